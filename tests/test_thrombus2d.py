"""CPU checks of the paper's 2-D thrombosis example set-up (section 4.1): geometry and
the adhesion region whose cell count is the level of the temporary plateau the paper
reports for the area above 10% of P_max."""
import numpy as np

import clot_inputs as ci
from oracle import clot_oracle as oc
from paper_2304_09180_amd import thrombus2d


def test_example_geometry_and_adhesion_region():
    d = thrombus2d.channel()
    assert (d["nx"], d["ny"], d["nz"]) == (128, 32, 1)
    assert d["Lx"] == 0.24 and d["Ly"] == 0.06
    dx = d["Lx"] / d["nx"]                              # 1.875 um
    assert abs(dx - 1.875e-3) < 1e-15
    # a ~90 um patch: the bottom-wall faces whose centre lies in it
    assert ci.n_injury_faces(d) == 48
    # cells over the patch whose centre lies within one platelet diameter (3 um) of the
    # wall: centres at 0.9375 and 2.8125 um, so two layers of 48
    o = oc.Oracle(d, np.zeros((15, ci.ncell(d))), np.zeros((2, 48)))
    hadh = o.hadh.reshape(32, 128)
    assert int((hadh > 0).sum()) == 96
    assert (hadh[:2] > 0).sum() == 96 and (hadh[2:] > 0).sum() == 0
