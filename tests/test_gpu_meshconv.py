"""The mesh-convergence driver end to end on the GPU, shortened: three nested meshes of
the test channel in one context for 100 common steps."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_mesh_convergence_driver_runs_and_reports_finite_errors(capsys):
    from paper_2304_09180_amd import meshconv
    assert meshconv.main(["--h", "3", "1.5", "0.75", "--dt", "4e-6", "--seconds", "4e-4", "--chunk", "50"]) == 0
    res = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    print(res, flush=True)
    assert res["grids"] == [[40, 10], [80, 20], [160, 40]] and res["steps"] == 100
    assert res["status"] == ["OK", "OK", "OK"]
    assert all(abs(t - 4e-4) < 1e-12 for t in res["t"])
    for q in ("S1", "E1", "PMU", "E2+E2B"):
        e = res["quantities"][q]["errors"]
        assert len(e) == 2 and all(np.isfinite(x) and x >= 0.0 for x in e), (q, e)
        assert np.isfinite(res["quantities"][q]["rate"])


def test_mesh_convergence_study_resumes_from_a_checkpoint(tmp_path, capsys):
    """A study split over two calls (stop after 50 steps, save; load, finish) reports the
    same errors, bit for bit, as one call of 100 steps."""
    from paper_2304_09180_amd import meshconv
    base = ["--h", "3", "1.5", "0.75", "--dt", "4e-6", "--seconds", "4e-4", "--chunk", "25"]
    assert meshconv.main(base) == 0
    whole = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    ck = str(tmp_path / "state.npy")
    assert meshconv.main(base + ["--max-steps", "50", "--save", ck]) == 0
    first = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert first["stopped_at"] == 50 and first["of"] == 100
    assert meshconv.main(base + ["--load", ck]) == 0
    rest = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert rest["steps"] == 100 and rest["status"] == ["OK", "OK", "OK"]
    assert rest["quantities"] == whole["quantities"]
