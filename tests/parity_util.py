"""Relative-l2 parity metric shared by the GPU tests.

Fields that stay near zero make the relative l2 of the field itself 0/0 or dominated
by round-off carried from larger fields; the denominator is floored at
1e-12 * s * sqrt(N) with s the field's scale (a field that stays at round-off is compared on its scale), and
velocity and flux components are measured against the norm of the whole vector."""
import numpy as np

# Scales for the relative-l2 floor of fields that stay near zero: err = ||a-b|| / max(||b||, 1e-12 s sqrt(N)).
SCALE = {"UX": 62.5, "UY": 62.5, "UZ": 62.5, "P": 2e4, "PMU": 2.5e5, "PMA": 2.5e5, "PBA": 6.67e7, "PBSE": 6.67e7,
         "ADP": 2e-3, "S1": 1.7e-4, "S2": 1.4e-3, "E1": 1.7e-4, "E2": 1.4e-3, "S1B": 1.7e-4, "S2B": 1.4e-3,
         "E1B": 1.7e-4, "E2B": 1.4e-3, "C1": 1.4e-3, "C2": 1.4e-3, "E0": 1.5e-7, "C0": 1.5e-7, "ETA": 1.0,
         "SIGMA": 1.0, "PHIX": 1e-2, "PHIY": 1e-2, "PHIZ": 1e-2, "I": 3.4e-3, "E2I": 1.4e-3}


def rel_l2(a, b, name):
    floor = 1e-12 * SCALE[name] * np.sqrt(max(b.size, 1))
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), floor)


VECTOR = {"UX": ("UX", "UY", "UZ"), "UY": ("UX", "UY", "UZ"), "UZ": ("UX", "UY", "UZ"),
          "PHIX": ("PHIX", "PHIY", "PHIZ"), "PHIY": ("PHIX", "PHIY", "PHIZ"), "PHIZ": ("PHIX", "PHIY", "PHIZ")}


def compare(gpu, ref, tol, names=None):
    """Relative l2 per field; velocity and flux components are measured against the
    norm of the whole vector (the transverse components are ~1e-3 of the axial one)."""
    worst = {}
    for n in (names or ref.keys()):
        if n not in gpu:
            continue
        if n in VECTOR:
            den = np.sqrt(sum(np.linalg.norm(ref[c]) ** 2 for c in VECTOR[n] if c in ref))
            size = sum(ref[c].size for c in VECTOR[n] if c in ref)
            den = max(den, 1e-12 * SCALE[n] * np.sqrt(max(size, 1)))    # no flow: a zero vector
            worst[n] = np.linalg.norm(gpu[n] - ref[n]) / den
        else:
            worst[n] = rel_l2(gpu[n], ref[n], n)
    bad = {k: v for k, v in worst.items() if not v <= tol}
    print({k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    assert not bad, bad




# ---- comparison with the oracle goldens of the full-size workloads ---------------------
GOLDEN_SPECIES = ["PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2", "S1B", "S2B", "E1B", "E2B", "C1", "C2"]


def load_golden(path):
    """A golden written by tests/golden/make_workload_goldens.py: (meta, arrays)."""
    import json
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    return meta, {k: z[k] for k in z.files if k != "meta"}


def compare_golden(fields, meta, g, tol, names=None, report=("P", "ETA")):
    """Relative l2 of a GPU run's fields against the oracle golden of the same workload
    and step count: on the golden's cell sample (velocity as one vector; each species
    with the near-zero floor, on the sample's size), on the full-field norms, and on the
    injury-face species in full.  Pressure and eta are reported, not checked."""
    idx = g["idx"]
    dim = meta["desc"]["dim"]
    vel = ["UX", "UY"] + (["UZ"] if dim == 3 else [])
    errs = {}
    den = np.sqrt(sum(np.linalg.norm(g["s_" + c]) ** 2 for c in vel))
    errs["U(sample)"] = np.sqrt(sum(np.linalg.norm(fields[c][idx] - g["s_" + c]) ** 2 for c in vel)) / den
    nfull = np.sqrt(sum(float(g["n_" + c]) ** 2 for c in vel))
    ngot = np.sqrt(sum(np.linalg.norm(fields[c]) ** 2 for c in vel))
    errs["U(norm)"] = abs(ngot - nfull) / nfull
    for n in (names or GOLDEN_SPECIES):
        b = g["s_" + n]
        floor = 1e-12 * SCALE[n] * np.sqrt(max(b.size, 1))
        errs[n + "(sample)"] = np.linalg.norm(fields[n][idx] - b) / max(np.linalg.norm(b), floor)
        nb = float(g["n_" + n])
        ffloor = 1e-12 * SCALE[n] * np.sqrt(max(fields[n].size, 1))
        errs[n + "(norm)"] = abs(np.linalg.norm(fields[n]) - nb) / max(nb, ffloor)
    for n in ("E0", "C0"):
        b = g["f_" + n]
        if b.size:
            errs[n] = rel_l2(fields[n], b, n)
    rep = {}
    for n in report:
        b = g["s_" + n]
        rep[n] = np.linalg.norm(fields[n][idx] - b) / max(np.linalg.norm(b), 1e-300)
    print({k: f"{v:.2e}" for k, v in errs.items()}, {k: f"{v:.2e}" for k, v in rep.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    return errs, bad
