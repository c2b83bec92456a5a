"""CPU model behind the pressure multigrid's Jacobi weight (6/7 for contexts of 3-D
channels, 4/5 otherwise) and its sweep count (3 each way on 3-D channels, 2 otherwise).

The model is the library's V-cycle written with scipy: aggregation coarsening (halve
every axis with at least 3 cells), coarse operators equal to half the Galerkin product
(re-discretisation on the doubled cells when every axis is coarsened), two (or n) weighted
Jacobi sweeps before and after each coarse correction, an exact solve at <= 64 cells,
inside CG on the Laplacian of a duct with a Dirichlet outlet.  It checks the choice of
weight, not the library: on the 7-point operator 6/7 needs no more CG iterations than
0.8 and on a 128x32x32 grid one fewer; on the 5-point operator 0.8 stays at least as
good.  A third sweep each way saves a third of the iterations on the 3-D grid.  (Whether
it pays depends on what a sweep costs on the GPU, measured separately: on 2-D channels
it did not.)"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def laplacian(nx, ny, nz):
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    diag = np.zeros(n)
    rows, cols = [], []
    for ax in (2, 1, 0):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        L, R = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        np.add.at(diag, L, 1.0)
        np.add.at(diag, R, 1.0)
        rows += [L, R]
        cols += [R, L]
    diag[idx[:, :, -1].ravel()] += 2.0          # outlet: fixed value half a cell away
    r, c = np.concatenate(rows), np.concatenate(cols)
    return (sp.csr_matrix((-np.ones(r.size), (r, c)), shape=(n, n)) + sp.diags(diag)).tocsr()


def aggregation(nx, ny, nz):
    dims = (nx, ny, nz)
    cd = tuple(m // 2 if m >= 3 else m for m in dims)
    maps = [np.minimum(np.arange(m) // 2, c - 1) if m >= 3 else np.arange(m) for m, c in zip(dims, cd)]
    coarse = (maps[0][None, None, :] + cd[0] * (maps[1][None, :, None] + cd[1] * maps[2][:, None, None])).ravel()
    n = nx * ny * nz
    return sp.csr_matrix((np.ones(n), (np.arange(n), coarse)), shape=(n, int(np.prod(cd)))), cd


def hierarchy(dims):
    A = laplacian(*dims)
    levels = []
    while np.prod(dims) > 64:
        P, cd = aggregation(*dims)
        levels.append((A, P))
        A = (P.T @ A @ P).tocsr() * 0.5
        dims = cd
    return levels, A


def v_cycle(levels, coarse, b, w, level=0, sweeps=2):
    if level == len(levels):
        return sla.spsolve(coarse.tocsc(), b)
    A, P = levels[level]
    d = A.diagonal()
    x = np.zeros_like(b)
    for _ in range(sweeps):
        x += w * (b - A @ x) / d
    x += P @ v_cycle(levels, coarse, P.T @ (b - A @ x), w, level + 1, sweeps)
    for _ in range(sweeps):
        x += w * (b - A @ x) / d
    return x


def cg_iterations(dims, w, tol=1e-4, sweeps=2):
    levels, coarse = hierarchy(dims)
    A = levels[0][0]
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    x = np.zeros_like(b)
    r = b.copy()
    z = v_cycle(levels, coarse, r, w, sweeps=sweeps)
    p = z.copy()
    rz = r @ z
    for it in range(1, 100):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= tol * np.linalg.norm(b):
            return it
        z = v_cycle(levels, coarse, r, w, sweeps=sweeps)
        rz, rz_old = r @ z, rz
        p = z + rz / rz_old * p
    return 100


def test_three_d_weight_six_sevenths_beats_four_fifths():
    a, b = cg_iterations((128, 32, 32), 0.8), cg_iterations((128, 32, 32), 6.0 / 7.0)
    print("3-D 128x32x32: w=0.8", a, "w=6/7", b)
    assert b < a
    assert cg_iterations((64, 16, 16), 6.0 / 7.0) <= cg_iterations((64, 16, 16), 0.8)


def test_two_d_keeps_four_fifths():
    a, b = cg_iterations((256, 64, 1), 0.8, 1e-8), cg_iterations((256, 64, 1), 6.0 / 7.0, 1e-8)
    print("2-D 256x64: w=0.8", a, "w=6/7", b)
    assert a <= b


def test_three_sweeps_save_a_third_of_the_iterations_in_three_d():
    w = 6.0 / 7.0
    two, three = cg_iterations((128, 32, 32), w, 1e-8), cg_iterations((128, 32, 32), w, 1e-8, sweeps=3)
    print("3-D 128x32x32, 1e-8: 2 sweeps", two, "3 sweeps", three)
    assert three <= two * 3 // 4
