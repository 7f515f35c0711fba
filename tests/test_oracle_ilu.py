"""Pins of the oracle's block ILU(0) preconditioner (CPU only).

ILU(0) is fixed by its defining property rather than by its algorithm: the
unit block-lower L and block-upper U keep A's pattern and their product
equals A on every block of that pattern (Saad, Iterative Methods for Sparse
Linear Systems, Sec. 10.3).  Checked here densely on small momentum
Jacobians; on a pattern without fill (block tridiagonal) the factorization
is the exact block LU, so the preconditioner inverts A."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from paper_2402_10348_amd import workloads as W


def dense_factors(lu, dinv, rowptr, col, n, bs):
    L = np.eye(n * bs)
    U = np.zeros((n * bs, n * bs))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = col[p]
            blk = lu[p].reshape(bs, bs)
            if j < i:
                L[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = blk
            else:
                U[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = blk
    return L, U


@pytest.mark.parametrize("name,seed", [("sphere3d_3", 1), ("disk2d_6", 2)])
def test_ilu0_product_matches_a_on_the_pattern(name, seed):
    prob = W.cavity_sphere_3d(n=3) if name == "sphere3d_3" else W.cavity_disk_2d(n=6)
    lvl, it = W.perturbed_state(prob, seed=seed)
    c = O.Case(prob)
    R, J = c.ns_assemble(lvl, it)
    rowptr, col = c.graph()
    n, bs = prob.n_nodes, prob.dim + 1
    lu, dinv, st = c.ilu0(J)
    assert st == 0
    L, U = dense_factors(lu.reshape(-1, bs * bs), dinv, rowptr, col, n, bs)
    LU = L @ U
    A = np.zeros_like(LU)
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            A[i * bs:(i + 1) * bs, col[p] * bs:(col[p] + 1) * bs] = J.reshape(-1, bs, bs)[p]
    scale = np.abs(A).max()
    on = np.zeros(LU.shape, dtype=bool)
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            on[i * bs:(i + 1) * bs, col[p] * bs:(col[p] + 1) * bs] = True
    assert np.abs(LU - A)[on].max() <= 1e-11 * scale
    # something is dropped off the pattern (otherwise the test would not see fill)
    assert np.abs(LU[~on]).max() > 1e-6 * scale
    # dinv holds the inverses of U's diagonal blocks
    for i in range(n):
        Uii = U[i * bs:(i + 1) * bs, i * bs:(i + 1) * bs]
        assert np.allclose(dinv[i].reshape(bs, bs) @ Uii, np.eye(bs), atol=1e-10)
    # the application solves L U z = r
    r = np.random.default_rng(seed).standard_normal(n * bs)
    z = c.ilu0_apply(lu, dinv, r)
    assert np.abs(LU @ z - r).max() <= 1e-10 * np.abs(r).max() * max(1.0, np.abs(LU).max() * np.abs(z).max() / np.abs(r).max())


def test_ilu0_exact_without_fill():
    """Block tridiagonal (a chain): no fill, ILU(0) = block LU, M^-1 A = I."""
    rng = np.random.default_rng(3)
    n, bs = 9, 4
    rowptr, col, blocks = [0], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                col.append(j)
                b = rng.standard_normal((bs, bs)) + (6.0 * np.eye(bs) if i == j else 0.0)
                blocks.append(b)
        rowptr.append(len(col))
    rowptr = np.array(rowptr, dtype=np.int32)
    col = np.array(col, dtype=np.int32)
    val = np.ascontiguousarray(np.stack(blocks).reshape(-1))
    lu = np.zeros_like(val)
    dinv = np.zeros(n * bs * bs)
    L = O.lib()
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    assert L.orc_ilu0(bs, n, ip(rowptr), ip(col), dp(val), dp(lu), dp(dinv)) == 0
    x = rng.standard_normal(n * bs)
    Ax = np.zeros(n * bs)
    L.orc_spmv(bs, n, ip(rowptr), ip(col), dp(val), dp(x), dp(Ax))
    z = np.zeros(n * bs)
    L.orc_ilu0_apply(bs, n, ip(rowptr), ip(col), dp(lu), dp(dinv), dp(Ax), dp(z))
    assert np.abs(z - x).max() <= 1e-12 * np.abs(x).max() * 10


def test_ilu0_reports_a_singular_pivot():
    prob = W.cavity_sphere_3d(n=3)
    lvl, it = W.perturbed_state(prob, seed=1)
    c = O.Case(prob)
    _, J = c.ns_assemble(lvl, it)
    rowptr, col = c.graph()
    bs = 4
    Jz = J.reshape(-1, bs * bs).copy()
    p = [q for q in range(rowptr[5], rowptr[6]) if col[q] == 5][0]
    Jz[p] = 0.0
    _, _, st = c.ilu0(Jz.reshape(J.shape))
    assert st == 1 + 5
