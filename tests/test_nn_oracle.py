"""Pins of the FP64 reference of the learned preconditioner (no GPU).

The backward pass is checked against central differences of the loss; the
forward pass against what its definition fixes exactly: block-Jacobi when the
output layer is zero, Dirichlet dofs untouched, equivariance under scaling of
the input, and the aggregation transpose."""
import numpy as np
import pytest

import oracle as O
from oracle import nn_oracle as NN
from paper_2402_10348_amd import workloads as W

H, L = 8, 2


def small_system(name="disk2d"):
    prob = W.cavity_disk_2d(n=5) if name == "disk2d" else W.cavity_sphere_3d(n=3)
    c = O.Case(prob)
    lvl, it = W.perturbed_state(prob, seed=3)
    R, J = c.ns_assemble(lvl, it)
    rowptr, col = c.graph()
    bs = prob.dim + 1
    J = J.reshape(-1, bs, bs)
    mask = np.ones((prob.n_nodes, bs))
    for k in range(bs):
        sel = (prob.dir_mask >> k) & 1 == 1
        mask[prob.dir_node[sel], k] = 0.0
    return prob, rowptr, col, J, NN.block_inverses(rowptr, col, J), mask, bs


def random_theta(bs, seed, out_scale=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {}
    for name, shp in NN.layout(bs, H, L):
        fan = shp[0] if len(shp) == 2 else 1
        P[name] = rng.standard_normal(shp) / np.sqrt(fan) * (out_scale if name == "W_out" else 1.0)
        if name.startswith("b"):
            P[name] = 0.1 * rng.standard_normal(shp)
    return NN.pack(P, bs, H, L)


def spmv(rowptr, col, J, x):
    N = rowptr.shape[0] - 1
    y = np.zeros_like(x)
    for i in range(N):
        for k in range(rowptr[i], rowptr[i + 1]):
            y[i] += J[k] @ x[col[k]]
    return y


@pytest.mark.parametrize("name", ["disk2d", "sphere3d"])
def test_gradient_matches_central_differences(name):
    prob, rowptr, col, J, Dinv, mask, bs = small_system(name)
    rng = np.random.Generator(np.random.PCG64(11))
    N = prob.n_nodes
    e = mask * rng.standard_normal((N, bs))
    r = spmv(rowptr, col, J, e)
    theta = random_theta(bs, 5)
    loss, g = NN.loss_and_grad(theta, rowptr, col, Dinv, mask, r, e, bs, H, L)
    assert loss > 0.0
    idx = rng.choice(theta.size, size=60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = NN.loss_and_grad(tp, rowptr, col, Dinv, mask, r, e, bs, H, L)
        lm, _ = NN.loss_and_grad(tm, rowptr, col, Dinv, mask, r, e, bs, H, L)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_output_layer_is_block_jacobi_and_dirichlet_untouched():
    prob, rowptr, col, J, Dinv, mask, bs = small_system()
    rng = np.random.Generator(np.random.PCG64(2))
    r = rng.standard_normal((prob.n_nodes, bs))
    theta = random_theta(bs, 7)
    P = NN.unpack(theta, bs, H, L)
    P["W_out"][:] = 0.0
    z = NN.forward(NN.pack(P, bs, H, L), rowptr, col, Dinv, mask, r, bs, H, L)
    u = np.einsum("nij,nj->ni", Dinv, r)
    assert np.array_equal(z, u)
    z2 = NN.forward(theta, rowptr, col, Dinv, mask, r, bs, H, L)
    assert np.array_equal(z2[mask == 0], u[mask == 0])
    assert np.abs(z2 - u).max() > 0


def test_scale_equivariance():
    prob, rowptr, col, J, Dinv, mask, bs = small_system("sphere3d")
    rng = np.random.Generator(np.random.PCG64(4))
    r = rng.standard_normal((prob.n_nodes, bs))
    theta = random_theta(bs, 8)
    z1 = NN.forward(theta, rowptr, col, Dinv, mask, r, bs, H, L)
    z2 = NN.forward(theta, rowptr, col, Dinv, mask, 37.5 * r, bs, H, L)
    assert np.allclose(z2, 37.5 * z1, rtol=1e-12, atol=0)


def test_aggregation_transpose():
    prob, rowptr, col, J, Dinv, mask, bs = small_system("sphere3d")
    rng = np.random.Generator(np.random.PCG64(6))
    h = rng.standard_normal((prob.n_nodes, 5))
    y = rng.standard_normal((prob.n_nodes, 5))
    lhs = np.sum(NN.mean_agg(rowptr, col, h) * y)
    rhs = np.sum(h * NN.mean_agg_T(rowptr, col, y))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # a constant field is a fixed point of the mean
    assert np.allclose(NN.mean_agg(rowptr, col, np.ones((prob.n_nodes, 2))), 1.0)


def test_exact_pair_has_zero_loss():
    prob, rowptr, col, J, Dinv, mask, bs = small_system()
    rng = np.random.Generator(np.random.PCG64(9))
    r = rng.standard_normal((prob.n_nodes, bs))
    theta = random_theta(bs, 1)
    P = NN.unpack(theta, bs, H, L)
    P["W_out"][:] = 0.0
    th = NN.pack(P, bs, H, L)
    u = np.einsum("nij,nj->ni", Dinv, r)
    loss, g = NN.loss_and_grad(th, rowptr, col, Dinv, mask, r, u, bs, H, L)
    assert loss == 0.0 and np.all(g == 0.0)


def test_device_arithmetic_mode_stays_near_the_definition():
    """The BF16/FP32 emulation of the reference stays within the BF16
    rounding (a few 1e-3) of the FP64 definition, and its BF16 rounding is
    to nearest even on the FP32 bit pattern."""
    b = NN._bf16(np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, 1.5 * 2.0 ** -20]))
    assert b[0] == 1.0                      # a tie rounds to the even neighbour
    assert b[1] == 1.0 + 2.0 ** -6          # a tie rounds to the even neighbour (upwards)
    assert b[2] == 1.0                      # below half an ulp
    assert b[3] == 1.5 * 2.0 ** -20         # exactly representable
    prob, rowptr, col, J, Dinv, mask, bs = small_system("sphere3d")
    rng = np.random.Generator(np.random.PCG64(4))
    r = rng.standard_normal((prob.n_nodes, bs))
    theta = random_theta(bs, 6, out_scale=1.0)
    z = NN.forward(theta, rowptr, col, Dinv, mask, r, bs, H, L)
    zm = NN.forward(theta, rowptr, col, Dinv, mask, r, bs, H, L, emulate=True)
    u = np.einsum("nij,nj->ni", Dinv, r)
    d = np.abs(zm - z).max() / np.abs(z - u).max()
    assert 1e-5 < d < 3e-2
