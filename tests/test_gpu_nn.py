"""Learned right preconditioner on the GPU (through the C ABI) against its
FP64 numpy reference, and what training it buys over block Jacobi.

Tolerances: the dense layers use BF16 operands (8-bit mantissa) with FP32
accumulation, so forward outputs and gradients are compared at 2e-2 and 5e-2
relative (a dropped term or a transposed operand moves them by O(1))."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import nn_oracle as NNO
from paper_2402_10348_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def setup(prob, **over):
    from paper_2402_10348_amd.eft import Context
    ctx = Context(prob, **over)
    c = O.Case(prob)
    rowptr, col = c.graph()
    bs = prob.dim + 1
    mask = np.ones((prob.n_nodes, bs))
    for k in range(bs):
        sel = (prob.dir_mask >> k) & 1 == 1
        mask[prob.dir_node[sel], k] = 0.0
    return ctx, c, rowptr, col, mask, bs


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def active_theta(ctx, seed):
    """The initialized parameters with a random nonzero output layer."""
    theta = ctx.nn_params().astype(np.float64)
    sh = ctx.nn_shape()
    bs = ctx.bs
    lay = NNO.layout(bs, sh["hidden"], sh["layers"])
    rng = np.random.Generator(np.random.PCG64(seed))
    o = 0
    for name, shp in lay:
        n = int(np.prod(shp))
        if name == "W_out":
            theta[o:o + n] = 0.2 * rng.standard_normal(n)
        if name.startswith("b"):
            theta[o:o + n] = 0.05 * rng.standard_normal(n)
        o += n
    return theta.astype(np.float32)


@pytest.mark.parametrize("name", ["disk2d", "sphere3d"])
def test_forward_and_gradient_match_reference(torch_cuda, name):
    prob = W.cavity_disk_2d(n=8) if name == "disk2d" else W.cavity_sphere_3d(n=6)
    say(f"[nn] forward/gradient {name} N={prob.n_nodes}")
    ctx, c, rowptr, col, mask, bs = setup(prob)
    ctx.nn_init(seed=3)
    sh = ctx.nn_shape()
    H, L = sh["hidden"], sh["layers"]
    assert sh["n_params"] == NNO.n_params(bs, H, L)
    rng = np.random.Generator(np.random.PCG64(1))
    u = rng.standard_normal((prob.n_nodes, bs))
    e = mask * rng.standard_normal((prob.n_nodes, bs))
    ud, ed = ctx.tensor(u), ctx.tensor(e)
    ident = np.broadcast_to(np.eye(bs), (prob.n_nodes, bs, bs))
    # zero output layer: exactly block Jacobi (the identity on u here)
    z0 = ctx.nn_apply(ud).cpu().numpy()
    assert np.array_equal(z0, u)
    theta = active_theta(ctx, 4)
    ctx.nn_params(theta)
    z = ctx.nn_apply(ud).cpu().numpy()
    zr = NNO.forward(theta.astype(np.float64), rowptr, col, ident, mask, u, bs, H, L)
    # against the FP64 definition (BF16 operands: about 1e-2) and, tightly,
    # against the same map in the device's arithmetic (BF16 operands of the
    # matrix-core products, FP32 storage), which pins the kernels' terms
    zm = NNO.forward(theta.astype(np.float64), rowptr, col, ident, mask, u, bs, H, L, emulate=True)
    say(f"  forward rel {rel(z - u, zr - u):.2e} (FP64 reference), {rel(z - u, zm - u):.2e} (device arithmetic)")
    assert rel(z - u, zr - u) < 2e-2
    assert rel(z - u, zm - u) < 2e-5
    assert np.array_equal(z[mask == 0], u[mask == 0])
    loss, g = ctx.nn_loss_grad(ud, ed)
    lr_, gr = NNO.loss_and_grad(theta.astype(np.float64), rowptr, col, ident, mask, u, e, bs, H, L)
    # (the pair is handed to the device in FP32)
    lm, gm = NNO.loss_and_grad(theta.astype(np.float64), rowptr, col, ident, mask, u.astype(np.float32), e, bs, H,
                               L, emulate=True)
    say(f"  loss gpu {loss:.6e} ref {lr_:.6e} device arithmetic {lm:.6e}")
    assert abs(loss - lr_) <= 2e-2 * lr_
    assert abs(loss - lm) <= 2e-6 * lm
    o = 0
    for nm, shp in NNO.layout(bs, H, L):
        n = int(np.prod(shp))
        e_t, e_m = rel(g[o:o + n], gr[o:o + n]), rel(g[o:o + n], gm[o:o + n])
        say(f"  grad {nm}: rel {e_t:.2e} (FP64 reference), {e_m:.2e} (device arithmetic)")
        assert e_t < 5e-2, nm
        assert e_m < 2.5e-4, nm
        o += n
    ctx.close()


def test_training_reduces_krylov_iterations(torch_cuda):
    """Pairs harvested from the block-Jacobi solves of two cavity steps; after
    training, FGMRES with the learned preconditioner needs fewer iterations
    than block Jacobi on a new system and reaches the same solution."""
    torch = torch_cuda
    prob = W.cavity_sphere_3d(n=12)
    say(f"[nn] training sphere3d n=12 N={prob.n_nodes}")
    ctx, c, rowptr, col, mask, bs = setup(prob, precond=0, lin_rtol=1e-8, restart=100, lin_maxit=5000)
    ctx.nn_init(seed=7)
    ctx.nn_harvest(256)
    st = ctx.device_state(prob.state_copy())
    t, k = 0.0, 0
    for _ in range(2):
        info = ctx.step(st, t=t, step=k)
        t, k = info["t"], info["step"]
    pairs = ctx.nn_shape()["pairs"]
    say(f"  harvested pairs {pairs}")
    assert pairs >= 32
    losses = ctx.nn_train(steps=400, batch=4, lr=2e-3, seed=1)
    a, b = float(np.mean(losses[:20])), float(np.mean(losses[-20:]))
    say(f"  loss first {a:.4f} last {b:.4f}")
    assert b < 0.8 * a
    lvl, it = W.perturbed_state(prob, seed=31, amp_v=0.05, amp_p=0.01, amp_phi=0.0, amp_B=0.0, amp_rate=0.05)
    R = ctx.assemble(ctx.device_state(lvl), ctx.device_state(it))
    res = {}
    for pc in (0, 2):
        ctx.set_params(precond=pc)
        x, si = ctx.fgmres(-R)
        r = -R - ctx.spmv(x)
        rr = float(torch.linalg.norm(r) / torch.linalg.norm(R))
        say(f"  precond={pc} iters={si['iters']} rel_res={rr:.2e}")
        assert si["converged"] == 1 and rr <= 1.0001e-8
        res[pc] = (x.cpu().numpy(), si["iters"])
    assert res[2][1] < res[0][1]
    # the same solution: two solves to 1e-8 differ by up to cond(A) 1e-8, so
    # the answers are compared after solving to 1e-12
    xs = {}
    for pc in (0, 2):
        ctx.set_params(precond=pc, lin_rtol=1e-12)
        x, si = ctx.fgmres(-R)
        assert si["converged"] == 1
        xs[pc] = x.cpu().numpy()
    say(f"  solutions at 1e-12: rel diff {rel(xs[2], xs[0]):.2e}")
    assert rel(xs[2], xs[0]) < 1e-7
    ctx.close()


def test_multigrid_base(torch_cuda):
    """nn_base = 1: with the initial zero output layer the learned
    preconditioner is the V-cycle itself (the same solve, bit for bit); pairs
    (V-cycle of A z_j, z_j) are harvested from multigrid steps (the harvest
    runs one ungated V-cycle per solve besides the gated ones of the columns),
    training runs on them, and the trained network still reaches the
    multigrid solution."""
    torch = torch_cuda
    prob = W.cavity_sphere_3d(n=16)
    say(f"[nn] multigrid base sphere3d n=16 N={prob.n_nodes}")
    ctx, c, rowptr, col, mask, bs = setup(prob, precond=1, nn_base=1, lin_rtol=1e-8, restart=50, lin_maxit=2000)
    ctx.nn_init(seed=5)
    lvl, it = W.perturbed_state(prob, seed=33, amp_v=0.05, amp_p=0.01, amp_phi=0.0, amp_B=0.0, amp_rate=0.05)
    R = ctx.assemble(ctx.device_state(lvl), ctx.device_state(it))
    b = (-R).contiguous()
    sol = {}
    for pc in (1, 2):
        ctx.set_params(precond=pc)
        x, si = ctx.fgmres(b)
        say(f"  untrained precond={pc}: iters={si['iters']} rel_res={si['rel_res']:.2e}")
        assert si["converged"] == 1 and si["fallback"] == 0
        sol[pc] = (x.clone(), si["iters"])
    assert sol[1][1] == sol[2][1] and torch.equal(sol[1][0], sol[2][0])
    # harvest from multigrid steps, train
    ctx.set_params(precond=1)
    ctx.nn_harvest(256)
    st = ctx.device_state(prob.state_copy())
    t, k = 0.0, 0
    for _ in range(3):
        info = ctx.step(st, t=t, step=k)
        t, k = info["t"], info["step"]
    pairs = ctx.nn_shape()["pairs"]
    say(f"  harvested pairs {pairs}")
    assert pairs >= 32
    losses = ctx.nn_train(steps=300, batch=4, lr=1e-3, seed=2)
    a, l1 = float(np.mean(losses[:20])), float(np.mean(losses[-20:]))
    # (reported, not asserted: these pairs are the multigrid-preconditioned
    # Krylov directions, where the V-cycle is least accurate, and a local
    # network that sees only its output gains little on them)
    say(f"  loss first {a:.4f} last {l1:.4f}")
    assert np.all(np.isfinite(losses))
    ctx.nn_harvest(0)
    ctx.set_params(precond=2, lin_rtol=1e-12)
    x2, si = ctx.fgmres(b)
    say(f"  trained precond=2 at 1e-12: iters={si['iters']} fallback={si['fallback']}")
    ctx.set_params(precond=1, lin_rtol=1e-12)
    x1, s1 = ctx.fgmres(b)
    say(f"  multigrid at 1e-12: iters={s1['iters']}; solutions rel diff {rel(x2.cpu().numpy(), x1.cpu().numpy()):.2e}")
    assert si["converged"] == 1 and s1["converged"] == 1
    assert rel(x2.cpu().numpy(), x1.cpu().numpy()) < 1e-7
    ctx.close()
