"""The Galerkin coarse operators of the multigrid preconditioner: every
coarse level equals P^T A P of the level above, computed here with scipy from
the exported fine operator and the interpolation of the nested Kuhn meshes
(weights 1 and 1/2, masked on the Dirichlet dofs of both levels; unit rows
for the coarse level's Dirichlet dofs), up to the FP32 storage of the
intermediate levels; and FGMRES preconditioned with it (also with more
smoothing sweeps on the coarse levels) reaches the solution of the same
system as point-block Jacobi."""
import sys

import numpy as np
import pytest

from paper_2402_10348_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def interpolation(dim, nf, fmask, cmask):
    """P: fine dofs x coarse dofs for cells nf (fine) -> nf/2 (coarse)."""
    import scipy.sparse as sp
    bs = dim + 1
    nc = [n // 2 for n in nf]
    fx, fy = nf[0] + 1, nf[1] + 1
    cx, cy = nc[0] + 1, nc[1] + 1
    Nf = int(np.prod([n + 1 for n in nf]))
    rows, cols, vals = [], [], []
    for f in range(Nf):
        c = [f % fx, (f // fx) % fy, f // (fx * fy) if dim == 3 else 0]
        odd = [v & 1 for v in c]
        base = [v >> 1 for v in c]
        par = [(base, 1.0)]
        if any(odd):
            par = [(base, 0.5), ([b + o for b, o in zip(base, odd)], 0.5)]
        for p, w in par:
            I = p[0] + cx * (p[1] + cy * (p[2] if dim == 3 else 0))
            for k in range(bs):
                if (fmask[f] >> k) & 1 and (cmask[I] >> k) & 1:
                    rows.append(f * bs + k)
                    cols.append(I * bs + k)
                    vals.append(w)
    Nc = int(np.prod([n + 1 for n in nc]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(Nf * bs, Nc * bs))


def bsr(rowptr, col, val):
    import scipy.sparse as sp
    bs = val.shape[1]
    n = rowptr.shape[0] - 1
    return sp.bsr_matrix((val, col, rowptr), shape=(n * bs, n * bs)).tocsr()


@pytest.mark.parametrize("name", ["disk2d_16", "sphere3d_8", "floes_16x8x4"])
def test_galerkin_levels_equal_ptap(name):
    from paper_2402_10348_amd.eft import Context
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    prob = {"disk2d_16": lambda: W.cavity_disk_2d(n=16), "sphere3d_8": lambda: W.cavity_sphere_3d(n=8),
            "floes_16x8x4": lambda: W.floe_field_3d(nx=16, ny=8, nz=4, n_floes=2)}[name]()
    dim, bs = prob.dim, prob.dim + 1
    say(f"[galerkin] {name} N={prob.n_nodes}")
    lvl, it = W.perturbed_state(prob, seed=9)
    ctx = Context(prob, mg_galerkin=1, precond=1)
    ctx.assemble(ctx.device_state(lvl), ctx.device_state(it))
    full = (1 << bs) - 1
    dm = np.zeros(prob.n_nodes, np.uint8)
    for n, m in zip(prob.dir_node, prob.dir_mask):
        dm[n] |= m
    fmask = (full & ~dm).astype(np.uint8)
    nf = [int(g) for g in prob.grid[:dim]]
    rp, cl, va, nlev = ctx.mg_level(0)
    Af = bsr(to_np(rp), to_np(cl), to_np(va))
    assert nlev >= 3
    # fine node of each level's node (injection), for the coarse masks
    inj = np.arange(prob.n_nodes)
    for lev in range(1, nlev):
        nc = [n // 2 for n in nf]
        fx, fy = nf[0] + 1, nf[1] + 1
        cx, cy = nc[0] + 1, nc[1] + 1
        Nc = int(np.prod([n + 1 for n in nc]))
        I = np.arange(Nc)
        ci, cj = I % cx, (I // cx) % cy
        ck = I // (cx * cy) if dim == 3 else np.zeros_like(I)
        fnode = 2 * ci + fx * (2 * cj + fy * 2 * ck)
        cinj = inj[fnode]
        cmask = (full & ~dm[cinj]).astype(np.uint8)
        P = interpolation(dim, nf, fmask, cmask)
        Ac = (P.T @ Af @ P).tolil()
        for Ic in range(Nc):
            for k in range(bs):
                if not (cmask[Ic] >> k) & 1:
                    Ac[Ic * bs + k, :] = 0.0
                    Ac[Ic * bs + k, Ic * bs + k] = 1.0
        Ac = Ac.tocsr()
        rp, cl, va, _ = ctx.mg_level(lev)
        G = bsr(to_np(rp), to_np(cl), to_np(va))
        err = abs(G - Ac).max() / abs(Ac).max()
        say(f"  level {lev}: N={Nc} max rel err {err:.2e}")
        assert err < 2e-6, (lev, err)
        Af, fmask, nf, inj = G, cmask, nc, cinj
    ctx.close()


@pytest.mark.parametrize("name", ["sphere3d_16", "floes_32x16x8"])
def test_galerkin_multigrid_same_solution(name):
    from paper_2402_10348_amd.eft import Context
    import torch
    prob = {"sphere3d_16": lambda: W.cavity_sphere_3d(n=16),
            "floes_32x16x8": lambda: W.floe_field_3d(nx=32, ny=16, nz=8, n_floes=3)}[name]()
    say(f"[galerkin solve] {name} N={prob.n_nodes}")
    lvl, it = W.perturbed_state(prob, seed=10)
    sols = {}
    for tag, over in (("bj", dict(precond=0)), ("mg", dict(precond=1, mg_galerkin=0)),
                      ("galerkin", dict(precond=1, mg_galerkin=1)),
                      ("galerkin_coarse8", dict(precond=1, mg_galerkin=1, mg_cnu=8, mg_cnu_post=8))):
        ctx = Context(prob, lin_rtol=1e-12, restart=200, lin_maxit=40000, **over)
        R = ctx.assemble(ctx.device_state(lvl), ctx.device_state(it))
        x, info = ctx.fgmres(-R)
        say(f"  {tag}: iters {info['iters']} converged {info['converged']} fallback {info['fallback']}")
        assert info["converged"] == 1 and info["fallback"] == 0
        sols[tag] = (to_np(x), info["iters"])
        ctx.close()
    ref = sols["bj"][0]
    for tag in ("mg", "galerkin", "galerkin_coarse8"):
        e = np.linalg.norm(sols[tag][0] - ref) / np.linalg.norm(ref)
        assert e < 1e-8, (tag, e)
    assert sols["galerkin"][1] < sols["bj"][1]
    # more smoothing on the coarse levels strengthens the coarse correction
    assert sols["galerkin_coarse8"][1] <= sols["galerkin"][1]


def test_lagged_coarse_levels_reach_the_same_step():
    """mg_lag = 1 keeps the coarse levels of a step's first nonlinear
    iteration: the preconditioner changes, the converged fields do not
    (both runs solved tightly)."""
    import torch
    from paper_2402_10348_amd.eft import Context
    prob = W.cavity_sphere_3d(n=16)
    say("[mg] lagged coarse levels, sphere3d n=16, 3 steps")
    out = {}
    for lag in (0, 1):
        ctx = Context(prob, mg_lag=lag, mg_galerkin=1, lin_rtol=1e-12, nl_rtol=1e-9, nl_max=30)
        st = ctx.device_state(prob.state_copy())
        t, k, its = 0.0, 0, []
        for _ in range(3):
            info = ctx.step(st, t=t, step=k)
            t, k = info["t"], info["step"]
            its.append((info["nl_iters"], info["lin_iters_block"][0], info["converged"]))
        torch.cuda.synchronize()
        say(f"  mg_lag={lag}: (nonlinear, momentum Krylov, converged) per step {its}")
        assert all(c == 1 for _, _, c in its)
        out[lag] = {n: v.cpu().numpy() for n, v in st.items()}
        ctx.close()
    for n in out[0]:
        a, b = out[0][n], out[1][n]
        d = float(np.abs(a - b).max()) / max(float(np.abs(a).max()), 1e-300)
        say(f"  {n}: rel diff {d:.2e}")
        assert d <= 1e-7, n
