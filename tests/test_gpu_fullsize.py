"""The GPU path at the full sizes of the workload family, in the launch
configuration of the benchmark, against the oracle on sampled rows.

Sizes: falling sphere 96 x 96 x 192 (10.6M tets), hull among 16 floes
256 x 128 x 64 (12.6M tets, 18 indicators, 17 solids), cavity 128^3 (12.6M
tets).  The whole oracle assembly is too slow at these sizes, so it evaluates
sampled rows only (random rows, rows in every diffuse interface, boundary
rows); bands are compared whole (they are integer sets).  Tolerances as the
small cases: 1e-11 relative to the scale of the sampled rows."""
import sys

import numpy as np
import pytest

import oracle as O
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


CASES = {
    "falling_96x96x192": lambda: W.falling_sphere_3d(n=96),
    "floes_256x128x64": lambda: W.floe_field_3d(),
    "cavity_128": lambda: W.cavity_sphere_3d(n=128),
}


def predictor(prob):
    lvl = prob.state_copy()
    it = {k: lvl[k].copy() for k in ("vp", "phi", "B")}
    for k in range(prob.dim + 1):
        sel = (prob.dir_mask >> k) & 1 == 1
        it["vp"][prob.dir_node[sel], k] = prob.dir_val[sel, k]
    return lvl, it


def sample_rows(prob, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = set(rng.choice(prob.n_nodes, 300, replace=False).tolist())
    for k in range(prob.phi.shape[0]):
        near = np.nonzero(np.abs(prob.phi[k]) < 0.9)[0]
        if near.size:
            rows |= set(rng.choice(near, min(24, near.size), replace=False).tolist())
    rows |= set(rng.choice(prob.dir_node, min(24, prob.dir_node.size), replace=False).tolist())
    return np.array(sorted(rows), dtype=np.int32)


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_assembly_spmv_and_bands(torch_cuda, name):
    torch = torch_cuda
    from paper_2402_10348_amd.eft import Context
    prob = CASES[name]()
    say(f"[full size] {name} N={prob.n_nodes} E={prob.n_elems} indicators={prob.phi.shape[0]} "
        f"solids={prob.B.shape[0]}")
    ctx = Context(prob)
    c = O.Case(prob)
    lvl, it = predictor(prob)
    L = ctx.device_state(lvl)
    R = ctx.assemble(L, ctx.device_state(it))
    rows = sample_rows(prob, 7)
    say(f"  sampled rows {rows.size}")
    R0, J0 = c.ns_rows(lvl, it, rows)
    Rg = R[torch.as_tensor(rows.astype(np.int64), device=R.device)].cpu().numpy()
    scale = float(np.abs(R0).max())
    say(f"  residual: max|R| {scale:.3e}, max diff {float(np.abs(Rg - R0).max()):.3e}")
    assert scale > 0.0 and float(np.abs(Rg - R0).max()) <= 1e-11 * scale
    rowptr, col, val = ctx.matrix()
    rp = rowptr.cpu().numpy()
    x = np.random.Generator(np.random.PCG64(3)).standard_normal((prob.n_nodes, prob.dim + 1))
    y = ctx.spmv(ctx.tensor(x)).cpu().numpy()
    worst_j = worst_y = 0.0
    for q, r in enumerate(rows):
        cols, blocks = J0[q]
        gcols = col[rp[r]:rp[r + 1]].cpu().numpy()
        gval = val[rp[r]:rp[r + 1]].cpu().numpy()
        assert np.array_equal(gcols, cols)
        js = max(float(np.abs(blocks).max()), 1e-300)
        worst_j = max(worst_j, float(np.abs(gval - blocks).max()) / js)
        y0 = np.einsum("kij,kj->i", blocks, x[cols])
        ys = float(np.einsum("kij,kj->i", np.abs(blocks), np.abs(x[cols])).max())
        worst_y = max(worst_y, float(np.abs(y[r] - y0).max()) / max(ys, 1e-300))
    say(f"  Jacobian rows rel {worst_j:.2e}, SpMV rows rel {worst_y:.2e}")
    assert worst_j <= 1e-11 and worst_y <= 1e-11
    del rowptr, col, val
    ctx.bands_build(L)
    for k in range(prob.phi.shape[0]):
        be, fr = ctx.band_export(k)
        be0, fr0 = c.band(lvl["phi"][k])
        assert np.array_equal(be.cpu().numpy(), be0), k
        assert np.array_equal(fr.cpu().numpy(), fr0), k
    say(f"  bands equal for {prob.phi.shape[0]} indicators")
    ctx.close()


@pytest.mark.parametrize("name", ["falling_96x96x192", "cavity_128", "floes_256x128x64"])
def test_full_size_step(torch_cuda, name):
    """One time step at full size: the nonlinear loop runs to its stop rule
    (or the cap), and the last momentum solve's true residual meets lin_rtol;
    indicators stay within the bound the oracle shows for them."""
    torch = torch_cuda
    from paper_2402_10348_amd.eft import Context
    prob = CASES[name]()
    say(f"[full size step] {name} N={prob.n_nodes}")
    ctx = Context(prob, nl_max=6, lin_maxit=4000)
    st = ctx.device_state(prob.state_copy())
    info = ctx.step(st)
    say(f"  nl={info['nl_iters']} conv={info['converged']} lin={info['lin_iters_total']} "
        f"by block={info['lin_iters_block'][:4]} t_asm={info['t_assemble']:.3f} t_solve={info['t_solve']:.3f} "
        f"t_transport={info['t_transport']:.3f}")
    for k in ("vp", "phi", "B"):
        assert bool(torch.isfinite(st[k]).all()), k
    assert float(st["phi"].abs().max()) <= 1.01
    R = ctx.assemble(ctx.device_state(prob.state_copy()), {k: st[k] for k in ("vp", "phi", "B")})
    x, si = ctx.fgmres(-R)
    r = -R - ctx.spmv(x)
    rr = float(torch.linalg.norm(r) / torch.linalg.norm(R))
    say(f"  final solve iters={si['iters']} rel_res={rr:.2e}")
    assert si["converged"] == 1 and rr <= prob.params.lin_rtol * 1.0001
    ctx.close()
