"""The allocation-free FGMRES entry point (eft_fgmres_noalloc) against
eft_fgmres, through the C ABI, on two calls in a row: a 3D cavity system
first, then a smaller 2D one, so the second call runs in the fixed workspace
the first one left filled.  Both solves run the same kernels in the same
order on the same matrix, so the answers agree to the FP64 parity bar
(1e-10 relative; in practice bit for bit), with the same iteration counts.
"""
import sys

import numpy as np
import pytest

from paper_2402_10348_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solve_pair(prob, seed, **over):
    import torch
    from paper_2402_10348_amd.eft import Context
    lvl, it = W.perturbed_state(prob, seed=seed)
    ctx = Context(prob, **over)
    R = ctx.assemble(ctx.device_state(lvl), ctx.device_state(it))
    b = -R
    x_ref, info_ref = ctx.fgmres(b)
    x_na, info_na = ctx.fgmres_noalloc(b)
    torch.cuda.synchronize()
    a, r = x_na.cpu().numpy(), x_ref.cpu().numpy()
    ctx.close()
    return a, r, info_na, info_ref


@pytest.mark.parametrize("precond", [0, 1])
def test_noalloc_fgmres_matches_fgmres_twice(precond):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cases = [("sphere3d_8", W.cavity_sphere_3d(n=8), 31), ("disk2d_16", W.cavity_disk_2d(n=16), 32)]
    for name, prob, seed in cases:
        say(f"[noalloc fgmres] case={name} precond={precond} N={prob.n_nodes} seed={seed}")
        a, r, ina, iref = _solve_pair(prob, seed, precond=precond, lin_rtol=1e-12, restart=60, lin_maxit=6000)
        err = float(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300))
        say(f"  iters {ina['iters']} vs {iref['iters']}, rel diff {err:.2e}")
        assert ina["converged"] == 1 and iref["converged"] == 1
        assert ina["iters"] == iref["iters"]
        assert err <= 1e-10


def test_noalloc_fgmres_rejects_oversized_system():
    """A system past the fixed workspace's limit returns EFT_EINVAL with a
    message (nothing is launched for it)."""
    import torch
    from paper_2402_10348_amd.eft import Context, EftError, EINVAL
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    prob = W.cavity_sphere_3d(n=40)   # 68,921 nodes x 4 dofs x (2*50 + 3) > 8 Mi doubles
    say(f"[noalloc fgmres] oversized N={prob.n_nodes}")
    ctx = Context(prob, restart=50)
    b = torch.zeros((prob.n_nodes, 4), dtype=torch.float64, device=ctx.dev)
    with pytest.raises(EftError) as ei:
        ctx.fgmres_noalloc(b)
    assert ei.value.status == EINVAL and "too large" in str(ei.value)
    ctx.close()
