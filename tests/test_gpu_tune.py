"""The autotuner (eft_tune): it times candidates of the solver's run-time
knobs on the caller's state, keeps the fastest, leaves the state and the
definition parameters alone, and a second context of the same configuration
reads its choice back from the cache file.  Tuned and default knobs reach
the same time step (the knobs change only the preconditioner)."""
import sys

import numpy as np
import pytest

from paper_2402_10348_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_tune_keeps_answer_and_caches(tmp_path):
    import torch
    from paper_2402_10348_amd.eft import Context
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    prob = W.cavity_sphere_3d(n=16)
    say(f"[tune] cavity 16^3 N={prob.n_nodes}")
    over = dict(nl_fixed=2, lin_rtol=1e-12, restart=80, lin_maxit=20000)
    ref = Context(prob, **over)
    s0 = ref.device_state(prob.state_copy())
    ref.step(s0)
    ctx = Context(prob, **over)
    st = ctx.device_state(prob.state_copy())
    before = {k: v.cpu().numpy().copy() for k, v in st.items()}
    cache = str(tmp_path / "tune.txt")
    info = ctx.tune(st, cache_path=cache, budget=12)
    say(f"  {info}")
    assert info["from_cache"] == 0 and info["evaluated"] >= 2
    assert info["best_seconds"] <= info["default_seconds"] * 1.5
    for k, v in st.items():
        assert np.array_equal(v.cpu().numpy(), before[k]), k
    ctx.step(st)
    for k in ("vp", "phi", "B"):
        a, b = st[k].cpu().numpy(), s0[k].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b), k
    c2 = Context(prob, **over)
    st2 = c2.device_state(prob.state_copy())
    info2 = c2.tune(st2, cache_path=cache)
    assert info2["from_cache"] == 1
    for k in ("mg_nu", "mg_nu_post", "mg_smoother", "band_sweeps"):
        assert info2[k] == info[k], k
    assert abs(info2["mg_omega"] - info["mg_omega"]) < 1e-12
    assert abs(info2["band_omega"] - info["band_omega"]) < 1e-12
    for c in (ref, ctx, c2):
        c.close()
