#!/usr/bin/env python3
"""Throughput of the hot path on one MI355X: converged time steps per second
of the 3D lid-driven cavity with one elastic sphere (64^3 cells split into
1,572,864 P1 tets, 274,625 nodes, 4 dof per node), every time step running
the partitioned nonlinear iteration (momentum/mass assembly + FGMRES,
Allen-Cahn and B band transport) to the stop rule ||dx||/||x|| < 5e-4 with
linear solves to 1e-8 relative residual.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  The line carries
  roofline      the fine-level multigrid smoother sweep (the kernel with the
                largest share of the step), every launch in the timed steps
                bracketed by HIP events on the library's stream: algorithmic
                bytes / summed launch time, vs the 8 TB/s HBM peak; traffic
                is the rocprofv3-measured HBM bytes per launch when the
                kernel's sources match the ones profiled;
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the same
                workload on the host cores (see --no-cpu).
Inputs are seeded and synthetic and resident in device memory before the
timed region starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="cells per axis of the cavity (64 = the benchmark)")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64, 1 FP32 Jacobian values")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--precond", type=int, default=1, help="1 multigrid V-cycle, 0 point-block Jacobi")
    ap.add_argument("--mg-nu", type=int, default=1, help="multigrid pre-smoothing sweeps (the first from zero)")
    ap.add_argument("--mg-nu-post", type=int, default=3, help="multigrid post-smoothing sweeps")
    ap.add_argument("--mg-smoother", type=int, default=0, help="0 damped block Jacobi, 1 multicolour block Gauss-Seidel")
    ap.add_argument("--band-sweeps", type=int, default=None,
                    help="damped block-Jacobi sweeps preconditioning the Allen-Cahn and B systems")
    ap.add_argument("--band-omega", type=float, default=None)
    ap.add_argument("--mg-omega", type=float, default=0.75)
    ap.add_argument("--mg-bf16", type=int, default=1, help="1: finest multigrid level's matrix copy in BF16, 0: FP32")
    ap.add_argument("--kernel-role", type=int, default=1,
                    help="kernel of the roofline object: 1 fine-level smoother sweep, 2 momentum SpMV in FGMRES, "
                         "3 assembly (all three are timed with HIP events over the timed steps); 0 no timing")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the mixed-precision (FP32 Jacobian) run of the same steps")
    ap.add_argument("--no-learned", dest="learned", action="store_false",
                    help="skip the learned-vs-plain preconditioner comparison")
    ap.add_argument("--learned-n", type=int, default=32)
    ap.add_argument("--learned-pairs", type=int, default=256)
    ap.add_argument("--learned-train", type=int, default=400)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB copied by a plain device copy before the timed steps (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-full-domain", dest="full_domain", action="store_false",
                    help="skip the paper-literal variants (full-domain transport, background indicator)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


KERNEL_NAME_FP32 = ("k_sweep_blk<4, float, float> (finest-level multigrid smoother sweep, FP32 copy of the "
                    "4x4-block momentum Jacobian, one block per lane)")


def band_over(args):
    """Band-system preconditioner settings given on the command line."""
    o = {}
    if args.band_sweeps is not None:
        o["band_sweeps"] = args.band_sweeps
    if args.band_omega is not None:
        o["band_omega"] = args.band_omega
    return o


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


KERNEL_NAME = {1: "k_sweep_blk<4, eft_bf16, float> (finest-level multigrid smoother sweep, BF16 copy of the "
                  "4x4-block momentum Jacobian, FP32 block inverses, FP64 vectors and arithmetic, one block per lane)",
               2: "k_spmv_rows<4, double, true> (FP64 SpMV of the 4x4-block momentum Jacobian in FGMRES)",
               3: "k_ns_rows<3, double> (momentum/mass residual and Jacobian assembly, bytes: J, its BF16 or "
                  "FP32 copy for the multigrid and R written once, connectivity and node fields read once)"}


def timed_steps(ctx, st, steps, warmup, torch):
    t_sim, step_no = 0.0, 0
    for _ in range(warmup):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(steps):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        its.append(info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, its


def run_learned(args, torch):
    """Learned vs plain preconditioner at 1e-8 on the n^3 cavity (default
    32^3, where block Jacobi still converges): the plain FP64 step with
    point-block Jacobi against the mixed-precision step with the learned
    preconditioner, trained in this run on pairs harvested from the plain
    run's own momentum solves (training time reported apart)."""
    from paper_2402_10348_amd import workloads as W
    from paper_2402_10348_amd.eft import Context
    prob = W.cavity_sphere_3d(n=args.learned_n)
    common = dict(lin_rtol=1e-8, restart=100, lin_maxit=20000)
    plain = Context(prob, precond=0, precision=0, **common)
    plain.nn_init(seed=7)
    plain.nn_harvest(args.learned_pairs)
    st = plain.device_state(prob.state_copy())
    el0, its0 = timed_steps(plain, st, args.steps, args.warmup, torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = plain.nn_train(steps=args.learned_train, batch=4, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    theta = plain.nn_params()
    plain.close()
    learned = Context(prob, precond=2, precision=1, **common)
    learned.nn_init(seed=7)
    learned.nn_params(theta)
    st = learned.device_state(prob.state_copy())
    el1, its1 = timed_steps(learned, st, args.steps, args.warmup, torch)
    learned.close()

    def line(el, its):
        return dict(steps_per_s=round(args.steps / el, 4), ms_per_step=round(1e3 * el / args.steps, 2),
                    nl_iters_per_step=sum(i["nl_iters"] for i in its) / len(its),
                    momentum_krylov_iters_per_step=sum(i["lin_iters_block"][0] for i in its) / len(its))
    return dict(workload=f"3D cavity with elastic sphere, {args.learned_n}^3 x 6 P1 tets, FGMRES(100) to 1e-8",
                plain=dict(precond="point-block Jacobi", dtype="f64", **line(el0, its0)),
                learned=dict(precond="learned (block Jacobi + network)", dtype="f64 residual/Krylov, f32 Jacobian",
                             **line(el1, its1)),
                training=dict(pairs=args.learned_pairs, adam_steps=args.learned_train, seconds=round(t_train, 3),
                              loss_first=float(losses[:10].mean()), loss_last=float(losses[-10:].mean())),
                speedup=round(el0 / el1, 4))


def diagnostics(ctx, st, prob):
    """Wall time per call of the solid diagnostics on the final state: the
    centre of mass of every indicator's region (Sec. 3) and one particle
    tracking step (Appendix) of 16 particles around the sphere's centre."""
    import numpy as np
    reps = 20
    ctx.center_of_mass(st["phi"])
    t0 = time.perf_counter()
    for _ in range(reps):
        xc, m = ctx.center_of_mass(st["phi"])
    t_com = (time.perf_counter() - t0) / reps
    rng = np.random.Generator(np.random.PCG64(0))
    pts = 0.5 + rng.uniform(-0.15, 0.15, (16, prob.dim))
    ctx.track_particles(st["vp"], pts, prob.params.dt)
    t0 = time.perf_counter()
    for _ in range(reps):
        pts, el = ctx.track_particles(st["vp"], pts, prob.params.dt)
    t_pt = (time.perf_counter() - t0) / reps
    # order parameter of a triangulated sphere (r = 1/4, 20,480 triangles)
    # on the 64^3 mesh, 8^3 grid cells, against tanh of the exact distance;
    # the centre is moved off the mesh planes by fractions of a cell so that
    # no +X ray is tangent to the sphere at a vertex (such a ray counts as a
    # crossing in the method)
    from paper_2402_10348_amd import workloads as W
    ctr = np.array([0.5 + 1.0 / 192, 0.5 + 1.0 / 320, 0.5 + 1.0 / 448])
    v, t = W.icosphere(0.25, ctr, 5)
    eps = 1.5 / 64
    ctx.init_phase(v, t, eps, [8, 8, 8])
    torch = ctx.torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        phi, cr = ctx.init_phase(v, t, eps, [8, 8, 8])
    t_init = (time.perf_counter() - t0) / 5
    d = 0.25 - np.linalg.norm(prob.xyz - ctr, axis=1)
    ref = np.tanh(d / (np.sqrt(2.0) * eps))
    e2 = float(np.linalg.norm(phi.cpu().numpy() - ref) / np.linalg.norm(ref))
    return dict(center_of_mass_us=round(1e6 * t_com, 1), sphere_center=[round(float(v_), 6) for v_ in xc[0]],
                sphere_measure=float(m[0]), track_particles_us=round(1e6 * t_pt, 1), n_particles=16,
                particles_found=int((el >= 0).sum()),
                init_phase=dict(ms=round(1e3 * t_init, 3), triangles=int(t.shape[0]), grid_cells=[8, 8, 8],
                                rel_l2_error_vs_exact_sdf=e2, most_crossings=int(cr[0])))


def run_variant(args, prob, torch, **over):
    """The bench's warmup and timed steps on a variant of the workload;
    returns the timing line and the final fields."""
    import numpy as np
    from paper_2402_10348_amd.eft import Context
    ctx = Context(prob, lin_rtol=1e-8, restart=args.restart, lin_maxit=20000, precision=args.precision,
                  precond=args.precond, mg_nu=args.mg_nu, mg_omega=args.mg_omega, mg_bf16=args.mg_bf16,
                  mg_nu_post=args.mg_nu_post, mg_smoother=args.mg_smoother, **dict(band_over(args), **over))
    st = ctx.device_state(prob.state_copy())
    t_sim, step_no = 0.0, 0
    for _ in range(args.warmup):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(args.steps):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        its.append(info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fin = {k: st[k].cpu().numpy() for k in ("vp", "phi", "B")}
    ctx.close()
    line = dict(value=round(args.steps / el, 4), unit="steps/s", ms_per_step=round(1e3 * el / args.steps, 2),
                transport_ms_per_step=round(1e3 * float(np.mean([i["t_transport"] for i in its])), 2),
                nl_iters_per_step=float(np.mean([i["nl_iters"] for i in its])),
                krylov_iters_per_step_by_block=[float(v) for v in np.mean([i["lin_iters_block"] for i in its],
                                                                          axis=0)])
    return line, fin


def run_full_domain(args, prob, torch, band_final):
    """The same steps with the transport on the whole mesh (band_flat < 0:
    no band), and the band's truncation: the relative difference of the
    final fields of the banded and the full-domain runs."""
    import numpy as np
    line, fin = run_variant(args, prob, torch, band_flat=-1.0)
    line["band_truncation_rel"] = {k: float(np.linalg.norm(band_final[k] - fin[k]) /
                                            max(np.linalg.norm(fin[k]), 1e-300)) for k in fin}
    return line


def run_background(args, prob, torch):
    """The same steps with one transported order parameter per phase, the
    background fluid included (two Allen-Cahn systems instead of one)."""
    from paper_2402_10348_amd import workloads as W
    pb = W.with_background_indicator(prob)
    line, _ = run_variant(args, pb, torch)
    line["indicators"] = pb.n_ind
    return line


def run_mixed(args, prob, torch):
    """The same steps with the mixed path: the momentum Jacobian assembled,
    stored and applied in FP32 inside the FP64 Newton/Krylov iteration."""
    from paper_2402_10348_amd.eft import Context
    ctx = Context(prob, lin_rtol=1e-8, restart=args.restart, lin_maxit=20000, precision=1, precond=args.precond,
                  mg_nu=args.mg_nu, mg_omega=args.mg_omega, mg_nu_post=args.mg_nu_post,
                  mg_smoother=args.mg_smoother, **band_over(args))
    st = ctx.device_state(prob.state_copy())
    t_sim, step_no = 0.0, 0
    for _ in range(args.warmup):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(args.steps):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        its.append(info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    return dict(value=round(args.steps / el, 4), unit="steps/s", ms_per_step=round(1e3 * el / args.steps, 2),
                dtype="f64 residual/Krylov, f32 Jacobian",
                nl_iters_per_step=sum(i["nl_iters"] for i in its) / len(its),
                krylov_iters_per_step=sum(i["lin_iters_total"] for i in its) / len(its))

# HBM bytes per launch of the fine-level sweep from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters, with the hash of the kernel's sources when they were
# taken: a changed kernel has no measured traffic.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_blk_cavity64_hbm_traffic.md")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2402_10348_amd", "csrc", f) for f in ("bsr_rows.h", "k_mg.hip")]


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of the fine-level sweep from the committed counter
    summary, if it was taken on this kernel variant and these sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    if kv.get("sources_sha256") != sources_hash() or not kernel.startswith(kv.get("kernel", "?") + " "):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calib_copy(torch, mib):
    """A plain device-to-device copy of known size (mib MiB read, mib MiB
    written), three times: the reference dispatches for scaling the HBM
    counters of a profiled run."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def cpu_baseline(prob, counts, args):
    """Time the FP64 CPU oracle on the host on a bounded sample of the
    benchmark step, then scale to steps/s with the GPU run's per-step counts.

    The sample, all on the full 64^3 workload at its initial state with the
    step's predictor: one momentum/mass assembly, the band of every indicator
    with its mobility and Lagrange multiplier, one Allen-Cahn assembly, one B
    assembly per solid, and ``its`` FGMRES iterations of each of these three
    systems (the oracle's point-block Jacobi preconditioner).  One step of the
    oracle is then  nl * (assemblies) + sum_block K_block * (time per Krylov
    iteration of that block)  with nl and K_block the GPU's mean nonlinear and
    Krylov iterations per step.  The oracle's preconditioner needs far more
    iterations than the GPU's multigrid, so the CPU figure is optimistic."""
    import numpy as np

    import oracle as O
    nl, kblk = counts
    c = O.Case(prob)
    st = prob.state_copy()
    dim, dt, ri = prob.dim, prob.params.dt, prob.params.rho_inf
    it = dict(vp=st["vp"].copy(), phi=st["phi"].copy(), B=st["B"].copy())
    its = 40   # Krylov iterations sampled per block (about 10-15 s of oracle work in all)
    tm = {}

    def timed(key, fn, *a, **kw):
        t0 = time.perf_counter()
        out = fn(*a, **kw)
        tm[key] = tm.get(key, 0.0) + time.perf_counter() - t0
        return out

    R, J = timed("ns_asm", c.ns_assemble, st, it)
    _, inf = timed("ns_kry", c.fgmres, J, -R.ravel(), rtol=1e-30, restart=its, maxit=its)
    t_ns_it = tm["ns_kry"] / max(inf["iters"], 1)
    del J
    va, _ = O.level_values(ri, dt, st["vp"][:, :dim], st["vdot"], it["vp"][:, :dim])
    n_ind = st["phi"].shape[0]
    t_blk = [t_ns_it]
    t_tr_asm = 0.0
    bands = []
    for k in range(n_ind):
        t0 = time.perf_counter()
        be, fr = c.band(st["phi"][k])
        fa, fd = O.level_values(ri, dt, st["phi"][k], st["phidot"][k], it["phi"][k])
        g = c.mobility(va, fa)
        b = c.beta(fa, be)
        R, J = c.ac_assemble(va, fa, fd, g, b, be, fr)
        t_tr_asm += time.perf_counter() - t0
        bands.append((be, fr))
        t0 = time.perf_counter()
        _, inf = c.fgmres(J, -R, rtol=1e-30, restart=its, maxit=its)
        t_blk.append((time.perf_counter() - t0) / max(inf["iters"], 1))
    fa_all, _ = O.level_values(ri, dt, st["phi"], st["phidot"], it["phi"])
    af, _, _ = c.nodal_properties(fa_all)
    s = 0
    for ph_i, ph in enumerate(prob.phases):
        if ph.kind != 1:
            continue
        k = sum(1 for p in prob.phases[:ph_i] if p.transported)
        t0 = time.perf_counter()
        Ba, Bd = O.level_values(ri, dt, st["B"][s], st["Bdot"][s], it["B"][s])
        R, J = c.b_assemble(va, af[ph_i], Ba, Bd, bands[k][0], bands[k][1])
        t_tr_asm += time.perf_counter() - t0
        t0 = time.perf_counter()
        _, inf = c.fgmres(J, -R.ravel(), rtol=1e-30, restart=its, maxit=its)
        t_blk.append((time.perf_counter() - t0) / max(inf["iters"], 1))
        s += 1
    t_step = nl * (tm["ns_asm"] + t_tr_asm) + sum(k * t for k, t in zip(kblk, t_blk))
    sample_s = tm["ns_asm"] + tm["ns_kry"] + t_tr_asm + sum(t_blk[1:]) * its
    return dict(value=1.0 / t_step, unit="steps/s", cores=1, kind="oracle",
                sample=(f"{prob.n_nodes}-node 64^3 cavity, one host core, {sample_s:.1f} s of oracle work: "
                        f"momentum/mass assembly {tm['ns_asm']:.2f} s, band + Allen-Cahn + B assembly "
                        f"{t_tr_asm:.2f} s, Krylov iteration (ms) per block "
                        + "/".join(f"{1e3 * t:.0f}" for t in t_blk)
                        + f"; scaled by the GPU's {nl:.2f} nonlinear and "
                        + "/".join(f"{k:.0f}" for k in kblk) + " Krylov iterations per step"))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the multi-GPU sharding is a "
              "design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2402_10348_amd import workloads as W
    from paper_2402_10348_amd.eft import Context

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    prob = W.cavity_sphere_3d(n=args.n)
    ctx = Context(prob, lin_rtol=1e-8, restart=args.restart, lin_maxit=20000, precision=args.precision,
                  precond=args.precond, mg_nu=args.mg_nu, mg_omega=args.mg_omega, mg_bf16=args.mg_bf16,
                  mg_nu_post=args.mg_nu_post, mg_smoother=args.mg_smoother, **band_over(args))
    st = ctx.device_state(prob.state_copy())
    log(args, f"[bench] {args.n}^3 cavity N={prob.n_nodes} E={prob.n_elems} precision={args.precision}")
    t_sim, step_no = 0.0, 0
    for w in range(args.warmup):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        log(args, f"[bench] warmup {w}: nl={info['nl_iters']} lin={info['lin_iters_total']}")
    if args.calib_copy:
        calib_copy(torch, args.calib_copy)
    if args.kernel_role:
        ctx.time_kernel(1, 2, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, info in enumerate(infos):
        log(args, f"[bench] step {i}: nl={info['nl_iters']} lin={info['lin_iters_total']} conv={info['converged']} "
                  f"asm={info['t_assemble']:.3f}s solve={info['t_solve']:.3f}s transport={info['t_transport']:.3f}s")
    value = args.steps / elapsed
    nl_mean = float(np.mean([i["nl_iters"] for i in infos]))
    lin_mean = float(np.mean([i["lin_iters_total"] for i in infos]))
    kblk = [float(v) for v in np.mean([i["lin_iters_block"] for i in infos], axis=0)]

    kts = {r: ctx.kernel_time(r) for r in (1, 2, 3)} if args.kernel_role else {}
    final = {k: st[k].cpu().numpy() for k in ("vp", "phi", "B")} if args.full_domain else None
    diag = diagnostics(ctx, st, prob)
    ctx.close()

    def hbm(role, traffic=None):
        kt = kts.get(role)
        if not kt or kt["launches"] == 0 or kt["seconds"] <= 0:
            return None
        achieved = kt["bytes"] / kt["seconds"] / 1e9
        return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=(KERNEL_NAME_FP32 if role == 1 and not args.mg_bf16 else KERNEL_NAME[role]),
                    launches=kt["launches"], active_launches=kt["active"],
                    bytes_per_launch=round(kt["bytes"] / kt["launches"]), mean_launch_s=kt["seconds"] / kt["launches"])

    roofline = None
    if args.kernel_role:
        kname = KERNEL_NAME_FP32 if args.kernel_role == 1 and not args.mg_bf16 else KERNEL_NAME[args.kernel_role]
        roofline = hbm(args.kernel_role, measured_traffic(kname) if args.kernel_role == 1 else None)
    others = {name: hbm(r) for name, r in (("spmv", 2), ("assembly", 3)) if args.kernel_role and r != args.kernel_role}

    mixed = None
    if args.mixed:
        mixed = run_mixed(args, prob, torch)
    full = background = None
    if args.full_domain:
        full = run_full_domain(args, prob, torch, final)
        background = run_background(args, prob, torch)
    learned = None
    if args.learned:
        log(args, "[bench] learned vs plain preconditioner ...")
        learned = run_learned(args, torch)
    cpu = None
    if not args.no_cpu:
        log(args, "[bench] timing the CPU oracle sample ...")
        cpu = cpu_baseline(prob, (nl_mean, kblk), args)

    line = {
        "metric": "converged time steps/s (3D cavity, elastic sphere, FP64, FGMRES to 1e-8)",
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64+f32J",
        "data": "synthetic (seeded cavity, tanh sphere indicator, B = I, v = 0 at t = 0)",
        "config": {"workload": f"3D lid-driven cavity with one elastic sphere, {args.n}^3 x 6 P1 tets",
                   "n_nodes": prob.n_nodes, "n_elems": prob.n_elems, "dt": prob.params.dt,
                   "lin_rtol": 1e-8, "restart": args.restart, "nl_rtol": prob.params.nl_rtol,
                   "nl_iters_per_step": nl_mean, "krylov_iters_per_step": lin_mean,
                   "krylov_iters_per_step_by_block": kblk,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": others,
        "mixed_precision": mixed,
        "full_domain_transport": full,
        "diagnostics": diag,
        "background_indicator": background,
        "learned_vs_plain_precond": learned,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
