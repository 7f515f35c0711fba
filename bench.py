#!/usr/bin/env python3
"""Throughput of the hot path on one MI355X: converged time steps per second
of the largest single-GPU workload, the hull among 16 ice floes in an
air-water box (256 x 128 x 64 cells split into 12,582,912 P1 tets, 2,154,945
nodes, 4 dof per node, 18 transported indicators, 17 solids).  Every time
step runs the partitioned nonlinear iteration (momentum/mass assembly +
FGMRES, Allen-Cahn and B band transport of every indicator and solid) to the
stop rule ||dx||/||x|| < 5e-4 on every block, at most 20 iterations, with
linear solves to 1e-8 relative residual; only steps that meet the stop rule
count.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Beside the headline it carries
  roofline      the assembly + SpMV pair of the momentum/mass system (the
                pair whose HBM fraction the method's target names): summed
                algorithmic bytes / summed launch time of every assembly and
                every FGMRES SpMV launch in --kernel-steps further steps after
                the timed ones, each bracketed by HIP events on the library's
                stream, vs the 8 TB/s HBM peak;
                traffic = the rocprofv3-counted HBM bytes of those launches
                (per-launch counter figures of profiles/, when the kernels'
                sources match the ones profiled);
  kernels       the same per kernel (assembly, SpMV, finest multigrid sweep);
  secondary     the 128^3 and 64^3 cavities with the elastic sphere;
  cpu_baseline  the FP64 CPU oracle (OpenMP timing copy) on a bounded sample
                of the headline workload, on all host threads and on one.
Inputs are seeded and synthetic and resident in device memory before the
timed region starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
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
    ap.add_argument("--workload", default="floes", choices=["floes", "cavity128", "cavity64"],
                    help="headline workload (floes = the hull among 16 floes, 256x128x64)")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64, 1 FP32 Jacobian values")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--precond", type=int, default=1, help="1 multigrid V-cycle, 0 point-block Jacobi")
    ap.add_argument("--mg-nu", type=int, default=1, help="multigrid pre-smoothing sweeps (the first from zero)")
    ap.add_argument("--mg-nu-post", type=int, default=3, help="multigrid post-smoothing sweeps")
    ap.add_argument("--mg-smoother", type=int, default=0, help="0 damped block Jacobi, 1 multicolour block Gauss-Seidel")
    ap.add_argument("--mg-omega", type=float, default=0.85,
                    help="multigrid damping before tuning (the tuner searches 0.65-0.95)")
    ap.add_argument("--mg-bf16", type=int, default=1, help="1: finest multigrid level's matrix copy in BF16, 0: FP32")
    ap.add_argument("--band-sweeps", type=int, default=None,
                    help="damped block-Jacobi sweeps preconditioning the Allen-Cahn and B systems")
    ap.add_argument("--band-omega", type=float, default=None)
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="keep the default solver knobs (no autotuning before the warmup)")
    ap.add_argument("--no-secondary", dest="secondary", action="store_false",
                    help="skip the 128^3 and 64^3 cavity lines")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the mixed-precision (FP32 Jacobian) run of the headline steps")
    ap.add_argument("--no-learned", dest="learned", action="store_false",
                    help="skip the learned-vs-plain preconditioner comparison")
    ap.add_argument("--learned-n", type=int, default=32)
    ap.add_argument("--learned-pairs", type=int, default=1024)
    ap.add_argument("--learned-train", type=int, default=400)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB copied by a plain device copy before the timed steps (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the paper-literal variants and diagnostics (64^3 cavity)")
    ap.add_argument("--graphs", type=int, default=1, help="1: momentum Krylov columns replayed as HIP graphs")
    ap.add_argument("--mg-lag", type=int, default=1,
                    help="1: coarse multigrid levels refreshed at the first nonlinear iteration of a step only, "
                         "0: at every nonlinear iteration")
    ap.add_argument("--kernel-steps", type=int, default=2,
                    help="steps after the timed ones with per-launch HIP-event timing of the roofline kernels")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


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


def make_workload(name):
    from paper_2402_10348_amd import workloads as W
    if name == "floes":
        p = W.floe_field_3d()
        return p, "hull among 16 ice floes in an air-water box, 256x128x64 x 6 P1 tets, 18 indicators, 17 solids"
    n = 128 if name == "cavity128" else 64
    p = W.cavity_sphere_3d(n=n)
    return p, f"3D lid-driven cavity with one elastic sphere, {n}^3 x 6 P1 tets"


KERNEL_NAME = {1: "k_sweep_blk<4, eft_bf16, eft_bf16, true, float, float> (finest-level multigrid smoother sweep: "
                  "BF16 copy of the 4x4-block momentum Jacobian with its pattern in stencil form (row masks, no "
                  "column indices), BF16 block inverses, FP32 iterate, FP64 right-hand side and arithmetic)",
               2: "k_spmv_stn<4, true> (FP64 SpMV of the 4x4-block momentum Jacobian in FGMRES, pattern in "
                  "stencil form)",
               3: "k_ns_rows<3, double, true> (momentum/mass residual and Jacobian assembly with the node records "
                  "staged per workgroup: J, its BF16 copy for the multigrid and R written once, connectivity and "
                  "node fields read once)"}
KERNEL_KEY = {1: "k_sweep_blk", 2: "k_spmv_stn", 3: "k_ns_rows"}
# sources each kernel's counter figures were taken on
KERNEL_SOURCES = {1: ("bsr_rows.h", "k_mg.hip"), 2: ("bsr_rows.h", "k_sparse.hip"),
                  3: ("k_assemble.hip", "dev_common.h")}


def sources_hash(role):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[role]:
        h.update(open(os.path.join(ROOT, "paper_2402_10348_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(role, workload):
    """HBM bytes per launch of a kernel from the committed counter summary
    profiles/<kernel>_<workload>_hbm_traffic.md, if it was taken on these
    sources."""
    path = os.path.join(ROOT, "profiles", f"{KERNEL_KEY[role]}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    if kv.get("sources_sha256") != sources_hash(role):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_steps(args, prob, torch, label, time_kernels=True, **over):
    """Warmup and timed steps of one workload; converged steps per second,
    the per-step counts and the kernel timings of the timed steps."""
    import numpy as np
    from paper_2402_10348_amd.eft import Context
    kw = dict(lin_rtol=1e-8, restart=args.restart, lin_maxit=20000, precision=args.precision,
              precond=args.precond, mg_nu=args.mg_nu, mg_omega=args.mg_omega, mg_bf16=args.mg_bf16,
              mg_nu_post=args.mg_nu_post, mg_smoother=args.mg_smoother, nl_max=20, graphs=args.graphs,
              mg_lag=args.mg_lag)
    kw.update(band_over(args))
    kw.update(over)
    t0 = time.perf_counter()
    ctx = Context(prob, **kw)
    st = ctx.device_state(prob.state_copy())
    torch.cuda.synchronize()
    log(args, f"[bench] {label}: N={prob.n_nodes} E={prob.n_elems} set-up {time.perf_counter() - t0:.1f}s")
    tune = None
    if args.tune:
        t0 = time.perf_counter()
        tune = ctx.tune(st)
        tune["seconds"] = round(time.perf_counter() - t0, 2)
        log(args, f"[bench] {label} tuned in {tune['seconds']}s: {tune}")
    t_sim, step_no = 0.0, 0
    for w in range(args.warmup):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        log(args, f"[bench] {label} warmup {w}: nl={info['nl_iters']} conv={info['converged']} "
                  f"lin={info['lin_iters_block'][:3]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no = info["t"], info["step"]
        infos.append(info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for i, info in enumerate(infos):
        log(args, f"[bench] {label} step {i}: nl={info['nl_iters']} conv={info['converged']} "
                  f"lin={info['lin_iters_block'][:3]} asm={info['t_assemble']:.3f}s solve={info['t_solve']:.3f}s "
                  f"transport={info['t_transport']:.3f}s")
    kts = {}
    if time_kernels and args.kernel_steps > 0:
        # the kernel timings: further steps, each launch of the timed roles
        # bracketed by HIP events (which also keeps the momentum columns out
        # of HIP graphs, so these steps are not part of the headline)
        ctx.time_kernel(1, 2, 3)
        for _ in range(args.kernel_steps):
            info = ctx.step(st, t=t_sim, step=step_no)
            t_sim, step_no = info["t"], info["step"]
        torch.cuda.synchronize()
        kts = {r: ctx.kernel_time(r) for r in (1, 2, 3)}
        ctx.time_kernel()
    conv = sum(1 for i in infos if i["converged"])
    out = dict(value=round(conv / el, 4), unit="steps/s", ms_per_step=round(1e3 * el / args.steps, 2),
               converged_steps=conv, nonconverged_steps=args.steps - conv,
               nl_iters_per_step=float(np.mean([i["nl_iters"] for i in infos])),
               krylov_iters_per_step_by_block=[round(float(v), 2) for v in
                                               np.mean([i["lin_iters_block"] for i in infos], axis=0)],
               transport_ms_per_step=round(1e3 * float(np.mean([i["t_transport"] for i in infos])), 2))
    if tune is not None:
        out["tuning"] = dict(seconds=tune["seconds"], candidates=tune["evaluated"],
                             momentum_solve_s_default=round(tune["default_seconds"], 5),
                             momentum_solve_s_tuned=round(tune["best_seconds"], 5),
                             momentum_iters_default=tune["default_iters"], momentum_iters_tuned=tune["best_iters"],
                             transport_s_default=round(tune["band_default_seconds"], 5),
                             transport_s_tuned=round(tune["band_best_seconds"], 5),
                             knobs={k: tune[k] for k in ("mg_nu", "mg_nu_post", "mg_smoother", "mg_omega",
                                                         "mg_galerkin", "mg_cnu", "mg_cnu_post", "band_sweeps",
                                                         "band_omega")})
    return out, kts, ctx, st, el


def kernel_line(kts, role, workload):
    kt = kts.get(role)
    if not kt or kt["launches"] == 0 or kt["seconds"] <= 0:
        return None
    achieved = kt["bytes"] / kt["seconds"] / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(role, workload),
                kernel=KERNEL_NAME[role], launches=kt["launches"], active_launches=kt["active"],
                bytes_per_launch=round(kt["bytes"] / max(kt["active"], 1)),
                mean_launch_s=kt["seconds"] / kt["launches"])


def pair_line(kts, workload):
    """Assembly + SpMV of the momentum/mass system over the kernel-timing steps."""
    a, s = kts.get(3), kts.get(2)
    if not a or not s or a["seconds"] <= 0 or s["seconds"] <= 0:
        return None
    byt = a["bytes"] + s["bytes"]
    sec = a["seconds"] + s["seconds"]
    achieved = byt / sec / 1e9
    ta, ts = measured_traffic(3, workload), measured_traffic(2, workload)
    traffic = None
    if ta is not None and ts is not None:
        traffic = round(ta * a["active"] + ts * s["active"])
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel="k_ns_rows + k_spmv_stn (assembly and FGMRES SpMV of the momentum/mass system, FP64)",
                traffic_unit="HBM bytes of all their launches in the kernel-timing steps (rocprofv3 FETCH_SIZE + "
                             "WRITE_SIZE per launch, scaled by a plain copy, times the launches)",
                algorithmic_bytes=round(byt), seconds=round(sec, 6),
                launches={"assembly": a["active"], "spmv": s["active"]})


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
    return time.perf_counter() - t0, its


def harvest_and_train(args, prob, torch, base):
    """Pairs (base of A z_j, z_j) harvested from the plain steps of the n^3
    cavity (multigrid solves for the V-cycle base, point-block Jacobi for
    the block-Jacobi base) until the ring holds --learned-pairs or 40 steps
    ran, then --learned-train Adam steps; (parameters, training record)."""
    from paper_2402_10348_amd.eft import Context
    pc = 1 if base == 1 else 0
    ctx = Context(prob, precond=pc, precision=0, nn_base=base, lin_rtol=1e-8, restart=100, lin_maxit=20000)
    ctx.nn_init(seed=7)
    ctx.nn_harvest(args.learned_pairs)
    st = ctx.device_state(prob.state_copy())
    t_sim, step_no, nsteps = 0.0, 0, 0
    t0 = time.perf_counter()
    while ctx.nn_shape()["pairs"] < args.learned_pairs and nsteps < 40:
        info = ctx.step(st, t=t_sim, step=step_no)
        t_sim, step_no, nsteps = info["t"], info["step"], nsteps + 1
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    pairs = ctx.nn_shape()["pairs"]
    t0 = time.perf_counter()
    losses = ctx.nn_train(steps=args.learned_train, batch=4, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    theta = ctx.nn_params()
    ctx.close()
    return theta, dict(base="multigrid V-cycle" if base == 1 else "point-block Jacobi", pairs=pairs,
                       harvest_steps=nsteps, harvest_seconds=round(t_h, 3), adam_steps=args.learned_train,
                       batch=4, seconds=round(t_train, 3), loss_first=float(losses[:10].mean()),
                       loss_last=float(losses[-10:].mean()))


def run_learned(args, torch):
    """Learned vs plain preconditioner at 1e-8 per converged step.  The
    network is local, so it is trained on the --learned-n cavity (pairs from
    that size's own momentum solves) and its parameters are applied to the
    128^3 cavity (the configuration of the comparison): there the plain
    FP64 step with the multigrid V-cycle (the product's preconditioner)
    against the mixed-precision step with the learned preconditioner on the
    V-cycle.  At the training size the table adds the plain preconditioners
    that judge the learned one (point-block Jacobi, ILU(0)) and the learned
    one on block Jacobi.  The network's forward pass at 128^3 is timed on
    its own (its dense layers are the MFMA work)."""
    import numpy as np
    from paper_2402_10348_amd import workloads as W
    from paper_2402_10348_amd.eft import Context
    common = dict(lin_rtol=1e-8, restart=100, lin_maxit=20000)

    def line(el, its, steps, **kw):
        conv = sum(1 for i in its if i["converged"])
        return dict(converged_steps_per_s=round(conv / el, 4), ms_per_step=round(1e3 * el / steps, 2),
                    nl_iters_per_step=sum(i["nl_iters"] for i in its) / len(its),
                    momentum_krylov_iters_per_step=sum(i["lin_iters_block"][0] for i in its) / len(its), **kw)

    small = W.cavity_sphere_3d(n=args.learned_n)
    log(args, f"[bench] learned: training at {args.learned_n}^3 ...")
    th_mg, tr_mg = harvest_and_train(args, small, torch, 1)
    th_bj, tr_bj = harvest_and_train(args, small, torch, 0)
    table = {}
    for name, kw, theta in (("plain multigrid (f64)", dict(precond=1, precision=0), None),
                            ("plain point-block Jacobi (f64)", dict(precond=0, precision=0), None),
                            ("plain ILU(0) (f64)", dict(precond=3, precision=0), None),
                            ("learned on multigrid (mixed)", dict(precond=2, nn_base=1, precision=1), th_mg),
                            ("learned on block Jacobi (mixed)", dict(precond=2, nn_base=0, precision=1), th_bj)):
        c = Context(small, **common, **kw)
        if theta is not None:
            c.nn_init(seed=7)
            c.nn_params(theta)
        st = c.device_state(small.state_copy())
        el, its = timed_steps(c, st, args.steps, args.warmup, torch)
        c.close()
        table[name] = line(el, its, args.steps)
        log(args, f"[bench] learned {args.learned_n}^3 {name}: {table[name]}")
    big = W.cavity_sphere_3d(n=128)
    out = {}
    for name, kw, theta in (("plain", dict(precond=1, precision=0), None),
                            ("learned", dict(precond=2, nn_base=1, precision=1), th_mg)):
        c = Context(big, **common, **kw)
        if theta is not None:
            c.nn_init(seed=7)
            c.nn_params(theta)
        st = c.device_state(big.state_copy())
        el, its = timed_steps(c, st, args.steps, args.warmup, torch)
        if theta is not None:
            # the network's forward pass alone on a base-sized vector
            u = torch.randn((big.n_nodes, 4), dtype=torch.float64, device="cuda")
            c.nn_apply(u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                c.nn_apply(u)
            torch.cuda.synchronize()
            t_fw = (time.perf_counter() - t0) / 10
            sh = c.nn_shape()
            H, L = sh["hidden"], sh["layers"]
            flop = 2.0 * big.n_nodes * (8 * H + L * 2 * H * H + H * 4)
        c.close()
        out[name] = line(el, its, args.steps)
        log(args, f"[bench] learned 128^3 {name}: {out[name]}")
    return dict(workload="3D cavity with elastic sphere, 128^3 x 6 P1 tets (2,146,689 nodes), FGMRES(100) to 1e-8",
                plain=dict(precond="multigrid V-cycle", dtype="f64", **out["plain"]),
                learned=dict(precond="learned correction of the V-cycle (trained at the small size)",
                             dtype="f64 residual/Krylov, f32 Jacobian", **out["learned"]),
                speedup=round(out["learned"]["converged_steps_per_s"] / max(out["plain"]["converged_steps_per_s"], 1e-12), 4),
                network_forward=dict(seconds=round(t_fw, 6), flop=flop, tflops=round(flop / t_fw / 1e12, 3),
                                     mfma_peak_tflops=2500.0, frac=round(flop / t_fw / 1e12 / 2500.0, 6),
                                     note="dense layers on BF16 MFMA with FP32 accumulation; the pass is bound "
                                          "by the activations' memory traffic, not by the matrix cores"),
                training_size=dict(workload=f"3D cavity with elastic sphere, {args.learned_n}^3", table=table),
                training=[tr_mg, tr_bj])


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



def oracle_sample(prob, its):
    """Time the oracle's pieces of one nonlinear iteration on prob at its
    initial state (after the predictor): the momentum/mass assembly, `its`
    FGMRES iterations of that system, and for indicator 0 and indicator 1 (the
    largest band and a smaller one) the band, mobility, beta and Allen-Cahn
    assembly with `its` iterations, and for solid 0 the B assembly with `its`
    iterations.  Seconds per piece (per Krylov iteration for the solves)."""
    import oracle as O
    c = O.Case(prob)
    st = prob.state_copy()
    dim, dt, ri = prob.dim, prob.params.dt, prob.params.rho_inf
    it = dict(vp=st["vp"].copy(), phi=st["phi"].copy(), B=st["B"].copy())
    for q, n in enumerate(prob.dir_node):
        for i in range(dim + 1):
            if (prob.dir_mask[q] >> i) & 1:
                it["vp"][n, i] = prob.dir_val[q, i]
    out = {}
    t0 = time.perf_counter()
    R, J = c.ns_assemble(st, it)
    out["ns_asm"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, inf = c.fgmres(J, -R.ravel(), rtol=1e-30, restart=its, maxit=its)
    out["ns_it"] = (time.perf_counter() - t0) / max(inf["iters"], 1)
    del J
    va, _ = O.level_values(ri, dt, st["vp"][:, :dim], st["vdot"], it["vp"][:, :dim])
    bands = {}
    for k in range(min(2, st["phi"].shape[0])):
        t0 = time.perf_counter()
        be, fr = c.band(st["phi"][k])
        fa, fd = O.level_values(ri, dt, st["phi"][k], st["phidot"][k], it["phi"][k])
        g = c.mobility(va, fa)
        b = c.beta(fa, be)
        R, J = c.ac_assemble(va, fa, fd, g, b, be, fr)
        out[f"ac_asm{k}"] = time.perf_counter() - t0
        bands[k] = (be, fr)
        t0 = time.perf_counter()
        _, inf = c.fgmres(J, -R, rtol=1e-30, restart=its, maxit=its)
        out[f"ac_it{k}"] = (time.perf_counter() - t0) / max(inf["iters"], 1)
    fa_all, _ = O.level_values(ri, dt, st["phi"], st["phidot"], it["phi"])
    af, _, _ = c.nodal_properties(fa_all)
    solid = [i for i, p in enumerate(prob.phases) if p.kind == 1]
    if solid:
        ph = solid[0]
        k = sum(1 for p in prob.phases[:ph] if p.transported)
        be, fr = bands[k] if k in bands else c.band(st["phi"][k])
        t0 = time.perf_counter()
        Ba, Bd = O.level_values(ri, dt, st["B"][0], st["Bdot"][0], it["B"][0])
        R, J = c.b_assemble(va, af[ph], Ba, Bd, be, fr)
        out["b_asm"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, inf = c.fgmres(J, -R.ravel(), rtol=1e-30, restart=its, maxit=its)
        out["b_it"] = (time.perf_counter() - t0) / max(inf["iters"], 1)
    return out


def oracle_step_seconds(tm, nl, kblk, n_ind, n_s, scale_e=1.0, scale_n=1.0):
    """One oracle time step from the sampled pieces and the GPU run's per-step
    counts: nl nonlinear iterations of (assemblies of every system) plus the
    Krylov iterations of every block; the oracle solves each indicator's and
    each solid's system on its own, so every member pays the union's count.
    Indicators past the first two are charged like the second (the smaller
    band), solids like the first.  scale_e / scale_n scale element- and
    node-proportional pieces from the sampled mesh to the workload's."""
    ac1 = "ac_asm1" if "ac_asm1" in tm else "ac_asm0"
    ai1 = "ac_it1" if "ac_it1" in tm else "ac_it0"
    asm = tm["ns_asm"] + tm["ac_asm0"] + max(n_ind - 1, 0) * tm[ac1] + n_s * tm.get("b_asm", 0.0)
    k_ac = kblk[1] if n_ind > 0 else 0.0
    k_b = kblk[1 + n_ind] if n_s > 0 else 0.0
    kry = (kblk[0] * tm["ns_it"] + k_ac * (tm["ac_it0"] + max(n_ind - 1, 0) * tm[ai1])
           + n_s * k_b * tm.get("b_it", 0.0))
    return scale_e * nl * asm + scale_n * kry


def cpu_baseline(prob, wname, gpu_line, args):
    """The FP64 CPU oracle as it stands, built here as its OpenMP timing copy
    (bit-identical results), on a bounded sample of the headline workload:
    one nonlinear iteration's pieces timed at a quarter of the resolution
    with all host threads (at full size the oracle's dense loop over the 17
    solids per element would take minutes), scaled by the element and node
    counts to the full mesh and to a converged step with the GPU run's
    nonlinear and Krylov counts (the oracle's point-block Jacobi needs far
    more Krylov iterations than the GPU's multigrid, and small vectors stay
    in the host caches, so the CPU figure flatters the CPU); the same pieces
    on one thread at an eighth of the resolution give the 1-thread figure."""
    import oracle as O
    from paper_2402_10348_amd import workloads as W
    its = 10
    O.use_library(O.timing_build(tempfile.mkdtemp(prefix="orc_timing_")))
    nthr = O.threads()
    nl = gpu_line["nl_iters_per_step"]
    kblk = gpu_line["krylov_iters_per_step_by_block"]
    n_ind, n_s = prob.phi.shape[0], prob.B.shape[0]

    def reduced(div):
        if wname == "floes":
            return W.floe_field_3d(nx=256 // div, ny=128 // div, nz=64 // div)
        return W.cavity_sphere_3d(n=(128 if wname == "cavity128" else 64) // div)

    res = {}
    for label, div, thr in (("all", 4, nthr), ("one", 8, 1)):
        small = reduced(div)
        O.set_threads(thr)
        t0 = time.perf_counter()
        tm = oracle_sample(small, its)
        wall = time.perf_counter() - t0
        step = oracle_step_seconds(tm, nl, kblk, n_ind, n_s, prob.n_elems / small.n_elems,
                                   prob.n_nodes / small.n_nodes)
        res[label] = (small, tm, wall, step)
    O.set_threads(nthr)
    small, tm, wall, step_n = res["all"]
    small1, _, wall1, step_1 = res["one"]
    kb = kblk[:1] + kblk[1:2] + kblk[1 + n_ind:2 + n_ind]
    return dict(value=round(1.0 / step_n, 6), unit="steps/s", cores=nthr, kind="oracle",
                value_1thread=round(1.0 / step_1, 6),
                sample=(f"{wname} workload at a quarter of the resolution ({small.n_elems} elements) at its "
                        f"initial state, OpenMP timing copy of the oracle on {nthr} threads, {wall:.1f} s: "
                        f"momentum/mass assembly {tm['ns_asm']:.2f} s, {1e3 * tm['ns_it']:.1f} ms per momentum "
                        f"Krylov iteration, band + Allen-Cahn assembly {tm['ac_asm0']:.2f} s (largest band) and "
                        f"{tm.get('ac_asm1', 0):.2f} s, B assembly {tm.get('b_asm', 0):.2f} s; scaled by "
                        f"{prob.n_elems / small.n_elems:.0f}x elements and {prob.n_nodes / small.n_nodes:.1f}x "
                        f"nodes to the full mesh and to a step with the GPU's {nl:.2f} nonlinear and "
                        f"{'/'.join(f'{k:.0f}' for k in kb)} (momentum/Allen-Cahn/B) Krylov iterations per step, "
                        f"every indicator and solid solved on its own.  value_1thread: the same pieces on one "
                        f"thread at an eighth of the resolution ({small1.n_elems} elements, {wall1:.1f} s), "
                        f"scaled the same way"))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the multi-GPU sharding is a "
              "design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2402_10348_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    prob, wdesc = make_workload(args.workload)
    if args.calib_copy:
        calib_copy(torch, args.calib_copy)
    head, kts, ctx, st, elapsed = run_steps(args, prob, torch, args.workload)
    ctx.close()
    del st
    roofline = pair_line(kts, args.workload)
    kernels = {name: kernel_line(kts, r, args.workload) for name, r in (("assembly", 3), ("spmv", 2),
                                                                         ("mg_sweep", 1))}
    mixed = None
    if args.mixed:
        # the same steps with FP32 Jacobian values and the FP64 run's tuned
        # knobs (so that only the precision differs between the two lines)
        am = argparse.Namespace(**vars(args))
        am.tune = False
        knobs = dict((head.get("tuning") or {}).get("knobs") or {})
        m, _, c2, s2, _ = run_steps(am, prob, torch, args.workload + " mixed", time_kernels=False, precision=1,
                                    **knobs)
        c2.close()
        del s2
        mixed = dict(m, dtype="f64 residual/Krylov, f32 Jacobian", knobs=knobs or None)
    secondary = {}
    if args.secondary:
        for name in ("cavity128", "cavity64"):
            if name == args.workload:
                continue
            pb, desc = make_workload(name)
            line, kt2, c2, s2, _ = run_steps(args, pb, torch, name)
            c2.close()
            del s2
            secondary[name] = dict(line, workload=desc, roofline=pair_line(kt2, name),
                                   kernels={nm: kernel_line(kt2, r, name) for nm, r in
                                            (("assembly", 3), ("spmv", 2), ("mg_sweep", 1))})
    variants = None
    if args.variants:
        pb = W.cavity_sphere_3d(n=64)
        a2 = argparse.Namespace(**vars(args))
        base, fin = run_variant(a2, pb, torch)
        full = run_full_domain(a2, pb, torch, fin)
        background = run_background(a2, pb, torch)
        from paper_2402_10348_amd.eft import Context
        c3 = Context(pb)
        s3 = c3.device_state(pb.state_copy())
        c3.step(s3)
        diag = diagnostics(c3, s3, pb)
        c3.close()
        variants = dict(workload="3D cavity with elastic sphere, 64^3", banded=base, full_domain_transport=full,
                        background_indicator=background, diagnostics=diag)
    learned = None
    if args.learned:
        log(args, "[bench] learned vs plain preconditioner ...")
        learned = run_learned(args, torch)
    cpu = None
    if not args.no_cpu:
        log(args, "[bench] timing the CPU oracle sample ...")
        cpu = cpu_baseline(prob, args.workload, head, args)

    line = {
        "metric": "converged time steps/s (FP64, every nonlinear iteration to ||dx||/||x|| < 5e-4, FGMRES to 1e-8)",
        "value": head["value"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64+f32J",
        "data": "synthetic (seeded geometry, tanh indicators of analytic signed distances, B = I, v = 0 at t = 0)",
        "config": {"workload": wdesc, "n_nodes": prob.n_nodes, "n_elems": prob.n_elems,
                   "indicators": int(prob.phi.shape[0]), "solids": int(prob.B.shape[0]), "dt": prob.params.dt,
                   "lin_rtol": 1e-8, "restart": args.restart, "nl_rtol": prob.params.nl_rtol, "nl_max": 20,
                   "converged_steps": head["converged_steps"], "nonconverged_steps": head["nonconverged_steps"],
                   "nl_iters_per_step": head["nl_iters_per_step"],
                   "krylov_iters_per_step_by_block": head["krylov_iters_per_step_by_block"],
                   "transport_ms_per_step": head["transport_ms_per_step"], "tuning": head.get("tuning"),
                   "preconditioner": {0: "point-block Jacobi", 1: "multigrid V-cycle", 2: "learned",
                                      3: "block ILU(0)"}[args.precond]
                   + (" (coarse levels kept within a step)" if args.precond == 1 and args.mg_lag else ""),
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "mixed_precision": mixed,
        "secondary": secondary,
        "variants": variants,
        "learned_vs_plain_precond": learned,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
