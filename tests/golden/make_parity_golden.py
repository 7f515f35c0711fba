#!/usr/bin/env python3
"""Writes the FP64 oracle's fields after several time steps for the GPU parity
tests at sizes the oracle needs minutes for (the tests compare the HIP path
with these files element by element).  It calls only the oracle (its OpenMP
build, bit-identical to the portable one) and the seeded input generator.

    python tests/golden/make_parity_golden.py [name ...]

Each case: workload, steps, solver settings (FGMRES to 1e-13 unless the case
says otherwise).  Output: tests/golden/parity_<name>.npz with the final vp,
vdot, phi, phidot, B, Bdot and the per-step nonlinear iteration counts.
"""
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2402_10348_amd import workloads as W  # noqa: E402

TIGHT = dict(lin_rtol=1e-13, restart=200, lin_maxit=400000)

# name: (problem factory, steps, oracle overrides)
CASES = {
    # the 2D cavity with the elastic disk exactly as configured (32^2, 10
    # steps x 3 nonlinear iterations, FGMRES with block Jacobi to 1e-10)
    "disk2d_32_configured": (lambda: W.cavity_disk_2d(n=32), 10, dict(restart=200, lin_maxit=400000)),
    # the same steps with the linear solves to 1e-13 (parity at 1e-10)
    "disk2d_32_tight": (lambda: W.cavity_disk_2d(n=32), 10, TIGHT),
    # the 3D cavity with the elastic sphere, 50 steps at 24^3 (the largest
    # size whose 50 oracle steps finish in about half an hour here)
    "cavity_24_50": (lambda: W.cavity_sphere_3d(n=24), 50, TIGHT),
    # the falling sphere on the block at a quarter of its resolution
    # (24 x 24 x 48), two steps
    "falling_24_2": (lambda: W.falling_sphere_3d(n=24), 2, TIGHT),
    # the hull among all 16 floes at an eighth of its resolution (32 x 16 x
    # 8), two steps: the largest floe field whose oracle steps (point-block
    # Jacobi on the stiff hull and floes) finish in minutes here
    "floes_32_2": (lambda: W.floe_field_3d(nx=32, ny=16, nz=8), 2, TIGHT),
}


def run(name):
    make, steps, over = CASES[name]
    prob = make()
    c = O.Case(prob, **over)
    st = prob.state_copy()
    nl = []
    t0 = time.time()
    for s in range(steps):
        info = c.step(st)
        nl.append(info["nl_iters"])
        print(f"{name}: step {s} nl={info['nl_iters']} lin={info['lin_iters_total']} status={info['status']} "
              f"{time.time() - t0:.0f}s", flush=True)
    out = os.path.join(HERE, f"parity_{name}.npz")
    np.savez_compressed(out, steps=steps, nl_iters=np.array(nl), **{k: st[k] for k in
                                                                      ("vp", "vdot", "phi", "phidot", "B", "Bdot")})
    print(f"wrote {out} ({os.path.getsize(out) / 1e6:.2f} MB)", flush=True)


if __name__ == "__main__":
    O.use_library(O.timing_build(tempfile.mkdtemp(prefix="orc_golden_")))
    for name in (sys.argv[1:] or list(CASES)):
        run(name)
