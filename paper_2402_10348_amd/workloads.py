"""Seeded synthetic inputs shared by the HIP path, the tests and the bench.

This module builds meshes, boundary-condition sets, material tables, solver
parameters and initial states for the cavity / falling-body / floe workloads.
It holds none of the method's arithmetic (no residuals, tangents, mobility,
Lagrange multiplier or solver steps): only geometry, bookkeeping and the
tanh initial profile of the order parameter (Sec. 3, phi = tanh(d/(sqrt(2) eps))
truncated to +-1 beyond 3 eps).

Random numbers come from numpy's PCG64 with an explicit seed.

Mesh convention
---------------
* Box [lo, hi] with ``n[k]`` cells per axis, nodes at lo + i*h, numbered
  lexicographically with x fastest.
* 2D: each cell is split by its (0,0)-(1,1) diagonal into two triangles.
* 3D: Kuhn split of each hex into 6 tets, one per axis permutation pi:
  (v0, v0+e_pi0, v0+e_pi0+e_pi1, v7); odd permutations have two nodes swapped
  so that every simplex has positive volume.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional

import numpy as np

# ---------------------------------------------------------------- mesh ----


def box_mesh(dim: int, n, lo=None, hi=None, mirror_z: bool = False):
    """Structured simplex mesh of a box.

    Returns ``xyz`` float64 [N][dim], ``conn`` int32 [E][dim+1] (positive
    orientation) and ``grid`` int32 [3] (cell counts; 1 for unused axes).
    3D cells are split into the 6 Kuhn tetrahedra along the cell diagonal
    (0,0,0)-(1,1,1); with mirror_z the cells of the upper half (k >= nz/2) use
    the split reflected in z (diagonal (0,0,1)-(1,1,0)), which keeps the mesh
    conforming (the mid-plane faces keep their x-y diagonal) and makes it
    symmetric under z -> 1 - z.
    """
    n = [int(v) for v in n]
    assert len(n) == dim
    lo = np.zeros(dim) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.ones(dim) if hi is None else np.asarray(hi, dtype=np.float64)
    axes = [lo[k] + (hi[k] - lo[k]) * np.arange(n[k] + 1) / n[k] for k in range(dim)]
    if dim == 2:
        Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
        xyz = np.stack([X.ravel(), Y.ravel()], axis=1)
        nx1 = n[0] + 1
        j, i = np.meshgrid(np.arange(n[1]), np.arange(n[0]), indexing="ij")
        v00 = (i + nx1 * j).ravel()
        v10, v01, v11 = v00 + 1, v00 + nx1, v00 + nx1 + 1
        t1 = np.stack([v00, v10, v11], axis=1)
        t2 = np.stack([v00, v11, v01], axis=1)
        conn = np.stack([t1, t2], axis=1).reshape(-1, 3)
        grid = np.array([n[0], n[1], 1], dtype=np.int32)
    elif dim == 3:
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        sx, sy = 1, n[0] + 1
        sz = (n[0] + 1) * (n[1] + 1)
        k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
        up = (k >= n[2] // 2).ravel() if mirror_z else np.zeros(k.size, dtype=bool)
        # start corner and z step of every cell (reflected cells start on top)
        v0 = (i * sx + j * sy + k * sz).ravel() + np.where(up, sz, 0)
        zs = np.where(up, -sz, sz)
        tets = []
        for perm in itertools.permutations(range(3)):
            steps = [np.full(v0.shape, sx), np.full(v0.shape, sy), zs]
            a = v0 + steps[perm[0]]
            b = a + steps[perm[1]]
            c = b + steps[perm[2]]
            # parity of the permutation decides the orientation; a reflected
            # cell has the opposite one
            inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
            even = (inv % 2 == 0) != up
            tets.append(np.where(even[:, None], np.stack([v0, a, b, c], axis=1), np.stack([v0, b, a, c], axis=1)))
        conn = np.stack(tets, axis=1).reshape(-1, 4)
        grid = np.array(n, dtype=np.int32)
    else:
        raise ValueError("dim must be 2 or 3")
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(conn, dtype=np.int32), grid


# ------------------------------------------------------ initial profile ----


def tanh_profile(d: np.ndarray, eps: float) -> np.ndarray:
    """Order parameter from a signed distance d (positive inside the phase).

    phi = tanh(d / (sqrt(2) eps)) for |d| <= 3 eps, +-1 beyond (Sec. 3.1).
    """
    d = np.asarray(d, dtype=np.float64)
    phi = np.tanh(d / (math.sqrt(2.0) * eps))
    far = np.abs(d) > 3.0 * eps
    phi[far] = np.sign(d[far])
    return phi


def sdf_ball(xyz, centre, radius):
    return radius - np.linalg.norm(xyz - np.asarray(centre)[None, :], axis=1)


def sdf_box(xyz, lo, hi):
    """Signed distance to an axis-aligned box, positive inside."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo)
    q = np.abs(xyz - c[None, :]) - h[None, :]
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = np.minimum(np.max(q, axis=1), 0.0)
    return -(outside + inside)


def sdf_disc(xyz, centre, radius, thickness):
    """Signed distance to a vertical-axis cylinder (disc) of given thickness."""
    c = np.asarray(centre, dtype=np.float64)
    r = np.linalg.norm(xyz[:, :2] - c[None, :2], axis=1) - radius
    z = np.abs(xyz[:, 2] - c[2]) - 0.5 * thickness
    q = np.stack([r, z], axis=1)
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = np.minimum(np.max(q, axis=1), 0.0)
    return -(outside + inside)


# ------------------------------------------------------------ problem ----

PHASE_FLUID = 0
PHASE_SOLID = 1


@dataclass
class Phase:
    kind: int            # PHASE_FLUID or PHASE_SOLID
    transported: int     # 0 = background complement, 1 = own order parameter
    rho: float
    mu: float
    mu_L: float = 0.0


@dataclass
class Params:
    dt: float
    rho_inf: float = 0.0
    eps: float = 0.0
    eta: float = 0.2
    C_I: float = 36.0
    di_cut: float = 0.9
    nl_rtol: float = 5e-4
    nl_max: int = 20
    nl_fixed: int = 0
    lin_rtol: float = 1e-8
    restart: int = 50
    lin_maxit: int = 1000
    precond: int = 1          # 1: geometric multigrid (structured boxes), 0: point-block Jacobi
    precision: int = 0
    band_flat: float = 1e-6
    band_cell: int = 4
    band_halo: int = 1
    mg_nu: int = 1            # pre-smoothing sweeps (the first from zero)
    mg_omega: float = 0.75
    mg_bf16: int = 1          # finest multigrid level's matrix copy in BF16 (0: FP32)
    mg_nu_post: int = 3
    mg_smoother: int = 0      # 0 damped block Jacobi, 1 multicolour block Gauss-Seidel
    band_sweeps: int = 2      # Allen-Cahn and B systems: damped block-Jacobi sweeps from zero
    band_omega: float = 0.6   # below 2 / 2.5: P1 consistent mass has lambda_max(D^-1 M) <= 2.5
    mg_galerkin: int = 0       # multigrid coarse operators: 0 rediscretized, 1 Galerkin P^T A P
    nn_maxit: int = 0          # learned preconditioner: iterations before block Jacobi takes over (0: lin_maxit/2)
    band_reserve: float = 0.0  # band storage for all indicators together, in mesh element counts (0: auto)
    graphs: int = 1           # momentum Krylov columns captured into HIP graphs and replayed
    nn_base: int = 0          # learned preconditioner corrects: 0 point-block Jacobi, 1 the multigrid V-cycle
    mg_lag: int = 0           # 1: coarse multigrid levels refreshed once per time step (first nonlinear iteration)
    mg_cnu: int = 0           # coarse multigrid levels' sweeps before / after the correction (0: as the finest)
    mg_cnu_post: int = 0


@dataclass
class Problem:
    name: str
    dim: int
    xyz: np.ndarray
    conn: np.ndarray
    grid: np.ndarray
    dir_node: np.ndarray     # int32 [n_dir]
    dir_mask: np.ndarray     # uint8 [n_dir]; bit k<dim velocity comp k, bit dim pressure
    dir_val: np.ndarray      # float64 [n_dir][dim+1]
    phases: List[Phase]
    g: np.ndarray            # float64 [3]
    params: Params
    # initial state at time level n
    vp: np.ndarray           # [N][dim+1]
    vdot: np.ndarray         # [N][dim]
    phi: np.ndarray          # [n_ind][N]
    phidot: np.ndarray       # [n_ind][N]
    B: np.ndarray            # [n_s][N][nv]
    Bdot: np.ndarray         # [n_s][N][nv]
    info: Dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.xyz.shape[0]

    @property
    def n_elems(self):
        return self.conn.shape[0]

    @property
    def n_ind(self):
        return sum(1 for p in self.phases if p.transported)

    @property
    def n_solid(self):
        return sum(1 for p in self.phases if p.kind == PHASE_SOLID)

    @property
    def nv(self):
        return 6 if self.dim == 3 else 3

    def state_copy(self):
        return dict(vp=self.vp.copy(), vdot=self.vdot.copy(), phi=self.phi.copy(),
                    phidot=self.phidot.copy(), B=self.B.copy(), Bdot=self.Bdot.copy())


def identity_voigt(dim: int, n: int) -> np.ndarray:
    """B = I in Voigt order [11,22,33,12,23,13] (3D) or [11,22,12] (2D)."""
    nv = 6 if dim == 3 else 3
    B = np.zeros((n, nv))
    B[:, :dim] = 1.0
    return B


def cavity_dirichlet(xyz: np.ndarray, dim: int, lid_axis: int = 1, lid_speed: float = 1.0,
                     pin_pressure: bool = True, tol: float = 1e-12):
    """No-slip walls, lid v_x = lid_speed on nodes strictly inside the face
    x[lid_axis] = max; edge/corner nodes keep the wall value 0; p = 0 pinned at
    node 0 of a closed cavity."""
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    on_bnd = np.zeros(xyz.shape[0], dtype=bool)
    for k in range(dim):
        on_bnd |= np.abs(xyz[:, k] - lo[k]) < tol
        on_bnd |= np.abs(xyz[:, k] - hi[k]) < tol
    lid = np.abs(xyz[:, lid_axis] - hi[lid_axis]) < tol
    for k in range(dim):
        if k == lid_axis:
            continue
        lid &= (xyz[:, k] > lo[k] + tol) & (xyz[:, k] < hi[k] - tol)
    nodes = np.nonzero(on_bnd)[0]
    mask = np.full(nodes.shape[0], (1 << dim) - 1, dtype=np.uint8)
    val = np.zeros((nodes.shape[0], dim + 1))
    val[lid[nodes], 0] = lid_speed
    if pin_pressure:
        if nodes.size and nodes[0] == 0:
            mask[0] |= (1 << dim)
        else:
            nodes = np.concatenate([[0], nodes])
            mask = np.concatenate([[1 << dim], mask]).astype(np.uint8)
            val = np.concatenate([np.zeros((1, dim + 1)), val])
    return nodes.astype(np.int32), mask.astype(np.uint8), val


def _finish(name, dim, xyz, conn, grid, dirs, phases, g, params, sdfs, eps, info=None):
    N = xyz.shape[0]
    n_ind = sum(1 for p in phases if p.transported)
    n_s = sum(1 for p in phases if p.kind == PHASE_SOLID)
    assert len(sdfs) == n_ind
    phi = np.stack([tanh_profile(d, eps) for d in sdfs]) if n_ind else np.zeros((0, N))
    nv = 6 if dim == 3 else 3
    B = np.stack([identity_voigt(dim, N) for _ in range(n_s)]) if n_s else np.zeros((0, N, nv))
    vp = np.zeros((N, dim + 1))
    # the initial velocity satisfies the boundary data
    dn, dm, dv = dirs
    for k in range(dim + 1):
        sel = (dm >> k) & 1 == 1
        vp[dn[sel], k] = dv[sel, k]
    return Problem(name=name, dim=dim, xyz=xyz, conn=conn, grid=grid,
                   dir_node=dn, dir_mask=dm, dir_val=dv, phases=phases,
                   g=np.asarray(g, dtype=np.float64), params=params,
                   vp=vp, vdot=np.zeros((N, dim)), phi=np.ascontiguousarray(phi),
                   phidot=np.zeros_like(phi), B=np.ascontiguousarray(B), Bdot=np.zeros_like(B),
                   info=info or {})


def cavity_disk_2d(n: int = 32, dt: float = 0.01, lin_rtol: float = 1e-10, nl_fixed: int = 3,
                   mu_L: float = 0.1) -> Problem:
    """2D lid-driven cavity with one elastic disk (r=0.2 at (0.6,0.5)).

    Fluid rho=1, mu=0.01; solid rho=1, mu=0.01, shear modulus mu_L;
    interface width eps = 2h, eta = 0.2; lid v_x = 1 on y = 1.
    """
    xyz, conn, grid = box_mesh(2, (n, n))
    h = 1.0 / n
    eps = 2.0 * h
    dirs = cavity_dirichlet(xyz, 2, lid_axis=1)
    phases = [Phase(PHASE_FLUID, 0, 1.0, 0.01), Phase(PHASE_SOLID, 1, 1.0, 0.01, mu_L)]
    params = Params(dt=dt, eps=eps, eta=0.2, nl_fixed=nl_fixed, lin_rtol=lin_rtol)
    sdf = sdf_ball(xyz, (0.6, 0.5), 0.2)
    return _finish(f"cavity_disk_2d_{n}", 2, xyz, conn, grid, dirs, phases, (0.0, 0.0, 0.0),
                   params, [sdf], eps, dict(h=h))


def cavity_sphere_3d(n: int = 64, dt: float = 0.005, lin_rtol: float = 1e-8, nl_fixed: int = 0,
                     mu_L: float = 0.1, eps_h: float = 1.5, mirror_z: bool = False) -> Problem:
    """3D lid-driven cavity with one elastic sphere (r=0.2 at (0.6,0.5,0.5)).

    Fluid rho=1, mu=0.01; solid rho=1, mu=0.01, shear modulus mu_L; interface
    width eps = 1.5h; eta = 0.2; lid v_x = 1 on y = 1.
    """
    xyz, conn, grid = box_mesh(3, (n, n, n), mirror_z=mirror_z)
    h = 1.0 / n
    eps = eps_h * h
    dirs = cavity_dirichlet(xyz, 3, lid_axis=1)
    phases = [Phase(PHASE_FLUID, 0, 1.0, 0.01), Phase(PHASE_SOLID, 1, 1.0, 0.01, mu_L)]
    params = Params(dt=dt, eps=eps, eta=0.2, nl_fixed=nl_fixed, lin_rtol=lin_rtol)
    sdf = sdf_ball(xyz, (0.6, 0.5, 0.5), 0.2)
    return _finish(f"cavity_sphere_3d_{n}", 3, xyz, conn, grid, dirs, phases, (0.0, 0.0, 0.0),
                   params, [sdf], eps, dict(h=h))


def falling_sphere_3d(n: int = 96, dt: float = 1e-3, lin_rtol: float = 1e-8) -> Problem:
    """Elastic sphere above an elastic block in water, z up, gravity -9.81.

    Box [0,1]x[0,1]x[0,2] with n x n x 2n cells; sphere r=0.15 at
    (0.5,0.5,1.5), rho=1500, shear modulus 1e5, no viscosity of its own; block
    [0.1,0.9]^2 x [0,0.3], rho=1200, shear modulus 5e4; water rho=1000,
    mu=1e-3; eps = h, eta = 0.1; no-slip walls, traction-free top.
    """
    xyz, conn, grid = box_mesh(3, (n, n, 2 * n), hi=(1.0, 1.0, 2.0))
    h = 1.0 / n
    eps = h
    lo, hi = xyz.min(0), xyz.max(0)
    tol = 1e-12
    wall = np.zeros(xyz.shape[0], dtype=bool)
    for k in range(3):
        wall |= np.abs(xyz[:, k] - lo[k]) < tol
        if k < 2:
            wall |= np.abs(xyz[:, k] - hi[k]) < tol
    nodes = np.nonzero(wall)[0].astype(np.int32)
    mask = np.full(nodes.shape[0], 0b111, dtype=np.uint8)
    val = np.zeros((nodes.shape[0], 4))
    phases = [Phase(PHASE_FLUID, 0, 1000.0, 1e-3),
              Phase(PHASE_SOLID, 1, 1500.0, 0.0, 1e5),
              Phase(PHASE_SOLID, 1, 1200.0, 0.0, 5e4)]
    params = Params(dt=dt, eps=eps, eta=0.1, lin_rtol=lin_rtol)
    sdfs = [sdf_ball(xyz, (0.5, 0.5, 1.5), 0.15), sdf_box(xyz, (0.1, 0.1, -1.0), (0.9, 0.9, 0.3))]
    return _finish(f"falling_sphere_3d_{n}", 3, xyz, conn, grid, (nodes, mask, val), phases,
                   (0.0, 0.0, -9.81), params, sdfs, eps, dict(h=h))


def floe_positions(n_floes: int, seed: int, x_range=(1.4, 3.9), width: float = 2.0,
                   r_range=(0.1, 0.3), max_tries: int = 100000):
    """Non-overlapping disc centres (x, y) and radii by rejection sampling:
    radius uniform in r_range, centre x uniform in x_range, y keeping the disc
    inside [0, width]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    tries = 0
    while len(out) < n_floes:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("floe placement failed")
        r = rng.uniform(*r_range)
        x = rng.uniform(*x_range)
        y = rng.uniform(r, width - r)
        if all((x - a) ** 2 + (y - b) ** 2 > (r + c) ** 2 for a, b, c in out):
            out.append((x, y, r))
    return out


def floe_field_3d(nx: int = 256, ny: int = 128, nz: int = 64, dt: float = 1e-3, lin_rtol: float = 1e-8,
                  n_floes: int = 16, seed: int = 0, thickness: float = 0.02, water: float = 0.6) -> Problem:
    """A box-like hull moving at 1 m/s among ice floes in an air-water domain.

    Box [0,4]x[0,2]x[0,1] (z up, g = -9.81) at nx x ny x nz cells; water
    (rho 1000, mu 1e-3) below z = water, air (1.2, 1.8e-5) above as the
    background phase; hull box [0.5,1.1]x[0.85,1.15]x[0.5,0.75] (rho 500,
    shear modulus 1e9) whose interior nodes carry v = (1, 0, 0); n_floes discs
    of the given thickness centred on the water line (rho 900, shear modulus
    1e8, radius uniform in [0.1, 0.3], centres x in [1.4, 3.9], seeded and
    non-overlapping); solid viscosity 1e-3; eps = h, eta = 1000.  Slip walls
    on the x and y sides (normal velocity 0), no-slip bottom, open top.  One
    transported indicator per phase except the air: water, hull, floes.
    """
    xyz, conn, grid = box_mesh(3, (nx, ny, nz), hi=(4.0, 2.0, 1.0))
    h = 4.0 / nx
    eps = h
    lo, hi = xyz.min(0), xyz.max(0)
    tol = 1e-12
    N = xyz.shape[0]
    mask = np.zeros(N, dtype=np.uint8)
    for k in range(2):
        side = (np.abs(xyz[:, k] - lo[k]) < tol) | (np.abs(xyz[:, k] - hi[k]) < tol)
        mask[side] |= np.uint8(1 << k)
    mask[np.abs(xyz[:, 2] - lo[2]) < tol] |= np.uint8(0b111)
    hull_lo, hull_hi = (0.5, 0.85, 0.5), (1.1, 1.15, 0.75)
    d_hull = sdf_box(xyz, hull_lo, hull_hi)
    inside = d_hull > 0.0
    mask[inside] |= np.uint8(0b111)
    nodes = np.nonzero(mask)[0].astype(np.int32)
    val = np.zeros((nodes.shape[0], 4))
    val[inside[nodes], 0] = 1.0
    floes = floe_positions(n_floes, seed)
    phases = [Phase(PHASE_FLUID, 0, 1.2, 1.8e-5), Phase(PHASE_FLUID, 1, 1000.0, 1e-3),
              Phase(PHASE_SOLID, 1, 500.0, 1e-3, 1e9)]
    phases += [Phase(PHASE_SOLID, 1, 900.0, 1e-3, 1e8) for _ in floes]
    sdfs = [water - xyz[:, 2], d_hull]
    sdfs += [sdf_disc(xyz, (x, y, water), r, thickness) for x, y, r in floes]
    params = Params(dt=dt, eps=eps, eta=1000.0, lin_rtol=lin_rtol)
    return _finish(f"floe_field_3d_{nx}x{ny}x{nz}", 3, xyz, conn, grid, (nodes, mask[nodes], val), phases,
                   (0.0, 0.0, -9.81), params, sdfs, eps, dict(h=h, floes=floes))


# ------------------------------------------------ closed surface meshes ----


def icosphere(radius: float, center, level: int):
    """Triangulated sphere: the icosahedron with every face split into four
    `level` times and the vertices pushed onto the sphere.  Returns (vert
    [nv][3], tri [nt][3]); edge length about 1.05 r / 2^level."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    for _ in range(level):
        mid, nf = {}, []

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    vert = np.array(verts) * radius + np.asarray(center, dtype=np.float64)
    return vert, np.array(f, dtype=np.int32)


def cube_surface(lo, hi, m: int):
    """Surface of the box [lo, hi]^3: every face an m x m grid of squares,
    each split into two triangles (shared vertices).  Returns (vert, tri)."""
    lo, hi = float(lo), float(hi)
    g = np.linspace(lo, hi, m + 1)
    index, verts, tris = {}, [], []

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in index:
            index[key] = len(verts)
            verts.append(p)
        return index[key]
    for axis in range(3):
        for side in (lo, hi):
            a1, a2 = [k for k in range(3) if k != axis]
            for i in range(m):
                for j in range(m):
                    q = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = np.zeros(3)
                        p[axis], p[a1], p[a2] = side, g[i + di], g[j + dj]
                        q.append(vid(p))
                    tris += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    return np.array(verts), np.array(tris, dtype=np.int32)


# ------------------------------------------- paper-literal indicator set ----


def with_background_indicator(prob: Problem) -> Problem:
    """The variant with one transported order parameter per phase, the
    background included (the default treats the background as the complement
    of the others).  Its indicator starts from that complement: alpha_bg =
    clamp(1 - sum of the other fractions), phi_bg = 2 alpha_bg - 1; the
    indicators keep the phase order."""
    bg = [i for i, p in enumerate(prob.phases) if not p.transported]
    if not bg:
        return prob
    b = bg[0]
    alpha = np.clip(0.5 * (1.0 + prob.phi), 0.0, 1.0)
    a_bg = np.clip(1.0 - alpha.sum(axis=0), 0.0, 1.0)
    rows, rates, k = [], [], 0
    for i, p in enumerate(prob.phases):
        if i == b:
            rows.append(2.0 * a_bg - 1.0)
            rates.append(np.zeros(prob.n_nodes))
        elif p.transported:
            rows.append(prob.phi[k])
            rates.append(prob.phidot[k])
            k += 1
    phases = [replace(p, transported=1) if i == b else p for i, p in enumerate(prob.phases)]
    return replace(prob, name=prob.name + "+background", phases=phases, phi=np.array(rows), phidot=np.array(rates),
                   info=dict(prob.info))


# ------------------------------------------------- random perturbations ----


def perturbed_state(prob: Problem, seed: int, amp_v: float = 0.3, amp_p: float = 0.1,
                    amp_phi: float = 0.05, amp_B: float = 0.05, amp_rate: float = 0.2):
    """A seeded, smooth-ish random state for parity tests.

    Returns (level_n, iterate): two dicts of arrays.  The iterate differs from
    the level-n state by small random increments so that every time-level
    combination in the residual is exercised.  Dirichlet values are respected
    in both.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N, dim = prob.n_nodes, prob.dim
    lvl = prob.state_copy()
    it = dict(vp=None, phi=None, B=None)
    lvl["vp"] = lvl["vp"] + np.concatenate([amp_v * rng.standard_normal((N, dim)),
                                            amp_p * rng.standard_normal((N, 1))], axis=1)
    lvl["vdot"] = amp_rate * rng.standard_normal((N, dim))
    if prob.n_ind:
        lvl["phi"] = np.clip(lvl["phi"] + amp_phi * rng.standard_normal(lvl["phi"].shape), -1.0, 1.0)
        lvl["phidot"] = amp_rate * rng.standard_normal(lvl["phidot"].shape)
    if prob.n_solid:
        lvl["B"] = lvl["B"] + amp_B * rng.standard_normal(lvl["B"].shape)
        lvl["Bdot"] = amp_rate * rng.standard_normal(lvl["Bdot"].shape)
    it["vp"] = lvl["vp"] + 0.1 * amp_v * rng.standard_normal(lvl["vp"].shape)
    it["phi"] = lvl["phi"] + 0.1 * amp_phi * rng.standard_normal(lvl["phi"].shape)
    it["B"] = lvl["B"] + 0.1 * amp_B * rng.standard_normal(lvl["B"].shape)
    for d in (lvl, it):
        vp = d["vp"]
        for k in range(dim + 1):
            sel = (prob.dir_mask >> k) & 1 == 1
            vp[prob.dir_node[sel], k] = prob.dir_val[sel, k]
    return lvl, it


def make(name: str, **kw) -> Problem:
    """Workload by name: 'c1' (2D cavity, 32^2), 'c2' (3D cavity, 64^3),
    'c3' (falling sphere, 96x96x192), 'c4' (hull among floes, 256x128x64),
    'c5' (3D cavity, 128^3) or a builder name with keywords."""
    if name == "c1":
        return cavity_disk_2d(**kw)
    if name == "c2":
        return cavity_sphere_3d(**kw)
    if name == "c3":
        return falling_sphere_3d(**kw)
    if name == "c4":
        return floe_field_3d(**kw)
    if name == "c5":
        return cavity_sphere_3d(**dict(dict(n=128), **kw))
    return globals()[name](**kw)
