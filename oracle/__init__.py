"""FP64 CPU oracle of the Eulerian phase-field FSI time step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the bench use it to check the HIP library.  It never imports the HIP
package, and the HIP package never imports it.  Problems are passed in as any
object with the attributes of a workload description (dim, xyz, conn, grid,
dir_node, dir_mask, dir_val, phases, g, params).

Every function is pinned by a check independent of its own code (see the
tests): closed forms, printed values, invariants, finite differences, a dense
solve, manufactured-solution convergence rates of the momentum/mass and
Allen-Cahn discretizations, and, for the grid-cell band (a definition of this
implementation's own), a brute-force restatement plus the geometric decay of
its difference to the full-domain transport with the halo width.  Parity
unpinned: only the paper's physical trajectories (figures without data) and
the bound |phi| <= 1 + delta.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eft_oracle.c")
_LIB = os.path.join(_HERE, "_liborc.so")

dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int)
u8p = C.POINTER(C.c_uint8)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (portable flags: the library may run on
    another host's CPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def timing_build(out_dir: str) -> str:
    """Compile the timing copy of the oracle into out_dir: -O3 -march=native
    with OpenMP (parallel element evaluation and SpMV rows).  -ffp-contract=off
    keeps every product and sum rounded as in the portable build, and the
    assembly adds element contributions in element order, so the results
    are bit-identical with any thread count.  Built where it runs (the
    native flags target the host's CPU)."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "_liborc_omp.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-std=c99", "-shared",
                           "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)
    return out


def use_library(path: str) -> None:
    """Route every later oracle call through the library at path (the timing
    copy); the default is the portable build."""
    global _lib
    _lib = None
    _setup(C.CDLL(path))


def threads() -> int:
    """Threads of the loaded library's parallel loops."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the parallel loops of the timing copy (no effect on the
    portable build)."""
    lib().orc_set_threads(int(n))


class Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n_nodes", C.c_int), ("n_elems", C.c_int),
        ("xyz", dp), ("conn", ip), ("grid", C.c_int * 3),
        ("n_dir", C.c_int), ("dir_node", ip), ("dir_mask", u8p), ("dir_val", dp),
        ("n_phase", C.c_int), ("kind", ip), ("transported", ip),
        ("rho", dp), ("mu", dp), ("muL", dp),
        ("g", C.c_double * 3),
        ("dt", C.c_double), ("rho_inf", C.c_double), ("eps", C.c_double), ("eta", C.c_double),
        ("C_I", C.c_double), ("di_cut", C.c_double), ("nl_rtol", C.c_double),
        ("nl_max", C.c_int), ("nl_fixed", C.c_int),
        ("lin_rtol", C.c_double), ("restart", C.c_int), ("lin_maxit", C.c_int),
        ("band_flat", C.c_double), ("band_cell", C.c_int), ("band_halo", C.c_int),
    ]


class State(C.Structure):
    _fields_ = [("vp", dp), ("vdot", dp), ("phi", dp), ("phidot", dp), ("B", dp), ("Bdot", dp)]


class StepInfo(C.Structure):
    _fields_ = [("nl_iters", C.c_int), ("converged", C.c_int), ("lin_iters_total", C.c_int),
                ("lin_failures", C.c_int), ("n_blocks", C.c_int),
                ("block_ratio", C.c_double * 66), ("gamma", C.c_double * 64), ("beta", C.c_double * 64)]


_lib = None


def _setup(L):
    global _lib
    _lib = L
    L.orc_threads.restype = C.c_int
    L.orc_graph_nnz.restype = C.c_int
    L.orc_fgmres.restype = C.c_int
    L.orc_ilu0.restype = C.c_int
    L.orc_mobility.restype = C.c_double
    L.orc_beta.restype = C.c_double
    L.orc_step.restype = C.c_int
    L.orc_simplex_geometry.restype = C.c_double
    L.orc_center_of_mass.restype = C.c_double
    L.orc_track_particle.restype = C.c_int


def lib():
    if _lib is None:
        _setup(C.CDLL(build()))
    return _lib


def _d(a):
    return a.ctypes.data_as(dp)


def _i(a):
    return a.ctypes.data_as(ip)


def _u8(a):
    return a.ctypes.data_as(u8p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Case:
    """Owns the contiguous arrays behind an orc_problem."""

    def __init__(self, prob, **overrides):
        self.dim = int(prob.dim)
        self.xyz = _f64(prob.xyz)
        self.conn = np.ascontiguousarray(prob.conn, dtype=np.int32)
        self.N = self.xyz.shape[0]
        self.E = self.conn.shape[0]
        self.nv = 6 if self.dim == 3 else 3
        self.bs = self.dim + 1
        self.dir_node = np.ascontiguousarray(prob.dir_node, dtype=np.int32)
        self.dir_mask = np.ascontiguousarray(prob.dir_mask, dtype=np.uint8)
        self.dir_val = _f64(prob.dir_val).reshape(-1, self.dim + 1)
        ph = prob.phases
        self.kind = np.array([p.kind for p in ph], dtype=np.int32)
        self.transported = np.array([p.transported for p in ph], dtype=np.int32)
        self.rho = np.array([p.rho for p in ph], dtype=np.float64)
        self.mu = np.array([p.mu for p in ph], dtype=np.float64)
        self.muL = np.array([p.mu_L for p in ph], dtype=np.float64)
        self.n_ind = int(self.transported.sum())
        self.n_s = int((self.kind == 1).sum())
        pr = prob.params
        P = Problem()
        P.dim, P.n_nodes, P.n_elems = self.dim, self.N, self.E
        P.xyz, P.conn = _d(self.xyz), _i(self.conn)
        for k in range(3):
            P.grid[k] = int(prob.grid[k])
        P.n_dir = self.dir_node.shape[0]
        P.dir_node, P.dir_mask, P.dir_val = _i(self.dir_node), _u8(self.dir_mask), _d(self.dir_val)
        P.n_phase = len(ph)
        P.kind, P.transported = _i(self.kind), _i(self.transported)
        P.rho, P.mu, P.muL = _d(self.rho), _d(self.mu), _d(self.muL)
        for k in range(3):
            P.g[k] = float(prob.g[k])
        vals = dict(dt=pr.dt, rho_inf=pr.rho_inf, eps=pr.eps, eta=pr.eta, C_I=pr.C_I, di_cut=pr.di_cut,
                    nl_rtol=pr.nl_rtol, nl_max=pr.nl_max, nl_fixed=pr.nl_fixed, lin_rtol=pr.lin_rtol,
                    restart=pr.restart, lin_maxit=pr.lin_maxit, band_flat=pr.band_flat,
                    band_cell=pr.band_cell, band_halo=pr.band_halo)
        vals.update(overrides)
        for k, v in vals.items():
            setattr(P, k, v)
        self.P = P
        self._graph = None

    # ---------------------------------------------------------------- graph
    def graph(self):
        if self._graph is None:
            L = lib()
            nnz = L.orc_graph_nnz(C.byref(self.P))
            rowptr = np.zeros(self.N + 1, dtype=np.int32)
            col = np.zeros(nnz, dtype=np.int32)
            L.orc_graph(C.byref(self.P), _i(rowptr), _i(col))
            self._graph = (rowptr, col)
        return self._graph

    def _state(self, st):
        keep = {k: _f64(st[k]) for k in ("vp", "vdot", "phi", "phidot", "B", "Bdot")}
        S = State()
        for k, a in keep.items():
            setattr(S, k, _d(a))
        return S, keep

    # ------------------------------------------------------------- assembly
    def ns_assemble(self, lvl, it, bc=True):
        """Residual [N][dim+1] and BSR values [nnz][bs][bs] of eq. (PG_NS)."""
        rowptr, col = self.graph()
        S, keep = self._state(lvl)
        vp, phi, B = _f64(it["vp"]), _f64(it["phi"]), _f64(it["B"])
        R = np.zeros((self.N, self.bs))
        J = np.zeros((col.shape[0], self.bs, self.bs))
        lib().orc_ns_assemble(C.byref(self.P), C.byref(S), _d(vp), _d(phi), _d(B), _i(rowptr), _i(col), _d(R), _d(J))
        if bc:
            lib().orc_ns_apply_bc(C.byref(self.P), _i(rowptr), _i(col), _d(R), _d(J))
        return R, J

    def ns_rows(self, lvl, it, rows):
        """Rows `rows` of the residual and Jacobian of eq. (PG_NS) with the
        boundary rows applied, without assembling the rest: R [nr][bs] and a
        list of (columns, blocks [len][bs][bs]) per row."""
        rowptr, col = self.graph()
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        S, keep = self._state(lvl)
        vp, phi, B = _f64(it["vp"]), _f64(it["phi"]), _f64(it["B"])
        lens = rowptr[rows + 1] - rowptr[rows]
        R = np.zeros((rows.shape[0], self.bs))
        J = np.zeros((int(lens.sum()), self.bs, self.bs))
        lib().orc_ns_rows(C.byref(self.P), C.byref(S), _d(vp), _d(phi), _d(B), _i(rowptr), _i(col),
                          int(rows.shape[0]), _i(rows), _d(R), _d(J))
        out, o = [], 0
        for q, r in enumerate(rows):
            out.append((col[rowptr[r]:rowptr[r + 1]].copy(), J[o:o + lens[q]]))
            o += lens[q]
        return R, out

    def level_values(self, xn, xdn, xnp1):
        xn, xdn, xnp1 = _f64(xn), _f64(xdn), _f64(xnp1)
        xa, xd = np.zeros_like(xn), np.zeros_like(xn)
        lib().orc_level_values(C.c_double(self.P.rho_inf), C.c_double(self.P.dt), xn.size, _d(xn), _d(xdn),
                               _d(xnp1), _d(xa), _d(xd))
        return xa, xd

    def nodal_properties(self, phi_a):
        phi_a = _f64(phi_a)
        af = np.zeros((len(self.kind), self.N))
        rho = np.zeros(self.N)
        mu = np.zeros(self.N)
        lib().orc_nodal_properties(C.byref(self.P), _d(phi_a), _d(af), _d(rho), _d(mu))
        return af, rho, mu

    def mobility(self, v_a, phi_a):
        return lib().orc_mobility(C.byref(self.P), _d(_f64(v_a)), _d(_f64(phi_a)))

    def band(self, phi_n):
        be = np.zeros(self.E, dtype=np.uint8)
        fr = np.zeros(self.N, dtype=np.uint8)
        lib().orc_band(C.byref(self.P), _d(_f64(phi_n)), _u8(be), _u8(fr))
        return be, fr

    def beta(self, phi_a, band_elem=None):
        be = None if band_elem is None else np.ascontiguousarray(band_elem, dtype=np.uint8)
        return lib().orc_beta(C.byref(self.P), _d(_f64(phi_a)), None if be is None else _u8(be))

    def ac_assemble(self, v_a, phi_a, phid_am, gamma, beta, band_elem, free_node):
        rowptr, col = self.graph()
        R = np.zeros(self.N)
        J = np.zeros(col.shape[0])
        be = np.ascontiguousarray(band_elem, dtype=np.uint8)
        fr = np.ascontiguousarray(free_node, dtype=np.uint8)
        lib().orc_ac_assemble(C.byref(self.P), _d(_f64(v_a)), _d(_f64(phi_a)), _d(_f64(phid_am)),
                              C.c_double(gamma), C.c_double(beta), _u8(be), _u8(fr), _i(rowptr), _i(col), _d(R), _d(J))
        return R, J

    def b_assemble(self, v_a, afrac, B_a, Bd_am, band_elem, free_node):
        rowptr, col = self.graph()
        nv = self.nv
        R = np.zeros((self.N, nv))
        J = np.zeros((col.shape[0], nv, nv))
        be = np.ascontiguousarray(band_elem, dtype=np.uint8)
        fr = np.ascontiguousarray(free_node, dtype=np.uint8)
        lib().orc_b_assemble(C.byref(self.P), _d(_f64(v_a)), _d(_f64(afrac)), _d(_f64(B_a)), _d(_f64(Bd_am)),
                             _u8(be), _u8(fr), _i(rowptr), _i(col), _d(R), _d(J))
        return R, J

    # ------------------------------------------------------------ algebra
    def spmv(self, J, x):
        rowptr, col = self.graph()
        J = _f64(J)
        bs = int(round((J.size // col.shape[0]) ** 0.5))
        x = _f64(x)
        y = np.zeros_like(x)
        lib().orc_spmv(bs, self.N, _i(rowptr), _i(col), _d(J), _d(x), _d(y))
        return y

    def fgmres(self, J, b, rtol=None, restart=None, maxit=None):
        rowptr, col = self.graph()
        J = _f64(J)
        bs = int(round((J.size // col.shape[0]) ** 0.5))
        b = _f64(b)
        x = np.zeros_like(b)
        its = C.c_int(0)
        rr = C.c_double(0.0)
        st = lib().orc_fgmres(bs, self.N, _i(rowptr), _i(col), _d(J), _d(b), _d(x),
                              restart or self.P.restart, maxit or self.P.lin_maxit,
                              C.c_double(self.P.lin_rtol if rtol is None else rtol), C.byref(its), C.byref(rr))
        return x, dict(status=st, iters=its.value, relres=rr.value)

    def ilu0(self, J):
        """Block ILU(0) factors of J on the node graph (natural order):
        (lu [nnz][bs*bs] holding L below and U on and above the diagonal,
        dinv [N][bs*bs] = U_ii^-1, status 0 or 1 + the first singular row)."""
        rowptr, col = self.graph()
        J = _f64(J)
        bs = int(round((J.size // col.shape[0]) ** 0.5))
        lu = np.zeros_like(J)
        dinv = np.zeros((self.N, bs * bs))
        st = lib().orc_ilu0(bs, self.N, _i(rowptr), _i(col), _d(J), _d(lu), _d(dinv))
        return lu, dinv, st

    def ilu0_apply(self, lu, dinv, r):
        """z = (L U)^-1 r with the factors of ilu0."""
        rowptr, col = self.graph()
        lu = _f64(lu)
        bs = int(round((lu.size // col.shape[0]) ** 0.5))
        r = _f64(r)
        z = np.zeros_like(r)
        lib().orc_ilu0_apply(bs, self.N, _i(rowptr), _i(col), _d(lu), _d(_f64(dinv)), _d(r), _d(z))
        return z

    # ---------------------------------------------------------- diagnostics
    def center_of_mass(self, phi):
        """(x_c [dim], int alpha dOmega) of the region of one order parameter."""
        xc = np.zeros(3)
        m = lib().orc_center_of_mass(C.byref(self.P), _d(_f64(phi)), _d(xc))
        return xc[:self.dim].copy(), m

    def track_particle(self, vp, x, dt, tol=1e-10):
        """Moves the particle x [dim] by one explicit step; returns (x_new,
        element or -1, shape functions)."""
        xx = _f64(np.array(x, dtype=np.float64).copy())
        Nv = np.zeros(4)
        e = lib().orc_track_particle(C.byref(self.P), _d(_f64(vp)), C.c_double(dt), C.c_double(tol), _d(xx), _d(Nv))
        return xx, e, Nv[:self.dim + 1].copy()

    def init_phase(self, vert, tri, eps, ncell, chi=1e-12):
        """Order parameter of the solid inside the closed surface (vert
        [nv][3], tri [nt][3]) on the mesh nodes (3D); returns (phi, stats)."""
        vert = _f64(vert)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        nc = np.ascontiguousarray(ncell, dtype=np.int32)
        phi = np.zeros(self.N)
        stats = np.zeros(2, dtype=np.int32)
        lib().orc_init_phase(C.byref(self.P), vert.shape[0], _d(vert), tri.shape[0], _i(tri), C.c_double(eps),
                             _i(nc), C.c_double(chi), _d(phi), _i(stats))
        return phi, stats

    # --------------------------------------------------------------- step
    def step(self, st):
        """Advance the state dict in place by one time step; returns info."""
        S, keep = self._state(st)
        info = StepInfo()
        status = lib().orc_step(C.byref(self.P), C.byref(S), C.byref(info))
        for k, a in keep.items():
            st[k] = a
        nb = info.n_blocks
        return dict(status=status, nl_iters=info.nl_iters, converged=info.converged,
                    lin_iters_total=info.lin_iters_total, lin_failures=info.lin_failures,
                    block_ratio=list(info.block_ratio[:nb]), gamma=list(info.gamma[:self.n_ind]),
                    beta=list(info.beta[:self.n_ind]))


# -------------------------------------------------------- element probes ----

def simplex_geometry(dim, X):
    X3 = np.zeros((4, 3))
    X3[:dim + 1, :dim] = X
    dN = np.zeros((4, 3))
    G = np.zeros((3, 3))
    vol = lib().orc_simplex_geometry(dim, _d(X3), _d(dN), _d(G))
    return vol, dN[:dim + 1, :dim].copy(), G[:dim, :dim].copy()


def level_values(rho_inf, dt, xn, xdn, xnp1):
    """Value at n+alpha and rate at n+alpha_m from x^n, xdot^n and x^{n+1}."""
    xn, xdn, xnp1 = _f64(xn), _f64(xdn), _f64(xnp1)
    xa, xd = np.zeros_like(xn), np.zeros_like(xn)
    lib().orc_level_values(C.c_double(rho_inf), C.c_double(dt), xn.size, _d(xn), _d(xdn), _d(xnp1), _d(xa), _d(xd))
    return xa, xd


def galpha(rho_inf, dt):
    out = np.zeros(5)
    lib().orc_galpha(C.c_double(rho_inf), C.c_double(dt), _d(out))
    return dict(alpha=out[0], alpha_m=out[1], varsigma=out[2], ct=out[3], kappa=out[4])


def ns_element(dim, rho_inf, dt, C_I, g, X, v, acc, p, rho, mu, alphas=(), Bv=(), muL=(), vref=None):
    """Element residual [nn][bs] and tangent [nn][nn][bs][bs] of eq. (PG_NS).
    vref: linearization point of tau_m, tau_c and the SUPG weight (default v)."""
    nn, bs = dim + 1, dim + 1
    nv = 6 if dim == 3 else 3

    def pad(a, shape):
        out = np.zeros(shape)
        a = np.asarray(a, dtype=np.float64)
        out[tuple(slice(0, s) for s in a.shape)] = a
        return out

    n_s = len(muL)
    X4, v4, a4 = pad(X, (4, 3)), pad(v, (4, 3)), pad(acc, (4, 3))
    w4 = v4 if vref is None else pad(vref, (4, 3))
    p4, r4, m4 = pad(p, (4,)), pad(rho, (4,)), pad(mu, (4,))
    as_ = np.zeros((max(n_s, 1), 4))
    Bv_ = np.zeros((max(n_s, 1), 4, 6))
    for s in range(n_s):
        as_[s, :nn] = alphas[s]
        Bv_[s, :nn, :nv] = Bv[s]
    muL_ = np.zeros(max(n_s, 1))
    muL_[:n_s] = muL
    g3 = pad(g, (3,))
    re = np.zeros((4, 4))
    Ke = np.zeros((4, 4, 4, 4))
    lib().orc_ns_element(dim, C.c_double(rho_inf), C.c_double(dt), C.c_double(C_I), _d(g3), _d(X4), _d(v4), _d(w4), _d(a4),
                         _d(p4), _d(r4), _d(m4), n_s, _d(as_), _d(Bv_), _d(muL_), _d(re), _d(Ke))
    return re[:nn, :bs].copy(), Ke[:nn, :nn, :bs, :bs].copy()


def ac_element(dim, rho_inf, dt, eps, gamma, beta, X, v, phi, phid, phiref=None):
    """Element residual and tangent of eq. (PPV_AC); phiref freezes tau_phi."""
    nn = dim + 1
    X4 = np.zeros((4, 3)); X4[:nn, :dim] = X
    v4 = np.zeros((4, 3)); v4[:nn, :dim] = v
    f4 = np.zeros(4); f4[:nn] = phi
    fd4 = np.zeros(4); fd4[:nn] = phid
    fr4 = f4.copy()
    if phiref is not None:
        fr4[:nn] = phiref
    re = np.zeros(4)
    Ke = np.zeros((4, 4))
    lib().orc_ac_element(dim, C.c_double(rho_inf), C.c_double(dt), C.c_double(eps), C.c_double(gamma),
                         C.c_double(beta), _d(X4), _d(v4), _d(f4), _d(fr4), _d(fd4), _d(re), _d(Ke))
    return re[:nn].copy(), Ke[:nn, :nn].copy()


def b_element(dim, rho_inf, dt, X, v, afr, Bv, Bd):
    nn = dim + 1
    nv = 6 if dim == 3 else 3
    X4 = np.zeros((4, 3)); X4[:nn, :dim] = X
    v4 = np.zeros((4, 3)); v4[:nn, :dim] = v
    a4 = np.zeros(4); a4[:nn] = afr
    B4 = np.zeros(4 * nv); B4[:nn * nv] = np.asarray(Bv, dtype=np.float64).ravel()
    D4 = np.zeros(4 * nv); D4[:nn * nv] = np.asarray(Bd, dtype=np.float64).ravel()
    re = np.zeros((4, 6))
    Ke = np.zeros((4, 4, 6, 6))
    lib().orc_b_element(dim, C.c_double(rho_inf), C.c_double(dt), _d(X4), _d(v4), _d(a4), _d(B4), _d(D4),
                        _d(re), _d(Ke))
    return re[:nn, :nv].copy(), Ke[:nn, :nn, :nv, :nv].copy()


def l2_project(dim, xyz, conn, fq):
    """Appendix A projection of quadrature-point values fq [E][nq] to nodes."""
    xyz = _f64(xyz).reshape(-1, dim)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    fq = _f64(fq)
    out = np.zeros(xyz.shape[0])
    lib().orc_l2_project(dim, xyz.shape[0], conn.shape[0], _d(xyz), _i(conn), _d(fq), _d(out))
    return out


def quad_points(dim):
    """Barycentric coordinates of the degree-2 rule (same rule the C code
    uses), for building quadrature-point data in tests."""
    if dim == 1:
        s = 0.5 / np.sqrt(3.0)
        return np.array([[0.5 + s, 0.5 - s], [0.5 - s, 0.5 + s]])
    if dim == 2:
        return np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    a, b = (5 + 3 * np.sqrt(5)) / 20, (5 - np.sqrt(5)) / 20
    return np.full((4, 4), b) + np.eye(4) * (a - b)
