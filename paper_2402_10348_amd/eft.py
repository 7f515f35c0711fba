"""Python binding of include/eft.h (ctypes; argument marshalling only).

Device memory and streams come from PyTorch (ROCm build): every field or
vector is a contiguous float64 torch tensor on the GPU; the HIP library does
all of the work.  Importing this module loads ``_libeft.so`` and raises if it
is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_libeft.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, ENAN, EBAND_OVERFLOW, EUNSUPPORTED = range(9)
STATUS = {0: "EFT_OK", 1: "EFT_EINVAL", 2: "EFT_ENOMEM", 3: "EFT_EDEVICE", 4: "EFT_ENOTCONV",
          5: "EFT_EBREAKDOWN", 6: "EFT_ENAN", 7: "EFT_EBAND_OVERFLOW", 8: "EFT_EUNSUPPORTED"}

vp_ = C.c_void_p
dp = C.POINTER(C.c_double)


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("n_elems", C.c_int64),
                ("xyz", vp_), ("conn", vp_), ("n_dir", C.c_int64), ("dir_node", vp_), ("dir_mask", vp_),
                ("dir_val", vp_), ("grid", C.c_int32 * 3)]


class Phase(C.Structure):
    _fields_ = [("kind", C.c_int32), ("transported", C.c_int32), ("rho", C.c_double), ("mu", C.c_double),
                ("mu_L", C.c_double)]


class Materials(C.Structure):
    _fields_ = [("n_phases", C.c_int32), ("phase", vp_), ("g", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("rho_inf", C.c_double), ("eps", C.c_double), ("eta", C.c_double),
                ("C_I", C.c_double), ("di_cut", C.c_double), ("nl_rtol", C.c_double),
                ("nl_max", C.c_int32), ("nl_fixed", C.c_int32), ("lin_rtol", C.c_double),
                ("restart", C.c_int32), ("lin_maxit", C.c_int32), ("precond", C.c_int32),
                ("precision", C.c_int32), ("band_flat", C.c_double), ("band_cell", C.c_int32),
                ("band_halo", C.c_int32), ("mg_nu", C.c_int32), ("mg_omega", C.c_double),
                ("mg_bf16", C.c_int32), ("mg_nu_post", C.c_int32), ("mg_smoother", C.c_int32),
                ("band_sweeps", C.c_int32), ("band_omega", C.c_double), ("mg_galerkin", C.c_int32),
                ("nn_maxit", C.c_int32),
                ("band_reserve", C.c_double), ("graphs", C.c_int32),
                ("nn_base", C.c_int32), ("mg_lag", C.c_int32), ("mg_cnu", C.c_int32),
                ("mg_cnu_post", C.c_int32)]


class State(C.Structure):
    _fields_ = [("vp", vp_), ("vdot", vp_), ("phi", vp_), ("phidot", vp_), ("B", vp_), ("Bdot", vp_),
                ("t", C.c_double), ("step", C.c_int64)]


class Iterate(C.Structure):
    _fields_ = [("vp", vp_), ("phi", vp_), ("B", vp_)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("fallback_used", C.c_int32), ("rel_res0", C.c_double), ("rel_res", C.c_double)]


class TransportInfo(C.Structure):
    _fields_ = [("n_ind", C.c_int32), ("n_solid", C.c_int32), ("gamma", C.c_double * 64),
                ("beta", C.c_double * 64), ("band_nodes", C.c_int64 * 64), ("band_elems", C.c_int64 * 64),
                ("lin_iters", C.c_int32 * 128), ("ratio", C.c_double * 128), ("ac_iters", C.c_int32),
                ("b_iters", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("nl_iters", C.c_int32), ("converged", C.c_int32), ("lin_iters_total", C.c_int32),
                ("n_blocks", C.c_int32), ("block_ratio", C.c_double * 129), ("t_assemble", C.c_double),
                ("t_solve", C.c_double), ("t_transport", C.c_double), ("lin_iters_block", C.c_int32 * 129)]


class TuneInfo(C.Structure):
    _fields_ = [("evaluated", C.c_int32), ("from_cache", C.c_int32), ("default_seconds", C.c_double),
                ("best_seconds", C.c_double), ("default_iters", C.c_int32), ("best_iters", C.c_int32),
                ("band_default_seconds", C.c_double), ("band_best_seconds", C.c_double),
                ("mg_nu", C.c_int32), ("mg_nu_post", C.c_int32), ("mg_smoother", C.c_int32),
                ("mg_omega", C.c_double), ("mg_galerkin", C.c_int32), ("band_sweeps", C.c_int32),
                ("band_omega", C.c_double), ("mg_cnu", C.c_int32), ("mg_cnu_post", C.c_int32)]


class KernelTime(C.Structure):
    _fields_ = [("launches", C.c_int64), ("active", C.c_int64), ("seconds", C.c_double), ("bytes", C.c_double)]


EXPORTS = ["eft_create", "eft_destroy", "eft_last_error", "eft_set_params", "eft_ns_matrix", "eft_matrix_shape",
           "eft_matrix_export", "eft_matrix_import", "eft_assemble", "eft_spmv", "eft_fgmres", "eft_fgmres_noalloc", "eft_bands_build", "eft_band_export",
           "eft_band_system", "eft_transport_solids", "eft_step", "eft_tune", "eft_time_kernel",
           "eft_kernel_time_read", "eft_nn_init", "eft_nn_shape", "eft_nn_params", "eft_nn_harvest", "eft_nn_train",
           "eft_nn_loss_grad", "eft_nn_apply", "eft_center_of_mass", "eft_track_particles", "eft_init_phase",
           "eft_mg_export", "eft_ilu_export"]

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: run `python -m paper_2402_10348_amd.build`")
    L = C.CDLL(LIB_PATH)
    for name in EXPORTS:
        getattr(L, name).restype = C.c_int
    L.eft_last_error.restype = C.c_char_p
    L.eft_create.argtypes = [C.POINTER(Mesh), C.POINTER(Materials), C.POINTER(Params), vp_, C.POINTER(vp_)]
    L.eft_track_particles.argtypes = [vp_, vp_, C.c_int32, C.c_double, C.c_double, vp_, vp_]
    L.eft_init_phase.argtypes = [vp_, C.POINTER(Surface), C.c_double, vp_, C.c_double, vp_, vp_]
    _lib = L
    return L


class Surface(C.Structure):
    _fields_ = [("n_vert", C.c_int32), ("n_tri", C.c_int32), ("vert", C.c_void_p), ("tri", C.c_void_p)]


class EftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def params_struct(p, **over):
    vals = dict(dt=p.dt, rho_inf=p.rho_inf, eps=p.eps, eta=p.eta, C_I=p.C_I, di_cut=p.di_cut, nl_rtol=p.nl_rtol,
                nl_max=p.nl_max, nl_fixed=p.nl_fixed, lin_rtol=p.lin_rtol, restart=p.restart,
                lin_maxit=p.lin_maxit, precond=p.precond, precision=p.precision, band_flat=p.band_flat,
                band_cell=p.band_cell, band_halo=p.band_halo, mg_nu=p.mg_nu, mg_omega=p.mg_omega,
                mg_bf16=p.mg_bf16, mg_nu_post=p.mg_nu_post, mg_smoother=p.mg_smoother,
                band_sweeps=p.band_sweeps, band_omega=p.band_omega, mg_galerkin=p.mg_galerkin, nn_maxit=p.nn_maxit, band_reserve=p.band_reserve,
                graphs=p.graphs, nn_base=p.nn_base, mg_lag=p.mg_lag, mg_cnu=p.mg_cnu,
                mg_cnu_post=p.mg_cnu_post)
    vals.update(over)
    P = Params()
    for k, v in vals.items():
        setattr(P, k, v)
    return P


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


class Context:
    """One eft_ctx: a mesh, materials and parameters on the current GPU."""

    def __init__(self, prob, stream=None, **overrides):
        import torch
        self.torch = torch
        self.L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP library needs a device")
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.dim = prob.dim
        self.N = prob.n_nodes
        self.E = prob.n_elems
        self.bs = self.dim + 1
        self.nv = 6 if self.dim == 3 else 3
        self.n_ind = prob.n_ind
        self.n_s = prob.n_solid
        self._keep = dict(
            xyz=np.ascontiguousarray(prob.xyz, dtype=np.float64),
            conn=np.ascontiguousarray(prob.conn, dtype=np.int32),
            dir_node=np.ascontiguousarray(prob.dir_node, dtype=np.int32),
            dir_mask=np.ascontiguousarray(prob.dir_mask, dtype=np.uint8),
            dir_val=np.ascontiguousarray(prob.dir_val, dtype=np.float64))
        k = self._keep
        M = Mesh()
        M.dim, M.n_nodes, M.n_elems = self.dim, self.N, self.E
        M.xyz, M.conn = k["xyz"].ctypes.data, k["conn"].ctypes.data
        M.n_dir = k["dir_node"].shape[0]
        M.dir_node, M.dir_mask, M.dir_val = k["dir_node"].ctypes.data, k["dir_mask"].ctypes.data, k["dir_val"].ctypes.data
        for i in range(3):
            M.grid[i] = int(prob.grid[i])
        ph = (Phase * len(prob.phases))()
        for i, p in enumerate(prob.phases):
            ph[i].kind, ph[i].transported, ph[i].rho, ph[i].mu, ph[i].mu_L = p.kind, p.transported, p.rho, p.mu, p.mu_L
        mat = Materials()
        mat.n_phases = len(prob.phases)
        mat.phase = C.cast(ph, vp_)
        for i in range(3):
            mat.g[i] = float(prob.g[i])
        self.params = params_struct(prob.params, **overrides)
        if stream is None:
            stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.stream = stream
        self.ctx = vp_()
        st = self.L.eft_create(C.byref(M), C.byref(mat), C.byref(self.params), vp_(stream), C.byref(self.ctx))
        if st != OK:
            msg = self.L.eft_last_error(self.ctx).decode() if self.ctx else ""
            if self.ctx:
                self.L.eft_destroy(self.ctx)
            self.ctx = None
            raise EftError(st, msg)
        self.J = vp_()
        self._check(self.L.eft_ns_matrix(self.ctx, C.byref(self.J)))

    # -------------------------------------------------------------- helpers
    def _check(self, st, allow=()):
        if st != OK and st not in allow:
            raise EftError(st, self.L.eft_last_error(self.ctx).decode())
        return st

    def close(self):
        if getattr(self, "ctx", None):
            self.torch.cuda.synchronize()
            self.L.eft_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tensor(self, a, dtype=None):
        t = self.torch
        return t.as_tensor(np.ascontiguousarray(a), device=self.dev, dtype=dtype or t.float64).contiguous()

    def device_state(self, st):
        """Dict of numpy arrays (vp, vdot, phi, phidot, B, Bdot) -> device tensors."""
        return {k: self.tensor(st[k]) for k in ("vp", "vdot", "phi", "phidot", "B", "Bdot") if k in st}

    def _state(self, d, t=0.0, step=0):
        S = State()
        for k in ("vp", "vdot", "phi", "phidot", "B", "Bdot"):
            v = d.get(k)
            setattr(S, k, _ptr(v) if v is not None and v.numel() else None)
        S.t, S.step = t, step
        return S

    def _iterate(self, d):
        I = Iterate()
        for k in ("vp", "phi", "B"):
            v = d.get(k)
            setattr(I, k, _ptr(v) if v is not None and v.numel() else None)
        return I

    def set_params(self, **over):
        p = self.params
        for k, v in over.items():
            setattr(p, k, v)
        self._check(self.L.eft_set_params(self.ctx, C.byref(p)))

    def tune(self, st, cache_path=None, budget=0):
        """Autotune the solver's run-time knobs on the device state dict st
        (unchanged); returns the outcome and keeps the chosen knobs."""
        S = self._state(st)
        out = TuneInfo()
        cp = cache_path.encode() if cache_path else None
        self._check(self.L.eft_tune(self.ctx, C.byref(S), C.c_char_p(cp) if cp else None, C.c_int32(budget),
                                    C.byref(out)))
        for k in ("mg_nu", "mg_nu_post", "mg_smoother", "mg_omega", "mg_galerkin", "band_sweeps", "band_omega"):
            setattr(self.params, k, getattr(out, k))
        return {f[0]: getattr(out, f[0]) for f in TuneInfo._fields_}

    def time_kernel(self, *roles):
        """Start HIP-event timing of kernel roles (1 fine-level smoother
        sweep, 2 momentum SpMV inside FGMRES, 3 momentum/mass assembly); no
        roles turns timing off.  Resets the counters."""
        mask = 0
        for r in roles:
            mask |= 1 << r
        self._check(self.L.eft_time_kernel(self.ctx, C.c_int32(mask)))

    def kernel_time(self, role):
        out = KernelTime()
        self._check(self.L.eft_kernel_time_read(self.ctx, C.c_int32(role), C.byref(out)))
        return dict(launches=out.launches, active=out.active, seconds=out.seconds, bytes=out.bytes)

    # ---------------------------------------------- learned preconditioner
    def nn_init(self, seed=0):
        self._check(self.L.eft_nn_init(self.ctx, C.c_uint64(seed)))

    def nn_shape(self):
        h, l, npar, pairs = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        self._check(self.L.eft_nn_shape(self.ctx, C.byref(h), C.byref(l), C.byref(npar), C.byref(pairs)))
        return dict(hidden=h.value, layers=l.value, n_params=npar.value, pairs=pairs.value)

    def nn_params(self, theta=None):
        """Export the parameters (theta None) or import theta (FP32 array)."""
        n = self.nn_shape()["n_params"]
        if theta is None:
            out = np.zeros(n, dtype=np.float32)
            self._check(self.L.eft_nn_params(self.ctx, out.ctypes.data_as(C.POINTER(C.c_float)), C.c_int64(n), 0))
            return out
        th = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(self.L.eft_nn_params(self.ctx, th.ctypes.data_as(C.POINTER(C.c_float)), C.c_int64(th.size), 1))

    def nn_harvest(self, capacity):
        self._check(self.L.eft_nn_harvest(self.ctx, C.c_int32(capacity)))

    def nn_train(self, steps, batch=1, lr=1e-3, seed=0):
        losses = np.zeros(max(steps, 1))
        self._check(self.L.eft_nn_train(self.ctx, C.c_int32(steps), C.c_int32(batch), C.c_double(lr),
                                        C.c_uint64(seed), losses.ctypes.data_as(C.POINTER(C.c_double))))
        return losses[:steps]

    def nn_loss_grad(self, u, e):
        n = self.nn_shape()["n_params"]
        g = np.zeros(n, dtype=np.float32)
        loss = C.c_double()
        self._check(self.L.eft_nn_loss_grad(self.ctx, _ptr(u), _ptr(e), g.ctypes.data_as(C.POINTER(C.c_float)),
                                            C.byref(loss)))
        return loss.value, g

    def nn_apply(self, u):
        z = self.torch.empty_like(u)
        self._check(self.L.eft_nn_apply(self.ctx, _ptr(u), _ptr(z)))
        return z

    # ------------------------------------------------------------- the ABI
    def assemble(self, lvl, it, with_J=True):
        """Residual [N][d+1] (and the context Jacobian) at the iterate."""
        R = self.torch.empty((self.N, self.bs), dtype=self.torch.float64, device=self.dev)
        S, I = self._state(lvl), self._iterate(it)
        self._check(self.L.eft_assemble(self.ctx, C.byref(S), C.byref(I), _ptr(R), self.J if with_J else None))
        return R

    def matrix_shape(self):
        n, nnz, bs = C.c_int64(), C.c_int64(), C.c_int32()
        self._check(self.L.eft_matrix_shape(self.J, C.byref(n), C.byref(nnz), C.byref(bs)))
        return n.value, nnz.value, bs.value

    def matrix(self):
        """(rowptr, col, val[nnzb][bs][bs]) of the momentum Jacobian as device tensors."""
        t = self.torch
        n, nnz, bs = self.matrix_shape()
        rowptr = t.empty(n + 1, dtype=t.int32, device=self.dev)
        col = t.empty(nnz, dtype=t.int32, device=self.dev)
        val = t.empty((nnz, bs, bs), dtype=t.float64, device=self.dev)
        self._check(self.L.eft_matrix_export(self.ctx, self.J, _ptr(rowptr), _ptr(col), _ptr(val)))
        return rowptr, col, val

    def matrix_import(self, val):
        """Overwrite the context matrix's values with val [nnzb][bs][bs] (device FP64)."""
        self._check(self.L.eft_matrix_import(self.ctx, self.J, _ptr(val.contiguous())))

    def mg_level(self, level):
        """(rowptr, col, val[nnzb][bs][bs]) of multigrid level `level` (device
        tensors, FP64) and the number of levels."""
        t = self.torch
        nl, n, nnz = C.c_int32(), C.c_int64(), C.c_int64()
        self._check(self.L.eft_mg_export(self.ctx, C.c_int32(level), C.byref(nl), C.byref(n), C.byref(nnz),
                                         None, None, None))
        rowptr = t.empty(n.value + 1, dtype=t.int32, device=self.dev)
        col = t.empty(nnz.value, dtype=t.int32, device=self.dev)
        val = t.empty((nnz.value, self.bs, self.bs), dtype=t.float64, device=self.dev)
        self._check(self.L.eft_mg_export(self.ctx, C.c_int32(level), None, None, None, _ptr(rowptr), _ptr(col),
                                         _ptr(val)))
        return rowptr, col, val, nl.value

    def ilu_factors(self):
        """Block ILU(0) factors of the current momentum matrix (precond = 3):
        (lu [nnzb][bs*bs], dinv [n][bs*bs]) device tensors."""
        n, nnz, bs = self.matrix_shape()
        lu = self.torch.empty((nnz, bs * bs), dtype=self.torch.float64, device=self.dev)
        dinv = self.torch.empty((n, bs * bs), dtype=self.torch.float64, device=self.dev)
        self._check(self.L.eft_ilu_export(self.ctx, _ptr(lu), _ptr(dinv)))
        return lu, dinv
    def spmv(self, x, y=None):
        if y is None:
            y = self.torch.empty_like(x)
        self._check(self.L.eft_spmv(self.ctx, self.J, _ptr(x), _ptr(y)))
        return y

    def fgmres(self, b, x=None):
        if x is None:
            x = self.torch.empty_like(b)
        info = SolveInfo()
        st = self._check(self.L.eft_fgmres(self.ctx, self.J, _ptr(b), _ptr(x), C.byref(info)), allow=(ENOTCONV,))
        return x, dict(status=st, iters=info.iters, restarts=info.restarts, converged=info.converged,
                       rel_res=info.rel_res, fallback=info.fallback_used)

    def fgmres_noalloc(self, b, x=None):
        """eft_fgmres with the Krylov workspace in the library's fixed device
        array (allocates nothing)."""
        if x is None:
            x = self.torch.empty_like(b)
        info = SolveInfo()
        st = self._check(self.L.eft_fgmres_noalloc(self.ctx, self.J, _ptr(b), _ptr(x), C.byref(info)),
                         allow=(ENOTCONV,))
        return x, dict(status=st, iters=info.iters, restarts=info.restarts, converged=info.converged,
                       rel_res=info.rel_res, fallback=info.fallback_used)

    def bands_build(self, lvl):
        self._check(self.L.eft_bands_build(self.ctx, C.byref(self._state(lvl))))

    def band_export(self, k):
        t = self.torch
        be = t.empty(self.E, dtype=t.uint8, device=self.dev)
        fr = t.empty(self.N, dtype=t.uint8, device=self.dev)
        self._check(self.L.eft_band_export(self.ctx, k, _ptr(be), _ptr(fr)))
        return be, fr

    def band_system(self, lvl, it, kind, index):
        """Assembled band system (test hook): dict with node, rowptr, col, R, J
        (device tensors) and gamma, beta for kind 0 (Allen-Cahn)."""
        t = self.torch
        S, I = self._state(lvl), self._iterate(it)
        n, nnz = C.c_int64(), C.c_int64()
        self._check(self.L.eft_band_system(self.ctx, C.byref(S), C.byref(I), kind, index, C.byref(n), C.byref(nnz),
                                           None, None, None, None, None, None))
        bs = 1 if kind == 0 else self.nv
        n, nnz = n.value, nnz.value
        node = t.empty(max(n, 1), dtype=t.int32, device=self.dev)
        rowptr = t.empty(n + 1, dtype=t.int32, device=self.dev)
        col = t.empty(max(nnz, 1), dtype=t.int32, device=self.dev)
        R = t.empty((max(n, 1), bs), dtype=t.float64, device=self.dev)
        J = t.empty((max(nnz, 1), bs, bs), dtype=t.float64, device=self.dev)
        gb = (C.c_double * 2)()
        self._check(self.L.eft_band_system(self.ctx, C.byref(S), C.byref(I), kind, index, C.byref(C.c_int64(n)),
                                           C.byref(C.c_int64(nnz)), _ptr(node), _ptr(rowptr), _ptr(col), _ptr(R),
                                           _ptr(J), gb))
        return dict(node=node[:n], rowptr=rowptr, col=col[:nnz], R=R[:n], J=J[:nnz], gamma=gb[0], beta=gb[1])

    def transport(self, lvl, it):
        info = TransportInfo()
        S, I = self._state(lvl), self._iterate(it)
        st = self._check(self.L.eft_transport_solids(self.ctx, C.byref(S), C.byref(I), C.byref(info)),
                         allow=(ENOTCONV,))
        ni, ns = info.n_ind, info.n_solid
        return dict(status=st, gamma=list(info.gamma[:ni]), beta=list(info.beta[:ni]),
                    band_nodes=list(info.band_nodes[:ni]), band_elems=list(info.band_elems[:ni]),
                    lin_iters=list(info.lin_iters[:ni + ns]), ratio=list(info.ratio[:ni + ns]),
                    ac_iters=info.ac_iters, b_iters=info.b_iters)

    def center_of_mass(self, phi):
        """Centre of mass [n_ind][dim] and measure int alpha dOmega [n_ind] of
        the region of every order parameter of phi [n_ind][N] (device)."""
        import numpy as np
        K = self.n_ind
        xc = np.zeros((max(K, 1), 3))
        m = np.zeros(max(K, 1))
        self._check(self.L.eft_center_of_mass(self.ctx, _ptr(phi), xc.ctypes.data_as(C.c_void_p),
                                               m.ctypes.data_as(C.c_void_p)))
        return xc[:K, :self.dim].copy(), m[:K].copy()

    def track_particles(self, vp, x, dt, tol=1e-10):
        """One explicit step of the particles x [n_p][dim] (host) in the
        velocity of vp [N][dim+1] (device); returns (x_new, element or -1)."""
        import numpy as np
        xx = np.ascontiguousarray(np.array(x, dtype=np.float64).reshape(-1, self.dim))
        el = np.zeros(xx.shape[0], dtype=np.int32)
        self._check(self.L.eft_track_particles(self.ctx, _ptr(vp), xx.shape[0], float(dt), float(tol),
                                                xx.ctypes.data_as(C.c_void_p), el.ctypes.data_as(C.c_void_p)))
        return xx, el

    def init_phase(self, vert, tri, eps, ncell, chi=1e-12):
        """Order parameter [N] (device tensor) of the solid inside the closed
        surface (vert [nv][3], tri [nt][3], host); returns (phi, crossings)."""
        import numpy as np
        v = np.ascontiguousarray(vert, dtype=np.float64)
        t = np.ascontiguousarray(tri, dtype=np.int32)
        nc = np.ascontiguousarray(ncell, dtype=np.int32)
        S = Surface(v.shape[0], t.shape[0], v.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p))
        phi = self.torch.empty(self.N, dtype=self.torch.float64, device=self.dev)
        cr = np.zeros(2, dtype=np.int32)
        self._check(self.L.eft_init_phase(self.ctx, C.byref(S), float(eps), nc.ctypes.data_as(C.c_void_p),
                                           float(chi), _ptr(phi), cr.ctypes.data_as(C.c_void_p)))
        return phi, cr

    def step(self, st, t=0.0, step=0, dt=0.0):
        """Advance the device state dict in place by one time step."""
        S = self._state(st, t, step)
        info = StepInfo()
        self._check(self.L.eft_step(self.ctx, C.byref(S), C.c_double(dt), C.byref(info)))
        nb = info.n_blocks
        return dict(nl_iters=info.nl_iters, converged=info.converged, lin_iters_total=info.lin_iters_total,
                    block_ratio=list(info.block_ratio[:nb]), t_assemble=info.t_assemble, t_solve=info.t_solve,
                    t_transport=info.t_transport, t=S.t, step=S.step,
                    lin_iters_block=list(info.lin_iters_block[:nb]))
