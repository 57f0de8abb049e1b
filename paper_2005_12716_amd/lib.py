"""ctypes binding of libswense.so (argument marshalling only).

Every computation runs in the HIP library; this module converts numpy host
arrays and torch device tensors to the plain pointers of the C ABI declared
in include/swense.h.  torch is imported first so that the library shares
torch's HIP runtime, device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswense.so")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ERANGE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
PHI, U, V, W, P, PHI_T, U_T, V_T, W_T, ETA, ETA_T = (1 << i for i in range(11))
ALL_FIELDS = (1 << 11) - 1
FIELD_BITS = [PHI, U, V, W, P, PHI_T, U_T, V_T, W_T, ETA, ETA_T]
PHYSICAL, SPECTRAL = 0, 1
KERNELS = ["yinv", "xpass", "yfwd", "yinv_eval", "xeval", "xeval_surf", "interp", "interp_div", "bind", "aux"]


class HosDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("lx", C.c_double), ("ly", C.c_double),
                ("depth", C.c_double), ("g", C.c_double), ("rho", C.c_double), ("order_m", C.c_int),
                ("dealias", C.c_int), ("precision", C.c_int), ("dt", C.c_double), ("t0", C.c_double)]


class GridDesc(C.Structure):
    _fields_ = [("gx", C.c_int), ("gy", C.c_int), ("ix0", C.c_int), ("iy0", C.c_int), ("wx", C.c_int),
                ("wy", C.c_int), ("nl", C.c_int), ("z", C.POINTER(C.c_double))]


class SeaDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("hs", C.c_double), ("kp", C.c_double), ("gamma", C.c_double),
                ("spreading", C.c_int), ("mode", C.c_int), ("ka", C.c_double)]


class StreamDesc(C.Structure):
    _fields_ = [("depth", C.c_double), ("height", C.c_double), ("wavelength", C.c_double), ("g", C.c_double),
                ("rho", C.c_double), ("n", C.c_int)]


class FnoDesc(C.Structure):
    _fields_ = [("n", C.c_int), ("channels", C.c_int), ("layers", C.c_int), ("p_modes", C.c_int),
                ("q_modes", C.c_int), ("hidden", C.c_int), ("in_channels", C.c_int), ("max_batch", C.c_int)]


class SurrogateDesc(C.Structure):
    _fields_ = [("stride_s", C.c_int), ("sigma_eta", C.c_double), ("sigma_phi", C.c_double), ("rho", C.c_double),
                ("tol", C.c_double), ("audit_every", C.c_int), ("cooldown", C.c_int), ("energy_tol", C.c_double),
                ("probation", C.c_int), ("base_substeps", C.c_int), ("drift_tol", C.c_double),
                ("base_only", C.c_int)]


class SurrogateStats(C.Structure):
    _fields_ = [("calls", C.c_longlong), ("surrogate_calls", C.c_longlong), ("hos_calls", C.c_longlong),
                ("audits", C.c_longlong), ("fallbacks", C.c_longlong), ("guard_trips", C.c_longlong),
                ("max_audit_err", C.c_double), ("last_audit_err", C.c_double), ("bound_calls", C.c_longlong),
                ("drift_est", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SwenseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"swense error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the built library; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2005_12716_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, dp, fp = C.c_void_p, C.POINTER(C.c_double), C.c_void_p
    sig = {
        "swense_version": (C.c_char_p, []),
        "swense_last_error": (C.c_char_p, [vp]),
        "swense_sea_spectrum": (C.c_int, [C.POINTER(HosDesc), C.POINTER(SeaDesc), vp, vp, vp]),
        "swense_hos_init": (C.c_int, [C.POINTER(HosDesc), vp, vp, C.c_int, vp, C.POINTER(vp)]),
        "swense_hos_workspace_bytes": (C.c_int, [C.POINTER(HosDesc), C.POINTER(C.c_size_t)]),
        "swense_hos_init_ws": (C.c_int, [C.POINTER(HosDesc), vp, vp, C.c_int, vp, vp, C.c_size_t, C.POINTER(vp)]),
        "swense_hos_set_state": (C.c_int, [vp, vp, vp, C.c_int, C.c_double]),
        "swense_hos_step": (C.c_int, [vp, C.c_int]),
        "swense_hos_tune_padding": (C.c_int, [C.POINTER(HosDesc), C.c_int, vp, C.POINTER(C.c_int), dp]),
        "swense_hos_step_exp": (C.c_int, [vp, C.c_double, C.c_int]),
        "swense_hos_get_state": (C.c_int, [vp, vp, vp, dp, C.c_int]),
        "swense_hos_rhs": (C.c_int, [vp, vp, vp]),
        "swense_hos_modes": (C.c_int, [vp, vp, vp, vp]),
        "swense_hos_energy": (C.c_int, [vp, dp]),
        "swense_eval_grid": (C.c_int, [vp, C.POINTER(GridDesc), C.c_uint, fp]),
        "swense_eval_grid_size": (C.c_size_t, [vp, C.POINTER(GridDesc), C.c_uint]),
        "swense_cells_bind": (C.c_int, [vp, C.POINTER(GridDesc), C.c_longlong, vp, C.POINTER(vp)]),
        "swense_cells_workspace_bytes": (C.c_int, [vp, C.POINTER(GridDesc), C.c_longlong, C.c_uint,
                                                   C.POINTER(C.c_size_t)]),
        "swense_cells_bind_ws": (C.c_int, [vp, C.POINTER(GridDesc), C.c_longlong, vp, C.c_uint, vp, C.c_size_t,
                                           C.POINTER(vp)]),
        "swense_interp_cells": (C.c_int, [vp, vp, C.c_uint, fp, C.POINTER(C.c_longlong)]),
        "swense_interp_cells_noalloc": (C.c_int, [vp, vp, C.c_uint, fp, C.POINTER(C.c_longlong)]),
        "swense_eval_points_direct": (C.c_int, [vp, C.c_longlong, vp, C.c_uint, vp]),
        "swense_hos_snapshot": (C.c_int, [vp]),
        "swense_stream_solve": (C.c_int, [C.POINTER(StreamDesc), vp]),
        "swense_stream_eval": (C.c_int, [C.POINTER(StreamDesc), vp, C.c_double, C.c_longlong, vp, C.c_uint, vp, vp]),
        "swense_hos_set_eval_time": (C.c_int, [vp, C.c_double]),
        "swense_cells_alpha": (C.c_int, [vp, C.c_longlong, vp, vp, vp, vp]),
        "swense_cells_pstar": (C.c_int, [vp, C.c_longlong, vp, vp, C.c_double, vp]),
        "swense_cells_relax": (C.c_int, [vp, C.c_longlong, C.c_int, vp, vp, vp, vp]),
        "swense_interp_divergence": (C.c_int, [vp, vp, fp]),
        "swense_interp_step": (C.c_int, [vp, vp, C.c_uint, fp, C.c_int]),
        "swense_fv_divergence": (C.c_int, [vp, C.POINTER(GridDesc), vp, C.c_int, vp, C.c_int, vp, C.c_int, fp,
                                           dp, dp]),
        "swense_profile_enable": (C.c_int, [vp, C.c_int]),
        "swense_profile_read": (C.c_int, [vp, C.c_int, dp, C.POINTER(C.c_longlong)]),
        "swense_profile_bytes": (C.c_int, [vp, C.c_int, dp]),
        "swense_profile_transform_bytes": (C.c_int, [vp, C.c_int, dp]),
        "swense_selfcheck_launch_geometry": (C.c_int, [C.c_int]),
        "swense_batch_create": (C.c_int, [C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_uint), C.POINTER(vp),
                                          C.c_int, C.c_int, vp, C.POINTER(vp)]),
        "swense_batch_run": (C.c_int, [vp]),
        "swense_batch_autotune": (C.c_int, [vp, C.c_char_p, C.POINTER(C.c_int), dp]),
        "swense_batch_last_error": (C.c_char_p, [vp]),
        "swense_batch_destroy": (None, [vp]),
        "swense_hos_destroy": (None, [vp]),
        "swense_cells_destroy": (None, [vp]),
        "swense_fno_param_count": (C.c_size_t, [C.POINTER(FnoDesc)]),
        "swense_fno_create": (C.c_int, [C.POINTER(FnoDesc), vp, vp, C.POINTER(vp)]),
        "swense_fno_forward": (C.c_int, [vp, vp, vp, C.c_int]),
        "swense_fno_loss": (C.c_int, [vp, vp, vp, vp, C.c_int, C.POINTER(C.c_float)]),
        "swense_fno_backward": (C.c_int, [vp, vp, vp, vp, C.c_int]),
        "swense_fno_train_step": (C.c_int, [vp, vp, vp, C.c_int, C.c_float, C.POINTER(C.c_float)]),
        "swense_fno_get": (C.c_int, [vp, C.c_int, vp]),
        "swense_fno_set": (C.c_int, [vp, C.c_int, vp]),
        "swense_fno_get_activations": (C.c_int, [vp, vp]),
        "swense_fno_set_trace": (C.c_int, [vp, vp]),
        "swense_fno_last_error": (C.c_char_p, [vp]),
        "swense_fno_destroy": (None, [vp]),
        "swense_gemm_bf16": (C.c_int, [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp]),
        "swense_surrogate_create": (C.c_int, [vp, vp, C.POINTER(SurrogateDesc), C.POINTER(vp)]),
        "swense_surrogate_features": (C.c_int, [vp, vp, vp]),
        "swense_surrogate_target": (C.c_int, [vp, vp, vp, vp]),
        "swense_surrogate_advance": (C.c_int, [vp, C.c_int, C.POINTER(SurrogateStats)]),
        "swense_surrogate_reset": (C.c_int, [vp]),
        "swense_surrogate_last_error": (C.c_char_p, [vp]),
        "swense_surrogate_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ["swense_version", "swense_last_error", "swense_sea_spectrum", "swense_hos_init",
            "swense_hos_workspace_bytes", "swense_hos_init_ws", "swense_cells_workspace_bytes", "swense_cells_bind_ws",
            "swense_hos_set_state", "swense_hos_step", "swense_hos_tune_padding", "swense_hos_step_exp", "swense_hos_get_state", "swense_hos_rhs",
            "swense_hos_modes", "swense_hos_energy", "swense_eval_grid", "swense_eval_grid_size",
            "swense_cells_bind", "swense_interp_cells", "swense_interp_cells_noalloc", "swense_eval_points_direct", "swense_hos_snapshot", "swense_hos_set_eval_time", "swense_stream_solve", "swense_stream_eval", "swense_cells_alpha", "swense_cells_pstar", "swense_cells_relax",
            "swense_interp_divergence", "swense_interp_step", "swense_fv_divergence", "swense_profile_enable",
            "swense_profile_read", "swense_profile_bytes", "swense_profile_transform_bytes",
            "swense_selfcheck_launch_geometry", "swense_batch_create", "swense_batch_run", "swense_batch_autotune",
            "swense_batch_last_error", "swense_batch_destroy", "swense_hos_destroy",
            "swense_cells_destroy", "swense_fno_param_count", "swense_fno_create", "swense_fno_forward",
            "swense_fno_loss", "swense_fno_backward", "swense_fno_train_step", "swense_fno_get", "swense_fno_set",
            "swense_fno_get_activations", "swense_fno_set_trace", "swense_fno_last_error", "swense_fno_destroy", "swense_gemm_bf16", "swense_surrogate_create",
            "swense_surrogate_features", "swense_surrogate_target", "swense_surrogate_advance", "swense_surrogate_reset",
            "swense_surrogate_last_error", "swense_surrogate_destroy"]


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def hos_desc(dim, nx, ny, lx, ly, depth, order_m=3, dt=0.1, g=1.0, rho=1.0, dealias=1, precision=0, t0=0.0):
    return HosDesc(dim, nx, ny, lx, ly, depth, g, rho, order_m, dealias, precision, dt, t0)


def tune_padding(desc, nsteps=3, stream=None):
    """Faster product-grid policy for this descriptor (1 or 2) and the timed
    ms per step of each (-1: not timed, the lengths coincide)."""
    best = C.c_int(0)
    ms = np.zeros(2)
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    rc = load().swense_hos_tune_padding(C.byref(desc), nsteps, C.c_void_p(st), C.byref(best),
                                        ms.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != OK:
        raise SwenseError(rc, "swense_hos_tune_padding failed")
    return best.value, ms


def grid_desc(gx, gy, z, window=None):
    z = np.ascontiguousarray(z, dtype=np.float64)
    ix0, iy0, wx, wy = window if window is not None else (0, 0, gx, gy)
    gd = GridDesc(gx, gy, ix0, iy0, wx, wy, z.size, z.ctypes.data_as(C.POINTER(C.c_double)))
    gd._z = z  # keep alive
    return gd


def stream_solve(depth, height, wavelength, n, g=1.0, rho=1.0):
    """Stream-function regular wave (host solve): (desc, sol[2n+4]) with sol =
    eta at the n+1 surface points (crest to trough), B_1..B_n, c, Q, R."""
    d = StreamDesc(depth, height, wavelength, g, rho, n)
    sol = np.zeros(2 * n + 4)
    rc = load().swense_stream_solve(C.byref(d), _ptr(sol))
    if rc != OK:
        raise SwenseError(rc, "stream_solve")
    return d, sol


def stream_eval(desc: StreamDesc, sol, t, xyz: torch.Tensor, mask, out=None):
    """Fields of `mask` of a solved regular wave at device FP64 points [3][n]
    and time t (FP64 [F][n], fields in bit order)."""
    assert xyz.is_cuda and xyz.dtype == torch.float64 and xyz.dim() == 2 and xyz.shape[0] == 3
    xyz = xyz.contiguous()
    n = xyz.shape[1]
    nf = bin(mask).count("1")
    if out is None:
        out = torch.empty((nf, n), dtype=torch.float64, device="cuda")
    sol = np.ascontiguousarray(sol, dtype=np.float64)
    st = torch.cuda.current_stream()
    rc = load().swense_stream_eval(C.byref(desc), _ptr(sol), float(t), n, _ptr(xyz), mask, _ptr(out),
                                   C.c_void_p(st.cuda_stream))
    if rc != OK:
        raise SwenseError(rc, "stream_eval")
    return out


def hos_workspace_bytes(desc: HosDesc):
    """Device bytes of a realisation's workspace (swense_hos_workspace_bytes)."""
    b = C.c_size_t()
    rc = load().swense_hos_workspace_bytes(C.byref(desc), C.byref(b))
    if rc != OK:
        raise SwenseError(rc, "hos_workspace_bytes")
    return b.value


def sea_spectrum(desc: HosDesc, kind=0, hs=0.0, kp=1.0, gamma=3.3, spreading=0, mode=0, ka=0.0, phases=None):
    """Initial half spectra (eta_hat, phis_hat) as complex128 [ny][nx/2+1]."""
    L = load()
    ny = 1 if desc.dim == 2 else desc.ny
    nxh = desc.nx // 2 + 1
    e = np.zeros((ny, nxh), dtype=np.complex128)
    p = np.zeros((ny, nxh), dtype=np.complex128)
    ph = None if phases is None else np.ascontiguousarray(phases, dtype=np.float64)
    sd = SeaDesc(kind, hs, kp, gamma, spreading, mode, ka)
    rc = L.swense_sea_spectrum(C.byref(desc), C.byref(sd), _ptr(ph), _ptr(e), _ptr(p))
    if rc != OK:
        raise SwenseError(rc, "sea_spectrum")
    return e, p


class Hos:
    """One HOS realisation on the current torch device and stream."""

    def __init__(self, desc: HosDesc, eta, phis, layout=SPECTRAL, stream=None, workspace=None):
        self.L = load()
        self.desc = desc
        self.ny = 1 if desc.dim == 2 else desc.ny
        self.nxh = desc.nx // 2 + 1
        eta = np.ascontiguousarray(eta, dtype=np.complex128 if layout == SPECTRAL else np.float64)
        phis = np.ascontiguousarray(phis, dtype=np.complex128 if layout == SPECTRAL else np.float64)
        st = stream if stream is not None else torch.cuda.current_stream()
        self.stream = st
        h = C.c_void_p()
        self.workspace = workspace
        if workspace is None:
            rc = self.L.swense_hos_init(C.byref(desc), _ptr(eta), _ptr(phis), layout, C.c_void_p(st.cuda_stream),
                                        C.byref(h))
        else:
            # caller-owned device memory (a torch uint8 buffer kept alive by this object)
            assert workspace.is_cuda and workspace.dtype == torch.uint8
            rc = self.L.swense_hos_init_ws(C.byref(desc), _ptr(eta), _ptr(phis), layout, C.c_void_p(st.cuda_stream),
                                           _ptr(workspace), workspace.numel(), C.byref(h))
        if rc != OK:
            raise SwenseError(rc, "hos_init")
        self.h = h

    def _check(self, rc, what):
        if rc not in (OK,):
            msg = self.L.swense_last_error(self.h)
            raise SwenseError(rc, f"{what}: {msg.decode() if msg else ''}")

    def step(self, n=1):
        self._check(self.L.swense_hos_step(self.h, n), "step")

    def step_exp(self, tau, nsub=1):
        """Advance by tau with nsub integrating-factor RK4 substeps."""
        self._check(self.L.swense_hos_step_exp(self.h, tau, nsub), "step_exp")

    def set_state(self, eta, phis, layout=SPECTRAL, t=0.0):
        eta = np.ascontiguousarray(eta, dtype=np.complex128 if layout == SPECTRAL else np.float64)
        phis = np.ascontiguousarray(phis, dtype=np.complex128 if layout == SPECTRAL else np.float64)
        self._check(self.L.swense_hos_set_state(self.h, _ptr(eta), _ptr(phis), layout, t), "set_state")

    def state(self, layout=SPECTRAL):
        if layout == SPECTRAL:
            e = np.zeros((self.ny, self.nxh), dtype=np.complex128)
            p = np.zeros_like(e)
        else:
            e = np.zeros((self.ny, self.desc.nx))
            p = np.zeros_like(e)
        t = C.c_double()
        self._check(self.L.swense_hos_get_state(self.h, _ptr(e), _ptr(p), C.byref(t), layout), "get_state")
        return e, p, t.value

    def rhs(self):
        e = np.zeros((self.ny, self.nxh), dtype=np.complex128)
        p = np.zeros_like(e)
        self._check(self.L.swense_hos_rhs(self.h, _ptr(e), _ptr(p)), "rhs")
        return e, p

    def modes(self):
        a = np.zeros((self.ny, self.nxh), dtype=np.complex128)
        at = np.zeros_like(a)
        et = np.zeros_like(a)
        self._check(self.L.swense_hos_modes(self.h, _ptr(a), _ptr(at), _ptr(et)), "modes")
        return a, at, et

    def energy(self):
        e = C.c_double()
        self._check(self.L.swense_hos_energy(self.h, C.byref(e)), "energy")
        return e.value

    def profile(self, enable=True):
        self._check(self.L.swense_profile_enable(self.h, 1 if enable else 0), "profile_enable")

    def profile_bytes(self):
        """{kernel class: compulsory HBM bytes of the recorded launches}."""
        out = {}
        for k, name in enumerate(KERNELS):
            b = C.c_double()
            self._check(self.L.swense_profile_bytes(self.h, k, C.byref(b)), "profile_bytes")
            out[name] = b.value
        return out

    def profile_transform_bytes(self):
        """{kernel class: two-pass transform-model bytes of the recorded launches}."""
        out = {}
        for k, name in enumerate(KERNELS):
            b = C.c_double()
            self._check(self.L.swense_profile_transform_bytes(self.h, k, C.byref(b)), "profile_transform_bytes")
            out[name] = b.value
        return out

    def profile_read(self):
        """{kernel class: (total ms, launches)} since profiling was enabled."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms = C.c_double()
            cnt = C.c_longlong()
            self._check(self.L.swense_profile_read(self.h, k, C.byref(ms), C.byref(cnt)), "profile_read")
            out[name] = (ms.value, cnt.value)
        return out

    def grid_size(self, gd, mask):
        return int(self.L.swense_eval_grid_size(self.h, C.byref(gd), mask))

    def eval_grid(self, gd, mask, out=None):
        n = self.grid_size(gd, mask)
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device="cuda")
        assert out.is_cuda and out.dtype == torch.float32 and out.numel() >= n
        self._check(self.L.swense_eval_grid(self.h, C.byref(gd), mask, _ptr(out)), "eval_grid")
        return out

    def snapshot(self):
        """Record the current spectra and time as the start of an interval."""
        self._check(self.L.swense_hos_snapshot(self.h), "snapshot")

    def set_eval_time(self, t):
        """Evaluate at time t in [snapshot time, current time] (Hermite in time)."""
        self._check(self.L.swense_hos_set_eval_time(self.h, float(t)), "set_eval_time")

    def eval_points_direct(self, xyz: torch.Tensor, mask, out=None):
        """Fields of `mask` at device FP64 points [3][n] by the modal sums
        themselves (FP64 [F][n], fields in bit order)."""
        assert xyz.is_cuda and xyz.dtype == torch.float64 and xyz.dim() == 2 and xyz.shape[0] == 3
        xyz = xyz.contiguous()
        n = xyz.shape[1]
        nf = bin(mask).count("1")
        if out is None:
            out = torch.empty((nf, n), dtype=torch.float64, device="cuda")
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == (nf, n)
        self._check(self.L.swense_eval_points_direct(self.h, n, _ptr(xyz), mask, _ptr(out)), "eval_points_direct")
        return out

    def cells_alpha(self, eta: torch.Tensor, zc: torch.Tensor, dz: torch.Tensor, out=None):
        """Incident volume fraction of cells (FP32 eta, dz; FP64 zc; all [n])."""
        n = eta.numel()
        for t, dt in ((eta, torch.float32), (zc, torch.float64), (dz, torch.float32)):
            assert t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == n
        out = torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out
        self._check(self.L.swense_cells_alpha(self.h, n, _ptr(eta), _ptr(zc), _ptr(dz), _ptr(out)), "cells_alpha")
        return out

    def cells_pstar(self, p: torch.Tensor, alpha: torch.Tensor, rho_air: float, out=None):
        """Modified incident pressure rho p / rho_water (FP32 [n])."""
        n = p.numel()
        for t in (p, alpha):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n
        out = torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out
        self._check(self.L.swense_cells_pstar(self.h, n, _ptr(p), _ptr(alpha), float(rho_air), _ptr(out)),
                    "cells_pstar")
        return out

    def cells_relax(self, x: torch.Tensor, alpha_i=None, alpha=None, uc=None):
        """Relaxation-zone blending in place (FP32): alpha [n] towards alpha_i,
        uc [ncomp][n] towards zero."""
        n = x.numel()
        ncomp = 0 if uc is None else uc.shape[0]
        for t in (x, alpha_i, alpha, uc):
            if t is not None:
                assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape[-1] == n
        self._check(self.L.swense_cells_relax(self.h, n, ncomp, _ptr(x), _ptr(alpha_i), _ptr(alpha), _ptr(uc)),
                    "cells_relax")

    def bind(self, gd, xyz: torch.Tensor, workspace=None, ws_mask=None):
        return Cells(self, gd, xyz, workspace, ws_mask)

    def cells_workspace_bytes(self, gd, n, mask=None):
        b = C.c_size_t()
        self._check(self.L.swense_cells_workspace_bytes(self.h, C.byref(gd), n, ALL_FIELDS if mask is None else mask,
                                                        C.byref(b)), "cells_workspace_bytes")
        return b.value

    def fv_divergence(self, gd, xe, ye, ze):
        """Finite-volume divergence on the structured mesh with edges xe, ye
        (None in 2D), ze: (div [nz][ny][nx] device FP32, rms, max |div|)."""
        xe = np.ascontiguousarray(xe, dtype=np.float64)
        ze = np.ascontiguousarray(ze, dtype=np.float64)
        ye = None if ye is None else np.ascontiguousarray(ye, dtype=np.float64)
        nx, nz = xe.size - 1, ze.size - 1
        ny = 1 if ye is None else ye.size - 1
        div = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
        rms, mx = C.c_double(), C.c_double()
        self._check(self.L.swense_fv_divergence(self.h, C.byref(gd), _ptr(xe), nx, _ptr(ye), ny, _ptr(ze), nz,
                                                _ptr(div), C.byref(rms), C.byref(mx)), "fv_divergence")
        return div, rms.value, mx.value

    def close(self):
        if getattr(self, "h", None):
            self.L.swense_hos_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cells:
    """A bound static point cloud (device FP64 coordinates [3][n])."""

    def __init__(self, hos: Hos, gd, xyz: torch.Tensor, workspace=None, ws_mask=None):
        assert xyz.is_cuda and xyz.dtype == torch.float64 and xyz.dim() == 2 and xyz.shape[0] == 3
        xyz = xyz.contiguous()
        self.hos = hos
        self.n = xyz.shape[1]
        c = C.c_void_p()
        self.workspace = workspace
        if workspace is None:
            rc = hos.L.swense_cells_bind(hos.h, C.byref(gd), self.n, _ptr(xyz), C.byref(c))
        else:
            assert workspace.is_cuda and workspace.dtype == torch.uint8
            rc = hos.L.swense_cells_bind_ws(hos.h, C.byref(gd), self.n, _ptr(xyz),
                                            ALL_FIELDS if ws_mask is None else ws_mask, _ptr(workspace),
                                            workspace.numel(), C.byref(c))
        hos._check(rc, "cells_bind")
        self.c = c
        self.gd = gd
        self._xyz = xyz

    @property
    def xyz_host(self):
        return self._xyz.cpu().numpy()

    def interp(self, mask, out=None, count=True):
        nf = bin(mask).count("1")
        if out is None:
            out = torch.empty((nf, self.n), dtype=torch.float32, device="cuda")
        nbad = C.c_longlong(-1)
        rc = self.hos.L.swense_interp_cells(self.hos.h, self.c, mask, _ptr(out), C.byref(nbad) if count else None)
        if rc not in (OK, ERANGE):
            self.hos._check(rc, "interp_cells")
        return out, (nbad.value if count else None)

    def interp_noalloc(self, mask, out=None, count=True):
        """swense_interp_cells_noalloc: the same fields with the library's
        fixed device scratch (no device allocation in the call)."""
        nf = bin(mask).count("1")
        if out is None:
            out = torch.empty((nf, self.n), dtype=torch.float32, device="cuda")
        nbad = C.c_longlong(-1)
        rc = self.hos.L.swense_interp_cells_noalloc(self.hos.h, self.c, mask, _ptr(out),
                                                     C.byref(nbad) if count else None)
        if rc not in (OK, ERANGE):
            self.hos._check(rc, "interp_cells_noalloc")
        return out, (nbad.value if count else None)

    def interp_step(self, mask, out=None, nsteps=1):
        """Fields of the current state into out while the state advances nsteps."""
        nf = bin(mask).count("1")
        if out is None:
            out = torch.empty((nf, self.n), dtype=torch.float32, device="cuda")
        self.hos._check(self.hos.L.swense_interp_step(self.hos.h, self.c, mask, _ptr(out), nsteps), "interp_step")
        return out

    def divergence(self, out=None):
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self.hos._check(self.hos.L.swense_interp_divergence(self.hos.h, self.c, _ptr(out)), "divergence")
        return out

    def close(self):
        if getattr(self, "c", None):
            self.hos.L.swense_cells_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many realisations advanced (and interpolated) by one graph launch."""

    def __init__(self, hoses, cells=None, masks=None, outs=None, nsteps=1, stream=None):
        self.L = load()
        n = len(hoses)
        self.hoses, self.cells_list, self.outs = list(hoses), cells, outs
        H = (C.c_void_p * n)(*[h.h for h in hoses])
        Cc = (C.c_void_p * n)(*[(c.c if c is not None else None) for c in cells]) if cells else None
        Mm = (C.c_uint * n)(*masks) if masks else None
        Oo = (C.c_void_p * n)(*[(o.data_ptr() if o is not None else None) for o in outs]) if outs else None
        st = stream if stream is not None else torch.cuda.current_stream()
        b = C.c_void_p()
        rc = self.L.swense_batch_create(H, Cc, Mm, Oo, n, nsteps, C.c_void_p(st.cuda_stream), C.byref(b))
        if rc != OK:
            raise SwenseError(rc, "batch_create")
        self.b = b

    def _check(self, rc, what):
        if rc != OK:
            msg = self.L.swense_batch_last_error(self.b)
            raise SwenseError(rc, f"{what}: {msg.decode() if msg else ''}")

    def run(self):
        self._check(self.L.swense_batch_run(self.b), "batch_run")

    def autotune(self, cache_path=None):
        k = C.c_int()
        ms = C.c_double()
        self._check(self.L.swense_batch_autotune(self.b, cache_path.encode() if cache_path else None,
                                                 C.byref(k), C.byref(ms)), "batch_autotune")
        return k.value, ms.value

    def close(self):
        if getattr(self, "b", None):
            self.L.swense_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- surrogate network

def fno_desc(n=256, channels=64, layers=8, p_modes=32, q_modes=31, hidden=128, max_batch=8, in_channels=2):
    return FnoDesc(n, channels, layers, p_modes, q_modes, hidden, in_channels, max_batch)


def fno_names(desc: FnoDesc):
    """Names and shapes of the packed parameter vector, in order."""
    C_, H = desc.channels, desc.hidden
    nq = 2 * desc.q_modes + 1
    out = [("W0", (C_, desc.in_channels)), ("b0", (C_,))]
    for l in range(1, desc.layers + 1):
        out += [(f"W{l}", (C_, C_)), (f"b{l}", (C_,)), (f"R{l}", (nq, desc.p_modes, C_, C_))]
    out += [("Q1", (H, C_)), ("c1", (H,)), ("Q2", (2, H)), ("c2", (2,))]
    return out


def fno_pack(desc: FnoDesc, params: dict) -> np.ndarray:
    """Dict of arrays (R complex) -> packed FP32 vector of the C ABI."""
    parts = []
    for name, shape in fno_names(desc):
        a = np.asarray(params[name])
        assert a.shape == shape, (name, a.shape, shape)
        if np.iscomplexobj(a):
            a = np.stack([a.real, a.imag], axis=-1)
        parts.append(a.astype(np.float32).ravel())
    v = np.concatenate(parts)
    assert v.size == load().swense_fno_param_count(C.byref(desc))
    return v


def fno_unpack(desc: FnoDesc, vec: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in fno_names(desc):
        if name.startswith("R"):
            m = int(np.prod(shape)) * 2
            a = vec[o:o + m].reshape(shape + (2,)).astype(np.float64)
            out[name] = a[..., 0] + 1j * a[..., 1]
        else:
            m = int(np.prod(shape))
            out[name] = vec[o:o + m].reshape(shape).astype(np.float64)
        o += m
    return out


def fno_init(desc: FnoDesc, seed: int) -> np.ndarray:
    """Seeded initial weights (packed FP32): pointwise weights ~ N(0, 1/fan_in),
    spectral weights uniform in [-1, 1] (re, im) / C^2, biases zero, the last
    projection scaled by 0.1."""
    rng = np.random.default_rng(seed)
    C_, H = desc.channels, desc.hidden
    nq = 2 * desc.q_modes + 1
    ci = desc.in_channels
    P = {"W0": rng.standard_normal((C_, ci)) / np.sqrt(ci), "b0": np.zeros(C_),
         "Q1": rng.standard_normal((H, C_)) / np.sqrt(C_), "c1": np.zeros(H),
         "Q2": rng.standard_normal((2, H)) / np.sqrt(H) * 0.1, "c2": np.zeros(2)}
    for l in range(1, desc.layers + 1):
        P[f"W{l}"] = rng.standard_normal((C_, C_)) / np.sqrt(C_)
        P[f"b{l}"] = np.zeros(C_)
        sh = (nq, desc.p_modes, C_, C_)
        P[f"R{l}"] = (rng.uniform(-1, 1, sh) + 1j * rng.uniform(-1, 1, sh)) / (C_ * C_)
    return fno_pack(desc, P)


class Fno:
    """Handle of the spectral neural operator (weights, Adam state, workspaces)."""

    def __init__(self, desc: FnoDesc, params: np.ndarray, stream=None):
        L = load()
        self.desc = desc
        st = stream if stream is not None else torch.cuda.current_stream()
        self.n_params = int(L.swense_fno_param_count(C.byref(desc)))
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.size == self.n_params
        h = C.c_void_p()
        rc = L.swense_fno_create(C.byref(desc), params.ctypes.data_as(C.c_void_p), C.c_void_p(st.cuda_stream),
                                 C.byref(h))
        if rc != OK:
            raise SwenseError(rc, "swense_fno_create failed")
        self.h = h

    def _check(self, rc, what):
        if rc != OK:
            raise SwenseError(rc, f"{what}: {load().swense_fno_last_error(self.h).decode()}")

    def forward(self, x: torch.Tensor, y: torch.Tensor = None) -> torch.Tensor:
        b = x.shape[0]
        if y is None:
            y = torch.empty((b, 2, self.desc.n, self.desc.n), dtype=torch.float32, device=x.device)
        self._check(load().swense_fno_forward(self.h, _ptr(x), _ptr(y), b), "forward")
        return y

    def loss(self, y, t, gy=None):
        if gy is None:
            gy = torch.empty_like(y)
        v = C.c_float()
        self._check(load().swense_fno_loss(self.h, _ptr(y), _ptr(t), _ptr(gy), y.shape[0], C.byref(v)), "loss")
        return v.value, gy

    def backward(self, x, gy, want_gx=False):
        gx = torch.empty_like(x) if want_gx else None
        self._check(load().swense_fno_backward(self.h, _ptr(x), _ptr(gy), _ptr(gx), x.shape[0]), "backward")
        return gx

    def train_step(self, x, t, lr):
        v = C.c_float()
        self._check(load().swense_fno_train_step(self.h, _ptr(x), _ptr(t), x.shape[0], lr, C.byref(v)), "train")
        return v.value

    def get(self, what=0) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(load().swense_fno_get(self.h, what, out.ctypes.data_as(C.c_void_p)), "get")
        return out

    def set(self, vec: np.ndarray, what=0):
        vec = np.ascontiguousarray(vec, dtype=np.float32)
        assert vec.size == self.n_params
        self._check(load().swense_fno_set(self.h, what, vec.ctypes.data_as(C.c_void_p)), "set")

    def activations(self, batch):
        """The last forward's activations (host FP32): v [L+1][batch][C][n][n],
        z [L][batch][C][n][n] (z[l-1] is layer l's pre-activation), zq and h
        [batch][H][n][n]."""
        d = self.desc
        C, H, n, L = d.channels, d.hidden, d.n, d.layers
        cblk, hblk = batch * C * n * n, batch * H * n * n
        buf = np.empty((2 * L + 1) * cblk + 2 * hblk, dtype=np.float32)
        self._check(load().swense_fno_get_activations(self.h, _ptr(buf)), "get_activations")
        v = buf[:(L + 1) * cblk].reshape(L + 1, batch, C, n, n)
        z = buf[(L + 1) * cblk:(2 * L + 1) * cblk].reshape(L, batch, C, n, n)
        o = (2 * L + 1) * cblk
        return {"v": v, "z": z, "zq": buf[o:o + hblk].reshape(batch, H, n, n),
                "h": buf[o + hblk:o + 2 * hblk].reshape(batch, H, n, n)}

    def set_trace(self, trace):
        """A device FP32 buffer of at least trace_floats() that later backward
        passes fill with dL/dz_1..dL/dz_L, dL/dv_0 and dL/dzq (None: off)."""
        self._trace = trace
        self._check(load().swense_fno_set_trace(self.h, _ptr(trace) if trace is not None else None), "set_trace")

    def trace_floats(self):
        d = self.desc
        return (d.layers + 1) * d.max_batch * d.channels * d.n * d.n + d.max_batch * d.hidden * d.n * d.n

    def close(self):
        if getattr(self, "h", None):
            load().swense_fno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """C = bf16(A) bf16(B) with FP32 accumulation (device FP32 row-major)."""
    M, K = a.shape
    K2, N = b.shape
    assert K == K2 and a.is_contiguous() and b.is_contiguous()
    c = torch.empty((M, N), dtype=torch.float32, device=a.device)
    rc = load().swense_gemm_bf16(M, N, K, _ptr(a), _ptr(b), _ptr(c), None)
    if rc != OK:
        raise SwenseError(rc, "swense_gemm_bf16 failed")
    return c


def surrogate_desc(stride_s=10, sigma_eta=1.0, sigma_phi=1.0, rho=1.0, tol=1e-3, audit_every=4, cooldown=4,
                   energy_tol=0.0, probation=2, base_substeps=0, drift_tol=None, base_only=False):
    """drift_tol defaults to tol (the accumulated error held to the same
    bound as one call's); 0 switches the bound off."""
    return SurrogateDesc(stride_s, sigma_eta, sigma_phi, rho, tol, audit_every, cooldown, energy_tol, probation,
                         base_substeps, tol if drift_tol is None else drift_tol, 1 if base_only else 0)


class Surrogate:
    """A network tied to one square realisation (same stream), advancing it
    with HOS as fallback and judge."""

    def __init__(self, hos: Hos, net: Fno, desc: SurrogateDesc):
        self.hos, self.net, self.desc = hos, net, desc
        self.n = net.desc.n
        h = C.c_void_p()
        rc = load().swense_surrogate_create(hos.h, net.h, C.byref(desc), C.byref(h))
        if rc != OK:
            raise SwenseError(rc, "swense_surrogate_create failed")
        self.h = h
        self.stats = SurrogateStats()

    def _check(self, rc, what):
        if rc != OK:
            raise SwenseError(rc, f"{what}: {load().swense_surrogate_last_error(self.h).decode()}")

    def features(self, x=None, lin=None, want_lin=True):
        dev = torch.device("cuda")
        if x is None:
            x = torch.empty((2, self.n, self.n), dtype=torch.float32, device=dev)
        if want_lin and lin is None:
            lin = torch.empty((2, self.n, self.n), dtype=torch.float32, device=dev)
        self._check(load().swense_surrogate_features(self.h, _ptr(x), _ptr(lin) if want_lin else None), "features")
        return x, lin

    def target(self, x_next, lin, t=None):
        if t is None:
            t = torch.empty_like(lin)
        self._check(load().swense_surrogate_target(self.h, _ptr(x_next), _ptr(lin), _ptr(t)), "target")
        return t

    def advance(self, ncalls):
        self._check(load().swense_surrogate_advance(self.h, ncalls, C.byref(self.stats)), "advance")
        return self.stats.as_dict()

    def reset(self):
        """New rollout: judge state and drift estimate cleared (stats too)."""
        self._check(load().swense_surrogate_reset(self.h), "reset")
        self.stats = SurrogateStats()

    def close(self):
        if getattr(self, "h", None):
            load().swense_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
