"""ctypes binding of libcdg2.so (C ABI in include/cdg2.h).

Argument marshalling only: every step of the operator runs in the HIP library.
torch tensors are used for device memory and streams.  The functions keep the
C names (cdg2_create, cdg2_apply_operator, ...); :class:`Operator` wraps a handle.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdg2.so")

CDG2_OK, CDG2_EINVAL, CDG2_ENOMEM, CDG2_EHIP, CDG2_ENONFINITE, CDG2_EDOMAIN = 0, -1, -2, -3, -4, -5
CDG2_ENOCONV = -6
CDG2_FP64, CDG2_FP32 = 0, 1
CDG2_LLF_ALL, CDG2_LLF_CELLS = 0, 1
CDG2_FLUX_CDG2, CDG2_FLUX_BR2, CDG2_FLUX_IP, CDG2_FLUX_BO, CDG2_FLUX_CDG = 0, 1, 2, 3, 4
FLUXES = {"cdg2": CDG2_FLUX_CDG2, "br2": CDG2_FLUX_BR2, "ip": CDG2_FLUX_IP, "bo": CDG2_FLUX_BO,
          "cdg": CDG2_FLUX_CDG}

COEFF_NAMES = [
    "mu1", "mu2", "mu3", "nu1", "nu2", "nu3",
    "chi0_11", "chi0_13", "chi0_21", "chi0_22",
    "chith_11", "chith_13", "chith_21", "chith_22",
    "d1", "d2", "gamma", "alpha1", "alpha2", "f1", "k",
    "beta1", "beta2", "sigma", "c1_star", "c1_sstar",
]

_d = ctypes.c_double


class cdg2_coeffs(ctypes.Structure):
    _fields_ = [("mu", _d * 3), ("nu", _d * 3), ("chi0", _d * 4), ("chith", _d * 4),
                ("d1", _d), ("d2", _d), ("gamma", _d), ("alpha1", _d), ("alpha2", _d),
                ("f1", _d), ("k", _d), ("beta1", _d), ("beta2", _d), ("sigma", _d),
                ("c1_star", _d), ("c1_sstar", _d)]


class cdg2_config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("order", ctypes.c_int),
                ("precision", ctypes.c_int), ("wall_axis", ctypes.c_int),
                ("llf_mode", ctypes.c_int), ("gamma1_in", _d * 2), ("coeffs", cdg2_coeffs),
                ("diff_flux", ctypes.c_int), ("reserved", ctypes.c_int), ("flux_eta", _d)]


class cdg2_implicit_opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("max_newton", ctypes.c_int), ("krylov_dim", ctypes.c_int),
                ("newton_rtol", _d), ("krylov_rtol", _d)]


class cdg2_implicit_stats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("krylov_iters", ctypes.c_int),
                ("converged", ctypes.c_int), ("pad", ctypes.c_int), ("max_residual", _d)]


class CDG2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cdg2 error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libcdg2.so; raise if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1403_1157_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.cdg2_create.argtypes = [ctypes.POINTER(cdg2_config), ctypes.POINTER(P)]
    L.cdg2_destroy.argtypes = [P]
    L.cdg2_set_stream.argtypes = [P, P]
    L.cdg2_set_coeffs.argtypes = [P, ctypes.POINTER(cdg2_coeffs)]
    L.cdg2_num_dofs.argtypes = [P]
    L.cdg2_num_dofs.restype = ctypes.c_size_t
    L.cdg2_apply_operator.argtypes = [P, P, P]
    L.cdg2_rk_step.argtypes = [P, P, _d, ctypes.c_int]
    L.cdg2_rk_step_noalloc.argtypes = [P, P, _d, ctypes.c_int]
    L.cdg2_max_dt.argtypes = [P, P, _d, ctypes.POINTER(_d)]
    L.cdg2_sync.argtypes = [P]
    L.cdg2_rho_hat.argtypes = [P]
    L.cdg2_rho_hat.restype = _d
    L.cdg2_apply_adjoint.argtypes = [P, P, P, P, ctypes.POINTER(_d)]
    L.cdg2_rk_step_adjoint.argtypes = [P, P, P, P, _d, ctypes.POINTER(_d)]
    L.cdg2_rk_adjoint_segment.argtypes = [P, P, ctypes.c_int, _d, P, ctypes.POINTER(_d)]
    L.cdg2_dirk_step.argtypes = [P, P, _d, ctypes.POINTER(cdg2_implicit_opts),
                                 ctypes.POINTER(cdg2_implicit_stats)]
    L.cdg2_batch_create.argtypes = [ctypes.POINTER(cdg2_config), ctypes.c_int, ctypes.c_int, ctypes.POINTER(P)]
    L.cdg2_batch_autotune.argtypes = [P, ctypes.POINTER(_d)]
    L.cdg2_batch_set_graph.argtypes = [P, ctypes.c_int]
    L.cdg2_batch_destroy.argtypes = [P]
    L.cdg2_batch_set_stream.argtypes = [P, P]
    L.cdg2_batch_num_dofs.argtypes = [P]
    L.cdg2_batch_num_dofs.restype = ctypes.c_size_t
    L.cdg2_batch_offset.argtypes = [P, ctypes.c_int]
    L.cdg2_batch_offset.restype = ctypes.c_size_t
    L.cdg2_batch_set_schedule.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.cdg2_batch_rk.argtypes = [P, P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_d), ctypes.c_int]
    L.cdg2_batch_sync.argtypes = [P]
    L.cdg2_tri_create.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.POINTER(cdg2_coeffs), _d, _d,
                                  ctypes.POINTER(P)]
    L.cdg2_tri_destroy.argtypes = [P]
    L.cdg2_tri_set_stream.argtypes = [P, P]
    L.cdg2_tri_num_dofs.argtypes = [P]
    L.cdg2_tri_num_dofs.restype = ctypes.c_size_t
    L.cdg2_tri_apply_operator.argtypes = [P, P, P]
    L.cdg2_tri_rk_step.argtypes = [P, P, _d, ctypes.c_int]
    L.cdg2_tri_sync.argtypes = [P]
    L.cdg2_tet_create.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.POINTER(cdg2_coeffs), _d, _d,
                                  ctypes.POINTER(P)]
    L.cdg2_tet_destroy.argtypes = [P]
    L.cdg2_tet_set_stream.argtypes = [P, P]
    L.cdg2_tet_num_dofs.argtypes = [P]
    L.cdg2_tet_num_dofs.restype = ctypes.c_size_t
    L.cdg2_tet_apply_operator.argtypes = [P, P, P]
    L.cdg2_tet_rk_step.argtypes = [P, P, _d, ctypes.c_int]
    L.cdg2_tet_sync.argtypes = [P]
    L.cdg2_last_error.argtypes = []
    L.cdg2_last_error.restype = ctypes.c_char_p
    for name in ("cdg2_create", "cdg2_destroy", "cdg2_set_stream", "cdg2_set_coeffs",
                 "cdg2_apply_operator", "cdg2_rk_step", "cdg2_rk_step_noalloc", "cdg2_max_dt", "cdg2_sync",
                 "cdg2_apply_adjoint", "cdg2_rk_step_adjoint", "cdg2_rk_adjoint_segment",
                 "cdg2_dirk_step",
                 "cdg2_batch_create",
                 "cdg2_batch_destroy", "cdg2_batch_set_stream", "cdg2_batch_set_schedule",
                 "cdg2_batch_rk", "cdg2_batch_sync", "cdg2_batch_autotune", "cdg2_batch_set_graph",
                 "cdg2_tri_create", "cdg2_tri_destroy", "cdg2_tri_set_stream", "cdg2_tri_apply_operator",
                 "cdg2_tri_rk_step", "cdg2_tri_sync", "cdg2_tet_create", "cdg2_tet_destroy",
                 "cdg2_tet_set_stream", "cdg2_tet_apply_operator", "cdg2_tet_rk_step", "cdg2_tet_sync"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != CDG2_OK:
        raise CDG2Error(rc, lib().cdg2_last_error().decode())


def make_coeffs(c: dict) -> cdg2_coeffs:
    v = [float(c[k]) for k in COEFF_NAMES]
    s = cdg2_coeffs()
    s.mu[:] = v[0:3]
    s.nu[:] = v[3:6]
    s.chi0[:] = v[6:10]
    s.chith[:] = v[10:14]
    (s.d1, s.d2, s.gamma, s.alpha1, s.alpha2, s.f1, s.k,
     s.beta1, s.beta2, s.sigma, s.c1_star, s.c1_sstar) = v[14:26]
    return s


def make_config(dim: int, n, order: int, coeffs: dict, precision: str = "fp64",
                wall_axis: int | None = None, llf_mode: str = "all",
                gamma1_in=(0.0, 1.0), diff_flux: str = "cdg2", flux_eta: float = 0.0) -> cdg2_config:
    cfg = cdg2_config()
    cfg.dim = int(dim)
    nn = list(n) + [1] * (3 - len(n))
    cfg.n[:] = [int(v) for v in nn[:3]]
    cfg.order = int(order)
    cfg.precision = CDG2_FP32 if precision == "fp32" else CDG2_FP64
    cfg.wall_axis = dim - 1 if wall_axis is None else int(wall_axis)
    cfg.llf_mode = CDG2_LLF_CELLS if llf_mode == "cells" else CDG2_LLF_ALL
    cfg.gamma1_in[:] = [float(gamma1_in[0]), float(gamma1_in[1])]
    cfg.coeffs = make_coeffs(coeffs)
    cfg.diff_flux = FLUXES[diff_flux]
    cfg.flux_eta = float(flux_eta)
    return cfg


# ---- C-named entry points ----------------------------------------------------

def cdg2_create(cfg: cdg2_config) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().cdg2_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def cdg2_destroy(h) -> None:
    _check(lib().cdg2_destroy(h))


def cdg2_set_stream(h, stream: int) -> None:
    _check(lib().cdg2_set_stream(h, ctypes.c_void_p(stream)))


def cdg2_set_coeffs(h, c: dict) -> None:
    s = make_coeffs(c)
    _check(lib().cdg2_set_coeffs(h, ctypes.byref(s)))


def cdg2_num_dofs(h) -> int:
    return int(lib().cdg2_num_dofs(h))


def cdg2_apply_operator(h, U_ptr: int, out_ptr: int) -> None:
    _check(lib().cdg2_apply_operator(h, ctypes.c_void_p(U_ptr), ctypes.c_void_p(out_ptr)))


def cdg2_rk_step(h, U_ptr: int, dt: float, nsteps: int) -> None:
    _check(lib().cdg2_rk_step(h, ctypes.c_void_p(U_ptr), float(dt), int(nsteps)))


def cdg2_rk_step_noalloc(h, U_ptr: int, dt: float, nsteps: int) -> None:
    _check(lib().cdg2_rk_step_noalloc(h, ctypes.c_void_p(U_ptr), float(dt), int(nsteps)))


def cdg2_max_dt(h, U_ptr: int, cfl: float) -> float:
    dt = _d()
    _check(lib().cdg2_max_dt(h, ctypes.c_void_p(U_ptr), float(cfl), ctypes.byref(dt)))
    return dt.value


def cdg2_apply_adjoint(h, U_ptr: int, w_ptr: int, out_ptr: int, want_theta: bool = False):
    """Returns the 21 parameter derivatives (list) when want_theta, else None."""
    arr = (_d * 21)() if want_theta else None
    _check(lib().cdg2_apply_adjoint(h, ctypes.c_void_p(U_ptr), ctypes.c_void_p(w_ptr),
                                    ctypes.c_void_p(out_ptr), arr))
    return list(arr) if want_theta else None


def cdg2_rk_step_adjoint(h, Un_ptr: int, lam_np1_ptr: int, lam_n_ptr: int, dt: float,
                         dtheta_acc_ptr: int = 0):
    """dtheta_acc_ptr: 0 or the device address of 21 float64 accumulators."""
    _check(lib().cdg2_rk_step_adjoint(h, ctypes.c_void_p(Un_ptr), ctypes.c_void_p(lam_np1_ptr),
                                      ctypes.c_void_p(lam_n_ptr), float(dt),
                                      ctypes.cast(ctypes.c_void_p(dtheta_acc_ptr or None),
                                                  ctypes.POINTER(_d))))


def cdg2_rk_adjoint_segment(h, U_start_ptr: int, nsteps: int, dt: float, lam_ptr: int,
                            dtheta_acc_ptr: int = 0):
    """lam_ptr: device buffer, dL/dU at the end of the segment in, at its start out;
    dtheta_acc_ptr: 0 or the device address of 21 float64 accumulators."""
    _check(lib().cdg2_rk_adjoint_segment(h, ctypes.c_void_p(U_start_ptr), int(nsteps), float(dt),
                                         ctypes.c_void_p(lam_ptr),
                                         ctypes.cast(ctypes.c_void_p(dtheta_acc_ptr or None),
                                                     ctypes.POINTER(_d))))


def cdg2_dirk_step(h, U_ptr: int, dt: float, opts: cdg2_implicit_opts | None = None) -> dict:
    """One implicit SDIRK step in place; returns the solver statistics."""
    st = cdg2_implicit_stats()
    rc = lib().cdg2_dirk_step(h, ctypes.c_void_p(U_ptr), float(dt),
                              ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    stats = {"newton_iters": st.newton_iters, "krylov_iters": st.krylov_iters,
             "converged": bool(st.converged), "max_residual": st.max_residual}
    if rc != CDG2_OK:
        err = CDG2Error(rc, lib().cdg2_last_error().decode())
        err.stats = stats
        raise err
    return stats


def cdg2_batch_create(cfgs, autotune: bool = False) -> ctypes.c_void_p:
    arr = (cdg2_config * len(cfgs))(*cfgs)
    h = ctypes.c_void_p()
    _check(lib().cdg2_batch_create(arr, len(cfgs), 1 if autotune else 0, ctypes.byref(h)))
    return h


def cdg2_batch_autotune(b) -> tuple:
    """Native autotuner: returns ((eb, nwg, order), ms per step) of the chosen schedule."""
    best = (_d * 4)()
    _check(lib().cdg2_batch_autotune(b, best))
    return (int(best[0]), int(best[1]), int(best[2])), float(best[3])


def cdg2_batch_set_graph(b, on: bool) -> None:
    _check(lib().cdg2_batch_set_graph(b, 1 if on else 0))


def cdg2_batch_destroy(b) -> None:
    _check(lib().cdg2_batch_destroy(b))


def cdg2_batch_set_stream(b, stream: int) -> None:
    _check(lib().cdg2_batch_set_stream(b, ctypes.c_void_p(stream)))


def cdg2_batch_num_dofs(b) -> int:
    return int(lib().cdg2_batch_num_dofs(b))


def cdg2_batch_offset(b, i: int) -> int:
    return int(lib().cdg2_batch_offset(b, int(i)))


def cdg2_batch_set_schedule(b, eb: int, nwg: int, order: int) -> None:
    _check(lib().cdg2_batch_set_schedule(b, int(eb), int(nwg), int(order)))


def cdg2_batch_rk(b, U_ptr: int, offsets, dts, nsteps: int) -> None:
    """offsets: None (the library's packing) or a sequence of element offsets."""
    arr = (_d * len(dts))(*[float(x) for x in dts])
    offs = None if offsets is None else (ctypes.c_size_t * len(offsets))(*[int(x) for x in offsets])
    _check(lib().cdg2_batch_rk(b, ctypes.c_void_p(U_ptr), offs, arr, int(nsteps)))


def cdg2_batch_sync(b) -> None:
    _check(lib().cdg2_batch_sync(b))


def cdg2_sync(h) -> None:
    _check(lib().cdg2_sync(h))


def cdg2_rho_hat(h) -> float:
    return float(lib().cdg2_rho_hat(h))


# ---- convenience wrapper -------------------------------------------------------

class Operator:
    """One grid / order / coefficient set; tensors are torch CUDA tensors of shape
    (6, E, (p+1)^dim) in float64 (or float32 with precision="fp32")."""

    def __init__(self, dim, n, order, coeffs, precision="fp64", wall_axis=None,
                 llf_mode="all", gamma1_in=(0.0, 1.0), diff_flux="cdg2", flux_eta=0.0):
        self.dim, self.order = int(dim), int(order)
        self.n = tuple(int(v) for v in n)[:dim]
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.cfg = make_config(dim, n, order, coeffs, precision, wall_axis, llf_mode, gamma1_in,
                               diff_flux, flux_eta)
        self.h = cdg2_create(self.cfg)
        self.E = 1
        for v in self.n:
            self.E *= v
        self.nm = (order + 1) ** dim
        self.shape = (6, self.E, self.nm)
        assert cdg2_num_dofs(self.h) == 6 * self.E * self.nm

    def _arg(self, t: torch.Tensor) -> int:
        if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and t.numel() == 6 * self.E * self.nm):
            raise ValueError(f"expected a contiguous CUDA {self.dtype} tensor of {self.shape}")
        return t.data_ptr()

    def _stream(self):
        cdg2_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def apply(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(U)
        self._stream()
        cdg2_apply_operator(self.h, self._arg(U), self._arg(out))
        return out

    def rk_step(self, U: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        self._stream()
        cdg2_rk_step(self.h, self._arg(U), dt, nsteps)
        return U

    def rk_step_noalloc(self, U: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        """rk_step with the intermediate states in the library's static scratch
        memory (no device allocation; states up to 32 MiB)."""
        self._stream()
        cdg2_rk_step_noalloc(self.h, self._arg(U), dt, nsteps)
        return U

    def max_dt(self, U: torch.Tensor, cfl: float = 0.9) -> float:
        self._stream()
        return cdg2_max_dt(self.h, self._arg(U), cfl)

    def apply_adjoint(self, U, w, out=None, want_theta=False):
        """J(U)^T w (and d(w . f(U))/d theta for the 21 coefficients if asked)."""
        if out is None:
            out = torch.empty_like(U)
        self._stream()
        th = cdg2_apply_adjoint(self.h, self._arg(U), self._arg(w), self._arg(out), want_theta)
        return (out, th) if want_theta else out

    def rk_step_adjoint(self, U_n, lam_np1, lam_n, dt, dtheta_acc=None):
        """dtheta_acc: None or a CUDA float64 tensor of 21 entries, added to in place."""
        self._stream()
        ptr = 0
        if dtheta_acc is not None:
            if not (dtheta_acc.is_cuda and dtheta_acc.dtype == torch.float64
                    and dtheta_acc.is_contiguous() and dtheta_acc.numel() == 21):
                raise ValueError("dtheta_acc must be a contiguous CUDA float64 tensor of 21 entries")
            ptr = dtheta_acc.data_ptr()
        cdg2_rk_step_adjoint(self.h, self._arg(U_n), self._arg(lam_np1), self._arg(lam_n), dt, ptr)
        return lam_n

    def dirk_step(self, U: torch.Tensor, dt: float, order: int = 3, max_newton: int = 10,
                  krylov_dim: int = 30, newton_rtol: float = 1e-10, krylov_rtol: float = 1e-3) -> dict:
        """One implicit SDIRK step (orders 2-4, Jacobian-free Newton-GMRES) in place;
        returns the solver statistics (raises CDG2Error, code CDG2_ENOCONV, if a
        stage does not converge; U is then unchanged)."""
        self._stream()
        opts = cdg2_implicit_opts(order, max_newton, krylov_dim, newton_rtol, krylov_rtol)
        return cdg2_dirk_step(self.h, self._arg(U), dt, opts)

    def rk_adjoint_segment(self, U_start, nsteps, dt, lam, dtheta_acc=None):
        """Adjoint of nsteps steps from U_start: lam (in place) goes from dL/dU at the
        end of the segment to dL/dU at its start; dtheta_acc as in rk_step_adjoint."""
        self._stream()
        ptr = 0
        if dtheta_acc is not None:
            if not (dtheta_acc.is_cuda and dtheta_acc.dtype == torch.float64
                    and dtheta_acc.is_contiguous() and dtheta_acc.numel() == 21):
                raise ValueError("dtheta_acc must be a contiguous CUDA float64 tensor of 21 entries")
            ptr = dtheta_acc.data_ptr()
        cdg2_rk_adjoint_segment(self.h, self._arg(U_start), nsteps, dt, self._arg(lam), ptr)
        return lam

    def set_coeffs(self, coeffs: dict) -> None:
        # the parameter upload is queued on the handle's stream: bind the current
        # one first, so it is ordered after the work already queued there
        self._stream()
        cdg2_set_coeffs(self.h, coeffs)

    def sync(self) -> None:
        self._stream()
        cdg2_sync(self.h)

    @property
    def rho_hat(self) -> float:
        return cdg2_rho_hat(self.h)

    def close(self):
        if self.h is not None:
            cdg2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cdg2_last_error() -> str:
    return lib().cdg2_last_error().decode()


# ---- unstructured triangle meshes ------------------------------------------------------

def cdg2_tri_create(order: int, xy, nbr, nbe, coeffs: dict, gamma1_in=(0.0, 1.0)) -> int:
    import numpy as np
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    nbe = np.ascontiguousarray(nbe, dtype=np.int32)
    E = xy.shape[0]
    if xy.shape != (E, 3, 2) or nbr.shape != (E, 3) or nbe.shape != (E, 3):
        raise ValueError("xy must be [E, 3, 2], nbr and nbe [E, 3]")
    h = ctypes.c_void_p()
    c = make_coeffs(coeffs)
    _check(lib().cdg2_tri_create(int(order), E, xy.ctypes.data, nbr.ctypes.data, nbe.ctypes.data, ctypes.byref(c),
                                 float(gamma1_in[0]), float(gamma1_in[1]), ctypes.byref(h)))
    return h.value


def cdg2_tri_destroy(h) -> None:
    _check(lib().cdg2_tri_destroy(h))


def cdg2_tri_set_stream(h, stream) -> None:
    _check(lib().cdg2_tri_set_stream(h, stream))


def cdg2_tri_num_dofs(h) -> int:
    return int(lib().cdg2_tri_num_dofs(h))


def cdg2_tri_apply_operator(h, U: int, F: int) -> None:
    _check(lib().cdg2_tri_apply_operator(h, U, F))


def cdg2_tri_rk_step(h, U: int, dt: float, nsteps: int) -> None:
    _check(lib().cdg2_tri_rk_step(h, U, float(dt), int(nsteps)))


def cdg2_tri_sync(h) -> None:
    _check(lib().cdg2_tri_sync(h))


class TriOperator:
    """The operator on a triangle mesh (xy [E, 3, 2], nbr, nbe [E, 3]; see
    cdg2_tri_create in include/cdg2.h); states are contiguous CUDA float64 tensors
    (6, E, (k+1)(k+2)/2)."""

    def __init__(self, order, xy, nbr, nbe, coeffs, gamma1_in=(0.0, 1.0)):
        self.order = int(order)
        self.E = int(len(xy))
        self.nb = (self.order + 1) * (self.order + 2) // 2
        self.shape = (6, self.E, self.nb)
        self.h = cdg2_tri_create(order, xy, nbr, nbe, coeffs, gamma1_in)
        assert cdg2_tri_num_dofs(self.h) == 6 * self.E * self.nb

    def _arg(self, t: torch.Tensor) -> int:
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"expected a contiguous CUDA float64 tensor of {self.shape}")
        return t.data_ptr()

    def _stream(self):
        cdg2_tri_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def apply(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(U)
        self._stream()
        cdg2_tri_apply_operator(self.h, self._arg(U), self._arg(out))
        return out

    def rk_step(self, U: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        self._stream()
        cdg2_tri_rk_step(self.h, self._arg(U), dt, nsteps)
        return U

    def sync(self) -> None:
        self._stream()
        cdg2_tri_sync(self.h)

    def close(self):
        if self.h is not None:
            cdg2_tri_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- unstructured tetrahedral meshes ---------------------------------------------------

def cdg2_tet_create(order: int, xyz, vid, nbr, nbe, coeffs: dict, gamma1_in=(0.0, 1.0)) -> int:
    import numpy as np
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    vid = np.ascontiguousarray(vid, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    nbe = np.ascontiguousarray(nbe, dtype=np.int32)
    E = xyz.shape[0]
    if xyz.shape != (E, 4, 3) or vid.shape != (E, 4) or nbr.shape != (E, 4) or nbe.shape != (E, 4):
        raise ValueError("xyz must be [E, 4, 3], vid, nbr and nbe [E, 4]")
    h = ctypes.c_void_p()
    c = make_coeffs(coeffs)
    _check(lib().cdg2_tet_create(int(order), E, xyz.ctypes.data, vid.ctypes.data, nbr.ctypes.data, nbe.ctypes.data,
                                 ctypes.byref(c), float(gamma1_in[0]), float(gamma1_in[1]), ctypes.byref(h)))
    return h.value


def cdg2_tet_destroy(h) -> None:
    _check(lib().cdg2_tet_destroy(h))


def cdg2_tet_set_stream(h, stream) -> None:
    _check(lib().cdg2_tet_set_stream(h, stream))


def cdg2_tet_num_dofs(h) -> int:
    return int(lib().cdg2_tet_num_dofs(h))


def cdg2_tet_apply_operator(h, U: int, F: int) -> None:
    _check(lib().cdg2_tet_apply_operator(h, U, F))


def cdg2_tet_rk_step(h, U: int, dt: float, nsteps: int) -> None:
    _check(lib().cdg2_tet_rk_step(h, U, float(dt), int(nsteps)))


def cdg2_tet_sync(h) -> None:
    _check(lib().cdg2_tet_sync(h))


class TetOperator:
    """The operator on a tetrahedral mesh (xyz [E, 4, 3], vid, nbr, nbe [E, 4]; see
    cdg2_tet_create in include/cdg2.h); states are contiguous CUDA float64 tensors
    (6, E, (k+1)(k+2)(k+3)/6)."""

    def __init__(self, order, xyz, vid, nbr, nbe, coeffs, gamma1_in=(0.0, 1.0)):
        self.order = int(order)
        self.E = int(len(xyz))
        self.nb = (self.order + 1) * (self.order + 2) * (self.order + 3) // 6
        self.shape = (6, self.E, self.nb)
        self.h = cdg2_tet_create(order, xyz, vid, nbr, nbe, coeffs, gamma1_in)
        assert cdg2_tet_num_dofs(self.h) == 6 * self.E * self.nb

    def _arg(self, t: torch.Tensor) -> int:
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"expected a contiguous CUDA float64 tensor of {self.shape}")
        return t.data_ptr()

    def _stream(self):
        cdg2_tet_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def apply(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(U)
        self._stream()
        cdg2_tet_apply_operator(self.h, self._arg(U), self._arg(out))
        return out

    def rk_step(self, U: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        self._stream()
        cdg2_tet_rk_step(self.h, self._arg(U), dt, nsteps)
        return U

    def sync(self) -> None:
        self._stream()
        cdg2_tet_sync(self.h)

    def close(self):
        if self.h is not None:
            cdg2_tet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
