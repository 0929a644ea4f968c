"""Thin ctypes binding of libdisco.so (the C ABI in include/disco.h).

Argument marshalling only: every step of the objective, its derivatives and the
Gauss-Newton step runs in the HIP kernels of the library.  PyTorch provides device
memory and the current HIP stream.  There is no CPU fallback: importing this module
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdisco.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(hipcc, gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (mirror include/disco.h) -------------------------------------------------
OK = 0
ERR_ARG, ERR_SHAPE, ERR_STATE, ERR_NONFINITE, ERR_NOMEM, ERR_LIMIT, ERR_HIP = -1, -2, -3, -4, -5, -6, -100
STATUS_FOLD, STATUS_PCG_BREAKDOWN, STATUS_LS_FAIL = 1, 2, 4
STORAGE_FP32, STORAGE_FP16 = 0, 1
FLAG_LS_DEVICE = 1
BUF_GRAD_R, BUF_GRAD_T, BUF_SCACHE = 0, 1, 2
REPORT_FIELDS = ["J", "D", "S", "V", "K", "gnorm", "t", "pcg_iters", "pcg_res", "gtp",
                 "J_new", "D_new", "S_new", "V_new", "K_new", "ls_trials", "B", "B_new"]
REP_SIZE = len(REPORT_FIELDS)
TERM_FIELDS = ["J", "D", "S", "V", "K", "B", "nfold", "gnorm"]
PROF_HV, PROF_GRAD, PROF_EVAL, PROF_IMGRAD, PROF_ADJT = 0, 1, 2, 3, 4


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3)]


class _Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
                ("delta", ctypes.c_double), ("tau", ctypes.c_double), ("armijo_c1", ctypes.c_double),
                ("pcg_tol", ctypes.c_double), ("pcg_iters", ctypes.c_int32), ("ls_max", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("beta", ctypes.c_double)]


class _Lbfgs(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("curv_eps", ctypes.c_double), ("h0_tol", ctypes.c_double),
                ("m", ctypes.c_int32), ("h0_iters", ctypes.c_int32)]


MAX_LEVELS = 8
OPT_GN, OPT_LBFGS = 0, 1


class _Multilevel(ctypes.Structure):
    _fields_ = [("params", _Params), ("lbfgs", _Lbfgs), ("levels", ctypes.c_int32), ("optimizer", ctypes.c_int32),
                ("adaptive_delta", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("iters", ctypes.c_int32 * MAX_LEVELS)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32

_SIGS = {
    "disco_create": ([ctypes.POINTER(_Geom), _I, ctypes.POINTER(_P)], ctypes.c_int),
    "disco_destroy": ([_P], None),
    "disco_set_images": ([_P, _P, _P, _P], ctypes.c_int),
    "disco_set_moving": ([_P, _P, _P], ctypes.c_int),
    "disco_set_images_noalloc": ([_P, _P, _P, _P], ctypes.c_int),
    "disco_batch_set_tile": ([_P, _I], ctypes.c_int),
    "disco_set_keypoints": ([_P, _I, _P, _P, _P], ctypes.c_int),
    "disco_set_reference": ([_P, _P, _P], ctypes.c_int),
    "ngf_eval": ([_P, _D, _P, _P, _P], ctypes.c_int),
    "ngf_grad": ([_P, _D, _P, _P, _P, _P, _P], ctypes.c_int),
    "ngf_hessvec": ([_P, _P, _P, _P], ctypes.c_int),
    "ngf_grad_T": ([_P, _D, _P, _P, _P, _P], ctypes.c_int),
    "curvature_apply": ([_P, _D, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "volchange_eval": ([_P, _D, _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "keypoint_penalty": ([_P, _D, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "gn_hessvec": ([_P, ctypes.POINTER(_Params), _P, _P, _P], ctypes.c_int),
    "gn_pcg_step": ([_P, ctypes.POINTER(_Params), _P, _P, _P, _P], ctypes.c_int),
    "lbfgs_step": ([_P, ctypes.POINTER(_Params), ctypes.POINTER(_Lbfgs), _P, _P, _P, _P], ctypes.c_int),
    "lbfgs_reset": ([_P], ctypes.c_int),
    "disco_set_masks": ([_P, _P, _P, _P], ctypes.c_int),
    "disco_kp_create": ([_P, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "disco_kp_destroy": ([_P], None),
    "disco_kp_set_images": ([_P, _P, _P, _D, _P], ctypes.c_int),
    "disco_kp_cost": ([_P, _I, _P, _I, _P, _P], ctypes.c_int),
    "disco_kp_regularise": ([_P, _I, _P, _P, _I, _P, _D, _D, _P, _P, _P, _P], ctypes.c_int),
    "objective_linearise": ([_P, ctypes.POINTER(_Params), _P, _P, _P, _P, _P], ctypes.c_int),
    "objective_eval": ([_P, ctypes.POINTER(_Params), _P, _P, _P], ctypes.c_int),
    "pyramid_plan": ([_P, _P, _I, _P, _P, _P, _P], ctypes.c_int),
    "pyramid_downsample": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "pyramid_prolong": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "multilevel_register": ([ctypes.POINTER(_Geom), _P, _P, _I, _P, _P, ctypes.POINTER(_Multilevel), _P, _P, _P,
                             _P, _P], ctypes.c_int),
    "disco_copy_buffer": ([_P, _I, _P, _P], ctypes.c_int),
    "disco_profile": ([_P, _I], ctypes.c_int),
    "disco_profile_read": ([_P, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_D)], ctypes.c_int),
    "disco_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "disco_batch_create": ([_I, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "disco_batch_destroy": ([_P], None),
    "disco_batch_prepare": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "disco_batch_gn_step": ([_P, _P], ctypes.c_int),
    "disco_batch_set_launch": ([_P, _I, _I], ctypes.c_int),
    "disco_batch_graph_capture": ([_P, _I], ctypes.c_int),
    "disco_batch_graph_launch": ([_P, _P], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTS = tuple(_SIGS)


class DiscoError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {_lib.disco_status_string(code).decode()} (code {code})")


def _check(code: int, where: str):
    if code != OK:
        raise DiscoError(code, where)


@dataclasses.dataclass
class Params:
    eta: float = 10.0
    alpha: float = 1.0
    gamma: float = 0.1
    delta: float = 0.0
    tau: float = 0.0
    armijo_c1: float = 1e-4
    pcg_tol: float = 0.0
    pcg_iters: int = 20
    ls_max: int = 10
    flags: int = 0
    beta: float = 0.0

    def c(self) -> _Params:
        return _Params(self.eta, self.alpha, self.gamma, self.delta, self.tau, self.armijo_c1, self.pcg_tol,
                       self.pcg_iters, self.ls_max, self.flags, self.beta)


@dataclasses.dataclass
class Lbfgs:
    """L-BFGS settings (Sec. II-D3): history m, H0 = alpha C_H L^T L + tau I solved by
    h0_iters Jacobi-PCG iterations (or to |r| <= h0_tol |q|), pairs used only when
    s.y > curv_eps |s||y|."""
    m: int = 5
    tau: float = 10.0
    curv_eps: float = 1e-10
    h0_iters: int = 30
    h0_tol: float = 1e-6

    def c(self) -> _Lbfgs:
        return _Lbfgs(self.tau, self.curv_eps, self.h0_tol, self.m, self.h0_iters)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class _Token:
    """Identity of a tensor's contents at one moment.  The token keeps the tensor alive, so
    no other allocation can take its address: a tensor with the same address, shape,
    strides and in-place version (shared by every view of the same storage) holds the
    same values."""

    def __init__(self, t: torch.Tensor):
        self.t = t
        self.version = t._version

    def same(self, x: torch.Tensor) -> bool:
        t = self.t
        return (x.data_ptr() == t.data_ptr() and x.device == t.device and x.dtype == t.dtype
                and tuple(x.shape) == tuple(t.shape) and x.stride() == t.stride() and x._version == self.version)


class Disco:
    """One image-pair context on the current (or given) HIP device."""

    def __init__(self, shape: Sequence[int], spacing: Sequence[float], storage: str = "fp32",
                 device: Optional[torch.device] = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.shape = tuple(int(s) for s in shape)
        self.spacing = tuple(float(h) for h in spacing)
        nx, ny, nz = self.shape
        self.nodes = (nx // 4 + 1, ny // 4 + 1, nz // 4 + 1)
        self.storage = STORAGE_FP16 if storage == "fp16" else STORAGE_FP32
        geom = _Geom((ctypes.c_int32 * 3)(*self.shape), (ctypes.c_double * 3)(*self.spacing))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.disco_create(ctypes.byref(geom), self.storage, ctypes.byref(h)), "disco_create")
        self._h = h
        self._scalars = torch.zeros(64, dtype=torch.float64, device=self.device)
        self._images = None
        self._ints = torch.zeros(8, dtype=torch.int32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            _lib.disco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers ------------------------------------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def node_field(self) -> torch.Tensor:
        nx, ny, nz = self.nodes
        return torch.empty((3, nz, ny, nx), dtype=torch.float32, device=self.device)

    def _field(self, t: torch.Tensor, name: str) -> torch.Tensor:
        nx, ny, nz = self.nodes
        if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
        if tuple(t.shape) != (3, nz, ny, nx):
            raise ValueError(f"{name} must have shape (3, {nz}, {ny}, {nx}), got {tuple(t.shape)}")
        return t

    def _volume(self, t: torch.Tensor, name: str) -> torch.Tensor:
        nx, ny, nz = self.shape
        if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
        if tuple(t.shape) != (nz, ny, nx):
            raise ValueError(f"{name} must have shape ({nz}, {ny}, {nx}), got {tuple(t.shape)}")
        return t

    # ---- state --------------------------------------------------------------------------
    def set_images(self, R: torch.Tensor, T: torch.Tensor):
        self._images = None
        _check(_lib.disco_set_images(self._h, _ptr(self._volume(R, "R")), _ptr(self._volume(T, "T")),
                                     self._stream()), "disco_set_images")
        self._images = (_Token(R), _Token(T))

    def set_images_noalloc(self, R: torch.Tensor, T: torch.Tensor):
        """set_images without any device allocation (static scratch; see disco.h)."""
        self._images = None
        _check(_lib.disco_set_images_noalloc(self._h, _ptr(self._volume(R, "R")), _ptr(self._volume(T, "T")),
                                             self._stream()), "disco_set_images_noalloc")
        self._images = (_Token(R), _Token(T))

    def set_moving(self, T: torch.Tensor):
        """Replace T only (grad R is kept)."""
        R = self._images[0] if self._images else None
        self._images = None
        _check(_lib.disco_set_moving(self._h, _ptr(self._volume(T, "T")), self._stream()), "disco_set_moving")
        if R is not None:
            self._images = (R, _Token(T))

    def holds_images(self, R: torch.Tensor, T: torch.Tensor) -> bool:
        """Whether the gradient volumes were built from these very tensors, unmodified since."""
        return self._images is not None and self._images[0].same(R) and self._images[1].same(T)

    def use_images(self, R: torch.Tensor, T: torch.Tensor):
        """Make (R, T) the context's images, rebuilding only what changed."""
        if self._images is not None and self._images[0].same(R):
            if not self._images[1].same(T):
                self.set_moving(T)
        else:
            self.set_images(R, T)

    def set_keypoints(self, x_mm, t_mm):
        import numpy as np
        x = np.ascontiguousarray(np.asarray(x_mm, dtype=np.float32).reshape(-1, 3))
        t = np.ascontiguousarray(np.asarray(t_mm, dtype=np.float32).reshape(-1, 3))
        if x.shape != t.shape:
            raise ValueError("keypoints and targets differ in shape")
        _check(_lib.disco_set_keypoints(self._h, len(x), x.ctypes.data_as(_P), t.ctypes.data_as(_P),
                                        self._stream()), "disco_set_keypoints")

    def set_masks(self, bF: Optional[torch.Tensor], bM: Optional[torch.Tensor]):
        """Binary lung masks (uint8 CUDA tensors [Nz][Ny][Nx]) of the lung-boundary term;
        None, None clears them."""
        if bF is None and bM is None:
            _check(_lib.disco_set_masks(self._h, None, None, self._stream()), "disco_set_masks")
            return
        nx, ny, nz = self.shape
        for t in (bF, bM):
            if t.dtype != torch.uint8 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (nz, ny, nx):
                raise ValueError("masks must be contiguous uint8 CUDA tensors [Nz][Ny][Nx]")
        _check(_lib.disco_set_masks(self._h, _ptr(bF), _ptr(bM), self._stream()), "disco_set_masks")

    def objective_linearise(self, params: Params, u: torch.Tensor, grad: bool = True, diag: bool = True,
                            terms: bool = True, g_out: Optional[torch.Tensor] = None):
        """J and its terms (dict of TERM_FIELDS, read back to the host when `terms`), grad J
        (into g_out when given) and the GN diagonal at u (sets the linearisation used by
        gn_hessvec)."""
        tv = torch.zeros(8, dtype=torch.float64, device=self.device) if terms else None
        g = (torch.empty_like(u) if g_out is None else self._field(g_out, "g_out")) if grad else None
        d = torch.empty_like(u) if diag else None
        p = params.c()
        _check(_lib.objective_linearise(self._h, ctypes.byref(p), _ptr(self._field(u, "u")), _ptr(tv), _ptr(g),
                                        _ptr(d), self._stream()), "objective_linearise")
        out = dict(zip(TERM_FIELDS, tv.cpu().tolist())) if terms else {}
        out["g"] = g
        out["diag"] = d
        return out

    def objective_eval(self, params: Params, u: torch.Tensor, terms: Optional[torch.Tensor] = None) -> torch.Tensor:
        """J and its terms at u, no derivatives: device float64 tensor [8] in TERM_FIELDS order
        (gnorm NaN); the linearisation is left unchanged."""
        out = torch.empty(8, dtype=torch.float64, device=self.device) if terms is None else terms
        p = params.c()
        _check(_lib.objective_eval(self._h, ctypes.byref(p), _ptr(self._field(u, "u")), _ptr(out), self._stream()),
               "objective_eval")
        return out

    def set_reference(self, u_ref: Optional[torch.Tensor]):
        _check(_lib.disco_set_reference(self._h, _ptr(None if u_ref is None else self._field(u_ref, "u_ref")),
                                        self._stream()), "disco_set_reference")

    # ---- single terms -------------------------------------------------------------------
    def ngf_eval(self, u: torch.Tensor, eta: float) -> torch.Tensor:
        D = self._scalars[0:1]
        _check(_lib.ngf_eval(self._h, eta, _ptr(self._field(u, "u")), _ptr(D), self._stream()), "ngf_eval")
        return D.clone()

    def ngf_grad(self, u: torch.Tensor, eta: float, diag: bool = True):
        g = self.node_field()
        d = self.node_field() if diag else None
        D = self._scalars[1:2]
        _check(_lib.ngf_grad(self._h, eta, _ptr(self._field(u, "u")), _ptr(D), _ptr(g), _ptr(d), self._stream()),
               "ngf_grad")
        return D.clone(), g, d

    def ngf_hessvec(self, v: torch.Tensor) -> torch.Tensor:
        out = self.node_field()
        _check(_lib.ngf_hessvec(self._h, _ptr(self._field(v, "v")), _ptr(out), self._stream()), "ngf_hessvec")
        return out

    def ngf_grad_T(self, u: torch.Tensor, eta: float, out: Optional[torch.Tensor] = None,
                   scale: Optional[torch.Tensor] = None) -> torch.Tensor:
        """scale * dD/dT at displacement u (volume [Nz][Ny][Nx], into `out` when given);
        scale (optional) is a one-element float64 tensor on the context's device, read by the
        kernels (an upstream gradient, without a host round trip)."""
        nx, ny, nz = self.shape
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device) if out is None \
            else self._volume(out, "out")
        sp = None
        if scale is not None:
            if scale.dtype != torch.float64 or scale.numel() != 1 or scale.device != self.device:
                raise ValueError("scale must be a one-element float64 tensor on the context's device")
            scale = scale.contiguous()
            sp = _ptr(scale)
        _check(_lib.ngf_grad_T(self._h, eta, _ptr(self._field(u, "u")), sp, _ptr(out), self._stream()),
               "ngf_grad_T")
        return out

    def curvature_apply(self, alpha: float, u: torch.Tensor, u_ref: Optional[torch.Tensor] = None,
                        energy: bool = True, grad: bool = True, diag: bool = False):
        S = self._scalars[2:3] if energy else None
        out = self.node_field() if grad else None
        d = self.node_field() if diag else None
        _check(_lib.curvature_apply(self._h, alpha, _ptr(self._field(u, "u")),
                                    _ptr(None if u_ref is None else self._field(u_ref, "u_ref")), _ptr(S), _ptr(out),
                                    _ptr(d), self._stream()), "curvature_apply")
        return (None if S is None else S.clone()), out, d

    def volchange_eval(self, gamma: float, u: torch.Tensor, v: Optional[torch.Tensor] = None,
                       energy: bool = True, grad: bool = True, diag: bool = True):
        V = self._scalars[3:4] if energy else None
        g = self.node_field() if grad else None
        d = self.node_field() if diag else None
        Hv = self.node_field() if v is not None else None
        nf = self._ints[0:1]
        _check(_lib.volchange_eval(self._h, gamma, _ptr(self._field(u, "u")), _ptr(V), _ptr(g), _ptr(d),
                                   _ptr(None if v is None else self._field(v, "v")), _ptr(Hv), _ptr(nf),
                                   self._stream()), "volchange_eval")
        return dict(V=None if V is None else V.clone(), g=g, diag=d, Hv=Hv, nfold=nf.clone())

    def keypoint_penalty(self, delta: float, u: torch.Tensor, v: Optional[torch.Tensor] = None,
                         energy: bool = True, grad: bool = True, diag: bool = True):
        K = self._scalars[4:5] if energy else None
        g = self.node_field() if grad else None
        d = self.node_field() if diag else None
        Hv = self.node_field() if v is not None else None
        _check(_lib.keypoint_penalty(self._h, delta, _ptr(self._field(u, "u")), _ptr(K), _ptr(g), _ptr(d),
                                     _ptr(None if v is None else self._field(v, "v")), _ptr(Hv), self._stream()),
               "keypoint_penalty")
        return dict(K=None if K is None else K.clone(), g=g, diag=d, Hv=Hv)

    # ---- Gauss-Newton ---------------------------------------------------------------------
    def gn_hessvec(self, params: Params, v: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.node_field() if out is None else out
        p = params.c()
        _check(_lib.gn_hessvec(self._h, ctypes.byref(p), _ptr(self._field(v, "v")), _ptr(out), self._stream()),
               "gn_hessvec")
        return out

    def gn_pcg_step(self, params: Params, u: torch.Tensor, report: Optional[torch.Tensor] = None,
                    status: Optional[torch.Tensor] = None):
        """One GN step in place on u.  Returns (report tensor [REP_SIZE] float64, status int32 tensor)."""
        rep = torch.zeros(REP_SIZE, dtype=torch.float64, device=self.device) if report is None else report
        st = torch.zeros(1, dtype=torch.int32, device=self.device) if status is None else status
        p = params.c()
        _check(_lib.gn_pcg_step(self._h, ctypes.byref(p), _ptr(self._field(u, "u")), _ptr(rep), _ptr(st),
                                self._stream()), "gn_pcg_step")
        return rep, st

    def lbfgs_step(self, params: Params, lb: Lbfgs, u: torch.Tensor, report: Optional[torch.Tensor] = None,
                   status: Optional[torch.Tensor] = None):
        """One L-BFGS iteration in place on u (the history of this context advances).
        Returns (report tensor [REP_SIZE] float64, status int32 tensor); the CG slots describe
        the H0 solve."""
        rep = torch.zeros(REP_SIZE, dtype=torch.float64, device=self.device) if report is None else report
        st = torch.zeros(1, dtype=torch.int32, device=self.device) if status is None else status
        p = params.c()
        q = lb.c()
        _check(_lib.lbfgs_step(self._h, ctypes.byref(p), ctypes.byref(q), _ptr(self._field(u, "u")), _ptr(rep),
                               _ptr(st), self._stream()), "lbfgs_step")
        return rep, st

    def lbfgs_reset(self):
        _check(_lib.lbfgs_reset(self._h), "lbfgs_reset")

    @staticmethod
    def report_dict(rep: torch.Tensor) -> dict:
        vals = rep.cpu().tolist()
        return dict(zip(REPORT_FIELDS, vals))

    # ---- buffers and profiling -----------------------------------------------------------
    def copy_buffer(self, which: int) -> torch.Tensor:
        nx, ny, nz = self.shape
        out = torch.empty((nz, ny, nx, 3), dtype=torch.float32, device=self.device)
        _check(_lib.disco_copy_buffer(self._h, which, _ptr(out), self._stream()), "disco_copy_buffer")
        return out

    def profile(self, enable: bool):
        _check(_lib.disco_profile(self._h, 1 if enable else 0), "disco_profile")

    def profile_read(self, kernel: int):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_lib.disco_profile_read(self._h, kernel, ctypes.byref(n), ctypes.byref(ms)), "disco_profile_read")
        return n.value, ms.value


class Batch:
    """Several contexts stepped together: one launch per phase of the GN step for all
    pairs (see disco_batch_* in include/disco.h)."""

    PASS_BRICK, PASS_NODE, PASS_VEC = 0, 1, 2

    def __init__(self, ctxs: Sequence[Disco]):
        self.ctxs = list(ctxs)
        self.device = self.ctxs[0].device
        arr = (_P * len(self.ctxs))(*[c._h for c in self.ctxs])
        h = ctypes.c_void_p()
        _check(_lib.disco_batch_create(len(self.ctxs), arr, ctypes.byref(h)), "disco_batch_create")
        self._h = h
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            _lib.disco_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def prepare(self, params: Sequence[Params], us: Sequence[torch.Tensor]):
        """Fix the per-pair parameters and displacement fields (updated in place by every
        step).  Returns (report [npairs][REP_SIZE] float64, status [npairs] int32) tensors that
        every step rewrites."""
        n = len(self.ctxs)
        if len(params) != n or len(us) != n:
            raise ValueError("one Params and one u per pair")
        for c, u in zip(self.ctxs, us):
            c._field(u, "u")
        rep = torch.zeros((n, REP_SIZE), dtype=torch.float64, device=self.device)
        st = torch.zeros(n, dtype=torch.int32, device=self.device)
        self._prepare(list(params), list(us), rep, st)
        return rep, st

    def _prepare(self, params, us, rep, st):
        n = len(self.ctxs)
        pa = (_Params * n)(*[p.c() for p in params])
        ua = (_P * n)(*[u.data_ptr() for u in us])
        _check(_lib.disco_batch_prepare(self._h, pa, ua, _ptr(rep), _ptr(st)), "disco_batch_prepare")
        self._keep = (params, us, rep, st)

    def gn_step(self):
        _check(_lib.disco_batch_gn_step(self._h, self._stream()), "disco_batch_gn_step")

    def set_launch(self, pass_: int, wg_per_cu: int):
        _check(_lib.disco_batch_set_launch(self._h, pass_, wg_per_cu), "disco_batch_set_launch")

    def set_tile(self, cells_z: int):
        """Brick tile of the batched passes (16 x 4 x cells_z cells, cells_z 4 or 2); a
        prepared batch is prepared again with the same parameters, fields and report tensors."""
        _check(_lib.disco_batch_set_tile(self._h, int(cells_z)), "disco_batch_set_tile")
        if self._keep is not None:
            self._prepare(*self._keep)

    def graph_capture(self, nsteps: int):
        _check(_lib.disco_batch_graph_capture(self._h, nsteps), "disco_batch_graph_capture")

    def graph_launch(self):
        _check(_lib.disco_batch_graph_launch(self._h, self._stream()), "disco_batch_graph_launch")


def status_string(code: int) -> str:
    return _lib.disco_status_string(code).decode()


# ---- multilevel scheme (Sec. II-D3) ----------------------------------------------------

def _i3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def pyramid_plan(shape: Sequence[int], spacing: Sequence[float], levels: int):
    """Host-only: list of (shape (Nx, Ny, Nz), spacing, halve) per level, finest first."""
    n_out = (ctypes.c_int32 * (3 * levels))()
    h_out = (ctypes.c_double * (3 * levels))()
    hv_out = (ctypes.c_int32 * (3 * levels))()
    L = ctypes.c_int32()
    _check(_lib.pyramid_plan(_i3(shape), (ctypes.c_double * 3)(*[float(h) for h in spacing]), levels,
                             ctypes.byref(L), n_out, h_out, hv_out), "pyramid_plan")
    return [(tuple(n_out[3 * l:3 * l + 3]), tuple(h_out[3 * l:3 * l + 3]), tuple(hv_out[3 * l:3 * l + 3]))
            for l in range(L.value)]


def _stream_of(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def pyramid_downsample(img: torch.Tensor, halve: Sequence[int]) -> torch.Tensor:
    """One pyramid step of a float32 CUDA volume [Nz][Ny][Nx]."""
    if img.dtype != torch.float32 or not img.is_cuda or not img.is_contiguous() or img.dim() != 3:
        raise ValueError("img must be a contiguous float32 CUDA tensor [Nz][Ny][Nx]")
    nz, ny, nx = img.shape
    out_shape = tuple(n // 2 if h else n for n, h in zip((nz, ny, nx), tuple(halve)[::-1]))
    out = torch.empty(out_shape, dtype=torch.float32, device=img.device)
    work = None
    if sum(int(h) for h in halve) >= 2:
        work = torch.empty(img.numel() // 2 + img.numel() // 4 + 1, dtype=torch.float32, device=img.device)
    _check(_lib.pyramid_downsample(_ptr(img), _i3((nx, ny, nz)), _i3(halve), _ptr(out), _ptr(work),
                                   _stream_of(img)), "pyramid_downsample")
    return out


def pyramid_prolong(uc: torch.Tensor, halve: Sequence[int]) -> torch.Tensor:
    """Node field [3][nz][ny][nx] of a coarse level to the next finer level."""
    if uc.dtype != torch.float32 or not uc.is_cuda or not uc.is_contiguous() or uc.dim() != 4 or uc.shape[0] != 3:
        raise ValueError("uc must be a contiguous float32 CUDA tensor [3][nz][ny][nx]")
    _, nz, ny, nx = uc.shape
    f = tuple(2 * (n - 1) + 1 if h else n for n, h in zip((nx, ny, nz), halve))
    out = torch.empty((3, f[2], f[1], f[0]), dtype=torch.float32, device=uc.device)
    _check(_lib.pyramid_prolong(_ptr(uc), _i3((nx, ny, nz)), _i3(halve), _ptr(out), _stream_of(uc)),
           "pyramid_prolong")
    return out


@dataclasses.dataclass
class Multilevel:
    """Coarse-to-fine settings: levels requested, optimiser ("lbfgs" or "gn"), iterations
    per level (coarsest built level first), adaptive keypoint weight, storage."""
    levels: int = 4
    optimizer: str = "lbfgs"
    iters: Sequence[int] = (10, 10, 10, 10)
    adaptive_delta: bool = True
    storage: str = "fp32"


def multilevel_register(R: torch.Tensor, T: torch.Tensor, spacing: Sequence[float], kp_x, kp_t, params: Params,
                        ml: Multilevel, lbfgs: Optional[Lbfgs] = None):
    """Whole coarse-to-fine registration on the device.  Returns (u on the finest level,
    reports [rows][REP_SIZE] float64 with NaN rows for iterations not run, levels, delta)."""
    import numpy as np
    for t in (R, T):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 3:
            raise ValueError("R and T must be contiguous float32 CUDA tensors [Nz][Ny][Nx]")
    if R.shape != T.shape:
        raise ValueError("R and T differ in shape")
    nz, ny, nx = R.shape
    g = _Geom((ctypes.c_int32 * 3)(nx, ny, nz), (ctypes.c_double * 3)(*[float(h) for h in spacing]))
    if len(ml.iters) > MAX_LEVELS:
        raise ValueError("too many levels")
    its = (ctypes.c_int32 * MAX_LEVELS)(*([int(i) for i in ml.iters] + [0] * (MAX_LEVELS - len(ml.iters))))
    cfg = _Multilevel(params.c(), (lbfgs or Lbfgs()).c(), ml.levels, OPT_LBFGS if ml.optimizer == "lbfgs" else OPT_GN,
                      1 if ml.adaptive_delta else 0, STORAGE_FP16 if ml.storage == "fp16" else STORAGE_FP32, its)
    x = np.ascontiguousarray(np.asarray(kp_x, dtype=np.float32).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(kp_t, dtype=np.float32).reshape(-1, 3))
    if x.shape != t.shape:
        raise ValueError("keypoints and targets differ in shape")
    u = torch.empty((3, nz // 4 + 1, ny // 4 + 1, nx // 4 + 1), dtype=torch.float32, device=R.device)
    rows = sum(int(i) for i in ml.iters[:ml.levels])
    rep = torch.empty((max(rows, 1), REP_SIZE), dtype=torch.float64, device=R.device)
    L = ctypes.c_int32()
    delta = ctypes.c_double()
    with torch.cuda.device(R.device):
        _check(_lib.multilevel_register(ctypes.byref(g), _ptr(R), _ptr(T), len(x), x.ctypes.data_as(_P),
                                        t.ctypes.data_as(_P), ctypes.byref(cfg), _ptr(u), _ptr(rep), ctypes.byref(L),
                                        ctypes.byref(delta), _stream_of(R)), "multilevel_register")
    return u, rep[:rows], L.value, delta.value


# ---- keypoint stage (Sec. II-C2, II-C3) -------------------------------------------------

class KeypointStage:
    """NGF matching cost over a displacement grid and its regularisation on a tree of
    keypoints (see disco_kp_* in include/disco.h)."""

    def __init__(self, shape: Sequence[int], spacing: Sequence[float] = (1.0, 1.0, 1.0),
                 device: Optional[torch.device] = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.shape = tuple(int(s) for s in shape)
        self.spacing = tuple(float(h) for h in spacing)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.disco_kp_create(_i3(self.shape), (ctypes.c_double * 3)(*self.spacing), ctypes.byref(h)),
                   "disco_kp_create")
        self._h = h

    def close(self):
        if self._h:
            _lib.disco_kp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def set_images(self, F: torch.Tensor, M: torch.Tensor, eta: float):
        nx, ny, nz = self.shape
        for t in (F, M):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (nz, ny, nx):
                raise ValueError("images must be contiguous float32 CUDA tensors [Nz][Ny][Nx]")
        self._imgs = (F, M)
        _check(_lib.disco_kp_set_images(self._h, _ptr(F), _ptr(M), float(eta), self._stream()), "disco_kp_set_images")

    def cost(self, kp_vox: torch.Tensor, R: int = 16) -> torch.Tensor:
        """D_KP [nkp][(2R+1)^3] for int32 CUDA keypoints [nkp][3] (voxel indices x, y, z)."""
        if kp_vox.dtype != torch.int32 or not kp_vox.is_cuda or not kp_vox.is_contiguous():
            raise ValueError("keypoints must be a contiguous int32 CUDA tensor [nkp][3]")
        n = kp_vox.shape[0]
        out = torch.empty((n, (2 * R + 1) ** 3), dtype=torch.float32, device=self.device)
        _check(_lib.disco_kp_cost(self._h, n, _ptr(kp_vox), R, _ptr(out), self._stream()), "disco_kp_cost")
        return out

    def regularise(self, x_mm, inten, cost: torch.Tensor, R: int = 16, alpha_kp: float = 1.0 / 45.0,
                   sigma_I: float = 150.0, marginals: bool = True):
        """Min-sum belief propagation on the keypoint MST.  Returns (min-marginals or None,
        labels int32 CUDA [nkp], parent numpy int32 [nkp])."""
        import numpy as np
        x = np.ascontiguousarray(np.asarray(x_mm, dtype=np.float32).reshape(-1, 3))
        it = np.ascontiguousarray(np.asarray(inten, dtype=np.float32).ravel())
        n = len(x)
        marg = torch.empty_like(cost) if marginals else None
        lab = torch.empty(n, dtype=torch.int32, device=self.device)
        par = np.empty(n, dtype=np.int32)
        _check(_lib.disco_kp_regularise(self._h, n, x.ctypes.data_as(_P), it.ctypes.data_as(_P), R, _ptr(cost),
                                        float(alpha_kp), float(sigma_I), _ptr(marg), _ptr(lab),
                                        par.ctypes.data_as(_P), self._stream()), "disco_kp_regularise")
        return marg, lab, par
