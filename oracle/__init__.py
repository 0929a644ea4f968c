"""FP64 CPU oracle of the dense registration objective (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It never imports the GPU library and the GPU library never
imports it; both receive the same seeded inputs from ``synth``.

The element-wise work is in ``disco_oracle.c`` (plain loops, double precision).
This module composes the joint objective of eq. 11

    J(u) = D(u) + alpha S(u) + beta B(u) + gamma Vhat(u) + delta K(u)

(the lung-boundary term B only when masks are given and beta != 0)
its gradient, the Gauss-Newton matrix-vector product, the adaptive keypoint weight
(Sec. II-D2: delta such that D = delta K at the start), and one Gauss-Newton step
with a Jacobi-preconditioned CG solve and Armijo backtracking.

Arrays: volumes float32 [Nz][Ny][Nx]; node fields [3][nz][ny][nx] (converted to
float64 here); keypoints [n][3] in mm.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "disco_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libdisco_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (double precision, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.or_image_gradient.argtypes = [P, P, P, P]
        lib.or_image_gradient.restype = None
        lib.or_sample_points.argtypes = [P, P, P, I64, P, P, P]
        lib.or_sample_points.restype = None
        lib.or_ngf.argtypes = [P, P, P, D, P, P, P, P, P, P, P, P]
        lib.or_ngf.restype = D
        lib.or_ngf_hv.argtypes = [P, P, P, P, P, P]
        lib.or_ngf_hv.restype = None
        lib.or_curvature.argtypes = [P, P, P, P, P]
        lib.or_curvature.restype = D
        lib.or_vcc.argtypes = [P, P, P, P, P, P, P, P, P]
        lib.or_vcc.restype = D
        lib.or_vcc_cell_expansion.argtypes = [P, P, P, P, P, P, P, P]
        lib.or_vcc_cell_expansion.restype = None
        lib.or_keypoints.argtypes = [P, P, I64, P, P, P, P, P, P, P]
        lib.or_keypoints.restype = D
        lib.or_det_voxels.argtypes = [P, P, P, P, P]
        lib.or_det_voxels.restype = None
        lib.or_ngf_grad_T.argtypes = [P, P, P, D, P, P, P, P]
        lib.or_ngf_grad_T.restype = None
        lib.or_mask.argtypes = [P, P, P, P, P, P, P, P, P, P]
        lib.or_mask.restype = D
        lib.or_ngf_ties.argtypes = [P, P, P, D, P, P, P, P, P, P, P, P]
        lib.or_ngf_ties.restype = I64
        lib.or_mask_ties.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
        lib.or_mask_ties.restype = I64
        lib.or_kp_cost.argtypes = [P, P, P, I64, P, D, I64, I64, P]
        lib.or_kp_cost.restype = None
        lib.or_num_threads.argtypes = []
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_threads.argtypes = [ctypes.c_int]
        lib.or_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().or_num_threads())


def set_threads(n: int) -> None:
    """Set the thread count of the oracle's parallel loops (timing runs)."""
    _load().or_set_threads(int(n))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


# ------------------------------------------------------------------------------------
# element functions
# ------------------------------------------------------------------------------------

def image_gradient(img: np.ndarray, spacing) -> np.ndarray:
    """Central-difference gradient with replicated border, [Nz][Ny][Nx][3] float64."""
    img = _f32(img)
    nz, ny, nx = img.shape
    out = np.empty((nz, ny, nx, 3), np.float64)
    _load().or_image_gradient(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(img), _p(out))
    return out


def sample_points(grad: np.ndarray, spacing, q: np.ndarray):
    """Trilinear, zero-padded sampling of a [Nz][Ny][Nx][3] field at continuous voxel
    indices q ([n][3], x,y,z order).  Returns (G [n][3], JG [n][3][3] = dG_c/dy_a)."""
    grad = _f64(grad)
    nz, ny, nx, _ = grad.shape
    q = _f64(q).reshape(-1, 3)
    G = np.empty((len(q), 3))
    JG = np.empty((len(q), 3, 3))
    _load().or_sample_points(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(grad), len(q), _p(q), _p(G), _p(JG))
    return G, JG


def node_shape(shape):
    return tuple(int(s) // 4 + 1 for s in shape)


def ngf(gR, gT, spacing, eta, u, m=(4, 4, 4), want=("g", "diag", "s", "r", "c")):
    """NGF distance (eq. 1) and its derivatives.  Returns dict with D and the requested
    arrays (g, diag: node fields; s: [N][3]; r, c: [N])."""
    gR = _f64(gR)
    gT = _f64(gT)
    nz, ny, nx, _ = gR.shape
    n = _i64([nx, ny, nz])
    mm = _i64(m)
    nn = [nx // m[0] + 1, ny // m[1] + 1, nz // m[2] + 1]
    u = _f64(u)
    assert u.shape == (3, nn[2], nn[1], nn[0]), (u.shape, nn)
    g = np.empty((3, nn[2], nn[1], nn[0])) if "g" in want else None
    diag = np.empty((3, nn[2], nn[1], nn[0])) if "diag" in want else None
    s = np.empty((nz, ny, nx, 3)) if "s" in want else None
    r = np.empty((nz, ny, nx)) if "r" in want else None
    c = np.empty((nz, ny, nx)) if "c" in want else None
    D = _load().or_ngf(_p(n), _p(_f64(spacing)), _p(mm), float(eta), _p(gR), _p(gT), _p(u),
                       _p(g), _p(diag), _p(s), _p(r), _p(c))
    return dict(D=D, g=g, diag=diag, s=s, r=r, c=c)


def ngf_ties(gR, gT, spacing, eta, u, v=None, m=(4, 4, 4), want_s=False):
    """Sample-cell ties of eq. 1 at u (see ``or_ngf_ties``): voxels whose warped point
    lies within single-precision rounding of a cell face of the moving image, where
    either one-sided derivative is correct.  Returns dict(n = number of such voxels,
    g, diag [, hv] = per-node allowance fields (sum over those voxels of the largest
    difference between the one-sided choices), s = per-voxel allowance of the s
    vectors when want_s)."""
    gR = _f64(gR)
    gT = _f64(gT)
    nz, ny, nx, _ = gR.shape
    nn = [nx // m[0] + 1, ny // m[1] + 1, nz // m[2] + 1]
    u = _f64(u)
    assert u.shape == (3, nn[2], nn[1], nn[0]), (u.shape, nn)
    g = np.empty((3, nn[2], nn[1], nn[0]))
    diag = np.empty_like(g)
    hv = np.empty_like(g) if v is not None else None
    s = np.empty((nz, ny, nx, 3)) if want_s else None
    nt = _load().or_ngf_ties(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(_i64(m)), float(eta), _p(gR), _p(gT),
                             _p(u), _p(None if v is None else _f64(v)), _p(g), _p(diag), _p(hv), _p(s))
    return dict(n=int(nt), g=g, diag=diag, hv=hv, s=s)


def mask_ties(bF, bM, spacing, u, v=None, m=(4, 4, 4), want_s=False):
    """Sample-cell ties of the lung-boundary term (eq. 6), as ``ngf_ties``; the per-voxel
    field (when want_s) is the allowance of the mask gradient sb."""
    bF = _f64(bF)
    bM = _f64(bM)
    nz, ny, nx = bF.shape
    nn = [nx // m[0] + 1, ny // m[1] + 1, nz // m[2] + 1]
    u = _f64(u)
    g = np.empty((3, nn[2], nn[1], nn[0]))
    diag = np.empty_like(g)
    hv = np.empty_like(g) if v is not None else None
    sb = np.empty((nz, ny, nx, 3)) if want_s else None
    nt = _load().or_mask_ties(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(_i64(m)), _p(bF), _p(bM), _p(u),
                              _p(None if v is None else _f64(v)), _p(g), _p(diag), _p(hv), _p(sb))
    return dict(n=int(nt), g=g, diag=diag, hv=hv, s=sb)


def ngf_grad_T(gR, gT, spacing, eta, u, m=(4, 4, 4)):
    """dD/dT (eq. 1 through the gradient stencil and the trilinear sampling), [Nz][Ny][Nx]."""
    gR = _f64(gR)
    gT = _f64(gT)
    nz, ny, nx, _ = gR.shape
    out = np.empty((nz, ny, nx))
    _load().or_ngf_grad_T(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(_i64(m)), float(eta), _p(gR), _p(gT),
                          _p(_f64(u)), _p(out))
    return out


def ngf_hv(s, spacing, v, m=(4, 4, 4)):
    """Gauss-Newton product of the NGF term with the per-voxel vectors s."""
    s = _f64(s)
    nz, ny, nx, _ = s.shape
    nn = [nx // m[0] + 1, ny // m[1] + 1, nz // m[2] + 1]
    v = _f64(v)
    out = np.empty((3, nn[2], nn[1], nn[0]))
    _load().or_ngf_hv(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(_i64(m)), _p(s), _p(v), _p(out))
    return out


def mask_term(bF, bM, spacing, u, m=(4, 4, 4), want=("g", "diag", "sb", "res")):
    """Lung-boundary term of eq. 6 and its derivatives: B, and the requested arrays
    (g, diag: node fields; sb: [N][3] gradient of the interpolated moving mask at the
    warped voxel; res: [N] residual b_M(y) - b_F)."""
    bF = _f64(bF)
    bM = _f64(bM)
    nz, ny, nx = bF.shape
    nn = [nx // m[0] + 1, ny // m[1] + 1, nz // m[2] + 1]
    u = _f64(u)
    assert u.shape == (3, nn[2], nn[1], nn[0]), (u.shape, nn)
    g = np.empty((3, nn[2], nn[1], nn[0])) if "g" in want else None
    diag = np.empty((3, nn[2], nn[1], nn[0])) if "diag" in want else None
    sb = np.empty((nz, ny, nx, 3)) if "sb" in want else None
    res = np.empty((nz, ny, nx)) if "res" in want else None
    B = _load().or_mask(_p(_i64([nx, ny, nz])), _p(_f64(spacing)), _p(_i64(m)), _p(bF), _p(bM), _p(u), _p(g),
                        _p(diag), _p(sb), _p(res))
    return dict(B=B, g=g, diag=diag, sb=sb, res=res)


def mask_hv(sb, spacing, v, m=(4, 4, 4)):
    """Gauss-Newton product of the lung-boundary term, h^3 sum_v phi_v sb_v (sb_v . Pv):
    the NGF product routine computes 2 h^3 sum_v phi_v s_v (s_v . Pv), so it is called
    with s = sb / sqrt(2)."""
    return ngf_hv(_f64(sb) * np.sqrt(0.5), spacing, v, m)


def curvature(w, H):
    """S(w) (eq. 5 on the node grid), C_H L^T L w, C_H diag(L^T L)."""
    w = _f64(w)
    _, nz, ny, nx = w.shape
    out = np.empty_like(w)
    diag = np.empty_like(w)
    S = _load().or_curvature(_p(_i64([nx, ny, nz])), _p(_f64(H)), _p(w), _p(out), _p(diag))
    return dict(S=S, g=out, diag=diag)


def vcc(u, H, v=None):
    """Vhat (eq. 9), its gradient, GN diagonal, optional GN product, fold count, d range."""
    u = _f64(u)
    _, nz, ny, nx = u.shape
    g = np.empty_like(u)
    diag = np.empty_like(u)
    Hv = np.empty_like(u) if v is not None else None
    nfold = np.zeros(1, np.int64)
    dmm = np.zeros(2)
    V = _load().or_vcc(_p(_i64([nx, ny, nz])), _p(_f64(H)), _p(u), _p(None if v is None else _f64(v)),
                       _p(g), _p(diag), _p(Hv), _p(nfold), _p(dmm))
    return dict(V=V, g=g, diag=diag, Hv=Hv, nfold=int(nfold[0]), dmin=dmm[0], dmax=dmm[1])


def vcc_cell_expansion(u, H, cell, xi):
    """(alpha[64], d[64], exact det grad y) of one cell at local coordinate xi."""
    u = _f64(u)
    _, nz, ny, nx = u.shape
    alpha = np.empty(64)
    d = np.empty(64)
    det = np.zeros(1)
    _load().or_vcc_cell_expansion(_p(_i64([nx, ny, nz])), _p(_f64(H)), _p(u), _p(_i64(cell)), _p(_f64(xi)),
                                  _p(alpha), _p(d), _p(det))
    return alpha, d, float(det[0])


def keypoints(u, H, x, t, v=None):
    """K (eq. 10), 2 P^T res, diag 2 P^T P, optional 2 P^T P v."""
    u = _f64(u)
    _, nz, ny, nx = u.shape
    x = _f64(x).reshape(-1, 3)
    t = _f64(t).reshape(-1, 3)
    g = np.empty_like(u)
    diag = np.empty_like(u)
    Hv = np.empty_like(u) if v is not None else None
    K = _load().or_keypoints(_p(_i64([nx, ny, nz])), _p(_f64(H)), len(x), _p(x), _p(t), _p(u),
                             _p(None if v is None else _f64(v)), _p(g), _p(diag), _p(Hv))
    if np.isnan(K):
        raise ValueError("keypoint outside the image domain")
    return dict(K=K, g=g, diag=diag, Hv=Hv)


def det_voxels(u, spacing, shape, m=(4, 4, 4)):
    """Exact det(grad y) at every voxel centre (diagnostic)."""
    nx, ny, nz = shape
    out = np.empty((nz, ny, nx))
    _load().or_det_voxels(_p(_i64([nx, ny, nz])), _p(_i64(m)), _p(_f64(spacing)), _p(_f64(u)), _p(out))
    return out


# ------------------------------------------------------------------------------------
# composite problem: eq. 11 with beta = 0
# ------------------------------------------------------------------------------------

@dataclasses.dataclass
class Weights:
    eta: float = 10.0
    alpha: float = 1.0
    gamma: float = 0.1
    delta: float = 0.0
    beta: float = 0.0     # lung-boundary weight (eq. 6, eq. 11); needs masks


class Problem:
    """One registration pair: J(u) = D + alpha S + gamma Vhat + delta K."""

    def __init__(self, R, T, spacing, kp_x=None, kp_t=None, weights: Weights = Weights(),
                 u_ref=None, m=(4, 4, 4), bF=None, bM=None):
        self.spacing = tuple(float(s) for s in spacing)
        self.m = tuple(int(a) for a in m)
        self.shape = (R.shape[2], R.shape[1], R.shape[0])
        self.H = tuple(self.spacing[a] * self.m[a] for a in range(3))
        self.gR = image_gradient(R, self.spacing)
        self.gT = image_gradient(T, self.spacing)
        self.kp_x = None if kp_x is None else _f64(kp_x).reshape(-1, 3)
        self.kp_t = None if kp_t is None else _f64(kp_t).reshape(-1, 3)
        self.w = dataclasses.replace(weights)
        nn = node_shape(self.shape)
        self.nodes = nn
        self.u_ref = np.zeros((3, nn[2], nn[1], nn[0])) if u_ref is None else _f64(u_ref)
        self.bF = None if bF is None else _f64(bF)
        self.bM = None if bM is None else _f64(bM)
        self._s = None
        self._sb = None

    # individual terms ---------------------------------------------------------------
    def ngf(self, u, want=("g", "diag", "s", "r", "c")):
        return ngf(self.gR, self.gT, self.spacing, self.w.eta, u, self.m, want)

    def curvature(self, u):
        return curvature(_f64(u) - self.u_ref, self.H)

    def vcc(self, u, v=None):
        return vcc(u, self.H, v)

    def keypoints(self, u, v=None):
        if self.kp_x is None or len(self.kp_x) == 0:
            z = np.zeros_like(_f64(u))
            return dict(K=0.0, g=z, diag=z.copy(), Hv=None if v is None else z.copy())
        return keypoints(u, self.H, self.kp_x, self.kp_t, v)

    def mask(self, u, want=("g", "diag", "sb", "res")):
        if self.bF is None:
            z = np.zeros_like(_f64(u))
            return dict(B=0.0, g=z, diag=z.copy(), sb=None, res=None)
        return mask_term(self.bF, self.bM, self.spacing, u, self.m, want)

    def adaptive_beta(self, u0):
        """beta such that D = 100 beta B at the start of the registration (Sec. II-D2)."""
        D = self.ngf(u0, want=())["D"]
        B = self.mask(u0, want=())["B"]
        return D / (100.0 * B) if B > 0 else 0.0

    def adaptive_delta(self, u0):
        """delta such that D = delta K at the start of the registration (Sec. II-D2)."""
        D = self.ngf(u0, want=())["D"]
        K = self.keypoints(u0)["K"]
        return D / K if K > 0 else 0.0

    def ties(self, u, v=None):
        """Allowance fields of the sample-cell ties at u for the joint gradient, GN
        diagonal and (with v) GN product of eq. 11: the NGF term's plus beta times the
        boundary term's (the other terms take no sampling decision)."""
        t = ngf_ties(self.gR, self.gT, self.spacing, self.w.eta, u, v, self.m)
        if self.w.beta != 0.0 and self.bF is not None:
            tb = mask_ties(self.bF, self.bM, self.spacing, u, v, self.m)
            t["n"] += tb["n"]
            for k in ("g", "diag", "hv"):
                if t[k] is not None:
                    t[k] = t[k] + self.w.beta * tb[k]
        return t

    # joint objective -----------------------------------------------------------------
    def objective(self, u):
        """Terms and total of eq. 11 (beta = 0); total is +inf on a fold."""
        w = self.w
        D = self.ngf(u, want=())["D"]
        S = self.curvature(u)["S"]
        vc = self.vcc(u)
        K = self.keypoints(u)["K"]
        B = self.mask(u, want=())["B"] if w.beta != 0.0 else 0.0
        # Vhat = +inf on a fold (eq. 9); the term only exists when gamma > 0
        folded = vc["nfold"] > 0 and w.gamma != 0.0
        vterm = w.gamma * vc["V"] if w.gamma != 0.0 else 0.0
        J = np.inf if folded else D + w.alpha * S + w.beta * B + vterm + w.delta * K
        return dict(J=J, D=D, S=S, V=vc["V"], K=K, B=B, nfold=vc["nfold"])

    def linearise(self, u):
        """Objective, gradient and GN diagonal at u; keeps s for gn_hv."""
        w = self.w
        nd = self.ngf(u, want=("g", "diag", "s"))
        cv = self.curvature(u)
        vc = self.vcc(u)
        kp = self.keypoints(u)
        self._s = nd["s"]
        self._u = _f64(u).copy()
        g = nd["g"] + w.alpha * cv["g"] + w.delta * kp["g"]
        diag = nd["diag"] + w.alpha * cv["diag"] + w.delta * kp["diag"]
        B = 0.0
        if w.beta != 0.0:
            mk = self.mask(u)
            self._sb = mk["sb"]
            B = mk["B"]
            g = g + w.beta * mk["g"]
            diag = diag + w.beta * mk["diag"]
        if w.gamma != 0.0:
            g = g + w.gamma * vc["g"]
            diag = diag + w.gamma * vc["diag"]
        folded = vc["nfold"] > 0 and w.gamma != 0.0
        vterm = w.gamma * vc["V"] if w.gamma != 0.0 else 0.0
        J = np.inf if folded else nd["D"] + w.alpha * cv["S"] + w.beta * B + vterm + w.delta * kp["K"]
        return dict(J=J, D=nd["D"], S=cv["S"], V=vc["V"], K=kp["K"], B=B, nfold=vc["nfold"], g=g, diag=diag)

    def gn_hv(self, v, terms=("D", "S", "V", "K", "B")):
        """Gauss-Newton matrix of eq. 11 times v, at the last linearisation point."""
        assert self._s is not None, "call linearise first"
        w = self.w
        v = _f64(v)
        out = np.zeros_like(v)
        if "D" in terms:
            out += ngf_hv(self._s, self.spacing, v, self.m)
        if "S" in terms and w.alpha != 0.0:
            out += w.alpha * curvature(v, self.H)["g"]
        if "V" in terms and w.gamma != 0.0:
            out += w.gamma * vcc(self._u, self.H, v)["Hv"]
        if "K" in terms and w.delta != 0.0:
            out += w.delta * self.keypoints(self._u, v)["Hv"]
        if "B" in terms and w.beta != 0.0:
            out += w.beta * mask_hv(self._sb, self.spacing, v, self.m)
        return out


# ------------------------------------------------------------------------------------
# one Gauss-Newton step: Jacobi-PCG on H p = -g, then Armijo backtracking
# ------------------------------------------------------------------------------------

@dataclasses.dataclass
class StepParams:
    pcg_iters: int = 20
    pcg_tol: float = 0.0          # stop when |r| <= tol |g| (0: run all iterations)
    ls_max: int = 10
    armijo_c1: float = 1e-4
    tau: float = 0.0              # optional damping tau I added to the GN matrix


def pcg(hv, b, diag, iters, tol=0.0, tau=0.0):
    """Jacobi-preconditioned CG for (H + tau I) x = b from x0 = 0.

    Preconditioner M = diag(H) + tau + 1e-12 max(diag(H)).  Stops after `iters`
    iterations, when |r| <= tol |b|, or when p^T H p <= 0 (breakdown)."""
    M = diag + tau + 1e-12 * float(np.max(diag))
    x = np.zeros_like(b)
    r = b.copy()
    z = r / M
    p = z.copy()
    rz = float(np.sum(r * z))
    bnorm = float(np.sqrt(np.sum(b * b)))
    hist = []
    breakdown = False
    it = 0
    while it < iters:
        q = hv(p) + tau * p
        pq = float(np.sum(p * q))
        if not pq > 0.0:
            breakdown = True
            break
        a = rz / pq
        x = x + a * p
        r = r - a * q
        it += 1
        rn = float(np.sqrt(np.sum(r * r)))
        hist.append(rn)
        if tol > 0.0 and rn <= tol * bnorm:
            break
        z = r / M
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, dict(iters=it, breakdown=breakdown, res=hist)


def gn_pcg_step(prob: Problem, u, params: StepParams = StepParams()):
    """One GN step: linearise, solve H p = -g by Jacobi-PCG, Armijo line search on
    t in {1, 1/2, ...} rejecting folded trial points.  Returns (u_new, report)."""
    lin = prob.linearise(u)
    g = lin["g"]
    p, info = pcg(lambda v: prob.gn_hv(v), -g, lin["diag"], params.pcg_iters, params.pcg_tol, params.tau)
    gtp = float(np.sum(g * p))
    t = 1.0
    accepted = False
    trial = None
    for _ in range(params.ls_max):
        trial = prob.objective(_f64(u) + t * p)
        if np.isfinite(trial["J"]) and trial["J"] <= lin["J"] + params.armijo_c1 * t * gtp:
            accepted = True
            break
        t *= 0.5
    u_new = _f64(u) + t * p if accepted else _f64(u).copy()
    rep = dict(J=lin["J"], D=lin["D"], S=lin["S"], V=lin["V"], K=lin["K"], B=lin["B"],
               gnorm=float(np.sqrt(np.sum(g * g))), t=t if accepted else 0.0, accepted=accepted,
               p=p, gtp=gtp, pcg=info, trial=trial, g=g, diag=lin["diag"])
    return u_new, rep


# ------------------------------------------------------------------------------------
# L-BFGS (Sec. II-D3): limited memory m, initial inverse Hessian H0^-1 with
# H0 = alpha C_H L^T L + tau I (the Hessian of the curvature term plus tau I)
# ------------------------------------------------------------------------------------

def h0_apply(prob: Problem, v, tau: float):
    """H0 v = alpha C_H L^T L v + tau v (node field)."""
    v = _f64(v)
    return prob.w.alpha * curvature(v, prob.H)["g"] + tau * v


def h0_solve(prob: Problem, q, tau: float, rtol: float = 1e-12):
    """H0^-1 q for the symmetric positive definite H0 (tau > 0), by conjugate gradients
    (scipy) run to a relative residual of rtol, i.e. exactly up to rounding."""
    from scipy.sparse.linalg import LinearOperator, cg
    q = _f64(q)
    n = q.size
    A = LinearOperator((n, n), matvec=lambda x: h0_apply(prob, x.reshape(q.shape), tau).ravel(), dtype=np.float64)
    x, info = cg(A, q.ravel(), rtol=rtol, atol=0.0, maxiter=20 * n)
    if info != 0:
        raise RuntimeError("H0 solve did not converge")
    return x.reshape(q.shape)


def lbfgs_direction(g, S, Y, h0inv):
    """Two-loop recursion: returns -H_k g, where H_k is the inverse Hessian approximation
    obtained from h0inv (a function applying H0^-1) by BFGS updates with the pairs (S[i],
    Y[i]), oldest first.  Pairs with s.y <= 0 carry rho = 0 and change nothing."""
    q = _f64(g).copy()
    rho = [1.0 / float(np.sum(s * y)) if float(np.sum(s * y)) > 0.0 else 0.0 for s, y in zip(S, Y)]
    alpha = [0.0] * len(S)
    for i in reversed(range(len(S))):
        alpha[i] = rho[i] * float(np.sum(S[i] * q))
        q = q - alpha[i] * Y[i]
    r = h0inv(q)
    for i in range(len(S)):
        beta = rho[i] * float(np.sum(Y[i] * r))
        r = r + (alpha[i] - beta) * S[i]
    return -r


@dataclasses.dataclass
class LbfgsParams:
    m: int = 5                # history length
    tau: float = 10.0         # H0 = alpha C_H L^T L + tau I
    ls_max: int = 10
    armijo_c1: float = 1e-4
    curv_eps: float = 1e-10   # pair stored only if s.y > curv_eps |s| |y|


def lbfgs_run(prob, u0, iters: int, params: LbfgsParams = LbfgsParams(), fg=None, f=None, h0inv=None):
    """L-BFGS iterations from u0 with Armijo backtracking on t in {1, 1/2, ...} (trial
    points with J = +inf rejected).  fg(u) -> (J, g), f(u) -> J and h0inv(q) default to the
    registration objective of eq. 11 of `prob` and the exact H0 solve.  A pair (s, y) with
    s.y <= curv_eps |s||y| is stored as zeros (rho = 0), so the history still advances.
    Returns (u, per-iteration reports)."""
    if fg is None:
        def fg(u):
            lin = prob.linearise(u)
            return lin["J"], lin["g"]
    if f is None:
        def f(u):
            return prob.objective(u)["J"]
    if h0inv is None:
        def h0inv(q):
            return h0_solve(prob, q, params.tau)
    u = _f64(u0).copy()
    J, g = fg(u)
    S, Y = [], []
    reps = []
    for _ in range(iters):
        p = lbfgs_direction(g, S, Y, h0inv)
        gtp = float(np.sum(g * p))
        t, accepted, Jt = 1.0, False, np.inf
        for _ in range(params.ls_max):
            Jt = f(u + t * p)
            if np.isfinite(Jt) and Jt <= J + params.armijo_c1 * t * gtp:
                accepted = True
                break
            t *= 0.5
        reps.append(dict(J=J, gnorm=float(np.sqrt(np.sum(g * g))), gtp=gtp, t=t if accepted else 0.0,
                         accepted=accepted, J_new=Jt, p=p))
        if not accepted:
            break
        u_new = u + t * p
        J_new, g_new = fg(u_new)
        s, y = u_new - u, g_new - g
        sy = float(np.sum(s * y))
        if sy <= params.curv_eps * float(np.linalg.norm(s) * np.linalg.norm(y)):
            s, y = s * 0.0, y * 0.0
        S.append(s)
        Y.append(y)
        if len(S) > params.m:
            S.pop(0)
            Y.pop(0)
        u, J, g = u_new, J_new, g_new
    return u, reps


# ------------------------------------------------------------------------------------
# multilevel scheme (Sec. II-D3): image pyramid by Gaussian smoothing and downsampling
# toward isotropic voxels, control grid halved with the voxels, coarse-to-fine
# optimisation with the displacement prolonged by trilinear interpolation
# ------------------------------------------------------------------------------------

PYR_SIGMA = 1.0   # Gaussian sigma in voxels of the finer level, along halved axes
PYR_RADIUS = 3    # taps at -3 .. 3 (truncated at 3 sigma), renormalised


def pyramid_halving(shape, spacing):
    """Axes halved to go one level coarser, (hx, hy, hz) in {0, 1}: among the non-empty
    subsets whose axes have a size divisible by 8 (so the coarse size stays a multiple
    of 4) and a coarse size of at least 8 voxels, the one whose coarse spacing is most
    nearly isotropic (smallest max h / min h); ties go to more halved axes, then to the
    subset that halves x before y before z.  None if no subset qualifies."""
    best = None
    for mask in range(1, 8):
        S = tuple((mask >> a) & 1 for a in range(3))
        if any(S[a] and (shape[a] % 8 != 0 or shape[a] // 2 < 8) for a in range(3)):
            continue
        h = [float(spacing[a]) * (2.0 if S[a] else 1.0) for a in range(3)]
        key = (max(h) / min(h), -sum(S), mask)
        if best is None or key < best[0]:
            best = (key, S)
    return None if best is None else best[1]


def pyramid_plan(shape, spacing, levels):
    """Levels finest first, at most `levels`: dicts with shape (Nx, Ny, Nz), spacing and
    the axes halved from the next finer level ((0, 0, 0) on the finest)."""
    plan = [dict(shape=tuple(int(n) for n in shape), spacing=tuple(float(h) for h in spacing), halve=(0, 0, 0))]
    while len(plan) < levels:
        last = plan[-1]
        S = pyramid_halving(last["shape"], last["spacing"])
        if S is None:
            break
        plan.append(dict(shape=tuple(n // 2 if s else n for n, s in zip(last["shape"], S)),
                         spacing=tuple(h * 2.0 if s else h for h, s in zip(last["spacing"], S)), halve=S))
    return plan


def gaussian_taps(sigma: float = PYR_SIGMA, radius: int = PYR_RADIUS):
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (k / sigma) ** 2)
    return w / np.sum(w)


def smooth_axis(img, axis: int, sigma: float = PYR_SIGMA, radius: int = PYR_RADIUS):
    """Gaussian smoothing of a volume [Nz][Ny][Nx] along image axis `axis` (0 = x), with
    the border value replicated: out(i) = sum_k w_k img(clamp(i + k))."""
    img = _f64(img)
    ax = 2 - axis
    n = img.shape[ax]
    w = gaussian_taps(sigma, radius)
    out = np.zeros_like(img)
    for j, k in enumerate(range(-radius, radius + 1)):
        idx = np.clip(np.arange(n) + k, 0, n - 1)
        out += w[j] * np.take(img, idx, axis=ax)
    return out


def downsample(img, halve):
    """One pyramid step: Gaussian smoothing along every halved axis, then each coarse
    voxel is the mean of the two finer voxels it covers along each halved axis (the
    smoothed image at the coarse voxel centre, which lies midway between them)."""
    out = _f64(img)
    for a in range(3):
        if halve[a]:
            out = smooth_axis(out, a)
    for a in range(3):
        if halve[a]:
            ax = 2 - a
            n = out.shape[ax]
            even = np.take(out, np.arange(0, n, 2), axis=ax)
            odd = np.take(out, np.arange(1, n, 2), axis=ax)
            out = 0.5 * (even + odd)
    return out


def prolong(uc, halve):
    """Coarse node field [3][nz][ny][nx] to the next finer level: along a halved axis the
    fine node q sits at coarse coordinate q/2, so even nodes copy a coarse node and odd
    nodes average the two coarse nodes beside it.  This is the coarse trilinear field
    evaluated at the fine nodes, and it represents that field exactly (the coarse cells
    are unions of fine cells).  Displacements are in mm and are not rescaled."""
    u = _f64(uc)
    for a in range(3):
        if halve[a]:
            ax = 3 - a
            n = u.shape[ax]
            shp = list(u.shape)
            shp[ax] = 2 * (n - 1) + 1
            out = np.empty(shp)
            sl = [slice(None)] * 4
            sl[ax] = slice(0, None, 2)
            out[tuple(sl)] = u
            sl[ax] = slice(1, None, 2)
            lo = np.take(u, np.arange(0, n - 1), axis=ax)
            hi = np.take(u, np.arange(1, n), axis=ax)
            out[tuple(sl)] = 0.5 * (lo + hi)
            u = out
    return u


@dataclasses.dataclass
class MultilevelParams:
    levels: int = 4
    iters: tuple = (10, 10, 10, 10)   # iterations per level, coarsest first
    optimizer: str = "lbfgs"          # "lbfgs" or "gn"
    lbfgs: LbfgsParams = dataclasses.field(default_factory=LbfgsParams)
    step: StepParams = dataclasses.field(default_factory=StepParams)


def multilevel_run(R, T, spacing, kp_x, kp_t, weights: Weights, params: MultilevelParams = MultilevelParams()):
    """Coarse-to-fine registration: the pyramid of pyramid_plan; on the coarsest level
    u = 0, on each finer level u = prolong(u of the coarser level); `iters` iterations of
    the optimiser per level (a fresh L-BFGS history per level; GN steps stop early when
    the line search fails).  With weights.delta < 0 the keypoint weight is set once on
    the coarsest level at u = 0 so that D = delta K (Sec. II-D2).  Level images are
    computed in FP64 and stored as float32 (the precision of the input volumes).
    Returns (u on the finest level, per-level dicts with shape, delta and reports)."""
    plan = pyramid_plan((R.shape[2], R.shape[1], R.shape[0]), spacing, params.levels)
    Rs, Ts = [np.asarray(R, np.float32)], [np.asarray(T, np.float32)]
    for lv in plan[1:]:
        Rs.append(downsample(Rs[-1], lv["halve"]).astype(np.float32))
        Ts.append(downsample(Ts[-1], lv["halve"]).astype(np.float32))
    L = len(plan)
    delta = weights.delta
    u = None
    out = []
    for li in range(L - 1, -1, -1):
        lv = plan[li]
        w = dataclasses.replace(weights, delta=0.0 if delta < 0 else delta)
        P = Problem(Rs[li], Ts[li], lv["spacing"], kp_x, kp_t, w)
        nn = P.nodes
        if u is None:
            u = np.zeros((3, nn[2], nn[1], nn[0]))
            if delta < 0:
                delta = P.adaptive_delta(u)
                P.w.delta = delta
        else:
            u = prolong(u, plan[li + 1]["halve"])
        iters = params.iters[L - 1 - li]
        if params.optimizer == "lbfgs":
            u, reps = lbfgs_run(P, u, iters, params.lbfgs)
        else:
            reps = []
            for _ in range(iters):
                u, rep = gn_pcg_step(P, u, params.step)
                reps.append(rep)
                if not rep["accepted"]:
                    break
        out.append(dict(shape=lv["shape"], spacing=lv["spacing"], delta=delta, reports=reps,
                        J_final=P.objective(u)["J"]))
    return u, out


# ------------------------------------------------------------------------------------
# keypoint stage (Sec. II-C2, II-C3): NGF matching cost over a displacement grid, a
# minimum spanning tree over the keypoints, min-sum belief propagation on the tree
# ------------------------------------------------------------------------------------

KP_PATCH = (-3, -1, 1, 3)   # patch offsets per axis: a 7^3 patch with stride 2 (64 voxels)


def kp_labels(R: int = 16, step: int = 2):
    """Label displacements in voxels, [(2R+1)^3][3] (x, y, z), ordered [iz][iy][ix]."""
    i = np.arange(2 * R + 1) - R
    dz, dy, dx = np.meshgrid(i, i, i, indexing="ij")
    return step * np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1)


def kp_cost_volume(F, M, spacing, kps, eta, R: int = 16, step: int = 2):
    """D_KP(k, d) of eq. 2 for keypoints kps (integer voxel indices [n][3], x, y, z) and
    labels d = step (i - R) voxels, i = 0..2R per axis: [n][(2R+1)^3] (label order of
    kp_labels).  Gradients by central differences (HU/mm), zero outside the volume."""
    gF = image_gradient(F, spacing)
    gM = image_gradient(M, spacing)
    nz, ny, nx = np.asarray(F).shape
    kps = _i64(np.asarray(kps).reshape(-1, 3))
    nl = 2 * R + 1
    out = np.empty((len(kps), nl ** 3))
    _load().or_kp_cost(_p(_i64([nx, ny, nz])), _p(gF), _p(gM), len(kps), _p(kps), float(eta), int(R), int(step),
                       _p(out))
    return out


def kp_edge_weight(x, inten, k, q, sigma_I: float = 150.0):
    """Spatial-plus-intensity distance of two keypoints (the denominator of eq. 3)."""
    return float(np.linalg.norm(x[k] - x[q]) + abs(float(inten[k]) - float(inten[q])) / sigma_I)


def kp_mst(x, inten, sigma_I: float = 150.0):
    """Minimum spanning tree over all keypoint pairs with the edge cost of eq. 3's
    denominator.  Ties between edge costs are broken by the strict order (cost, lower
    index, higher index), which makes the tree unique; Kruskal's algorithm on that order.
    The tree is rooted at keypoint 0 and visited breadth first (neighbours in increasing
    order).  Returns (parent [n] with parent[0] = -1, visit order)."""
    x = _f64(x).reshape(-1, 3)
    inten = _f64(inten).ravel()
    n = len(x)
    ii, jj = np.triu_indices(n, 1)
    d = x[jj] - x[ii]
    w = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]) + np.abs(inten[jj] - inten[ii]) / sigma_I
    srt = np.lexsort((jj, ii, w))
    uf = list(range(n))

    def find(a):
        while uf[a] != a:
            uf[a] = uf[uf[a]]
            a = uf[a]
        return a

    adj = [[] for _ in range(n)]
    taken = 0
    for e in srt:
        if taken == n - 1:
            break
        a, b = int(ii[e]), int(jj[e])
        ra, rb = find(a), find(b)
        if ra == rb:
            continue
        uf[max(ra, rb)] = min(ra, rb)
        adj[a].append(b)
        adj[b].append(a)
        taken += 1
    parent = np.full(n, -1, np.int64)
    seen = np.zeros(n, bool)
    seen[0] = True
    order = [0]
    h = 0
    while h < len(order):
        a = order[h]
        h += 1
        for b in sorted(adj[a]):
            if not seen[b]:
                seen[b] = True
                parent[b] = a
                order.append(b)
    return parent, np.asarray(order, np.int64)


def kp_mincon_bruteforce(f, c, R: int = 16, step: int = 2):
    """out(d_q) = min over d_k of f(d_k) + c |d_k - d_q|^2 (labels of kp_labels, |.| in
    voxels): the plain definition, O(L^2)."""
    lab = kp_labels(R, step).astype(np.float64)
    f = _f64(f).ravel()
    out = np.empty_like(f)
    for qi in range(len(f)):
        out[qi] = np.min(f + c * np.sum((lab - lab[qi]) ** 2, axis=1))
    return out


def kp_mincon(f, c, R: int = 16, step: int = 2):
    """The same minimum by separability of |.|^2: a 1-D minimum along x, then y, then z
    (each over the 2R+1 labels of its line)."""
    nl = 2 * R + 1
    g = _f64(f).reshape(nl, nl, nl)
    i = np.arange(nl)
    pen = c * (step * (i[:, None] - i[None, :])) ** 2   # [out][in]
    for ax in (2, 1, 0):
        gm = np.moveaxis(g, ax, -1)                          # [..., in]
        g = np.moveaxis(np.min(gm[..., None, :] + pen, axis=-1), -1, ax)
    return g.ravel()


def kp_belief_propagation(D, parent, order, x, inten, alpha_kp: float, sigma_I: float = 150.0, R: int = 16,
                          step: int = 2, mincon=None):
    """Min-sum belief propagation on the tree (eq. 4 with the regulariser of eq. 3):
    inward pass from the leaves, m_kq(d_q) = min_{d_k} h_k(d_k) + R_KP(d_k, d_q) with
    h_k = D(k, .) + sum of the messages of k's children; outward pass from the root,
    m_qk(d_k) = min_{d_q} (M_q(d_q) - m_kq(d_q)) + R_KP(d_q, d_k), and min-marginals
    M_k = h_k + m_qk (M_root = h_root).  R_KP = alpha_kp |d_k - d_q|^2 / w_kq with the
    label displacement in mm (voxel size 1 mm at the keypoint stage).  Returns
    (min-marginals [n][L], inward messages [n][L])."""
    mincon = mincon or kp_mincon
    D = _f64(D)
    n, L = D.shape
    x = _f64(x).reshape(-1, 3)
    h = D.copy()
    msg = np.zeros_like(D)
    cw = np.zeros(n)
    for k in range(n):
        if parent[k] >= 0:
            cw[k] = alpha_kp / kp_edge_weight(x, inten, k, parent[k], sigma_I)
    for k in order[::-1]:
        if parent[k] >= 0:
            msg[k] = mincon(h[k], cw[k], R, step)
            h[parent[k]] += msg[k]
    marg = np.empty_like(D)
    marg[order[0]] = h[order[0]]
    for k in order[1:]:
        q = parent[k]
        marg[k] = h[k] + mincon(marg[q] - msg[k], cw[k], R, step)
    return marg, msg


def kp_argmin(marg):
    """Label of smallest min-marginal per keypoint (lowest index on ties)."""
    return np.argmin(_f64(marg), axis=1)
