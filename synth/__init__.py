"""Seeded synthetic lung-CT-shaped inputs for the dense registration objective.

This module only *makes inputs*: a thorax-like fixed volume R, a moving volume T
obtained by warping R with a known smooth field, the matching displacement at the
control-grid nodes, keypoint pairs and random direction vectors.  It holds none
of the registration method's arithmetic (no NGF, regulariser, volume-change or
keypoint terms) and is shared by the FP64 oracle tests and by the GPU path, which
never import each other.

The shapes, spacings and intensity ranges follow the lung CT data the paper
evaluates on (512 x 512 voxels per slice, about 120 slices, 0.59-0.74 mm in plane
and 2.5 mm slice distance; Sec. III-A).  The data sets themselves are not used or
reproduced: the phantom below stands in for them.

Conventions
-----------
* ``shape`` is (Nx, Ny, Nz); volumes are stored as ``[Nz][Ny][Nx]`` float32.
* ``spacing`` is (hx, hy, hz) in mm; voxel (i, j, k) has its centre at
  ((i + 1/2) hx, (j + 1/2) hy, (k + 1/2) hz).
* The control grid has 4 voxels per cell and axis, i.e. (N/4 + 1) nodes per axis
  at positions p * 4h; node fields are float32 ``[3][nz][ny][nx]`` (components x, y, z).
* T(z) = (R(psi(z)) + 1000) * det(grad psi(z)) - 1000 with psi(z) = z + w(z), so the
  exact registration transformation is y = psi^{-1} and the true displacement is
  u_true = psi^{-1} - id.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy import ndimage

__all__ = ["PairConfig", "CONFIGS", "make_pair", "batch_configs", "node_shape",
           "random_direction", "Field"]

AIR_HU = -1000.0
BODY_HU = 40.0
LUNG_HU = -850.0
VESSEL_HU = 40.0
CELL = 4  # voxels per control-grid cell and axis


@dataclasses.dataclass(frozen=True)
class PairConfig:
    shape: Tuple[int, int, int]                 # (Nx, Ny, Nz)
    spacing: Tuple[float, float, float]         # (hx, hy, hz) mm
    n_tubes: int = 40
    field: str = "gauss"                        # "gauss" | "breathing"
    field_max: float = 6.0                      # gauss: max |w| in mm
    amp_z: float = 25.0                         # breathing: craniocaudal amplitude (mm)
    amp_y: float = 8.0                          # breathing: anterior-posterior amplitude (mm)
    n_kp: int = 200
    kp_noise: float = 0.0                       # std of N(0, s^2) added per target component
    texture_sd: float = 20.0
    smooth_sigma: float = 0.5                   # voxels; 0 disables
    seed: int = 0


CONFIGS: Dict[str, PairConfig] = {
    # plain method, small: oracle finishes in seconds
    "cfg0": PairConfig(shape=(64, 64, 48), spacing=(1.5, 1.5, 1.5), n_tubes=40,
                       field="gauss", field_max=6.0, n_kp=200, seed=0),
    # full-size plain GPU path: 512 x 512 x 128 at 0.7 x 0.7 x 2.5 mm
    "cfg1": PairConfig(shape=(512, 512, 128), spacing=(0.7, 0.7, 2.5), n_tubes=300,
                       field="breathing", amp_z=25.0, amp_y=8.0, n_kp=2000,
                       kp_noise=1.0, seed=1),
    # differentiation form: one of 8 pairs (seeds 200..207) of 192 x 192 x 160 at 1 mm
    "cfg2": PairConfig(shape=(192, 192, 160), spacing=(1.0, 1.0, 1.0), n_tubes=120,
                       field="breathing", amp_z=25.0, amp_y=8.0, n_kp=2000,
                       kp_noise=1.0, seed=200),
    # keypoint stage: the full-size field of view resampled to 1 mm isotropic, 3500
    # keypoints in the lungs
    "kp": PairConfig(shape=(356, 356, 320), spacing=(1.0, 1.0, 1.0), n_tubes=300,
                     field="breathing", amp_z=25.0, amp_y=8.0, n_kp=3500, seed=5),
    # precision form: 512 x 512 x 256 at 0.7 x 0.7 x 1.25 mm
    "cfg4": PairConfig(shape=(512, 512, 256), spacing=(0.7, 0.7, 1.25), n_tubes=300,
                       field="breathing", amp_z=25.0, amp_y=8.0, n_kp=2000,
                       kp_noise=1.0, seed=4),
}

# Pyramid shapes of the batching form; spacings keep the field of view fixed at
# 358.4 x 358.4 x 320 mm.
PYRAMID_SHAPES = [((64, 64, 32), (5.6, 5.6, 10.0)),
                  ((128, 128, 64), (2.8, 2.8, 5.0)),
                  ((256, 256, 96), (1.4, 1.4, 320.0 / 96.0)),
                  ((512, 512, 128), (0.7, 0.7, 2.5))]


def batch_configs(n_pairs: int = 24, shape_seed: int = 300, first_pair_seed: int = 301,
                  tubes_per_mm3: Optional[float] = None) -> List[PairConfig]:
    """Uneven batch: each pair's shape is drawn uniformly from the pyramid shapes."""
    rng = np.random.default_rng(shape_seed)
    picks = rng.integers(0, len(PYRAMID_SHAPES), size=n_pairs)
    out = []
    for p, s in enumerate(picks):
        shape, spacing = PYRAMID_SHAPES[int(s)]
        out.append(PairConfig(shape=shape, spacing=spacing, n_tubes=60 + 40 * int(s),
                              field="breathing", amp_z=25.0, amp_y=8.0, n_kp=500,
                              kp_noise=1.0, seed=first_pair_seed + p))
    return out


def node_shape(shape: Tuple[int, int, int]) -> Tuple[int, int, int]:
    """(nx, ny, nz) node counts of the 4-voxel control grid."""
    return tuple(s // CELL + 1 for s in shape)  # type: ignore[return-value]


# --------------------------------------------------------------------------------------
# Smooth deformation psi(z) = z + w(z), evaluated analytically (value and Jacobian)
# --------------------------------------------------------------------------------------

class Field:
    """w(z) as an analytic sum of smooth terms, with its 3x3 Jacobian."""

    def __init__(self, cfg: PairConfig, rng: np.random.Generator):
        nx, ny, nz = cfg.shape
        hx, hy, hz = cfg.spacing
        self.ext = np.array([nx * hx, ny * hy, nz * hz])
        self.kind = cfg.field
        ext = self.ext
        # Gaussian bumps: centres in the central 60 % of the box, sigma in [15, 30] mm
        n_g = 8 if cfg.field == "gauss" else 4
        self.mu = ext * (0.2 + 0.6 * rng.random((n_g, 3)))
        self.sig = 15.0 + 15.0 * rng.random(n_g)
        amp = rng.standard_normal((n_g, 3))
        self.amp = amp
        self.scale_g = 1.0
        self.scale_b = 1.0
        self.amp_z = cfg.amp_z
        self.amp_y = cfg.amp_y
        # normalise the Gaussian part on a ~2 mm sample grid
        pts = self._sample_points()
        gmax = np.max(np.linalg.norm(self._gauss(pts)[0], axis=-1))
        target = cfg.field_max if cfg.field == "gauss" else 3.0
        self.scale_g = target / max(gmax, 1e-12)
        # keep the warp a diffeomorphism with a comfortable margin
        for _ in range(20):
            dmin = np.min(np.linalg.det(np.eye(3) + self.jac(pts)))
            if dmin > 0.2:
                break
            self.scale_g *= 0.8
            self.scale_b *= 0.8
        self.min_det = float(dmin)

    def _sample_points(self) -> np.ndarray:
        g = [np.linspace(0.0, e, max(int(e / 2.0), 8)) for e in self.ext]
        zz, yy, xx = np.meshgrid(g[2], g[1], g[0], indexing="ij")
        return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=-1)

    def _gauss(self, p: np.ndarray, want_jac: bool = True):
        w = np.zeros_like(p)
        jac = np.zeros(p.shape + (3,)) if want_jac else None
        for mu, sig, a in zip(self.mu, self.sig, self.amp):
            d = p - mu
            e = np.exp(-np.sum(d * d, axis=-1) / (2.0 * sig * sig))
            w += e[..., None] * a
            if want_jac:
                # d/dz_b of a_c * e = -a_c * e * d_b / sig^2
                jac += -(a[None, :, None] * (e[..., None] * d)[..., None, :]) / (sig * sig)
        return w * self.scale_g, (jac * self.scale_g if want_jac else None)

    def _breathing(self, p: np.ndarray, want_jac: bool = True):
        ex, ey, ez = self.ext
        cx, cy = ex / 2.0, ey / 2.0
        sx, sy = 0.3 * ex, 0.3 * ey
        z = p[..., 2]
        prof = 0.5 * (1.0 + np.cos(np.pi * np.clip(z / ez, 0.0, 1.0)))   # 1 at base, 0 at apex
        lat = np.exp(-((p[..., 0] - cx) ** 2 / (2 * sx * sx) + (p[..., 1] - cy) ** 2 / (2 * sy * sy)))
        w = np.zeros_like(p)
        az, ay = -self.amp_z * self.scale_b, self.amp_y * self.scale_b
        w[..., 2] = az * prof * lat
        w[..., 1] = ay * prof * lat
        if not want_jac:
            return w, None
        dprof = -0.5 * np.pi / ez * np.sin(np.pi * np.clip(z / ez, 0.0, 1.0))
        dlat_x = -lat * (p[..., 0] - cx) / (sx * sx)
        dlat_y = -lat * (p[..., 1] - cy) / (sy * sy)
        jac = np.zeros(p.shape + (3,))
        for c, a in ((2, az), (1, ay)):
            jac[..., c, 0] = a * prof * dlat_x
            jac[..., c, 1] = a * prof * dlat_y
            jac[..., c, 2] = a * dprof * lat
        return w, jac

    def value(self, p: np.ndarray) -> np.ndarray:
        w, _ = self._gauss(p, want_jac=False)
        if self.kind == "breathing":
            w = w + self._breathing(p, want_jac=False)[0]
        return w

    def jac(self, p: np.ndarray) -> np.ndarray:
        _, j = self._gauss(p)
        if self.kind == "breathing":
            j = j + self._breathing(p)[1]
        return j

    def grid(self, xs: np.ndarray, ys: np.ndarray, zs: np.ndarray):
        """w and det(I + grad w) on the tensor grid zs x ys x xs (float32 [nz][ny][nx]),
        using that every term is a product of one-dimensional factors."""
        shp = (len(zs), len(ys), len(xs))
        X = xs[None, None, :]
        Y = ys[:, None][None]
        Z = zs[:, None, None]
        w = [np.zeros(shp, np.float32) for _ in range(3)]
        J = [[np.zeros(shp, np.float32) for _ in range(3)] for _ in range(3)]
        for mu, sig, a in zip(self.mu, self.sig, self.amp):
            s2 = 2.0 * sig * sig
            ex = np.exp(-(xs - mu[0]) ** 2 / s2)
            ey = np.exp(-(ys - mu[1]) ** 2 / s2)
            ez = np.exp(-(zs - mu[2]) ** 2 / s2)
            dx = -(xs - mu[0]) / (sig * sig) * ex
            dy = -(ys - mu[1]) / (sig * sig) * ey
            dz = -(zs - mu[2]) / (sig * sig) * ez
            e = (ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).astype(np.float32)
            de = [(ez[:, None, None] * ey[None, :, None] * dx[None, None, :]).astype(np.float32),
                  (ez[:, None, None] * dy[None, :, None] * ex[None, None, :]).astype(np.float32),
                  (dz[:, None, None] * ey[None, :, None] * ex[None, None, :]).astype(np.float32)]
            for c in range(3):
                ac = np.float32(a[c] * self.scale_g)
                w[c] += ac * e
                for b in range(3):
                    J[c][b] += ac * de[b]
        if self.kind == "breathing":
            ex_, ey_, ez_ = self.ext
            cx, cy = ex_ / 2.0, ey_ / 2.0
            sx, sy = 0.3 * ex_, 0.3 * ey_
            zc = np.clip(zs / ez_, 0.0, 1.0)
            prof = 0.5 * (1.0 + np.cos(np.pi * zc))
            dprof = -0.5 * np.pi / ez_ * np.sin(np.pi * zc)
            lx = np.exp(-(xs - cx) ** 2 / (2 * sx * sx))
            ly = np.exp(-(ys - cy) ** 2 / (2 * sy * sy))
            dlx = -lx * (xs - cx) / (sx * sx)
            dly = -ly * (ys - cy) / (sy * sy)
            base = (prof[:, None, None] * ly[None, :, None] * lx[None, None, :]).astype(np.float32)
            d_x = (prof[:, None, None] * ly[None, :, None] * dlx[None, None, :]).astype(np.float32)
            d_y = (prof[:, None, None] * dly[None, :, None] * lx[None, None, :]).astype(np.float32)
            d_z = (dprof[:, None, None] * ly[None, :, None] * lx[None, None, :]).astype(np.float32)
            for c, a in ((2, -self.amp_z * self.scale_b), (1, self.amp_y * self.scale_b)):
                a = np.float32(a)
                w[c] += a * base
                J[c][0] += a * d_x
                J[c][1] += a * d_y
                J[c][2] += a * d_z
        for c in range(3):
            J[c][c] += np.float32(1.0)
        det = (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))
        return w, det

    def inverse(self, x: np.ndarray, iters: int = 60) -> np.ndarray:
        """psi^{-1}(x): solve z + w(z) = x by fixed-point iteration z <- x - w(z)."""
        z = x.copy()
        for _ in range(iters):
            z_new = x - self.value(z)
            if np.max(np.abs(z_new - z)) < 1e-9:
                z = z_new
                break
            z = z_new
        return z


# --------------------------------------------------------------------------------------
# Phantom
# --------------------------------------------------------------------------------------

def _axes_mm(shape, spacing):
    return [(np.arange(n) + 0.5) * h for n, h in zip(shape, spacing)]


def _lungs(ext):
    ex, ey, ez = ext
    centres = [np.array([0.5 * ex - 0.21 * ex, 0.52 * ey, 0.55 * ez]),
               np.array([0.5 * ex + 0.21 * ex, 0.52 * ey, 0.55 * ez])]
    semi = np.array([0.16 * ex, 0.27 * ey, 0.42 * ez])
    return centres, semi


def _in_lung(p, ext):
    centres, semi = _lungs(ext)
    inside = np.zeros(p.shape[:-1], dtype=bool)
    for c in centres:
        inside |= np.sum(((p - c) / semi) ** 2, axis=-1) <= 1.0
    return inside


def _random_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _tube_segments(cfg: PairConfig, rng: np.random.Generator, ext) -> List[Tuple[np.ndarray, np.ndarray, float]]:
    """Branching tubes inside the lungs: radius x0.8 per generation, segments 8-25 mm,
    branch probability 0.3, radii between 0.7 and 3 mm."""
    centres, semi = _lungs(ext)
    segs = []
    for _ in range(cfg.n_tubes):
        lung = int(rng.integers(0, 2))
        while True:
            p0 = centres[lung] + semi * (2.0 * rng.random(3) - 1.0)
            if _in_lung(p0[None], ext)[0]:
                break
        stack = [(p0, _random_unit(rng), 2.0 + rng.random())]
        count = 0
        while stack and count < 40:
            p, d, r = stack.pop()
            if r < 0.7:
                continue
            length = 8.0 + 17.0 * rng.random()
            q = p + length * d
            segs.append((p, q, r))
            count += 1
            # continuation with a gently bent direction
            d1 = d + 0.35 * _random_unit(rng)
            stack.append((q, d1 / np.linalg.norm(d1), 0.8 * r))
            if rng.random() < 0.3:
                d2 = d + 0.9 * _random_unit(rng)
                stack.append((q, d2 / np.linalg.norm(d2), 0.8 * r))
    return segs


def _raster_segments(vol, segs, shape, spacing, value):
    nx, ny, nz = shape
    h = np.asarray(spacing)
    for p, q, r in segs:
        lo = np.floor((np.minimum(p, q) - r) / h - 0.5).astype(int)
        hi = np.ceil((np.maximum(p, q) + r) / h - 0.5).astype(int)
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, np.array([nx - 1, ny - 1, nz - 1]))
        if np.any(hi < lo):
            continue
        xs = (np.arange(lo[0], hi[0] + 1) + 0.5) * h[0]
        ys = (np.arange(lo[1], hi[1] + 1) + 0.5) * h[1]
        zs = (np.arange(lo[2], hi[2] + 1) + 0.5) * h[2]
        d = q - p
        dd = float(d @ d)
        # distance from each voxel centre to the segment
        px = xs[None, None, :] - p[0]
        py = ys[None, :, None] - p[1]
        pz = zs[:, None, None] - p[2]
        t = np.clip((px * d[0] + py * d[1] + pz * d[2]) / max(dd, 1e-12), 0.0, 1.0)
        dist2 = (px - t * d[0]) ** 2 + (py - t * d[1]) ** 2 + (pz - t * d[2]) ** 2
        sub = vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        sub[dist2 <= r * r] = value


def _phantom(cfg: PairConfig, rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    nx, ny, nz = cfg.shape
    ext = np.array([nx * cfg.spacing[0], ny * cfg.spacing[1], nz * cfg.spacing[2]])
    xs, ys, zs = _axes_mm(cfg.shape, cfg.spacing)
    X = xs[None, None, :]
    Y = ys[None, :, None]
    Z = zs[:, None, None]
    body = ((X - 0.5 * ext[0]) / (0.46 * ext[0])) ** 2 + ((Y - 0.5 * ext[1]) / (0.40 * ext[1])) ** 2 \
        + ((Z - 0.5 * ext[2]) / (0.80 * ext[2])) ** 2 <= 1.0
    vol = np.full((nz, ny, nx), AIR_HU, dtype=np.float32)
    vol[body] = BODY_HU
    centres, semi = _lungs(ext)
    lung = np.zeros((nz, ny, nx), dtype=bool)
    for c in centres:
        lung |= ((X - c[0]) / semi[0]) ** 2 + ((Y - c[1]) / semi[1]) ** 2 + ((Z - c[2]) / semi[2]) ** 2 <= 1.0
    tex = rng.standard_normal(int(lung.sum()), dtype=np.float32) * np.float32(cfg.texture_sd)
    vol[lung] = np.float32(LUNG_HU) + tex
    vessels = np.zeros((nz, ny, nx), dtype=np.float32)
    _raster_segments(vessels, _tube_segments(cfg, rng, ext), cfg.shape, cfg.spacing, 1.0)
    vol = np.where(lung & (vessels > 0), np.float32(VESSEL_HU), vol).astype(np.float32)
    if cfg.smooth_sigma > 0:
        vol = ndimage.gaussian_filter(vol, cfg.smooth_sigma, mode="nearest").astype(np.float32)
    return vol, lung


def _warp_moving(R: np.ndarray, field: Field, cfg: PairConfig, lung: Optional[np.ndarray] = None):
    """T(z) = (R(psi(z)) + 1000) det(grad psi(z)) - 1000, evaluated slab by slab; with the
    fixed lung mask given, also the moving lung mask (lung(psi(z)) by linear interpolation,
    thresholded at 1/2) as uint8."""
    nx, ny, nz = cfg.shape
    h = np.asarray(cfg.spacing)
    xs, ys, zs = _axes_mm(cfg.shape, cfg.spacing)
    T = np.empty_like(R)
    mT = None if lung is None else np.empty(R.shape, np.uint8)
    lf = None if lung is None else lung.astype(np.float32)
    slab = max(1, int(4_000_000 // (nx * ny)))
    for k0 in range(0, nz, slab):
        k1 = min(nz, k0 + slab)
        w, det = field.grid(xs, ys, zs[k0:k1])
        # continuous voxel index (z, y, x order) of psi(z) = z + w(z)
        qz = (zs[k0:k1, None, None] + w[2]) / h[2] - 0.5
        qy = (ys[None, :, None] + w[1]) / h[1] - 0.5
        qx = (xs[None, None, :] + w[0]) / h[0] - 0.5
        coords = np.stack([qz.ravel(), qy.ravel(), qx.ravel()], axis=0).astype(np.float32)
        Rw = ndimage.map_coordinates(R, coords, order=1, mode="nearest").reshape(w[0].shape)
        T[k0:k1] = ((Rw + 1000.0) * det - 1000.0).astype(np.float32)
        if lf is not None:
            mw = ndimage.map_coordinates(lf, coords, order=1, mode="nearest").reshape(w[0].shape)
            mT[k0:k1] = (mw >= 0.5).astype(np.uint8)
    return T if lung is None else (T, mT)


def random_direction(nodes: Tuple[int, int, int], seed: int) -> np.ndarray:
    """v ~ N(0, 1 mm^2) per node and component, float32 [3][nz][ny][nx]."""
    nx, ny, nz = nodes
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, nz, ny, nx)).astype(np.float32)


def make_pair(cfg: PairConfig | str, seed: Optional[int] = None) -> dict:
    """Generate one synthetic pair.

    Returns a dict with R, T (float32 [Nz][Ny][Nx]), shape, spacing, nodes,
    u_true (float32 [3][nz][ny][nx]), kp_x, kp_t (float32 [n][3], mm),
    v (float32 node field for Hessian-vector tests), min_det of grad psi, and the binary
    lung masks mask_R, mask_T (uint8 [Nz][Ny][Nx]) of the fixed and moving images.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if seed is not None:
        cfg = dataclasses.replace(cfg, seed=seed)
    for s in cfg.shape:
        if s % CELL:
            raise ValueError("every volume dimension must be a multiple of 4")
    rng = np.random.default_rng(cfg.seed)
    R, lung = _phantom(cfg, rng)
    field = Field(cfg, rng)
    T, mask_T = _warp_moving(R, field, cfg, lung)
    nodes = node_shape(cfg.shape)
    H = np.asarray(cfg.spacing) * CELL
    pz, py, px = np.meshgrid(np.arange(nodes[2]), np.arange(nodes[1]), np.arange(nodes[0]), indexing="ij")
    Xn = np.stack([px * H[0], py * H[1], pz * H[2]], axis=-1).astype(np.float64)
    un = field.inverse(Xn) - Xn
    u_true = np.ascontiguousarray(np.moveaxis(un, -1, 0)).astype(np.float32)
    # keypoints uniform inside the lungs (and strictly inside the box)
    ext = np.array([cfg.shape[i] * cfg.spacing[i] for i in range(3)])
    pts = []
    need = cfg.n_kp
    while need > 0:
        cand = ext * (0.02 + 0.96 * rng.random((4 * need + 16, 3)))
        cand = cand[_in_lung(cand, ext)]
        pts.append(cand[:need])
        need -= len(pts[-1])
    kp_x = np.concatenate(pts, axis=0) if pts else np.zeros((0, 3))
    kp_t = field.inverse(kp_x) if len(kp_x) else np.zeros((0, 3))
    if cfg.kp_noise > 0 and len(kp_t):
        kp_t = kp_t + cfg.kp_noise * rng.standard_normal(kp_t.shape)
    v = random_direction(nodes, cfg.seed + 1000)
    return dict(R=R, T=T, shape=cfg.shape, spacing=cfg.spacing, nodes=nodes,
                u_true=u_true, kp_x=kp_x.astype(np.float32), kp_t=kp_t.astype(np.float32),
                v=v, lung=lung, mask_R=lung.astype(np.uint8), mask_T=mask_T, min_det=field.min_det, cfg=cfg)


def small_pair(shape=(16, 16, 12), spacing=(1.5, 1.5, 1.5), seed=0, n_tubes=6, n_kp=20,
               field_max=3.0) -> dict:
    """A tiny pair for brute-force and parity tests (same recipe, fewer voxels)."""
    cfg = PairConfig(shape=shape, spacing=spacing, n_tubes=n_tubes, field="gauss",
                     field_max=field_max, n_kp=n_kp, seed=seed)
    return make_pair(cfg)
