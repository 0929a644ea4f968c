"""Pins of the FP64 oracle against facts fixed outside it.

Each test ties one part of the oracle to a library routine, a closed form, an
invariant stated in the paper, finite differences, or brute force on tiny inputs,
chosen so that a dropped term, a wrong sign/index or a transposed operand fails.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy import ndimage

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def rng(seed=0):
    return np.random.default_rng(seed)


def smooth_volume(shape_zyx, seed, sigma=1.5, scale=100.0):
    r = rng(seed).standard_normal(shape_zyx)
    return (ndimage.gaussian_filter(r, sigma) * scale).astype(np.float32)


def grid_sample_vec(field, q):
    """Library trilinear sampling: torch grid_sample, align_corners=False, zero padding.
    field [Nz][Ny][Nx][3] (float64), q [n][3] continuous voxel index (x, y, z)."""
    nz, ny, nx, _ = field.shape
    inp = torch.from_numpy(np.ascontiguousarray(np.moveaxis(field, -1, 0)))[None]
    n = np.array([nx, ny, nz], np.float64)
    g = (2.0 * q + 1.0) / n - 1.0
    grid = torch.from_numpy(g)[None, None, None]
    out = F.grid_sample(inp, grid, mode="bilinear", padding_mode="zeros", align_corners=False)
    return out[0, :, 0, 0, :].numpy().T


def conv_gradient(img, h):
    """Library central differences with replicate padding (torch conv3d), [Nz][Ny][Nx][3]."""
    t = torch.from_numpy(img.astype(np.float64))[None, None]
    t = F.pad(t, (1, 1, 1, 1, 1, 1), mode="replicate")
    outs = []
    for axis in range(3):  # x, y, z
        k = torch.zeros(3, 3, 3, dtype=torch.float64)
        if axis == 0:
            k[1, 1, 0], k[1, 1, 2] = -1.0, 1.0
        elif axis == 1:
            k[1, 0, 1], k[1, 2, 1] = -1.0, 1.0
        else:
            k[0, 1, 1], k[2, 1, 1] = -1.0, 1.0
        outs.append(F.conv3d(t, k[None, None])[0, 0].numpy() / (2.0 * h[axis]))
    return np.stack(outs, axis=-1)


def trilinear_nodes(u, H, pts):
    """Library trilinear evaluation of a node field at physical points (scipy)."""
    coords = np.stack([pts[:, 2] / H[2], pts[:, 1] / H[1], pts[:, 0] / H[0]], axis=0)
    return np.stack([ndimage.map_coordinates(u[c], coords, order=1, mode="nearest") for c in range(3)], axis=-1)


# ---------------------------------------------------------------------------------
# image gradients and sampling (eq. 1 ingredients)
# ---------------------------------------------------------------------------------

def test_image_gradient_matches_library_stencil():
    img = smooth_volume((7, 9, 11), 1)
    h = (0.7, 0.9, 2.5)
    np.testing.assert_allclose(oracle.image_gradient(img, h), conv_gradient(img, h), rtol=0, atol=1e-12)


def test_sampling_matches_grid_sample_including_outside():
    f = rng(2).standard_normal((6, 7, 8, 3))
    q = rng(3).uniform(-2.5, 9.5, size=(500, 3))
    G, _ = oracle.sample_points(f, (1.0, 1.0, 1.0), q)
    np.testing.assert_allclose(G, grid_sample_vec(f, q), rtol=0, atol=1e-12)


def test_sampling_integer_points_return_grid_values():
    f = rng(4).standard_normal((5, 6, 7, 3))
    idx = np.stack(np.meshgrid(np.arange(7), np.arange(6), np.arange(5), indexing="ij"), -1).reshape(-1, 3)
    G, _ = oracle.sample_points(f, (1.0, 1.0, 1.0), idx.astype(np.float64))
    np.testing.assert_array_equal(G, f[idx[:, 2], idx[:, 1], idx[:, 0]])


def test_sampling_jacobian_is_derivative_of_library_interpolant():
    f = rng(5).standard_normal((6, 6, 6, 3))
    h = np.array([0.7, 1.1, 2.5])
    base = rng(6).integers(0, 5, size=(200, 3)) + rng(7).uniform(0.1, 0.9, size=(200, 3))
    _, JG = oracle.sample_points(f, h, base)
    eps = 1e-4
    for a in range(3):
        d = np.zeros(3)
        d[a] = eps
        fd = (grid_sample_vec(f, base + d) - grid_sample_vec(f, base - d)) / (2 * eps * h[a])
        np.testing.assert_allclose(JG[:, :, a], fd, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------------
# NGF (eq. 1)
# ---------------------------------------------------------------------------------

def small_case(seed=0, shape=(16, 16, 12), spacing=(1.5, 1.5, 1.5)):
    return synth.small_pair(shape=shape, spacing=spacing, seed=seed)


def test_ngf_identical_images_zero_distance_and_gradient():
    d = small_case()
    gR = oracle.image_gradient(d["R"], d["spacing"])
    u = np.zeros_like(d["u_true"], np.float64)
    res = oracle.ngf(gR, gR, d["spacing"], 10.0, u)
    assert res["D"] == 0.0
    assert np.all(res["g"] == 0.0)


@pytest.mark.parametrize("axis,k", [(0, 3), (1, 2), (2, -2)])
def test_ngf_integer_translation_zero_inside(axis, k):
    """T(x) = R(x - k h e_a) and u = k h e_a align every voxel whose stencil stays in
    the copied region; the opposite displacement does not."""
    nx, ny, nz = 24, 20, 16
    h = (1.5, 1.25, 2.0)
    R = smooth_volume((nz, ny, nx), 11)
    T = np.roll(R, k, axis=2 - axis)
    gR = oracle.image_gradient(R, h)
    gT = oracle.image_gradient(T, h)
    nn = oracle.node_shape((nx, ny, nz))
    u = np.zeros((3, nn[2], nn[1], nn[0]))
    u[axis] = k * h[axis]
    c = oracle.ngf(gR, gT, h, 5.0, u)["c"]
    n_ax = (nx, ny, nz)[axis]
    idx = np.arange(n_ax)
    inside = (idx + k - 1 >= max(k, 0) + 0) & (idx + k + 1 <= n_ax - 1 + min(k, 0)) & (idx + k - 1 >= 0)
    # the rolled copy wraps around: only voxels whose warped stencil avoids the seam count
    sl = [slice(None)] * 3
    sl[2 - axis] = inside
    assert np.max(c[tuple(sl)]) < 1e-20
    u[axis] = -k * h[axis]
    c_wrong = oracle.ngf(gR, gT, h, 5.0, u)["c"]
    assert np.mean(c_wrong[tuple(sl)]) > 1e-3


def test_ngf_large_eta_limit_is_gradient_ssd():
    """eta -> inf: eta^2 (1 - r^2) -> |a - b|^2, so eta^2 D -> h^3 sum |grad T(y) - grad R|^2.
    a is sampled with torch grid_sample, b with a library stencil: independent of the oracle."""
    d = small_case(1)
    h = d["spacing"]
    gR = oracle.image_gradient(d["R"], h)
    gT = oracle.image_gradient(d["T"], h)
    u = d["u_true"].astype(np.float64)
    eta = 1e7  # leading correction is O(|grad T|^2 / eta^2) ~ 1e-9 here
    D = oracle.ngf(gR, gT, h, eta, u, want=())["D"]
    nx, ny, nz = d["shape"]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vox = np.stack([(i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]], -1).reshape(-1, 3)
    H = [4 * s for s in h]
    uv = trilinear_nodes(u, H, vox)
    q = (vox + uv) / np.array(h) - 0.5
    a = grid_sample_vec(conv_gradient(d["T"], h), q)
    b = conv_gradient(d["R"], h).reshape(-1, 3)
    ssd = np.prod(h) * np.sum((a - b) ** 2)
    assert abs(eta ** 2 * D - ssd) / ssd < 1e-7


def test_ngf_stable_form_equals_naive_form():
    d = small_case(2)
    h = d["spacing"]
    gR = oracle.image_gradient(d["R"], h)
    gT = oracle.image_gradient(d["T"], h)
    res = oracle.ngf(gR, gT, h, 10.0, d["u_true"])
    np.testing.assert_allclose(res["c"], 1.0 - res["r"] ** 2, rtol=0, atol=1e-12)
    assert np.all(res["c"] >= 0) and np.all(np.abs(res["r"]) <= 1.0 + 1e-15)


def _fd_check(fun, grad, x, coords, eps_list=(1e-4, 1e-5, 1e-6)):
    """Return the worst (over coords) best (over eps) relative central-FD error."""
    worst = 0.0
    scale = np.max(np.abs(grad)) + 1e-300
    for c in coords:
        best = np.inf
        for eps in eps_list:
            xp = x.copy()
            xm = x.copy()
            xp[c] += eps
            xm[c] -= eps
            fd = (fun(xp) - fun(xm)) / (2 * eps)
            best = min(best, abs(fd - grad[c]) / max(abs(grad[c]), 1e-3 * scale))
        worst = max(worst, best)
    return worst


def random_coords(shape, n, seed):
    r = rng(seed)
    return [tuple(int(r.integers(0, s)) for s in shape) for _ in range(n)]


def test_ngf_gradient_matches_finite_differences():
    d = small_case(3)
    h = d["spacing"]
    gR = oracle.image_gradient(d["R"], h)
    gT = oracle.image_gradient(d["T"], h)
    u = d["u_true"].astype(np.float64) * 0.7 + 0.013  # generic positions, off the integer grid
    g = oracle.ngf(gR, gT, h, 10.0, u)["g"]
    err = _fd_check(lambda x: oracle.ngf(gR, gT, h, 10.0, x, want=())["D"], g, u, random_coords(u.shape, 25, 1))
    assert err < 1e-5


def test_ngf_residual_jacobian_matches_finite_differences():
    """J v = s_v . (P v)(x_v): checked against central differences of the residual r(u)."""
    d = small_case(4)
    h = d["spacing"]
    gR = oracle.image_gradient(d["R"], h)
    gT = oracle.image_gradient(d["T"], h)
    u = d["u_true"].astype(np.float64) * 0.5 + 0.021
    res = oracle.ngf(gR, gT, h, 10.0, u)
    v = rng(8).standard_normal(u.shape)
    nx, ny, nz = d["shape"]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vox = np.stack([(i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]], -1).reshape(-1, 3)
    Pv = trilinear_nodes(v, [4 * s for s in h], vox)  # library interpolation of v
    Jv = np.sum(res["s"].reshape(-1, 3) * Pv, axis=1)
    eps = 1e-6
    rp = oracle.ngf(gR, gT, h, 10.0, u + eps * v, want=("r",))["r"].ravel()
    rm = oracle.ngf(gR, gT, h, 10.0, u - eps * v, want=("r",))["r"].ravel()
    fd = (rp - rm) / (2 * eps)
    assert np.linalg.norm(fd - Jv) / np.linalg.norm(Jv) < 1e-5


def test_ngf_gauss_newton_matrix_dense_brute_force_8cubed():
    """8^3 volume, 2x2x2 cells, 27 nodes, 81 unknowns: J assembled column by column from
    finite differences of r(u); 2 h^3 J^T J equals the oracle's GN product and diagonal."""
    d = synth.small_pair(shape=(8, 8, 8), spacing=(2.0, 2.0, 2.0), seed=5, n_tubes=3, n_kp=4)
    h = d["spacing"]
    gR = oracle.image_gradient(d["R"], h)
    gT = oracle.image_gradient(d["T"], h)
    u = d["u_true"].astype(np.float64) * 0.6 + 0.017
    res = oracle.ngf(gR, gT, h, 5.0, u)
    n = u.size
    Jm = np.empty((d["R"].size, n))
    eps = 1e-6
    for col in range(n):
        e = np.zeros(n)
        e[col] = eps
        e = e.reshape(u.shape)
        rp = oracle.ngf(gR, gT, h, 5.0, u + e, want=("r",))["r"].ravel()
        rm = oracle.ngf(gR, gT, h, 5.0, u - e, want=("r",))["r"].ravel()
        Jm[:, col] = (rp - rm) / (2 * eps)
    Hd = 2 * np.prod(h) * Jm.T @ Jm
    Ho = np.stack([oracle.ngf_hv(res["s"], h, np.eye(n)[c].reshape(u.shape)).ravel() for c in range(n)], 1)
    assert np.linalg.norm(Ho - Hd) / np.linalg.norm(Hd) < 1e-6
    np.testing.assert_allclose(res["diag"].ravel(), np.diag(Ho), rtol=1e-12, atol=1e-12 * np.max(np.diag(Ho)))
    assert np.allclose(Ho, Ho.T, rtol=1e-12, atol=1e-12 * np.abs(Ho).max())
    assert np.linalg.eigvalsh(0.5 * (Ho + Ho.T)).min() > -1e-10 * np.abs(Ho).max()


# ---------------------------------------------------------------------------------
# curvature (eq. 5)
# ---------------------------------------------------------------------------------

def node_coords(nn, H):
    pz, py, px = np.meshgrid(np.arange(nn[2]), np.arange(nn[1]), np.arange(nn[0]), indexing="ij")
    return px * H[0], py * H[1], pz * H[2]


def test_curvature_affine_has_zero_energy():
    nn = (7, 6, 5)
    H = (2.8, 2.8, 10.0)
    X, Y, Z = node_coords(nn, H)
    A = rng(9).standard_normal((3, 3))
    w = np.stack([A[c, 0] * X + A[c, 1] * Y + A[c, 2] * Z + c for c in range(3)])
    res = oracle.curvature(w, H)
    assert abs(res["S"]) < 1e-18
    assert np.max(np.abs(res["g"])) < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_curvature_quadratic_closed_form(axis):
    """w_j = c x_a^2 has Laplacian 2c at nodes interior along a and zero elsewhere, so
    S = 1/2 C_H (2c)^2 (number of such nodes)."""
    nn = (7, 6, 5)
    H = (2.8, 2.4, 10.0)
    coords = node_coords(nn, H)
    c = 0.37
    w = np.zeros((3,) + coords[0].shape)
    w[1] = c * coords[axis] ** 2
    S = oracle.curvature(w, H)["S"]
    count = (nn[axis] - 2) * np.prod(nn) // nn[axis]
    expect = 0.5 * np.prod(H) * (2 * c) ** 2 * count
    assert abs(S - expect) / expect < 1e-12


def test_curvature_gradient_fd_and_exact_hessian():
    nn = (5, 6, 4)
    H = (2.0, 3.0, 4.0)
    w = rng(10).standard_normal((3, nn[2], nn[1], nn[0]))
    res = oracle.curvature(w, H)
    err = _fd_check(lambda x: oracle.curvature(x, H)["S"], res["g"], w, random_coords(w.shape, 20, 2))
    assert err < 1e-7
    v = rng(11).standard_normal(w.shape)
    # quadratic: gradient is linear, so g(w + v) - g(w) is the Hessian times v exactly
    np.testing.assert_allclose(oracle.curvature(w + v, H)["g"] - res["g"], oracle.curvature(v, H)["g"],
                               rtol=1e-9, atol=1e-9)
    n = w.size
    Hm = np.stack([oracle.curvature(np.eye(n)[c].reshape(w.shape), H)["g"].ravel() for c in range(n)], 1)
    np.testing.assert_allclose(np.diag(Hm), res["diag"].ravel(), rtol=1e-12)
    assert np.allclose(Hm, Hm.T, atol=1e-12 * np.abs(Hm).max())


# ---------------------------------------------------------------------------------
# volume change control (eq. 7-9)
# ---------------------------------------------------------------------------------

def psi(t):
    return (t - 1.0) ** 2 / t


def test_vcc_identity_is_zero():
    nn = (5, 4, 6)
    H = (2.8, 2.8, 10.0)
    res = oracle.vcc(np.zeros((3, nn[2], nn[1], nn[0])), H)
    # d = (H_x H_y H_z) / C up to the rounding of the two products
    assert abs(res["V"]) < 1e-20 and abs(res["dmin"] - 1.0) < 1e-15 and abs(res["dmax"] - 1.0) < 1e-15
    assert np.max(np.abs(res["g"])) < 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vcc_affine_closed_form(seed):
    """y = A x: every d_abc equals det A, so Vhat = 64 C (#cells) psi(det A)."""
    nn = (4, 5, 3)
    H = (2.8, 2.0, 10.0)
    X, Y, Z = node_coords(nn, H)
    A = np.eye(3) + 0.2 * rng(seed).standard_normal((3, 3))
    assert np.linalg.det(A) > 0
    u = np.stack([(A[c, 0] - (c == 0)) * X + (A[c, 1] - (c == 1)) * Y + (A[c, 2] - (c == 2)) * Z
                  for c in range(3)])
    res = oracle.vcc(u, H)
    ncell = (nn[0] - 1) * (nn[1] - 1) * (nn[2] - 1)
    expect = 64 * np.prod(H) * ncell * psi(np.linalg.det(A))
    assert abs(res["V"] - expect) <= 1e-10 * expect
    assert abs(res["dmin"] - np.linalg.det(A)) < 1e-12 and abs(res["dmax"] - np.linalg.det(A)) < 1e-12


def test_vcc_scaling_symmetry_psi_t_equals_psi_inverse_t():
    """psi(t) = psi(1/t): uniform scaling by s and by 1/s give the same Vhat (d = s^3)."""
    nn = (4, 4, 4)
    H = (2.0, 2.0, 2.0)
    X, Y, Z = node_coords(nn, H)
    vals = []
    for s in (1.3, 1.0 / 1.3):
        u = np.stack([(s - 1) * X, (s - 1) * Y, (s - 1) * Z])
        res = oracle.vcc(u, H)
        assert abs(res["dmin"] - s ** 3) < 1e-12
        vals.append(res["V"])
    assert abs(vals[0] - vals[1]) <= 1e-12 * vals[0]


def _rand_field(nn, seed, amp):
    return amp * rng(seed).standard_normal((3, nn[2], nn[1], nn[0]))


def test_vcc_eq8_expansion_matches_exact_determinant():
    """alpha in [0,1], sum alpha = 1, sum alpha d = det grad y (computed here by central
    differences of the library trilinear interpolant), and min d <= det <= max d."""
    nn = (4, 4, 3)
    H = (2.8, 2.4, 5.0)
    u = _rand_field(nn, 12, 0.4)
    r = rng(13)
    for _ in range(40):
        cell = [int(r.integers(0, nn[a] - 1)) for a in range(3)]
        xi = r.uniform(0.05, 0.95, 3)
        alpha, d, _ = oracle.vcc_cell_expansion(u, H, cell, xi)
        assert np.all(alpha >= 0) and np.all(alpha <= 1) and abs(alpha.sum() - 1) < 1e-14
        x0 = (np.array(cell) + xi) * np.array(H)
        Jm = np.empty((3, 3))
        eps = 1e-3
        for a in range(3):
            e = np.zeros(3)
            e[a] = eps
            yp = x0 + e + trilinear_nodes(u, H, (x0 + e)[None])[0]
            ym = x0 - e + trilinear_nodes(u, H, (x0 - e)[None])[0]
            Jm[:, a] = (yp - ym) / (2 * eps)
        det = np.linalg.det(Jm)
        assert abs(np.dot(alpha, d) - det) < 1e-9
        assert d.min() - 1e-12 <= det <= d.max() + 1e-12


def test_vcc_jensen_upper_bound():
    """Vhat >= V = int psi(det grad y) dx (dense midpoint quadrature of the exact det)."""
    nn = (4, 4, 4)
    H = (2.0, 2.0, 2.0)
    u = _rand_field(nn, 14, 0.15)
    Vhat = oracle.vcc(u, H)["V"]
    det = oracle.det_voxels(u, (0.25, 0.25, 0.25), (24, 24, 24), m=(8, 8, 8))
    V = np.sum(psi(det)) * 0.25 ** 3
    assert np.all(det > 0)
    assert Vhat >= V


def test_vcc_fold_gives_infinity():
    nn = (4, 4, 4)
    H = (2.0, 2.0, 2.0)
    u = np.zeros((3, 4, 4, 4))
    u[0, 1, 1, 1] = -5.0  # push a node past its left neighbour: folding
    res = oracle.vcc(u, H)
    assert np.isinf(res["V"]) and res["nfold"] > 0 and res["dmin"] <= 0


def test_vcc_gradient_fd():
    nn = (4, 5, 3)
    H = (2.8, 2.4, 5.0)
    u = _rand_field(nn, 15, 0.2)
    g = oracle.vcc(u, H)["g"]
    err = _fd_check(lambda x: oracle.vcc(x, H)["V"], g, u, random_coords(u.shape, 25, 3))
    assert err < 1e-6


def test_vcc_gauss_newton_from_fd_of_coefficients():
    """GN matrix C sum psi''(d) grad d grad d^T with grad d from central differences of
    the 64 coefficients of every cell (2x2x2 cells, 81 unknowns)."""
    nn = (3, 3, 3)
    H = (2.0, 2.5, 3.0)
    u = _rand_field(nn, 16, 0.2)
    cells = [(i, j, k) for k in range(2) for j in range(2) for i in range(2)]

    def all_d(x):
        return np.concatenate([oracle.vcc_cell_expansion(x, H, c, [0.5, 0.5, 0.5])[1] for c in cells])

    d0 = all_d(u)
    n = u.size
    Jd = np.empty((d0.size, n))
    eps = 1e-6
    for col in range(n):
        e = np.zeros(n)
        e[col] = eps
        e = e.reshape(u.shape)
        Jd[:, col] = (all_d(u + e) - all_d(u - e)) / (2 * eps)
    C = np.prod(H)
    Hbf = C * Jd.T @ (2.0 / d0 ** 3 * Jd.T).T
    Ho = np.stack([oracle.vcc(u, H, np.eye(n)[c].reshape(u.shape))["Hv"].ravel() for c in range(n)], 1)
    assert np.linalg.norm(Ho - Hbf) / np.linalg.norm(Hbf) < 1e-7
    np.testing.assert_allclose(oracle.vcc(u, H)["diag"].ravel(), np.diag(Ho), rtol=1e-10)


# ---------------------------------------------------------------------------------
# keypoints (eq. 10)
# ---------------------------------------------------------------------------------

def test_keypoints_constant_displacement_closed_form():
    nn = (5, 5, 4)
    H = (2.8, 2.8, 10.0)
    ext = np.array([(nn[a] - 1) * H[a] for a in range(3)])
    x = rng(17).uniform(0, 1, (30, 3)) * ext
    t = x + rng(18).standard_normal((30, 3))
    c = np.array([0.3, -1.2, 2.5])
    u = np.broadcast_to(c[:, None, None, None], (3, nn[2], nn[1], nn[0])).copy()
    K = oracle.keypoints(u, H, x, t)["K"]
    assert abs(K - np.sum((x + c - t) ** 2)) < 1e-10


def test_keypoint_on_node_and_on_upper_border():
    nn = (4, 4, 4)
    H = (2.0, 2.0, 2.0)
    u = rng(19).standard_normal((3, 4, 4, 4))
    x = np.array([[2.0, 4.0, 2.0], [6.0, 6.0, 6.0]])  # an interior node and the far corner
    t = np.zeros_like(x)
    K = oracle.keypoints(u, H, x, t)["K"]
    y0 = x[0] + u[:, 1, 2, 1]
    y1 = x[1] + u[:, 3, 3, 3]
    assert abs(K - (np.sum(y0 ** 2) + np.sum(y1 ** 2))) < 1e-12
    with pytest.raises(ValueError):
        oracle.keypoints(u, H, np.array([[6.5, 1.0, 1.0]]), np.zeros((1, 3)))


def test_keypoints_gradient_and_hessian():
    nn = (4, 5, 3)
    H = (2.8, 2.4, 5.0)
    ext = np.array([(nn[a] - 1) * H[a] for a in range(3)])
    x = rng(20).uniform(0, 1, (15, 3)) * ext
    t = x + rng(21).standard_normal((15, 3))
    u = _rand_field(nn, 22, 0.5)
    res = oracle.keypoints(u, H, x, t)
    err = _fd_check(lambda z: oracle.keypoints(z, H, x, t)["K"], res["g"], u, random_coords(u.shape, 20, 4))
    assert err < 1e-7
    v = _rand_field(nn, 23, 1.0)
    Hv = oracle.keypoints(u, H, x, t, v)["Hv"]
    np.testing.assert_allclose(oracle.keypoints(u + v, H, x, t)["g"] - res["g"], Hv, rtol=1e-9, atol=1e-9)
    # library interpolation of v at the keypoints: <v, Hv> = 2 |P v|^2
    Pv = trilinear_nodes(v, H, x)
    assert abs(np.sum(v * Hv) - 2 * np.sum(Pv ** 2)) < 1e-9 * np.sum(Pv ** 2)


# ---------------------------------------------------------------------------------
# joint GN matrix, PCG and one GN step (eq. 11)
# ---------------------------------------------------------------------------------

def tiny_problem(seed=6, gamma=0.1, shape=(8, 8, 8)):
    d = synth.small_pair(shape=shape, spacing=(2.0, 2.0, 2.0), seed=seed, n_tubes=3, n_kp=6)
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"],
                       oracle.Weights(eta=5.0, alpha=1.0, gamma=gamma))
    u0 = np.zeros(d["u_true"].shape)
    P.w.delta = P.adaptive_delta(u0)
    return P, d


def test_adaptive_delta_balances_data_terms():
    P, d = tiny_problem()
    u0 = np.zeros(d["u_true"].shape)
    o = P.objective(u0)
    assert abs(o["D"] - P.w.delta * o["K"]) < 1e-12 * o["D"]


def test_gn_matrix_symmetric_psd():
    P, d = tiny_problem()
    u = d["u_true"].astype(np.float64) * 0.5
    P.linearise(u)
    n = u.size
    Hm = np.stack([P.gn_hv(np.eye(n)[c].reshape(u.shape)).ravel() for c in range(n)], 1)
    assert np.allclose(Hm, Hm.T, atol=1e-11 * np.abs(Hm).max())
    assert np.linalg.eigvalsh(0.5 * (Hm + Hm.T)).min() > -1e-9 * np.abs(Hm).max()


def test_pcg_reaches_dense_solve():
    P, d = tiny_problem()
    u = d["u_true"].astype(np.float64) * 0.5
    lin = P.linearise(u)
    n = u.size
    Hm = np.stack([P.gn_hv(np.eye(n)[c].reshape(u.shape)).ravel() for c in range(n)], 1)
    x_ref = np.linalg.solve(Hm, -lin["g"].ravel())
    x, info = oracle.pcg(P.gn_hv, -lin["g"], lin["diag"], iters=4 * n)
    assert np.linalg.norm(x.ravel() - x_ref) / np.linalg.norm(x_ref) < 1e-8
    assert not info["breakdown"]


def test_quadratic_objective_one_gn_step_reaches_minimiser():
    """With a flat image pair (D = 0) and gamma = 0 the objective alpha S + delta K is
    quadratic and its GN matrix exact: one converged step zeroes the gradient."""
    d = synth.small_pair(shape=(12, 12, 8), spacing=(2.0, 2.0, 2.0), seed=7, n_tubes=2, n_kp=10)
    flat = np.full_like(d["R"], -850.0)
    P = oracle.Problem(flat, flat, d["spacing"], d["kp_x"], d["kp_t"],
                       oracle.Weights(eta=5.0, alpha=1.0, gamma=0.0, delta=3.0))
    u0 = np.zeros(d["u_true"].shape)
    u1, rep = oracle.gn_pcg_step(P, u0, oracle.StepParams(pcg_iters=2000, pcg_tol=1e-13))
    assert rep["accepted"] and rep["t"] == 1.0
    g1 = P.linearise(u1)["g"]
    assert np.linalg.norm(g1) < 1e-9 * rep["gnorm"]


def test_gn_step_decreases_objective_and_keeps_det_positive():
    P, d = tiny_problem(gamma=0.1, shape=(16, 16, 12))
    u0 = np.zeros(d["u_true"].shape)
    u1, rep = oracle.gn_pcg_step(P, u0, oracle.StepParams(pcg_iters=20))
    assert rep["accepted"]
    assert rep["trial"]["J"] < rep["J"]
    assert rep["trial"]["nfold"] == 0
    det = oracle.det_voxels(u1, d["spacing"], d["shape"])
    assert det.min() > 0


def test_line_search_rejects_folding_step():
    """A step that folds the grid has Vhat = inf (eq. 9) and must not be taken at t = 1."""
    P, d = tiny_problem(gamma=0.1)
    u = np.zeros(d["u_true"].shape)
    bad = np.zeros_like(u)
    bad[0, 1, 1, 1] = -20.0
    o = P.objective(u + bad)
    assert np.isinf(o["J"]) and o["nfold"] > 0


# ---------------------------------------------------------------------------------
# derivative with respect to the moving image (differentiation form)
# ---------------------------------------------------------------------------------

def test_ngf_grad_T_matches_finite_differences_in_T():
    """dD/dT by central differences of D in single voxel values of T (D recomputed
    from scratch: gradient image, sampling, NGF)."""
    d = small_case(8, shape=(16, 12, 12))
    h = d["spacing"]
    u = d["u_true"].astype(np.float64) * 0.8 + 0.017
    gR = oracle.image_gradient(d["R"], h)
    T = d["T"].astype(np.float64)
    dT = oracle.ngf_grad_T(gR, oracle.image_gradient(T.astype(np.float32), h), h, 10.0, u)

    def D_of(Tv):
        # image_gradient of the oracle takes float32 input: do the stencil in float64 here
        return oracle.ngf(gR, conv_gradient(Tv, h), h, 10.0, u, want=())["D"]

    r = rng(30)
    scale = np.max(np.abs(dT))
    for _ in range(25):
        idx = tuple(int(r.integers(0, s)) for s in T.shape)
        best = np.inf
        for eps in (1e-2, 1e-3, 1e-4):
            Tp = T.copy()
            Tm = T.copy()
            Tp[idx] += eps
            Tm[idx] -= eps
            fd = (D_of(Tp) - D_of(Tm)) / (2 * eps)
            best = min(best, abs(fd - dT[idx]) / max(abs(dT[idx]), 1e-3 * scale))
        assert best < 1e-5, (idx, best)


# ---------------------------------------------------------------------------------
# L-BFGS (Sec. II-D3)
# ---------------------------------------------------------------------------------

def _spd(r, n, lo=0.5):
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    return Q @ np.diag(lo + r.random(n) * 3.0) @ Q.T


def test_lbfgs_two_loop_equals_dense_bfgs_update():
    """The two-loop recursion applies the inverse BFGS matrix built by the explicit
    update H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T from H0^-1, oldest pair first."""
    r = rng(40)
    n = 12
    H0 = _spd(r, n)
    B = _spd(r, n)
    S = [r.standard_normal(n) for _ in range(4)]
    Y = [B @ s + 0.05 * r.standard_normal(n) for s in S]
    assert all(float(s @ y) > 0 for s, y in zip(S, Y))
    Hinv = np.linalg.inv(H0)
    for s, y in zip(S, Y):
        rho = 1.0 / float(s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        Hinv = V.T @ Hinv @ V + rho * np.outer(s, s)
    g = r.standard_normal(n)
    p = oracle.lbfgs_direction(g, S, Y, lambda q: np.linalg.solve(H0, q))
    assert np.allclose(p, -Hinv @ g, rtol=1e-10, atol=1e-12)
    # the secant condition of the newest pair: H_k y = s
    p_y = oracle.lbfgs_direction(-Y[-1], S, Y, lambda q: np.linalg.solve(H0, q))
    assert np.allclose(p_y, S[-1], rtol=1e-9, atol=1e-11)


def test_lbfgs_without_history_is_preconditioned_gradient():
    r = rng(41)
    H0 = _spd(r, 9)
    g = r.standard_normal(9)
    p = oracle.lbfgs_direction(g, [], [], lambda q: np.linalg.solve(H0, q))
    assert np.allclose(p, -np.linalg.solve(H0, g), rtol=1e-12)


def test_lbfgs_minimises_a_quadratic():
    r = rng(42)
    n = 30
    A = _spd(r, n, lo=0.2)
    b = r.standard_normal(n)
    x_star = np.linalg.solve(A, b)
    fg = lambda u: (0.5 * u @ A @ u - b @ u, A @ u - b)
    f = lambda u: 0.5 * u @ A @ u - b @ u
    u, reps = oracle.lbfgs_run(None, np.zeros(n), 80, oracle.LbfgsParams(m=5, ls_max=30), fg=fg, f=f,
                               h0inv=lambda q: q)
    assert np.linalg.norm(u - x_star) <= 1e-8 * np.linalg.norm(x_star)
    Js = [rep["J"] for rep in reps]
    assert all(b_ <= a_ + 1e-14 for a_, b_ in zip(Js, Js[1:]))


def test_h0_solve_matches_dense_solve():
    """H0 = alpha C_H L^T L + tau I on a small node grid: symmetric, eigenvalues >= tau,
    and the solve equals numpy's dense solve."""
    d = small_case(9, shape=(12, 8, 8))
    P = oracle.Problem(d["R"], d["T"], d["spacing"], weights=oracle.Weights(alpha=1.7))
    shape = (3,) + tuple(P.nodes[::-1])
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(oracle.h0_apply(P, e.reshape(shape), 10.0).ravel())
    A = np.array(cols).T
    assert np.allclose(A, A.T, atol=1e-9 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() >= 10.0 - 1e-8
    q = rng(43).standard_normal(shape)
    x = oracle.h0_solve(P, q, 10.0)
    assert np.allclose(x.ravel(), np.linalg.solve(A, q.ravel()), rtol=1e-9, atol=1e-12)


def test_lbfgs_registration_decreases_objective():
    d = small_case(10, shape=(16, 12, 12))
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"], oracle.Weights(eta=10.0, alpha=1.0,
                                                                                           gamma=0.1))
    P.w.delta = P.adaptive_delta(np.zeros_like(d["u_true"], np.float64))
    u, reps = oracle.lbfgs_run(P, np.zeros_like(d["u_true"], np.float64), 4)
    assert len(reps) == 4 and all(rep["accepted"] for rep in reps)
    Js = [rep["J"] for rep in reps] + [reps[-1]["J_new"]]
    assert all(b_ < a_ for a_, b_ in zip(Js, Js[1:]))


# ---- multilevel scheme (Sec. II-D3) ----------------------------------------------------

def test_pyramid_plan_examples():
    """Coarse levels approach isotropic voxels: worked by hand from the halving rule."""
    plan = oracle.pyramid_plan((512, 512, 128), (0.7, 0.7, 2.5), 4)
    assert [l["shape"] for l in plan] == [(512, 512, 128), (256, 256, 128), (128, 128, 128), (64, 64, 64)]
    assert [l["halve"] for l in plan] == [(0, 0, 0), (1, 1, 0), (1, 1, 0), (1, 1, 1)]
    np.testing.assert_allclose(plan[-1]["spacing"], (5.6, 5.6, 5.0))
    plan = oracle.pyramid_plan((64, 64, 48), (1.5, 1.5, 1.5), 4)
    assert [l["shape"] for l in plan] == [(64, 64, 48), (32, 32, 24), (16, 16, 12), (8, 8, 12)]
    # 12 is not divisible by 8 and 8 // 2 < 8: the pyramid stops early
    plan = oracle.pyramid_plan((48, 32, 24), (1.2, 1.4, 2.2), 4)
    assert [l["shape"] for l in plan] == [(48, 32, 24), (24, 16, 24), (12, 8, 12)]
    assert oracle.pyramid_halving((12, 8, 12), (4.8, 5.6, 4.4)) is None


def test_pyramid_halving_is_the_most_isotropic_choice():
    """Brute force over all subsets on random shapes and spacings: no valid subset gives a
    smaller anisotropy than the chosen one."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        shape = tuple(int(x) for x in rng.choice([8, 12, 16, 24, 32, 40, 64], 3))
        spacing = tuple(float(x) for x in rng.uniform(0.5, 3.0, 3))
        S = oracle.pyramid_halving(shape, spacing)
        ratios = []
        for mask in range(1, 8):
            T = [(mask >> a) & 1 for a in range(3)]
            if any(T[a] and (shape[a] % 8 or shape[a] < 16) for a in range(3)):
                continue
            h = [spacing[a] * (1 + T[a]) for a in range(3)]
            ratios.append(max(h) / min(h))
        if not ratios:
            assert S is None
            continue
        h = [spacing[a] * (1 + S[a]) for a in range(3)]
        assert max(h) / min(h) <= min(ratios) + 1e-15


def test_smooth_axis_matches_scipy_gaussian_filter():
    from scipy.ndimage import gaussian_filter1d
    rng = np.random.default_rng(6)
    img = rng.normal(size=(10, 12, 14))
    for a in range(3):
        ref = gaussian_filter1d(img, sigma=1.0, axis=2 - a, mode="nearest", truncate=3.0)
        np.testing.assert_allclose(oracle.smooth_axis(img, a), ref, rtol=0, atol=1e-13)


def test_downsample_constant_and_linear_ramp():
    """A constant stays constant; a linear function of position is reproduced exactly at
    the coarse voxel centres wherever the smoothing stencil stays inside the volume (the
    symmetric kernel preserves linear functions; the pair mean is the midpoint value)."""
    Nz, Ny, Nx = 16, 24, 32
    c = oracle.downsample(np.full((Nz, Ny, Nx), 3.25), (1, 1, 1))
    assert c.shape == (8, 12, 16)
    np.testing.assert_allclose(c, 3.25, rtol=0, atol=1e-13)
    h = (0.7, 0.9, 2.0)
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) * hh for n, hh in zip((Nz, Ny, Nx), h[::-1])], indexing="ij")
    f = 1.0 + 0.3 * x - 0.2 * y + 0.05 * z
    for halve in ((1, 0, 0), (1, 1, 0), (1, 1, 1), (0, 0, 1)):
        d = oracle.downsample(f, halve)
        hc = [hh * (1 + s) for hh, s in zip(h, halve)]
        shp = d.shape
        zc, yc, xc = np.meshgrid(*[(np.arange(n) + 0.5) * hh for n, hh in zip(shp, hc[::-1])], indexing="ij")
        ref = 1.0 + 0.3 * xc - 0.2 * yc + 0.05 * zc
        # interior: coarse index i with fine stencil 2i - 3 .. 2i + 4 inside along halved axes
        sl = []
        for ax, a in zip(range(3), (2, 1, 0)):
            n = shp[ax]
            sl.append(slice(2, n - 2) if halve[a] else slice(None))
        np.testing.assert_allclose(d[tuple(sl)], ref[tuple(sl)], rtol=0, atol=1e-12)


def test_prolong_represents_the_coarse_trilinear_field():
    """The prolonged node field and the coarse field define the same trilinear function
    (scipy RegularGridInterpolator on both grids at random points)."""
    from scipy.interpolate import RegularGridInterpolator
    rng = np.random.default_rng(7)
    Hc = (4.0, 3.0, 5.0)
    nc = (5, 4, 6)  # nodes x, y, z
    uc = rng.normal(size=(3, nc[2], nc[1], nc[0]))
    for halve in ((1, 1, 1), (1, 0, 1), (0, 1, 0)):
        uf = oracle.prolong(uc, halve)
        Hf = tuple(H / (1 + s) for H, s in zip(Hc, halve))
        nf = (uf.shape[3], uf.shape[2], uf.shape[1])
        assert nf == tuple(2 * (n - 1) + 1 if s else n for n, s in zip(nc, halve))
        pts = rng.uniform(0, 1, size=(200, 3)) * np.array([(n - 1) * H for n, H in zip(nc, Hc)])[::-1]
        for c in range(3):
            gc = RegularGridInterpolator([np.arange(n) * H for n, H in zip(nc[::-1], Hc[::-1])], uc[c])
            gf = RegularGridInterpolator([np.arange(n) * H for n, H in zip(nf[::-1], Hf[::-1])], uf[c])
            np.testing.assert_allclose(gf(pts), gc(pts), rtol=0, atol=1e-12)


def test_multilevel_run_decreases_objective_on_every_level():
    d = synth.small_pair(shape=(32, 32, 24), spacing=(1.5, 1.5, 2.0), seed=8, n_tubes=6, n_kp=20, field_max=3.0)
    w = oracle.Weights(eta=10.0, alpha=1.0, gamma=0.1, delta=-1.0)
    prm = oracle.MultilevelParams(levels=3, iters=(4, 3, 2), optimizer="lbfgs")
    u, levels = oracle.multilevel_run(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"], w, prm)
    assert [l["shape"] for l in levels] == [(8, 8, 12), (16, 16, 12), (32, 32, 24)]
    for lv in levels:
        assert lv["delta"] > 0
        r = lv["reports"]
        assert r[-1]["J_new"] < r[0]["J"]
    assert u.shape == (3, 7, 9, 9)


# ---- lung-boundary term (eq. 6) ---------------------------------------------------------

def mask_case(seed=12, shape=(16, 16, 12), spacing=(1.5, 1.5, 2.0)):
    d = synth.small_pair(shape=shape, spacing=spacing, seed=seed, n_tubes=4, n_kp=10, field_max=4.0)
    return d, d["mask_R"].astype(np.float64), d["mask_T"].astype(np.float64)


def test_mask_term_zero_for_identical_masks():
    d, bF, _ = mask_case()
    u = np.zeros_like(d["u_true"], np.float64)
    res = oracle.mask_term(bF, bF, d["spacing"], u)
    assert res["B"] == 0.0 and np.all(res["g"] == 0.0) and np.all(res["res"] == 0.0)


def test_mask_term_integer_translation_brute_force():
    """b_M(z) = b_F(z - k h_x e_x) and u = k h_x e_x: inside, b_M(y(x)) = b_F(x); the last
    k voxel columns sample beyond the volume (zero), so B = 1/2 h^3 sum of b_F there."""
    d, _, _ = mask_case(13)
    bF = (rng(13).random(d["mask_R"].shape) > 0.5).astype(np.float64)  # reaches every border
    h = d["spacing"]
    k = 2
    bM = np.zeros_like(bF)
    bM[:, :, k:] = bF[:, :, :-k]
    u = np.zeros_like(d["u_true"], np.float64)
    u[0] = k * h[0]
    res = oracle.mask_term(bF, bM, h, u)
    expect = 0.5 * np.prod(h) * np.sum(bF[:, :, -k:] ** 2)
    assert expect > 0
    assert abs(res["B"] - expect) <= 1e-12 * expect
    np.testing.assert_array_equal(res["res"][:, :, :-k], 0.0)


def test_mask_sampling_matches_grid_sample():
    d, bF, bM = mask_case(14)
    h = d["spacing"]
    u = d["u_true"].astype(np.float64) * 0.8 + 0.031
    res = oracle.mask_term(bF, bM, h, u)
    nx, ny, nz = d["shape"]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vox = np.stack([(i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]], -1).reshape(-1, 3)
    uv = trilinear_nodes(u, [4 * s for s in h], vox)
    q = (vox + uv) / np.array(h) - 0.5
    ref = grid_sample_vec(np.repeat(bM[..., None], 3, axis=-1), q)[:, 0]
    np.testing.assert_allclose(res["res"].ravel() + bF.ravel(), ref, rtol=0, atol=1e-12)
    # the interpolant's gradient: central differences of the library sampler in mm
    eps = 1e-6
    for a in range(3):
        dq = np.zeros(3)
        dq[a] = eps / h[a]
        fd = (grid_sample_vec(np.repeat(bM[..., None], 3, -1), q + dq)[:, 0]
              - grid_sample_vec(np.repeat(bM[..., None], 3, -1), q - dq)[:, 0]) / (2 * eps)
        # points within eps of a cell face have a one-sided derivative: skip them
        frac = q[:, a] - np.floor(q[:, a])
        okp = (frac > 1e-4) & (frac < 1 - 1e-4)
        np.testing.assert_allclose(res["sb"].reshape(-1, 3)[okp, a], fd[okp], rtol=0, atol=1e-7)


def test_mask_gradient_matches_finite_differences():
    d, bF, bM = mask_case(15)
    h = d["spacing"]
    u = d["u_true"].astype(np.float64) * 0.7 + 0.023
    g = oracle.mask_term(bF, bM, h, u)["g"]
    err = _fd_check(lambda x: oracle.mask_term(bF, bM, h, x, want=())["B"], g, u, random_coords(u.shape, 25, 3))
    assert err < 1e-5


def test_mask_gauss_newton_matrix_dense_brute_force_8cubed():
    """h^3 J^T J with J from finite differences of the residual equals the oracle's GN
    product (columns) and diagonal; symmetric positive semi-definite."""
    d = synth.small_pair(shape=(8, 8, 8), spacing=(2.0, 2.0, 2.0), seed=16, n_tubes=3, n_kp=4, field_max=3.0)
    bF = d["mask_R"].astype(np.float64)
    bM = d["mask_T"].astype(np.float64)
    if bF.sum() == 0:
        bF[2:6, 2:6, 2:6] = 1.0
        bM[3:7, 2:6, 1:5] = 1.0
    h = d["spacing"]
    u = d["u_true"].astype(np.float64) * 0.6 + 0.017
    res = oracle.mask_term(bF, bM, h, u)
    n = u.size
    Jm = np.empty((bF.size, n))
    eps = 1e-6
    for col in range(n):
        e = np.zeros(n)
        e[col] = eps
        e = e.reshape(u.shape)
        rp = oracle.mask_term(bF, bM, h, u + e, want=("res",))["res"].ravel()
        rm = oracle.mask_term(bF, bM, h, u - e, want=("res",))["res"].ravel()
        Jm[:, col] = (rp - rm) / (2 * eps)
    Hd = np.prod(h) * Jm.T @ Jm
    Ho = np.stack([oracle.mask_hv(res["sb"], h, np.eye(n)[c].reshape(u.shape)).ravel() for c in range(n)], 1)
    assert np.linalg.norm(Hd) > 0
    assert np.linalg.norm(Ho - Hd) / np.linalg.norm(Hd) < 1e-6
    np.testing.assert_allclose(res["diag"].ravel(), np.diag(Ho), rtol=1e-12, atol=1e-12 * np.max(np.diag(Ho)))
    assert np.linalg.eigvalsh(0.5 * (Ho + Ho.T)).min() > -1e-10 * np.abs(Ho).max()


def test_problem_with_boundary_term_and_adaptive_beta():
    """J includes beta B; the adaptive beta gives D = 100 beta B at u = 0 (Sec. II-D2); the
    GN step with the term decreases J."""
    d, bF, bM = mask_case(17, shape=(24, 24, 16))
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"], oracle.Weights(eta=10.0, alpha=1.0,
                       gamma=0.1, delta=0.0), bF=bF, bM=bM)
    u0 = np.zeros_like(d["u_true"], np.float64)
    beta = P.adaptive_beta(u0)
    P.w.beta = beta
    o = P.objective(u0)
    assert abs(o["D"] - 100.0 * beta * o["B"]) <= 1e-12 * o["D"]
    P0 = oracle.Problem(d["R"], d["T"], d["spacing"], weights=oracle.Weights(eta=10.0, alpha=1.0, gamma=0.1))
    assert abs(o["J"] - (P0.objective(u0)["J"] + beta * o["B"])) <= 1e-12 * o["J"]
    u1, rep = oracle.gn_pcg_step(P, u0, oracle.StepParams(pcg_iters=10))
    assert rep["accepted"] and rep["trial"]["J"] < rep["J"]


# ---- keypoint stage (Sec. II-C2, II-C3) ------------------------------------------------

def kp_images(seed=31, shape=(40, 36, 32)):
    d = synth.small_pair(shape=shape, spacing=(1.0, 1.0, 1.0), seed=seed, n_tubes=8, n_kp=12, field_max=3.0)
    return d


def test_kp_cost_zero_for_identical_images_at_zero_displacement():
    d = kp_images()
    kps = np.array([[5, 6, 7], [20, 18, 16], [1, 34, 30], [39, 0, 0]])  # incl. border keypoints
    D = oracle.kp_cost_volume(d["R"], d["R"], (1.0, 1.0, 1.0), kps, 12.0, R=3, step=2)
    zero = (3 * 7 + 3) * 7 + 3  # label d = 0
    np.testing.assert_array_equal(D[:, zero], 0.0)
    assert np.all(D >= 0.0) and np.all(D <= 1.0)


def test_kp_cost_translation_has_zero_at_the_shift():
    """M(z) = F(z - t) with t = (2, -4, 6): D(k, t) = 0 where patch and gradient
    stencils stay inside the volume, and t is the arg-min."""
    d = kp_images(32, shape=(48, 48, 48))
    F = d["R"]
    t = (2, -4, 6)
    M = np.roll(F, shift=(t[2], t[1], t[0]), axis=(0, 1, 2))
    kps = np.array([[20, 22, 18], [24, 26, 20], [18, 24, 22]])
    D = oracle.kp_cost_volume(F, M, (1.0, 1.0, 1.0), kps, 12.0, R=4, step=2)
    lab = oracle.kp_labels(4, 2)
    it = int(np.where((lab == np.array(t)).all(axis=1))[0][0])
    assert np.all(D[:, it] < 1e-15)
    assert np.all(np.argmin(D, axis=1) == it)


def test_kp_cost_matches_library_gradients_and_plain_formula():
    """Eq. 2 evaluated with torch central differences and numpy at sampled labels; and the
    eta -> infinity limit eta^2 D -> mean |a - b|^2."""
    d = kp_images(33)
    F, M = d["R"], d["T"]
    gF = conv_gradient(F, (1.0, 1.0, 1.0))
    gM = conv_gradient(M, (1.0, 1.0, 1.0))
    nz, ny, nx = F.shape
    kps = np.array([[10, 12, 9], [30, 20, 25], [2, 33, 3]])
    R, step = 3, 2
    lab = oracle.kp_labels(R, step)
    off = np.array(np.meshgrid(*[oracle.KP_PATCH] * 3, indexing="ij")).reshape(3, -1).T[:, ::-1]

    def grad_at(g, pts):
        out = np.zeros((len(pts), 3))
        ok = (pts[:, 0] >= 0) & (pts[:, 0] < nx) & (pts[:, 1] >= 0) & (pts[:, 1] < ny) & (pts[:, 2] >= 0) & (pts[:, 2] < nz)
        out[ok] = g[pts[ok, 2], pts[ok, 1], pts[ok, 0]]
        return out

    for eta, tol in ((12.0, 1e-12), (1e7, 1e-6)):
        D = oracle.kp_cost_volume(F, M, (1.0, 1.0, 1.0), kps, eta, R=R, step=step)
        for k in range(len(kps)):
            for li in rng(k).integers(0, len(lab), 12):
                p = kps[k] + off
                b = grad_at(gF, p)
                a = grad_at(gM, p + lab[li])
                if eta < 1e6:
                    r2 = (eta ** 2 + np.sum(a * b, 1)) ** 2 / ((eta ** 2 + np.sum(a * a, 1)) * (eta ** 2 + np.sum(b * b, 1)))
                    ref = np.mean(1.0 - r2)
                    assert abs(D[k, li] - ref) <= tol, (k, li)
                else:
                    ref = np.mean(np.sum((a - b) ** 2, 1))
                    assert abs(eta ** 2 * D[k, li] - ref) <= tol * max(ref, 1.0), (k, li)


def test_kp_mst_is_a_minimum_spanning_tree():
    from scipy.sparse.csgraph import minimum_spanning_tree
    r = rng(34)
    x = r.uniform(0, 100, (60, 3))
    inten = r.normal(-800, 100, 60)
    parent, order = oracle.kp_mst(x, inten)
    W = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1)) + np.abs(inten[:, None] - inten[None]) / 150.0
    ref = minimum_spanning_tree(W).sum()
    ours = sum(W[k, parent[k]] for k in range(60) if parent[k] >= 0)
    assert abs(ours - ref) <= 1e-9 * ref
    assert parent[0] == -1 and np.sum(parent >= 0) == 59 and order[0] == 0
    pos = {int(k): i for i, k in enumerate(order)}
    assert all(pos[int(parent[k])] < pos[k] for k in range(1, 60))  # parents come first: a tree


def test_kp_mincon_separable_equals_brute_force():
    r = rng(35)
    for R, step, c in ((2, 2, 0.37), (1, 2, 5.0), (3, 1, 0.01)):
        f = r.normal(size=(2 * R + 1) ** 3)
        np.testing.assert_allclose(oracle.kp_mincon(f, c, R, step), oracle.kp_mincon_bruteforce(f, c, R, step),
                                   rtol=0, atol=1e-12)


def test_kp_belief_propagation_gives_exact_min_marginals():
    """On a 4-node tree with 27 labels the min-marginals equal brute-force minimisation of
    sum_k D(k, d_k) + sum_edges R_KP over all 27^4 joint labelings with d_k fixed."""
    r = rng(36)
    n, R, step = 4, 1, 2
    L = (2 * R + 1) ** 3
    x = r.uniform(0, 20, (n, 3))
    inten = r.normal(-800, 80, n)
    D = r.uniform(0, 1, (n, L))
    parent, order = oracle.kp_mst(x, inten)
    alpha = 0.8
    marg, _ = oracle.kp_belief_propagation(D, parent, order, x, inten, alpha, R=R, step=step,
                                           mincon=oracle.kp_mincon_bruteforce)
    lab = oracle.kp_labels(R, step).astype(np.float64)
    idx = np.array(np.meshgrid(*[np.arange(L)] * n, indexing="ij")).reshape(n, -1)
    E = sum(D[k][idx[k]] for k in range(n))
    for k in range(n):
        if parent[k] >= 0:
            w = oracle.kp_edge_weight(x, inten, k, parent[k])
            E = E + alpha / w * np.sum((lab[idx[k]] - lab[idx[parent[k]]]) ** 2, axis=1)
    for k in range(n):
        ref = np.full(L, np.inf)
        np.minimum.at(ref, idx[k], E)
        np.testing.assert_allclose(marg[k], ref, rtol=1e-12, atol=1e-12)
    marg2, _ = oracle.kp_belief_propagation(D, parent, order, x, inten, alpha, R=R, step=step)
    np.testing.assert_allclose(marg2, marg, rtol=1e-12, atol=1e-12)


def test_kp_mst_ties_follow_the_edge_order():
    """Keypoints on a unit lattice with equal intensities: every nearest-neighbour edge
    costs 1, so the tree is fixed by the order (cost, lower index, higher index); brute
    force over Kruskal's rule written out for this case gives the same edges."""
    g = np.array([[i, j, 0] for j in range(3) for i in range(4)], np.float64)
    inten = np.zeros(len(g))
    parent, order = oracle.kp_mst(g, inten)
    edges = {tuple(sorted((k, int(parent[k])))) for k in range(len(g)) if parent[k] >= 0}
    # by hand: unit edges sorted by (lower, higher) are (0,1), (0,4), (1,2), (1,5), (2,3),
    # (2,6), (3,7), (4,5), (4,8), ...; Kruskal keeps the first row's horizontal edges and
    # every vertical edge, all later horizontal edges close a cycle
    expect = {(0, 1), (1, 2), (2, 3), (0, 4), (1, 5), (2, 6), (3, 7), (4, 8), (5, 9), (6, 10), (7, 11)}
    assert edges == expect
    assert list(order[:3]) == [0, 1, 4]


def test_kp_min_marginals_do_not_depend_on_the_root():
    """The two-pass schedule gives exact min-marginals, so re-rooting the tree (here at
    several keypoints, the device schedules from the tree's centre) leaves them unchanged
    up to rounding."""
    r = rng(37)
    n, R, step = 30, 2, 2
    L = (2 * R + 1) ** 3
    x = r.uniform(0, 40, (n, 3))
    inten = r.normal(-800, 80, n)
    D = r.uniform(0, 1, (n, L))
    parent, order = oracle.kp_mst(x, inten)
    ref, _ = oracle.kp_belief_propagation(D, parent, order, x, inten, 0.5, R=R, step=step)
    adj = [[] for _ in range(n)]
    for k in range(n):
        if parent[k] >= 0:
            adj[k].append(int(parent[k]))
            adj[int(parent[k])].append(k)
    for root in (7, 13, n - 1):
        par = np.full(n, -1)
        seen = np.zeros(n, bool)
        seen[root] = True
        ordr = [root]
        for a in ordr:
            for b in sorted(adj[a]):
                if not seen[b]:
                    seen[b] = True
                    par[b] = a
                    ordr.append(b)
        marg, _ = oracle.kp_belief_propagation(D, par, ordr, x, inten, 0.5, R=R, step=step)
        np.testing.assert_allclose(marg, ref, rtol=1e-12, atol=1e-12)
