"""Pins of the oracle's sample-cell rule and tie allowances, and of the joint objective of
eq. 11 at non-unit weights.

Sample cell (eq. 1 evaluated at the warped point).  The cell of a sample point is the
floor of q = i + u/h, which equals i + floor(u/h) exactly; a displacement far below the
voxel index must therefore still pick its side of the face.  Where u/h lies within
single-precision rounding of an integer, both one-sided derivatives are correct results;
the oracle's tie routine returns allowance fields that bracket the difference between
them.  These tests pin both against brute force: explicit left/right evaluations, and
single-precision evaluations of the voxel displacement in several operation orders.

Joint objective (eq. 11, weights of Sec. II-D2).  The gradient of the weighted sum is
checked by central differences of the weighted objective, and the GN matrix against the
weighted sum of the term matrices, each built from the term routines pinned elsewhere,
at alpha = 1.7, gamma = 0.3, delta = 2.5, beta = 0.4, so a dropped or squared weight
fails.
"""
import numpy as np
import pytest

import oracle
import synth


def rng(seed=0):
    return np.random.default_rng(seed)


def grads(d):
    h = d["spacing"]
    return oracle.image_gradient(d["R"], h), oracle.image_gradient(d["T"], h)


def case(seed=41, shape=(16, 16, 12), spacing=(1.5, 1.25, 2.0)):
    return synth.small_pair(shape=shape, spacing=spacing, seed=seed, n_tubes=6, n_kp=12, field_max=4.0)


# ---------------------------------------------------------------------------------
# sample cell: floor(i + u/h) = i + floor(u/h)
# ---------------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sample_cell_keeps_displacements_far_below_the_index(axis):
    """u_a = -1e-30 mm puts every sample point just left of its voxel centre: the sample
    cell is the left one, so s equals the one at a clearly-left displacement (-1e-7 voxel)
    and differs from the clearly-right one.  Forming i + u/h in double precision first
    would round -1e-30 away and pick the right cell."""
    d = case()
    gR, gT = grads(d)
    h = d["spacing"]
    u0 = 0.6 * d["u_true"].astype(np.float64) + 0.37
    res = {}
    for name, off in (("tiny", -1e-30), ("left", -1e-7 * h[axis]), ("right", +1e-7 * h[axis])):
        u = u0.copy()
        u[axis] = off
        res[name] = oracle.ngf(gR, gT, h, 10.0, u, want=("s",))["s"]
    sc = np.max(np.abs(res["left"]))
    assert np.max(np.abs(res["tiny"] - res["left"])) < 1e-5 * sc
    assert np.max(np.abs(res["tiny"] - res["right"])) > 1e-2 * sc


def test_ties_flag_nothing_at_generic_and_zero_points():
    d = case()
    gR, gT = grads(d)
    h = d["spacing"]
    u = 0.6 * d["u_true"].astype(np.float64) + 0.0137
    assert oracle.ngf_ties(gR, gT, h, 10.0, u)["n"] == 0
    z = oracle.ngf_ties(gR, gT, h, 10.0, np.zeros_like(u), want_s=True)
    assert z["n"] == 0 and np.all(z["g"] == 0) and np.all(z["s"] == 0)


@pytest.mark.parametrize("axis,k", [(0, 1), (1, -2), (2, 1)])
def test_tie_allowance_brackets_the_two_one_sided_results(axis, k):
    """u_a = k h_a exactly: every voxel's sample point lies on a face along a.  The
    oracle takes the right-hand cell; the left-hand result is the oracle evaluated at
    u_a = k h_a (1 - 1e-12).  The per-voxel s allowance equals |s_right - s_left|, and the
    gradient, diagonal and GN-product differences stay within their allowance fields."""
    d = case(42)
    gR, gT = grads(d)
    h = d["spacing"]
    eta = 10.0
    base = 0.5 * d["u_true"].astype(np.float64) + 0.0137
    u = base.copy()
    u[axis] = k * h[axis]
    ul = base.copy()
    ul[axis] = k * h[axis] * (1 - 1e-12) if k > 0 else k * h[axis] * (1 + 1e-12)
    v = rng(3).standard_normal(u.shape)
    ties = oracle.ngf_ties(gR, gT, h, eta, u, v, want_s=True)
    nvox = int(np.prod(d["shape"]))
    assert ties["n"] == nvox
    R = oracle.ngf(gR, gT, h, eta, u, want=("g", "diag", "s", "r"))
    L = oracle.ngf(gR, gT, h, eta, ul, want=("g", "diag", "s", "r"))
    sc = np.max(np.abs(R["s"]))
    ds = np.abs(R["s"] - L["s"])
    assert np.max(ds) > 1e-2 * sc  # the derivative really jumps
    # only axis a is a tie: the allowance is exactly the other side's difference
    np.testing.assert_allclose(ties["s"], ds, rtol=0, atol=1e-9 * sc)
    h3 = np.prod(h)
    Pv = interp_nodes(v, d["shape"])
    swR = np.sum(R["s"] * Pv, -1, keepdims=True)
    swL = np.sum(L["s"] * Pv, -1, keepdims=True)
    per_voxel = {
        "g": (np.abs(2 * h3 * (R["r"][..., None] * R["s"] - L["r"][..., None] * L["s"])), False),
        "diag": (np.abs(2 * h3 * (R["s"] ** 2 - L["s"] ** 2)), True),
        "hv": (np.abs(2 * h3 * (R["s"] * swR - L["s"] * swL)), False),
    }
    fields = {"g": (R["g"], L["g"]), "diag": (R["diag"], L["diag"]),
              "hv": (oracle.ngf_hv(R["s"], h, v), oracle.ngf_hv(L["s"], h, v))}
    for key, (fr, fl) in fields.items():
        a = ties[key]
        scale = np.max(np.abs(fr))
        # the allowance is the phi-weighted sum of the per-voxel one-sided differences
        # (scattered here independently of the oracle)...
        vals, sq = per_voxel[key]
        np.testing.assert_allclose(a, scatter_nodes(vals, d["shape"], sq), rtol=1e-9, atol=1e-9 * scale)
        # ...so it bounds the difference of the two one-sided fields
        assert np.all(np.abs(fr - fl) <= a + 1e-9 * scale), key
        assert np.max(a) > 1e-3 * scale, key


def _phi(shape):
    """Per-voxel node indices and trilinear weights of the control grid (4 voxels per
    cell, voxel i at xi = (i mod 4 + 1/2)/4 in cell i // 4)."""
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = 1.0
                idx = []
                for ax, dd in ((i, dx), (j, dy), (k, dz)):
                    xi = (ax % 4 + 0.5) / 4
                    w = w * (xi if dd else 1 - xi)
                    idx.append(ax // 4 + dd)
                out.append((idx[2], idx[1], idx[0], w))
    return out


def interp_nodes(f, shape):
    """(Pf)(x_v) for a node field f [3][nz][ny][nx]: [Nz][Ny][Nx][3]."""
    res = 0.0
    for kz, jy, ix, w in _phi(shape):
        res = res + w[..., None] * np.moveaxis(f[:, kz, jy, ix], 0, -1)
    return res


def scatter_nodes(vals, shape, squared):
    """sum_v phi_v vals_v (phi^2 when squared) onto the nodes, [3][nz][ny][nx]."""
    nx, ny, nz = shape
    out = np.zeros((3, nz // 4 + 1, ny // 4 + 1, nx // 4 + 1))
    for kz, jy, ix, w in _phi(shape):
        ww = w * w if squared else w
        for c in range(3):
            np.add.at(out[c], (kz, jy, ix), ww * vals[..., c])
    return out


def _f32_voxel_displacements(u, m, h, order):
    """Voxel displacement u/h evaluated in single precision in one operation order."""
    f = np.float32
    _, nz, ny, nx = u.shape
    u32 = u.astype(np.float32)
    out = np.empty((3, (nz - 1) * m, (ny - 1) * m, (nx - 1) * m), np.float32)
    xi = ((np.arange(m) + 0.5) / m).astype(np.float32)
    inv_h = [f(1.0 / hh) for hh in h]
    for a in range(3):
        U = u32[a]
        for kz in range((nz - 1) * m):
            cz, wz = kz // m, xi[kz % m]
            for jy in range((ny - 1) * m):
                cy, wy = jy // m, xi[jy % m]
                cx = np.arange((nx - 1) * m) // m
                wx = xi[np.arange((nx - 1) * m) % m]
                c = {(dz, dy, dx): U[cz + dz, cy + dy, cx + dx] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)}
                if order == "xzy":  # lerp a0 + w (a1 - a0) along x, then z, then y
                    lx = {(dz, dy): c[dz, dy, 0] + wx * (c[dz, dy, 1] - c[dz, dy, 0]) for dz in (0, 1) for dy in (0, 1)}
                    lz = {dy: lx[0, dy] + wz * (lx[1, dy] - lx[0, dy]) for dy in (0, 1)}
                    val = lz[0] + wy * (lz[1] - lz[0])
                elif order == "zyx":  # (1 - w) a0 + w a1 along z, then y, then x
                    lz = {(dy, dx): (f(1) - wz) * c[0, dy, dx] + wz * c[1, dy, dx] for dy in (0, 1) for dx in (0, 1)}
                    ly = {dx: (f(1) - wy) * lz[0, dx] + wy * lz[1, dx] for dx in (0, 1)}
                    val = (f(1) - wx) * ly[0] + wx * ly[1]
                else:  # eight weights, summed in single precision
                    val = np.zeros_like(wx)
                    for (dz, dy, dx), cv in c.items():
                        w = (wx if dx else f(1) - wx) * (wy if dy else f(1) - wy) * (wz if dz else f(1) - wz)
                        val = val + w * cv
                out[a, kz, jy] = (val * inv_h[a]).astype(np.float32)
    return out


@pytest.mark.parametrize("order", ["xzy", "zyx", "sum8"])
def test_tie_rule_covers_single_precision_evaluations(order):
    """Node fields built to sit next to cell faces (near-integer u/h with relative noise
    around single-precision rounding, and tiny values of mixed sign): wherever a
    single-precision evaluation of u/h floors differently from the double-precision
    one, the voxel must be a tie (its s allowance is nonzero)."""
    shape = (24, 16, 12)
    h = (0.7, 0.9, 2.5)
    r = rng(7)
    R = (r.standard_normal(shape[::-1]) * 200).astype(np.float32)
    T = (r.standard_normal(shape[::-1]) * 200).astype(np.float32)
    gR = oracle.image_gradient(R, h)
    gT = oracle.image_gradient(T, h)
    nn = oracle.node_shape(shape)
    u = np.empty((3, nn[2], nn[1], nn[0]))
    for a in range(3):
        kint = r.integers(-3, 4, size=u[a].shape)
        near = (kint + kint * r.standard_normal(u[a].shape) * 2.0 ** -23) * h[a]
        tiny = r.choice([-1.0, 0.0, 1.0], size=u[a].shape) * 5.7e-14
        u[a] = np.where(r.random(u[a].shape) < 0.5, near, tiny)
    u = u.astype(np.float32).astype(np.float64)  # the inputs are single precision on both sides
    uh32 = _f32_voxel_displacements(u, 4, h, order)
    nz, ny, nx = shape[2], shape[1], shape[0]
    uh64 = np.empty((3, nz, ny, nx))
    xi = (np.arange(4) + 0.5) / 4
    for a in range(3):
        U = u[a]
        k = np.arange(nz)[:, None, None]
        j = np.arange(ny)[None, :, None]
        i = np.arange(nx)[None, None, :]
        cz, cy, cx = k // 4, j // 4, i // 4
        wz, wy, wx = xi[k % 4], xi[j % 4], xi[i % 4]
        val = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = (wx if dx else 1 - wx) * (wy if dy else 1 - wy) * (wz if dz else 1 - wz)
                    val = val + w * U[cz + dz, cy + dy, cx + dx]
        uh64[a] = val / h[a]
    differ = np.any(np.floor(uh32.astype(np.float64)) != np.floor(uh64), axis=0)
    if order != "sum8":  # summing the eight products rarely flips on these fields
        assert differ.sum() > 0, "the construction must produce single-precision flips"
    ties = oracle.ngf_ties(gR, gT, h, 10.0, u, want_s=True)
    flagged = np.any(ties["s"] > 0, axis=-1)
    # a sample point with every corner outside the volume samples zero on both sides
    # (s = 0 either way): nothing to allow for there
    idx = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), 0)
    idx = np.moveaxis(idx, (1, 2, 3), (3, 2, 1))
    q = idx + uh64
    outside = np.any((q <= -1.0) | (q >= np.array([nx, ny, nz])[:, None, None, None]), axis=0)
    missed = differ & ~flagged & ~outside
    assert not missed.any(), f"{missed.sum()} of {differ.sum()} flips not covered"
    # the rule is not vacuous: most voxels are not ties
    assert ties["n"] < 0.8 * np.prod(shape)


def test_mask_ties_bracket_the_two_one_sided_results():
    d = synth.small_pair(shape=(16, 16, 12), spacing=(1.5, 1.5, 2.0), seed=12, n_tubes=4, n_kp=10, field_max=4.0)
    bF = d["mask_R"].astype(np.float64)
    bM = d["mask_T"].astype(np.float64)
    h = d["spacing"]
    base = 0.5 * d["u_true"].astype(np.float64) + 0.0137
    u = base.copy()
    u[1] = 2 * h[1]
    ul = base.copy()
    ul[1] = 2 * h[1] * (1 - 1e-12)
    v = rng(5).standard_normal(u.shape)
    t = oracle.mask_ties(bF, bM, h, u, v, want_s=True)
    R = oracle.mask_term(bF, bM, h, u)
    L = oracle.mask_term(bF, bM, h, ul)
    ds = np.abs(R["sb"] - L["sb"])
    assert np.max(ds) > 0.05
    np.testing.assert_allclose(t["s"], ds, rtol=0, atol=1e-9)
    for key, fr, fl in (("g", R["g"], L["g"]), ("diag", R["diag"], L["diag"]),
                        ("hv", oracle.mask_hv(R["sb"], h, v), oracle.mask_hv(L["sb"], h, v))):
        assert np.all(np.abs(fr - fl) <= t[key] + 1e-9 * np.max(np.abs(fr))), key
    assert oracle.mask_ties(bF, bM, h, base)["n"] == 0


# ---------------------------------------------------------------------------------
# eq. 11 at non-unit weights
# ---------------------------------------------------------------------------------

W_JOINT = dict(eta=8.0, alpha=1.7, gamma=0.3, delta=2.5, beta=0.4)


def joint_problem(shape=(12, 12, 8), seed=43):
    d = synth.small_pair(shape=shape, spacing=(2.0, 1.5, 2.5), seed=seed, n_tubes=4, n_kp=10, field_max=3.0)
    bF = d["mask_R"].astype(np.float64)
    bM = d["mask_T"].astype(np.float64)
    if bF.sum() == 0 or bM.sum() == 0:
        bF[2:6, 3:9, 3:9] = 1.0
        bM[3:7, 2:8, 4:10] = 1.0
    nn = oracle.node_shape(d["shape"])
    u_ref = 0.1 * rng(9).standard_normal((3, nn[2], nn[1], nn[0]))
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"], oracle.Weights(**W_JOINT),
                       u_ref=u_ref, bF=bF, bM=bM)
    return P, d


def test_joint_gradient_matches_finite_differences_of_the_weighted_objective():
    P, d = joint_problem()
    u = 0.6 * d["u_true"].astype(np.float64) + 0.0137
    lin = P.linearise(u)
    assert P.ties(u)["n"] == 0
    o = P.objective(u)
    # every term is present and weighted as eq. 11 states
    assert o["D"] > 0 and o["S"] > 0 and o["V"] > 0 and o["K"] > 0 and o["B"] > 0
    w = P.w
    J = o["D"] + w.alpha * o["S"] + w.gamma * o["V"] + w.delta * o["K"] + w.beta * o["B"]
    assert abs(o["J"] - J) <= 1e-13 * abs(J)
    g = lin["g"]
    coords = [tuple(int(rng(11 + c).integers(0, s)) for s in u.shape) for c in range(30)]
    scale = np.max(np.abs(g))
    worst = 0.0
    for c in coords:
        best = np.inf
        for eps in (1e-4, 1e-5, 1e-6):
            up = u.copy()
            um = u.copy()
            up[c] += eps
            um[c] -= eps
            fd = (P.objective(up)["J"] - P.objective(um)["J"]) / (2 * eps)
            best = min(best, abs(fd - g[c]) / max(abs(g[c]), 1e-3 * scale))
        worst = max(worst, best)
    assert worst < 1e-5


def test_joint_gn_matrix_is_the_weighted_sum_of_the_term_matrices():
    P, d = joint_problem(shape=(8, 8, 8), seed=44)
    u = 0.6 * d["u_true"].astype(np.float64) + 0.0137
    lin = P.linearise(u)
    n = u.size
    h = d["spacing"]
    nd = oracle.ngf(P.gR, P.gT, h, P.w.eta, u, want=("s", "diag"))
    mk = oracle.mask_term(P.bF, P.bM, h, u)
    cv = oracle.curvature(u - P.u_ref, P.H)
    vc = oracle.vcc(u, P.H)
    kp = oracle.keypoints(u, P.H, P.kp_x, P.kp_t)
    w = P.w
    cols = []
    cols_ref = []
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        e = e.reshape(u.shape)
        cols.append(P.gn_hv(e).ravel())
        # curvature and keypoint terms are quadratic: their Hessian columns are exact
        # differences of their gradients
        d_curv = oracle.curvature(u - P.u_ref + e, P.H)["g"] - cv["g"]
        d_kp = oracle.keypoints(u + e, P.H, P.kp_x, P.kp_t)["g"] - kp["g"]
        col = (oracle.ngf_hv(nd["s"], h, e) + w.alpha * d_curv + w.gamma * oracle.vcc(u, P.H, e)["Hv"]
               + w.delta * d_kp + w.beta * oracle.mask_hv(mk["sb"], h, e))
        cols_ref.append(col.ravel())
    Hm = np.stack(cols, 1)
    Hr = np.stack(cols_ref, 1)
    assert np.linalg.norm(Hm - Hr) <= 1e-10 * np.linalg.norm(Hr)
    diag_ref = nd["diag"] + w.alpha * cv["diag"] + w.gamma * vc["diag"] + w.delta * kp["diag"] + w.beta * mk["diag"]
    np.testing.assert_allclose(lin["diag"], diag_ref, rtol=1e-12, atol=1e-12 * np.max(diag_ref))
    np.testing.assert_allclose(np.diag(Hm), diag_ref.ravel(), rtol=1e-9, atol=1e-9 * np.max(diag_ref))
    assert np.allclose(Hm, Hm.T, atol=1e-10 * np.abs(Hm).max())
    assert np.linalg.eigvalsh(0.5 * (Hm + Hm.T)).min() > -1e-9 * np.abs(Hm).max()
    # the weights matter: unit weights give a different matrix
    P1 = oracle.Problem(d["R"], d["T"], h, d["kp_x"], d["kp_t"], oracle.Weights(eta=W_JOINT["eta"], alpha=1.0,
                        gamma=1.0, delta=1.0, beta=1.0), u_ref=P.u_ref, bF=P.bF, bM=P.bM)
    P1.linearise(u)
    e0 = np.zeros(u.shape)
    e0[2, 1, 1, 1] = 1.0
    assert np.linalg.norm(P1.gn_hv(e0) - P.gn_hv(e0)) > 1e-3 * np.linalg.norm(P.gn_hv(e0))
