"""GPU parity: every entry point of the HIP library against the FP64 oracle.

Tolerances (FP32 storage and arithmetic, FP64 reductions): objective values rel 1e-5;
gradient, GN diagonal, s vectors and GN products rel-L2 1e-4 and element-wise 1e-4 of
the field's largest entry, beyond the oracle's sample-cell tie allowance (see
``tests/fields.py``); the GN step (after a 10-iteration FP32 CG) 1e-3 on the step and
identical accept decisions.  The numerical status paths of the step (a folded trial
rejected, no step accepted, CG breakdown) are compared with the oracle's decisions.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.fields import check_field, rel, rel_l2, say, say_ties

pytestmark = pytest.mark.gpu

TOL_OBJ = 1e-5
TOL_FIELD = 1e-4


@pytest.fixture(scope="module")
def disco():
    from paper_1807_00467_amd import disco as d
    return d


DEV = torch.device("cuda:0")

CASES = {
    # name: (shape, spacing, seed)
    "small": ((32, 24, 20), (1.5, 1.5, 2.0), 11),
    # cells (19, 9, 7): ragged in every brick dimension (16 x 4 x 4 cells per brick)
    "ragged": ((76, 36, 28), (1.2, 1.4, 2.2), 12),
    # one cell row/layer in y and z
    "thin": ((68, 4, 4), (1.0, 1.0, 1.0), 13),
}


def make_case(name):
    shape, spacing, seed = CASES[name]
    return synth.small_pair(shape=shape, spacing=spacing, seed=seed, n_tubes=8, n_kp=40, field_max=4.0)


class Setup:
    def __init__(self, disco, d, eta=10.0, alpha=1.0, gamma=0.1, delta=2.0):
        self.d = d
        self.ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
        self.ctx.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV))
        self.ctx.set_keypoints(d["kp_x"], d["kp_t"])
        self.P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"],
                                oracle.Weights(eta=eta, alpha=alpha, gamma=gamma, delta=delta))
        self.params = disco.Params(eta=eta, alpha=alpha, gamma=gamma, delta=delta)

    def t(self, a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def lin_points(d):
    rng = np.random.default_rng(5)
    return {
        "zero": np.zeros_like(d["u_true"]),
        "true": d["u_true"],
        # off every cell face: no sample-cell ties, the allowance is zero
        "generic": (d["u_true"] + np.float32(0.0137)).astype(np.float32),
        "rand": (0.6 * d["u_true"] + 0.3 * rng.standard_normal(d["u_true"].shape)).astype(np.float32),
    }


@pytest.mark.parametrize("case", list(CASES))
def test_image_gradients(disco, case):
    say(f"[image_gradients] case={case}")
    d = make_case(case)
    s = Setup(disco, d)
    gR = s.ctx.copy_buffer(disco.BUF_GRAD_R).cpu().numpy()
    gT = s.ctx.copy_buffer(disco.BUF_GRAD_T).cpu().numpy()
    assert rel_l2(gR, s.P.gR) < 1e-6
    assert rel_l2(gT, s.P.gT) < 1e-6


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("point", ["zero", "true", "generic", "rand"])
def test_ngf_eval_grad_hessvec(disco, case, point):
    say(f"[ngf] case={case} point={point}")
    d = make_case(case)
    s = Setup(disco, d)
    u = lin_points(d)[point]
    u64 = u.astype(np.float64)
    ref = s.P.ngf(u64, want=("g", "diag", "s"))
    ties = oracle.ngf_ties(s.P.gR, s.P.gT, d["spacing"], s.params.eta, u64, d["v"], want_s=True)
    say_ties(point, ties)
    if point in ("zero", "generic"):
        assert ties["n"] == 0
    D = s.ctx.ngf_eval(s.t(u), s.params.eta).item()
    assert rel(D, ref["D"]) < TOL_OBJ
    D2, g, diag = s.ctx.ngf_grad(s.t(u), s.params.eta)
    assert rel(D2.item(), ref["D"]) < TOL_OBJ
    check_field("grad", g, ref["g"], ties["g"], TOL_FIELD)
    check_field("diag", diag, ref["diag"], ties["diag"], TOL_FIELD)
    sc = s.ctx.copy_buffer(disco.BUF_SCACHE)
    check_field("s", sc, ref["s"], ties["s"], TOL_FIELD)
    hv = s.ctx.ngf_hessvec(s.t(d["v"]))
    hv_ref = oracle.ngf_hv(ref["s"], d["spacing"], d["v"])
    check_field("NGF Hv", hv, hv_ref, ties["hv"], TOL_FIELD)


@pytest.mark.parametrize("case", list(CASES))
def test_curvature(disco, case):
    say(f"[curvature] case={case}")
    d = make_case(case)
    s = Setup(disco, d)
    u = lin_points(d)["rand"]
    uref = (0.5 * d["u_true"]).astype(np.float32)
    alpha = 1.7
    ref = oracle.curvature(u.astype(np.float64) - uref, s.P.H)
    S, out, diag = s.ctx.curvature_apply(alpha, s.t(u), s.t(uref), energy=True, grad=True, diag=True)
    assert rel(S.item(), alpha * ref["S"]) < TOL_OBJ
    check_field("curvature grad", out, alpha * ref["g"], None, TOL_FIELD)
    check_field("curvature diag", diag, alpha * ref["diag"], None, 1e-6)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("point", ["zero", "true", "rand"])
def test_volchange(disco, case, point):
    say(f"[vcc] case={case} point={point}")
    d = make_case(case)
    s = Setup(disco, d)
    u = lin_points(d)[point]
    gamma = 0.3
    ref = oracle.vcc(u.astype(np.float64), s.P.H, d["v"])
    out = s.ctx.volchange_eval(gamma, s.t(u), s.t(d["v"]))
    assert int(out["nfold"].item()) == ref["nfold"] == 0
    if point == "zero":
        # Vhat = 0 up to FP32 rounding of d = 1
        assert abs(out["V"].item()) <= 1e-9 * np.prod(s.P.H) * 64 * np.prod([n - 1 for n in s.P.nodes])
        assert np.max(np.abs(out["g"].cpu().numpy())) < 1e-4
    else:
        assert rel(out["V"].item(), gamma * ref["V"]) < 1e-4
        check_field("VCC grad", out["g"], gamma * ref["g"], None, TOL_FIELD)
    check_field("VCC diag", out["diag"], gamma * ref["diag"], None, TOL_FIELD)
    check_field("VCC Hv", out["Hv"], gamma * ref["Hv"], None, TOL_FIELD)


def test_volchange_fold_is_infinite(disco):
    say("[vcc fold]")
    d = make_case("small")
    s = Setup(disco, d)
    u = np.zeros_like(d["u_true"])
    u[0, 2, 2, 2] = -8.0  # pushes a node past its neighbour along x (H_x = 6 mm)
    ref = oracle.vcc(u.astype(np.float64), s.P.H)
    out = s.ctx.volchange_eval(0.1, s.t(u), None)
    assert ref["nfold"] > 0 and np.isinf(ref["V"])
    assert int(out["nfold"].item()) == ref["nfold"]
    assert np.isinf(out["V"].item())


@pytest.mark.parametrize("case", list(CASES))
def test_keypoints(disco, case):
    say(f"[keypoints] case={case}")
    d = make_case(case)
    s = Setup(disco, d)
    u = lin_points(d)["rand"]
    delta = 2.5
    ref = oracle.keypoints(u.astype(np.float64), s.P.H, d["kp_x"], d["kp_t"], d["v"])
    out = s.ctx.keypoint_penalty(delta, s.t(u), s.t(d["v"]))
    assert rel(out["K"].item(), delta * ref["K"]) < TOL_OBJ
    check_field("keypoint grad", out["g"], delta * ref["g"], None, TOL_FIELD)
    check_field("keypoint diag", out["diag"], delta * ref["diag"], None, TOL_FIELD)
    check_field("keypoint Hv", out["Hv"], delta * ref["Hv"], None, TOL_FIELD)


def test_keypoints_empty_and_border(disco):
    say("[keypoints empty/border]")
    d = make_case("small")
    s = Setup(disco, d)
    u = s.t(d["u_true"])
    s.ctx.set_keypoints(np.zeros((0, 3)), np.zeros((0, 3)))
    out = s.ctx.keypoint_penalty(1.0, u, s.t(d["v"]))
    assert out["K"].item() == 0.0 and float(out["g"].abs().max()) == 0.0
    ext = np.array(d["shape"]) * np.array(d["spacing"])
    x = np.array([[0.0, 0.0, 0.0], ext, [ext[0], 0.0, ext[2] / 2]], np.float32)
    t = x + 1.0
    s.ctx.set_keypoints(x, t)
    ref = oracle.keypoints(d["u_true"].astype(np.float64), s.P.H, x, t)
    out = s.ctx.keypoint_penalty(1.0, u)
    assert rel(out["K"].item(), ref["K"]) < TOL_OBJ
    with pytest.raises(disco.DiscoError) as e:
        s.ctx.set_keypoints(np.array([[ext[0] + 0.1, 1.0, 1.0]]), np.zeros((1, 3)))
    assert e.value.code == disco.ERR_SHAPE


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("point", ["zero", "true", "generic"])
@pytest.mark.parametrize("alpha", [1.0, 1.7])
def test_gn_hessvec_full(disco, case, point, alpha):
    say(f"[gn_hessvec] case={case} point={point} alpha={alpha}")
    d = make_case(case)
    s = Setup(disco, d, alpha=alpha, gamma=0.3, delta=2.5)
    u = lin_points(d)[point]
    s.ctx.ngf_grad(s.t(u), s.params.eta)
    hv = s.ctx.gn_hessvec(s.params, s.t(d["v"]))
    s.P.linearise(u.astype(np.float64))
    ref = s.P.gn_hv(d["v"].astype(np.float64))
    ties = s.P.ties(u.astype(np.float64), d["v"])
    say_ties(point, ties)
    check_field("GN Hv", hv, ref, ties["hv"], TOL_FIELD)


@pytest.mark.parametrize("case", ["small", "ragged"])
@pytest.mark.parametrize("ls_device", [False, True])
@pytest.mark.parametrize("alpha", [1.0, 1.7])
def test_gn_pcg_step(disco, case, ls_device, alpha):
    say(f"[gn_pcg_step] case={case} ls_device={ls_device} alpha={alpha}")
    d = make_case(case)
    s = Setup(disco, d, alpha=alpha, gamma=0.3)
    u0 = np.zeros_like(d["u_true"], np.float64)
    s.P.w.delta = s.P.adaptive_delta(u0)
    s.params.delta = s.P.w.delta
    s.params.pcg_iters = 10
    s.params.flags = disco.FLAG_LS_DEVICE if ls_device else 0
    u_gpu = s.t(u0)
    rep, st = s.ctx.gn_pcg_step(s.params, u_gpu)
    r = disco.Disco.report_dict(rep)
    u1, ref = oracle.gn_pcg_step(s.P, u0, oracle.StepParams(pcg_iters=10))
    say(f"  gpu J {r['J']:.6e} -> {r['J_new']:.6e} t={r['t']}  oracle J {ref['J']:.6e} -> {ref['trial']['J']:.6e} "
        f"t={ref['t']}")
    assert int(st.item()) == 0
    for k in ("J", "D", "S", "K"):
        assert rel(r[k], ref[k]) < TOL_OBJ, k
    assert rel(r["gnorm"], ref["gnorm"]) < TOL_FIELD
    assert r["t"] == ref["t"] and r["pcg_iters"] == 10
    step_gpu = u_gpu.cpu().numpy().astype(np.float64) - u0
    check_field("step", step_gpu, u1 - u0, None, 1e-3)
    assert r["J_new"] < r["J"]
    assert rel(r["J_new"], ref["trial"]["J"]) < 1e-4


def fold_case(disco):
    """Crossing keypoint pairs (two points one cell apart along x with their targets
    swapped and pushed past each other) under a weak curvature weight: the full GN step
    folds the grid (Vhat = +inf, eq. 9), the half step does not."""
    d = make_case("small")
    H = np.array(d["spacing"]) * 4
    xs, ts = [], []
    for c in [(2, 2, 2), (4, 3, 2), (5, 2, 3)]:
        p0 = (np.array(c) + 0.5) * H
        p1 = p0 + np.array([H[0], 0, 0])
        xs += [p0, p1]
        ts += [p1 + np.array([0.3 * H[0], 0, 0]), p0 - np.array([0.3 * H[0], 0, 0])]
    d["kp_x"] = np.array(xs, np.float32)
    d["kp_t"] = np.array(ts, np.float32)
    return Setup(disco, d, alpha=0.01, gamma=0.01, delta=100.0), d


@pytest.mark.parametrize("ls_device", [False, True])
def test_gn_step_rejects_folded_trial(disco, ls_device):
    say(f"[gn_pcg_step fold] ls_device={ls_device}")
    s, d = fold_case(disco)
    s.params.pcg_iters = 10
    s.params.flags = disco.FLAG_LS_DEVICE if ls_device else 0
    u0 = np.zeros_like(d["u_true"], np.float64)
    u1, ref = oracle.gn_pcg_step(s.P, u0, oracle.StepParams(pcg_iters=10))
    full = s.P.objective(u0 + ref["p"])
    half = s.P.objective(u0 + 0.5 * ref["p"])
    say(f"  oracle: t=1 trial folds {full['nfold']} coefficients; t=1/2 folds {half['nfold']}; accepted t={ref['t']}")
    assert full["nfold"] > 0 and half["nfold"] == 0 and ref["t"] == 0.5 and ref["accepted"]
    u_gpu = s.t(u0)
    rep, st = s.ctx.gn_pcg_step(s.params, u_gpu)
    r = disco.Disco.report_dict(rep)
    say(f"  gpu: t={r['t']} trials={r['ls_trials']} J {r['J']:.6e} -> {r['J_new']:.6e} status {int(st.item())}")
    assert int(st.item()) == 0
    assert r["t"] == ref["t"] and r["ls_trials"] == 2
    assert np.isfinite(r["J_new"]) and rel(r["J_new"], ref["trial"]["J"]) < 1e-4
    check_field("step", u_gpu.cpu().numpy().astype(np.float64) - u0, u1 - u0, None, 1e-3)
    # the device's own volume-change evaluation agrees that the full step folds
    vf = s.ctx.volchange_eval(s.params.gamma, s.t(u0 + ref["p"]), None)
    assert int(vf["nfold"].item()) > 0 and np.isinf(vf["V"].item())


@pytest.mark.parametrize("ls_device", [False, True])
def test_gn_step_line_search_failure(disco, ls_device):
    """Armijo constant 0.9999 with one trial: a GN step decreases J by about half its
    linear prediction, so no step is accepted; status LS_FAIL and u unchanged."""
    say(f"[gn_pcg_step LS_FAIL] ls_device={ls_device}")
    d = make_case("small")
    s = Setup(disco, d)
    s.params.pcg_iters = 10
    s.params.armijo_c1 = 0.9999
    s.params.ls_max = 1
    s.params.flags = disco.FLAG_LS_DEVICE if ls_device else 0
    u0 = (0.5 * d["u_true"]).astype(np.float32)
    u1, ref = oracle.gn_pcg_step(s.P, u0.astype(np.float64), oracle.StepParams(pcg_iters=10, armijo_c1=0.9999,
                                                                                ls_max=1))
    assert not ref["accepted"]
    u_gpu = s.t(u0)
    rep, st = s.ctx.gn_pcg_step(s.params, u_gpu)
    r = disco.Disco.report_dict(rep)
    say(f"  gpu: status {int(st.item())} t={r['t']} trials={r['ls_trials']}; oracle accepted={ref['accepted']}")
    assert int(st.item()) == disco.STATUS_LS_FAIL
    assert r["t"] == 0.0 and r["ls_trials"] == 1
    assert np.array_equal(u_gpu.cpu().numpy(), u0)


@pytest.mark.parametrize("ls_device", [False, True])
def test_gn_step_pcg_breakdown(disco, ls_device):
    """T = R = 0 with alpha = gamma = delta = 0: every NGF quantity is exactly zero (both
    image gradients vanish), so grad J = 0, the GN matrix is zero and the first p^T H p is
    not positive.  Status PCG_BREAKDOWN, the zero step accepted at t = 1 (J = 0 <= 0 + 0),
    u unchanged."""
    say(f"[gn_pcg_step breakdown] ls_device={ls_device}")
    d = make_case("small")
    zero = np.zeros_like(d["R"])
    d = dict(d, R=zero, T=zero.copy())
    s = Setup(disco, d, alpha=0.0, gamma=0.0, delta=0.0)
    s.params.pcg_iters = 10
    s.params.flags = disco.FLAG_LS_DEVICE if ls_device else 0
    u0 = np.zeros_like(d["u_true"])
    with np.errstate(invalid="ignore", divide="ignore"):
        u1, ref = oracle.gn_pcg_step(s.P, u0.astype(np.float64), oracle.StepParams(pcg_iters=10))
    assert ref["pcg"]["breakdown"] and ref["pcg"]["iters"] == 0 and ref["accepted"] and ref["t"] == 1.0
    u_gpu = s.t(u0)
    rep, st = s.ctx.gn_pcg_step(s.params, u_gpu)
    r = disco.Disco.report_dict(rep)
    say(f"  gpu: status {int(st.item())} t={r['t']} pcg_iters={r['pcg_iters']} gnorm={r['gnorm']}")
    assert int(st.item()) == disco.STATUS_PCG_BREAKDOWN
    assert r["pcg_iters"] == 0 and r["t"] == 1.0 and r["gnorm"] == 0.0
    assert np.array_equal(u_gpu.cpu().numpy(), u0)


def test_gn_pcg_step_converged_tolerance(disco):
    say("[gn_pcg_step tol]")
    d = make_case("small")
    s = Setup(disco, d)
    s.params.pcg_iters = 200
    s.params.pcg_tol = 1e-2
    u = s.t(np.zeros_like(d["u_true"]))
    rep, st = s.ctx.gn_pcg_step(s.params, u)
    r = disco.Disco.report_dict(rep)
    assert r["pcg_iters"] < 200
    assert r["pcg_res"] <= 1e-2 * r["gnorm"] * (1 + 1e-6)


def test_determinism_bitwise(disco):
    say("[determinism]")
    d = make_case("ragged")
    s = Setup(disco, d)
    u = s.t(d["u_true"])
    v = s.t(d["v"])
    outs = []
    for _ in range(2):
        D, g, diag = s.ctx.ngf_grad(u, s.params.eta)
        hv = s.ctx.gn_hessvec(s.params, v)
        outs.append((D.item(), g.cpu().numpy(), diag.cpu().numpy(), hv.cpu().numpy()))
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1:], outs[1][1:]):
        assert np.array_equal(a, b)


def test_state_and_argument_errors(disco):
    say("[errors]")
    d = make_case("small")
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    v = torch.zeros(ctx.nodes[::-1], device=DEV)
    v = torch.zeros((3,) + tuple(ctx.nodes[::-1]), device=DEV)
    with pytest.raises(disco.DiscoError) as e:
        ctx.ngf_eval(v, 10.0)
    assert e.value.code == disco.ERR_STATE
    with pytest.raises(disco.DiscoError) as e:
        ctx.ngf_hessvec(v)
    assert e.value.code == disco.ERR_STATE
    ctx.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV))
    with pytest.raises(disco.DiscoError) as e:
        ctx.ngf_eval(v, float("nan"))
    assert e.value.code == disco.ERR_NONFINITE
    with pytest.raises(disco.DiscoError) as e:
        ctx.gn_hessvec(disco.Params(), v)
    assert e.value.code == disco.ERR_STATE
    with pytest.raises(disco.DiscoError) as e:
        ctx.gn_pcg_step(disco.Params(pcg_iters=0), v)
    assert e.value.code == disco.ERR_ARG
    ctx.close()
