"""GPU parity: every entry point of the HIP library against the FP64 oracle.

Tolerances (FP32 storage and arithmetic, FP64 reductions): objective values rel 1e-5;
gradient, GN diagonal and GN products rel-L2 1e-4; the GN step (after a 10-iteration
FP32 CG) rel-L2 1e-3 on the step and identical accept decisions.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_OBJ = 1e-5
TOL_FIELD = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


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
@pytest.mark.parametrize("point", ["zero", "true", "rand"])
def test_ngf_eval_grad_hessvec(disco, case, point):
    say(f"[ngf] case={case} point={point}")
    d = make_case(case)
    s = Setup(disco, d)
    u = lin_points(d)[point]
    ref = s.P.ngf(u.astype(np.float64), want=("g", "diag", "s"))
    D = s.ctx.ngf_eval(s.t(u), s.params.eta).item()
    assert rel(D, ref["D"]) < TOL_OBJ
    D2, g, diag = s.ctx.ngf_grad(s.t(u), s.params.eta)
    assert rel(D2.item(), ref["D"]) < TOL_OBJ
    assert rel_l2(g.cpu().numpy(), ref["g"]) < TOL_FIELD
    assert rel_l2(diag.cpu().numpy(), ref["diag"]) < TOL_FIELD
    sc = s.ctx.copy_buffer(disco.BUF_SCACHE).cpu().numpy()
    assert rel_l2(sc, ref["s"]) < TOL_FIELD
    hv = s.ctx.ngf_hessvec(s.t(d["v"])).cpu().numpy()
    hv_ref = oracle.ngf_hv(ref["s"], d["spacing"], d["v"])
    assert rel_l2(hv, hv_ref) < TOL_FIELD


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
    assert rel_l2(out.cpu().numpy(), alpha * ref["g"]) < TOL_FIELD
    assert rel_l2(diag.cpu().numpy(), alpha * ref["diag"]) < 1e-6


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
        assert rel_l2(out["g"].cpu().numpy(), gamma * ref["g"]) < TOL_FIELD
    assert rel_l2(out["diag"].cpu().numpy(), gamma * ref["diag"]) < TOL_FIELD
    assert rel_l2(out["Hv"].cpu().numpy(), gamma * ref["Hv"]) < TOL_FIELD


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
    assert rel_l2(out["g"].cpu().numpy(), delta * ref["g"]) < TOL_FIELD
    assert rel_l2(out["diag"].cpu().numpy(), delta * ref["diag"]) < TOL_FIELD
    assert rel_l2(out["Hv"].cpu().numpy(), delta * ref["Hv"]) < TOL_FIELD


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
@pytest.mark.parametrize("point", ["zero", "true"])
def test_gn_hessvec_full(disco, case, point):
    say(f"[gn_hessvec] case={case} point={point}")
    d = make_case(case)
    s = Setup(disco, d)
    u = lin_points(d)[point]
    s.ctx.ngf_grad(s.t(u), s.params.eta)
    hv = s.ctx.gn_hessvec(s.params, s.t(d["v"])).cpu().numpy()
    s.P.linearise(u.astype(np.float64))
    ref = s.P.gn_hv(d["v"].astype(np.float64))
    assert rel_l2(hv, ref) < TOL_FIELD


@pytest.mark.parametrize("case", ["small", "ragged"])
@pytest.mark.parametrize("ls_device", [False, True])
def test_gn_pcg_step(disco, case, ls_device):
    say(f"[gn_pcg_step] case={case} ls_device={ls_device}")
    d = make_case(case)
    s = Setup(disco, d)
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
    assert rel_l2(step_gpu, u1 - u0) < 1e-3
    assert r["J_new"] < r["J"]
    assert rel(r["J_new"], ref["trial"]["J"]) < 1e-4


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
