"""Batched form: one launch per phase of the GN step over many pairs of uneven sizes.

The batched kernels run the single-pair device bodies on (pair, block) work items, so every
pair's step must agree with gn_pcg_step (device line search) on the same inputs up to
rounding: the two are separately compiled kernels, in which the compiler may fuse
different multiply-adds.  The single-pair step is checked against the FP64 oracle
elsewhere, and one pair is checked against the oracle here as well.  A captured graph of
two steps must reproduce the eager batched steps bitwise on every replay (same kernels),
with eager work and synchronisation in between.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.fields import check_field, say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ETA, ALPHA, GAMMA = 10.0, 1.0, 0.1

# uneven shapes (voxels), spacings, seeds; the first is the largest
CASES = [((64, 48, 32), (1.5, 1.5, 2.0), 51), ((76, 36, 28), (1.2, 1.4, 2.2), 54), ((48, 32, 24), (1.2, 1.4, 2.2), 53),
         ((32, 24, 20), (1.5, 1.5, 2.0), 52), ((16, 16, 12), (1.5, 1.5, 1.5), 55)]


@pytest.fixture(scope="module")
def disco():
    from paper_1807_00467_amd import disco as d
    return d


@pytest.fixture(scope="module")
def pairs():
    return [synth.small_pair(shape=sh, spacing=sp, seed=sd, n_tubes=8, n_kp=30, field_max=4.0) for sh, sp, sd in CASES]


def make_ctx(disco, d, storage="fp32"):
    ctx = disco.Disco(d["shape"], d["spacing"], storage=storage, device=DEV)
    ctx.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV))
    ctx.set_keypoints(d["kp_x"], d["kp_t"])
    return ctx


def params_for(disco, ctx, d, iters=6, ls_max=6):
    z = torch.zeros((3,) + tuple(ctx.nodes[::-1]), device=DEV)
    D0 = ctx.ngf_eval(z, ETA).item()
    K0 = ctx.keypoint_penalty(1.0, z, grad=False, diag=False)["K"].item()
    return disco.Params(eta=ETA, alpha=ALPHA, gamma=GAMMA, delta=D0 / K0, pcg_iters=iters, ls_max=ls_max,
                        flags=disco.FLAG_LS_DEVICE)


@pytest.mark.parametrize("tile", [4, 2])
@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_batch_step_equals_single_pair(disco, pairs, storage, tile):
    """Both brick tiles (16 x 4 x 4 and 16 x 4 x 2 cells): the tile changes the order in
    which brick contributions are summed, so the comparison is to rounding."""
    say(f"[batch] {len(pairs)} pairs, storage={storage}, tile cells_z={tile}")
    cb = [make_ctx(disco, d, storage) for d in pairs]
    cs = [make_ctx(disco, d, storage) for d in pairs]
    params = [params_for(disco, c, d) for c, d in zip(cb, pairs)]
    u0 = [torch.from_numpy(d["u_true"]).to(DEV) * 0.5 for d in pairs]
    ub = [u.clone() for u in u0]
    us = [u.clone() for u in u0]
    batch = disco.Batch(cb)
    rep, st = batch.prepare(params, ub)
    batch.set_tile(tile)
    batch.gn_step()
    torch.cuda.synchronize()
    rep1 = rep.clone()
    ub1 = [u.clone() for u in ub]
    batch.gn_step()
    torch.cuda.synchronize()
    for i, (c, p) in enumerate(zip(cs, params)):
        rs, ss = c.gn_pcg_step(p, us[i])
        torch.cuda.synchronize()
        rb, rsd = disco.Disco.report_dict(rep1[i]), disco.Disco.report_dict(rs)
        for k in ("J", "D", "S", "V", "K", "gnorm", "J_new"):
            assert abs(rb[k] - rsd[k]) <= 1e-6 * abs(rsd[k]) + 1e-12, (i, k, rb[k], rsd[k])
        assert rb["t"] == rsd["t"] and rb["pcg_iters"] == rsd["pcg_iters"] and int(st[i].item()) == int(ss.item())
        say(f"  pair {i}:")
        check_field("step 1", ub1[i] - u0[i], us[i] - u0[i], None, 1e-5)
        rs, ss = c.gn_pcg_step(p, us[i])
        torch.cuda.synchronize()
        check_field("after 2 steps", ub[i] - u0[i], us[i] - u0[i], None, 1e-4)
    r0 = disco.Disco.report_dict(rep[0])
    say(f"  pair 0: J {r0['J']:.6e} -> {r0['J_new']:.6e}, t={r0['t']}")
    assert r0["J_new"] < r0["J"]
    batch.close()


@pytest.mark.parametrize("tile", [4, 2])
def test_batch_step_matches_oracle(disco, pairs, tile):
    """The largest pair of the batch, one step from u_true / 2, against the FP64 oracle."""
    say(f"[batch] oracle check, tile cells_z={tile}")
    cb = [make_ctx(disco, d) for d in pairs]
    params = [params_for(disco, c, d) for c, d in zip(cb, pairs)]
    u0 = [(torch.from_numpy(d["u_true"]) * 0.5).to(DEV) for d in pairs]
    batch = disco.Batch(cb)
    batch.set_tile(tile)
    rep, st = batch.prepare(params, u0)
    batch.gn_step()
    torch.cuda.synchronize()
    d = pairs[0]
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"],
                       oracle.Weights(eta=ETA, alpha=ALPHA, gamma=GAMMA, delta=params[0].delta))
    uo = d["u_true"].astype(np.float64) * 0.5
    u1, ref = oracle.gn_pcg_step(P, uo, oracle.StepParams(pcg_iters=6, ls_max=6))
    r = disco.Disco.report_dict(rep[0])
    for k in ("J", "D", "S", "K"):
        assert abs(r[k] - ref[k]) <= 1e-5 * abs(ref[k]), k
    assert abs(r["V"] - ref["V"]) <= 1e-4 * abs(ref["V"])
    assert r["t"] == ref["t"]
    step = u0[0].cpu().numpy().astype(np.float64) - uo
    check_field("step", step, u1 - uo, None, 1e-3)
    batch.close()


def test_batch_graph_replays_match_eager(disco, pairs):
    say("[batch] graph of 2 steps, 3 replays")
    cb = [make_ctx(disco, d) for d in pairs]
    params = [params_for(disco, c, d) for c, d in zip(cb, pairs)]
    u0 = [(torch.from_numpy(d["u_true"]) * 0.5).to(DEV) for d in pairs]
    us = [u.clone() for u in u0]
    batch = disco.Batch(cb)
    rep, st = batch.prepare(params, us)
    for _ in range(2):
        batch.gn_step()
    torch.cuda.synchronize()
    ref_u = [u.clone() for u in us]
    ref_rep = rep.clone()
    batch.graph_capture(2)
    for k in range(3):
        for u, a in zip(us, u0):
            u.copy_(a)
        rep.zero_()
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        batch.graph_launch()
        torch.cuda.synchronize()
        assert bool(torch.isfinite(junk))
        for i in range(len(us)):
            assert torch.equal(us[i], ref_u[i]), f"replay {k}, pair {i}"
        assert torch.equal(rep, ref_rep), f"replay {k}: report"
    batch.close()


def test_batch_argument_errors(disco, pairs):
    cb = [make_ctx(disco, d) for d in pairs[:2]]
    params = [params_for(disco, c, d) for c, d in zip(cb, pairs[:2])]
    us = [(torch.from_numpy(d["u_true"]) * 0.0).to(DEV) for d in pairs[:2]]
    with pytest.raises(disco.DiscoError) as e:
        disco.Batch([cb[0], cb[0]])
    assert e.value.code == disco.ERR_ARG
    batch = disco.Batch(cb)
    with pytest.raises(disco.DiscoError) as e:
        batch.gn_step()  # not prepared
    assert e.value.code == disco.ERR_STATE
    with pytest.raises(disco.DiscoError) as e:
        batch.graph_launch()
    assert e.value.code == disco.ERR_STATE
    host_ls = [disco.Params(**{**p.__dict__, "flags": 0}) for p in params]
    with pytest.raises(disco.DiscoError) as e:
        batch.prepare(host_ls, us)  # the batch needs the device line search
    assert e.value.code == disco.ERR_ARG
    mixed = [params[0], disco.Params(**{**params[1].__dict__, "gamma": 0.0})]
    with pytest.raises(disco.DiscoError) as e:
        batch.prepare(mixed, us)  # terms present must agree
    assert e.value.code == disco.ERR_ARG
    with pytest.raises(disco.DiscoError) as e:
        batch.set_launch(3, 4)
    assert e.value.code == disco.ERR_ARG
    batch.close()


@pytest.mark.parametrize("shape", [(0, 0, 0), (1, 2, 2), (4, 16, 16), (3, 0, 8)])
def test_batch_launch_shapes_agree(disco, pairs, shape):
    """The launch shape only changes which workgroup takes which work item: persistent grids
    of 1..16 workgroups per compute unit (capped at each kernel's residency) and one
    workgroup per item (0) give the same step bitwise."""
    say(f"[batch] launch shape {shape}")
    ctx_a = [make_ctx(disco, d) for d in pairs]
    ctx_b = [make_ctx(disco, d) for d in pairs]
    params = [params_for(disco, c, d) for c, d in zip(ctx_a, pairs)]
    u0 = [torch.from_numpy(d["u_true"]).to(DEV) * 0.5 for d in pairs]
    ua = [u.clone() for u in u0]
    ub = [u.clone() for u in u0]
    ba, bb = disco.Batch(ctx_a), disco.Batch(ctx_b)
    ra, _ = ba.prepare(params, ua)
    rb, _ = bb.prepare(params, ub)
    for p_, w in enumerate(shape):
        bb.set_launch(p_, w)
    for _ in range(2):
        ba.gn_step()
        bb.gn_step()
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    for x, y in zip(ua, ub):
        assert torch.equal(x, y)
    ba.close()
    bb.close()


def test_autotune_choice_and_cache(disco, pairs, tmp_path, monkeypatch):
    """The tuner returns a tile and launch shapes from its candidate sets, stores them under
    the batch's key, and a later call with the same key returns the stored choice without
    timing anything; the choice applied to a prepared batch steps like the default."""
    from paper_1807_00467_amd import autotune
    say("[batch] autotune")
    ctxs = [make_ctx(disco, d) for d in pairs]
    params = [params_for(disco, c, d, iters=3, ls_max=3) for c, d in zip(ctxs, pairs)]
    u0 = [torch.from_numpy(d["u_true"]).to(DEV) * 0.5 for d in pairs]
    keep = [u.clone() for u in u0]
    cache = str(tmp_path / "autotune.json")
    choice = autotune.tune(ctxs, params, u0, reps=1, cache=cache, log=say)
    say(f"  choice {choice}")
    assert set(choice) == set(autotune.CANDIDATES)
    for k, w in choice.items():
        assert w in autotune.CANDIDATES[k]
    for a, b in zip(u0, keep):
        assert torch.equal(a, b)  # the timing ran on copies
    import json
    with open(cache) as f:
        table = json.load(f)
    assert table[autotune.batch_key(ctxs, params)] == {str(k): v for k, v in choice.items()}

    def no_timing(*a, **k):
        raise AssertionError("a cache hit must not time")

    monkeypatch.setattr(autotune, "_time_steps", no_timing)
    assert autotune.tune(ctxs, params, u0, cache=cache) == choice
    # the choice applied after prepare (set_tile prepares again) against the default shapes
    ua = [u.clone() for u in u0]
    ub = [u.clone() for u in u0]
    ba, bb = disco.Batch(ctxs), disco.Batch([make_ctx(disco, d) for d in pairs])
    ra, _ = ba.prepare(params, ua)
    autotune.apply(ba, choice)
    rb, _ = bb.prepare(params, ub)
    ba.gn_step()
    bb.gn_step()
    torch.cuda.synchronize()
    for i in range(len(pairs)):
        x, y = disco.Disco.report_dict(ra[i]), disco.Disco.report_dict(rb[i])
        assert abs(x["J_new"] - y["J_new"]) <= 1e-6 * abs(y["J_new"]), (i, x["J_new"], y["J_new"])
        assert x["t"] == y["t"]
    ba.close()
    bb.close()
