"""Multilevel scheme on the device against the FP64 oracle: pyramid downsampling and
prolongation element by element, and a whole coarse-to-fine registration (L-BFGS and GN)
iteration by iteration."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.fields import check_field

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    from paper_1807_00467_amd import disco as d
    return d


# (Nx, Ny, Nz): x spans several 256-wide rows with a ragged tail
@pytest.mark.parametrize("shape", [(600, 20, 12), (36, 44, 28), (8, 6, 10)])
@pytest.mark.parametrize("halve", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 1, 1), (0, 1, 1)])
def test_downsample_matches_oracle(disco, shape, halve):
    say(f"[pyramid] downsample shape={shape} halve={halve}")
    rng = np.random.default_rng(sum(shape) + 7 * sum(halve))
    img = (rng.normal(size=shape[::-1]) * 300.0 - 500.0).astype(np.float32)
    got = disco.pyramid_downsample(torch.from_numpy(img).to(DEV), halve).cpu().numpy()
    ref = oracle.downsample(img, halve)
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err < 2e-6, err


def test_downsample_full_size_sampled(disco):
    """512x512x128 with the first halving of the headline pyramid (x and y): sampled
    coarse voxels against the oracle evaluated on the sub-volumes they depend on."""
    say("[pyramid] downsample 512x512x128, sampled")
    d = synth.make_pair("cfg1")
    R = d["R"]
    got = disco.pyramid_downsample(torch.from_numpy(R).to(DEV), (1, 1, 0)).cpu().numpy()
    assert got.shape == (128, 256, 256)
    rng = np.random.default_rng(3)
    for _ in range(64):
        z, y, x = int(rng.integers(0, 128)), int(rng.integers(0, 256)), int(rng.integers(0, 256))
        # a window of 16 x 16 fine voxels around the coarse voxel, clamped to the volume:
        # the oracle on the window gives the same value as on the whole volume as long as
        # every tap lies inside the window or is clamped the same way
        x0, y0 = min(max(2 * x - 6, 0), 512 - 16), min(max(2 * y - 6, 0), 512 - 16)
        win = R[z:z + 1, y0:y0 + 16, x0:x0 + 16]
        ref_win = oracle.downsample(win, (1, 1, 0))
        # taps of coarse voxel i reach fine 2i - 3 .. 2i + 4: inside the window, or clamped
        # at a volume border that the window shares
        cx, cy = x - x0 // 2, y - y0 // 2
        ref = ref_win[0, cy, cx]
        assert abs(got[z, y, x] - ref) <= 2e-6 * max(1.0, abs(ref)), (z, y, x)


@pytest.mark.parametrize("halve", [(1, 1, 1), (1, 0, 1), (0, 1, 0)])
def test_prolong_matches_oracle(disco, halve):
    say(f"[pyramid] prolong halve={halve}")
    rng = np.random.default_rng(17)
    uc = rng.normal(size=(3, 9, 70, 65)).astype(np.float32) * 5.0
    got = disco.pyramid_prolong(torch.from_numpy(uc).to(DEV), halve).cpu().numpy()
    ref = oracle.prolong(uc, halve)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("optimizer,levels,iters", [("lbfgs", 3, (5, 4, 3)), ("gn", 2, (3, 2))])
def test_multilevel_register_matches_oracle(disco, optimizer, levels, iters):
    say(f"[pyramid] multilevel {optimizer} levels={levels} iters={iters}")
    d = synth.small_pair(shape=(32, 32, 24), spacing=(1.5, 1.5, 2.0), seed=9, n_tubes=8, n_kp=30, field_max=4.0)
    prm = disco.Params(eta=10.0, alpha=1.0, gamma=0.1, delta=0.0, pcg_iters=8, ls_max=10,
                       flags=disco.FLAG_LS_DEVICE)
    lb = disco.Lbfgs(m=5, tau=10.0, h0_iters=60, h0_tol=1e-7)
    ml = disco.Multilevel(levels=levels, optimizer=optimizer, iters=iters, adaptive_delta=True)
    u, rep, L, delta = disco.multilevel_register(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV),
                                                 d["spacing"], d["kp_x"], d["kp_t"], prm, ml, lb)
    torch.cuda.synchronize()
    w = oracle.Weights(eta=10.0, alpha=1.0, gamma=0.1, delta=-1.0)
    op = oracle.MultilevelParams(levels=levels, iters=iters, optimizer=optimizer,
                                 lbfgs=oracle.LbfgsParams(m=5, tau=10.0, ls_max=10),
                                 step=oracle.StepParams(pcg_iters=8, ls_max=10))
    uo, lv = oracle.multilevel_run(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"], w, op)
    assert L == len(lv) == levels
    assert abs(delta - lv[0]["delta"]) <= 1e-5 * lv[0]["delta"]
    rep = rep.cpu().numpy()
    row = 0
    for k, lvl in enumerate(lv):
        for i in range(iters[k]):
            r = rep[row + i]
            if i < len(lvl["reports"]):
                o = lvl["reports"][i]
                say(f"  level {k} it {i}: J {r[0]:.8e} / {o['J']:.8e} t {r[6]} / {o['t']}")
                assert abs(r[0] - o["J"]) <= 1e-5 * abs(o["J"]), (k, i)
                assert r[6] == o["t"], (k, i)
            else:
                assert np.all(np.isnan(r)), (k, i)
        row += iters[k]
    check_field("final u", u, uo, None, 2e-3)


def test_multilevel_register_fp16_storage_runs(disco):
    """A coarse-to-fine run with FP16 storage on every level lowers J on every level."""
    say("[pyramid] multilevel, FP16 storage")
    d = synth.small_pair(shape=(32, 32, 24), spacing=(1.5, 1.5, 2.0), seed=10, n_tubes=8, n_kp=30, field_max=4.0)
    prm = disco.Params(eta=10.0, alpha=1.0, gamma=0.1, delta=0.0, ls_max=10, flags=disco.FLAG_LS_DEVICE)
    ml = disco.Multilevel(levels=3, optimizer="lbfgs", iters=(4, 3, 2), adaptive_delta=True, storage="fp16")
    u, rep, L, delta = disco.multilevel_register(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV),
                                                 d["spacing"], d["kp_x"], d["kp_t"], prm, ml,
                                                 disco.Lbfgs(h0_iters=60, h0_tol=1e-7))
    torch.cuda.synchronize()
    rep = rep.cpu().numpy()
    assert L == 3 and delta > 0 and torch.isfinite(u).all()
    row = 0
    for n in (4, 3, 2):
        r = rep[row:row + n]
        r = r[~np.isnan(r[:, 0])]
        assert len(r) >= 1 and r[-1, 10] < r[0, 0]
        row += n
