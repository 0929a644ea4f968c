"""Keypoint stage (Sec. II-C2, II-C3) on the device against the FP64 oracle: the NGF
matching cost of eq. 2 over all 33^3 displacements (keypoints in the interior, at the
border and of every voxel parity), sampled at the benchmark's workload, and the
regularisation by min-sum belief propagation on the keypoint MST, where both sides take
the oracle's cost volume as the data term."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ETA = 12.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    from paper_1807_00467_amd import disco as d
    return d


def stage(disco, d):
    st = disco.KeypointStage(d["shape"], d["spacing"], device=DEV)
    st.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV), ETA)
    return st


def vox_of(d):
    return np.floor(np.asarray(d["kp_x"], np.float64) / np.asarray(d["spacing"])).astype(np.int32)


@pytest.mark.parametrize("R", [16, 3])
def test_kp_cost_matches_oracle(disco, R):
    say(f"[kp] cost R={R}")
    d = synth.small_pair(shape=(64, 56, 44), spacing=(1.0, 1.0, 1.0), seed=41, n_tubes=10, n_kp=6, field_max=4.0)
    nx, ny, nz = d["shape"]
    kps = np.concatenate([vox_of(d), np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [1, ny - 2, 5], [nx - 2, 3, nz - 1],
                                                [31, 28, 22], [32, 27, 21]], np.int32)]).astype(np.int32)
    st = stage(disco, d)
    got = st.cost(torch.from_numpy(kps).to(DEV), R).cpu().numpy()
    ref = oracle.kp_cost_volume(d["R"], d["T"], d["spacing"], kps, ETA, R=R, step=2)
    err = np.max(np.abs(got - ref))
    say(f"  {len(kps)} keypoints x {ref.shape[1]} labels: max abs error {err:.2e}")
    assert err < 2e-6


def test_kp_cost_fullsize_sampled(disco):
    """The benchmark's workload (1 mm, 3500 keypoints in the lungs): 12 keypoints against
    the oracle over all labels."""
    say("[kp] cost, benchmark workload sampled")
    d = synth.make_pair("kp")
    st = stage(disco, d)
    kps = vox_of(d)
    got = st.cost(torch.from_numpy(kps).to(DEV), 16)
    idx = np.random.default_rng(5).choice(len(kps), 12, replace=False)
    ref = oracle.kp_cost_volume(d["R"], d["T"], d["spacing"], kps[idx], ETA, R=16, step=2)
    err = float(np.max(np.abs(got[torch.from_numpy(idx).to(DEV)].cpu().numpy() - ref)))
    say(f"  {len(kps)} keypoints; sampled max abs error {err:.2e}")
    assert len(kps) == 3500 and err < 2e-6


def test_kp_regularise_matches_oracle(disco):
    say("[kp] belief propagation")
    d = synth.small_pair(shape=(64, 56, 44), spacing=(1.0, 1.0, 1.0), seed=42, n_tubes=10, n_kp=40, field_max=4.0)
    st = stage(disco, d)
    kps = vox_of(d)
    # both sides regularise the oracle's data cost (single precision, the device's input type)
    D32 = oracle.kp_cost_volume(d["R"], d["T"], d["spacing"], kps, ETA, R=16, step=2).astype(np.float32)
    cost = torch.from_numpy(D32).to(DEV)
    x = (kps + 0.5) * np.asarray(d["spacing"])
    inten = d["R"][kps[:, 2], kps[:, 1], kps[:, 0]]
    alpha = 1.0 / 45.0
    marg, lab, par = st.regularise(x, inten, cost, 16, alpha, 150.0)
    torch.cuda.synchronize()
    parent, order = oracle.kp_mst(x.astype(np.float32), inten)
    np.testing.assert_array_equal(par, parent)
    om, _ = oracle.kp_belief_propagation(D32.astype(np.float64), parent, order, x.astype(np.float32), inten, alpha,
                                         R=16, step=2)
    gm = marg.cpu().numpy()
    scale = np.max(np.abs(om), axis=1, keepdims=True)
    err = float(np.max(np.abs(gm - om) / scale))
    say(f"  {len(kps)} keypoints, tree depth {tree_depth(parent, order)}: marginals max rel error {err:.2e}")
    assert err < 1e-5
    # labels: the unique minimum must agree; near-ties only need an equally good label
    gl = lab.cpu().numpy()
    ol = oracle.kp_argmin(om)
    tol = 2e-5 * scale[:, 0]
    srt = np.sort(om, axis=1)
    for k in range(len(kps)):
        if srt[k, 1] - srt[k, 0] > tol[k]:
            assert gl[k] == ol[k], k
        else:
            assert om[k, gl[k]] - srt[k, 0] <= tol[k], k


def tree_depth(parent, order):
    dep = np.zeros(len(parent), int)
    for k in order[1:]:
        dep[k] = dep[parent[k]] + 1
    return int(dep.max())


def test_kp_argument_errors(disco):
    d = synth.small_pair(shape=(16, 16, 12), spacing=(1.0, 1.0, 1.0), seed=43)
    st = disco.KeypointStage(d["shape"], d["spacing"], device=DEV)
    kp = torch.zeros((1, 3), dtype=torch.int32, device=DEV)
    with pytest.raises(disco.DiscoError) as e:
        st.cost(kp, 4)  # images not set
    assert e.value.code == disco.ERR_STATE
    st.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV), ETA)
    with pytest.raises(disco.DiscoError) as e:
        st.cost(kp, 17)
    assert e.value.code == disco.ERR_ARG


@pytest.mark.parametrize("n", [3500, 4200])
def test_kp_tree_and_messages_at_scale(disco, n):
    """3500 and 4200 keypoints: the MST (Boruvka rounds on the device) equals the oracle's
    (Kruskal's algorithm under the same edge order), and the min-marginals agree, with 27
    labels (R = 1)."""
    say(f"[kp] MST + BP with {n} keypoints")
    d = synth.small_pair(shape=(64, 56, 44), spacing=(1.0, 1.0, 1.0), seed=44, n_tubes=10, n_kp=8, field_max=4.0)
    r = np.random.default_rng(n)
    nx, ny, nz = d["shape"]
    flat = r.choice(nx * ny * nz, n, replace=False)  # distinct keypoints
    kps = np.stack([flat % nx, (flat // nx) % ny, flat // (nx * ny)], 1).astype(np.int32)
    st = stage(disco, d)
    D32 = oracle.kp_cost_volume(d["R"], d["T"], d["spacing"], kps, ETA, R=1, step=2).astype(np.float32)
    cost = torch.from_numpy(D32).to(DEV)
    x = (kps + 0.5).astype(np.float32)
    inten = d["R"][kps[:, 2], kps[:, 1], kps[:, 0]]
    marg, lab, par = st.regularise(x, inten, cost, 1, 1.0 / 45.0, 150.0)
    torch.cuda.synchronize()
    parent, order = oracle.kp_mst(x, inten)
    np.testing.assert_array_equal(par, parent)
    om, _ = oracle.kp_belief_propagation(D32.astype(np.float64), parent, order, x, inten, 1.0 / 45.0, R=1, step=2)
    gm = marg.cpu().numpy()
    err = float(np.max(np.abs(gm - om) / np.max(np.abs(om), axis=1, keepdims=True)))
    say(f"  tree depth {tree_depth(parent, order)}; marginals max rel error {err:.2e}")
    assert err < 1e-5


def test_kp_regularise_reuses_work_memory(disco):
    """Calls on one handle of growing size, with and without the min-marginals output (the
    handle's work memory is grown, then reused): labels and marginals equal those of a
    fresh handle bitwise, and the labels match the oracle's."""
    say("[kp] work memory reuse")
    d = synth.small_pair(shape=(64, 56, 44), spacing=(1.0, 1.0, 1.0), seed=45, n_tubes=10, n_kp=8, field_max=4.0)
    st = stage(disco, d)
    r = np.random.default_rng(9)
    nx, ny, nz = d["shape"]
    runs = []
    for n, marginals in ((30, True), (90, False), (60, True)):
        flat = r.choice(nx * ny * nz, n, replace=False)
        kps = np.stack([flat % nx, (flat // nx) % ny, flat // (nx * ny)], 1).astype(np.int32)
        cost = st.cost(torch.from_numpy(kps).to(DEV), 4)
        x = (kps + 0.5).astype(np.float32)
        inten = d["R"][kps[:, 2], kps[:, 1], kps[:, 0]]
        marg, lab, par = st.regularise(x, inten, cost, 4, 1.0 / 45.0, 150.0, marginals=marginals)
        fresh = stage(disco, d)
        marg2, lab2, _ = fresh.regularise(x, inten, cost, 4, 1.0 / 45.0, 150.0, marginals=True)
        torch.cuda.synchronize()
        assert torch.equal(lab, lab2), n
        if marginals:
            assert torch.equal(marg, marg2), n
        parent, order = oracle.kp_mst(x, inten)
        om, _ = oracle.kp_belief_propagation(cost.cpu().numpy().astype(np.float64), parent, order, x, inten,
                                             1.0 / 45.0, R=4, step=2)
        ol = oracle.kp_argmin(om)
        scale = np.max(np.abs(om), axis=1)
        srt = np.sort(om, axis=1)
        gl = lab.cpu().numpy()
        for k in range(n):
            if srt[k, 1] - srt[k, 0] > 2e-5 * scale[k]:
                assert gl[k] == ol[k], (n, k)
        runs.append(n)
    say(f"  sizes {runs} ok")


@pytest.mark.parametrize("n", [1, 2, 3])
def test_kp_regularise_tiny_trees(disco, n):
    """Degenerate trees: one keypoint (its min-marginals are its data cost, bitwise), two
    and three keypoints (against the oracle)."""
    say(f"[kp] tiny tree n={n}")
    d = synth.small_pair(shape=(40, 36, 32), spacing=(1.0, 1.0, 1.0), seed=46, n_tubes=6, n_kp=4, field_max=4.0)
    st = stage(disco, d)
    kps = np.array([[12, 10, 8], [20, 18, 15], [27, 25, 21]], np.int32)[:n]
    cost = st.cost(torch.from_numpy(kps).to(DEV), 16)
    x = (kps + 0.5).astype(np.float32)
    inten = d["R"][kps[:, 2], kps[:, 1], kps[:, 0]]
    marg, lab, par = st.regularise(x, inten, cost, 16, 1.0 / 45.0, 150.0)
    torch.cuda.synchronize()
    parent, order = oracle.kp_mst(x, inten)
    np.testing.assert_array_equal(par, parent)
    if n == 1:
        assert torch.equal(marg, cost)
        assert int(lab[0]) == int(torch.argmin(cost[0]))
        return
    om, _ = oracle.kp_belief_propagation(cost.cpu().numpy().astype(np.float64), parent, order, x, inten, 1.0 / 45.0,
                                         R=16, step=2)
    err = float(np.max(np.abs(marg.cpu().numpy() - om) / np.max(np.abs(om), axis=1, keepdims=True)))
    say(f"  marginals max rel error {err:.2e}")
    assert err < 1e-5


def test_kp_regularise_fullsize_invariants(disco):
    """The benchmark's workload (3500 keypoints, 35 937 labels), where the oracle's full
    belief propagation is too slow to run: the tree equals the oracle's, every keypoint's
    smallest min-marginal is the same number (the minimum of the joint energy), and the
    labels the device picks form a labeling whose energy, evaluated in FP64 from the data
    costs and eq. 3 on the tree, is that minimum.  Bound 1e-5 relative: FP32 messages are
    summed along paths of about 160 tree levels (measured spread 4e-6)."""
    say("[kp] full-size invariants")
    d = synth.make_pair("kp")
    st = stage(disco, d)
    kps = vox_of(d)
    # both sides regularise the oracle's data cost (single precision, the device's input type)
    D32 = oracle.kp_cost_volume(d["R"], d["T"], d["spacing"], kps, ETA, R=16, step=2).astype(np.float32)
    cost = torch.from_numpy(D32).to(DEV)
    x = (kps + 0.5) * np.asarray(d["spacing"])
    inten = d["R"][kps[:, 2], kps[:, 1], kps[:, 0]]
    alpha = 1.0 / 45.0
    marg, lab, par = st.regularise(x, inten, cost, 16, alpha, 150.0)
    torch.cuda.synchronize()
    parent, _ = oracle.kp_mst(x.astype(np.float32), inten)
    np.testing.assert_array_equal(par, parent)
    mins = marg.min(dim=1).values.double().cpu().numpy()
    labs = lab.long()
    data = cost[torch.arange(len(kps), device=DEV), labs].double().cpu().numpy()
    disp = oracle.kp_labels(16, 2).astype(np.float64)[labs.cpu().numpy()]
    E = float(np.sum(data))
    for k in range(len(kps)):
        if parent[k] >= 0:
            w = oracle.kp_edge_weight(x.astype(np.float32).astype(np.float64), inten, k, parent[k])
            E += alpha / w * float(np.sum((disp[k] - disp[parent[k]]) ** 2))
    spread = float((mins.max() - mins.min()) / abs(E))
    err = abs(float(np.median(mins)) - E) / abs(E)
    say(f"  {len(kps)} keypoints: min energy {E:.6f}; min-marginal spread {spread:.2e}, vs labeling {err:.2e}")
    assert len(kps) == 3500
    assert spread < 1e-5 and err < 1e-5
