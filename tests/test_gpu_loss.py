"""Differentiable loss form: NGFLoss forward/backward through the C ABI.

dL/du comes from the gradient passes (D, S, Vhat); dL/dT from ngf_grad_T (the adjoint of
the warped trilinear sampling and of the central-difference stencil).  Checked against
the FP64 oracle: the full fields (oracle.ngf_grad_T is pinned by finite differences in
the CPU tests), and central finite differences of the oracle objective at 64 random
coordinates in u (h = 1e-3 mm, at the coordinates where no sample-cell face is
crossed) and in T (h = 1e-3 HU) on a 192 x 192 x 160 pair at 1 mm.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.fields import check_field, rel_l2, say, say_ties

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ETA, ALPHA, GAMMA = 10.0, 1.0, 0.1


@pytest.fixture(scope="module")
def mods():
    from paper_1807_00467_amd import disco as d
    from paper_1807_00467_amd import loss as l
    return d, l


def oracle_loss_grads(d, u, T=None):
    """Oracle value and gradients of D + alpha S + gamma Vhat at u (FP64), and the tie
    allowance of dL/du."""
    T = d["T"] if T is None else T
    P = oracle.Problem(d["R"], T, d["spacing"], None, None,
                       oracle.Weights(eta=ETA, alpha=ALPHA, gamma=GAMMA))
    ob = P.objective(u)
    gD = P.ngf(u, want=("g",))["g"]
    H = P.H
    gS = oracle.curvature(u, H)["g"]
    gV = oracle.vcc(u, H)["g"]
    gT = oracle.ngf_grad_T(P.gR, P.gT, d["spacing"], ETA, u)
    ties = oracle.ngf_ties(P.gR, P.gT, d["spacing"], ETA, u)
    return ob["J"], gD + ALPHA * gS + GAMMA * gV, gT, ties


@pytest.mark.parametrize("shape,spacing,seed", [((32, 24, 20), (1.5, 1.5, 2.0), 31),
                                                ((76, 36, 28), (1.2, 1.4, 2.2), 32)])
@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_ngf_grad_T_matches_oracle(mods, shape, spacing, seed, storage):
    disco, _ = mods
    say(f"[grad_T] shape={shape} storage={storage}")
    d = synth.small_pair(shape=shape, spacing=spacing, seed=seed, n_tubes=8, n_kp=10, field_max=4.0)
    ctx = disco.Disco(d["shape"], d["spacing"], storage=storage, device=DEV)
    ctx.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV))
    dT = ctx.ngf_grad_T(torch.from_numpy(d["u_true"]).to(DEV), ETA).cpu().numpy()
    gR = oracle.image_gradient(d["R"], d["spacing"])
    gT = oracle.image_gradient(d["T"], d["spacing"])
    ref = oracle.ngf_grad_T(gR, gT, d["spacing"], ETA, d["u_true"].astype(np.float64))
    # the sample weights are continuous across cell faces: no tie allowance is needed
    check_field("dD/dT", dT, ref, None, 1e-4 if storage == "fp32" else 2e-2)


@pytest.mark.parametrize("amp", [0.3, 12.0])
def test_ngf_grad_T_field_strength(mods, amp):
    """dD/dT under node displacements drawn uniformly in +-amp voxels.  With amp = 0.3 the
    sample corners of a 16 x 4 x 8 voxel tile fit the kernel's LDS box (at most 18 x 6 x 10
    of its 1600 points) and are added there in fixed point; with amp = 12 the box of most
    tiles spans tens of voxels in every axis (far over 1600 points) and the voxels add their
    corners to the field directly."""
    disco, _ = mods
    say(f"[grad_T] random node field +-{amp} voxels")
    shape, spacing = (76, 36, 28), (1.2, 1.4, 2.2)
    d = synth.small_pair(shape=shape, spacing=spacing, seed=33, n_tubes=8, n_kp=10, field_max=4.0)
    rng = np.random.default_rng(3300 + int(amp))
    u = (rng.uniform(-amp, amp, size=d["u_true"].shape)
         * np.asarray(spacing, np.float64)[:, None, None, None]).astype(np.float32)
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    ctx.set_images(torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV))
    dT = ctx.ngf_grad_T(torch.from_numpy(u).to(DEV), ETA).cpu().numpy()
    gR = oracle.image_gradient(d["R"], d["spacing"])
    gT = oracle.image_gradient(d["T"], d["spacing"])
    ref = oracle.ngf_grad_T(gR, gT, d["spacing"], ETA, u.astype(np.float64))
    check_field("dD/dT", dT, ref, None, 1e-4)


def test_ngf_loss_matches_oracle_small(mods):
    disco, loss = mods
    say("[NGFLoss small]")
    d = synth.small_pair(shape=(32, 24, 20), spacing=(1.5, 1.5, 2.0), seed=33, n_tubes=8, n_kp=10, field_max=4.0)
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    R = torch.from_numpy(d["R"]).to(DEV)
    u = torch.from_numpy(d["u_true"]).to(DEV).requires_grad_(True)
    T = torch.from_numpy(d["T"]).to(DEV).requires_grad_(True)
    L = loss.ngf_loss(ctx, u, T, R, ETA, ALPHA, GAMMA)
    L.backward()
    J, gu, gT, ties = oracle_loss_grads(d, d["u_true"].astype(np.float64))
    say_ties("u_true", ties)
    eL = abs(L.item() - J) / abs(J)
    say(f"  loss rel {eL:.2e}")
    assert eL < 1e-5
    check_field("dL/du", u.grad, gu, ties["g"], 1e-4)
    check_field("dL/dT", T.grad, gT, None, 1e-4)


def test_ngf_loss_two_forwards_before_backward(mods):
    """Two forward passes with different moving images on one context, then backward on
    the first: its gradients must be those of the first pair (the context's volumes are
    rebuilt from the saved images), and then those of the second."""
    disco, loss = mods
    say("[NGFLoss two forwards, one context]")
    d = synth.small_pair(shape=(32, 24, 20), spacing=(1.5, 1.5, 2.0), seed=35, n_tubes=8, n_kp=10, field_max=4.0)
    d2 = synth.small_pair(shape=(32, 24, 20), spacing=(1.5, 1.5, 2.0), seed=36, n_tubes=8, n_kp=10, field_max=4.0)
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    R = torch.from_numpy(d["R"]).to(DEV)
    u1 = torch.from_numpy(d["u_true"]).to(DEV).requires_grad_(True)
    u2 = (torch.from_numpy(d["u_true"]).to(DEV) * 0.5).requires_grad_(True)
    T1 = torch.from_numpy(d["T"]).to(DEV).requires_grad_(True)
    T2 = torch.from_numpy(d2["T"]).to(DEV).requires_grad_(True)
    L1 = loss.ngf_loss(ctx, u1, T1, R, ETA, ALPHA, GAMMA)
    L2 = loss.ngf_loss(ctx, u2, T2, R, ETA, ALPHA, GAMMA)
    L1.backward()
    L2.backward()
    for name, u, T, L, Tn in (("first", u1, T1, L1, d["T"]), ("second", u2, T2, L2, d2["T"])):
        uu = u.detach().cpu().numpy().astype(np.float64)
        J, gu, gT, ties = oracle_loss_grads(d, uu, Tn)
        say(f"  {name}: loss rel {abs(L.item() - J) / abs(J):.2e}")
        assert abs(L.item() - J) <= 1e-5 * abs(J)
        check_field(f"dL/du ({name})", u.grad, gu, ties["g"], 1e-4)
        check_field(f"dL/dT ({name})", T.grad, gT, None, 1e-4)
    # a moving image modified in place after the forward pass is refused by autograd
    T3 = torch.from_numpy(d["T"]).to(DEV).requires_grad_(True)
    T3c = T3.detach().clone().requires_grad_(True)
    L3 = loss.ngf_loss(ctx, u1.detach(), T3c, R, ETA, ALPHA, GAMMA)
    with torch.no_grad():
        T3c.add_(1.0)
    with pytest.raises(RuntimeError):
        L3.backward()


def test_ngf_loss_no_grad_paths(mods):
    """Only the inputs that need a gradient get one; the loss is a plain float64 scalar."""
    disco, loss = mods
    d = synth.small_pair(shape=(16, 16, 12), spacing=(1.5, 1.5, 1.5), seed=34)
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    R = torch.from_numpy(d["R"]).to(DEV)
    u = torch.from_numpy(d["u_true"]).to(DEV).requires_grad_(True)
    T = torch.from_numpy(d["T"]).to(DEV)
    L = loss.ngf_loss(ctx, u, T, R, ETA, ALPHA, GAMMA)
    assert L.dim() == 0 and L.dtype == torch.float64
    (gu,) = torch.autograd.grad(L, (u,))
    assert gu.shape == u.shape and bool(torch.isfinite(gu).all())


@pytest.fixture(scope="module")
def cfg2(mods):
    say("[NGFLoss 192x192x160] generating ...")
    return synth.make_pair("cfg2")


def test_ngf_loss_fd_u_cfg2(mods, cfg2):
    disco, loss = mods
    d = cfg2
    say("[NGFLoss 192x192x160] dL/du: full field and 64 FD coordinates")
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    R = torch.from_numpy(d["R"]).to(DEV)
    u = torch.from_numpy(d["u_true"]).to(DEV).requires_grad_(True)
    T = torch.from_numpy(d["T"]).to(DEV)
    L = loss.ngf_loss(ctx, u, T, R, ETA, ALPHA, GAMMA)
    (gu,) = torch.autograd.grad(L, (u,))
    gu = gu.cpu().numpy().astype(np.float64)
    u0 = d["u_true"].astype(np.float64)
    J, gref, _, ties = oracle_loss_grads(d, u0)
    say_ties("u_true", ties)
    check_field("dL/du", gu, gref, ties["g"], 1e-4)
    P = oracle.Problem(d["R"], d["T"], d["spacing"], None, None, oracle.Weights(eta=ETA, alpha=ALPHA, gamma=GAMMA))
    rng = np.random.default_rng(2001)
    flat = np.flatnonzero(np.abs(gref).ravel() > np.median(np.abs(gref)))
    picks = rng.choice(flat, size=64, replace=False)

    def fd_at(p, h):
        up = u0.copy().ravel()
        um = u0.copy().ravel()
        up[p] += h
        um[p] -= h
        return (P.objective(up.reshape(u0.shape))["J"] - P.objective(um.reshape(u0.shape))["J"]) / (2 * h)

    fd3 = np.array([fd_at(p, 1e-3) for p in picks])
    fd4 = np.array([fd_at(p, 1e-4) for p in picks])
    # The trilinear sample of grad T is only continuous across the faces of its sample
    # cells, so D has kinks in u.  A coordinate is smooth on the stencil when the two
    # step sizes agree (a central difference of a smooth function changes by O(h^2));
    # a step that straddles a face changes it by O(h).  Only smooth coordinates are
    # compared, and they must be the large majority.
    smooth = np.abs(fd3 - fd4) <= 1e-5 * np.abs(fd4) + 1e-6
    e_fd = rel_l2(gu.ravel()[picks][smooth], fd3[smooth])
    e_orc = rel_l2(gref.ravel()[picks][smooth], fd3[smooth])
    say(f"  loss rel {abs(L.item() - J) / abs(J):.2e}  FD h=1e-3 on {int(smooth.sum())}/64 "
        f"smooth coordinates: gpu {e_fd:.2e} oracle {e_orc:.2e}")
    assert abs(L.item() - J) / abs(J) < 1e-5
    assert smooth.sum() >= 48
    assert e_fd < 1e-4 and e_orc < 1e-5


def test_ngf_loss_fd_T_cfg2(mods, cfg2):
    disco, loss = mods
    d = cfg2
    say("[NGFLoss 192x192x160] dL/dT: full field and 64 FD coordinates")
    ctx = disco.Disco(d["shape"], d["spacing"], device=DEV)
    R = torch.from_numpy(d["R"]).to(DEV)
    u = torch.from_numpy(d["u_true"]).to(DEV)
    T = torch.from_numpy(d["T"]).to(DEV).requires_grad_(True)
    L = loss.ngf_loss(ctx, u, T, R, ETA, ALPHA, GAMMA)
    (gT,) = torch.autograd.grad(L, (T,))
    gT = gT.cpu().numpy().astype(np.float64)
    u0 = d["u_true"].astype(np.float64)
    gR = oracle.image_gradient(d["R"], d["spacing"])
    ref = oracle.ngf_grad_T(gR, oracle.image_gradient(d["T"], d["spacing"]), d["spacing"], ETA, u0)
    check_field("dL/dT", gT, ref, None, 1e-4)
    rng = np.random.default_rng(2002)
    flat = np.flatnonzero(np.abs(ref).ravel() > np.median(np.abs(ref)))
    picks = rng.choice(flat, size=64, replace=False)
    h = 1e-3
    h3 = float(np.prod(d["spacing"]))
    gT0 = oracle.image_gradient(d["T"], d["spacing"])
    fd = np.empty(64)
    for n, p in enumerate(picks):
        # grad T is linear in T: perturbing T at voxel p by +-h moves it by +-h times the
        # stencil's response to a unit impulse at p (exact in the oracle's float input)
        e = np.zeros(d["T"].size, np.float32)
        e[p] = 1.0
        G1 = oracle.image_gradient(e.reshape(d["T"].shape), d["spacing"])
        # D is a sum of per-voxel terms: differencing the term arrays cancels every voxel
        # the perturbation does not reach exactly
        cp = oracle.ngf(gR, gT0 + h * G1, d["spacing"], ETA, u0, want=("c",))["c"]
        cm = oracle.ngf(gR, gT0 - h * G1, d["spacing"], ETA, u0, want=("c",))["c"]
        fd[n] = h3 * float(np.sum(cp - cm)) / (2 * h)
    e_fd = rel_l2(gT.ravel()[picks], fd)
    e_orc = rel_l2(ref.ravel()[picks], fd)
    say(f"  FD: gpu {e_fd:.2e} oracle {e_orc:.2e}")
    assert e_fd < 1e-4 and e_orc < 1e-5


def test_ngf_loss_module_batch_of_pairs(mods):
    """NGFLoss over a batch equals the sum of the single-pair losses, and so do the gradients."""
    disco, loss = mods
    say("[NGFLoss batch]")
    pairs = [synth.small_pair(shape=(32, 24, 20), spacing=(1.5, 1.5, 2.0), seed=40 + b, n_tubes=8, n_kp=10,
                              field_max=4.0) for b in range(3)]
    shape, spacing = pairs[0]["shape"], pairs[0]["spacing"]
    Rs = [torch.from_numpy(p["R"]).to(DEV) for p in pairs]
    mod = loss.NGFLoss(shape, spacing, Rs, eta=ETA, alpha=ALPHA, gamma=GAMMA)
    u = torch.stack([torch.from_numpy(p["u_true"]) for p in pairs]).to(DEV).requires_grad_(True)
    T = torch.stack([torch.from_numpy(p["T"]) for p in pairs]).to(DEV).requires_grad_(True)
    L = mod(u, T)
    L.backward()
    Js = 0.0
    for b, p in enumerate(pairs):
        J, gu, gT, ties = oracle_loss_grads(p, p["u_true"].astype(np.float64))
        Js += J
        check_field(f"dL/du pair {b}", u.grad[b], gu, ties["g"], 1e-4)
        check_field(f"dL/dT pair {b}", T.grad[b], gT, None, 1e-4)
    assert abs(L.item() - Js) / abs(Js) < 1e-5


@pytest.mark.parametrize("batched", [False, True])
def test_ngf_loss_upstream_gradient(mods, batched):
    """A non-unit upstream gradient (L scaled by -2.5 before backward): dL/du and dL/dT are
    the oracle's times -2.5 (dL/dT takes the factor inside its stencil pass)."""
    disco, loss = mods
    say(f"[NGFLoss upstream gradient, batched={batched}]")
    k = -2.5
    pairs = [synth.small_pair(shape=(32, 24, 20), spacing=(1.5, 1.5, 2.0), seed=50 + b, n_tubes=8, n_kp=10,
                              field_max=4.0) for b in range(2 if batched else 1)]
    shape, spacing = pairs[0]["shape"], pairs[0]["spacing"]
    Rs = [torch.from_numpy(p["R"]).to(DEV) for p in pairs]
    u = torch.stack([torch.from_numpy(p["u_true"]) for p in pairs]).to(DEV).requires_grad_(True)
    T = torch.stack([torch.from_numpy(p["T"]) for p in pairs]).to(DEV).requires_grad_(True)
    if batched:
        L = loss.NGFLoss(shape, spacing, Rs, eta=ETA, alpha=ALPHA, gamma=GAMMA)(u, T)
    else:
        ctx = disco.Disco(shape, spacing, device=DEV)
        L = loss.ngf_loss(ctx, u[0], T[0], Rs[0], ETA, ALPHA, GAMMA)
    (k * L).backward()
    for b, p in enumerate(pairs):
        J, gu, gT, ties = oracle_loss_grads(p, p["u_true"].astype(np.float64))
        check_field(f"dL/du pair {b}", u.grad[b], k * gu, abs(k) * ties["g"], 1e-4)
        check_field(f"dL/dT pair {b}", T.grad[b], k * gT, None, 1e-4)
