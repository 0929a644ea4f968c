"""Comparison of device results with the FP64 oracle, shared by the GPU tests.

A node or voxel field passes when
  * element by element, |got - ref| <= elem_tol * max|ref| + allow, and
  * the part of the error beyond the allowance, e = max(|got - ref| - allow, 0), has
    ||e|| / ||ref|| <= tol (relative L2),
where allow is the oracle's sample-cell tie allowance (zero where no voxel's warped
point lies within single-precision rounding of a cell face; see ``oracle.ngf_ties``).
The element-wise bound catches errors confined to a few nodes (a brick face, a ragged
edge) that a whole-field norm would average away.  Every check prints its figures and,
on failure, the worst element.
"""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def as64(a):
    if torch.is_tensor(a):
        a = a.detach().cpu().numpy()
    return np.asarray(a, np.float64)


def rel_l2(a, b):
    a = as64(a)
    b = as64(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def check_field(name, got, ref, allow=None, tol=1e-4, elem_tol=None):
    """Assert the field criteria above; returns the raw relative L2 error."""
    got = as64(got)
    ref = as64(ref)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    elem_tol = tol if elem_tol is None else elem_tol
    err = np.abs(got - ref)
    a = np.zeros_like(ref) if allow is None else as64(allow)
    nref = max(float(np.linalg.norm(ref)), 1e-300)
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    raw = float(np.linalg.norm(err)) / nref
    beyond = float(np.linalg.norm(np.maximum(err - a, 0.0))) / nref
    slack = err - (elem_tol * scale + a)
    worst = int(np.argmax(slack)) if slack.size else 0
    n_allow = int(np.count_nonzero(a))
    msg = (f"  {name}: rel-L2 {raw:.2e} (beyond allowance {beyond:.2e}, bound {tol:.0e}); "
           f"max elem err {float(err.max()) / max(scale, 1e-300) if err.size else 0.0:.2e} x max|ref|; "
           f"{n_allow} elements with allowance")
    say(msg)
    if slack.size and slack.flat[worst] > 0:
        idx = np.unravel_index(worst, ref.shape)
        raise AssertionError(f"{name}: element {idx}: got {got.flat[worst]!r} ref {ref.flat[worst]!r} "
                             f"allowance {a.flat[worst]!r} (bound {elem_tol:.0e} x max|ref| = {elem_tol * scale:.3e})")
    assert beyond <= tol, f"{name}: relative L2 error beyond the allowance {beyond:.3e} > {tol:.0e}"
    return raw


def say_ties(label, ties):
    say(f"  {label}: {ties['n']} voxels with a sample-cell tie")


def pcg_vector_rounding(hv, b, diag, iters):
    """The Jacobi-PCG iteration of the oracle (x0 = 0, M = diag + 1e-12 max diag, a fixed
    number of iterations) with every vector rounded to single precision after each update
    (dot products in double precision, products hv in double precision then rounded).
    It measures how far single-precision vector storage alone moves a fixed-iteration CG
    result from the double-precision one on a given system: the tolerance of a
    single-precision implementation's step is derived from it."""
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    M = f32(diag + 1e-12 * float(np.max(diag)))
    x = np.zeros_like(b)
    r = f32(b)
    z = f32(r / M)
    p = z.copy()
    rz = float(np.sum(r * z))
    for _ in range(iters):
        q = f32(hv(p))
        pq = float(np.sum(p * q))
        if not pq > 0.0:
            break
        a = np.float32(rz / pq)
        x = f32(x + a * p)
        r = f32(r - a * q)
        z = f32(r / M)
        rz_new = float(np.sum(r * z))
        p = f32(z + np.float32(rz_new / rz) * p)
        rz = rz_new
    return x
