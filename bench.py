"""Benchmark of the dense DIS-CO objective hot path on one MI355X.

One step = one pass of the whole path on the 512 x 512 x 128 (0.7 x 0.7 x 2.5 mm)
synthetic lung-CT pair: image gradients of R and T, then one Gauss-Newton step from
the true displacement (linearisation: objective, gradient, GN diagonal and the
per-voxel GN vectors; 20 Jacobi-PCG iterations, each one full GN product of eq. 11;
Armijo line search).  The step's inputs are resident in HBM before timing starts.

value = GN products per second over the timed steps (20 per step).  The roofline
entry is for the dominant kernel, the voxel-brick GN-product pass, timed with HIP
events on its launch stream during the timed steps.  The CPU baseline times the FP64
oracle on a bounded sample of the same workload (GN products at full size).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--storage fp32|fp16] [--calib-copy-mib M]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GN Hv products/s + Gvoxel/s at 512²×128; achieved HBM GB/s vs 8 TB/s peak"
HBM_PEAK_GBS = 8000.0
PCG_ITERS = 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_1807_00467_amd/csrc/kernels.hpp", "paper_1807_00467_amd/csrc/disco.hip",
                  "paper_1807_00467_amd/csrc/solver.hpp", "paper_1807_00467_amd/csrc/adjoint.hpp",
                  "paper_1807_00467_amd/csrc/batch.hpp", "paper_1807_00467_amd/csrc/keypoint.hpp",
                  "paper_1807_00467_amd/csrc/pyramid.hpp", "paper_1807_00467_amd/build.py"]


def kernel_source_hash():
    """sha256 over the sources the measured kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this kernel
    and workload; None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "counters_" + kernel_tag + ".md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    """Host cores available to this process and the CPU model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(d, params, budget_s=12.0):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload, with the
    thread count it is given (OMP_NUM_THREADS): the objective and the linearisation
    (objective + gradient + GN diagonal + s vectors) once each, then as many full-size
    GN products as fit in the budget (at least one); then one GN product on one thread."""
    import numpy as np
    import oracle
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"],
                       oracle.Weights(eta=params.eta, alpha=params.alpha, gamma=params.gamma, delta=params.delta))
    u = d["u_true"].astype(np.float64)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    P.objective(u)
    t_obj = time.perf_counter() - t0
    t0 = time.perf_counter()
    P.linearise(u)
    t_lin = time.perf_counter() - t0
    v = d["v"].astype(np.float64)
    n = 0
    t0 = time.perf_counter()
    while True:
        P.gn_hv(v)
        n += 1
        el = time.perf_counter() - t0
        if el + el / n > budget_s or n >= 16:
            break
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        P.gn_hv(v)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    return dict(value=n / el, unit="Hv/s", cores=threads, kind="oracle",
                sample=f"{n} full GN products of eq. 11 at 512x512x128 (FP64 C oracle, {threads} threads) after "
                       f"one objective evaluation ({t_obj:.2f} s) and one linearisation ({t_lin:.2f} s); "
                       f"{el:.1f} s timed; then one GN product on one thread ({t1:.2f} s)",
                objective_s=t_obj, objective_gradient_s=t_lin,
                one_thread={"value": 1.0 / t1, "unit": "Hv/s", "cores": 1},
                **host_info())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; 10 L-BFGS iterations with --lbfgs, the workload its "
                         "figures are quoted on)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cfg1")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ls", default="host", choices=["host", "device"],
                    help="Armijo line search decided on the host (stops at the accepted trial) or on "
                         "the device (all ls_max trials enqueued, later ones exit at once)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="batched form instead: 24 uneven pyramid-shape pairs, 5 GN iterations (15 PCG each), "
                         "one launch per phase and one graph, against the same steps pair by pair")
    ap.add_argument("--loss", action="store_true",
                    help="differentiable loss instead: NGFLoss forward + backward on 8 pairs of 192x192x160")
    ap.add_argument("--boundary", action="store_true",
                    help="add the lung-boundary term (eq. 6) with the adaptive beta (D = 100 beta B at u = 0)")
    ap.add_argument("--lbfgs", action="store_true",
                    help="L-BFGS iterations (m = 5, H0 = alpha C_H L^T L + tau I) on the same workload instead")
    ap.add_argument("--tau", type=float, default=10.0, help="tau of the L-BFGS initial Hessian")
    ap.add_argument("--ls-max", type=int, default=30,
                    help="Armijo trials at most per L-BFGS iteration (t >= 2^(1-n)); next to a fold the accepted "
                         "t falls below 2^-9, so 10 trials end the run there")
    ap.add_argument("--keypoints", action="store_true",
                    help="keypoint stage instead: NGF matching cost of 3500 keypoints over 33^3 displacements "
                         "(1 mm images) and its regularisation by belief propagation on the keypoint MST")
    ap.add_argument("--multilevel", action="store_true",
                    help="whole coarse-to-fine registrations (4-level pyramid) instead")
    ap.add_argument("--optimizer", default="lbfgs", choices=["lbfgs", "gn"],
                    help="optimiser of --multilevel")
    ap.add_argument("--iters", default="40,20,10,5", help="--multilevel iterations per level, coarsest first")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 10 if args.lbfgs else 20
    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_1807_00467_amd import disco

    if args.loss:
        return bench_loss(args)
    if args.batched:
        return bench_batched(args)
    if args.lbfgs:
        return bench_lbfgs(args)
    if args.multilevel:
        return bench_multilevel(args)
    if args.keypoints:
        return bench_keypoints(args)

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst

    log(f"[bench] generating {args.config} ...")
    t0 = time.perf_counter()
    d = synth.make_pair(args.config)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s; shape {d['shape']} spacing {d['spacing']}")
    dev = torch.device("cuda:0")
    R = torch.from_numpy(d["R"]).to(dev)
    T = torch.from_numpy(d["T"]).to(dev)
    u_true = torch.from_numpy(d["u_true"]).to(dev)
    ctx = disco.Disco(d["shape"], d["spacing"], storage=args.storage, device=dev)
    ctx.set_images(R, T)
    ctx.set_keypoints(d["kp_x"], d["kp_t"])
    zero = torch.zeros_like(u_true)
    # adaptive keypoint weight: D = delta K at the start (u = 0)
    D0 = ctx.ngf_eval(zero, 10.0).item()
    K0 = ctx.keypoint_penalty(1.0, zero, grad=False, diag=False)["K"].item()
    params = disco.Params(eta=10.0, alpha=1.0, gamma=0.1, delta=D0 / K0 if K0 > 0 else 0.0,
                          pcg_iters=PCG_ITERS, pcg_tol=0.0, ls_max=10,
                          flags=disco.FLAG_LS_DEVICE if args.ls == "device" else 0)
    log(f"[bench] delta = {params.delta:.4g}")
    if args.boundary:
        ctx.set_masks(torch.from_numpy(d["mask_R"]).to(dev), torch.from_numpy(d["mask_T"]).to(dev))
        B0 = ctx.objective_linearise(disco.Params(eta=10.0, alpha=0.0, gamma=0.0, delta=0.0, beta=1.0), zero,
                                     grad=False, diag=False)["B"]
        params.beta = D0 / (100.0 * B0) if B0 > 0 else 0.0
        log(f"[bench] beta = {params.beta:.4g}")
    u = torch.empty_like(u_true)
    rep = torch.zeros(disco.REP_SIZE, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)

    def step():
        u.copy_(u_true)
        ctx.set_images(R, T)
        ctx.gn_pcg_step(params, u, rep, st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    n_hv, ms_hv = ctx.profile_read(disco.PROF_HV)
    n_gr, ms_gr = ctx.profile_read(disco.PROF_GRAD)
    n_ev, ms_ev = ctx.profile_read(disco.PROF_EVAL)
    n_ig, ms_ig = ctx.profile_read(disco.PROF_IMGRAD)
    r = disco.Disco.report_dict(rep)
    log(f"[bench] last step report: {r}; status {int(st.item())}")

    nvox = int(np.prod(d["shape"]))
    nx, ny, nz = ctx.nodes
    nnodes = nx * ny * nz
    bpv = 12 if args.storage == "fp32" else 8
    hv_bytes = bpv * nvox + 36 * nnodes           # s stream + v, u (VCC) read + Hv write
    hv_s = ms_hv / max(n_hv, 1) / 1e3
    achieved = hv_bytes / hv_s / 1e9
    hv_total = PCG_ITERS * args.steps
    value = hv_total / elapsed
    kernel_tag = f"brick_hv_{d['shape'][0]}x{d['shape'][1]}x{d['shape'][2]}_{args.storage}"
    if args.boundary:
        kernel_tag += "_boundary"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Hv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "f16-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: R,T {d['shape'][0]}x{d['shape'][1]}x{d['shape'][2]} at "
                        f"{d['spacing'][0]}x{d['spacing'][1]}x{d['spacing'][2]} mm, node grid {nx}x{ny}x{nz}, "
                        f"{len(d['kp_x'])} keypoints; step = image gradients + GN step "
                        f"(linearise + {PCG_ITERS} PCG GN products + Armijo)"
                        + ("; with the lung-boundary term" if args.boundary else ""),
            "eta": params.eta, "alpha": params.alpha, "gamma": params.gamma, "delta": params.delta,
            "beta": params.beta, "storage": args.storage, "line_search": args.ls,
        },
        "gvoxel_per_s_hv_kernel": nvox / hv_s / 1e9,
        "hv_kernel_us": hv_s * 1e6,
        "grad_kernel_us": 1e3 * ms_gr / max(n_gr, 1),
        "eval_kernel_us": 1e3 * ms_ev / max(n_ev, 1),
        "imgrad_kernel_us": 1e3 * ms_ig / max(n_ig, 1),
        "launches": {"hv": n_hv, "grad": n_gr, "eval": n_ev, "imgrad": n_ig},
        "roofline": {
            "kernel": "k_brick<HV> (NGF + VCC + keypoint GN product pass)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_from_profiles(kernel_tag),
            "algorithmic_bytes_per_launch": hv_bytes,
        },
        "cpu_baseline": None,
    }
    if args.storage == "fp16":
        # the same steps with FP32 storage on the same GPU: the speedup of the storage form
        log("[bench] the same steps with FP32 storage ...")
        ctx32 = disco.Disco(d["shape"], d["spacing"], storage="fp32", device=dev)
        ctx32.set_keypoints(d["kp_x"], d["kp_t"])
        rep32 = torch.zeros_like(rep)

        def step32():
            u.copy_(u_true)
            ctx32.set_images(R, T)
            ctx32.gn_pcg_step(params, u, rep32, st)

        for _ in range(args.warmup):
            step32()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step32()
        torch.cuda.synchronize()
        ms32 = 1e3 * (time.perf_counter() - t0) / args.steps
        r32 = disco.Disco.report_dict(rep32)
        out["fp32_storage_ms_per_step"] = ms32
        out["speedup_vs_fp32_storage"] = ms32 / out["ms_per_step"]
        out["J_new_rel_diff_vs_fp32_storage"] = abs(r["J_new"] - r32["J_new"]) / abs(r32["J_new"])
        ctx32.close()
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(d, params)
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_lbfgs(args):
    """L-BFGS on the full-size workload: the first K iterations of a run from u = 0
    (timed after W untimed runs of the same iterations; the history is reset before each
    run).  One iteration = J and grad J at u, two-loop recursion over the stored pairs
    (full from the sixth iteration on), H0 solve (Jacobi-PCG, 30 iterations at most,
    relative residual 1e-6), Armijo trials."""
    import numpy as np
    import torch
    import synth
    from paper_1807_00467_amd import disco

    log(f"[bench] generating {args.config} ...")
    d = synth.make_pair(args.config)
    dev = torch.device("cuda:0")
    ctx = disco.Disco(d["shape"], d["spacing"], storage=args.storage, device=dev)
    ctx.set_images(torch.from_numpy(d["R"]).to(dev), torch.from_numpy(d["T"]).to(dev))
    ctx.set_keypoints(d["kp_x"], d["kp_t"])
    zero = torch.zeros((3,) + tuple(ctx.nodes[::-1]), device=dev)
    D0 = ctx.ngf_eval(zero, 10.0).item()
    K0 = ctx.keypoint_penalty(1.0, zero, grad=False, diag=False)["K"].item()
    params = disco.Params(eta=10.0, alpha=1.0, gamma=0.1, delta=D0 / K0 if K0 > 0 else 0.0, ls_max=args.ls_max,
                          flags=disco.FLAG_LS_DEVICE)
    lb = disco.Lbfgs(m=5, tau=args.tau, h0_iters=30, h0_tol=1e-6)
    u = zero.clone()
    rep = torch.zeros(disco.REP_SIZE, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        ctx.lbfgs_reset()
        u.zero_()
        for _ in range(args.steps):
            ctx.lbfgs_step(params, lb, u, rep, st)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    ctx.lbfgs_reset()
    u.zero_()
    reps = []
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.lbfgs_step(params, lb, u, rep, st)
        reps.append(rep.clone())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    n_gr, ms_gr = ctx.profile_read(disco.PROF_GRAD)
    n_ev, ms_ev = ctx.profile_read(disco.PROF_EVAL)
    rs = [disco.Disco.report_dict(r) for r in reps]
    trials = sum(int(r["ls_trials"]) for r in rs)
    h0 = [int(r["pcg_iters"]) for r in rs]
    for k, r in enumerate(rs):
        log(f"[bench]   it {k}: J {r['J']:.6e} |g| {r['gnorm']:.3e} g.p {r['gtp']:.3e} t {r['t']} "
            f"trials {int(r['ls_trials'])} J_new {r['J_new']:.6e} V_new {r['V_new']:.3e}")
    log(f"[bench] J {rs[0]['J']:.6e} -> {rs[-1]['J_new']:.6e}; trials {trials}; H0 CG iterations {h0}; "
        f"status {int(st.item())}")
    nx, ny, nz = ctx.nodes
    out = {
        "metric": "L-BFGS iterations/s",
        "value": args.steps / elapsed,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "f16-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: R,T {d['shape'][0]}x{d['shape'][1]}x{d['shape'][2]}, node grid "
                        f"{nx}x{ny}x{nz}; step = one L-BFGS iteration (m 5, H0 tau {args.tau:g}, <= 30 H0 CG "
                        f"iterations, Armijo on the device, {args.ls_max} trials at most); the first {args.steps} "
                        f"iterations from u = 0",
            "storage": args.storage,
        },
        "grad_kernel_us": 1e3 * ms_gr / max(n_gr, 1),
        "eval_kernel_us": 1e3 * ms_ev / max(n_ev, 1),
        "ls_trials_per_iter": trials / args.steps,
        "h0_cg_iters": h0,
        "J_first": rs[0]["J"],
        "J_last": rs[-1]["J_new"],
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def tree_depths(parent, root):
    """Hop distance of every node from root in the tree given by a parent array."""
    import numpy as np
    n = len(parent)
    adj = [[] for _ in range(n)]
    for k, p in enumerate(parent):
        if p >= 0:
            adj[k].append(int(p))
            adj[int(p)].append(k)
    dep = np.full(n, -1, int)
    dep[root] = 0
    queue = [root]
    for a in queue:
        for b in adj[a]:
            if dep[b] < 0:
                dep[b] = dep[a] + 1
                queue.append(b)
    return dep


def _make_pair_seeded(a):
    import synth
    cfg, seed = a
    return synth.make_pair(cfg, seed=seed)


def make_pairs(cfg, seeds):
    """Synthetic pairs generated in worker processes (before anything touches the GPU)."""
    import multiprocessing as mp
    nproc = max(1, min(len(seeds), len(os.sched_getaffinity(0)), 16))
    with mp.get_context("fork").Pool(nproc) as pool:
        return pool.map(_make_pair_seeded, [(cfg, s) for s in seeds])


def cpu_baseline_loss(d, eta, alpha, gamma, budget_s=20.0):
    """The FP64 oracle's loss forward and backward for one pair: J (eq. 11 without the
    keypoint term), dJ/du and dD/dT, timed on one pair of the same workload."""
    import numpy as np
    import oracle
    P = oracle.Problem(d["R"], d["T"], d["spacing"], None, None,
                       oracle.Weights(eta=eta, alpha=alpha, gamma=gamma, delta=0.0))
    u = d["u_true"].astype(np.float64)
    n = 0
    t0 = time.perf_counter()
    while True:
        P.objective(u)
        P.linearise(u)
        oracle.ngf_grad_T(P.gR, P.gT, d["spacing"], eta, u)
        n += 1
        el = time.perf_counter() - t0
        if el + el / n > budget_s or n >= 8:
            break
    return dict(value=n / el, unit="pairs/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{n} forward + backward passes of one {d['shape'][0]}x{d['shape'][1]}x{d['shape'][2]} "
                       f"pair (FP64 C oracle: objective, gradient in u, derivative in T); {el:.1f} s",
                **host_info())


def bench_loss(args):
    """Differentiable loss (NGFLoss, a torch.autograd.Function per pair) on 8 pairs of
    192 x 192 x 160 at 1 mm (node grid 49 x 49 x 41): one step = the forward pass (sum
    over the pairs of D + alpha S + gamma Vhat, eq. 11 without the keypoint and
    lung-boundary terms) and the backward pass (dL/du and dL/dT of every pair).  Each
    pair keeps its gradient volumes resident: they are built at the first forward pass,
    before timing (the images do not change between steps, as when a network is trained
    on a fixed set of pairs)."""
    import numpy as np
    import torch
    from paper_1807_00467_amd import disco
    from paper_1807_00467_amd.loss import NGFLoss

    npairs = 8
    eta, alpha, gamma = 10.0, 1.0, 0.1
    log(f"[bench] generating {npairs} cfg2 pairs ...")
    t0 = time.perf_counter()
    pairs = make_pairs("cfg2", [2000 + i for i in range(npairs)])
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s")
    d0 = pairs[0]
    dev = torch.device("cuda:0")
    R = [torch.from_numpy(p["R"]).to(dev) for p in pairs]
    T = torch.stack([torch.from_numpy(p["T"]) for p in pairs]).to(dev).requires_grad_(True)
    u = torch.stack([torch.from_numpy(p["u_true"]) for p in pairs]).to(dev).requires_grad_(True)
    crit = NGFLoss(d0["shape"], d0["spacing"], R, eta=eta, alpha=alpha, gamma=gamma, storage=args.storage)

    def step():
        u.grad = None
        T.grad = None
        loss = crit(u, T)
        loss.backward()
        return loss

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    for c in crit.ctxs:
        c.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for c in crit.ctxs:
        c.profile(False)
    kinds = {"grad": disco.PROF_GRAD, "eval": disco.PROF_EVAL, "adjT": disco.PROF_ADJT}
    prof = {}
    for name, k in kinds.items():
        n_tot, ms_tot = 0, 0.0
        for c in crit.ctxs:
            n, ms = c.profile_read(k)
            n_tot += n
            ms_tot += ms
        prof[name] = (n_tot, ms_tot)
    nvox = int(np.prod(d0["shape"]))
    nx, ny, nz = crit.ctxs[0].nodes
    nnodes = nx * ny * nz
    bpv = 12 if args.storage == "fp32" else 8
    # algorithmic bytes per launch: objective pass (grad R and the sample of grad T per
    # voxel, u per node); gradient pass (the same plus the s cache written; u read, g and
    # diag written per node); derivative in T (clear of the 3-vector field, grad R and the
    # sample of grad T read, the field scattered (read and written), the stencil pass
    # reading it and writing dT; u per node)
    bytes_per = {"eval": 2 * bpv * nvox + 12 * nnodes, "grad": 3 * bpv * nvox + 36 * nnodes,
                 "adjT": (12 + 2 * bpv + 24 + 12 + 4) * nvox + 12 * nnodes}
    names = {"eval": "k_brick<EVAL> (objective pass, forward)", "grad": "k_brick<GRAD> (gradient pass, backward in u)",
             "adjT": "k_fill + k_adjT_scatter + k_adjT_stencil (backward in T)"}
    dom = max(prof, key=lambda k: prof[k][1])
    n_dom, ms_dom = prof[dom]
    t_dom = ms_dom / max(n_dom, 1) / 1e3
    achieved = bytes_per[dom] / t_dom / 1e9
    out = {
        "metric": "loss forward + backward pairs/s (8 pairs of 192x192x160)",
        "value": npairs * args.steps / elapsed,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "f16-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": f"cfg2: {npairs} pairs of {d0['shape'][0]}x{d0['shape'][1]}x{d0['shape'][2]} at 1 mm, "
                        f"node grid {nx}x{ny}x{nz}; step = NGFLoss forward (D + alpha S + gamma Vhat summed "
                        f"over the pairs) + backward (dL/du and dL/dT of every pair), gradient volumes resident",
            "eta": eta, "alpha": alpha, "gamma": gamma, "storage": args.storage,
        },
        "kernel_us": {k: 1e3 * v[1] / max(v[0], 1) for k, v in prof.items()},
        "launches": {k: v[0] for k, v in prof.items()},
        "loss": float(loss.item()),
        "roofline": {
            "kernel": names[dom],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": bytes_per[dom],
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on one pair ...")
        out["cpu_baseline"] = cpu_baseline_loss(d0, eta, alpha, gamma)
    print(json.dumps(out), flush=True)
    crit.close()


def bench_keypoints(args):
    """Keypoint stage at the paper's size: 3500 keypoints, 33^3 = 35937 displacements, 64
    patch voxels each (8.05e9 NGF terms); K cost evaluations timed with events on the
    launch stream after W untimed ones, then the regularisation (MST + belief propagation)."""
    import numpy as np
    import torch
    import synth
    from paper_1807_00467_amd import disco

    log("[bench] generating the 1 mm keypoint workload ...")
    d = synth.make_pair("kp")
    dev = torch.device("cuda:0")
    st = disco.KeypointStage(d["shape"], d["spacing"], device=dev)
    st.set_images(torch.from_numpy(d["R"]).to(dev), torch.from_numpy(d["T"]).to(dev), 12.0)
    kps = np.floor(np.asarray(d["kp_x"], np.float64) / np.asarray(d["spacing"])).astype(np.int32)
    kpt = torch.from_numpy(kps).to(dev)
    R = 16
    L = (2 * R + 1) ** 3
    for _ in range(args.warmup):
        cost = st.cost(kpt, R)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        cost = st.cost(kpt, R)
    e1.record()
    torch.cuda.synchronize()
    cost_s = e0.elapsed_time(e1) / 1e3 / args.steps
    x = (kps + 0.5) * np.asarray(d["spacing"])
    inten = d["R"][kps[:, 2], kps[:, 1], kps[:, 0]]
    st.regularise(x, inten, cost, R)  # warm (allocates the handle's work memory)
    torch.cuda.synchronize()
    reg = []
    for _ in range(3):
        t0 = time.perf_counter()
        marg, lab, par = st.regularise(x, inten, cost, R)
        torch.cuda.synchronize()
        reg.append(time.perf_counter() - t0)
    reg_s = float(np.median(reg))
    dep = tree_depths(par, 0)
    far = int(np.argmax(dep))
    diameter = int(tree_depths(par, far).max())
    terms = len(kps) * L * 64
    flops = 10.0 * terms  # per term: 4-component dot and r^2 accumulation, 5 fused multiply-adds
    achieved = flops / cost_s / 1e12
    peak = 157.3
    labs = lab.cpu().numpy()
    disp = 2 * (np.stack([labs % 33, (labs // 33) % 33, labs // 1089], 1) - R)
    out = {
        "metric": "keypoint NGF cost terms/s",
        "value": terms / cost_s,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * cost_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"keypoint stage: F, M {d['shape'][0]}x{d['shape'][1]}x{d['shape'][2]} at 1 mm, "
                        f"{len(kps)} keypoints in the lungs, {L} displacements (0, +-2, ..., +-32 mm), 64-voxel "
                        f"patches; step = one cost volume (eq. 2)",
        },
        "cost_ms": 1e3 * cost_s,
        "regularise_ms": 1e3 * reg_s,
        "tree_depth": int(dep.max()),
        "bp_levels": (diameter + 1) // 2,
        "roofline": {
            "kernel": "k_kp_cost (NGF matching cost, eq. 2)",
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "algorithmic_flops_per_launch": flops,
        },
        "median_abs_displacement_mm": float(np.median(np.abs(disp))),
    }
    print(json.dumps(out), flush=True)
    st.close()


def bench_multilevel(args):
    """Whole registrations of the full-size pair: pyramid build, coarse-to-fine optimisation
    on every level, prolongation; K registrations timed after W untimed ones."""
    import numpy as np
    import torch
    import synth
    from paper_1807_00467_amd import disco

    log(f"[bench] generating {args.config} ...")
    d = synth.make_pair(args.config)
    dev = torch.device("cuda:0")
    R = torch.from_numpy(d["R"]).to(dev)
    T = torch.from_numpy(d["T"]).to(dev)
    iters = tuple(int(x) for x in args.iters.split(","))
    prm = disco.Params(eta=10.0, alpha=1.0, gamma=0.1, delta=0.0, pcg_iters=PCG_ITERS, ls_max=10,
                       flags=disco.FLAG_LS_DEVICE)
    lb = disco.Lbfgs(m=5, tau=args.tau, h0_iters=30, h0_tol=1e-6)
    ml = disco.Multilevel(levels=4, optimizer=args.optimizer, iters=iters, adaptive_delta=True, storage=args.storage)
    plan = disco.pyramid_plan(d["shape"], d["spacing"], 4)
    log(f"[bench] pyramid: {[p[0] for p in plan]}")
    for _ in range(args.warmup):
        disco.multilevel_register(R, T, d["spacing"], d["kp_x"], d["kp_t"], prm, ml, lb)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, rep, L, delta = disco.multilevel_register(R, T, d["spacing"], d["kp_x"], d["kp_t"], prm, ml, lb)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    rep = rep.cpu().numpy()
    row, per_level = 0, []
    for k, n in enumerate(iters[:L]):
        r = rep[row:row + n]
        ran = r[~np.isnan(r[:, 0])]
        per_level.append(dict(shape=plan[L - 1 - k][0], iters_run=int(len(ran)),
                              J_first=float(ran[0, 0]) if len(ran) else None,
                              J_last=float(ran[-1, 10]) if len(ran) else None,
                              trials=int(ran[:, 15].sum()) if len(ran) else 0))
        row += n
    for lv in per_level:
        log(f"[bench]   level {lv}")
    # distance of the result to the generating field (mm, RMS over nodes inside the lungs is
    # not tracked here: all nodes)
    rms = float(torch.sqrt(torch.mean((u - torch.from_numpy(d["u_true"]).to(dev)) ** 2)).item())
    rms0 = float(torch.sqrt(torch.mean(torch.from_numpy(d["u_true"]) ** 2)).item())
    elapsed = sum(times)
    out = {
        "metric": "registrations/s",
        "value": args.steps / elapsed,
        "unit": "registrations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "f16-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: R,T {d['shape'][0]}x{d['shape'][1]}x{d['shape'][2]}, {L}-level pyramid "
                        f"{[p[0] for p in plan]}, {args.optimizer} iterations per level {list(iters[:L])} "
                        f"(coarsest first), adaptive delta; step = one whole registration from u = 0",
            "storage": args.storage,
        },
        "delta": delta,
        "levels": per_level,
        "rms_u_minus_u_true_mm": rms,
        "rms_u_true_mm": rms0,
    }
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """24 uneven pairs (pyramid shapes 64^2x32 ... 512^2x128 at a fixed field of view),
    5 GN iterations with 15 PCG products and a device line search (6 trials) each.
    Timed three ways on the same inputs: pair by pair (gn_pcg_step), batched eager (one
    launch per phase for all pairs) and one captured graph of all 5 iterations."""
    import numpy as np
    import torch
    import synth
    from paper_1807_00467_amd import autotune, disco

    dev = torch.device("cuda:0")
    iters, pcg, ls_max = 5, 15, 6
    cfgs = synth.batch_configs(24)
    t0 = time.perf_counter()
    pairs = []
    for i, c in enumerate(cfgs):
        pairs.append(synth.make_pair(c))
        log(f"[bench-batched] pair {i}: {c.shape} ({time.perf_counter() - t0:.1f} s)")
    log(f"[bench-batched] generated {len(pairs)} pairs in {time.perf_counter() - t0:.1f} s; "
        f"{sum(int(np.prod(p['shape'])) for p in pairs) / 1e6:.1f} M voxels")

    def contexts():
        cs = []
        for d in pairs:
            c = disco.Disco(d["shape"], d["spacing"], device=dev)
            c.set_images(torch.from_numpy(d["R"]).to(dev), torch.from_numpy(d["T"]).to(dev))
            c.set_keypoints(d["kp_x"], d["kp_t"])
            cs.append(c)
        return cs

    ctxs = contexts()
    params = []
    for c, d in zip(ctxs, pairs):
        z = torch.zeros((3,) + tuple(c.nodes[::-1]), device=dev)
        D0 = c.ngf_eval(z, 10.0).item()
        K0 = c.keypoint_penalty(1.0, z, grad=False, diag=False)["K"].item()
        params.append(disco.Params(eta=10.0, alpha=1.0, gamma=0.1, delta=D0 / K0, pcg_iters=pcg, ls_max=ls_max,
                                   flags=disco.FLAG_LS_DEVICE))
    u0 = [torch.from_numpy(d["u_true"]).to(dev) for d in pairs]
    us = [u.clone() for u in u0]

    def reset():
        for u, a in zip(us, u0):
            u.copy_(a)
        torch.cuda.synchronize()

    def timed(fn):
        reset()
        fn()  # warm-up run
        reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def pair_by_pair():
        for c, p, u in zip(ctxs, params, us):
            for _ in range(iters):
                c.gn_pcg_step(p, u)

    ms_seq = timed(pair_by_pair)
    log(f"[bench-batched] pair by pair: {ms_seq:.2f} ms")
    cache = os.path.join(os.path.expanduser("~"), ".cache", "paper_1807_00467_amd", "autotune.json")
    launch = autotune.tune(ctxs, params, u0, cache=cache, log=log)
    log(f"[bench-batched] launch shape (workgroups per CU: brick, node, vector): {launch}")
    batch = disco.Batch(ctxs)
    rep, st = batch.prepare(params, us)
    autotune.apply(batch, launch)

    def eager():
        for _ in range(iters):
            batch.gn_step()

    ms_eager = timed(eager)
    log(f"[bench-batched] batched eager: {ms_eager:.2f} ms")
    batch.graph_capture(iters)
    ms_graph = timed(batch.graph_launch)
    log(f"[bench-batched] batched graph: {ms_graph:.2f} ms; status {st.cpu().tolist()}")
    nvox = sum(int(np.prod(d["shape"])) for d in pairs)
    n_hv = len(pairs) * iters * pcg
    out = {
        "metric": "GN Hv products/s, batched form (24 uneven pairs)",
        "value": n_hv / (ms_graph / 1e3),
        "unit": "Hv/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": 1,
        "ms_per_step": ms_graph / iters,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"24 pairs drawn from 64x64x32, 128x128x64, 256x256x96, 512x512x128 at a "
                               f"358.4x358.4x320 mm field of view ({nvox / 1e6:.1f} M voxels); per pair "
                               f"{iters} GN iterations x ({pcg} PCG GN products + device line search, "
                               f"{ls_max} trials)", "launch": {str(k): v for k, v in launch.items()}},
        "ms_pair_by_pair": ms_seq,
        "ms_batched_eager": ms_eager,
        "ms_batched_graph": ms_graph,
        "speedup_graph_vs_pair_by_pair": ms_seq / ms_graph,
        "speedup_eager_vs_pair_by_pair": ms_seq / ms_eager,
        "gvoxel_steps_per_s": nvox * iters / (ms_graph / 1e3) / 1e9,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
