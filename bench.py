"""Benchmark of the FGA hot path on one MI355X.

One step = one whole registration of the LiDAR-shaped pair (two 64-beam x
1024-azimuth ring scans, 65,536 points each; Barnes-Hut theta = 0.5, FP32
forces with Kahan tiles, FP64 rigid state, NIV masses): normalisation and
masses, tree build, 100 iterations of Alg. 2 (two launches each: forces,
ODE and per-block moments; then the moment sum and the Kabsch step),
de-normalisation. The
iteration count is fixed (tol = 0) so every step does the same work.

Printed on stdout: one JSON line. `value` is force interactions per second
over the whole step (inputs already resident in HBM). Extra fields report the
Barnes-Hut iteration against the FP32 vector peak (`roofline`), the
direct-sum kernel on the 131,072 x 131,072 precision-study shape, batched
versus plain registrations/s on the 256-pair workload, the 1,024-point FP64
mixture, the 1,048,576-point mesh (Barnes-Hut theta sweep against the
direct sum), and the FP64 oracle timed on the host cores on a bounded sample
(`cpu_baseline`).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_INTERACTION = 20          # conventional n-body count (3 sub, 3+3 fma, rsqrt, 3 mul, 3 fma)
PEAK_FP32_VECTOR = 157.3e12        # MI355X published FP32 vector peak (packed), FLOP/s
PEAK_FP32_NONPACKED = 78.6e12      # 256 CU x 64 lanes x 2 flop x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=100, help="iterations per registration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra workloads")
    ap.add_argument("--extras", default="direct,batched,mixture,mesh",
                    help="comma list of extra workloads to run: direct, batched, mixture, mesh")
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--plain-pairs", type=int, default=32,
                    help="pairs of the batch timed with sequential plain solves")
    ap.add_argument("--precision-study", action="store_true",
                    help="also run the 131,072-point precision study (force errors and final pose per mode)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (a known-size kernel for HBM counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2009_14005_amd as fga
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:  # one elementwise kernel reading 256 MiB and writing 256 MiB
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    log("generating LiDAR-shaped pair (65,536 + 65,536 points)")
    X, Y, R_gt, t_gt = synth.lidar_pair()
    Xd = torch.as_tensor(X, dtype=torch.float32, device=dev)
    Yd = torch.as_tensor(Y, dtype=torch.float32, device=dev)
    p = fga.default_params(theta=0.5, max_iter=args.iters, tol=0.0)

    for k in range(args.warmup):
        fga.register(Xd, Yd, p)
        log(f"warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    inter = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        R, t, rep = fga.register(Xd, Yd, p)
        inter += rep.interactions
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    value = inter / elapsed
    log(f"timed {args.steps} registrations: {ms_step:.2f} ms/step, {value:.3e} interactions/s")
    phi = float(np.degrees(np.arccos(np.clip(0.5 * (np.trace(R_gt.T @ R) - 1), -1, 1))))
    diag = float(np.linalg.norm(X.max(0) - X.min(0)))

    # the dominant work: one BH iteration (force launch + reduction launch),
    # timed with events on the library's stream
    st = fga.State(Xd, Yd, p)
    st.step(5)
    torch.cuda.synchronize()
    _, _, r0 = st.get()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_it = args.iters
    e0.record(stream)
    st.step(n_it)
    e1.record(stream)
    torch.cuda.synchronize()
    _, _, r1 = st.get()
    st.close()
    it_ms = e0.elapsed_time(e1) / n_it
    it_inter = (r1.interactions - r0.interactions) / n_it
    achieved = it_inter * FLOP_PER_INTERACTION / (it_ms * 1e-3)
    log(f"BH iteration: {it_ms * 1e3:.1f} us, {it_inter:.3e} interactions/iteration, "
        f"{achieved / 1e12:.2f} TFLOP/s")
    out = {
        "metric": "force interactions/s (% FP32 VALU peak) + registrations/s, batched vs plain",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lidar_ring_scan_pair_65536_bh_theta0.5", "points": [len(X), len(Y)],
                   "theta": 0.5, "iterations": args.iters, "masses": "niv",
                   "precision": "fp32_kahan_forces_fp64_state", "parallelism": "single_gpu"},
        "registrations_per_s": args.steps / elapsed,
        "pct_fp32_vector_peak": 100.0 * value * FLOP_PER_INTERACTION / PEAK_FP32_VECTOR,
        "accuracy_vs_ground_truth": {"phi_deg": phi, "dt_over_diag": float(np.linalg.norm(t - t_gt) / diag)},
        "roofline": {
            "kernel": KERNEL_NAMES.get(r1.traversal, "?") + " + k_reduce_step (one iteration: pose, forces, "
                      "ODE, moments; then ordered moment sum and Kabsch step)",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR,
            "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
            "traffic": measured_traffic(),
            "avg_launch_us": it_ms * 1e3,
            "launches_per_iteration": 2,
            "interactions_per_launch": it_inter,
            "flop_per_interaction": FLOP_PER_INTERACTION,
        },
    }

    extras = set() if args.no_extras else set(args.extras.split(","))
    if "direct" in extras:
        out["direct"] = bench_direct(fga, torch, synth, dev, stream)
    if "batched" in extras:
        out["batched"] = bench_batched(fga, torch, synth, dev, args)
    if "mixture" in extras:
        out["mixture_fp64_direct"] = bench_mixture(fga, torch, synth, dev)
    if "mesh" in extras:
        out["mesh"] = bench_mesh(fga, torch, synth, dev, stream)
    if args.precision_study:
        out["precision_study"] = precision_study(fga, torch, synth, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, Y)
    print(json.dumps(out), flush=True)


KERNEL_NAMES = {0: "k_iteration<float, direct, FP32_KAHAN>",
                1: "k_iteration<float, BH per-particle walk, FP32_KAHAN>",
                64: "k_iteration_group<FP32_KAHAN, 1> (group walk, 64 particles per wave)",
                128: "k_iteration_group<FP32_KAHAN, 2> (group walk, 128 particles per wave)"}


def measured_traffic():
    """HBM bytes per launch of the iteration kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary, scaled by the calibration kernel; None
    when the kernel sources have changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "bh_group_iteration_lidar65536_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def bench_direct(fga, torch, synth, dev, stream):
    """Direct all-pairs kernel on the 131,072 x 131,072 precision-study shape,
    as the iteration of a registration (FP32 Kahan tiles)."""
    log("direct kernel: 131,072 x 131,072")
    X, Y, _, _ = synth.precision_pair()
    Xd = torch.as_tensor(X, dtype=torch.float32, device=dev)
    Yd = torch.as_tensor(Y, dtype=torch.float32, device=dev)
    res = {}
    for name, prec in (("fp32_kahan", fga.PREC_FP32_KAHAN), ("fp32", fga.PREC_FP32)):
        st = fga.State(Xd, Yd, fga.default_params(theta=0.0, tol=0.0, precision=prec))
        st.step(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n_it = 5
        e0.record(stream)
        st.step(n_it)
        e1.record(stream)
        torch.cuda.synchronize()
        st.close()
        ms = e0.elapsed_time(e1) / n_it
        ips = len(X) * len(Y) / (ms * 1e-3)
        res[name] = {"ms_per_iteration": ms, "interactions_per_s": ips,
                     "tflops": ips * FLOP_PER_INTERACTION / 1e12,
                     "frac_fp32_vector_peak": ips * FLOP_PER_INTERACTION / PEAK_FP32_VECTOR}
        log(f"  {name}: {ms:.2f} ms/iteration, {ips:.3e} interactions/s")
    return res


def bench_mesh(fga, torch, synth, dev, stream):
    """1,048,576 + 1,048,576 points on a weighted triangle mesh: one
    iteration of the registration with Barnes-Hut at theta 0.3, 0.5, 0.8
    (group walk, autotuned) and with the direct sum, and the Barnes-Hut force
    error against the direct sum on 4,096 template points (uniform masses,
    the mesh's own coordinates)."""
    log("mesh workload: 1,048,576 + 1,048,576 points")
    X, Y, _, _ = synth.mesh_pair()
    Xd = torch.as_tensor(X, dtype=torch.float32, device=dev)
    Yd = torch.as_tensor(Y, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}

    def timed(theta, warm, n_it):
        st = fga.State(Xd, Yd, fga.default_params(theta=theta, tol=0.0))
        st.step(warm)
        torch.cuda.synchronize()
        _, _, r0 = st.get()
        e0.record(stream)
        st.step(n_it)
        e1.record(stream)
        torch.cuda.synchronize()
        _, _, r1 = st.get()
        st.close()
        ms = e0.elapsed_time(e1) / n_it
        inter = (r1.interactions - r0.interactions) / n_it
        return {"ms_per_iteration": ms, "interactions_per_particle": inter / len(Y),
                "interactions_per_s": inter / (ms * 1e-3)}

    res["direct"] = timed(0.0, 1, 2)
    log(f"  direct: {res['direct']['ms_per_iteration']:.1f} ms/iteration")
    idx = np.random.default_rng(2).choice(len(Y), 4096, replace=False)
    Ys = Yd[torch.as_tensor(idx, device=dev)].contiguous()
    mX = torch.full((len(X),), 1.0 / len(X), dtype=torch.float32, device=dev)
    Fd, _ = fga.forces(Ys, Xd, mX, None, 0.0)
    Fd = Fd.cpu().numpy().astype(np.float64)
    nd = np.linalg.norm(Fd, axis=1)
    for th in (0.3, 0.5, 0.8):
        r = timed(th, 2, 10)
        Fb, _ = fga.forces(Ys, Xd, mX, None, th, fga.default_params(group_width=64))
        e = np.linalg.norm(Fb.cpu().numpy().astype(np.float64) - Fd, axis=1) / nd
        r["force_rel_err_vs_direct_median"] = float(np.median(e))
        r["force_rel_err_vs_direct_p99"] = float(np.percentile(e, 99))
        r["speedup_vs_direct"] = res["direct"]["ms_per_iteration"] / r["ms_per_iteration"]
        res[f"theta_{th}"] = r
        log(f"  theta {th}: {r['ms_per_iteration'] * 1e3:.0f} us/iteration, "
            f"{r['interactions_per_particle']:.0f} interactions/particle, "
            f"error vs direct median {r['force_rel_err_vs_direct_median']:.1e}")
    return res


def bench_mixture(fga, torch, synth, dev):
    """The 1,024 / 900-point Gaussian-mixture registration: direct sum in
    FP64, 200 fixed iterations (launch-bound at this size)."""
    X, Y, Rg, tg = synth.mixture_pair()
    Xd = torch.as_tensor(X, dtype=torch.float64, device=dev)
    Yd = torch.as_tensor(Y, dtype=torch.float64, device=dev)
    p = fga.default_params(theta=0.0, tol=0.0, max_iter=200, precision=fga.PREC_FP64)
    fga.register(Xd, Yd, p)
    torch.cuda.synchronize()
    n = 10
    t0 = time.perf_counter()
    for _ in range(n):
        R, t, rep = fga.register(Xd, Yd, p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / n * 1e3
    phi = float(np.degrees(np.arccos(np.clip(0.5 * (np.trace(Rg.T @ R) - 1), -1, 1))))
    log(f"mixture FP64 direct: {ms:.2f} ms per 200-iteration registration")
    return {"ms_per_registration": ms, "iterations": rep.iters, "interactions_per_s": rep.interactions / (ms * 1e-3),
            "phi_deg_vs_ground_truth": phi}


def precision_study(fga, torch, synth, dev):
    """131,072 x 131,072 direct sums: per precision mode, the relative force
    error on 512 sampled template points against the FP64 oracle (max and
    median), and the final pose after 100 iterations against the FP64 device
    path on the same FP32-rounded coordinates (whose agreement with the
    oracle's Alg. 2 is pinned on the 1,024-point mixture to 1e-11), as rotation
    angle and translation / diagonal."""
    import oracle
    oracle.build(force=False)
    X, Y, _, _ = synth.precision_pair()
    X32 = np.ascontiguousarray(X, dtype=np.float32).astype(np.float64)
    Y32 = np.ascontiguousarray(Y, dtype=np.float32).astype(np.float64)
    n = len(X32)
    mX = np.full(n, 1.0 / n)
    idx = np.random.default_rng(1).choice(len(Y32), 512, replace=False)
    ref = oracle.direct_forces(Y32[idx], X32, mX)
    diag = float(np.linalg.norm(X.max(0) - X.min(0)))
    log("precision study: FP64 reference registration")
    p64 = fga.default_params(theta=0.0, tol=0.0, max_iter=100, precision=fga.PREC_FP64)
    R64, t64, _ = fga.register(torch.as_tensor(X32, dtype=torch.float64, device=dev),
                               torch.as_tensor(Y32, dtype=torch.float64, device=dev), p64)
    res = {}
    # pure FP32 (force tiles and moment sums); FP32 tiles with FP64 moment
    # and state reductions; the same with Kahan-compensated tiles
    modes = (("pure_fp32", fga.PREC_FP32_ALL), ("fp32_tiles_fp64_reductions", fga.PREC_FP32),
             ("fp32_kahan_tiles_fp64_reductions", fga.PREC_FP32_KAHAN))
    Xd = torch.as_tensor(X32, dtype=torch.float32, device=dev)
    Yd = torch.as_tensor(Y32, dtype=torch.float32, device=dev)
    for name, prec in modes:
        prm = fga.default_params(precision=prec)
        F, _ = fga.forces(Yd, Xd, torch.as_tensor(mX, dtype=torch.float32, device=dev), None, 0.0, prm)
        Fs = F.cpu().numpy().astype(np.float64)[idx]
        e = np.linalg.norm(Fs - ref, axis=1) / np.linalg.norm(ref, axis=1)
        R, t, _ = fga.register(Xd, Yd,
                               fga.default_params(theta=0.0, tol=0.0, max_iter=100, precision=prec))
        A = R64.T @ R  # small-angle form: arccos of the trace saturates below ~1e-6 deg
        phi = float(np.degrees(np.arcsin(min(1.0, 0.5 * np.linalg.norm(
            [A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])))))
        res[name] = {"force_rel_err_max": float(e.max()), "force_rel_err_median": float(np.median(e)),
                     "rotation_deg_vs_fp64": phi, "translation_vs_fp64_over_diag": float(np.linalg.norm(t - t64) / diag)}
        log(f"  {name}: force err max {e.max():.2e} median {np.median(e):.2e}; pose {phi:.2e} deg")
    return res


def bench_batched(fga, torch, synth, dev, args):
    """256 mixture pairs with log-uniform sizes: one batched registration
    (persistent work-queue launches replayed from a HIP graph, FP32 forces)
    against sequential plain registrations (FP64 forces and reductions) of a
    subset, both with per-pair convergence (Alg. 2 stop rule, tol 1e-8 on the
    squared step, at most 200 iterations)."""
    k = args.batch_pairs
    log(f"batched workload: {k} pairs")
    pairs = synth.batch_pairs(k)
    Xs = [torch.as_tensor(pp[0], dtype=torch.float32, device=dev) for pp in pairs]
    Ys = [torch.as_tensor(pp[1], dtype=torch.float32, device=dev) for pp in pairs]
    pb = fga.default_params(theta=0.5, max_iter=200)
    fga.register_batch(Xs[:4], Ys[:4], pb)  # warm the code paths
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R, t, reps = fga.register_batch(Xs, Ys, pb)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log(f"  batched: {tb * 1e3:.1f} ms for {k} pairs")
    nplain = min(args.plain_pairs, k)
    Xs64 = [torch.as_tensor(pp[0], dtype=torch.float64, device=dev) for pp in pairs[:nplain]]
    Ys64 = [torch.as_tensor(pp[1], dtype=torch.float64, device=dev) for pp in pairs[:nplain]]
    pp64 = fga.default_params(theta=0.5, max_iter=200, precision=fga.PREC_FP64)
    fga.register(Xs64[0], Ys64[0], pp64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    errs = []
    for j in range(nplain):
        Rp, tp, rp = fga.register(Xs64[j], Ys64[j], pp64)
        diag = np.linalg.norm(pairs[j][0].max(0) - pairs[j][0].min(0))
        c = np.clip(0.5 * (np.trace(Rp.T @ R[j]) - 1), -1, 1)
        errs.append((float(np.degrees(np.arccos(c))), float(np.linalg.norm(tp - t[j]) / diag)))
    torch.cuda.synchronize()
    tp_total = time.perf_counter() - t0
    log(f"  plain FP64: {tp_total * 1e3:.1f} ms for {nplain} pairs")
    errs = np.array(errs)
    gt = []
    for j in range(k):
        Rg, tg = pairs[j][2], pairs[j][3]
        c = np.clip(0.5 * (np.trace(Rg.T @ R[j]) - 1), -1, 1)
        gt.append(float(np.degrees(np.arccos(c))))
    return {
        "pairs": k,
        "batched_registrations_per_s": k / tb,
        "plain_registrations_per_s": nplain / tp_total,
        "plain_pairs_timed": nplain,
        "speedup": (k / tb) / (nplain / tp_total),
        "batched_vs_plain_max_phi_deg": float(errs[:, 0].max()),
        "batched_vs_plain_max_dt_over_diag": float(errs[:, 1].max()),
        "median_iters": float(np.median([r.iters for r in reps])),
        "median_phi_vs_ground_truth_deg": float(np.median(gt)),
    }


def cpu_baseline(X, Y):
    """The FP64 oracle (plain C, OpenMP over template particles) on the host
    cores: Alg. 2 with the literal BH tree on the same LiDAR pair, timed over
    a bounded number of iterations after its one-off setup."""
    import oracle
    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"cpu baseline: FP64 oracle, {threads} threads")
    Xn, Yn, _ = oracle.normalise(X, Y)
    p = oracle.Params(theta=0.5)
    mX, mY = oracle.masses(Xn, Yn, p)
    st = oracle.Stepper(Xn, Yn, mX, mY, p)
    t0 = time.perf_counter()
    iters = 0
    while iters < 100 and (iters < 2 or time.perf_counter() - t0 < 15.0):
        st.step()
        iters += 1
    el = time.perf_counter() - t0
    log(f"  oracle: {iters} iterations in {el:.1f} s")
    return {"value": st.interactions / el, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{iters} Alg. 2 iterations (literal BH tree, theta 0.5, FP64) of the "
                      f"65,536-point LiDAR pair; tree build excluded",
            "ms_per_iteration": 1e3 * el / iters}


if __name__ == "__main__":
    main()
