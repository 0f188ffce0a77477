"""Benchmark of the FGA hot path on one MI355X.

One step = one whole registration of the large inhomogeneous pair: two
independent 1,048,576-point samples of a weighted 2,000-triangle mesh
(template rotated up to 45 degrees), Barnes-Hut theta = 0.5, FP32 forces with
Kahan tiles, FP64 moments and rigid state, NIV masses: normalisation and
masses, tree build, 100 iterations of Alg. 2 (two launches each: forces, ODE
and per-block moments; then the moment sum and the Kabsch step), and the
de-normalisation. The iteration count is fixed (tol = 0) so every step does
the same work.

`value` counts the method's own work: the interactions that Alg. 2 makes for
every particle (accepted nodes plus the points of opened leaves), taken from a
registration with the per-particle walk, which makes exactly those
decisions, over the same inputs and parameters. The default group walk shares
one walk between 64 particles and evaluates more terms than that (its MAC is
tested against the group's box); those are reported as
`interactions_evaluated`. `roofline` is the force launch of the group walk
against the FP32 vector peak, timed with HIP events around every launch on
the library's stream.

Printed on stdout: one JSON line. Progress goes to stderr. Every reported
pose carries its error against the FP64 oracle, read from
tests/golden/oracle_runs.json (written by tests/golden/make_oracle_runs.py,
which calls only the oracle) or computed live where the oracle is fast enough.
`cpu_baseline` times the oracle on the host cores on bounded samples.
"""
import argparse
import ctypes
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
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
GOLDEN_FORCES = os.path.join(ROOT, "tests", "golden", "oracle_forces.npz")
KERNEL_NAMES = {0: "k_iteration<float, direct, FP32_KAHAN>",
                1: "k_iteration<float, BH per-particle walk, FP32_KAHAN>",
                32: "k_iteration_group<FP32_KAHAN, 1> (group walk, groups of 32 held twice per wave)",
                64: "k_iteration_group<FP32_KAHAN, 1> (group walk, 64 particles per wave)",
                128: "k_iteration_group<FP32_KAHAN, 2> (group walk, 128 particles per wave)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=100, help="iterations per registration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra workloads")
    ap.add_argument("--extras",
                    default="sweep,lidar,direct,precision,batched,odometry,mixture,landmarks,planar,energy",
                    help="comma list of extra workloads: sweep (mesh theta 0.3/0.8 and direct), "
                         "lidar, direct, precision, batched, odometry, mixture, landmarks, "
                         "planar (D = 2), energy")
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--leaf", type=int, default=0,
                    help="leaf size of the group-walk registrations (0 = autotuned)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (a known-size kernel for HBM counters)")
    return ap.parse_args()


# ------------------------------------------------------------------ helpers
def phi_deg(Ra, Rb):
    """Rotation angle of Ra^T Rb, accurate for small angles too."""
    A = Ra.T @ Rb
    s = 0.5 * np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    c = 0.5 * (np.trace(A) - 1.0)
    return float(np.degrees(np.arctan2(s, c)))


def diag_of(X):
    return float(np.linalg.norm(X.max(0) - X.min(0)))


def golden():
    try:
        return json.load(open(GOLDEN))
    except (OSError, ValueError):
        return {}


def golden_forces():
    """Stored FP64 oracle direct-sum forces on sampled template points of the
    mesh and precision pairs (sample indices included)."""
    try:
        with np.load(GOLDEN_FORCES, allow_pickle=False) as z:
            return {k: z[k] for k in z.files}
    except (OSError, ValueError):
        return {}


def vs_oracle(rec, R, t, X, at=None, iters=None):
    """Pose error against a stored FP64 oracle registration (None if absent).
    With `iters`, the record's pose after that many iterations (its final
    pose or a stored checkpoint), else None."""
    if not rec:
        return None
    if iters is not None and rec.get("iters") != iters:
        at = iters
    if at is not None:
        rec = rec.get("at", {}).get(str(at))
        if rec is None:
            return None
    Ro, to = np.array(rec["R"]), np.array(rec["t"])
    return {"phi_deg": phi_deg(Ro, R), "dt_over_diag": float(np.linalg.norm(t - to) / diag_of(X))}


def omp_threads(n):
    """Sets the OpenMP thread count of this thread's parallel regions (the
    oracle's loops)."""
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def all_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Registration:
    """Timed registrations of one pair, the Alg. 2 interaction count of the
    same registration, and a profiled pass with per-launch HIP events."""

    def __init__(self, fga, torch, X, Y, params, dtype=None):
        self.fga, self.torch = fga, torch
        dtype = dtype or torch.float32
        self.X, self.Y = X, Y
        self.Xd = torch.as_tensor(X, dtype=dtype, device="cuda:0")
        self.Yd = torch.as_tensor(Y, dtype=dtype, device="cuda:0")
        self.p = params

    def timed(self, steps, warmup, label=""):
        fga, torch = self.fga, self.torch
        for k in range(warmup):
            fga.register(self.Xd, self.Yd, self.p)
            log(f"  {label}warmup {k + 1}/{warmup} done")
        torch.cuda.synchronize()
        evaluated = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            R, t, rep = fga.register(self.Xd, self.Yd, self.p)
            evaluated += rep.interactions
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        self.R, self.t, self.rep = R, t, rep
        return el, evaluated / steps

    def tree_build_ms(self, reps=5):
        """Wall time of one Alg. 1 tree build over the reference cloud (device
        copy, Morton sort, octree, node relayout) at the registration's leaf
        size, averaged over `reps` builds."""
        fga, torch = self.fga, self.torch
        p = type(self.p).from_buffer_copy(self.p)
        p.leaf_size = self.rep.leaf_size
        m = torch.ones(self.Xd.shape[0], dtype=self.Xd.dtype, device="cuda:0")
        fga.Tree(self.Xd, m, p).close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fga.Tree(self.Xd, m, p).close()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    def alg2_count(self):
        """Interactions of Alg. 2's per-particle decisions over one whole
        registration: the per-particle walk makes exactly those decisions."""
        p = type(self.p).from_buffer_copy(self.p)
        p.group_width, p.tile, p.leaf_size = 1, 1, 1
        _, _, rep = self.fga.register(self.Xd, self.Yd, p)
        return rep.interactions

    def profile(self, iters):
        """Per-launch HIP-event times (force launch, reduction launch) over
        `iters` iterations after the first, and the interactions evaluated."""
        st = self.fga.State(self.Xd, self.Yd, self.p)
        st.step(1)
        _, _, r0 = st.get()
        f_ms, r_ms = st.step_profile(iters)
        _, _, r1 = st.get()
        st.close()
        return f_ms / iters, r_ms / iters, (r1.interactions - r0.interactions) / iters, r1.traversal


def roofline(kernel, alg2_per_launch, force_ms, traffic=None, evaluated=None):
    achieved = alg2_per_launch * FLOP_PER_INTERACTION / (force_ms * 1e-3)
    out = {"kernel": kernel, "bound": "alu", "achieved": achieved / 1e12,
           "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
           "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED, "traffic": traffic,
           "avg_launch_us": force_ms * 1e3, "alg2_interactions_per_launch": alg2_per_launch,
           "flop_per_interaction": FLOP_PER_INTERACTION}
    if evaluated is not None:
        out["interactions_evaluated_per_launch"] = evaluated
    return out


def measured_traffic(name):
    """HBM bytes per force launch from a committed FETCH_SIZE / WRITE_SIZE
    summary, scaled by the calibration kernel; None when the kernel sources
    have changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


# ----------------------------------------------------------------- headline
def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; use --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2009_14005_amd as fga
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    gold = golden()
    if args.calibrate_copy:  # one elementwise kernel reading 256 MiB and writing 256 MiB
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    log("mesh pair: 1,048,576 + 1,048,576 points, Barnes-Hut theta 0.5")
    X, Y, R_gt, t_gt = synth.mesh_pair()
    p = fga.default_params(theta=0.5, max_iter=args.iters, tol=0.0, leaf_size=args.leaf)
    reg = Registration(fga, torch, X, Y, p)
    elapsed, evaluated = reg.timed(args.steps, args.warmup)
    ms_step = 1e3 * elapsed / args.steps
    alg2 = reg.alg2 = reg.alg2_count()
    value = alg2 * args.steps / elapsed
    f_ms, r_ms, ev_it, trav = reg.profile(args.iters)
    tree_ms = reg.tree_build_ms()
    log(f"timed {args.steps} registrations: {ms_step:.2f} ms/step; Alg. 2 interactions "
        f"{alg2:.4e} per registration -> {value:.3e}/s; force launch {f_ms * 1e3:.1f} us, "
        f"reduction launch {r_ms * 1e3:.1f} us")
    R, t = reg.R, reg.t
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
        "config": {"workload": "weighted_mesh_pair_1048576_bh_theta0.5", "points": [len(X), len(Y)],
                   "theta": 0.5, "iterations": args.iters, "masses": "niv",
                   "precision": "fp32_kahan_forces_fp64_state", "parallelism": "single_gpu",
                   "leaf_size": reg.rep.leaf_size, "traversal": reg.rep.traversal},
        "registrations_per_s": args.steps / elapsed,
        "pct_fp32_vector_peak": 100.0 * value * FLOP_PER_INTERACTION / PEAK_FP32_VECTOR,
        "alg2_interactions_per_registration": alg2,
        "interactions_evaluated_per_registration": evaluated,
        "interactions_evaluated_per_s": evaluated * args.steps / elapsed,
        "ms_per_iteration": {"force_launch": f_ms, "reduction_launch": r_ms},
        "tree_build_ms": tree_ms,
        "error_vs_oracle": vs_oracle(gold.get("mesh_1048576_bh0.5"), R, t, X, iters=args.iters),
        "oracle_alg2_interactions_per_registration": (gold.get("mesh_1048576_bh0.5") or {}).get("interactions"),
        "accuracy_vs_ground_truth": {"phi_deg": phi_deg(R_gt, R),
                                     "dt_over_diag": float(np.linalg.norm(t - t_gt) / diag_of(X))},
        "roofline": roofline(KERNEL_NAMES.get(trav, "?") + " force launch", alg2 / args.iters, f_ms,
                             measured_traffic("bh_group_iteration_mesh1048576_traffic.json"), ev_it),
    }

    extras = set() if args.no_extras else set(args.extras.split(","))
    ctx = dict(fga=fga, torch=torch, synth=synth, gold=gold, args=args)
    if "sweep" in extras:
        out["mesh_theta_sweep"] = bench_sweep(reg, **ctx)
    if "lidar" in extras:
        out["lidar"] = bench_lidar(**ctx)
    if "direct" in extras:
        out["direct"] = bench_direct(**ctx)
    if "precision" in extras:
        out["precision_study"] = precision_study(**ctx)
    if "batched" in extras:
        out["batched"] = bench_batched(**ctx)
    if "odometry" in extras:
        out["odometry"] = bench_odometry(**ctx)
    if "mixture" in extras:
        out["mixture_fp64_direct"] = bench_mixture(**ctx)
    if "landmarks" in extras:
        out["landmarks"] = bench_landmarks(**ctx)
    if "planar" in extras:
        out["planar"] = bench_planar(**ctx)
    if "energy" in extras:
        out["energy"] = bench_energy(**ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, Y, extras, out, **ctx)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------- extras
def bench_sweep(reg, fga, torch, synth, gold, args):
    """The same mesh pair at theta 0.3 and 0.8 (whole registrations, poses
    against the oracle's) and with the direct sum (one iteration); forces of
    every variant on 4,096 sampled template points against the FP64 oracle's
    direct sum (uniform masses, the mesh's own coordinates), stored with
    their sample indices."""
    X, Y = reg.X, reg.Y
    res = {}
    gf = golden_forces()
    Fo, idx = gf.get("mesh_F"), gf.get("mesh_idx")
    Ys = torch.as_tensor(np.ascontiguousarray(Y[idx] if idx is not None else Y[:4096], dtype=np.float32),
                         device="cuda:0")
    mXd = torch.full((len(X),), 1.0 / len(X), dtype=torch.float32, device="cuda:0")

    def ferr(theta, **kw):
        if Fo is None:
            return None
        F, _ = fga.forces(Ys, reg.Xd, mXd, None, theta, fga.default_params(**kw))
        e = np.linalg.norm(F.cpu().numpy().astype(np.float64) - Fo, axis=1) / np.linalg.norm(Fo, axis=1)
        return {"median": float(np.median(e)), "p99": float(np.percentile(e, 99)), "max": float(e.max())}

    # direct sum: one registration iteration, timed with events
    st = fga.State(reg.Xd, reg.Yd, fga.default_params(theta=0.0, tol=0.0))
    st.step(1)
    f_ms, r_ms = st.step_profile(2)
    st.close()
    f_ms /= 2
    ips = len(X) * len(Y) / (f_ms * 1e-3)
    res["direct"] = {"ms_per_iteration": f_ms + r_ms / 2, "force_launch_ms": f_ms, "interactions_per_s": ips,
                     "frac_fp32_vector_peak": ips * FLOP_PER_INTERACTION / PEAK_FP32_VECTOR,
                     "force_rel_err_vs_oracle": ferr(0.0)}
    log(f"  direct: {f_ms:.1f} ms per force launch, {ips:.3e} interactions/s")
    for th in (0.3, 0.5, 0.8):
        if th == 0.5:  # the headline's registrations
            sub, r, a2 = reg, {}, reg.alg2
        else:
            sub = Registration(fga, torch, X, Y, fga.default_params(theta=th, max_iter=args.iters, tol=0.0,
                                                                    leaf_size=args.leaf))
            el, _ = sub.timed(3, 1, f"theta {th} ")
            r, a2 = {"ms_per_registration": el / 3 * 1e3}, sub.alg2_count()
        f_ms, r_ms, ev, _ = sub.profile(args.iters)
        r.update({"force_launch_us": f_ms * 1e3, "reduction_launch_us": r_ms * 1e3,
                  "interactions_evaluated_per_particle": ev / len(Y),
                  "force_rel_err_vs_oracle_direct": {"group_walk": ferr(th, group_width=64),
                                                     "per_particle_walk": ferr(th, group_width=1)},
                  "speedup_vs_direct": res["direct"]["force_launch_ms"] / f_ms})
        r["alg2_interactions_per_particle"] = a2 / args.iters / len(Y)
        r["alg2_interactions_per_s_force_launch"] = a2 / args.iters / (f_ms * 1e-3)
        r["error_vs_oracle"] = vs_oracle(gold.get(f"mesh_1048576_bh{th}"), sub.R, sub.t, X, iters=args.iters)
        res[f"theta_{th}"] = r
        log(f"  theta {th}: force launch {f_ms * 1e3:.0f} us")
    return res


def bench_lidar(fga, torch, synth, gold, args):
    """The 65,536-point LiDAR-shaped pair (two 64-beam ring scans), theta 0.5,
    100 iterations per registration."""
    log("LiDAR pair: 65,536 + 65,536 points")
    X, Y, R_gt, t_gt = synth.lidar_pair()
    reg = Registration(fga, torch, X, Y, fga.default_params(theta=0.5, max_iter=args.iters, tol=0.0,
                                                            leaf_size=args.leaf))
    el, evaluated = reg.timed(10, 2)
    alg2 = reg.alg2_count()
    f_ms, r_ms, ev_it, trav = reg.profile(args.iters)
    tree_ms = reg.tree_build_ms()
    log(f"  {el / 10 * 1e3:.2f} ms per registration; force launch {f_ms * 1e3:.1f} us")
    return {"ms_per_registration": el / 10 * 1e3, "registrations_per_s": 10 / el,
            "alg2_interactions_per_s": alg2 * 10 / el, "alg2_interactions_per_registration": alg2,
            "interactions_evaluated_per_registration": evaluated,
            "oracle_alg2_interactions_per_registration": (gold.get("lidar_65536_bh0.5") or {}).get("interactions"),
            "error_vs_oracle": vs_oracle(gold.get("lidar_65536_bh0.5"), reg.R, reg.t, X, iters=args.iters),
            "accuracy_vs_ground_truth": {"phi_deg": phi_deg(R_gt, reg.R),
                                         "dt_over_diag": float(np.linalg.norm(reg.t - t_gt) / diag_of(X))},
            "leaf_size": reg.rep.leaf_size, "tree_build_ms": tree_ms,
            "roofline": roofline(KERNEL_NAMES.get(trav, "?") + " force launch", alg2 / args.iters, f_ms,
                                 measured_traffic("bh_group_iteration_lidar65536_traffic.json"), ev_it),
            "reduction_launch_us": r_ms * 1e3}


def bench_direct(fga, torch, synth, gold, args):
    """Direct all-pairs kernel on the 131,072 x 131,072 precision-study shape,
    as the force launch of a registration iteration."""
    log("direct kernel: 131,072 x 131,072")
    X, Y, _, _ = synth.precision_pair()
    Xd = torch.as_tensor(X, dtype=torch.float32, device="cuda:0")
    Yd = torch.as_tensor(Y, dtype=torch.float32, device="cuda:0")
    res = {}
    for name, prec in (("fp32_kahan", fga.PREC_FP32_KAHAN), ("fp32", fga.PREC_FP32)):
        st = fga.State(Xd, Yd, fga.default_params(theta=0.0, tol=0.0, precision=prec))
        st.step(1)
        f_ms, r_ms = st.step_profile(5)
        st.close()
        f_ms /= 5
        ips = len(X) * len(Y) / (f_ms * 1e-3)
        res[name] = {"force_launch_ms": f_ms, "reduction_launch_ms": r_ms / 5, "interactions_per_s": ips,
                     "tflops": ips * FLOP_PER_INTERACTION / 1e12,
                     "frac_fp32_vector_peak": ips * FLOP_PER_INTERACTION / PEAK_FP32_VECTOR,
                     "frac_of_nonpacked_peak": ips * FLOP_PER_INTERACTION / PEAK_FP32_NONPACKED}
        log(f"  {name}: {f_ms:.2f} ms per force launch, {ips:.3e} interactions/s")
    return res


def precision_study(fga, torch, synth, gold, args):
    """131,072 x 131,072 direct sums in the three precision modes: relative
    force error on 512 sampled template points against the FP64 oracle (max,
    median), and the pose after 10 and 100 registration iterations against the
    oracle's registration of the same FP32-rounded pair (both stored)."""
    log("precision study: 131,072 x 131,072")
    X, Y, _, _ = synth.precision_pair()
    X32 = np.ascontiguousarray(X, dtype=np.float32).astype(np.float64)
    Y32 = np.ascontiguousarray(Y, dtype=np.float32).astype(np.float64)
    n = len(X32)
    mX = np.full(n, 1.0 / n)
    gf = golden_forces()
    ref, idx = gf.get("precision_F"), gf.get("precision_idx")
    rec = gold.get("precision_131072_direct")
    modes = (("pure_fp32", fga.PREC_FP32_ALL), ("fp32_tiles_fp64_reductions", fga.PREC_FP32),
             ("fp32_kahan_tiles_fp64_reductions", fga.PREC_FP32_KAHAN))
    Xd = torch.as_tensor(X32, dtype=torch.float32, device="cuda:0")
    Yd = torch.as_tensor(Y32, dtype=torch.float32, device="cuda:0")
    mXd = torch.as_tensor(mX, dtype=torch.float32, device="cuda:0")
    res = {}
    for name, prec in modes:
        F, _ = fga.forces(Yd, Xd, mXd, None, 0.0, fga.default_params(precision=prec))
        if ref is not None:
            Fs = F.cpu().numpy().astype(np.float64)[idx]
            e = np.linalg.norm(Fs - ref, axis=1) / np.linalg.norm(ref, axis=1)
        else:
            e = np.full(1, np.nan)
        st = fga.State(Xd, Yd, fga.default_params(theta=0.0, tol=0.0, precision=prec))
        st.step(10)
        R10, t10, _ = st.get()
        st.step(90)
        R, t, _ = st.get()
        st.close()
        res[name] = {"force_rel_err_max": float(e.max()), "force_rel_err_median": float(np.median(e)),
                     "pose_vs_oracle_10_iterations": vs_oracle(rec, R10, t10, X32, at=10),
                     "pose_vs_oracle_100_iterations": vs_oracle(rec, R, t, X32)}
        log(f"  {name}: force err max {e.max():.2e} median {np.median(e):.2e}")
    return res


def bench_batched(fga, torch, synth, gold, args):
    """256 mixture pairs with log-uniform sizes: one batched registration
    (persistent work-queue launches replayed from a HIP graph, FP32 forces)
    against sequential plain registrations of every pair (FP64 forces and
    reductions), both with the per-pair Alg. 2 stop rule (at most 200
    iterations), at tol 1e-8 (the default) and 1e-4 on the squared step.
    Pose errors of both against the oracle's registrations of every pair."""
    k = args.batch_pairs
    log(f"batched workload: {k} pairs")
    pairs = synth.batch_pairs(k)
    Xs = [torch.as_tensor(pp[0], dtype=torch.float32, device="cuda:0") for pp in pairs]
    Ys = [torch.as_tensor(pp[1], dtype=torch.float32, device="cuda:0") for pp in pairs]
    X64 = [torch.as_tensor(np.ascontiguousarray(pp[0], dtype=np.float32), dtype=torch.float64,
                           device="cuda:0") for pp in pairs]
    Y64 = [torch.as_tensor(np.ascontiguousarray(pp[1], dtype=np.float32), dtype=torch.float64,
                           device="cuda:0") for pp in pairs]
    res = {"pairs": k}
    for tol in (1e-8, 1e-4):
        # fixed configuration: tau option 2, part cap 16, Alg. 1 leaves
        pf = fga.default_params(theta=0.5, max_iter=200, tol=tol, tile=16, leaf_size=1)
        fga.register_batch(Xs[:4], Ys[:4], pf)  # warm the code paths
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fga.register_batch(Xs, Ys, pf)
        torch.cuda.synchronize()
        t_fixed = time.perf_counter() - t0
        # autotuned: (tau option, part cap, leaf size) chosen on this batch by
        # a first call, whose choice later calls of the same shape reuse
        pb = fga.default_params(theta=0.5, max_iter=200, tol=tol, tile=0, leaf_size=0)
        t0 = time.perf_counter()
        fga.register_batch(Xs, Ys, pb)
        torch.cuda.synchronize()
        t_tuning = time.perf_counter() - t0
        t0 = time.perf_counter()
        Rb, tb, reps = fga.register_batch(Xs, Ys, pb)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        pp64 = fga.default_params(theta=0.5, max_iter=200, tol=tol, precision=fga.PREC_FP64)
        fga.register(X64[0], Y64[0], pp64)
        torch.cuda.synchronize()
        plain = []
        t0 = time.perf_counter()
        for j in range(k):
            plain.append(fga.register(X64[j], Y64[j], pp64))
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        recs = gold.get(f"batch_256_bh0.5_tol{tol:g}") or []
        eb, ep, ebp = [], [], []
        for j in range(k):
            diag = diag_of(pairs[j][0])
            Rp, tp, _ = plain[j]
            ebp.append((phi_deg(Rp, Rb[j]), float(np.linalg.norm(tp - tb[j]) / diag)))
            if j < len(recs):
                e1 = vs_oracle(recs[j], Rb[j], tb[j], pairs[j][0])
                e2 = vs_oracle(recs[j], Rp, tp, pairs[j][0])
                eb.append((e1["phi_deg"], e1["dt_over_diag"]))
                ep.append((e2["phi_deg"], e2["dt_over_diag"]))
        gt = [phi_deg(pairs[j][2], Rb[j]) for j in range(k)]

        def summ(a):
            if not a:
                return None
            a = np.array(a)
            return {"phi_deg_max": float(a[:, 0].max()), "phi_deg_median": float(np.median(a[:, 0])),
                    "dt_over_diag_max": float(a[:, 1].max()), "dt_over_diag_median": float(np.median(a[:, 1])),
                    "pairs": len(a)}
        alg2_walk = None
        if tol == 1e-8:
            # the batch with the per-particle walk: Alg. 2's own node
            # decisions in FP32 (Kahan), so its poses differ from the plain
            # FP64 registrations by rounding only
            pw = fga.default_params(theta=0.5, max_iter=200, tol=tol, group_width=1, leaf_size=1)
            fga.register_batch(Xs[:4], Ys[:4], pw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Rw, tw, repw = fga.register_batch(Xs, Ys, pw)
            torch.cuda.synchronize()
            t_walk = time.perf_counter() - t0
            ew, ewp = [], []
            for j in range(k):
                diag = diag_of(pairs[j][0])
                ewp.append((phi_deg(plain[j][0], Rw[j]), float(np.linalg.norm(plain[j][1] - tw[j]) / diag)))
                if j < len(recs):
                    e3 = vs_oracle(recs[j], Rw[j], tw[j], pairs[j][0])
                    ew.append((e3["phi_deg"], e3["dt_over_diag"]))
            alg2_walk = {"registrations_per_s": k / t_walk, "ms": t_walk * 1e3, "speedup_vs_plain": t_plain / t_walk,
                         "median_iters": float(np.median([r.iters for r in repw])),
                         "vs_oracle": None, "vs_plain": None}
            log(f"  tol {tol:g}: batched per-particle walk {t_walk * 1e3:.1f} ms")
        res[f"tol_{tol:g}"] = {
            "batched_registrations_per_s": k / t_batch, "plain_registrations_per_s": k / t_plain,
            "batched_interactions_evaluated_per_s": sum(r.interactions for r in reps) / t_batch,
            "batched_fixed_config_registrations_per_s": k / t_fixed, "tuning_call_ms": t_tuning * 1e3,
            "tuned_leaf_size": reps[0].leaf_size,
            "speedup": t_plain / t_batch, "batched_ms": t_batch * 1e3, "plain_ms": t_plain * 1e3,
            "median_iters_batched": float(np.median([r.iters for r in reps])),
            "median_iters_plain": float(np.median([pl[2].iters for pl in plain])),
            "batched_vs_oracle": summ(eb), "plain_vs_oracle": summ(ep), "batched_vs_plain": summ(ebp),
            "median_phi_vs_ground_truth_deg": float(np.median(gt))}
        if alg2_walk is not None:
            alg2_walk["vs_oracle"], alg2_walk["vs_plain"] = summ(ew), summ(ewp)
            res[f"tol_{tol:g}"]["batched_per_particle_walk"] = alg2_walk
        log(f"  tol {tol:g}: batched {t_batch * 1e3:.1f} ms (fixed configuration {t_fixed * 1e3:.1f} ms), "
            f"plain FP64 {t_plain * 1e3:.1f} ms for {k} pairs")
    return res


def bench_odometry(fga, torch, synth, gold, args, nframes=32):
    """Sequential LiDAR odometry: a 32-frame drive through the LiDAR scene
    (65,536-point ring scans, 1 m per frame), every frame registered to the
    previous one in one call (theta 0.5, 100 iterations per pair, each
    frame's tree built once) and the poses composed. Frames per second,
    relative-pose error against the ground truth, end-point drift over the
    path length, and the first 8 pairs against the oracle's registrations."""
    log(f"odometry: {nframes} frames of 65,536 points")
    scans, poses = synth.lidar_sequence(nframes)
    frames = [torch.as_tensor(np.ascontiguousarray(sc, np.float32), device="cuda:0") for sc in scans]
    p = fga.default_params(theta=0.5, tol=0.0, max_iter=args.iters)
    fga.register_sequence(frames[:3], p)  # warm the code paths
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Rr, tr, Ra, ta, reps = fga.register_sequence(frames, p)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    R0, p0 = poses[0]
    rel, gt_abs = [], []
    for k in range(nframes - 1):
        Rk, pk = poses[k]
        Rn, pn = poses[k + 1]
        rel.append((phi_deg(Rk.T @ Rn, Rr[k]), float(np.linalg.norm(tr[k] - Rk.T @ (pn - pk)))))
    path = sum(float(np.linalg.norm(poses[k + 1][1] - poses[k][1])) for k in range(nframes - 1))
    end_err = float(np.linalg.norm(ta[-1] - R0.T @ (poses[-1][1] - p0)))
    recs = gold.get("odometry_lidar_pairs_bh0.5") or []
    vo = [vs_oracle(recs[k], Rr[k], tr[k], scans[k], iters=args.iters) for k in range(min(len(recs), nframes - 1))]
    rel = np.array(rel)
    log(f"  {el * 1e3:.1f} ms for {nframes - 1} pairs ({(nframes - 1) / el:.1f} frames/s), drift {end_err / path:.4f}")
    return {"frames": nframes, "ms_total": el * 1e3, "frames_per_s": (nframes - 1) / el,
            "ms_per_frame": el * 1e3 / (nframes - 1),
            "relative_phi_deg_vs_ground_truth_median": float(np.median(rel[:, 0])),
            "relative_dt_m_vs_ground_truth_median": float(np.median(rel[:, 1])),
            "end_point_drift_over_path_length": end_err / path, "path_length_m": path,
            "vs_oracle_max_phi_deg": max((v["phi_deg"] for v in vo), default=None),
            "vs_oracle_max_dt_over_diag": max((v["dt_over_diag"] for v in vo), default=None),
            "pairs_vs_oracle": len(vo)}


def bench_mixture(fga, torch, synth, gold, args):
    """The 1,024 / 900-point Gaussian-mixture registration: direct sum in
    FP64, 200 fixed iterations (launch-bound at this size); pose against the
    stored oracle registration of the same FP64 pair and the ground truth."""
    X, Y, Rg, tg = synth.mixture_pair()
    Xd = torch.as_tensor(X, dtype=torch.float64, device="cuda:0")
    Yd = torch.as_tensor(Y, dtype=torch.float64, device="cuda:0")
    p = fga.default_params(theta=0.0, tol=0.0, max_iter=200, precision=fga.PREC_FP64)
    fga.register(Xd, Yd, p)
    torch.cuda.synchronize()
    n = 10
    t0 = time.perf_counter()
    for _ in range(n):
        R, t, rep = fga.register(Xd, Yd, p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / n * 1e3
    log(f"mixture FP64 direct: {ms:.2f} ms per 200-iteration registration")
    return {"ms_per_registration": ms, "registrations_per_s": 1e3 / ms, "iterations": rep.iters,
            "ms_per_iteration": ms / rep.iters, "interactions_per_s": rep.interactions / (ms * 1e-3),
            "error_vs_oracle": vs_oracle(gold.get("mixture_1024_direct_fp64"), R, t, X),
            "accuracy_vs_ground_truth": {"phi_deg": phi_deg(Rg, R),
                                         "dt_over_diag": float(np.linalg.norm(t - tg) / diag_of(X))}}


def emb3(R2):
    """A 2 x 2 rotation as the 3 x 3 rotation about z."""
    R = np.eye(3)
    R[:2, :2] = R2
    return R


def bench_planar(fga, torch, synth, gold, args):
    """The planar mixture (D = 2: 262,144 reference and 196,608 template
    points, quadtree, theta 0.5, FP32 Kahan forces, 100 iterations per
    registration): registrations/s, Alg. 2 interactions per second over whole
    registrations (the per-particle walk's count of the same registration),
    and the pose against the stored oracle registration and the ground
    truth."""
    log("planar mixture (D = 2): 262,144 + 196,608 points, theta 0.5")
    X, Y, R_gt, t_gt = synth.planar_pair()
    Xd = torch.as_tensor(np.ascontiguousarray(X, np.float32), device="cuda:0")
    Yd = torch.as_tensor(np.ascontiguousarray(Y, np.float32), device="cuda:0")
    p = fga.default_params(theta=0.5, max_iter=args.iters, tol=0.0, leaf_size=args.leaf)
    fga.register_2d(Xd, Yd, p)  # tunes the walk, warms the code paths
    torch.cuda.synchronize()
    n = 5
    t0 = time.perf_counter()
    for _ in range(n):
        R, t, rep = fga.register_2d(Xd, Yd, p)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / n
    pa = type(p).from_buffer_copy(p)
    pa.group_width, pa.tile, pa.leaf_size = 1, 1, 1
    _, _, ra = fga.register_2d(Xd, Yd, pa)
    rec = gold.get("planar_262144_bh0.5")
    ev = None
    if rec:
        ev = {"phi_deg": phi_deg(emb3(np.array(rec["R"])), emb3(R)),
              "dt_over_diag": float(np.linalg.norm(t - np.array(rec["t"])) / diag_of(X))}
    log(f"  {el * 1e3:.2f} ms per registration, {ra.interactions / el:.3e} Alg. 2 interactions/s")
    return {"ms_per_registration": el * 1e3, "registrations_per_s": 1.0 / el,
            "alg2_interactions_per_registration": ra.interactions,
            "alg2_interactions_per_s": ra.interactions / el,
            "interactions_evaluated_per_registration": rep.interactions,
            "oracle_alg2_interactions_per_registration": (rec or {}).get("interactions"),
            "traversal": rep.traversal, "leaf_size": rep.leaf_size, "error_vs_oracle": ev,
            "accuracy_vs_ground_truth": {"phi_deg": phi_deg(emb3(R_gt), emb3(R)),
                                         "dt_over_diag": float(np.linalg.norm(t - t_gt) / diag_of(X))}}


def bench_energy(fga, torch, synth, gold, args):
    """Plummer energy (the convergence diagnostic; its negative gradient is
    Eq. GAForce), uniform reference masses 1/n and unit template masses: the
    direct sum over the 131,072-point precision pair and the Alg. 2 traversal
    (theta 0.5, per-particle decisions, tree build included) over the mesh
    pair. Time per evaluation (best of 3), interactions/s, and the relative
    difference from the stored oracle values."""
    log("Plummer energy: direct 131,072 x 131,072, Barnes-Hut 1,048,576 x 1,048,576")
    recs = gold.get("energy") or {}
    res = {}
    for key, pair, theta in (("precision_131072_direct", synth.precision_pair, 0.0),
                             ("mesh_1048576_bh0.5", synth.mesh_pair, 0.5)):
        X, Y, _, _ = pair()
        Xd = torch.as_tensor(np.ascontiguousarray(X, np.float32), device="cuda:0")
        Yd = torch.as_tensor(np.ascontiguousarray(Y, np.float32), device="cuda:0")
        mX = torch.full((len(X),), 1.0 / len(X), dtype=torch.float32, device="cuda:0")
        fga.energy(Yd, Xd, mX, None, theta)
        torch.cuda.synchronize()
        best = 1e9
        for _ in range(3):
            t0 = time.perf_counter()
            E, cnt = fga.energy(Yd, Xd, mX, None, theta)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        rec = recs.get(key)
        res[key] = {"ms_per_evaluation": best * 1e3, "interactions": cnt, "interactions_per_s": cnt / best,
                    "E": E, "rel_diff_vs_oracle": abs(E - rec["E"]) / abs(rec["E"]) if rec else None,
                    "oracle_interactions": rec["interactions"] if rec else None}
        log(f"  {key}: {best * 1e3:.2f} ms, {cnt / best:.3e} interactions/s")
    return res


def bench_landmarks(fga, torch, synth, gold, args, samples=32):
    """Registration under large misalignment (full overlap, Euler angles up
    to 90 degrees about each axis, 1,888 points) with 0, 1 and 3 prior correspondences as
    RBF landmark masses (Eq. RBF_function, S = N o B): success rate (RMSE of
    the registered template under 1% of the bounding-box diagonal), time per
    registration, and the pose against the stored oracle registrations of
    the first samples."""
    log(f"landmark masses: {samples} misaligned pairs, 0 / 1 / 3 prior matches")
    p = fga.default_params(theta=0.0, max_iter=300, tol=1e-8)
    res = {}
    lm_gold = gold.get("landmarks_misaligned90") or {}
    for k in (0, 1, 3):
        recs = lm_gold.get(f"priors_{k}") or []
        ok, ms, err = 0, [], []
        for j in range(samples):
            X, Y, Rg, tg, idx = synth.misaligned_pair(j, max_deg=90.0)
            lm = None
            if k:
                pick = synth.landmark_picks(j, k, len(Y))
                lm = (idx[pick], pick)
            Xd = torch.as_tensor(X, dtype=torch.float32, device="cuda:0")
            Yd = torch.as_tensor(Y, dtype=torch.float32, device="cuda:0")
            fga.register(Xd, Yd, p, landmarks=lm) if j == 0 else None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R, t, rep = fga.register(Xd, Yd, p, landmarks=lm)
            ms.append((time.perf_counter() - t0) * 1e3)
            rmse = float(np.sqrt(np.mean(np.sum((Y @ R.T + t - X[idx]) ** 2, 1))))
            ok += rmse < 0.01 * diag_of(X)
            if j < len(recs):
                v = vs_oracle(recs[j], R, t, X)
                err.append((v["phi_deg"], v["dt_over_diag"]))
        e = np.array(err) if err else np.full((1, 2), np.nan)
        res[f"priors_{k}"] = {"success_rate": ok / samples, "ms_per_registration_median": float(np.median(ms)),
                              "registrations_per_s": 1e3 / float(np.mean(ms)),
                              "vs_oracle_max_phi_deg": float(e[:, 0].max()),
                              "vs_oracle_max_dt_over_diag": float(e[:, 1].max()), "pairs_vs_oracle": len(err)}
        log(f"  {k} priors: success {ok}/{samples}, {np.median(ms):.2f} ms per registration")
    return res


# ------------------------------------------------------------- CPU baseline
def cpu_baseline(X, Y, extras, out, fga, torch, synth, gold, args):
    """The FP64 oracle (plain C loops, OpenMP over template particles) on the
    host cores, on bounded samples of each workload. The headline figure is
    one Alg. 2 iteration of the mesh pair with the literal tree at theta 0.5
    (tree build timed apart) on all threads."""
    import oracle
    oracle.build(force=False)
    nth = all_threads()
    log(f"cpu baseline: FP64 oracle, {nth} threads ({cpu_model()})")

    def f64(a):
        return np.ascontiguousarray(a, dtype=np.float32).astype(np.float64)

    Xn, Yn, _ = oracle.normalise(f64(X), f64(Y))
    prm = oracle.Params(theta=0.5)
    mX, mY = oracle.masses(Xn, Yn, prm)
    omp_threads(nth)
    t0 = time.perf_counter()
    tree = oracle.BHTree(Xn, mX)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, cnt = tree.forces(Yn, None, prm.G, prm.eps, prm.theta, count=True)
    el = time.perf_counter() - t0
    sub = np.random.default_rng(3).choice(len(Yn), 16384, replace=False)
    omp_threads(1)
    t0 = time.perf_counter()
    _, cnt1 = tree.forces(Yn[sub], None, prm.G, prm.eps, prm.theta, count=True)
    el1 = time.perf_counter() - t0
    del tree
    res = {"value": cnt / el, "unit": "interactions/s", "cores": nth, "kind": "oracle",
           "sample": "one Alg. 2 force evaluation (literal uncompressed tree, theta 0.5, FP64) of the "
                     "1,048,576-point mesh pair at its initial pose; tree build timed apart",
           "cpu_model": cpu_model(), "tree_build_s": t_tree, "iteration_s": el,
           "one_thread": {"interactions_per_s": cnt1 / el1,
                          "sample": "the same evaluation for 16,384 random template points"}}
    if out.get("ms_per_step"):
        est = (t_tree + args.iters * el) * 1e3
        res["registration_ms_estimate"] = est
        res["registration_estimate_note"] = ("extrapolated: tree build + iterations x the measured iteration "
                                             "(the pose changes little the count)")
    per = {}
    # C0: the whole 200-iteration FP64 direct registration, all threads and one
    Xm, Ym, _, _ = synth.mixture_pair()
    for th in (nth, 1):
        omp_threads(th)
        t0 = time.perf_counter()
        oracle.register(Xm, Ym, oracle.Params(max_iter=200))
        per.setdefault("mixture_1024_direct_200it", {})[f"threads_{th}_s"] = time.perf_counter() - t0
    # C1: one BH iteration with one thread, the whole 100-iteration registration with all
    if "lidar" in extras:
        Xl, Yl, _, _ = synth.lidar_pair()
        Xn, Yn, _ = oracle.normalise(f64(Xl), f64(Yl))
        mX, mY = oracle.masses(Xn, Yn, prm)
        omp_threads(nth)
        stp = oracle.Stepper(Xn, Yn, mX, mY, oracle.Params(theta=0.5))
        t0 = time.perf_counter()
        for _ in range(args.iters):
            stp.step()
        t_all = time.perf_counter() - t0
        c_all = stp.interactions
        omp_threads(1)
        t0 = time.perf_counter()
        stp.step()
        t_one = time.perf_counter() - t0
        per["lidar_65536_bh0.5"] = {f"threads_{nth}_registration_s": t_all, "threads_1_iteration_s": t_one,
                                    "interactions_per_s_all_threads": c_all / t_all,
                                    "interactions_per_s_one_thread": (stp.interactions - c_all) / t_one,
                                    "note": "tree build excluded"}
    # C2 direct: the oracle's direct sum for 4,096 template points, all threads
    if "sweep" in extras:
        Xs = f64(X)
        Ys = f64(Y[np.random.default_rng(2).choice(len(Y), 4096, replace=False)])
        omp_threads(nth)
        t0 = time.perf_counter()
        oracle.direct_forces(Ys, Xs, np.full(len(Xs), 1.0 / len(Xs)))
        t = time.perf_counter() - t0
        per["mesh_1048576_direct"] = {"threads": nth, "sample": "4,096 template points x 1,048,576 references",
                                      "interactions_per_s": 4096 * len(X) / t,
                                      "iteration_s_extrapolated": t * len(Y) / 4096}
    # C3: one full FP64 direct force evaluation, all threads (the 100-iteration
    # registration is extrapolated from it); one thread on 1,024 template points
    if "precision" in extras:
        Xp, Yp, _, _ = synth.precision_pair()
        Xp, Yp = f64(Xp), f64(Yp)
        mp_ = np.full(len(Xp), 1.0 / len(Xp))
        omp_threads(nth)
        t0 = time.perf_counter()
        oracle.direct_forces(Yp, Xp, mp_)
        t_all = time.perf_counter() - t0
        omp_threads(1)
        t0 = time.perf_counter()
        oracle.direct_forces(Yp[:1024], Xp, mp_)
        t_one = time.perf_counter() - t0
        per["precision_131072_direct"] = {f"threads_{nth}_iteration_s": t_all,
                                          "threads_1_interactions_per_s": 1024 * len(Xp) / t_one,
                                          "registration_100it_s_extrapolated": 100 * t_all}
    # C4: 8 randomly chosen pairs registered sequentially, extrapolated to 256
    if "batched" in extras:
        sel = np.random.default_rng(4).choice(synth.BATCH_PAIRS, 8, replace=False)
        omp_threads(nth)
        t0 = time.perf_counter()
        for j in sel:
            Xb, Yb, _, _ = synth.batch_pair(int(j))
            oracle.register(f64(Xb), f64(Yb), oracle.Params(theta=0.5, max_iter=200, tol=1e-8))
        t8 = time.perf_counter() - t0
        per["batch_256_bh0.5"] = {"pairs_timed": [int(j) for j in sel], "seconds": t8,
                                  "registrations_per_s": 8 / t8,
                                  "batch_s_extrapolated": t8 / 8 * synth.BATCH_PAIRS}
    # planar (D = 2): one Alg. 2 iteration (quadtree, theta 0.5), all threads
    if "planar" in extras:
        X2, Y2, _, _ = synth.planar_pair()
        Xn, Yn, _ = oracle.normalise(f64(X2), f64(Y2))
        mX, mY = oracle.masses(Xn, Yn, prm)
        omp_threads(nth)
        stp = oracle.Stepper(Xn, Yn, mX, mY, oracle.Params(theta=0.5))
        t0 = time.perf_counter()
        stp.step()
        t_it = time.perf_counter() - t0
        per["planar_262144_bh0.5"] = {f"threads_{nth}_iteration_s": t_it,
                                      "interactions_per_s": stp.interactions / t_it,
                                      "registration_100it_s_extrapolated": 100 * t_it,
                                      "note": "tree build excluded"}
    omp_threads(nth)
    res["per_workload"] = per
    log(f"  oracle: {res['value']:.3e} interactions/s on {nth} threads")
    return res


if __name__ == "__main__":
    main()
