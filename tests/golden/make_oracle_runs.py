"""Writes tests/golden/oracle_runs.json: FP64 oracle registrations of the
benchmark workloads at their full sizes, for the parity tests and the
benchmark's error columns (the benchmark never runs the oracle itself outside
its CPU-baseline timing), and tests/golden/oracle_forces.npz: the oracle's
direct-sum forces on sampled template points of the mesh and precision pairs.

Only `oracle/` and the seeded input generators in `synth/` are used. Every
input is rounded to FP32 first, exactly as the HIP path receives it; each
record stores a SHA-256 of those FP32 inputs so that a reader can tell when
the generators have changed since the record was written.

Usage:  python tests/golden/make_oracle_runs.py [section ...]
Sections: lidar, mesh, precision, batch, odometry, mixture, landmarks, forces,
planar, energy (default: all). Existing records of other sections are kept. The whole run
takes about an hour on 8 cores.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")
FORCES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_forces.npz")


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def input_hash(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(f32(a).tobytes())
    return h.hexdigest()


def run(X, Y, checkpoints=(), round32=True, landmarks=None, **kw):
    """Oracle registration of the pair (rounded to FP32 first unless the HIP
    path receives it in FP64); poses (caller frame) at the listed iteration
    counts and at the end."""
    if round32:
        X64, Y64 = f32(X).astype(np.float64), f32(Y).astype(np.float64)
    else:
        X64, Y64 = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    p = oracle.Params(**kw)
    t0 = time.time()
    res = oracle.register(X64, Y64, p, trace=bool(checkpoints), landmarks=landmarks)
    rec = {"R": res["R"].tolist(), "t": res["t"].tolist(), "iters": res["iters"],
           "converged": bool(res["converged"]), "interactions": int(res["interactions"]),
           "params": {k: v for k, v in vars(p).items() if k != "extras"},
           "seconds": time.time() - t0}
    if checkpoints:
        rec["at"] = {}
        for k in checkpoints:
            R, tn, _ = res["history"][k - 1]
            rec["at"][str(k)] = {"R": R.tolist(), "t": oracle.denormalise_t(R, tn, res["info"]).tolist()}
    return rec


def save(db):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, OUT)


def main(sections):
    db = json.load(open(OUT)) if os.path.exists(OUT) else {}
    db["_about"] = ("FP64 oracle (oracle/) registrations of the FP32-rounded synthetic workloads "
                    "(synth/); written by tests/golden/make_oracle_runs.py")
    if "lidar" in sections:
        X, Y, _, _ = synth.lidar_pair()
        rec = run(X, Y, checkpoints=(6,), theta=0.5, max_iter=100)
        rec["input_sha256"] = input_hash(X, Y)
        db["lidar_65536_bh0.5"] = rec
        save(db)
        print("lidar", rec["seconds"], flush=True)
    if "precision" in sections:
        X, Y, _, _ = synth.precision_pair()
        rec = run(X, Y, checkpoints=(10,), theta=0.0, max_iter=100)
        rec["input_sha256"] = input_hash(X, Y)
        db["precision_131072_direct"] = rec
        save(db)
        print("precision", rec["seconds"], flush=True)
    if "mesh" in sections:
        X, Y, _, _ = synth.mesh_pair()
        for th in (0.5, 0.8, 0.3):
            rec = run(X, Y, checkpoints=(3,), theta=th, max_iter=100)
            rec["input_sha256"] = input_hash(X, Y)
            db[f"mesh_1048576_bh{th}"] = rec
            save(db)
            print("mesh", th, rec["seconds"], flush=True)
    if "batch" in sections:
        for tol in (1e-8, 1e-4):
            key = f"batch_256_bh0.5_tol{tol:g}"
            recs = db.get(key, [])
            for pidx in range(len(recs), synth.BATCH_PAIRS):
                X, Y, _, _ = synth.batch_pair(pidx)
                rec = run(X, Y, theta=0.5, max_iter=200, tol=tol)
                rec["input_sha256"] = input_hash(X, Y)
                recs.append(rec)
                if pidx % 16 == 15:
                    db[key] = recs
                    save(db)
                    print(key, pidx + 1, flush=True)
            db[key] = recs
            save(db)
    if "odometry" in sections:
        # the first 8 frame pairs of the 32-frame drive: frame k+1 registered to frame k
        scans, _ = synth.lidar_sequence(9)
        recs = []
        for k in range(8):
            rec = run(scans[k], scans[k + 1], theta=0.5, max_iter=100)
            rec["input_sha256"] = input_hash(scans[k], scans[k + 1])
            recs.append(rec)
            print("odometry", k, rec["seconds"], flush=True)
        db["odometry_lidar_pairs_bh0.5"] = recs
        save(db)
    if "mixture" in sections:
        # the 1,024 / 900-point mixture pair, given to the HIP path in FP64
        X, Y, _, _ = synth.mixture_pair()
        rec = run(X, Y, round32=False, theta=0.0, max_iter=200)
        rec["input_sha256"] = input_hash(X, Y)
        db["mixture_1024_direct_fp64"] = rec
        save(db)
        print("mixture", rec["seconds"], flush=True)
    if "landmarks" in sections:
        # misaligned pairs 0..3 (Euler angles up to 90 degrees) with 0, 1 and
        # 3 prior correspondences as RBF landmark masses
        lm_db = {}
        for k in (0, 1, 3):
            recs = []
            for j in range(4):
                X, Y, _, _, idx = synth.misaligned_pair(j, max_deg=90.0)
                lm = None
                if k:
                    pick = synth.landmark_picks(j, k, len(Y))
                    lm = (idx[pick], pick)
                rec = run(X, Y, landmarks=lm, theta=0.0, max_iter=300, tol=1e-8)
                rec["input_sha256"] = input_hash(X, Y)
                recs.append(rec)
            lm_db[f"priors_{k}"] = recs
            print("landmarks", k, flush=True)
        db["landmarks_misaligned90"] = lm_db
        save(db)
    if "planar" in sections:
        # the planar mixture (D = 2, quadtree), theta 0.5, 100 iterations
        X, Y, _, _ = synth.planar_pair()
        rec = run(X, Y, checkpoints=(3,), theta=0.5, max_iter=100)
        rec["input_sha256"] = input_hash(X, Y)
        db["planar_262144_bh0.5"] = rec
        save(db)
        print("planar", rec["seconds"], flush=True)
    if "energy" in sections:
        # Plummer energy (uniform reference masses 1/n, unit template
        # masses) of the FP32-rounded pairs: the direct sum on the precision
        # pair, the Alg. 2 traversal at theta 0.5 on the mesh pair
        en = {}
        X, Y, _, _ = synth.precision_pair()
        X64, Y64 = f32(X).astype(np.float64), f32(Y).astype(np.float64)
        t0 = time.time()
        e = oracle.gpe(Y64, X64, np.full(len(X64), 1.0 / len(X64)))
        en["precision_131072_direct"] = {"E": e, "interactions": len(X64) * len(Y64),
                                         "input_sha256": input_hash(X, Y), "seconds": time.time() - t0}
        X, Y, _, _ = synth.mesh_pair()
        X64, Y64 = f32(X).astype(np.float64), f32(Y).astype(np.float64)
        t0 = time.time()
        e, cnt = oracle.BHTree(X64, np.full(len(X64), 1.0 / len(X64))).gpe(Y64, None, theta=0.5, count=True)
        en["mesh_1048576_bh0.5"] = {"E": e, "interactions": cnt, "input_sha256": input_hash(X, Y),
                                    "seconds": time.time() - t0}
        db["energy"] = en
        save(db)
        print("energy", {k: v["seconds"] for k, v in en.items()}, flush=True)
    if "forces" in sections:
        # Eq. (GAForce) with uniform masses 1/n on the FP32-rounded clouds
        # (no normalisation), on 4,096 template points of the mesh pair and
        # 512 of the precision pair
        arr = {}
        for name, pair, count, seed in (("mesh", synth.mesh_pair, 4096, 2),
                                        ("precision", synth.precision_pair, 512, 1)):
            X, Y, _, _ = pair()
            X64, Y64 = f32(X).astype(np.float64), f32(Y).astype(np.float64)
            idx = np.random.default_rng(seed).choice(len(Y64), count, replace=False)
            t0 = time.time()
            F = oracle.direct_forces(np.ascontiguousarray(Y64[idx]), X64, np.full(len(X64), 1.0 / len(X64)))
            arr[f"{name}_idx"] = idx.astype(np.int32)
            arr[f"{name}_F"] = F
            arr[f"{name}_input_sha256"] = np.array(input_hash(X, Y))
            print("forces", name, time.time() - t0, flush=True)
        np.savez_compressed(FORCES, **arr)


if __name__ == "__main__":
    main(sys.argv[1:] or ["lidar", "precision", "mesh", "batch", "odometry", "mixture", "landmarks", "forces",
                          "planar", "energy"])
