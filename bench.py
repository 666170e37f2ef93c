"""Benchmark: FP64 logm of the n = 4096 rotation-scaling workload on one MI355X.

One step = one full logm_forward (Algorithm 1: square roots, degree selection,
graph polynomial, 2^s rescale) of a resident n x n matrix.  The value is
algorithmic FP64 flops per second, counted from the call's own decisions:
2n^3 per inverse and per matrix product plus 2n^2 per matrix-vector product.

Prints one JSON line (rank 0).  Single GPU only.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_FP64_PEAK_TFLOPS = 78.6     # MI355X dense fp64 matrix peak
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel, from the rocprofv3 FETCH_SIZE and
# WRITE_SIZE counter runs summarised in profiles/, each scaled by what the same
# counter reads for a plain copy of known size (--copy-calibration).  Tied to the
# kernel source it was measured on: any later edit of that file voids it.
TRAFFIC = {"bytes_per_launch": 4.1700e+08,
           "source_sha256": "c24f1d8bc90a5f6792bb754830a8434d1751e42317c1610f4ce7e43a3d91b34a"}
TRAFFIC_SOURCE = os.path.join(ROOT, "paper_2401_10089_amd", "csrc", "gemm_f64.hip")
COPY_CALIBRATION_DOUBLES = 1 << 27   # 1 GiB read + 1 GiB written


def traffic_per_launch():
    if TRAFFIC is None:
        return None
    import hashlib
    with open(TRAFFIC_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return TRAFFIC["bytes_per_launch"] if sha == TRAFFIC["source_sha256"] else None

WORKLOAD = "rotscale4096"
N = 4096
BATCH_COUNT = 10000   # batched workload: SPD matrices, n ~ U{8..128}
BATCH_SEED = 3001
BWD_SEED = 4001      # differentiation workload


def cpu_baseline(A, budget_s: float = 30.0):
    """The oracle (test infrastructure) on a bounded sample of the same workload:
    Denman-Beavers iterations of the first square root of the n = 4096 matrix."""
    import numpy as np
    import oracle

    try:
        from threadpoolctl import threadpool_info
        cores = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    n = A.shape[0]
    iters = 0
    t0 = time.perf_counter()
    elapsed = 0.0
    n_inv = 0
    # one iteration at a time until the budget is used (each costs 1-2 inverses)
    for it in (1, 2, 3):
        t1 = time.perf_counter()
        _, done, _, ninv = oracle.db_sqrt(A, force_iters=it)
        elapsed = time.perf_counter() - t1
        iters, n_inv = done, ninv
        if time.perf_counter() - t0 + elapsed * 1.7 > budget_s:
            break
    flops = 2.0 * n ** 3 * n_inv
    return {
        "value": flops / elapsed / 1e12,
        "unit": "TFLOP/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"{iters} Denman-Beavers iterations ({n_inv} inverses, 2n^3 each) of the first square "
                  f"root of the n={n} workload matrix, NumPy/LAPACK fp64, {elapsed:.1f} s",
    }


def batched_section(lm, torch, dev, reps: int = 3, per_matrix_sample: int = 40, autotune: bool = True):
    """Batched forward over 10,000 SPD matrices (n ~ U{8..128}, seed 3001): logm/s of the
    one-launch batched path against the single-matrix path on a sample of the same batch."""
    import numpy as np
    from workloads import spd_batch

    mats = spd_batch(BATCH_COUNT, BATCH_SEED)
    plan = lm.BatchPlan([m.shape[0] for m in mats], dev)
    flat = torch.from_numpy(np.concatenate([m.reshape(-1) for m in mats])).to(dev)
    # the class boundary (8-wave kernel above it) is chosen by timing this batch
    if autotune:
        split, _ = lm.autotune_batched(flat, plan)
    else:
        lm.set_batched_split(64)
        split = 64
    L, st = lm.logm_batched(flat, plan)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lm.logm_batched(flat, plan, L_flat=L)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    status = st.cpu().numpy()
    Ls = [x.cpu().numpy() for x in plan.unpack(L)]
    errs = []
    for i in range(0, BATCH_COUNT, BATCH_COUNT // 20):
        w, V = np.linalg.eigh(mats[i])
        Le = (V * np.log(w)) @ V.T
        errs.append(float(np.linalg.norm(Ls[i] - Le) / np.linalg.norm(Le)))
    # the single-matrix path (host-driven decisions, one matrix per call) on a sample
    sample = [torch.from_numpy(m).to(dev) for m in mats[:per_matrix_sample]]
    lm.logm(sample[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for A in sample:
        lm.logm(A)
    torch.cuda.synchronize()
    per_matrix_rate = per_matrix_sample / (time.perf_counter() - t1)
    return {
        "metric": "logm/s batched n<=128",
        "value": BATCH_COUNT / dt,
        "unit": "logm/s",
        "ms_per_batch": 1e3 * dt,
        "workload": f"spd_batch: {BATCH_COUNT} SPD A_i = X_i^T X_i / 64 + 1e-3 I, X_i 64 x n_i N(0,1), "
                    f"n_i ~ U{{8..128}}, seed {BATCH_SEED}, packed row-major",
        "class_split": split,
        "class_split_autotuned": bool(autotune),
        "status_codes": {str(c): int(v) for c, v in zip(*np.unique(status[:, 0], return_counts=True))},
        "mean_s": float(status[:, 1].mean()),
        "max_rel_err_vs_eigh_log_sample": max(errs),
        "per_matrix_path_logm_per_s": per_matrix_rate,
        "per_matrix_path_sample": per_matrix_sample,
        "speedup_vs_per_matrix_path": (BATCH_COUNT / dt) / per_matrix_rate,
    }


def backward_section(lm, torch, dev, A_big, fwd_big_ms, sample: int = 32):
    """fwd+bwd / fwd time ratio of the reverse mode (logm_backward): on a sample of
    the differentiation batch (n = 64, rotation-scaling spectra with r in [1e-2, 1e2])
    and on the n = 4096 matrix of the main metric."""
    import numpy as np
    from workloads import rotscale_matrix

    rng = np.random.default_rng(BWD_SEED + 1)
    mats = [torch.from_numpy(rotscale_matrix(64, BWD_SEED + i, 1e-2, 1e2)[0]).to(dev) for i in range(sample)]
    grads = [torch.from_numpy(rng.standard_normal((64, 64))).to(dev) for _ in range(sample)]
    ws = torch.empty(lm.backward_workspace_size(64, tape_mats=48), dtype=torch.uint8, device=dev)
    lm.logm(mats[0])
    lm.logm_backward(mats[0], grads[0], workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A in mats:
        lm.logm(A)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    for A, G in zip(mats, grads):
        lm.logm_backward(A, G, workspace=ws)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    # the taped pair (what the autograd wrapper runs): forward with tape, then backward
    tape = lm.Tape(64, dev, tape_mats=48)
    t_tf = t_tb = 0.0
    for A, G in zip(mats, grads):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lm.logm_forward_taped(A, tape)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lm.logm_backward_taped(G, tape)
        torch.cuda.synchronize()
        t_tf += t1 - t0
        t_tb += time.perf_counter() - t1
    out = {
        "metric": "fwd+bwd/fwd time ratio",
        "value": (t_tf + t_tb) / t_fwd,
        "definition": "(taped forward + taped backward) / plain forward, as the autograd wrapper runs",
        "workload": f"{sample} of the differentiation batch: n = 64, rotscale construction with "
                    f"r ~ logU[1e-2, 1e2], seeds {BWD_SEED}+i, G iid N(0,1) seed {BWD_SEED + 1}",
        "fwd_ms_per_matrix": 1e3 * t_fwd / sample,
        "taped_fwd_ms_per_matrix": 1e3 * t_tf / sample,
        "taped_bwd_ms_per_matrix": 1e3 * t_tb / sample,
        "self_contained_bwd_ms_per_matrix": 1e3 * t_bwd / sample,
        "self_contained_ratio": (t_fwd + t_bwd) / t_fwd,
    }
    del ws
    G = torch.from_numpy(np.random.default_rng(BWD_SEED + 2).standard_normal(A_big.shape)).to(dev)
    # room for every taped inverse of the call (80 at this workload), so no root is replayed
    tape = lm.Tape(A_big.shape[0], dev, tape_mats=48)
    wsb = tape.ws
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm.logm_forward_taped(A_big, tape)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, info = lm.logm_backward_taped(G, tape)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lm.logm_backward(A_big, G, workspace=wsb)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out["n4096"] = {
        "fwd_ms": fwd_big_ms,
        "taped_fwd_ms": 1e3 * (t1 - t0),
        "taped_bwd_ms": 1e3 * (t2 - t1),
        "ratio": (1e3 * (t2 - t0)) / fwd_big_ms,
        "self_contained_bwd_ms": 1e3 * (t3 - t2),
        "self_contained_ratio": (fwd_big_ms + 1e3 * (t3 - t2)) / fwd_big_ms,
        "taped_bwd_tflops": info["flops"] / (t2 - t1) / 1e12,
        "workspace_gib": wsb.numel() / 2 ** 30,
    }
    del tape
    del wsb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain copy (torch.neg) of 1 GiB so that "
                         "counter runs can scale FETCH_SIZE / WRITE_SIZE to bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the single-matrix logm is not sharded); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2401_10089_amd as lm
    from workloads import CONFIG_SEEDS, rotscale_matrix

    lm.load_library()
    dev = torch.device("cuda:0")
    A_np, L_exact = rotscale_matrix(N, CONFIG_SEEDS[WORKLOAD])
    A = torch.from_numpy(A_np).to(dev)
    out = torch.empty_like(A)
    ws = torch.empty(lm.workspace_size(N), dtype=torch.uint8, device=dev)
    # the library's launch-shape autotuner picks the trailing-update workgroup cap for
    # this size (outside the timed region)
    lookahead_wgs, _ = lm.autotune(N, dev, ws) if not args.no_autotune else (None, None)
    lookahead_wgs = dict(zip(("search", "reordered"), lookahead_wgs)) if lookahead_wgs else None
    torch.cuda.synchronize()

    info = None
    for _ in range(args.warmup):
        _, info = lm.logm(A, out=out, workspace=ws)
    torch.cuda.synchronize()

    lm.profile_reset()
    lm.profile_enable(True)
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    flops = 0.0
    for _ in range(args.steps):
        _, info = lm.logm(A, out=out, workspace=ws)
        flops += info["flops"]
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lm.profile_enable(False)
    prof = lm.profile_get()
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / args.steps
    value = flops / wall / 1e12

    if args.copy_calibration:
        src = torch.ones(COPY_CALIBRATION_DOUBLES, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    L = out.cpu().numpy()
    rel_err = float(np.linalg.norm(L - L_exact) / np.linalg.norm(L_exact))

    # precision variant (untimed for the metric): graph products on the fp32 matrix cores
    out32 = torch.empty_like(A)
    torch.cuda.synchronize()
    t32 = time.perf_counter()
    lm.logm(A, out=out32, workspace=ws, graph_fp32=True)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t32
    L32 = out32.cpu().numpy()
    fp32_check = {
        "graph_fp32_rel_err_vs_fp64_path": float(np.linalg.norm(L32 - L) / np.linalg.norm(L)),
        "graph_fp32_rel_err_vs_exact_log": float(np.linalg.norm(L32 - L_exact) / np.linalg.norm(L_exact)),
        "graph_fp32_ms": 1e3 * t32,
    }
    del out32

    achieved = prof["flops"] / (prof["ms"] * 1e-3) / 1e12 if prof["ms"] > 0 else None
    roofline = {
        "bound": "mfma",
        "kernel": "gemm_kernel<GjeOuterOp> (Gauss-Jordan rank-256 trailing update)",
        "achieved": achieved,
        "peak": MFMA_FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": (achieved / MFMA_FP64_PEAK_TFLOPS) if achieved else None,
        "traffic": traffic_per_launch(),
        "launches": prof["launches"],
        "algorithmic_bytes_per_launch": prof["bytes"] / max(prof["launches"], 1),
        "avg_launch_ms": prof["ms"] / max(prof["launches"], 1),
        "algorithmic_flops_per_launch": prof["flops"] / max(prof["launches"], 1),
    }
    line = {
        "metric": "FP64 TFLOP/s logm at n=4096",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "rotscale4096: A = V blockdiag(r [[cos t, sin t], [-sin t, cos t]]) V^-1, "
                        "V = I + 0.1 N(0,1)/sqrt(n), log r ~ U[log 1e-3, log 1e3], t ~ U(-0.9pi, 0.9pi), seed 2002",
            "n": N,
            "s": info["s"],
            "k": info["k"],
            "db_iters": info["db_iters"],
            "n_inv": info["n_inv"],
            "n_gemm": info["n_gemm"],
            "n_matvec": info["n_matvec"],
            "n_inv_reordered": info["n_inv_reordered"],
            "n_order_rejected": info["n_order_rejected"],
            "algorithmic_flops_per_step": info["flops"],
            "event_ms_per_step": ev_ms / args.steps,
            "lookahead_wgs": lookahead_wgs,
        },
        "check": {"rel_frobenius_err_vs_exact_log": rel_err, **fp32_check},
        "roofline": roofline,
    }
    if not args.no_batched:
        line["batched"] = batched_section(lm, torch, dev, autotune=not args.no_autotune)
    if not args.no_backward:
        del ws
        line["backward"] = backward_section(lm, torch, dev, A, ms_per_step)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A_np)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
