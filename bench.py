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
TRAFFIC = {"bytes_per_launch": 7.5688e+08,
           "source_sha256": "5520fea9bf0e0381abab966dc08e8a5f6f043412574565e6fd56c76438c255ce"}
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
BWD_COUNT = 1024


def cpu_baseline(A, iters: int = 3):
    """The oracle (test infrastructure) on a bounded sample of the same workload: the
    first `iters` Denman-Beavers iterations of the first square root of the n = 4096
    matrix (2 * iters - 1 inverses, about 15 s on 16 host threads), run once."""
    import numpy as np
    import oracle

    try:
        from threadpoolctl import threadpool_info
        cores = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    n = A.shape[0]
    t0 = time.perf_counter()
    _, done, _, n_inv = oracle.db_sqrt(np.asarray(A), force_iters=iters)
    elapsed = time.perf_counter() - t0
    flops = 2.0 * n ** 3 * n_inv
    return {
        "value": flops / elapsed / 1e12,
        "unit": "TFLOP/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"{done} Denman-Beavers iterations ({n_inv} inverses, 2n^3 each) of the first square "
                  f"root of the n={n} workload matrix, NumPy/LAPACK fp64, {elapsed:.1f} s",
    }


def batch_flops(dims, status):
    """Algorithmic flops of a batch from each matrix's decisions: 2n^3 per inverse
    (sum over roots of 2 * iterations - 1) and per matrix product ((k - 1) graph
    products, plus B^2 at s = 0); the estimator's matrix-vector products are not
    counted.  The status keeps the iteration counts of the first six roots: a root
    beyond them counts one inverse, so the total is a lower bound when s > 6."""
    total = 0.0
    beyond = 0
    for n, (code, s, k, packed) in zip(dims, status):
        if code != 0:
            continue
        its = [(int(packed) >> (5 * r)) & 31 for r in range(min(int(s), 6))]
        n_inv = sum(2 * it - 1 for it in its) + max(int(s) - 6, 0)
        beyond += int(s) > 6
        total += 2.0 * float(n) ** 3 * (n_inv + (int(k) - 1) + (1 if s == 0 else 0))
    return total, beyond


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
    dt_eager = (time.perf_counter() - t0) / reps
    # the launch sequence captured in a HIP graph (no host synchronisation inside),
    # replayed: the batched configuration as specified
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        lm.logm_batched(flat, plan, L_flat=L)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        lm.logm_batched(flat, plan, L_flat=L)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    status = plan.status.view(-1, 4).cpu().numpy()
    flops, beyond = batch_flops([m.shape[0] for m in mats], status)
    Ls = [x.cpu().numpy() for x in plan.unpack(L)]
    errs = []
    for i in range(0, BATCH_COUNT, BATCH_COUNT // 20):
        w, V = np.linalg.eigh(mats[i])
        Le = (V * np.log(w)) @ V.T
        errs.append(float(np.linalg.norm(Ls[i] - Le) / np.linalg.norm(Le)))
    del graph
    # the single-matrix path (host-driven decisions, one matrix per call) on a sample
    sample = [torch.from_numpy(m).to(dev) for m in mats[:per_matrix_sample]]
    lm.logm(sample[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for A in sample:
        lm.logm(A)
    torch.cuda.synchronize()
    per_matrix_rate = per_matrix_sample / (time.perf_counter() - t1)
    achieved = flops / dt / 1e12
    return {
        "metric": "logm/s batched n<=128",
        "value": BATCH_COUNT / dt,
        "unit": "logm/s",
        "timing": "HIP graph replay of the whole batched call (capture of the launch sequence)",
        "ms_per_batch": 1e3 * dt,
        "eager_ms_per_batch": 1e3 * dt_eager,
        "eager_logm_per_s": BATCH_COUNT / dt_eager,
        "roofline": {
            "bound": "alu",
            "kernel": "batched_logm_kernel (Gauss-Jordan elimination in registers, vector fp64 FMA)",
            "achieved": achieved,
            "peak": MFMA_FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / MFMA_FP64_PEAK_TFLOPS,
            "algorithmic_flops_per_batch": flops,
            "flops_note": "2n^3 per inverse and per product from each matrix's status; "
                          f"lower bound: {beyond} matrices with s > 6 count one inverse per extra root",
            "peak_note": "fp64 vector peak of MI355X (256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz)",
        },
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


def backward_section(lm, torch, dev, A_big, fwd_big_ms, count: int = BWD_COUNT):
    """fwd+bwd / fwd time ratio of the reverse mode: over the whole differentiation
    batch (1024 matrices n = 64, rotation-scaling spectra with r in [1e-2, 1e2]), each
    side timed as one loop over the batch with one synchronisation at its end, and on
    the n = 4096 matrix of the main metric."""
    import numpy as np
    from workloads import rotscale_matrix

    rng = np.random.default_rng(BWD_SEED + 1)
    mats = [torch.from_numpy(rotscale_matrix(64, BWD_SEED + i, 1e-2, 1e2)[0]).to(dev) for i in range(count)]
    grads = [torch.from_numpy(rng.standard_normal((64, 64))).to(dev) for _ in range(count)]
    ws = torch.empty(lm.backward_workspace_size(64, tape_mats=48), dtype=torch.uint8, device=dev)
    tape = lm.Tape(64, dev, tape_mats=48)
    lm.logm(mats[0])
    lm.logm_forward_taped(mats[0], tape)
    lm.logm_backward_taped(grads[0], tape)
    lm.logm_backward(mats[0], grads[0], workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A in mats:
        lm.logm(A)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # the taped pair (what the autograd wrapper runs): forward with tape, then backward
    t0 = time.perf_counter()
    for A, G in zip(mats, grads):
        lm.logm_forward_taped(A, tape)
        lm.logm_backward_taped(G, tape)
    torch.cuda.synchronize()
    t_pair = time.perf_counter() - t0
    t0 = time.perf_counter()
    for A in mats:
        lm.logm_forward_taped(A, tape)
    torch.cuda.synchronize()
    t_tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    for A, G in zip(mats, grads):
        lm.logm_backward(A, G, workspace=ws)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    out = {
        "metric": "fwd+bwd/fwd time ratio",
        "value": t_pair / t_fwd,
        "definition": "(taped forward + taped backward) / plain forward over the whole batch, as the "
                      "autograd wrapper runs; each side one loop, synchronised once at its end",
        "workload": f"differentiation batch: {count} matrices n = 64, rotscale construction with "
                    f"r ~ logU[1e-2, 1e2], seeds {BWD_SEED}+i, G iid N(0,1) seed {BWD_SEED + 1}",
        "fwd_ms_per_matrix": 1e3 * t_fwd / count,
        "taped_fwd_ms_per_matrix": 1e3 * t_tf / count,
        "taped_bwd_ms_per_matrix": 1e3 * (t_pair - t_tf) / count,
        "self_contained_bwd_ms_per_matrix": 1e3 * t_bwd / count,
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
        "kernel": "gemm_kernel<GjeOuterOp, 128, 128> (Gauss-Jordan rank-256 trailing update)",
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
