#!/usr/bin/env python3
"""Throughput benchmark of the Householder-reflector hot path on one MI355X.

Default workload (the headline metric): Q X with Q = H_1 ... H_64 on
N = 2^18 vectors of length n = 4096, synthetic Gaussian data resident in HBM,
through the C ABI of libhh.so.  The compact-WY form in BF16 on the matrix
cores is the reported value; the fused FP32 sequential-reflector kernel on
the same shape is timed beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one library call over the whole batch (reflector setup included).
Prints one JSON line.  Other workloads (--workload) exist for measurement runs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
MFMA_BF16_TFLOPS = 2500.0      # dense
MFMA_F32_TFLOPS = 157.3        # dense FP32 matrix cores
FP32_VALU_TFLOPS = 78.6        # unpacked FP32 FMA (packed FP32 is switched off)
FP64_VALU_TFLOPS = 78.6

WORKLOADS = {
    # name: (op, n, h, N, compute, description)
    "qx_n4096_h64": ("apply", 4096, 64, 1 << 18, "bf16",
                     "Q X, n=4096, h=64, N=2^18; compact-WY BF16 (FP32 accumulate)"),
    "qx_n4096_h64_fused": ("apply", 4096, 64, 1 << 18, "f32",
                           "Q X, n=4096, h=64, N=2^18; fused sequential FP32"),
    "sym_n1024_h10": ("sym", 1024, 10, 1 << 20, "f32",
                      "Q diag(lam) Q^T X, n=1024, h=10, N=2^20; fused FP32"),
    "sym_d_n1024_h10": ("sym_d", 1024, 10, 1 << 20, "f32",
                        "D Q diag(lam) Q^T D X (eq. thesbar with a random sign diagonal D), n=1024, "
                        "h=10, N=2^20; fused FP32"),
    "mahal_n512_h9": ("mahal", 512, 9, 1 << 22, "f32",
                      "Mahalanobis distances, n=512, h=9, N=2^22 pairs; fused FP32"),
    "mahal_fb_n512_h9": ("mahal_fb", 512, 9, 1 << 22, "f32",
                         "Mahalanobis forward + backward to U and lam, n=512, h=9, N=2^22; fused FP32"),
    "qx_n64_h4_f64": ("apply", 64, 4, 1024, "f64",
                      "Q X, n=64, h=4, N=1024; fused FP64"),
    "qx_fb_n4096_h64": ("apply_fb", 4096, 64, 1 << 18, "bf16",
                        "Q X forward + backward (dX, dU), n=4096, h=64, N=2^18; compact-WY BF16"),
    "sym_fb_n8192_h128": ("sym_fb", 8192, 128, 1 << 16, "f16",
                          "Q diag(lam) Q^T X forward + backward (dX, dU, dlam), n=8192, h=128, "
                          "N=2^16; compact-WY FP16"),
    "qr_n512_h511": ("apply_qr", 512, 511, 1 << 20, "f32",
                     "Q X with h = n - 1 reflectors of Householder QR structure (k - 1 leading "
                     "zeros, the remark after Result 3), n=512, N=2^20; fused FP32"),
    "knn_n40_h6": ("knn", 40, 6, 49000, "f32",
                   "k-NN (k = 5) in the learned metric, n=40, h=6, 21000 queries against 49000 "
                   "database vectors (the sizes of the paper's MNIST split, synthetic Gaussian data): "
                   "transform both sets, then all-pairs distances on the matrix cores and top-k"),
    "copy_n4096_bf16": ("copy", 4096, 0, 1 << 18, "bf16",
                        "device copy of the Q X batch (2 GiB in, 2 GiB out): HBM calibration"),
}
DEFAULT = "qx_n4096_h64"
KNN_QUERIES, KNN_K = 21000, 5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the fused FP32 kernel beside the default workload")
    return ap.parse_args()


def algorithmic(op, n, h, N, io_bytes, param_bytes=4):
    """Bytes (one read of each input, one write of each output) and flops
    (operation counts of the paper: 4nh per Q x, (8h+1)n per symmetric
    product; (4h+3)n per distance) for one call over N vectors."""
    if op in ("apply", "copy"):
        return 2 * n * io_bytes * N, 4 * n * h * N
    if op == "apply_qr":   # reflector k has n - k + 1 nonzeros: 4(n - k + 1) operations
        return 2 * n * io_bytes * N, 4 * sum(n - k + 1 for k in range(1, h + 1)) * N
    if op == "sym":
        return 2 * n * io_bytes * N, (8 * h + 1) * n * N
    if op == "sym_d":      # the two diagonal products: 2n more
        return 2 * n * io_bytes * N, (8 * h + 3) * n * N
    if op == "mahal":
        return (2 * n * io_bytes + param_bytes) * N, (4 * h + 3) * n * N
    if op == "apply_fb":   # forward: X in, Y out; backward: X, dY in, dX out
        return 5 * n * io_bytes * N, (4 * n * h + 2 * h * h) * 4 * N
    if op == "sym_fb":     # ~24 n h per vector for forward + backward on the matrix cores
        return 5 * n * io_bytes * N, 24 * n * h * N
    if op == "knn":        # transforms of both sets, then the all-pairs products (n padded to 4)
        nq = KNN_QUERIES
        npad = (n + 3) // 4 * 4
        return (N + nq) * n * io_bytes * 2, 2 * npad * nq * N + 4 * n * h * (N + nq)
    if op == "mahal_fb":  # the forward writes each pair's h dot products, the backward reads them
        fwd = (2 * n * io_bytes + param_bytes + h * param_bytes) * N
        bwd = (2 * n * io_bytes + param_bytes + h * param_bytes) * N
        # backward: the chain again by its updates (2nh), then per reflector the
        # rebuild, one dot product, the update and the two dU terms (10nh), and 6n
        return fwd + bwd, ((4 * h + 3) * n + 12 * n * h + 6 * n) * N
    raise ValueError(op)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the workload's dominant kernel from the committed
    rocprofv3 counter summary, if the counters were taken on the current
    sources of that kernel (the entry lists them with their hash); else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            e = json.load(f).get(workload)
        if not e or e.get("source_hash") != source_hash(e["sources"]):
            return None
        return e.get("bytes_per_launch")
    except (OSError, ValueError, KeyError):
        return None


def orthogonality(P, U, n, tdt, dev):
    """||Q^T Q - I||_F / sqrt(n) and max |(Q^T Q - I)_ij| of the path's Q and
    Q^T, each column of Q being the path applied to a unit vector."""
    import torch
    res = {}
    eye = torch.eye(n, dtype=torch.float64, device=dev)
    for trans in (False, True):
        Qt = P.apply_raw(U, eye.to(tdt), trans=trans, compute=tdt).double()
        E = Qt @ Qt.T - eye
        res["QT" if trans else "Q"] = {"fro_over_sqrt_n": float(E.norm()) / math.sqrt(n),
                                        "max_abs": float(E.abs().max())}
        del Qt, E
    res["fro_over_sqrt_n"] = max(r["fro_over_sqrt_n"] for r in (res["Q"], res["QT"]))
    res["max_abs"] = max(r["max_abs"] for r in (res["Q"], res["QT"]))
    del eye
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs "
                          "are not part of this build (--gpus must be 1)"}))
        sys.exit(2)

    import torch
    import synth
    import paper_1811_07624_amd as P

    op, n, h, N, comp, desc = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
           "f16": torch.float16}[comp]
    io_dt = tdt
    pdt = torch.float64 if comp == "f64" else torch.float32

    if op == "apply_qr":
        U = torch.tensor(synth.structured_reflectors(n, h, seed=0), dtype=pdt, device=dev)
    else:
        U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=pdt, device=dev)
    lam_np = (synth.eig_loguniform(n, seed=0) if op == "sym_fb" else synth.eig_uniform(n, seed=0))
    lam = torch.tensor(lam_np, dtype=pdt, device=dev)
    X = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_X, device=dev, dtype=io_dt)
    Xb = None
    w = None
    if op in ("mahal", "mahal_fb"):
        Xb = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_XB, device=dev, dtype=io_dt)
    if op == "mahal_fb":
        w = synth.device_gaussian((N,), seed=0, stream=synth.STREAM_W, device=dev, dtype=pdt)
    Gd = None
    if op in ("apply_fb", "sym_fb"):
        Gd = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_G, device=dev, dtype=io_dt)
    Y = torch.empty_like(X) if op in ("apply", "apply_qr", "sym", "sym_d", "copy", "apply_fb",
                                      "sym_fb") else None
    Xq = None
    if op == "knn":
        Xq = synth.device_gaussian((KNN_QUERIES, n), seed=0, stream=synth.STREAM_XB, device=dev,
                                   dtype=io_dt)
    dsig = None
    if op == "sym_d":
        dsig = torch.tensor(np.where(synth.host_rng(0, 11).random(n) < 0.5, -1.0, 1.0), dtype=pdt, device=dev)
    torch.cuda.synchronize()

    def step():
        if op == "copy":
            Y.copy_(X)
        elif op == "apply":
            P.apply_raw(U, X, compute=tdt, out=Y)
        elif op == "apply_qr":
            P.apply_raw(U, X, compute=tdt, out=Y, algo="fused_qr")
        elif op == "sym":
            P.sym_raw(U, lam, X, compute=tdt, out=Y)
        elif op == "sym_d":
            P.signed_raw("sym", U, X, d_in=dsig, d_out=dsig, lam=lam, compute=tdt, out=Y)
        elif op == "mahal":
            P.mahal_raw(U, lam, X, Xb)
        elif op == "knn":
            P.knn(U, lam, Xq, X, KNN_K)
        elif op == "apply_fb":  # the forward keeps its WY coefficients for the backward
            _, rec = P.apply_raw(U, X, compute=tdt, out=Y, save=True)
            P.apply_bwd_raw(U, X, Gd, compute=tdt, saved=rec)
        elif op == "sym_fb":
            _, rec = P.sym_raw(U, lam, X, compute=tdt, out=Y, save=True)
            P.sym_bwd_raw(U, lam, X, Gd, compute=tdt, saved=rec)
        else:  # the forward keeps each pair's dot products for the backward
            _, rec = P.mahal_raw(U, lam, X, Xb, save=True)
            P.mahal_bwd_raw(U, lam, X, Xb, w, need_dX=False, saved=rec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]  # ms per call, on the launch stream
    ms_call = float(np.mean(per))
    ms_wall = wall * 1e3 / args.steps
    value = (KNN_QUERIES if op == "knn" else N) / (ms_wall * 1e-3)

    # The main kernel's duration: a call also launches the per-call setup
    # kernels (normalisation, T), so the same call on a single vector is timed
    # the same way and subtracted (its main kernel is one tile, a few us).
    ms_setup = 0.0
    if op in ("apply", "apply_qr", "sym", "sym_d", "mahal"):
        X1 = X[:1]
        Y1 = Y[:1] if Y is not None else None
        Xb1 = Xb[:1] if Xb is not None else None

        def step1():
            if op in ("apply", "apply_qr"):
                P.apply_raw(U, X1, compute=tdt, out=Y1, algo="fused_qr" if op == "apply_qr" else "auto")
            elif op == "sym":
                P.sym_raw(U, lam, X1, compute=tdt, out=Y1)
            elif op == "sym_d":
                P.signed_raw("sym", U, X1, d_in=dsig, d_out=dsig, lam=lam, compute=tdt, out=Y1)
            else:
                P.mahal_raw(U, lam, X1, Xb1)
        for _ in range(2):
            step1()
        torch.cuda.synchronize()
        e1 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(10)]
        for a, b in e1:
            a.record(stream)
            step1()
            b.record(stream)
        torch.cuda.synchronize()
        ms_setup = float(np.mean([a.elapsed_time(b) for a, b in e1]))
    ms_ev = ms_call - ms_setup  # main kernel (whole step for the forward+backward workloads)
    timed = "main kernel" if ms_setup > 0 else "whole step"
    if ms_ev < 0.25 * ms_call:
        # a launch-bound call (setup and launches take most of it): the difference
        # of two short timings is noise, so the roofline uses the whole call
        ms_ev, timed = ms_call, "whole call (launch-bound)"

    io_bytes = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[comp]
    abytes, aflops = algorithmic(op, n, h, N, io_bytes, 8 if comp == "f64" else 4)
    if op == "knn":
        bound, peak, unit = "mfma", MFMA_F32_TFLOPS, "TFLOP/s"
        ach = aflops / (ms_ev * 1e-3) / 1e12
    elif comp in ("bf16", "f16"):
        bound, peak, unit, ach = "hbm", HBM_PEAK_GBS, "GB/s", abytes / (ms_ev * 1e-3) / 1e9
        if op == "sym_fb" and aflops / (MFMA_BF16_TFLOPS * 1e12) > abytes / (HBM_PEAK_GBS * 1e9):
            bound, peak, unit = "mfma", MFMA_BF16_TFLOPS, "TFLOP/s"
            ach = aflops / (ms_ev * 1e-3) / 1e12
    else:
        t_hbm = abytes / (HBM_PEAK_GBS * 1e9)
        t_alu = aflops / ((FP64_VALU_TFLOPS if comp == "f64" else FP32_VALU_TFLOPS) * 1e12)
        if t_alu > t_hbm:
            bound, peak, unit = "alu", (FP64_VALU_TFLOPS if comp == "f64" else FP32_VALU_TFLOPS), "TFLOP/s"
            ach = aflops / (ms_ev * 1e-3) / 1e12
        else:
            bound, peak, unit = "hbm", HBM_PEAK_GBS, "GB/s"
            ach = abytes / (ms_ev * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)

    out = {
        "metric": "vectors/s for Q.X at n=4096,h=64 (BF16 compact-WY vs FP32 fused)",
        "value": value,
        "unit": "queries/s" if op == "knn" else "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": comp,
        "data": "synthetic (seeded Gaussian data, Gaussian unit reflectors)",
        "config": {"workload": args.workload, "description": desc, "n": n, "h": h, "N": N,
                   "op": op},
        "roofline": {"bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                     "frac": ach / peak, "traffic": traffic,
                     "kernel_ms_events": ms_ev, "timed": timed, "call_ms_events": ms_call,
                     "setup_ms_events": ms_setup, "algorithmic_bytes": abytes,
                     "algorithmic_flops": aflops},
    }
    if bound == "alu" and comp == "f32":  # the same rate against the FP32 matrix cores
        out["roofline"]["peak_fp32_matrix"] = MFMA_F32_TFLOPS
        out["roofline"]["frac_fp32_matrix"] = ach / MFMA_F32_TFLOPS

    # orthogonality of the operator the path applies: Q (and Q^T) applied to
    # the identity (exact in every compute type) at this workload's n and h,
    # with the same arithmetic; E = Q^T Q - I formed in FP64
    if op != "copy":
        out["orth"] = orthogonality(P, U, n, tdt, dev)

    # the fused FP32 kernel on the same Q X shape, timed beside the headline
    if args.workload == DEFAULT and not args.no_compare:
        del Y
        Xf = X.float()
        Yf = torch.empty_like(Xf)
        for _ in range(1):
            P.apply_raw(U, Xf, out=Yf)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kf = max(1, min(args.steps, 5))
        a.record(stream)
        for _ in range(kf):
            P.apply_raw(U, Xf, out=Yf)
        b.record(stream)
        torch.cuda.synchronize()
        msf = a.elapsed_time(b) / kf
        out["fused_f32"] = {"vectors_per_s": N / (msf * 1e-3), "ms_per_call": msf,
                            "wy_speedup": (N / (ms_wall * 1e-3)) / (N / (msf * 1e-3))}
        del Xf, Yf
        Y = None

    # k-NN: the search kernel alone (transforms excluded), and the oracle on a
    # bounded sample of queries (every pair's distance by definition, sorted)
    if op == "knn":
        sq = torch.sqrt(lam)
        Zq = P.signed_raw("apply_T", U, Xq, d_out=sq)
        Zd = P.signed_raw("apply_T", U, X, d_out=sq)
        P.knn_raw(Zq, Zd, KNN_K)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kf = max(1, min(args.steps, 5))
        a.record(stream)
        for _ in range(kf):
            P.knn_raw(Zq, Zd, KNN_K)
        b.record(stream)
        torch.cuda.synchronize()
        msk = a.elapsed_time(b) / kf
        npad = (n + 3) // 4 * 4
        out["knn_kernel"] = {"ms_per_call": msk, "queries": KNN_QUERIES, "database": N, "k": KNN_K,
                             "tflops_products": 2 * npad * KNN_QUERIES * N / (msk * 1e-3) / 1e12}
        if not args.no_cpu:
            import oracle
            Uh, lh = U.double().cpu().numpy(), lam.double().cpu().numpy()
            S = 8
            xq, xd = Xq[:S].double().cpu().numpy(), X.double().cpu().numpy()
            t = time.perf_counter()
            Dh = oracle.mahal(Uh, lh, np.repeat(xq, N, axis=0), np.tile(xd, (S, 1))).reshape(S, N)
            ref = np.sort(Dh, axis=1)[:, :KNN_K]
            tcpu = time.perf_counter() - t
            dg, _ = P.knn(U, lam, Xq[:S], X, KNN_K)
            dg = dg.double().cpu().numpy()
            out["cpu_baseline"] = {"value": S / tcpu, "unit": "queries/s", "cores": oracle.num_threads(),
                                   "kind": "oracle",
                                   "sample": f"first {S} of {KNN_QUERIES} queries against all {N} "
                                             "database vectors, FP64, all pairs then sort"}
            out["max_rel_err_sample"] = float(np.max(np.abs(dg - ref) / ref))

    # the same reflectors through the dense kernels, timed beside
    if op == "apply_qr":
        P.apply_raw(U, X, out=Y, algo="fused")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kf = max(1, min(args.steps, 5))
        a.record(stream)
        for _ in range(kf):
            P.apply_raw(U, X, out=Y, algo="fused")
        b.record(stream)
        torch.cuda.synchronize()
        msd = a.elapsed_time(b) / kf
        out["dense_kernels"] = {"ms_per_call": msd, "vectors_per_s": N / (msd * 1e-3),
                                "skip_speedup": msd / ms_wall}

    # accuracy on a sample of vectors, and the oracle's own speed on it
    if not args.no_cpu and op in ("apply_fb", "sym_fb"):
        import oracle
        Uh = U.double().cpu().numpy()
        lh = lam.double().cpu().numpy()
        S = min(N, 256)
        Xs, Gs = X[:S], Gd[:S]
        if op == "apply_fb":
            Yg, rg = P.apply_raw(U, Xs, compute=tdt, save=True)
            dXg, dUg = P.apply_bwd_raw(U, Xs, Gs, compute=tdt, saved=rg)
        else:
            Yg, rg = P.sym_raw(U, lam, Xs, compute=tdt, save=True)
            dXg, dUg, dlg = P.sym_bwd_raw(U, lam, Xs, Gs, compute=tdt, saved=rg)
        torch.cuda.synchronize()
        xh, gh = Xs.double().cpu().numpy(), Gs.double().cpu().numpy()
        t = time.perf_counter()
        if op == "apply_fb":
            ry = oracle.apply(Uh, xh)
            rdx, rdu = oracle.apply_bwd(Uh, xh, gh)
        else:
            ry = oracle.sym(Uh, lh, xh)
            rdx, rdu, rdl = oracle.sym_bwd(Uh, lh, xh, gh)
        tcpu = time.perf_counter() - t

        def rr(a, b):
            a = a.double().cpu().numpy()
            return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))

        def rf(a, b):
            a = a.double().cpu().numpy()
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out["max_rel_err_sample"] = {"Y": rr(Yg, ry), "dX": rr(dXg, rdx), "dU": rf(dUg, rdu)}
        if op == "sym_fb":
            out["max_rel_err_sample"]["dlam"] = rf(dlg, rdl)
        out["cpu_baseline"] = {"value": S / tcpu, "unit": "vectors/s (forward + backward)",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"first {S} of {N} vectors of the same batch, FP64"}
    if not args.no_cpu and op in ("apply", "apply_qr", "sym", "sym_d", "mahal", "mahal_fb"):
        import oracle
        Uh = U.double().cpu().numpy()
        lh = lam.double().cpu().numpy()
        S = min(N, 64)
        Xs = X[:S].double().cpu().numpy()
        t = time.perf_counter()
        dh = dsig.double().cpu().numpy() if dsig is not None else None
        if op in ("apply", "apply_qr"):
            ref = oracle.apply(Uh, Xs)
        elif op == "sym":
            ref = oracle.sym(Uh, lh, Xs)
        elif op == "sym_d":
            ref = oracle.signed("sym", Uh, Xs, d_in=dh, d_out=dh, lam=lh)
        else:
            ref = oracle.mahal(Uh, lh, Xs, Xb[:S].double().cpu().numpy())
        t1 = time.perf_counter() - t
        # size a sample that takes about cpu_seconds
        S2 = int(min(N, max(S, S * args.cpu_seconds / max(t1, 1e-4))))
        Xs2 = X[:S2].double().cpu().numpy()
        t = time.perf_counter()
        if op in ("apply", "apply_qr"):
            oracle.apply(Uh, Xs2)
        elif op == "sym":
            oracle.sym(Uh, lh, Xs2)
        elif op == "sym_d":
            oracle.signed("sym", Uh, Xs2, d_in=dh, d_out=dh, lam=lh)
        elif op == "mahal":
            oracle.mahal(Uh, lh, Xs2, Xb[:S2].double().cpu().numpy())
        else:
            Xbs = Xb[:S2].double().cpu().numpy()
            oracle.mahal(Uh, lh, Xs2, Xbs)
            oracle.mahal_bwd(Uh, lh, Xs2, Xbs, w[:S2].double().cpu().numpy())
        tcpu = time.perf_counter() - t
        out["cpu_baseline"] = {"value": S2 / tcpu, "unit": "vectors/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"first {S2} of {N} vectors of the same batch, FP64"}
        if op in ("apply", "apply_qr", "sym", "sym_d"):
            Yg = (P.apply_raw(U, X[:S], compute=tdt) if op in ("apply", "apply_qr") else
                  P.sym_raw(U, lam, X[:S], compute=tdt) if op == "sym" else
                  P.signed_raw("sym", U, X[:S], d_in=dsig, d_out=dsig, lam=lam, compute=tdt)
                  ).double().cpu().numpy()
            err = float(np.max(np.linalg.norm(Yg - ref, axis=1) / np.linalg.norm(ref, axis=1)))
        else:
            dg = P.mahal_raw(U, lam, X[:S], Xb[:S]).double().cpu().numpy()
            err = float(np.max(np.abs(dg - ref) / np.abs(ref)))
        out["max_rel_err_sample"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
