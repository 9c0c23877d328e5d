#!/usr/bin/env python3
"""Throughput of the LRAMM hot path on one MI355X.

A step is one full forward pass of the method over one batch of synthetic
input that is already resident in HBM: quantisation of A and B, the seeded
Gaussian test matrix, the sketch, CholeskyQR2, the power iterations, the
projection and the two quantised products (all stages of the library's
lramm_forward).  Default workload: A, B 4096 x 4096 FP32, A with singular
values exp(-i/128) plus entrywise noise of variance 1e-4 (relative to unit-RMS
entries), B ~ N(0, 1); r = 256, p = 16, q = 1, int8 in every stage.

Prints ONE JSON line: effective 2 m n k / s, per-stage times (HIP events on
the launch stream inside the timed region), the roofline of the dominant
kernel, the dense bf16 / fp32 comparators on the same GPU, the error against
the exact FP64 product and against the FP64 oracle, and the oracle's own
time on the host cores (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--r 256] [--q 1] [--fmt int8]
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective 2MNK/s + speedup vs dense GEMM at fixed rel-Frobenius error (1 GPU)"
PEAK = {"int8": 5.03e15, "int4": 5.03e15, "bf16": 2.52e15, "fp32": 157.3e12, "fp64": 78.6e12}
HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=4096)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--k", type=int, default=4096)
    ap.add_argument("--r", type=int, default=256)
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--tau", type=float, default=128.0)
    ap.add_argument("--noise", type=float, default=1e-4)
    ap.add_argument("--fmt", default="int8", help="one format for every stage, or four comma-separated")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="finish with one plain device copy of MIB MiB (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Stages whose timed region is one kernel launch (the roofline is reported
# for the dominant one); composite stages (the whole orthonormalisation,
# column quantisers with their max / quantise / scale kernels) are excluded.
SINGLE_KERNEL = ("sketch_gemm", "power_gemm_Z", "power_gemm_Y", "proj_gemm", "g1_gemm", "g2_gemm",
                 "quant_A_rows", "quant_Bt_rows", "quant_Q_rows", "quant_Tt_rows", "cholqr2.gram",
                 "cholqr2.chol_panel", "cholqr2.solve", "cholqr2.series", "cholqr2.apply")


# HBM bytes per launch of the dominant kernel, from two rocprofv3 counter
# passes (FETCH_SIZE, WRITE_SIZE) of this bench's default workload, scaled by
# the same counters on a plain device copy; recorded with a hash of the
# kernel's source file and reported only while that file is unchanged.
TRAFFIC = {"cholqr2.chol_panel": ("profiles/chol_panel_4096_r256_q1_int8_hbm_traffic.md",
                                  "paper_2405_16917_amd/csrc/cholqr.hip")}


def measured_traffic(stage):
    if stage not in TRAFFIC:
        return None
    summary, src = (os.path.join(ROOT, x) for x in TRAFFIC[stage])
    try:
        import hashlib
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        fields = {}
        for line in open(summary):
            if ":" in line and line.strip().startswith(("source_sha256", "traffic_bytes_per_launch")):
                key, val = line.split(":", 1)
                fields[key.strip()] = val.strip().strip("`")
        if fields.get("source_sha256") != digest:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def stage_work(name, m, n, k, l, fmt, q):
    """Algorithmic work of ONE launch of a stage: (ops, bytes, peak key).

    GEMM ops count 2 M N K; bytes count each operand read once and the
    output written once.  Quantiser bytes count the FP input read once and
    the codes written.  FP64 orthonormalisation (rows = m = k here, l' = l
    rounded up to 32): Gram rows * l * (l + 1) flops (symmetric) reading X
    once; Cholesky plus block inverse 2 l'^3 / 3 flops per factorisation
    (split over its launches by the caller); the two solve products rows * l^2 flops (triangular factor)
    reading X and writing Q; the expansion 2 l^3 flops."""
    fs, fp, f1, f2 = fmt
    cb = {"int8": 1.0, "int4": 0.5, "bf16": 2.0}
    lw = (l + 31) // 32 * 32
    rows = m
    if name in ("sketch_gemm", "power_gemm_Y"):
        return 2.0 * m * l * k, m * k * cb[fs] + l * k * cb[fs] + m * l * 4, fs
    if name == "power_gemm_Z":
        return 2.0 * k * l * m, k * m * cb[fp] + l * m * cb[fp] + k * l * 4, fp
    if name == "proj_gemm":
        return 2.0 * l * k * m, l * m * cb[fp] + k * m * cb[fp] + l * k * 4, fp
    if name == "g1_gemm":
        return 2.0 * n * l * k, n * k * cb[f1] + l * k * cb[f1] + n * l * 4, f1
    if name == "g2_gemm":
        return 2.0 * m * n * l, m * l * cb[f2] + n * l * cb[f2] + m * n * 4, f2
    if name == "quant_A_rows":
        return 0.0, m * k * 4 + m * k * cb[fs], None
    if name == "quant_Bt_rows":
        return 0.0, l * k * 4 + l * k * cb[f1], None
    if name == "quant_Q_rows":
        return 0.0, m * l * 8 + m * l * cb[f2], None
    if name == "quant_Tt_rows":
        return 0.0, n * l * 4 + n * l * cb[f2], None
    if name == "cholqr2.gram":          # average over the FP32 (Y) and FP64 (Q1) inputs
        return rows * l * (l + 1.0), rows * l * 6.0, "fp64"
    if name == "cholqr2.chol_panel":
        # one Cholesky + block inverse (l'^3/3 + l'^3/3 flops; G's lower half
        # read once, L's and L^-1's lower halves written once); the caller
        # divides by the launches per Cholesky it measured (one for the
        # one-launch chain)
        return 2.0 * lw ** 3 / 3.0, 1.5 * lw * lw * 8, "fp64"
    if name in ("cholqr2.solve", "cholqr2.apply"):
        return rows * l * float(l), rows * l * (4.0 + 8.0), "fp64"
    if name == "cholqr2.series":
        return 2.0 * l ** 3, 2.0 * lw * lw * 8, "fp64"
    return 0.0, 0.0, None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the multi-GPU path is a "
              "design in DESIGN.md and is not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2405_16917_amd as lramm
    import synth

    lramm.load()
    lramm.lramm_init()
    m, n, k, r, p, q = args.m, args.n, args.k, args.r, args.p, args.q
    l = r + p
    fmt = tuple(args.fmt.split(",")) if "," in args.fmt else (args.fmt,) * 4
    dev = torch.device("cuda:0")

    t = time.time()
    A_np, sigma = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), args.tau), 0, noise_var=args.noise)
    B_np = synth.gaussian(k, n, 100)
    log(f"inputs generated in {time.time() - t:.1f}s")
    A = torch.from_numpy(A_np).to(dev)
    B = torch.from_numpy(B_np).to(dev)
    seed = 1

    plan = lramm.LrammPlan(m, n, k, r, p, q, fmt, torch.float32, torch.float32, torch.float32, seed)
    ws = plan.workspace(dev)
    C = torch.empty((m, n), dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        plan.forward(A, B, ws, C=C)
    torch.cuda.synchronize()
    plan.status(ws)
    # timed region: K whole forward passes, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(A, B, ws, C=C)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags = plan.status(ws)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = 2.0 * m * n * k / (ms_step * 1e-3) / 1e12
    log(f"LRAMM {ms_step:.3f} ms/step, effective {value:.1f} TFLOP/s, flags {flags}")
    # second timed region of K passes with HIP events around every stage and
    # every launch of the orthonormalisation, recorded on the launch stream
    plan.stage_times()                          # clear anything recorded so far
    plan.set_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(A, B, ws, C=C)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    plan.set_timing(False)
    stages = plan.stage_times()
    ms_step_instr = (t3 - t2) * 1e3 / args.steps

    stage_ms = {kk: (v[0] / args.steps, v[1] / args.steps) for kk, v in stages.items() if v[1]}
    # roofline of the dominant single-kernel stage
    cand = [st for st in stage_ms if st in SINGLE_KERNEL]
    dom = max(cand, key=lambda st: stage_ms[st][0])
    ops, byt, pk = stage_work(dom, m, n, k, l, fmt, q)
    per_launch_ms = stage_ms[dom][0] / max(1e-9, stage_ms[dom][1])
    if dom == "cholqr2.chol_panel":
        # work per Cholesky -> per launch: 1 + 2q Cholesky factorisations per forward
        per_chol = stage_ms[dom][1] / (1 + 2 * q)
        ops, byt = ops / per_chol, byt / per_chol
    if pk is not None and ops > 0 and (ops / byt) >= PEAK[pk] / HBM:
        roof = {"bound": "mfma", "achieved": ops / (per_launch_ms * 1e-3) / 1e12, "peak": PEAK[pk] / 1e12,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": byt / (per_launch_ms * 1e-3) / 1e9, "peak": HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom)
    roof["kernel"] = dom
    roof["peak_dtype"] = pk
    roof["launch_ms"] = per_launch_ms
    roof["launches_per_step"] = stage_ms[dom][1]

    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "ms_per_step_instrumented": ms_step_instr,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": fmt[0] if len(set(fmt)) == 1 else "+".join(fmt), "data": "synthetic",
        "config": {"workload": f"plain LRAMM at scale: A,B {m}x{k}x{n} FP32, sigma_i=exp(-i/{args.tau:g}) + "
                               f"noise var {args.noise:g}, B~N(0,1); r={r} p={p} q={q}, formats {','.join(fmt)}, "
                               "seeded Philox Omega",
                   "m": m, "n": n, "k": k, "r": r, "p": p, "q": q, "l": l, "formats": list(fmt)},
        "stages_ms": {st: round(v[0], 5) for st, v in stage_ms.items()},
        "roofline": roof,
    }

    if not args.no_dense:
        Ab, Btb = A.to(torch.bfloat16), B.t().contiguous().to(torch.bfloat16)
        Bt32 = B.t().contiguous()
        Cd = torch.empty((m, n), dtype=torch.float32, device=dev)
        dense = {}
        for name, (L, R) in {"bf16": (Ab, Btb), "fp32": (A, Bt32)}.items():
            for _ in range(2):
                lramm.lramm_dense_gemm_nt(L, R, Cd)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record()
            for _ in range(reps):
                lramm.lramm_dense_gemm_nt(L, R, Cd)
            e1.record()
            torch.cuda.synchronize()
            dms = e0.elapsed_time(e1) / reps
            entry = {"ms": dms, "tflops": 2.0 * m * n * k / (dms * 1e-3) / 1e12}
            entry["frac_peak"] = entry["tflops"] * 1e12 / PEAK[name]
            if not args.no_error:
                entry["Cd"] = Cd.double().cpu().numpy()
            dense[name] = entry
        out["dense"] = dense
        out["speedup_vs_dense_bf16"] = dense["bf16"]["ms"] / ms_step
        out["speedup_vs_dense_fp32"] = dense["fp32"]["ms"] / ms_step
        out["speedup_vs_bf16_roofline"] = (2.0 * m * n * k / PEAK["bf16"] * 1e3) / ms_step

    Cg = C.double().cpu().numpy()
    if not args.no_error:
        t = time.time()
        A64 = A_np.astype(np.float64)
        B64 = B_np.astype(np.float64)
        Cex = A64 @ B64
        nrm = np.linalg.norm(Cex)
        err = {"rel_fro_vs_exact": float(np.linalg.norm(Cg - Cex) / nrm),
               "max_abs_vs_exact": float(np.max(np.abs(Cg - Cex))),
               "sigma_next": float(sigma[l]) if l < len(sigma) else 0.0,
               "tail_rank_l": float(math.sqrt(float(np.sum(sigma[l:] ** 2))))}
        if "dense" in out:
            for name in ("bf16", "fp32"):
                Cd = out["dense"][name].pop("Cd")
                out["dense"][name]["rel_fro_vs_exact"] = float(np.linalg.norm(Cd - Cex) / nrm)
        out["error"] = err
        log(f"errors computed in {time.time() - t:.1f}s")
    elif "dense" in out:
        for name in ("bf16", "fp32"):
            out["dense"][name].pop("Cd", None)

    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info, threadpool_limits

        from oracle import lramm as OL
        cores = len(os.sched_getaffinity(0))
        with threadpool_limits(limits=cores):
            used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
            t = time.time()
            ref = OL.lramm_forward(A_np.astype(np.float64), B_np.astype(np.float64), r, p, q, fmt, seed=seed,
                                   keep=False)
            dt = time.time() - t
        out["cpu_baseline"] = {"value": 2.0 * m * n * k / dt / 1e12, "unit": "TFLOP/s", "cores": used,
                               "kind": "oracle", "seconds": dt,
                               "sample": f"one full oracle forward of the same workload ({m}x{k}x{n}, r={r}, "
                                         f"p={p}, q={q}, {','.join(fmt)}) in FP64 numpy"}
        out.setdefault("error", {})["rel_fro_vs_oracle"] = float(OL.rel_fro(Cg, ref["C"]))
        log(f"oracle {dt:.1f}s on {used} threads; GPU vs oracle rel-F {out['error']['rel_fro_vs_oracle']:.2e}")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
