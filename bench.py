#!/usr/bin/env python3
"""Throughput of the LRAMM hot path on one MI355X, at fixed accuracy.

A step is one full forward pass of the method over one batch of synthetic
input already resident in HBM: the seeded Gaussian test matrix and its codes,
the sketch, CholeskyQR2, the power iterations, the projection, every
quantisation (or bf16 rounding) and the two chained products (all stages of
the library's lramm_forward).

Default workload (the headline): A, B 8192 x 8192 bf16, A = U diag(sigma) V^T
with Haar U, V and sigma_i = exp(-i/64), B ~ N(0, 1); the fastest setting
(sketch width l = r + p, power iterations q, per-stage formats) whose
relative Frobenius error against the exact product of the bf16 inputs is at
most 1e-2, as found by ``--sweep``.  The same is reported for decay rates 128
and 256 (``other_decays``), next to the hand-written dense bf16 GEMM on the
same inputs and the dense bf16 roofline.

Prints ONE JSON line: effective 2 m n k / s, speedups, per-stage times (HIP
events on the launch stream in a second, instrumented region), the roofline
of the kernel with the largest share of the step, the error against the
exact FP64 product and against the FP64 oracle with the Eckart-Young floor,
and the oracle's own time on the host cores (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--tau 64] [--l 448 --q 0 --fmt bf16]
    python bench.py --sweep [--taus 64,128,256]     # the setting search
    python bench.py --workload at-scale             # 4096^3 FP32 int8 (throughput / parity workload)
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective 2MNK/s + speedup vs dense GEMM at fixed rel-Frobenius error (1 GPU)"
PEAK = {"int8": 5.0e15, "int4": 5.0e15, "fp8": 5.0e15, "bf16": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}
HBM = 8.0e12
TARGET_RELF = 1e-2

# Fastest setting per decay rate with rel-F <= 1e-2 on 8192^3 bf16, from
# ``bench.py --sweep`` (summary: profiles/target_8192_setting_sweep.md):
# (l, p, q, formats, test matrix, orthonormalisation).  None: no setting
# within l <= 1024 reaches 1e-2; the closest one is reported instead.
BEST = {
    64.0: (416, 32, 0, ("bf16",) * 4, "srht", "cholqr"),
    128.0: (896, 32, 0, ("bf16",) * 4, "srht", "cholqr"),
    256.0: None,
}
CLOSEST = {256.0: (1024, 32, 1, ("bf16",) * 4, "gaussian", "cholqr")}

SWEEP = {
    64.0: [256, 320, 384, 416, 448, 480, 512],
    128.0: [512, 640, 768, 896, 1024],
    256.0: [768, 896, 1024],
}
SWEEP_FMTS = {"bf16": ("bf16",) * 4, "int8_sketch": ("int8", "bf16", "bf16", "bf16"),
              "fp8": ("fp8",) * 4, "int8": ("int8",) * 4, "srht+bf16": (("bf16",) * 4, "srht"),
              "srht+fp8": (("fp8",) * 4, "srht"), "srht+bf16+1pass": (("bf16",) * 4, "srht", "cholqr"),
              "bf16+1pass": (("bf16",) * 4, "gaussian", "cholqr")}


def setting_parts(setting):
    """(l, p, q, formats, test matrix, orthonormalisation) of a setting tuple
    (the last two optional: "gaussian", "cholqr2")."""
    l, p, q, fmt = setting[:4]
    sketch = setting[4] if len(setting) > 4 else "gaussian"
    orth = setting[5] if len(setting) > 5 else "cholqr2"
    return l, p, q, fmt, sketch, orth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="target", choices=["target", "at-scale"])
    ap.add_argument("--tau", type=float, default=None, help="decay rate of sigma_i = exp(-i/tau)")
    ap.add_argument("--l", type=int, default=None, help="sketch width l = r + p (with --q and --fmt)")
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--q", type=int, default=None)
    ap.add_argument("--fmt", default=None, help="one format for every stage, or four comma-separated")
    ap.add_argument("--sketch", default=None, choices=["gaussian", "srht"],
                    help="test matrix of the first sketch (default: the setting's)")
    ap.add_argument("--orth", default=None, choices=["cholqr2", "cholqr"],
                    help="orthonormalisation: two Cholesky QR passes or one (default: the setting's)")
    ap.add_argument("--sweep", action="store_true", help="search (l, q, formats) per decay rate")
    ap.add_argument("--taus", default="64,128,256")
    ap.add_argument("--precision-sweep", action="store_true",
                    help="two-sided Alg. 3 budgets 888/884/844/444 against DQ8/DQ4 on uniform, exponential and "
                         "normal matrices (the paper's precision test)")
    ap.add_argument("--size", type=int, default=1024, help="matrix size of --precision-sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-other-decays", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="finish with one plain device copy of MIB MiB (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------ workloads --

def make_inputs(workload, tau, dev):
    """(A, B on the GPU, A and B as float64 host arrays, info) for a workload.
    info holds the spectrum of A's low-rank part in the units of A, the
    Frobenius norm of A and of the rounding or noise added to it."""
    import numpy as np
    import torch

    import synth
    t = time.time()
    if workload == "target":
        m = n = k = 8192
        A32, sigma = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, dtype="fp32")
        A_np = synth.to_dtype(A32, "bf16")
        B_np = synth.gaussian(k, n, 100, dtype="bf16")
        dt = torch.bfloat16
        pert = float(np.linalg.norm(A_np.astype(np.float64) - A32.astype(np.float64)))
        del A32
    else:
        m = n = k = 4096
        info0 = {}
        A_np, sigma = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, noise_var=1e-4, info=info0)
        B_np = synth.gaussian(k, n, 100)
        dt = torch.float32
        pert = info0["noise_fro"]
    log(f"inputs ({workload}, tau {tau:g}) generated in {time.time() - t:.1f}s")
    A = torch.from_numpy(A_np).to(dev).to(dt)
    B = torch.from_numpy(B_np).to(dev).to(dt)
    A64, B64 = A_np.astype(np.float64), B_np.astype(np.float64)
    info = {"sigma": sigma, "A_fro": float(np.linalg.norm(A64)), "perturbation_fro": pert, "dtype": dt}
    return A, B, A64, B64, info


def exact_product(A64, B64):
    t = time.time()
    C = A64 @ B64
    log(f"exact FP64 product in {time.time() - t:.1f}s")
    return C


def run_setting(lramm, A, B, setting, steps, warmup, seed=1, timing=False):
    """Time `steps` forwards of one setting; returns (ms per step, C, plan, ws)."""
    import torch
    l, p, q, fmt, sketch, orth = setting_parts(setting)
    m, k = A.shape
    n = B.shape[1]
    plan = lramm.LrammPlan(m, n, k, l - p, p, q, fmt, A.dtype, B.dtype, A.dtype, seed, exclusive=True,
                           sketch=sketch, orth=orth)
    ws = plan.workspace(A.device)
    C = torch.empty((m, n), dtype=A.dtype, device=A.device)
    for _ in range(warmup):
        plan.forward(A, B, ws, C=C)
    torch.cuda.synchronize()
    plan.status(ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(A, B, ws, C=C)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.status(ws)
    return ms, C, plan, ws


def rel_errors(C, Cex, nrm):
    import numpy as np
    Cg = C.double().cpu().numpy()
    d = Cg - Cex
    return float(np.linalg.norm(d) / nrm), float(np.max(np.abs(d))), Cg


def floors(info, r, l):
    """Eckart-Young floors of the low-rank part of A (relative to ||A||_F):
    sigma_{r+1}, the rank-r and rank-l tails; and the size of what was added
    to it (bf16 rounding or entrywise noise)."""
    import numpy as np
    s = np.sort(np.asarray(info["sigma"], np.float64))[::-1]
    a = info["A_fro"]
    return {"sigma_r1_rel": float(s[r] / a) if r < len(s) else 0.0,
            "tail_rank_r_rel": float(math.sqrt(float(np.sum(s[r:] ** 2))) / a),
            "tail_rank_l_rel": float(math.sqrt(float(np.sum(s[l:] ** 2))) / a),
            "perturbation_rel": info["perturbation_fro"] / a}


# ----------------------------------------------------- measurement work --

def stage_work(name, m, n, k, l, fmt, c_bytes, sketch="gaussian"):
    """Algorithmic work of ONE launch of a stage: (flops, bytes, peak key).

    GEMM: 2 M N K flops; bytes = each operand read once (1 byte per int8 /
    fp8 code, 1/2 for int4, 2 for bf16) and the output written once.
    Quantisers: the input read once and the codes written.  FP64
    orthonormalisation: the Gram rows * l * (l + 1) flops over its lower
    half; the Cholesky l^3 / 3 per factorisation (the unpadded l, no inverse);
    the solve and the second-pass product rows * l^2."""
    fs, fp, f1, f2 = fmt
    cb = {"int8": 1.0, "int4": 0.5, "fp8": 1.0, "bf16": 2.0}
    if name == "sketch_gemm" and sketch == "srht":
        # structured sketch: A read once (input dtype, c_bytes per element),
        # Y written; k' log2 k' additions per row
        kp = 1 << max(1, (k - 1).bit_length())
        return m * kp * math.log2(kp), m * k * c_bytes + m * l * 4.0, "fp32"
    if name in ("sketch_gemm", "power_gemm_Y"):
        return 2.0 * m * l * k, m * k * cb[fs] + l * k * cb[fs] + m * l * 4, fs
    if name == "power_gemm_Z":
        return 2.0 * k * l * m, k * m * cb[fp] + l * m * cb[fp] + k * l * 4, fp
    if name == "proj_gemm":
        return 2.0 * l * k * m, l * m * cb[fp] + k * m * cb[fp] + l * k * 4, fp
    if name == "g1_gemm":
        return 2.0 * n * l * k, n * k * cb[f1] + l * k * cb[f1] + n * l * 4, f1
    if name == "g2_gemm":
        return 2.0 * m * n * l, m * l * cb[f2] + n * l * cb[f2] + m * n * c_bytes, f2
    if name == "cholqr2.gram":
        return m * l * (l + 1.0), m * l * 6.0, "fp64"
    if name == "cholqr2.chol_panel":
        return l ** 3 / 3.0, l * l * 8.0, "fp64"
    if name in ("cholqr2.solve", "cholqr2.apply"):
        return m * l * float(l), m * l * (4.0 + 8.0), "fp64"
    return 0.0, 0.0, None


KERNEL_OF = {"sketch_gemm": "gemm_nt_kernel", "power_gemm_Z": "gemm_nt_kernel", "power_gemm_Y": "gemm_nt_kernel",
             "proj_gemm": "gemm_nt_kernel", "g1_gemm": "gemm_nt_kernel", "g2_gemm": "gemm_nt_kernel",
             "cholqr2.gram": "gram_kernel", "cholqr2.chol_panel": "chol_chain_kernel",
             "cholqr2.solve": "tsmul_kernel", "cholqr2.apply": "tsmul_kernel"}

# HBM bytes per launch of a kernel at the headline setting, from rocprofv3
# FETCH_SIZE / WRITE_SIZE passes scaled by the same counters on a plain
# device copy; reported only while the kernel's source is unchanged.
TRAFFIC = {"gemm_nt_kernel": ("profiles/target_8192_l416_srht_bf16_hbm_traffic.md",
                              "paper_2405_16917_amd/csrc/gemm_nt.hip")}


def measured_traffic(kernel):
    if kernel not in TRAFFIC:
        return None
    summary, src = (os.path.join(ROOT, x) for x in TRAFFIC[kernel])
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        fields = {}
        for line in open(summary):
            if ":" in line and line.strip().startswith((kernel + ".",)):
                key, val = line.split(":", 1)
                fields[key.strip()] = val.strip().strip("`")
        if fields.get(kernel + ".source_sha256") != digest:
            return None
        return float(fields[kernel + ".traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def roofline(stage_ms, m, n, k, l, fmt, c_bytes, sketch="gaussian"):
    """Roofline of the kernel with the largest time per step: its algorithmic
    work per launch over its average event-measured launch duration, against
    the MI355X peak of its bound (intensity against the ridge point of its
    dtype)."""
    per_kernel = {}
    for st, (ms, cnt) in stage_ms.items():
        kern = "srht_kernel" if (st == "sketch_gemm" and sketch == "srht") else KERNEL_OF.get(st)
        if kern is None or cnt <= 0:
            continue
        fl, by, pk = stage_work(st, m, n, k, l, fmt, c_bytes, sketch)
        e = per_kernel.setdefault(kern, {"ms": 0.0, "launches": 0.0, "flops": 0.0, "bytes": 0.0, "peak": pk})
        e["ms"] += ms
        e["launches"] += cnt
        e["flops"] += fl * cnt
        e["bytes"] += by * cnt
    out = {}
    for kern, e in per_kernel.items():
        launch_ms = e["ms"] / e["launches"]
        fl, by = e["flops"] / e["launches"], e["bytes"] / e["launches"]
        pk = e["peak"]
        if fl > 0 and fl / by >= PEAK[pk] / HBM:
            r = {"bound": "mfma", "achieved": fl / (launch_ms * 1e-3) / 1e12, "peak": PEAK[pk] / 1e12,
                 "unit": "TFLOP/s"}
        else:
            r = {"bound": "hbm", "achieved": by / (launch_ms * 1e-3) / 1e9, "peak": HBM / 1e9, "unit": "GB/s"}
        r["frac"] = r["achieved"] / r["peak"]
        r.update(kernel=kern, peak_dtype=pk, launch_ms=launch_ms, launches_per_step=e["launches"],
                 ms_per_step=e["ms"], flops_per_launch=fl, bytes_per_launch=by)
        out[kern] = r
    dom = max(out, key=lambda kk: out[kk]["ms_per_step"])
    top = dict(out[dom])
    tb = measured_traffic(dom)
    top["traffic"] = tb
    return top, out


# ------------------------------------------------------------- the runs --

def dense_bf16(lramm, A, B, reps=10):
    """The hand-written dense bf16 NT-GEMM on the same inputs (B transposed
    beforehand, outside the timing): ms per product and its C (FP32)."""
    import torch
    Bt = B.t().contiguous()
    m, n = A.shape[0], B.shape[1]
    Cd = torch.empty((m, n), dtype=torch.float32, device=A.device)
    for _ in range(2):
        lramm.lramm_dense_gemm_nt(A, Bt, Cd)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        lramm.lramm_dense_gemm_nt(A, Bt, Cd)
    e1.record()
    torch.cuda.synchronize()
    del Bt
    return e0.elapsed_time(e1) / reps, Cd


def dense_library(A, B, reps=10):
    """The vendor library's dense bf16 GEMM (torch.matmul, which calls
    hipBLASLt) on the same inputs, bf16 output: ms per product with B as
    stored (row-major, NN) and with B transposed beforehand outside the
    timing (NT).  A comparator only: no LRAMM stage calls it."""
    import torch
    out = {}
    for name, Bx in (("nn", B), ("nt", B.t().contiguous().t())):
        for _ in range(3):
            C = A @ Bx
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            C = A @ Bx
        e1.record()
        torch.cuda.synchronize()
        out[f"ms_{name}"] = e0.elapsed_time(e1) / reps
        del C, Bx
    out["ms"] = min(out["ms_nn"], out["ms_nt"])
    return out


def sweep(args, lramm, dev):
    import torch
    taus = [float(x) for x in args.taus.split(",")]
    best = {}
    for tau in taus:
        A, B, A64, B64, info = make_inputs("target", tau, dev)
        Cex = exact_product(A64, B64)
        import numpy as np
        nrm = float(np.linalg.norm(Cex))
        cands = []
        for l in SWEEP.get(tau, SWEEP[64.0]):
            for q in (0, 1):
                for fname, fmt in SWEEP_FMTS.items():
                    sk, orth = "gaussian", "cholqr2"
                    if isinstance(fmt[0], tuple):
                        fmt, sk, orth = (tuple(fmt) + ("cholqr2",))[:3]
                    setting = (l, 32, q, fmt, sk, orth)
                    try:
                        ms, C, plan, ws = run_setting(lramm, A, B, setting, 5, 2)
                    except lramm.LrammError as e:
                        print(json.dumps({"tau": tau, "l": l, "q": q, "fmt": fname, "error": str(e)}), flush=True)
                        continue
                    e, mx, _ = rel_errors(C, Cex, nrm)
                    row = {"tau": tau, "l": l, "q": q, "fmt": fname, "ms": round(ms, 4), "rel_fro": e, "max_abs": mx}
                    print(json.dumps(row), flush=True)
                    cands.append(row)
                    del plan, ws, C
                    torch.cuda.empty_cache()
        ok = [c for c in cands if c["rel_fro"] <= TARGET_RELF]
        # none within the target: the lowest error, the fastest among equal ones
        pick = min(ok, key=lambda c: c["ms"]) if ok else min(cands, key=lambda c: (c["rel_fro"], c["ms"]))
        best[tau] = dict(pick, reaches_target=bool(ok))
        del A, B, A64, B64, Cex
    print(json.dumps({"sweep_best": best}), flush=True)


def precision_sweep(args, lramm, dev):
    """The paper's precision test (Sec. 4, its Fig. 3) on seeded synthetic
    inputs: N x N matrices with i.i.d. entries U(0, 1), Exp(1) or N(0, 1);
    relative Frobenius error against the exact FP64 product of the two-sided
    method (RSVD in bf16, q = 0 as the paper chooses, p = 8) for each budget
    d1 d2 d3 and rank r, and of the direct quantised products DQ8 and DQ4."""
    import numpy as np
    import torch
    N = args.size
    rng_draw = {"uniform": lambda g, s: g.uniform(0.0, 1.0, s), "exponential": lambda g, s: g.exponential(1.0, s),
                "normal": lambda g, s: g.standard_normal(s)}
    budgets = {"888": ("int8", "int8", "int8"), "884": ("int8", "int8", "int4"), "844": ("int8", "int4", "int4"),
               "444": ("int4", "int4", "int4"), "bf16": ("bf16", "bf16", "bf16")}
    ranks = [r for r in (8, 16, 32, 48, 64, 96, 120) if r + 8 <= min(N, 128)]
    summary = {}
    for dist, draw in rng_draw.items():
        g0 = np.random.default_rng(1000 + len(dist))
        A_np = draw(g0, (N, N)).astype(np.float32)
        B_np = draw(g0, (N, N)).astype(np.float32)
        A, B = torch.from_numpy(A_np).to(dev), torch.from_numpy(B_np).to(dev)
        Cex = A_np.astype(np.float64) @ B_np.astype(np.float64)
        nrm = float(np.linalg.norm(Cex))
        row = {"dist": dist, "N": N}
        for name, fmt in (("DQ8", "int8"), ("DQ4", "int4")):
            Lq, dL = lramm.lramm_quantize(A, fmt)
            Rq, dR = lramm.lramm_quantize(B, fmt, transpose=True)
            C = lramm.lramm_gemm_nt(N, N, N, fmt, Lq, dL, Rq, dR)
            row[name] = float(np.linalg.norm(C.double().cpu().numpy() - Cex) / nrm)
        for r in ranks:
            for bname, d in budgets.items():
                plan = lramm.LrammTsPlan(N, N, N, r, 8, 0, ("bf16", "bf16"), d, seed=5)
                ws = plan.workspace(dev)
                C = plan.forward(A, B, ws)
                plan.status(ws)
                row[f"r{r}_{bname}"] = float(np.linalg.norm(C.double().cpu().numpy() - Cex) / nrm)
                del plan, ws, C
        print(json.dumps(row), flush=True)
        first = {}
        for bname in budgets:
            beat = [r for r in ranks if row[f"r{r}_{bname}"] < row["DQ4"]]
            first[bname] = beat[0] if beat else None
        summary[dist] = {"DQ8": row["DQ8"], "DQ4": row["DQ4"], "smallest_r_beating_DQ4": first}
    print(json.dumps({"precision_sweep_summary": summary, "ranks": ranks}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the library runs on one GPU, "
              "and its row-sharded multi-GPU form is designed but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2405_16917_amd as lramm

    lramm.load()
    lramm.lramm_init()
    dev = torch.device("cuda:0")
    if args.sweep:
        sweep(args, lramm, dev)
        return
    if args.precision_sweep:
        precision_sweep(args, lramm, dev)
        return

    if args.workload == "target":
        tau = 64.0 if args.tau is None else args.tau
        setting = BEST.get(tau) or CLOSEST.get(tau) or BEST[64.0]
    else:
        tau = 128.0 if args.tau is None else args.tau
        setting = (272, 16, 1, ("int8",) * 4)
    if args.l is not None:
        p = args.p if args.p is not None else setting[1]
        fmt = tuple(args.fmt.split(",")) if args.fmt and "," in args.fmt else ((args.fmt,) * 4 if args.fmt
                                                                                else setting[3])
        setting = (args.l, p, args.q if args.q is not None else setting[2], fmt) + setting_parts(setting)[4:]
    l, p, q, fmt, sketch, orth = setting_parts(setting)
    sketch = args.sketch or sketch
    orth = args.orth or orth
    setting = (l, p, q, fmt, sketch, orth)
    r = l - p

    A, B, A64, B64, info = make_inputs(args.workload, tau, dev)
    m, k = A.shape
    n = B.shape[1]
    c_bytes = 2 if A.dtype == torch.bfloat16 else 4
    seed = 1
    # timed region: K whole forward passes, no instrumentation
    ms_step, C, plan, ws = run_setting(lramm, A, B, setting, args.steps, args.warmup, seed)
    value = 2.0 * m * n * k / (ms_step * 1e-3) / 1e12
    log(f"LRAMM {ms_step:.3f} ms/step, effective {value:.1f} TFLOP/s")
    # second region with HIP events around every stage and every launch of
    # the orthonormalisation, recorded on the stream that launches them
    plan.stage_times()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(A, B, ws, C=C)
    torch.cuda.synchronize()
    ms_instr = (time.perf_counter() - t2) * 1e3 / args.steps
    plan.set_timing(False)
    stages = plan.stage_times()
    stage_ms = {kk: (v[0] / args.steps, v[1] / args.steps) for kk, v in stages.items() if v[1]}
    top, kernels = roofline(stage_ms, m, n, k, l, fmt, c_bytes, sketch)

    dtype = fmt[0] if len(set(fmt)) == 1 else "+".join(fmt)
    wl = (f"{'target' if args.workload == 'target' else 'at-scale'}: A,B {m}x{k}x{n} "
          f"{'bf16' if c_bytes == 2 else 'fp32'}, A = U diag(sigma) V^T, sigma_i = exp(-i/{tau:g})"
          f"{' + entrywise noise var 1e-4' if args.workload != 'target' else ''}, B ~ N(0,1); "
          f"l = {l} (r = {r}, p = {p}), q = {q}, formats {','.join(fmt)}, "
          f"{'structured (SRHT)' if sketch == 'srht' else 'Gaussian'} test matrix from Philox seed {seed}, "
          f"{'one Cholesky QR pass' if orth == 'cholqr' else 'CholeskyQR2'} per orthonormalisation")
    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "ms_per_step_instrumented": ms_instr,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic (seeded low-rank A with exponential singular-value decay, Gaussian B)",
        "config": {"workload": wl, "m": m, "n": n, "k": k, "tau": tau, "r": r, "p": p, "q": q, "l": l,
                   "formats": list(fmt), "sketch": sketch, "orth": orth,
                   "io": "bf16" if c_bytes == 2 else "fp32"},
        "stages_ms": {st: round(v[0], 5) for st, v in stage_ms.items()},
        "roofline": top,
        "kernels": kernels,
    }

    if orth == "cholqr" and not args.no_other_decays:
        # the same setting with CholeskyQR2, untimed by the line's value
        ms2q, C2q, plan2q, ws2q = run_setting(lramm, A, B, setting[:5] + ("cholqr2",), args.steps, args.warmup, seed)
        out["cholqr2_same_setting"] = {"ms_per_step": ms2q, "value": 2.0 * m * n * k / (ms2q * 1e-3) / 1e12}
        C2q_keep = C2q
        del plan2q, ws2q
    Cex = None
    if not args.no_error or not args.no_dense:
        Cex = exact_product(A64, B64)
    nrm = float(np.linalg.norm(Cex)) if Cex is not None else 1.0
    if not args.no_error:
        e, mx, Cg = rel_errors(C, Cex, nrm)
        out["error"] = {"rel_fro_vs_exact": e, "max_abs_vs_exact": mx, "max_abs_exact": float(np.max(np.abs(Cex))),
                        "target_rel_fro": TARGET_RELF, "meets_target": e <= TARGET_RELF}
        out["error"].update(floors(info, r, l))
        if "cholqr2_same_setting" in out:
            out["cholqr2_same_setting"]["rel_fro_vs_exact"] = rel_errors(C2q_keep, Cex, nrm)[0]
            out["error"]["rel_fro_one_pass_vs_cholqr2"] = float(
                np.linalg.norm(Cg - C2q_keep.double().cpu().numpy()) / nrm)
    del C, plan, ws
    torch.cuda.empty_cache()

    if not args.no_dense:
        dms, Cd = dense_bf16(lramm, A if A.dtype == torch.bfloat16 else A.to(torch.bfloat16),
                             B if B.dtype == torch.bfloat16 else B.to(torch.bfloat16))
        ed, _, _ = rel_errors(Cd, Cex, nrm)
        del Cd
        roof_ms = 2.0 * m * n * k / PEAK["bf16"] * 1e3
        out["dense_bf16"] = {"ms": dms, "tflops": 2.0 * m * n * k / (dms * 1e-3) / 1e12,
                             "frac_peak": 2.0 * m * n * k / (dms * 1e-3) / PEAK["bf16"], "rel_fro_vs_exact": ed,
                             "roofline_ms": roof_ms}
        out["speedup_vs_dense_bf16"] = dms / ms_step
        out["speedup_vs_dense_bf16_roofline"] = roof_ms / ms_step
        lib_d = dense_library(A if A.dtype == torch.bfloat16 else A.to(torch.bfloat16),
                              B if B.dtype == torch.bfloat16 else B.to(torch.bfloat16))
        lib_d["tflops"] = 2.0 * m * n * k / (lib_d["ms"] * 1e-3) / 1e12
        out["dense_bf16_library"] = lib_d
        out["speedup_vs_dense_bf16_library"] = lib_d["ms"] / ms_step
        log(f"dense bf16: own kernel {dms:.3f} ms, library {lib_d['ms']:.3f} ms "
            f"(NN {lib_d['ms_nn']:.3f}, NT {lib_d['ms_nt']:.3f})")

    if args.workload == "target" and not args.no_other_decays and args.tau is None and args.l is None:
        others = {}
        for t2_ in (128.0, 256.0):
            st = BEST.get(t2_)
            reach = st is not None
            st = st or CLOSEST[t2_]
            A2, B2, A2_64, B2_64, info2 = make_inputs("target", t2_, dev)
            ms2, C2, plan2, ws2 = run_setting(lramm, A2, B2, st, max(5, args.steps // 4), 2, seed)
            Cex2 = exact_product(A2_64, B2_64)
            e2, mx2, _ = rel_errors(C2, Cex2, float(np.linalg.norm(Cex2)))
            row = {"l": st[0], "p": st[1], "q": st[2], "formats": list(st[3]),
                   "sketch": setting_parts(st)[4], "orth": setting_parts(st)[5], "ms_per_step": ms2,
                   "value": 2.0 * m * n * k / (ms2 * 1e-3) / 1e12, "rel_fro_vs_exact": e2, "max_abs_vs_exact": mx2,
                   "reaches_target": reach and e2 <= TARGET_RELF}
            row.update(floors(info2, st[0] - st[1], st[0]))
            if "dense_bf16" in out:
                row["speedup_vs_dense_bf16"] = out["dense_bf16"]["ms"] / ms2
                row["speedup_vs_dense_bf16_roofline"] = out["dense_bf16"]["roofline_ms"] / ms2
                row["speedup_vs_dense_bf16_library"] = out["dense_bf16_library"]["ms"] / ms2
            others[f"tau={t2_:g}"] = row
            del A2, B2, A2_64, B2_64, C2, plan2, ws2, Cex2
            torch.cuda.empty_cache()
        out["other_decays"] = others

    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info, threadpool_limits

        from oracle import lramm as OL
        cores = len(os.sched_getaffinity(0))
        with threadpool_limits(limits=cores):
            used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
            t = time.time()
            ref = OL.lramm_forward(A64, B64, r, p, q, fmt, seed=seed, keep=False, sketch=sketch,
                                   one_pass=orth == "cholqr")
            dt = time.time() - t
        out["cpu_baseline"] = {"value": 2.0 * m * n * k / dt / 1e12, "unit": "TFLOP/s", "cores": used,
                               "kind": "oracle", "seconds": dt,
                               "sample": f"one whole oracle forward of the same workload and setting "
                                         f"({m}x{k}x{n}, l={l}, q={q}, {','.join(fmt)}) in FP64 numpy"}
        if "error" in out:
            Cg32 = Cg.astype(np.float32).astype(np.float64) if c_bytes == 4 else Cg
            refC = ref["C"] if c_bytes == 4 else synth_bf16(ref["C"])
            d = Cg32 - refC
            out["error"]["rel_fro_vs_oracle"] = float(np.linalg.norm(d) / np.linalg.norm(refC))
            out["error"]["max_abs_vs_oracle"] = float(np.max(np.abs(d)))
        log(f"oracle {dt:.1f}s on {used} threads")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    print(json.dumps(out), flush=True)


def synth_bf16(X):
    import synth
    return synth.to_dtype(X, "bf16").astype("float64")


if __name__ == "__main__":
    main()
