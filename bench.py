#!/usr/bin/env python3
"""FP64 randUTV throughput on one MI355X.

One step = one full randUTV factorization A = U T V^T (U and V built) of the
12000 x 12000 matrix A = P diag(0.99^i) Q^T (P, Q Haar), block size b = 256,
q = 2 power steps, sketch seed 0 -- every block step of the method (sketch,
power iteration, QR of the sketch, right transform of all rows and of V, panel
QR, left transform, U update, b x b SVDs and their applications) runs inside
the timed region; A, U, T, V are resident in HBM before it starts, and nothing
but the factorizations runs inside it (no event records).

value = F_std / t in TFLOP/s, with the leading-order count
F_std = (1+2q)(m n^2 - n^3/3) + 2 m n^2 + 4/3 n^3 + 4 m^2 n  (1.843e13 here).

The roofline entry is the dominant kernel, the FP64 matrix-core GEMM (all its
operand layouts): its algorithmic flops per launch over its average launch
duration, from HIP events recorded on the launching stream around every GEMM
launch of one more factorization in which each GEMM launch runs alone on the
chip (the library waits for all queued work before it), so that the duration
is the kernel's own and not a share of a chip that the other streams' kernels
occupy as well.  The same figure with the streams overlapping, as they do in
the timed steps, is reported as roofline.in_place.  The roofline is refused
(null, with the reason) when the GEMM launches of one factorization, run
alone, take longer in total than a timed step.  traffic is the HBM bytes per
launch from committed rocprofv3 counters when they were taken on the current
kernel source.  cpu_baseline times the FP64 CPU oracle on the first block
steps of the same problem.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=12000)
    ap.add_argument("--n", type=int, default=12000)
    ap.add_argument("--b", type=int, default=256)
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--spectrum", default="exp")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="block steps of the same problem timed for the CPU oracle baseline (0: skip)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the factorizations after the timed region that time the kernels")
    ap.add_argument("--roofline-pass-only", action="store_true",
                    help="run only the warmup and the factorization whose GEMM launches run alone "
                         "(for a profiler run that measures the same launches)")
    ap.add_argument("--mixed-modes", default="sk32,sk48,sk16,sk32_up32,sk48_up32",
                    help="reduced-precision modes timed beside the FP64 run: skNN = sketch products "
                         "in NN bits (32 FP32, 48 split BF16 x3, 16 BF16), upNN = compact-WY updates too")
    ap.add_argument("--mixed-sizes", default="12000,16000",
                    help="square sizes of the mixed-precision comparison (FP64 and each mode)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the runs beside the FP64 headline: the reduced-precision modes, "
                         "the differentiable truncation and HQRRP")
    ap.add_argument("--ooc-n", type=int, default=12000,
                    help="size of the out-of-core run (0: skip)")
    ap.add_argument("--ooc-budget-gib", type=float, default=1.0,
                    help="HBM tile cache of the out-of-core run")
    ap.add_argument("--grad-batch", type=int, default=16,
                    help="matrices of the differentiable-truncation run (2048 x 2048, b=128; 0: skip)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the residual/orthogonality check of the timed output (profiler runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the factorizations, run one plain device copy of this many MiB "
                         "(a kernel of known HBM traffic, to scale hardware byte counters)")
    return ap.parse_args()


MODES = {"sk32": (32, 64), "sk48": (48, 64), "sk16": (16, 64), "sk32_up32": (32, 32),
         "sk48_up32": (48, 32), "sk32_up48": (32, 48)}
MODE_TEXT = {32: "fp32 matrix cores", 48: "bf16 matrix cores, split operands hi*hi + hi*lo + lo*hi",
             16: "bf16 matrix cores", 64: "fp64 matrix cores"}


def traffic_entry(kernel: str, launches: int):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary, if one exists for the current kernel source and the same launch
    list (launches per factorization; else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        import hashlib

        with open(path) as f:
            rec = json.load(f)
        src = os.path.join(ROOT, "paper_2002_06960_amd", "csrc", rec["source"])
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if digest != rec["sha256"] or rec.get("kernel") != kernel:
            return None
        if rec.get("launches_per_factorization") != launches:
            return None
        return rec["bytes_per_launch"]
    except Exception:
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stream_summary(trace):
    """Busy and idle time of each library stream in one factorization, from
    the per-launch record (overlapping launches of a stream counted once)."""
    if not trace:
        return None
    span = max(t0 + d for _, _, t0, d in trace) - min(t0 for _, _, t0, _ in trace)
    out = {"span_ms": round(span, 3)}
    for name in ("T", "P", "UV", "S"):
        iv = sorted((t0, t0 + d) for _, sname, t0, d in trace if sname == name)
        busy, end = 0.0, None
        for a, b in iv:
            if end is None or a >= end:
                busy += b - a
                end = b
            elif b > end:
                busy += b - end
                end = b
        out[name] = {"launches": len(iv), "busy_ms": round(busy, 3),
                     "idle_ms": round((iv[-1][1] - iv[0][0] - busy) if iv else 0.0, 3)}
    return out


def gemm_totals(stats):
    gemm = [k for k in stats if k.startswith("dgemm_") and stats[k][0]]
    return (sum(stats[k][0] for k in gemm), sum(stats[k][1] for k in gemm),
            sum(stats[k][2] for k in gemm))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the factorization has "
                                   "no multi-GPU path (use --gpus 1)"}))
        sys.exit(2)
    import torch

    import paper_2002_06960_amd as pkg
    from randutv_inputs import make_matrix_device

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    pkg.load()  # fails loudly without the HIP library
    m, n, b, q = args.m, args.n, args.b, args.q
    dev = "cuda:0"
    A = make_matrix_device(args.spectrum, m, n, seed=0, device=dev)
    U = pkg.colmajor_empty(m, m, dev)
    T = pkg.colmajor_empty(m, n, dev)
    V = pkg.colmajor_empty(n, n, dev)
    if args.copy_calibration_mib > 0:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"# copy calibration: {nel * 8} bytes read, {nel * 8} bytes written")
        del src, dst
    torch.cuda.synchronize()
    log(f"# workload randutv fp64 {m}x{n} b={b} q={q} spectrum={args.spectrum}")

    def factor(**kw):
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V, **kw)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        factor()
        torch.cuda.synchronize()
        log(f"# warmup {w}: {time.perf_counter() - t0:.3f} s")

    if args.roofline_pass_only:
        pkg.randutv_set_timing(True, serialize_gemm=True)
        factor()
        torch.cuda.synchronize()
        st = pkg.randutv_kernel_stats()
        by = pkg.randutv_kernel_bytes()
        pkg.randutv_set_timing(False)
        la, ms, fl = gemm_totals(st)
        gb = sum(v for k, v in by.items() if k.startswith("dgemm_"))
        log(f"# GEMM launches run alone: {la} launches, {ms:.3f} ms, {ms / la:.4f} ms per launch, "
            f"{fl / (ms * 1e-3) / 1e12:.3f} TFLOP/s, algorithmic bytes {gb / la:.4g} per launch")
        return

    # ---- timed region: the factorizations alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        factor()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / max(args.steps, 1)
    log(f"# timed {args.steps} steps: {ms_step:.2f} ms/step")

    # ---- kernel timing, after the timed region: (1) HIP events around every
    # GEMM launch with the streams overlapping as in the timed steps; (2) every
    # GEMM launch alone on the chip; (3) every kernel class (per-class table)
    stats_inplace = stats_alone = cls_stats = bytes_alone = {}
    trace = []
    if not args.no_kernel_timing:
        pkg.randutv_set_timing(True, gemm_only=True)
        factor()
        torch.cuda.synchronize()
        stats_inplace = pkg.randutv_kernel_stats()
        pkg.randutv_set_timing(True, serialize_gemm=True)
        t1 = time.perf_counter()
        factor()
        torch.cuda.synchronize()
        log(f"# factorization with every GEMM launch alone: {time.perf_counter() - t1:.3f} s")
        stats_alone = pkg.randutv_kernel_stats()
        bytes_alone = pkg.randutv_kernel_bytes()
        pkg.randutv_set_timing(True)
        factor()
        torch.cuda.synchronize()
        cls_stats = pkg.randutv_kernel_stats()
        trace = pkg.randutv_kernel_trace()
        pkg.randutv_set_timing(False)

    F = pkg.flops_std(m, n, q)
    value = F / (ms_step * 1e-3) / 1e12

    # correctness of the timed output
    res = orth_u = orth_v = None
    nA = torch.linalg.norm(A)
    if not args.no_check:
        res = (torch.linalg.norm(A - U @ T @ V.T) / nA).item()
        eye_m = torch.eye(m, dtype=torch.float64, device=dev)
        orth_u = (U.T @ U - eye_m).abs().max().item()
        del eye_m
        eye_n = torch.eye(n, dtype=torch.float64, device=dev)
        orth_v = (V.T @ V - eye_n).abs().max().item()
        del eye_n

    # ---- the same factorization in reduced-precision modes, at the headline
    # size and at 16000 x 16000: errors against the FP64 factorization of the
    # same matrix (which the GPU tests pin to the FP64 oracle)
    mixed = None
    if not args.no_mixed:
        mixed = {}
        for size in [int(x) for x in args.mixed_sizes.split(",") if x]:
            mixed[f"{size}x{size}"] = mixed_block(pkg, torch, size, b, q, args, dev,
                                                  (A, U, T, V, ms_step) if (size == m == n) else None)

    trunc_grad = None
    if args.grad_batch > 0 and not args.no_mixed:
        trunc_grad = truncation_grad_block(pkg, torch, args, dev)

    ooc = None
    if args.ooc_n > 0 and not args.no_mixed:
        ooc = ooc_block(pkg, torch, args, dev)

    # HQRRP (randomized blocked column-pivoted QR) of the same matrix, block b
    hq = None
    if not args.no_mixed:
        pkg.randutv_hqrrp(A, b, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fh, tauh, jph = pkg.randutv_hqrrp(A, b, 0)
        torch.cuda.synchronize()
        ms_hq = 1e3 * (time.perf_counter() - t0)
        f_qr = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
        del Fh, tauh, jph
        # the unpivoted blocked Householder QR of the same matrix (the same
        # step loop without the sketch, the pivots and the exchanges)
        pkg.randutv_geqrf_blocked(A, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fq, tauq = pkg.randutv_geqrf_blocked(A, b)
        torch.cuda.synchronize()
        ms_qr = 1e3 * (time.perf_counter() - t0)
        del Fq, tauq
        hq = {"workload": f"hqrrp {m}x{n} b={b}, FP64", "ms": round(ms_hq, 3),
              "qr_flops": f_qr, "tflops_qr_count": round(f_qr / (ms_hq * 1e-3) / 1e12, 3),
              "unpivoted_blocked_qr_ms": round(ms_qr, 3), "ratio_to_unpivoted": round(ms_hq / ms_qr, 3)}
        log(f"# hqrrp: {ms_hq:.2f} ms; unpivoted blocked QR of the same matrix {ms_qr:.2f} ms")

    roofline = None
    refused = None
    kern = {}
    if stats_alone:
        for name, (launches, ms, fl) in cls_stats.items():
            if launches:
                kern[name] = {"launches": launches, "ms_per_step": ms,
                              "tflops": (fl / (ms * 1e-3) / 1e12) if ms > 0 and fl > 0 else None}
        la, ms_alone, fl = gemm_totals(stats_alone)
        li, ms_in, fli = gemm_totals(stats_inplace)
        achieved = fl / (ms_alone * 1e-3) / 1e12
        if ms_alone > ms_step:
            refused = (f"the GEMM launches of one factorization take {ms_alone:.1f} ms run alone, "
                       f"more than the {ms_step:.1f} ms step")
        else:
            roofline = {"bound": "mfma", "kernel": "dgemm_mfma_kernel", "achieved": round(achieved, 3),
                        "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                        "traffic": traffic_entry("dgemm_mfma_kernel", la),
                        "avg_launch_ms": ms_alone / la, "launches": la, "flops_per_launch": fl / la,
                        "algorithmic_bytes_per_launch": sum(v for k, v in bytes_alone.items()
                                                            if k.startswith("dgemm_")) / la,
                        "timing": "every GEMM launch of one factorization run alone (HIP events on "
                                  "the launching stream)",
                        "gemm_ms_alone_per_step": round(ms_alone, 3),
                        "in_place": {"achieved": round(fli / (ms_in * 1e-3) / 1e12, 3),
                                     "avg_launch_ms": ms_in / li,
                                     "timing": "HIP events around the same launches with the four "
                                               "streams overlapping as in the timed steps"},
                        "device_ms_share": round(sum(cls_stats[k][1] for k in cls_stats
                                                     if k.startswith("dgemm_"))
                                                 / max(1e-9, sum(v[1] for v in cls_stats.values())), 4)}
        log(f"# GEMM alone: {la} launches {ms_alone:.1f} ms ({achieved:.2f} TFLOP/s); in place "
            f"{ms_in:.1f} ms")
        for name in sorted(stats_alone):
            l_, t_, f_ = stats_alone[name]
            if name.startswith("dgemm_") and l_:
                log(f"#   alone {name}: {l_} launches {t_:.1f} ms {f_ / (t_ * 1e-3) / 1e12:.2f} TFLOP/s")
        ss = stream_summary(trace)
        if ss:
            log("# streams (busy / idle ms within a " + f"{ss['span_ms']:.1f} ms factorization): " +
                ", ".join(f"{k} {ss[k]['busy_ms']:.1f} / {ss[k]['idle_ms']:.1f}" for k in ("T", "P", "UV", "S")))
        log("# kernel classes (ms/step, launches/step, TFLOP/s):")
        for name, kv in sorted(kern.items(), key=lambda x: -x[1]["ms_per_step"]):
            log(f"#   {name:20s} {kv['ms_per_step']:9.3f} {kv['launches']:6d} {kv['tflops']}")
        if refused:
            log(f"# roofline refused: {refused}")

    cpu = None
    if args.cpu_steps > 0:
        from oracle import randutv_oracle as ro

        Ah = A.cpu().numpy()
        threads = os.cpu_count()
        t0 = time.perf_counter()
        ro.randutv(Ah, b, q, 0, max_steps=args.cpu_steps)
        tc = time.perf_counter() - t0
        fe = ro.flops_exact(m, n, b, q, max_steps=args.cpu_steps)
        scale = F / ro.flops_exact(m, n, b, q)  # express in F_std units
        cpu = {"value": round(fe * scale / tc / 1e12, 5), "unit": "TFLOP/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"first {args.cpu_steps} of {-(-n // b)} block steps of the same "
                         f"{m}x{n} b={b} q={q} factorization (U, V built), {tc:.1f} s"}
        log(f"# cpu oracle: {tc:.1f} s for {args.cpu_steps} steps")

    out = {
        "metric": "randUTV TFLOP/s (FP64, standard flop count) at n=12000",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"randutv_fp64_{m}x{n}_b{b}_q{q}_{args.spectrum}",
                   "m": m, "n": n, "b": b, "q": q, "spectrum": args.spectrum, "build_uv": True,
                   "parallelism": "single-gpu"},
        "frac_of_fp64_peak": round(value / PEAK_FP64_TFLOPS, 4),
        "residual": res,
        "orth_u": orth_u,
        "orth_v": orth_v,
        "flops_std": F,
        "roofline": roofline,
        "roofline_refused": refused,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "truncation_grad": trunc_grad,
        "hqrrp": hq,
        "ooc": ooc,
        "kernels": kern,
        "streams": stream_summary(trace),
    }
    print(json.dumps(out), flush=True)


def _aligned_col_err(X, Y, k):
    """||X(:, :k) S - Y(:, :k)||_F / sqrt(k), S the column signs that align X with Y."""
    import torch
    s = torch.sign((X[:, :k] * Y[:, :k]).sum(0))
    s[s == 0] = 1.0
    return (torch.linalg.norm(X[:, :k] * s[None, :] - Y[:, :k]) / k ** 0.5).item()


def mixed_block(pkg, torch, size, b, q, args, dev, reuse):
    """FP64 and each reduced-precision mode on the size x size exp matrix:
    time per factorization, F_std rate, residual, orthogonality, and errors
    against the FP64 factorization: T, the leading 1024 columns of U and V
    (sign-aligned), and the rank-k truncations for k in {64, 256, 1024}."""
    from randutv_inputs import make_matrix_device

    F = pkg.flops_std(size, size, q)
    if reuse is not None:
        A, U, T, V, ms64 = reuse
    else:
        A = make_matrix_device("exp", size, size, seed=0, device=dev)
        U = pkg.colmajor_empty(size, size, dev)
        T = pkg.colmajor_empty(size, size, dev)
        V = pkg.colmajor_empty(size, size, dev)
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V)
        torch.cuda.synchronize()
        ms64 = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
    nA = torch.linalg.norm(A)
    ks = [k for k in (64, 256, 1024) if k <= size]
    ref_err = {}
    for k in ks:
        Ak = pkg.randutv_truncate(U, T, V, k)
        ref_err[k] = (Ak, (torch.linalg.norm(A - Ak) / nA).item())
    block = {"workload": f"randutv {size}x{size} b={b} q={q} exp", "fp64": {
        "ms_per_step": round(ms64, 3), "value": round(F / (ms64 * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
        "frac_of_fp64_peak": round(F / (ms64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
        "rank_k_trunc_err": {str(k): ref_err[k][1] for k in ks}}}
    log(f"# mixed {size}x{size}: fp64 {ms64:.2f} ms/step")
    U2 = pkg.colmajor_empty(size, size, dev)
    T2 = pkg.colmajor_empty(size, size, dev)
    V2 = pkg.colmajor_empty(size, size, dev)
    eye = torch.eye(size, dtype=torch.float64, device=dev)
    for name in [x for x in args.mixed_modes.split(",") if x]:
        sk, up = MODES[name]
        kw = dict(U=U2, T=T2, V=V2, sketch_bits=sk, update_bits=up)
        pkg.randutv_factor(A, b, q, 0, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pkg.randutv_factor(A, b, q, 0, **kw)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
        rec = {"sketch": MODE_TEXT[sk], "updates": MODE_TEXT[up], "ms_per_step": round(ms, 3),
               "value": round(F / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
               "frac_of_fp64_peak": round(F / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
               "speedup_vs_fp64": round(ms64 / ms, 4)}
        if not args.no_check:
            rec["residual"] = (torch.linalg.norm(A - U2 @ T2 @ V2.T) / nA).item()
            rec["orth_u"] = (U2.T @ U2 - eye).abs().max().item()
            rec["orth_v"] = (V2.T @ V2 - eye).abs().max().item()
            ranks = {}
            for k in ks:
                Ak2 = pkg.randutv_truncate(U2, T2, V2, k)
                ranks[str(k)] = {"trunc_err": (torch.linalg.norm(A - Ak2) / nA).item(),
                                 "vs_fp64": (torch.linalg.norm(Ak2 - ref_err[k][0]) / nA).item()}
                del Ak2
            rec["rank_k"] = ranks
            kk = min(1024, size)
            rec["vs_fp64"] = {"T": (torch.linalg.norm(T2 - T) / nA).item(),
                              "U_1024": _aligned_col_err(U2, U, kk),
                              "V_1024": _aligned_col_err(V2, V, kk)}
        block[name] = rec
        log(f"# mixed {size}x{size} {name}: {ms:.2f} ms/step")
    del U2, T2, V2, eye
    for k in ks:
        del ref_err[k]
    if reuse is None:
        del A, U, T, V
    torch.cuda.empty_cache()
    return block


def truncation_grad_block(pkg, torch, args, dev):
    """Differentiable rank-k truncation on the 2048 x 2048 workload: a batch of
    float32 matrices (s_i = 0.98^i), b = 128, q = 2, k = 128 (and k = 64), loss
    ||A_k - B||_F^2 for a seeded Gaussian B, through pkg.truncation (forward
    from the first step, reverse pass randutv_truncate_grad_k; the library
    computes in FP64).  Forward and reverse timed over the whole batch."""
    from randutv_inputs import make_matrix_device

    gm, gb, gq = 2048, 128, 2
    gen = torch.Generator(device=dev)
    gen.manual_seed(77)
    A = torch.stack([make_matrix_device("exp98", gm, gm, seed=100 + i, device=dev)
                     for i in range(args.grad_batch)]).to(torch.float32)
    B = torch.randn(A.shape, dtype=torch.float32, device=dev, generator=gen)

    def fwd_bwd(k, full=False):
        X = A.detach().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ak = pkg.truncation(X, gb, gq, 0, k, full_factorization=full)
        loss = ((Ak - B) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        return 1e3 * (t1 - t0) / len(A), 1e3 * (time.perf_counter() - t1) / len(A)

    fwd_bwd(gb)
    f128, b128 = fwd_bwd(gb)
    f64, b64 = fwd_bwd(64)
    ffull, _ = fwd_bwd(gb, full=True)
    log(f"# truncation grad batch of {len(A)}: k=128 forward {f128:.2f} + backward {b128:.2f} ms per "
        f"matrix; k=64 {f64:.2f} + {b64:.2f} ms; forward through the whole factorization {ffull:.2f} ms")
    return {"workload": f"{args.grad_batch} x {gm}x{gm} float32, s_i = 0.98^i, b={gb}, q={gq}, k={gb}, "
                        "loss ||A_k - B||_F^2 (computed in FP64)",
            "ms_forward_per_matrix": round(f128, 3), "ms_backward_per_matrix": round(b128, 3),
            "ms_forward_backward_per_matrix": round(f128 + b128, 3),
            "k64": {"ms_forward_per_matrix": round(f64, 3), "ms_backward_per_matrix": round(b64, 3)},
            "ms_forward_full_factorization_per_matrix": round(ffull, 3)}


def ooc_block(pkg, torch, args, dev):
    """Out-of-core factorization (Section 3.2) of the n x n exp matrix held in
    page-locked host memory, with an HBM tile cache of args.ooc_budget_gib,
    in the three variants of Section 3.2.4: wall time against the summed
    compute and copy times, the paper's Table 1 quantities."""
    from randutv_inputs import make_matrix_device

    n, b, q = args.ooc_n, 256, 2
    Ad = make_matrix_device("exp", n, n, seed=0, device=dev)
    Ah = pkg.host_colmajor_empty(n, n)
    Ah.copy_(Ad.cpu())
    del Ad
    budget = int(args.ooc_budget_gib * (1 << 30))
    U = pkg.host_colmajor_empty(n, n)
    T = pkg.host_colmajor_empty(n, n)
    V = pkg.host_colmajor_empty(n, n)
    out = {"workload": f"randutv {n}x{n} b={b} q={q} exp, A/U/T/V in page-locked host memory "
                       f"({3 * 8 * n * n / 2**30:.2f} GiB), HBM tile cache {args.ooc_budget_gib} GiB",
           "modes": {}}
    for mode in ("overlapped", "cached", "traditional"):
        _, _, _, st = pkg.randutv_factor_ooc(Ah, b, q, 0, budget, mode, U=U, T=T, V=V)
        e = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
        e["real_over_compute"] = round(st["real_ms"] / st["compute_ms"], 3)
        e["compute_over_io"] = round(st["compute_ms"] / st["io_ms"], 3) if st["io_ms"] > 0 else None
        out["modes"][mode] = e
        log(f"# ooc {n}^2 {mode}: real {st['real_ms']:.0f} ms, compute {st['compute_ms']:.0f} ms, "
            f"I/O {st['io_ms']:.0f} ms (in {st['h2d_ms']:.0f}, out {st['d2h_ms']:.0f}), "
            f"{(st['h2d_bytes'] + st['d2h_bytes']) / 1e9:.1f} GB moved")
    return out

if __name__ == "__main__":
    main()
