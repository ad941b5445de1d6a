#!/usr/bin/env python3
"""FP64 randUTV throughput on one MI355X.

One step = one full randUTV factorization A = U T V^T (U and V built) of the
12000 x 12000 matrix A = P diag(0.99^i) Q^T (P, Q Haar), block size b = 256,
q = 2 power steps, sketch seed 0 -- every block step of the method (sketch,
power iteration, QR of the sketch, right transform of all rows and of V, panel
QR, left transform, U update, b x b SVDs and their applications) runs inside
the timed region; A, U, T, V are resident in HBM before it starts.

value = F_std / t in TFLOP/s, with the leading-order count
F_std = (1+2q)(m n^2 - n^3/3) + 2 m n^2 + 4/3 n^3 + 4 m^2 n  (1.843e13 here).
The roofline entry is the dominant kernel, the FP64 matrix-core GEMM (all its
operand layouts): algorithmic flops per launch over its average launch time,
from HIP events recorded on the launching stream around every launch in the
timed steps, against the FP64 matrix-core peak (78.6 TFLOP/s); traffic is the
HBM bytes per launch from committed rocprofv3 counters when they were taken on
the current kernel source.  cpu_baseline
times the FP64 CPU oracle on the first block steps of the same problem.
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
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--all-classes-timed", action="store_true",
                    help="time every kernel class inside the timed region (default: the GEMM "
                         "launches there, the other classes in one more factorization after it)")
    ap.add_argument("--mixed-modes", default="fp32,bf16x3,bf16",
                    help="reduced-precision sketch modes timed beside the FP64 run")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the runs beside the FP64 headline: the reduced-precision sketches, "
                         "the differentiable truncation and HQRRP")
    ap.add_argument("--grad-batch", type=int, default=16,
                    help="matrices of the differentiable-truncation run (2048 x 2048, b=128; 0: skip)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the residual/orthogonality check of the timed output (profiler runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the factorizations, run one plain device copy of this many MiB "
                         "(a kernel of known HBM traffic, to scale hardware byte counters)")
    return ap.parse_args()


def traffic_entry(kernel: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary, if one exists for the current kernel source (else None)."""
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
        return rec["bytes_per_launch"]
    except Exception:
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the factorization has "
                                   "no multi-GPU path (use --gpus 1)"}))
        sys.exit(2)
    import numpy as np
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
        print(f"# copy calibration: {nel * 8} bytes read, {nel * 8} bytes written", file=sys.stderr)
        del src, dst
    torch.cuda.synchronize()
    print(f"# workload randutv fp64 {m}x{n} b={b} q={q} spectrum={args.spectrum}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V)
        torch.cuda.synchronize()
        print(f"# warmup {w}: {time.perf_counter() - t0:.3f} s", file=sys.stderr, flush=True)

    # HIP events around every GEMM launch of the timed factorizations (on the
    # stream it is launched on) give the dominant kernel's average duration;
    # the other kernel classes are timed in one more factorization after the
    # timed region (all classes timed at once cost ~2% of the step time)
    timing = not args.no_kernel_timing
    pkg.randutv_set_timing(timing, gemm_only=not args.all_classes_timed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = pkg.randutv_kernel_stats() if timing else {}
    pkg.randutv_set_timing(False)
    cls_stats, cls_steps = stats, args.steps
    if timing and not args.all_classes_timed:
        pkg.randutv_set_timing(True)
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V)
        torch.cuda.synchronize()
        cls_stats, cls_steps = pkg.randutv_kernel_stats(), 1
        pkg.randutv_set_timing(False)
    ms_step = 1e3 * elapsed / max(args.steps, 1)
    print(f"# timed {args.steps} steps: {ms_step:.2f} ms/step", file=sys.stderr, flush=True)

    F = pkg.flops_std(m, n, q)
    value = F / (ms_step * 1e-3) / 1e12

    # correctness of the timed output
    res = orth_u = orth_v = None
    if not args.no_check:
        nA = torch.linalg.norm(A)
        res = (torch.linalg.norm(A - U @ T @ V.T) / nA).item()
        eye_m = torch.eye(m, dtype=torch.float64, device=dev)
        orth_u = (U.T @ U - eye_m).abs().max().item()
        del eye_m
        eye_n = torch.eye(n, dtype=torch.float64, device=dev)
        orth_v = (V.T @ V - eye_n).abs().max().item()
        del eye_n

    # the same factorization with the sketch and power-iteration products in
    # reduced precision (every transform of T, U, V still FP64): FP32 matrix
    # cores, three BF16 products of split operands, one BF16 product
    mixed = None
    if not args.no_mixed:
        mixed = {}
        U2 = pkg.colmajor_empty(m, m, dev)
        T2 = pkg.colmajor_empty(m, n, dev)
        V2 = pkg.colmajor_empty(n, n, dev)
        modes = {"fp32": (32, "fp32 matrix cores (FP64 storage); all transforms FP64"),
                 "bf16x3": (48, "bf16 matrix cores, operands split x = hi + lo, hi*hi + hi*lo + lo*hi, "
                                "fp32 accumulation (FP64 storage); all transforms FP64"),
                 "bf16": (16, "bf16 matrix cores, operands rounded to bf16, fp32 accumulation "
                              "(FP64 storage); all transforms FP64")}
        for name in args.mixed_modes.split(","):
            bits, what = modes[name]
            pkg.randutv_factor(A, b, q, 0, U=U2, T=T2, V=V2, sketch_bits=bits)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                pkg.randutv_factor(A, b, q, 0, U=U2, T=T2, V=V2, sketch_bits=bits)
            torch.cuda.synchronize()
            ms_mixed = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
            print(f"# {name}-sketch: {ms_mixed:.2f} ms/step", file=sys.stderr, flush=True)
            rec = {"sketch": what, "ms_per_step": round(ms_mixed, 3),
                   "value": round(F / (ms_mixed * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
                   "frac_of_fp64_peak": round(F / (ms_mixed * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
            if not args.no_check:
                nA = torch.linalg.norm(A)
                rec["residual"] = (torch.linalg.norm(A - U2 @ T2 @ V2.T) / nA).item()
                ranks = {}
                for k in (kk for kk in (64, 256, 1024) if kk <= n):
                    Ak = pkg.randutv_truncate(U, T, V, k)
                    Ak2 = pkg.randutv_truncate(U2, T2, V2, k)
                    ranks[str(k)] = {"fp64_trunc_err": (torch.linalg.norm(A - Ak) / nA).item(),
                                     "mixed_trunc_err": (torch.linalg.norm(A - Ak2) / nA).item(),
                                     "mixed_vs_fp64": (torch.linalg.norm(Ak2 - Ak) / nA).item()}
                    del Ak, Ak2
                rec["rank_k"] = ranks
                rec["T_vs_fp64"] = (torch.linalg.norm(T2 - T) / nA).item()
            mixed[name] = rec
        del U2, T2, V2

    # differentiable first-block truncation: a batch of 2048 x 2048 matrices
    # (s_i = 0.98^i), b = 128, q = 2, k = 128; loss ||A_k - B||_F^2 for a
    # seeded Gaussian B; forward (randutv_factor + randutv_truncate) and
    # reverse pass (randutv_truncate_grad) timed separately
    trunc_grad = None
    if args.grad_batch > 0 and not args.no_mixed:
        gm, gb, gq = 2048, 128, 2
        gen = torch.Generator(device=dev)
        gen.manual_seed(77)
        As = [make_matrix_device("exp98", gm, gm, seed=100 + i, device=dev) for i in range(args.grad_batch)]
        Bs = [torch.randn(gm, gm, dtype=torch.float64, device=dev, generator=gen) for _ in As]

        def fwd_bwd(Ai, Bi, first_step_only=False):
            X = Ai.detach().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Ak = pkg.first_block_truncation(X, gb, gq, 0, first_step_only=first_step_only)
            loss = ((Ak - Bi) ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            return t1 - t0, time.perf_counter() - t1

        fwd_bwd(As[0], Bs[0])
        tf = tb = 0.0
        for Ai, Bi in zip(As, Bs):
            a, c = fwd_bwd(Ai, Bi)
            tf += a
            tb += c
        tf1 = 0.0
        for Ai, Bi in zip(As, Bs):
            tf1 += fwd_bwd(Ai, Bi, first_step_only=True)[0]
        trunc_grad = {"workload": f"{args.grad_batch} x {gm}x{gm}, s_i = 0.98^i, b={gb}, q={gq}, k={gb}, FP64, "
                                  "loss ||A_k - B||_F^2",
                      "ms_forward_per_matrix": round(1e3 * tf / len(As), 3),
                      "ms_forward_first_step_per_matrix": round(1e3 * tf1 / len(As), 3),
                      "ms_backward_per_matrix": round(1e3 * tb / len(As), 3),
                      "ms_batch": round(1e3 * (tf + tb), 3)}
        print(f"# truncation grad batch: forward {1e3 * tf / len(As):.2f} ms (first step only "
              f"{1e3 * tf1 / len(As):.2f} ms), backward {1e3 * tb / len(As):.2f} ms per matrix",
              file=sys.stderr, flush=True)
        del As, Bs

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
        hq = {"workload": f"hqrrp {m}x{n} b={b}, FP64", "ms": round(ms_hq, 3),
              "qr_flops": f_qr, "tflops_qr_count": round(f_qr / (ms_hq * 1e-3) / 1e12, 3)}
        print(f"# hqrrp: {ms_hq:.2f} ms", file=sys.stderr, flush=True)
        del Fh, tauh, jph

    roofline = None
    kern = {}
    if stats:
        for name, (launches, ms, fl) in cls_stats.items():
            if launches:
                kern[name] = {"launches": launches // cls_steps, "ms_per_step": ms / cls_steps,
                              "tflops": (fl / (ms * 1e-3) / 1e12) if ms > 0 and fl > 0 else None}
        # the dominant kernel: the FP64 matrix-core GEMM (one HIP kernel,
        # instantiated per operand layout; its classes together take most of
        # the device time)
        gemm = [k for k in stats if k.startswith("dgemm_") and stats[k][0]]
        launches = sum(stats[k][0] for k in gemm)
        ms = sum(stats[k][1] for k in gemm)
        fl = sum(stats[k][2] for k in gemm)
        achieved = fl / (ms * 1e-3) / 1e12
        tb = traffic_entry("dgemm_mfma_kernel")
        roofline = {"bound": "mfma", "kernel": "dgemm_mfma_kernel", "achieved": round(achieved, 3),
                    "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                    "traffic": tb, "avg_launch_ms": ms / launches, "launches": launches,
                    "flops_per_launch": fl / launches,
                    "device_ms_share": round(sum(cls_stats[k][1] for k in gemm if k in cls_stats)
                                             / sum(v[1] for v in cls_stats.values()), 4)}
        print("# kernel classes (ms/step, launches/step, TFLOP/s):", file=sys.stderr)
        for name, kv in sorted(kern.items(), key=lambda x: -x[1]["ms_per_step"]):
            print(f"#   {name:20s} {kv['ms_per_step']:9.3f} {kv['launches']:6d} {kv['tflops']}",
                  file=sys.stderr)

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
               "kind": "oracle",
               "sample": f"first {args.cpu_steps} of {-(-n // b)} block steps of the same "
                         f"{m}x{n} b={b} q={q} factorization (U, V built), {tc:.1f} s"}
        print(f"# cpu oracle: {tc:.1f} s for {args.cpu_steps} steps", file=sys.stderr)

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
        "cpu_baseline": cpu,
        "mixed": mixed,
        "truncation_grad": trunc_grad,
        "hqrrp": hq,
        "kernels": kern,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
