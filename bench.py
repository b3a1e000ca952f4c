#!/usr/bin/env python3
"""Benchmark: effective complex GFLOPS of multi-component LU on one MI355X.

A step is one pass of the whole hot path over one synthetic input: canonicalised
complex double-double A (n = 4096, entries uniform[-1,1], lower components
c_k = c_{k-1} 2^-53 U(-1,1)), blocked right-looking LU with partial pivoting (panel 64,
3M trailing update), then the forward / backward solve for b = A 1.  All inputs are
resident in HBM before the timed region; each step factors its own copy of A.

value = 8 n^3 / 3 / t_step (the LAPACK zgetrf operation count; the solve is inside the
step but not counted).  Besides the headline line, the JSON carries: the backward error
of the last solve (exact-enough residual computed on the GPU in quadruple-double), the
4M / triple-double / quadruple-double variants, the roofline of the dominant kernel (the
3M trailing-update GEMM, timed live with HIP events), the complex matrix-product
benchmark of Sec. 2.4 (C := A B, n = 2048, every product form), the first trailing update
of the factorisation in every product form including Strassen-Winograd, the real (Im = 0)
gesv and the CPU oracle baseline.
`--panel-sweep 32,64,96,128` instead runs the panel-width sweep on the paper's LU workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096] [--panel 64]
"""
from __future__ import annotations

import argparse
import ctypes as ct
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("effective complex GFLOPS of DD/TD/QD getrf at n=4096 (3M vs 4M vs split-MFMA) "
          "+ backward err")
PEAK_FP64_TFLOPS = 78.6   # 256 CU x 64 FP64 lanes/clk x 2 (FMA) x 2.4 GHz
# algorithmic FP64 flops of one real multiply-accumulate in the level accumulator of the
# trailing update (FMA counted as 2; 12 / 45 / 112 FP64 instructions for DD / TD / QD);
# 3M uses three real MACs per complex MAC, 4M four
FLOPS_PER_REAL_MAC = {2: 15, 3: 51, 4: 122}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=4096)
    p.add_argument("--panel", type=int, default=64)
    p.add_argument("--method", default="3m")
    p.add_argument("--no-variants", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-roofline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target length of the CPU oracle sample")
    p.add_argument("--no-matmul", action="store_true")
    p.add_argument("--matmul-n", type=int, default=2048,
                   help="size of the square complex matrix-product benchmark (Sec. 2.4)")
    p.add_argument("--panel-sweep", default="",
                   help="comma-separated panel widths: instead of the headline, run the "
                        "panel-width sweep on the paper's LU workload at --n and print it")
    p.add_argument("--calib-copy", action="store_true",
                   help="first run one plain 1 GiB device-to-device copy (a reference for "
                        "hardware memory counters)")
    return p.parse_args()


def eff_gflops(n, seconds):
    return 8.0 * n ** 3 / 3.0 / seconds / 1e9


def backward_error(mp, torch, A0, X, B0):
    """eta = ||b - A x||_inf / (||A||_inf ||x||_inf); residual formed by the library in
    quadruple-double (widening is exact), norms from the leading components."""
    A4 = mp.convert(A0, 4)
    X4 = mp.convert(X, 4)
    R4 = mp.convert(B0, 4)
    mp.gemm(A4, X4, R4, alpha=-1, method="4m")
    hi = lambda T: torch.complex(T[0, 0], T[1, 0]).transpose(0, 1)
    nr = hi(R4).abs().max().item()
    nA = hi(A0).abs().sum(dim=1).max().item()
    nx = hi(X).abs().max().item()
    return nr / (nA * nx)


def make_problem(mp, torch, synthgen, n, C, seed=0):
    A0 = torch.from_numpy(synthgen.uniform(n, n, C, seed)).cuda()
    mp.renorm_(A0)
    X1 = torch.from_numpy(synthgen.ones(n, 1, C)).cuda()
    B0 = mp.gemm(A0, X1, None, method="4m")   # b = A 1 in the working precision
    return A0, B0


def time_gesv(mp, torch, A0, B0, steps, warmup, panel, method):
    """Factor + solve `steps` resident copies back to back; returns (ms/step, X, info)."""
    C, n = A0.shape[1], A0.shape[2]
    nb = ct.c_size_t()
    o = mp._opts(panel, method)
    mp.lib().mplu_zgesv_wsbytes(C, n, 1, ct.byref(o), ct.byref(nb))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    As = [A0.clone() for _ in range(warmup + steps)]
    Bs = [B0.clone() for _ in range(warmup + steps)]
    for w in range(warmup):
        mp.gesv(As[w], Bs[w], panel=panel, method=method, work=work)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    infos = []
    t0 = time.perf_counter()
    ev0.record()
    for s in range(steps):
        _, info = mp.gesv(As[warmup + s], Bs[warmup + s], panel=panel, method=method, work=work)
        infos.append(info)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / steps
    info = max(int(i.item()) for i in infos)
    X = Bs[-1]
    del As
    return ms, wall, X, info


def gemm_roofline(mp, torch, A0, panel, method):
    """Replay the trailing updates of one factorisation (m = n - j - K, k = K for every
    panel step j) through mplu_zgemm on the stream, each launch bracketed by HIP events."""
    C, n = A0.shape[1], A0.shape[2]
    M = A0.clone()
    L = mp.lib()
    ld, ps = n, n * n
    base = M.data_ptr()
    meth = mp._METHODS[method]
    stream = ct.c_void_p(torch.cuda.current_stream().cuda_stream)

    def sub(i, j):
        return mp.ZMat(base + 8 * (j * ld + i), ld, ps)

    launches = []
    for j in range(0, n - panel, panel):
        r = n - j - panel
        # products with fewer than 512 tiles of 32 x 32 go to the 16 x 16 kernel; the
        # replay covers the launches of the 32 x 32 kernel, the dominant one
        if r <= 0 or ((r + 31) // 32) ** 2 < 512:
            break
        launches.append((j, r))
    # warm up the kernel once
    rc = L.mplu_zgemm(C, b"N", b"N", launches[0][1], launches[0][1], panel, -1,
                      sub(panel, 0), sub(0, panel), 1, sub(panel, panel), meth, None, None, 0,
                      stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    evs = []
    for (j, r) in launches:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        rc = L.mplu_zgemm(C, b"N", b"N", r, r, panel, -1, sub(j + panel, j), sub(j, j + panel),
                          1, sub(j + panel, j + panel), meth, None, None, 0, stream)
        e1.record()
        assert rc == 0, rc
        evs.append((e0, e1))
    torch.cuda.synchronize()
    total_ms = sum(a.elapsed_time(b) for a, b in evs)
    macs = sum(r * r * panel for (_, r) in launches)
    real_per_complex = 3 if method == "3m" else 4
    flops = macs * real_per_complex * FLOPS_PER_REAL_MAC[C]
    achieved = flops / (total_ms / 1e3) / 1e12
    return {
        "kernel": f"k_gemm<{C},{'3M' if method == '3m' else '4M'},32x32 tiles> trailing update",
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": committed_traffic("k_gemm.hip") if (C, method) == (2, "3m") else None,
        "launches": len(launches),
        "avg_launch_ms": round(total_ms / len(launches), 4),
        "flops_per_launch": flops / len(launches),
    }


INT8_PEAK_TOPS = 5000.0  # MI355X dense INT8 MFMA


def split_roofline(mp, torch, A0, panel, n_launch=12):
    """MFMA rate of the INT8 split trailing update (DD, S = 17 slices): the first n_launch
    trailing updates of one factorisation with panel width `panel`, each (slicing and
    product kernels) bracketed by HIP events on the stream.  Counted work: the digit-pair
    MFMAs, S (S + 1) / 2 pairs per 64-deep chunk, for each of the three real products."""
    C, n = A0.shape[1], A0.shape[2]
    M = A0.clone()
    L = mp.lib()
    ld, ps = n, n * n
    base = M.data_ptr()
    stream = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    S = 17
    opts = mp._gemm_opts("split_i8")
    nb = ct.c_size_t()
    r0 = n - panel
    assert L.mplu_zgemm_wsbytes(C, r0, r0, panel, 3, ct.byref(opts), ct.byref(nb)) == 0
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")

    def sub(i, j):
        return mp.ZMat(base + 8 * (j * ld + i), ld, ps)

    launches = [(j, n - j - panel) for j in range(0, panel * n_launch, panel)]
    evs = []
    for it, (j, r) in enumerate([launches[0]] + launches):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        rc = L.mplu_zgemm(C, b"N", b"N", r, r, panel, -1, sub(j + panel, j), sub(j, j + panel), 1,
                          sub(j + panel, j + panel), 3, ct.byref(opts), work.data_ptr(),
                          work.numel(), stream)
        e1.record()
        assert rc == 0, rc
        if it > 0:
            evs.append((e0, e1))
    torch.cuda.synchronize()
    total_ms = sum(a.elapsed_time(b) for a, b in evs)
    kpad = (panel + 63) // 64 * 64
    ops = sum(3 * (S * (S + 1) // 2) * 2 * r * r * kpad for (_, r) in launches)
    achieved = ops / (total_ms / 1e3) / 1e12
    return {"kernel": "k_slice + k_split_i8<2,17> (DD split INT8 trailing update)",
            "bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS,
            "unit": "TOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4),
            "launches": len(launches), "avg_launch_ms": round(total_ms / len(launches), 4),
            "panel": panel}


def mp_diff(torch, X4, R4):
    """Leading-order value of X - R for two quadruple-double plane tensors, as complex128
    (component differences summed in binary64; both agree to far more than 53 bits, so
    this carries the difference to a few digits)."""
    d = (X4 - R4).sum(dim=1)
    return torch.complex(d[0], d[1])


def hi_abs(torch, T):
    """cabs1 of the leading components, as a (rows, cols) float64 matrix."""
    return (T[0, 0].abs() + T[1, 0].abs()).transpose(0, 1)


def matmul_bench(mp, torch, synthgen, n, reps=3):
    """The complex matrix-product benchmark of Sec. 2.4: C := A B with square n x n
    operands whose leading components are uniform on [0, 1], for DD / TD / QD and each
    product form (4M, 3M, split INT8, split FP64, one level of Strassen-Winograd over 3M).  Each product is timed with HIP events
    on the stream (one warm-up, then the mean of `reps`).  Error: max over elements of
    |C - C_ref| / (|A| |B|)_ij, C_ref the quadruple-double 4M product of the same
    (exactly widened) operands; for QD this is the difference from QD 4M itself."""
    out = {}
    for C in (2, 3, 4):
        A = torch.from_numpy(synthgen.uniform(n, n, C, 11, lo=0.0, hi=1.0)).cuda()
        B = torch.from_numpy(synthgen.uniform(n, n, C, 12, lo=0.0, hi=1.0)).cuda()
        mp.renorm_(A)
        mp.renorm_(B)
        ref = mp.gemm(mp.convert(A, 4), mp.convert(B, 4), None, method="4m")
        scale = hi_abs(torch, A) @ hi_abs(torch, B)
        for meth in ("4m", "3m", "split_i8", "split_f64", "strassen"):
            times = []
            for r in range(reps + 1):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                Cm = mp.gemm(A, B, None, method=meth)
                e1.record()
                torch.cuda.synchronize()
                if r:
                    times.append(e0.elapsed_time(e1))
            d = mp_diff(torch, mp.convert(Cm, 4), ref).transpose(0, 1)
            err = (d.real.abs() + d.imag.abs()).div(scale).max().item()
            ms = sum(times) / len(times)
            key = f"{['', '', 'DD', 'TD', 'QD'][C]}_{meth}"
            out[key] = {"ms": round(ms, 3), "gflops": round(8.0 * n ** 3 / (ms / 1e3) / 1e9, 2),
                        "err": err}
            print(f"[bench] matmul n={n} {key}: {out[key]}", file=sys.stderr, flush=True)
            del Cm
        del A, B, ref, scale
        torch.cuda.empty_cache()
    return {"n": n, "op": "C := A B, complex, leading components uniform[0,1]",
            "flops": "8 n^3 per product", "results": out}


def update_forms(mp, torch, synthgen, n, K, reps=5):
    """The first trailing update of the factorisation, A22 := A22 - L21 U12 with
    m = n - K rows and columns and depth K, in every product form the update could use:
    4M, 3M, split INT8, split FP64, and one level of Strassen-Winograd over 3M (Sec. 2.1;
    the paper's Strassen LU of Table 1).  Mean of `reps` HIP-event-timed launches after a
    warm-up; DD and QD."""
    m = n - K
    out = {}
    for C in (2, 4):
        L21 = torch.from_numpy(synthgen.uniform(m, K, C, 21)).cuda()
        U12 = torch.from_numpy(synthgen.uniform(K, m, C, 22)).cuda()
        A22 = torch.from_numpy(synthgen.uniform(m, m, C, 23)).cuda()
        for T in (L21, U12, A22):
            mp.renorm_(T)
        for meth in ("4m", "3m", "split_i8", "split_f64", "strassen"):
            times = []
            for r in range(reps + 1):
                T = A22.clone()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                mp.gemm(L21, U12, T, alpha=-1, method=meth)
                e1.record()
                torch.cuda.synchronize()
                if r:
                    times.append(e0.elapsed_time(e1))
                del T
            ms = sum(times) / len(times)
            key = f"{['', '', 'DD', 'TD', 'QD'][C]}_{meth}"
            out[key] = {"ms": round(ms, 4),
                        "gflops": round(8.0 * m * m * K / (ms / 1e3) / 1e9, 2)}
            print(f"[bench] update n={n} K={K} {key}: {out[key]}", file=sys.stderr, flush=True)
        del L21, U12, A22
        torch.cuda.empty_cache()
    return {"m": m, "n": m, "k": K, "op": "A22 := A22 - L21 U12 (first trailing update)",
            "flops": "8 m^2 k per update", "results": out}


def panel_sweep(mp, torch, synthgen, n, panels, steps=2):
    """Panel width (the paper's block size K) sweep on the paper's LU workload of Sec. 4:
    leading components uniform on [0, 1], x_k = k + k i, b = A x formed in quadruple-double
    and rounded to the working format (exact to 2^-209 relative for DD and TD; for QD the
    rounding of b is itself of the order of the working precision).  Reports gesv time,
    the normwise backward error and the maximum relative error max_k |x_k - x*_k| / |x*_k|."""
    out = []
    for C in (2, 3, 4):
        A0 = torch.from_numpy(synthgen.uniform(n, n, C, 0, lo=0.0, hi=1.0)).cuda()
        mp.renorm_(A0)
        xt4 = torch.from_numpy(synthgen.k_plus_ki(n, 4)).cuda()
        b4 = mp.gemm(mp.convert(A0, 4), xt4, None, method="4m")
        B0 = mp.convert(b4, C)
        xmod = hi_abs(torch, xt4)[:, 0] / 2 ** 0.5   # |k + k i| = sqrt(2) k
        for meth in ("4m", "3m", "split_i8", "split_f64"):
            for K in panels:
                ms, _, X, info = time_gesv(mp, torch, A0, B0, steps, 1, K, meth)
                eta = backward_error(mp, torch, A0, X, B0)
                d = mp_diff(torch, mp.convert(X, 4), xt4).transpose(0, 1)[:, 0]
                rel = (d.abs() / xmod).max().item()
                rec = {"prec": ["", "", "DD", "TD", "QD"][C], "method": meth, "panel": K,
                       "ms": round(ms, 3), "gflops": round(eff_gflops(n, ms / 1e3), 2),
                       "eta": eta, "max_rel_err": rel, "info": info}
                print(f"[sweep] {rec}", file=sys.stderr, flush=True)
                out.append(rec)
                del X
        del A0, B0, b4, xt4
        torch.cuda.empty_cache()
    return out


def real_bench(mp, torch, synthgen, n, panel, steps=2):
    """Real DD / QD gesv (the Im = 0 case, mplu_dgesv) on the real part of the headline
    matrix, b = A 1, with the real product and with the INT8 split; effective GFLOPS from
    the real LU count 2 n^3 / 3; eta from the QD residual of the complex embedding."""
    out = {}
    for C in (2, 4):
        Z, _ = make_problem(mp, torch, synthgen, n, C)
        A0 = Z[0].clone()
        del Z
        X1 = torch.from_numpy(synthgen.ones(n, 1, C)[0]).cuda()
        B0 = mp.dgemm(A0, X1)
        emb = lambda R: torch.stack([R, torch.zeros_like(R)])
        for meth in ("3m", "split_i8"):
            nb = ct.c_size_t()
            o = mp._opts(panel, meth)
            mp.lib().mplu_dgesv_wsbytes(C, n, 1, ct.byref(o), ct.byref(nb))
            work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
            As = [A0.clone() for _ in range(steps + 1)]
            Bs = [B0.clone() for _ in range(steps + 1)]
            mp.dgesv(As[0], Bs[0], panel=panel, method=meth, work=work)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            infos = [mp.dgesv(As[s], Bs[s], panel=panel, method=meth, work=work)[1]
                     for s in range(1, steps + 1)]
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            eta = backward_error(mp, torch, emb(A0), emb(Bs[-1]), emb(B0))
            key = f"{['', '', 'DD', 'TD', 'QD'][C]}_{'real_product' if meth == '3m' else meth}"
            out[key] = {"ms": round(ms, 3),
                        "gflops": round(2.0 * n ** 3 / 3.0 / (ms / 1e3) / 1e9, 2),
                        "eta": eta, "info": max(int(i.item()) for i in infos)}
            print(f"[bench] real {key}: {out[key]}", file=sys.stderr, flush=True)
            del As, Bs, work
            torch.cuda.empty_cache()
        del A0, B0
        torch.cuda.empty_cache()
    return {"n": n, "panel": panel, "op": "real gesv (mplu_dgesv), 1 RHS",
            "flops": "2 n^3 / 3 per factorisation", "results": out}


def committed_traffic(kernel_src):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, or None when that kernel's source changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "gemm_dd_3m_n4096_counters.txt")
    src = os.path.join(ROOT, "paper_2403_16013_amd", "csrc", kernel_src)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != h:
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_baseline(synthgen, n, target_s):
    """The oracle's unblocked 4M LU (the paper's Normal LU) on the same n x n DD matrix,
    stopped after k columns so that the sample takes about target_s seconds."""
    import oracle

    threads = oracle.set_threads(0)
    A = oracle.canon(synthgen.uniform(n, n, 2, 0))
    # calibrate on one column
    t0 = time.perf_counter()
    oracle.getf2(A, kmax=1)
    t1 = time.perf_counter() - t0
    kmax = max(1, min(n, int(target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.getf2(A, kmax=kmax)
    dt = time.perf_counter() - t0
    macs = sum((n - k - 1) ** 2 for k in range(kmax))
    return {"value": round(8.0 * macs / dt / 1e9, 4), "unit": "GFLOPS", "cores": threads,
            "kind": "oracle",
            "sample": f"unblocked 4M LU of the n={n} DD matrix, first {kmax} columns "
                      f"({macs:.3e} complex MACs, {dt:.1f} s, {threads} OpenMP threads)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "runs the factorisation on one GPU", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2403_16013_amd as mp
    import synthgen

    n, panel, method = args.n, args.panel, args.method
    if args.panel_sweep:
        panels = [int(k) for k in args.panel_sweep.split(",")]
        res = panel_sweep(mp, torch, synthgen, n, panels)
        print(json.dumps({"panel_sweep": {"n": n, "workload": "the paper's LU workload: "
                          "A uniform[0,1] complex, x_k = k + k i", "results": res}}))
        return
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] DD n={n} panel={panel} {method}: building inputs", file=sys.stderr,
          flush=True)
    A0, B0 = make_problem(mp, torch, synthgen, n, 2)
    ms, wall, X, info = time_gesv(mp, torch, A0, B0, args.steps, args.warmup, panel, method)
    eta = backward_error(mp, torch, A0, X, B0)
    print(f"[bench] DD {method}: {ms:.2f} ms/step info={info} eta={eta:.3e}", file=sys.stderr,
          flush=True)
    line = {
        "metric": METRIC,
        "value": round(eff_gflops(n, ms / 1e3), 2),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"complex double-double gesv (getrf + getrs), n={n}, panel {panel}, "
                               f"{method.upper()} trailing update, A uniform[-1,1] DD, b = A*1",
                   "n": n, "prec": "DD", "panel": panel, "method": method, "nrhs": 1},
        "eta": eta,
        "info": info,
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_roofline:
        line["roofline"] = gemm_roofline(mp, torch, A0, panel, method)
        print(f"[bench] roofline {line['roofline']}", file=sys.stderr, flush=True)
    if not args.no_roofline:
        line["roofline_split_i8"] = split_roofline(mp, torch, A0, 128)
        print(f"[bench] split roofline {line['roofline_split_i8']}", file=sys.stderr, flush=True)
        line["roofline_split_i8_k64"] = split_roofline(mp, torch, A0, 64)
        print(f"[bench] split roofline K=64 {line['roofline_split_i8_k64']}", file=sys.stderr,
              flush=True)
    if not args.no_variants:
        var = {}
        # the metric's grid: DD / TD / QD x {4M, 3M, split INT8, split FP64}, panels 64
        # and 128 (DD 3M at the headline's panel is the headline itself), and the
        # Strassen-Winograd LU of Table 1
        runs = ((2, "4m", panel, 2), (2, "3m", 128, 2), (2, "split_i8", panel, 2),
                (2, "split_i8", 128, 2), (2, "split_f64", panel, 1), (2, "split_f64", 128, 1),
                (2, "strassen", panel, 1))
        for C in (3, 4):
            runs += ((C, "3m", panel, 1), (C, "3m", 128, 1), (C, "4m", panel, 1),
                     (C, "split_i8", panel, 1), (C, "split_i8", 128, 1),
                     (C, "split_f64", panel, 1), (C, "strassen", panel, 1))
        probs = {2: (A0, B0)}
        for (C, meth, pnl, steps) in runs:
            if C not in probs:
                probs = {2: (A0, B0), C: make_problem(mp, torch, synthgen, n, C)}
                torch.cuda.empty_cache()
            A, B = probs[C]
            vms, _, VX, vinfo = time_gesv(mp, torch, A, B, steps, 1, pnl, meth)
            veta = backward_error(mp, torch, A, VX, B)
            key = f"{['', '', 'DD', 'TD', 'QD'][C]}_{meth}_K{pnl}"
            var[key] = {"ms": round(vms, 3), "gflops": round(eff_gflops(n, vms / 1e3), 2),
                        "eta": veta, "info": vinfo}
            print(f"[bench] variant {key}: {var[key]}", file=sys.stderr, flush=True)
            del VX
            torch.cuda.empty_cache()
        del probs
        line["variants"] = var
        line["variants_eta"] = ("eta of every variant is formed by the library itself (a QD "
                                "residual on the GPU): accurate far below the DD and TD "
                                "working precisions, but itself at working precision for "
                                "QD solutions; the exact-residual figures "
                                "of the same grid are asserted by tests/test_gpu_fullsize.py")
    if not args.no_matmul:
        line["matmul"] = matmul_bench(mp, torch, synthgen, args.matmul_n)
        line["update_forms"] = [update_forms(mp, torch, synthgen, n, K)
                                for K in sorted({panel, 128})]
    if not args.no_variants:
        line["real"] = real_bench(mp, torch, synthgen, n, panel)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(synthgen, n, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
