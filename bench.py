#!/usr/bin/env python3
"""Benchmark of the drag update v' = exp(dt K) v on one MI355X.

One step = one drag update of every cell of the workload (drag_expm_apply:
coefficients, ||dt K||_1, Alg. 1, Taylor stage, squarings, apply), with all
inputs resident in HBM before the timed region.  The default workload is the
stiff N = 16 case the headline metric is quoted on: 2^20 cells, 16 dust
species log-spaced over [1e-6, 1e2] dt, 3 velocity components, FP64.

Printed: one JSON line with the throughput in cell-updates/s, the roofline
of the dominant kernel (algorithmic FP64 flops per launch over the launch
time, both measured here with HIP events on the launch stream) and the
oracle's rate on the host as a reported CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix), public spec
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, public spec
METRIC = "FP64 cell-updates/s of exp(dt·K)·v at N=16, %FP64 peak; fwd+bwd vs fwd"

TABLE_Q = {1: 1, 2: 2, 3: 2, 4: 3, 5: 3, 6: 4, 7: 4, 8: 5, 9: 5}
TABLE_R = {1: 2, 2: 2, 3: 3, 4: 3, 5: 4, 6: 4, 7: 5, 8: 5, 9: 6}


def algorithmic_flops(k, m, s, N, D):
    """FP64 flops of the paper's method per cell in its dense (N+1) form:
    (r-1+s) dense products 2n^3 (Horner and squarings), (q-1) powers of the
    arrowhead matrix 2n(3n-2), the Paterson-Stockmeyer sums 2 m n^2 and the
    apply 2 D n^2, with n = N + 1."""
    n = N + 1
    q = np.vectorize(TABLE_Q.get)(k)
    r = np.vectorize(TABLE_R.get)(k)
    return ((r - 1 + s) * 2.0 * n ** 3 + (q - 1) * 2.0 * n * (3 * n - 2)
            + 2.0 * m * n ** 2 + 2.0 * D * n ** 2)


# Paterson-Stockmeyer split (q, r) of the MFMA forward per k (structured
# powers are cheap there; see csrc/wave.hpp kPsQ / kPsR)
PS_Q = {1: 2, 2: 4, 3: 3, 4: 5, 5: 4, 6: 4, 7: 5, 8: 5, 9: 5}
PS_R = {1: 1, 2: 1, 3: 2, 4: 2, 5: 3, 6: 4, 7: 4, 8: 5, 9: 6}


def executed_flops(k, m, s, N, D, mapping):
    """FP64 flops the library executes per cell.  MFMA kernel: (r-1) Horner
    products, s squarings and the apply on 16 x 16 tiles with a contraction
    length of 4 ceil(N / 4) (2 * 16^2 * that each), (q-1) structured powers
    (4 * 16^2) and the B-bar sums (2 * 16^2 per coefficient, q r of them).
    Lane kernel: Horner in the structured matrix (4 N^2 per degree), s
    squarings (2 N^3) and the apply (2 D N^2)."""
    if mapping == "wave":
        t, tk = 16, 4 * ((N + 3) // 4)
        q = np.vectorize(PS_Q.get)(k)
        r = np.vectorize(PS_R.get)(k)
        return ((r - 1 + s + 1) * 2.0 * t * t * tk + (q - 1) * 4.0 * t * t
                + 2.0 * q * r * t * t)
    return (s * 2.0 * N ** 3 + m * 4.0 * N * N + 2.0 * D * N * N)


def algorithmic_bytes(C, N, D):
    """HBM bytes one step must move: read rho_g, rho_d, t_stop, v; write v'."""
    return 8.0 * C * (1 + 2 * N + 2 * D * (N + 1))


KERNEL_SOURCES = {"k_forward_wave": ("common.hpp", "wave.hpp"),
                  "k_forward_lane": ("common.hpp", "lane.hpp"),
                  "k_forward_lane_stream": ("common.hpp", "lane.hpp"),
                  "k_forward_pair": ("common.hpp", "lane.hpp", "pair.hpp"),
                  "k_backward_pair": ("common.hpp", "lane.hpp", "pair.hpp"),
                  "k_forward_big": ("common.hpp", "wave.hpp", "big.hpp"),
                  "k_rk1_lane": ("common.hpp", "rk1.hpp")}


def forward_kernel(N, mapping, n_cells, n_dim=3):
    """The kernel drag_expm_apply launches for N species under `mapping`
    (contiguous arrays: the streaming one-lane kernel needs the velocity
    array, n_dim (N + 1) rows of n_cells, within 2^32 bytes)."""
    if mapping == "wave":
        return "k_forward_wave" if N <= 16 else "k_forward_big"
    if N <= 6:
        return "k_forward_lane"
    if N <= 8:
        fits = 8 * n_dim * (N + 1) * n_cells < 1 << 32
        return "k_forward_lane_stream" if fits else "k_forward_lane"
    return "k_forward_pair"


def source_hash(kernel):
    """Short SHA-256 over the sources that define `kernel` and the compiler
    flags; a profile summary records the hash its counters were taken on."""
    import hashlib
    from paper_2509_25347_amd import _lib
    h = hashlib.sha256(" ".join(_lib.HIPCC_FLAGS).encode())
    csrc = os.path.join(ROOT, "paper_2509_25347_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 summary of this kernel
    and workload (FETCH_SIZE + WRITE_SIZE scaled by the copy calibration), or
    None when there is none or the sources have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("hbm_bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                fields[k] = v.strip()
    if fields.get("source_sha256") != source_hash(kernel) or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


def cpu_baseline(d, budget_s=12.0, chunk=4096):
    """The oracle (single thread) on a bounded prefix of the same workload."""
    import oracle
    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    C = d["rho_g"].shape[0]
    done, t_used = 0, 0.0
    while done < C and t_used < budget_s:
        sl = slice(done, min(C, done + chunk))
        t0 = time.perf_counter()
        oracle.apply_cells(d["rho_g"][sl], d["rho_d"][:, sl], d["t_stop"][:, sl],
                           d["v"][:, :, sl], d["dt"])
        t_used += time.perf_counter() - t0
        done = sl.stop
    return {"value": done / t_used, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} cells of the workload, single thread, {t_used:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="n16_stiff_3d")
    ap.add_argument("--cells", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the fused-adjoint and batched comparisons against the plain forward")
    ap.add_argument("--extra", action="store_true",
                    help="also time the other workloads, the fused adjoint and the batched launch")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the fused forward + adjoint (drag_expm_apply_backward) on the "
                         "workload instead of the forward (for profiling the adjoint kernels)")
    ap.add_argument("--batched", action="store_true",
                    help="time only the batched uneven-N graph (4096 blocks x 512 cells, K = 9, "
                         "autotuned) for profiling its kernels")
    ap.add_argument("--pin", default=None,
                    help="with --batched: LANE_MAX,MODE (e.g. 10,per_n) instead of the "
                         "autotuner's choice, so that profiling runs launch the same kernels")
    ap.add_argument("--rk1", action="store_true",
                    help="time the backward Euler step (drag_rk1_apply) on the workload instead "
                         "of the exponential, with its HBM roofline")
    ap.add_argument("--sweep", action="store_true",
                    help="time per cell of the exponential (K = 9 and the tuned cap) and of the "
                         "backward Euler step for N = 1..16 on 64^3 cells (the paper's Fig. 6 "
                         "axes); one JSON object")
    ap.add_argument("--k-sweep", action="store_true",
                    help="time every Taylor cap K = 2..9 per species count N = 1..16 (stiff and "
                         "jittered recipes, 2^18 cells, interleaved repeats); one JSON object")
    ap.add_argument("--mapping-sweep", action="store_true",
                    help="forward and fused-adjoint time per launch under every mapping that "
                         "takes N = 1..16 (stiff recipe, 2^18 cells); one JSON object")
    ap.add_argument("--squaring-cost", action="store_true",
                    help="the N = 16 stiff workload at dt 2^j, j = 0..4: one more squaring per "
                         "doubling at fixed k*, m*; the fitted cost per squaring; one JSON object")
    ap.add_argument("--report", action="store_true",
                    help="every workload configuration: GPU rate, roofline fractions, and the "
                         "oracle beside it (1-core and all-core rates, errors on the same "
                         "sample); one JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (3 times), the "
                         "reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--side-only", action="store_true",
                    help="only the side measurements of the default run (fused adjoint, "
                         "batched, RK1, bound test, Pade), one JSON object; the default run "
                         "takes them from a child process started this way")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the drag update is cell-local and would shard by cell ranges)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_25347_amd import _lib, ops, workloads

    _lib.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": src.numel() * 8,
                          "copy_calibration_bytes_written": dst.numel() * 8}), flush=True)
        return

    name = args.workload
    if args.report:
        print(json.dumps(config_report(torch, ops, _lib, workloads, dev)), flush=True)
        return
    if args.sweep:
        print(json.dumps(n_sweep(torch, ops, _lib, workloads, dev)), flush=True)
        return
    if args.k_sweep:
        print(json.dumps(k_sweep(torch, ops, _lib, workloads, dev)), flush=True)
        return
    if args.mapping_sweep:
        print(json.dumps(mapping_sweep(torch, ops, _lib, workloads, dev)), flush=True)
        return
    if args.squaring_cost:
        print(json.dumps(squaring_cost(torch, ops, workloads, dev)), flush=True)
        return
    if args.adjoint:
        print(json.dumps(adjoint_only(torch, ops, _lib, workloads, dev, name, args)), flush=True)
        return
    if args.batched:
        print(json.dumps(batched_only(torch, ops, workloads, dev, args)), flush=True)
        return
    if args.side_only:
        print(json.dumps(side_measurements(torch, ops, _lib, workloads, dev)), flush=True)
        return
    if args.rk1:
        print(json.dumps(rk1_only(torch, ops, workloads, dev, name, args)), flush=True)
        return
    d = workloads.make(name, args.cells)
    C = d["rho_g"].shape[0]
    N = d["rho_d"].shape[0]
    D = d["v"].shape[0]
    T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
    out = torch.empty_like(T["v"])
    mapping = {1: "lane", 2: "wave"}[_lib.get_mapping(N)]

    # per-cell (k*, m*, s*) for the flop count (outside the timed region)
    _, _, _, kk, mm, ss = ops.build(T["rho_g"], T["rho_d"], T["t_stop"], d["dt"])
    kk, mm, ss = (x.cpu().numpy() for x in (kk, mm, ss))
    f_alg = float(algorithmic_flops(kk, mm, ss, N, D).sum())
    f_exe = float(executed_flops(kk, mm, ss, N, D, mapping).sum())
    b_alg = algorithmic_bytes(C, N, D)

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], out=out)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    value = C * args.steps / (ms_total * 1e-3)

    achieved_tflops = f_alg / (ms_per_step * 1e-3) / 1e12
    roof = {
        "bound": "mfma" if mapping == "wave" else "alu",
        "achieved": round(achieved_tflops, 3),
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved_tflops / FP64_PEAK_TFLOPS, 4),
        "traffic": profiled_traffic(forward_kernel(N, mapping, C, D), name),
        "kernel": f"{forward_kernel(N, mapping, C, D)}<{N}>",
        "flops_per_launch": f_alg,
        "executed_flops_per_launch": f_exe,
        "executed_frac": round(f_exe / (ms_per_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
        "hbm_bytes_per_launch": b_alg,
        "hbm_frac": round(b_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "n_cells": C, "n_species": N, "n_dim": D,
                   "dt": d["dt"], "k_max": 9, "option": 2, "mapping": mapping,
                   "s_star": [int(ss.min()), int(ss.max())],
                   "m_star": [int(mm.min()), int(mm.max())]},
        "roofline": roof,
        "wall_s_timed": wall,
    }
    # The side measurements run in a child process (this script with
    # --side-only), so that the headline line above survives whatever happens
    # to them; each reports an error in place instead.
    if not args.no_comparisons:
        res.update(_side_in_child())
    if args.extra:
        try:
            res["extra"] = extra_measurements(torch, ops, workloads, dev)
        except Exception as e:  # noqa: BLE001
            res["extra"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        try:
            res["cpu_baseline"] = cpu_baseline(d)
        except Exception as e:  # noqa: BLE001
            res["cpu_baseline"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(res), flush=True)


SIDE_KEYS = ("fwd_bwd_vs_fwd", "batched_vs_plain", "rk1_vs_expm", "bound_test", "pade_vs_taylor")


def side_measurements(torch, ops, _lib, workloads, dev):
    """The comparisons beside the headline, each reporting an error in place."""
    res = {}
    fns = {"fwd_bwd_vs_fwd": lambda: adjoint_measurement(torch, ops, workloads, dev),
           "batched_vs_plain": lambda: batched_measurement(torch, ops, workloads, dev),
           "rk1_vs_expm": lambda: rk1_measurement(torch, ops, workloads, dev),
           "bound_test": lambda: bound_test_measurement(torch, ops, _lib, workloads, dev),
           "pade_vs_taylor": lambda: pade_measurement(torch, ops, _lib, workloads, dev)}
    for key in SIDE_KEYS:
        _progress(f"side measurement: {key}")
        try:
            res[key] = fns[key]()
        except Exception as e:  # noqa: BLE001
            res[key] = {"error": f"{type(e).__name__}: {e}"}
    return res


def _side_in_child(timeout_s=300):
    """Run side_measurements in a child process and return its result, or an
    error entry per key when the child fails (its stderr goes to ours)."""
    import subprocess
    try:
        p = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--side-only"],
                           stdout=subprocess.PIPE, timeout=timeout_s, check=False, text=True)
        lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
        if p.returncode == 0 and lines:
            return json.loads(lines[-1])
        why = f"side measurements exited with status {p.returncode}"
    except subprocess.TimeoutExpired:
        why = f"side measurements exceeded {timeout_s} s"
    return {k: {"error": why} for k in SIDE_KEYS}


def _progress(msg):
    """One progress line on stderr (the JSON result goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def _time(torch, fn, steps, warmup, chunks=1):
    """ms per call: HIP events around `steps` calls after `warmup`; with
    chunks > 1 the median over that many such runs (the per-launch time of
    the sub-millisecond kernels wanders by about 10 % between runs on these
    boxes, with no gaps between the kernels in their traces)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    runs = []
    for _ in range(chunks):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1) / steps)
    return float(np.median(runs))


def _interleaved(torch, fns, steps, warmup, rounds=5):
    """Median ms per call of each function, timed in alternation (`rounds`
    rounds of `steps` calls each) so that a ratio between them does not
    carry the drift of the GPU's clock from one run to the next."""
    for fn in fns:
        for _ in range(warmup):
            fn()
    torch.cuda.synchronize()
    runs = [[] for _ in fns]
    for _ in range(rounds):
        for i, fn in enumerate(fns):
            runs[i].append(_time(torch, fn, steps, 0))
    return [float(np.median(r)) for r in runs]


def _graph_time(torch, fn, launches=20, replays=20):
    """Device time per launch with the host out of the loop: `launches`
    calls captured into one HIP graph (torch.cuda.graph on its capture
    stream, which the library launches on) and replayed; ms per launch."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(launches):
            fn()
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (replays * launches)


def _oracle_rates(d, sample, threads):
    """Oracle (CPU leg) on the first `sample` cells: its outputs, the
    single-thread rate, and the rate with `threads` threads over chunks (the
    oracle is a C library; ctypes releases the GIL during each call)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    sl = slice(0, sample)
    args = (d["rho_g"][sl], d["rho_d"][:, sl], d["t_stop"][:, sl], d["v"][:, :, sl], d["dt"])
    t0 = time.perf_counter()
    ref, _, nrm, _ = oracle.apply_cells(*args)
    t1 = time.perf_counter() - t0
    bounds = np.linspace(0, sample, 4 * threads + 1).astype(int)
    chunks = [slice(a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]

    def run(c):
        oracle.apply_cells(d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c], d["v"][:, :, c],
                           d["dt"])

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, chunks))
    tp = time.perf_counter() - t0
    return ref, nrm, sample / t1, sample / tp


def _err_stats(got, ref, v):
    scale = np.abs(v).max(axis=1)
    scale = np.where(scale == 0, 1.0, scale)
    e = (np.abs(got - ref).max(axis=1) / scale).max(axis=0)
    return {"max": float(e.max()), "p99.9": float(np.quantile(e, 0.999)),
            "median": float(np.median(e))}


def _exact_stats(d, got, ref, dt):
    """Errors against the exact exponential (the oracle's long-double truth,
    no scaling and squaring) on the oracle's sample: the GPU's, the
    oracle's, and the GPU's excess over the oracle's own error per cell."""
    import oracle
    C = ref.shape[-1]
    v = d["v"][..., :C]
    tr = oracle.truth_apply(d["rho_g"][:C], d["rho_d"][:, :C], d["t_stop"][:, :C], v, dt)
    scale = np.abs(v).max(axis=1)
    scale = np.where(scale == 0, 1.0, scale)

    def per_cell(x, y):
        return (np.abs(x - y).max(axis=1) / scale).max(axis=0)

    e_gx, e_ox, e_go = per_cell(got, tr), per_cell(ref, tr), per_cell(got, ref)

    def stats(e):
        return {"max": float(e.max()), "p99.9": float(np.quantile(e, 0.999)),
                "median": float(np.median(e))}

    return {"gpu_vs_exact": stats(e_gx), "oracle_vs_exact": stats(e_ox),
            "max_gpu_vs_oracle_minus_oracle_vs_exact": float((e_go - e_ox).max())}


def config_report(torch, ops, _lib, workloads, dev):
    """All five workload configurations on one GPU, with the oracle timed
    beside the GPU on a bounded sample of the same cells (single thread and
    all cores) and the GPU's per-cell errors against it on that sample
    (error of a cell: max over components and species of |dv'| / ||v_in||_inf)."""
    threads = min(16, len(os.sched_getaffinity(0)))
    out = {"threads": threads}
    for cfg, name, sample in ((1, "n1_closed_form", 4096), (2, "n4_3d", 1 << 16),
                              (3, "n16_stiff_3d", 1 << 13), (5, "n8_adjoint_3d", 1 << 15)):
        _progress(f"report: config {cfg} ({name})")
        d = workloads.make(name)
        C, N, D = d["rho_g"].shape[0], d["rho_d"].shape[0], d["v"].shape[0]
        T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
        o = torch.empty_like(T["v"])
        ms = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                 d["dt"], out=o), 50, 5, chunks=5)
        got = o.cpu().numpy()
        _, _, _, kk, mm, ss = ops.build(T["rho_g"], T["rho_d"], T["t_stop"], d["dt"])
        kk, mm, ss = (x.cpu().numpy() for x in (kk, mm, ss))
        f_alg = float(algorithmic_flops(kk, mm, ss, N, D).sum())
        _progress(f"report: config {cfg} oracle")
        ref, nrm, r1, rp = _oracle_rates(d, min(sample, C), threads)
        _progress(f"report: config {cfg} errors")
        row = {"workload": name, "cells": C, "ms": ms, "cells_per_s": C / (ms * 1e-3),
               "fp64_frac": f_alg / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
               "hbm_frac": algorithmic_bytes(C, N, D) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "err_vs_oracle": _err_stats(got[..., :ref.shape[-1]], ref, d["v"][..., :ref.shape[-1]]),
               "err_vs_exact": _exact_stats(d, got[..., :ref.shape[-1]], ref, d["dt"]),
               "oracle_sample": int(ref.shape[-1]), "oracle_1core_cells_per_s": r1,
               "oracle_all_cores_cells_per_s": rp}
        if cfg == 1:  # launch-bound: the device time per launch, from graph replays
            row["graph_replay_us_per_launch"] = 1e3 * _graph_time(
                torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                              d["dt"], out=o))
        ms_auto = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                      d["dt"], k_max=_lib.K_AUTO, out=o), 50, 5,
                        chunks=5)
        row["taylor_cap_tuned"] = {"k_max": _lib.get_k_max(N), "ms": ms_auto,
                                   "cells_per_s": C / (ms_auto * 1e-3), "speedup_vs_k9": ms / ms_auto}
        if cfg == 5:
            dd = workloads.make(name, with_weights=True)
            Tw = torch.from_numpy(dd["w"]).to(dev)
            tf, tb = _interleaved(torch, [
                lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], out=o),
                lambda: ops.expm_apply_backward(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], Tw,
                                                d["dt"])], 20, 3)
            row["fwd_bwd_ms"] = tb
            row["fwd_ms_alternating"] = tf
            row["fwd_bwd_over_fwd"] = tb / tf
        out[f"config{cfg}"] = row
    # config 4: the batched launch; the oracle on the first 32 blocks
    _progress("report: config 4 (batched)")
    batch = workloads.make_batched()
    plan = ops.BatchPlan(batch["n_species"], batch["block_cells"], 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    vo = torch.empty_like(v)
    plan.autotune(fields, v, vo)
    _progress("report: config 4 timing")
    ms = _time(torch, lambda: plan.apply(fields, v, vo), 20, 3)
    cells = len(batch["blocks"]) * batch["block_cells"]
    # algorithmic work: the blocks of each N concatenated, (k*, m*, s*) from drag_build
    f_alg = 0.0
    for N in range(1, 17):
        bl = [blk for blk, n in zip(batch["blocks"], batch["n_species"]) if n == N]
        if not bl:
            continue
        cat = {k: np.concatenate([x[k] for x in bl], -1) for k in ("rho_g", "rho_d", "t_stop")}
        kk, mm, ss = _lib_select_cells(ops, cat, batch["dt"], dev)
        f_alg += float(algorithmic_flops(kk, mm, ss, N, 3).sum())
    # the oracle on the first 32 blocks: one thread, then one block per thread
    _progress("report: config 4 oracle")
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    sample = batch["blocks"][:32]

    def run(blk):
        return oracle.apply_cells(blk["rho_g"], blk["rho_d"], blk["t_stop"], blk["v"], batch["dt"])

    t0 = time.perf_counter()
    refs = [run(blk) for blk in sample]
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, sample))
    tp = time.perf_counter() - t0
    errs, ex = [], []
    for b, (blk, r) in enumerate(zip(sample, refs)):
        got = plan.block_view(vo, b).cpu().numpy()
        scale = np.abs(blk["v"]).max(axis=1)
        errs.append((np.abs(got - r[0]).max(axis=1) / np.where(scale == 0, 1, scale)).max(axis=0))
        ex.append(_exact_stats(blk, got, r[0], batch["dt"]))
    e = np.concatenate(errs)
    exact = {k: {s: max(x[k][s] for x in ex) for s in ("max", "p99.9")}
             for k in ("gpu_vs_exact", "oracle_vs_exact")}
    exact["note"] = "max over the 32 blocks of each block's max and p99.9"
    exact["max_gpu_vs_oracle_minus_oracle_vs_exact"] = max(
        x["max_gpu_vs_oracle_minus_oracle_vs_exact"] for x in ex)
    _progress("report: config 4 done")
    plan.close()
    out["config4"] = {"workload": "batched 4096 x 512, N_b ~ U{1..16}", "cells": cells, "ms": ms,
                      "cells_per_s": cells / (ms * 1e-3),
                      "fp64_frac": f_alg / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                      "err_vs_oracle": {"max": float(e.max()), "p99.9": float(np.quantile(e, 0.999)),
                                        "median": float(np.median(e))},
                      "err_vs_exact": exact,
                      "oracle_sample": int(e.size),
                      "oracle_1core_cells_per_s": e.size / t1,
                      "oracle_all_cores_cells_per_s": e.size / tp}
    return out


def _lib_select_cells(ops, blk, dt, dev):
    """(k*, m*, s*) of a block's cells from drag_build."""
    import torch
    T = {k: torch.from_numpy(np.ascontiguousarray(blk[k])).to(dev) for k in ("rho_g", "rho_d", "t_stop")}
    _, _, _, k, m, s = ops.build(T["rho_g"], T["rho_d"], T["t_stop"], dt)
    return k.cpu().numpy(), m.cpu().numpy(), s.cpu().numpy()


def adjoint_only(torch, ops, _lib, workloads, dev, name, args):
    """The fused forward + adjoint on one workload (loss weights w ~ N(0, 1))."""
    d = workloads.make(name, args.cells, with_weights=True)
    T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v", "w")}
    N = d["rho_d"].shape[0]
    C = d["rho_g"].shape[0]
    ms = _time(torch, lambda: ops.expm_apply_backward(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                      T["w"], d["dt"]), args.steps, args.warmup)
    return {"metric": "FP64 fused forward + adjoint cell-updates/s", "value": C / (ms * 1e-3),
            "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": name, "n_cells": C, "n_species": N}}


def batched_only(torch, ops, workloads, dev, args):
    """The batched uneven-N graph alone (K = 9, the plan autotuned on the
    data first, outside the timed launches)."""
    batch = workloads.make_batched()
    plan = ops.BatchPlan(batch["n_species"], batch["block_cells"], 3, batch["dt"], k_max=9)
    fields, v = plan.pack(batch["blocks"], dev)
    out = torch.empty_like(v)
    if args.pin:
        lm, mode = args.pin.split(",")
        plan.set_config(int(lm), mode)
    else:
        plan.autotune(fields, v, out)
    lane_max, mfma_mode = plan.config()
    ms = _time(torch, lambda: plan.apply(fields, v, out), args.steps, args.warmup)
    plan.close()
    cells = len(batch["blocks"]) * batch["block_cells"]
    return {"metric": "FP64 cell-updates/s of the batched uneven-N graph", "value": cells / (ms * 1e-3),
            "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "4096 blocks x 512 cells, N_b ~ U{1..16}, D = 3",
                       "n_cells": cells, "lane_max": lane_max, "mfma_mode": mfma_mode}}


def n_sweep(torch, ops, _lib, workloads, dev, cells=1 << 18):
    """Time per cell against the species count, as the paper plots it (Fig. 6:
    EXP and RK1 on 64^3 cells): stiff and jittered synthetic cells (the
    Dustywave stopping times are not available), D = 3, the default mapping."""
    out = {"cells": cells, "rows": []}
    for recipe, make in (("stiff", workloads.make_stiff), ("jittered", workloads.make_jittered)):
        for N in range(1, 17):
            d = make(N, cells)
            T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
                 for k in ("rho_g", "rho_d", "t_stop", "v")}
            o = torch.empty_like(T["v"])
            t9 = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                     d["dt"], out=o), 20, 3)
            ta = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                     d["dt"], k_max=_lib.K_AUTO, out=o), 20, 3)
            tr = _time(torch, lambda: ops.rk1_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                    d["dt"], out=o), 20, 3)
            out["rows"].append({"recipe": recipe, "N": N, "exp_k9_s_per_cell": t9 * 1e-3 / cells,
                                "exp_auto_s_per_cell": ta * 1e-3 / cells,
                                "rk1_s_per_cell": tr * 1e-3 / cells, "k_auto": _lib.get_k_max(N),
                                "exp_over_rk1": min(t9, ta) / tr})
    return out


def k_sweep(torch, ops, _lib, workloads, dev, cells=1 << 18, reps=3):
    """The Taylor cap K (Alg. 1's k_max: every K is u-accurate, it trades
    polynomial degree against squarings) against time, per species count and
    recipe: for each N, every K = 2..9 timed `reps` times in rotating order
    (20 launches each), medians; the fastest K is what the library's
    K_AUTO table should hold for that N."""
    out = {"cells": cells, "rows": []}
    Ks = list(range(2, 10))
    for recipe, make in (("stiff", workloads.make_stiff), ("jittered", workloads.make_jittered)):
        for N in range(1, 17):
            d = make(N, cells)
            T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
                 for k in ("rho_g", "rho_d", "t_stop", "v")}
            o = torch.empty_like(T["v"])
            times = {K: [] for K in Ks}
            for rep in range(reps):
                order = Ks[rep % len(Ks):] + Ks[:rep % len(Ks)]
                for K in order:
                    times[K].append(_time(torch, lambda: ops.expm_apply(
                        T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], k_max=K, out=o),
                        20, 2))
            med = {K: float(np.median(v)) for K, v in times.items()}
            best = min(med, key=med.get)
            out["rows"].append({"recipe": recipe, "N": N, "ms": med, "best_k": best,
                                "best_over_k9": med[best] / med[9],
                                "k_auto": _lib.get_k_max(N)})
    return out


def mapping_sweep(torch, ops, _lib, workloads, dev, cells=1 << 18):
    """Forward and fused adjoint time per launch under every mapping that
    takes N (stiff recipe, 2^18 cells, D = 3, K = 9): the lane mapping (one
    lane per cell to N = 8, two lanes per cell above) and the MFMA quad; the
    library's default per N is the faster one."""
    rows = []
    for N in range(1, 17):
        d = workloads.make_stiff(N, cells)
        T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
             for k in ("rho_g", "rho_d", "t_stop", "v")}
        w = torch.randn_like(T["v"])
        o = torch.empty_like(T["v"])
        row = {"N": N, "default": {1: "lane", 2: "wave"}[_lib.get_mapping(N)]}
        for name, mp in (("lane", _lib.MAP_LANE), ("wave", _lib.MAP_WAVE)):
            if mp == _lib.MAP_LANE and N > 12:
                continue
            try:
                _lib.set_mapping(N, mp)
                row[f"fwd_{name}_ms"] = _time(torch, lambda: ops.expm_apply(
                    T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], out=o), 10, 2)
                if mp == _lib.MAP_WAVE or N <= 10:
                    row[f"adj_{name}_ms"] = _time(torch, lambda: ops.expm_apply_backward(
                        T["rho_g"], T["rho_d"], T["t_stop"], T["v"], w, d["dt"]), 5, 1)
            finally:
                _lib.set_mapping(N, _lib.MAP_AUTO)
        rows.append(row)
    return {"cells": cells, "recipe": "stiff", "rows": rows}


def squaring_cost(torch, ops, workloads, dev, steps=50):
    """Cost of one squaring in the shipped N = 16 kernel: the stiff workload
    at dt 2^j, j = 0..4.  Each doubling of dt doubles ||dt K||_1, which in
    Alg. 1's scaled branch adds exactly one squaring (s* + 1) with the same
    k* and m* (the scaled norm 2^-s* ||dt K||_1 is the same number), so the
    time differences are the squarings' share, the rest (set-up, polynomial
    stage, apply, memory) the intercept."""
    d = workloads.make("n16_stiff_3d")
    C = d["rho_g"].shape[0]
    T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
    o = torch.empty_like(T["v"])
    rows = []
    for j in range(5):
        dt = d["dt"] * 2.0 ** j
        _, _, _, kk, mm, ss = ops.build(T["rho_g"], T["rho_d"], T["t_stop"], dt)
        ms = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], dt,
                                                 out=o), steps, 5)
        rows.append({"dt": dt, "ms": ms, "s_star": [int(ss.min()), int(ss.max())],
                     "k_star": [int(kk.min()), int(kk.max())], "m_star": [int(mm.min()), int(mm.max())]})
    x = np.array([r["s_star"][0] for r in rows], dtype=float)
    y = np.array([r["ms"] for r in rows])
    slope, icpt = np.polyfit(x, y, 1)
    simds, clock = 1024, 2.4e9
    per_cell = lambda ms: ms * 1e-3 * clock * simds / C  # noqa: E731
    return {"workload": "n16_stiff_3d", "cells": C, "rows": rows,
            "ms_per_squaring": float(slope),
            "simd_cycles_per_cell_per_squaring": float(per_cell(slope)),
            "mfma_cycles_per_cell_per_squaring": 4 * 64,
            "simd_cycles_per_cell_outside_squarings": float(per_cell(icpt)),
            "note": "one 16x16 product per squaring per cell: 4 FP64 MFMAs of 64 cycles"}


def rk1_roofline(ms, C, N, D, workload):
    """HBM roofline of the backward Euler kernel: it moves the same bytes as
    the exponential (read rho_g, rho_d, t_stop, v; write v')."""
    b = algorithmic_bytes(C, N, D)
    gbs = b / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": profiled_traffic("k_rk1_lane", workload),
            "kernel": f"k_rk1_lane<{N}>", "hbm_bytes_per_launch": b}


def rk1_only(torch, ops, workloads, dev, name, args):
    """The backward Euler step alone on one workload (for profiling k_rk1_lane)."""
    d = workloads.make(name, args.cells)
    T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
    out = torch.empty_like(T["v"])
    C, N, D = d["rho_g"].shape[0], d["rho_d"].shape[0], d["v"].shape[0]
    ms = _time(torch, lambda: ops.rk1_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"],
                                            out=out), args.steps, args.warmup)
    return {"metric": "FP64 backward Euler cell-updates/s", "value": C / (ms * 1e-3),
            "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": name, "n_cells": C, "n_species": N, "n_dim": D},
            "roofline": rk1_roofline(ms, C, N, D, name)}


def rk1_measurement(torch, ops, workloads, dev, names=("n16_stiff_3d", "n8_adjoint_3d", "n4_3d")):
    """The paper's yardstick beside the exponential: the backward Euler step
    (drag_rk1_apply) on the same cells, its HBM roofline, the time ratio
    EXP / RK1, and how far one RK1 step lands from exp(dt K) v (per cell:
    max |v'_rk1 - v'_exp| / ||v||_inf; median and max over the cells)."""
    res = {}
    for name in names:
        d = workloads.make(name)
        C, N, D = d["rho_g"].shape[0], d["rho_d"].shape[0], d["v"].shape[0]
        T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
        o1, o2 = torch.empty_like(T["v"]), torch.empty_like(T["v"])
        t_rk1 = _time(torch, lambda: ops.rk1_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                   d["dt"], out=o1), 30, 3, chunks=5)
        t_exp = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                    d["dt"], out=o2), 20, 3, chunks=5)
        scale = T["v"].abs().amax(dim=1)
        gap = ((o1 - o2).abs().amax(dim=1) / scale).amax(dim=0)
        res[name] = {"n_cells": C, "n_species": N, "rk1_ms": t_rk1, "expm_ms": t_exp,
                     "expm_over_rk1": t_exp / t_rk1, "rk1_cells_per_s": C / (t_rk1 * 1e-3),
                     "rk1_roofline": rk1_roofline(t_rk1, C, N, D, name),
                     "rk1_step_gap_to_exp": {"median": float(gap.median()), "max": float(gap.max())}}
    return res


def bound_test_measurement(torch, ops, _lib, workloads, dev):
    """Sastre's second modification (option bit DRAG_OPTION_BOUND_TEST, MFMA
    kernel) against the same MFMA kernel without it: time, and the cells
    whose result it changed (where a product was dropped and the rounding
    differs)."""
    res = {}
    for name in ("n16_stiff_3d", "n8_adjoint_3d", "n1_closed_form"):
        d = workloads.make(name)
        N = d["rho_d"].shape[0]
        T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
        o1, o2 = torch.empty_like(T["v"]), torch.empty_like(T["v"])
        try:
            _lib.set_mapping(N, _lib.MAP_WAVE)
            t0 = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                     d["dt"], out=o1), 20, 3)
        finally:
            _lib.set_mapping(N, _lib.MAP_AUTO)
        t1 = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                 d["dt"], option=2 | _lib.OPTION_BOUND_TEST,
                                                 out=o2), 20, 3)
        changed = int(((o1 - o2).abs().amax(dim=(0, 1)) > 0).sum())
        res[name] = {"mfma_ms": t0, "mfma_bound_test_ms": t1, "time_ratio": t1 / t0,
                     "cells_changed": changed, "n_cells": int(d["rho_g"].shape[0])}
    return res


def pade_measurement(torch, ops, _lib, workloads, dev, sample=128):
    """The diagonal Pade scaling step (option bit DRAG_OPTION_PADE, MFMA
    kernel) against the Taylor step: time (the default Taylor path, and the
    Taylor step on the same MFMA kernel), mean degree and squarings from
    drag_build, and the error against the exact exponential (long-double
    eigen-decomposition) on the first `sample` cells."""
    import oracle
    res = {}
    for name in ("n16_stiff_3d", "n8_adjoint_3d"):
        d = workloads.make(name)
        N = d["rho_d"].shape[0]
        T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
        o_t, o_w, o_p = (torch.empty_like(T["v"]) for _ in range(3))
        t_default = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                        d["dt"], out=o_t), 20, 3)
        try:
            _lib.set_mapping(N, _lib.MAP_WAVE)
            t_wave = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"],
                                                         T["v"], d["dt"], out=o_w), 20, 3)
        finally:
            _lib.set_mapping(N, _lib.MAP_AUTO)
        t_pade = _time(torch, lambda: ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                                     d["dt"], option=_lib.OPTION_PADE, out=o_p),
                       20, 3)
        row = {"n_cells": int(d["rho_g"].shape[0]), "taylor_default_ms": t_default,
               "taylor_mfma_ms": t_wave, "pade_mfma_ms": t_pade,
               "pade_over_taylor_mfma": t_pade / t_wave, "pade_over_taylor_default": t_pade / t_default}
        for lab, opt in (("taylor", 2), ("pade", _lib.OPTION_PADE)):
            _, _, _, kk, mm, ss = ops.build(T["rho_g"], T["rho_d"], T["t_stop"], d["dt"], option=opt)
            row[f"{lab}_mean_m"] = float(mm.double().mean())
            row[f"{lab}_mean_s"] = float(ss.double().mean())
        v = d["v"][..., :sample]
        exact = np.empty_like(v)
        for c in range(sample):
            E = oracle.truth_eigen(d["dt"], d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c])
            exact[:, :, c] = v[:, :, c] @ E.T
        scale = np.abs(v).max(axis=1)
        for lab, o in (("taylor", o_t), ("pade", o_p)):
            e = (np.abs(o[..., :sample].cpu().numpy() - exact).max(axis=1) / scale).max(axis=0)
            row[f"{lab}_err_vs_exact"] = {"max": float(e.max()), "median": float(np.median(e))}
        res[name] = row
    return res


def adjoint_measurement(torch, ops, workloads, dev):
    """Fused forward + adjoint against the plain forward, N = 8, 2^18 cells."""
    dd = workloads.make("n8_adjoint_3d", with_weights=True)
    TT = {k: torch.from_numpy(dd[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v", "w")}
    oo = torch.empty_like(TT["v"])
    tf, tb = _interleaved(torch, [
        lambda: ops.expm_apply(TT["rho_g"], TT["rho_d"], TT["t_stop"], TT["v"], dd["dt"], out=oo),
        lambda: ops.expm_apply_backward(TT["rho_g"], TT["rho_d"], TT["t_stop"], TT["v"],
                                        TT["w"], dd["dt"])], 10, 3)
    # FMAs per cell of the two as implemented, at the cells' own (m*, s*):
    # forward = structured Horner (2N^2 + N per degree), Y-form squarings
    # (N^3 each), apply (D N^2); fused (the two-lane kernel at N = 8) =
    # Horner on Y and dY with the direction as D outer products and the
    # vectors (Y + cI) ubar_d by their own O(N) recurrence
    # (4N^2 + 2N + D N^2 + 3 D N per degree), three products per squaring
    # (3 N^3), both applies (2 D N^2)
    _, _, _, _, mm, ss = ops.build(TT["rho_g"], TT["rho_d"], TT["t_stop"], dd["dt"])
    m, s = float(mm.double().mean()), float(ss.double().mean())
    N, D = int(TT["rho_d"].shape[0]), int(TT["v"].shape[0])
    fma_f = (2 * N * N + N) * m + N ** 3 * s + D * N * N
    fma_b = (4 * N * N + 2 * N + D * N * N + 3 * D * N) * m + 3 * N ** 3 * s + 2 * D * N * N
    return {"workload": "n8_adjoint_3d", "n_cells": int(dd["rho_g"].shape[0]),
            "fwd_ms": tf, "fwd_bwd_ms": tb, "fwd_bwd_over_fwd": tb / tf,
            "fma_per_cell": {"fwd": fma_f, "fwd_bwd": fma_b, "ratio": fma_b / fma_f,
                             "mean_m": m, "mean_s": s},
            "timing": "medians of 5 alternating runs of 10 calls each"}


def batched_measurement(torch, ops, workloads, dev):
    """The batched uneven-N graph against the plain per-N launches over the
    same cells (blocks grouped by N into contiguous arrays), first with the
    paper's K = 9 for every N, then with the Taylor cap tuned per N by the
    plan's autotuner (the plain launches then use the same per-N caps)."""
    import numpy as np
    from paper_2509_25347_amd import _lib
    batch = workloads.make_batched()
    groups = {}
    for b, blk in enumerate(batch["blocks"]):
        groups.setdefault(int(batch["n_species"][b]), []).append(blk)
    per = []
    for N, bl in sorted(groups.items()):
        cat = {k: torch.from_numpy(np.ascontiguousarray(np.concatenate([x[k] for x in bl], -1))).to(dev)
               for k in ("rho_g", "rho_d", "t_stop", "v")}
        per.append((N, cat, torch.empty_like(cat["v"])))
    cells = len(batch["blocks"]) * batch["block_cells"]
    res = {"workload": "4096 blocks x 512 cells, N_b ~ U{1..16}, D = 3", "n_cells": cells}
    for label, k_req in (("k9", 9), ("k_auto", _lib.K_AUTO)):
        plan = ops.BatchPlan(batch["n_species"], batch["block_cells"], 3, batch["dt"], k_max=k_req)
        fields, v = plan.pack(batch["blocks"], dev)
        out = torch.empty_like(v)
        plan.autotune(fields, v, out)
        lane_max, mfma_mode = plan.config()
        ks = plan.k_max()
        def plain():
            for N, cat, o in per:
                ops.expm_apply(cat["rho_g"], cat["rho_d"], cat["t_stop"], cat["v"], batch["dt"],
                               k_max=ks[N - 1], out=o)

        tb, tp = _interleaved(torch, [lambda: plan.apply(fields, v, out), plain], 5, 2)
        plan.close()
        row = {"batched_ms": tb, "plain_per_n_ms": tp, "batched_over_plain": tb / tp,
               "batched_cells_per_s": cells / (tb * 1e-3), "lane_max": lane_max,
               "mfma_mode": mfma_mode}
        if label == "k9":
            res.update(row)
        else:
            row["k_max_per_n"] = ks
            res["taylor_cap_tuned"] = row
    res["taylor_cap_tuned"]["speedup_vs_k9"] = res["batched_ms"] / res["taylor_cap_tuned"]["batched_ms"]
    return res


def extra_measurements(torch, ops, workloads, dev):
    ex = {}
    for name in ("n4_3d", "n8_adjoint_3d", "n1_closed_form"):
        dd = workloads.make(name)
        TT = {k: torch.from_numpy(dd[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
        oo = torch.empty_like(TT["v"])
        ms = _time(torch, lambda: ops.expm_apply(TT["rho_g"], TT["rho_d"], TT["t_stop"], TT["v"],
                                                 dd["dt"], out=oo), 20, 3)
        ex[name] = {"ms": ms, "cells_per_s": dd["rho_g"].shape[0] / (ms * 1e-3)}
    return ex


if __name__ == "__main__":
    main()
