"""Benchmark of the dense Pauli decomposition on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--N 14] [--no-cpu] [--no-fp64]
    python bench.py --workload batch      # 512 uneven matrices, N in 3..9
    python bench.py --workload backward   # 8 x N=11 forward + backward

Workload: one complex64 Hermitian 16384 x 16384 matrix (N = 14 qubits),
G = (A + A^H)/2 with A iid complex N(0,1) (numpy PCG64, seed 1014), resident in
HBM before timing.  One step = one full decomposition into all 4^14
coefficients (complex64 out) with a split matrix-core path, by default the
fixed-point int8 path (--algo split_fp16: the two-plane fp16 split,
--algo split_bf16: the three-plane bf16 split): the pack (scale reduction,
XOR gather, quantisation or split, operand layout) then the contraction
kernel (+-1 contraction, exact or binary64 recombination, phase, 2^-N,
store).

Printed: one JSON line with coefficients/s over the whole step, the roofline
of the contraction kernel (the method's own 4 * 8^N operations per launch /
its mean launch time from HIP events on its stream, against the dense
matrix-core peak of the path's data type: 5.0 POP/s int8, 2.5 PFLOP/s
fp16/bf16; the executed matrix-core operations of the split in separate
fields), the binary64 Gray-code GPU kernel on the same input for the speed
ratio and the error (max |c - c_fp64| / max |c_fp64|), another split path
timed on the same input (split_fp16 beside split_i8), and the CPU oracle
timed on a bounded sample of the same coefficients on the host's cores
(which also checks those coefficients).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "Pauli coeffs/sec + % MFMA peak at N=14, split-BF16 vs FP64 at err≤1e-6"
METRIC_HERM = ("Pauli coeffs/sec at N=14, Hermitian-aware decomposition (not the paper's general method), "
               "err<=1e-6")
PEAK_BF16_TFLOPS = 2500.0
PEAK_I8_TOPS = 5000.0   # dense int8 matrix-core peak
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2401_16378_amd/csrc/mfma_tile.hpp", "paper_2401_16378_amd/csrc/mfma.hip",
                  "paper_2401_16378_amd/csrc/common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_split_bf16_n14.json")
TRAFFIC_FILES = {"split_bf16": TRAFFIC_FILE,
                 "split_fp16": os.path.join(ROOT, "profiles", "traffic_split_fp16_n14.json"),
                 "split_i8": os.path.join(ROOT, "profiles", "traffic_split_i8_n14.json")}
I8_SOURCES = ["paper_2401_16378_amd/csrc/mfma_i8.hip", "paper_2401_16378_amd/csrc/mfma_tile.hpp",
              "paper_2401_16378_amd/csrc/common.hpp"]
TRAFFIC_SOURCES = {"split_i8": I8_SOURCES}
PLANES = {"split_bf16": 3, "split_fp16": 2, "fp32": 1, "split_i8": 3}
DTYPE = {"split_bf16": "bf16", "split_fp16": "fp16", "fp32": "f32", "split_i8": "i8"}
SPLITS = ("split_bf16", "split_fp16", "split_i8")
OTHER_SPLIT = {"split_fp16": "split_bf16", "split_bf16": "split_fp16", "split_i8": "split_fp16"}


def peak_of(algo):
    """(dense matrix-core peak, unit) of the algorithm's MFMA data type."""
    if algo == "split_i8":
        return PEAK_I8_TOPS, "TOP/s"
    return (157.3 if algo == "fp32" else PEAK_BF16_TFLOPS), "TFLOP/s"   # bf16 and fp16 share the dense peak
STRINGS_SOURCES = ["paper_2401_16378_amd/csrc/strings.hip", "paper_2401_16378_amd/csrc/common.hpp"]
STRINGS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_strings_n14.json")
FWHT_SOURCES = ["paper_2401_16378_amd/csrc/fwht.hip", "paper_2401_16378_amd/csrc/common.hpp"]
FWHT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fwht_n14.json")
FWHT_F32_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fwht_f32_n14.json")
HERM_TRAFFIC_FILES = {"split_bf16": os.path.join(ROOT, "profiles", "traffic_hermitian_n14.json"),
                      "split_fp16": os.path.join(ROOT, "profiles", "traffic_hermitian_fp16_n14.json"),
                      "split_i8": os.path.join(ROOT, "profiles", "traffic_hermitian_i8_n14.json")}


def source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the kernel as it stands now."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash(sources):
        return None
    return t.get("bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(G64: np.ndarray, c_gpu: np.ndarray, sample: int):
    import oracle
    cores = len(os.sched_getaffinity(0))
    N = G64.shape[0].bit_length() - 1
    import workloads
    ns = workloads.sample_indices(4 ** N, sample, seed=workloads.SEED_SAMPLE)
    t0 = time.perf_counter()
    ref = oracle.coeffs_at(G64, ns, threads=cores)
    dt = time.perf_counter() - t0
    got = c_gpu[ns.astype(np.int64)]
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    return {"value": sample / dt, "unit": "coeffs/s", "cores": cores, "kind": "oracle",
            "sample": "%d of the 4^%d coefficients (uniform without replacement, seed %d) of the same "
                      "matrix, binary64 Gray-code oracle, %d threads over disjoint ranges, %.1f s"
                      % (sample, N, workloads.SEED_SAMPLE, cores, dt)}, err


def timed(fn, steps, warmup, stream):
    """Mean ms per call of fn() over `steps` calls, after `warmup` calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record(stream)
    for _ in range(steps):
        fn()
    e.record(stream)
    torch.cuda.synchronize()
    return b.elapsed_time(e) / steps


def bench_batch(a):
    """512 complex64 matrices, N uniform on 3..9 (102 Hermitian): one graph
    replay (batched pack + persistent contraction) per step, against one
    decomposition launch per matrix on the same buffers."""
    import torch
    import paper_2401_16378_amd as pauli
    import workloads
    dev = torch.device("cuda:0")
    Ns, mats, herm = workloads.batch_spec()
    G = [torch.from_numpy(m).to(dev) for m in mats]
    outs = [torch.empty(1 << (2 * n), dtype=torch.complex64, device=dev) for n in Ns]
    stream = torch.cuda.current_stream(dev)
    algo = a.algo
    tile = pauli.autotune_batched(G, algo=algo, outs=outs)
    plan = pauli.BatchPlan(G, algo=algo, outs=outs)   # arguments marshalled once, as a serving loop would
    ms = timed(plan.run, a.steps, a.warmup, stream)
    ws = pauli.workspace(algo, 9, 1, dev)

    def per_matrix():
        for g, o in zip(G, outs):
            n = g.shape[-1].bit_length() - 1
            oo = pauli._opts(algo, 0, 0, 0, ctypes.c_void_p(stream.cuda_stream), ws)
            st = pauli.load_library().pauli_decompose(g.data_ptr(), n, 1, o.data_ptr(), ctypes.byref(oo))
            if st:
                raise RuntimeError(pauli.last_error())
    ms_each = timed(per_matrix, max(2, a.steps // 4), 1, stream)
    coeffs = float(sum(4 ** n for n in Ns))
    flops = float(sum(4 * PLANES[algo] * 8 ** n for n in Ns))
    line = {"metric": "Pauli coeffs/sec, uneven batch", "value": coeffs / (ms / 1e3), "unit": "coeffs/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[algo], "data": "synthetic",
            "config": {"workload": "512 complex64 matrices, N uniform on 3..9 (seed %d), 20%% Hermitian, "
                                   "%s, one HIP graph replay per step" % (workloads.SEED_BATCH, algo),
                       "batch": len(Ns), "tile": tile, "algo": algo},
            "executed_tflops": flops / (ms / 1e3) / 1e12,
            "useful_tflops": float(sum(4 * 8 ** n for n in Ns)) / (ms / 1e3) / 1e12,
            "per_matrix_launch_ms": ms_each, "speedup_vs_per_matrix": ms_each / ms}
    print(json.dumps(line), flush=True)


def bench_backward(a):
    """8 complex64 matrices at N=11: forward decomposition, loss
    sum w |c - t|^2 and the adjoint backward, through torch.autograd."""
    import torch
    import paper_2401_16378_amd as pauli
    import workloads
    dev = torch.device("cuda:0")
    G, G2, w = workloads.backward_problem(11, 8)
    Gd = torch.from_numpy(G).to(dev)
    # the loss runs in complex64 / binary32 (it only drives the gradient here;
    # the gradient tests use binary64 losses)
    t = pauli.decompose(torch.from_numpy(G2).to(dev))
    wd = torch.from_numpy(w).to(dev).to(torch.float32)
    stream = torch.cuda.current_stream(dev)

    algo = a.algo

    def step():
        g = Gd.detach().requires_grad_(True)
        c = pauli.PauliDecompose.apply(g, algo)
        # |c - t|^2 as re^2 + im^2 of a real view: no abs/sgn kernels in its gradient
        d = torch.view_as_real(c - t)
        loss = (wd * (d * d).sum(-1)).sum()
        loss.backward()
        return g.grad

    ms = timed(step, a.steps, a.warmup, stream)
    ms_fwd = timed(lambda: pauli.decompose(Gd, algo=algo), a.steps, a.warmup, stream)
    g = Gd.detach()
    gc = torch.randn(8, 4 ** 11, dtype=torch.complex64, device=dev)
    ms_bwd = timed(lambda: pauli.decompose_backward(gc, algo=algo), a.steps, a.warmup, stream)
    flops = 2 * 8 * 4 * PLANES[algo] * float(8 ** 11)
    line = {"metric": "forward+backward steps/sec, 8 x N=11", "value": 1e3 / ms, "unit": "steps/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[algo], "data": "synthetic",
            "config": {"workload": "8 complex64 2048x2048 matrices, L = sum w|c-t|^2 (complex64 / binary32), %s forward "
                                   "and adjoint backward through torch.autograd" % algo, "batch": 8, "N": 11,
                       "algo": algo},
            "forward_ms": ms_fwd, "backward_kernel_ms": ms_bwd,
            ("executed_tops_fwd_bwd_kernels" if algo == "split_i8" else "executed_tflops_fwd_bwd_kernels"):
                flops / ((ms_fwd + ms_bwd) / 1e3) / 1e12}
    print(json.dumps(line), flush=True)


def bench_strings(a):
    """Coefficients of a list of 65,536 Pauli strings (seeded uniform sample
    without replacement) of the N=14 complex64 Hermitian matrix: one
    pauli_coeffs_at call per step, binary64 sums."""
    import torch
    import paper_2401_16378_amd as pauli
    import workloads
    dev = torch.device("cuda:0")
    N, L = a.N, a.strings
    log("[bench] generating N=%d Hermitian complex64 input (seed %d)" % (N, workloads.SEED_N14))
    G = workloads.hermitian(N, workloads.SEED_N14)
    Gd = torch.from_numpy(G).to(dev)
    ns = workloads.sample_indices(4 ** N, L, seed=workloads.SEED_SAMPLE).astype(np.uint32)
    lib = pauli.load_library()
    ws = torch.empty(lib.pauli_coeffs_at_workspace_bytes(N, L), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    ms = timed(lambda: pauli.coeffs_at(Gd, ns, workspace_tensor=ws), a.steps, a.warmup, stream)
    got = pauli.coeffs_at(Gd, ns, out_dtype=torch.complex128, workspace_tensor=ws).cpu().numpy()
    # HBM bytes the method must move: the 16 XOR diagonals (16 x 2^N elements)
    # of every line group the list touches, read once, plus the coefficients.
    flips = np.bitwise_xor(ns & 0x55555555, (ns >> 1) & 0x55555555)
    x = np.zeros_like(ns)
    for t in range(N):
        x |= ((flips >> (2 * t)) & 1) << t
    groups = len(np.unique(x >> 4)) if N >= 4 else 1
    width = 16 if N >= 4 else 1 << N
    alg_bytes = groups * width * (1 << N) * 8 + L * 8
    achieved = alg_bytes / (ms / 1e3) / 1e9
    line = {"metric": "Pauli string coefficients/sec, list of %d strings at N=%d" % (L, N),
            "value": L / (ms / 1e3), "unit": "strings/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "coefficients of %d Pauli strings (uniform sample without replacement, "
                                   "seed %d) of one %dx%d complex64 Hermitian matrix (seed %d), binary64 sums, "
                                   "host list, one pauli_coeffs_at call per step"
                                   % (L, workloads.SEED_SAMPLE, 1 << N, 1 << N, workloads.SEED_N14),
                       "N": N, "strings": L, "line_groups": groups},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic(STRINGS_TRAFFIC_FILE, STRINGS_SOURCES)
                         if (N, L) == (14, 65536) else None,
                         "note": "whole call (plan copy, strings_kernel, strings_finish) on the stream, "
                                 "so a lower bound on the kernel's own rate"}}
    if not a.no_cpu:
        import oracle
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=cores)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": L / dt, "unit": "strings/s", "cores": cores, "kind": "oracle",
                                "sample": "the same %d strings, binary64 Gray-code oracle, %d threads over "
                                          "disjoint ranges, %.1f s" % (L, cores, dt)}
        line["max_err_vs_oracle"] = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(json.dumps(line), flush=True)


def bench_fwht(a):
    """All 4^N coefficients of the N=14 matrix by the fast Walsh-Hadamard
    algorithm (not the paper's O(8^N) evaluation): `--algo fwht` (binary64
    intermediate, the default here) or `--algo fwht_f32` (binary32
    intermediate)."""
    import torch
    import paper_2401_16378_amd as pauli
    import workloads
    dev = torch.device("cuda:0")
    N = a.N
    log("[bench] generating N=%d Hermitian complex64 input (seed %d)" % (N, workloads.SEED_N14))
    G = workloads.hermitian(N, workloads.SEED_N14)
    Gd = torch.from_numpy(G).to(dev)
    out = torch.empty(1 << (2 * N), dtype=torch.complex64, device=dev)
    lib = pauli.load_library()
    stream = torch.cuda.current_stream(dev)
    algo = a.algo if a.algo in ("fwht", "fwht_f32") else "fwht"
    narrow = algo == "fwht_f32"
    ws = pauli.workspace(algo, N, 1, dev)
    o = pauli._opts(algo, 0, 0, 0, ctypes.c_void_p(stream.cuda_stream), ws)

    def step():
        if lib.pauli_decompose(Gd.data_ptr(), N, 1, out.data_ptr(), ctypes.byref(o)) != 0:
            raise RuntimeError(pauli.last_error())
    ms = timed(step, a.steps, a.warmup, stream)
    c128 = pauli.decompose(Gd, algo=algo, out_dtype=torch.complex128)
    ref = pauli.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128)
    err = ((c128 - ref).abs().max() / ref.abs().max()).item()
    err64 = ((out.to(torch.complex128) - ref).abs().max() / ref.abs().max()).item()
    # the method's own minimum: read G once, write the coefficients once
    alg_bytes = float(4 ** N) * (8 + 8)
    achieved = alg_bytes / (ms / 1e3) / 1e9
    ub = 8 if narrow else 16
    line = {"metric": "Pauli coeffs/sec at N=%d, %s fast Walsh-Hadamard (not the paper's O(8^N) method)"
                      % (N, "binary32-intermediate" if narrow else "binary64"),
            "value": 4 ** N / (ms / 1e3), "unit": "coeffs/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "dense Pauli decomposition, N=%d (%dx%d complex64 Hermitian, seed %d), all 4^%d "
                                   "coefficients, algo %s (two passes through a %d B/element %s intermediate)"
                                   % (N, 1 << N, 1 << N, workloads.SEED_N14, N, algo, ub,
                                      "binary32" if narrow else "binary64"), "N": N, "algo": algo},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic(FWHT_F32_TRAFFIC_FILE if narrow else FWHT_TRAFFIC_FILE,
                                                     FWHT_SOURCES) if N == 14 else None,
                         "note": "achieved counts 16 B per element (G read once, coefficients written once); the "
                                 "two-pass design also writes and reads a %d B/element intermediate, and traffic "
                                 "is the measured HBM bytes of both passes of one decomposition" % ub},
            "max_err_vs_fp64_gray": err, "max_err_complex64_out": err64}
    if not a.no_cpu:
        line["cpu_baseline"], line["max_err_vs_oracle_sample"] = cpu_baseline(
            G.astype(np.complex128), c128.cpu().numpy(), min(a.cpu_sample, 65536))
    print(json.dumps(line), flush=True)


def bench_table(a):
    """Every single-matrix config of the workload list, every path: median
    time of `steps` calls (HIP events around each call, input in HBM),
    coefficients/s, the method's flops (4 * 8^N) and the executed flops as
    fractions of the matrix-core peak of the path's data type (int8 ops for
    split_i8), algorithmic HBM bytes (input read +
    coefficients written) per second, and the error against the binary64
    Gray kernel (which the tests hold bit-identical to the oracle).  One JSON
    line per (config, path) on stdout."""
    import torch
    import paper_2401_16378_amd as pauli
    import workloads
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    configs = [("N=6 complex128 iid", 6, workloads.iid_complex(6, workloads.SEED_N6)),
               ("N=10 complex128 iid", 10, workloads.iid_complex(10, workloads.SEED_N10)),
               ("N=12 complex64 Hermitian", 12, workloads.hermitian(12, workloads.SEED_N12)),
               ("N=14 complex64 Hermitian", 14, workloads.hermitian(14, workloads.SEED_N14))]
    peak = {algo: peak_of(algo)[0] for algo in ("split_i8", "split_fp16", "split_bf16", "fp32")}
    for name, N, G in configs:
        Gd = torch.from_numpy(G).to(dev)
        esz = 16 if Gd.dtype == torch.complex128 else 8
        ref = pauli.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128)
        mref = ref.abs().max().item()
        for algo in ("split_i8", "split_fp16", "split_bf16", "fp32", "fwht", "fwht_f32", "fp64_gray"):
            steps = a.steps if not (algo in ("fp64_gray", "fp32") and N == 14) else 3
            out = pauli.decompose(Gd, algo=algo)
            err = ((out.to(torch.complex128) - ref).abs().max().item()) / mref
            ts = []
            for _ in range(steps):
                b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                b.record(stream)
                pauli.decompose(Gd, algo=algo)
                e.record(stream)
                torch.cuda.synchronize()
                ts.append(b.elapsed_time(e))
            ms = float(np.median(ts))
            row = {"config": name, "algo": algo, "ms_median": ms, "steps": steps,
                   "coeffs_per_s": float(4 ** N) / (ms / 1e3),
                   "hbm_gbs_algorithmic": 2.0 * esz * float(4 ** N) / (ms / 1e3) / 1e9,
                   "max_err_vs_fp64_gray": err}
            if algo in peak:
                useful = 4.0 * float(8 ** N) / (ms / 1e3) / 1e12
                row.update({"useful_frac": useful / peak[algo],
                            "executed_frac": useful * PLANES[algo] / peak[algo], "peak": peak[algo],
                            "peak_unit": peak_of(algo)[1]})
            print(json.dumps(row), flush=True)
            del out
        del Gd, ref
        pauli.release_workspace()
        torch.cuda.empty_cache()


def bench_oracle(a):
    """The CPU oracle's own timings on this host (no GPU work): full
    decompositions single-threaded at N=6 and N=10 and on all cores at N=10
    and N=12, and at N=14 the 65,536-coefficient sample on one core and on
    all cores, extrapolated to all 4^14 coefficients."""
    import oracle
    import workloads
    cores = len(os.sched_getaffinity(0))
    rows = []

    def run(label, N, threads, fn):
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        rows.append({"case": label, "N": N, "threads": threads, "seconds": dt})
        log("[oracle] %s: %.3f s" % (label, dt))
        return dt

    G6 = workloads.iid_complex(6, workloads.SEED_N6)
    run("N=6 full, 1 thread", 6, 1, lambda: oracle.decompose(G6))
    G10 = workloads.iid_complex(10, workloads.SEED_N10)
    run("N=10 full, 1 thread", 10, 1, lambda: oracle.decompose(G10))
    run("N=10 full, all threads", 10, cores, lambda: oracle.decompose(G10, threads=cores))
    G12 = workloads.hermitian(12, workloads.SEED_N12).astype(np.complex128)
    run("N=12 full, all threads", 12, cores, lambda: oracle.decompose(G12, threads=cores))
    del G12
    G14 = workloads.hermitian(14, workloads.SEED_N14).astype(np.complex128)
    ns = workloads.sample_indices(4 ** 14, 65536, seed=workloads.SEED_SAMPLE)
    s1 = run("N=14 65,536-coefficient sample, 1 thread", 14, 1, lambda: oracle.coeffs_at(G14, ns))
    sa = run("N=14 65,536-coefficient sample, all threads", 14, cores,
             lambda: oracle.coeffs_at(G14, ns, threads=cores))
    line = {"oracle_timing": rows, "cores": cores,
            "n14_full_extrapolated_seconds": {"1 thread": s1 * 4096, "all threads": sa * 4096,
                                              "note": "extrapolated: the sample's time x 4096 (4^14 / 65,536)"}}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["n14", "hermitian", "batch", "backward", "strings", "fwht", "oracle",
                                           "table"],
                    default="n14")
    ap.add_argument("--strings", type=int, default=65536, help="list length of the strings workload")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=14)
    ap.add_argument("--algo", default=None,
                    help="path to time (default: split_i8 for n14, hermitian and backward, split_fp16 for "
                         "batch, fwht for fwht)")
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other split path")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=131072)
    ap.add_argument("--fp64-reps", type=int, default=3)
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a device copy of this many GiB (counter calibration)")
    a = ap.parse_args()
    if a.algo is None:
        a.algo = {"n14": "split_i8", "hermitian": "split_i8", "backward": "split_i8", "fwht": "fwht"}.get(
            a.workload, "split_fp16")
    if a.workload == "batch" and a.algo not in ("split_bf16", "split_fp16", "fp32"):
        raise SystemExit("bench.py: the batch workload runs split_bf16, split_fp16 or fp32, not %s" % a.algo)
    if a.workload == "backward" and a.algo not in ("split_bf16", "split_fp16", "fp32", "split_i8"):
        raise SystemExit("bench.py: the backward workload runs a matrix-core path, not %s" % a.algo)
    if a.gpus != 1:
        print("bench.py: the decomposition runs on one GPU (it is not sharded across devices); --gpus %d is not supported" % a.gpus,
              file=sys.stderr)
        sys.exit(2)

    if a.workload == "oracle":
        return bench_oracle(a)

    import torch
    import paper_2401_16378_amd as pauli
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_probe_gib > 0:
        # a device copy of known size, the calibration for HBM byte counters
        nb = int(a.copy_probe_gib * (1 << 30))
        src = torch.empty(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "batch":
        return bench_batch(a)
    if a.workload == "backward":
        return bench_backward(a)
    if a.workload == "strings":
        return bench_strings(a)
    if a.workload == "fwht":
        return bench_fwht(a)
    if a.workload == "table":
        return bench_table(a)
    N = a.N
    log("[bench] generating N=%d Hermitian complex64 input (seed %d)" % (N, workloads.SEED_N14))
    t0 = time.perf_counter()
    G = workloads.hermitian(N, workloads.SEED_N14)
    log("[bench] generated in %.1f s" % (time.perf_counter() - t0))
    Gd = torch.from_numpy(G).to(dev)
    out = torch.empty(1 << (2 * N), dtype=torch.complex64, device=dev)
    lib = pauli.load_library()
    import ctypes
    stream = torch.cuda.current_stream(dev)
    ws = pauli.workspace(a.algo, N, 1, dev)
    o = pauli._opts(a.algo, 0, 0, a.tile, ctypes.c_void_p(stream.cuda_stream), ws)
    herm = a.workload == "hermitian"
    if a.algo not in PLANES:
        raise SystemExit("bench.py: the n14 and hermitian workloads time a matrix-core algorithm (%s)"
                         % ", ".join(PLANES))
    mode = 3 if herm else 0   # 3: pauli_decompose_hermitian split at the kernel boundary

    def step(mid=None):
        # pauli_pack + pauli_contract is pauli_decompose split at the kernel
        # boundary, so the contraction kernel can be timed on its own.
        st = lib.pauli_pack(Gd.data_ptr(), N, 1, mode, ctypes.byref(o))
        if mid is not None:
            mid.record(stream)
        st = st or lib.pauli_contract(N, 1, mode, out.data_ptr(), ctypes.byref(o))
        if st != 0:
            raise RuntimeError(pauli.last_error())

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    log("[bench] warm-up done; timing %d steps" % a.steps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        evs[s][0].record(stream)
        step(evs[s][1])
        evs[s][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [m.elapsed_time(e) for b, m, e in evs]      # contraction kernel
    pack_ms = float(np.mean([b.elapsed_time(m) for b, m, e in evs]))
    step_ms = [b.elapsed_time(e) for b, m, e in evs]        # whole step, per step
    ms_step = wall * 1000.0 / a.steps
    mean_launch = float(np.mean(launch_ms))
    coeffs = float(4 ** N)
    value = coeffs / (ms_step / 1000.0)
    planes = PLANES[a.algo]
    flops_exec = 2.0 * 2.0 * planes * float(8 ** N)   # 2 (re,im) x 2 op/MAC x planes x D^3
    flops_useful = 4.0 * float(8 ** N)                 # the method's own work (section 3)
    if herm:
        # the Hermitian variant's algorithmic work: half of K and half of the
        # rows z for every flip mask (the first few flip-mask tiles walk more,
        # so this undercounts what they execute)
        flops_exec /= 4.0
        flops_useful /= 4.0
    achieved = flops_useful / (mean_launch / 1000.0) / 1e12
    executed = flops_exec / (mean_launch / 1000.0) / 1e12
    peak, peak_unit = peak_of(a.algo)
    log("[bench] %.3f ms/step (median %.3f), pack %.3f ms, contraction %.3f ms (median %.3f), "
        "%.1f TFLOP/s useful, %.1f executed"
        % (ms_step, float(np.median(step_ms)), pack_ms, mean_launch, float(np.median(launch_ms)), achieved,
           executed))

    c_bf16 = out.cpu().numpy()
    res = {}
    if not a.no_fp64:
        out64 = torch.empty(1 << (2 * N), dtype=torch.complex128, device=dev)
        o64 = pauli._opts("fp64_gray", 0, 1, 0, ctypes.c_void_p(stream.cuda_stream))
        st = lib.pauli_decompose(Gd.data_ptr(), N, 1, out64.data_ptr(), ctypes.byref(o64))
        if st != 0:
            raise RuntimeError(pauli.last_error())
        torch.cuda.synchronize()
        b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.record(stream)
        for _ in range(a.fp64_reps):
            lib.pauli_decompose(Gd.data_ptr(), N, 1, out64.data_ptr(), ctypes.byref(o64))
        e.record(stream)
        torch.cuda.synchronize()
        fp64_ms = b.elapsed_time(e) / a.fp64_reps
        c64 = out64.cpu().numpy()
        err = float(np.abs(c_bf16 - c64).max() / np.abs(c64).max())
        im_ratio = float(np.abs(c64.imag).max() / np.abs(c64).max())
        res.update({"fp64_gray_ms": round(fp64_ms, 3), "speedup_vs_fp64_gray": round(fp64_ms / ms_step, 2),
                    "max_err_vs_fp64": err, "fp64_imag_ratio": im_ratio})
        log("[bench] fp64 gray %.1f ms, ratio %.2f, err %.3g" % (fp64_ms, fp64_ms / ms_step, err))
        del out64

    if a.algo in SPLITS and not a.no_compare:
        # another split path on the same input: its time per step and error
        other = OTHER_SPLIT[a.algo]
        ws2 = pauli.workspace(other, N, 1, dev)
        o2 = pauli._opts(other, 0, 0, 0, ctypes.c_void_p(stream.cuda_stream), ws2)
        out2 = torch.empty_like(out)
        dec = lib.pauli_decompose_hermitian if herm else lib.pauli_decompose

        def step2():
            if dec(Gd.data_ptr(), N, 1, out2.data_ptr(), ctypes.byref(o2)) != 0:
                raise RuntimeError(pauli.last_error())
        ms2 = timed(step2, max(3, a.steps // 2), 1, stream)
        cmp = {"algo": other, "ms_per_step": ms2, "value": float(4 ** N) / (ms2 / 1000.0)}
        if not a.no_fp64:
            c2 = out2.cpu().numpy()
            cmp["max_err_vs_fp64"] = float(np.abs(c2 - c64).max() / np.abs(c64).max())
        res["other_split"] = cmp
        log("[bench] %s: %.3f ms/step" % (other, ms2))
        del out2, ws2
        pauli.release_workspace()

    cpu = None
    if not a.no_cpu:
        log("[bench] timing the CPU oracle on a %d-coefficient sample" % a.cpu_sample)
        cpu, err_cpu = cpu_baseline(G.astype(np.complex128), c_bf16.astype(np.complex128), a.cpu_sample)
        res["max_err_vs_oracle_sample"] = err_cpu
        log("[bench] oracle %.0f coeffs/s on %d cores, sample err %.3g" % (cpu["value"], cpu["cores"], err_cpu))

    # committed counter summaries cover the split kernels at N=14 only
    tile_used = a.tile if a.tile else (pauli.tile_selected_hermitian(N, a.algo) if herm
                                       else pauli.tile_selected(N, a.algo))
    if a.algo == "split_i8":
        tile_used = 1   # its one tile shape
    traffic = None
    if N == 14 and herm and a.algo in HERM_TRAFFIC_FILES:
        traffic = measured_traffic(HERM_TRAFFIC_FILES[a.algo], TRAFFIC_SOURCES.get(a.algo, KERNEL_SOURCES))
    elif N == 14 and not herm and a.algo in TRAFFIC_FILES:
        traffic = measured_traffic(TRAFFIC_FILES[a.algo], TRAFFIC_SOURCES.get(a.algo, KERNEL_SOURCES))
    if herm:
        res["imag_exactly_zero"] = bool(np.all(c_bf16.imag == 0))
    line = {
        "metric": METRIC_HERM if herm else (METRIC if a.algo in SPLITS else
                                            "Pauli coeffs/sec + %% MFMA peak at N=%d, %s matrix-core path"
                                            % (N, a.algo)), "value": value, "unit": "coeffs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "ms_per_step_median": float(np.median(step_ms)),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[a.algo], "data": "synthetic",
        "config": {"workload": "dense Pauli decomposition, N=%d (%dx%d complex64 Hermitian, "
                               "G=(A+A^H)/2, A iid N(0,1)), all 4^%d coefficients, %s%s"
                               % (N, 1 << N, 1 << N, N, a.algo,
                                  ", Hermitian variant (half of K and of the rows per flip mask, "
                                  "pauli_decompose_hermitian)"
                                  if herm else ""), "N": N, "batch": 1,
                   "algo": a.algo, "tile": tile_used},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": peak_unit,
                     "frac": achieved / peak, "traffic": traffic,
                     "counts": "the method's own flops, 4*8^N (re, im x 2 flop per term)%s; executed "
                               "matrix-core %s (%d %s planes) in executed_*"
                               % (", quartered" if herm else "", "int8 ops" if a.algo == "split_i8" else "flops",
                                  planes, "int8 digit" if a.algo == "split_i8" else DTYPE[a.algo]),
                     "flops_per_launch": flops_useful,
                     "executed_tflops": executed, "executed_frac": executed / peak,
                     "executed_flops_per_launch": flops_exec,
                     "launch_ms": mean_launch, "launch_ms_median": float(np.median(launch_ms)),
                     "kernel": ("i8_contract_kernel%s (split_i8, two walks over K)" % ("<16, HERM=true>" if herm else "<16>")
                                if a.algo == "split_i8" else
                                "%s%s (%s, tile %d)" % ("contract_lds_kernel" if tile_used >= 13 else "contract_kernel",
                                                        " <..., HERM=true>" if herm else "", a.algo, tile_used)),
                     "pack_ms": pack_ms},
        "cpu_baseline": cpu,
    }
    line.update(res)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
