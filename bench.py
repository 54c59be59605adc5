"""Benchmark: compressed state-vector passes on one MI355X.

One step is one pass of Algorithm 1 (Section II of the paper) over the whole
state: every slice is decompressed, normalised, updated by one gate and
recompressed.  The default workload is the largest configuration that fits one
GPU: 34-qubit Grover search (marked index from seed 0), 1024 slices of 2^24
amplitudes (an uncompressed FP64 state of 256 GiB, held only compressed),
absolute error bound 1e-8, FP64.  Inputs are synthetic (the paper's circuits
are not available).  The initial H layer runs untimed; the timed passes start
at the first Grover iteration's oracle and run into its diffusion layer, where
every slice holds nonzero amplitudes.  The same window is then run in FP32
mode, and both read-outs are compared on sampled amplitudes (with the exact
state beside them), and once more with zero-chunk, constant-chunk and
chunk-run records (the same amplitudes, smaller records).

Prints one JSON line: throughput in state amplitudes per second (amplitude-
passes: 2^34 per step), the compression ratio, per-pass latency percentiles,
the roofline position of the dominant kernel (device times from HIP events on
the library's stream), and the CPU oracle timed on sampled slices.

`--workload grover24 | qft30 | qft12 | serve` runs the other configurations;
`--copy-probe` times a plain device copy of known size, whose HBM counter
readings calibrate the per-kernel traffic figures below.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6
METRIC = "state amps/s via decompress+gate+compress at error bound; ratio; p99 latency"
KERNEL_SRC = os.path.join(ROOT, "paper_1811_05630_amd", "csrc", "kernels.hip")

# HBM bytes per launch of a kernel class, per workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script, each scaled by the
# reading of the same counter for the copy probe.  Valid only for the kernel
# source they were taken on (sha256 of kernels.hip).
MEASURED_TRAFFIC = {
    "grover34": {
        "decode": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 9196552035},
        "gate_quant": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 13767265397},
        "codebook": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 5864041},
        "encode": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 5773226182},
        "finish": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 1075019555},
    },
    "grover24": {
        "decode": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 149670621},
        "gate_quant": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 220343282},
        "codebook": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 5870640},
        "encode": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 78993272},
        "finish": {"kernels_sha256": "19bc40c8b65ed4589a884b0d0d9c1317bc7ee10729a95950a57a7f394cc5bf2a",
                 "bytes_per_launch": 16579607},
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed passes (default: 20; grover24: 1000)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed passes before them (default: 5; grover24: 100)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--chunk-log2", type=int, default=8)
    ap.add_argument("--latency-passes", type=int, default=None, help="single-pass calls timed for the "
                    "latency percentiles (default: 20; grover24: 200)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fp32", action="store_true",
                    help="grover24: FP32 mode (FP32 working values and gate arithmetic); grover34 runs both "
                         "precisions")
    ap.add_argument("--no-fp32", action="store_true", help="grover34: skip the FP32 leg")
    ap.add_argument("--no-codec-leg", action="store_true",
                    help="grover34: skip the leg with zero-chunk, constant-chunk and chunk-run records")
    ap.add_argument("--tune", action="store_true",
                    help="grover24: also report the chunk-length autotuner's table (sim_tune_chunk) on the circuit")
    ap.add_argument("--zero-chunks", action="store_true",
                    help="grover24, grover34: zero-chunk records (all-zero chunks stored with no words)")
    ap.add_argument("--const-chunks", action="store_true",
                    help="grover24, grover34: constant-chunk records (a chunk of equal values keeps its first only)")
    ap.add_argument("--opt", action="store_true",
                    help="grover24, grover34: optimised passes (SIM_OPT: groups where a gate's slice-index controls "
                         "fail are carried over unchanged)")
    ap.add_argument("--chunk-runs", action="store_true",
                    help="grover24, grover34: chunk-run records (runs of chunks with identical streams stored once)")
    ap.add_argument("--workload", choices=("grover34", "grover24", "qft30", "qft12", "serve"), default="grover34",
                    help="grover34 (default, the headline line: 34-qubit Grover search, FP64 and FP32); "
                         "grover24: 24-qubit Grover search; qft30: 30-qubit QFT of a product state in fused "
                         "mode; qft12: 12-qubit QFT as a captured graph; serve: the job server")
    ap.add_argument("--jobs", type=int, default=200, help="serve: jobs in the timed stream")
    ap.add_argument("--arrival-ms", type=float, default=60.0, help="serve: mean gap between arrivals")
    ap.add_argument("--max-active", type=int, default=4, help="serve: jobs running at once, at most")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="serve: device-memory budget")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 256 MiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    big = args.workload == "grover24"
    if args.steps is None:
        args.steps = 1000 if big else 20
    if args.warmup is None:
        args.warmup = 100 if big else 5
    if args.latency_passes is None:
        args.latency_passes = 200 if big else 20
    return args


def kernel_bytes(name, n_amps, c_in, c_out, n_slices, escapes, plane_bytes=16):
    """Algorithmic HBM bytes of one launch of each kernel class over the whole
    state (2^n amplitudes in two planes of plane_bytes / 2 bytes per value:
    16 for FP64 values, 8 for the compact int32 codes; one u16 symbol per
    value; 8 bytes per escaped difference; c_in / c_out compressed bytes read /
    written)."""
    planes = plane_bytes * n_amps
    syms = 4 * n_amps
    return {
        "decode": c_in + planes,                   # records in, FP64 planes out
        "gate_quant": planes + syms + 8 * escapes,  # planes in, symbols (+ escapes) out
        "codebook": n_slices * (4096 + 4096 + 2048 + 8192),  # histogram in; codes, table, decoder table out
        "encode": syms + 8 * escapes + c_out,      # symbols in, chunk streams out
        "header": n_slices * 8 * 1024,             # chunk sizes in, headers and offsets out (order of)
        "compact": 2 * c_out,                      # chunk streams moved into the records
    }.get(name)


def source_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def traffic_for(workload, kernel):
    rec = MEASURED_TRAFFIC.get(workload, {}).get(kernel)
    if not rec or rec["kernels_sha256"] != source_sha():
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(w, seconds, chunk_log2, fp32=False):
    import oracle
    threads = oracle.num_threads()
    sim = oracle.OracleSim(w.n_qubits, w.slice_log2, chunk_log2, w.error_bound, oracle.FP32 if fp32 else oracle.ABS)
    n0 = w.n_qubits  # bring the oracle to the timed region's starting point
    sim.apply(w.gates[:n0])
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < len(w.gates) - n0:
        sim.apply(w.gates[n0 + done:n0 + done + 1])
        done += 1
    dt = time.perf_counter() - t0
    # the same oracle on one thread, over the following passes, for a third of the time
    oracle.set_threads(1)
    n1 = n0 + done
    one = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < seconds / 3 and n1 + one < len(w.gates):
        sim.apply(w.gates[n1 + one:n1 + one + 1])
        one += 1
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    return {"value": done * (1 << w.n_qubits) / dt, "unit": "amps/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} passes of the 24-qubit Grover circuit after its H layer "
                      f"(gates {n0}..{n0 + done - 1}), {dt:.1f} s, OpenMP over slices",
            "one_thread": {"value": one * (1 << w.n_qubits) / max(dt1, 1e-9), "unit": "amps/s",
                           "sample": f"{one} further passes (gates {n1}..{n1 + one - 1}), {dt1:.1f} s"}}


def copy_probe():
    import torch
    n = 32 << 20  # 32 Mi doubles = 256 MiB read and 256 MiB written per launch
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    reps = 20
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)  # one elementwise kernel: reads n doubles, writes n doubles
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_probe": "torch.neg float64", "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "launches": reps, "ms_per_launch": ms, "GBps": 16 * n / ms / 1e6}), flush=True)


def compact_workspace(w, relative, chunk_log2):
    """Whether the passes of a plain-mode workload run on the compact int32
    workspace: an absolute bound whose codes fit int32 (|q| <= 1 / (2 eb) for a
    normalised state), chunks of at most 256 values and slices of at least
    1024 amplitudes (the wavefront-range gate kernels)."""
    return (not relative and chunk_log2 <= 8 and w.slice_log2 >= 10 and 1.0 / (2 * w.error_bound) < 2 ** 30)


def report(args, w, sim, value, K, Wm, dt, kt, st1, st2, lat, config, mfma_flops=None, extra=None,
           plane_bytes=16, nslices=None):
    """The JSON line shared by all workloads."""
    import numpy as np
    N = 1 << w.n_qubits
    comp = st2["compressed_bytes"]
    esc = (st2["escapes"] - st1["escapes"]) / K  # escapes coded per pass
    ms_launch = {k: v[0] / v[1] for k, v in kt.items() if v[1] > 0}
    per_pass = {k: v[1] / K for k, v in kt.items() if v[1] > 0}
    dom = max((k for k in ms_launch if k in ("decode", "gate_quant", "codebook", "encode", "header", "compact",
                                               "dense_mfma")), key=lambda k: kt[k][0])
    avg_ms = ms_launch[dom]
    if dom == "dense_mfma":
        flops = mfma_flops / kt[dom][1]  # per launch
        achieved = flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": MFMA_F64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / MFMA_F64_PEAK_TFLOPS, "traffic": None,
                "algorithmic_flops_per_launch": flops, "avg_launch_ms": avg_ms}
    else:
        algo = kernel_bytes(dom, N, comp, comp, nslices or sim.nslices, esc, plane_bytes) / per_pass[dom]
        achieved = algo / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic_for(args.workload, dom),
                "algorithmic_bytes_per_launch": algo, "avg_launch_ms": avg_ms}
    b = 8 if getattr(args, "fp32", False) else 16  # bytes per amplitude of the working form
    pipe_bytes = 2 * b * N + 2 * comp  # B_alg: planes written and read once + records in and out
    pipe_achieved = pipe_bytes * K / dt / 1e9
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "amps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if getattr(args, "fp32", False) else "f64",
        "data": "synthetic",
        "config": config,
        "ratio": st2["raw_bytes"] / comp,
        "min_ratio": st2["min_ratio"],
        "max_abs_codec_err": st2["max_abs_codec_err"],
        "kernel_ms_per_launch": ms_launch,
        "kernel_launches_per_pass": per_pass,
        "roofline": roof,
        "pipeline_roofline": {"bytes_per_pass": pipe_bytes, "achieved": pipe_achieved, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": pipe_achieved / HBM_PEAK_GBS},
    }
    if lat:
        line["latency_ms_per_pass"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}
    if mfma_flops and "dense_mfma" in kt and kt["dense_mfma"][0] > 0:
        t = mfma_flops / (kt["dense_mfma"][0] * 1e-3) / 1e12
        line["mfma"] = {"achieved": t, "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": t / MFMA_F64_PEAK_TFLOPS}
    if extra:
        line.update(extra)
    return line


def run_grover24(args):
    import torch
    import paper_1811_05630_amd as cq
    import qcircuits as qc

    w = qc.grover_workload(seed=args.seed)
    n = w.n_qubits
    N = 1 << n
    K, Wm = args.steps, args.warmup
    # record arenas sized up front for a ratio of 4 or better (the circuit
    # stays above 6), so that no reallocation falls inside a timed batch
    sim = cq.Sim(n, w.slice_log2, w.error_bound, chunk_log2=args.chunk_log2, arena_bytes=(16 << n) // 4,
                 fp32=args.fp32, zero_chunks=args.zero_chunks,
                 const_chunks=args.const_chunks, chunk_runs=args.chunk_runs, opt=args.opt)
    # initial H layer (untimed), then warm-up passes
    # the circuit is marshalled once, outside every timed region
    gates = cq.Circuit(w.gates)
    sim.apply(gates[:n])
    pos = n
    assert len(gates) >= pos + Wm + 3 * K + args.latency_passes
    sim.apply(gates[pos:pos + Wm])
    pos += Wm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.apply(gates[pos:pos + K])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pos += K
    value = K * N / dt

    # per-kernel device time over the same number of passes (HIP events
    # around every launch, on the library's stream)
    st1 = sim.stats()
    sim.kernel_times(True)
    sim.apply(gates[pos:pos + K])
    torch.cuda.synchronize()
    kt = sim.kernel_times(False)
    pos += K
    st2 = sim.stats()

    # the next K passes as one captured HIP graph (sim_graph_*), captured
    # outside the timed region: the same kernels without the gaps between
    # launches
    graph = sim.graph(gates[pos:pos + K])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert graph.launch() == K
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    graph.close()
    pos += K

    # per-pass latency: one sim_apply call per pass, host clock
    lat = []
    for i in range(args.latency_passes):
        torch.cuda.synchronize()
        a = time.perf_counter()
        sim.apply(gates[pos + i:pos + i + 1])
        lat.append((time.perf_counter() - a) * 1e3)
    config = {"workload": "grover24: 24-qubit Grover search, marked index from seed 0, 64 slices of 2^18 "
                          "amplitudes, absolute bound 1e-7, plain mode (one pass per gate)" +
                          (", FP32 mode" if args.fp32 else "") +
                          (", zero-chunk records" if args.zero_chunks else "") +
                          (", constant-chunk records" if args.const_chunks else "") +
                          (", chunk-run records" if args.chunk_runs else "") +
                          (", optimised passes" if args.opt else ""),
              "n_qubits": n, "slice_log2": w.slice_log2, "chunk_log2": args.chunk_log2,
              "error_bound": w.error_bound, "passes_timed": K, "first_timed_gate": n + Wm, "fp32": args.fp32,
              "zero_chunks": args.zero_chunks, "const_chunks": args.const_chunks, "chunk_runs": args.chunk_runs}
    line = report(args, w, sim, value, K, Wm, dt, kt, st1, st2, lat, config,
                  plane_bytes=8 if compact_workspace(w, False, args.chunk_log2) else 16)
    line["graph"] = {"value": K * N / t_graph, "unit": "amps/s", "ms_per_step": t_graph / K * 1e3,
                     "speedup_vs_launches": dt / t_graph,
                     "passes": "the %d passes after the timed window and its repeat, as one captured graph" % K}
    if args.tune:  # the H layer and 300 Grover gates on fresh handles, chunks of 2^5 .. 2^10
        best, table = cq.tune_chunk(n, w.slice_log2, w.error_bound, gates[:n + 300], lo=5, hi=10,
                                    fp32=args.fp32, zero_chunks=args.zero_chunks,
                 const_chunks=args.const_chunks)
        line["autotune"] = {"best_chunk_log2": best,
                            "ms_per_gate": {str(c): round(v[0], 4) for c, v in table.items()},
                            "record_bytes": {str(c): int(v[1]) for c, v in table.items()}}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, args.chunk_log2, args.fp32)
    return line


def run_qft12(args):
    """The 12-qubit QFT of a basis state (84 passes over 4 slices of 2^10,
    absolute bound 1e-6): a latency-bound program, applied again and again
    to the state (QFT^4 = I keeps it a QFT image of a basis state).  Timed as
    one captured graph per program (the value) and through sim_apply (the
    `eager_amps_per_s` beside it)."""
    import torch
    import paper_1811_05630_amd as cq
    import qcircuits as qc

    w = qc.qft_basis_workload(seed=args.seed)
    n, N = w.n_qubits, 1 << w.n_qubits
    R = max(1, args.steps // 10)  # programs per timed region
    # chunks of 32 values: 256 chunks decode in parallel (one lane each)
    sim = cq.Sim(n, w.slice_log2, w.error_bound, chunk_log2=5)
    sim.init_basis(w.basis)
    circ = cq.Circuit(w.gates)
    graph = sim.graph(circ)
    for _ in range(max(1, args.warmup // 10)):
        sim.apply(circ)
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(R):
        sim.apply(circ)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(R):
        graph.launch()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    K = R * len(w.gates)
    st1 = sim.stats()
    sim.kernel_times(True)
    sim.apply(circ)
    torch.cuda.synchronize()
    kt = sim.kernel_times(False)
    st2 = sim.stats()
    config = {"workload": "qft12: 12-qubit QFT of a basis state (seed 0), 4 slices of 2^10 amplitudes, absolute "
                          "bound 1e-6, chunks of 32 values, the 84-gate program captured as one HIP graph and launched %d "
                          "times" % R,
              "n_qubits": n, "slice_log2": w.slice_log2, "chunk_log2": 5, "error_bound": w.error_bound,
              "passes_timed": K}
    extra = {"eager_amps_per_s": K * N / t_eager, "graph_speedup": t_eager / t_graph,
             "ms_per_program": {"graph": t_graph / R * 1e3, "eager": t_eager / R * 1e3}}
    line = report(args, w, sim, K * N / t_graph, K, args.warmup, t_graph, kt, st1, st2, None, config, extra=extra)
    graph.close()
    return line


def run_qft30(args):
    """30-qubit QFT of a seeded product state in fused mode: 256 slices of
    2^22, relative bound 1e-4.  One step is one fused pass; the timed region
    is the whole circuit (after one untimed run of it)."""
    import torch
    import paper_1811_05630_amd as cq
    import qcircuits as qc

    w = qc.qft_product_workload(seed=args.seed)
    n, N = w.n_qubits, 1 << w.n_qubits
    plan = cq.plan(n, w.gates)
    K = len(plan)
    flops = sum(8 * (1 << len(q)) * N for (_, _, fused, q) in plan if fused and len(q) >= 3)
    sim = cq.Sim(n, w.slice_log2, w.error_bound, relative=True, chunk_log2=args.chunk_log2, fused=True,
                 workspace_bytes=64 << 30, arena_bytes=4 << 30)
    circ = cq.Circuit(w.gates)  # marshalled once, outside the timed region
    sim.init_product(w.factors)
    sim.apply(circ)  # warm-up: the whole circuit once
    sim.init_product(w.factors)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.apply(circ)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.init_product(w.factors)
    st1 = sim.stats()
    sim.kernel_times(True)
    sim.apply(circ)
    torch.cuda.synchronize()
    kt = sim.kernel_times(False)
    st2 = sim.stats()
    config = {"workload": "qft30_product: 30-qubit QFT of a product state (angles from seed 0), 256 slices of "
                          "2^22 amplitudes, relative bound 1e-4, fused mode (blocks of up to 5 qubits)",
              "n_qubits": n, "slice_log2": w.slice_log2, "chunk_log2": args.chunk_log2,
              "error_bound": w.error_bound, "gates": len(w.gates), "passes": K,
              "workspace_slots": st2["workspace_slots"]}
    extra = {"gate_amps_per_s": len(w.gates) * N / dt}
    line = report(args, w, sim, K * N / dt, K, 1, dt, kt, st1, st2, None, config, mfma_flops=flops, extra=extra)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_sample(w, args.cpu_seconds, args.chunk_log2, fused_k=5)
    return line


def grover_exact(n, marked, layer_done, idx):
    """Exact amplitudes at indices idx of the Grover circuit after its initial
    H layer, the first oracle and H on qubits 0..layer_done-1 of the first
    diffusion (uncompressed arithmetic: the state before the diffusion is
    c (1 - 2 [i = w]) with c = 2^(-n/2); H on the j low qubits maps it to
    c 2^(j/2) [low_j(i) = 0] - 2 c 2^(-j/2) (-1)^popcount(low_j(i) & w) [high(i) = high(w)])."""
    import numpy as np
    idx = np.asarray(idx, dtype=np.int64)
    j = layer_done
    c = 2.0 ** (-n / 2)
    low = (1 << j) - 1
    a = np.where((idx & low) == 0, c * 2.0 ** (j / 2), 0.0)
    par = np.array([bin(int(i) & marked & low).count("1") & 1 for i in idx])
    same = (idx >> j) == (marked >> j)
    a = a - np.where(same, 2 * c * 2.0 ** (-j / 2) * np.where(par == 1, -1.0, 1.0), 0.0)
    return a.astype(np.complex128)


def grover34_sample_ranges(n, sl, marked, seed=11):
    """Amplitude ranges read out for the precision comparison: 64 runs of 4096
    amplitudes at seeded slice offsets, plus the run holding the marked index."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    starts = sorted({int(x) << 12 for x in rng.integers(0, 1 << (n - 12), size=64)} | {(marked >> 12) << 12})
    return [(b, 4096) for b in starts]


def run_grover34_leg(args, w, fp32, K, Wm, codec=None):
    """One precision of the headline: the prelude untimed, Wm warm-up passes
    (the end of the initial H layer), K timed passes from the first oracle on;
    then the same window again from |0...0> with per-kernel event timing, and
    single-pass latencies after it."""
    import torch
    import numpy as np
    import paper_1811_05630_amd as cq
    n, N = w.n_qubits, 1 << w.n_qubits
    start = n  # the first oracle
    assert Wm <= start
    # record arenas sized up front for a ratio of 4 (the window's smallest is
    # about 6.6, in its first diffusion passes), so that no arena grows, and
    # no pass is run again, inside the timed region
    if codec is None:
        codec = dict(zero_chunks=args.zero_chunks, const_chunks=args.const_chunks, chunk_runs=args.chunk_runs,
                     opt=args.opt)
    sim = cq.Sim(n, w.slice_log2, w.error_bound, chunk_log2=args.chunk_log2, workspace_bytes=96 << 30,
                 arena_bytes=(16 << n) // 4, fp32=fp32, **codec)
    g = cq.Circuit(w.gates)  # marshalled once, outside the timed region
    assert len(g) >= start + K + args.latency_passes

    def prelude():
        sim.init_basis(0)
        sim.apply(g[:start - Wm])
        sim.apply(g[start - Wm:start])  # warm-up passes

    prelude()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.apply(g[start:start + K])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st2 = sim.stats()
    samples = grover34_sample_ranges(n, w.slice_log2, w.basis)
    read = np.concatenate([sim.amplitudes(b, c) for b, c in samples])
    # the same window with per-kernel events (HIP events on the library's stream)
    prelude()
    st1 = sim.stats()
    sim.kernel_times(True)
    sim.apply(g[start:start + K])
    torch.cuda.synchronize()
    kt = sim.kernel_times(False)
    st3 = sim.stats()
    lat = []
    for i in range(args.latency_passes):
        torch.cuda.synchronize()
        a = time.perf_counter()
        sim.apply(g[start + K + i:start + K + i + 1])
        lat.append((time.perf_counter() - a) * 1e3)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return dict(dt=dt, kt=kt, st1=st1, st2=st2, st3=st3, lat=lat, read=read, samples=samples)


def run_grover34(args):
    """The headline: 34-qubit Grover search (1024 slices of 2^24, absolute
    bound 1e-8), FP64, timed from the first oracle into its diffusion layer;
    the FP32 leg and a leg with the record variants (zero chunks, constant
    chunks, chunk runs) beside it."""
    import numpy as np
    import qcircuits as qc

    w = qc.grover_workload(n=34, slice_log2=24, eb=1e-8, seed=args.seed, iterations=1)
    n, N = w.n_qubits, 1 << w.n_qubits
    K, Wm = args.steps, args.warmup
    start = n
    print("[bench] grover34 FP64 leg", file=sys.stderr, flush=True)
    r64 = run_grover34_leg(args, w, False, K, Wm)
    layer_done = max(0, min(n, K - 1))  # diffusion H gates inside the window
    idx = np.concatenate([np.arange(b, b + c) for b, c in r64["samples"]])
    exact = grover_exact(n, w.basis, layer_done, idx) if K <= n + 1 else None

    def err(a, b):
        d = a - b
        return {"max_abs": float(np.max(np.abs(d))), "l2": float(np.linalg.norm(d)),
                "l2_rel": float(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300))}

    config = {"workload": "grover34: 34-qubit Grover search (marked index from seed %d), 1024 slices of 2^24 "
                          "amplitudes (raw FP64 state 256 GiB, held compressed), absolute bound 1e-8, plain mode, "
                          "FP64; passes %d..%d timed (the first oracle, then H on qubits 0..%d of its diffusion; "
                          "every slice holds nonzero amplitudes), after the initial H layer"
                          % (args.seed, start, start + K - 1, K - 2) +
                          (", zero-chunk records" if args.zero_chunks else "") +
                          (", constant-chunk records" if args.const_chunks else "") +
                          (", chunk-run records" if args.chunk_runs else "") +
                          (", optimised passes" if args.opt else ""),
              "n_qubits": n, "slice_log2": w.slice_log2, "chunk_log2": args.chunk_log2,
              "error_bound": w.error_bound, "passes_timed": K, "first_timed_pass": start,
              "workspace_slots": r64["st2"]["workspace_slots"], "fp32": False}
    line = report(args, w, None, K * N / r64["dt"], K, Wm, r64["dt"], r64["kt"], r64["st1"], r64["st3"],
                  r64["lat"], config, plane_bytes=8 if compact_workspace(w, False, args.chunk_log2) else 16,
                  nslices=1 << (n - w.slice_log2))
    acc = {"sample": "%d amplitudes in %d runs of 4096 (seeded offsets and the marked index's run)"
                     % (idx.size, len(r64["samples"]))}
    if exact is not None:
        acc["fp64_vs_exact"] = err(r64["read"], exact)
    if not args.no_fp32:
        print("[bench] grover34 FP32 leg", file=sys.stderr, flush=True)
        r32 = run_grover34_leg(args, w, True, K, Wm)
        acc["fp32_vs_fp64"] = err(r32["read"], r64["read"])
        if exact is not None:
            acc["fp32_vs_exact"] = err(r32["read"], exact)
        kt32 = r32["kt"]
        ms32 = {k: v[0] / v[1] for k, v in kt32.items() if v[1] > 0}
        line["fp32"] = {"value": K * N / r32["dt"], "unit": "amps/s", "ms_per_step": r32["dt"] / K * 1e3,
                        "ratio": r32["st3"]["raw_bytes"] / r32["st3"]["compressed_bytes"],
                        "min_ratio": r32["st3"]["min_ratio"], "kernel_ms_per_launch": ms32,
                        "max_abs_codec_err": r32["st3"]["max_abs_codec_err"],
                        "latency_ms_per_pass": {"p50": float(np.percentile(r32["lat"], 50)),
                                                "p99": float(np.percentile(r32["lat"], 99))}
                        if r32["lat"] else None}
    line["accuracy"] = acc
    if not args.no_codec_leg and not (args.chunk_runs or args.zero_chunks or args.const_chunks or args.opt):
        # the same window with the record variants past the Huffman stage
        # (zero chunks, constant chunks, chunk runs): the same codes and
        # amplitudes, smaller records
        print("[bench] grover34 chunk-run leg", file=sys.stderr, flush=True)
        rr = run_grover34_leg(args, w, False, K, Wm,
                              codec=dict(zero_chunks=True, const_chunks=True, chunk_runs=True))
        line["chunk_runs"] = {"value": K * N / rr["dt"], "unit": "amps/s", "ms_per_step": rr["dt"] / K * 1e3,
                              "ratio": rr["st3"]["raw_bytes"] / rr["st3"]["compressed_bytes"],
                              "min_ratio": rr["st3"]["min_ratio"],
                              "records": "zero-chunk, constant-chunk and chunk-run records",
                              "same_readout_as_plain": bool(np.array_equal(rr["read"], r64["read"]))}
    if not args.no_cpu:
        print("[bench] grover34 CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_grover34(w, args.cpu_seconds, args.chunk_log2, K)
    return line


def cpu_grover34(w, seconds, chunk_log2, K):
    """The oracle on sampled slices of the headline window: one slice of the
    state the window starts from (after the initial H layer every slice holds
    the same values, 2^-17, and the oracle compresses it itself) put through
    the window's slice-local passes (H on qubits 0, 1, ...) by
    oracle.pass_group, each worker on its own slice; all workers for `seconds`,
    then one for a third of that."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    import qcircuits as qc
    L = 1 << w.slice_log2
    amp = np.full(L, 2.0 ** (-w.n_qubits / 2))
    rec0, _ = oracle.compress_slice(amp, np.zeros(L), w.slice_log2, chunk_log2, w.error_bound, oracle.ABS)
    # the scale of the whole stored state: 1024 equal slices
    h = oracle.parse_header(rec0)
    s = oracle.rsqrt(oracle.norm(np.full(1 << (w.n_qubits - w.slice_log2), h["step"]),
                                 [h["sumsq"]] * (1 << (w.n_qubits - w.slice_log2))))
    gates = [qc.H(q) for q in range(min(K, w.slice_log2))]

    def worker(deadline):
        rec, done, t = rec0, 0, time.perf_counter()
        while time.perf_counter() < deadline:
            rec = oracle.pass_group(w.n_qubits, w.slice_log2, chunk_log2, w.error_bound, oracle.ABS,
                                    gates[done % len(gates)], s, [0], [rec])[0]
            done += 1
        return done

    threads = min(16, len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        counts = list(ex.map(worker, [t0 + seconds] * threads))
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    one = worker(t1 + seconds / 3)
    dt1 = time.perf_counter() - t1
    total = sum(counts)
    return {"value": total * L / dt, "unit": "amps/s", "cores": threads, "kind": "oracle",
            "sample": f"{total} single-slice passes (H on qubits 0..{len(gates) - 1} in turn) over slices of 2^"
                      f"{w.slice_log2} amplitudes of the window's starting state, compressed by the oracle; "
                      f"{threads} threads, one slice each, {dt:.1f} s",
            "one_thread": {"value": one * L / dt1, "unit": "amps/s",
                           "sample": f"{one} such passes on one thread, {dt1:.1f} s"}}


def serve_jobs(count, seed):
    """A seeded stream of independent jobs: n ~ U{16..24}, absolute bound
    log-uniform in [1e-7, 1e-4], FP32 or FP64 with equal odds, and one of three
    families with equal odds -- Grover (1..8 iterations, random marked index,
    from |0...0>), the QFT of a random basis state, or 20 random layers of U3
    gates and CZ on a random perfect matching (from |0...0>).  64 slices per
    state (at most 2^18 amplitudes each), chunks of 256 values."""
    import numpy as np
    import qcircuits as qc
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for i in range(count):
        n = int(rng.integers(16, 25))
        fam = int(rng.integers(0, 3))
        eb = float(10 ** rng.uniform(-7, -4))
        fp32 = bool(rng.integers(0, 2))
        job = dict(n=n, sl=min(18, n - 6), eb=eb, fp32=fp32, family=fam, init="zero", basis=0)
        if fam == 0:
            job["gates"] = qc.grover(n, int(rng.integers(0, 1 << n)), int(rng.integers(1, 9)))
        elif fam == 1:
            job["gates"] = qc.qft(n)
            job["init"], job["basis"] = "basis", int(rng.integers(0, 1 << n))
        else:
            job["gates"] = qc.random_layered(n, 20, seed=int(rng.integers(0, 1 << 31)))
        jobs.append(job)
    return jobs


def run_serve(args):
    """Serving: jobs arrive as a Poisson stream (mean gap --arrival-ms) and
    run on the job server, up to --max-active at once within a device-memory
    budget.  Value: amplitude-passes of all jobs per second of makespan (first
    arrival to last completion); beside it the job latency percentiles
    (completion - arrival).  A sample of jobs is run again alone and compared
    bit for bit."""
    import numpy as np
    import paper_1811_05630_amd as cq
    rng = np.random.Generator(np.random.PCG64(args.seed + 1))
    n_jobs = args.jobs
    jobs = serve_jobs(n_jobs + 2, args.seed)
    warm, jobs = jobs[:2], jobs[2:]
    for j in jobs + warm:
        j["circ"] = cq.Circuit(j["gates"])
    keep = 4096  # leading amplitudes returned per job (compared in the alone check)

    def submit(srv, j):
        return srv.submit(j["n"], j["sl"], j["eb"], j["circ"], family=j["family"], init=j["init"], basis=j["basis"],
                          fp32=j["fp32"], chunk_log2=args.chunk_log2, out_count=keep)

    budget = int(args.budget_gib * (1 << 30))
    srv = cq.Server(budget, args.max_active)
    for j in warm:
        submit(srv, j)
    srv.drain(timeout=600)
    gaps = rng.exponential(args.arrival_ms / 1e3, size=n_jobs)
    arrive = np.cumsum(gaps) - gaps[0]
    t_base = srv.clock()
    ids, done, k = {}, [], 0
    while k < n_jobs or len(done) < n_jobs:
        now = srv.clock() - t_base
        while k < n_jobs and arrive[k] <= now:
            ids[submit(srv, jobs[k])] = k
            k += 1
        wait = (arrive[k] - (srv.clock() - t_base)) if k < n_jobs else 1.0
        got = srv.wait(timeout=max(0.0, min(wait, 1.0)))
        done += got
        if got and len(done) % 50 < len(got):
            print(f"[serve] {len(done)}/{n_jobs} jobs done", file=sys.stderr, flush=True)
    srv.close()
    bad = [d for d in done if d["status"] != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} jobs failed, first: {bad[0]['error']}")
    t0 = min(d["t_submit"] for d in done)
    t1 = max(d["t_end"] for d in done)
    makespan = t1 - t0
    amp_passes = sum(d["stats"]["passes"] * (1 << jobs[ids[d["id"]]]["n"]) for d in done)
    lat = np.array([d["t_end"] - d["t_submit"] for d in done]) * 1e3
    wait_q = np.array([d["t_start"] - d["t_submit"] for d in done]) * 1e3
    service = np.array([d["t_end"] - d["t_start"] for d in done]) * 1e3
    # the same jobs alone (one at a time) give the same bits
    sample = [d for d in done if ids[d["id"]] < 6]
    alone = cq.Server(budget, 1)
    alone_ids = [submit(alone, jobs[ids[d["id"]]]) for d in sample]
    again = {r["id"]: r for r in alone.drain(600)}
    alone.close()
    same = all(np.array_equal(d["amplitudes"].view(np.uint64), again[a]["amplitudes"].view(np.uint64)) and
               d["stats"]["compressed_bytes"] == again[a]["stats"]["compressed_bytes"]
               for d, a in zip(sample, alone_ids))
    fams = ["grover", "qft", "layered"]
    return {
        "metric": METRIC, "value": amp_passes / makespan, "unit": "amps/s", "n_gpus": 1, "steps": n_jobs,
        "warmup": len(warm), "ms_per_step": makespan / n_jobs * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "serve: %d independent jobs, Poisson arrivals (mean gap %g ms), n ~ U{16..24} (the 16..28 "
                               "mix narrowed so that the stream finishes in seconds), "
                               "absolute bound log-uniform [1e-7, 1e-4], FP32/FP64 1:1, Grover (1..8 iterations) / "
                               "QFT of a basis state / 20 random U3+CZ layers 1:1:1, up to %d jobs at once within "
                               "%g GiB" % (n_jobs, args.arrival_ms, args.max_active, args.budget_gib),
                   "jobs": n_jobs, "max_active": args.max_active, "budget_bytes": budget,
                   "chunk_log2": args.chunk_log2, "seed": args.seed},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "queue_wait_ms": {"p50": float(np.percentile(wait_q, 50)), "p99": float(np.percentile(wait_q, 99))},
        "service_ms": {"p50": float(np.percentile(service, 50)), "p99": float(np.percentile(service, 99))},
        "jobs_per_s": n_jobs / makespan,
        "overlap": float(service.sum() / 1e3 / makespan),
        "ratio": {"final_median": float(np.median([d["stats"]["ratio"] for d in done])),
                  "min_over_jobs": float(min(d["stats"]["min_ratio"] for d in done))},
        "jobs_by_family": {f: sum(1 for d in done if d["family"] == i) for i, f in enumerate(fams)},
        "alone_equals_mixed": {"checked": len(sample), "identical": bool(same)},
        "roofline": None,
    }


def cpu_sample(w, seconds, chunk_log2, fused_k, fp32=False):
    """The oracle on a bounded sample of a large workload: one slice of the
    workload's shape, compressed by the oracle itself, put through repeated
    single-slice passes (a 5-qubit dense block for the fused workload, else
    H on qubit 3) on one host thread."""
    import numpy as np
    import oracle
    import qcircuits as qc
    L = 1 << w.slice_log2
    mode = (oracle.REL if w.relative else oracle.ABS) | (oracle.FP32 if fp32 else 0)
    if w.factors is not None:  # the product state's first slice
        f = np.asarray(w.factors)
        amp = np.ones(L, dtype=complex)
        idx = np.arange(L)
        for q in range(w.slice_log2):
            amp *= np.where((idx >> q) & 1, f[q, 1], f[q, 0])
        amp *= np.prod(f[w.slice_log2:, 0])
    else:  # the state after the H layer
        amp = np.full(L, 2.0 ** (-w.n_qubits / 2), dtype=complex)
    rec, _ = oracle.compress_slice(amp.real.copy(), amp.imag.copy(), w.slice_log2, chunk_log2, w.error_bound, mode)
    if fused_k:
        r = np.random.default_rng(1)
        a = r.standard_normal((32, 32)) + 1j * r.standard_normal((32, 32))
        gate = qc.U([0, 1, 2, 3, 4], np.linalg.qr(a)[0])
    else:
        gate = qc.H(3)
    oracle.set_threads(1)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        rec = oracle.pass_group(w.n_qubits, w.slice_log2, chunk_log2, w.error_bound, mode, gate,
                                1.0, [0], [rec])[0]
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done * L / dt, "unit": "amps/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} single-slice passes ({'5-qubit dense block' if fused_k else 'H on qubit 3'}) "
                      f"over one slice of 2^{w.slice_log2} amplitudes, {dt:.1f} s, one thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU slice sharding is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    run = {"grover34": run_grover34, "grover24": run_grover24, "qft30": run_qft30, "qft12": run_qft12,
           "serve": run_serve}[args.workload]
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
