"""Benchmark: compressed state-vector passes on one MI355X.

One step is one pass of Algorithm 1 (Section II of the paper) over the whole
state: every slice is decompressed, normalised, updated by one gate and
recompressed.  The workload is 24-qubit Grover search (marked index from seed
0), 64 slices of 2^18 amplitudes, absolute error bound 1e-7, FP64.  Inputs
are synthetic (the paper's circuits are not available); the timed passes are
Grover iterations (oracle + diffusion gates) after the initial H layer.

Prints one JSON line: throughput in state amplitudes per second (amplitude-
passes: 2^24 per step), the compression ratio, per-pass latency percentiles,
the roofline position of the dominant kernel (device times from HIP events on
the library's stream), and the CPU oracle timed on a bounded sample.

`--copy-probe` instead times a plain device copy of known size; its HBM
counter readings calibrate the per-kernel traffic figures below.
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
METRIC = "state amps/s via decompress+gate+compress at error bound; ratio; p99 latency"
KERNEL_SRC = os.path.join(ROOT, "paper_1811_05630_amd", "csrc", "kernels.hip")

# HBM bytes per launch of a kernel class at the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script, each scaled by
# the reading of the same counter for the copy probe.  Valid only for the
# kernel source they were taken on (sha256 of kernels.hip).
MEASURED_TRAFFIC = {
    "gate_quant": {"kernels_sha256": "cdb5c927671fefd55c23314847fb9638be8c8fb40c15a605233e42eaf6058a11",
                   "bytes_per_launch": 319003670},
    "decode": {"kernels_sha256": "cdb5c927671fefd55c23314847fb9638be8c8fb40c15a605233e42eaf6058a11",
               "bytes_per_launch": 263631444},
    "encode": {"kernels_sha256": "cdb5c927671fefd55c23314847fb9638be8c8fb40c15a605233e42eaf6058a11",
               "bytes_per_launch": 83419676},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--chunk-log2", type=int, default=8)
    ap.add_argument("--latency-passes", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 256 MiB device copy (counter calibration) and exit")
    return ap.parse_args()


def kernel_bytes(name, n_amps, c_in, c_out, n_slices, escapes):
    """Algorithmic HBM bytes of one launch of each kernel class over the whole
    state (2^n amplitudes in two FP64 planes; one u16 symbol per value; 8 bytes
    per escaped difference; c_in / c_out compressed bytes read / written)."""
    planes = 16 * n_amps
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


def traffic_for(kernel):
    rec = MEASURED_TRAFFIC.get(kernel)
    if not rec or rec["kernels_sha256"] != source_sha():
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(w, seconds, chunk_log2):
    import oracle
    threads = oracle.num_threads()
    sim = oracle.OracleSim(w.n_qubits, w.slice_log2, chunk_log2, w.error_bound)
    n0 = w.n_qubits  # bring the oracle to the timed region's starting point
    sim.apply(w.gates[:n0])
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < len(w.gates) - n0:
        sim.apply(w.gates[n0 + done:n0 + done + 1])
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done * (1 << w.n_qubits) / dt, "unit": "amps/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} passes of the 24-qubit Grover circuit after its H layer "
                      f"(gates {n0}..{n0 + done - 1}), {dt:.1f} s, OpenMP over slices"}


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(the multi-GPU slice sharding is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    import numpy as np
    import torch
    import paper_1811_05630_amd as cq
    import qcircuits as qc

    w = qc.grover_workload(seed=args.seed)
    n = w.n_qubits
    N = 1 << n
    K, Wm = args.steps, args.warmup
    sim = cq.Sim(n, w.slice_log2, w.error_bound, chunk_log2=args.chunk_log2)
    # initial H layer (untimed), then warm-up passes
    sim.apply(w.gates[:n])
    pos = n
    gates = w.gates
    assert len(gates) >= pos + Wm + 2 * K + args.latency_passes
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

    # per-pass latency: one sim_apply call per pass, host clock
    lat = []
    for i in range(args.latency_passes):
        torch.cuda.synchronize()
        a = time.perf_counter()
        sim.apply(gates[pos + i:pos + i + 1])
        lat.append((time.perf_counter() - a) * 1e3)
    pos += args.latency_passes

    comp = st2["compressed_bytes"]
    esc = (st2["escapes"] - st1["escapes"]) / K  # escapes coded per pass
    ms_launch = {k: v[0] / v[1] for k, v in kt.items() if v[1] > 0}
    dom = max((k for k in ms_launch if k in ("decode", "gate_quant", "codebook", "encode", "header", "compact")),
              key=lambda k: kt[k][0])
    avg_ms = ms_launch[dom]
    algo = kernel_bytes(dom, N, comp, comp, sim.nslices, esc)
    achieved = algo / (avg_ms * 1e-3) / 1e9
    traffic = traffic_for(dom)
    pipe_bytes = 2 * 16 * N + 2 * comp  # B_alg: planes written and read once + records in and out
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grover24: 24-qubit Grover search, marked index from seed 0, 64 slices of 2^18 "
                               "amplitudes, absolute bound 1e-7, plain mode (one pass per gate)",
                   "n_qubits": n, "slice_log2": w.slice_log2, "chunk_log2": args.chunk_log2,
                   "error_bound": w.error_bound, "passes_timed": K, "first_timed_gate": n + Wm},
        "ratio": N * 16 / comp,
        "min_ratio": st2["min_ratio"],
        "max_abs_codec_err": st2["max_abs_codec_err"],
        "latency_ms_per_pass": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "kernel_ms_per_launch": ms_launch,
        "kernel_launches_per_pass": {k: v[1] / K for k, v in kt.items() if v[1] > 0},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": algo, "avg_launch_ms": avg_ms},
        "pipeline_roofline": {"bytes_per_pass": pipe_bytes, "achieved": pipe_achieved, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": pipe_achieved / HBM_PEAK_GBS},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, args.chunk_log2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
