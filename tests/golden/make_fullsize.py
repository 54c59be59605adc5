"""Write the expected results of full-size runs (tests/golden/*_full.json).

Calls only the CPU oracle (oracle.CodeSim: Algorithm 1 at the level of the
quantised codes, whose amplitudes equal the full oracle's) and the exact
closed forms; nothing here runs or reads the HIP library.

    python tests/golden/make_fullsize.py grover24 [--checkpoint DIR] [--threads T]
    python tests/golden/make_fullsize.py qft30 [--threads T]

grover24: 24-qubit Grover search, marked index from seed 0, 64 slices of 2^18
amplitudes, absolute bound 1e-7, floor(pi/4 sqrt(2^24)) = 3216 iterations
(315,192 passes).  The run takes hours on a few cores; it saves its state
every --every passes under --checkpoint and resumes from there.

qft30: 30-qubit QFT of the product state from seed 0, fused mode (blocks of
up to 5 qubits), 256 slices of 2^22, relative bound 1e-4; about half an hour
on eight cores and some 30 GB of memory.  The matrix cores sum in another
order than the oracle, so the GPU's read-out is compared with the exact state
only: qft30_full.json records the oracle's distance from it (the QFT of a
product state in closed form) and the tolerance, 1.5 x that distance.

The grover24 file records the run's read-out (SHA-256 of all amplitudes as interleaved
little-endian FP64 re, im -- the layout sim_amplitudes writes -- and a sample
of them as hexadecimal floats), its error against the exact state (closed
form of Grover's algorithm, including the (-1)^k sign of this circuit's
diffusion), and the tolerance the GPU run is held to: 1.5 x the oracle's
measured 2-norm error, a rule fixed before the GPU run.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import qcircuits as qc  # noqa: E402
from brute import QftProductExact, grover_closed_form  # noqa: E402


def sample_indices(n, marked, count=64, seed=12345):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = sorted(set([0, marked, (1 << n) - 1] + [int(x) for x in rng.integers(0, 1 << n, size=count)]))
    return idx


def run_grover24(args):
    w = qc.grover_workload(seed=0)
    n, sl2, eb = w.n_qubits, w.slice_log2, w.error_bound
    k = qc.grover_iterations(n)
    gates = w.gates
    assert len(gates) == qc.grover_passes(n, k)
    sim = oracle.CodeSim(n, sl2, eb, oracle.ABS)
    ck = os.path.join(args.checkpoint, "grover24.npz")
    if os.path.exists(ck):
        d = dict(np.load(ck, allow_pickle=False))
        d["passes"] = int(d["passes"])
        d["max_err"] = float(d["max_err"])
        sim.set_state(d)
        print(f"resumed at pass {sim.passes}", flush=True)
    t0 = time.time()
    while sim.passes < len(gates):
        a = sim.passes
        b = min(len(gates), a + args.every)
        sim.apply(gates[a:b])
        st = sim.state()
        tmp = ck + ".tmp.npz"
        np.savez(tmp, **st)
        os.replace(tmp, ck)
        el = time.time() - t0
        print(f"pass {sim.passes}/{len(gates)}  {el:.0f} s", flush=True)
    words = sim.amplitude_words()
    sha = hashlib.sha256(words.astype("<f8").tobytes()).hexdigest()
    psi = words[0::2] + 1j * words[1::2]
    exact = grover_closed_form(n, w.basis, k)
    d = psi - exact
    err2 = float(np.linalg.norm(d))
    fid = float(abs(np.vdot(exact, psi)) ** 2 / (np.vdot(psi, psi).real * np.vdot(exact, exact).real))
    idx = sample_indices(n, w.basis)
    out = {
        "workload": "24-qubit Grover search, marked index from seed 0, 64 slices of 2^18 amplitudes, absolute "
                    "bound 1e-7, plain mode, the full circuit",
        "n_qubits": n, "slice_log2": sl2, "error_bound": eb, "marked": w.basis, "iterations": k,
        "passes": len(gates),
        "readout_sha256": sha,
        "max_abs_codec_err": sim.max_err(),
        "vs_closed_form": {"l2": err2, "max_abs": float(np.max(np.abs(d))), "fidelity": fid,
                           "marked_amplitude": [float(psi[w.basis].real), float(psi[w.basis].imag)],
                           "marked_exact": [float(exact[w.basis].real), float(exact[w.basis].imag)]},
        "tolerance": {"rule": "GPU l2 error vs the closed form <= 1.5 x the oracle's", "l2": 1.5 * err2},
        "sample": {str(i): [float(psi[i].real).hex(), float(psi[i].imag).hex()] for i in idx},
    }
    path = os.path.join(HERE, "grover24_full.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["vs_closed_form"]), flush=True)
    print("wrote", path)


def run_qft30(args):
    """30-qubit QFT of the product state from seed 0 in fused mode (blocks of
    up to 5 qubits), 256 slices of 2^22, relative bound 1e-4: the oracle's run
    of the whole circuit and its distance from the exact state."""
    w = qc.qft_product_workload()
    n, sl2, eb = w.n_qubits, w.slice_log2, w.error_bound
    plan = oracle.plan(w.gates)  # the oracle's own partition into passes
    sim = oracle.CodeSim(n, sl2, eb, oracle.REL)
    sim.init_product(w.factors)
    t0 = time.time()
    for k, (first, count, fused, qubits) in enumerate(plan):
        sim.apply(w.gates[first:first + count], fused=True)
        if k % 10 == 9 or k == len(plan) - 1:
            print(f"pass {k + 1}/{len(plan)}  {time.time() - t0:.0f} s", flush=True)
    m = 24
    ex = QftProductExact(w.factors, m)
    sq, mx, dot, norm2 = 0.0, 0.0, 0.0 + 0.0j, 0.0
    for hi in range(1 << (n - m)):
        got = sim.amplitudes(hi << m, 1 << m)
        want = ex.block(hi)
        d = got - want
        sq += float(np.vdot(d, d).real)
        mx = max(mx, float(np.max(np.abs(d))))
        dot += np.vdot(want, got)
        norm2 += float(np.vdot(got, got).real)
    err2 = math.sqrt(sq)
    out = {
        "workload": "30-qubit QFT of the product state from seed 0, 256 slices of 2^22 amplitudes, relative bound "
                    "1e-4, fused mode (blocks of up to 5 qubits), the whole circuit",
        "n_qubits": n, "slice_log2": sl2, "error_bound": eb, "passes": len(plan), "gates": len(w.gates),
        "vs_closed_form": {"l2": err2, "max_abs": mx, "fidelity": float(abs(dot) ** 2 / norm2)},
        "tolerance": {"rule": "GPU l2 error vs the closed form <= 1.5 x the oracle's", "l2": 1.5 * err2},
    }
    path = os.path.join(HERE, "qft30_full.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["vs_closed_form"]), flush=True)
    print("wrote", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=("grover24", "qft30"))
    ap.add_argument("--checkpoint", default="/tmp/cqsim_golden")
    ap.add_argument("--every", type=int, default=5000)
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    os.makedirs(args.checkpoint, exist_ok=True)
    if args.threads:
        oracle.set_threads(args.threads)
    {"grover24": run_grover24, "qft30": run_qft30}[args.which](args)


if __name__ == "__main__":
    main()
