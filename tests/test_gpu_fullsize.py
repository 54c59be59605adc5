"""Full-size checks of the benchmark configurations on the GPU (through the C ABI).

* 12-qubit QFT of a basis state (4 slices of 2^10, absolute bound 1e-6): the
  whole circuit, byte-equal to the oracle and within the first-order bound of
  the closed form.
* 34-qubit Grover search (1024 slices of 2^24, absolute bound 1e-8, several
  workspace batches per pass): a pass at a time, sampled slice groups are
  recomputed by the oracle from the GPU's input records and the normalisation
  of the whole stored state; the output records must be byte-equal.  The
  passes cover slice-local gates, slice-index targets (groups of two slices),
  the oracle's phase and the diffusion, every slice occupied.
* 30-qubit QFT of a product state in fused mode (256 slices of 2^22, relative
  bound 1e-4): sampled slice groups of fused passes recomputed the same way,
  within one quantisation step (the matrix-core sums round differently).
* Fused blocks whose kernel makes several trips through its grid-stride loop,
  and a state of more than 1024 slices (the tree of the norm reduction
  starts from per-thread blocks).

Each case prints its name, geometry and pass before it touches the GPU."""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import qcircuits as qc
from tests.brute import qft_basis_closed_form

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def tolerances():
    with open(os.path.join(GOLDEN, "tolerances.json")) as f:
        return json.load(f)


def oracle_scale(sim):
    """The oracle's normalisation (Normalize of Algorithm 1) of the GPU's
    stored state, from the step and sum p^2 in every record header."""
    return oracle.scale_from_records(sim.headers())


def values(rec):
    """p * step of a record (the quantised values before normalisation)."""
    h = oracle.parse_header(rec)
    return oracle.decompress_slice(rec, h["step"])


def check_groups_exact(sim, n, sl, cl, eb, mode, gate, groups, label):
    """One pass of `gate` on the GPU against the oracle's pass of the same
    gate on the sampled groups, from the same input records: byte equality."""
    s = oracle_scale(sim)
    need = sorted({j for g in groups for j in g})
    before = dict(zip(need, sim.records(need)))
    assert sim.apply([gate]) == 1
    after = dict(zip(need, sim.records(need)))
    for mem in groups:
        want = oracle.pass_group(n, sl, cl, eb, mode, gate, s, mem, [before[j] for j in mem])
        for j, w in zip(mem, want):
            if after[j] != w:
                ha, hb = oracle.parse_header(after[j]), oracle.parse_header(w)
                diff = ", ".join(f"{k}: gpu {ha[k]} oracle {hb[k]}" for k in ha if ha[k] != hb[k])
                pytest.fail(f"{label}: slice {j}: {diff or 'payload differs'}")


# ------------------------------------------------------------------ c1

def test_qft12_basis_closed_form():
    w = qc.qft_basis_workload()
    tol = tolerances()["qft12_basis"]["l2"]
    say("qft12 full circuit", w.n_qubits, w.slice_log2, w.error_bound)
    sim = cq.Sim(w.n_qubits, w.slice_log2, w.error_bound)
    orc = oracle.OracleSim(w.n_qubits, w.slice_log2, 10, w.error_bound)
    sim.init_basis(w.basis)
    orc.init_basis(w.basis)
    assert sim.apply(w.gates) == len(w.gates)
    orc.apply(w.gates)
    assert sim.records() == orc.records()
    a = sim.amplitudes()
    assert np.array_equal(a, orc.amplitudes())
    err = float(np.linalg.norm(a - qft_basis_closed_form(w.n_qubits, w.basis)))
    print(f"  l2 error vs closed form {err:.3e} (tolerance {tol:.3e})", flush=True)
    assert err <= tol


# ------------------------------------------------------------------ c4

def test_grover34_sampled_groups():
    n, sl, eb, cl = 34, 24, 1e-8, 8
    w = qc.grover_workload(n=n, slice_log2=sl, eb=eb, seed=0, iterations=1)
    mslice = w.basis >> sl
    say("grover34 sampled groups", n, sl, eb, "chunk", cl, "marked slice", mslice)
    # 32 slots of 2^24 amplitudes: 32 batches per pass
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, workspace_bytes=32 << 30, arena_bytes=16 << 30)
    assert sim.stats()["workspace_slots"] == 32
    oracle.set_threads(0)
    rng = np.random.default_rng(7)
    other = int(rng.integers(0, 1024))
    checks = {  # pass -> sampled groups (members in the order of the gate's slice bits)
        5: [[0], [1], [other]],
        24: [[0, 1], [2, 3]],
        33: [[0, 512], [mslice & 511, (mslice & 511) | 512]],
        34: [[0], [mslice], [1023]],
        35 + 3: [[mslice], [other], [0]],
        35 + 27: [[j, j | 8] for j in sorted({mslice & ~8, other & ~8})],
    }
    done = 0
    for g in sorted(checks):
        sim.apply(w.gates[done:g])
        gate = w.gates[g]
        say(f"grover34 pass {g} ({gate.name} {gate.targets}) groups {checks[g]}")
        check_groups_exact(sim, n, sl, cl, eb, oracle.ABS, gate, checks[g], f"pass {g}")
        done = g + 1
    st = sim.stats()
    assert st["passes"] == done


# ------------------------------------------------------------------ c3

def test_qft30_fused_sampled_groups():
    w = qc.qft_product_workload()
    n, sl, rel, cl = w.n_qubits, w.slice_log2, w.error_bound, 8
    plan = cq.plan(n, w.gates)
    say("qft30 fused sampled groups", n, sl, rel, "chunk", cl, "passes", len(plan))
    sim = cq.Sim(n, sl, rel, relative=True, chunk_log2=cl, fused=True, workspace_bytes=64 << 30,
                 arena_bytes=4 << 30)
    sim.init_product(w.factors)
    oracle.set_threads(0)
    rng = np.random.default_rng(3)
    done = 0
    for pi in (2, 6):  # qubits (17..20, 29) and (1..4, 29): groups of two slices
        first, count, fused, qubits = plan[pi]
        assert fused
        sim.apply(w.gates[plan[done][0]:first])
        U = oracle.block_matrix(w.gates, first, count, qubits)
        gate = qc.U(list(qubits), U)
        gm = sum(1 << (q - sl) for q in qubits if q >= sl)
        leaders = [j for j in range(1 << (n - sl)) if not j & gm]
        pick = [leaders[0], leaders[int(rng.integers(1, len(leaders)))]]
        groups = [oracle.group_members(n, sl, gate, j0) for j0 in pick]
        say(f"qft30 fused pass {pi} qubits {qubits} groups {groups}")
        s = oracle_scale(sim)
        need = sorted({j for g in groups for j in g})
        before = dict(zip(need, sim.records(need)))
        assert sim.apply(w.gates[first:first + count]) == count
        after = dict(zip(need, sim.records(need)))
        worst = 0.0
        for mem in groups:
            want = oracle.pass_group(n, sl, cl, rel, oracle.REL, gate, s, mem, [before[j] for j in mem])
            for j, rec in zip(mem, want):
                a, b = values(after[j]), values(rec)
                step = max(oracle.parse_header(after[j])["step"], oracle.parse_header(rec)["step"])
                d = float(np.max(np.abs(a - b)))
                worst = max(worst, d / step)
                # one quantisation step: a value within rounding of a step boundary may round
                # either way when the matrix-core sums differ in their last bits
                assert d <= step * (1 + 1e-12), f"pass {pi} slice {j}: {d} > step {step}"
        print(f"  largest difference {worst:.3f} steps", flush=True)
        done = pi + 1


def test_qft30_full_run_closed_form():
    """The whole 30-qubit fused QFT of the product state: the read-out against
    the exact QFT of the product state over all 2^30 amplitudes, within 1.5 x
    the oracle's own distance (tests/golden/qft30_full.json); the first-order
    bound summed from the steps the run's records hold is printed beside it."""
    from concurrent.futures import ThreadPoolExecutor
    from tests.brute import QftProductExact
    w = qc.qft_product_workload()
    n, sl, rel, cl = w.n_qubits, w.slice_log2, w.error_bound, 8
    plan = cq.plan(n, w.gates)
    say("qft30 full run", n, sl, rel, "chunk", cl, "passes", len(plan))
    sim = cq.Sim(n, sl, rel, relative=True, chunk_log2=cl, fused=True, workspace_bytes=64 << 30,
                 arena_bytes=4 << 30)
    L = 1 << sl

    def eps():
        steps = np.array([oracle.parse_header(h)["step"] for h in sim.headers()])
        return math.sqrt(float(np.sum(2 * L * (steps / 2) ** 2)))

    sim.init_product(w.factors)
    bound = 0.0
    e = eps()
    bound += e / (1 - e)
    circ = cq.Circuit(w.gates)
    for first, count, _, _ in plan:
        assert sim.apply(circ[first:first + count]) == count
        e = eps()
        bound += e / (1 - e)
    with open(os.path.join(GOLDEN, "qft30_full.json")) as f:
        want = json.load(f)
    assert (n, sl, rel, len(plan)) == (want["n_qubits"], want["slice_log2"], want["error_bound"], want["passes"])
    tol = want["tolerance"]["l2"]
    m = 24
    ex = QftProductExact(w.factors, m)

    def block(hi, got):
        want = ex.block(hi)
        d = got - want
        return float(np.vdot(d, d).real), float(np.max(np.abs(d))), np.vdot(want, got)

    parts, pending = [], []
    with ThreadPoolExecutor(8) as pool:
        for hi in range(1 << (n - m)):
            pending.append(pool.submit(block, hi, sim.amplitudes(hi << m, 1 << m)))
            if len(pending) >= 12:
                parts.append(pending.pop(0).result())
        parts += [f.result() for f in pending]
    l2 = math.sqrt(sum(p[0] for p in parts))
    mx = max(p[1] for p in parts)
    fid = abs(sum(p[2] for p in parts)) ** 2
    print(f"  l2 {l2:.4e} (oracle {want['vs_closed_form']['l2']:.4e}, tolerance {tol:.4e})  max_abs {mx:.4e}  "
          f"fidelity {fid:.12f}  first-order bound {1.01 * bound + 1e-12:.4e}", flush=True)
    assert l2 <= tol


# ---------------------------------------------------------- fused trips

def random_unitary(k, seed):
    r = np.random.default_rng(seed)
    a = r.standard_normal((1 << k, 1 << k)) + 1j * r.standard_normal((1 << k, 1 << k))
    q, rr = np.linalg.qr(a)
    return q * (np.diag(rr) / abs(np.diag(rr)))


def test_fused_blocks_many_grid_trips():
    """24 qubits in 64 slices of 2^18: 2^24 / 2^k bases per fused pass, more
    than the dense kernel's grid covers in one trip (4096 workgroups x 64
    bases) for k = 3, 4 and 5; each pass compared with the oracle's pass of
    the same block from the same records (within one step, per value)."""
    n, sl, cl, eb = 24, 18, 8, 1e-7
    say("fused many trips", n, sl, cl, eb)
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, fused=True)
    layer = [qc.H(q) for q in range(n)]
    assert sim.apply(layer) == n
    blocks = [(0, 3, 9, 19, 21), (17, 18, 19, 20), (1, 7, 22), (2, 4, 6, 8, 23)]
    oracle.set_threads(0)
    for i, qs in enumerate(blocks):
        U = random_unitary(len(qs), 40 + i)
        gates = [qc.U(list(qs), U), qc.H(qs[0]), qc.U([qs[0]], np.eye(2))]  # one fused pass on qs
        assert len(cq.plan(n, gates)) == 1
        say(f"fused many trips: block {qs}")
        recs = sim.records()
        orc = oracle.OracleSim(n, sl, cl, eb)
        orc.set_records(recs)
        orc.apply(gates, fused=True)
        assert sim.apply(gates) == len(gates)
        got = sim.records()
        worst = 0.0
        for j in range(orc.nslices):
            d = float(np.max(np.abs(values(got[j]) - values(orc.record(j)))))
            worst = max(worst, d)
        step = oracle.abs_step(eb)[0]
        print(f"  largest difference {worst / step:.3f} steps", flush=True)
        assert worst <= step * (1 + 1e-12)


# ------------------------------------------------------ more than 1024 slices

@pytest.mark.parametrize("n,sl,cl", [(12, 1, 1), (13, 2, 2)])
def test_more_than_1024_slices(n, sl, cl):
    say("many slices", n, sl, cl, "slices", 1 << (n - sl))
    from tests.test_gpu_parity import run_both
    gates = qc.random_layered(n, 1, seed=n) + qc.grover(n, 1234 % (1 << n), iterations=1)
    sim, orc = run_both(n, sl, cl, 1e-6, gates, check_every=max(1, len(gates) // 4))
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())


# ------------------------------------------------------------------ c2

def test_grover24_full_run():
    """The whole 24-qubit Grover circuit (315,192 passes over 64 slices of
    2^18, absolute bound 1e-7): the read-out bit-equal to the oracle's run of
    the same circuit (tests/golden/grover24_full.json, written by
    tests/golden/make_fullsize.py from the oracle alone) and within the stated
    distance of Grover's closed form."""
    import hashlib
    from tests.brute import grover_closed_form
    path = os.path.join(GOLDEN, "grover24_full.json")
    with open(path) as f:
        want = json.load(f)
    w = qc.grover_workload(seed=0)
    n, sl, eb = w.n_qubits, w.slice_log2, w.error_bound
    assert (n, sl, eb, w.basis, len(w.gates)) == (want["n_qubits"], want["slice_log2"], want["error_bound"],
                                                  want["marked"], want["passes"])
    say("grover24 full run", n, sl, eb, "passes", len(w.gates))
    sim = cq.Sim(n, sl, eb, chunk_log2=8, arena_bytes=(16 << n) // 4)
    circ = cq.Circuit(w.gates)
    step = 40000
    for a in range(0, len(circ), step):
        assert sim.apply(circ[a:a + step]) == min(step, len(circ) - a)
        print(f"  pass {min(a + step, len(circ))}", flush=True)
    amp = sim.amplitudes()
    words = np.empty(2 * amp.size)
    words[0::2], words[1::2] = amp.real, amp.imag
    sha = hashlib.sha256(words.astype("<f8").tobytes()).hexdigest()
    for i, (re, im) in want["sample"].items():
        i = int(i)
        assert (amp[i].real, amp[i].imag) == (float.fromhex(re), float.fromhex(im)), f"amplitude {i}"
    assert sha == want["readout_sha256"]
    exact = grover_closed_form(n, w.basis, want["iterations"])
    err = float(np.linalg.norm(amp - exact))
    print(f"  l2 error vs closed form {err:.4e} (oracle {want['vs_closed_form']['l2']:.4e}, "
          f"tolerance {want['tolerance']['l2']:.4e})", flush=True)
    assert err <= want["tolerance"]["l2"]
    st = sim.stats()
    assert st["passes"] == len(w.gates) and st["max_abs_codec_err"] <= eb
