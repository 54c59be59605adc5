"""GPU parity in fused mode (SIM_FUSED) through the C ABI.

Blocks of one or two qubits run through the plain kernels and are checked
byte for byte against the oracle's fused mode.  Blocks of three to five
qubits run on FP64 matrix cores, whose sums round in a different order than
the oracle's; there the quantisation codes can differ by one step wherever a
value falls within rounding of a step boundary, so amplitudes are compared
within a stated tolerance (and against exact results), and the records the
GPU writes must decode, by the oracle's own decoder, to exactly the
amplitudes the GPU reads out.  Each case prints its name before it touches
the GPU."""
import math
import sys

import numpy as np
import pytest

import oracle
import qcircuits as qc
from tests.brute import grover_closed_form

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def random_unitary(k, seed):
    r = np.random.default_rng(seed)
    a = r.standard_normal((1 << k, 1 << k)) + 1j * r.standard_normal((1 << k, 1 << k))
    q, rr = np.linalg.qr(a)
    return q * (np.diag(rr) / abs(np.diag(rr)))


def decoded_state(sim):
    """The GPU's stored state decoded by the oracle, scaled like a read-out."""
    recs = sim.records()
    s = oracle.scale_from_records(recs)
    out = []
    for r in recs:
        out.append(oracle.decompress_slice(r, oracle.parse_header(r)["step"] * s))
    return np.concatenate(out)


def both(n, sl, cl, eb, gates, rel=False, init=None):
    mode = oracle.REL if rel else oracle.ABS
    orc = oracle.OracleSim(n, sl, cl, eb, mode)
    sim = cq.Sim(n, sl, eb, relative=rel, chunk_log2=cl, fused=True)
    if init is not None:
        orc.init_product(init)
        sim.init_product(init)
    assert orc.apply(gates, fused=True) == len(gates)
    assert sim.apply(gates) == len(gates)
    return sim, orc


def test_narrow_blocks_are_byte_identical():
    n, sl, cl, eb = 9, 5, 4, 1e-6
    say("fused narrow", n, sl, cl)
    gates = []
    for q in range(n):
        gates += [qc.H(q), qc.P(q, 0.3 + q), qc.CP(q, (q + 1) % n, 0.7), qc.MCZ(n)]
    assert all(len(p[3]) <= 2 for p in oracle.plan(gates))
    sim, orc = both(n, sl, cl, eb, gates)
    for j in range(orc.nslices):
        assert sim.record(j) == orc.record(j), f"slice {j}"
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())


@pytest.mark.parametrize("k,qubits,sl", [(3, (0, 1, 2), 6), (4, (1, 3, 6, 8), 6), (5, (0, 2, 5, 7, 9), 7),
                                         (5, (4, 5, 6, 7, 8), 5), (3, (7, 8, 9), 5), (4, (0, 5, 6, 9), 4)])
def test_one_wide_block_each_layout(k, qubits, sl):
    n, cl, eb = 10, 3, 1e-7
    say("fused block", k, qubits, "slice_log2", sl)
    U = random_unitary(k, 31 + k)
    gates = qc.random_layered(n, 1, seed=k) + [qc.U(list(qubits), U), qc.U([qubits[0]], np.eye(2))]
    plan = oracle.plan(gates)
    assert plan[-1][2] and set(qubits) <= set(plan[-1][3])
    sim, orc = both(n, sl, cl, eb, gates)
    a, b = sim.amplitudes(), orc.amplitudes()
    assert np.max(np.abs(a - b)) <= 4 * eb
    assert np.array_equal(decoded_state(sim), a)
    exact = oracle.sv_run(n, gates)
    assert np.linalg.norm(a - exact) < len(plan) * math.sqrt(2 << n) * eb
    same = sum(sim.record(j) == orc.record(j) for j in range(orc.nslices))
    print(f"  identical records: {same} of {orc.nslices}", flush=True)


def test_qft_of_product_state_relative_bound():
    n, sl, cl, rel = 12, 8, 6, 1e-4
    say("fused qft product", n, sl, cl, rel)
    theta, phi = qc.product_angles(n, 3)
    f = qc.product_factors(theta, phi)
    gates = qc.qft(n)
    sim, orc = both(n, sl, cl, rel, gates, rel=True, init=f)
    a, b = sim.amplitudes(), orc.amplitudes()
    exact = math.sqrt(1 << n) * np.fft.ifft(oracle.product_state(f))
    amax = np.max(np.abs(exact))
    assert np.max(np.abs(a - b)) <= 4 * 2 * rel * amax
    npass = len(oracle.plan(gates))
    assert np.linalg.norm(a - exact) < npass * math.sqrt(2 << n) * 2 * rel * amax
    assert np.array_equal(decoded_state(sim), a)


def test_relative_bound_blocks_take_their_slot_min_max():
    """Slices of 2^10: 5-qubit blocks inside the slice take each slot's min/max
    of their outputs in the block kernel (the relative bound's step), blocks
    with slice-index targets leave it to the min/max kernel.  Every pass's
    records carry the same power-of-two step as the oracle's, and the state
    stays within the bound of the oracle's and of the exact one."""
    n, sl, cl, rel = 13, 10, 6, 1e-4
    say("fused relative min/max", n, sl, cl, rel)
    theta, phi = qc.product_angles(n, 5)
    f = qc.product_factors(theta, phi)
    gates = qc.qft(n)
    plan = oracle.plan(gates)
    inside = [p for p in plan if p[2] and max(p[3]) < sl and len(p[3]) == 5]
    assert inside, "the plan has 5-qubit blocks inside the slice"
    orc = oracle.OracleSim(n, sl, cl, rel, oracle.REL)
    sim = cq.Sim(n, sl, rel, relative=True, chunk_log2=cl, fused=True)
    orc.init_product(f)
    sim.init_product(f)
    for i, p in enumerate(plan):
        g = gates[p[0]:p[0] + p[1]]
        orc.apply(g, fused=True)
        assert sim.apply(g) == len(g)
        for j in range(orc.nslices):
            hs, ho = oracle.parse_header(sim.record(j)), oracle.parse_header(orc.record(j))
            assert hs["step"] == ho["step"], f"pass {i}, slice {j}: step {hs['step']} against {ho['step']}"
    a, b = sim.amplitudes(), orc.amplitudes()
    exact = math.sqrt(1 << n) * np.fft.ifft(oracle.product_state(f))
    amax = np.max(np.abs(exact))
    assert np.max(np.abs(a - b)) <= 4 * 2 * rel * amax
    assert np.linalg.norm(a - exact) < len(plan) * math.sqrt(2 << n) * 2 * rel * amax
    assert np.array_equal(decoded_state(sim), a)


def test_grover_with_cross_slice_blocks():
    n, sl, cl, eb = 11, 5, 4, 1e-7
    say("fused grover", n, sl, cl, eb)
    w = 1234
    k = 4
    gates = qc.grover(n, w, iterations=k)
    sim, orc = both(n, sl, cl, eb, gates)
    a = sim.amplitudes()
    assert np.max(np.abs(a - orc.amplitudes())) <= 4 * eb
    npass = len(oracle.plan(gates))
    assert np.linalg.norm(a - grover_closed_form(n, w, k)) < npass * math.sqrt(2 << n) * eb
    assert np.array_equal(decoded_state(sim), a)


def test_fused_counts_gates_and_stops_at_an_invalid_one():
    n, sl, cl, eb = 8, 5, 4, 1e-6
    say("fused invalid gate", n, sl)
    good = [qc.H(0), qc.H(1), qc.CP(0, 1, 0.3), qc.H(7)]
    bad = qc.Gate(qc.DENSE, (0,), matrix=np.eye(2))
    bad.targets = (9,)
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, fused=True)
    rc, applied = sim.apply_partial(good + [bad, qc.H(2)])
    assert rc == -1 and applied == len(good)
    orc = oracle.OracleSim(n, sl, cl, eb)
    orc.apply(good, fused=True)
    for j in range(orc.nslices):
        assert sim.record(j) == orc.record(j)
