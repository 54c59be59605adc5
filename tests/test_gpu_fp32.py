"""GPU parity in FP32 mode (SIM_FP32) through the C ABI: the working values,
gate matrices and every product and sum of the gate arithmetic are FP32, the
quantiser and norm FP64, so plain mode is again deterministic end to end and
the records must be byte-identical with the oracle's FP32 mode after every
checked pass.  Fused blocks of three or more qubits (FP64 matrix cores, output
rounded to FP32) are compared within the fused-mode tolerance.  Each case
prints its name before it touches the GPU."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from tests.test_gpu_parity import assert_same_records, gate_zoo, run_both, say

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")

GEOMETRIES = [  # n, slice_log2, chunk_log2, eb: whole tiles, short slices, wavefront ranges
    (6, 3, 2, 1e-7), (10, 5, 5, 1e-6), (12, 11, 10, 1e-6), (12, 10, 8, 1e-6), (13, 11, 7, 1e-7),
    (13, 12, 8, 1e-8),
]


@pytest.mark.parametrize("n,sl,cl,eb", GEOMETRIES)
def test_fp32_gate_zoo(n, sl, cl, eb):
    say("fp32 zoo", n, sl, cl, eb)
    gates = qc.random_layered(n, 2, seed=n + 1) + gate_zoo(n, n + 1)
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=max(1, len(gates) // 12), fp32=True)
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())
    st = sim.stats()
    assert st["raw_bytes"] == 8 << n


def test_fp32_qft12_every_pass():
    w = qc.qft_basis_workload()
    say("fp32 qft12")
    run_both(w.n_qubits, w.slice_log2, 10, w.error_bound, w.gates, init=("basis", w.basis), fp32=True)


@pytest.mark.parametrize("n,sl,cl", [(10, 6, 5), (12, 10, 8)])
def test_fp32_relative_product_qft(n, sl, cl):
    say("fp32 rel qft", n, sl, cl)
    theta, phi = qc.product_angles(n, 4)
    f = qc.product_factors(theta, phi)
    sim, orc = run_both(n, sl, cl, 1e-4, qc.qft(n), rel=True, init=("product", f), check_every=7, fp32=True)
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())


def test_fp32_grover_small():
    n, sl, cl, eb = 10, 6, 6, 1e-7
    say("fp32 grover10")
    gates = qc.grover(n, 613, 4)
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=23, fp32=True)
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())


def decoded_state32(recs):
    """The stored state decoded by the oracle in FP32 mode, scaled like a read-out."""
    s = oracle.scale_from_records(recs)
    return np.concatenate([oracle.decompress_slice(r, oracle.parse_header(r)["step"] * s, oracle.FP32)
                           for r in recs])


def test_fp32_fused_blocks():
    """Fused QFT in FP32 mode, one pass at a time against the oracle's FP32
    fused pass from the same records.  Blocks of 1-2 qubits run the plain
    kernels: byte-equal.  Blocks of 3-5 qubits: the oracle rounds every
    product and partial sum to FP32, the matrix cores sum in FP64 and round
    once, so a gate output may differ by up to
        ((2^k + 2) sqrt(2) sqrt(2^k) + 1) 2^-24 max|a|
    (recursive summation of the 2^k complex terms, |sum_c u_rc a_c| <=
    ||u_r|| ||a|| <= sqrt(2^k) max|a| for a unitary row), and its code by that
    plus one step."""
    n, sl, cl, eb = 11, 8, 6, 1e-7
    say("fp32 fused", n, sl, cl, eb)
    gates = qc.qft(n)
    x = 1234
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, fused=True, fp32=True)
    sim.init_basis(x)
    step = oracle.abs_step(eb)[0]
    plan = cq.plan(n, gates)
    bound = 0.0  # first-order bound of the distance to the exact result
    for first, count, fused, qubits in plan:
        recs = sim.records()
        orc = oracle.OracleSim(n, sl, cl, eb, oracle.FP32)
        orc.set_records(recs)
        amax = float(np.max(np.abs(decoded_state32(recs))))
        k = len(qubits) if fused else len(gates[first].targets)
        rnd = ((2 ** k + 2) * math.sqrt(2) * math.sqrt(2 ** k) + 1) * 2.0 ** -24 * amax
        bound += math.sqrt(2 << n) * (eb + rnd)
        orc.apply(gates[first:first + count], fused=True)
        assert sim.apply(gates[first:first + count]) == count
        got = sim.records()
        if not fused or len(qubits) <= 2:
            assert got == orc.records(), f"pass at gate {first}"
            continue
        tol = step + rnd
        for j in range(orc.nslices):
            a = oracle.decompress_slice(got[j], oracle.parse_header(got[j])["step"], oracle.FP32)
            b = oracle.decompress_slice(orc.record(j), oracle.parse_header(orc.record(j))["step"], oracle.FP32)
            d = float(np.max(np.abs(a - b)))
            assert d <= tol, f"pass at gate {first}, slice {j}: {d} > {tol}"
    a = sim.amplitudes()
    assert np.array_equal(a.real, a.real.astype(np.float32).astype(np.float64))
    assert np.array_equal(decoded_state32(sim.records()), a)
    want = np.exp(2j * np.pi * x * np.arange(1 << n) / (1 << n)) / math.sqrt(1 << n)
    # first-order bound against the exact result: each pass adds at most
    # sqrt(2N) (eb + the FP32 rounding of its gate outputs)
    assert np.linalg.norm(a - want) <= bound
    assert abs(np.vdot(want, a)) ** 2 > 0.999


def test_fp32_and_fp64_differ_and_agree():
    """The two precisions give different records, and amplitudes within the
    FP32 rounding of each other."""
    n, sl, cl, eb = 12, 10, 8, 1e-7
    say("fp32 vs fp64", n, sl, cl, eb)
    gates = qc.random_layered(n, 3, seed=2)
    a = cq.Sim(n, sl, eb, chunk_log2=cl)
    b = cq.Sim(n, sl, eb, chunk_log2=cl, fp32=True)
    a.apply(gates)
    b.apply(gates)
    assert a.records() != b.records()
    assert np.linalg.norm(a.amplitudes() - b.amplitudes()) < 1e-4
