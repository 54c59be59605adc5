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


def test_fp32_fused_blocks():
    n, sl, cl, eb = 11, 8, 6, 1e-7
    say("fp32 fused", n, sl, cl, eb)
    gates = qc.qft(n)
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, fused=True, fp32=True)
    orc = oracle.OracleSim(n, sl, cl, eb, oracle.FP32)
    x = 1234
    sim.init_basis(x)
    orc.init_basis(x)
    assert sim.apply(gates) == len(gates)
    orc.apply(gates, fused=True)
    a, b = sim.amplitudes(), orc.amplitudes()
    assert np.array_equal(a.real, a.real.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(a - b)) <= 4 * eb * len(cq.plan(n, gates))
    want = np.exp(2j * np.pi * x * np.arange(1 << n) / (1 << n)) / math.sqrt(1 << n)
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
