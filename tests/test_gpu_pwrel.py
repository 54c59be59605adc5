"""GPU parity in pointwise-relative mode (SIM_EB_PWREL) through the C ABI.

Each value is stored as the nearest FP64 number with b mantissa bits; the
codes are integers from the bit pattern and the slice norms FP64 pairwise
trees in a fixed order, so plain mode is deterministic end to end: records
byte-identical with the oracle's pointwise-relative mode after every checked
pass, read-out bit-identical.  Each case prints its name before it touches
the GPU."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from tests.test_gpu_parity import assert_same_records, gate_zoo, say

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def run_both(n, sl, cl, eb, gates, init=None, check_every=1, fp32=False, workspace_bytes=0):
    mode = oracle.PWREL | (oracle.FP32 if fp32 else 0)
    orc = oracle.OracleSim(n, sl, cl, eb, mode)
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, pointwise=True, fp32=fp32, workspace_bytes=workspace_bytes)
    if init is not None:
        orc.init_product(init)
        sim.init_product(init)
    assert_same_records(sim, orc, "initial state")
    for i in range(0, len(gates), check_every):
        chunk = gates[i:i + check_every]
        orc.apply(chunk)
        assert sim.apply(chunk) == len(chunk)
        assert_same_records(sim, orc, f"after gate {i + len(chunk)} ({chunk[-1].name})")
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())
    return sim, orc


GEOMETRIES = [  # n, slice_log2, chunk_log2, eb: whole tiles of 1024, short slices, slice-index targets
    (10, 5, 4, 0.01), (11, 10, 8, 1e-3), (12, 11, 10, 0.01), (12, 6, 6, 1e-4), (9, 3, 2, 0.2),
]


@pytest.mark.parametrize("n,sl,cl,eb", GEOMETRIES)
def test_pwrel_product_qft_and_zoo(n, sl, cl, eb):
    say("pwrel", n, sl, cl, eb)
    f = qc.product_factors(*qc.product_angles(n, n + 3))
    gates = qc.qft(n) + gate_zoo(n, n)
    run_both(n, sl, cl, eb, gates, init=f, check_every=max(1, len(gates) // 10))


def test_pwrel_fp32_and_small_workspace():
    n, sl, cl, eb = 11, 7, 6, 1e-3
    say("pwrel fp32, several batches", n, sl, cl, eb)
    f = qc.product_factors(*qc.product_angles(n, 2))
    sim, orc = run_both(n, sl, cl, eb, qc.random_layered(n, 2, seed=4), init=f, check_every=9, fp32=True,
                        workspace_bytes=400_000)
    assert sim.stats()["workspace_slots"] == 2  # eight batches per pass


def test_pwrel_grover_keeps_small_amplitudes():
    n, sl, cl, eb = 12, 8, 8, 0.01
    say("pwrel grover", n, sl, cl, eb)
    w, k = 1234, 6
    sim, orc = run_both(n, sl, cl, eb, qc.grover(n, w, k), check_every=50)
    a = sim.amplitudes()
    from tests.brute import grover_closed_form
    exact = grover_closed_form(n, w, k)
    # every stored value keeps its relative precision, small ones included
    assert np.count_nonzero(a) == np.count_nonzero(exact)


def test_pwrel_records_checked_on_import():
    n, sl, cl, eb = 10, 6, 5, 0.01
    say("pwrel import", n, sl, cl, eb)
    a = cq.Sim(n, sl, eb, chunk_log2=cl, pointwise=True)
    a.apply(qc.qft(n))
    recs = a.records()
    b = cq.Sim(n, sl, eb, chunk_log2=cl, pointwise=True)
    for j, r in enumerate(recs):
        b.import_record(j, r)
    assert b.records() == recs
    assert np.array_equal(b.amplitudes(), a.amplitudes())
    plain = cq.Sim(n, sl, eb, chunk_log2=cl)
    with pytest.raises(cq.SimError) as e:
        plain.import_record(0, recs[0])  # a pointwise-relative record in an absolute-bound handle
    assert e.value.rc == -4
    other = cq.Sim(n, sl, 1e-3, chunk_log2=cl, pointwise=True)
    with pytest.raises(cq.SimError) as e:
        other.import_record(0, recs[0])  # other mantissa bits
    assert e.value.rc == -4


def test_pwrel_refused_configurations():
    say("pwrel refused")
    for eb in (0.5, 1e-9):
        with pytest.raises(cq.SimError) as e:
            cq.Sim(6, 3, eb, pointwise=True)
        assert e.value.rc == -1
    with pytest.raises(cq.SimError):
        cq.Sim(6, 3, 0.01, pointwise=True, relative=True)
