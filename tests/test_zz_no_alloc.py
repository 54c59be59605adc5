"""The allocation-free entry point sim_apply_noalloc against sim_apply, through
the C ABI: twin handles run the same program, one through each entry point,
and must hold byte-identical records and bit-identical amplitudes.  Two calls
in a row, the second with a smaller state, so that the second runs on what
the first left in the shared scratch array; the handle's device bytes do not
change during the calls.  Each case prints its name before it touches the
GPU."""
import sys

import numpy as np
import pytest

import qcircuits as qc

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def twin_run(n, sl, cl, eb, gates, init=None, **kw):
    a = cq.Sim(n, sl, eb, chunk_log2=cl, arena_bytes=64 << 20, **kw)
    b = cq.Sim(n, sl, eb, chunk_log2=cl, arena_bytes=64 << 20, **kw)
    for s in (a, b):
        if init is not None:
            s.init_product(init)
    assert a.apply(gates) == len(gates)
    before = b.stats()["device_bytes"]
    rc, applied = b.apply_noalloc(gates)
    assert rc == 0, f"sim_apply_noalloc failed with {rc}: {cq.lib().sim_last_error().decode()}"
    assert applied == len(gates)
    assert b.stats()["device_bytes"] == before
    assert a.records() == b.records()
    assert np.array_equal(a.amplitudes(), b.amplitudes())
    sa, sb = a.stats(), b.stats()
    assert sa["compressed_bytes"] == sb["compressed_bytes"] and sa["passes"] == sb["passes"]
    return a, b


def test_noalloc_two_calls_second_smaller():
    # 16 slices of 2^17 through a scratch array of 8 slots (two batches per pass),
    # slice-index targets (groups of two slices)
    n, sl, cl, eb = 21, 17, 8, 1e-7
    say("noalloc call 1", n, sl, cl, eb)
    gates = qc.random_layered(n, 2, seed=5) + qc.grover(n, 777777, iterations=1)
    twin_run(n, sl, cl, eb, gates)
    # a smaller state next, relative bound and fused blocks (matrices in the array)
    n2, sl2, cl2 = 11, 7, 5
    say("noalloc call 2", n2, sl2, cl2)
    theta, phi = qc.product_angles(n2, 1)
    twin_run(n2, sl2, cl2, 1e-4, qc.qft(n2), init=qc.product_factors(theta, phi), relative=True, fused=True)


def test_noalloc_refuses_what_does_not_fit():
    n, sl, eb = 22, 21, 1e-6
    say("noalloc too large", n, sl)
    s = cq.Sim(n, sl, eb, chunk_log2=8)
    recs = s.records()
    rc, applied = s.apply_noalloc([qc.H(0)])
    assert rc == -2 and applied == 0
    assert "scratch" in cq.lib().sim_last_error().decode()
    assert s.records() == recs
    # an arena too small for the program: refused, the completed passes kept
    n, sl, cl = 14, 10, 8
    a = cq.Sim(n, sl, 1e-9, chunk_log2=cl)
    b = cq.Sim(n, sl, 1e-9, chunk_log2=cl, arena_bytes=1 << 16)
    gates = qc.random_layered(n, 2, seed=3)
    rc, applied = b.apply_noalloc(gates)
    assert rc == -2 and applied < len(gates)
    assert a.apply(gates[:applied]) == applied
    assert a.records() == b.records()
