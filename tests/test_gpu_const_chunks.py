"""GPU parity of constant-chunk records (SIM_CONST_CHUNKS, alone and with
SIM_ZERO_CHUNKS): byte-equal records to the oracle's after every checked
pass, on both decode paths, both precisions and chunk sizes 2^3..2^10; the
record checks on import.  Each case prints its name before it touches the
GPU."""
import struct

import numpy as np
import pytest

import oracle
import qcircuits as qc
from test_gpu_parity import run_both, say

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


@pytest.mark.parametrize("cl", [3, 5, 8, 10])
@pytest.mark.parametrize("zc", [False, True])
def test_grover_constant_chunks_match_the_oracle(cl, zc):
    n, sl, eb = 12, 10, 1e-6
    gates = qc.grover(n, 1234, 1)
    say(f"constant chunks: grover n={n} sl={sl} cl={cl} zero={zc}")
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=5, const_chunks=True, zero_chunks=zc)
    assert np.array_equal(sim.amplitudes().view(np.float64), orc.amplitudes().view(np.float64))
    st = sim.stats()
    assert st["compressed_bytes"] == orc.total_bytes() and st["peak_compressed"] == orc.peak_bytes()


def test_constant_chunks_are_used_and_save_bytes():
    n, sl, cl, eb = 14, 11, 6, 1e-7
    gates = qc.grover(n, 77, 1)
    say("constant chunks: bytes saved on a Grover iteration")
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=len(gates), const_chunks=True)
    plain = cq.Sim(n, sl, eb, chunk_log2=cl)
    plain.apply(gates)
    recs = sim.records()
    assert sum(int(oracle.constant_chunks(r).sum()) for r in recs) > 0
    assert all(oracle.parse_header(r)["flags"] == 2 for r in recs)
    assert sim.stats()["compressed_bytes"] < plain.stats()["compressed_bytes"]
    assert np.array_equal(sim.amplitudes().view(np.float64), plain.amplitudes().view(np.float64))


def test_constant_chunks_fp32_relative_and_basis_state():
    n, sl, cl = 11, 8, 5
    gates = qc.grover(n, 300, 1)
    say("constant chunks: FP32, absolute bound")
    run_both(n, sl, cl, 1e-6, gates, check_every=7, fp32=True, const_chunks=True)
    say("constant chunks: relative bound (FP64 workspace)")
    run_both(n, sl, cl, 1e-4, gates, rel=True, check_every=7, const_chunks=True, zero_chunks=True)
    say("constant chunks: QFT of a basis state")
    run_both(10, 7, 4, 1e-6, qc.qft(10), init=("basis", 3), check_every=11, const_chunks=True)


def test_constant_chunk_records_import_and_checks():
    n, sl, cl, eb = 10, 7, 4, 1e-6
    gates = qc.grover(n, 5, 1)[:n + 4]
    say("constant chunks: export / import")
    src = cq.Sim(n, sl, eb, chunk_log2=cl, const_chunks=True)
    src.apply(gates)
    dst = cq.Sim(n, sl, eb, chunk_log2=cl)  # a handle without the mode reads such records too
    recs = src.records()
    marked = [j for j, r in enumerate(recs) if oracle.constant_chunks(r).any()]
    assert marked
    for j, r in enumerate(recs):
        dst.import_record(j, r)
    assert np.array_equal(dst.amplitudes().view(np.float64), src.amplitudes().view(np.float64))
    after = cq.Sim(n, sl, eb, chunk_log2=cl)
    for j, r in enumerate(recs):
        after.import_record(j, r)
    g = gates[:3]
    dst.apply(g)
    src.apply(g)
    assert np.array_equal(dst.amplitudes().view(np.float64), src.amplitudes().view(np.float64))
    bad = bytearray(recs[marked[0]])
    struct.pack_into("<I", bad, 56, 0)  # marks without the flag
    with pytest.raises(cq.SimError) as e:
        after.import_record(marked[0], bytes(bad))
    assert e.value.rc == -4
