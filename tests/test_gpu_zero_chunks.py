"""GPU parity of zero-chunk records (SIM_ZERO_CHUNKS): byte-equal records to
the oracle's after every checked pass, on both decode paths (int32 and FP64
workspace), both precisions, short and long chunks; and the record checks
on import.  Each case prints its name before it touches the GPU."""
import struct

import numpy as np
import pytest

import oracle
import qcircuits as qc
from test_gpu_parity import assert_same_records, run_both, say

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def empty_chunks(rec):
    return int((np.diff(oracle.chunk_offsets(rec)) == 0).sum())


@pytest.mark.parametrize("cl", [3, 5, 8, 10])
def test_grover_zero_chunks_match_the_oracle(cl):
    n, sl, eb = 12, 10, 1e-6
    gates = qc.grover(n, 1234, 1)
    say(f"zero chunks: grover n={n} sl={sl} cl={cl}")
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=5, zero_chunks=True)
    assert np.array_equal(sim.amplitudes().view(np.float64), orc.amplitudes().view(np.float64))
    st = sim.stats()
    assert st["compressed_bytes"] == orc.total_bytes() and st["peak_compressed"] == orc.peak_bytes()


def test_zero_chunks_are_used_and_save_bytes():
    n, sl, cl, eb = 12, 9, 5, 1e-6
    gates = qc.grover(n, 77, 1)[:n + 6]  # H layer, oracle, part of the diffusion's H layer
    say("zero chunks: bytes saved on a sparse state")
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=len(gates), zero_chunks=True)
    plain = cq.Sim(n, sl, eb, chunk_log2=cl)
    plain.apply(gates)
    recs = sim.records()
    assert sum(empty_chunks(r) for r in recs) > 0
    assert all(oracle.parse_header(r)["flags"] == 1 for r in recs)
    assert sim.stats()["compressed_bytes"] < plain.stats()["compressed_bytes"]
    assert np.array_equal(sim.amplitudes().view(np.float64), plain.amplitudes().view(np.float64))


def test_zero_chunks_fp32_and_relative_bound():
    n, sl, cl = 11, 8, 5
    gates = qc.grover(n, 300, 1)
    say("zero chunks: FP32, absolute bound")
    run_both(n, sl, cl, 1e-6, gates, check_every=7, fp32=True, zero_chunks=True)
    say("zero chunks: relative bound (FP64 workspace)")
    run_both(n, sl, cl, 1e-4, gates, rel=True, check_every=7, zero_chunks=True)
    say("zero chunks: QFT of a basis state, FP64 workspace on the first pass")
    run_both(10, 7, 4, 1e-6, qc.qft(10), init=("basis", 3), check_every=11, zero_chunks=True)


def test_zero_chunk_records_import_and_checks():
    n, sl, cl, eb = 10, 7, 4, 1e-6
    gates = qc.grover(n, 5, 1)[:n + 4]
    say("zero chunks: export / import")
    src = cq.Sim(n, sl, eb, chunk_log2=cl, zero_chunks=True)
    src.apply(gates)
    dst = cq.Sim(n, sl, eb, chunk_log2=cl)  # a handle without the mode reads such records too
    recs = src.records()
    withempty = [j for j, r in enumerate(recs) if empty_chunks(r) and oracle.parse_header(r)["n_used"] > 1]
    assert withempty
    for j, r in enumerate(recs):
        dst.import_record(j, r)
    assert np.array_equal(dst.amplitudes().view(np.float64), src.amplitudes().view(np.float64))
    bad = bytearray(recs[withempty[0]])
    struct.pack_into("<I", bad, 56, 0)  # flag cleared: an empty chunk is now corrupt
    with pytest.raises(cq.SimError) as e:
        dst.import_record(withempty[0], bytes(bad))
    assert e.value.rc == -4


def test_graph_recaptures_when_zero_chunk_records_arrive():
    """A graph captured with the plain decoder is captured again once the
    handle holds imported zero-chunk records; it matches sim_apply."""
    n, sl, cl, eb = 10, 7, 4, 1e-6
    head = qc.grover(n, 5, 1)[:n + 4]
    prog = [qc.H(0), qc.H(1)]  # two passes: the graph starts from its own arena parity again
    say("zero chunks: graph, then imported zero-chunk records")
    src = cq.Sim(n, sl, eb, chunk_log2=cl, zero_chunks=True)
    src.apply(head)
    dst = cq.Sim(n, sl, eb, chunk_log2=cl)
    ref = cq.Sim(n, sl, eb, chunk_log2=cl)
    g = dst.graph(prog)
    assert g.launch() == len(prog)
    ref.apply(prog)
    recs = src.records()
    assert any(empty_chunks(r) and oracle.parse_header(r)["n_used"] > 1 for r in recs)
    for j, r in enumerate(recs):
        dst.import_record(j, r)
        ref.import_record(j, r)
    assert g.launch() == len(prog)
    ref.apply(prog)
    assert np.array_equal(dst.amplitudes().view(np.float64), ref.amplitudes().view(np.float64))
    assert dst.records() == ref.records()
    g.close()
