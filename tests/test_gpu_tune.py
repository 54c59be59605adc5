"""GPU test of the chunk-length autotuner (sim_tune_chunk): it returns the
fastest candidate of its own table, and each candidate's record total is
what a handle of that chunk length reaches on the same program."""
import sys

import pytest

import qcircuits as qc

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_tuner_picks_the_fastest_of_its_table():
    n, sl, eb = 14, 11, 1e-6
    gates = cq.Circuit(qc.grover(n, 4321, 1))
    say("tune: grover n=14, chunks 2^5..2^9")
    best, table = cq.tune_chunk(n, sl, eb, gates, lo=5, hi=9)
    assert sorted(table) == [5, 6, 7, 8, 9]
    assert all(ms > 0 and b > 0 for ms, b in table.values())
    fastest = min(table, key=lambda c: (table[c][0], table[c][1]))
    assert best == fastest
    for cl in (5, best):
        s = cq.Sim(n, sl, eb, chunk_log2=cl)
        s.apply(gates)
        assert s.stats()["compressed_bytes"] == table[cl][1]
        s.close()


def test_tuner_refuses_bad_ranges():
    gates = [qc.H(0), qc.H(1)]
    with pytest.raises(cq.SimError) as e:
        cq.tune_chunk(6, 4, 1e-6, gates, lo=8, hi=5)
    assert e.value.rc == -1
    with pytest.raises(cq.SimError) as e:
        cq.tune_chunk(6, 4, 1e-6, gates[:1], lo=3, hi=4)
    assert e.value.rc == -1
