"""Captured gate programs (sim_graph_*): every replay gives the records the
same program gives through sim_apply, byte for byte, with eager work and
synchronisation between replays, from both arena parities, across arena
growth, in plain and fused mode.  Each case prints its name before it
touches the GPU."""
import numpy as np
import pytest

import oracle
import qcircuits as qc
from tests.test_gpu_parity import assert_same_records, say

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def same(a, b, label):
    ra, rb = a.records(), b.records()
    for j, (x, y) in enumerate(zip(ra, rb)):
        if x != y:
            pytest.fail(f"{label}: slice {j} differs")


def test_graph_replays_match_eager_with_work_between():
    n, sl, cl, eb = 12, 8, 6, 1e-7
    say("graph replays", n, sl, cl, eb)
    it = qc.grover(n, 1234, 1)[n:]  # one Grover iteration (after the H layer)
    assert len(it) % 2 == 0
    g_sim = cq.Sim(n, sl, eb, chunk_log2=cl)
    e_sim = cq.Sim(n, sl, eb, chunk_log2=cl)
    orc = oracle.OracleSim(n, sl, cl, eb)
    head = qc.grover(n, 1234, 0)  # the H layer
    for s in (g_sim, e_sim):
        s.apply(head)
    orc.apply(head)
    graph = g_sim.graph(it)
    for rep in range(3):
        assert graph.launch() == len(it)
        e_sim.apply(it)
        orc.apply(it)
        same(g_sim, e_sim, f"replay {rep}")
        assert_same_records(g_sim, orc, f"replay {rep} vs oracle")
        extra = [qc.P(3, 0.1 * rep), qc.H(5)]  # eager work between replays (even: same parity)
        g_sim.apply(extra)
        e_sim.apply(extra)
        orc.apply(extra)
    # an odd number of eager passes: the next replay starts from the other parity
    g_sim.apply([qc.X(2)])
    e_sim.apply([qc.X(2)])
    assert graph.launch() == len(it)
    e_sim.apply(it)
    same(g_sim, e_sim, "other parity")
    graph.close()
    assert np.array_equal(g_sim.amplitudes(), e_sim.amplitudes())


def test_graph_with_odd_pass_count():
    n, sl, cl, eb = 10, 6, 5, 1e-6
    say("graph odd", n, sl, cl, eb)
    prog = qc.qft(n)
    if len(prog) % 2 == 0:
        prog = prog + [qc.H(0)]
    a = cq.Sim(n, sl, eb, chunk_log2=cl)
    b = cq.Sim(n, sl, eb, chunk_log2=cl)
    a.init_basis(77)
    b.init_basis(77)
    graph = a.graph(prog)
    for rep in range(3):  # parities alternate: captured, other, captured
        assert graph.launch() == len(prog)
        b.apply(prog)
        same(a, b, f"odd replay {rep}")


def test_graph_survives_arena_growth():
    n, sl, cl, eb = 12, 7, 6, 1e-7
    say("graph growth", n, sl, cl, eb)
    prog = qc.random_layered(n, 2, seed=3)
    if len(prog) % 2:
        prog = prog + [qc.Z(0)]
    a = cq.Sim(n, sl, eb, chunk_log2=cl, arena_bytes=4096)
    orc = oracle.OracleSim(n, sl, cl, eb)
    graph = a.graph(prog)  # captured on arenas the records will outgrow
    for rep in range(2):
        assert graph.launch() == len(prog)
        orc.apply(prog)
        assert_same_records(a, orc, f"growth replay {rep}")
    assert a.stats()["arena_bytes"] > 2 * 4096


def test_graph_fused_mode():
    n, sl, cl, eb = 11, 8, 6, 1e-7
    say("graph fused", n, sl, cl, eb)
    prog = qc.qft(n)
    a = cq.Sim(n, sl, eb, chunk_log2=cl, fused=True)
    b = cq.Sim(n, sl, eb, chunk_log2=cl, fused=True)
    a.init_basis(5)
    b.init_basis(5)
    graph = a.graph(prog)
    for rep in range(2):
        assert graph.launch() == len(prog)
        b.apply(prog)
        same(a, b, f"fused replay {rep}")


def test_graph_rejects_invalid_program():
    say("graph invalid")
    a = cq.Sim(6, 3, 1e-6)
    with pytest.raises(cq.SimError) as e:
        a.graph([qc.H(0), qc.H(9)])
    assert e.value.rc == -1
    a.close()
