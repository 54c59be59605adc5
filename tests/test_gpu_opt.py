"""GPU parity of optimised passes (SIM_OPT): byte-equal records to the
oracle's optimised passes after every checked pass -- groups where a gate's
slice-index controls fail carried over unchanged, SWAPs of two slice-index
qubits relabelling the slices -- with other modes, several batches, arena
growth and captured graphs; the refusals.  Each case prints its name before it
touches the GPU."""
import numpy as np
import pytest

import oracle
import qcircuits as qc
from test_gpu_parity import run_both, say

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def opt_program(n, sl, seed):
    """Gates with controls on slice-index qubits, slice-index targets and
    index SWAPs, between ordinary layers."""
    rng = np.random.default_rng(seed)
    hi = list(range(sl, n))
    g = qc.random_layered(n, 1, seed=seed)
    for _ in range(3):
        a, b = (int(x) for x in rng.choice(hi, 2, replace=False))
        t = int(rng.integers(0, sl))
        g += [qc.SWAP(a, b),
              qc.U([t], qc.H(t).matrix, ctrl_mask=1 << a, ctrl_vals=1 << a),
              qc.CP(t, b, 0.3 + a),
              qc.U([a], qc.H(a).matrix, ctrl_mask=(1 << b) | 1, ctrl_vals=1 << b),
              qc.MCPHASE((1 << n) - 1, int(rng.integers(0, 1 << n)), -1.0),
              qc.SWAP(t, a)]  # an in-slice qubit: an ordinary pass
    return g + qc.random_layered(n, 1, seed=seed + 1)


@pytest.mark.parametrize("n,sl,cl", [(10, 6, 4), (12, 8, 5), (11, 5, 3)])
def test_opt_program_matches_the_oracle(n, sl, cl):
    say(f"opt: program n={n} sl={sl} cl={cl}")
    sim, orc = run_both(n, sl, cl, 1e-6, opt_program(n, sl, n), opt=True)
    assert np.array_equal(sim.amplitudes().view(np.float64), orc.amplitudes().view(np.float64))
    assert sim.stats()["compressed_bytes"] == orc.total_bytes()


def test_opt_grover():
    n, sl, cl = 12, 7, 5
    say("opt: grover")
    run_both(n, sl, cl, 1e-7, qc.grover(n, 2024, 2), opt=True, check_every=3)


def test_opt_with_other_modes():
    n, sl, cl = 11, 7, 4
    g = opt_program(n, sl, 5)
    say("opt: FP32")
    run_both(n, sl, cl, 1e-6, g, opt=True, fp32=True, check_every=2)
    say("opt: relative bound")
    run_both(n, sl, cl, 1e-4, g, opt=True, rel=True, check_every=2)
    say("opt: zero chunks, constant chunks, chunk runs")
    run_both(n, sl, cl, 1e-6, g, opt=True, zero_chunks=True, const_chunks=True, chunk_runs=True, check_every=2)


def test_opt_batches_and_arena_growth():
    n, sl, cl = 13, 7, 5
    say("opt: several batches, arena growth")
    run_both(n, sl, cl, 1e-6, opt_program(n, sl, 9), opt=True, check_every=4, workspace_bytes=1_200_000,
             arena_bytes=4096)


def test_opt_graph_and_refusals():
    n, sl, cl = 10, 6, 4
    g = opt_program(n, sl, 3)
    say("opt: captured graph")
    a = cq.Sim(n, sl, 1e-6, chunk_log2=cl, opt=True)
    b = cq.Sim(n, sl, 1e-6, chunk_log2=cl, opt=True)
    cq.Graph(a, g).launch()
    b.apply(g)
    assert a.records() == b.records()
    say("opt: refusals")
    assert b.apply_noalloc(g[:2])[0] == -1
    with pytest.raises(cq.SimError) as e:
        cq.Sim(n, sl, 1e-6, chunk_log2=cl, opt=True, fused=True)
    assert e.value.rc == -1
