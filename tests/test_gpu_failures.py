"""Failure handling of the record arenas on the GPU (through the C ABI).

A pass that overflows its output arena is run again after the arena grows.
When the device memory for that growth cannot be had (here: an allocator hook
that refuses on request), sim_apply must report SIM_ENOMEM with the passes
that completed, leave the state of the last completed pass, and work again
once memory is available.  Each case prints its name before it touches the
GPU."""
import sys

import numpy as np
import pytest

import oracle
import qcircuits as qc

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


class Hooks:
    """Device memory from torch, refused while `refuse` is set."""

    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}
        self.refuse = False
        self.refused = 0

        def _alloc(nbytes, ctx):
            if self.refuse:
                self.refused += 1
                return None
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            self.live.pop(ptr, None)

        self.pair = (cq.ALLOC_FN(_alloc), cq.FREE_FN(_free))


def test_arena_growth_refused_then_granted():
    n, sl, cl, eb = 12, 8, 6, 1e-7
    say("arena growth refused", n, sl, cl, eb)
    hooks = Hooks()
    gates = qc.random_layered(n, 3, seed=9)
    sim = cq.Sim(n, sl, eb, chunk_log2=cl, arena_bytes=8192, allocator=hooks.pair)
    hooks.refuse = True
    rc, applied = sim.apply_partial(gates)
    assert rc == -2, f"expected SIM_ENOMEM, got {rc} after {applied} gates"
    assert hooks.refused > 0 and applied < len(gates)
    orc = oracle.OracleSim(n, sl, cl, eb)
    orc.apply(gates[:applied])
    assert sim.records() == orc.records()
    # nothing can run while memory is refused
    rc2, applied2 = sim.apply_partial(gates[applied:])
    assert rc2 == -2 and applied2 < len(gates) - applied
    orc.apply(gates[applied:applied + applied2])
    assert sim.records() == orc.records()
    hooks.refuse = False
    rest = gates[applied + applied2:]
    assert sim.apply(rest) == len(rest)
    orc.apply(rest)
    assert sim.records() == orc.records()
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())
    sim.close()
