"""The C ABI's named gate kinds, statistics and plan on a handle (GPU).

Named kinds (H, X, Z, P, CP, CZ, SWAP, U3, MCZ, U1Q) are expanded by the
library on the host; a program of them must give records byte-identical to
the same program written as DENSE and PHASE gates with the matrices and
phases of qcircuits (and so to the oracle, which is fed those).  Each case
prints its name before it touches the GPU."""
import math
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


def programs(n, seed):
    rng = np.random.default_rng(seed)
    named, plain = [], []
    for q in range(n):
        th, ph, la = (float(x) for x in rng.uniform(0, 2 * math.pi, 3))
        named += [cq.Named(cq.GATE_H, (q,)), cq.Named(cq.GATE_U3, (q,), (th, ph, la)),
                  cq.Named(cq.GATE_P, (q,), (th,)), cq.Named(cq.GATE_Z, ((q + 1) % n,))]
        plain += [qc.H(q), qc.U3(q, th, ph, la), qc.P(q, th), qc.Z((q + 1) % n)]
    for a, b in [(0, n - 1), (1, n // 2), (n - 2, 2)]:
        th = float(rng.uniform(0, math.pi))
        named += [cq.Named(cq.GATE_CP, (a, b), (th,)), cq.Named(cq.GATE_CZ, (b, a)), cq.Named(cq.GATE_SWAP, (a, b)),
                  cq.Named(cq.GATE_X, (b,), ctrl_mask=1 << a, ctrl_vals=1 << a)]
        plain += [qc.CP(a, b, th), qc.CZ(b, a), qc.SWAP(a, b),
                  qc.Gate(qc.DENSE, (b,), ctrl_mask=1 << a, ctrl_vals=1 << a, matrix=qc.X(b).matrix)]
    m = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))[0]
    named += [cq.Named(cq.GATE_U1Q, (n - 1,), matrix=m), cq.Named(cq.GATE_MCZ, (0, 2, 3, n - 1))]
    plain += [qc.U([n - 1], m), qc.MCPHASE(1 | 4 | 8 | (1 << (n - 1)), 1 | 4 | 8 | (1 << (n - 1)), -1)]
    return named, plain


@pytest.mark.parametrize("n,sl,cl,fused", [(10, 6, 5, False), (12, 10, 8, False), (11, 7, 6, True)])
def test_named_kinds_equal_dense_and_phase(n, sl, cl, fused):
    say("named kinds", n, sl, cl, "fused" if fused else "plain")
    named, plain = programs(n, n)
    a = cq.Sim(n, sl, 1e-7, chunk_log2=cl, fused=fused)
    b = cq.Sim(n, sl, 1e-7, chunk_log2=cl, fused=fused)
    assert a.apply(named) == len(named)
    assert b.apply(plain) == len(plain)
    assert a.records() == b.records()
    assert np.array_equal(a.amplitudes(), b.amplitudes())
    assert cq.plan(a, named) == cq.plan(n, plain)
    if not fused:
        orc = oracle.OracleSim(n, sl, cl, 1e-7)
        orc.apply(plain)
        assert a.records() == orc.records()


def test_stats_gates_and_slice_ratio():
    n, sl, cl = 12, 8, 6
    say("stats fields", n, sl, cl)
    s = cq.Sim(n, sl, 1e-6, chunk_log2=cl, fused=True)
    gates = qc.qft(n)
    s.apply(gates)
    st = s.stats()
    assert st["gates"] == len(gates)
    assert st["passes"] == len(cq.plan(n, gates)) < len(gates)
    lens = [len(r) for r in s.records()]
    assert st["min_slice_ratio"] == (16 << sl) / max(lens)
    assert st["min_slice_ratio"] <= st["ratio"]


def test_named_kind_errors():
    s = cq.Sim(6, 3, 1e-6)
    say("named kind errors")
    for bad in (cq.Named(cq.GATE_CZ, (1,)), cq.Named(cq.GATE_H, (1, 2)), cq.Named(99, (0,)),
                cq.Named(cq.GATE_Z, (2,), ctrl_mask=4, ctrl_vals=4), cq.Named(cq.GATE_U1Q, (0,))):
        rc, applied = s.apply_partial([qc.H(0), bad, qc.H(1)])
        assert rc == -1 and applied == 1
