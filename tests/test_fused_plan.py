"""Fused mode on the host: the library's pass partition (sim_plan, host code
that needs no device) against the oracle's own implementation of the same
rule, hand-worked partitions, the oracle's block product against a brute-
force product of Kronecker-embedded gates, and the oracle's fused runs
against exact results."""
import math

import numpy as np
import pytest

import oracle
import paper_1811_05630_amd as cq
import qcircuits as qc
from tests.brute import full_operator, grover_closed_form


def programs():
    yield "qft9", 9, qc.qft(9)
    yield "grover8", 8, qc.grover(8, 77)[:120]
    yield "layers10", 10, qc.random_layered(10, 3, seed=4)
    yield "inverse-qft7", 7, qc.inverse(qc.qft(7))
    zoo = [qc.H(0), qc.U([3, 1], np.eye(4)), qc.MCZ(6), qc.X(5), qc.P(2, 0.3), qc.CP(0, 5, 0.1),
           qc.U([0, 1, 2, 3, 4], np.eye(32)), qc.Z(4), qc.MCPHASE(0, 0, 1j), qc.SWAP(2, 3)]
    yield "zoo6", 6, zoo


@pytest.mark.parametrize("name,n,gates", list(programs()), ids=[p[0] for p in programs()])
def test_library_plan_equals_oracle_plan(name, n, gates):
    assert cq.plan(n, gates) == oracle.plan(gates)


def test_hand_worked_partitions():
    # QFT(3) involves 3 qubits: one fused pass of all 7 gates
    assert oracle.plan(qc.qft(3)) == [(0, 7, True, (0, 1, 2))]
    # a 6-qubit MCZ alone exceeds the width: passes of its own, no fusion across it
    g = [qc.H(0), qc.H(1), qc.MCZ(6), qc.H(2)]
    assert oracle.plan(g) == [(0, 2, True, (0, 1)), (2, 1, False, ()), (3, 1, False, ())]
    # width grows to 5 and the sixth qubit starts a new pass
    g = [qc.H(q) for q in range(7)]
    assert oracle.plan(g) == [(0, 5, True, (0, 1, 2, 3, 4)), (5, 2, True, (5, 6))]
    # controls count as involved qubits
    g = [qc.U([0], np.eye(2), ctrl_mask=0b111110, ctrl_vals=0), qc.H(0)]
    assert oracle.plan(g) == [(0, 1, False, ()), (1, 1, False, ())]
    # global phases involve no qubit
    g = [qc.MCPHASE(0, 0, 1j), qc.MCPHASE(0, 0, -1j)]
    assert oracle.plan(g) == [(0, 2, True, ())]
    assert cq.plan(7, [qc.H(q) for q in range(7)]) == oracle.plan([qc.H(q) for q in range(7)])


def embed(g, qubits):
    """The gate as a matrix over `qubits` (block bit i = qubits[i]), by brute
    force: the full operator on len(qubits) qubits after relabelling."""
    k = len(qubits)
    relabel = {q: i for i, q in enumerate(qubits)}
    h = qc.Gate(g.kind, tuple(relabel[t] for t in g.targets),
                ctrl_mask=sum(1 << relabel[b] for b in range(64) if (g.ctrl_mask >> b) & 1),
                ctrl_vals=sum(1 << relabel[b] for b in range(64) if (g.ctrl_vals >> b) & 1),
                phase=g.phase, matrix=g.matrix)
    return full_operator(h, k)


@pytest.mark.parametrize("name,n,gates", list(programs()), ids=[p[0] for p in programs()])
def test_block_matrix_is_the_product_of_embedded_gates(name, n, gates):
    for first, count, fused, qubits in oracle.plan(gates):
        if not fused:
            continue
        U = oracle.block_matrix(gates, first, count, qubits)
        ref = np.eye(1 << len(qubits), dtype=complex)
        for g in gates[first:first + count]:
            ref = embed(g, qubits) @ ref
        assert np.max(np.abs(U - ref)) < 1e-14


def test_oracle_fused_qft_of_product_state_matches_fft():
    n, sl, cl, rel = 10, 6, 5, 1e-4
    theta, phi = qc.product_angles(n, 7)
    f = qc.product_factors(theta, phi)
    psi0 = oracle.product_state(f)
    exact = math.sqrt(1 << n) * np.fft.ifft(psi0)
    sim = oracle.OracleSim(n, sl, cl, rel, oracle.REL)
    sim.init_product(f)
    assert sim.apply(qc.qft(n), fused=True) == len(qc.qft(n))
    a = sim.amplitudes()
    # REL: per slice eb_j <= rel * range_j <= 2 rel max|a|; unitary passes add
    # at most sqrt(2N) eb per pass to the 2-norm error (first order)
    npass = len(oracle.plan(qc.qft(n)))
    bound = npass * math.sqrt(2 << n) * 2 * rel * np.max(np.abs(exact))
    assert np.linalg.norm(a - exact) < bound
    assert np.linalg.norm(a - exact) < 1e-2


def test_oracle_fused_grover_matches_closed_form():
    n, sl, cl, eb = 8, 5, 4, 1e-7
    w = 77
    gates = qc.grover(n, w)
    k = qc.grover_iterations(n)
    sim = oracle.OracleSim(n, sl, cl, eb)
    sim.apply(gates, fused=True)
    a = sim.amplitudes()
    N = 1 << n
    exact = grover_closed_form(n, w, k)
    npass = len(oracle.plan(gates))
    assert np.linalg.norm(a - exact) < npass * math.sqrt(2 * N) * eb
    assert npass < len(gates) / 2  # fusion shortens the pass list


def test_fused_and_plain_oracle_runs_agree_within_the_bound():
    n, sl, cl, eb = 9, 5, 4, 1e-6
    gates = qc.random_layered(n, 3, seed=9)
    a = oracle.OracleSim(n, sl, cl, eb)
    b = oracle.OracleSim(n, sl, cl, eb)
    a.apply(gates)
    b.apply(gates, fused=True)
    exact = oracle.sv_run(n, gates)
    for sim, npass in ((a, len(gates)), (b, len(oracle.plan(gates)))):
        assert np.linalg.norm(sim.amplitudes() - exact) < npass * math.sqrt(2 << n) * eb


def test_plan_rejects_invalid_gates():
    bad = qc.Gate(qc.DENSE, (0,), matrix=np.eye(2))
    bad.targets = (9,)
    with pytest.raises(cq.SimError) as e:
        cq.plan(8, [qc.H(0), bad])
    assert e.value.rc == -1
