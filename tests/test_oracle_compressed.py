"""Pins for the oracle's whole compressed simulation (Algorithm 1, Section II):
decompress, normalise, gate, compress for every gate and every slice.

The exact state is known in closed form (QFT of a basis state, Grover) or by
numpy's FFT; the lossy run must stay within the error the bound allows.  Per
pass the quantiser moves the state by at most sqrt(2N)*eb in 2-norm; unitary
gates keep that distance; renormalising y with |y - psi| = e <= 1/2 onto the
unit sphere gives a distance of at most e/(1-e).  The recursion below turns
that into a guaranteed bound per run."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from brute import grover_closed_form, qft_basis_closed_form


def guaranteed_bound(n, passes, eb):
    q = math.sqrt(2 * (1 << n)) * eb
    e = q  # initial compression
    for _ in range(passes):
        e = (e + q) / (1 - (e + q))  # renormalise, gate, quantise
    return e / (1 - e)  # the final read-out is normalised too


def test_qft12_basis_state_within_guaranteed_bound():
    w = qc.qft_basis_workload()
    s = oracle.OracleSim(w.n_qubits, w.slice_log2, 10, w.error_bound)
    s.init_basis(w.basis)
    assert s.apply(w.gates) == len(w.gates) == 84
    a = s.amplitudes()
    err = np.linalg.norm(a - qft_basis_closed_form(w.n_qubits, w.basis))
    bound = guaranteed_bound(w.n_qubits, len(w.gates), w.error_bound)
    assert bound < 1.6e-2
    assert err <= bound
    assert err < 1e-3  # measured ~7e-5; far inside the bound
    assert s.max_err() <= w.error_bound
    fid = abs(np.vdot(qft_basis_closed_form(w.n_qubits, w.basis), a)) ** 2
    assert fid > 0.9999


@pytest.mark.parametrize("n,slice_log2,k", [(8, 5, 4), (10, 6, 3)])
def test_small_grover_within_guaranteed_bound(n, slice_log2, k):
    marked = (29 * n + 3) % (1 << n)
    eb = 1e-7
    gates = qc.grover(n, marked, k)
    s = oracle.OracleSim(n, slice_log2, 6, eb)
    s.apply(gates)
    a = s.amplitudes()
    err = np.linalg.norm(a - grover_closed_form(n, marked, k))
    assert err <= guaranteed_bound(n, len(gates), eb)


def test_qft_of_product_state_rel_bound_matches_fft():
    n, slice_log2, rel = 10, 6, 1e-4
    theta, phi = qc.product_angles(n, 2)
    f = qc.product_factors(theta, phi)
    s = oracle.OracleSim(n, slice_log2, 5, rel, oracle.REL)
    s.init_product(f)
    s.apply(qc.qft(n))
    a = s.amplitudes()
    psi0 = oracle.product_state(f)
    want = math.sqrt(1 << n) * np.fft.ifft(psi0)
    # REL bound: eb_j <= rel * (range of the slice) <= 2 rel max|a|
    assert np.linalg.norm(a - want) < 0.05
    assert abs(np.vdot(want, a)) ** 2 > 0.99


def test_initial_product_state_is_quantised_within_bound():
    n, slice_log2, rel = 8, 5, 1e-5
    theta, phi = qc.product_angles(n, 4)
    f = qc.product_factors(theta, phi)
    s = oracle.OracleSim(n, slice_log2, 5, rel, oracle.REL)
    s.init_product(f)
    psi0 = oracle.product_state(f)
    L = 1 << slice_log2
    for j, rec in enumerate(s.records()):
        h = oracle.parse_header(rec)
        v = np.concatenate([psi0[j * L:(j + 1) * L].real, psi0[j * L:(j + 1) * L].imag])
        step, _, ebj = oracle.rel_step(rel, v)
        assert h["step"] == step
        p = oracle.decode_p(rec)
        assert np.all(np.abs(v - p * step) <= ebj)


def test_normalised_readout_has_unit_norm():
    w = qc.qft_basis_workload()
    s = oracle.OracleSim(w.n_qubits, w.slice_log2, 10, w.error_bound)
    s.init_basis(w.basis)
    s.apply(w.gates[:30])
    assert abs(np.linalg.norm(s.amplitudes()) - 1) < 1e-14


def test_deterministic_across_thread_counts():
    n, sl = 12, 8
    g = qc.random_layered(n, 3, seed=9)
    recs = []
    for t in (1, 4):
        oracle.set_threads(t)
        s = oracle.OracleSim(n, sl, 7, 1e-6)
        s.apply(g)
        recs.append(s.records())
    oracle.set_threads(0)
    assert recs[0] == recs[1]


def test_pass_group_reproduces_simulator_pass():
    """Recomputing one group from the stored records gives the same bytes as
    the simulator's own pass (the entry used to check large states slice by slice)."""
    n, sl, cl, eb = 10, 6, 6, 1e-6
    s = oracle.OracleSim(n, sl, cl, eb)
    s.apply(qc.grover(n, 77, 1)[:15])
    before = s.records()
    scale = oracle.scale_from_records(before)
    assert scale == s.scale()
    for g in [qc.H(2), qc.H(8), qc.SWAP(1, 9), qc.MCZ(n), qc.U([7, 9, 3], np.eye(8))]:
        s2 = oracle.OracleSim(n, sl, cl, eb)
        s2.apply(qc.grover(n, 77, 1)[:15])
        s2.apply([g])
        after = s2.records()
        for j0 in (0, 3, 5):
            mem = oracle.group_members(n, sl, g, j0 & ~sum(1 << (t - sl) for t in g.targets if t >= sl))
            out = oracle.pass_group(n, sl, cl, eb, oracle.ABS, g, scale, mem, [before[j] for j in mem])
            for j, r in zip(mem, out):
                assert r == after[j]


def test_failed_pass_leaves_state_unchanged():
    n, sl = 6, 3
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleSim(n, sl, 3, 1e-15)  # |p| of the amplitude 1 is 5e14 >= 2^48
    assert e.value.rc == -3
    s = oracle.OracleSim(n, sl, 3, 1e-6)
    s.apply([qc.H(0), qc.H(4)])
    ref = s.records()
    s2 = oracle.OracleSim(n, sl, 3, 1e-6)
    bad = qc.Gate(qc.DENSE, (0,), matrix=np.eye(2))
    bad.targets = (7,)  # beyond the register: refused when its pass starts
    with pytest.raises(oracle.OracleError) as e:
        s2.apply([qc.H(0), qc.H(4), bad, qc.H(1)])
    assert e.value.rc == -1
    assert s2.records() == ref


def test_compression_ratio_and_peak_tracking():
    w = qc.qft_basis_workload()
    s = oracle.OracleSim(w.n_qubits, w.slice_log2, 10, w.error_bound)
    s.init_basis(w.basis)
    raw = 16 << w.n_qubits
    s.apply(w.gates)
    assert s.peak_bytes() >= s.total_bytes()
    assert raw / s.peak_bytes() > 1.5
