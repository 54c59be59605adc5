"""Pins for the oracle's uncompressed FP64 gate arithmetic (GateComputation of
Algorithm 1, Section II), checked against brute-force Kronecker operators,
closed forms and numpy's FFT -- never against the oracle itself."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from brute import full_operator, grover_closed_form, qft_basis_closed_form


def rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def rand_unitary(k, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / abs(np.diag(r)))


def gate_zoo(n, seed):
    """Every gate kind at many positions, with and without controls."""
    rng = np.random.default_rng(seed)
    g = []
    for t in range(n):
        g += [qc.H(t), qc.X(t), qc.Z(t), qc.P(t, 0.3 + t), qc.U3(t, 0.1 + t, 0.7, 2.1 - t)]
        g.append(qc.U([t], rand_unitary(1, seed + t)))
    for a in range(n):
        for b in range(n):
            if a != b:
                g += [qc.CP(a, b, 0.5 + a - b), qc.CZ(a, b), qc.SWAP(a, b),
                      qc.U([a, b], rand_unitary(2, 100 * a + b + seed))]
    for k in range(3, min(n, 5) + 1):
        tg = [int(x) for x in rng.permutation(n)[:k]]
        g.append(qc.U(tg, rand_unitary(k, seed + k)))
    # controlled dense gates with both control values
    for t in range(n):
        others = [q for q in range(n) if q != t]
        if not others:
            continue
        m = 0
        for q in others[:2]:
            m |= 1 << q
        vals = m & int(rng.integers(0, 1 << n))
        g.append(qc.U([t], rand_unitary(1, seed + 7 * t), ctrl_mask=m, ctrl_vals=vals))
    full = (1 << n) - 1
    g += [qc.MCZ(n), qc.MCPHASE(full, int(rng.integers(0, 1 << n)), -1.0),
          qc.MCPHASE(full & 0b101, 0b001 & full, complex(math.cos(0.4), math.sin(0.4)))]
    return g


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_every_gate_matches_kron_operator(n):
    for i, g in enumerate(gate_zoo(n, 11 * n)):
        psi = rand_state(n, 1000 * n + i)
        got = oracle.sv_apply(n, psi, g)
        want = full_operator(g, n) @ psi
        assert np.max(np.abs(got - want)) < 1e-13, (n, i, g.name, g.targets)


@pytest.mark.parametrize("n", [3, 5, 6])
def test_slicing_invariance_bit_identical(n):
    """Applying a gate group by group over slices gives the same bits as on the
    whole vector, for every slice size (cross-slice groups included)."""
    gates = gate_zoo(n, 5 * n)
    for slice_log2 in range(1, n + 1):
        L = 1 << slice_log2
        for i, g in enumerate(gates):
            psi = rand_state(n, 77 + i)
            want = oracle.sv_apply(n, psi, g)
            got = psi.copy()
            tbits = 0
            if g.kind == qc.DENSE:
                for t in g.targets:
                    if t >= slice_log2:
                        tbits |= 1 << (t - slice_log2)
            for j0 in range(1 << (n - slice_log2)):
                if j0 & tbits:
                    continue
                mem = oracle.group_members(n, slice_log2, g, j0)
                planes = [psi[j * L:(j + 1) * L] for j in mem]
                out = oracle.group_apply(g, slice_log2, mem, planes)
                for j, o in zip(mem, out):
                    got[j * L:(j + 1) * L] = o
            assert np.array_equal(got, want), (slice_log2, i, g.name)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_qft_of_basis_state_closed_form(n):
    for x in {0, 1, (1 << n) - 1, (5 * n + 3) % (1 << n)}:
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[x] = 1
        got = oracle.sv_run(n, qc.qft(n), psi0)
        assert np.max(np.abs(got - qft_basis_closed_form(n, x))) < 1e-12


@pytest.mark.parametrize("n", [2, 4, 7, 9])
def test_qft_equals_scaled_inverse_fft(n):
    psi = rand_state(n, n)
    got = oracle.sv_run(n, qc.qft(n), psi)
    want = math.sqrt(1 << n) * np.fft.ifft(psi)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (6, 3), (8, 12), (10, 25)])
def test_grover_closed_form(n, k):
    w = (37 * n + 5) % (1 << n)
    psi = oracle.sv_run(n, qc.grover(n, w, k))
    assert np.max(np.abs(psi - grover_closed_form(n, w, k))) < 1e-12


def test_grover_pass_count():
    # n initial H + k * (oracle + 4n diffusion gates + MCZ)
    assert qc.grover_passes(24, qc.grover_iterations(24)) == 315192
    assert len(qc.grover(5, 3)) == qc.grover_passes(5, qc.grover_iterations(5))
    assert qc.grover_iterations(24) == 3216 and qc.grover_iterations(34) == 102943


def test_norm_invariant_and_mirror_circuit():
    n = 6
    g = qc.random_layered(n, 8, seed=3)
    psi = oracle.sv_run(n, g)
    assert abs(np.linalg.norm(psi) - 1) < 1e-14
    back = oracle.sv_run(n, qc.inverse(g), psi)
    e0 = np.zeros(1 << n)
    e0[0] = 1
    assert np.max(np.abs(back - e0)) < 1e-12


def test_product_state_is_kron_of_factors():
    theta, phi = qc.product_angles(5, 1)
    f = qc.product_factors(theta, phi)
    want = np.ones(1, dtype=np.complex128)
    for q in range(4, -1, -1):
        want = np.kron(want, f[q])
    got = oracle.product_state(f)
    assert np.max(np.abs(got - want)) < 1e-15
    assert abs(np.linalg.norm(got) - 1) < 1e-14


@pytest.mark.parametrize("n,m", [(6, 2), (10, 4), (11, 11)])
def test_qft_product_closed_form_blocks(n, m):
    """The block-wise closed form used for the 30-qubit check equals sqrt(N)
    ifft of the Kronecker product state and the oracle's run of the QFT."""
    from brute import QftProductExact
    theta, phi = qc.product_angles(n, 2)
    f = qc.product_factors(theta, phi)
    psi = np.ones(1, dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        psi = np.kron(psi, f[q])
    want = math.sqrt(1 << n) * np.fft.ifft(psi)
    ex = QftProductExact(f, m)
    got = np.concatenate([ex.block(h) for h in range(1 << (n - m))])
    assert np.max(np.abs(got - want)) < 1e-13
    assert np.max(np.abs(got - oracle.sv_run(n, qc.qft(n), psi))) < 1e-12
