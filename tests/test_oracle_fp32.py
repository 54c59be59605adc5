"""Pins for the oracle's FP32 mode (amplitudes, matrix entries, initial
factors and every product and sum of the gate arithmetic in FP32; the
quantiser, its bound check and the norm in FP64).  The gate arithmetic is
checked bit for bit against numpy float32 scalar arithmetic in the operation
order of the complex multiply-add; compressed runs against closed forms and
the FFT within bounds that add the FP32 rounding to the codec's."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from brute import grover_closed_form, qft_basis_closed_form

F = np.float32


def f32_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    return v.real.astype(F), v.imag.astype(F)


def rand_unitary(k, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / abs(np.diag(r)))


def float32_gate(n, re, im, g):
    """The gate on an FP32 state in numpy float32 scalar arithmetic: every
    output is sum_c U[r][c] * a[c] in ascending c, each complex product as
    (ur*ar - ui*ai, ur*ai + ui*ar), added to the running sum."""
    re, im = re.copy(), im.copy()
    if g.kind == qc.PHASE:
        pr, pi = F(g.phase.real), F(g.phase.imag)
        for i in range(1 << n):
            if (i & g.ctrl_mask) == g.ctrl_vals:
                ar, ai = re[i], im[i]
                re[i] = F(0) + (pr * ar - pi * ai)
                im[i] = F(0) + (pr * ai + pi * ar)
        return re, im
    k = len(g.targets)
    dim = 1 << k
    tmask = sum(1 << t for t in g.targets)
    U = g.matrix
    out_r, out_i = re.copy(), im.copy()
    for base in range(1 << n):
        if base & tmask or (base & g.ctrl_mask) != g.ctrl_vals:
            continue
        idx = []
        for m in range(dim):
            gi = base
            for t in range(k):
                if (m >> t) & 1:
                    gi |= 1 << g.targets[t]
            idx.append(gi)
        for r in range(dim):
            cr, ci = F(0), F(0)
            for c in range(dim):
                ur, ui = F(U[r, c].real), F(U[r, c].imag)
                ar, ai = re[idx[c]], im[idx[c]]
                cr = cr + (ur * ar - ui * ai)
                ci = ci + (ur * ai + ui * ar)
            out_r[idx[r]], out_i[idx[r]] = cr, ci
    return out_r, out_i


def gates_for(n, seed):
    g = [qc.H(0), qc.U3(n - 1, 0.3, 1.1, 0.2), qc.U([1], rand_unitary(1, seed)),
         qc.U([0, n - 1], rand_unitary(2, seed + 1)), qc.U([2, 0, 3], rand_unitary(3, seed + 2)),
         qc.CP(1, 2, 0.7), qc.P(3, -0.4), qc.MCZ(n),
         qc.U([2], rand_unitary(1, seed + 3), ctrl_mask=0b1001, ctrl_vals=0b0001)]
    return g


@pytest.mark.parametrize("seed", [1, 2])
def test_fp32_gate_arithmetic_is_float32(seed):
    n = 4
    re, im = f32_state(n, seed)
    for g in gates_for(n, 10 * seed):
        want_r, want_i = float32_gate(n, re, im, g)
        got = oracle.sv_apply(n, re.astype(np.float64) + 1j * im.astype(np.float64), g, oracle.FP32)
        assert np.array_equal(got.real, want_r.astype(np.float64)), g.name
        assert np.array_equal(got.imag, want_i.astype(np.float64)), g.name
        # and it differs from the FP64 arithmetic somewhere (the rounding is not a no-op)
        re, im = want_r, want_i
    f64 = oracle.sv_apply(n, re.astype(np.float64) + 1j * im.astype(np.float64), qc.H(1))
    f32 = oracle.sv_apply(n, re.astype(np.float64) + 1j * im.astype(np.float64), qc.H(1), oracle.FP32)
    assert not np.array_equal(f64, f32)


def fp32_bound(n, passes, eb):
    """FP64 codec bound per pass (quantisation, sqrt(2N) eb in norm) plus the
    FP32 rounding of one pass: the decoded values (2^-24 relative) and a gate
    output of at most 32 terms (each product and partial sum rounded:
    at most 2 * 33 * 2^-24 relative in norm, as the gate is unitary)."""
    q = math.sqrt(2 * (1 << n)) * eb + 70 * 2.0 ** -24
    e = q
    for _ in range(passes):
        e = (e + q) / (1 - (e + q))
    return e / (1 - e)


def test_fp32_qft_basis_within_bound_and_fp32_valued():
    w = qc.qft_basis_workload()
    s = oracle.OracleSim(w.n_qubits, w.slice_log2, 10, w.error_bound, oracle.FP32)
    s.init_basis(w.basis)
    assert s.apply(w.gates) == len(w.gates)
    a = s.amplitudes()
    assert np.array_equal(a.real, a.real.astype(F).astype(np.float64))
    assert np.array_equal(a.imag, a.imag.astype(F).astype(np.float64))
    want = qft_basis_closed_form(w.n_qubits, w.basis)
    assert np.linalg.norm(a - want) <= fp32_bound(w.n_qubits, len(w.gates), w.error_bound)
    s64 = oracle.OracleSim(w.n_qubits, w.slice_log2, 10, w.error_bound)
    s64.init_basis(w.basis)
    s64.apply(w.gates)
    assert not np.array_equal(s64.amplitudes(), a)  # the two modes do differ
    assert s.max_err() <= w.error_bound


def test_fp32_grover_within_bound():
    n, sl, k, eb = 8, 5, 4, 1e-7
    marked = 77
    gates = qc.grover(n, marked, k)
    s = oracle.OracleSim(n, sl, 6, eb, oracle.FP32)
    s.apply(gates)
    err = np.linalg.norm(s.amplitudes() - grover_closed_form(n, marked, k))
    assert err <= fp32_bound(n, len(gates), eb)


def test_fp32_rel_product_qft_matches_fft():
    n, sl, rel = 10, 6, 1e-4
    theta, phi = qc.product_angles(n, 3)
    f = qc.product_factors(theta, phi)
    s = oracle.OracleSim(n, sl, 5, rel, oracle.REL | oracle.FP32)
    s.init_product(f)
    s.apply(qc.qft(n))
    a = s.amplitudes()
    want = math.sqrt(1 << n) * np.fft.ifft(oracle.product_state(f))
    assert np.linalg.norm(a - want) < 0.05
    assert abs(np.vdot(want, a)) ** 2 > 0.99


def test_fp32_initial_product_uses_fp32_factors():
    """The product state is the FP32 MAC chain over FP32-rounded factors."""
    n = 3
    theta, phi = qc.product_angles(n, 5)
    f = qc.product_factors(theta, phi)
    s = oracle.OracleSim(n, 2, 2, 1e-9, oracle.FP32)
    s.init_product(f)
    got = s.amplitudes()
    ff = np.asarray(f, dtype=np.complex128).reshape(n, 2)
    want = []
    for i in range(1 << n):
        ar, ai = F(1), F(0)
        for q in range(n):
            b = (i >> q) & 1
            ur, ui = F(ff[q, b].real), F(ff[q, b].imag)
            ar, ai = F(0) + (ur * ar - ui * ai), F(0) + (ur * ai + ui * ar)
        want.append(complex(ar, ai))
    want = np.array(want)
    # stored within 1e-9 of those values, then normalised (norm within 1e-8 of 1)
    assert np.max(np.abs(got - want / np.linalg.norm(want))) < 1e-7
