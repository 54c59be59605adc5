"""The oracle's code-level runner (oracle.CodeSim) against the full oracle.

CodeSim follows Algorithm 1 on the quantised codes only, eliding the codec's
lossless stages; it must give exactly the full simulator's codes, steps,
amplitudes and largest codec error after every checked pass, in plain and
fused mode, both bounds and both precisions.  Its gate routine (local
addressing of a group's members) must equal the oracle's gate routine bit for
bit."""
import numpy as np
import pytest

import oracle
import qcircuits as qc


def unitary(k, seed):
    r = np.random.default_rng(seed)
    a = r.standard_normal((1 << k, 1 << k)) + 1j * r.standard_normal((1 << k, 1 << k))
    return np.linalg.qr(a)[0]


def same(full, codes, label):
    assert np.array_equal(full.amplitudes().view(np.float64), codes.amplitudes().view(np.float64)), label
    st = codes.state()
    for j in range(full.nslices):
        rec = full.record(j)
        assert np.array_equal(oracle.decode_p(rec), st["codes"][j].astype(np.int64)), f"{label}: slice {j}"
        h = oracle.parse_header(rec)
        assert h["step"] == st["step"][j] and h["sumsq"] == (int(st["hi"][j]) << 64) | int(st["lo"][j])
    assert full.max_err() == codes.max_err()


CASES = [  # n, slice_log2, eb, mode
    (9, 4, 1e-6, oracle.ABS), (9, 9, 1e-6, oracle.ABS), (10, 3, 1e-5, oracle.ABS | oracle.FP32),
    (10, 6, 1e-3, oracle.REL), (9, 5, 1e-3, oracle.REL | oracle.FP32),
]


@pytest.mark.parametrize("n,sl,eb,mode", CASES)
def test_plain_mode_equals_full_oracle(n, sl, eb, mode):
    f = qc.product_factors(*qc.product_angles(n, n))
    gates = (qc.random_layered(n, 2, seed=n) + qc.qft(n)[: 3 * n] +
             [qc.U([0, n - 1], unitary(2, 1)), qc.U([1, n - 2, 2], unitary(3, 2), ctrl_mask=1 << 5, ctrl_vals=0),
              qc.MCPHASE(0b101 << (n - 3), 0b100 << (n - 3), 1j), qc.SWAP(0, n - 1)])
    a = oracle.OracleSim(n, sl, min(sl, 5), eb, mode)
    b = oracle.CodeSim(n, sl, eb, mode)
    a.init_product(f)
    b.init_product(f)
    same(a, b, "initial state")
    for i in range(0, len(gates), 7):
        a.apply(gates[i:i + 7])
        b.apply(gates[i:i + 7])
        same(a, b, f"after gate {i + 7}")


def test_fused_mode_and_basis_state():
    n, sl, eb = 10, 5, 1e-7
    gates = qc.qft(n) + qc.grover(n, 700, iterations=1)
    a = oracle.OracleSim(n, sl, 4, eb)
    b = oracle.CodeSim(n, sl, eb)
    a.init_basis(321)
    b.init_basis(321)
    assert a.apply(gates, fused=True) == b.apply(gates, fused=True) == len(gates)
    same(a, b, "fused")


def test_grover_full_run_small():
    n, sl, eb = 12, 6, 1e-7
    w = qc.grover_workload(n=n, slice_log2=sl, eb=eb, seed=4)
    a = oracle.OracleSim(n, sl, 8, eb)
    b = oracle.CodeSim(n, sl, eb)
    a.apply(w.gates)
    b.apply(w.gates)
    same(a, b, "grover12")


def test_checkpoint_resume_is_seamless():
    n, sl, eb = 10, 4, 1e-6
    gates = qc.random_layered(n, 3, seed=8)
    a = oracle.CodeSim(n, sl, eb)
    a.apply(gates)
    b = oracle.CodeSim(n, sl, eb)
    b.apply(gates[:17])
    c = oracle.CodeSim(n, sl, eb)
    c.set_state(b.state())
    c.apply(gates[17:])
    assert np.array_equal(a.amplitudes(), c.amplitudes())
    assert c.passes == len(gates)


def test_codes_beyond_int32_are_refused():
    with pytest.raises(oracle.OracleError) as e:
        oracle.CodeSim(4, 2, 1e-11)  # the code of |0...0>, 1 / (2e-11), is above 2^31
    assert e.value.rc == -3
    b = oracle.CodeSim(4, 2, 4e-10)  # 1 / (8e-10) < 2^31: fits
    b.apply([qc.H(0), qc.H(1)])


@pytest.mark.parametrize("fp32", [False, True])
def test_local_addressing_equals_the_gate_routine(fp32):
    rng = np.random.default_rng(3)
    sl = 4
    for trial in range(12):
        k = int(rng.integers(1, 6))
        qs = [int(x) for x in rng.choice(8, size=k, replace=False)]
        rest = [q for q in range(8) if q not in qs]
        cm = 0
        if rest and trial % 2:
            cm = 1 << int(rng.choice(rest))
        g = qc.U(qs, unitary(k, trial), ctrl_mask=cm, ctrl_vals=cm if trial % 4 == 1 else 0)
        members = oracle.group_members(8, sl, g, 0)
        planes = [rng.standard_normal(1 << sl) + 1j * rng.standard_normal(1 << sl) for _ in members]
        if fp32:
            planes = [p.real.astype(np.float32) + 1j * p.imag.astype(np.float32) for p in planes]
        want = oracle.group_apply(g, sl, members, planes) if not fp32 else None
        got = oracle.group_apply_local(g, sl, members, planes, fp32=fp32)
        if not fp32:
            for w, x in zip(want, got):
                assert np.array_equal(w.view(np.float64), x.view(np.float64))
        else:  # FP32: against the oracle's FP32 state-vector gate on the assembled group
            full = np.zeros(1 << 8, dtype=complex)
            for u, j in enumerate(members):
                full[j << sl:(j + 1) << sl] = planes[u]
            ref = oracle.sv_apply(8, full, g, oracle.FP32)
            for u, j in enumerate(members):
                assert np.array_equal(ref[j << sl:(j + 1) << sl].view(np.float64), got[u].view(np.float64))
