"""Pins for the oracle's optimised passes (mode bit OPT): a gate controlled on
slice-index qubits leaves the slice groups whose index bits fail those
controls untouched, and a SWAP of two slice-index qubits relabels the slices.
Checked against the definition (untouched records byte-equal to the input,
the other records equal to a plain pass of the same gate from the same
records; a relabelled read-out equal, bit for bit, to the permuted read-out
before it) and against Grover's closed form."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from brute import grover_closed_form

OPT = oracle.ABS | oracle.OPT


def slice_bits(gate, sl):
    lo = (1 << sl) - 1
    return (gate.ctrl_mask & ~lo) >> sl, (gate.ctrl_vals & ~lo) >> sl


@pytest.mark.parametrize("gate", [
    qc.MCZ(10),                                                  # phase on the all-ones index
    qc.MCPHASE((1 << 10) - 1, 0b1011001110, -1.0),               # Grover's oracle on a marked index
    qc.U([2], qc.H(2).matrix, ctrl_mask=0b1100000000, ctrl_vals=0b0100000000),
    qc.U([7], qc.H(7).matrix, ctrl_mask=0b1000000001, ctrl_vals=0b1000000001),  # a slice-index target
    qc.CP(3, 9, 0.7),
])
def test_skipped_groups_keep_their_records(gate):
    n, sl, cl, eb = 10, 6, 4, 1e-6
    prep = qc.random_layered(n, 2, seed=3)
    o = oracle.OracleSim(n, sl, cl, eb, OPT)
    o.apply(prep)
    before = o.records()
    o.apply([gate])
    after = o.records()
    # the same gate as a plain pass from the same records
    p = oracle.OracleSim(n, sl, cl, eb, oracle.ABS)
    p.set_records(before)
    p.apply([gate])
    plain = p.records()
    smask, svals = slice_bits(gate, sl)
    skipped = 0
    for j in range(1 << (n - sl)):
        if (j & smask) != svals:
            assert after[j] == before[j], j
            skipped += 1
        else:
            assert after[j] == plain[j], j
    assert skipped > 0


@pytest.mark.parametrize("a,b", [(6, 9), (8, 7), (9, 6)])
def test_slice_index_swap_relabels(a, b):
    n, sl, cl, eb = 10, 6, 4, 1e-6
    o = oracle.OracleSim(n, sl, cl, eb, OPT)
    o.apply(qc.random_layered(n, 2, seed=11))
    before, amp = o.records(), o.amplitudes()
    o.apply([qc.SWAP(a, b)])
    after = o.records()
    sa, sb = a - sl, b - sl
    for j in range(1 << (n - sl)):
        t = j if ((j >> sa) & 1) == ((j >> sb) & 1) else j ^ ((1 << sa) | (1 << sb))
        assert after[t] == before[j]
    i = np.arange(1 << n)
    perm = np.where(((i >> a) & 1) == ((i >> b) & 1), i, i ^ ((1 << a) | (1 << b)))
    got = o.amplitudes()
    assert np.array_equal(got[perm].view(np.float64), amp.view(np.float64))


def test_swap_with_an_in_slice_qubit_is_a_pass():
    n, sl, cl, eb = 10, 6, 4, 1e-6
    o = oracle.OracleSim(n, sl, cl, eb, OPT)
    p = oracle.OracleSim(n, sl, cl, eb, oracle.ABS)
    g = qc.random_layered(n, 1, seed=2) + [qc.SWAP(2, 8), qc.SWAP(7, 9)]
    o.apply(g[:-1])
    p.apply(g[:-1])
    assert o.records() == p.records()  # no slice-index controls, and SWAP(2, 8) is an ordinary pass


def test_grover_with_optimised_passes_is_within_the_first_order_bound():
    n, sl, cl, eb = 12, 8, 5, 1e-7
    w, k = 1234, 3
    gates = qc.grover(n, w, k)
    o = oracle.OracleSim(n, sl, cl, eb, OPT)
    o.apply(gates)
    err = np.linalg.norm(o.amplitudes() - grover_closed_form(n, w, k))
    assert err < len(gates) * math.sqrt(2 << n) * eb


def test_optimised_passes_are_plain_mode_only():
    o = oracle.OracleSim(8, 5, 3, 1e-6, OPT)
    with pytest.raises(oracle.OracleError):
        o.apply(qc.qft(8), fused=True)
    with pytest.raises(oracle.OracleError):
        oracle.CodeSim(8, 5, 1e-6, OPT)
