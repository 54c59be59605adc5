"""Pins of the oracle's pointwise-relative mode (ORC_PWREL): every value v is
stored as the nearest FP64 number with b mantissa bits, b the least integer
with 2^-(b+1) <= eb, so |v - v'| <= eb |v| and zeros stay zero.

The rounding is checked against an independent construction (frexp, an
integer mantissa rounded half to even by numpy, ldexp), the code against its
definition (the rounded bit pattern shifted right by 52 - b, signed), the
norm field against the pairwise tree and math.fsum, and whole runs against
exact results within the first-order bound."""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc


def bits_for(eb):
    b = 0
    while 2.0 ** -(b + 1) > eb:
        b += 1
    return b


def nearest_with_bits(v, b):
    """Round-to-nearest-even of v to b mantissa bits (after the leading one)."""
    out = np.zeros_like(v)
    for i, x in enumerate(v):
        if x == 0.0:
            continue
        m, e = math.frexp(abs(x))  # |x| = m 2^e, m in [0.5, 1)
        k = np.rint(m * 2.0 ** (b + 1))  # integer mantissa with b + 1 bits, half to even
        out[i] = math.copysign(math.ldexp(float(k), e - b - 1), x)
    return out


@pytest.mark.parametrize("eb,b", [(0.01, 6), (2.0 ** -7, 6), (0.3, 1), (1e-4, 13), (2.0 ** -21, 20)])
def test_bits_from_the_bound(eb, b):
    assert bits_for(eb) == b
    L = 8
    v = np.linspace(0.1, 0.9, 2 * L)
    rec, st = oracle.compress_slice(v[:L], v[L:], 3, 3, eb, oracle.PWREL)
    assert oracle.parse_header(rec)["pw_bits"] == b and oracle.parse_header(rec)["flags"] & 4


def test_values_are_the_nearest_with_b_bits():
    rng = np.random.default_rng(1)
    L = 1 << 10
    eb = 0.01
    b = bits_for(eb)
    v = rng.standard_normal(2 * L) * 10.0 ** rng.uniform(-12, 0, 2 * L)
    v[::17] = 0.0
    v[5] = -0.0
    # exact halfway cases: 1 + (2j + 1) 2^-(b+1) lies between two b-bit mantissas
    v[7] = 1.0 + 2.0 ** -(b + 1)            # rounds down to 1 (even)
    v[9] = 1.0 + 3 * 2.0 ** -(b + 1)        # rounds up to 1 + 2^-(b-1)
    v[11] = -(2.0 - 2.0 ** -(b + 2))        # rounds up to -2 (into the next binade)
    rec, st = oracle.compress_slice(v[:L], v[L:], 10, 8, eb, oracle.PWREL)
    back = oracle.decompress_slice(rec, 1.0)
    got = np.concatenate([back.real, back.imag])
    want = nearest_with_bits(v, b)
    assert np.array_equal(got, want)
    assert got[7] == 1.0 and got[9] == 1.0 + 2.0 ** -(b - 1) and got[11] == -2.0
    nz = v != 0
    assert np.all(np.abs(got - v)[nz] <= eb * np.abs(v[nz]))
    assert np.all(got[~nz] == 0.0)
    # codes: the rounded magnitude's bit pattern >> (52 - b), with the value's sign
    p = oracle.decode_p(rec)
    mag = np.abs(want).view(np.uint64) >> np.uint64(52 - b)
    assert np.array_equal(np.abs(p).astype(np.uint64), mag)
    assert np.all((p < 0) == (want < 0))


def test_norm_field_is_the_pairwise_tree_of_squares():
    rng = np.random.default_rng(2)
    L = 1 << 9
    v = rng.standard_normal(2 * L) * 1e-2
    rec, st = oracle.compress_slice(v[:L], v[L:], 9, 6, 1e-3, oracle.PWREL)
    h = oracle.parse_header(rec)
    assert h["step"] == 1.0 and h["sumsq"] >> 64 == 0
    got = np.array([h["sumsq"]], dtype=np.uint64).view(np.float64)[0]
    back = oracle.decompress_slice(rec, 1.0)
    x = np.concatenate([back.real, back.imag]) ** 2
    while x.size > 1:
        x = x[0::2] + x[1::2]
    assert got == x[0]
    assert abs(got - math.fsum(np.concatenate([back.real, back.imag]) ** 2)) <= 1e-15 * got
    assert oracle.norm([1.0], [h["sumsq"]], oracle.PWREL) == got


def test_run_within_first_order_bound_of_exact():
    n, sl, eb = 10, 6, 1e-4
    f = qc.product_factors(*qc.product_angles(n, 5))
    s = oracle.OracleSim(n, sl, 5, eb, oracle.PWREL)
    s.init_product(f)
    gates = qc.qft(n)
    s.apply(gates)
    exact = math.sqrt(1 << n) * np.fft.ifft(oracle.product_state(f))
    a = s.amplitudes()
    # each pass adds an error of at most eb |v| per value, at most eb in 2-norm
    # for a unit state (plus the initial compression)
    assert np.linalg.norm(a - exact) <= (len(gates) + 1) * eb * 1.01
    assert s.max_err() > 0.0


def test_refused_and_corrupt():
    with pytest.raises(oracle.OracleError):
        oracle.compress_slice(np.ones(4), np.ones(4), 2, 2, 0.7, oracle.PWREL)  # bound out of range
    with pytest.raises(oracle.OracleError):
        oracle.compress_slice(np.ones(4), np.ones(4), 2, 2, 1e-9, oracle.PWREL)  # more than 20 bits
    rec, _ = oracle.compress_slice(np.full(4, 0.25), np.zeros(4), 2, 2, 0.01, oracle.PWREL)
    bad = bytearray(rec)
    bad[60] = 30  # bit count beyond the limit
    with pytest.raises(oracle.OracleError):
        oracle.decompress_slice(bytes(bad), 1.0)
    bad = bytearray(rec)
    bad[56] &= ~4  # the bit count without the flag
    with pytest.raises(oracle.OracleError):
        oracle.decompress_slice(bytes(bad), 1.0)
