"""Pins for the oracle's constant-chunk records (mode bit CONST_CHUNKS): a
chunk whose values all equal its head keeps only the head's code, marked by
bit 31 of its word offset; nothing else changes.

Checks against a hand-derived record, against chunk sizes and marks computed
here from the decoded codes, and against the same data coded without the mode
(same code table, same codes, same run of Algorithm 1)."""
import struct

import numpy as np
import pytest

import oracle
import qcircuits as qc

CC = oracle.ABS | oracle.CONST_CHUNKS
M = 0x80000000


def raw_offsets(rec):
    h = oracle.parse_header(rec)
    o = 64 + ((2 * h["n_used"] + 3) & ~3)
    return [int(x) for x in np.frombuffer(rec[o:o + 4 * (h["n_chunks"] + 1)], dtype="<u4")]


def test_hand_derived_constant_chunk_record():
    # L = 4, chunks of B = 2 values: Re = (5, 5, 0, 3) steps, Im = 0.
    # Differences per chunk: (5, 0), (0, 3), (0, 0), (0, 0) -> symbols 517,
    # 512 x 6, 515.  Lengths: 515 and 517 two bits, 512 one; canonical codes
    # 512 -> 0, 515 -> 10, 517 -> 11.  Chunks 0, 2 and 3 are constant and keep
    # their head only: "11", "0", "0"; chunk 1 is coded whole: "0" "10".
    eb = 1e-6
    step = (2.0 * eb) * (1.0 - 2.0 ** -20)
    re = np.array([5, 5, 0, 3]) * step
    rec, _ = oracle.compress_slice(re, np.zeros(4), 2, 1, eb, CC)
    h = oracle.parse_header(rec)
    assert h["flags"] == 2 and h["n_used"] == 3 and h["n_words"] == 4
    assert oracle.symtab(rec) == [(512, 1), (515, 2), (517, 2)]
    assert raw_offsets(rec) == [0 | M, 1, 2 | M, 3 | M, 4]
    words = struct.unpack_from("<4I", rec, len(rec) - 16)
    assert words == (0xC0000000, 0x40000000, 0, 0)
    assert list(oracle.decode_p(rec)) == [5, 5, 0, 3, 0, 0, 0, 0]
    # with zero chunks as well, the two all-zero chunks keep nothing and no mark
    rz, _ = oracle.compress_slice(re, np.zeros(4), 2, 1, eb, CC | oracle.ZERO_CHUNKS)
    assert oracle.parse_header(rz)["flags"] == 3
    assert raw_offsets(rz) == [0 | M, 1, 2, 2, 2]
    assert list(oracle.decode_p(rz)) == [5, 5, 0, 3, 0, 0, 0, 0]


def _piecewise_planes(L, B, seed):
    rng = np.random.default_rng(seed)
    step = 2e-6 * (1.0 - 2.0 ** -20)
    lev = rng.integers(-3000, 3000, size=2 * L // B).astype(float)
    v = np.repeat(lev, B) * step
    noisy = np.repeat(rng.random(2 * L // B) < 0.3, B)  # some chunks not constant
    v[noisy] += rng.integers(-40, 40, size=int(noisy.sum())) * step
    return v[:L].copy(), v[L:].copy()


def _bits_per_position(p, B):
    d = p.copy()
    for c in range(0, p.size, B):
        d[c + 1:c + B] = p[c + 1:c + B] - p[c:c + B - 1]
    esc = np.abs(d) >= 512
    sym = np.where(esc, 0, d + 512)
    lens = oracle.huffman_lengths(np.bincount(sym, minlength=1024))
    nb = np.array([int(z).bit_length() for z in np.where(d >= 0, 2 * d, -2 * d - 1)])
    return (lens[sym].astype(np.int64) + np.where(esc, 6 + nb, 0)).reshape(-1, B), d.reshape(-1, B)


@pytest.mark.parametrize("seed", range(4))
def test_constant_chunk_sizes_and_marks_follow_definition(seed):
    slice_log2, chunk_log2, eb = 10, 4, 1e-6
    B = 1 << chunk_log2
    re, im = _piecewise_planes(1 << slice_log2, B, seed)
    rec, _ = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb, CC)
    p = oracle.decode_p(rec)
    bits, d = _bits_per_position(p, B)
    const = ~(d[:, 1:] != 0).any(axis=1)
    assert const.sum() > 0 and (~const).sum() > 0
    words = np.where(const, (bits[:, 0] + 31) // 32, (bits.sum(axis=1) + 31) // 32)
    assert np.array_equal(oracle.constant_chunks(rec), const)
    assert np.array_equal(np.diff(oracle.chunk_offsets(rec)), words)
    plain, _ = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb)
    assert np.array_equal(oracle.decode_p(plain), p)
    assert oracle.symtab(plain) == oracle.symtab(rec)
    assert len(rec) < len(plain)


def test_constant_marks_need_the_flag_and_stay_off_the_last_offset():
    eb = 1e-6
    step = (2.0 * eb) * (1.0 - 2.0 ** -20)
    rec, _ = oracle.compress_slice(np.array([5, 5, 0, 3]) * step, np.zeros(4), 2, 1, eb, CC)
    bad = bytearray(rec)
    struct.pack_into("<I", bad, 56, 0)  # marks without the flag
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))
    bad = bytearray(rec)
    o = 64 + 8 + 4 * 4  # the last offset
    struct.pack_into("<I", bad, o, struct.unpack_from("<I", bad, o)[0] | M)
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))


@pytest.mark.parametrize("extra", [0, oracle.ZERO_CHUNKS, oracle.FP32])
def test_constant_chunk_run_equals_plain_run(extra):
    """Algorithm 1 with constant chunks: the same codes after every pass,
    fewer bytes."""
    n, sl, cl, eb = 10, 7, 4, 1e-6
    gates = qc.grover(n, 345, 1)
    base = oracle.ABS | (extra & oracle.FP32)
    a = oracle.OracleSim(n, sl, cl, eb, CC | extra)
    b = oracle.OracleSim(n, sl, cl, eb, base)
    for i in range(0, len(gates), 9):
        a.apply(gates[i:i + 9])
        b.apply(gates[i:i + 9])
        for j in range(a.nslices):
            ra, rb = a.record(j), b.record(j)
            assert np.array_equal(oracle.decode_p(ra), oracle.decode_p(rb))
            assert len(ra) <= len(rb)
    assert np.array_equal(a.amplitudes().view(np.float64), b.amplitudes().view(np.float64))
    assert a.total_bytes() < b.total_bytes()
