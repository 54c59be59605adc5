"""Pins for the oracle's zero-chunk records (mode bit ZERO_CHUNKS): a chunk
whose codes are all zero is stored with no words, and nothing else changes.

Checks against a hand-derived record, against chunk sizes computed here from
the decoded codes, and against the same data coded without the mode (same
code table, same codes, same run of Algorithm 1)."""
import struct

import numpy as np
import pytest

import oracle
import qcircuits as qc
from test_oracle_codec import _chunk_bits_independent

ZC = oracle.ABS | oracle.ZERO_CHUNKS


def test_hand_derived_zero_chunk_record():
    # L = 4, chunks of B = 2 values: Re = (0, 0, 3 step, 0), Im = 0.
    # Differences per chunk: (0, 0), (3, -3), (0, 0), (0, 0) -> symbols
    # 512 x 6, 515, 509.  Package-merge: 509 and 515 get 2 bits, 512 gets 1;
    # canonical codes by (length, symbol): 512 -> 0, 509 -> 10, 515 -> 11.
    # Only chunk 1 is coded: 11 10 -> one word 0xE0000000.
    eb = 1e-6
    step = (2.0 * eb) * (1.0 - 2.0 ** -20)
    re = np.array([0.0, 0.0, 3 * step, 0.0])
    im = np.zeros(4)
    rec, st = oracle.compress_slice(re, im, 2, 1, eb, ZC)
    h = oracle.parse_header(rec)
    assert h["flags"] == 1 and h["n_used"] == 3 and h["n_words"] == 1 and h["n_escapes"] == 0
    assert oracle.symtab(rec) == [(512, 1), (509, 2), (515, 2)]
    assert list(oracle.chunk_offsets(rec)) == [0, 0, 1, 1, 1]
    assert struct.unpack_from("<I", rec, len(rec) - 4)[0] == 0xE0000000
    assert len(rec) == 64 + 8 + 4 * 5 + 4
    assert list(oracle.decode_p(rec)) == [0, 0, 3, 0, 0, 0, 0, 0]
    # without the mode every chunk takes its word
    plain, _ = oracle.compress_slice(re, im, 2, 1, eb)
    assert oracle.parse_header(plain)["flags"] == 0
    assert list(oracle.chunk_offsets(plain)) == [0, 1, 2, 3, 4]
    assert len(plain) == len(rec) + 12


def _sparse_planes(L, seed, B):
    rng = np.random.default_rng(seed)
    re = rng.normal(0, 1e-3, L) * (rng.random(L) < 0.2)
    im = np.zeros(L)
    # whole chunks of zeros, some chunks with a single small value
    mask = np.repeat(rng.random(L // B) < 0.6, B)
    re[mask] = 0.0
    im[rng.integers(0, L, 5)] = 2e-5
    return re, im


@pytest.mark.parametrize("seed", range(4))
def test_zero_chunk_sizes_follow_definition(seed):
    slice_log2, chunk_log2, eb = 10, 5, 1e-6
    B = 1 << chunk_log2
    re, im = _sparse_planes(1 << slice_log2, seed, B)
    rec, st = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb, ZC)
    p = oracle.decode_p(rec)
    bits, nesc, nused = _chunk_bits_independent(p, B)
    zero = ~p.reshape(-1, B).any(axis=1)
    assert zero.sum() > 0 and (~zero).sum() > 0
    words = np.where(zero, 0, (bits + 31) // 32)
    assert np.array_equal(np.diff(oracle.chunk_offsets(rec)), words)
    h = oracle.parse_header(rec)
    assert h["n_words"] == int(words.sum()) and h["n_used"] == nused and h["n_escapes"] == nesc
    assert h["flags"] == 1


@pytest.mark.parametrize("seed", range(3))
def test_zero_chunks_change_only_the_stream(seed):
    slice_log2, chunk_log2, eb = 9, 4, 1e-6
    re, im = _sparse_planes(1 << slice_log2, seed + 10, 1 << chunk_log2)
    a, sa = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb, ZC)
    b, sb = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb)
    assert oracle.symtab(a) == oracle.symtab(b)
    assert sa == sb
    assert np.array_equal(oracle.decode_p(a), oracle.decode_p(b))
    ha, hb = oracle.parse_header(a), oracle.parse_header(b)
    assert ha["n_words"] < hb["n_words"]
    assert {k: v for k, v in ha.items() if k not in ("n_words", "total", "flags")} == \
           {k: v for k, v in hb.items() if k not in ("n_words", "total", "flags")}


def test_empty_chunk_without_the_flag_is_corrupt():
    eb = 1e-6
    step = (2.0 * eb) * (1.0 - 2.0 ** -20)
    rec, _ = oracle.compress_slice(np.array([0.0, 0.0, 3 * step, 0.0]), np.zeros(4), 2, 1, eb, ZC)
    bad = bytearray(rec)
    struct.pack_into("<I", bad, 56, 0)
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))
    struct.pack_into("<I", bad, 56, 4)  # unknown flag
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))


def test_one_symbol_code_needs_no_flag():
    # every value zero: a one-symbol code of no bits, every chunk empty
    rec, _ = oracle.compress_slice(np.zeros(64), np.zeros(64), 6, 3, 1e-6)
    assert oracle.parse_header(rec)["n_words"] == 0
    assert not oracle.decode_p(rec).any()


@pytest.mark.parametrize("fp32", [False, True])
def test_zero_chunk_run_equals_plain_run(fp32):
    """Algorithm 1 with zero chunks: the same codes after every gate (so the
    same amplitudes), fewer bytes."""
    n, sl, cl, eb = 10, 7, 4, 1e-6
    gates = qc.grover(n, 345, 1)
    fmode = oracle.FP32 if fp32 else 0
    a = oracle.OracleSim(n, sl, cl, eb, ZC | fmode)
    b = oracle.OracleSim(n, sl, cl, eb, oracle.ABS | fmode)
    smaller = 0
    for i in range(0, len(gates), 7):
        a.apply(gates[i:i + 7])
        b.apply(gates[i:i + 7])
        for j in range(a.nslices):
            ra, rb = a.record(j), b.record(j)
            assert np.array_equal(oracle.decode_p(ra), oracle.decode_p(rb))
            assert len(ra) <= len(rb)
            smaller += len(ra) < len(rb)
    assert smaller > 0
    assert np.array_equal(a.amplitudes().view(np.float64), b.amplitudes().view(np.float64))
    assert a.total_bytes() < b.total_bytes()
