"""Pins for the oracle's chunk-run records (mode bit CHUNK_RUNS): consecutive
chunks with identical streams store the stream once, behind a table of run
ends and word offsets, where that makes the record smaller and there are at
most MAX_RUNS runs; codes and amplitudes do not change.

Checks against a hand-derived record, against runs recomputed here from the
plain record of the same data (its chunk offsets and words), against the
size rule, and against the same run of Algorithm 1 without the mode."""
import struct

import numpy as np
import pytest

import oracle
import qcircuits as qc

RUNS = oracle.ABS | oracle.CHUNK_RUNS
M = 0x80000000


def step_of(eb):
    return 2.0 * eb * (1.0 - 2.0 ** -20)


def test_hand_derived_chunk_run_record():
    # L = 4, chunks of B = 2: Re = (5, 5, 5, 5) steps, Im = 0.  Differences
    # (5, 0) (5, 0) (0, 0) (0, 0): symbols 517 twice, 512 six times; two used
    # symbols, one bit each, canonical 512 -> 0, 517 -> 1.  Streams "10",
    # "10", "00", "00": chunk words 0x80000000 twice, then 0 twice.  Two runs
    # (ends 2, 4; word offsets 0, 1, 2) and two stored words make 24 + 8
    # bytes against the plain 20 + 16.
    eb = 1e-6
    re = np.full(4, 5.0) * step_of(eb)
    rec, _ = oracle.compress_slice(re, np.zeros(4), 2, 1, eb, RUNS)
    h = oracle.parse_header(rec)
    assert h["flags"] == 8 and h["n_used"] == 2 and h["n_words"] == 2 and h["total"] == 100 == len(rec)
    assert oracle.symtab(rec) == [(512, 1), (517, 1)]
    assert struct.unpack_from("<6I", rec, 68) == (2, 2, 4, 0, 1, 2)
    assert struct.unpack_from("<2I", rec, 92) == (0x80000000, 0)
    assert list(oracle.decode_p(rec)) == [5, 5, 5, 5, 0, 0, 0, 0]
    plain, _ = oracle.compress_slice(re, np.zeros(4), 2, 1, eb, oracle.ABS)
    assert len(plain) == 104 and oracle.parse_header(plain)["flags"] == 0


def runs_from_plain(plain):
    """Runs of equal chunk streams, recomputed from a plain record."""
    h = oracle.parse_header(plain)
    o = 64 + ((2 * h["n_used"] + 3) & ~3)
    raw = np.frombuffer(plain[o:o + 4 * (h["n_chunks"] + 1)], dtype="<u4").astype(np.int64)
    words = np.frombuffer(plain[o + 4 * (h["n_chunks"] + 1):], dtype="<u4")
    off, mark = raw & 0x7FFFFFFF, raw >> 31
    streams = [(int(mark[c]), words[off[c]:off[c + 1]].tobytes()) for c in range(h["n_chunks"])]
    starts = [c for c in range(h["n_chunks"]) if c == 0 or streams[c] != streams[c - 1]]
    return starts, streams


def check_against_plain(runs_rec, plain):
    starts, streams = runs_from_plain(plain)
    hp, hr = oracle.parse_header(plain), oracle.parse_header(runs_rec)
    W = sum(len(streams[c][1]) // 4 for c in starts)
    R = len(starts)
    smaller = 8 * R + 8 + 4 * W < 4 * (hp["n_chunks"] + 1) + 4 * hp["n_words"]
    if R <= oracle.MAX_RUNS and smaller:
        ends, woff = oracle.chunk_runs(runs_rec)
        assert list(ends) == starts[1:] + [hp["n_chunks"]]
        w = 0
        for r, c in enumerate(starts):
            assert woff[r] == (w | (M if streams[c][0] else 0))
            w += len(streams[c][1]) // 4
        assert woff[R] == w == hr["n_words"]
        body = runs_rec[len(runs_rec) - 4 * w:]
        assert body == b"".join(streams[c][1] for c in starts)
        assert hr["flags"] == hp["flags"] | 8
        assert hr["total"] == hp["total"] - 4 * (hp["n_chunks"] + 1) - 4 * hp["n_words"] + 8 * R + 8 + 4 * W
        for k in ("n_used", "n_escapes", "step", "sumsq", "pw_bits"):
            assert hr[k] == hp[k]
    else:
        assert runs_rec == plain
    assert np.array_equal(oracle.decode_p(runs_rec), oracle.decode_p(plain))


def periodic_planes(L, period, seed, eb):
    rng = np.random.default_rng(seed)
    base = rng.integers(-600, 600, size=period).astype(float)
    re = np.tile(base, L // period) * step_of(eb)
    return re, np.zeros(L)


@pytest.mark.parametrize("L,B,period", [(256, 16, 4), (1024, 32, 32), (4096, 64, 8), (1024, 8, 16)])
@pytest.mark.parametrize("extra", [0, oracle.ZERO_CHUNKS, oracle.CONST_CHUNKS, oracle.ZERO_CHUNKS | oracle.CONST_CHUNKS])
def test_runs_match_the_plain_record(L, B, period, extra):
    eb = 1e-6
    re, im = periodic_planes(L, period, L + B, eb)
    sl, cl = L.bit_length() - 1, B.bit_length() - 1
    plain, _ = oracle.compress_slice(re, im, sl, cl, eb, oracle.ABS | extra)
    runs, _ = oracle.compress_slice(re, im, sl, cl, eb, RUNS | extra)
    check_against_plain(runs, plain)
    if period <= B:  # every chunk of a plane the same: runs pay
        assert oracle.parse_header(runs)["flags"] & 8


def test_no_repeats_give_the_plain_record():
    rng = np.random.default_rng(4)
    eb = 1e-6
    re = rng.integers(-5000, 5000, size=1024) * step_of(eb)
    im = rng.integers(-5000, 5000, size=1024) * step_of(eb)
    plain, _ = oracle.compress_slice(re, im, 10, 4, eb, oracle.ABS)
    runs, _ = oracle.compress_slice(re, im, 10, 4, eb, RUNS)
    assert runs == plain


def test_run_cap():
    # 8192 chunks of 2 values; chunk pairs repeat, so runs are pairs: 4096
    # runs fit the cap, one more break (4097 runs) falls back to the plain table
    eb = 1e-6
    L = 8192
    vals = np.repeat(np.arange(4096) % 700 + 1.0, 4) * step_of(eb)  # chunks (v, v), pairs of equal chunks
    re, im = vals[:L].copy(), vals[L:].copy()
    runs, _ = oracle.compress_slice(re, im, 13, 1, eb, RUNS)
    plain, _ = oracle.compress_slice(re, im, 13, 1, eb, oracle.ABS)
    starts, _ = runs_from_plain(plain)
    assert len(starts) == oracle.MAX_RUNS
    assert oracle.parse_header(runs)["flags"] & 8
    check_against_plain(runs, plain)
    re2 = re.copy()
    re2[2] = 900 * step_of(eb)  # breaks the first pair: one more run
    runs2, _ = oracle.compress_slice(re2, im, 13, 1, eb, RUNS)
    plain2, _ = oracle.compress_slice(re2, im, 13, 1, eb, oracle.ABS)
    assert len(runs_from_plain(plain2)[0]) == oracle.MAX_RUNS + 1
    assert runs2 == plain2


@pytest.mark.parametrize("mode", [oracle.ABS, oracle.REL, oracle.FP32, oracle.PWREL,
                                  oracle.ZERO_CHUNKS | oracle.CONST_CHUNKS])
def test_algorithm1_run_has_the_same_codes(mode):
    n, sl, cl = 11, 8, 5
    eb = 0.002 if mode == oracle.PWREL else 1e-6
    gates = qc.grover(n, 300, 2)
    a = oracle.OracleSim(n, sl, cl, eb, mode)
    b = oracle.OracleSim(n, sl, cl, eb, mode | oracle.CHUNK_RUNS)
    used = 0
    for k in range(0, len(gates), 7):
        a.apply(gates[k:k + 7])
        b.apply(gates[k:k + 7])
        for ra, rb in zip(a.records(), b.records()):
            check_against_plain(rb, ra)
            used += bool(oracle.parse_header(rb)["flags"] & 8)
    assert used > 0
    assert np.array_equal(a.amplitudes(), b.amplitudes())


def corrupt(rec, word_index, value):
    b = bytearray(rec)
    struct.pack_into("<I", b, word_index * 4, value)
    return bytes(b)


def test_corrupt_run_tables_are_refused():
    eb = 1e-6
    re = np.full(4, 5.0) * step_of(eb)
    rec, _ = oracle.compress_slice(re, np.zeros(4), 2, 1, eb, RUNS)
    # words 17.. : R, ends (2), woff (3), stream (2)
    assert struct.unpack_from("<I", rec, 68)[0] == 2
    bad = [
        corrupt(rec, 17, 0),                # no runs
        corrupt(rec, 17, 5),                # more runs than chunks
        corrupt(rec, 18, 4),                # ends not increasing
        corrupt(rec, 19, 3),                # last end short of n_chunks
        corrupt(rec, 22, 3),                # last word offset beyond n_words
        corrupt(rec, 22, 2 | M),            # a mark on the last offset
        corrupt(rec, 20, M),                # a constant mark without header bit 1
        corrupt(rec, 21, 0),                # word offsets decreasing
        corrupt(rec, 14, 16),               # an unknown flag
    ]
    for r in bad:
        with pytest.raises(oracle.OracleError):
            oracle.decode_p(r)
