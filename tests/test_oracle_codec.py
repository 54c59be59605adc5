"""Pins for the oracle's slice codec (Compress / Decompress of Algorithm 1,
Section II; SZ-style error-bounded quantisation named in Section I).

Each check compares the oracle with something it does not compute itself:
hand-derived records, the canonical-code example of RFC 1951, exhaustive
search and textbook Huffman for code lengths, numpy's rint for the quantiser,
math.fsum for the norm."""
import json
import math
import os
import struct

import numpy as np
import pytest

import oracle
from brute import best_limited_cost, huffman_cost

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------ Huffman lengths

def test_hand_worked_huffman_lengths():
    g = load("huffman_hand.json")
    assert list(oracle.huffman_lengths(g["hist"])) == g["lengths"]


def test_canonical_codes_rfc1951_example():
    g = load("rfc1951_canonical.json")
    lens = np.array(g["lengths"], dtype=np.uint8)
    codes = oracle.canonical_codes(lens, lmax=12)
    got = [format(int(c), "0%db" % l) for c, l in zip(codes, lens)]
    assert got == g["codes"]


@pytest.mark.parametrize("seed", range(40))
def test_length_limited_optimal_vs_exhaustive(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    lmax = int(rng.integers(max(2, math.ceil(math.log2(n))), 6))
    w = rng.integers(1, 60, size=n) ** rng.integers(1, 4)
    lens = oracle.huffman_lengths(w, lmax=lmax)
    assert max(lens) <= lmax and min(lens) >= 1
    assert sum(2.0 ** -int(l) for l in lens) == 1.0  # complete prefix code
    assert int(np.dot(w, lens.astype(np.int64))) == best_limited_cost(w, lmax)


@pytest.mark.parametrize("seed", range(20))
def test_unconstrained_equals_textbook_huffman(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 300))
    w = rng.integers(1, 1000, size=n)
    lens = oracle.huffman_lengths(w, lmax=30)
    assert int(np.dot(w, lens.astype(np.int64))) == huffman_cost(w)


def test_length_limit_binds_on_geometric_weights():
    w = [2 ** i for i in range(20)]  # unconstrained Huffman would need depth 19
    lens = oracle.huffman_lengths(w, lmax=12)
    assert max(lens) == 12
    assert sum(2.0 ** -int(l) for l in lens) == 1.0


def test_single_used_symbol_needs_no_bits():
    h = np.zeros(1024, dtype=np.uint64)
    h[512] = 777
    lens = oracle.huffman_lengths(h)
    assert lens.sum() == 0


# ---------------------------------------------------------------- records

@pytest.mark.parametrize("case", load("records_hand.json")["records"], ids=lambda c: c["name"])
def test_hand_derived_records_bytes(case):
    rec, st = oracle.compress_slice(np.array(case["re"]), np.array(case["im"]), case["slice_log2"],
                                    case["chunk_log2"], case["eb"], case["mode"])
    assert rec.hex() == case["hex"]
    p = oracle.decode_p(rec)
    assert list(p) == [int(x) for x in case["re"] + case["im"]]


def _rand_planes(L, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(L) * scale, rng.standard_normal(L) * scale


@pytest.mark.parametrize("slice_log2,chunk_log2,eb", [(4, 2, 1e-3), (10, 10, 1e-6), (12, 8, 1e-7),
                                                      (12, 12, 1e-4), (3, 5, 1e-2)])
def test_abs_quantiser_matches_numpy_rint_and_bound(slice_log2, chunk_log2, eb):
    L = 1 << slice_log2
    re, im = _rand_planes(L, slice_log2)
    rec, st = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb, oracle.ABS)
    step = (2.0 * eb) * (1.0 - 2.0 ** -20)
    r = 1.0 / step
    v = np.concatenate([re, im])
    want_p = np.rint(v * r).astype(np.int64)
    p = oracle.decode_p(rec)
    assert np.array_equal(p, want_p)
    assert np.all(np.abs(v - p * step) <= eb)
    h = oracle.parse_header(rec)
    assert h["step"] == step
    assert h["sumsq"] == sum(int(x) * int(x) for x in want_p)
    assert st["max_err"] <= eb


def test_rel_step_is_power_of_two_and_bounded():
    for seed in range(10):
        re, im = _rand_planes(256, seed, scale=10.0 ** (seed - 5))
        v = np.concatenate([re, im])
        rel = [1e-2, 1e-4, 3e-5][seed % 3]
        step, r, ebj = oracle.rel_step(rel, v)
        assert ebj == rel * (v.max() - v.min())
        m, e = math.frexp(step)
        assert m == 0.5  # a power of two
        assert step <= 2 * ebj < 2 * step
        rec, _ = oracle.compress_slice(re, im, 8, 6, rel, oracle.REL)
        p = oracle.decode_p(rec)
        assert np.array_equal(p, np.rint(v / step).astype(np.int64))
        assert np.all(np.abs(v - p * step) <= ebj)


def test_rel_constant_slice_uses_magnitude_floor():
    v = np.full(16, 0.3)
    step, r, ebj = oracle.rel_step(1e-3, v)
    assert ebj == 1e-3 * (0.3 * 2.0 ** -24)
    re = np.zeros(8)
    step0, _, e0 = oracle.rel_step(1e-3, np.zeros(16))
    assert step0 == 1.0 and e0 == 0.0
    rec, _ = oracle.compress_slice(re, re, 3, 3, 1e-3, oracle.REL)
    assert np.all(oracle.decode_p(rec) == 0)


def _chunk_bits_independent(p, B):
    """Bits of every chunk from the stream definition, recomputed here."""
    d = p.copy()
    for c in range(0, p.size, B):
        d[c + 1:c + B] = p[c + 1:c + B] - p[c:c + B - 1]
    esc = np.abs(d) >= 512
    sym = np.where(esc, 0, d + 512)
    hist = np.bincount(sym, minlength=1024)
    lens = oracle.huffman_lengths(hist)
    zz = np.where(d >= 0, 2 * d, -2 * d - 1).astype(np.uint64)
    nb = np.array([int(z).bit_length() for z in zz])
    bits = lens[sym].astype(np.int64) + np.where(esc, 6 + nb, 0)
    return bits.reshape(-1, B).sum(axis=1), int(esc.sum()), int((hist > 0).sum())


@pytest.mark.parametrize("seed", range(6))
def test_stream_sizes_follow_definition(seed):
    slice_log2, chunk_log2 = 11, 7
    re, im = _rand_planes(1 << slice_log2, seed, scale=[1e-4, 1e-2, 1.0][seed % 3])
    eb = 1e-6
    rec, st = oracle.compress_slice(re, im, slice_log2, chunk_log2, eb)
    p = oracle.decode_p(rec)
    cb, nesc, nused = _chunk_bits_independent(p, 1 << chunk_log2)
    h = oracle.parse_header(rec)
    assert h["n_escapes"] == nesc == st["n_escapes"]
    assert h["n_used"] == nused
    words = (cb + 31) // 32
    assert h["n_words"] == int(words.sum())
    sym_bytes = (2 * nused + 3) // 4 * 4
    offs = np.frombuffer(rec[64 + sym_bytes:64 + sym_bytes + 4 * (h["n_chunks"] + 1)], dtype="<u4")
    assert np.array_equal(np.diff(offs.astype(np.int64)), words)
    assert h["total"] == len(rec) == 64 + sym_bytes + 4 * (h["n_chunks"] + 1) + 4 * h["n_words"]


def test_special_inputs():
    # constant slice: one escape (the chunk head) per chunk, zeros elsewhere
    L, B = 256, 64
    step = (2.0 * 1e-6) * (1.0 - 2.0 ** -20)
    re = np.full(L, 1000 * step)
    im = np.zeros(L)
    rec, _ = oracle.compress_slice(re, im, 8, 6, 1e-6)
    h = oracle.parse_header(rec)
    assert h["n_escapes"] == L // B  # only Re chunks start at 1000 >= R
    assert [s for s, _ in oracle.symtab(rec)] == [0, 512]
    # linear ramp: constant difference
    re = np.arange(L) * step
    rec, _ = oracle.compress_slice(re, np.zeros(L), 8, 6, 1e-6)
    syms = [s for s, _ in oracle.symtab(rec)]
    assert 513 in syms and 512 in syms
    # basis state: zero everywhere except one amplitude
    re = np.zeros(L)
    re[37] = 1.0
    rec, _ = oracle.compress_slice(re, np.zeros(L), 8, 6, 1e-6)
    h = oracle.parse_header(rec)
    assert h["n_escapes"] == 2  # the jump up and the jump back down
    p = oracle.decode_p(rec)
    assert p[37] == round(1.0 / step) and np.count_nonzero(p) == 1


def test_out_of_range_codes_are_refused():
    re = np.full(4, 1.0)
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress_slice(re, re, 2, 2, 1e-16)  # |p| ~ 5e15 >= 2^48
    assert e.value.rc == -3


def test_corrupted_record_is_detected():
    re, im = _rand_planes(64, 3)
    rec, _ = oracle.compress_slice(re, im, 6, 4, 1e-5)
    bad = bytearray(rec)
    bad[0] ^= 1  # magic
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))
    bad = bytearray(rec)
    bad[64 + 1] ^= 0x10  # a code length in the symbol table -> Kraft sum != 1
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))
    bad = bytearray(rec)
    struct.pack_into("<I", bad, 28, len(rec) + 4)  # total size
    with pytest.raises(oracle.OracleError):
        oracle.decode_p(bytes(bad))


# ----------------------------------------------------------- normalisation

def test_norm_equals_fsum_of_decoded_state():
    recs = []
    for j in range(8):
        re, im = _rand_planes(128, 50 + j, scale=0.03)
        rec, _ = oracle.compress_slice(re, im, 7, 5, 1e-7)
        recs.append(rec)
    hs = [oracle.parse_header(r) for r in recs]
    N = oracle.norm(np.array([h["step"] for h in hs]), [h["sumsq"] for h in hs])
    terms = []
    for r, h in zip(recs, hs):
        p = oracle.decode_p(r)
        terms += list((p * h["step"]) ** 2)
    assert abs(N - math.fsum(terms)) <= 1e-15 * N
    s = oracle.rsqrt(N)
    assert abs(s - 1 / math.sqrt(N)) <= 2e-16 / math.sqrt(N)
    # after scaling, the decoded state has unit norm
    tot = math.fsum(float(x) for r, h in zip(recs, hs) for x in np.abs(oracle.decompress_slice(r, h["step"] * s)) ** 2)
    assert abs(tot - 1) < 1e-14


def test_rsqrt_newton_converges_over_range():
    for N in [0.3, 0.9, 1.0, 1.0 + 1e-7, 1.7, 2.5]:
        s = oracle.rsqrt(N)
        assert abs(s * math.sqrt(N) - 1) < 4e-16
