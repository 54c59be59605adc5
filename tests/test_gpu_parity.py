"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Plain mode is deterministic end to end (integer codes, fixed FP64 operation
order, exact integer norm), so the bar is byte equality of every slice record
after every checked pass, and bit equality of the read-out amplitudes.
Each case prints its name before it touches the GPU."""
import math
import sys

import numpy as np
import pytest

import oracle
import qcircuits as qc

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def header_diff(a: bytes, b: bytes) -> str:
    ha, hb = oracle.parse_header(a), oracle.parse_header(b)
    return ", ".join(f"{k}: gpu {ha[k]} oracle {hb[k]}" for k in ha if ha[k] != hb[k]) or "payload differs"


def assert_same_records(sim, orc, label, which=None):
    idx = list(range(orc.nslices)) if which is None else list(which)
    g = sim.records(idx)
    for j, r in zip(idx, g):
        o = orc.record(j)
        if r != o:  # no assertion rewriting: a diff of two large records takes minutes
            pytest.fail(f"{label}: slice {j}: {header_diff(r, o)}")


def run_both(n, sl, cl, eb, gates, rel=False, init=None, check_every=1, workspace_bytes=0, arena_bytes=0,
             use_torch=None, fp32=False, zero_chunks=False, const_chunks=False, chunk_runs=False, pointwise=False,
             opt=False):
    mode = ((oracle.REL if rel else oracle.PWREL if pointwise else oracle.ABS) | (oracle.FP32 if fp32 else 0) |
            (oracle.ZERO_CHUNKS if zero_chunks else 0) | (oracle.CONST_CHUNKS if const_chunks else 0) |
            (oracle.CHUNK_RUNS if chunk_runs else 0) | (oracle.OPT if opt else 0))
    orc = oracle.OracleSim(n, sl, cl, eb, mode)
    sim = cq.Sim(n, sl, eb, relative=rel, chunk_log2=cl, workspace_bytes=workspace_bytes,
                 arena_bytes=arena_bytes, use_torch=use_torch, fp32=fp32, zero_chunks=zero_chunks,
                 const_chunks=const_chunks, chunk_runs=chunk_runs, pointwise=pointwise, opt=opt)
    if init is not None:
        kind, arg = init
        if kind == "basis":
            orc.init_basis(arg)
            sim.init_basis(arg)
        else:
            orc.init_product(arg)
            sim.init_product(arg)
    assert_same_records(sim, orc, "initial state")
    for i in range(0, len(gates), check_every):
        chunk = gates[i:i + check_every]
        orc.apply(chunk)
        assert sim.apply(chunk) == len(chunk)
        assert_same_records(sim, orc, f"after gate {i + len(chunk)} ({chunk[-1].name})")
    return sim, orc


def gate_zoo(n, seed):
    rng = np.random.default_rng(seed)

    def ru(k, s):
        r = np.random.default_rng(s)
        a = r.standard_normal((1 << k, 1 << k)) + 1j * r.standard_normal((1 << k, 1 << k))
        q, rr = np.linalg.qr(a)
        return q * (np.diag(rr) / abs(np.diag(rr)))

    g = []
    for t in range(n):
        g += [qc.H(t), qc.U3(t, 0.3 + t, 1.1, 0.2 * t), qc.Z(t), qc.X(t), qc.P(t, 0.7 - t)]
    for a, b in [(0, n - 1), (n - 1, 1), (n // 2, 0), (1, n // 2 + 1)]:
        if a != b and max(a, b) < n:
            g += [qc.CP(a, b, 0.4), qc.SWAP(a, b), qc.CZ(a, b), qc.U([a, b], ru(2, a * 7 + b))]
    for k in range(3, min(n, 5) + 1):
        tg = [int(x) for x in rng.permutation(n)[:k]]
        g.append(qc.U(tg, ru(k, k + seed)))
    if n >= 3:
        t = n - 1
        g.append(qc.U([t], ru(1, 99), ctrl_mask=0b11, ctrl_vals=0b01))
        g.append(qc.U([0], ru(1, 98), ctrl_mask=1 << (n - 1), ctrl_vals=1 << (n - 1)))
    g += [qc.MCZ(n), qc.MCPHASE((1 << n) - 1, int(rng.integers(0, 1 << n)), -1.0)]
    return g


# ------------------------------------------------------------------ cases

@pytest.mark.parametrize("cl", [1, 2, 4, 5, 6, 7, 8, 9, 10])
def test_sparse_periodic_escapes_every_group_size(cl):
    """The escape buffer keeps each group of min(chunk, 256) positions'
    escapes at the group's start (ranks from ballots, across the wavefronts
    of a tile through LDS).  A Grover state after its oracle, then H on the
    low qubits, has escapes every 2^t positions in its real plane (differences
    of about 780 and more steps against R = 512), and the dense two-qubit gates
    take the tile kernels: records byte-equal to the oracle after every pass."""
    n, sl, eb = 13, 11, 1e-5
    say("sparse escapes", n, sl, cl, eb)
    rng = np.random.default_rng(cl)

    def ru2(s):
        r = np.random.default_rng(s)
        a = r.standard_normal((4, 4)) + 1j * r.standard_normal((4, 4))
        q, rr = np.linalg.qr(a)
        return q * (np.diag(rr) / abs(np.diag(rr)))

    marked = int(rng.integers(0, 1 << n))
    gates = [qc.H(t) for t in range(n)] + [qc.MCPHASE((1 << n) - 1, marked, -1.0)]
    gates += [qc.H(t) for t in range(8)] + [qc.U([0, 1], ru2(cl)), qc.U([3, 6], ru2(cl + 50)), qc.H(9)]
    sim, orc = run_both(n, sl, cl, eb, gates)
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())
    assert sim.stats()["max_abs_codec_err"] <= eb


def test_qft12_basis_every_pass_identical():
    w = qc.qft_basis_workload()
    say("qft12 basis", w.n_qubits, w.slice_log2, w.error_bound)
    sim, orc = run_both(w.n_qubits, w.slice_log2, 10, w.error_bound, w.gates, init=("basis", w.basis))
    a_gpu, a_orc = sim.amplitudes(), orc.amplitudes()
    assert np.array_equal(a_gpu, a_orc)
    st = sim.stats()
    assert st["compressed_bytes"] == orc.total_bytes()
    assert st["peak_compressed"] == orc.peak_bytes()
    assert st["max_abs_codec_err"] <= w.error_bound
    assert st["passes"] == 84
    p = sim.probabilities()
    assert np.array_equal(p, a_gpu.real * a_gpu.real + a_gpu.imag * a_gpu.imag)


GEOMETRIES = [  # n, slice_log2, chunk_log2, eb
    (3, 1, 1, 1e-6), (4, 2, 1, 1e-5), (5, 3, 7, 1e-6), (6, 3, 2, 1e-7), (7, 7, 3, 1e-6),
    (8, 4, 3, 1e-6), (9, 6, 4, 1e-8), (10, 5, 5, 1e-6), (11, 9, 6, 1e-7), (12, 11, 10, 1e-6),
    # slices of 2^10 .. 2^12 with chunks of at most 256 values (the wavefront-range kernels):
    # targets inside a range (lanes, v), range pairs in a slice, slice pairs
    (12, 10, 8, 1e-6), (13, 11, 7, 1e-7), (14, 12, 5, 1e-6), (13, 12, 8, 1e-8),
]


@pytest.mark.parametrize("n,sl,cl,eb", GEOMETRIES)
def test_gate_zoo_geometries(n, sl, cl, eb):
    say("zoo", n, sl, cl, eb)
    gates = qc.random_layered(n, 2, seed=n) + gate_zoo(n, n)
    run_both(n, sl, cl, eb, gates)


@pytest.mark.parametrize("n,sl,cl", [(10, 6, 5), (12, 8, 10), (6, 2, 1)])
def test_relative_bound_product_state_qft(n, sl, cl):
    say("rel qft", n, sl, cl)
    theta, phi = qc.product_angles(n, 3)
    f = qc.product_factors(theta, phi)
    sim, orc = run_both(n, sl, cl, 1e-4, qc.qft(n), rel=True, init=("product", f))
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())


def test_grover_small_full_run():
    n, sl, cl, eb = 10, 6, 6, 1e-7
    say("grover10 full", n, sl, cl, eb)
    w = 613
    gates = qc.grover(n, w)
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=41)
    assert np.array_equal(sim.amplitudes(), orc.amplitudes())


def test_workspace_batches_and_arena_growth():
    n, sl, cl, eb = 14, 8, 7, 1e-6
    say("batches+growth", n, sl, cl, eb)
    nch = (2 << sl) >> cl
    stage_words = ((1 << cl) * 68 + 31) // 32 + 1
    per_slot = (2 * (1 << sl) * 18 + 1024 * 6 + 4 * 32 * (1024 + 8) + 12 * nch + 4 * nch * stage_words + 4 * 1024 +
                8 * 4096 + 140 + nch + 8 * ((nch + 1023) // 1024) + 4 * 1024)  # ... chunk-run tables
    gates = qc.random_layered(n, 2, seed=5) + [qc.U([13, 12, 3], np.eye(8)[::-1]), qc.H(13)]
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=7, workspace_bytes=8 * per_slot, arena_bytes=8192)
    st = sim.stats()
    assert st["workspace_slots"] == 8
    assert st["arena_bytes"] > 2 * 8192  # grew at least once


def test_arena_overflow_inside_one_batch():
    """One batch from a minimal arena: the records outgrow it mid-batch, the
    failed pass and those after it are replayed into a larger arena."""
    n, sl, cl, eb = 12, 7, 6, 1e-7
    say("overflow mid-batch", n, sl, cl, eb)
    gates = qc.random_layered(n, 3, seed=9)
    sim, orc = run_both(n, sl, cl, eb, gates, check_every=len(gates), arena_bytes=4096)
    assert sim.stats()["arena_bytes"] > 2 * 4096


def test_circuit_slices_match_gate_lists():
    n, sl, cl, eb = 11, 7, 6, 1e-6
    say("circuit slices", n, sl, cl, eb)
    gates = gate_zoo(n, seed=4)
    a = cq.Sim(n, sl, eb, chunk_log2=cl)
    b = cq.Sim(n, sl, eb, chunk_log2=cl)
    circ = cq.Circuit(gates)
    h = len(gates) // 2
    a.apply(gates[:h])
    a.apply(gates[h:])
    b.apply(circ[:h])
    b.apply(circ[h:])
    assert a.records() == b.records()


def test_invalid_gate_stops_with_completed_prefix():
    n, sl, cl, eb = 8, 5, 4, 1e-6
    say("invalid gate", n, sl)
    good = [qc.H(0), qc.H(7), qc.CP(0, 7, 0.3)]
    sim = cq.Sim(n, sl, eb, chunk_log2=cl)
    bad = qc.Gate(qc.DENSE, (0,), matrix=np.eye(2))
    bad.targets = (9,)
    rc, applied = sim.apply_partial(good + [bad, qc.H(1)])
    assert rc == -1 and applied == 3
    orc = oracle.OracleSim(n, sl, cl, eb)
    orc.apply(good)
    assert_same_records(sim, orc, "prefix")


def test_codes_beyond_int32_switch_the_workspace_format():
    """With a bound of 1e-10 a concentrated state has codes |q| > 2^31: the
    passes after it decode to an FP64 workspace, those after a spread state to
    the compact int32 one; the records match the oracle's through every switch."""
    n, sl, cl, eb = 12, 10, 8, 1e-10
    say("wide codes", n, sl, cl, eb)
    layer = [qc.H(q) for q in range(n)]
    gates = ([qc.H(0), qc.H(11), qc.X(3)] + layer + [qc.P(5, 0.3), qc.H(2), qc.H(2)] + layer +
             [qc.CP(1, 10, 0.7), qc.H(7), qc.H(10)])
    run_both(n, sl, cl, eb, gates, check_every=1)


def test_too_fine_bound_is_refused():
    say("ebound")
    with pytest.raises(cq.SimError) as e:
        cq.Sim(6, 3, 1e-15)
    assert e.value.rc == -3


def test_export_import_round_trip():
    n, sl, cl, eb = 10, 6, 5, 1e-6
    say("export/import", n, sl)
    g = qc.random_layered(n, 2, seed=11)
    a = cq.Sim(n, sl, eb, chunk_log2=cl)
    a.apply(g)
    recs = a.records()
    b = cq.Sim(n, sl, eb, chunk_log2=cl)
    for j, r in enumerate(recs):
        b.import_record(j, r)
    assert b.records() == recs
    assert np.array_equal(a.amplitudes(), b.amplitudes())
    more = qc.random_layered(n, 1, seed=12)
    a.apply(more)
    b.apply(more)
    assert a.records() == b.records()
    bad = bytearray(recs[0])
    bad[65] ^= 0x04  # a code length changes by one: no longer a complete prefix code
    with pytest.raises(cq.SimError) as e:
        b.import_record(0, bytes(bad))
    assert e.value.rc == -4
    with pytest.raises(cq.SimError) as e:
        b.import_record(0, recs[0][:-4])  # truncated
    assert e.value.rc == -4
    assert b.records() == a.records()  # refused imports leave the state alone


def test_deterministic_and_allocator_independent():
    n, sl, cl, eb = 12, 7, 6, 1e-6
    say("determinism", n, sl)
    g = qc.random_layered(n, 3, seed=2)
    out = []
    for use_torch in (True, False, True):
        s = cq.Sim(n, sl, eb, chunk_log2=cl, use_torch=use_torch)
        s.apply(g)
        out.append(s.records())
    assert out[0] == out[1] == out[2]


@pytest.mark.parametrize("cl", [8, 10])
def test_grover24_full_size_window(cl):
    """The benchmark geometry (24 qubits, 64 slices of 2^18, bound 1e-7) over the
    initial H layer, one oracle and the first diffusion gates."""
    w = qc.grover_workload()
    say("grover24 window", w.n_qubits, w.slice_log2, w.error_bound, "chunk", cl)
    gates = w.gates[:24 + 1 + 10]
    oracle.set_threads(0)
    sim, orc = run_both(w.n_qubits, w.slice_log2, cl, w.error_bound, gates, check_every=len(gates))
    idx = [0, 1, 17, 63]
    a = sim.amplitudes(0, 1 << 12)
    assert np.array_equal(a, orc.amplitudes(0, 1 << 12))
    st = sim.stats()
    assert st["compressed_bytes"] == orc.total_bytes()
