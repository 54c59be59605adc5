"""CPU oracle for the compressed state-vector simulation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The simulator library never calls it:
it shares no code, header or table with the HIP path.  The arithmetic lives in
``cqsim_oracle.c`` (plain C, FP64, compiled by ``oracle/build.py``); this file
only marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CQ_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

ABS = 0
REL = 1
FP32 = 2  # mode bit: FP32 working values and gate arithmetic (quantiser and norm stay FP64)
ZERO_CHUNKS = 8  # mode bit: a chunk whose codes are all zero is stored with no words
CONST_CHUNKS = 16  # mode bit: a chunk whose values all equal its head keeps only the head (offset bit 31)
PWREL = 32  # mode bit: pointwise-relative bound (|v - v'| <= eb |v| for every value)
CHUNK_RUNS = 64  # mode bit: runs of chunks with identical streams store the stream once (flags bit 3)
MAX_RUNS = 4096  # chunk-run records hold at most this many runs
OPT = 128  # mode bit: passes skip slice groups where a gate's slice-index controls fail, relabel index SWAPs

R = 512
NSYM = 1024
LMAX = 12


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"oracle {what} failed with code {rc}")
        self.rc = rc


class _Gate(C.Structure):
    _fields_ = [
        ("kind", C.c_uint32),
        ("n_targets", C.c_uint32),
        ("targets", C.c_uint32 * 5),
        ("pad", C.c_uint32),
        ("ctrl_mask", C.c_uint64),
        ("ctrl_vals", C.c_uint64),
        ("phase_re", C.c_double),
        ("phase_im", C.c_double),
        ("matrix", C.POINTER(C.c_double)),
    ]


class _Pass(C.Structure):
    _fields_ = [("first", C.c_uint32), ("count", C.c_uint32), ("fused", C.c_uint32), ("k", C.c_uint32),
                ("qubits", C.c_uint32 * 5), ("pad", C.c_uint32)]


class _CStats(C.Structure):
    _fields_ = [("max_err", C.c_double), ("n_escapes", C.c_uint64), ("sumsq_lo", C.c_uint64),
                ("sumsq_hi", C.c_uint64), ("step", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_sv_apply.argtypes = [C.c_int, P, P, C.POINTER(_Gate)]
        L.orc_sv_apply_mode.argtypes = [C.c_int, P, P, C.POINTER(_Gate), C.c_uint32]
        L.orc_abs_step.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_rel_step.argtypes = [C.c_double, P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]
        L.orc_huffman_lengths.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_canonical_codes.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_compress_slice.argtypes = [P, P, C.c_int, C.c_int, C.c_double, C.c_uint32,
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.POINTER(_CStats)]
        L.orc_decode_p.argtypes = [P, C.c_uint64, P]
        L.orc_decompress_slice.argtypes = [P, C.c_uint64, C.c_double, P, P]
        L.orc_decompress_slice_mode.argtypes = [P, C.c_uint64, C.c_double, C.c_uint32, P, P]
        L.orc_norm.argtypes = [C.c_int, P, P, P]
        L.orc_norm.restype = C.c_double
        L.orc_norm_mode.argtypes = [C.c_int, P, P, P, C.c_uint32]
        L.orc_norm_mode.restype = C.c_double
        L.orc_rsqrt.argtypes = [C.c_double]
        L.orc_rsqrt.restype = C.c_double
        L.orc_sim_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_uint32]
        L.orc_sim_create.restype = C.c_void_p
        L.orc_sim_destroy.argtypes = [C.c_void_p]
        L.orc_sim_init.argtypes = [C.c_void_p, C.c_int, C.c_uint64, P]
        L.orc_sim_apply.argtypes = [C.c_void_p, C.POINTER(_Gate), C.c_uint64, C.POINTER(C.c_uint64)]
        L.orc_sim_scale.argtypes = [C.c_void_p]
        L.orc_sim_scale.restype = C.c_double
        L.orc_sim_set_record.argtypes = [C.c_void_p, C.c_uint64, P, C.c_uint64]
        L.orc_sim_nslices.argtypes = [C.c_void_p]
        L.orc_sim_nslices.restype = C.c_uint64
        L.orc_sim_record_len.argtypes = [C.c_void_p, C.c_uint64]
        L.orc_sim_record_len.restype = C.c_uint64
        L.orc_sim_record.argtypes = [C.c_void_p, C.c_uint64, P, C.c_uint64]
        L.orc_sim_total_bytes.argtypes = [C.c_void_p]
        L.orc_sim_total_bytes.restype = C.c_uint64
        L.orc_sim_peak_bytes.argtypes = [C.c_void_p]
        L.orc_sim_peak_bytes.restype = C.c_uint64
        L.orc_sim_max_err.argtypes = [C.c_void_p]
        L.orc_sim_max_err.restype = C.c_double
        L.orc_sim_amplitudes.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, P]
        L.orc_pass_group.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_uint32, C.POINTER(_Gate),
                                     C.c_double, C.c_int, P, P, P, P, P]
        L.orc_group_apply.argtypes = [C.POINTER(_Gate), C.c_int, C.c_int, P, P, P]
        L.orc_plan.argtypes = [C.POINTER(_Gate), C.c_uint64, C.POINTER(_Pass), C.c_uint64, C.POINTER(C.c_uint64)]
        L.orc_block_matrix.argtypes = [C.POINTER(_Gate), C.POINTER(_Pass), P]
        L.orc_sim_apply_fused.argtypes = [C.c_void_p, C.POINTER(_Gate), C.c_uint64, C.POINTER(C.c_uint64)]
        L.orc_group_apply_local.argtypes = [C.POINTER(_Gate), C.c_int, C.c_int, P, P, P, C.c_int]
        L.orc_vsim_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_uint32]
        L.orc_vsim_create.restype = C.c_void_p
        L.orc_vsim_destroy.argtypes = [C.c_void_p]
        L.orc_vsim_init.argtypes = [C.c_void_p, C.c_int, C.c_uint64, P]
        L.orc_vsim_apply.argtypes = [C.c_void_p, C.POINTER(_Gate), C.c_uint64, C.POINTER(C.c_uint64)]
        L.orc_vsim_apply_fused.argtypes = [C.c_void_p, C.POINTER(_Gate), C.c_uint64, C.POINTER(C.c_uint64)]
        L.orc_vsim_amplitudes.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, P]
        L.orc_vsim_scale.argtypes = [C.c_void_p]
        L.orc_vsim_scale.restype = C.c_double
        L.orc_vsim_get.argtypes = [C.c_void_p, P, P, P, P]
        L.orc_vsim_set.argtypes = [C.c_void_p, P, P, P, P, C.c_uint64, C.c_double]
        L.orc_vsim_passes.argtypes = [C.c_void_p]
        L.orc_vsim_passes.restype = C.c_uint64
        L.orc_vsim_max_err.argtypes = [C.c_void_p]
        L.orc_vsim_max_err.restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


_libc = C.CDLL(None)
_libc.free.argtypes = [C.c_void_p]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _gate_struct(g) -> Tuple[_Gate, Optional[np.ndarray]]:
    s = _Gate()
    s.kind = g.kind
    s.n_targets = len(g.targets)
    for i, t in enumerate(g.targets):
        s.targets[i] = t
    s.ctrl_mask = g.ctrl_mask
    s.ctrl_vals = g.ctrl_vals
    ph = complex(g.phase)
    s.phase_re = ph.real
    s.phase_im = ph.imag
    keep = None
    if g.matrix is not None and g.kind == 1:
        keep = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128)).view(np.float64).copy()
        s.matrix = keep.ctypes.data_as(C.POINTER(C.c_double))
    return s, keep


def gate_array(gates: Sequence) -> Tuple[C.Array, list]:
    arr = (_Gate * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        s, k = _gate_struct(g)
        arr[i] = s
        keep.append(k)
    return arr, keep


# ------------------------------------------------------------ state vector

def sv_apply(n: int, psi: np.ndarray, gate, mode: int = 0) -> np.ndarray:
    """Apply one gate to an uncompressed state (returns a new array); mode
    FP32: the state holds FP32 values and the gate runs in FP32 arithmetic."""
    re = np.ascontiguousarray(psi.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(psi.imag, dtype=np.float64).copy()
    s, keep = _gate_struct(gate)
    rc = lib().orc_sv_apply_mode(n, _ptr(re), _ptr(im), C.byref(s), mode)
    if rc:
        raise OracleError(rc, "sv_apply")
    return re + 1j * im


def sv_run(n: int, gates: Sequence, psi0: Optional[np.ndarray] = None) -> np.ndarray:
    """Uncompressed FP64 simulation of a gate list (planes kept in place)."""
    if psi0 is None:
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[0] = 1
    re = np.ascontiguousarray(psi0.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(psi0.imag, dtype=np.float64).copy()
    L = lib()
    for g in gates:
        s, keep = _gate_struct(g)
        rc = L.orc_sv_apply(n, _ptr(re), _ptr(im), C.byref(s))
        if rc:
            raise OracleError(rc, "sv_apply")
    return re + 1j * im


def group_apply(gate, slice_log2: int, members: Sequence[int], planes: List[np.ndarray]) -> List[np.ndarray]:
    """Apply a gate to one slice group given as complex arrays (one per member)."""
    s, keep = _gate_struct(gate)
    m = len(members)
    re = [np.ascontiguousarray(p.real, dtype=np.float64).copy() for p in planes]
    im = [np.ascontiguousarray(p.imag, dtype=np.float64).copy() for p in planes]
    rp = (C.c_void_p * m)(*[a.ctypes.data for a in re])
    ip = (C.c_void_p * m)(*[a.ctypes.data for a in im])
    mem = np.array(members, dtype=np.uint64)
    rc = lib().orc_group_apply(C.byref(s), slice_log2, m, _ptr(mem), C.cast(rp, C.c_void_p), C.cast(ip, C.c_void_p))
    if rc:
        raise OracleError(rc, "group_apply")
    return [r + 1j * i for r, i in zip(re, im)]


def product_state(factors: np.ndarray) -> np.ndarray:
    """prod_q f_q(b_q) multiplied from (1, 0), qubit 0 first, with the same
    complex product order as the gates (the oracle's initial-state rule)."""
    n = factors.shape[0]
    N = 1 << n
    idx = np.arange(N, dtype=np.uint64)
    ar = np.ones(N)
    ai = np.zeros(N)
    for q in range(n):
        b = ((idx >> np.uint64(q)) & np.uint64(1)).astype(bool)
        fr = np.where(b, factors[q, 1].real, factors[q, 0].real)
        fi = np.where(b, factors[q, 1].imag, factors[q, 0].imag)
        pr = fr * ar
        pi = fi * ai
        qr = fr * ai
        qi = fi * ar
        ar = 0.0 + (pr - pi)
        ai = 0.0 + (qr + qi)
    return ar + 1j * ai


# ------------------------------------------------------------------ codec

def abs_step(eb: float) -> Tuple[float, float]:
    st, r = C.c_double(), C.c_double()
    lib().orc_abs_step(eb, C.byref(st), C.byref(r))
    return st.value, r.value


def rel_step(rel: float, values: np.ndarray) -> Tuple[float, float, float]:
    v = np.ascontiguousarray(values, dtype=np.float64)
    st, r, e = C.c_double(), C.c_double(), C.c_double()
    lib().orc_rel_step(rel, _ptr(v), v.size, C.byref(st), C.byref(r), C.byref(e))
    return st.value, r.value, e.value


def huffman_lengths(hist: Sequence[int], lmax: int = LMAX) -> np.ndarray:
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint64))
    lens = np.zeros(h.size, dtype=np.uint8)
    rc = lib().orc_huffman_lengths(_ptr(h), h.size, lmax, _ptr(lens))
    if rc:
        raise OracleError(rc, "huffman_lengths")
    return lens


def canonical_codes(lens: np.ndarray, lmax: int = LMAX) -> np.ndarray:
    l8 = np.ascontiguousarray(np.asarray(lens, dtype=np.uint8))
    codes = np.zeros(l8.size, dtype=np.uint32)
    lib().orc_canonical_codes(_ptr(l8), l8.size, lmax, _ptr(codes))
    return codes


def compress_slice(re: np.ndarray, im: np.ndarray, slice_log2: int, chunk_log2: int, eb: float,
                   mode: int = ABS) -> Tuple[bytes, dict]:
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    assert re.size == im.size == (1 << slice_log2)
    out = C.c_void_p()
    n = C.c_uint64()
    st = _CStats()
    rc = lib().orc_compress_slice(_ptr(re), _ptr(im), slice_log2, chunk_log2, eb, mode, C.byref(out),
                                  C.byref(n), C.byref(st))
    if rc:
        raise OracleError(rc, "compress_slice")
    data = C.string_at(out.value, n.value)
    _libc.free(out)
    stats = dict(max_err=st.max_err, n_escapes=st.n_escapes,
                 sumsq=(st.sumsq_hi << 64) | st.sumsq_lo, step=st.step)
    return data, stats


def decode_p(rec: bytes) -> np.ndarray:
    hdr = parse_header(rec)
    p = np.zeros(2 << hdr["slice_log2"], dtype=np.int64)
    buf = np.frombuffer(rec, dtype=np.uint8).copy()
    rc = lib().orc_decode_p(_ptr(buf), len(rec), _ptr(p))
    if rc:
        raise OracleError(rc, "decode_p")
    return p


def decompress_slice(rec: bytes, kscale: float, mode: int = 0) -> np.ndarray:
    hdr = parse_header(rec)
    L = 1 << hdr["slice_log2"]
    re = np.zeros(L)
    im = np.zeros(L)
    buf = np.frombuffer(rec, dtype=np.uint8).copy()
    rc = lib().orc_decompress_slice_mode(_ptr(buf), len(rec), kscale, mode, _ptr(re), _ptr(im))
    if rc:
        raise OracleError(rc, "decompress_slice")
    return re + 1j * im


def parse_header(rec: bytes) -> dict:
    """Header fields of a slice record (little-endian, 64 bytes)."""
    u32 = np.frombuffer(rec[:32], dtype="<u4")
    step = float(np.frombuffer(rec[32:40], dtype="<f8")[0])
    lo, hi = (int(x) for x in np.frombuffer(rec[40:56], dtype="<u8"))
    flags = int(np.frombuffer(rec[56:60], dtype="<u4")[0])
    pw_bits = int(np.frombuffer(rec[60:64], dtype="<u4")[0])
    return dict(magic=int(u32[0]), slice_log2=int(u32[1]), chunk_log2=int(u32[2]), n_used=int(u32[3]),
                n_chunks=int(u32[4]), n_words=int(u32[5]), n_escapes=int(u32[6]), total=int(u32[7]),
                step=step, sumsq=(hi << 64) | lo, flags=flags, pw_bits=pw_bits)


def chunk_offsets(rec: bytes) -> np.ndarray:
    """The n_chunks + 1 word offsets of a record's chunks."""
    h = parse_header(rec)
    o = 64 + ((2 * h["n_used"] + 3) & ~3)
    return np.frombuffer(rec[o:o + 4 * (h["n_chunks"] + 1)], dtype="<u4").astype(np.int64) & 0x7FFFFFFF


def chunk_runs(rec: bytes):
    """A chunk-run record's runs as (ends, word offsets with their marks), or
    None for a record with a plain offsets table."""
    h = parse_header(rec)
    if not h["flags"] & 8:
        return None
    o = 64 + ((2 * h["n_used"] + 3) & ~3)
    R = int(np.frombuffer(rec[o:o + 4], dtype="<u4")[0])
    ends = np.frombuffer(rec[o + 4:o + 4 + 4 * R], dtype="<u4").astype(np.int64)
    woff = np.frombuffer(rec[o + 4 + 4 * R:o + 8 + 8 * R], dtype="<u4").astype(np.int64)
    return ends, woff


def constant_chunks(rec: bytes) -> np.ndarray:
    """The chunks marked constant (bit 31 of their word offset)."""
    h = parse_header(rec)
    o = 64 + ((2 * h["n_used"] + 3) & ~3)
    return (np.frombuffer(rec[o:o + 4 * h["n_chunks"]], dtype="<u4") >> 31).astype(bool)


def symtab(rec: bytes) -> List[Tuple[int, int]]:
    h = parse_header(rec)
    e = np.frombuffer(rec[64:64 + 2 * h["n_used"]], dtype="<u2")
    return [(int(x) & 1023, int(x) >> 10) for x in e]


def norm(steps: np.ndarray, sumsq: Sequence[int], mode: int = 0) -> float:
    """N of the stored state from every slice's step and sum field (mode
    PWREL: the sum fields hold FP64 squared norms)."""
    st = np.ascontiguousarray(steps, dtype=np.float64)
    lo = np.array([int(s) & ((1 << 64) - 1) for s in sumsq], dtype=np.uint64)
    hi = np.array([int(s) >> 64 for s in sumsq], dtype=np.uint64)
    return lib().orc_norm_mode(st.size, _ptr(st), _ptr(lo), _ptr(hi), mode)


def rsqrt(N: float) -> float:
    return lib().orc_rsqrt(N)


def scale_from_records(records: Sequence[bytes]) -> float:
    """The normalisation of a stored state from its records (or their headers)."""
    hs = [parse_header(r) for r in records]
    pw = PWREL if any(h["flags"] & 4 for h in hs) else 0
    return rsqrt(norm(np.array([h["step"] for h in hs]), [h["sumsq"] for h in hs], pw))


def pass_group(n: int, slice_log2: int, chunk_log2: int, eb: float, mode: int, gate, scale: float,
               members: Sequence[int], records: Sequence[bytes]) -> List[bytes]:
    """Algorithm 1 for one slice group, from given input records."""
    s, keep = _gate_struct(gate)
    m = len(members)
    mem = np.array(members, dtype=np.uint64)
    bufs = [np.frombuffer(r, dtype=np.uint8).copy() for r in records]
    inp = (C.c_void_p * m)(*[b.ctypes.data for b in bufs])
    inl = np.array([len(r) for r in records], dtype=np.uint64)
    outp = (C.c_void_p * m)()
    outl = np.zeros(m, dtype=np.uint64)
    rc = lib().orc_pass_group(n, slice_log2, chunk_log2, eb, mode, C.byref(s), scale, m, _ptr(mem),
                              C.cast(inp, C.c_void_p), _ptr(inl), C.cast(outp, C.c_void_p), _ptr(outl))
    res = []
    for u in range(m):
        if outp[u]:
            if rc == 0:
                res.append(C.string_at(outp[u], int(outl[u])))
            _libc.free(outp[u])
    if rc:
        raise OracleError(rc, "pass_group")
    return res


def group_apply_local(gate, slice_log2: int, members: Sequence[int], planes: List[np.ndarray],
                      fp32: bool = False) -> List[np.ndarray]:
    """group_apply through the code-level runner's addressing (local index
    member * L + offset) instead of the search over members."""
    s, keep = _gate_struct(gate)
    m = len(members)
    re = [np.ascontiguousarray(p.real, dtype=np.float64).copy() for p in planes]
    im = [np.ascontiguousarray(p.imag, dtype=np.float64).copy() for p in planes]
    rp = (C.c_void_p * m)(*[a.ctypes.data for a in re])
    ip = (C.c_void_p * m)(*[a.ctypes.data for a in im])
    mem = np.array(members, dtype=np.uint64)
    rc = lib().orc_group_apply_local(C.byref(s), slice_log2, m, _ptr(mem), C.cast(rp, C.c_void_p),
                                     C.cast(ip, C.c_void_p), int(fp32))
    if rc:
        raise OracleError(rc, "group_apply_local")
    return [r + 1j * i for r, i in zip(re, im)]


def group_members(n: int, slice_log2: int, gate, j0: int) -> List[int]:
    bits = [t - slice_log2 for t in gate.targets if t >= slice_log2] if gate.kind == 1 else []
    mem = []
    for u in range(1 << len(bits)):
        j = j0
        for b, bit in enumerate(bits):
            if (u >> b) & 1:
                j |= 1 << bit
        mem.append(j)
    return mem


# ---------------------------------------------------------- fused passes

def plan(gates: Sequence) -> List[Tuple[int, int, bool, Tuple[int, ...]]]:
    """Fused-mode pass partition: (first gate, gate count, fused, qubits)."""
    arr, keep = gate_array(gates)
    n = C.c_uint64()
    lib().orc_plan(arr, len(gates), None, 0, C.byref(n))
    out = (_Pass * max(1, n.value))()
    rc = lib().orc_plan(arr, len(gates), out, n.value, C.byref(n))
    if rc:
        raise OracleError(rc, "plan")
    return [(p.first, p.count, bool(p.fused), tuple(p.qubits[i] for i in range(p.k))) for p in out[:n.value]]


def block_matrix(gates: Sequence, first: int, count: int, qubits: Sequence[int]) -> np.ndarray:
    """U = G_last ... G_first of gates[first:first + count] over `qubits`."""
    arr, keep = gate_array(gates)
    p = _Pass()
    p.first, p.count, p.fused, p.k = first, count, 1, len(qubits)
    for i, q in enumerate(qubits):
        p.qubits[i] = q
    dim = 1 << len(qubits)
    U = np.zeros(2 * dim * dim)
    rc = lib().orc_block_matrix(arr, C.byref(p), _ptr(U))
    if rc:
        raise OracleError(rc, "block_matrix")
    return (U[0::2] + 1j * U[1::2]).reshape(dim, dim)


# ------------------------------------------------------------- simulator

class OracleSim:
    """Algorithm 1 on the CPU with the oracle codec (plain mode)."""

    def __init__(self, n: int, slice_log2: int, chunk_log2: int, eb: float, mode: int = ABS):
        self.n, self.slice_log2, self.chunk_log2, self.eb, self.mode = n, slice_log2, chunk_log2, eb, mode
        self._h = lib().orc_sim_create(n, slice_log2, chunk_log2, eb, mode)
        if not self._h:
            raise OracleError(-1, "sim_create")
        rc = lib().orc_sim_init(self._h, 0, 0, None)
        if rc:
            raise OracleError(rc, "sim_init")

    def close(self):
        if self._h:
            lib().orc_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_basis(self, x: int):
        rc = lib().orc_sim_init(self._h, 1, x, None)
        if rc:
            raise OracleError(rc, "sim_init")

    def init_product(self, factors: np.ndarray):
        f = np.ascontiguousarray(np.asarray(factors, dtype=np.complex128)).view(np.float64).copy()
        rc = lib().orc_sim_init(self._h, 2, 0, _ptr(f))
        if rc:
            raise OracleError(rc, "sim_init")

    def apply(self, gates: Sequence, fused: bool = False) -> int:
        arr, keep = gate_array(gates)
        applied = C.c_uint64()
        fn = lib().orc_sim_apply_fused if fused else lib().orc_sim_apply
        rc = fn(self._h, arr, len(gates), C.byref(applied))
        if rc:
            raise OracleError(rc, f"sim_apply (after {applied.value} gates)")
        return applied.value

    @property
    def nslices(self) -> int:
        return int(lib().orc_sim_nslices(self._h))

    def record(self, j: int) -> bytes:
        n = int(lib().orc_sim_record_len(self._h, j))
        buf = np.zeros(n, dtype=np.uint8)
        rc = lib().orc_sim_record(self._h, j, _ptr(buf), n)
        if rc:
            raise OracleError(rc, "record")
        return buf.tobytes()

    def records(self) -> List[bytes]:
        return [self.record(j) for j in range(self.nslices)]

    def set_records(self, records: Sequence[bytes]):
        """Replace every stored record (a state built elsewhere)."""
        assert len(records) == self.nslices
        for j, r in enumerate(records):
            b = np.frombuffer(r, dtype=np.uint8).copy()
            rc = lib().orc_sim_set_record(self._h, j, _ptr(b), len(r))
            if rc:
                raise OracleError(rc, f"set_record {j}")

    def scale(self) -> float:
        return lib().orc_sim_scale(self._h)

    def amplitudes(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - begin
        out = np.zeros(2 * count)
        rc = lib().orc_sim_amplitudes(self._h, begin, count, _ptr(out))
        if rc:
            raise OracleError(rc, "amplitudes")
        return out[0::2] + 1j * out[1::2]

    def total_bytes(self) -> int:
        return int(lib().orc_sim_total_bytes(self._h))

    def peak_bytes(self) -> int:
        return int(lib().orc_sim_peak_bytes(self._h))

    def max_err(self) -> float:
        return float(lib().orc_sim_max_err(self._h))


class CodeSim:
    """Algorithm 1 at the level of the quantised codes (the lossless stages of
    the codec elided, since they return the codes they are given): the same
    amplitudes as OracleSim, for runs too long for the full codec.  Codes are
    held as int32 (a pass that needs more fails with ORC_EBOUND)."""

    def __init__(self, n: int, slice_log2: int, eb: float, mode: int = ABS):
        self.n, self.slice_log2, self.eb, self.mode = n, slice_log2, eb, mode
        self._h = lib().orc_vsim_create(n, slice_log2, eb, mode)
        if not self._h:
            raise OracleError(-2, "vsim_create")
        self._init(0, 0, None)

    def _init(self, kind, x, f):
        rc = lib().orc_vsim_init(self._h, kind, x, None if f is None else _ptr(f))
        if rc:
            raise OracleError(rc, "vsim_init")

    def close(self):
        if self._h:
            lib().orc_vsim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nslices(self) -> int:
        return 1 << (self.n - self.slice_log2)

    def init_basis(self, x: int):
        self._init(1, x, None)

    def init_product(self, factors: np.ndarray):
        self._init(2, 0, np.ascontiguousarray(np.asarray(factors, dtype=np.complex128)).view(np.float64).copy())

    def apply(self, gates: Sequence, fused: bool = False) -> int:
        arr, keep = gate_array(gates)
        applied = C.c_uint64()
        fn = lib().orc_vsim_apply_fused if fused else lib().orc_vsim_apply
        rc = fn(self._h, arr, len(gates), C.byref(applied))
        if rc:
            raise OracleError(rc, f"vsim_apply (after {applied.value} gates)")
        return applied.value

    def amplitudes(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - begin
        out = np.zeros(2 * count)
        rc = lib().orc_vsim_amplitudes(self._h, begin, count, _ptr(out))
        if rc:
            raise OracleError(rc, "vsim_amplitudes")
        return out[0::2] + 1j * out[1::2]

    def amplitude_words(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        """The read-out as interleaved (re, im) FP64 values (the layout of
        sim_amplitudes), without the complex conversion."""
        if count is None:
            count = (1 << self.n) - begin
        out = np.zeros(2 * count)
        rc = lib().orc_vsim_amplitudes(self._h, begin, count, _ptr(out))
        if rc:
            raise OracleError(rc, "vsim_amplitudes")
        return out

    def scale(self) -> float:
        return lib().orc_vsim_scale(self._h)

    def state(self) -> dict:
        S, L2 = self.nslices, 2 << self.slice_log2
        d = dict(codes=np.zeros((S, L2), dtype=np.int32), step=np.zeros(S), lo=np.zeros(S, dtype=np.uint64),
                 hi=np.zeros(S, dtype=np.uint64))
        lib().orc_vsim_get(self._h, _ptr(d["codes"]), _ptr(d["step"]), _ptr(d["lo"]), _ptr(d["hi"]))
        d["passes"] = int(lib().orc_vsim_passes(self._h))
        d["max_err"] = float(lib().orc_vsim_max_err(self._h))
        return d

    def set_state(self, d: dict):
        S, L2 = self.nslices, 2 << self.slice_log2
        codes = np.ascontiguousarray(d["codes"], dtype=np.int32)
        assert codes.shape == (S, L2)
        st = np.ascontiguousarray(d["step"], dtype=np.float64)
        lo = np.ascontiguousarray(d["lo"], dtype=np.uint64)
        hi = np.ascontiguousarray(d["hi"], dtype=np.uint64)
        lib().orc_vsim_set(self._h, _ptr(codes), _ptr(st), _ptr(lo), _ptr(hi), int(d["passes"]),
                           float(d["max_err"]))

    def codes(self, j: int) -> np.ndarray:
        return self.state()["codes"][j].astype(np.int64)

    @property
    def passes(self) -> int:
        return int(lib().orc_vsim_passes(self._h))

    def max_err(self) -> float:
        return float(lib().orc_vsim_max_err(self._h))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(t: int):
    lib().orc_set_threads(t)
