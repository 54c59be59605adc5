"""cqsim: compressed full-amplitude quantum circuit simulation on one MI355X.

Python binding of ``libcqsim.so`` (the C ABI of ``include/cqsim.h``).  This
module only marshals arguments: every step of the per-gate, per-slice loop --
Decompress, Normalize, GateComputation, Compress (Algorithm 1, Section II of
Wu et al., "Memory-Efficient Quantum Circuit Simulation by Using Lossy Data
Compression") -- runs in the library's HIP kernels on gfx950.  PyTorch, when
present, provides the device memory (its caching allocator) and the stream.

There is no CPU fallback: if the library is missing or no gfx950 device is
usable, the constructor raises.
"""
from __future__ import annotations

import ctypes as C
import weakref
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcqsim.so")

SIM_EB_ABS = 0x0
SIM_EB_REL = 0x1
SIM_FP32 = 0x2
SIM_FUSED = 0x4
SIM_ZERO_CHUNKS = 0x8
SIM_CONST_CHUNKS = 0x10
SIM_EB_PWREL = 0x20
SIM_CHUNK_RUNS = 0x40
SIM_OPT = 0x80
GATE_DENSE = 1
GATE_PHASE = 2
# named kinds (include/cqsim.h): matrices and phases made by the library from params
GATE_H, GATE_X, GATE_Z, GATE_P, GATE_CP, GATE_CZ, GATE_SWAP, GATE_U3, GATE_MCZ, GATE_U1Q = range(3, 13)

ERRORS = {-1: "SIM_EINVAL", -2: "SIM_ENOMEM", -3: "SIM_EBOUND", -4: "SIM_ECORRUPT", -5: "SIM_EDEVICE"}

# every entry point declared in include/cqsim.h
EXPORTS = ("sim_create", "sim_create_ex", "sim_destroy", "sim_last_error", "sim_init_basis", "sim_init_product",
           "sim_set_allocator", "sim_set_stream", "sim_apply", "sim_apply_noalloc", "sim_amplitudes", "sim_probabilities", "sim_stats",
           "sim_record_size", "sim_record_headers", "sim_export_slice", "sim_import_slice", "sim_kernel_times", "sim_plan", "sim_plan_qubits",
           "sim_graph_create", "sim_graph_launch", "sim_graph_destroy", "sim_footprint",
           "sim_tune_chunk", "srv_create", "srv_submit", "srv_wait", "srv_clock", "srv_projected_bytes",
           "srv_destroy")

SRV_INIT_ZERO, SRV_INIT_BASIS, SRV_INIT_PRODUCT = 0, 1, 2
SRV_FAMILIES = 16


class SimError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"{ERRORS.get(rc, rc)}: {msg}")
        self.rc = rc


class GateStruct(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("n_targets", C.c_uint32), ("targets", C.c_uint32 * 5),
                ("reserved", C.c_uint32), ("ctrl_mask", C.c_uint64), ("ctrl_vals", C.c_uint64),
                ("params", C.c_double * 3), ("matrix", C.POINTER(C.c_double))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ConfigStruct(C.Structure):
    _fields_ = [("n_qubits", C.c_int), ("slice_log2", C.c_int), ("chunk_log2", C.c_int),
                ("error_bound", C.c_double), ("mode", C.c_uint32), ("workspace_bytes", C.c_uint64),
                ("alloc", ALLOC_FN), ("free_fn", FREE_FN), ("alloc_ctx", C.c_void_p), ("stream", C.c_void_p),
                ("arena_bytes", C.c_uint64)]


class PassStruct(C.Structure):
    _fields_ = [("first_gate", C.c_uint32), ("n_gates", C.c_uint32), ("fused", C.c_uint32),
                ("n_qubits", C.c_uint32), ("qubits", C.c_uint32 * 5), ("reserved", C.c_uint32)]


class StatsStruct(C.Structure):
    _fields_ = [("raw_bytes", C.c_uint64), ("compressed_bytes", C.c_uint64), ("peak_compressed", C.c_uint64),
                ("ratio", C.c_double), ("min_ratio", C.c_double), ("passes", C.c_uint64),
                ("escapes", C.c_uint64), ("last_norm", C.c_double), ("max_abs_codec_err", C.c_double),
                ("elapsed_s", C.c_double), ("arena_bytes", C.c_uint64), ("workspace_slots", C.c_uint64),
                ("device_bytes", C.c_uint64), ("min_slice_ratio", C.c_double), ("gates", C.c_uint64)]


class SrvJobStruct(C.Structure):
    _fields_ = [("cfg", ConfigStruct), ("family", C.c_uint32), ("init", C.c_uint32), ("basis", C.c_uint64),
                ("factors", C.c_void_p), ("gates", C.POINTER(GateStruct)), ("n_gates", C.c_size_t),
                ("out", C.c_void_p), ("out_begin", C.c_uint64), ("out_count", C.c_uint64)]


class SrvDoneStruct(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int), ("family", C.c_uint32), ("applied", C.c_uint64),
                ("projected_bytes", C.c_uint64), ("device_bytes", C.c_uint64), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_end", C.c_double), ("stats", StatsStruct),
                ("error", C.c_char * 160)]


_lib = None


def lib():
    """Load libcqsim.so (built in-tree by build.py); raises if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python {HERE}/build.py`")
        # A process can drive the GPU through one HIP runtime only.  PyTorch
        # ships its own libamdhip64.so.7; loading it first makes the library
        # bind to that same copy (same soname) instead of a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.sim_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_uint32, C.POINTER(P)]
        L.sim_create_ex.argtypes = [C.POINTER(ConfigStruct), C.POINTER(P)]
        L.sim_destroy.argtypes = [P]
        L.sim_destroy.restype = None
        L.sim_last_error.restype = C.c_char_p
        L.sim_init_basis.argtypes = [P, C.c_uint64]
        L.sim_init_product.argtypes = [P, P]
        L.sim_set_allocator.argtypes = [P, ALLOC_FN, FREE_FN, P]
        L.sim_set_stream.argtypes = [P, P]
        L.sim_apply.argtypes = [P, C.POINTER(GateStruct), C.c_size_t, C.POINTER(C.c_size_t)]
        L.sim_apply_noalloc.argtypes = [P, C.POINTER(GateStruct), C.c_size_t, C.POINTER(C.c_size_t)]
        L.sim_amplitudes.argtypes = [P, C.c_uint64, C.c_uint64, P]
        L.sim_probabilities.argtypes = [P, C.c_uint64, C.c_uint64, P]
        L.sim_stats.argtypes = [P, C.POINTER(StatsStruct)]
        L.sim_record_size.argtypes = [P, C.c_uint64]
        L.sim_record_size.restype = C.c_uint64
        L.sim_export_slice.argtypes = [P, C.c_uint64, P, C.c_uint64, C.POINTER(C.c_uint64)]
        L.sim_record_headers.argtypes = [P, C.c_uint64, C.c_uint64, P]
        L.sim_import_slice.argtypes = [P, C.c_uint64, P, C.c_uint64]
        L.sim_kernel_times.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_char_p)]
        L.sim_graph_create.argtypes = [P, C.POINTER(GateStruct), C.c_size_t, C.POINTER(P)]
        L.sim_graph_launch.argtypes = [P, P, C.POINTER(C.c_size_t)]
        L.sim_graph_destroy.argtypes = [P]
        L.sim_graph_destroy.restype = None
        L.sim_plan.argtypes = [P, C.POINTER(GateStruct), C.c_size_t, C.POINTER(PassStruct), C.c_size_t,
                               C.POINTER(C.c_size_t)]
        L.sim_plan_qubits.argtypes = [C.c_int, C.POINTER(GateStruct), C.c_size_t, C.POINTER(PassStruct), C.c_size_t,
                                      C.POINTER(C.c_size_t)]
        L.sim_footprint.argtypes = [C.POINTER(ConfigStruct), C.POINTER(C.c_uint64)]
        L.sim_tune_chunk.argtypes = [C.POINTER(ConfigStruct), C.POINTER(GateStruct), C.c_size_t, C.c_int, C.c_int,
                                     C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        L.srv_create.argtypes = [C.c_uint64, C.c_int, C.POINTER(P)]
        L.srv_submit.argtypes = [P, C.POINTER(SrvJobStruct), C.POINTER(C.c_uint64)]
        L.srv_wait.argtypes = [P, C.POINTER(SrvDoneStruct), C.c_size_t, C.POINTER(C.c_size_t), C.c_double]
        L.srv_clock.argtypes = [P]
        L.srv_clock.restype = C.c_double
        L.srv_projected_bytes.argtypes = [P, C.POINTER(SrvJobStruct), C.POINTER(C.c_uint64)]
        L.srv_destroy.argtypes = [P]
        L.srv_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise SimError(rc, f"{what}: {lib().sim_last_error().decode()}")


class Named:
    """A gate of a named kind (GATE_H .. GATE_U1Q): the library makes its
    matrix or phase from `params`."""

    def __init__(self, kind: int, targets: Sequence[int] = (), params: Sequence[float] = (), ctrl_mask: int = 0,
                 ctrl_vals: int = 0, matrix=None):
        self.kind, self.targets, self.params = int(kind), tuple(targets), tuple(params)
        self.ctrl_mask, self.ctrl_vals, self.matrix = ctrl_mask, ctrl_vals, matrix


def gate_struct(g) -> Tuple[GateStruct, Optional[np.ndarray]]:
    """sim_gate from any object with kind, targets, ctrl_mask, ctrl_vals and
    matrix or phase (DENSE / PHASE), or params (named kinds)."""
    s = GateStruct()
    s.kind = int(g.kind)
    tg = tuple(g.targets) if g.kind != GATE_PHASE else ()
    s.n_targets = len(tg)
    for i, t in enumerate(tg):
        s.targets[i] = int(t)
    s.ctrl_mask = int(g.ctrl_mask)
    s.ctrl_vals = int(g.ctrl_vals)
    if g.kind == GATE_PHASE:
        ph = complex(getattr(g, "phase", 1.0))
        s.params[0], s.params[1] = ph.real, ph.imag
    else:
        for i, v in enumerate(getattr(g, "params", ())[:3]):
            s.params[i] = float(v)
    keep = None
    if getattr(g, "matrix", None) is not None and g.kind in (GATE_DENSE, GATE_U1Q):
        keep = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128)).view(np.float64).copy()
        s.matrix = keep.ctypes.data_as(C.POINTER(C.c_double))
    return s, keep


def gate_array(gates: Sequence):
    arr = (GateStruct * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        s, k = gate_struct(g)
        arr[i] = s
        keep.append(k)
    return arr, keep


class Circuit:
    """Gates marshalled once into a sim_gate array (with the matrices they
    point to), so that applying them, or any contiguous range of them, does no
    per-gate Python work. Slicing with a step of 1 returns a view."""

    def __init__(self, gates: Sequence = (), _base=None, _start: int = 0, _n: int = 0):
        if _base is None:
            self._arr, self._keep = gate_array(gates)
            self._start, self._n = 0, len(gates)
        else:
            self._arr, self._keep = _base._arr, _base._keep
            self._start, self._n = _start, _n

    def __len__(self):
        return self._n

    def __getitem__(self, key):
        if not isinstance(key, slice):
            raise TypeError("Circuit supports slices only")
        a, b, step = key.indices(self._n)
        if step != 1:
            raise ValueError("Circuit slices need a step of 1")
        return Circuit(_base=self, _start=self._start + a, _n=max(0, b - a))

    def pointer(self):
        return C.cast(C.byref(self._arr, self._start * C.sizeof(GateStruct)), C.POINTER(GateStruct))


def _gate_ptr(gates):
    """(pointer, count, keep-alive) for a Circuit or any sequence of gates."""
    if isinstance(gates, Circuit):
        return gates.pointer(), len(gates), gates
    arr, keep = gate_array(gates)
    return C.cast(arr, C.POINTER(GateStruct)), len(gates), (arr, keep)


def plan(n_qubits, gates: Sequence) -> List[Tuple[int, int, bool, Tuple[int, ...]]]:
    """sim_plan (n_qubits a Sim) or sim_plan_qubits (n_qubits an int): the
    fused-mode passes as (first gate, gate count, fused, qubits)."""
    arr, keep = gate_array(gates)
    n = C.c_size_t()
    if isinstance(n_qubits, Sim):
        fn, first, name = lib().sim_plan, n_qubits._h, "sim_plan"
    else:
        fn, first, name = lib().sim_plan_qubits, int(n_qubits), "sim_plan_qubits"
    _check(fn(first, arr, len(gates), None, 0, C.byref(n)), name)
    out = (PassStruct * max(1, n.value))()
    _check(fn(first, arr, len(gates), out, n.value, C.byref(n)), name)
    return [(p.first_gate, p.n_gates, bool(p.fused), tuple(p.qubits[i] for i in range(p.n_qubits)))
            for p in out[:n.value]]


class _TorchMemory:
    """Device memory and stream from PyTorch (its caching allocator)."""

    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
                # The caching allocator may hand out a block whose last use is
                # still queued on torch's current stream; the library may run
                # on another stream (its own, when torch's is the null
                # stream), so that work must finish before the block is used.
                torch.cuda.current_stream().synchronize()
            except Exception:
                return None
            p = t.data_ptr()
            self.live[p] = t
            return p

        def _free(ptr, ctx):
            self.live.pop(ptr, None)

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)

    def stream(self):
        return self.torch.cuda.current_stream().cuda_stream


def _torch_ready() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


class Sim:
    """A compressed state of n qubits on the GPU (see include/cqsim.h)."""

    def __init__(self, n_qubits: int, slice_log2: int, error_bound: float, relative: bool = False,
                 chunk_log2: int = 0, workspace_bytes: int = 0, use_torch: Optional[bool] = None,
                 arena_bytes: int = 0, fused: bool = False, fp32: bool = False, zero_chunks: bool = False,
                 const_chunks: bool = False, allocator=None, pointwise: bool = False, chunk_runs: bool = False,
                 opt: bool = False):
        """allocator: optional (ALLOC_FN, FREE_FN) pair of device-memory hooks
        (sim_config.alloc / free_fn); the caller keeps them alive as long as
        the Sim.  Otherwise torch's caching allocator (when torch sees a
        device) or hipMalloc."""
        L = lib()
        cfg = _config(n_qubits, slice_log2, error_bound, relative=relative, chunk_log2=chunk_log2,
                      workspace_bytes=workspace_bytes, arena_bytes=arena_bytes, fused=fused, fp32=fp32,
                      zero_chunks=zero_chunks, const_chunks=const_chunks, pointwise=pointwise,
                      chunk_runs=chunk_runs, opt=opt)
        self._mem = None
        if use_torch is None:
            use_torch = _torch_ready()
        if allocator is not None:
            cfg.alloc, cfg.free_fn = allocator
            self._hooks = allocator
        elif use_torch:
            self._mem = _TorchMemory()
            cfg.alloc = self._mem.alloc
            cfg.free_fn = self._mem.free
            cfg.stream = self._mem.stream()
        h = C.c_void_p()
        self._h = None
        _check(L.sim_create_ex(C.byref(cfg), C.byref(h)), "sim_create")
        self._h = h
        self.n, self.slice_log2, self.error_bound, self.relative = n_qubits, slice_log2, error_bound, relative
        self.fused = fused
        self.fp32 = fp32
        self.zero_chunks = zero_chunks
        self.const_chunks = const_chunks
        self.pointwise = pointwise
        self.chunk_runs = chunk_runs
        self.opt = opt
        self.chunk_log2 = min(chunk_log2 or 10, slice_log2)

    def close(self):
        for g in list(getattr(self, "_graphs", ())):  # a graph must go before its handle
            g.close()
        if self._h:
            lib().sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def nslices(self) -> int:
        return 1 << (self.n - self.slice_log2)

    def init_basis(self, x: int):
        _check(lib().sim_init_basis(self._h, x), "sim_init_basis")

    def init_product(self, factors: np.ndarray):
        f = np.ascontiguousarray(np.asarray(factors, dtype=np.complex128)).view(np.float64).copy()
        assert f.size == 4 * self.n
        _check(lib().sim_init_product(self._h, f.ctypes.data_as(C.c_void_p)), "sim_init_product")

    def apply(self, gates: Sequence) -> int:
        """Apply a Circuit (or a sequence of gates, marshalled on each call)."""
        ptr, cnt, keep = _gate_ptr(gates)
        n = C.c_size_t()
        rc = lib().sim_apply(self._h, ptr, cnt, C.byref(n))
        if rc:
            raise SimError(rc, f"sim_apply after {n.value} gates: {lib().sim_last_error().decode()}")
        return n.value

    def apply_noalloc(self, gates: Sequence) -> Tuple[int, int]:
        """sim_apply_noalloc: the passes on the library's scratch array, with
        no device allocation; returns (status, gates applied)."""
        ptr, cnt, keep = _gate_ptr(gates)
        n = C.c_size_t()
        rc = lib().sim_apply_noalloc(self._h, ptr, cnt, C.byref(n))
        return rc, n.value

    def apply_partial(self, gates: Sequence) -> Tuple[int, int]:
        """Like apply, but returns (status, gates applied) instead of raising."""
        ptr, cnt, keep = _gate_ptr(gates)
        n = C.c_size_t()
        rc = lib().sim_apply(self._h, ptr, cnt, C.byref(n))
        return rc, n.value

    def amplitudes(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - begin
        out = np.zeros(2 * count)
        _check(lib().sim_amplitudes(self._h, begin, count, out.ctypes.data_as(C.c_void_p)), "sim_amplitudes")
        return out[0::2] + 1j * out[1::2]

    def probabilities(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - begin
        out = np.zeros(count)
        _check(lib().sim_probabilities(self._h, begin, count, out.ctypes.data_as(C.c_void_p)),
               "sim_probabilities")
        return out

    def stats(self) -> dict:
        st = StatsStruct()
        _check(lib().sim_stats(self._h, C.byref(st)), "sim_stats")
        return {k: getattr(st, k) for k, _ in StatsStruct._fields_}

    def record(self, j: int) -> bytes:
        n = int(lib().sim_record_size(self._h, j))
        buf = np.zeros(max(n, 1), dtype=np.uint8)
        ln = C.c_uint64()
        _check(lib().sim_export_slice(self._h, j, buf.ctypes.data_as(C.c_void_p), n, C.byref(ln)),
               "sim_export_slice")
        return buf[:ln.value].tobytes()

    def headers(self, first: int = 0, count: Optional[int] = None) -> List[bytes]:
        """The 64-byte headers of the stored records of slices [first, first + count)."""
        if count is None:
            count = self.nslices - first
        buf = np.zeros(64 * max(count, 1), dtype=np.uint8)
        _check(lib().sim_record_headers(self._h, first, count, buf.ctypes.data_as(C.c_void_p)),
               "sim_record_headers")
        b = buf.tobytes()
        return [b[64 * i:64 * (i + 1)] for i in range(count)]

    def records(self, which: Optional[Iterable[int]] = None) -> List[bytes]:
        return [self.record(j) for j in (range(self.nslices) if which is None else which)]

    def import_record(self, j: int, rec: bytes):
        b = np.frombuffer(rec, dtype=np.uint8).copy()
        _check(lib().sim_import_slice(self._h, j, b.ctypes.data_as(C.c_void_p), len(rec)), "sim_import_slice")

    def graph(self, gates: Sequence) -> "Graph":
        """sim_graph_create: the program captured once, to be applied with
        Graph.launch() as often as needed."""
        return Graph(self, gates)

    def kernel_times(self, enable: Optional[bool] = None) -> dict:
        """Per-kernel-class device time since the last reset, as
        {class: (milliseconds, launches)}; enable=True/False switches the event
        timing on/off (and resets the sums)."""
        out = (C.c_double * 64)()
        names = C.c_char_p()
        k = lib().sim_kernel_times(self._h, -1 if enable is None else int(bool(enable)), out, 64,
                                   C.byref(names))
        if k < 0:
            _check(k, "sim_kernel_times")
        cls = names.value.decode().split(",")
        return {cls[i]: (out[i], int(out[k + i])) for i in range(k)}


class Graph:
    """A gate program captured into a HIP graph on one Sim (sim_graph_*).
    launch() applies it to the Sim's current state, like Sim.apply."""

    def __init__(self, sim: "Sim", gates: Sequence):
        ptr, cnt, keep = _gate_ptr(gates)
        h = C.c_void_p()
        _check(lib().sim_graph_create(sim._h, ptr, cnt, C.byref(h)), "sim_graph_create")
        self._h, self.sim, self.n_gates = h, sim, cnt
        if not hasattr(sim, "_graphs"):
            sim._graphs = weakref.WeakSet()
        sim._graphs.add(self)

    def launch(self) -> int:
        n = C.c_size_t()
        rc = lib().sim_graph_launch(self.sim._h, self._h, C.byref(n))
        if rc:
            raise SimError(rc, f"sim_graph_launch after {n.value} gates: {lib().sim_last_error().decode()}")
        return n.value

    def close(self):
        if self._h:
            lib().sim_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _config(n_qubits: int, slice_log2: int, error_bound: float, relative: bool = False, chunk_log2: int = 0,
            workspace_bytes: int = 0, arena_bytes: int = 0, fused: bool = False, fp32: bool = False,
            zero_chunks: bool = False, const_chunks: bool = False, pointwise: bool = False,
            chunk_runs: bool = False, opt: bool = False) -> ConfigStruct:
    cfg = ConfigStruct()
    cfg.n_qubits = n_qubits
    cfg.slice_log2 = slice_log2
    cfg.chunk_log2 = chunk_log2
    cfg.error_bound = error_bound
    cfg.mode = ((SIM_EB_REL if relative else SIM_EB_ABS) | (SIM_FUSED if fused else 0) | (SIM_FP32 if fp32 else 0) |
                (SIM_ZERO_CHUNKS if zero_chunks else 0) | (SIM_CONST_CHUNKS if const_chunks else 0) |
                (SIM_EB_PWREL if pointwise else 0) | (SIM_CHUNK_RUNS if chunk_runs else 0) | (SIM_OPT if opt else 0))
    cfg.workspace_bytes = workspace_bytes
    cfg.arena_bytes = arena_bytes
    return cfg


def footprint(n_qubits: int, slice_log2: int, error_bound: float, **kw) -> int:
    """sim_footprint: device bytes a new Sim of this configuration holds (host-only)."""
    b = C.c_uint64()
    _check(lib().sim_footprint(C.byref(_config(n_qubits, slice_log2, error_bound, **kw)), C.byref(b)),
           "sim_footprint")
    return b.value


def tune_chunk(n_qubits: int, slice_log2: int, error_bound: float, gates: Sequence, lo: int = 5, hi: int = 10,
               **kw) -> Tuple[int, dict]:
    """sim_tune_chunk: the fastest chunk_log2 in [lo, hi] for this
    configuration and gate sample, and {chunk_log2: (ms per gate, record bytes)}."""
    cfg = _config(n_qubits, slice_log2, error_bound, **kw)
    ptr, cnt, keep = _gate_ptr(gates)
    k = hi - lo + 1
    ms = (C.c_double * max(k, 1))()  # a bad range is refused by the library
    by = (C.c_uint64 * max(k, 1))()
    best = C.c_int()
    _check(lib().sim_tune_chunk(C.byref(cfg), ptr, cnt, lo, hi, C.byref(best), ms, by), "sim_tune_chunk")
    return best.value, {lo + i: (ms[i], by[i]) for i in range(k)}


class Server:
    """A job server (srv_*): independent simulations run side by side on the
    device, admitted first come, first served within a device-memory budget.

    submit() queues a job and returns its id; wait() returns finished jobs as
    dicts (id, status, times on the server clock, statistics, and the
    requested amplitudes as a complex array)."""

    def __init__(self, budget_bytes: int, max_active: int = 4):
        h = C.c_void_p()
        self._h = None
        _check(lib().srv_create(int(budget_bytes), int(max_active), C.byref(h)), "srv_create")
        self._h = h
        self._keep = {}  # job id -> objects that must outlive the job (gates, factors, output)

    def _job(self, n_qubits, slice_log2, error_bound, gates=(), family=0, init="zero", basis=0, factors=None,
             out_count=0, out_begin=0, **cfg):
        j = SrvJobStruct()
        j.cfg = _config(n_qubits, slice_log2, error_bound, **cfg)
        j.family = family
        j.init = {"zero": SRV_INIT_ZERO, "basis": SRV_INIT_BASIS, "product": SRV_INIT_PRODUCT}[init]
        j.basis = basis
        keep = []
        if factors is not None:
            f = np.ascontiguousarray(np.asarray(factors, dtype=np.complex128)).view(np.float64).copy()
            assert f.size == 4 * n_qubits
            j.factors = f.ctypes.data_as(C.c_void_p)
            keep.append(f)
        if len(gates):
            ptr, cnt, k = _gate_ptr(gates)
            j.gates, j.n_gates = ptr, cnt
            keep.append(k)
        out = None
        if out_count:
            out = np.zeros(2 * out_count)
            j.out, j.out_begin, j.out_count = out.ctypes.data_as(C.c_void_p), out_begin, out_count
        return j, keep, out

    def submit(self, n_qubits: int, slice_log2: int, error_bound: float, gates: Sequence = (), **kw) -> int:
        """Queue a job.  Keywords: family, init ('zero' | 'basis' | 'product'),
        basis, factors, out_count / out_begin (amplitudes to return), and the
        Sim configuration (relative, chunk_log2, workspace_bytes, arena_bytes,
        fused, fp32)."""
        j, keep, out = self._job(n_qubits, slice_log2, error_bound, gates, **kw)
        i = C.c_uint64()
        _check(lib().srv_submit(self._h, C.byref(j), C.byref(i)), "srv_submit")
        self._keep[i.value] = (keep, out)
        return i.value

    def projected_bytes(self, n_qubits: int, slice_log2: int, error_bound: float, **kw) -> int:
        j, keep, out = self._job(n_qubits, slice_log2, error_bound, **kw)
        b = C.c_uint64()
        _check(lib().srv_projected_bytes(self._h, C.byref(j), C.byref(b)), "srv_projected_bytes")
        return b.value

    def clock(self) -> float:
        return lib().srv_clock(self._h)

    def wait(self, timeout: float = 0.0, cap: int = 256) -> List[dict]:
        buf = (SrvDoneStruct * cap)()
        n = C.c_size_t()
        _check(lib().srv_wait(self._h, buf, cap, C.byref(n), float(timeout)), "srv_wait")
        res = []
        for d in buf[:n.value]:
            r = {k: getattr(d, k) for k, _ in SrvDoneStruct._fields_ if k not in ("stats", "error")}
            r["stats"] = {k: getattr(d.stats, k) for k, _ in StatsStruct._fields_}
            r["error"] = d.error.decode()
            keep, out = self._keep.pop(d.id, (None, None))
            if out is not None:
                r["amplitudes"] = out[0::2] + 1j * out[1::2]
            res.append(r)
        return res

    def drain(self, timeout: float = 600.0) -> List[dict]:
        """Wait until every submitted job has finished; returns them all."""
        res = []
        while self._keep:
            got = self.wait(timeout)
            if not got:
                raise TimeoutError(f"jobs {sorted(self._keep)} not finished within {timeout} s")
            res += got
        return res

    def close(self):
        if self._h:
            lib().srv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
