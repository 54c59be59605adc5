"""Host-only checks of the C ABI boundary: the library loads, exports every
entry point include/cqsim.h declares, and the binding's structure layouts
match the header as a C compiler sees it.  No kernel is launched."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

import paper_1811_05630_amd as cq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cqsim.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:sim|srv)_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(cq.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(cq.LIB_PATH):
        pytest.skip("libcqsim.so not built (run __graft_entry__.build())")
    L = C.CDLL(cq.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", cq.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT ((?:sim|srv)_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "cqsim.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("sim_gate %zu\n", sizeof(sim_gate));
  printf("sim_config %zu\n", sizeof(sim_config));
  printf("sim_stats_t %zu\n", sizeof(sim_stats_t));
  printf("sim_pass %zu\n", sizeof(sim_pass));
  F(sim_pass, n_qubits); F(sim_pass, qubits);
  F(sim_gate, targets); F(sim_gate, ctrl_mask); F(sim_gate, params); F(sim_gate, matrix);
  F(sim_config, error_bound); F(sim_config, workspace_bytes); F(sim_config, alloc); F(sim_config, stream);
  F(sim_config, arena_bytes);
  F(sim_stats_t, ratio); F(sim_stats_t, max_abs_codec_err); F(sim_stats_t, workspace_slots);
  F(sim_stats_t, device_bytes); F(sim_stats_t, min_slice_ratio); F(sim_stats_t, gates);
  printf("srv_job %zu\n", sizeof(srv_job));
  printf("srv_done %zu\n", sizeof(srv_done));
  F(srv_job, family); F(srv_job, basis); F(srv_job, factors); F(srv_job, gates); F(srv_job, n_gates);
  F(srv_job, out); F(srv_job, out_count);
  F(srv_done, status); F(srv_done, applied); F(srv_done, t_submit); F(srv_done, stats); F(srv_done, error);
  return 0;
}
"""


def test_struct_layouts_match_header():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write(LAYOUT_C)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), "-o", exe, src], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.strip().splitlines())
    py = {
        "sim_gate": C.sizeof(cq.GateStruct), "sim_config": C.sizeof(cq.ConfigStruct),
        "sim_stats_t": C.sizeof(cq.StatsStruct), "sim_pass": C.sizeof(cq.PassStruct),
        "sim_pass.n_qubits": cq.PassStruct.n_qubits.offset, "sim_pass.qubits": cq.PassStruct.qubits.offset,
        "sim_gate.targets": cq.GateStruct.targets.offset, "sim_gate.ctrl_mask": cq.GateStruct.ctrl_mask.offset,
        "sim_gate.params": cq.GateStruct.params.offset, "sim_gate.matrix": cq.GateStruct.matrix.offset,
        "sim_config.error_bound": cq.ConfigStruct.error_bound.offset,
        "sim_config.workspace_bytes": cq.ConfigStruct.workspace_bytes.offset,
        "sim_config.alloc": cq.ConfigStruct.alloc.offset, "sim_config.stream": cq.ConfigStruct.stream.offset,
        "sim_config.arena_bytes": cq.ConfigStruct.arena_bytes.offset,
        "sim_stats_t.ratio": cq.StatsStruct.ratio.offset,
        "sim_stats_t.max_abs_codec_err": cq.StatsStruct.max_abs_codec_err.offset,
        "sim_stats_t.workspace_slots": cq.StatsStruct.workspace_slots.offset,
        "sim_stats_t.device_bytes": cq.StatsStruct.device_bytes.offset,
        "sim_stats_t.min_slice_ratio": cq.StatsStruct.min_slice_ratio.offset,
        "sim_stats_t.gates": cq.StatsStruct.gates.offset,
        "srv_job": C.sizeof(cq.SrvJobStruct), "srv_done": C.sizeof(cq.SrvDoneStruct),
        **{f"srv_job.{f}": getattr(cq.SrvJobStruct, f).offset
           for f in ("family", "basis", "factors", "gates", "n_gates", "out", "out_count")},
        **{f"srv_done.{f}": getattr(cq.SrvDoneStruct, f).offset
           for f in ("status", "applied", "t_submit", "stats", "error")},
    }
    assert {k: int(v) for k, v in got.items()} == py
    assert py["sim_gate"] == 80
    assert py["sim_pass"] == 40


def test_binding_converts_gates_without_the_device():
    import numpy as np
    import qcircuits as qc
    arr, keep = cq.gate_array([qc.H(3), qc.CP(1, 4, 0.25), qc.SWAP(0, 7)])
    assert arr[0].kind == cq.GATE_DENSE and arr[0].n_targets == 1 and arr[0].targets[0] == 3
    assert arr[1].kind == cq.GATE_PHASE and arr[1].ctrl_mask == 0b10010
    assert abs(complex(arr[1].params[0], arr[1].params[1]) - complex(np.cos(0.25), np.sin(0.25))) < 1e-15
    m = np.ctypeslib.as_array(arr[2].matrix, shape=(32,))
    assert m[2 * (1 * 4 + 2)] == 1.0  # SWAP row 1, column 2


def test_named_kinds_marshal_their_params():
    g = cq.Named(cq.GATE_U3, (5,), (0.1, 0.2, 0.3), ctrl_mask=1, ctrl_vals=1)
    arr, keep = cq.gate_array([g, cq.Named(cq.GATE_CZ, (1, 2))])
    assert arr[0].kind == cq.GATE_U3 and arr[0].n_targets == 1 and arr[0].targets[0] == 5
    assert list(arr[0].params) == [0.1, 0.2, 0.3] and not arr[0].matrix
    assert arr[1].kind == cq.GATE_CZ and arr[1].n_targets == 2


def test_plan_expands_named_kinds_without_the_device():
    """sim_plan_qubits is host code: named kinds plan like the gates they stand for."""
    if not os.path.exists(cq.LIB_PATH):
        pytest.skip("libcqsim.so not built")
    import qcircuits as qc
    named = [cq.Named(cq.GATE_H, (0,)), cq.Named(cq.GATE_CP, (0, 1), (0.5,)), cq.Named(cq.GATE_SWAP, (2, 7)),
             cq.Named(cq.GATE_MCZ, (0, 1, 2, 3, 4, 5)[:5])]
    plain = [qc.H(0), qc.CP(0, 1, 0.5), qc.SWAP(2, 7), qc.MCPHASE(0b11111, 0b11111, -1)]
    assert cq.plan(10, named) == cq.plan(10, plain)
    with pytest.raises(cq.SimError) as e:
        cq.plan(10, [cq.Named(cq.GATE_CZ, (3,))])
    assert e.value.rc == -1


def test_circuit_slices_point_into_one_marshalled_array():
    import ctypes as C
    import qcircuits as qc
    gates = [qc.H(q) for q in range(6)] + [qc.CP(1, 4, 0.5), qc.SWAP(0, 5)]
    circ = cq.Circuit(gates)
    assert len(circ) == 8
    base = C.addressof(circ.pointer().contents)
    sub = circ[2:7][1:3]  # gates 3 and 4
    assert len(sub) == 2
    assert C.addressof(sub.pointer().contents) == base + 3 * C.sizeof(cq.GateStruct)
    assert sub.pointer()[0].targets[0] == 3 and sub.pointer()[1].targets[0] == 4
    assert len(circ[7:100]) == 1 and len(circ[5:2]) == 0
    with pytest.raises(ValueError):
        circ[::2]


def test_no_device_means_a_loud_failure():
    """Without a GPU the library refuses to run (no CPU fallback)."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    if not os.path.exists(cq.LIB_PATH):
        pytest.skip("libcqsim.so not built")
    with pytest.raises(cq.SimError) as e:
        cq.Sim(4, 2, 1e-6, use_torch=False)
    assert e.value.rc == -5


def test_footprint_without_the_device():
    """sim_footprint is host arithmetic: arenas count twice, the workspace
    budget bounds the slot buffers, bad configurations are refused."""
    if not os.path.exists(cq.LIB_PATH):
        pytest.skip("libcqsim.so not built")
    base = cq.footprint(14, 10, 1e-6, arena_bytes=1 << 20)
    assert cq.footprint(14, 10, 1e-6, arena_bytes=3 << 20) - base == 2 * (2 << 20)
    assert cq.footprint(15, 10, 1e-6, arena_bytes=1 << 20) > base
    small = cq.footprint(14, 10, 1e-6, arena_bytes=1 << 20, workspace_bytes=1)  # one slot
    assert small < base
    # FP32 changes the raw size only, not the buffers of a handle
    assert cq.footprint(14, 10, 1e-6, arena_bytes=1 << 20, fp32=True) == base
    with pytest.raises(cq.SimError) as e:
        cq.footprint(14, 15, 1e-6)
    assert e.value.rc == -1


def test_server_without_a_device_fails_loudly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    if not os.path.exists(cq.LIB_PATH):
        pytest.skip("libcqsim.so not built")
    with pytest.raises(cq.SimError) as e:
        cq.Server(1 << 30, 2)
    assert e.value.rc == -5
