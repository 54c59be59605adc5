"""Seeded synthetic inputs shared by the simulator and its test oracle.

This module only *describes* circuits and initial states: gate lists with
explicit FP64 matrices, and per-qubit factors of product states.  It holds
none of the compression method's arithmetic (no quantisation, no coding, no
gate application), so that both the HIP library and the CPU oracle can be fed
the very same numbers without sharing any of the code under test.

Conventions (the paper fixes none of them, Section II only says the program is
processed gate by gate):

* amplitude index ``i = sum_q b_q 2^q``; qubit 0 is the least significant bit;
* a dense gate on targets ``(t_0, .., t_{k-1})`` uses local index
  ``m = sum_k bit(i, t_k) 2^k`` and a row-major ``2^k x 2^k`` complex matrix;
* a phase gate multiplies amplitude ``i`` by one complex factor wherever
  ``i & ctrl_mask == ctrl_vals``;
* every matrix entry is computed here, on the host, once; numbers such as
  ``sqrt(1/2)`` are the correctly rounded FP64 values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

DENSE = 1
PHASE = 2

SQRT_HALF = math.sqrt(0.5)  # correctly rounded sqrt(1/2) = 0x1.6a09e667f3bcdp-1


@dataclass
class Gate:
    """One gate of a program, as the simulator applies it."""

    kind: int
    targets: Tuple[int, ...] = ()
    ctrl_mask: int = 0
    ctrl_vals: int = 0
    matrix: Optional[np.ndarray] = None  # complex128, 2^k x 2^k, row-major
    phase: complex = 1.0 + 0.0j
    name: str = ""

    def __post_init__(self):
        if self.kind == DENSE:
            k = len(self.targets)
            if not 1 <= k <= 5:
                raise ValueError("dense gates act on 1..5 targets")
            m = np.ascontiguousarray(np.asarray(self.matrix, dtype=np.complex128))
            if m.shape != (1 << k, 1 << k):
                raise ValueError("matrix shape does not match the number of targets")
            self.matrix = m
            tmask = 0
            for t in self.targets:
                tmask |= 1 << t
            if len(set(self.targets)) != k:
                raise ValueError("repeated target")
            if tmask & self.ctrl_mask:
                raise ValueError("controls overlap targets")
        elif self.kind == PHASE:
            self.targets = ()
        else:
            raise ValueError("unknown gate kind")
        if self.ctrl_vals & ~self.ctrl_mask:
            raise ValueError("control values outside the control mask")

    def max_qubit(self) -> int:
        q = -1
        for t in self.targets:
            q = max(q, t)
        if self.ctrl_mask:
            q = max(q, self.ctrl_mask.bit_length() - 1)
        return q


# ----------------------------------------------------------------- gate library

def H(t: int) -> Gate:
    s = SQRT_HALF
    return Gate(DENSE, (t,), matrix=np.array([[s, s], [s, -s]], dtype=np.complex128), name="H")


def X(t: int) -> Gate:
    return Gate(DENSE, (t,), matrix=np.array([[0, 1], [1, 0]], dtype=np.complex128), name="X")


def Z(t: int) -> Gate:
    return Gate(PHASE, ctrl_mask=1 << t, ctrl_vals=1 << t, phase=-1.0 + 0.0j, name="Z")


def P(t: int, theta: float) -> Gate:
    return Gate(PHASE, ctrl_mask=1 << t, ctrl_vals=1 << t,
                phase=complex(math.cos(theta), math.sin(theta)), name="P")


def CP(c: int, t: int, theta: float) -> Gate:
    m = (1 << c) | (1 << t)
    return Gate(PHASE, ctrl_mask=m, ctrl_vals=m, phase=complex(math.cos(theta), math.sin(theta)),
                name="CP")


def CZ(a: int, b: int) -> Gate:
    m = (1 << a) | (1 << b)
    return Gate(PHASE, ctrl_mask=m, ctrl_vals=m, phase=-1.0 + 0.0j, name="CZ")


def SWAP(a: int, b: int) -> Gate:
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = m[1, 2] = m[2, 1] = m[3, 3] = 1
    return Gate(DENSE, (a, b), matrix=m, name="SWAP")


def U3(t: int, theta: float, phi: float, lam: float) -> Gate:
    """OpenQASM 2 ``u3(theta, phi, lambda)``."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    m = np.array([[c, -complex(math.cos(lam), math.sin(lam)) * s],
                  [complex(math.cos(phi), math.sin(phi)) * s,
                   complex(math.cos(phi + lam), math.sin(phi + lam)) * c]], dtype=np.complex128)
    return Gate(DENSE, (t,), matrix=m, name="U3")


def U(targets: Sequence[int], matrix, ctrl_mask: int = 0, ctrl_vals: int = 0) -> Gate:
    return Gate(DENSE, tuple(targets), ctrl_mask=ctrl_mask, ctrl_vals=ctrl_vals, matrix=matrix,
                name="U")


def MCPHASE(mask: int, vals: int, phase: complex) -> Gate:
    return Gate(PHASE, ctrl_mask=mask, ctrl_vals=vals, phase=complex(phase), name="MCPHASE")


def MCZ(n: int) -> Gate:
    """-1 on |1...1> of n qubits."""
    m = (1 << n) - 1
    return Gate(PHASE, ctrl_mask=m, ctrl_vals=m, phase=-1.0 + 0.0j, name="MCZ")


# ------------------------------------------------------------------- circuits

def qft(n: int) -> List[Gate]:
    """Textbook QFT: for j = n-1..0: H(j), then CP(m, j, pi/2^(j-m)) for m = j-1..0;
    then SWAP(q, n-1-q) for q < n/2.  On this index convention it maps a state
    psi to sqrt(N) * ifft(psi) (numpy's inverse DFT)."""
    g: List[Gate] = []
    for j in range(n - 1, -1, -1):
        g.append(H(j))
        for m in range(j - 1, -1, -1):
            g.append(CP(m, j, math.pi / (1 << (j - m))))
    for q in range(n // 2):
        g.append(SWAP(q, n - 1 - q))
    return g


def grover_iterations(n: int) -> int:
    return int(math.floor(math.pi / 4 * math.sqrt(float(1 << n))))


def grover(n: int, marked: int, iterations: Optional[int] = None, initial_layer: bool = True) -> List[Gate]:
    """Grover search on n qubits for one marked index.

    Initial H on every qubit; each iteration is the oracle (phase -1 on the
    marked index) followed by the diffusion H^n X^n MCZ X^n H^n, each layer
    with qubits ascending.  This diffusion equals -(2|s><s| - I), so after k
    iterations the amplitudes are (-1)^k times the textbook ones."""
    if iterations is None:
        iterations = grover_iterations(n)
    full = (1 << n) - 1
    g: List[Gate] = []
    if initial_layer:
        g += [H(q) for q in range(n)]
    for _ in range(iterations):
        g.append(MCPHASE(full, marked, -1.0))
        g += [H(q) for q in range(n)]
        g += [X(q) for q in range(n)]
        g.append(MCZ(n))
        g += [X(q) for q in range(n)]
        g += [H(q) for q in range(n)]
    return g


def grover_passes(n: int, iterations: int) -> int:
    return n + iterations * (4 * n + 2)


def random_layered(n: int, depth: int, seed: int) -> List[Gate]:
    """Layers of U3 with angles ~ U[0, 2pi) on every qubit (ascending), then CZ on
    a seeded random perfect matching of the qubits (floor(n/2) disjoint pairs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g: List[Gate] = []
    for _ in range(depth):
        ang = rng.uniform(0.0, 2 * math.pi, size=(n, 3))
        for q in range(n):
            g.append(U3(q, float(ang[q, 0]), float(ang[q, 1]), float(ang[q, 2])))
        perm = rng.permutation(n)
        for k in range(n // 2):
            g.append(CZ(int(perm[2 * k]), int(perm[2 * k + 1])))
    return g


def inverse(gates: Sequence[Gate]) -> List[Gate]:
    """The inverse program (each gate's adjoint, reversed order)."""
    out: List[Gate] = []
    for gt in reversed(gates):
        if gt.kind == PHASE:
            out.append(Gate(PHASE, ctrl_mask=gt.ctrl_mask, ctrl_vals=gt.ctrl_vals,
                            phase=complex(gt.phase).conjugate(), name=gt.name + "^-1"))
        else:
            out.append(Gate(DENSE, gt.targets, ctrl_mask=gt.ctrl_mask, ctrl_vals=gt.ctrl_vals,
                            matrix=np.ascontiguousarray(gt.matrix.conj().T), name=gt.name + "^-1"))
    return out


# --------------------------------------------------------------- initial states

def basis_index(n: int, seed: int) -> int:
    rng = np.random.Generator(np.random.PCG64(seed))
    return int(rng.integers(0, 1 << n))


def product_angles(n: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """theta_q ~ U[0, pi], phi_q ~ U[0, 2pi) per qubit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(0.0, math.pi, size=n)
    phi = rng.uniform(0.0, 2 * math.pi, size=n)
    return theta, phi


def product_factors(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Per-qubit single-qubit states f_q = (cos(theta/2), e^{i phi} sin(theta/2)),
    as an (n, 2) complex128 array; the product state is prod_q f_q(b_q)."""
    n = len(theta)
    f = np.empty((n, 2), dtype=np.complex128)
    for q in range(n):
        c, s = math.cos(theta[q] / 2), math.sin(theta[q] / 2)
        f[q, 0] = c
        f[q, 1] = complex(math.cos(phi[q]) * s, math.sin(phi[q]) * s)
    return f


@dataclass
class Workload:
    """A named benchmark configuration: circuit family, sizes and error bound."""

    name: str
    n_qubits: int
    slice_log2: int
    error_bound: float
    relative: bool
    gates: List[Gate] = field(default_factory=list)
    init: str = "zero"  # "zero", "basis" or "product"
    basis: int = 0
    factors: Optional[np.ndarray] = None


def qft_basis_workload(n: int = 12, slice_log2: int = 10, eb: float = 1e-6, seed: int = 0) -> Workload:
    """12-qubit QFT of a seeded basis state, 4 slices of 1024 amplitudes, absolute bound 1e-6."""
    x = basis_index(n, seed)
    return Workload(f"qft{n}_basis", n, slice_log2, eb, False, qft(n), init="basis", basis=x)


def grover_workload(n: int = 24, slice_log2: int = 18, eb: float = 1e-7, seed: int = 0,
                    iterations: Optional[int] = None) -> Workload:
    """24-qubit Grover search, marked index from the seed, 64 slices of 2^18, absolute bound 1e-7."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = int(rng.integers(0, 1 << n))
    return Workload(f"grover{n}", n, slice_log2, eb, False, grover(n, w, iterations), init="zero",
                    basis=w)


def qft_product_workload(n: int = 30, slice_log2: int = 22, rel: float = 1e-4, seed: int = 0) -> Workload:
    theta, phi = product_angles(n, seed)
    return Workload(f"qft{n}_product", n, slice_log2, rel, True, qft(n), init="product",
                    factors=product_factors(theta, phi))
