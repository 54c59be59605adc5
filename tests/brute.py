"""Independent brute-force references used to pin the oracle.

Full 2^n x 2^n operators are assembled from Kronecker products of 2x2 matrix
units (numpy.kron), a different route from the oracle's index arithmetic.
Qubit q is kron factor n-1-q (qubit 0 is the least significant index bit).
"""
import heapq
import itertools
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)


def unit(r, c):
    m = np.zeros((2, 2), dtype=np.complex128)
    m[r, c] = 1
    return m


def kron_all(ops_by_qubit, n):
    out = np.ones((1, 1), dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        out = np.kron(out, ops_by_qubit.get(q, I2))
    return out


def control_projector(n, mask, vals):
    ops = {}
    for q in range(n):
        if (mask >> q) & 1:
            v = (vals >> q) & 1
            ops[q] = unit(v, v)
    return kron_all(ops, n)


def full_operator(gate, n):
    """2^n x 2^n matrix of one gate (dense with controls, or a phase on a pattern)."""
    N = 1 << n
    if gate.kind == 2:  # phase on every index matching the pattern
        P = control_projector(n, gate.ctrl_mask, gate.ctrl_vals)
        return np.eye(N, dtype=np.complex128) + (complex(gate.phase) - 1) * P
    k = len(gate.targets)
    U = np.zeros((N, N), dtype=np.complex128)
    for r in range(1 << k):
        for c in range(1 << k):
            if gate.matrix[r, c] == 0:
                continue
            ops = {}
            for q in range(n):
                if (gate.ctrl_mask >> q) & 1:
                    v = (gate.ctrl_vals >> q) & 1
                    ops[q] = unit(v, v)
            for i, t in enumerate(gate.targets):
                ops[t] = unit((r >> i) & 1, (c >> i) & 1)
            U += gate.matrix[r, c] * kron_all(ops, n)
    if gate.ctrl_mask:
        P = control_projector(n, gate.ctrl_mask, gate.ctrl_vals)
        U += np.eye(N, dtype=np.complex128) - P
    return U


def huffman_cost(weights):
    """Textbook Huffman: total cost = sum of all merged weights (heap of weights)."""
    w = [int(x) for x in weights if x > 0]
    if len(w) <= 1:
        return 0
    heapq.heapify(w)
    cost = 0
    while len(w) > 1:
        a = heapq.heappop(w)
        b = heapq.heappop(w)
        cost += a + b
        heapq.heappush(w, a + b)
    return cost


def best_limited_cost(weights, lmax):
    """Exhaustive search over all length vectors in [1, lmax]^n with Kraft sum <= 1."""
    w = [int(x) for x in weights]
    n = len(w)
    if n == 1:
        return 0
    best = None
    for ls in itertools.product(range(1, lmax + 1), repeat=n):
        if sum(2.0 ** -l for l in ls) > 1.0:
            continue
        c = sum(a * b for a, b in zip(w, ls))
        if best is None or c < best:
            best = c
    return best


def grover_closed_form(n, marked, k):
    """Amplitudes after the initial H layer and k iterations of oracle + diffusion
    H X MCZ X H, which is -(2|s><s| - I): (-1)^k times the textbook values."""
    N = 1 << n
    theta = math.asin(1 / math.sqrt(N))
    sgn = -1.0 if k % 2 else 1.0
    good = sgn * math.sin((2 * k + 1) * theta)
    bad = sgn * math.cos((2 * k + 1) * theta) / math.sqrt(N - 1)
    psi = np.full(N, bad, dtype=np.complex128)
    psi[marked] = good
    return psi


def qft_basis_closed_form(n, x):
    N = 1 << n
    y = np.arange(N)
    return np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)


class QftProductExact:
    """Exact QFT of a product state, a block of 2^m output indices at a time.

    QFT maps psi to sqrt(N) * ifft(psi); for psi(x) = prod_q f_q(x_q) the sum
    over x factorises: out(y) = prod_q (f_q(0) + f_q(1) w^(2^q y)) / sqrt 2 with
    w = exp(2 pi i / N).  Write y = hi 2^m + lo: for q >= n - m the factor
    depends on lo alone (2^q hi 2^m is a multiple of N), so their product is
    one vector over lo; for q < n - m, w^(2^q y) = w^(2^(q+m) hi) w^(2^q lo)."""

    def __init__(self, factors, m):
        f = np.asarray(factors, dtype=np.complex128)
        self.n, self.m = len(f), m
        n, N = self.n, 1 << self.n
        self.f = f
        lo = np.arange(1 << m, dtype=np.int64)
        self.low = np.ones(1 << m, dtype=np.complex128)
        self.e = {}
        for q in range(n):
            ang = (2 * math.pi / N) * ((lo << q) & (N - 1)).astype(np.float64)
            e = np.cos(ang) + 1j * np.sin(ang)
            if q >= n - m:
                self.low *= (f[q, 0] + f[q, 1] * e) / math.sqrt(2)
            else:
                self.e[q] = e

    def block(self, hi):
        """Amplitudes at y = hi 2^m .. hi 2^m + 2^m - 1."""
        n, N = self.n, 1 << self.n
        out = self.low.copy()
        t = np.empty_like(out)
        for q, e in self.e.items():
            k = (hi << (q + self.m)) & (N - 1)
            c = complex(math.cos(2 * math.pi * k / N), math.sin(2 * math.pi * k / N))
            np.multiply(e, self.f[q, 1] * c, out=t)
            t += self.f[q, 0]
            t *= 1 / math.sqrt(2)
            out *= t
        return out
