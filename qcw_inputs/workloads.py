"""Circuits of the paper's example workloads, built from the named gates.

* ghz_chain(nq): H on qubit 1, then CNOT from qubit 1 to each other qubit in
  turn (§5, MVn-Noise): |0..0> -> (|0..0> + |1..1>)/sqrt2.
* bell_and_inverse(): the Bell circuit CNOT_12 H_1 followed by its inverse
  H_1 CNOT_12 (§5, MV2-Noise): |00> -> |00>.
* grover(n, marked, iterations): textbook Grover search over the n "data"
  qubits 1..n (the paper lists Grover among its applications, §6d, without
  giving its circuit; this is the standard construction).  Start |0..0>,
  Hadamard on every data qubit, then `iterations` times: the oracle flips the
  sign of |marked>, and the diffusion reflects about the uniform state
  (H^n X^n C^{n-1}Z X^n H^n).  The sign flip of |1..1> on m qubits
  (C^{m-1}Z) is Z, CZ or CCZ for m <= 3; for m > 3 it is a Toffoli ladder onto
  m - 2 ancilla qubits n+1..2n-2 (left in |0>), a CZ, and the ladder undone.
  With N = 2^n and sin(theta) = N^(-1/2), the marked amplitude after k
  iterations is (-1)^k sin((2k+1) theta) and every other data amplitude
  (-1)^k cos((2k+1) theta) / sqrt(N-1): the oracle is I - 2|w><w| and the
  diffusion as built is I - 2|s><s|, so each iteration is minus the textbook
  Grover operator.

Only gate lists are built here; no gate is applied.
"""
from __future__ import annotations

import math

import numpy as np

from . import CNOT, CZ, TOFFOLI, Circuit, H, X, Z

CCZ = np.diag([1, 1, 1, 1, 1, 1, 1, -1]).astype(np.complex128)


def ghz_chain(nq: int) -> Circuit:
    c = Circuit(nq).add(H, 1)
    for t in range(2, nq + 1):
        c.add(CNOT, 1, t)
    return c


def bell_and_inverse() -> Circuit:
    return Circuit(2).add(H, 1).add(CNOT, 1, 2).add(CNOT, 1, 2).add(H, 1)


def grover_qubits(n: int) -> int:
    """Qubits of grover(n, ...): the n data qubits, plus the n - 2 ancillas of
    the Toffoli ladder when n > 3."""
    return n if n <= 3 else 2 * n - 2


def _sign_flip_all_ones(c: Circuit, qs: list[int], anc: list[int]) -> None:
    """Multiply |1..1> on qubits qs by -1 (C^{m-1}Z)."""
    m = len(qs)
    if m == 1:
        c.add(Z, qs[0])
    elif m == 2:
        c.add(CZ, qs[0], qs[1])
    elif m == 3:
        c.add(CCZ, *qs)
    else:
        # ladder: anc[0] = q0 q1, anc[i] = anc[i-1] q_{i+1}, ..., anc[m-3]
        c.add(TOFFOLI, qs[0], qs[1], anc[0])
        for i in range(1, m - 2):
            c.add(TOFFOLI, anc[i - 1], qs[i + 1], anc[i])
        c.add(CZ, anc[m - 3], qs[m - 1])
        for i in range(m - 3, 0, -1):
            c.add(TOFFOLI, anc[i - 1], qs[i + 1], anc[i])
        c.add(TOFFOLI, qs[0], qs[1], anc[0])


def grover(n: int, marked: int, iterations: int) -> Circuit:
    """Grover search for the data basis state `marked` (0 <= marked < 2^n, the
    data qubits' bits MSB first), on grover_qubits(n) qubits."""
    if n < 1 or not 0 <= marked < (1 << n):
        raise ValueError("bad n or marked")
    nq = grover_qubits(n)
    data = list(range(1, n + 1))
    anc = list(range(n + 1, nq + 1))
    c = Circuit(nq)
    for q in data:
        c.add(H, q)
    zeros = [q for q in data if not (marked >> (n - q)) & 1]
    for _ in range(iterations):
        for q in zeros:                       # oracle: |marked> -> -|marked>
            c.add(X, q)
        _sign_flip_all_ones(c, data, anc)
        for q in zeros:
            c.add(X, q)
        for q in data:                        # diffusion
            c.add(H, q)
        for q in data:
            c.add(X, q)
        _sign_flip_all_ones(c, data, anc)
        for q in data:
            c.add(X, q)
        for q in data:
            c.add(H, q)
    return c


def grover_amplitudes(n: int, iterations: int) -> tuple[float, float]:
    """(marked, other) data amplitudes after `iterations` rounds (ancillas |0>)."""
    theta = math.asin(1.0 / math.sqrt(1 << n))
    sign = -1.0 if iterations % 2 else 1.0
    a = sign * math.sin((2 * iterations + 1) * theta)
    b = sign * math.cos((2 * iterations + 1) * theta) / math.sqrt((1 << n) - 1)
    return a, b


def grover_optimal_iterations(n: int) -> int:
    """floor(pi / (4 theta)), the usual choice."""
    theta = math.asin(1.0 / math.sqrt(1 << n))
    return int(math.floor(math.pi / (4 * theta)))
