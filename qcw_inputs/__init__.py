"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws numbers and builds constant gate tables.  It holds
none of the gate-sweep arithmetic (no gate is ever applied here), so that the
oracle under ``oracle/`` and the HIP library under ``paper_1101_1785_amd/``
can both consume identical bytes without sharing any code of the method.

Conventions (QCWAVE, Tabakin & Julia-Diaz, arXiv:1101.1785):

* An nq-qubit state is a complex128 vector of length N = 2**nq; amplitude n
  sits at offset n, and qubit 1 is the most significant bit of n (§2c,
  Eq. staten).  Qubit ``is`` therefore owns bit b = nq - is.
* A k-qubit gate is a dense m x m complex matrix (m = 2**k), row-major,
  U[r, c] = <r|U|c>, whose local index r = sum_j q_{is_j} 2**(k-j) takes the
  first listed target as its most significant bit (§3b, Eq. resmat2 and the
  V_{ij;kl} = <ij|V|kl> definition that follows it).
* A circuit is a list of gates in application order.

Draw recipe (all via numpy PCG64 ``default_rng`` seeded with integer lists,
so every stream is independent and reproducible):

* state(seed, nq, tag): chunks of 2**20 amplitudes; chunk c draws
  2*len uniforms on [0, 1) from default_rng([seed, tag, STATE, c]), maps them
  to U[-1, 1) as 2u - 1 (re, im interleaved) and the whole vector is scaled to
  unit 2-norm (the paper normalises every state, §2a-§2c).
* circuit(seed, nq, G, tag): one default_rng([seed, tag, CIRCUIT]) draws, per
  gate in order: k from {1: .50, 2: .35, 3: .15} restricted to k <= nq; the
  ordered targets rng.choice(nq, k, replace=False) + 1; then an m x m complex
  matrix with re/im uniform on [-1, 1) drawn row-major (re block then im
  block), made unitary by modified Gram-Schmidt over its columns.  Dense random
  unitaries play the part of the "general random rotation" the paper allows as
  a gate or noise operator (§5, error-correction subsection).
* batch(seed, count, nq_lo, nq_hi): instance i takes nq uniform on
  [nq_lo, nq_hi] (one draw from default_rng([seed, BATCH]) per instance), a
  state from state(seed, nq, 1000 + i) and a circuit from
  circuit(seed, nq, 4*nq, 1000 + i).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

STATE = 11
CIRCUIT = 23
BATCH = 37
ARRIVALS = 41
CHUNK_LOG2 = 20

K_PROBS = {1: 0.50, 2: 0.35, 3: 0.15}


def _threads() -> int:
    n = os.environ.get("OMP_NUM_THREADS")
    try:
        v = int(n) if n else (os.cpu_count() or 1)
    except ValueError:
        v = os.cpu_count() or 1
    return max(1, min(v, 16))


# ---------------------------------------------------------------- states
def state(seed: int, nq: int, tag: int = 0, threads: int | None = None) -> np.ndarray:
    """Normalised random nq-qubit state, complex128, length 2**nq."""
    if nq < 0 or nq > 34:
        raise ValueError("nq out of range")
    N = 1 << nq
    flat = np.empty(2 * N, dtype=np.float64)
    chunk = 1 << CHUNK_LOG2
    nchunks = (N + chunk - 1) // chunk

    def fill(c: int) -> float:
        lo = c * chunk
        hi = min(N, lo + chunk)
        seg = flat[2 * lo:2 * hi]
        np.random.default_rng([seed, tag, STATE, c]).random(out=seg)
        seg *= 2.0
        seg -= 1.0
        return float(np.dot(seg, seg))

    nt = threads or _threads()
    if nchunks == 1 or nt == 1:
        sums = [fill(c) for c in range(nchunks)]
    else:
        with ThreadPoolExecutor(nt) as ex:
            sums = list(ex.map(fill, range(nchunks)))
    norm = math.sqrt(math.fsum(sums))
    inv = 1.0 / norm

    def scale(c: int) -> None:
        lo = c * chunk
        hi = min(N, lo + chunk)
        flat[2 * lo:2 * hi] *= inv

    if nchunks == 1 or nt == 1:
        for c in range(nchunks):
            scale(c)
    else:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(scale, range(nchunks)))
    return flat.view(np.complex128)


def basis_state(nq: int, n: int) -> np.ndarray:
    """|n> in the computational basis (§2c, Eq. ampn)."""
    v = np.zeros(1 << nq, dtype=np.complex128)
    v[n] = 1.0
    return v


# ---------------------------------------------------------------- gates
def mgs_unitary(a: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt over the columns of a square complex matrix."""
    q = np.array(a, dtype=np.complex128, copy=True)
    m = q.shape[0]
    for j in range(m):
        for i in range(j):
            q[:, j] -= np.vdot(q[:, i], q[:, j]) * q[:, i]
        q[:, j] /= np.linalg.norm(q[:, j])
    return q


def random_unitary(rng: np.random.Generator, m: int) -> np.ndarray:
    re = rng.uniform(-1.0, 1.0, size=(m, m))
    im = rng.uniform(-1.0, 1.0, size=(m, m))
    return mgs_unitary(re + 1j * im)


def random_matrix(rng: np.random.Generator, m: int) -> np.ndarray:
    """A general (non-unitary) complex matrix; the sweep is linear in it."""
    re = rng.uniform(-1.0, 1.0, size=(m, m))
    im = rng.uniform(-1.0, 1.0, size=(m, m))
    return re + 1j * im


class Circuit:
    """Ordered gate list: ks[g], targets[g] (1-based, length ks[g]), mats[g]."""

    def __init__(self, nq: int):
        self.nq = nq
        self.ks: list[int] = []
        self.targets: list[tuple[int, ...]] = []
        self.mats: list[np.ndarray] = []

    def add(self, U, *targets: int) -> "Circuit":
        U = np.asarray(U, dtype=np.complex128)
        k = len(targets)
        if U.shape != (1 << k, 1 << k):
            raise ValueError("matrix shape does not match target count")
        self.ks.append(k)
        self.targets.append(tuple(int(t) for t in targets))
        self.mats.append(U)
        return self

    def __len__(self) -> int:
        return len(self.ks)

    def inverse(self) -> "Circuit":
        c = Circuit(self.nq)
        for k, t, U in zip(reversed(self.ks), reversed(self.targets), reversed(self.mats)):
            c.add(U.conj().T, *t)
        return c

    # Packed form consumed by both C interfaces: gate rows of 8 int64
    # (k, t1, t2, t3, mat_offset_in_complex, 0, 0, 0) and one flat complex
    # matrix array.
    def packed(self):
        rows = np.zeros((len(self), 8), dtype=np.int64)
        off = 0
        chunks = []
        for g, (k, t, U) in enumerate(zip(self.ks, self.targets, self.mats)):
            rows[g, 0] = k
            rows[g, 1:1 + k] = t
            rows[g, 4] = off
            chunks.append(np.ascontiguousarray(U).reshape(-1))
            off += U.size
        mats = np.concatenate(chunks) if chunks else np.zeros(0, np.complex128)
        return rows, np.ascontiguousarray(mats, dtype=np.complex128)


def draw_k(rng: np.random.Generator, nq: int) -> int:
    ks = [k for k in (1, 2, 3) if k <= nq]
    p = np.array([K_PROBS[k] for k in ks])
    return int(rng.choice(ks, p=p / p.sum()))


def circuit(seed: int, nq: int, G: int, tag: int = 0, unitary: bool = True) -> Circuit:
    rng = np.random.default_rng([seed, tag, CIRCUIT])
    c = Circuit(nq)
    for _ in range(G):
        k = draw_k(rng, nq)
        t = tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False))
        m = 1 << k
        U = random_unitary(rng, m) if unitary else random_matrix(rng, m)
        c.add(U, *t)
    return c


# ---------------------------------------------------------------- batches
def batch_nqs(seed: int, count: int, nq_lo: int, nq_hi: int) -> np.ndarray:
    """nq per instance, uniform on [nq_lo, nq_hi], i.e. log-uniform in size."""
    rng = np.random.default_rng([seed, BATCH])
    return rng.integers(nq_lo, nq_hi + 1, size=count).astype(np.int64)


def batch(seed: int, count: int, nq_lo: int, nq_hi: int, gates_per_qubit: int = 4,
          nqs: np.ndarray | None = None):
    """List of (nq, psi0, Circuit) for `count` independent instances."""
    if nqs is None:
        nqs = batch_nqs(seed, count, nq_lo, nq_hi)
    out = []
    for i, nq in enumerate(nqs):
        nq = int(nq)
        out.append((nq, state(seed, nq, 1000 + i, threads=1),
                    circuit(seed, nq, gates_per_qubit * nq, 1000 + i)))
    return out


def poisson_arrivals(seed: int, rate: float, seconds: float) -> np.ndarray:
    """Open-loop arrival times (s): exponential gaps of mean 1/rate."""
    rng = np.random.default_rng([seed, ARRIVALS])
    n = int(rate * seconds * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < seconds]


# ---------------------------------------------------------------- named gates
# Fixed matrices the paper names; each is <out|U|in> in the local basis.
S2 = 1.0 / math.sqrt(2.0)
I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)          # NOT = sigma_x (§3a)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)       # sigma_y (§3 footnote)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)         # sigma_z
H = np.array([[S2, S2], [S2, -S2]], dtype=np.complex128)     # Hadamard (§3a, Eq. NOTH)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                dtype=np.complex128)                         # control = first target
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                dtype=np.complex128)
TOFFOLI = np.eye(8, dtype=np.complex128)
TOFFOLI[6:8, 6:8] = X                                        # |110> <-> |111>


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """A general one-qubit rotation, the alternative noise operator of the
    multiverse scheme (§5, the general-rotation option beside the Pauli
    operators): exp(-i theta n.sigma / 2) = cos(theta/2) I - i sin(theta/2)
    (n_x X + n_y Y + n_z Z), with theta uniform on [0, 2 pi) and the axis n
    uniform on the unit sphere (z = cos of the polar angle uniform on [-1, 1],
    azimuth uniform on [0, 2 pi)).  Draw order: theta, z, azimuth."""
    theta = rng.uniform(0.0, 2.0 * np.pi)
    z = rng.uniform(-1.0, 1.0)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    r = np.sqrt(max(0.0, 1.0 - z * z))
    nx, ny = r * np.cos(phi), r * np.sin(phi)
    c, sn = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c - 1j * sn * z, -1j * sn * (nx - 1j * ny)],
                     [-1j * sn * (nx + 1j * ny), c + 1j * sn * z]], dtype=np.complex128)


def cphase(phi: float) -> np.ndarray:
    """Controlled phase: diag(1, 1, 1, e^{i phi}) (§4b)."""
    return np.diag([1, 1, 1, np.exp(1j * phi)]).astype(np.complex128)
