"""FP64 CPU oracle for the QCWAVE gate sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product library: the two share nothing but
the seeded input generator in ``qcw_inputs``.

Three independent formulations of the same definition (QCWAVE, Tabakin &
Julia-Diaz, arXiv:1101.1785):

* ``apply`` / ``circuit`` / ``apply_at`` -- the per-amplitude formula of §3a
  Eq. oneopres and §3b Eq. twoopA, written in plain C (``qcw_oracle.c``,
  no FMA contraction), output-driven and out of place.
* ``apply_tensor`` -- numpy: view the state as an nq-axis 2x2x...x2 tensor
  (qubit 1 = axis 0, §2c Eq. staten), move the target axes to the front in
  argument order, contract with the m x m matrix, move them back.  This is the
  tensor-product structure of the operator (§3, opening paragraphs).
* ``apply_kron`` -- numpy: the full 2^nq x 2^nq operator 1 x ... x U x ... x 1
  for contiguous ascending targets, times the state (what the method avoids
  storing, §3a last paragraphs).

``pick`` is the brute-force scan for Pick_k (§4a-§4c).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qcw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libqcw_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (plain scalar C, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-std=c99", "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.orc_apply.argtypes = [i32, i32, P, P, P, P]
        L.orc_apply_ld.argtypes = [i32, i32, P, P, P, P]
        L.orc_apply_at.argtypes = [i32, i32, P, P, P, P, i64, P]
        L.orc_circuit.argtypes = [i32, i32, P, P, P, P, P, P]
        L.orc_circuit_batch.argtypes = [i32, P, P, P, P, P, P, P, P, P]
        L.orc_pick.argtypes = [i32, i32, P, P]
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _targets(targets, k: int) -> np.ndarray:
    t = np.zeros(3, dtype=np.int32)
    t[:k] = targets
    return t


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def apply(U, targets, psi, nq: int | None = None, long_double: bool = False) -> np.ndarray:
    """psi_f = Op_k[U, targets..., psi] (out of place)."""
    U = _c128(U)
    psi = _c128(psi)
    if nq is None:
        nq = int(psi.size).bit_length() - 1
    k = len(targets)
    out = np.empty_like(psi)
    f = lib().orc_apply_ld if long_double else lib().orc_apply
    rc = f(nq, k, _ptr(_targets(targets, k)), _ptr(U), _ptr(psi), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def apply_at(U, targets, psi, idx, nq: int | None = None) -> np.ndarray:
    U = _c128(U)
    psi = _c128(psi)
    if nq is None:
        nq = int(psi.size).bit_length() - 1
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    k = len(targets)
    out = np.empty(idx.size, dtype=np.complex128)
    rc = lib().orc_apply_at(nq, k, _ptr(_targets(targets, k)), _ptr(U), _ptr(psi),
                            _ptr(idx), idx.size, _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def _pack(circ):
    G = len(circ)
    ks = np.array(circ.ks, dtype=np.int32)
    tg = np.zeros((max(G, 1), 3), dtype=np.int32)
    offs = np.zeros(max(G, 1), dtype=np.int64)
    mats = []
    off = 0
    for g in range(G):
        tg[g, :ks[g]] = circ.targets[g]
        offs[g] = off
        mats.append(_c128(circ.mats[g]).reshape(-1))
        off += circ.mats[g].size
    M = np.concatenate(mats) if mats else np.zeros(1, np.complex128)
    return ks, tg, _c128(M), offs


def circuit(circ, psi) -> np.ndarray:
    """Apply every gate of `circ` in list order; returns a new state."""
    psi = np.array(psi, dtype=np.complex128, copy=True)
    ks, tg, M, offs = _pack(circ)
    scratch = np.empty_like(psi)
    rc = lib().orc_circuit(circ.nq, len(circ), _ptr(ks), _ptr(tg), _ptr(M),
                           _ptr(offs), _ptr(psi), _ptr(scratch))
    if rc != 0:
        raise ValueError("oracle rejected the circuit")
    return psi


def circuit_batch(instances):
    """instances: list of (nq, psi0, Circuit); returns list of final states."""
    n = len(instances)
    nqs = np.array([i[0] for i in instances], dtype=np.int32)
    sizes = np.array([1 << int(q) for q in nqs], dtype=np.int64)
    soff = np.zeros(n, dtype=np.int64)
    if n:
        soff[1:] = np.cumsum(sizes)[:-1]
    states = np.concatenate([_c128(i[1]) for i in instances]) if n else np.zeros(1, np.complex128)
    ng = np.array([len(i[2]) for i in instances], dtype=np.int32)
    goff = np.zeros(n, dtype=np.int64)
    if n:
        goff[1:] = np.cumsum(ng)[:-1]
    ks_all, tg_all, M_all, off_all = [], [], [], []
    moff = 0
    for (_, _, c) in instances:
        ks, tg, M, offs = _pack(c)
        G = len(c)
        ks_all.append(ks[:G])
        tg_all.append(tg[:G])
        off_all.append(offs[:G] + moff)
        M_all.append(M[:sum(x.size for x in c.mats)])
        moff += sum(x.size for x in c.mats)
    ks = np.concatenate(ks_all).astype(np.int32) if ks_all else np.zeros(1, np.int32)
    tg = np.ascontiguousarray(np.concatenate(tg_all), dtype=np.int32) if tg_all else np.zeros((1, 3), np.int32)
    offs = np.concatenate(off_all).astype(np.int64) if off_all else np.zeros(1, np.int64)
    M = _c128(np.concatenate(M_all)) if M_all else np.zeros(1, np.complex128)
    rc = lib().orc_circuit_batch(n, _ptr(nqs), _ptr(soff), _ptr(ng), _ptr(goff), _ptr(ks),
                                 _ptr(tg), _ptr(M), _ptr(offs), _ptr(states))
    if rc != 0:
        raise ValueError("oracle rejected the batch")
    return [states[soff[i]:soff[i] + sizes[i]].copy() for i in range(n)]


def pick(nq: int, targets) -> np.ndarray:
    """Pick_k labels, shape (2^nq / m, m): groups ascending, members by local index."""
    k = len(targets)
    out = np.empty(1 << nq, dtype=np.uint64)
    rc = lib().orc_pick(nq, k, _ptr(_targets(targets, k)), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out.reshape(-1, 1 << k)


# ---------------------------------------------------------------- numpy forms
def apply_tensor(U, targets, psi) -> np.ndarray:
    """Tensor-axis form: qubit i is axis i-1 of the (2,)*nq view of psi."""
    psi = _c128(psi)
    nq = int(psi.size).bit_length() - 1
    k = len(targets)
    U = _c128(U).reshape((2,) * (2 * k))
    T = psi.reshape((2,) * nq)
    axes = [t - 1 for t in targets]
    T = np.moveaxis(T, axes, list(range(k)))
    # out[a1..ak, rest] = sum_{b1..bk} U[a1..ak, b1..bk] T[b1..bk, rest]
    T = np.tensordot(U, T, axes=(list(range(k, 2 * k)), list(range(k))))
    T = np.moveaxis(T, list(range(k)), axes)
    return np.ascontiguousarray(T).reshape(-1)


def kron_operator(U, first: int, k: int, nq: int) -> np.ndarray:
    """1_{2^(first-1)} x U x 1_{2^(nq-first-k+1)} for targets first..first+k-1."""
    left = np.eye(1 << (first - 1), dtype=np.complex128)
    right = np.eye(1 << (nq - first - k + 1), dtype=np.complex128)
    return np.kron(np.kron(left, _c128(U)), right)


def apply_kron(U, targets, psi) -> np.ndarray:
    psi = _c128(psi)
    nq = int(psi.size).bit_length() - 1
    k = len(targets)
    first = targets[0]
    if list(targets) != list(range(first, first + k)):
        raise ValueError("kron form needs contiguous ascending targets")
    return kron_operator(U, first, k, nq) @ psi
