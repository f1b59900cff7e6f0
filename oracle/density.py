"""FP64 CPU oracle for the multiverse density-matrix step -- TEST INFRASTRUCTURE ONLY.

Written from QCWAVE §5 (Tabakin & Julia-Diaz, arXiv:1101.1785), with the
density matrix held as a full 2^nq x 2^nq numpy array and every operator built
as a full matrix by Kronecker products (qubit 1 leftmost, §2c Eq. staten).
Nothing here is shared with the HIP library.

* channel(rho, p, terms): the ensemble average over paths, Eq. rhoE1 --
  rho_f = p rho + sum_b w_b K_b rho K_b^dagger -- where each path's operator
  K_b is one one-qubit operator, or two one-qubit operators on two distinct
  qubits (the single and double hits of the noise model, Eq. rhoE4; the
  weight of a term is eps * p_s / n_p there).
* conjugate(rho, U, targets): rho -> U rho U^dagger for an algorithm gate
  (the Omega_A factors of Eq. rhoE4).
* observables(rho, psi0): trace, purity Tr rho^2, fidelity with a pure
  reference Tr sqrt(sqrt(rho0) rho sqrt(rho0)) = sqrt(<psi0|rho|psi0>) when
  rho0 = |psi0><psi0|, and each qubit's polarisation vector P = Tr[sigma rho]
  (§5, the ideal and noisy channels; the storage case).
* eigen_observables: eigenvalues, von Neumann entropy (in bits, so that the
  classical limit is nq) via numpy's Hermitian eigensolver, for pins only.
* pair_polarization(rho, a, b): the 15 parameters of the two-qubit form in
  the footnote to §5's density-matrix paragraph, for qubits a and b: the
  polarisations P1 = Tr[(sigma x 1) rho], P2 = Tr[(1 x sigma) rho] and the
  3 x 3 spin correlation tensor C_ij = Tr[(sigma_i x sigma_j) rho] (the
  footnote's traces omit rho; read as in the one-qubit case before it).
"""
from __future__ import annotations

import numpy as np

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _nq(rho):
    return int(rho.shape[0]).bit_length() - 1


def embed(ops: dict, nq: int) -> np.ndarray:
    """Full operator: ops maps qubit (1-based) -> 2x2 matrix; identity elsewhere."""
    M = np.array([[1.0 + 0j]])
    for q in range(1, nq + 1):
        M = np.kron(M, ops.get(q, np.eye(2, dtype=np.complex128)))
    return M


def gate_operator(U, targets, nq: int) -> np.ndarray:
    """Full 2^nq operator of a k-qubit gate on ordered targets (first = MSB of r)."""
    k = len(targets)
    N = 1 << nq
    bits = [nq - t for t in targets]
    mask = sum(1 << b for b in bits)
    M = np.zeros((N, N), dtype=np.complex128)
    for n in range(N):
        r = 0
        for b in bits:
            r = (r << 1) | ((n >> b) & 1)
        rest = n & ~mask
        for c in range(1 << k):
            src = rest
            for j, b in enumerate(bits):
                if (c >> (k - 1 - j)) & 1:
                    src |= 1 << b
            M[n, src] = U[r, c]
    return M


def pure(psi) -> np.ndarray:
    psi = np.asarray(psi, dtype=np.complex128)
    return np.outer(psi, psi.conj())


def channel(rho, p_keep: float, terms) -> np.ndarray:
    """terms: list of (weight, {qubit: 2x2 matrix}) -- one or two qubits each."""
    nq = _nq(rho)
    out = p_keep * rho
    for w, ops in terms:
        K = embed(ops, nq)
        out = out + w * (K @ rho @ K.conj().T)
    return out


def conjugate(rho, U, targets) -> np.ndarray:
    M = gate_operator(np.asarray(U, dtype=np.complex128), list(targets), _nq(rho))
    return M @ rho @ M.conj().T


def observables(rho, psi0=None) -> dict:
    nq = _nq(rho)
    out = {"trace": complex(np.trace(rho)),
           "purity": float(np.real(np.trace(rho @ rho)))}
    if psi0 is not None:
        psi0 = np.asarray(psi0, dtype=np.complex128)
        f2 = np.real(psi0.conj() @ rho @ psi0)
        out["fidelity"] = float(np.sqrt(max(f2, 0.0)))
    P = np.zeros((nq, 3))
    for q in range(1, nq + 1):
        for i, s in enumerate((SX, SY, SZ)):
            P[q - 1, i] = np.real(np.trace(embed({q: s}, nq) @ rho))
    out["polarization"] = P
    return out


def pair_polarization(rho, a: int, b: int) -> np.ndarray:
    """[P1 (x, y, z), P2 (x, y, z), C row-major (i for qubit a, j for b)]:
    traces of rho with Pauli operators on qubits a and b (1-based,
    distinct), each operator embedded as a full 2^nq matrix."""
    nq = _nq(rho)
    S = (SX, SY, SZ)
    out = [np.real(np.trace(embed({a: s}, nq) @ rho)) for s in S]
    out += [np.real(np.trace(embed({b: s}, nq) @ rho)) for s in S]
    out += [np.real(np.trace(embed({a: si, b: sj}, nq) @ rho)) for si in S for sj in S]
    return np.array(out)


def eigen_observables(rho) -> dict:
    lam = np.linalg.eigvalsh((rho + rho.conj().T) / 2)
    lam_pos = lam[lam > 1e-300]
    return {"eigenvalues": lam, "entropy_bits": float(-np.sum(lam_pos * np.log2(lam_pos)))}


def fidelity_general(rho, rho0) -> float:
    """Tr sqrt(sqrt(rho0) rho sqrt(rho0)) by eigendecomposition (pins only)."""
    w, V = np.linalg.eigh((rho0 + rho0.conj().T) / 2)
    s = (V * np.sqrt(np.clip(w, 0, None))) @ V.conj().T
    m = s @ rho @ s
    ev = np.linalg.eigvalsh((m + m.conj().T) / 2)
    return float(np.sum(np.sqrt(np.clip(ev, 0, None))))


def partial_trace(rho, keep) -> np.ndarray:
    """Reduced density matrix of the qubits `keep` (1-based), kept in qubit order:
    the traced qubits' row and column indices are summed together."""
    nq = _nq(rho)
    keep = sorted(keep)
    letters = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"
    rows = [letters[q - 1] for q in range(1, nq + 1)]
    cols = [letters[nq + q - 1] if q in keep else letters[q - 1] for q in range(1, nq + 1)]
    out = [letters[q - 1] for q in keep] + [letters[nq + q - 1] for q in keep]
    T = np.einsum("".join(rows + cols) + "->" + "".join(out), rho.reshape((2,) * (2 * nq)))
    nk = len(keep)
    return T.reshape(1 << nk, 1 << nk)
