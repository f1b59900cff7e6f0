"""Pins of the density-matrix (multiverse) oracle against the paper's closed
forms and invariants (QCWAVE §5)."""
import numpy as np
import pytest

import qcw_inputs as qi
from oracle import density as D

EPS = 2.0 ** -53


def _rand_rho(rng, nq, rank=3):
    A = rng.normal(size=(1 << nq, rank)) + 1j * rng.normal(size=(1 << nq, rank))
    r = A @ A.conj().T
    return r / np.trace(r)


def _pauli_terms(rng, nq, n_p, eps, p1=0.95, p2=0.05, paulis=(D.SX, D.SY, D.SZ)):
    """n_p single hits and n_p double hits, each path weighted eps * p_s / n_p."""
    terms = []
    for _ in range(n_p):
        q = int(rng.integers(1, nq + 1))
        terms.append((eps * p1 / n_p, {q: paulis[int(rng.integers(len(paulis)))]}))
    if nq >= 2:
        for _ in range(n_p):
            a, b = (int(x) + 1 for x in rng.choice(nq, 2, replace=False))
            terms.append((eps * p2 / n_p, {a: paulis[int(rng.integers(len(paulis)))],
                                           b: paulis[int(rng.integers(len(paulis)))]}))
    return terms


def test_trace_and_hermiticity_preserved():
    """Eq. rhoE1: with unitary path operators and p + sum of weights = 1, Tr = 1
    and rho stays Hermitian."""
    rng = np.random.default_rng(0)
    for nq in (1, 2, 4):
        rho = _rand_rho(rng, nq)
        eps = 0.2
        terms = _pauli_terms(rng, nq, 8, eps) if nq > 1 else \
            [(eps / 8, {1: [D.SX, D.SY, D.SZ][i % 3]}) for i in range(8)]
        w = sum(t[0] for t in terms)
        out = D.channel(rho, 1 - w, terms)
        assert abs(np.trace(out) - 1) <= 64 * EPS
        assert np.max(np.abs(out - out.conj().T)) <= 64 * EPS


def test_kraus_completeness():
    """Eq. rhoE2: K0 = sqrt(p) 1, Kn = sqrt(eps/n_p) Omega_n satisfy sum K^dag K = 1."""
    rng = np.random.default_rng(1)
    nq, n_p, eps = 3, 6, 0.2
    Ks = [np.sqrt(1 - eps) * np.eye(8)]
    for _ in range(n_p):
        q = int(rng.integers(1, nq + 1))
        U = qi.random_unitary(rng, 2)
        Ks.append(np.sqrt(eps / n_p) * D.embed({q: U}, nq))
    S = sum(K.conj().T @ K for K in Ks)
    assert np.max(np.abs(S - np.eye(8))) <= 64 * EPS


@pytest.mark.parametrize("nx,ny,nz", [(1, 1, 1), (2, 0, 1), (0, 3, 1), (4, 0, 0)])
def test_one_qubit_pauli_channel_closed_form(nx, ny, nz):
    """Storage case (§5): with n_X, n_Y, n_Z of the n_p paths hit by X, Y, Z, the
    polarisation shrinks as P_x -> [1 - 2 eps (n_Y + n_Z)/n_p] P_x (cyclic)."""
    n_p, eps = nx + ny + nz, 0.2
    P = np.array([0.3, -0.5, 0.6])
    rho = 0.5 * (np.eye(2) + P[0] * D.SX + P[1] * D.SY + P[2] * D.SZ)
    terms = [(eps / n_p, {1: D.SX})] * nx + [(eps / n_p, {1: D.SY})] * ny + \
            [(eps / n_p, {1: D.SZ})] * nz
    out = D.channel(rho, 1 - eps, terms)
    got = D.observables(out)["polarization"][0]
    expect = P * np.array([1 - 2 * eps * (ny + nz) / n_p, 1 - 2 * eps * (nx + nz) / n_p,
                           1 - 2 * eps * (nx + ny) / n_p])
    assert np.max(np.abs(got - expect)) <= 16 * EPS


def test_fidelity_after_one_hadamard():
    """§5, MV1-Noise: without noise the fidelity drops to 1/sqrt2 after one H."""
    psi0 = qi.basis_state(1, 0)
    rho = D.conjugate(D.pure(psi0), qi.H, (1,))
    f = D.observables(rho, psi0)["fidelity"]
    assert abs(f - 2 ** -0.5) <= 4 * EPS
    assert abs(D.fidelity_general(rho, D.pure(psi0)) - 2 ** -0.5) <= 1e-12
    back = D.conjugate(rho, qi.H, (1,))
    assert abs(D.observables(back, psi0)["fidelity"] - 1.0) <= 4 * EPS


def test_bell_state_observables():
    """§5, MV2-Noise: CNOT_12 H_1 |00> is pure and each qubit is unpolarised; a
    double X hit leaves it unchanged."""
    rho = D.pure(qi.basis_state(2, 0))
    rho = D.conjugate(rho, qi.H, (1,))
    rho = D.conjugate(rho, qi.CNOT, (1, 2))
    ob = D.observables(rho)
    assert abs(ob["purity"] - 1) <= 8 * EPS
    assert np.max(np.abs(ob["polarization"])) <= 8 * EPS
    hit = D.channel(rho, 0.0, [(1.0, {1: D.SX, 2: D.SX})])
    assert np.max(np.abs(hit - rho)) <= 8 * EPS


def test_classical_limit():
    """§5 (classical limit): repeated X and Z noise drives rho to 1/2^nq: all
    eigenvalues 1/2^nq and entropy nq bits.  Z noise alone removes the
    coherences but keeps the populations."""
    rng = np.random.default_rng(3)
    nq = 3
    rho = _rand_rho(rng, nq)
    xz = [(0.3 / (2 * nq), {q: s}) for q in range(1, nq + 1) for s in (D.SX, D.SZ)]
    for _ in range(600):
        rho = D.channel(rho, 0.7, xz)
    ev = D.eigen_observables(rho)
    assert np.max(np.abs(ev["eigenvalues"] - 1 / 8)) <= 1e-12
    assert abs(ev["entropy_bits"] - nq) <= 1e-10
    rho = _rand_rho(rng, nq)
    pops = np.real(np.diag(rho)).copy()
    z = [(0.3 / nq, {q: D.SZ}) for q in range(1, nq + 1)]
    for _ in range(200):
        rho = D.channel(rho, 0.7, z)
    assert np.max(np.abs(rho - np.diag(np.diag(rho)))) <= 1e-12
    assert np.max(np.abs(np.real(np.diag(rho)) - pops)) <= 1e-12


def test_gate_operator_matches_sweep_definition():
    """The full gate operator equals the tensor-axis form of the state oracle."""
    import oracle
    rng = np.random.default_rng(4)
    for t in [(2,), (3, 1), (1, 4, 2)]:
        U = qi.random_matrix(rng, 1 << len(t))
        psi = rng.normal(size=16) + 1j * rng.normal(size=16)
        assert np.max(np.abs(D.gate_operator(U, t, 4) @ psi - oracle.apply_tensor(U, t, psi))) <= 1e-13


def test_planted_transpose_mistake_caught():
    """K rho K^T in place of K rho K^dagger breaks the Y-channel closed form."""
    rho = 0.5 * (np.eye(2) + 0.4 * D.SY)

    def wrong(rho, p, terms):
        out = p * rho
        for w, ops in terms:
            K = D.embed(ops, 1)
            out = out + w * (K @ rho @ K.T)
        return out
    good = D.channel(rho, 0.8, [(0.2, {1: D.SY})])
    bad = wrong(rho, 0.8, [(0.2, {1: D.SY})])
    Py = lambda r: np.real(np.trace(D.SY @ r))
    assert abs(Py(good) - 0.4) <= 8 * EPS            # Y hits keep P_y
    assert abs(Py(bad) - 0.4) > 0.1


def test_partial_trace_pins():
    """Tracing out one qubit of a product state leaves the other factor; of a
    Bell state, the maximally mixed 1/2 (entropy 1 bit)."""
    rng = np.random.default_rng(8)
    a, b = _rand_rho(rng, 1, 2), _rand_rho(rng, 2, 2)
    prod = np.kron(a, b)                                  # qubit 1 x qubits 2, 3
    assert np.max(np.abs(D.partial_trace(prod, [1]) - a)) <= 1e-15
    assert np.max(np.abs(D.partial_trace(prod, [2, 3]) - b)) <= 1e-15
    rho = D.conjugate(D.conjugate(D.pure(qi.basis_state(2, 0)), qi.H, (1,)), qi.CNOT, (1, 2))
    r1 = D.partial_trace(rho, [2])
    assert np.max(np.abs(r1 - np.eye(2) / 2)) <= 1e-15
    assert abs(D.eigen_observables(r1)["entropy_bits"] - 1.0) <= 1e-14
    assert abs(np.trace(D.partial_trace(_rand_rho(rng, 4), [1, 3])) - 1) <= 1e-14


def test_eigen_pins():
    """Pure state: eigenvalues {0, ..., 0, 1}, entropy 0; maximally mixed: all
    1/2^nq, entropy nq; eigenvalues sum to the trace; fidelity of a state with
    itself is 1 and with an orthogonal pure state 0."""
    rng = np.random.default_rng(9)
    psi = qi.state(4, 3)
    ev = D.eigen_observables(D.pure(psi))
    assert np.max(np.abs(ev["eigenvalues"] - np.r_[np.zeros(7), 1.0])) <= 1e-14
    assert abs(ev["entropy_bits"]) <= 1e-12
    ev = D.eigen_observables(np.eye(8) / 8)
    assert abs(ev["entropy_bits"] - 3) <= 1e-14
    r = _rand_rho(rng, 3)
    assert abs(np.sum(D.eigen_observables(r)["eigenvalues"]) - 1) <= 1e-14
    assert abs(D.fidelity_general(r, r) - 1) <= 1e-7
    assert abs(D.fidelity_general(D.pure(qi.basis_state(2, 0)), D.pure(qi.basis_state(2, 3)))) <= 1e-7


def _bloch(P):
    """One-qubit rho = (1 + P . sigma) / 2 (§5, the one-qubit form)."""
    return (np.eye(2) + P[0] * D.SX + P[1] * D.SY + P[2] * D.SZ) / 2


def test_pair_polarization_pins():
    """The two-qubit form of §5's footnote, rho = (1 + P1 . sigma x 1 + P2 .
    1 x sigma + C . sigma x sigma) / 4:
    * a product of one-qubit states (1 + P . sigma)/2 has polarisations P
      and C_ij = P1_i P2_j, with the pair anywhere in a larger product and in
      either order (C transposes);
    * the Bell state (|00> + |11>)/sqrt2 has P1 = P2 = 0 and C = diag(1, -1, 1);
    * for any rho the 15 numbers rebuild the pair's reduced matrix by the
      footnote's formula."""
    rng = np.random.default_rng(21)
    Ps = [rng.normal(size=3) for _ in range(4)]
    Ps = [P / np.linalg.norm(P) * rng.uniform(0.2, 1.0) for P in Ps]
    rho = _bloch(Ps[0])
    for P in Ps[1:]:
        rho = np.kron(rho, _bloch(P))                      # qubits 1..4
    for a, b in ((1, 2), (2, 4), (4, 1), (3, 1)):
        v = D.pair_polarization(rho, a, b)
        Pa, Pb = Ps[a - 1], Ps[b - 1]
        assert np.max(np.abs(v[:3] - Pa)) <= 1e-15 and np.max(np.abs(v[3:6] - Pb)) <= 1e-15
        assert np.max(np.abs(v[6:].reshape(3, 3) - np.outer(Pa, Pb))) <= 1e-15
    bell = D.conjugate(D.conjugate(D.pure(qi.basis_state(2, 0)), qi.H, (1,)), qi.CNOT, (1, 2))
    v = D.pair_polarization(bell, 1, 2)
    assert np.max(np.abs(v[:6])) <= 8 * EPS
    assert np.max(np.abs(v[6:].reshape(3, 3) - np.diag([1.0, -1.0, 1.0]))) <= 8 * EPS
    S = (D.SX, D.SY, D.SZ)
    r = _rand_rho(rng, 4)
    for a, b in ((1, 3), (2, 4)):
        v = D.pair_polarization(r, a, b)
        re = np.eye(4, dtype=np.complex128)
        for i in range(3):
            re = re + v[i] * np.kron(S[i], np.eye(2)) + v[3 + i] * np.kron(np.eye(2), S[i])
            for j in range(3):
                re = re + v[6 + 3 * i + j] * np.kron(S[i], S[j])
        assert np.max(np.abs(re / 4 - D.partial_trace(r, [a, b]))) <= 1e-15
    assert np.max(np.abs(D.pair_polarization(r, 2, 4)[:3] - D.observables(r)["polarization"][1])) <= 1e-15


def test_planted_pair_index_mistake_caught():
    """The pins fail for a plausible slip: C with its indices swapped."""
    rng = np.random.default_rng(22)
    Pa, Pb = rng.normal(size=3), rng.normal(size=3)
    rho = np.kron(_bloch(Pa / 2), _bloch(Pb / 3))
    v = D.pair_polarization(rho, 1, 2)
    swapped = v[6:].reshape(3, 3).T
    assert np.max(np.abs(swapped - np.outer(Pa / 2, Pb / 3))) > 1e-3
