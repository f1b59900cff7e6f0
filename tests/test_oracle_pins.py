"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses a worked example
stated in the text, a closed form, an invariant, or an independent formulation
(tensor-axis contraction, explicit Kronecker operator, brute-force label scan).
The mutation tests at the end plant plausible mistakes in an oracle-shaped
function and show that the same pins catch every one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
import qcw_inputs as qi
from golden_io import all_golden

EPS = 2.0 ** -53
GOLDEN = all_golden()


def _rand_state(rng, nq):
    v = rng.uniform(-1, 1, 1 << nq) + 1j * rng.uniform(-1, 1, 1 << nq)
    return v / np.linalg.norm(v)


def _targets_all(nq, k):
    return list(itertools.permutations(range(1, nq + 1), k))


# --------------------------------------------------------------- worked examples
@pytest.mark.parametrize("g", GOLDEN, ids=[g.name for g in GOLDEN])
def test_golden_worked_examples(g):
    g.check(oracle.circuit(g.circ, g.init))


def test_e1_exact_bits():
    """H_1|000>: C_0 and C_4 are exactly the stored entry fl(1/sqrt2) (Sec. 4a)."""
    out = oracle.apply(qi.H, (1,), qi.basis_state(3, 0))
    assert out[0] == qi.S2 and out[4] == qi.S2
    assert np.count_nonzero(out) == 2


@pytest.mark.parametrize("nq", [1, 2, 5, 9])
def test_hadamard_all_closed_form(nq):
    """OmegaALL[H, |0...0>] has every amplitude 2^(-nq/2) (Sec. 4a)."""
    psi = qi.basis_state(nq, 0)
    for q in range(1, nq + 1):
        psi = oracle.apply(qi.H, (q,), psi)
    assert np.max(np.abs(psi - 2.0 ** (-nq / 2))) <= 4 * nq * EPS


@pytest.mark.parametrize("nq", [2, 3, 6, 10])
def test_ghz_chain_any_size(nq):
    """CNOT_1n ... CNOT_12 H_1 |0..0> = (|0..0> + |1..1>)/sqrt2 (Sec. 5, MVn-Noise)."""
    c = qi.Circuit(nq).add(qi.H, 1)
    for t in range(2, nq + 1):
        c.add(qi.CNOT, 1, t)
    out = oracle.circuit(c, qi.basis_state(nq, 0))
    ref = np.zeros(1 << nq, complex)
    ref[0] = ref[-1] = qi.S2
    assert np.array_equal(out, ref)


# --------------------------------------------------------------- independent forms
def test_tensor_form_matches_kron_operator():
    """The tensor-axis form equals the explicit 1 x U x 1 operator (Sec. 3 intro)."""
    rng = np.random.default_rng(5)
    for nq in range(1, 7):
        psi = _rand_state(rng, nq)
        for k in range(1, min(3, nq) + 1):
            for first in range(1, nq - k + 2):
                U = qi.random_matrix(rng, 1 << k)
                t = tuple(range(first, first + k))
                a = oracle.apply_tensor(U, t, psi)
                b = oracle.apply_kron(U, t, psi)
                assert np.max(np.abs(a - b)) <= 64 * EPS


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5])
def test_oracle_vs_tensor_every_target_tuple(nq):
    rng = np.random.default_rng(100 + nq)
    psi = _rand_state(rng, nq)
    for k in range(1, min(3, nq) + 1):
        for t in _targets_all(nq, k):
            U = qi.random_matrix(rng, 1 << k)
            a = oracle.apply(U, t, psi)
            b = oracle.apply_tensor(U, t, psi)
            assert np.max(np.abs(a - b)) <= 64 * EPS, (k, t)


@pytest.mark.parametrize("nq", [6, 8, 11])
def test_oracle_vs_tensor_sampled_targets(nq):
    rng = np.random.default_rng(200 + nq)
    psi = _rand_state(rng, nq)
    for k in (1, 2, 3):
        for _ in range(6):
            t = tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False))
            U = qi.random_unitary(rng, 1 << k)
            a = oracle.apply(U, t, psi)
            b = oracle.apply_tensor(U, t, psi)
            assert np.linalg.norm(a - b) <= 64 * EPS, (k, t)


def test_oracle_vs_explicit_element_operator():
    """Full operator <n|Op|n'> = U[r(n), r(n')] when n, n' agree off the targets."""
    rng = np.random.default_rng(7)
    nq = 4
    N = 1 << nq
    psi = _rand_state(rng, nq)
    for t in [(2,), (4, 1), (3, 1, 4)]:
        k = len(t)
        U = qi.random_matrix(rng, 1 << k)
        bits = [nq - x for x in t]
        mask = sum(1 << b for b in bits)
        M = np.zeros((N, N), complex)
        for n in range(N):
            for n2 in range(N):
                if (n & ~mask) == (n2 & ~mask):
                    r = int("".join(str((n >> b) & 1) for b in bits), 2)
                    c = int("".join(str((n2 >> b) & 1) for b in bits), 2)
                    M[n, n2] = U[r, c]
        assert np.max(np.abs(M @ psi - oracle.apply(U, t, psi))) <= 64 * EPS


# --------------------------------------------------------------- structure
@pytest.mark.parametrize("nq,a,b", [(3, 1, 3), (5, 4, 2), (6, 6, 1)])
def test_two_qubit_product_factorises(nq, a, b):
    """Op2(A x B; a, b) = Op1(A; a) Op1(B; b): the tensor product of Sec. 3."""
    rng = np.random.default_rng(nq * 10 + a)
    A, B = qi.random_matrix(rng, 2), qi.random_matrix(rng, 2)
    psi = _rand_state(rng, nq)
    two = oracle.apply(np.kron(A, B), (a, b), psi)
    one = oracle.apply(A, (a,), oracle.apply(B, (b,), psi))
    assert np.max(np.abs(two - one)) <= 64 * EPS


def test_three_qubit_product_factorises():
    rng = np.random.default_rng(3)
    nq = 5
    A, B, C = (qi.random_matrix(rng, 2) for _ in range(3))
    psi = _rand_state(rng, nq)
    t = (4, 1, 3)
    three = oracle.apply(np.kron(np.kron(A, B), C), t, psi)
    one = oracle.apply(A, (4,), oracle.apply(B, (1,), oracle.apply(C, (3,), psi)))
    assert np.max(np.abs(three - one)) <= 128 * EPS


def test_argument_order_swap():
    """Op2(V; a, b) = Op2(SWAP V SWAP; b, a): local index follows argument order."""
    rng = np.random.default_rng(9)
    psi = _rand_state(rng, 4)
    V = qi.random_matrix(rng, 4)
    a = oracle.apply(V, (1, 3), psi)
    b = oracle.apply(qi.SWAP @ V @ qi.SWAP, (3, 1), psi)
    assert np.max(np.abs(a - b)) <= 16 * EPS


def test_unitary_preserves_norm_and_inverts():
    """Unitary gates keep sum |C_n|^2 = 1 (Sec. 2) and U then U^dagger is identity."""
    rng = np.random.default_rng(11)
    nq = 9
    psi0 = _rand_state(rng, nq)
    c = qi.circuit(0, nq, 20, tag=3)
    out = oracle.circuit(c, psi0)
    assert abs(np.linalg.norm(out) - 1.0) <= 1e-13
    back = oracle.circuit(c.inverse(), out)
    assert np.linalg.norm(back - psi0) <= 1e-13


def test_linearity_in_the_matrix():
    rng = np.random.default_rng(13)
    psi = _rand_state(rng, 5)
    U, W = qi.random_matrix(rng, 4), qi.random_matrix(rng, 4)
    a = oracle.apply(2.0 * U - 3j * W, (2, 5), psi)
    b = 2.0 * oracle.apply(U, (2, 5), psi) - 3j * oracle.apply(W, (2, 5), psi)
    assert np.max(np.abs(a - b)) <= 256 * EPS


def test_permutation_gates_exact():
    """Signed-permutation gates (entries 0, +-1, +-i) move values without rounding."""
    rng = np.random.default_rng(17)
    nq = 6
    psi = _rand_state(rng, nq)
    for U, t in [(qi.X, (2,)), (qi.Y, (6,)), (qi.Z, (1,)), (qi.CNOT, (5, 2)),
                 (qi.CZ, (1, 6)), (qi.SWAP, (3, 4)), (qi.TOFFOLI, (6, 1, 3))]:
        out = oracle.apply(U, t, psi)
        assert np.array_equal(np.sort(np.abs(out)), np.sort(np.abs(psi)))
        assert np.array_equal(out, oracle.apply_tensor(U, t, psi))


def test_sampled_outputs_match_full():
    rng = np.random.default_rng(19)
    nq = 10
    psi = _rand_state(rng, nq)
    U = qi.random_unitary(rng, 8)
    t = (7, 2, 10)
    idx = rng.choice(1 << nq, 200, replace=False).astype(np.uint64)
    full = oracle.apply(U, t, psi)
    assert np.array_equal(oracle.apply_at(U, t, psi, idx), full[idx.astype(np.int64)])


def test_oracle_rounding_vs_long_double():
    """The double oracle stays within 1e-14 of the same sums carried in long double."""
    rng = np.random.default_rng(23)
    nq = 12
    psi = _rand_state(rng, nq)
    for t in [(5,), (12, 1), (3, 9, 6)]:
        U = qi.random_unitary(rng, 1 << len(t))
        a = oracle.apply(U, t, psi)
        b = oracle.apply(U, t, psi, long_double=True)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-14


def test_batch_equals_each_instance():
    inst = qi.batch(2, 12, 3, 7)
    outs = oracle.circuit_batch(inst)
    for (nq, psi0, c), o in zip(inst, outs):
        assert np.array_equal(o, oracle.circuit(c, psi0))


def test_oracle_rejects_bad_arguments():
    psi = qi.basis_state(3, 0)
    for t in [(0,), (4,), (2, 2), (1, 2, 3, 1)]:
        with pytest.raises((ValueError, IndexError)):
            oracle.apply(np.eye(1 << len(t)), t, psi)


# --------------------------------------------------------------- Pick
@pytest.mark.parametrize("nq", [1, 3, 6, 10])
def test_pick_structure(nq):
    """Pick_k: 2^nq/m groups, closed-form partners, every label exactly once."""
    rng = np.random.default_rng(nq)
    for k in range(1, min(3, nq) + 1):
        tl = _targets_all(nq, k) if nq <= 3 else \
            [tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False)) for _ in range(5)]
        for t in tl:
            P = oracle.pick(nq, t).astype(np.int64)
            m = 1 << k
            assert P.shape == ((1 << nq) // m, m)                       # Sec. 3a-3c counts
            assert np.array_equal(np.sort(P.reshape(-1)), np.arange(1 << nq))
            stride = [1 << (nq - x) for x in t]
            base = P[:, 0]
            assert np.all(np.diff(base) > 0)                            # ascending groups
            for s in stride:
                assert np.all((base & s) == 0)                          # all targets 0
            for r in range(m):
                off = sum(stride[j] for j in range(k) if (r >> (k - 1 - j)) & 1)
                assert np.array_equal(P[:, r], base + off)
            if k == 1:
                assert np.array_equal(P[:, 1], P[:, 0] + stride[0])     # n1 = n0 + 2^(nq-is)
            if k == 2:                                                  # quartet relations
                assert np.array_equal(P[:, 1], P[:, 0] + stride[1])
                assert np.array_equal(P[:, 2], P[:, 0] + stride[0])
                assert np.array_equal(P[:, 3], P[:, 0] + stride[0] + stride[1])


def test_pick_partner_formula_pair0_pair1():
    """Eqs. pair0/pair1: n0 = n - q_is 2^(nq-is), n1 = n - (q_is - 1) 2^(nq-is)."""
    nq, s = 4, 2
    P = oracle.pick(nq, (s,)).astype(np.int64)
    st = 1 << (nq - s)
    for n in range(1 << nq):
        q = (n >> (nq - s)) & 1
        n0, n1 = n - q * st, n - (q - 1) * st
        row = np.nonzero(P[:, 0] == n0)[0]
        assert row.size == 1 and P[row[0], 1] == n1


# --------------------------------------------------------------- mutation checks
def _pin_suite(apply_fn):
    """The pins above, against an arbitrary apply(U, targets, psi) callable.

    Returns True when every pin holds."""
    def circ(c, psi):
        for U, t in zip(c.mats, c.targets):
            psi = apply_fn(U, t, psi)
        return psi
    try:
        for g in GOLDEN:
            g.check(circ(g.circ, g.init), tol=1e-12)
        rng = np.random.default_rng(77)
        for nq in (3, 4):
            psi = _rand_state(rng, nq)
            for k in (1, 2, 3):
                for t in _targets_all(nq, k)[:8]:
                    U = qi.random_matrix(rng, 1 << k)
                    if np.max(np.abs(apply_fn(U, t, psi) - oracle.apply_tensor(U, t, psi))) > 1e-12:
                        return False
                    if list(t) == list(range(t[0], t[0] + k)):
                        if np.max(np.abs(apply_fn(U, t, psi) - oracle.apply_kron(U, t, psi))) > 1e-12:
                            return False
    except AssertionError:
        return False
    return True


def _mutant(kind):
    def f(U, t, psi):
        U = np.asarray(U)
        t = tuple(t)
        if kind == "transposed":
            U = U.T
        elif kind == "reversed_targets":
            t = t[::-1]
        elif kind == "conjugated":
            U = U.conj()
        elif kind == "dropped_offdiagonal_term" and U.shape[0] > 1:
            U = U.copy()
            U[0, -1] = 0
        elif kind == "lsb_first_qubit_order":
            nq = int(psi.size).bit_length() - 1
            t = tuple(nq + 1 - x for x in t)
        elif kind == "complex_product_sign":
            # re = ur*xr + ui*xi instead of ur*xr - ui*xi
            Ur, Ui = U.real + 0j, U.imag + 0j
            xr, xi = psi.real + 0j, psi.imag + 0j
            re = oracle.apply(Ur, t, xr) + oracle.apply(Ui, t, xi)
            im = oracle.apply(Ur, t, xi) + oracle.apply(Ui, t, xr)
            return re.real + 1j * im.real
        return oracle.apply(U, t, psi)
    return f


def test_pins_accept_the_oracle():
    assert _pin_suite(oracle.apply)


@pytest.mark.parametrize("kind", ["transposed", "reversed_targets", "conjugated",
                                  "dropped_offdiagonal_term", "lsb_first_qubit_order",
                                  "complex_product_sign"])
def test_pins_reject_planted_mistakes(kind):
    assert not _pin_suite(_mutant(kind))
