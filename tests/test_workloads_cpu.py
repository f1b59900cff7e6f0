"""The paper's example workloads as circuits (qcw_inputs.workloads), checked on
the oracle against closed forms: the GHZ chain (§5, MVn-Noise), Bell followed
by its inverse (§5, MV2-Noise), and textbook Grover search (listed among the
applications, §6d): after k iterations the marked amplitude is
(-1)^k sin((2k+1) theta), sin theta = 2^(-n/2), every other data amplitude
(-1)^k cos((2k+1) theta)/sqrt(2^n - 1), and the ancillas are back in |0>."""
import numpy as np
import pytest

import oracle
import qcw_inputs as qi
from qcw_inputs import workloads as W

TOL = 1e-12


def grover_expected(n, marked, k):
    nq = W.grover_qubits(n)
    a, b = W.grover_amplitudes(n, k)
    ref = np.zeros(1 << nq, complex)
    for d in range(1 << n):
        ref[d << (nq - n)] = a if d == marked else b
    return ref


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_grover_closed_form(n):
    rng = np.random.default_rng(n)
    kopt = W.grover_optimal_iterations(n)
    for marked in rng.choice(1 << n, min(3, 1 << n), replace=False):
        for k in sorted({0, 1, kopt, kopt + 1}):
            c = W.grover(n, int(marked), k)
            out = oracle.circuit(c, qi.basis_state(c.nq, 0))
            assert np.max(np.abs(out - grover_expected(n, int(marked), k))) <= TOL, (n, marked, k)


def test_grover_success_probability_near_one_at_optimum():
    for n in range(2, 8):
        a, _ = W.grover_amplitudes(n, W.grover_optimal_iterations(n))
        assert a * a > 0.94


def test_grover_gate_count_and_qubits():
    c = W.grover(5, 19, 2)
    assert c.nq == 8 and max(c.ks) == 3
    assert all(max(t) <= c.nq for t in c.targets)


def test_bell_and_inverse_returns_to_00():
    out = oracle.circuit(W.bell_and_inverse(), qi.basis_state(2, 0))
    ref = np.zeros(4, complex)
    ref[0] = 1.0
    assert np.max(np.abs(out - ref)) <= 4e-16


@pytest.mark.parametrize("nq", [2, 5, 9])
def test_ghz_chain_builder(nq):
    out = oracle.circuit(W.ghz_chain(nq), qi.basis_state(nq, 0))
    ref = np.zeros(1 << nq, complex)
    ref[0] = ref[-1] = qi.S2
    assert np.array_equal(out, ref)
