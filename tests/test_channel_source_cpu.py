"""The tiled channel kernel that a channel compiles at creation (host side).

qcw_debug_channel_source returns the source that qcw_channel_create hands
to the run-time compiler for a channel's tiled plan, without a device.  These
tests check which channels get one, that it depends on the plan's structure
and not on the coefficients (channels of one structure share a compiled
kernel), and that it compiles for gfx950.  That it computes the channel is
checked on the GPU, bit for bit against the generic tiled kernel and against
the oracle (tests/test_gpu_density.py).
"""
import numpy as np
import pytest

import qcw_inputs as qi


@pytest.fixture(scope="module")
def L():
    from paper_1101_1785_amd import _lib
    return _lib


def _pauli(rng, nq, n_p=16, eps=0.2):
    P = [qi.X, qi.Y, qi.Z]
    terms = []
    for s, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(n_p):
            qs = [int(x) + 1 for x in rng.choice(nq, s, replace=False)]
            terms.append((eps * ps / n_p, {q: P[int(rng.integers(3))] for q in qs}))
    return terms


@pytest.mark.parametrize("nq", [7, 10, 13, 15])
def test_pauli_channel_has_a_source(L, nq):
    src, _, _ = L.channel_kernel_source(nq, _pauli(np.random.default_rng(nq), nq))
    assert "qcw_channel_tiled_spec" in src
    assert "typedef double CT;" in src  # Pauli coefficients are real
    assert src.count("const double2 own") == 4  # the thread's four own elements, read once


def test_no_source_without_a_tiled_plan(L):
    rng = np.random.default_rng(1)
    assert L.channel_kernel_source(6, _pauli(rng, 6))[0] == ""     # below 7 qubits
    general = [(0.1, {1: qi.random_unitary(rng, 2)})]                # not permutation type
    assert L.channel_kernel_source(9, general)[0] == ""


def test_source_depends_on_structure_not_weights(L):
    """Same qubits and operator kinds with other weights and p: one source,
    so the compiled kernel is shared.  Another flip pattern: another source."""
    nq = 9
    a = _pauli(np.random.default_rng(5), nq)
    b = [(w * 0.37, ops) for w, ops in a]
    sa = L.channel_kernel_source(nq, a)[0]
    assert sa == L.channel_kernel_source(nq, b)[0]
    c = [(w, {q: (qi.Z if K is qi.X else K) for q, K in ops.items()}) for w, ops in a]
    assert any(K is qi.X for _, ops in a for K in ops.values())
    assert L.channel_kernel_source(nq, c)[0] != sa


def test_complex_coefficients_select_complex_tables(L):
    rng = np.random.default_rng(3)
    ph = np.diag([1.0, np.exp(0.7j)])
    terms = _pauli(rng, 8) + [(0.01, {2: ph}), (0.01, {5: qi.X, 7: ph})]
    src, _, _ = L.channel_kernel_source(8, terms)
    assert "typedef double2 CT;" in src


@pytest.mark.parametrize("nq,seed", [(8, 11), (13, 5)])
def test_source_compiles_for_gfx950(L, nq, seed):
    """The run-time compiler (hipRTC, no device needed) turns the source into
    a code object."""
    rng = np.random.default_rng([seed, 7])
    src, code, ver = L.channel_kernel_source(nq, _pauli(rng, nq), compile=True)
    assert src and code > 1000
    assert ver >= 700  # the ROCm 7 installation's compiler


def test_bad_terms_rejected(L):
    with pytest.raises(RuntimeError):
        L.channel_kernel_source(0, [])
    with pytest.raises(RuntimeError):
        L.channel_kernel_source(9, [(0.1, {10: qi.X})])


def test_permutation_gate_gets_a_kernel_of_its_own(L):
    """qcw_channel_apply_gate folds a monomial gate (a permutation with
    phases) into the compiled kernel's stores: its source differs from the
    plain one only there, names the gate's bits, and compiles; a gate that
    mixes basis states (H) has no kernel of its own."""
    nq = 10
    terms = _pauli(np.random.default_rng(9), nq)
    plain = L.channel_kernel_source(nq, terms)[0]
    src, code, _ = L.channel_kernel_source(nq, terms, compile=True, gate=(qi.CNOT, (1, nq)))
    assert "gate_perm" in src and "gate_perm" not in plain and code > 1000
    # CNOT(1, nq): local index 2 q1 + q_nq on bits nq - 1 and 0; pi = (0, 1, 3, 2)
    assert "(((n >> 9) & 1u) << 1) | (((n >> 0) & 1u) << 0)" in src
    assert f"{0 | 1 << 3 | 3 << 6 | 2 << 9}u" in src
    assert L.channel_kernel_source(nq, terms, gate=(qi.H, (1,)))[0] == ""
    assert "gate_ur" not in src  # a plain permutation multiplies nothing
    # a monomial gate (phases) carries its phases, exactly
    z, codez, _ = L.channel_kernel_source(nq, terms, compile=True, gate=(np.diag([1.0, 1j]), (4,)))
    assert "gate_ur" in z and "0x1p+0" in z and codez > 1000
    toff, code3, _ = L.channel_kernel_source(nq, terms, compile=True, gate=(qi.TOFFOLI, (1, 2, 3)))
    assert "gate_perm" in toff and code3 > 1000


def test_observables_variant_compiles(L):
    """The kernel of qcw_channel_step_obs sums the observables as it stores:
    with and without a folded gate it compiles, and it writes one record of
    four sums per (tile, wave)."""
    nq = 9
    terms = _pauli(np.random.default_rng(4), nq)
    for gate in (None, (qi.CNOT, (1, nq)), (np.diag([1.0, -1.0]), (3,))):
        src, code, _ = L.channel_kernel_source(nq, terms, compile=True, gate=gate, observables=True)
        assert "o_pu" in src and "double *__restrict__ part" in src and code > 1000
        assert "wave_sum(o_pu)" in src  # register moves between lanes, no LDS round trip
    assert "o_pu" not in L.channel_kernel_source(nq, terms)[0]


def test_general_gate_on_the_last_qubits_gets_a_kernel(L):
    """A gate that mixes basis states is folded when every target is among
    the four last qubits (state bits 0..3, whose rows and columns each tile
    holds complete): the kernel runs U over the rows and conj(U) over the
    columns of the tile's outputs in LDS, its matrix passed with the launch.
    So the source depends on the targets, not on the matrix.  A target
    outside those qubits: no kernel of its own."""
    nq = 10
    rng = np.random.default_rng(12)
    terms = _pauli(rng, nq)
    h, code, _ = L.channel_kernel_source(nq, terms, compile=True, gate=(qi.H, (nq,)))
    assert "struct GateU { double v[8]; }" in h and "gu.v" in h and code > 1000
    assert "gate_perm" not in h  # no moved stores
    assert "gx[" in h  # the tile's outputs pass through LDS between the two passes
    rot = qi.random_unitary(rng, 2)
    assert L.channel_kernel_source(nq, terms, gate=(rot, (nq,)))[0] == h  # the matrix is an argument
    assert L.channel_kernel_source(nq, terms, gate=(qi.H, (nq - 1,)))[0] != h
    for U, t in ((qi.random_unitary(rng, 4), (nq, nq - 3)),
                 (qi.random_unitary(rng, 8), (nq - 1, nq - 3, nq))):
        for obs in (False, True):
            src, code, _ = L.channel_kernel_source(nq, terms, compile=True, gate=(U, t), observables=obs)
            assert f"double v[{2 * len(U) ** 2}]" in src and code > 1000
    for t in ((nq - 4,), (1,)):
        assert L.channel_kernel_source(nq, terms, gate=(qi.H, t))[0] == ""
    assert L.channel_kernel_source(nq, terms, gate=(qi.random_unitary(rng, 4), (nq, 2)))[0] == ""
