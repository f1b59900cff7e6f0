"""GPU parity of the one-gate sweep and the plain circuit path against the oracle.

Tolerances (FP64): a single gate or a circuit of G gates must satisfy
  ||psi_gpu - psi_oracle||_2 <= 1e-12 * max(1, G/64) * ||psi_oracle||_2 and
  max_n |psi_gpu[n] - psi_oracle[n]| <= 1e-12 * ||psi_oracle||_2.
A gate adds at most a few ulp per amplitude (m products and sums, one FMA
order on the GPU, plain products on the CPU): about 2*sqrt(2)*m^1.5*2^-53,
i.e. below 1e-14 at m = 8, so 1e-12 leaves room for ~100 gates.
Signed-permutation gates (X, Y, Z, CNOT, CZ, SWAP, Toffoli) move values
without rounding on both sides and must agree bit for bit.
"""
import itertools

import numpy as np
import pytest

import oracle
import qcw_inputs as qi
from golden_io import all_golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_1785_amd import _lib
    return _lib


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def close(a, b, G=1):
    nb = np.linalg.norm(b)
    scale = max(nb, 1e-300)
    assert np.linalg.norm(a - b) <= TOL * max(1.0, G / 64) * scale, np.linalg.norm(a - b) / scale
    assert np.max(np.abs(a - b)) <= TOL * scale


def rand_state(rng, nq):
    v = rng.uniform(-1, 1, 1 << nq) + 1j * rng.uniform(-1, 1, 1 << nq)
    return v / np.linalg.norm(v)


GOLDEN = all_golden()


@pytest.mark.parametrize("g", GOLDEN, ids=[g.name for g in GOLDEN])
def test_golden_on_gpu(L, g):
    print(f"[gpu] golden {g.name}", flush=True)
    psi = dev(g.init)
    L.circuit(psi, g.circ)
    g.check(host(psi))


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5])
def test_every_target_tuple_small(L, nq):
    print(f"[gpu] every target tuple nq={nq}", flush=True)
    rng = np.random.default_rng(300 + nq)
    psi0 = rand_state(rng, nq)
    for k in range(1, min(3, nq) + 1):
        for t in itertools.permutations(range(1, nq + 1), k):
            U = qi.random_matrix(rng, 1 << k)
            psi = dev(psi0)
            L.qcw_opk(k, t, U, psi)
            close(host(psi), oracle.apply(U, t, psi0))


@pytest.mark.parametrize("nq", [6, 7, 9, 11, 12, 13, 16, 20])
def test_sampled_targets_ragged_and_multi_tile(L, nq):
    """Sizes from a fraction of one block up to thousands of blocks (ragged tails)."""
    print(f"[gpu] sampled targets nq={nq}", flush=True)
    rng = np.random.default_rng(400 + nq)
    psi0 = rand_state(rng, nq)
    cases = [(1, (nq,)), (1, (1,)), (2, (nq, nq - 1)), (2, (1, nq)), (3, (nq, 1, nq // 2 + 1)),
             (3, (1, 2, 3)), (3, (nq - 2, nq, nq - 1))]
    for _ in range(4):
        k = int(rng.integers(1, 4))
        cases.append((k, tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False))))
    for k, t in cases:
        U = qi.random_matrix(rng, 1 << k)
        psi = dev(psi0)
        L.qcw_opk(k, t, U, psi)
        close(host(psi), oracle.apply(U, t, psi0))


def test_op1_op2_op3_entry_points(L):
    rng = np.random.default_rng(1)
    nq = 8
    psi0 = rand_state(rng, nq)
    U1, U2, U3 = (qi.random_unitary(rng, m) for m in (2, 4, 8))
    psi = dev(psi0)
    L.qcw_op1(U1, 3, psi)
    L.qcw_op2(U2, 7, 2, psi)
    L.qcw_op3(U3, 5, 8, 1, psi)
    ref = oracle.apply(U3, (5, 8, 1), oracle.apply(U2, (7, 2), oracle.apply(U1, (3,), psi0)))
    close(host(psi), ref, G=3)


def test_out_of_place_and_aliasing(L):
    rng = np.random.default_rng(2)
    nq = 10
    psi0 = rand_state(rng, nq)
    U = qi.random_unitary(rng, 4)
    a, b = dev(psi0), torch.zeros(1 << nq, dtype=torch.complex128, device="cuda")
    L.qcw_opk_to(2, (4, 9), U, a, b)
    ref = oracle.apply(U, (4, 9), psi0)
    close(host(b), ref)
    assert np.array_equal(host(a), psi0)            # input untouched
    L.qcw_opk_to(2, (4, 9), U, a, a)                # exact aliasing = in place
    assert np.array_equal(host(a), host(b))
    buf = torch.zeros(3 << nq, dtype=torch.complex128, device="cuda")
    with pytest.raises(L.QcwError, match="overlap"):
        L.qcw_opk_to(2, (4, 9), U, buf[: 1 << nq], buf[8: 8 + (1 << nq)])


def test_buffer_too_short_rejected(L):
    psi = torch.zeros(1 << 10, dtype=torch.complex128, device="cuda")
    with pytest.raises(L.QcwError, match="overrun"):
        L.qcw_op1(qi.H, 1, psi, nq=30)
    cpu = torch.zeros(8, dtype=torch.complex128)
    with pytest.raises(TypeError):
        L.qcw_op1(qi.H, 1, cpu)


@pytest.mark.parametrize("nq", [1, 3, 8, 15])
def test_omega_all(L, nq):
    psi = dev(qi.basis_state(nq, 0))
    L.qcw_omega_all(qi.H, psi)
    out = host(psi)
    assert np.max(np.abs(out - 2.0 ** (-nq / 2))) <= 4 * nq * 2.0 ** -53
    rng = np.random.default_rng(nq)
    psi0 = rand_state(rng, nq)
    U = qi.random_unitary(rng, 2)
    psi = dev(psi0)
    L.qcw_omega_all(U, psi)
    ref = psi0
    for q in range(1, nq + 1):
        ref = oracle.apply(U, (q,), ref)
    close(host(psi), ref, G=nq)


def _low_cases(nq):
    return [(nq, nq - 1), (nq - 1, nq), (nq, nq - 1, nq - 2), (nq - 2, nq, nq - 1),
            (nq - 1, nq, nq - 11), (nq - 11, nq - 1, nq)]


@pytest.mark.parametrize("nq", [12, 13, 17, 22])
def test_lowest_qubit_gates_tile_kernel(L, nq):
    """Gates on qubits nq and nq-1 with every target among the lowest 12 label
    bits run as contiguous LDS tiles: within the FP64 tolerance of the oracle,
    and bit for bit the one-gate fused pass (the sweep's arithmetic), in place
    and out of place."""
    print(f"[gpu] lowest-qubit tile kernel nq={nq}", flush=True)
    rng = np.random.default_rng(200 + nq)
    psi0 = rand_state(rng, nq)
    for t in _low_cases(nq):
        k = len(t)
        U = qi.random_unitary(rng, 1 << k)
        a = dev(psi0)
        L.qcw_opk(k, t, U, a)
        b = dev(psi0)
        L.circuit_fused(b, qi.Circuit(nq).add(U, *t), 12, low_bits=3)
        c = torch.empty_like(a)
        L.qcw_opk_to(k, t, U, dev(psi0), c)
        ha = host(a)
        assert np.array_equal(ha, host(b)), t
        assert np.array_equal(ha, host(c)), t
        close(ha, oracle.apply(U, t, psi0), G=1)


@pytest.mark.parametrize("nq", [21, 22, 25])
def test_omega_all_large_equals_sweeps_bitwise(L, nq):
    """From 22 qubits OmegaALL runs as fused passes: bit for bit the nq
    one-qubit sweeps (21 still runs the sweeps), and H on |0..0> gives the
    closed form 2^(-nq/2) everywhere."""
    print(f"[gpu] omega_all nq={nq}", flush=True)
    rng = np.random.default_rng(100 + nq)
    psi0 = rand_state(rng, nq)
    U = qi.random_unitary(rng, 2)
    a, b = dev(psi0), dev(psi0)
    L.qcw_omega_all(U, a)
    for q in range(1, nq + 1):
        L.qcw_op1(U, q, b)
    assert np.array_equal(host(a), host(b))
    psi = dev(qi.basis_state(nq, 0))
    L.qcw_omega_all(qi.H, psi)
    assert np.max(np.abs(host(psi) - 2.0 ** (-nq / 2))) <= 4 * nq * 2.0 ** -53


def test_permutation_gates_bit_exact(L):
    rng = np.random.default_rng(3)
    nq = 12
    psi0 = rand_state(rng, nq)
    for U, t in [(qi.X, (5,)), (qi.Y, (12,)), (qi.Z, (1,)), (qi.CNOT, (11, 3)),
                 (qi.CZ, (1, 12)), (qi.SWAP, (6, 7)), (qi.TOFFOLI, (12, 1, 6)),
                 (qi.TOFFOLI, (2, 3, 4))]:
        psi = dev(psi0)
        L.qcw_opk(len(t), t, U, psi)
        assert np.array_equal(host(psi), oracle.apply(U, t, psi0)), t


@pytest.mark.parametrize("nq", [3, 5, 9, 12, 16])
def test_random_circuits(L, nq):
    print(f"[gpu] circuit nq={nq}", flush=True)
    G = 4 * nq
    psi0 = qi.state(0, nq, tag=7)
    c = qi.circuit(0, nq, G, tag=7)
    psi = dev(psi0)
    L.circuit(psi, c)
    close(host(psi), oracle.circuit(c, psi0), G=G)


def test_pick_device_bit_exact(L):
    rng = np.random.default_rng(4)
    for nq in (1, 3, 7, 12, 18):
        for k in range(1, min(3, nq) + 1):
            for _ in range(3):
                t = tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False))
                assert np.array_equal(L.qcw_debug_pick_device(nq, t), oracle.pick(nq, t)), (nq, t)


@pytest.mark.parametrize("nq,G", [(1, 5), (3, 12), (5, 40), (8, 70), (11, 44)])
def test_small_state_circuit_equals_sweeps(L, nq, G):
    """States of at most 11 qubits run the whole circuit in one launch (a
    further launch per 32 gates or 224 matrix entries: G = 40 and 70 need
    several) with the state in LDS; the result equals one sweep per gate
    (qcw_opk on each gate, the path of larger states) bit for bit, and the
    launches are counted as QCW_KERNEL_SMALL."""
    c = qi.circuit(5, nq, G, tag=11)
    psi0 = qi.state(6, nq)
    a, b = dev(psi0), dev(psi0)
    L.qcw_timing_reset()
    L.qcw_timing_enable(True)
    try:
        L.circuit(a, c)
        n_small, _ = L.qcw_timing_read(L.QCW_KERNEL_SMALL)
    finally:
        L.qcw_timing_enable(False)
    for k, t, U in zip(c.ks, c.targets, c.mats):
        L.qcw_opk(k, t, U, b)
    assert np.array_equal(host(a), host(b))
    entries = [1 << (2 * k) for k in c.ks]
    launches, g, m = 1, 0, 0
    for e in entries:
        if g == 32 or m + e > 224:
            launches, g, m = launches + 1, 0, 0
        g, m = g + 1, m + e
    assert n_small == launches


def test_timing_counts_launches(L):
    psi = dev(qi.state(0, 12))
    L.qcw_timing_reset()
    L.qcw_timing_enable(True)
    try:
        for _ in range(3):
            L.qcw_op2(qi.CNOT, 1, 2, psi)
        n, ms = L.qcw_timing_read(L.QCW_KERNEL_SWEEP2)
    finally:
        L.qcw_timing_enable(False)
    assert n == 3 and ms > 0


# ------------------------------------------------------------------ full size
FULL_NQ = 31


@pytest.fixture(scope="module")
def full_state():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    need = 16 << FULL_NQ
    if free < 2 * need + (4 << 30):
        pytest.skip("not enough device memory for the full-size state")
    print(f"[gpu] generating the nq={FULL_NQ} state", flush=True)
    psi0 = qi.state(1, FULL_NQ)
    return psi0


@pytest.fixture(scope="module")
def state28():
    free, _ = torch.cuda.mem_get_info()
    if free < (2 * (16 << 28) + (4 << 30)):
        pytest.skip("not enough device memory")
    print("[gpu] generating the nq=28 state", flush=True)
    return qi.state(28, 28)


@pytest.mark.parametrize("k,targets", [(1, (15,)), (2, (28, 27)), (3, (1, 14, 28))])
def test_full_compare_nq28(L, state28, k, targets):
    """nq = 28 (4 GiB): every output of one gate against the oracle, the full
    elementwise comparison of the measurement plan (k = 2 on the two lowest
    qubits runs as LDS tiles)."""
    print(f"[gpu] full compare nq=28 k={k} targets={targets}", flush=True)
    rng = np.random.default_rng(280 + k)
    U = qi.random_unitary(rng, 1 << k)
    psi = dev(state28)
    L.qcw_opk(k, targets, U, psi)
    got = host(psi)
    del psi
    torch.cuda.empty_cache()
    close(got, oracle.apply(U, targets, state28), G=1)


@pytest.mark.parametrize("k,targets", [
    (1, (FULL_NQ,)), (1, (1,)), (1, (16,)),
    (2, (FULL_NQ, FULL_NQ - 1)), (2, (1, 2)), (2, (3, 29)),
    (3, (FULL_NQ, FULL_NQ - 1, FULL_NQ - 2)), (3, (1, 2, 3)), (3, (30, 4, 17))])
def test_fullsize_single_gate_sampled(L, full_state, k, targets):
    """nq = 31 (32 GiB), the benchmark's launch shape: 2^16 sampled outputs
    against the oracle's per-amplitude formula, plus the norm."""
    print(f"[gpu] full size k={k} targets={targets}", flush=True)
    rng = np.random.default_rng(k * 100 + targets[0])
    U = qi.random_unitary(rng, 1 << k)
    psi = torch.from_numpy(full_state).to("cuda")
    L.qcw_opk(k, targets, U, psi)
    idx = np.concatenate([np.arange(64), (1 << FULL_NQ) - 1 - np.arange(64),
                          rng.integers(0, 1 << FULL_NQ, 1 << 16)]).astype(np.int64)
    got = psi[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    ref = oracle.apply_at(U, targets, full_state, idx.astype(np.uint64))
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref))
    nrm = torch.linalg.vector_norm(psi).item()
    assert abs(nrm - 1.0) <= 1e-12
    del psi
    torch.cuda.empty_cache()


def test_fullsize_circuit_roundtrip(L, full_state):
    """nq = 31: a 124-gate random circuit keeps the norm, and the circuit then its
    inverse returns the input (a property that holds at any size)."""
    print("[gpu] full size circuit roundtrip", flush=True)
    c = qi.circuit(1, FULL_NQ, 4 * FULL_NQ)
    psi = torch.from_numpy(full_state).to("cuda")
    L.circuit(psi, c)
    nrm = torch.linalg.vector_norm(psi).item()
    assert abs(nrm - 1.0) <= 1e-11
    L.circuit(psi, c.inverse())
    ref = torch.from_numpy(full_state).to("cuda")
    err = torch.linalg.vector_norm(psi - ref).item()
    assert err <= TOL * max(1.0, 2 * len(c) / 64)
    del psi, ref
    torch.cuda.empty_cache()
