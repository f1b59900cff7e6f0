"""GPU parity of the multiverse density-matrix step against the density oracle.

Tolerance: elementwise |rho_gpu - rho_oracle| <= 1e-12 (rho has unit trace,
so its elements are at most 1); observables within 1e-12.
"""
import numpy as np
import pytest

import qcw_inputs as qi
from oracle import density as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_1785_amd import _lib
    return _lib


def dev(r):
    return torch.from_numpy(np.ascontiguousarray(r, dtype=np.complex128).reshape(-1)).to("cuda")


def host(t, nq):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(1 << nq, 1 << nq)


def _rand_rho(rng, nq, rank=3):
    A = rng.normal(size=(1 << nq, rank)) + 1j * rng.normal(size=(1 << nq, rank))
    r = A @ A.conj().T
    return r / np.trace(r)


def _terms(rng, nq, n_p, eps, unitary=True):
    terms = []
    for s, ps in ((1, 0.95), (2, 0.05)):
        if s == 2 and nq < 2:
            continue
        for _ in range(n_p):
            qs = [int(x) + 1 for x in rng.choice(nq, s, replace=False)]
            ops = {q: (qi.random_unitary(rng, 2) if unitary else qi.random_matrix(rng, 2))
                   for q in qs}
            terms.append((eps * ps / n_p, ops))
    return terms


def _pauli_terms(rng, nq, n_p=16, eps=0.2):
    P = [qi.X, qi.Y, qi.Z]
    terms = []
    for s, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(n_p):
            qs = [int(x) + 1 for x in rng.choice(nq, s, replace=False)]
            terms.append((eps * ps / n_p, {q: P[int(rng.integers(3))] for q in qs}))
    return terms


def _apply(L, ch, rho0, nq, force_gather=-1):
    ch.plan(force_gather)
    a, b = dev(rho0), torch.empty(1 << (2 * nq), dtype=torch.complex128, device="cuda")
    ch.apply(a, b)
    return host(b, nq)


@pytest.mark.parametrize("nq", [2, 5, 7, 9])
@pytest.mark.parametrize("kernel", ["auto", "gather"])
def test_pauli_channel_matches_oracle(L, nq, kernel):
    """Pauli-type hits (each output element gathers the flipped elements).
    From nq = 7 a channel of such terms runs the tiled kernel; the gather
    kernel (forced here) visits elements in its cache-ordered sequence there.
    Neither order may change a result."""
    rng = np.random.default_rng(90 + nq)
    rho0 = _rand_rho(rng, nq)
    terms = _pauli_terms(rng, nq)
    ch = L.Channel(nq, 0.8, terms)
    out = _apply(L, ch, rho0, nq, 1 if kernel == "gather" else 0)
    assert ch.plan()["gather_kernel"] == (1 if kernel == "gather" or nq < 7 else 0)
    assert np.max(np.abs(out - D.channel(rho0, 0.8, terms))) <= TOL
    ch.close()


@pytest.mark.parametrize("kernel", ["auto", "gather"])
def test_pauli_channel_many_terms_matches_oracle(L, kernel):
    """300 Pauli-type hits: more than the gather kernel stages in LDS (256),
    so that kernel chooses coefficients from scalar registers; the tiled
    kernel groups them into mask groups of many segments."""
    nq = 7
    rng = np.random.default_rng(97)
    rho0 = _rand_rho(rng, nq)
    terms = _pauli_terms(rng, nq, n_p=150)
    ch = L.Channel(nq, 0.8, terms)
    out = _apply(L, ch, rho0, nq, 1 if kernel == "gather" else 0)
    assert np.max(np.abs(out - D.channel(rho0, 0.8, terms))) <= TOL
    ch.close()


def _phase(rng):
    return np.diag([np.exp(1j * rng.uniform(0, 2 * np.pi)), np.exp(1j * rng.uniform(0, 2 * np.pi))])


def _flip_phase(rng):
    return np.array([[0, np.exp(1j * rng.uniform(0, 2 * np.pi))],
                     [np.exp(1j * rng.uniform(0, 2 * np.pi)), 0]])


def _tiled_case(kind, nq, seed):
    """Permutation-type channels shaped to reach every part of the tiled plan.
    pauli: the multiverse noise of Eq. rhoE4 (real coefficients); phase: Pauli
    operators mixed with random phases and phased flips (complex
    coefficients); zheavy: many Z and ZZ hits (flip-free group of several
    segments) and flips on bits 0..3 (the tile itself staged); pairs: a flip
    on one of up to four far qubits with one on bits 0..3 (partners read by several
    read sets, staged)."""
    rng = np.random.default_rng(seed)
    P = [qi.X, qi.Y, qi.Z]
    terms = []
    if kind == "pauli":
        return _pauli_terms(rng, nq)
    if kind == "phase":
        ops = [qi.X, qi.Y, qi.Z, D.SX, _phase, _flip_phase]
        for s in (1, 2) * 12:
            qs = [int(x) + 1 for x in rng.choice(nq, s, replace=False)]
            op = {}
            for q in qs:
                o = ops[int(rng.integers(len(ops)))]
                op[q] = o(rng) if callable(o) else o
            terms.append((0.2 / 24, op))
        return terms
    if kind == "zheavy":
        for _ in range(20):
            qs = [int(x) + 1 for x in rng.choice(nq, 1 + int(rng.integers(2)), replace=False)]
            terms.append((0.1 / 20, {q: qi.Z for q in qs}))
        for _ in range(10):   # flips among the four lowest bits (qubits nq-3 .. nq)
            q = nq - int(rng.integers(4))
            terms.append((0.1 / 10, {q: P[int(rng.integers(2))]}))
        return terms
    if kind == "pairs":   # a flip on one of four far qubits (bits >= 4) with one on bits 0..3
        far = [int(x) + 1 for x in rng.choice(nq - 4, min(4, nq - 4), replace=False)]
        for _ in range(24):
            qa, lo = far[int(rng.integers(len(far)))], nq - int(rng.integers(4))
            terms.append((0.2 / 24, {qa: P[int(rng.integers(2))], lo: P[int(rng.integers(3))]}))
        return terms
    raise ValueError(kind)


TILED_CASES = [("pauli", 7, 1), ("pauli", 10, 2), ("phase", 8, 3), ("phase", 9, 4),
               ("zheavy", 8, 5), ("pairs", 9, 6), ("pairs", 7, 7)]


@pytest.mark.parametrize("kind,nq,seed", TILED_CASES)
def test_tiled_channel_matches_oracle(L, kind, nq, seed):
    """The tiled channel kernel against the oracle's Kronecker-product channel,
    elementwise (Eqs. rhoE1, rhoE4)."""
    rng = np.random.default_rng(1000 + seed)
    rho0 = _rand_rho(rng, nq)
    terms = _tiled_case(kind, nq, seed)
    ch = L.Channel(nq, 0.8, terms)
    assert ch.plan()["tiled_plan"] == 1
    out = _apply(L, ch, rho0, nq, 0)
    assert ch.plan()["compiled_kernel"] == 1
    assert np.max(np.abs(out - D.channel(rho0, 0.8, terms))) <= TOL
    ch.close()


@pytest.mark.parametrize("kind,nq,seed", TILED_CASES + [("pauli", 12, 8), ("pauli", 13, 9)])
def test_compiled_tiled_kernel_equals_generic(L, kind, nq, seed):
    """The tiled kernel compiled for the channel's plan at creation against
    the generic tiled kernel, which reads the same plan from memory: the same
    groups, segments and operations in the same order, so the outputs agree
    bit for bit (nq = 13: a 1 GiB rho, several thousand tiles per XCD)."""
    print(f"[gpu] compiled vs generic tiled channel {kind} nq={nq}", flush=True)
    rng = np.random.default_rng(2000 + seed)
    terms = _pauli_terms(rng, nq) if nq >= 12 else _tiled_case(kind, nq, seed)
    ch = L.Channel(nq, 0.8, terms)
    assert ch.plan(L.Channel.KERNEL_TILED)["compiled_kernel"] == 1
    NN = 1 << (2 * nq)
    g = torch.Generator(device="cuda").manual_seed(seed)
    a = torch.complex(torch.randn(NN, dtype=torch.float64, device="cuda", generator=g),
                      torch.randn(NN, dtype=torch.float64, device="cuda", generator=g))
    b1 = torch.full_like(a, float("nan"))
    b2 = torch.full_like(a, float("nan"))
    ch.apply(a, b1)
    assert ch.plan(L.Channel.KERNEL_TILED_GENERIC)["compiled_kernel"] == 0
    ch.apply(a, b2)
    ch.apply(a, b2)  # twice: the ticket counters start from zero again
    torch.cuda.synchronize()
    ch.close()
    assert not bool(torch.isnan(b1).any())
    assert torch.equal(torch.view_as_real(b1), torch.view_as_real(b2))


def _step_gates(nq):
    """Algorithm gates for the one-call step: permutation and monomial
    matrices (phases, Y, CZ, a phased swap) with targets among the tile's
    thread bits (the last qubits), its E bits or the rest; gates that mix
    basis states on the four last qubits (H, a rotation, dense two- and
    three-qubit unitaries: also one pass); and two that mix basis states with
    a target outside them (the two-kernel path)."""
    S = np.diag([1.0, 1j])
    CZ = np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128)
    phased_swap = np.array([[np.exp(0.3j), 0, 0, 0], [0, 0, -1j, 0], [0, np.exp(-1.1j), 0, 0],
                            [0, 0, 0, 0.6 - 0.8j]])
    rot = np.array([[np.cos(0.4), -np.sin(0.4)], [np.sin(0.4), np.cos(0.4)]], dtype=np.complex128)
    return [(qi.CNOT, (1, 2)), (qi.CNOT, (nq, 1)), (qi.CNOT, (nq - 1, nq)), (qi.CNOT, (3, nq - 2)),
            (qi.X, (nq // 2,)), (qi.SWAP, (2, nq)), (qi.TOFFOLI, (nq, 1, nq - 3)),
            (S, (nq - 1,)), (qi.Z, (1,)), (qi.Y, (nq,)), (CZ, (nq - 2, 2)),
            (phased_swap, (nq, nq // 2)), (qi.H, (1,)), (rot, (nq - 1,)), (qi.H, (nq,)),
            (qi.random_unitary(np.random.default_rng(nq), 4), (nq, nq - 3)),
            (qi.random_unitary(np.random.default_rng(nq + 3), 4), (nq, nq - 1)),
            (qi.random_unitary(np.random.default_rng(nq + 1), 8), (nq - 1, nq - 3, nq)),
            (qi.random_unitary(np.random.default_rng(nq + 2), 4), (nq - 2, 2))]


def _monomial(U):
    nz = np.abs(U) != 0
    return bool(np.all(nz.sum(0) == 1) and np.all(nz.sum(1) == 1))


def _one_pass(U, t, nq):
    """Whether the compiled kernel takes the gate in the channel's pass: a
    monomial gate anywhere, any other gate with every target among the four
    last qubits (state bits 0..3, complete in each tile)."""
    return _monomial(U) or all(nq - q <= 3 for q in t)


@pytest.mark.parametrize("kind,nq,seed", [("pauli", 9, 1), ("phase", 8, 3), ("zheavy", 8, 5),
                                          ("pairs", 9, 6), ("pauli", 12, 8), ("pauli", 13, 9)])
def test_channel_apply_gate_equals_channel_then_conjugation(L, kind, nq, seed):
    """One multiverse step in one call (qcw_channel_apply_gate): for a
    monomial gate (U|l> = u_l |pi(l)>) the compiled kernel stores output
    (n, m), times u_l(n) conj(u_l(m)), at (pi(n), pi(m)); for any other gate
    on the four last qubits it applies U to the rows and conj(U) to the
    columns of each tile's outputs in LDS; either way the step is one pass.
    It must equal the channel followed by qcw_rho_conjugate exactly (values
    equal; only zeros may differ in sign), and, up to nq = 9, the oracle's
    channel and conjugation to 1e-12.  The timing counters show which path
    ran."""
    print(f"[gpu] channel + gate in one call {kind} nq={nq}", flush=True)
    rng = np.random.default_rng(3000 + seed)
    terms = _pauli_terms(rng, nq) if kind == "pauli" else _tiled_case(kind, nq, seed)
    ch = L.Channel(nq, 0.8, terms)
    assert ch.plan()["compiled_kernel"] == 1
    NN = 1 << (2 * nq)
    g = torch.Generator(device="cuda").manual_seed(seed)
    a = torch.complex(torch.randn(NN, dtype=torch.float64, device="cuda", generator=g),
                      torch.randn(NN, dtype=torch.float64, device="cuda", generator=g))
    for U, t in _step_gates(nq):
        perm = _one_pass(U, t, nq)
        b1 = torch.full_like(a, float("nan"))
        b2 = torch.full_like(a, float("nan"))
        torch.cuda.synchronize()
        L.qcw_timing_reset()
        L.qcw_timing_enable(True)
        ch.apply_gate(a, b1, U, t)
        n_ch, _ = L.qcw_timing_read(L.QCW_KERNEL_CHANNEL)
        n_cj, _ = L.qcw_timing_read(L.QCW_KERNEL_CONJ)
        L.qcw_timing_enable(False)
        assert (n_ch, n_cj) == ((1, 0) if perm else (1, 1)), (t, n_ch, n_cj)
        ch.apply(a, b2)
        L.qcw_rho_conjugate(len(t), t, U, b2)
        torch.cuda.synchronize()
        assert not bool(torch.isnan(b1).any()), t
        assert torch.equal(b1, b2), t
        if perm and nq <= 9:  # the folded step against the oracle directly
            want = D.conjugate(D.channel(host(a, nq), 0.8, terms), U, t)
            assert np.max(np.abs(host(b1, nq) - want)) <= TOL, t
    ch.close()


def test_channel_apply_gate_other_kernels(L):
    """Without the compiled tiled kernel (the gather kernel, the generic
    tiled kernel, or nq below the tiled range) the call is the channel then
    the conjugation, with the same result."""
    for nq, choice in ((6, -1), (8, 1), (8, 2)):
        rng = np.random.default_rng(40 + nq + choice)
        terms = _pauli_terms(rng, nq)
        ch = L.Channel(nq, 0.8, terms)
        ch.plan(choice)
        rho0 = _rand_rho(rng, nq)
        for U, t in ((qi.CNOT, (1, nq)), (qi.H, (2,))):
            a = dev(rho0)
            b1 = torch.empty_like(a)
            b2 = torch.empty_like(a)
            ch.apply_gate(a, b1, U, t)
            ch.apply(a, b2)
            L.qcw_rho_conjugate(len(t), t, U, b2)
            assert torch.equal(b1, b2)
            want = D.conjugate(D.channel(rho0, 0.8, terms), U, t)
            assert np.max(np.abs(host(b1, nq) - want)) <= TOL
        ch.close()


@pytest.mark.parametrize("kind,nq,seed,choice", [("pauli", 9, 1, -1), ("phase", 8, 3, -1),
                                                 ("pauli", 12, 8, -1), ("pauli", 6, 2, -1),
                                                 ("pauli", 8, 4, 1), ("pauli", 8, 5, 2)])
def test_channel_step_obs_matches_observables(L, kind, nq, seed, choice):
    """qcw_channel_step_obs: the step equals qcw_channel_apply_gate (or the
    channel alone), and its four observables equal qcw_rho_observables of the
    result to 1e-12, the same bits on a repeated call.  Summed in the
    compiled kernel (nq = 8, 9, 12 with the default kernel choice) or by the
    observables kernels (nq = 6; the gather and generic tiled kernels).  The
    polarisations come from the same kernel as qcw_rho_observables': equal
    bits."""
    print(f"[gpu] step with observables {kind} nq={nq} kernel={choice}", flush=True)
    rng = np.random.default_rng(5000 + seed)
    terms = _pauli_terms(rng, nq) if kind == "pauli" else _tiled_case(kind, nq, seed)
    ch = L.Channel(nq, 0.8, terms)
    ch.plan(choice)
    rho0 = _rand_rho(rng, nq)
    psi = rng.normal(size=1 << nq) + 1j * rng.normal(size=1 << nq)
    psi /= np.linalg.norm(psi)
    psi_d = torch.from_numpy(psi).to("cuda")
    a = dev(rho0)
    obs = torch.empty(4 + 3 * nq, dtype=torch.float64, device="cuda")
    for U, t in ((qi.CNOT, (1, nq)), (qi.Z, (2,)), (qi.H, (1,)), (qi.H, (nq,)),
                 (qi.random_unitary(rng, 4), (nq - 1, nq - 2)), (None, ())):
        b1 = torch.full_like(a, float("nan"))
        b2 = torch.full_like(a, float("nan"))
        ch.step_obs(a, b1, obs, U, t, psi0=psi_d)
        o1 = obs.cpu().numpy().copy()
        ch.step_obs(a, b1, obs, U, t, psi0=psi_d)
        o2 = obs.cpu().numpy().copy()
        assert np.array_equal(o1, o2), t
        if U is None:
            ch.apply(a, b2)
        else:
            ch.apply_gate(a, b2, U, t)
        torch.cuda.synchronize()
        assert torch.equal(b1, b2), t
        ref = L.qcw_rho_observables(b2, psi0=psi)
        want = [ref["trace"].real, ref["trace"].imag, ref["purity"], ref["fidelity"]]
        assert np.max(np.abs(o1[:4] - np.array(want))) <= 1e-12, (t, o1[:4], want)
        assert np.array_equal(o1[4:].reshape(nq, 3), ref["polarization"]), t
    ch.step_obs(a, b1, obs, qi.CNOT, (1, 2))  # no psi0: NaN fidelity
    assert np.isnan(obs.cpu().numpy()[3])
    ch.close()


def test_channel_apply_gate_rejects_bad_input(L):
    ch = L.Channel(8, 0.8, _pauli_terms(np.random.default_rng(1), 8))
    a = torch.zeros(1 << 16, dtype=torch.complex128, device="cuda")
    b = torch.zeros_like(a)
    with pytest.raises(RuntimeError):
        ch.apply_gate(a, b, qi.CNOT, (1, 1))       # repeated target
    with pytest.raises(RuntimeError):
        ch.apply_gate(a, b, qi.CNOT, (1, 9))       # target outside [1, nq]
    with pytest.raises(RuntimeError):
        ch.apply_gate(a, a, qi.CNOT, (1, 2))       # rho_in == rho_out
    obs = torch.empty(4 + 3 * 8, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        ch.step_obs(a, b, obs, qi.CNOT, (2, 2))    # repeated target
    with pytest.raises(RuntimeError):
        ch.step_obs(a, a, obs, qi.CNOT, (1, 2))    # rho_in == rho_out
    ch.close()


def test_tiled_channel_plan_coverage(L):
    """The cases above reach every part of the tiled kernel: partners staged
    in LDS and read directly, the tile itself staged, segments on the tile
    bits, groups of several segments, real and complex coefficients."""
    seen = {"staged": 0, "direct": 0, "own_staged": 0, "etouch_segments": 0, "multi_seg": 0,
            "real": set()}
    for kind, nq, seed in TILED_CASES:
        ch = L.Channel(nq, 0.8, _tiled_case(kind, nq, seed))
        p = ch.plan()
        ch.close()
        for k in ("staged", "direct", "own_staged", "etouch_segments"):
            seen[k] += p[k]
        seen["multi_seg"] += p["segments"] > p["groups"]
        seen["real"].add(p["real"])
    assert seen["staged"] and seen["direct"] and seen["own_staged"], seen
    assert seen["etouch_segments"] and seen["multi_seg"], seen
    assert seen["real"] == {0, 1}, seen


def test_tiled_channel_without_terms(L):
    """A channel of no paths keeps p rho: the tiled kernel's plan is the tile
    itself with no groups, and every output is p times its input exactly."""
    nq = 8
    rng = np.random.default_rng(300)
    rho0 = _rand_rho(rng, nq)
    ch = L.Channel(nq, 0.7, [])
    assert ch.plan()["tiled_plan"] == 1 and ch.plan()["groups"] == 0
    out = _apply(L, ch, rho0, nq, 0)
    assert ch.plan()["compiled_kernel"] == 1
    ch.close()
    assert np.array_equal(out, 0.7 * rho0)


def test_tiled_channel_15_qubits_basis_state(L):
    """nq = 15, the largest state of the tiled kernel (2^30 elements, 16 GiB
    each for input and output): on |0..0><0..0| a Pauli hit moves weight w_t
    to the diagonal element at its flip mask, so the output is p at (0, 0)
    plus the flip-free hits, w summed per flip mask f at (f, f), and zero
    elsewhere (the output starts as NaN, so every element must be written)."""
    nq = 15
    N = 1 << nq
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 2 * 16 * N * N + (8 << 30):
        pytest.skip("needs 40 GiB of free device memory")
    print(f"[gpu] tiled pauli channel nq={nq} on a basis state", flush=True)
    rng = np.random.default_rng(15)
    P = {"X": qi.X, "Y": qi.Y, "Z": qi.Z}
    terms, expect = [], {0: 0.8}
    for s_, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(16):
            qs = [int(x) + 1 for x in rng.choice(nq, s_, replace=False)]
            names = {q: "XYZ"[int(rng.integers(3))] for q in qs}
            w = 0.2 * ps / 16
            terms.append((w, {q: P[n] for q, n in names.items()}))
            f = sum(1 << (nq - q) for q, n in names.items() if n != "Z")
            expect[f] = expect.get(f, 0.0) + w
    ch = L.Channel(nq, 0.8, terms)
    assert ch.plan()["gather_kernel"] == 0
    a = torch.zeros(N * N, dtype=torch.complex128, device="cuda")
    a[0] = 1.0
    b = torch.full_like(a, float("nan"))
    ch.apply(a, b)
    ch.close()
    del a
    assert not bool(torch.isnan(b).any())
    assert int(torch.count_nonzero(b).item()) == len(expect)
    idx = torch.tensor([f * N + f for f in expect], device="cuda")
    got = b[idx].cpu().numpy()
    assert np.allclose(got, list(expect.values()), rtol=0, atol=1e-15)
    assert abs(complex(b.sum().item()) - 1.0) <= 1e-14
    del b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nq,kind", [(11, "pauli"), (12, "pauli"), (12, "phase")])
def test_tiled_channel_equals_gather_kernel(L, nq, kind):
    """Beyond the oracle's reach: the tiled and the gather kernels, two
    independent evaluations of the same sums, agree elementwise on a random
    density matrix."""
    print(f"[gpu] tiled vs gather channel nq={nq} {kind}", flush=True)
    rng = np.random.default_rng(2000 + nq)
    rho0 = _rand_rho(rng, nq)
    terms = _tiled_case(kind, nq, 50 + nq)
    ch = L.Channel(nq, 0.8, terms)
    t = _apply(L, ch, rho0, nq, 0)
    g = _apply(L, ch, rho0, nq, 1)
    ch.close()
    assert np.max(np.abs(t - g)) <= TOL
    assert abs(np.trace(t) - 1) <= 1e-12 and np.max(np.abs(t - t.conj().T)) <= TOL


@pytest.mark.parametrize("nq", [1, 2, 3, 5, 7])
def test_conjugate_matches_oracle(L, nq):
    rng = np.random.default_rng(nq)
    rho0 = _rand_rho(rng, nq)
    for k in range(1, min(3, nq) + 1):
        t = tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False))
        U = qi.random_unitary(rng, 1 << k)
        r = dev(rho0)
        L.qcw_rho_conjugate(k, t, U, r)
        assert np.max(np.abs(host(r, nq) - D.conjugate(rho0, U, t))) <= TOL


@pytest.mark.parametrize("nq", [5, 6, 8, 11])
def test_conjugate_equals_two_sweeps(L, nq):
    """From nq = 5 qcw_rho_conjugate applies U and conj(U) in one pass of LDS
    tiles; the result equals the sweep of U on the row qubits followed by the
    sweep of conj(U) on the column qubits (qcw_opk on rho read as a
    2nq-qubit state) bit for bit, for k = 1, 2, 3, targets in any order and
    targets among the lowest qubits (whose bits are always tile bits)."""
    rng = np.random.default_rng(400 + nq)
    rho0 = _rand_rho(rng, nq)
    cases = [(1, (nq,)), (1, (1,)), (2, (nq, nq - 1)), (2, (1, nq)), (2, (nq - 1, 2)),
             (3, (nq - 2, 1, nq)), (3, (2, nq - 1, 3)),
             (3, tuple(int(x) + 1 for x in rng.choice(nq, 3, replace=False)))]
    for k, t in cases:
        U = qi.random_unitary(rng, 1 << k)
        a = dev(rho0)
        L.qcw_rho_conjugate(k, t, U, a)
        b = dev(rho0)
        L.qcw_opk(k, t, U, b, nq=2 * nq)
        L.qcw_opk(k, tuple(x + nq for x in t), np.conj(U), b, nq=2 * nq)
        assert np.array_equal(host(a, nq), host(b, nq)), (k, t)
        if nq <= 8:
            assert np.max(np.abs(host(a, nq) - D.conjugate(rho0, U, t))) <= TOL, (k, t)


@pytest.mark.parametrize("nq", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("unitary", [True, False])
def test_channel_matches_oracle(L, nq, unitary):
    rng = np.random.default_rng(10 * nq + unitary)
    rho0 = _rand_rho(rng, nq)
    terms = _terms(rng, nq, 8, 0.2, unitary)
    ch = L.Channel(nq, 0.8, terms)
    a, b = dev(rho0), torch.empty(1 << (2 * nq), dtype=torch.complex128, device="cuda")
    ch.apply(a, b)
    assert np.max(np.abs(host(b, nq) - D.channel(rho0, 0.8, terms))) <= TOL
    ch.close()


@pytest.mark.parametrize("nq", [1, 3, 6])
def test_observables_match_oracle(L, nq):
    rng = np.random.default_rng(20 + nq)
    rho = _rand_rho(rng, nq)
    psi0 = qi.state(2, nq)
    got = L.qcw_rho_observables(dev(rho), psi0=psi0)
    ref = D.observables(rho, psi0)
    assert abs(got["trace"] - ref["trace"]) <= TOL
    assert abs(got["purity"] - ref["purity"]) <= TOL
    assert abs(got["fidelity"] - ref["fidelity"]) <= TOL
    assert np.max(np.abs(got["polarization"] - ref["polarization"])) <= TOL
    assert np.isnan(L.qcw_rho_observables(dev(rho))["fidelity"])


def _run_sequence(L, nq, psi0, schedule, p_keep, terms):
    """schedule: list of gates (U, targets) or 'noise'; returns per-step observables
    from the GPU and the oracle."""
    rho_o = D.pure(psi0)
    a = dev(rho_o)
    b = torch.empty_like(a)
    ch = L.Channel(nq, p_keep, terms)
    gpu, orc = [], []
    for step in schedule:
        if step == "noise":
            ch.apply(a, b)
            a, b = b, a
            rho_o = D.channel(rho_o, p_keep, terms)
        else:
            U, t = step
            L.qcw_rho_conjugate(len(t), t, U, a)
            rho_o = D.conjugate(rho_o, U, t)
        gpu.append(L.qcw_rho_observables(a, psi0=psi0))
        orc.append(D.observables(rho_o, psi0))
    ch.close()
    return gpu, orc, host(a, nq), rho_o


def test_mv1_sequence(L):
    """§5 MV1-Noise: |0>, H at step 1, noise, H at step 3, then noise; without
    noise the fidelity is 1/sqrt2 after the first H and 1 after the second."""
    psi0 = qi.basis_state(1, 0)
    sched = [(qi.H, (1,)), "noise", (qi.H, (1,))] + ["noise"] * 6
    xyz = [(0.2 / 3, {1: s}) for s in (D.SX, D.SY, D.SZ)]
    gpu, orc, r_g, r_o = _run_sequence(L, 1, psi0, sched, 0.8, xyz)
    for g, o in zip(gpu, orc):
        assert abs(g["fidelity"] - o["fidelity"]) <= TOL
        assert abs(g["purity"] - o["purity"]) <= TOL
    assert np.max(np.abs(r_g - r_o)) <= TOL
    gpu0, _, _, _ = _run_sequence(L, 1, psi0, sched, 1.0, [])
    assert abs(gpu0[0]["fidelity"] - 2 ** -0.5) <= 4e-16
    assert abs(gpu0[2]["fidelity"] - 1.0) <= 4e-16


def test_mv2_sequence(L):
    """§5 MV2-Noise: Bell circuit, noise, inverse Bell, noise (X/Y/Z single and
    double hits)."""
    rng = np.random.default_rng(5)
    psi0 = qi.basis_state(2, 0)
    sched = [(qi.H, (1,)), "noise", (qi.CNOT, (1, 2)), "noise", (qi.CNOT, (1, 2)),
             (qi.H, (1,))] + ["noise"] * 4
    paulis = (D.SX, D.SY, D.SZ)
    terms = [(0.2 * 0.95 / 8, {int(rng.integers(1, 3)): paulis[i % 3]}) for i in range(8)] + \
            [(0.2 * 0.05 / 8, {1: paulis[i % 3], 2: paulis[(i + 1) % 3]}) for i in range(8)]
    gpu, orc, r_g, r_o = _run_sequence(L, 2, psi0, sched, 0.8, terms)
    for g, o in zip(gpu, orc):
        assert abs(g["fidelity"] - o["fidelity"]) <= TOL
        assert np.max(np.abs(g["polarization"] - o["polarization"])) <= TOL
    assert np.max(np.abs(r_g - r_o)) <= TOL


def test_mvn_ghz_with_noise(L):
    """§5 MVn-Noise: five qubits, H_1 then the CNOT_1j chain, noise between steps."""
    rng = np.random.default_rng(6)
    nq = 5
    psi0 = qi.basis_state(nq, 0)
    sched = [(qi.H, (1,)), "noise"]
    for t in range(2, nq + 1):
        sched += [(qi.CNOT, (1, t)), "noise"]
    terms = _terms(rng, nq, 16, 0.2)
    gpu, orc, r_g, r_o = _run_sequence(L, nq, psi0, sched, 0.8, terms)
    assert np.max(np.abs(r_g - r_o)) <= TOL
    assert abs(gpu[-1]["purity"] - orc[-1]["purity"]) <= TOL


def test_large_rho_properties(L):
    """nq = 12 (16M elements): trace and hermiticity preserved by the channel."""
    nq = 12
    rng = np.random.default_rng(7)
    v = qi.state(3, nq)
    a = dev(np.outer(v, v.conj()))
    b = torch.empty_like(a)
    ch = L.Channel(nq, 0.8, _terms(rng, nq, 16, 0.2))
    ch.apply(a, b)
    ob = L.qcw_rho_observables(b)
    assert abs(ob["trace"] - 1) <= 1e-12
    assert ob["purity"] < 1.0
    m = b.reshape(1 << nq, 1 << nq)
    assert torch.max(torch.abs(m - m.conj().T)).item() <= 1e-15
    ch.close()


def test_channel_validation(L):
    with pytest.raises(L.QcwError):
        L.Channel(3, 0.5, [(0.5, {4: D.SX})])
    with pytest.raises(L.QcwError):
        L.Channel(18, 0.5, [])
    ch = L.Channel(2, 1.0, [])
    a = torch.zeros(16, dtype=torch.complex128, device="cuda")
    with pytest.raises(L.QcwError, match="overlap"):
        ch.apply(a, a)
    ch.close()


# ------------------------------------------------------------------ eigen observables
@pytest.mark.parametrize("nq", [1, 2, 3, 5, 6])
def test_eigvals_and_entropy(L, nq):
    rng = np.random.default_rng(40 + nq)
    for rank in (1, 3, 1 << nq):
        rho = _rand_rho(rng, nq, rank)
        ev, S = L.qcw_rho_eigvals(dev(rho))
        ref = D.eigen_observables(rho)
        assert np.max(np.abs(ev - ref["eigenvalues"])) <= 1e-13
        assert abs(S - ref["entropy_bits"]) <= 1e-11


def test_classical_limit_on_gpu(L):
    """Repeated X and Z noise on every qubit drives the eigenvalues to 1/2^nq and
    the entropy to nq bits (§5, classical limit)."""
    nq = 3
    rng = np.random.default_rng(50)
    a = dev(_rand_rho(rng, nq))
    b = torch.empty_like(a)
    xz = [(0.3 / (2 * nq), {q: s}) for q in range(1, nq + 1) for s in (D.SX, D.SZ)]
    ch = L.Channel(nq, 0.7, xz)
    for _ in range(300):
        ch.apply(a, b)
        a, b = b, a
    ev, S = L.qcw_rho_eigvals(a)
    assert np.max(np.abs(ev - 1 / 8)) <= 1e-12 and abs(S - nq) <= 1e-10
    ch.close()


# Fidelity bar.  Full-rank pairs: 1e-12 against the oracle (the definition
# written out with numpy's Hermitian solver).  Rank-deficient inputs (pure
# states): the oracle's square roots of rounding-level eigenvalues add ~1e-8
# each, so those cases are checked against closed forms instead, at 1e-12:
# F(rho, |psi0><psi0|) = sqrt(<psi0|rho|psi0>), and by the symmetry of F,
# F(|psi><psi|, rho0) = sqrt(<psi|rho0|psi>); F(rho, rho) = 1.
FID_TOL = 1e-12


@pytest.mark.parametrize("nq", [1, 2, 4, 5, 6])
def test_general_fidelity(L, nq):
    rng = np.random.default_rng(60 + nq)
    full = 1 << nq
    r, r0 = _rand_rho(rng, nq, full), _rand_rho(rng, nq, full)
    assert abs(L.qcw_rho_fidelity(dev(r), dev(r0)) - D.fidelity_general(r, r0)) <= FID_TOL
    # pure reference (the paper's case: fidelity against the initial state)
    psi0 = qi.state(3, nq)
    f = L.qcw_rho_fidelity(dev(r), dev(D.pure(psi0)))
    assert abs(f - D.observables(r, psi0)["fidelity"]) <= FID_TOL
    # pure state against a mixed reference
    psi = qi.state(4, nq)
    g = L.qcw_rho_fidelity(dev(D.pure(psi)), dev(r0))
    assert abs(g - np.sqrt(np.real(psi.conj() @ r0 @ psi))) <= FID_TOL
    # a state against itself: full rank, rank 3, pure
    for x in (r, _rand_rho(rng, nq, min(3, full)), D.pure(psi)):
        assert abs(L.qcw_rho_fidelity(dev(x), dev(x)) - 1.0) <= FID_TOL


def test_fidelity_after_one_hadamard_general(L):
    """§5, MV1-Noise: 1/sqrt2 after one H, through the general (mixed-reference) path."""
    psi0 = qi.basis_state(1, 0)
    rho = D.conjugate(D.pure(psi0), qi.H, (1,))
    assert abs(L.qcw_rho_fidelity(dev(rho), dev(D.pure(psi0))) - 2 ** -0.5) <= 4e-16


def test_fidelity_orthogonal_and_mixed_limits(L):
    """F = 0 for orthogonal pure states; against the maximally mixed reference
    F = Tr sqrt(rho) / sqrt(n), i.e. sum sqrt(lambda) / sqrt(n)."""
    nq = 3
    a, b = qi.basis_state(nq, 0), qi.basis_state(nq, 5)
    assert abs(L.qcw_rho_fidelity(dev(D.pure(a)), dev(D.pure(b)))) <= FID_TOL
    rng = np.random.default_rng(61)
    r = _rand_rho(rng, nq, 8)
    lam = np.linalg.eigvalsh(r)
    ref = np.sum(np.sqrt(lam)) / np.sqrt(8)
    assert abs(L.qcw_rho_fidelity(dev(r), dev(np.eye(8) / 8)) - ref) <= FID_TOL


# ------------------------------------------------------------------ batched eigensolver
def _rho_batch(rng, nq, count):
    """count density matrices of nq qubits with ranks cycling over 1, 2, 3 and full."""
    ranks = [1, 2, 3, 1 << nq]
    return [_rand_rho(rng, nq, min(ranks[i % 4], 1 << nq)) for i in range(count)]


@pytest.mark.parametrize("nq,count", [(1, 5), (2, 33), (3, 300), (4, 257), (5, 600), (6, 1100)])
def test_eigvals_batch_against_lapack(L, nq, count):
    """Every matrix of one persistent launch (more matrices than resident
    blocks at nq = 6, so blocks take several) against numpy's Hermitian
    solver: eigenvalues and entropy within 1e-12; matrices spaced by a stride
    above 4^nq (the gaps are never read as matrix data)."""
    rng = np.random.default_rng(300 + nq)
    n = 1 << nq
    rhos = _rho_batch(rng, nq, count)
    stride = n * n + 7
    flat = np.full(count * stride, np.nan + 1j * np.nan, dtype=np.complex128)
    for i, r in enumerate(rhos):
        flat[i * stride:i * stride + n * n] = r.reshape(-1)
    ev, S = L.qcw_rho_eigvals_batch(dev(flat), nq, count, stride)
    torch.cuda.synchronize()
    ev, S = ev.cpu().numpy(), S.cpu().numpy()
    for i, r in enumerate(rhos):
        ref = D.eigen_observables(r)
        assert np.max(np.abs(ev[i] - ref["eigenvalues"])) <= 1e-12, i
        assert abs(S[i] - ref["entropy_bits"]) <= 1e-12, i
        assert np.all(np.diff(ev[i]) >= 0)


def test_eigvals_batch_equals_single_calls(L):
    """The synchronous one-matrix call runs the same kernel: same bits."""
    rng = np.random.default_rng(310)
    nq = 5
    rhos = _rho_batch(rng, nq, 12)
    ev, S = L.qcw_rho_eigvals_batch(dev(np.stack(rhos)), nq, len(rhos))
    torch.cuda.synchronize()
    ev, S = ev.cpu().numpy(), S.cpu().numpy()
    for i, r in enumerate(rhos):
        e1, s1 = L.qcw_rho_eigvals(dev(r))
        assert np.array_equal(e1, ev[i]) and s1 == S[i]


def test_eigvals_batch_classical_limit_and_pure(L):
    """Closed forms: the maximally mixed state has every eigenvalue 1/n and
    entropy nq bits; a pure state has eigenvalues {0, ..., 0, 1} and entropy 0."""
    nq = 6
    n = 1 << nq
    psi = qi.state(5, nq)
    ev, S = L.qcw_rho_eigvals_batch(dev(np.stack([np.eye(n) / n, D.pure(psi)])), nq, 2)
    torch.cuda.synchronize()
    ev, S = ev.cpu().numpy(), S.cpu().numpy()
    assert np.max(np.abs(ev[0] - 1 / n)) <= 1e-15 and abs(S[0] - nq) <= 1e-13
    assert np.max(np.abs(ev[1] - np.r_[np.zeros(n - 1), 1.0])) <= 1e-14 and abs(S[1]) <= 1e-12


@pytest.mark.parametrize("nq,count", [(2, 40), (5, 300), (6, 520)])
def test_fidelity_batch(L, nq, count):
    """Pairs (full-rank rho_i, full-rank rho0_i) against the oracle, and one
    shared pure reference (rho0 stride 0) against the closed form."""
    rng = np.random.default_rng(320 + nq)
    n = 1 << nq
    rs = [_rand_rho(rng, nq, n) for _ in range(count)]
    r0s = [_rand_rho(rng, nq, n) for _ in range(count)]
    F = L.qcw_rho_fidelity_batch(dev(np.stack(rs)), dev(np.stack(r0s)), nq, count)
    psi0 = qi.state(6, nq)
    Fp = L.qcw_rho_fidelity_batch(dev(np.stack(rs)), dev(D.pure(psi0)), nq, count, rho0_stride=0)
    torch.cuda.synchronize()
    F, Fp = F.cpu().numpy(), Fp.cpu().numpy()
    for i in range(count):
        assert abs(F[i] - D.fidelity_general(rs[i], r0s[i])) <= FID_TOL, i
        assert abs(Fp[i] - D.observables(rs[i], psi0)["fidelity"]) <= FID_TOL, i
    # the one-pair call runs the same kernel
    assert L.qcw_rho_fidelity(dev(rs[3]), dev(r0s[3])) == F[3]


def test_eigen_batch_validation(L):
    nq, n = 3, 8
    rho = dev(np.stack([np.eye(n) / n] * 4))
    eig = torch.empty((4, n), dtype=torch.float64, device="cuda")
    with pytest.raises(L.QcwError):     # stride below 4^nq
        L.qcw_rho_eigvals_batch(rho, nq, 4, n * n - 1, eig)
    # negative count (through the C call: the binding would not allocate for it)
    assert L.lib().qcw_rho_eigvals_batch(rho.data_ptr(), nq, -1, n * n, eig.data_ptr(), None,
                                         None) == L.QCW_EINVAL
    with pytest.raises(L.QcwError):     # nq above 6
        L.qcw_rho_eigvals_batch(dev(np.zeros(1 << 14)), 7, 1)
    with pytest.raises(L.QcwError):     # rho stride 0 is only for the reference
        L.qcw_rho_fidelity_batch(rho, rho, nq, 2, rho_stride=0)
    # count 0 is a no-op
    L.qcw_rho_eigvals_batch(rho, nq, 0, n * n, eig)


@pytest.mark.parametrize("nq,keep", [(2, [1]), (2, [2]), (3, [1, 3]), (5, [2, 3, 5]), (8, [4]),
                                     (8, [1, 2, 7, 8])])
def test_partial_trace(L, nq, keep):
    rng = np.random.default_rng(70 + nq)
    rho = _rand_rho(rng, nq)
    got = L.qcw_rho_partial_trace(dev(rho), keep)
    ref = D.partial_trace(rho, keep)
    assert np.max(np.abs(host(got, len(keep)) - ref)) <= 1e-14


def test_bell_subsystem_entropy(L):
    rho = D.conjugate(D.conjugate(D.pure(qi.basis_state(2, 0)), qi.H, (1,)), qi.CNOT, (1, 2))
    red = L.qcw_rho_partial_trace(dev(rho), [2])
    ev, S = L.qcw_rho_eigvals(red)
    assert np.max(np.abs(ev - 0.5)) <= 1e-15 and abs(S - 1.0) <= 1e-14


@pytest.mark.parametrize("nq", [1, 3, 7])
def test_channel_mixed_monomial_and_dense_terms(L, nq):
    """Diagonal/anti-diagonal terms take the flip-mask path (grouped by mask),
    all others (random unitaries, one-column and rank-one operators) the table
    path; both together must match the oracle."""
    rng = np.random.default_rng(80 + nq)
    rho0 = _rand_rho(rng, nq)
    P = [D.SX, D.SY, D.SZ, np.eye(2, dtype=complex), np.array([[0, 1j], [0.5, 0]]),
         np.array([[0.3, 0], [0.7j, 0]]), np.array([[0, 0.4], [0, 0]]),
         np.diag([1.0, 0.6])]
    terms = []
    for i in range(12):
        qs = [int(x) + 1 for x in rng.choice(nq, min(nq, 1 + i % 2), replace=False)]
        ops = {q: (P[int(rng.integers(len(P)))] if i % 3 else qi.random_unitary(rng, 2))
               for q in qs}
        terms.append((0.2 / 12, ops))
    ch = L.Channel(nq, 0.8, terms)
    a, b = dev(rho0), torch.empty(1 << (2 * nq), dtype=torch.complex128, device="cuda")
    ch.apply(a, b)
    assert np.max(np.abs(host(b, nq) - D.channel(rho0, 0.8, terms))) <= TOL
    ch.close()


@pytest.mark.parametrize("nq", [2, 5])
def test_channel_random_rotation_noise(L, nq):
    """The general-rotation noise option of the multiverse scheme (random
    rotations exp(-i theta n.sigma/2) as the hit operators instead of Pauli
    operators), single and double hits: equal to the oracle, trace and
    hermiticity kept."""
    rng = np.random.default_rng(90 + nq)
    rho0 = _rand_rho(rng, nq)
    terms = []
    for i in range(8):
        qs = [int(x) + 1 for x in rng.choice(nq, min(nq, 1 + i % 2), replace=False)]
        terms.append((0.2 / 8, {q: qi.random_rotation(rng) for q in qs}))
    ch = L.Channel(nq, 0.8, terms)
    a, b = dev(rho0), torch.empty(1 << (2 * nq), dtype=torch.complex128, device="cuda")
    ch.apply(a, b)
    out = host(b, nq)
    assert np.max(np.abs(out - D.channel(rho0, 0.8, terms))) <= TOL
    assert abs(np.trace(out) - 1) <= TOL and np.max(np.abs(out - out.conj().T)) <= TOL
    ch.close()


def test_pauli_channel_16_qubits_basis_state(L):
    """nq = 16 (above the tiled kernel's range, so the gather kernel): 2^32
    elements, more than one launch grid can address, so the kernel's blocks
    stride over the matrix.  On |0..0><0..0| a Pauli hit
    moves weight w_t to the diagonal element at its flip mask (X and Y flip
    their qubit, Z does not; |entries| = 1), so the output is p at (0, 0) plus
    the weights of the flip-free hits, w summed per flip mask f at (f, f), and
    zero everywhere else (the output starts as NaN, so every element must be
    written)."""
    nq = 16
    N = 1 << nq
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 2 * 16 * N * N + (8 << 30):
        pytest.skip("needs 128 GiB of free device memory")
    print(f"[gpu] pauli channel nq={nq} on a basis state", flush=True)
    rng = np.random.default_rng(16)
    P = {"X": qi.X, "Y": qi.Y, "Z": qi.Z}
    terms, expect = [], {0: 0.8}
    for s, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(16):
            qs = [int(x) + 1 for x in rng.choice(nq, s, replace=False)]
            names = {q: "XYZ"[int(rng.integers(3))] for q in qs}
            w = 0.2 * ps / 16
            terms.append((w, {q: P[n] for q, n in names.items()}))
            f = sum(1 << (nq - q) for q, n in names.items() if n != "Z")
            expect[f] = expect.get(f, 0.0) + w
    ch = L.Channel(nq, 0.8, terms)
    a = torch.zeros(N * N, dtype=torch.complex128, device="cuda")
    a[0] = 1.0
    b = torch.full_like(a, float("nan"))
    ch.apply(a, b)
    ch.close()
    del a
    assert not bool(torch.isnan(b).any())
    assert int(torch.count_nonzero(b).item()) == len(expect)
    idx = torch.tensor([f * N + f for f in expect], device="cuda")
    got = b[idx].cpu().numpy()
    assert np.allclose(got, list(expect.values()), rtol=0, atol=1e-15)
    assert abs(complex(b.sum().item()) - 1.0) <= 1e-14
    del b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nq,pairs", [(2, ((1, 2), (2, 1))), (3, ((1, 3), (3, 2))),
                                      (5, ((2, 4), (5, 1), (4, 5))), (8, ((1, 8), (7, 3), (6, 7)))])
def test_pair_polarization_matches_oracle(L, nq, pairs):
    """qcw_rho_pair_polarization: P1, P2 and the correlation tensor of two
    qubits (the two-qubit form of §5's footnote) against the oracle's traces
    with full Pauli operators, to 1e-13; the same bits on a repeated call."""
    print(f"[gpu] pair polarisation nq={nq}", flush=True)
    rng = np.random.default_rng(900 + nq)
    rho0 = _rand_rho(rng, nq)
    a = dev(rho0)
    for qa, qb in pairs:
        got = L.qcw_rho_pair_polarization(a, qa, qb).cpu().numpy()
        again = L.qcw_rho_pair_polarization(a, qa, qb).cpu().numpy()
        assert np.array_equal(got, again)
        want = D.pair_polarization(rho0, qa, qb)
        assert np.max(np.abs(got - want)) <= 1e-13, (qa, qb, got - want)


def test_pair_polarization_product_state_closed_form(L):
    """At nq = 12 (beyond the oracle's full operators): for a product of
    one-qubit states (1 + P . sigma)/2 the pair's polarisations are the
    factors' P and C = P_a P_b^T; P1 also equals qcw_rho_observables'
    polarisation of qa."""
    nq = 12
    print(f"[gpu] pair polarisation product state nq={nq}", flush=True)
    rng = np.random.default_rng(77)
    Ps = [rng.normal(size=3) for _ in range(nq)]
    Ps = [P / np.linalg.norm(P) * rng.uniform(0.3, 1.0) for P in Ps]
    rho = np.array([[1.0 + 0j]])
    for P in Ps:
        rho = np.kron(rho, (np.eye(2) + P[0] * D.SX + P[1] * D.SY + P[2] * D.SZ) / 2)
    a = dev(rho)
    obs = L.qcw_rho_observables(a)
    for qa, qb in ((1, 12), (12, 1), (5, 6), (3, 10)):
        v = L.qcw_rho_pair_polarization(a, qa, qb).cpu().numpy()
        Pa, Pb = Ps[qa - 1], Ps[qb - 1]
        assert np.max(np.abs(v[:3] - Pa)) <= 1e-13 and np.max(np.abs(v[3:6] - Pb)) <= 1e-13
        assert np.max(np.abs(v[6:].reshape(3, 3) - np.outer(Pa, Pb))) <= 1e-13
        assert np.max(np.abs(v[:3] - obs["polarization"][qa - 1])) <= 1e-13
    for bad in ((3, 3), (0, 2), (2, 13)):
        with pytest.raises(RuntimeError):
            L.qcw_rho_pair_polarization(a, *bad)
