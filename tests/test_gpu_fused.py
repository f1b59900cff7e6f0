"""GPU parity of the fused multi-gate passes (qcw_circuit_fused).

A fused pass runs each gate's group update with the same arithmetic as the
one-gate sweep, so with no plan flags the result must equal the plain path bit
for bit, and the oracle within the FP64 circuit tolerance.  The plan flags
(QCW_PLAN_COMMUTE: gates on disjoint qubits reordered; QCW_PLAN_FUSE: gates
merged inside a pass; QCW_PLAN_3M: the three-product complex arithmetic) keep
the operator and change only the rounding: their
results must equal the plain path and the oracle within that tolerance.
"""
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


COMMUTE, FUSE, M3 = 1, 2, 4


def _run(L, psi0, c, fused, tile_bits=0, low_bits=0, plan=0):
    psi = torch.from_numpy(psi0).to("cuda")
    if fused:
        L.circuit_fused(psi, c, tile_bits, low_bits=low_bits, plan=plan)
    else:
        L.circuit(psi, c)
    torch.cuda.synchronize()
    return psi.cpu().numpy()


@pytest.mark.parametrize("nq", [9, 10, 12, 14, 18, 22])
@pytest.mark.parametrize("tile_bits,low_bits", [(8, 5), (10, 5), (12, 5), (11, 3), (12, 3),
                                                (13, 3), (13, 4), (12, 4)])
def test_fused_equals_plain_bitwise(L, nq, tile_bits, low_bits):
    print(f"[gpu] fused nq={nq} tile_bits={tile_bits} low_bits={low_bits}", flush=True)
    psi0 = qi.state(11, nq, tag=tile_bits)
    c = qi.circuit(11, nq, 4 * nq, tag=tile_bits)
    a = _run(L, psi0, c, True, tile_bits, low_bits)
    b = _run(L, psi0, c, False)
    assert np.array_equal(a, b)
    if nq <= 18:
        r = oracle.circuit(c, psi0)
        assert np.linalg.norm(a - r) <= TOL * max(1, len(c) / 64) * np.linalg.norm(r)


@pytest.mark.parametrize("tile_bits,low_bits,threads", [(12, 3, 256), (12, 3, 1024), (12, 5, 1024),
                                                        (12, 4, 1024), (13, 3, 512), (13, 5, 1024)])
@pytest.mark.parametrize("nq", [12, 13, 17, 21])
def test_fused_threads_per_tile(L, tile_bits, low_bits, threads, nq):
    """Every block shape, including the warp-specialised pipelined kernel
    (tile_bits = 12, threads = 1024): one tile, a few tiles per block, and many."""
    psi0 = qi.state(12, nq)
    c = qi.circuit(12, nq, 4 * nq)
    psi = torch.from_numpy(psi0).to("cuda")
    L.circuit_fused(psi, c, tile_bits, low_bits=low_bits, threads=threads)
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), _run(L, psi0, c, False))


def _close(a, b, G):
    return np.linalg.norm(a - b) <= TOL * max(1, G / 64) * np.linalg.norm(b)


@pytest.mark.parametrize("plan", [COMMUTE, FUSE, COMMUTE | FUSE, M3, COMMUTE | FUSE | M3])
@pytest.mark.parametrize("nq", [9, 12, 14, 18, 22])
@pytest.mark.parametrize("tile_bits,low_bits", [(8, 5), (11, 3), (12, 4), (13, 4)])
def test_fused_plan_equals_plain_to_rounding(L, nq, tile_bits, low_bits, plan):
    print(f"[gpu] fused plan={plan} nq={nq} tile_bits={tile_bits} low_bits={low_bits}", flush=True)
    psi0 = qi.state(13, nq, tag=tile_bits)
    c = qi.circuit(13, nq, 4 * nq, tag=tile_bits + 100 * plan)
    a = _run(L, psi0, c, True, tile_bits, low_bits, plan)
    b = _run(L, psi0, c, False)
    assert _close(a, b, len(c))
    if nq <= 18:
        assert _close(a, oracle.circuit(c, psi0), len(c))


@pytest.mark.parametrize("tile_bits,low_bits,threads", [(12, 3, 256), (12, 4, 1024), (13, 5, 1024),
                                                        (13, 3, 512), (11, 4, 512)])
@pytest.mark.parametrize("nq", [13, 21])
def test_fused_plan_threads_per_tile(L, tile_bits, low_bits, threads, nq):
    psi0 = qi.state(14, nq)
    c = qi.circuit(14, nq, 6 * nq)
    psi = torch.from_numpy(psi0).to("cuda")
    L.circuit_fused(psi, c, tile_bits, low_bits=low_bits, threads=threads, plan=COMMUTE | FUSE | M3)
    torch.cuda.synchronize()
    assert _close(psi.cpu().numpy(), _run(L, psi0, c, False), len(c))


def test_fused_plan_ghz_and_inverse(L):
    """GHZ chain on 16 qubits under all three flags: (|0..0> + |1..1>)/sqrt2
    and zeros elsewhere, then back to |0..0> under the inverse circuit.  The
    three-product form rounds a + b before the shared product, so even these
    permutation and real gates are exact only to about an ulp per gate: the
    bound is 64 ulp (a wrong gate is off by O(1))."""
    nq = 16
    c = qi.Circuit(nq).add(qi.H, 1)
    for t in range(2, nq + 1):
        c.add(qi.CNOT, 1, t)
    psi = torch.from_numpy(qi.basis_state(nq, 0)).to("cuda")
    L.circuit_fused(psi, c, plan=COMMUTE | FUSE | M3)
    torch.cuda.synchronize()
    out = psi.cpu().numpy()
    ref = np.zeros(1 << nq, complex)
    ref[0] = ref[-1] = qi.S2
    assert np.abs(out - ref).max() <= 64 * 2.0 ** -53
    L.circuit_fused(psi, c.inverse(), plan=COMMUTE | FUSE | M3)
    torch.cuda.synchronize()
    back = psi.cpu().numpy()
    assert np.abs(back - qi.basis_state(nq, 0)).max() <= 128 * 2.0 ** -53


def test_fused_plan_cache_follows_the_request(L):
    """A stream reuses its last plan only for the same request: the same
    circuit twice, then the same gate list with one matrix entry changed, then
    other plan flags, each equal to the plain path."""
    nq = 16
    c = qi.circuit(15, nq, 40)
    g, m = L.pack_circuit(c)
    psi0 = qi.state(15, nq)
    a = torch.from_numpy(psi0).to("cuda")
    b = a.clone()
    s = torch.cuda.current_stream()
    for _ in range(2):
        L.qcw_circuit_fused_ex(a, nq, g, len(c), m, m.size, 12, 4, 0, COMMUTE | FUSE, s)
        L.qcw_circuit(b, nq, g, len(c), m, m.size, s)
    torch.cuda.synchronize()
    assert _close(a.cpu().numpy(), b.cpu().numpy(), 2 * len(c))
    m2 = m.copy()
    m2[5] *= -1j                                     # linear update: any matrix is fine
    for plan in (COMMUTE | FUSE, COMMUTE | FUSE | M3, 0):
        L.qcw_circuit_fused_ex(a, nq, g, len(c), m2, m2.size, 12, 4, 0, plan, s)
        L.qcw_circuit(b, nq, g, len(c), m2, m2.size, s)
        torch.cuda.synchronize()
        assert _close(a.cpu().numpy(), b.cpu().numpy(), 5 * len(c))


def test_fused_fewer_passes(L):
    c = qi.circuit(1, 31, 124)
    g, m = L.pack_circuit(c)
    n = L.qcw_fused_pass_count(31, g, len(c))
    assert 1 <= n < len(c) // 2
    low = qi.Circuit(20)
    for q in (20, 19, 18, 17, 16):
        low.add(qi.H, q)
    g, m = L.pack_circuit(low)
    assert L.qcw_fused_pass_count(20, g, len(low)) == 1


@pytest.mark.parametrize("g", [x for x in all_golden()], ids=[x.name for x in all_golden()])
def test_fused_golden(L, g):
    psi = torch.from_numpy(g.init).to("cuda")
    L.circuit_fused(psi, g.circ)
    torch.cuda.synchronize()
    g.check(psi.cpu().numpy())


def test_fused_ghz_large_bit_exact(L):
    nq = 16
    c = qi.Circuit(nq).add(qi.H, 1)
    for t in range(2, nq + 1):
        c.add(qi.CNOT, 1, t)
    out = _run(L, qi.basis_state(nq, 0), c, True)
    ref = np.zeros(1 << nq, complex)
    ref[0] = ref[-1] = qi.S2
    assert np.array_equal(out, ref)


def test_fused_validation(L):
    psi = torch.zeros(1 << 10, dtype=torch.complex128, device="cuda")
    c = qi.circuit(0, 10, 4)
    g, m = L.pack_circuit(c)
    with pytest.raises(L.QcwError, match="tile_bits"):
        L.qcw_circuit_fused(psi, 10, g, len(c), m, m.size, 14)
    bad = g.copy()
    bad[1]["q"][0] = 11
    with pytest.raises(L.QcwError, match="gate 1"):
        L.qcw_circuit_fused(psi, 10, bad, len(c), m, m.size)
    with pytest.raises(L.QcwError, match="threads"):
        L.qcw_circuit_fused_ex(psi, 10, g, len(c), m, m.size, 11, 3, 1024)
    with pytest.raises(L.QcwError, match="plan"):
        L.qcw_circuit_fused_ex(psi, 10, g, len(c), m, m.size, 12, 4, 0, 8)
    L.qcw_circuit_fused(psi, 10, g, 0, m, m.size)          # empty circuit is a no-op


FULL_NQ = 31


def test_fullsize_fused_equals_plain_and_roundtrips(L):
    """nq = 31: the 124-gate benchmark circuit, fused vs one sweep per gate
    (bitwise), then fused inverse back to the input."""
    free, _ = torch.cuda.mem_get_info()
    if free < (3 * (16 << FULL_NQ) + (4 << 30)):
        pytest.skip("not enough device memory")
    print("[gpu] full size fused", flush=True)
    psi0 = qi.state(1, FULL_NQ)
    c = qi.circuit(1, FULL_NQ, 4 * FULL_NQ)
    a = torch.from_numpy(psi0).to("cuda")
    b = a.clone()
    L.circuit_fused(a, c)
    L.circuit(b, c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    del b
    torch.cuda.empty_cache()
    L.circuit_fused(a, c.inverse())
    ref = torch.from_numpy(psi0).to("cuda")
    err = torch.linalg.vector_norm(a - ref).item()
    assert err <= TOL * max(1.0, 2 * len(c) / 64)
    del a, ref
    torch.cuda.empty_cache()


def test_fullsize_fused_plan_matches_plain(L):
    """nq = 31, the 124-gate benchmark circuit with all three plan flags (the
    benchmark's launch configuration): equal to one sweep per gate (whose
    single-gate outputs are checked against the oracle at this size) within
    the circuit tolerance, as a relative 2-norm and amplitude by amplitude."""
    free, _ = torch.cuda.mem_get_info()
    if free < (3 * (16 << FULL_NQ) + (4 << 30)):
        pytest.skip("not enough device memory")
    print("[gpu] full size fused plan", flush=True)
    psi0 = qi.state(1, FULL_NQ)
    c = qi.circuit(1, FULL_NQ, 4 * FULL_NQ)
    a = torch.from_numpy(psi0).to("cuda")
    b = a.clone()
    L.circuit_fused(a, c, plan=COMMUTE | FUSE | M3)
    L.circuit(b, c)
    torch.cuda.synchronize()
    tol = TOL * max(1.0, len(c) / 64)
    err = (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()
    assert err <= tol
    # every amplitude of this state has modulus about 2^-15.5; allow the same
    # relative error on each
    worst = (a - b).abs().max().item()
    assert worst <= tol * 2.0 ** -15.5 * 64
    del a, b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nq", [26, 28])
def test_fullsize_headline_plan_vs_oracle(L, nq):
    """The benchmark's exact configuration -- all three plan flags, default
    tiles (12 bits, 4 low bits, 512 threads), a 4*nq-gate random circuit --
    at sizes where the commute planner's search runs (24 qubits and up),
    against the full oracle circuit, element by element: normwise within the
    FP64 circuit tolerance and every amplitude within 1e-12 |psi|."""
    G = 4 * nq
    print(f"[gpu] headline plan vs oracle nq={nq} G={G}", flush=True)
    psi0 = qi.state(21, nq, tag=nq)
    c = qi.circuit(21, nq, G, tag=nq)
    g, _ = L.pack_circuit(c)
    assert L.qcw_fused_pass_count(nq, g, G, 0, 0, COMMUTE | FUSE | M3) < \
        L.qcw_fused_pass_count(nq, g, G, 0, 0, 0)
    got = _run(L, psi0, c, True, 0, 0, COMMUTE | FUSE | M3)
    ref = oracle.circuit(c, psi0)
    nr = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= TOL * max(1, G / 64) * nr
    assert np.max(np.abs(got - ref)) <= TOL * nr
