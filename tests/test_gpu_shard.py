"""GPU parity of one GPU's part of a gate on a state split over two GPUs by
qubit 1 (qcw_op_shard): both halves, each run against the other's pre-gate
half, must equal qcw_opk on the whole state bit for bit (same group
arithmetic), and the oracle within the FP64 tolerance."""
import numpy as np
import pytest

import oracle
import qcw_inputs as qi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_1785_amd import _lib
    return _lib


def _sharded(L, psi, k, t, U, nq):
    h = 1 << (nq - 1)
    s0 = torch.from_numpy(psi[:h].copy()).to("cuda")
    s1 = torch.from_numpy(psi[h:].copy()).to("cuda")
    r0, r1 = s1.clone(), s0.clone()          # what each rank received from the other
    L.qcw_op_shard(k, t, U, 0, s0, r0, nq)
    L.qcw_op_shard(k, t, U, 1, s1, r1, nq)
    torch.cuda.synchronize()
    return np.concatenate([s0.cpu().numpy(), s1.cpu().numpy()])


@pytest.mark.parametrize("nq", [2, 3, 5, 9, 14, 20])
def test_shard_equals_whole_state(L, nq):
    print(f"[gpu] shard nq={nq}", flush=True)
    rng = np.random.default_rng(nq)
    psi = qi.state(3, nq)
    cases = [(1, (1,))]
    if nq >= 2:
        cases += [(2, (1, nq)), (2, (nq, 1)), (2, (2, 3) if nq >= 3 else (2, 1))]
    if nq >= 3:
        cases += [(3, (1, 2, nq)), (3, (nq, 1, 2)), (3, (2, nq, 1)), (3, (2, 3, nq) if nq >= 4 else (2, 3, 1))]
    for k, t in cases:
        U = qi.random_unitary(rng, 1 << k)
        got = _sharded(L, psi, k, t, U, nq)
        whole = torch.from_numpy(psi.copy()).to("cuda")
        L.qcw_opk(k, t, U, whole)
        torch.cuda.synchronize()
        assert np.array_equal(got, whole.cpu().numpy()), (k, t)
        if nq <= 14:
            r = oracle.apply(U, t, psi, nq)
            assert np.max(np.abs(got - r)) <= TOL * np.linalg.norm(r)


def test_shard_validation(L):
    nq = 6
    a = torch.zeros(1 << (nq - 1), dtype=torch.complex128, device="cuda")
    b = torch.zeros_like(a)
    with pytest.raises(L.QcwError):
        L.qcw_op_shard(1, (1,), qi.H, 2, a, b, nq)            # rank_bit not 0/1
    with pytest.raises(L.QcwError):
        L.qcw_op_shard(2, (1, 1), qi.CNOT, 0, a, b, nq)       # repeated target
    with pytest.raises(L.QcwError):
        L.qcw_op_shard(1, (1,), qi.H, 0, a, a, nq)            # overlapping halves
    with pytest.raises(L.QcwError, match="overrun"):          # a 2^29-amplitude share
        L.qcw_op_shard(1, (1,), qi.H, 0, a, b, 30)            # claimed, 2^5 allocated


SHARD_NQ = 32


def test_fullsize_shard_roundtrip(L):
    """The real shape: a 32-qubit state (64 GiB) split in two 32 GiB halves.
    A gate on qubit 1 and one local qubit, then its inverse, each followed by
    the exchange, returns both halves to the input within the tolerance."""
    free, _ = torch.cuda.mem_get_info()
    if free < 6 * (16 << (SHARD_NQ - 1)) + (8 << 30):
        pytest.skip("not enough device memory")
    print("[gpu] full size shard", flush=True)
    h = 1 << (SHARD_NQ - 1)
    gen = torch.Generator(device="cuda").manual_seed(7)
    s0 = torch.randn(h, dtype=torch.complex128, device="cuda", generator=gen)
    s1 = torch.randn(h, dtype=torch.complex128, device="cuda", generator=gen)
    nrm = torch.sqrt(torch.linalg.vector_norm(s0) ** 2 + torch.linalg.vector_norm(s1) ** 2)
    s0 /= nrm
    s1 /= nrm
    orig0, orig1 = s0.clone(), s1.clone()
    U = qi.random_unitary(np.random.default_rng(8), 4)
    for M in (U, U.conj().T):
        r0, r1 = s1.clone(), s0.clone()
        L.qcw_op_shard(2, (1, 17), M, 0, s0, r0, SHARD_NQ)
        L.qcw_op_shard(2, (1, 17), M, 1, s1, r1, SHARD_NQ)
        torch.cuda.synchronize()
        del r0, r1
    e = max((s0 - orig0).abs().max().item(), (s1 - orig1).abs().max().item())
    del s0, s1, orig0, orig1
    torch.cuda.empty_cache()
    assert e <= 2 * TOL
