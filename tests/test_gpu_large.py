"""States above 31 qubits (64-bit labels in the sweep and the fused passes).

Pins that need no full-size oracle run:
* a gate on a basis state: Op_k of |0..0> is column 0 of U placed at the k
  labels its targets span (§3a-§3c), every other amplitude zero, and the
  products against the single nonzero input are exact, so the check is bit
  for bit;
* OmegaALL of H on |0..0> (§4a): 2^(-nq/2) on every amplitude;
* list-order fused passes equal one sweep per gate bit for bit, and with all
  plan flags a circuit followed by its inverse returns the input (a property
  that holds at any size).
Each case is skipped when the device lacks the memory.
"""
import numpy as np
import pytest

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


def _need(nbytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (8 << 30):
        pytest.skip(f"needs {nbytes / 2**30:.0f} GiB of free device memory")


def _label(nq, targets, r):
    """Label of local index r of the group at base 0 (first target most significant)."""
    k = len(targets)
    return sum(1 << (nq - t) for j, t in enumerate(targets) if (r >> (k - 1 - j)) & 1)


@pytest.mark.parametrize("nq", [32, 33])
def test_basis_state_gate_64bit_labels(L, nq):
    _need(16 << nq)
    rng = np.random.default_rng(nq)
    psi = torch.zeros(1 << nq, dtype=torch.complex128, device="cuda")
    for targets in ((1,), (1, nq), (1, nq // 2, nq), (nq, 2, 1)):
        k = len(targets)
        print(f"[gpu] basis state nq={nq} targets={targets}", flush=True)
        U = qi.random_unitary(rng, 1 << k)
        psi.zero_()
        psi[0] = 1.0
        L.qcw_opk(k, targets, U, psi)
        labels = [_label(nq, targets, r) for r in range(1 << k)]
        got = psi[torch.tensor(labels, device="cuda")].cpu().numpy()
        assert np.array_equal(got, U[:, 0])
        assert int(torch.count_nonzero(psi).item()) == int(np.count_nonzero(U[:, 0]))
    del psi
    torch.cuda.empty_cache()


def test_omega_all_h_33_qubits(L):
    nq = 33
    _need(16 << nq)
    print(f"[gpu] omega_all H nq={nq}", flush=True)
    psi = torch.zeros(1 << nq, dtype=torch.complex128, device="cuda")
    psi[0] = 1.0
    L.qcw_omega_all(qi.H, psi)
    v = 2.0 ** (-nq / 2)
    re = psi.real
    assert abs(re.max().item() - v) <= 4 * nq * 2.0 ** -53 * v
    assert abs(re.min().item() - v) <= 4 * nq * 2.0 ** -53 * v
    assert psi.imag.abs().max().item() == 0.0
    del psi, re
    torch.cuda.empty_cache()


def test_fused_32_qubits(L):
    nq = 32
    _need(3 * (16 << nq))
    print(f"[gpu] fused nq={nq}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(32)
    psi0 = torch.randn(1 << nq, dtype=torch.complex128, device="cuda", generator=g)
    psi0 /= torch.linalg.vector_norm(psi0)
    c = qi.circuit(32, nq, 24)
    a = psi0.clone()
    b = psi0.clone()
    L.circuit_fused(a, c)                      # list order
    L.circuit(b, c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    del b
    torch.cuda.empty_cache()
    a.copy_(psi0)
    L.circuit_fused(a, c, plan=L.QCW_PLAN_COMMUTE | L.QCW_PLAN_FUSE | L.QCW_PLAN_3M)
    L.circuit_fused(a, c.inverse(), plan=L.QCW_PLAN_COMMUTE | L.QCW_PLAN_FUSE | L.QCW_PLAN_3M)
    torch.cuda.synchronize()
    err = torch.linalg.vector_norm(a - psi0).item()
    assert err <= TOL * max(1.0, 2 * len(c) / 64)
    del a, psi0
    torch.cuda.empty_cache()
