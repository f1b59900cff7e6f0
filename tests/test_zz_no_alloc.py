"""qcw_circuit_fused_noalloc (the fused passes with their plan tables in the
library's static per-GPU array, for callers that cannot allocate) against
qcw_circuit_fused_ex, through the C ABI: the same kernels and plans, so the
same bits.  Two calls in a row with different requests, the second on a
smaller state, then the first request again (its plan is planned and uploaded
anew into the shared array); a plan whose tables exceed the array is rejected."""
import ctypes

import numpy as np
import pytest

import qcw_inputs as qi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_1785_amd import _lib
    return _lib


def _both(L, nq, seed, plan):
    c = qi.circuit(seed, nq, 4 * nq, tag=40)
    g, m = L.pack_circuit(c)
    psi0 = torch.from_numpy(qi.state(seed, nq, tag=40)).to("cuda")
    a, b = psi0.clone(), psi0.clone()
    s = torch.cuda.current_stream().cuda_stream
    print(f"[gpu] noalloc nq={nq} seed={seed} plan={plan}", flush=True)
    rc = L.lib().qcw_circuit_fused_noalloc(a.data_ptr(), nq, g.ctypes.data, len(c), m.ctypes.data,
                                           m.size, 0, 0, 0, plan, ctypes.c_void_p(s))
    assert rc == L.QCW_OK, L.lib().qcw_last_error()
    rc = L.lib().qcw_circuit_fused_ex(b.data_ptr(), nq, g.ctypes.data, len(c), m.ctypes.data,
                                      m.size, 0, 0, 0, plan, ctypes.c_void_p(s))
    assert rc == L.QCW_OK, L.lib().qcw_last_error()
    torch.cuda.synchronize()
    return a, b, psi0


@pytest.mark.parametrize("plan", [0, 7])
def test_noalloc_equals_fused_ex(L, plan):
    for nq, seed in ((22, 1), (14, 2), (22, 1)):
        a, b, psi0 = _both(L, nq, seed, plan)
        assert torch.equal(a, b)
        assert not torch.equal(a, psi0)


def test_noalloc_rejects_oversized_plan(L):
    # 3000 one-qubit gates on a 12-qubit state, no fusion: one pass of 3000
    # gate records (1.6 KiB each) does not fit the 4 MiB array
    nq, G = 12, 3000
    rng = np.random.default_rng(3)
    g = np.zeros(G, dtype=L.GATE_DTYPE)
    g["k"] = 1
    g["q"][:, 0] = rng.integers(1, nq + 1, G)
    g["mat"] = 0
    m = np.ascontiguousarray(qi.H, dtype=np.complex128).reshape(-1)
    psi = torch.zeros(1 << nq, dtype=torch.complex128, device="cuda")
    rc = L.lib().qcw_circuit_fused_noalloc(psi.data_ptr(), nq, g.ctypes.data, G, m.ctypes.data,
                                           m.size, 0, 0, 0, 0, None)
    assert rc == L.QCW_EINVAL
    assert b"no-allocation buffer" in L.lib().qcw_last_error()
    # the same request through the allocating entry point runs
    rc = L.lib().qcw_circuit_fused_ex(psi.data_ptr(), nq, g.ctypes.data, G, m.ctypes.data,
                                      m.size, 0, 0, 0, 0, None)
    assert rc == L.QCW_OK
    torch.cuda.synchronize()
