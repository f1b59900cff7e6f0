"""GPU parity of the fused multi-gate passes (qcw_circuit_fused).

A fused pass runs each gate's group update with the same arithmetic as the
one-gate sweep, so the result must equal the plain path bit for bit, and the
oracle within the FP64 circuit tolerance.
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


def _run(L, psi0, c, fused, tile_bits=0, low_bits=0):
    psi = torch.from_numpy(psi0).to("cuda")
    if fused:
        L.circuit_fused(psi, c, tile_bits, low_bits=low_bits)
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

