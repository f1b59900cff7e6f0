"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qcw.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qcw_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1101_1785_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "qcw_op1" in names and "qcw_circuit" in names
    for n in names:
        assert hasattr(L.lib(), n), n


def test_binding_covers_header(L):
    assert set(_declared()) == set(L.exported_names())


def test_version_and_strerror(L):
    assert L.lib().qcw_version() >= 100
    assert L.lib().qcw_strerror(-1) == b"invalid argument"
    assert L.lib().qcw_strerror(0) == b"ok"


# Argument validation happens on the host before any HIP call, so it runs here.
def _U(m):
    return np.eye(m, dtype=np.complex128)


@pytest.mark.parametrize("k,targets,nq,msg", [
    (1, [0], 3, "outside"), (1, [4], 3, "outside"), (2, [2, 2], 3, "repeated"),
    (3, [1, 2, 3], 2, "exceeds"), (4, [1, 2, 3], 5, "outside {1, 2, 3}"),
    (1, [1], 0, "nq=0"), (1, [1], 35, "nq=35")])
def test_invalid_targets_rejected(L, k, targets, nq, msg):
    lib = L.lib()
    t = np.array(targets + [0] * (3 - len(targets)), dtype=np.int32)
    U = _U(2 ** min(k, 3))
    rc = lib.qcw_opk(k, t.ctypes.data_as(ctypes.c_void_p), U.ctypes.data_as(ctypes.c_void_p),
                     ctypes.c_void_p(0x1000), nq, None)
    assert rc == L.QCW_EINVAL
    assert msg in lib.qcw_last_error().decode()


def test_null_pointers_rejected(L):
    lib = L.lib()
    t = np.array([1, 0, 0], dtype=np.int32)
    U = _U(2)
    assert lib.qcw_opk(1, t.ctypes.data_as(ctypes.c_void_p), None, ctypes.c_void_p(0x1000), 3, None) == L.QCW_EINVAL
    assert lib.qcw_opk(1, None, U.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(0x1000), 3, None) == L.QCW_EINVAL


def test_partial_overlap_rejected(L):
    lib = L.lib()
    t = np.array([1, 0, 0], dtype=np.int32)
    U = _U(2)
    rc = lib.qcw_opk_to(1, t.ctypes.data_as(ctypes.c_void_p), U.ctypes.data_as(ctypes.c_void_p),
                        ctypes.c_void_p(0x10000), ctypes.c_void_p(0x10010), 3, None)
    assert rc == L.QCW_EINVAL and "overlap" in lib.qcw_last_error().decode()


def test_circuit_validates_every_gate_first(L):
    lib = L.lib()
    gates = np.zeros(2, dtype=L.GATE_DTYPE)
    gates[0]["k"] = 1; gates[0]["q"][0] = 1; gates[0]["mat"] = 0
    gates[1]["k"] = 2; gates[1]["q"][:2] = [2, 2]; gates[1]["mat"] = 4
    mats = np.zeros(20, dtype=np.complex128)
    rc = lib.qcw_circuit(ctypes.c_void_p(0x1000), 3, gates.ctypes.data_as(ctypes.c_void_p), 2,
                         mats.ctypes.data_as(ctypes.c_void_p), mats.size, None)
    assert rc == L.QCW_EINVAL and "gate 1" in lib.qcw_last_error().decode()
    gates[1]["q"][:2] = [2, 3]
    rc = lib.qcw_circuit(ctypes.c_void_p(0x1000), 3, gates.ctypes.data_as(ctypes.c_void_p), 2,
                         mats.ctypes.data_as(ctypes.c_void_p), 10, None)
    assert rc == L.QCW_EINVAL and "matrix offset" in lib.qcw_last_error().decode()


def test_pack_circuit_layout(L):
    import qcw_inputs as qi
    c = qi.circuit(0, 5, 7)
    gates, mats = L.pack_circuit(c)
    assert gates.size == 7
    for g, (k, t, U) in enumerate(zip(c.ks, c.targets, c.mats)):
        assert gates[g]["k"] == k and tuple(gates[g]["q"][:k]) == t
        o = gates[g]["mat"]
        assert np.array_equal(mats[o:o + U.size].reshape(U.shape), U)


def test_single_hip_runtime_in_process():
    """Importing the binding alone must not load a second HIP runtime next to torch's."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1101_1785_amd import _lib\n"
            "import torch\n"
            "m = open('/proc/self/maps').read()\n"
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.stdout.strip() == "1", out.stdout + out.stderr


def test_pair_polarization_rejects_bad_qubits(L):
    """qcw_rho_pair_polarization checks nq and the two qubits before it looks
    at device memory."""
    lib = L.lib()
    rho, out = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    for nq, qa, qb in ((1, 1, 2), (18, 1, 2), (5, 3, 3), (5, 0, 2), (5, 2, 6)):
        rc = lib.qcw_rho_pair_polarization(rho, nq, qa, qb, out, None)
        assert rc == L.QCW_EINVAL, (nq, qa, qb)
        assert "qubit" in lib.qcw_last_error().decode() or "nq" in lib.qcw_last_error().decode()
