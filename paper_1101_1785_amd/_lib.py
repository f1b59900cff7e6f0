"""ctypes binding of libqcw.so: argument marshalling only.

Every function here has the name and argument order of its C counterpart in
include/qcw.h.  States are torch complex128 tensors on the GPU (torch supplies
device memory and the current stream); matrices and gate lists are numpy
arrays on the host.  Nothing is computed here: if the library is missing,
importing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcw.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1101_1785_amd.build`")

# torch ships its own HIP runtime.  Loading torch first makes libqcw.so bind to
# that same runtime (same SONAME), so device pointers and streams from torch are
# valid in the library; loading libqcw.so first would put a second HIP runtime
# in the process.
import torch  # noqa: E402,F401

_L = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i32 = ctypes.c_int
_i64 = ctypes.c_int64

QCW_OK, QCW_EINVAL, QCW_ENOMEM, QCW_EHIP, QCW_EAGAIN = 0, -1, -2, -3, -4
QCW_KERNEL_SWEEP1, QCW_KERNEL_SWEEP2, QCW_KERNEL_SWEEP3, QCW_KERNEL_BATCH = 1, 2, 3, 4
QCW_KERNEL_SMALL = 7
QCW_KERNEL_CONJ = 8
QCW_KERNEL_FUSED = 5
QCW_PLAN_COMMUTE, QCW_PLAN_FUSE, QCW_PLAN_3M = 1, 2, 4
QCW_KERNEL_CHANNEL = 6


class QcwError(RuntimeError):
    def __init__(self, code: int, fn: str):
        self.code = code
        msg = _L.qcw_last_error().decode(errors="replace")
        super().__init__(f"{fn}: {_L.qcw_strerror(code).decode()} ({code}): {msg}")


class qcw_gate(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("q", ctypes.c_int32 * 3), ("mat", ctypes.c_int64)]


GATE_DTYPE = np.dtype([("k", np.int32), ("q", np.int32, (3,)), ("mat", np.int64)], align=True)
assert GATE_DTYPE.itemsize == ctypes.sizeof(qcw_gate) == 24
INSTANCE_DTYPE = np.dtype([("nq", np.int32), ("ngates", np.int32), ("state_off", np.int64),
                           ("gate_off", np.int64)], align=True)
assert INSTANCE_DTYPE.itemsize == 24

_SIGS = {
    "qcw_strerror": ([_i32], ctypes.c_char_p),
    "qcw_last_error": ([], ctypes.c_char_p),
    "qcw_version": ([], _i32),
    "qcw_op1": ([_P, _i32, _P, _i32, _P], _i32),
    "qcw_op2": ([_P, _i32, _i32, _P, _i32, _P], _i32),
    "qcw_op3": ([_P, _i32, _i32, _i32, _P, _i32, _P], _i32),
    "qcw_opk": ([_i32, _P, _P, _P, _i32, _P], _i32),
    "qcw_opk_to": ([_i32, _P, _P, _P, _P, _i32, _P], _i32),
    "qcw_omega_all": ([_P, _P, _i32, _P], _i32),
    "qcw_circuit": ([_P, _i32, _P, _i32, _P, _i64, _P], _i32),
    "qcw_circuit_fused": ([_P, _i32, _P, _i32, _P, _i64, _i32, _P], _i32),
    "qcw_circuit_fused_ex": ([_P, _i32, _P, _i32, _P, _i64, _i32, _i32, _i32, _i32, _P], _i32),
    "qcw_circuit_fused_noalloc": ([_P, _i32, _P, _i32, _P, _i64, _i32, _i32, _i32, _i32, _P],
                                  _i32),
    "qcw_fused_pass_count": ([_i32, _P, _i32, _i32, _i32, _i32], _i32),
    "qcw_fused_plan": ([_i32, _P, _i32, _i32, _i32, _i32, _P, _P], _i32),
    "qcw_debug_pick_device": ([_i32, _i32, _P, _P], _i32),
    "qcw_debug_fused_tables": ([_i32, _P, _i32, _P, _i64, _i32, _i32, _i32, _i32, _i32, _P, _P,
                                _P, _P, _P, _P, _P], _i32),
    "qcw_op_shard": ([_i32, _P, _P, _i32, _P, _P, _i32, _P], _i32),
    "qcw_batch_create": ([_P, _P, _i32, _P, _i64, _P, _i64, _P, _i64, ctypes.c_char_p, _P], _i32),
    "qcw_batch_run": ([_P, _P], _i32),
    "qcw_batch_run_eager": ([_P, _P], _i32),
    "qcw_batch_run_repeat": ([_P, _i32, _P], _i32),
    "qcw_batch_info": ([_P, _i32, _P, _P, _P], _i32),
    "qcw_batch_destroy": ([_P], _i32),
    "qcw_batch_variant_name": ([_i32], ctypes.c_char_p),
    "qcw_batch_autotune": ([ctypes.c_char_p, _i32, _i32, _i32, _i32, _P], _i32),
    "qcw_fuse_circuit": ([_i32, _P, _i32, _P, _i64, _i32, _i32, _P, _P, _P, _i64, _P], _i32),
    "qcw_rho_conjugate": ([_i32, _P, _P, _P, _i32, _P], _i32),
    "qcw_channel_create": ([_P, _i32, ctypes.c_double, _P, _i32, _P, _i64], _i32),
    "qcw_channel_apply": ([_P, _P, _P, _P], _i32),
    "qcw_channel_destroy": ([_P], _i32),
    "qcw_channel_flops_per_element": ([_P], _i64),
    "qcw_debug_channel_plan": ([_P, _i32, _P], _i32),
    "qcw_debug_channel_source": ([_i32, _P, _i32, _P, _i64, _i32, _P, _P, _i32, _i32, _P,
                                  ctypes.c_size_t, _P, _P, _P], _i32),
    "qcw_channel_apply_gate": ([_P, _P, _P, _i32, _P, _P, _P], _i32),
    "qcw_channel_step_obs": ([_P, _P, _P, _i32, _P, _P, _P, _P, _P], _i32),
    "qcw_rho_observables": ([_P, _i32, _P, _P, _P], _i32),
    "qcw_rho_eigvals": ([_P, _i32, _P, _P], _i32),
    "qcw_rho_eigvals_batch": ([_P, _i32, _i64, _i64, _P, _P, _P], _i32),
    "qcw_rho_fidelity_batch": ([_P, _i64, _P, _i64, _i32, _i64, _P, _P], _i32),
    "qcw_rho_fidelity": ([_P, _P, _i32, _P, _P], _i32),
    "qcw_rho_partial_trace": ([_P, _i32, _P, _i32, _P, _P], _i32),
    "qcw_rho_pair_polarization": ([_P, _i32, _i32, _i32, _P, _P], _i32),
    "qcw_server_create": ([_P, _P], _i32),
    "qcw_server_submit": ([_P, _P, _P], _i32),
    "qcw_server_poll": ([_P, ctypes.c_uint64, _P, _P], _i32),
    "qcw_server_wait": ([_P, ctypes.c_uint64, _P, _P, ctypes.c_double], _i32),
    "qcw_server_counters_get": ([_P, _P], _i32),
    "qcw_server_destroy": ([_P], _i32),
    "qcw_timing_enable": ([_i32], _i32),
    "qcw_timing_reset": ([], _i32),
    "qcw_timing_read": ([_i32, _P, _P], _i32),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = _res


def lib():
    return _L


def exported_names():
    return list(_SIGS)


# ------------------------------------------------------------------ marshalling
def _check(rc: int, fn: str) -> None:
    if rc != QCW_OK:
        raise QcwError(rc, fn)


def _mat(U, k: int | None = None) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.complex128)
    if U.ndim != 2 or U.shape[0] != U.shape[1]:
        raise ValueError("gate matrix must be square")
    if k is not None and U.shape[0] != (1 << k):
        raise ValueError(f"gate matrix must be {1 << k} x {1 << k}")
    return U


def _hptr(a: np.ndarray):
    """Host address of a numpy array (an int, which ctypes passes as void*)."""
    return a.ctypes.data


def _dptr(t):
    """Device pointer of a torch complex128 GPU tensor (contiguous)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError("state must be a torch.complex128 tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("state tensor must be contiguous")
    return _P(t.data_ptr())


def _nq_of(t, nq):
    if nq is not None:
        return int(nq)
    n = t.numel()
    if n <= 0 or n & (n - 1):
        raise ValueError("state length must be a power of two")
    return n.bit_length() - 1


def _stream(stream):
    if stream is None:
        import torch
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def _targets(targets) -> np.ndarray:
    t = np.zeros(3, dtype=np.int32)
    t[:len(targets)] = targets
    return t


# ------------------------------------------------------------------ entry points
def qcw_op1(U, is_, psi, nq=None, stream=None):
    U = _mat(U, 1)
    _check(_L.qcw_op1(_hptr(U), int(is_), _dptr(psi), _nq_of(psi, nq), _stream(stream)), "qcw_op1")


def qcw_op2(V, is1, is2, psi, nq=None, stream=None):
    V = _mat(V, 2)
    _check(_L.qcw_op2(_hptr(V), int(is1), int(is2), _dptr(psi), _nq_of(psi, nq),
                      _stream(stream)), "qcw_op2")


def qcw_op3(W, is1, is2, is3, psi, nq=None, stream=None):
    W = _mat(W, 3)
    _check(_L.qcw_op3(_hptr(W), int(is1), int(is2), int(is3), _dptr(psi), _nq_of(psi, nq),
                      _stream(stream)), "qcw_op3")


def qcw_opk(k, targets, U, psi, nq=None, stream=None):
    U = _mat(U, k)
    t = _targets(targets)
    _check(_L.qcw_opk(int(k), _hptr(t), _hptr(U), _dptr(psi), _nq_of(psi, nq), _stream(stream)),
           "qcw_opk")


def qcw_opk_to(k, targets, U, psi_in, psi_out, nq=None, stream=None):
    U = _mat(U, k)
    t = _targets(targets)
    _check(_L.qcw_opk_to(int(k), _hptr(t), _hptr(U), _dptr(psi_in), _dptr(psi_out),
                         _nq_of(psi_in, nq), _stream(stream)), "qcw_opk_to")


def qcw_omega_all(U, psi, nq=None, stream=None):
    U = _mat(U, 1)
    _check(_L.qcw_omega_all(_hptr(U), _dptr(psi), _nq_of(psi, nq), _stream(stream)),
           "qcw_omega_all")


def pack_circuit(circ):
    """Circuit (qcw_inputs.Circuit) -> (gates structured array, mats complex array)."""
    G = len(circ)
    gates = np.zeros(G, dtype=GATE_DTYPE)
    mats = []
    off = 0
    for g, (k, t, U) in enumerate(zip(circ.ks, circ.targets, circ.mats)):
        gates[g]["k"] = k
        gates[g]["q"][:k] = t
        gates[g]["mat"] = off
        mats.append(np.ascontiguousarray(U, dtype=np.complex128).reshape(-1))
        off += U.size
    M = np.concatenate(mats) if mats else np.zeros(1, np.complex128)
    return gates, np.ascontiguousarray(M)


def qcw_circuit(psi, nq, gates, ngates, mats, nmats, stream=None):
    _check(_L.qcw_circuit(_dptr(psi), int(nq), _hptr(gates), int(ngates), _hptr(mats),
                          int(nmats), _stream(stream)), "qcw_circuit")


def circuit(psi, circ, stream=None):
    """Apply a qcw_inputs.Circuit to psi in place with qcw_circuit."""
    gates, mats = pack_circuit(circ)
    qcw_circuit(psi, circ.nq, gates, len(circ), mats, mats.size, stream)


def qcw_circuit_fused(psi, nq, gates, ngates, mats, nmats, tile_bits=0, stream=None):
    _check(_L.qcw_circuit_fused(_dptr(psi), int(nq), _hptr(gates), int(ngates), _hptr(mats),
                                int(nmats), int(tile_bits), _stream(stream)), "qcw_circuit_fused")


def qcw_circuit_fused_ex(psi, nq, gates, ngates, mats, nmats, tile_bits=0, low_bits=0,
                         threads=0, plan=0, stream=None):
    _check(_L.qcw_circuit_fused_ex(_dptr(psi), int(nq), _hptr(gates), int(ngates), _hptr(mats),
                                   int(nmats), int(tile_bits), int(low_bits), int(threads),
                                   int(plan), _stream(stream)), "qcw_circuit_fused_ex")


def circuit_fused(psi, circ, tile_bits=0, stream=None, low_bits=0, threads=0, plan=0):
    """Apply a qcw_inputs.Circuit in place with qcw_circuit_fused_ex."""
    gates, mats = pack_circuit(circ)
    qcw_circuit_fused_ex(psi, circ.nq, gates, len(circ), mats, mats.size, tile_bits, low_bits,
                         threads, plan, stream)


def qcw_op_shard(k, targets, U, rank_bit, psi_local, psi_remote, nq, stream=None):
    """One rank's half of a gate on a state split by qubit 1 (see include/qcw.h)."""
    t = _targets(targets)
    Uc = np.ascontiguousarray(U, dtype=np.complex128).reshape(-1)
    rem = _dptr(psi_remote) if psi_remote is not None else None
    _check(_L.qcw_op_shard(int(k), _hptr(t), _hptr(Uc), int(rank_bit), _dptr(psi_local), rem,
                           int(nq), _stream(stream)), "qcw_op_shard")


def qcw_fused_pass_count(nq, gates, ngates, tile_bits=0, low_bits=0, plan=0):
    n = _L.qcw_fused_pass_count(int(nq), _hptr(gates), int(ngates), int(tile_bits), int(low_bits),
                                int(plan))
    if n < 0:
        raise QcwError(n, "qcw_fused_pass_count")
    return n


def qcw_fused_plan(nq, gates, ngates, tile_bits=0, low_bits=0, plan=0):
    """(pass count, pass_of per gate, gate indices in execution order)."""
    pass_of = np.zeros(max(int(ngates), 1), dtype=np.int32)
    order = np.zeros(max(int(ngates), 1), dtype=np.int32)
    n = _L.qcw_fused_plan(int(nq), _hptr(gates), int(ngates), int(tile_bits), int(low_bits),
                          int(plan), _hptr(pass_of), _hptr(order))
    if n < 0:
        raise QcwError(n, "qcw_fused_plan")
    return n, pass_of[:ngates], order[:ngates]


def qcw_debug_fused_tables(nq, gates, ngates, mats, tile_bits=0, low_bits=0, plan=0):
    """The fused pass plan's device tables (host call): a dict with per-pass
    gate_off, ngates, T, L, outer_pos (list per pass), chunk_off (array per
    pass, 2^(T-L) entries) and per-gate k, sb (3), m3, off (8), u (m x m)."""
    cap_p, cap_g = 8, 8
    while True:
        ph = np.zeros(4 * cap_p, dtype=np.int32)
        op = np.zeros(40 * cap_p, dtype=np.int32)
        co = np.zeros(1024 * cap_p, dtype=np.uint64)
        gh = np.zeros(13 * cap_g, dtype=np.int32)
        gm = np.zeros(64 * cap_g, dtype=np.complex128)
        npass, ngate = ctypes.c_int(0), ctypes.c_int(0)
        rc = _L.qcw_debug_fused_tables(int(nq), _hptr(gates), int(ngates), _hptr(mats),
                                       int(mats.size), int(tile_bits), int(low_bits), int(plan),
                                       cap_p, cap_g, _hptr(ph), _hptr(op), _hptr(co), _hptr(gh),
                                       _hptr(gm), ctypes.byref(npass), ctypes.byref(ngate))
        if rc == QCW_OK:
            break
        if npass.value > cap_p or ngate.value > cap_g:
            cap_p, cap_g = max(cap_p, npass.value), max(cap_g, ngate.value)
            continue
        _check(rc, "qcw_debug_fused_tables")
    P, G = npass.value, ngate.value
    ph = ph.reshape(-1, 4)[:P]
    passes = []
    for p in range(P):
        T, Lb = int(ph[p, 2]), int(ph[p, 3])
        outer = [int(x) for x in op[40 * p:40 * p + 40] if x >= 0]
        passes.append({"gate_off": int(ph[p, 0]), "ngates": int(ph[p, 1]), "T": T, "L": Lb,
                       "outer_pos": outer,
                       "chunk_off": co[1024 * p:1024 * p + (1 << (T - Lb))].copy()})
    gates_out = []
    for g in range(G):
        h = gh[13 * g:13 * g + 13]
        k = int(h[0])
        m = 1 << k
        gates_out.append({"k": k, "sb": [int(x) for x in h[1:4]], "m3": int(h[4]),
                          "off": [int(x) for x in h[5:13]],
                          "u": gm[64 * g:64 * g + m * m].reshape(m, m).copy()})
    return {"passes": passes, "gates": gates_out}


def qcw_debug_pick_device(nq, targets):
    k = len(targets)
    out = np.empty(1 << nq, dtype=np.uint64)
    t = _targets(targets)
    _check(_L.qcw_debug_pick_device(int(nq), int(k), _hptr(t), _hptr(out)), "qcw_debug_pick_device")
    return out.reshape(-1, 1 << k)


def qcw_timing_enable(on: bool):
    _check(_L.qcw_timing_enable(1 if on else 0), "qcw_timing_enable")


def qcw_timing_reset():
    _check(_L.qcw_timing_reset(), "qcw_timing_reset")


def qcw_timing_read(kernel: int):
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(_L.qcw_timing_read(int(kernel), ctypes.byref(n), ctypes.byref(ms)), "qcw_timing_read")
    return int(n.value), float(ms.value)


# ------------------------------------------------------------------ batched form
def pack_batch(instances):
    """[(nq, Circuit), ...] -> (instance table, gates, mats, total state length).

    States are packed back to back in list order."""
    n = len(instances)
    inst = np.zeros(n, dtype=INSTANCE_DTYPE)
    gate_rows, mat_chunks = [], []
    soff = goff = moff = 0
    for i, (nq, circ) in enumerate(instances):
        g, m = pack_circuit(circ)
        g = g.copy()
        g["mat"] += moff
        inst[i] = (nq, len(circ), soff, goff)
        gate_rows.append(g)
        if len(circ):
            mat_chunks.append(m)
            moff += m.size
        soff += 1 << nq
        goff += len(circ)
    gates = np.concatenate(gate_rows) if gate_rows else np.zeros(0, GATE_DTYPE)
    mats = np.concatenate(mat_chunks) if mat_chunks else np.zeros(1, np.complex128)
    return inst, np.ascontiguousarray(gates), np.ascontiguousarray(mats), soff


def qcw_batch_create(inst, n, gates, ngates, mats, nmats, states, nstates, tune_table=None,
                     stream=None):
    h = _P()
    tt = tune_table.encode() if tune_table else None
    _check(_L.qcw_batch_create(ctypes.byref(h), _hptr(inst), int(n), _hptr(gates), int(ngates),
                               _hptr(mats), int(nmats), _dptr(states), int(nstates), tt,
                               _stream(stream)), "qcw_batch_create")
    return h


def qcw_batch_run(h, stream=None):
    _check(_L.qcw_batch_run(h, _stream(stream)), "qcw_batch_run")


def qcw_batch_run_eager(h, stream=None):
    _check(_L.qcw_batch_run_eager(h, _stream(stream)), "qcw_batch_run_eager")


def qcw_batch_run_repeat(h, reps, stream=None):
    _check(_L.qcw_batch_run_repeat(h, int(reps), _stream(stream)), "qcw_batch_run_repeat")


def qcw_batch_info(h, nq):
    v, b, l = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(_L.qcw_batch_info(h, int(nq), ctypes.byref(v), ctypes.byref(b), ctypes.byref(l)),
           "qcw_batch_info")
    return v.value, b.value, l.value


def qcw_batch_destroy(h):
    _check(_L.qcw_batch_destroy(h), "qcw_batch_destroy")


def fuse_circuit(nq, circ, max_qubits=3, regroup=False):
    """Gate fusion (host only): returns (gates, mats) in the packed layout of
    pack_circuit, blocks of gates spanning at most max_qubits qubits merged
    into one gate each (runs of consecutive gates, or with regroup also gates
    that commute past the gates between them)."""
    g, m = pack_circuit(circ)
    n = g.size
    og = np.zeros(max(n, 1), dtype=GATE_DTYPE)
    om = np.zeros(max(64 * n, 1), dtype=np.complex128)
    ng = ctypes.c_int(0)
    nm = ctypes.c_int64(0)
    _check(_L.qcw_fuse_circuit(int(nq), _hptr(g), int(n), _hptr(m), int(m.size), int(max_qubits),
                               int(bool(regroup)), _hptr(og), ctypes.byref(ng), _hptr(om), int(om.size),
                               ctypes.byref(nm)), "qcw_fuse_circuit")
    return og[:ng.value].copy(), om[:nm.value].copy()


def qcw_batch_variant_name(v):
    return _L.qcw_batch_variant_name(int(v)).decode()


def qcw_batch_autotune(out_path, nq_lo, nq_hi, ninst, gates_per_qubit=4, stream=None):
    _check(_L.qcw_batch_autotune(out_path.encode(), int(nq_lo), int(nq_hi), int(ninst),
                                 int(gates_per_qubit), _stream(stream)), "qcw_batch_autotune")


class Batch:
    """Owns a qcw_batch handle over a packed device state tensor."""

    def __init__(self, instances, states, tune_table=None, stream=None):
        self.inst, self.gates, self.mats, total = pack_batch(instances)
        if states.numel() < total:
            raise ValueError("states tensor shorter than the packed instances")
        self.states = states
        self.h = qcw_batch_create(self.inst, len(self.inst), self.gates, self.gates.size,
                                  self.mats, self.mats.size, states, states.numel(),
                                  tune_table, stream)

    def run(self, stream=None):
        qcw_batch_run(self.h, stream)

    def run_eager(self, stream=None):
        qcw_batch_run_eager(self.h, stream)

    def run_repeat(self, reps, stream=None):
        qcw_batch_run_repeat(self.h, reps, stream)

    def info(self, nq):
        return qcw_batch_info(self.h, nq)

    def close(self):
        if self.h:
            qcw_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
class qcw_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int),
                ("gates_per_tick", ctypes.c_int), ("max_nq", ctypes.c_int),
                ("tune_table", ctypes.c_char_p)]


class qcw_request(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_int), ("ngates", ctypes.c_int), ("gates", _P), ("mats", _P),
                ("nmats", ctypes.c_int64), ("psi0", _P)]


class qcw_req_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("ticks", ctypes.c_int),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


class qcw_server_counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "ticks",
                                                "peak_active", "peak_pending", "admit_waits")]


def qcw_server_create(cfg):
    h = _P()
    _check(_L.qcw_server_create(ctypes.byref(h), ctypes.byref(cfg)), "qcw_server_create")
    return h


def qcw_server_submit(h, req):
    t = ctypes.c_uint64(0)
    _check(_L.qcw_server_submit(h, ctypes.byref(req), ctypes.byref(t)), "qcw_server_submit")
    return t.value


def qcw_server_poll(h, ticket, out=None):
    st = qcw_req_stats()
    rc = _L.qcw_server_poll(h, ctypes.c_uint64(ticket), _hptr(out) if out is not None else None,
                            ctypes.byref(st))
    if rc not in (QCW_OK, QCW_EAGAIN):
        raise QcwError(rc, "qcw_server_poll")
    return rc, st


def qcw_server_wait(h, ticket, out=None, timeout_s=60.0):
    st = qcw_req_stats()
    rc = _L.qcw_server_wait(h, ctypes.c_uint64(ticket), _hptr(out) if out is not None else None,
                            ctypes.byref(st), float(timeout_s))
    if rc not in (QCW_OK, QCW_EAGAIN):
        raise QcwError(rc, "qcw_server_wait")
    return rc, st


def qcw_server_counters_get(h):
    c = qcw_server_counters()
    _check(_L.qcw_server_counters_get(h, ctypes.byref(c)), "qcw_server_counters_get")
    return {n: getattr(c, n) for n, _ in c._fields_}


def qcw_server_destroy(h):
    _check(_L.qcw_server_destroy(h), "qcw_server_destroy")


class Server:
    """Continuous-batching request loop on the current GPU."""

    def __init__(self, hbm_budget_bytes=1 << 30, max_slots=1024, gates_per_tick=0, max_nq=11,
                 tune_table=None):
        self._tt = tune_table.encode() if tune_table else None
        cfg = qcw_server_cfg(hbm_budget_bytes, max_slots, gates_per_tick, max_nq, self._tt)
        self.h = qcw_server_create(cfg)

    def submit(self, nq, circ=None, psi0=None, gates=None, mats=None):
        """Copies the request (a qcw_inputs.Circuit or packed gates/mats) and returns a ticket."""
        if circ is not None:
            gates, mats = pack_circuit(circ)
        psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
        if psi0.size != (1 << nq):
            raise ValueError("psi0 must hold 2^nq amplitudes")
        req = qcw_request(int(nq), int(len(gates)), _hptr(gates) if len(gates) else None,
                          _hptr(mats), int(mats.size), _hptr(psi0))
        return qcw_server_submit(self.h, req)

    def poll(self, ticket, nq):
        out = np.empty(1 << nq, np.complex128)
        rc, st = qcw_server_poll(self.h, ticket, out)
        return (out if rc == QCW_OK else None), st

    def wait(self, ticket, nq, timeout_s=60.0):
        out = np.empty(1 << nq, np.complex128)
        rc, st = qcw_server_wait(self.h, ticket, out, timeout_s)
        return (out if rc == QCW_OK else None), st

    def counters(self):
        return qcw_server_counters_get(self.h)

    def close(self):
        if self.h:
            qcw_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ density matrix
KRAUS_DTYPE = np.dtype([("nops", np.int32), ("q", np.int32, (2,)), ("pad", np.int32),
                        ("mat", np.int64, (2,)), ("weight", np.float64)], align=True)
assert KRAUS_DTYPE.itemsize == 40


def _rho_nq(rho, nq):
    if nq is not None:
        return int(nq)
    n = rho.numel()
    b = n.bit_length() - 1
    if n <= 0 or n & (n - 1) or b % 2:
        raise ValueError("rho must hold 4^nq elements")
    return b // 2


def qcw_rho_conjugate(k, targets, U, rho, nq=None, stream=None):
    U = _mat(U, k)
    t = _targets(targets)
    _check(_L.qcw_rho_conjugate(int(k), _hptr(t), _hptr(U), _dptr(rho), _rho_nq(rho, nq),
                                _stream(stream)), "qcw_rho_conjugate")


def pack_terms(terms):
    """[(weight, {qubit: 2x2}), ...] -> (term table, mats)."""
    tab = np.zeros(len(terms), dtype=KRAUS_DTYPE)
    mats = []
    off = 0
    for i, (w, ops) in enumerate(terms):
        if not 1 <= len(ops) <= 2:
            raise ValueError("a term has one or two one-qubit operators")
        tab[i]["nops"] = len(ops)
        tab[i]["weight"] = w
        for j, (q, K) in enumerate(ops.items()):
            tab[i]["q"][j] = q
            tab[i]["mat"][j] = off
            mats.append(np.ascontiguousarray(K, dtype=np.complex128).reshape(4))
            off += 4
    M = np.concatenate(mats) if mats else np.zeros(4, np.complex128)
    return tab, M


def channel_kernel_source(nq, terms, compile=False, gate=None, observables=False):
    """(source, code_bytes, compiler_version) of the tiled kernel a Channel
    over these terms compiles at creation (qcw_debug_channel_source; host
    only), or with gate = (U, targets) the one apply_gate compiles for that
    gate ("" unless U is monomial or every target is among the four last
    qubits).  source is "" when the
    channel has no tiled plan; code_bytes is None unless compile;
    compiler_version is major * 100 + minor."""
    tab, mats = pack_terms(terms)
    n, cb, ver = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_int32(0)
    gk, gt, gu = 0, None, None
    if gate is not None:
        gk = len(gate[1])
        gt, gu = _targets(gate[1]), _mat(gate[0], gk)
    args = (int(nq), _hptr(tab) if len(tab) else None, len(tab), _hptr(mats), mats.size, gk,
            _hptr(gt) if gt is not None else None, _hptr(gu) if gu is not None else None,
            int(bool(observables)))
    _check(_L.qcw_debug_channel_source(*args, 0, None, 0, ctypes.byref(n), None, None),
           "qcw_debug_channel_source")
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(_L.qcw_debug_channel_source(*args, int(bool(compile)), buf, n.value + 1, ctypes.byref(n),
                                       ctypes.byref(cb), ctypes.byref(ver)),
           "qcw_debug_channel_source")
    return buf.value.decode(), (cb.value if compile else None), ver.value


class Channel:
    """Ensemble-average channel rho -> p rho + sum w K rho K^dagger on the GPU."""

    def __init__(self, nq, p_keep, terms):
        tab, mats = pack_terms(terms)
        h = _P()
        _check(_L.qcw_channel_create(ctypes.byref(h), int(nq), float(p_keep),
                                     _hptr(tab) if len(tab) else None, len(tab), _hptr(mats),
                                     mats.size), "qcw_channel_create")
        self.h, self.nq = h, nq

    def apply(self, rho_in, rho_out, stream=None):
        _check(_L.qcw_channel_apply(self.h, _dptr(rho_in), _dptr(rho_out), _stream(stream)),
               "qcw_channel_apply")

    def apply_gate(self, rho_in, rho_out, U, targets, stream=None):
        """rho_out = U channel(rho_in) U^dagger (qcw_channel_apply_gate): one
        pass when the compiled tiled kernel runs and U is monomial or acts on
        the four last qubits only."""
        k = len(targets)
        t = _targets(targets)
        U = _mat(U, k)
        _check(_L.qcw_channel_apply_gate(self.h, _dptr(rho_in), _dptr(rho_out), k, _hptr(t),
                                         _hptr(U), _stream(stream)), "qcw_channel_apply_gate")

    def step_obs(self, rho_in, rho_out, obs, U=None, targets=(), psi0=None, stream=None):
        """qcw_channel_step_obs: rho_out = U channel(rho_in) U^dagger (no gate
        when U is None) and its trace (re, im), purity, root fidelity against
        psi0 (a device tensor, or None) and polarisations into obs (a device
        float64 tensor of 4 + 3 nq, laid out as qcw_rho_observables),
        asynchronously."""
        k = 0 if U is None else len(targets)
        t = _targets(targets) if k else None
        Um = _mat(U, k) if k else None
        _check(_L.qcw_channel_step_obs(self.h, _dptr(rho_in), _dptr(rho_out), k,
                                       _hptr(t) if k else None, _hptr(Um) if k else None,
                                       _dptr(psi0) if psi0 is not None else None, _dptr_f64(obs),
                                       _stream(stream)), "qcw_channel_step_obs")

    def flops_per_element(self):
        return int(_L.qcw_channel_flops_per_element(self.h))

    _PLAN_KEYS = ("tiled_plan", "gather_kernel", "e0", "e1", "partners", "staged", "direct",
                  "own_staged", "reads", "groups", "segments", "etouch_segments", "real",
                  "compiled_kernel", "grid", "vgprs", "compiler_version")
    KERNEL_TILED, KERNEL_GATHER, KERNEL_TILED_GENERIC = 0, 1, 2

    def plan(self, kernel=-1):
        """The tiled kernel's plan (qcw_debug_channel_plan) as a dict; kernel
        0/1/2 picks the tiled (compiled when available) / gather / generic
        tiled kernel from now on."""
        info = np.zeros(17, dtype=np.int32)
        _check(_L.qcw_debug_channel_plan(self.h, int(kernel), _hptr(info)),
               "qcw_debug_channel_plan")
        return dict(zip(self._PLAN_KEYS, (int(x) for x in info)))

    def close(self):
        if self.h:
            _check(_L.qcw_channel_destroy(self.h), "qcw_channel_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcw_rho_observables(rho, nq=None, psi0=None, stream=None):
    nq = _rho_nq(rho, nq)
    out = np.empty(4 + 3 * nq, dtype=np.float64)
    p = np.ascontiguousarray(psi0, dtype=np.complex128) if psi0 is not None else None
    _check(_L.qcw_rho_observables(_dptr(rho), nq, _hptr(p) if p is not None else None,
                                  _hptr(out), _stream(stream)), "qcw_rho_observables")
    return {"trace": complex(out[0], out[1]), "purity": float(out[2]),
            "fidelity": float(out[3]), "polarization": out[4:].reshape(nq, 3)}


def qcw_rho_eigvals(rho, nq=None, stream=None):
    """(eigenvalues ascending, entropy in bits)."""
    nq = _rho_nq(rho, nq)
    out = np.empty((1 << nq) + 1, dtype=np.float64)
    _check(_L.qcw_rho_eigvals(_dptr(rho), nq, _hptr(out), _stream(stream)), "qcw_rho_eigvals")
    return out[:-1], float(out[-1])


def qcw_rho_fidelity(rho, rho0, nq=None, stream=None):
    nq = _rho_nq(rho, nq)
    out = np.empty(1, dtype=np.float64)
    _check(_L.qcw_rho_fidelity(_dptr(rho), _dptr(rho0), nq, _hptr(out), _stream(stream)),
           "qcw_rho_fidelity")
    return float(out[0])


def _dptr_f64(t):
    """Device pointer of a contiguous torch float64 GPU tensor (or None)."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda \
            or not t.is_contiguous():
        raise TypeError("output must be a contiguous torch.float64 tensor on the GPU")
    return t.data_ptr()


def qcw_rho_eigvals_batch(rho, nq, count, stride=None, eig=None, entropy=None, stream=None):
    """Eigenvalues (count x 2^nq, ascending) and entropies in bits (count) of
    `count` density matrices, matrix i at element i * stride of the complex128
    device tensor rho; outputs are float64 device tensors (allocated here when
    not given).  Asynchronous on the stream.  Returns (eig, entropy)."""
    import torch
    n = 1 << nq
    stride = n * n if stride is None else stride
    if eig is None:
        eig = torch.empty((count, n), dtype=torch.float64, device=rho.device)
    if entropy is None:
        entropy = torch.empty(count, dtype=torch.float64, device=rho.device)
    _check(_L.qcw_rho_eigvals_batch(_dptr(rho), nq, count, stride, _dptr_f64(eig),
                                    _dptr_f64(entropy), _stream(stream)),
           "qcw_rho_eigvals_batch")
    return eig, entropy


def qcw_rho_fidelity_batch(rho, rho0, nq, count, rho_stride=None, rho0_stride=None, out=None,
                           stream=None):
    """Fidelities of `count` pairs (rho_i, rho0_i); rho0_stride = 0 compares
    every rho_i with one reference.  Asynchronous; returns the float64 device
    tensor of count values."""
    import torch
    nn = 1 << (2 * nq)
    rho_stride = nn if rho_stride is None else rho_stride
    rho0_stride = nn if rho0_stride is None else rho0_stride
    if out is None:
        out = torch.empty(count, dtype=torch.float64, device=rho.device)
    _check(_L.qcw_rho_fidelity_batch(_dptr(rho), rho_stride, _dptr(rho0), rho0_stride, nq, count,
                                     _dptr_f64(out), _stream(stream)), "qcw_rho_fidelity_batch")
    return out


def qcw_rho_pair_polarization(rho, qa, qb, nq=None, stream=None):
    """[P1 (3), P2 (3), C (3 x 3 row-major)] of qubits qa, qb (a device
    tensor of 15 doubles; qcw_rho_pair_polarization)."""
    import torch
    nq = _rho_nq(rho, nq)
    out = torch.empty(15, dtype=torch.float64, device=rho.device)
    _check(_L.qcw_rho_pair_polarization(_dptr(rho), nq, int(qa), int(qb), _dptr_f64(out),
                                        _stream(stream)), "qcw_rho_pair_polarization")
    return out


def qcw_rho_partial_trace(rho, keep, nq=None, stream=None):
    import torch
    nq = _rho_nq(rho, nq)
    k = np.ascontiguousarray(keep, dtype=np.int32)
    out = torch.empty(1 << (2 * len(keep)), dtype=torch.complex128, device=rho.device)
    _check(_L.qcw_rho_partial_trace(_dptr(rho), nq, _hptr(k), len(keep), _dptr(out),
                                    _stream(stream)), "qcw_rho_partial_trace")
    return out
