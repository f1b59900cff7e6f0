"""Builds and binds the scheduler test double (tests/sched/sched_harness.cpp)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1101_1785_amd", "csrc")
OUT = os.path.join(HERE, "_build", "libqcw_sched_test.so")


class Request(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_int), ("ngates", ctypes.c_int), ("gates", ctypes.c_void_p),
                ("mats", ctypes.c_void_p), ("nmats", ctypes.c_int64), ("psi0", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("ticks", ctypes.c_int), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class Counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "ticks",
                                                "peak_active", "peak_pending", "admit_waits")]


def build():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(CSRC, "server_core.cpp"), os.path.join(CSRC, "common.cpp"),
            os.path.join(HERE, "sched_harness.cpp")]
    # A temporary name per process: parallel test workers may build at once,
    # and each then renames its own complete file into place.
    tmp = f"{OUT}.{os.getpid()}.tmp"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-shared", "-fPIC", "-pthread",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "-o", tmp, *srcs]
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


def load():
    build()
    L = ctypes.CDLL(OUT)
    P, u64 = ctypes.c_void_p, ctypes.c_uint64
    L.qcws_create.restype = P
    L.qcws_create.argtypes = [u64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, u64]
    L.qcws_submit.argtypes = [P, P, P]
    L.qcws_poll.argtypes = [P, u64, P, P]
    L.qcws_wait.argtypes = [P, u64, P, P, ctypes.c_double]
    L.qcws_counters.argtypes = [P, P]
    L.qcws_violations.argtypes = [P]
    L.qcws_max_tick.argtypes = [P]
    L.qcws_stop.argtypes = [P]
    L.qcws_destroy.argtypes = [P]
    L.qcws_last_error.restype = ctypes.c_char_p
    return L


class FakeServer:
    def __init__(self, L, budget=1 << 24, max_slots=64, gates_per_tick=0, max_nq=11,
                 tick_seconds=0.0, fail_ticket=0):
        self.L = L
        self.h = L.qcws_create(budget, max_slots, gates_per_tick, max_nq, tick_seconds, fail_ticket)
        self._keep = {}

    def submit(self, nq, gates, mats, psi0):
        psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
        r = Request(nq, len(gates), gates.ctypes.data if len(gates) else None,
                    mats.ctypes.data, mats.size, psi0.ctypes.data)
        t = ctypes.c_uint64(0)
        rc = self.L.qcws_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        return rc, t.value

    def wait(self, ticket, nq, timeout=10.0):
        out = np.empty(1 << nq, np.complex128)
        st = Stats()
        rc = self.L.qcws_wait(self.h, ticket, out.ctypes.data, ctypes.byref(st), timeout)
        return rc, out, st

    def poll(self, ticket, nq):
        out = np.empty(1 << nq, np.complex128)
        st = Stats()
        rc = self.L.qcws_poll(self.h, ticket, out.ctypes.data, ctypes.byref(st))
        return rc, out, st

    def counters(self):
        c = Counters()
        self.L.qcws_counters(self.h, ctypes.byref(c))
        return c

    def violations(self):
        return self.L.qcws_violations(self.h)

    def max_tick(self):
        return self.L.qcws_max_tick(self.h)

    def stop(self):
        self.L.qcws_stop(self.h)

    def close(self):
        if self.h:
            self.L.qcws_destroy(self.h)
            self.h = None
