"""GPU tests of the continuous-batching request loop.

Each request's result must equal, bit for bit, the plain path run on that
request alone ("alone == in the mix"), and match the oracle within the plain
path's FP64 tolerance.
"""
import threading
import time

import numpy as np
import pytest

import oracle
import qcw_inputs as qi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_1785_amd import _lib
    return _lib


def _alone(L, nq, psi0, c):
    psi = torch.from_numpy(psi0).to("cuda")
    L.circuit(psi, c)
    torch.cuda.synchronize()
    return psi.cpu().numpy()


@pytest.mark.parametrize("gpt", [0, 5])
def test_alone_equals_in_the_mix(L, gpt):
    print(f"[gpu] server mix gates_per_tick={gpt}", flush=True)
    inst = qi.batch(3, 240, 3, 9)
    s = L.Server(hbm_budget_bytes=64 << 20, max_slots=128, gates_per_tick=gpt)
    tickets = []

    def client():
        for i, (nq, p, c) in enumerate(inst):
            tickets.append(s.submit(nq, c, p))
            if i % 16 == 0:
                time.sleep(0.0005)                    # arrivals spread over several ticks

    th = threading.Thread(target=client)
    th.start()
    th.join()
    outs = []
    for t, (nq, p, c) in zip(tickets, inst):
        out, st = s.wait(t, nq)
        assert out is not None and st.status == 0
        assert st.t_submit_ns <= st.t_admit_ns <= st.t_done_ns
        if gpt:
            assert st.ticks >= -(-len(c) // gpt)
        outs.append(out)
    cnt = s.counters()
    assert cnt["completed"] == len(inst) and cnt["ticks"] >= 1
    s.close()
    for out, (nq, p, c) in zip(outs, inst):
        assert np.array_equal(out, _alone(L, nq, p, c))
    refs = oracle.circuit_batch(inst)
    for out, r, (nq, p, c) in zip(outs, refs, inst):
        assert np.linalg.norm(out - r) <= 1e-12 * max(1, len(c) / 64) * np.linalg.norm(r)


def _device_bytes(nq, c):
    """A request's arena footprint as the server accounts it: state, 64-B gate
    rows and matrices, each rounded up to 256 B.  A server without a tune table
    runs the exact tile shapes, which take the circuit as given (no fusion)."""
    r = lambda x: (x + 255) // 256 * 256
    return r(16 << nq) + r(64 * len(c)) + r(16 * sum(x.size for x in c.mats))


def test_small_budget_admission_on_gpu(L):
    """A budget below the three smallest requests but above the largest: every
    request runs, never more than two at once."""
    inst = qi.batch(4, 40, 8, 9)
    fp = sorted(_device_bytes(nq, c) for nq, _, c in inst)
    budget = fp[0] + fp[1] + fp[2] - 256
    assert budget >= fp[-1]
    s = L.Server(hbm_budget_bytes=budget, max_slots=64)
    tickets = [s.submit(nq, c, p) for nq, p, c in inst]
    for t, (nq, p, c) in zip(tickets, inst):
        out, st = s.wait(t, nq)
        assert np.array_equal(out, _alone(L, nq, p, c))
    cnt = s.counters()
    assert 1 <= cnt["peak_active"] <= 2 and cnt["completed"] == 40
    s.close()


def test_invalid_request_rejected_others_fine(L):
    s = L.Server(hbm_budget_bytes=1 << 20, max_nq=9)
    nq, p, c = 5, qi.state(1, 5), qi.circuit(1, 5, 10)
    gates, mats = L.pack_circuit(c)
    bad = gates.copy()
    bad[2]["q"][1] = bad[2]["q"][0] if bad[2]["k"] > 1 else 9
    with pytest.raises(L.QcwError):
        s.submit(nq, psi0=p, gates=bad, mats=mats)
    with pytest.raises(L.QcwError):
        s.submit(10, qi.circuit(1, 10, 2), qi.state(1, 10))
    t = s.submit(nq, c, p)
    out, st = s.wait(t, nq)
    assert np.array_equal(out, _alone(L, nq, p, c))
    assert s.counters()["rejected"] == 2
    s.close()


def test_mfma_table_server_equals_batch_alone(L, tmp_path):
    """With the matrix-core tile shape selected, a request's circuit is fused at
    submit: its result must equal the batched form run on that request alone
    with the same table (same fusion, same kernel), bit for bit, and the
    oracle within tolerance."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    table = tmp_path / "mfma.txt"
    table.write_text(f"arch {arch}\n" + "".join(f"nq {q} variant amp4_mfma\n" for q in range(1, 12)))
    inst = qi.batch(13, 60, 2, 9)
    s = L.Server(hbm_budget_bytes=16 << 20, max_slots=32, tune_table=str(table))
    tickets = [s.submit(nq, c, p) for nq, p, c in inst]
    outs = []
    for t, (nq, p, c) in zip(tickets, inst):
        out, st = s.wait(t, nq)
        assert out is not None and st.status == 0
        outs.append(out)
    s.close()
    refs = oracle.circuit_batch(inst)
    for out, r, (nq, p, c) in zip(outs, refs, inst):
        assert np.linalg.norm(out - r) <= 1e-12 * max(1, len(c) / 64) * np.linalg.norm(r)
    for i in range(0, len(inst), 7):
        nq, p, c = inst[i]
        one = torch.from_numpy(p.copy()).to("cuda")
        b = L.Batch([(nq, c)], one, tune_table=str(table))
        b.run()
        torch.cuda.synchronize()
        assert np.array_equal(one.cpu().numpy(), outs[i]), i
        b.close()


def _burst_request(rng, pool, nq=11, G=500):
    """nq-qubit request of G three-qubit gates, matrices drawn from `pool` and
    stored one per gate (so the request carries 1 KiB of matrices per gate)."""
    from paper_1101_1785_amd import _lib
    gates = np.zeros(G, dtype=_lib.GATE_DTYPE)
    gates["k"] = 3
    gates["q"] = np.argsort(rng.random((G, nq)), axis=1)[:, :3] + 1
    gates["mat"] = np.arange(G, dtype=np.int64) * 64
    mats = np.ascontiguousarray(pool[rng.integers(0, len(pool), G)].reshape(-1))
    psi = qi.state(int(rng.integers(1 << 30)), nq)
    return gates, mats, psi


def test_staging_overflow_and_direct_upload(L):
    """Admission stages requests in a 64 MiB pinned buffer that each tick
    uploads.  Two paths beyond the common one:
    * a request larger than the staging buffer (1 100 001 X gates on 11 qubits,
      ~70 MiB of gate rows) is uploaded on its own; X gates only permute, so
      its result is exactly the input with qubit 1 flipped (each other qubit
      takes an even number of X);
    * a burst of 140 requests (~79 MiB) that arrives while that request's long
      tick runs is admitted during that tick (the scheduler keeps admitting
      while a tick runs), so the staging buffer fills mid-admission and is
      flushed (the flush waits for the tick in flight); every result must equal
      the plain path alone, bit for bit.
    """
    nq0, G0 = 11, 1_100_001
    print(f"[gpu] server staging: direct request of {G0} gates, then a 140-request burst", flush=True)
    g0 = np.zeros(G0, dtype=L.GATE_DTYPE)
    g0["k"] = 1
    g0["q"][:, 0] = np.arange(G0) % nq0 + 1
    m0 = np.ascontiguousarray(qi.X.reshape(-1))
    p0 = qi.state(70, nq0)
    rng = np.random.default_rng(71)
    pool = np.stack([qi.random_unitary(rng, 8) for _ in range(32)])
    burst = [_burst_request(rng, pool) for _ in range(140)]
    s = L.Server(hbm_budget_bytes=1 << 30, max_slots=256)
    t0 = s.submit(nq0, psi0=p0, gates=g0, mats=m0)
    time.sleep(0.05)                                   # its tick is running
    tickets = [s.submit(11, psi0=p, gates=g, mats=m) for g, m, p in burst]
    out0, st0 = s.wait(t0, nq0, timeout_s=100.0)
    assert out0 is not None and st0.status == 0
    flip = np.arange(1 << nq0) ^ (1 << (nq0 - 1))
    assert np.array_equal(out0, p0[flip])
    outs, admits, dones = [], [], []
    for t in tickets:
        out, st = s.wait(t, 11, timeout_s=100.0)
        assert out is not None and st.status == 0
        outs.append(out)
        admits.append(st.t_admit_ns)
        dones.append(st.t_done_ns)
    s.close()
    # Admission of the burst began while the long tick ran, and more of it was
    # admitted before that tick completed than the 64 MiB staging buffer
    # holds, so the buffer was flushed mid-admission (the flush waits for the
    # tick in flight).  Requests submitted while the flush held the scheduler
    # may be admitted after the next, short tick has finished part of the
    # burst: no order between admissions and completions is asserted.
    need = (16 << 11) + 64 * 500 + 16 * 64 * 500       # the server's bytes per burst request
    during = sum(need for a in admits if a < st0.t_done_ns)
    assert min(admits) < st0.t_done_ns and during > 64 << 20
    assert min(dones) > st0.t_done_ns                   # none finished inside the long tick
    for i, ((g, m, p), out) in enumerate(zip(burst, outs)):
        psi = torch.from_numpy(p).to("cuda")
        L.qcw_circuit(psi, 11, g, len(g), m, m.size)
        torch.cuda.synchronize()
        assert np.array_equal(psi.cpu().numpy(), out), i


def test_native_load_generator(L):
    """The native open-loop client (serve_load, built beside the library)
    drives the server with Poisson arrivals from two threads and collects
    every result: all requests complete, latencies are positive."""
    import os
    import bench
    exe = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1101_1785_amd", "serve_load")
    if not os.path.exists(exe):
        pytest.skip("serve_load not built")
    print("[gpu] native load generator, 2000 req/s for 0.3 s", flush=True)
    r = bench.bench_serving_native(L, qi, None, 0.3, rates=(2000,), pool=64)
    (row,) = r["server"]
    assert "error" not in row, row
    assert row["requests"] > 300 and row["failed"] == 0
    assert 0 < row["p50_ms"] <= row["p99_ms"]
