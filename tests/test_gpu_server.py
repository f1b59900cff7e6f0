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
