"""The paper's example workloads on the batched and served paths, checked
against their closed forms (qcw_inputs.workloads): Grover search instances with
different marked items and iteration counts in one launch, the GHZ chain and
Bell followed by its inverse."""
import numpy as np
import pytest

import qcw_inputs as qi
from qcw_inputs import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_1785_amd import _lib
    return _lib


def _grover_instances(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(2, 7))
        marked = int(rng.integers(0, 1 << n))
        k = int(rng.choice([0, 1, W.grover_optimal_iterations(n)]))
        c = W.grover(n, marked, k)
        out.append((n, marked, k, c))
    return out


def _expected(n, marked, k):
    nq = W.grover_qubits(n)
    a, b = W.grover_amplitudes(n, k)
    ref = np.zeros(1 << nq, complex)
    for d in range(1 << n):
        ref[d << (nq - n)] = a if d == marked else b
    return ref


def _forced_table(tmp_path, name):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    t = tmp_path / f"{name}.txt"
    t.write_text(f"arch {arch}\n" + "".join(f"nq {q} variant {name}\n" for q in range(1, 12)))
    return str(t)


@pytest.mark.parametrize("shape", ["amp4_lds", "amp4_mfma"])
def test_grover_batch_closed_form(L, tmp_path, shape):
    print(f"[gpu] grover batch {shape}", flush=True)
    inst = _grover_instances(5, 200)
    states = torch.from_numpy(np.concatenate([qi.basis_state(c.nq, 0) for *_, c in inst])).to("cuda")
    b = L.Batch([(c.nq, c) for *_, c in inst], states, tune_table=_forced_table(tmp_path, shape))
    b.run()
    torch.cuda.synchronize()
    flat = states.cpu().numpy()
    b.close()
    off = 0
    for n, marked, k, c in inst:
        out = flat[off:off + (1 << c.nq)]
        off += 1 << c.nq
        assert np.max(np.abs(out - _expected(n, marked, k))) <= TOL, (n, marked, k)


def test_grover_served_closed_form(L):
    inst = _grover_instances(6, 80)
    s = L.Server(hbm_budget_bytes=32 << 20, max_slots=64, max_nq=10)
    tickets = [s.submit(c.nq, c, qi.basis_state(c.nq, 0)) for *_, c in inst]
    for t, (n, marked, k, c) in zip(tickets, inst):
        out, st = s.wait(t, c.nq)
        assert out is not None and st.status == 0
        assert np.max(np.abs(out - _expected(n, marked, k))) <= TOL
    s.close()


def test_ghz_and_bell_in_one_batch(L):
    cs = [W.ghz_chain(n) for n in (2, 5, 9, 11)] + [W.bell_and_inverse()] * 3
    states = torch.from_numpy(np.concatenate([qi.basis_state(c.nq, 0) for c in cs])).to("cuda")
    b = L.Batch([(c.nq, c) for c in cs], states)
    b.run()
    torch.cuda.synchronize()
    flat = states.cpu().numpy()
    b.close()
    off = 0
    for c in cs:
        out = flat[off:off + (1 << c.nq)]
        off += 1 << c.nq
        ref = np.zeros(1 << c.nq, complex)
        if c.nq == 2 and len(c) == 4:          # Bell then inverse: back to |00>
            ref[0] = 1.0
            assert np.max(np.abs(out - ref)) <= 4e-16
        else:
            ref[0] = ref[-1] = qi.S2
            assert np.array_equal(out, ref)
