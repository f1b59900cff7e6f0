"""GPU parity of the batched form (one persistent launch in a hipGraph).

Every instance must equal, bit for bit, the plain path applied to that
instance alone (both run the same group arithmetic in the same FMA order),
and must match the oracle within the FP64 tolerance of the plain path.
Graph replays are checked one by one with eager work in between.
"""
import os

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


def _pack_states(instances):
    return np.concatenate([s for (_, s, _) in instances])


def _plain(L, instances):
    """Each instance alone through qcw_circuit."""
    outs = []
    for nq, psi0, c in instances:
        psi = torch.from_numpy(psi0).to("cuda")
        L.circuit(psi, c)
        outs.append(psi)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def _split(flat, instances):
    out, off = [], 0
    for nq, _, _ in instances:
        out.append(flat[off:off + (1 << nq)])
        off += 1 << nq
    return out


def _check_vs_oracle(outs, instances):
    refs = oracle.circuit_batch(instances)
    for o, r, (nq, _, c) in zip(outs, refs, instances):
        n = np.linalg.norm(r)
        assert np.linalg.norm(o - r) <= TOL * max(1, len(c) / 64) * n
        assert np.max(np.abs(o - r)) <= TOL * n


@pytest.mark.parametrize("lo,hi,count", [(3, 7, 300), (1, 11, 120), (9, 9, 64)])
def test_batch_equals_plain_and_oracle(L, lo, hi, count):
    print(f"[gpu] batch nq {lo}..{hi} x {count}", flush=True)
    inst = qi.batch(2, count, lo, hi)
    states = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states)
    b.run()
    torch.cuda.synchronize()
    outs = _split(states.cpu().numpy(), inst)
    plain = _plain(L, inst)
    for i, (o, p) in enumerate(zip(outs, plain)):
        assert np.array_equal(o, p), i
    _check_vs_oracle(outs, inst)
    b.close()


def test_every_variant_bit_identical(L, tmp_path):
    """Each tile shape gives the same bits (a table forcing one variant for all sizes)."""
    inst = qi.batch(5, 80, 2, 9)
    plain = _plain(L, inst)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    for v in range(5):  # the exact variants; amp4_mfma (5) has its own tests
        name = L.qcw_batch_variant_name(v)
        table = tmp_path / f"t{v}.txt"
        table.write_text(f"arch {arch}\n" + "".join(f"nq {q} variant {name}\n" for q in range(1, 12)))
        states = torch.from_numpy(_pack_states(inst)).to("cuda")
        b = L.Batch([(nq, c) for nq, _, c in inst], states, tune_table=str(table))
        assert L.qcw_batch_variant_name(b.info(5)[0]) == name
        b.run()
        torch.cuda.synchronize()
        for o, p in zip(_split(states.cpu().numpy(), inst), plain):
            assert np.array_equal(o, p), name
        b.close()


def _forced_table(L, tmp_path, name):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    table = tmp_path / f"{name}.txt"
    table.write_text(f"arch {arch}\n" + "".join(f"nq {q} variant {name}\n" for q in range(1, 12)))
    return str(table)


@pytest.mark.parametrize("lo,hi,count,seed", [(1, 11, 150, 8), (2, 3, 64, 9), (9, 9, 48, 10)])
def test_mfma_variant_matches_oracle_and_is_mix_independent(L, tmp_path, lo, hi, count, seed):
    """Two- and three-qubit gates on the matrix cores: a different summation
    order, so the bar is the oracle tolerance; each instance's bits must not
    depend on the other instances of the launch."""
    print(f"[gpu] mfma variant nq {lo}..{hi} x {count}", flush=True)
    table = _forced_table(L, tmp_path, "amp4_mfma")
    inst = qi.batch(seed, count, lo, hi)
    states = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states, tune_table=table)
    assert L.qcw_batch_variant_name(b.info(hi)[0]) == "amp4_mfma"
    b.run()
    torch.cuda.synchronize()
    outs = _split(states.cpu().numpy(), inst)
    b.close()
    _check_vs_oracle(outs, inst)
    for i in range(0, count, max(1, count // 8)):
        nq, p, c = inst[i]
        one = torch.from_numpy(p.copy()).to("cuda")
        b1 = L.Batch([(nq, c)], one, tune_table=table)
        b1.run()
        torch.cuda.synchronize()
        assert np.array_equal(one.cpu().numpy(), outs[i]), i
        b1.close()


def test_mfma_variant_named_gates_exact(L, tmp_path):
    """Permutation gates (CNOT, SWAP, Toffoli, X) have entries 0 and 1: every
    product is exact, so the matrix-core path must reproduce them exactly."""
    table = _forced_table(L, tmp_path, "amp4_mfma")
    rng = np.random.default_rng(12)
    inst = []
    for i in range(40):
        nq = int(rng.integers(3, 10))
        c = qi.Circuit(nq)
        for _ in range(3 * nq):
            k = int(rng.integers(1, 4))
            t = tuple(int(x) + 1 for x in rng.choice(nq, k, replace=False))
            c.add({1: qi.X, 2: qi.CNOT, 3: qi.TOFFOLI}[k] if i % 2 else
                  {1: qi.X, 2: qi.SWAP, 3: qi.TOFFOLI}[k], *t)
        inst.append((nq, qi.state(12, nq, i), c))
    states = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states, tune_table=table)
    b.run()
    torch.cuda.synchronize()
    outs = _split(states.cpu().numpy(), inst)
    b.close()
    for o, r in zip(outs, oracle.circuit_batch(inst)):
        assert np.array_equal(o, r)


def test_graph_replays_with_eager_work_between(L):
    inst = qi.batch(6, 50, 3, 8)
    states = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states)
    expect = [s.copy() for (_, s, _) in inst]
    for rep in range(3):
        b.run()
        torch.cuda.synchronize()
        scratch = torch.randn(1 << 16, device="cuda").sum().item()   # unrelated eager work
        assert np.isfinite(scratch)
        got = _split(states.cpu().numpy(), inst)
        nxt = []
        for (nq, _, c), e in zip(inst, expect):
            psi = torch.from_numpy(e).to("cuda")
            L.circuit(psi, c)
            nxt.append(psi.cpu().numpy())
        expect = nxt
        for i, (g, e) in enumerate(zip(got, expect)):
            assert np.array_equal(g, e), (rep, i)
    b.run_eager()
    torch.cuda.synchronize()
    got = _split(states.cpu().numpy(), inst)
    for (nq, _, c), e, g in zip(inst, expect, got):
        psi = torch.from_numpy(e).to("cuda")
        L.circuit(psi, c)
        assert np.array_equal(psi.cpu().numpy(), g)
    b.close()


@pytest.mark.parametrize("variant", [None, "amp4_mfma"])
def test_run_repeat_equals_single_replays(L, tmp_path, variant):
    """reps executions in one graph launch equal reps single replays, bit for
    bit, for the exact and the matrix-core shapes, with an oversize instance
    (plain sweeps) in the same graph; invalid counts are rejected."""
    inst = qi.batch(16, 60, 3, 9) + [(12, qi.state(16, 12, 9), qi.circuit(16, 12, 8, 9))]
    tt = None
    if variant:
        tt = str(tmp_path / "t.txt")
        with open(tt, "w") as f:
            f.write("arch gfx950\n" + "".join(f"nq {q} variant {variant}\n" for q in range(1, 12)))
    a = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = a.clone()
    ba = L.Batch([(nq, c) for nq, _, c in inst], a, tune_table=tt)
    bb = L.Batch([(nq, c) for nq, _, c in inst], b, tune_table=tt)
    for reps in (3, 1, 5):
        ba.run_repeat(reps)
        for _ in range(reps):
            bb.run()
        torch.cuda.synchronize()
        assert torch.equal(a, b), reps
    for bad in (0, -1, 1025):
        with pytest.raises(L.QcwError):
            ba.run_repeat(bad)
    ba.close()
    bb.close()


def test_oversize_instances_run_as_sweeps(L):
    """Instances above 11 qubits run as plain sweeps inside the same graph."""
    inst = [(12, qi.state(7, 12, 1), qi.circuit(7, 12, 10, 1)),
            (4, qi.state(7, 4, 2), qi.circuit(7, 4, 16, 2)),
            (13, qi.state(7, 13, 3), qi.circuit(7, 13, 6, 3))]
    states = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states)
    b.run()
    torch.cuda.synchronize()
    outs = _split(states.cpu().numpy(), inst)
    for o, p in zip(outs, _plain(L, inst)):
        assert np.array_equal(o, p)
    _check_vs_oracle(outs, inst)
    b.close()


def test_empty_and_gateless(L):
    states = torch.zeros(8, dtype=torch.complex128, device="cuda")
    b = L.Batch([], states)
    b.run()
    b.close()
    psi0 = qi.state(1, 3)
    states = torch.from_numpy(psi0.copy()).to("cuda")
    b = L.Batch([(3, qi.Circuit(3))], states)
    b.run()
    torch.cuda.synchronize()
    assert np.array_equal(states.cpu().numpy(), psi0)
    b.close()


def test_batch_validation(L):
    c = qi.circuit(0, 4, 4)
    states = torch.zeros(16 * 3, dtype=torch.complex128, device="cuda")
    inst, gates, mats, _ = L.pack_batch([(4, c), (4, c)])
    inst[1]["state_off"] = 8                                         # overlaps instance 0
    with pytest.raises(L.QcwError, match="overlap"):
        L.qcw_batch_create(inst, 2, gates, gates.size, mats, mats.size, states, states.numel())
    inst[1]["state_off"] = 40                                        # runs past the buffer
    with pytest.raises(L.QcwError, match="outside the states"):
        L.qcw_batch_create(inst, 2, gates, gates.size, mats, mats.size, states, states.numel())
    inst[1]["state_off"] = 16
    bad = gates.copy()
    bad[2]["q"][0] = 9
    with pytest.raises(L.QcwError, match="instance 0 gate 2"):
        L.qcw_batch_create(inst, 2, bad, bad.size, mats, mats.size, states, states.numel())


def test_tune_table_arch_checked(L, tmp_path):
    t = tmp_path / "other.txt"
    t.write_text("arch gfx000\nnq 3 variant amp4_sgpr\n")
    states = torch.zeros(8, dtype=torch.complex128, device="cuda")
    with pytest.raises(L.QcwError, match="gfx000"):
        L.Batch([(3, qi.circuit(0, 3, 2))], states, tune_table=str(t))


def test_autotune_writes_a_loadable_table(L, tmp_path):
    out = tmp_path / "tune.txt"
    L.qcw_batch_autotune(str(out), 3, 5, 64)
    text = out.read_text()
    assert "arch gfx" in text and "nq 5 variant" in text
    inst = qi.batch(8, 40, 3, 5)
    states = torch.from_numpy(_pack_states(inst)).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states, tune_table=str(out))
    chosen = {nq: L.qcw_batch_variant_name(b.info(nq)[0]) for nq in (3, 4, 5)}
    b.run()
    torch.cuda.synchronize()
    outs = _split(states.cpu().numpy(), inst)
    b.close()
    # exact variants reproduce the plain path bit for bit; the matrix-core one
    # agrees to rounding
    for o, p, (nq, _, _) in zip(outs, _plain(L, inst), inst):
        if chosen[nq] != "amp4_mfma":
            assert np.array_equal(o, p)
    _check_vs_oracle(outs, inst)


def test_committed_tune_table_loads(L):
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1101_1785_amd", "tune", "gfx950.txt")
    if not os.path.exists(path):
        pytest.skip("no committed tune table")
    states = torch.zeros(16, dtype=torch.complex128, device="cuda")
    b = L.Batch([(4, qi.circuit(0, 4, 3))], states, tune_table=path)
    b.close()
