"""Address maps of the fused passes, from the plan tables the host builds for
the device (qcw_debug_fused_tables; host code, no GPU).

A fused pass gives block b the tile of 2^T amplitudes whose local index i
has the label
    label(b, i) = sum_j bit_j(b) 2^outer_pos[j] + chunk_off[i >> L] + (i & (2^L - 1)),
loads it into LDS, applies its gates at the local positions
insert_zeros(j) + off[r] (a zero bit inserted at each local target bit, in
ascending order, §3a-§3c Pick), and stores it back to the same labels.  For
every tile shape the kernels accept (T = 8..13, L = 3..5, T - L <= 10), states
of up to 16 qubits and the plan flags, these tests check:
* the label map is a bijection of (block, local index) onto [0, 2^nq): every
  amplitude is loaded and stored by exactly one block, and none outside the
  state;
* each gate's groups cover the tile's local indices exactly once, inside the
  tile;
* running the passes through these tables on the CPU (numpy, all tiles of a
  pass at once) moves a random state as the oracle's circuit does;
* the same run with the last gate of each pass storing its outputs straight
  to their labels (no store of the tile afterwards) gives the same state, with
  every store inside the state.  That is the addressing of a kernel variant
  that was dropped after wrong results and a GPU fault on 11-bit tiles with
  3 low bits (nq = 14 among them); the tables it used are shown sound here.
"""
import numpy as np
import pytest

import oracle
import qcw_inputs as qi

COMMUTE, FUSE, M3 = 1, 2, 4
SHAPES = [(T, L) for T in range(8, 14) for L in (3, 4, 5) if T - L <= 10]


@pytest.fixture(scope="module")
def L():
    from paper_1101_1785_amd import _lib
    return _lib


def _insert_zeros(j, bits):
    x = j.copy()
    for b in sorted(bits):
        b = np.uint64(b)
        x = ((x >> b) << (b + np.uint64(1))) | (x & ((np.uint64(1) << b) - np.uint64(1)))
    return x


def _labels(P, nq):
    """(blocks, 2^T) array of labels, from the kernels' formula."""
    T, Lb = P["T"], P["L"]
    assert len(P["outer_pos"]) == nq - T
    b = np.arange(1 << (nq - T), dtype=np.uint64)
    base = np.zeros_like(b)
    for j, pos in enumerate(P["outer_pos"]):
        base |= ((b >> np.uint64(j)) & np.uint64(1)) << np.uint64(pos)
    i = np.arange(1 << T, dtype=np.uint64)
    loc = P["chunk_off"][i >> np.uint64(Lb)] + (i & np.uint64((1 << Lb) - 1))
    return base[:, None] + loc[None, :]


def _members(g, T):
    """(groups, m) local indices of a gate's groups, group order, local index order."""
    k = g["k"]
    j = np.arange(1 << (T - k), dtype=np.uint64)
    base = _insert_zeros(j, g["sb"][:k])
    return base[:, None] + np.array(g["off"][:1 << k], dtype=np.uint64)[None, :]


def _tables(L, nq, T, Lb, plan, seed):
    c = qi.circuit(seed, nq, 4 * nq)
    g, m = L.pack_circuit(c)
    return c, L.qcw_debug_fused_tables(nq, g, len(c), m, T, Lb, plan)


@pytest.mark.parametrize("T,Lb", SHAPES)
@pytest.mark.parametrize("nq", [9, 12, 14, 16])
@pytest.mark.parametrize("plan", [0, COMMUTE, COMMUTE | FUSE | M3])
def test_label_map_is_a_bijection(L, T, Lb, nq, plan):
    if T > nq:
        pytest.skip("tile larger than the state")
    c, tb = _tables(L, nq, T, Lb, plan, seed=nq + 17 * T + Lb)
    N = 1 << nq
    for P in tb["passes"]:
        assert (P["T"], P["L"]) == (T, Lb)
        assert P["chunk_off"].size == 1 << (T - Lb)
        lab = _labels(P, nq).reshape(-1)
        assert lab.max() < N
        assert np.array_equal(np.bincount(lab.astype(np.int64), minlength=N), np.ones(N, np.int64))
        for g in tb["gates"][P["gate_off"]:P["gate_off"] + P["ngates"]]:
            mem = _members(g, T).reshape(-1)
            assert mem.max() < (1 << T)
            assert np.array_equal(np.sort(mem), np.arange(1 << T, dtype=np.uint64))


def _run_passes(tb, psi, nq, direct_last):
    psi = psi.copy()
    N = 1 << nq
    for P in tb["passes"]:
        T = P["T"]
        lab = _labels(P, nq).astype(np.int64)
        tile = psi[lab]
        gl = tb["gates"][P["gate_off"]:P["gate_off"] + P["ngates"]]
        for gi, g in enumerate(gl):
            mem = _members(g, T).astype(np.int64)
            y = tile[:, mem] @ g["u"].T          # y[r] = sum_c U[r][c] x[c] per group
            if direct_last and gi == len(gl) - 1:
                out = lab[:, mem]                # the members' labels
                assert out.min() >= 0 and out.max() < N
                psi[out] = y
            else:
                tile[:, mem] = y
        if not direct_last:
            psi[lab] = tile
    return psi


@pytest.mark.parametrize("T,Lb", SHAPES)
@pytest.mark.parametrize("nq", [11, 14])
@pytest.mark.parametrize("plan", [0, COMMUTE | FUSE])
def test_passes_through_tables_match_oracle(L, T, Lb, nq, plan):
    if T > nq:
        pytest.skip("tile larger than the state")
    c, tb = _tables(L, nq, T, Lb, plan, seed=nq + 17 * T + Lb)
    psi0 = qi.state(nq + T, nq, tag=5)
    ref = oracle.circuit(c, psi0)
    got = _run_passes(tb, psi0, nq, direct_last=False)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    direct = _run_passes(tb, psi0, nq, direct_last=True)
    assert np.array_equal(direct, got)
