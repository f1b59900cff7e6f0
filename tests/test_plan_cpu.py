"""Pass planning of the fused path (qcw_fused_plan, host code).

The plan flag QCW_PLAN_COMMUTE lets a gate join an earlier pass ahead of
deferred gates it shares no qubit with: operators on disjoint qubits commute
(§2c tensor structure), so the circuit's operator is unchanged.  Pins, none of
which reads the planner's own rules back:
* every gate runs exactly once, and any two gates that share a qubit run in
  list order (the only order the operator fixes);
* each pass's tile holds the low bits and its gates' targets within tile_bits;
* the oracle, applying the gates in the planned order, moves a state as it does
  in list order (FP64 tolerance);
* with no flag the order is the list order and passes are maximal runs;
* two alternating gate sets on disjoint qubits that cannot share a tile take
  one pass each with the flag, and one pass per alternation without it.
"""
import numpy as np
import pytest

import oracle
import qcw_inputs as qi

TOL = 1e-12
COMMUTE, FUSE, M3 = 1, 2, 4


@pytest.fixture(scope="module")
def L():
    from paper_1101_1785_amd import _lib
    return _lib


def _check_plan(c, n, pass_of, order, tile_bits, low_bits):
    G = len(c)
    assert sorted(order.tolist()) == list(range(G))
    pos = np.empty(G, dtype=np.int64)
    pos[order] = np.arange(G)
    # passes run one after another: pass index never decreases along the order
    assert np.all(np.diff(pass_of[order]) >= 0)
    assert pass_of.min() == 0 and pass_of.max() == n - 1
    # gates sharing a qubit keep their list order
    for i in range(G):
        for j in range(i + 1, G):
            if set(c.targets[i]) & set(c.targets[j]):
                assert pos[i] < pos[j], (i, j)
    # tile budget: low bits plus the pass's target bits
    nq = c.nq
    for p in range(n):
        bits = set(range(min(low_bits, nq)))
        for g in np.nonzero(pass_of == p)[0]:
            bits |= {nq - q for q in c.targets[g]}
        assert len(bits) <= tile_bits
    return pos


@pytest.mark.parametrize("nq,seed", [(9, 1), (12, 2), (16, 3), (22, 4), (31, 1), (31, 2)])
@pytest.mark.parametrize("tile_bits,low_bits", [(8, 5), (12, 4), (13, 3)])
def test_commute_plan_is_a_valid_reordering(L, nq, seed, tile_bits, low_bits):
    c = qi.circuit(seed, nq, 4 * nq)
    g, _ = L.pack_circuit(c)
    n, pass_of, order = L.qcw_fused_plan(nq, g, len(c), tile_bits, low_bits, COMMUTE)
    _check_plan(c, n, pass_of, order, tile_bits, low_bits)
    n0 = L.qcw_fused_pass_count(nq, g, len(c), tile_bits, low_bits, 0)
    assert n <= n0
    assert L.qcw_fused_pass_count(nq, g, len(c), tile_bits, low_bits, COMMUTE | FUSE) == n
    assert L.qcw_fused_pass_count(nq, g, len(c), tile_bits, low_bits, COMMUTE | FUSE | M3) == n


@pytest.mark.parametrize("nq,seed", [(9, 5), (11, 6), (13, 7)])
def test_planned_order_moves_state_like_list_order(L, nq, seed):
    c = qi.circuit(seed, nq, 6 * nq)
    g, _ = L.pack_circuit(c)
    n, pass_of, order = L.qcw_fused_plan(nq, g, len(c), 8, 3, COMMUTE)
    assert n < len(c)
    assert not np.array_equal(order, np.arange(len(c)))   # something moved
    r = qi.Circuit(nq)
    for i in order:
        r.add(c.mats[i], *c.targets[i])
    psi = qi.state(seed, nq, 2)
    a, b = oracle.circuit(c, psi), oracle.circuit(r, psi)
    assert np.linalg.norm(a - b) <= TOL * np.linalg.norm(a)


def test_list_plan_is_maximal_runs(L):
    for seed in range(4):
        nq = 20
        c = qi.circuit(60 + seed, nq, 80)
        g, _ = L.pack_circuit(c)
        n, pass_of, order = L.qcw_fused_plan(nq, g, len(c), 12, 4, 0)
        assert np.array_equal(order, np.arange(len(c)))
        _check_plan(c, n, pass_of, order, 12, 4)
        # a pass ends only where the next gate would overflow the tile
        for i in range(len(c) - 1):
            if pass_of[i + 1] != pass_of[i]:
                bits = set(range(4))
                for j in np.nonzero(pass_of == pass_of[i])[0]:
                    bits |= {nq - q for q in c.targets[j]}
                bits |= {nq - q for q in c.targets[i + 1]}
                assert len(bits) > 12


def test_alternating_disjoint_sets(L):
    """Gates alternate between qubits 1..8 and 9..16 of a 24-qubit state; with
    4 low bits a 12-bit tile holds exactly one set.  Reordering may gather
    each set into one pass; list order needs a pass per alternation."""
    nq = 24
    c = qi.Circuit(nq)
    rounds = 5
    for r in range(rounds):
        for q in range(1, 9):
            c.add(qi.H, q)
        for q in range(9, 17):
            c.add(qi.H, q)
    g, _ = L.pack_circuit(c)
    assert L.qcw_fused_pass_count(nq, g, len(c), 12, 4, 0) == 2 * rounds
    n, pass_of, order = L.qcw_fused_plan(nq, g, len(c), 12, 4, COMMUTE)
    assert n == 2
    _check_plan(c, n, pass_of, order, 12, 4)


def test_plan_validation(L):
    c = qi.circuit(0, 12, 8)
    g, _ = L.pack_circuit(c)
    with pytest.raises(L.QcwError):
        L.qcw_fused_plan(12, g, len(c), 12, 4, 8)
    with pytest.raises(L.QcwError):
        L.qcw_fused_pass_count(12, g, len(c), 12, 4, -1)
    with pytest.raises(L.QcwError):
        L.qcw_fused_plan(12, g, len(c), 14, 4, 0)
    n, pass_of, order = L.qcw_fused_plan(8, *L.pack_circuit(qi.circuit(0, 8, 5))[:1], 5, 12, 4, COMMUTE)
    assert n == 5 and np.array_equal(order, np.arange(5))   # below 9 qubits: one sweep per gate
