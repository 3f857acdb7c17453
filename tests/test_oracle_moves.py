"""Pins of the move-application oracle (``oracle/moves.py``, the paper's
paragraph "Apply Moves").

* ``connectivity`` against hand-computed values;
* every applied sequence's gain equals the objective recomputed from
  scratch before and after it (the gain is the exact change of
  sum w(e) (lambda(e) - 1), however the pin counts cross zero);
* a reverted sequence leaves the partition as it was, a rejected one too,
  and rejection happens exactly when block i or j would exceed Lmax;
* moves of vertices that left their expected block (an earlier sequence
  moved them) are dropped.
"""
import numpy as np

from paper_2201_01556_amd import inputs
from oracle import moves


def _hg(nets, weights, V):
    return inputs.hypergraph_from_nets(V, nets, weights, [0], [V - 1])


def test_connectivity_by_hand():
    hg = _hg([[0, 1, 2], [2, 3], [0, 3, 4, 5]], [2, 1, 5], 6)
    block = np.array([0, 0, 1, 1, 2, 2])
    # lambda: 2, 1, 3 -> 2*1 + 1*0 + 5*2
    assert moves.connectivity(hg, block) == 12
    assert moves.connectivity(hg, np.zeros(6, int)) == 0


def _random_case(seed, V=60, E=90, k=4):
    rng = np.random.default_rng(seed)
    nets = [sorted(rng.choice(V, int(rng.integers(2, 7)), replace=False).tolist())
            for _ in range(E)]
    hg = _hg(nets, rng.integers(1, 4, E).tolist(), V)
    c = rng.integers(1, 4, V)
    block = rng.integers(0, k, V)
    seqs = []
    for _ in range(12):
        i, j = rng.choice(k, 2, replace=False)
        region = np.nonzero((block == i) | (block == j))[0]
        region = rng.choice(region, min(len(region), int(rng.integers(1, 15))), replace=False)
        region.sort()
        seqs.append(dict(pair=(int(i), int(j)), gid=region, expected=block[region].copy(),
                         side=rng.integers(0, 2, len(region)),
                         gain=int(rng.integers(-1, 4))))
    return hg, c, block, seqs


def test_gains_are_exact_and_reverts_restore():
    statuses = set()
    for seed in range(40):
        hg, c, block, seqs = _random_case(seed)
        k = 4
        lmax = int(np.ceil(c.sum() / k * (1.3 if seed % 2 else 1.05)))
        cur = block.copy()
        for s in seqs:
            before = moves.connectivity(hg, cur)
            bw = np.bincount(cur, weights=c, minlength=k)
            nxt, ((st, gain, nm),) = moves.apply_sequences(hg, cur, c, k, lmax, [s])
            after = moves.connectivity(hg, nxt)
            statuses.add(st)
            if st == moves.APPLIED:
                assert before - after == gain >= 0
                assert nm == int((nxt != cur).sum())
            else:
                assert (nxt == cur).all()
            if st == moves.REVERTED:
                assert gain < 0
            if st == moves.NOT_TRIED:
                assert s["gain"] <= 0
            i, j = s["pair"]
            # which moves survive the expected-block filter, and the weights
            # they would give blocks i and j
            wi, wj = bw[i], bw[j]
            for u, exp, x in zip(s["gid"], s["expected"], s["side"]):
                to = i if x else j
                if to != exp and cur[u] == exp:
                    d = c[u] if to == i else -c[u]
                    wi, wj = wi + d, wj - d
            if s["gain"] > 0:
                assert (st == moves.UNBALANCED) == (wi > lmax or wj > lmax)
            cur = nxt
        # the sequences applied in one call give the same result
        whole, _ = moves.apply_sequences(hg, block, c, k, lmax, seqs)
        assert (whole == cur).all()
    assert statuses == {0, 1, 2, 3}


def test_stale_moves_are_dropped():
    hg = _hg([[0, 1], [1, 2], [2, 3], [3, 0]], [1, 1, 1, 1], 4)
    c = np.ones(4, int)
    block = np.array([0, 0, 1, 1])
    # both sequences move vertex 1 from block 0 to block 1; the second finds
    # it in block 1 already and drops the move
    s = dict(pair=(0, 1), gid=np.array([1]), expected=np.array([0]), side=np.array([0]), gain=1)
    out_block, res = moves.apply_sequences(hg, block, c, 2, 10, [s, dict(s)])
    assert out_block.tolist() == [0, 1, 1, 1]
    assert res[0][0] == moves.APPLIED and res[0][2] == 1
    assert res[1] == (moves.APPLIED, 0, 0)


def test_refine_rounds_improve_and_stay_balanced():
    """The refinement rounds on a planted 4-block hypergraph with perturbed
    blocks: the objective never grows, every block stays within Lmax, and
    the trajectory equals the objective recomputed from the blocks."""
    import oracle
    oracle.build()
    bp = inputs.planted_block_pair_problems(2, num_vertices=4000, target_pins=16000, size_hi=40,
                                            k=4, noisy_pairs=3, swap_fraction=0.1,
                                            max_problems=6, threads=1)
    hg = bp.hypergraph
    blocks, traj, log = moves.refine(hg, bp.block, hg.vertex_weights, 4, max_rounds=4)
    assert traj[0] == moves.connectivity(hg, bp.block)
    assert traj[-1] == moves.connectivity(hg, blocks)
    assert all(a >= b for a, b in zip(traj, traj[1:]))
    assert traj[-1] < traj[0]
    bw = np.bincount(blocks, weights=hg.vertex_weights, minlength=4)
    cv = int(hg.vertex_weights.sum())
    assert bw.max() <= (103 * (-(-cv // 4))) // 100
    applied = [e for rnd in log for e in rnd if e[1] == moves.APPLIED]
    assert applied and sum(e[2] for e in applied) == traj[0] - traj[-1]
