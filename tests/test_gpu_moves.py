"""GPU parity of applying block-pair results to a partition on the device
(flow_partition_apply) against the oracle of the paragraph "Apply Moves"
(``oracle/moves.py``): statuses, exact gains, move counts, the final
blocks, block weights and objective, bit-exact."""
import numpy as np
import pytest

from paper_2201_01556_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-moves] {msg}", flush=True)


@pytest.fixture(scope="module")
def hf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_01556_amd import hyperflow
    hyperflow.load_library()
    return hyperflow


def _run(hf, bp, k, merge, lmax=None):
    """Regions on the device, one union batch with sides, then the moves
    applied on the device and by the oracle."""
    import torch
    from oracle import moves as omoves
    hg = bp.hypergraph
    pairs = [p.meta["pair"] for p in bp.problems]
    cuts = [p.meta["cut"] for p in bp.problems]
    caps = inputs.region_caps(bp.block_weights, pairs, cuts)
    lmax = bp.lmax if lmax is None else lmax
    with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                        hg.vertex_weights, bp.block, k, pairs, caps,
                        merge_identical=merge) as rg:
        probs = [rg.problem(q) for q in range(len(pairs))]
        try:
            with hf.FlowBatch(probs, with_cut=True) as plan:
                flows = plan.run(with_cut=True)
                torch.cuda.synchronize()
                sides = [t.cpu().numpy()[:rg.info(q)["n"]] for q, t in
                         enumerate(plan.vertex_sides)]
                gains = np.array([rg.info(q)["cut_before"] - int(flows[q])
                                  for q in range(len(pairs))], dtype=np.int64)
                with hf.FlowPartition(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                                      hg.vertex_weights, bp.block, k) as part:
                    _, bw0, obj0 = part.get()
                    st, g, mv = part.apply(rg, plan.vertex_sides, gains, lmax)
                    blocks, bw, obj = part.get()
        finally:
            for p in probs:
                p.close()
        seqs = []
        for q, (i, j) in enumerate(pairs):
            gid = rg.export(q)["vertex_ids"]
            seqs.append(dict(pair=(i, j), gid=gid, expected=bp.block[gid], side=sides[q],
                             gain=int(gains[q])))
    ref_block, ref = omoves.apply_sequences(hg, bp.block, hg.vertex_weights, k, lmax, seqs)
    return (st, g, mv, blocks, bw, obj, obj0, bw0), (ref_block, ref)


@pytest.mark.parametrize("merge", [False, True])
def test_apply_planted_pairs_vs_oracle(hf, merge):
    """Planted 16-block hypergraph (320,000 vertices, ~1.6M pins, 30 perturbed
    pairs), 100 heaviest pairs: the minimum cuts of perturbed pairs recover
    swapped vertices; statuses, gains, moves and the final partition equal
    the oracle's."""
    from oracle import moves as omoves
    bp = inputs.planted_block_pair_problems(0, num_vertices=320_000, target_pins=1_600_000,
                                            k=16, noisy_pairs=30, max_problems=100, threads=4)
    (st, g, mv, blocks, bw, obj, obj0, bw0), (ref_block, ref) = _run(hf, bp, 16, merge)
    _say(f"merge={merge}: statuses {np.bincount(st, minlength=4).tolist()}, "
         f"gain {int(g[st == 1].sum())}, objective {obj0} -> {obj}")
    assert [tuple(int(x) for x in r) for r in ref] == list(zip(st.tolist(), g.tolist(),
                                                               mv.tolist()))
    assert (blocks == ref_block).all()
    assert (bw == np.bincount(ref_block, weights=bp.hypergraph.vertex_weights,
                              minlength=16)).all()
    assert obj0 - obj == int(g[st == 1].sum())
    assert obj == omoves.connectivity(bp.hypergraph, ref_block)
    assert (st == 1).sum() > 0 and obj < obj0


def test_apply_tight_balance_and_conflicts(hf):
    """Random k = 8 partition with a tight Lmax (many sequences rejected)
    and overlapping regions (later sequences find moved vertices and drop
    them): still equal to the oracle."""
    bp = inputs.block_pair_problems(1, num_vertices=40_000, target_pins=200_000, size_hi=100,
                                    k=8, max_problems=28, threads=4)
    lmax = int(np.ceil(bp.block_weights.sum() / 8 * 1.01))
    (st, g, mv, blocks, bw, obj, obj0, bw0), (ref_block, ref) = _run(hf, bp, 8, False, lmax)
    _say(f"tight: statuses {np.bincount(st, minlength=4).tolist()}")
    assert [tuple(int(x) for x in r) for r in ref] == list(zip(st.tolist(), g.tolist(),
                                                               mv.tolist()))
    assert (blocks == ref_block).all()
    assert obj0 - obj == int(g[st == 1].sum())


def test_partition_errors(hf):
    hg = inputs.uniform_hypergraph(0)
    block = np.zeros(hg.num_vertices, np.int32)
    block[::2] = 1
    with pytest.raises(hf.HyperflowError) as ei:
        hf.FlowPartition(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                         hg.vertex_weights, block, 1)
    assert ei.value.name == "FP_ERR_INVALID"
    bad = block.copy()
    bad[5] = 2
    with pytest.raises(hf.HyperflowError) as ei:
        hf.FlowPartition(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                         hg.vertex_weights, bad, 2)
    assert ei.value.name == "FP_ERR_INVALID"
    with hf.FlowPartition(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                          hg.vertex_weights, block, 2) as part:
        blocks, bw, obj = part.get()
        assert (blocks == block).all()
        from oracle import moves as omoves
        assert obj == omoves.connectivity(hg, block)
        assert bw.tolist() == np.bincount(block, weights=hg.vertex_weights,
                                          minlength=2).astype(int).tolist()


@pytest.mark.parametrize("merge", [True, False])
def test_refine_rounds_vs_oracle(hf, merge):
    """Refinement rounds on the device (quotient graph, regions, union
    minimum cuts, moves) against the oracle's rounds on a planted 8-block
    hypergraph (24,000 vertices, ~100k pins, 6 perturbed pairs): the same
    trajectory of the objective and the same final blocks."""
    from oracle import moves as omoves
    import oracle
    oracle.build()
    bp = inputs.planted_block_pair_problems(3, num_vertices=24_000, target_pins=100_000,
                                            size_hi=200, k=8, noisy_pairs=6, max_problems=4,
                                            threads=4)
    hg = bp.hypergraph
    ref_block, ref_traj, _ = omoves.refine(hg, bp.block, hg.vertex_weights, 8, max_rounds=5)
    with hf.FlowPartition(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                          hg.vertex_weights, bp.block, 8) as part:
        res, traj = part.refine(max_rounds=5, merge_identical=merge)
        blocks, bw, obj = part.get()
    _say(f"refine merge={merge}: {res}, trajectory {traj.tolist()}")
    assert traj.tolist() == list(ref_traj)
    assert (blocks == ref_block).all()
    assert res["objective_after"] == obj == ref_traj[-1] < ref_traj[0]
