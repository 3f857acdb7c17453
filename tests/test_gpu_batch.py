"""GPU parity of the batch API (flow_batch_solve and batch plans) against
the CPU oracle, through the C ABI.

A batch runs the same device phases as the single-problem path under a
different schedule, so flow values and minimal source sides must match the
oracle bit-exactly for every configuration: the union schedule (the kept
problems as one network, the default) and the workers schedule (each
problem on its own stream).
"""
import os
import sys
import tempfile

import numpy as np
import pytest

from paper_2201_01556_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batch] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_01556_amd import hyperflow
    hyperflow.load_library()
    return hyperflow


def uneven_set(n, seed0=0):
    """Uniform hypergraphs of different sizes (uneven batch)."""
    out = []
    for i in range(n):
        V = 200 + 300 * (i % 7)
        out.append(inputs.uniform_hypergraph(seed0 + i, num_vertices=V,
                                             num_nets=int(1.5 * V), num_sources=V // 20,
                                             num_sinks=V // 20))
    return out


@pytest.fixture(scope="module")
def small_pairs():
    return inputs.block_pair_problems(0, num_vertices=20000, target_pins=100000, k=8,
                                      max_problems=50)


def _oracle_all(oracle_mod, hgs):
    return [oracle_mod.maxflow(h) for h in hgs]


def _check_sides(batch, hgs, refs, tag):
    for i, (h, r) in enumerate(zip(hgs, refs)):
        vs, ns = batch.sides(i)
        bad = np.nonzero(vs.astype(bool) != r.vertex_side.astype(bool))[0]
        assert bad.size == 0, f"{tag} problem {i}: {bad.size} vertex sides differ"
        badn = np.nonzero(ns != r.net_side)[0]
        assert badn.size == 0, f"{tag} problem {i}: {badn.size} net sides differ"


def test_batch_solve_uneven_vs_oracle(hf, oracle_mod):
    hgs = uneven_set(40)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say("flow_batch_solve, 40 uneven problems")
        flows = hf.flow_batch_solve([p.handle for p in probs])
        assert list(flows) == [r.flow for r in refs]
        # the default (union) schedule leaves the handles as they were
        with pytest.raises(hf.HyperflowError) as ei:
            probs[0].source_side()
        assert ei.value.name == "FP_ERR_STATE"
        # with the workers schedule a solved handle behaves as after maxflow_solve
        with hf.FlowBatch(probs, schedule=2, streams=4) as b:
            assert list(b.run()) == [r.flow for r in refs]
        for i in (0, 13, 39):
            vs, ns = probs[i].source_side()
            assert (vs.astype(bool) == refs[i].vertex_side.astype(bool)).all()
            assert (ns == refs[i].net_side).all()
            assert probs[i].solve() == refs[i].flow  # warm re-solve
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("lanes,schedule,streams", [(4, 2, 1), (8, 2, 4), (16, 2, 16),
                                                    (4, 1, 0), (8, 1, 0), (16, 0, 0)])
def test_batch_plan_configs_with_cut(hf, oracle_mod, lanes, schedule, streams):
    hgs = uneven_set(24, seed0=100)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say(f"plan lanes={lanes} schedule={schedule} streams={streams}")
        with hf.FlowBatch(probs, with_cut=True, group_lanes=lanes, schedule=schedule,
                          streams=streams) as b:
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            _check_sides(b, hgs, refs, f"lanes={lanes} schedule={schedule}")
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("gr", [-1, 1, 8, 64])
def test_batch_relabel_intervals(hf, oracle_mod, gr):
    hgs = uneven_set(12, seed0=200)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say(f"gr_interval={gr}")
        for schedule in (1, 2, 3):
            with hf.FlowBatch(probs, with_cut=True, gr_interval=gr, schedule=schedule,
                              streams=5) as b:
                flows = b.run(with_cut=True)
                assert list(flows) == [r.flow for r in refs]
                _check_sides(b, hgs, refs, f"gr={gr} schedule={schedule}")
    finally:
        for p in probs:
            p.close()


def test_batch_block_pairs_vs_oracle(hf, oracle_mod, small_pairs):
    hgs = small_pairs.problems
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say(f"{len(hgs)} block-pair problems")
        with hf.FlowBatch(probs, with_cut=True) as b:
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            _check_sides(b, hgs, refs, "block pairs")
            for h, f in zip(hgs, flows):
                assert 0 <= f <= h.meta["cut_before"]
            # a second run of the plan
            flows2 = b.run(with_cut=True)
            assert list(flows2) == list(flows)
            _check_sides(b, hgs, refs, "block pairs replay")
    finally:
        for p in probs:
            p.close()


def test_batch_skip_and_reset(hf, oracle_mod):
    hgs = uneven_set(10, seed0=300)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        skip = np.zeros(10, dtype=np.uint8)
        skip[[1, 4, 9]] = 1
        with hf.FlowBatch(probs, with_cut=True) as b:
            flows = b.run(skip=skip, with_cut=True)
            for i in range(10):
                assert flows[i] == (-1 if skip[i] else refs[i].flow)
            # skipped problems were left alone: still unsolved
            with pytest.raises(hf.HyperflowError):
                probs[1].source_side()
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            for p in probs:
                p.reset()
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            _check_sides(b, hgs, refs, "after reset")
    finally:
        for p in probs:
            p.close()


def test_batch_tune_and_cache(hf, oracle_mod):
    hgs = uneven_set(16, seed0=400)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        with tempfile.TemporaryDirectory() as d:
            cache = os.path.join(d, "tune.txt")
            with hf.FlowBatch(probs, with_cut=True) as b:
                cfg = b.tune(cache)
                assert cfg["group_lanes"] in (4, 8, 16)
                assert cfg["schedule"] in (1, 2, 3)
                assert 1 <= cfg["streams"] <= 64
                assert cfg["wg_threads"] in (256, 1024)
                assert b.config() == cfg
                flows = b.run(with_cut=True)
                assert list(flows) == [r.flow for r in refs]
                _check_sides(b, hgs, refs, "tuned")
            with open(cache) as f:
                assert len(f.read().strip().splitlines()) == 1
            with hf.FlowBatch(probs) as b2:
                assert b2.tune(cache) == cfg  # from the cache
            with open(cache) as f:
                assert len(f.read().strip().splitlines()) == 1
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("lanes,gr", [(4, 0), (8, -1), (16, 8), (8, 1)])
def test_batch_union_vs_oracle(hf, oracle_mod, lanes, gr):
    """Union schedule: the kept problems solved as one network; flows and
    minimal source sides per problem equal the oracle's."""
    hgs = uneven_set(24, seed0=600)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say(f"union schedule lanes={lanes} gr={gr}")
        with hf.FlowBatch(probs, with_cut=True, schedule=1, group_lanes=lanes,
                          gr_interval=gr) as b:
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            _check_sides(b, hgs, refs, f"union lanes={lanes} gr={gr}")
            skip = np.zeros(24, dtype=np.uint8)
            skip[[0, 5, 23]] = 1
            flows = b.run(skip=skip)
            for i in range(24):
                assert flows[i] == (-1 if skip[i] else refs[i].flow)
            assert list(b.run(skip=np.ones(24, dtype=np.uint8))) == [-1] * 24
    finally:
        for p in probs:
            p.close()


def test_batch_union_chunks(hf, oracle_mod):
    """A bound on the pins per union splits the kept problems over several
    unions (in index order); flows and sides are unchanged."""
    hgs = uneven_set(16, seed0=700)
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        for bound in (1, 3000, 20000):
            _say(f"union chunks of at most {bound} pins")
            with hf.FlowBatch(probs, with_cut=True, schedule=1, union_pins=bound) as b:
                flows = b.run(with_cut=True)
                assert list(flows) == [r.flow for r in refs]
                _check_sides(b, hgs, refs, f"union_pins={bound}")
    finally:
        for p in probs:
            p.close()


def test_batch_union_weight_sums(hf, oracle_mod):
    """Problems whose net weights each sum to nearly INT32_MAX go to separate
    unions (one union would overflow the int32 capacities); flows and sides
    are the oracle's."""
    hgs = [inputs.tiny_hypergraph(s) for s in (3, 9, 15, 21, 27)]  # weights near the guard
    assert sum(int(h.net_weights.astype(np.int64).sum()) for h in hgs) > 2**31
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say("union of problems with large weight sums")
        with hf.FlowBatch(probs, with_cut=True, schedule=1) as b:
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            _check_sides(b, hgs, refs, "weight sums")
    finally:
        for p in probs:
            p.close()


def test_batch_union_block_pairs_and_pierced(hf, oracle_mod, small_pairs):
    """Union schedule on block-pair regions, then with one problem pierced:
    the union takes each problem's current terminals."""
    hgs = small_pairs.problems
    refs = _oracle_all(oracle_mod, hgs)
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    twin = hf.FlowProblem.from_hypergraph(hgs[0])
    try:
        _say(f"union schedule, {len(hgs)} block-pair problems")
        with hf.FlowBatch(probs, with_cut=True, schedule=1) as b:
            flows = b.run(with_cut=True)
            assert list(flows) == [r.flow for r in refs]
            _check_sides(b, hgs, refs, "union block pairs")
            # pierce problem 0 (and its twin) on the source side
            probs[0].solve()
            twin.solve()
            vs, _ = probs[0].source_side()
            outside = np.nonzero(vs == 0)[0]
            v = int(outside[outside != hgs[0].sinks[0]][0])
            probs[0].pierce(0, [v])
            twin.pierce(0, [v])
            f_twin = twin.solve()
            twin_vs, twin_ns = twin.source_side()
            flows = b.run(with_cut=True)
            assert flows[0] == f_twin
            vs0, ns0 = b.sides(0)
            assert (vs0 == twin_vs).all() and (ns0 == twin_ns).all()
            assert list(flows[1:]) == [r.flow for r in refs[1:]]
    finally:
        twin.close()
        for p in probs:
            p.close()


def test_batch_errors(hf):
    hgs = uneven_set(3, seed0=500)
    probs = [hf.FlowProblem.from_hypergraph(h, round_budget=1) for h in hgs]
    try:
        with pytest.raises(hf.HyperflowError) as ei:
            hf.flow_batch_solve([probs[0].handle, probs[0].handle])
        assert ei.value.name == "FP_ERR_INVALID"
        with pytest.raises(hf.HyperflowError) as ei:
            hf.FlowBatch(probs, reserved0=512)
        assert ei.value.name == "FP_ERR_INVALID"
        with pytest.raises(hf.HyperflowError) as ei:
            hf.FlowBatch(probs, streams=65)
        assert ei.value.name == "FP_ERR_INVALID"
        with pytest.raises(hf.HyperflowError) as ei:
            hf.FlowBatch(probs, schedule=4)
        assert ei.value.name == "FP_ERR_INVALID"
        with pytest.raises(hf.HyperflowError) as ei:
            hf.FlowBatch(probs, schedule=3, wg_threads=512)
        assert ei.value.name == "FP_ERR_INVALID"
        with pytest.raises(hf.HyperflowError) as ei:
            hf.FlowBatch(probs, schedule=1, union_pins=-1)
        assert ei.value.name == "FP_ERR_INVALID"
        with hf.FlowBatch(probs) as b:
            with pytest.raises(hf.HyperflowError) as ei:
                b.run(with_cut=True)  # planned without side buffers
            assert ei.value.name == "FP_ERR_INVALID"
        with hf.FlowBatch(probs, schedule=2) as b:  # per-problem round budgets
            with pytest.raises(hf.HyperflowError) as ei:
                b.run()
            assert ei.value.name == "FP_ERR_ABORTED"
        assert len(hf.flow_batch_solve([])) == 0
    finally:
        for p in probs:
            p.close()


def _cut_weight(hg, side):
    off = hg.net_offsets.astype(np.int64)
    sizes = np.diff(off)
    inside = side[hg.pins].astype(np.int64)
    net_of = np.repeat(np.arange(hg.num_nets), sizes)
    cnt = np.bincount(net_of, weights=inside, minlength=hg.num_nets)
    cut = (cnt > 0) & (cnt < sizes)
    return int(hg.net_weights[cut].sum())


@pytest.mark.slow
def test_batch_full_block_pairs_vs_oracle(hf, oracle_mod):
    """The 2M-vertex, 10M-pin, k=64 instance as the benchmark runs it: all
    500 problems in one union plan with the cut, then in one persistent
    launch with a workgroup per problem, every problem's flow value,
    vertex side and net side compared with the oracle (run on a process
    pool), and every side a minimum cut certificate (cut weight = flow <=
    cut before)."""
    import torch
    _say("building the 10M-pin block-pair set")
    bp = inputs.block_pair_problems(0)
    hgs = bp.problems
    _say(f"{len(hgs)} problems, oracle on a process pool")
    refs = oracle_mod.maxflow_many(hgs)
    _say("creating on the device")
    probs = [hf.FlowProblem.from_hypergraph(h, device=True) for h in hgs]
    try:
        # the union, and the workgroups schedule as the tuner keeps it here
        for cfg in (dict(schedule=1, group_lanes=8, gr_interval=8),
                    dict(schedule=3, group_lanes=4, gr_interval=8)):
            with hf.FlowBatch(probs, with_cut=True, **cfg) as b:
                _say(f"solve + cut, {cfg}")
                flows = b.run(with_cut=True)
                torch.cuda.synchronize()
                for i, (h, (F, rvs, rns)) in enumerate(zip(hgs, refs)):
                    vs, ns = b.sides(i)
                    assert flows[i] == F, f"{cfg} problem {i}: flow {flows[i]} != oracle {F}"
                    assert (vs.astype(bool) == rvs.astype(bool)).all(), \
                        f"{cfg} problem {i}: vertex side"
                    assert (ns == rns).all(), f"{cfg} problem {i}: net side"
                    assert _cut_weight(h, vs) == flows[i], f"{cfg} problem {i}"
                    assert 0 <= flows[i] <= h.meta["cut_before"]
    finally:
        for p in probs:
            p.close()
