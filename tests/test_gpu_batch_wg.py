"""GPU parity of the workgroups batch schedule (schedule 3: one persistent
launch, each problem solved start to end inside one workgroup, replayed
from a captured HIP graph) against the CPU oracle: flow values and minimal
source sides (vertex and net bitmaps) of every problem, bit-exact."""
import sys

import numpy as np
import pytest

from paper_2201_01556_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batch-wg] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_01556_amd import hyperflow
    hyperflow.load_library()
    return hyperflow


def uneven_set(n, seed0=0):
    out = []
    for i in range(n):
        V = 200 + 300 * (i % 7)
        out.append(inputs.uniform_hypergraph(seed0 + i, num_vertices=V,
                                             num_nets=int(1.5 * V), num_sources=V // 20,
                                             num_sinks=V // 20))
    return out


def _check(batch, hgs, refs, flows, tag, skip=None):
    for i, (h, r) in enumerate(zip(hgs, refs)):
        if skip is not None and skip[i]:
            assert flows[i] == -1, f"{tag} problem {i}"
            continue
        assert flows[i] == r.flow, f"{tag} problem {i}"
        vs, ns = batch.sides(i)
        assert (vs.astype(bool) == r.vertex_side.astype(bool)).all(), f"{tag} problem {i}"
        assert (ns == r.net_side).all(), f"{tag} problem {i}"


@pytest.mark.parametrize("lanes,gr,threads", [(8, 0, 0), (4, -1, 256), (16, 8, 1024),
                                               (8, 1, 1024), (4, 0, 1024)])
def test_workgroups_vs_oracle(hf, oracle_mod, lanes, gr, threads):
    """24 uneven uniform problems (200..2,000 vertices): flows and sides equal
    the oracle's; skipped problems report -1."""
    hgs = uneven_set(24, seed0=800)
    refs = [oracle_mod.maxflow(h) for h in hgs]
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        _say(f"workgroups lanes={lanes} gr={gr} threads={threads}")
        with hf.FlowBatch(probs, with_cut=True, schedule=3, group_lanes=lanes,
                          gr_interval=gr, wg_threads=threads) as b:
            flows = b.run(with_cut=True)
            _check(b, hgs, refs, flows, f"lanes={lanes} gr={gr}")
            skip = np.zeros(24, dtype=np.uint8)
            skip[[1, 7, 22]] = 1
            flows = b.run(skip=skip)
            for i in range(24):
                assert flows[i] == (-1 if skip[i] else refs[i].flow)
            assert list(b.run(skip=np.ones(24, dtype=np.uint8))) == [-1] * 24
    finally:
        for p in probs:
            p.close()


def test_workgroups_replays_and_handles(hf, oracle_mod):
    """Tiny adversarial problems, uniform ones and 2,000-vertex ones in one
    plan, run five times from the captured launch with other device work
    and host synchronisation in between; every replay equals the oracle.
    The solved handles then behave as after maxflow_solve (source side,
    warm re-solve)."""
    import torch
    hgs = [inputs.tiny_hypergraph(s) for s in range(40)] + uneven_set(12, seed0=900) + \
        [inputs.uniform_hypergraph(s) for s in range(4)]
    refs = [oracle_mod.maxflow(h) for h in hgs]
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        with hf.FlowBatch(probs, with_cut=True, schedule=3, wg_threads=1024) as b:
            for rep in range(5):
                _say(f"replay {rep}")
                for vs in b.vertex_sides:
                    vs.fill_(7)
                x = torch.randn(1 << 20, device="cuda")
                float((x * x).sum())
                flows = b.run(with_cut=True)
                torch.cuda.synchronize()
                _check(b, hgs, refs, flows, f"replay {rep}")
        for i in (0, 17, 45, len(hgs) - 1):
            vs, ns = probs[i].source_side()
            assert (vs.astype(bool) == refs[i].vertex_side.astype(bool)).all()
            assert (ns == refs[i].net_side).all()
            assert probs[i].solve() == refs[i].flow
    finally:
        for p in probs:
            p.close()


def test_workgroups_block_pairs_and_pierced(hf, oracle_mod):
    """Block-pair regions of a partitioned hypergraph (up to a few thousand
    pins each), then one problem pierced: the schedule takes each problem's
    current terminals and starts from the zero flow."""
    bp = inputs.block_pair_problems(0, num_vertices=20000, target_pins=100000, k=8,
                                    max_problems=30)
    hgs = bp.problems
    refs = [oracle_mod.maxflow(h) for h in hgs]
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    twin = hf.FlowProblem.from_hypergraph(hgs[0])
    try:
        _say(f"workgroups, {len(hgs)} block-pair problems")
        with hf.FlowBatch(probs, with_cut=True, schedule=3) as b:
            flows = b.run(with_cut=True)
            _check(b, hgs, refs, flows, "block pairs")
            vs, _ = probs[0].source_side()
            twin.solve()
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


def test_workgroups_in_tuner(hf, oracle_mod):
    """The tuner times the workgroups schedule beside the others; whatever it
    keeps gives the oracle's flows."""
    hgs = uneven_set(48, seed0=1000)
    refs = [oracle_mod.maxflow(h) for h in hgs]
    probs = [hf.FlowProblem.from_hypergraph(h) for h in hgs]
    try:
        with hf.FlowBatch(probs) as b:
            cfg = b.tune()
            _say(f"tuned: {cfg}")
            assert cfg["schedule"] in (1, 2, 3)
            assert list(b.run()) == [r.flow for r in refs]
    finally:
        for p in probs:
            p.close()
