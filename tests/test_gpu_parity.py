"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Integer method: flow values and the minimal source side (vertex bitmap and
per-net bits) must match bit-exactly.  The minimal minimum cut is unique
(min cuts form a lattice), so every schedule must produce the same bits.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2201_01556_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_01556_amd import hyperflow
    hyperflow.load_library()
    return hyperflow


def gpu_solve(hf, hg, **opts):
    with hf.FlowProblem.from_hypergraph(hg, **opts) as p:
        F = p.solve()
        vs, ns = p.source_side()
        st = p.stats()
    return F, vs.astype(bool), ns, st


def assert_same(hg, oracle_res, F, vs, ns, tag=""):
    assert F == oracle_res.flow, f"{tag}: flow {F} != oracle {oracle_res.flow}"
    bad = np.nonzero(vs != oracle_res.vertex_side.astype(bool))[0]
    assert bad.size == 0, f"{tag}: {bad.size} vertex sides differ, first {bad[:10]}"
    badn = np.nonzero(ns != oracle_res.net_side)[0]
    assert badn.size == 0, f"{tag}: {badn.size} net sides differ, first {badn[:10]}"


def _fixtures():
    with open(os.path.join(HERE, "golden", "fixtures.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _fixtures(), ids=lambda c: c["name"])
def test_fixtures(hf, case):
    _say(f"fixture {case['name']}")
    hg = inputs.hypergraph_from_nets(case["V"], case["nets"], case["w"], case["S"], case["T"])
    F, vs, ns, _ = gpu_solve(hf, hg, debug_checks=1)
    x = np.zeros(case["V"], dtype=bool)
    x[case["x"]] = True
    assert F == case["F"]
    assert (vs == x).all()
    assert list(ns) == case["net_side"]


@pytest.mark.parametrize("block", range(3))
def test_tiny_vs_oracle(hf, oracle_mod, block):
    for seed in range(block * 100, block * 100 + 100):
        hg = inputs.tiny_hypergraph(seed)
        _say(f"tiny seed {seed}")
        r = oracle_mod.maxflow(hg)
        F, vs, ns, _ = gpu_solve(hf, hg, debug_checks=1 if seed % 4 == 0 else 0)
        assert_same(hg, r, F, vs, ns, f"tiny {seed}")


@pytest.mark.parametrize("block", range(4))
def test_uniform_vs_oracle(hf, oracle_mod, block):
    """2,000 vertices, 3,000 nets of size U{2..8}, weights U{1..4}."""
    for seed in range(block * 25, block * 25 + 25):
        hg = inputs.uniform_hypergraph(seed)
        _say(f"uniform seed {seed}")
        r = oracle_mod.maxflow(hg)
        F, vs, ns, _ = gpu_solve(hf, hg)
        assert_same(hg, r, F, vs, ns, f"uniform {seed}")


def test_debug_invariants_every_round(hf, oracle_mod):
    """Preflow feasibility and label validity after every round, on the
    device-wide path (debug mode runs every round device-wide)."""
    for seed in range(3):
        hg = inputs.uniform_hypergraph(seed)
        _say(f"debug uniform seed {seed}")
        r = oracle_mod.maxflow(hg)
        F, vs, ns, st = gpu_solve(hf, hg, debug_checks=1)
        assert_same(hg, r, F, vs, ns, f"debug {seed}")
        assert st["restarts"] == 0
    hg = inputs.zipf_hypergraph(3, num_vertices=20000, num_nets=40000, size_hi=300)
    _say("debug zipf 20k")
    r = oracle_mod.maxflow(hg)
    F, vs, ns, _ = gpu_solve(hf, hg, debug_checks=1)
    assert_same(hg, r, F, vs, ns, "debug zipf")
    # the blocking variant of the round keeps every label valid as well
    F, vs, ns, st = gpu_solve(hf, hg, debug_checks=1, relabel_blocking=1)
    assert_same(hg, r, F, vs, ns, "debug zipf blocking")
    assert st["restarts"] == 0


@pytest.mark.parametrize("opts", [
    dict(group_lanes=4), dict(group_lanes=8), dict(group_lanes=16), dict(tail_threshold=1),
    dict(tail_threshold=1 << 30), dict(relabel_factor_x16=1), dict(relabel_factor_x16=256),
    dict(big_degree=2), dict(big_degree=100000), dict(bfs_arc_parallel=1),
    dict(bottom_up_min=-1), dict(bottom_up_min=1), dict(gr_interval=-1, stale_rounds=-1),
    dict(gr_interval=1), dict(pull_min=1), dict(pull_min=1, tail_threshold=1),
    dict(pull_min=5000), dict(tail_gr_interval=-1), dict(tail_gr_interval=1),
    dict(tail_gr_interval=1000, tail_threshold=1 << 30),
    dict(bfs_flat=-1), dict(bfs_marks=-1), dict(bfs_flat=-1, bfs_marks=-1),
    dict(bfs_flat=-1, bottom_up_min=1, tail_threshold=1),
    dict(bfs_marks=-1, bottom_up_min=1, tail_threshold=1), dict(bfs_flat=1, big_degree=2),
    dict(relabel_blocking=1), dict(relabel_blocking=1, tail_threshold=1),
    dict(relabel_blocking=1, gr_interval=-1, stale_rounds=-1),
    dict(bfs_xcd=2), dict(bfs_xcd=2, bottom_up_min=1, tail_threshold=1),
    dict(bfs_xcd=2, bottom_up_min=1, big_degree=2), dict(bfs_xcd=-1),
], ids=str)
def test_schedule_invariance(hf, oracle_mod, opts):
    """Every tuning knob changes only the schedule, never the result."""
    for hg in (inputs.uniform_hypergraph(11),
               inputs.zipf_hypergraph(4, num_vertices=30000, num_nets=60000, size_hi=500)):
        _say(f"schedule {opts} V={hg.num_vertices}")
        r = oracle_mod.maxflow(hg)
        F, vs, ns, _ = gpu_solve(hf, hg, **opts)
        assert_same(hg, r, F, vs, ns, str(opts))


@pytest.mark.parametrize("opts", [dict(), dict(pull_min=1, tail_threshold=1),
                                  dict(bottom_up_min=1, tail_threshold=1),
                                  dict(bottom_up_min=1, tail_threshold=1, bfs_marks=-1),
                                  dict(bottom_up_min=-1, tail_threshold=1),
                                  dict(bfs_flat=-1, bfs_marks=-1, tail_threshold=1),
                                  dict(relabel_blocking=1),
                                  dict(bfs_xcd=2, bottom_up_min=1, tail_threshold=1),
                                  dict(bfs_xcd=2, bottom_up_min=1, tail_threshold=1,
                                       bfs_marks=1)], ids=str)
def test_labels_and_preflow_certificate(hf, oracle_mod, opts):
    """After the solve the labels are exact residual distances of the final
    state (the terminating global relabel), the state is a feasible preflow
    of the capped network, and the cut weight equals the flow value; with
    every multi-kernel BFS level pulled bottom-up or expanded as well."""
    hg = inputs.zipf_hypergraph(6, num_vertices=20000, num_nets=40000, size_hi=200)
    _say(f"labels / certificate {opts}")
    with hf.FlowProblem.from_hypergraph(hg, **opts) as p:
        F = p.solve()
        vs, ns = p.source_side()
        s = p.export_state(hg.num_pins)
    errs = oracle_mod.check_preflow(hg, s["f_in"], s["f_out"], s["f_b"], F)
    assert not errs, errs
    V, E = hg.num_vertices, hg.num_nets
    NB = (V + 1) & ~1
    N = NB + 2 * E
    dv, din, dout = oracle_mod.residual_labels(hg, s["f_in"], s["f_out"], s["f_b"])
    lab = s["labels"].astype(np.int64)
    exp_v = np.where(dv == -1, N, np.where(dv == -2, N + 1, dv))
    assert (lab[:V] == exp_v).all()
    assert (lab[V::2] == np.where(din == -1, N, din)).all()
    assert (lab[V + 1::2] == np.where(dout == -1, N, dout)).all()
    assert oracle_mod.cut_weight(hg, vs.astype(bool)) == F


def test_device_memory_inputs_and_outputs(hf, oracle_mod):
    import torch
    hg = inputs.uniform_hypergraph(42)
    _say("device memory")
    r = oracle_mod.maxflow(hg)
    with hf.FlowProblem.from_hypergraph(hg, device=True) as p:
        F = p.solve()
        vs = torch.zeros(hg.num_vertices, dtype=torch.uint8, device="cuda")
        ns = torch.zeros(hg.num_nets, dtype=torch.uint8, device="cuda")
        p.source_side(vs, ns)
        torch.cuda.synchronize()
        assert_same(hg, r, F, vs.cpu().numpy().astype(bool), ns.cpu().numpy(), "device")


def test_zipf_medium_vs_oracle(hf, oracle_mod):
    for seed in range(2):
        hg = inputs.zipf_hypergraph(seed, num_vertices=100_000, num_nets=200_000, size_hi=1000)
        _say(f"zipf 100k seed {seed}")
        r = oracle_mod.maxflow(hg)
        F, vs, ns, _ = gpu_solve(hf, hg)
        assert_same(hg, r, F, vs, ns, f"zipf100k {seed}")


@pytest.mark.parametrize("seed", range(3))
def test_zipf_full_size_vs_oracle(hf, oracle_mod, seed):
    """1M vertices, 2M nets, Zipf(2.2) sizes clamped to [2, 1000], unit
    weights, 1 % hash-selected sources and sinks: full comparison."""
    _say(f"zipf 1M seed {seed}: generating")
    hg = inputs.zipf_hypergraph(seed)
    _say(f"zipf 1M seed {seed}: oracle")
    r = oracle_mod.maxflow(hg)
    _say(f"zipf 1M seed {seed}: gpu")
    F, vs, ns, st = gpu_solve(hf, hg)
    _say(f"zipf 1M seed {seed}: F={F} stats={st}")
    assert_same(hg, r, F, vs, ns, f"zipf1M {seed}")


def test_edge_cases(hf, oracle_mod):
    cases = {
        "no nets": inputs.hypergraph_from_nets(4, [], [], [0], [3]),
        "only single-pin nets": inputs.hypergraph_from_nets(4, [[0], [1], [2], [3]],
                                                            [1, 2, 3, 4], [0], [3]),
        "empty nets everywhere": inputs.hypergraph_from_nets(
            5, [[], [0, 1], [], [1, 4], []], [3, 1, 3, 2, 3], [0], [4]),
        "odd vertex count": inputs.hypergraph_from_nets(3, [[0, 1, 2]], [5], [0], [2]),
        "weights near the guard": inputs.hypergraph_from_nets(
            4, [[0, 1], [1, 3], [0, 2], [2, 3]], [2**29, 2**29, 2**29, 2**29 - 1], [0], [3]),
        "hub vertex": inputs.hypergraph_from_nets(
            40, [[0, v, 39] if v % 3 == 0 else [v, 20] for v in range(1, 39) if v != 20]
            + [[20, 39]], list(range(1, 39)), [0], [39]),
        "one net with all vertices": inputs.hypergraph_from_nets(
            300, [list(range(300))] + [[i, i + 1] for i in range(299)],
            [7] + [1] * 299, [0, 1, 2], [297, 298, 299]),
        "sources everywhere": inputs.hypergraph_from_nets(
            6, [[0, 1, 2], [2, 3], [3, 4, 5]], [1, 2, 1], [0, 1, 2, 3], [5]),
    }
    for name, hg in cases.items():
        _say(f"edge case {name}")
        r = oracle_mod.maxflow(hg)
        F, vs, ns, _ = gpu_solve(hf, hg, debug_checks=1)
        assert_same(hg, r, F, vs, ns, name)


def test_error_paths(hf):
    _say("error paths")
    bad = [
        ("pin out of range", inputs.hypergraph_from_nets(3, [[0, 5]], [1], [0], [2])),
        ("zero weight", inputs.hypergraph_from_nets(3, [[0, 1]], [0], [0], [2])),
        ("duplicate pin", inputs.hypergraph_from_nets(3, [[0, 1, 1]], [1], [0], [2])),
        ("S and T overlap", inputs.hypergraph_from_nets(3, [[0, 1]], [1], [0, 1], [1, 2])),
        ("terminal out of range", inputs.hypergraph_from_nets(3, [[0, 1]], [1], [0], [7])),
    ]
    for name, hg in bad:
        with pytest.raises(hf.HyperflowError) as ei:
            hf.FlowProblem.from_hypergraph(hg)
        assert ei.value.name == "FP_ERR_INVALID", name
    hg = inputs.hypergraph_from_nets(3, [[0, 1], [1, 2]], [2**30, 2**30], [0], [2])
    with pytest.raises(hf.HyperflowError) as ei:
        hf.FlowProblem.from_hypergraph(hg)
    assert ei.value.name == "FP_ERR_OVERFLOW"
    off = np.array([0, 2, 1, 3], dtype=np.int32)
    with pytest.raises(hf.HyperflowError) as ei:
        hf.FlowProblem(3, off, np.array([0, 1, 2], np.int32), np.ones(3, np.int32),
                       np.array([0], np.int32), np.array([2], np.int32))
    assert ei.value.name == "FP_ERR_INVALID"
    # cut before solve
    hg = inputs.uniform_hypergraph(1)
    with hf.FlowProblem.from_hypergraph(hg) as p:
        with pytest.raises(hf.HyperflowError) as ei:
            p.source_side()
        assert ei.value.name == "FP_ERR_STATE"


def test_round_budget_abort_then_resume(hf, oracle_mod):
    hg = inputs.zipf_hypergraph(2, num_vertices=20000, num_nets=40000, size_hi=200)
    _say("round budget")
    r = oracle_mod.maxflow(hg)
    with hf.FlowProblem.from_hypergraph(hg, round_budget=2, tail_threshold=1) as p:
        with pytest.raises(hf.HyperflowError) as ei:
            p.solve()
        assert ei.value.name == "FP_ERR_ABORTED"
    # a generous budget finishes
    F, vs, ns, _ = gpu_solve(hf, hg, round_budget=1 << 30)
    assert_same(hg, r, F, vs, ns, "budget")
