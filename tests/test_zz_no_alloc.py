"""GPU test of maxflow_mincut_noalloc, the entry point that allocates
nothing (its device state lives in the library's fixed scratch array),
through the C ABI: its flow value, vertex side and net side must equal
those of the allocating sequence flow_problem_create -> maxflow_solve ->
mincut_source_side bit-exactly, on calls in a row whose later inputs are
smaller (so state a call leaves behind must not leak into the next one).
"""
import sys

import numpy as np
import pytest

from paper_2201_01556_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_01556_amd import hyperflow
    hyperflow.load_library()
    return hyperflow


def _allocating(hf, hg):
    with hf.FlowProblem.from_hypergraph(hg) as p:
        F = p.solve()
        vs, ns = p.source_side()
    return F, vs, ns


def _cases():
    return [inputs.uniform_hypergraph(0),  # 2,000 vertices, 3,000 nets
            inputs.uniform_hypergraph(1, num_vertices=500, num_nets=700, num_sources=20,
                                      num_sinks=20),
            inputs.zipf_hypergraph(2, num_vertices=20000, num_nets=40000, size_hi=300),
            inputs.tiny_hypergraph(3)]


def test_noalloc_host_memory_matches_create_solve_cut(hf, oracle_mod):
    hgs = _cases()
    # larger, smaller, larger, smallest: each call follows a different size
    for i in (0, 1, 2, 3, 0):
        hg = hgs[i]
        _say(f"host call on case {i}: V={hg.num_vertices} pins={hg.num_pins}")
        F0, vs0, ns0 = _allocating(hf, hg)
        F, vs, ns = hf.maxflow_mincut_noalloc(hg.num_vertices, hg.net_offsets, hg.pins,
                                              hg.net_weights, hg.sources, hg.sinks)
        assert F == F0
        assert (vs == vs0).all() and (ns == ns0).all()
        r = oracle_mod.maxflow(hg)
        assert F == r.flow and (vs.astype(bool) == r.vertex_side.astype(bool)).all()


def test_noalloc_device_memory_two_calls(hf):
    import torch
    for i in (2, 1):  # the second call's input is smaller
        hg = _cases()[i]
        _say(f"device call on case {i}")
        F0, vs0, ns0 = _allocating(hf, hg)
        arr = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
               for a in (hg.net_offsets, hg.pins, hg.net_weights, hg.sources, hg.sinks)]
        vs = torch.full((hg.num_vertices,), 7, dtype=torch.uint8, device="cuda")
        ns = torch.full((hg.num_nets,), 7, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        F, _, _ = hf.maxflow_mincut_noalloc(hg.num_vertices, *arr, vertex_side=vs, net_side=ns)
        torch.cuda.synchronize()
        assert F == F0
        assert (vs.cpu().numpy() == vs0).all() and (ns.cpu().numpy() == ns0).all()


def test_noalloc_rejects_oversized_problem(hf):
    """A problem that needs more than the scratch array holds is rejected
    with FP_ERR_OVERFLOW and a message naming both sizes; the next call
    still works."""
    big = inputs.zipf_hypergraph(0, 200_000, 400_000, size_hi=200)
    _say(f"oversized: pins={big.num_pins}")
    with pytest.raises(hf.HyperflowError) as ei:
        hf.maxflow_mincut_noalloc(big.num_vertices, big.net_offsets, big.pins, big.net_weights,
                                  big.sources, big.sinks)
    assert ei.value.name == "FP_ERR_OVERFLOW"
    assert "bytes of device scratch" in str(ei.value)
    hg = _cases()[1]
    F0, vs0, ns0 = _allocating(hf, hg)
    F, vs, ns = hf.maxflow_mincut_noalloc(hg.num_vertices, hg.net_offsets, hg.pins,
                                          hg.net_weights, hg.sources, hg.sinks)
    assert F == F0 and (vs == vs0).all() and (ns == ns0).all()


def test_noalloc_invalid_input(hf):
    hg = _cases()[1]
    bad = hg.pins.copy()
    bad[0] = hg.num_vertices  # pin id out of range
    with pytest.raises(hf.HyperflowError) as ei:
        hf.maxflow_mincut_noalloc(hg.num_vertices, hg.net_offsets, bad, hg.net_weights,
                                  hg.sources, hg.sinks)
    assert ei.value.name == "FP_ERR_INVALID"
    F0, vs0, ns0 = _allocating(hf, hg)
    F, vs, ns = hf.maxflow_mincut_noalloc(hg.num_vertices, hg.net_offsets, hg.pins,
                                          hg.net_weights, hg.sources, hg.sinks)
    assert F == F0 and (vs == vs0).all() and (ns == ns0).all()
