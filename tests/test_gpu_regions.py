"""GPU parity of the device region builder (flow_regions_build) against the
oracle of the section "Network Construction" (``oracle/regions.py``), and
of its problems' flows against the max-flow oracle.  Bit-exact: every
array of every pair (offsets, pins, weights, vertex weights, vertex and net
ids) and every fact."""
import numpy as np
import pytest

from paper_2201_01556_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-regions] {msg}", flush=True)


@pytest.fixture(scope="module")
def hf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_01556_amd import hyperflow
    hyperflow.load_library()
    return hyperflow


@pytest.fixture(scope="module")
def oreg():
    from oracle import regions
    return regions


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


def _instance(seed, V, k, target, size_hi, vw_hi=3, w_hi=3, shuffle=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = inputs.zipf_sizes_until(rng, target, 2.2, size_hi)
    pins = inputs._distinct_pins(rng, V, sizes).astype(np.int32)
    E = int(sizes.shape[0])
    off = np.zeros(E + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    if shuffle:
        for e in range(E):
            rng.shuffle(pins[off[e]:off[e + 1]])
    w = rng.integers(1, w_hi + 1, E).astype(np.int32)
    cv = rng.integers(1, vw_hi + 1, V).astype(np.int32)
    block = rng.integers(0, k, V).astype(np.int32)
    hg = inputs.Hypergraph(V, off.astype(np.int32), pins, w, cv, np.zeros(0, np.int32),
                           np.zeros(0, np.int32), {})
    return hg, block


def _heaviest_pairs(hg, block, k, count):
    """Block pairs by cut weight (descending, then ids); vectorised count."""
    E = hg.num_nets
    net = np.repeat(np.arange(E), np.diff(hg.net_offsets))
    bm = np.zeros(E, dtype=np.uint64)
    np.bitwise_or.at(bm, net, (np.uint64(1) << block[hg.pins].astype(np.uint64)))
    cuts = {}
    w = hg.net_weights
    for a in range(k):
        for b in range(a + 1, k):
            m = ((bm >> np.uint64(a)) & np.uint64(1)).astype(bool) & \
                ((bm >> np.uint64(b)) & np.uint64(1)).astype(bool)
            c = int(w[m].sum())
            if c:
                cuts[(a, b)] = c
    order = sorted(cuts, key=lambda p: (-cuts[p], p))[:count]
    return order, [cuts[p] for p in order]


def _compare(oreg, hg, block, regions, pairs, caps, merge, vnets=None, sample=None):
    if vnets is None:
        vnets = oreg.vertex_nets(hg)
    idx = range(len(pairs)) if sample is None else sample
    for q in idx:
        i, j = pairs[q]
        r = oreg.build_region(hg, block, hg.vertex_weights, i, j, int(caps[q][0]),
                              int(caps[q][1]), remove_identical=merge, vnets=vnets)
        g = regions.export(q)
        inf = g["info"]
        tag = f"pair {q} ({i},{j}) merge={merge}"
        assert inf["n"] == r["n"], tag
        assert inf["num_nets"] == len(r["net_offsets"]) - 1, tag
        assert inf["num_pins"] == len(r["pins"]), tag
        assert (g["vertex_ids"] == r["gid"]).all(), tag
        assert (g["vertex_weights"] == r["vw"]).all(), tag
        assert (g["net_offsets"] == r["net_offsets"]).all(), tag
        assert (g["pins"] == r["pins"]).all(), tag
        assert (g["net_weights"] == r["net_weights"]).all(), tag
        assert (g["net_ids"] == r["net_gid"]).all(), tag
        assert inf["cut_before"] == r["cut_before"], tag
        assert inf["boundary"] == r["boundary"], tag
        assert (inf["weight_i"], inf["weight_j"]) == tuple(r["side_weights"]), tag
        bins = [inf[k] for k in ("bin_2", "bin_4", "bin_8", "bin_16", "bin_64", "bin_256",
                                 "bin_more")]
        assert bins == r["bins"], tag


@pytest.mark.parametrize("merge", [False, True])
@pytest.mark.parametrize("seed,shuffle", [(0, False), (1, True)])
def test_regions_vs_oracle(hf, oreg, seed, shuffle, merge):
    """30,000 vertices, k = 8, Zipf sizes up to 200, vertex and net weights
    U{1..3}; the 12 heaviest pairs; pins in input order sorted or shuffled
    (the builder sorts them)."""
    hg, block = _instance(seed, 30_000, 8, 150_000, 200, shuffle=shuffle)
    pairs, cuts = _heaviest_pairs(hg, block, 8, 12)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=8).astype(np.int64)
    caps = inputs.region_caps(bw, pairs, cuts)
    _say(f"seed {seed} shuffle={shuffle} merge={merge}: {len(pairs)} pairs")
    with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                        hg.vertex_weights, block, 8, pairs, caps, merge_identical=merge) as rg:
        _compare(oreg, hg, block, rg, pairs, caps, merge)


def test_region_caps_and_small_blocks(hf, oreg):
    """Caps of 0, tight caps and unbounded caps (each side stops one vertex
    short of its block), k = 3 with uneven blocks."""
    hg, block = _instance(4, 3000, 3, 12_000, 40)
    block[:2500] = 0
    pairs = [(0, 1), (1, 2), (2, 0), (0, 2)]
    caps = np.array([[0, 0], [7, 3], [10 ** 12, 10 ** 12], [50, 10 ** 12]], dtype=np.int64)
    for merge in (False, True):
        with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                            hg.vertex_weights, block, 3, pairs, caps,
                            merge_identical=merge) as rg:
            _compare(oreg, hg, block, rg, pairs, caps, merge)
            assert rg.info(0)["n"] == 0


def test_region_problems_solve(hf, oreg, oracle_mod):
    """Problems created from the device copy: flows and minimal source sides
    equal the oracle's on the exported problems, merged or not."""
    hg, block = _instance(2, 20_000, 6, 90_000, 100)
    pairs, cuts = _heaviest_pairs(hg, block, 6, 8)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=6).astype(np.int64)
    caps = inputs.region_caps(bw, pairs, cuts)
    flows = {}
    for merge in (False, True):
        with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                            hg.vertex_weights, block, 6, pairs, caps,
                            merge_identical=merge) as rg:
            for q in range(len(pairs)):
                g = rg.export(q)
                n = g["info"]["n"]
                h = inputs.Hypergraph(n + 2, g["net_offsets"], g["pins"], g["net_weights"],
                                      g["vertex_weights"], np.array([n], np.int32),
                                      np.array([n + 1], np.int32), {})
                ref = oracle_mod.maxflow(h)
                with rg.problem(q) as p:
                    F = p.solve()
                    vs, _ = p.source_side()
                assert F == ref.flow, (q, merge)
                assert (vs.astype(bool) == ref.vertex_side.astype(bool)).all(), (q, merge)
                flows.setdefault(q, set()).add(F)
    assert all(len(v) == 1 for v in flows.values())  # merging changes no flow


def test_regions_device_inputs(hf):
    import torch
    hg, block = _instance(3, 20_000, 5, 80_000, 60)
    pairs, cuts = _heaviest_pairs(hg, block, 5, 6)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=5).astype(np.int64)
    caps = inputs.region_caps(bw, pairs, cuts)
    host = hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                          hg.vertex_weights, block, 5, pairs, caps)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
           for a in (hg.net_offsets, hg.pins, hg.net_weights, hg.vertex_weights, block)]
    torch.cuda.synchronize()
    with host, hf.FlowRegions(hg.num_vertices, *dev, 5, pairs, caps) as d:
        for q in range(len(pairs)):
            a, b = host.export(q), d.export(q)
            for key in ("net_offsets", "pins", "net_weights", "vertex_weights", "vertex_ids",
                        "net_ids"):
                assert (a[key] == b[key]).all(), (q, key)
            assert a["info"] == b["info"]


def test_regions_errors(hf):
    hg, block = _instance(6, 500, 4, 2000, 10)
    args = (hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights, hg.vertex_weights)
    caps = np.array([[5, 5]], dtype=np.int64)

    def expect(name, *a, **kw):
        with pytest.raises(hf.HyperflowError) as ei:
            hf.flow_regions_build(*a, **kw)
        assert ei.value.name == name

    expect("FP_ERR_INVALID", *args, block, 1, [(0, 1)], caps)
    expect("FP_ERR_INVALID", *args, block, 65, [(0, 1)], caps)
    expect("FP_ERR_INVALID", *args, block, 4, [(1, 1)], caps)
    expect("FP_ERR_INVALID", *args, block, 4, [(0, 4)], caps)
    expect("FP_ERR_INVALID", *args, block, 4, [(0, 1)], np.array([[-1, 5]]))
    bad = block.copy()
    bad[7] = 4
    expect("FP_ERR_INVALID", *args, bad, 4, [(0, 1)], caps)
    cw = hg.vertex_weights.copy()
    cw[3] = 0
    expect("FP_ERR_INVALID", hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights, cw,
           block, 4, [(0, 1)], caps)
    pins = hg.pins.copy()
    pins[0] = hg.num_vertices
    expect("FP_ERR_INVALID", hg.num_vertices, hg.net_offsets, pins, hg.net_weights,
           hg.vertex_weights, block, 4, [(0, 1)], caps)
    with hf.FlowRegions(*args, block, 4, np.zeros((0, 2), np.int32),
                        np.zeros((0, 2), np.int64)) as rg:
        assert rg.count == 0
        with pytest.raises(hf.HyperflowError):
            rg.info(0)


def test_regions_full_block_pairs(hf, oreg):
    """The 500 block pairs of the 2M-vertex workload (10M pins, k = 64, three
    label-propagation sweeps): without merging, every problem equals the
    host builder's (input generation) array for array; with merging, the
    union batch gives every problem the same flow; one pair is compared
    with the oracle both ways."""
    import torch
    _say("full block pairs: generating")
    bp = inputs.block_pair_problems(0, threads=0)
    hg = bp.hypergraph
    pairs = [p.meta["pair"] for p in bp.problems]
    cuts = [p.meta["cut"] for p in bp.problems]
    caps = inputs.region_caps(bp.block_weights, pairs, cuts)
    _say(f"full block pairs: {len(pairs)} pairs, building on the device")
    with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                        hg.vertex_weights, bp.block, 64, pairs, caps,
                        merge_identical=False) as rg:
        for q, p in enumerate(bp.problems):
            g = rg.export(q)
            assert g["info"]["num_vertices"] == p.num_vertices, q
            assert (g["net_offsets"] == p.net_offsets).all(), q
            assert (g["pins"] == p.pins).all(), q
            assert (g["net_weights"] == p.net_weights).all(), q
            assert (g["vertex_weights"] == p.vertex_weights).all(), q
            assert (g["vertex_ids"] == p.meta["gid"]).all(), q
            assert g["info"]["cut_before"] == p.meta["cut_before"], q
        # the learned scorer's features from the device statistics
        assert (rg.features(cuts, bp.block_weights) == inputs.scorer_features(bp.problems)).all()
    _say("full block pairs: unmerged equal to the host builder; merged flows")
    plain = [hf.FlowProblem.from_hypergraph(h, device=True) for h in bp.problems]
    try:
        with hf.FlowBatch(plain) as plan:
            f_plain = plan.run()
    finally:
        for p in plain:
            p.close()
    with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                        hg.vertex_weights, bp.block, 64, pairs, caps,
                        merge_identical=True) as rg:
        merged = [rg.problem(q) for q in range(len(pairs))]
        torch.cuda.synchronize()
        try:
            with hf.FlowBatch(merged) as plan:
                f_merged = plan.run()
        finally:
            for p in merged:
                p.close()
        assert list(f_merged) == list(f_plain)
        nets_removed = sum(rg.info(q)["merged"] for q in range(len(pairs)))
        _say(f"full block pairs: {nets_removed} identical nets merged; oracle on one pair")
        vnets = oreg.vertex_nets(hg)
        _compare(oreg, hg, bp.block, rg, pairs, caps, True, vnets=vnets, sample=[len(pairs) - 1])


def test_regions_solve_union(hf, oracle_mod):
    """flow_regions_solve (union networks built from the regions, no handle
    per pair): flows and minimal source sides equal the oracle's on the
    exported problems and the per-handle batch's; skipped pairs report -1
    and keep nothing; a solve before another keeps the latest sides."""
    import torch
    hg, block = _instance(8, 20_000, 6, 90_000, 100)
    pairs, cuts = _heaviest_pairs(hg, block, 6, 10)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=6).astype(np.int64)
    caps = inputs.region_caps(bw, pairs, cuts)
    with hf.FlowRegions(hg.num_vertices, hg.net_offsets, hg.pins, hg.net_weights,
                        hg.vertex_weights, block, 6, pairs, caps) as rg:
        with pytest.raises(hf.HyperflowError) as ei:
            rg.source_side(0)
        assert ei.value.name == "FP_ERR_STATE"
        skip = np.zeros(len(pairs), np.uint8)
        skip[::3] = 1
        f_skip = rg.solve(skip)
        assert all(f_skip[q] == -1 for q in range(len(pairs)) if skip[q])
        flows = rg.solve()
        probs = [rg.problem(q) for q in range(len(pairs))]
        try:
            with hf.FlowBatch(probs, with_cut=True) as plan:
                fb = plan.run(with_cut=True)
                torch.cuda.synchronize()
                for q in range(len(pairs)):
                    n = rg.info(q)["n"]
                    assert (rg.source_side(q) == plan.vertex_sides[q].cpu().numpy()[:n]).all()
        finally:
            for p in probs:
                p.close()
        assert list(flows) == list(fb)
        assert all(f_skip[q] == flows[q] for q in range(len(pairs)) if not skip[q])
        for q in range(len(pairs)):
            g = rg.export(q)
            n = g["info"]["n"]
            h = inputs.Hypergraph(n + 2, g["net_offsets"], g["pins"], g["net_weights"],
                                  g["vertex_weights"], np.array([n], np.int32),
                                  np.array([n + 1], np.int32), {})
            ref = oracle_mod.maxflow(h)
            assert flows[q] == ref.flow, q
            assert (rg.source_side(q).astype(bool) == ref.vertex_side[:n].astype(bool)).all(), q
