"""Pins of the region-construction oracle (``oracle/regions.py``).

The oracle follows the paper's section "Network Construction" (paragraphs
"Region Growing", "Construction Algorithms", "Identical Net Removal").  It
is pinned to things other than itself:

* the host region builder of the input generators (``regions.c``, written
  separately in C with the same readings) must produce the same problems
  net for net when identical nets are kept;
* the cut identity that makes the construction correct: for every choice X
  of region vertices on the source side, the cut of the built problem plus
  the weight of the discarded nets holding both s and t plus the weight of
  the untouched nets cut between the two blocks equals the weight of the
  nets cut between (V_i - B_i) u X and (V_j - B_j) u (B - X) in the
  original hypergraph (pins of other blocks ignored) -- with and without
  merging identical nets;
* merging: no two nets left equal, weights conserved, every net's pins in
  increasing local id;
* growth: each side inside its block, within its cap, with a vertex of the
  block left outside, level 0 = the block's pins on the nets cut between
  the two blocks.
"""
import numpy as np
import pytest

from paper_2201_01556_amd import inputs
from oracle import regions as oreg


def _instance(seed, V=2400, k=6, target=9000, size_hi=30, vw_hi=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = inputs.zipf_sizes_until(rng, target, 2.2, size_hi)
    pins = inputs._distinct_pins(rng, V, sizes)
    E = int(sizes.shape[0])
    off = np.zeros(E + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    w = rng.integers(1, 4, E).astype(np.int32)
    cv = rng.integers(1, vw_hi + 1, V).astype(np.int32)
    block = rng.integers(0, k, V).astype(np.int32)
    hg = inputs.Hypergraph(V, off.astype(np.int32), pins.astype(np.int32), w, cv,
                           np.zeros(0, np.int32), np.zeros(0, np.int32), {})
    return hg, block


def _pair_cut(hg, block, i, j, side_i):
    """Weight of the nets with a pin on each side, where side_i marks the
    vertices of blocks i and j that are on the i side; other blocks'
    pins are ignored."""
    tot = 0
    for e in range(hg.num_nets):
        ps = hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]
        a = any(block[u] in (i, j) and side_i[u] for u in ps)
        b = any(block[u] in (i, j) and not side_i[u] for u in ps)
        if a and b:
            tot += int(hg.net_weights[e])
    return tot


def _problem_cut(r, x_local):
    """Cut of the built problem for source side X u {s} (x_local marks the
    region vertices in X)."""
    n = r["n"]
    src = np.zeros(n + 2, dtype=bool)
    src[:n] = x_local
    src[n] = True
    tot = 0
    off, pins = r["net_offsets"], r["pins"]
    for e in range(len(off) - 1):
        ps = pins[off[e]:off[e + 1]]
        if src[ps].any() and not src[ps].all():
            tot += int(r["net_weights"][e])
    return tot


def _discarded_st_and_untouched(hg, block, i, j, members):
    """(weight of nets touching the region that would hold both s and t,
    weight of nets not touching the region with pins in both blocks)."""
    inside = set(int(u) for u in members)
    st = un = 0
    for e in range(hg.num_nets):
        ps = [int(u) for u in hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]]
        touch = any(u in inside for u in ps)
        has_i = any(block[u] == i and u not in inside for u in ps)
        has_j = any(block[u] == j and u not in inside for u in ps)
        if touch and has_i and has_j:
            st += int(hg.net_weights[e])
        if not touch and any(block[u] == i for u in ps) and any(block[u] == j for u in ps):
            un += int(hg.net_weights[e])
    return st, un


def _pairs(hg, block, k, count):
    """The heaviest block pairs by cut weight (then by ids)."""
    cuts = {}
    for e in range(hg.num_nets):
        bs = sorted({int(block[u]) for u in hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]})
        for a in range(len(bs)):
            for b in range(a + 1, len(bs)):
                cuts[(bs[a], bs[b])] = cuts.get((bs[a], bs[b]), 0) + int(hg.net_weights[e])
    order = sorted(cuts, key=lambda p: (-cuts[p], p))[:count]
    return order, [cuts[p] for p in order]


@pytest.mark.parametrize("seed", [0, 1])
def test_regions_match_the_host_builder(seed):
    hg, block = _instance(seed)
    k = 6
    bps = inputs._pair_problems(hg, block.copy(), seed, k, 0, 0.03, 16, 1, 8, 1)
    vnets = oreg.vertex_nets(hg)
    assert len(bps.problems) >= 6
    for p in bps.problems:
        i, j = p.meta["pair"]
        cut = p.meta["cut"]
        caps = inputs.region_caps(bps.block_weights, [(i, j)], [cut])[0]
        r = oreg.build_region(hg, bps.block, hg.vertex_weights, i, j, int(caps[0]),
                              int(caps[1]), remove_identical=False, vnets=vnets)
        assert r["n"] + 2 == p.num_vertices
        assert (r["gid"] == p.meta["gid"]).all()
        assert (r["vw"] == p.vertex_weights).all()
        assert (r["net_offsets"] == p.net_offsets).all()
        assert (r["pins"] == p.pins).all()
        assert (r["net_weights"] == p.net_weights).all()
        assert r["cut_before"] == p.meta["cut_before"]
        assert r["boundary"] == p.meta["boundary"]
        assert tuple(r["side_weights"]) == tuple(p.meta["side_weights"])
        assert r["bins"] == [int(x) for x in p.meta["features"][3:10]]


@pytest.mark.parametrize("merge", [False, True])
def test_cut_identity(merge):
    hg, block = _instance(7, V=600, k=4, target=2400, size_hi=12)
    rng = np.random.default_rng(3)
    pairs, cuts = _pairs(hg, block, 4, 4)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=4).astype(np.int64)
    caps = inputs.region_caps(bw, pairs, cuts)
    checked = 0
    for (i, j), cp in zip(pairs, caps):
        r = oreg.build_region(hg, block, hg.vertex_weights, i, j, int(cp[0]), int(cp[1]),
                              remove_identical=merge)
        st, un = _discarded_st_and_untouched(hg, block, i, j, r["gid"])
        members = r["gid"]
        for _ in range(12):
            x = rng.random(r["n"]) < rng.random()
            side_i = np.zeros(hg.num_vertices, dtype=bool)
            side_i[block == i] = True
            side_i[members] = x
            assert _problem_cut(r, x) + st + un == _pair_cut(hg, block, i, j, side_i)
            checked += 1
        # the current bipartition: X = the region's block-i vertices
        xi = block[members] == i
        assert _problem_cut(r, xi) == r["cut_before"]
    assert checked == 48


def test_merging_identical_nets():
    hg, block = _instance(11, V=400, k=3, target=3000, size_hi=6)
    pairs, cuts = _pairs(hg, block, 3, 3)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=3).astype(np.int64)
    caps = inputs.region_caps(bw, pairs, cuts)
    merged_any = False
    for (i, j), cp in zip(pairs, caps):
        a = oreg.build_region(hg, block, hg.vertex_weights, i, j, int(cp[0]), int(cp[1]),
                              remove_identical=False)
        b = oreg.build_region(hg, block, hg.vertex_weights, i, j, int(cp[0]), int(cp[1]),
                              remove_identical=True)
        nets_a = [tuple(a["pins"][a["net_offsets"][e]:a["net_offsets"][e + 1]])
                  for e in range(len(a["net_offsets"]) - 1)]
        nets_b = [tuple(b["pins"][b["net_offsets"][e]:b["net_offsets"][e + 1]])
                  for e in range(len(b["net_offsets"]) - 1)]
        assert len(set(nets_b)) == len(nets_b)
        assert all(list(t) == sorted(t) for t in nets_b)
        want = {}
        for t, w_ in zip(nets_a, a["net_weights"]):
            want[t] = want.get(t, 0) + int(w_)
        assert dict(zip(nets_b, (int(x) for x in b["net_weights"]))) == want
        # representatives are the smallest global ids of their groups
        first = {}
        for t, g in zip(nets_a, a["net_gid"]):
            first.setdefault(t, int(g))
        assert [first[t] for t in nets_b] == [int(g) for g in b["net_gid"]]
        merged_any |= len(nets_b) < len(nets_a)
        assert b["cut_before"] == a["cut_before"]
    assert merged_any


def test_growth_rules():
    hg, block = _instance(5, V=1500, k=4, target=6000, size_hi=20)
    pairs, cuts = _pairs(hg, block, 4, 6)
    bw = np.bincount(block, weights=hg.vertex_weights, minlength=4).astype(np.int64)
    vnets = oreg.vertex_nets(hg)
    for (i, j), cut in zip(pairs, cuts):
        for cap in (0, 5, 40, 10 ** 9):
            for blk in (i, j):
                added, wt, b0 = oreg.grow_side(hg, block, hg.vertex_weights, vnets, blk, i, j,
                                               cap)
                assert all(block[u] == blk for u in added)
                assert wt == int(hg.vertex_weights[added].sum()) <= cap
                assert len(added) <= int((block == blk).sum()) - 1
                assert len(set(added)) == len(added)
                # level 0: the block's pins on nets with pins in both blocks
                lvl0 = set()
                for e in range(hg.num_nets):
                    ps = hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]
                    if (block[ps] == i).any() and (block[ps] == j).any():
                        lvl0 |= {int(u) for u in ps if block[u] == blk}
                assert b0 == len(lvl0)
                if added:
                    first = sorted(lvl0)[:len(added)]
                    # growth starts with level 0 in increasing id
                    assert added[:min(len(added), len(lvl0))] == first[:min(len(added),
                                                                             len(lvl0))]
            if cap == 10 ** 9:
                # unbounded weight: the side stops only one vertex short of
                # the block or when the search runs out
                assert len(added) <= int((block == blk).sum()) - 1
