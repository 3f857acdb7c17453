"""Oracle of the flow-network construction around a block pair.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the HIP library and never imports it.

It follows the paper's section "Network Construction" (paragraphs "Region
Growing", "Construction Algorithms" and "Identical Net Removal") in plain
Python, one block pair at a time:

1. Region growing.  For the pair (i, j) two breadth-first searches grow
   B_i inside block i and B_j inside block j, each starting from its
   block's pins on the nets cut between the two blocks.  Readings (the
   paper leaves them open): a search visits each level in increasing vertex
   id and adds vertices while the side's weight stays within its cap and at
   least one vertex of the block stays outside; it stops for good at the
   first vertex that does not fit.  The next level is every vertex of the
   block, not yet visited, on a net of a vertex added in this level.  The
   weight caps are inputs (the caller's policy, e.g. the paper's
   (1 + alpha eps) ceil(c(V)/2) - c(other block) bound).
2. Construction (the first algorithm of the paragraph "Construction
   Algorithms"): every net with a pin in B_i u B_j, in increasing net id,
   keeps its region pins, gains the source s if it has a pin of block i
   outside the region and the sink t if it has a pin of block j outside;
   pins of other blocks are dropped; nets left with fewer than two pins or
   with both s and t are discarded (they cannot leave the cut).  Region
   vertices get local ids 0..n-1 in increasing global id, s = n, t = n + 1;
   each net's pins are listed in increasing local id.
3. Identical net removal: nets with the same pin set are merged into the
   one of smallest net id, which carries the sum of their weights (the
   paper detects them by fingerprints; here every group is found exactly by
   comparing pin tuples).

``build_region`` returns the problem plus its facts: the weight of the
constructed nets cut by the pair's current bipartition (region pins of
block i or s on one side, region pins of block j or t on the other), the
boundary (level-0 vertices of both searches), both side weights, and the
net-size histogram of the final nets (bins 2, 3-4, 5-8, 9-16, 17-64,
65-256, more).
"""
from __future__ import annotations

import numpy as np


def vertex_nets(hg):
    """Nets of every vertex, in increasing net id."""
    V, E = hg.num_vertices, hg.num_nets
    out = [[] for _ in range(V)]
    off = hg.net_offsets
    for e in range(E):
        for p in range(int(off[e]), int(off[e + 1])):
            out[int(hg.pins[p])].append(e)
    return out


def _net_pins(hg, e):
    return [int(u) for u in hg.pins[int(hg.net_offsets[e]):int(hg.net_offsets[e + 1])]]


def grow_side(hg, block, c, vnets, blk, i, j, cap_w):
    """Region growing of one side (paragraph "Region Growing"): returns
    (added vertices in the order added, weight, level-0 size)."""
    size_blk = int(np.count_nonzero(block == blk))
    cap_n = size_blk - 1
    visited = set()
    level = []
    for e in range(hg.num_nets):
        pins = _net_pins(hg, e)
        blocks = {int(block[u]) for u in pins}
        if i in blocks and j in blocks:
            for u in pins:
                if block[u] == blk and u not in visited:
                    visited.add(u)
                    level.append(u)
    level.sort()
    boundary = len(level)
    added, weight = [], 0
    while level:
        this = []
        for u in level:
            if weight + int(c[u]) > cap_w or len(added) + 1 > cap_n:
                return added, weight, boundary
            added.append(u)
            this.append(u)
            weight += int(c[u])
        nxt = []
        for u in this:
            for e in vnets[u]:
                for x in _net_pins(hg, e):
                    if block[x] == blk and x not in visited:
                        visited.add(x)
                        nxt.append(x)
        level = sorted(nxt)
    return added, weight, boundary


def _bin(size):
    for b, hi in enumerate((2, 4, 8, 16, 64, 256)):
        if size <= hi:
            return b
    return 6


def build_region(hg, block, c, i, j, cap_i, cap_j, remove_identical=True, vnets=None):
    """The flow problem of block pair (i, j): a dict with ``n`` (region
    vertices), ``gid`` (their global ids), ``vw`` (n + 2 weights: region
    vertices, then s = c(V_i) - c(B_i) and t = c(V_j) - c(B_j)),
    ``net_offsets``, ``pins`` (local ids), ``net_weights``, ``net_gid``
    (global id of each net, the smallest of a merged group), ``cut_before``,
    ``boundary``, ``side_weights`` and ``bins``."""
    block = np.asarray(block)
    c = np.asarray(c)
    if vnets is None:
        vnets = vertex_nets(hg)
    bi, wi, b0 = grow_side(hg, block, c, vnets, i, i, j, cap_i)
    bj, wj, b1 = grow_side(hg, block, c, vnets, j, i, j, cap_j)
    members = sorted(bi + bj)
    n = len(members)
    local = {u: k for k, u in enumerate(members)}
    touched = sorted({e for u in members for e in vnets[u]})
    nets, weights, gids = [], [], []
    cut_before = 0
    for e in touched:
        pins = _net_pins(hg, e)
        region = sorted(local[u] for u in pins if u in local)
        has_s = any(block[u] == i and u not in local for u in pins)
        has_t = any(block[u] == j and u not in local for u in pins)
        if has_s and has_t:
            continue
        out = region + ([n] if has_s else []) + ([n + 1] if has_t else [])
        if len(out) < 2:
            continue
        side_i = has_s or any(block[u] == i for u in pins if u in local)
        side_j = has_t or any(block[u] == j for u in pins if u in local)
        if side_i and side_j:
            cut_before += int(hg.net_weights[e])
        nets.append(tuple(out))
        weights.append(int(hg.net_weights[e]))
        gids.append(e)
    if remove_identical:
        first = {}
        keep = []
        for k, pins in enumerate(nets):
            if pins in first:
                weights[first[pins]] += weights[k]
            else:
                first[pins] = k
                keep.append(k)
        nets = [nets[k] for k in keep]
        weights = [weights[k] for k in keep]
        gids = [gids[k] for k in keep]
    off = [0]
    flat = []
    bins = [0] * 7
    for pins in nets:
        flat.extend(pins)
        off.append(len(flat))
        bins[_bin(len(pins))] += 1
    cvi = int(c[block == i].sum())
    cvj = int(c[block == j].sum())
    vw = [int(c[u]) for u in members] + [cvi - wi, cvj - wj]
    return dict(n=n, gid=np.array(members, dtype=np.int32), vw=np.array(vw, dtype=np.int64),
                net_offsets=np.array(off, dtype=np.int64), pins=np.array(flat, dtype=np.int64),
                net_weights=np.array(weights, dtype=np.int64),
                net_gid=np.array(gids, dtype=np.int64), cut_before=cut_before,
                boundary=b0 + b1, side_weights=(wi, wj), bins=bins)
