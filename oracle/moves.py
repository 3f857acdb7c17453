"""Oracle of applying the move sequences of block-pair refinements.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the HIP library and never imports it.

It follows the paper's section "Parallel Active Block Scheduling",
paragraph "Apply Moves", in plain Python, one sequence after another in
the given order:

1. A block pair's result is a source side X of its region; a region vertex
   of block i outside X moves to block j, one of block j inside X moves to
   block i.  Readings: a sequence is tried only when its expected gain
   (cut_before - F) is positive (the text's "claims an improvement"); the
   expected block of a vertex is its block when the region was built.
2. Moves whose vertex is no longer in its expected block are dropped.
3. If the remaining moves would leave block i or block j heavier than
   Lmax, none is applied (the other blocks do not change).
4. Otherwise the moves are applied one by one; for every net of a moved
   vertex, the gain grows by w(e) when the pin count of the source block
   drops to zero and shrinks by w(e) when the pin count of the target block
   rises to one (the exact change of the connectivity objective
   sum w(e) (lambda(e) - 1)).
5. If that gain is negative, every move of the sequence is undone.

``connectivity`` is the objective itself, for checks.

``refine`` runs synchronous refinement rounds around these steps (the
paper's algorithm "Parallel Flow-Based Refinement" with its section
"Parallel Active Block Scheduling"): every round takes the block pairs
with a cut of at least ``min_cut`` and an active block (all blocks at
first), heaviest cut first (then block ids), builds their regions
(``oracle.regions``), solves each by the max-flow oracle (minimum cut,
expected gain cut_before - F) and applies the sequences in that order;
the blocks of a pair applied with a positive gain are active next round.
Rounds stop when no pair is left, after ``max_rounds``, or when a round
improves the objective by less than ``min_improvement_ppm`` parts per
million.  Readings: rounds are synchronous (the paper interleaves them
through one queue); the flow-based refinement of a pair is its minimum
cut (FlowCutter's first iteration), so unbalanced results are left to the
balance check.
"""
from __future__ import annotations

import numpy as np

NOT_TRIED, APPLIED, UNBALANCED, REVERTED = 0, 1, 2, 3


def connectivity(hg, block) -> int:
    tot = 0
    for e in range(hg.num_nets):
        ps = hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]
        lam = len({int(block[u]) for u in ps})
        tot += int(hg.net_weights[e]) * max(lam - 1, 0)
    return tot


def apply_sequences(hg, block, vertex_weights, k, lmax, sequences, vnets=None):
    """Apply ``sequences`` in order to a copy of ``block``.

    Each sequence is a dict with ``pair`` (i, j), ``gid`` (global ids of the
    region vertices), ``expected`` (their blocks when the region was
    built), ``side`` (1 where the vertex is on the source side X) and
    ``gain`` (cut_before - F).  Returns (new block array, per-sequence list
    of (status, gain, moves applied))."""
    block = np.array(block, dtype=np.int64, copy=True)
    c = np.asarray(vertex_weights, dtype=np.int64)
    if vnets is None:
        vnets = [[] for _ in range(hg.num_vertices)]
        for e in range(hg.num_nets):
            for p in range(int(hg.net_offsets[e]), int(hg.net_offsets[e + 1])):
                vnets[int(hg.pins[p])].append(e)
    phi = {}
    for e in range(hg.num_nets):
        for u in hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]:
            key = (e, int(block[u]))
            phi[key] = phi.get(key, 0) + 1
    bw = np.bincount(block, weights=c, minlength=k).astype(np.int64)
    out = []
    for s in sequences:
        i, j = s["pair"]
        if s["gain"] <= 0:
            out.append((NOT_TRIED, 0, 0))
            continue
        moves = []
        for u, exp, x in zip(s["gid"], s["expected"], s["side"]):
            u, exp = int(u), int(exp)
            to = i if x else j
            if to == exp:
                continue
            if block[u] != exp:
                continue  # the vertex left its expected block
            moves.append((u, exp, to))
        wi, wj = int(bw[i]), int(bw[j])
        for u, frm, to in moves:
            if frm == i:
                wi, wj = wi - int(c[u]), wj + int(c[u])
            else:
                wi, wj = wi + int(c[u]), wj - int(c[u])
        if wi > lmax or wj > lmax:
            out.append((UNBALANCED, 0, 0))
            continue
        gain = 0
        for u, frm, to in moves:
            block[u] = to
            bw[frm] -= c[u]
            bw[to] += c[u]
            for e in vnets[u]:
                w = int(hg.net_weights[e])
                phi[(e, frm)] -= 1
                if phi[(e, frm)] == 0:
                    gain += w
                phi[(e, to)] = phi.get((e, to), 0) + 1
                if phi[(e, to)] == 1:
                    gain -= w
        if gain < 0:
            for u, frm, to in reversed(moves):
                block[u] = frm
                bw[to] -= c[u]
                bw[frm] += c[u]
                for e in vnets[u]:
                    phi[(e, to)] -= 1
                    phi[(e, frm)] += 1
            out.append((REVERTED, gain, len(moves)))
        else:
            out.append((APPLIED, gain, len(moves)))
    return block, out


def pair_cuts(hg, block, k):
    """Weight of the nets with pins in blocks a and b, for a < b."""
    cuts = {}
    for e in range(hg.num_nets):
        bs = sorted({int(block[u]) for u in hg.pins[hg.net_offsets[e]:hg.net_offsets[e + 1]]})
        for x in range(len(bs)):
            for y in range(x + 1, len(bs)):
                cuts[(bs[x], bs[y])] = cuts.get((bs[x], bs[y]), 0) + int(hg.net_weights[e])
    return cuts


def refine(hg, block, vertex_weights, k, max_rounds=16, min_cut=10, alpha=16, eps_percent=3,
           min_improvement_ppm=1000, max_pairs=0, maxflow=None):
    """Refinement rounds; returns (blocks, objective before and after each
    round, per-round lists of (pair, status, gain, moves))."""
    from . import _Plain
    from . import regions as oreg
    if maxflow is None:
        from . import maxflow
    block = np.array(block, dtype=np.int64, copy=True)
    c = np.asarray(vertex_weights, dtype=np.int64)
    cv = int(c.sum())
    lmax = (100 + eps_percent) * (-(-cv // k)) // 100
    vnets = oreg.vertex_nets(hg)
    active = [True] * k
    traj = [connectivity(hg, block)]
    log = []
    for _ in range(max_rounds):
        cuts = pair_cuts(hg, block, k)
        cand = [(w, a, b) for (a, b), w in cuts.items()
                if w >= min_cut and (active[a] or active[b])]
        cand.sort(key=lambda t: (-t[0], t[1], t[2]))
        if max_pairs:
            cand = cand[:max_pairs]
        if not cand:
            break
        bw = np.bincount(block, weights=c, minlength=k).astype(np.int64)
        seqs = []
        for w, a, b in cand:
            cvi, cvj = int(bw[a]), int(bw[b])
            lim = (100 + alpha * eps_percent) * ((cvi + cvj + 1) // 2) // 100
            side = (alpha // 2) * w
            cap_i = max(0, min(side, lim - cvj))
            cap_j = max(0, min(side, lim - cvi))
            r = oreg.build_region(hg, block, c, a, b, cap_i, cap_j, remove_identical=True,
                                  vnets=vnets)
            n = r["n"]
            h = _Plain((n + 2, r["net_offsets"].astype(np.int32), r["pins"].astype(np.int32),
                        r["net_weights"].astype(np.int32), np.array([n], np.int32),
                        np.array([n + 1], np.int32)))
            res = maxflow(h)
            seqs.append(dict(pair=(a, b), gid=r["gid"], expected=block[r["gid"]].copy(),
                             side=np.asarray(res.vertex_side)[:n],
                             gain=r["cut_before"] - res.flow))
        block, out = apply_sequences(hg, block, c, k, lmax, seqs, vnets=vnets)
        log.append([(s["pair"], st, g, m) for s, (st, g, m) in zip(seqs, out)])
        nxt = [False] * k
        for s, (st, g, m) in zip(seqs, out):
            if st == APPLIED and g > 0:
                nxt[s["pair"][0]] = nxt[s["pair"][1]] = True
        active = nxt
        prev = traj[-1]
        traj.append(connectivity(hg, block))
        if (prev - traj[-1]) * 1000000 < min_improvement_ppm * prev:
            break
    return block, traj, log
