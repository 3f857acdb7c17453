"""Seeded synthetic flow-problem inputs.

This module only *draws* inputs: hypergraphs in CSR form (net offsets, pins,
net weights, vertex weights) and terminal sets.  It contains none of the
max-flow / min-cut arithmetic, so both the CPU oracle tests and the HIP path
can take their inputs from here without sharing any of the method.

Workload families (the paper evaluates on unit-weight hypergraphs with
heavy-tailed net sizes, and on flow networks grown around cuts, see the
sections "Network Construction" and "Experimental Setup"):

* ``uniform_hypergraph`` -- small random hypergraph, net sizes uniform,
  integer net weights; random disjoint source / sink vertex sets.
* ``zipf_hypergraph``    -- large power-law hypergraph: net sizes Zipf(2.2)
  clamped to [2, hi], unit net weights, terminals chosen by a seeded
  splitmix64 hash of the vertex id (1 % smallest = sources, 1 % largest =
  sinks).
* ``block_pair_problems`` -- the flow problems of a k-way partition: a
  power-law hypergraph, a balanced random k-way partition refined by label
  propagation, and for each heavy block pair a region grown around the cut
  with the rest of each block contracted into a source / sink vertex (the
  construction itself is host C in ``regions.c``).
* ``tiny_hypergraph``    -- tiny random instances (<= 16 vertices) with the
  adversarial shapes used to pin the oracle (nets inside S or T, nets with
  both S and T pins, single-pin nets, a hub vertex, one all-vertex net, large
  weights).

Every generator is a pure function of its arguments and ``seed``
(numpy ``Generator(PCG64(seed))``).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Hypergraph",
    "splitmix64",
    "uniform_hypergraph",
    "zipf_hypergraph",
    "tiny_hypergraph",
    "hypergraph_from_nets",
    "hash_terminals",
    "zipf_sizes_until",
    "BlockPairSet",
    "block_pair_problems",
    "planted_block_pair_problems",
    "scorer_init_params",
    "scorer_features",
]


@dataclass
class Hypergraph:
    """A weighted hypergraph with a source set and a sink set.

    ``net_offsets[e]:net_offsets[e+1]`` indexes the pins of net ``e`` in
    ``pins``; all arrays are int32 and C-contiguous.
    """

    num_vertices: int
    net_offsets: np.ndarray
    pins: np.ndarray
    net_weights: np.ndarray
    vertex_weights: np.ndarray
    sources: np.ndarray
    sinks: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def num_nets(self) -> int:
        return int(self.net_offsets.shape[0] - 1)

    @property
    def num_pins(self) -> int:
        return int(self.pins.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.num_vertices).tobytes())
        for a in (self.net_offsets, self.pins, self.net_weights,
                  self.vertex_weights, self.sources, self.sinks):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def nets(self):
        """Yield the pin array of every net (slow; small inputs only)."""
        off = self.net_offsets
        for e in range(self.num_nets):
            yield self.pins[off[e]:off[e + 1]]


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def hypergraph_from_nets(num_vertices, nets, weights, sources, sinks,
                         vertex_weights=None, meta=None) -> Hypergraph:
    """Build a :class:`Hypergraph` from a list of pin lists."""
    sizes = [len(n) for n in nets]
    off = np.zeros(len(nets) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes, dtype=np.int64)
    pins = (np.concatenate([np.asarray(n, dtype=np.int64) for n in nets])
            if nets else np.zeros(0, dtype=np.int64))
    if vertex_weights is None:
        vertex_weights = np.ones(num_vertices, dtype=np.int32)
    return Hypergraph(int(num_vertices), _i32(off), _i32(pins), _i32(weights),
                      _i32(vertex_weights), _i32(sources), _i32(sinks),
                      dict(meta or {}))


_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014) on uint64, vectorised.

    A bijection on 64-bit words, so distinct keys never tie.
    """
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def hash_terminals(seed: int, num_vertices: int, fraction: float = 0.01):
    """Sources = the ``fraction`` of vertices with the smallest
    splitmix64((seed << 32) | v); sinks = the same count with the largest."""
    v = np.arange(num_vertices, dtype=np.uint64)
    key = (np.uint64(seed & 0xFFFFFFFF) << np.uint64(32)) | v
    h = splitmix64(key)
    order = np.argsort(h, kind="stable")
    k = max(1, int(round(fraction * num_vertices)))
    return _i32(np.sort(order[:k])), _i32(np.sort(order[-k:]))


def _distinct_pins(rng, num_vertices, sizes):
    """Uniform pins without replacement inside each net.

    All pins are drawn at once; pins that repeat inside their net are redrawn
    until no net holds a vertex twice (rejection sampling, distributionally
    identical to drawing each net without replacement).  Pins end up sorted
    inside each net.
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    total = int(sizes.sum())
    net_of = np.repeat(np.arange(sizes.shape[0], dtype=np.int64), sizes)
    pins = rng.integers(0, num_vertices, total, dtype=np.int64)
    while True:
        key = net_of * np.int64(num_vertices) + pins
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup = np.nonzero(sk[1:] == sk[:-1])[0]
        if dup.size == 0:
            return pins[order]
        redo = order[dup + 1]
        pins[redo] = rng.integers(0, num_vertices, redo.shape[0], dtype=np.int64)


def uniform_hypergraph(seed: int, num_vertices: int = 2000, num_nets: int = 3000,
                       size_lo: int = 2, size_hi: int = 8, w_lo: int = 1,
                       w_hi: int = 4, num_sources: int = 100,
                       num_sinks: int = 100) -> Hypergraph:
    """Random hypergraph with uniform net sizes and integer net weights.

    Draw order: net sizes U{size_lo..size_hi}; then per net its pins by
    ``rng.choice(V, size, replace=False)``; then net weights
    U{w_lo..w_hi}; then ``num_sources`` random vertices as S and
    ``num_sinks`` random vertices of V \\ S as T.  Vertex weights are 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(size_lo, size_hi + 1, num_nets)
    nets = [rng.choice(num_vertices, int(s), replace=False) for s in sizes]
    w = rng.integers(w_lo, w_hi + 1, num_nets)
    src = rng.choice(num_vertices, num_sources, replace=False)
    rest = np.setdiff1d(np.arange(num_vertices), src)
    snk = rng.choice(rest, num_sinks, replace=False)
    return hypergraph_from_nets(
        num_vertices, nets, w, np.sort(src), np.sort(snk),
        meta=dict(kind="uniform", seed=seed, V=num_vertices, E=num_nets))


def zipf_hypergraph(seed: int, num_vertices: int = 1_000_000,
                    num_nets: int = 2_000_000, zipf_a: float = 2.2,
                    size_hi: int = 1000, terminal_fraction: float = 0.01,
                    vertex_weight_hi: int = 1) -> Hypergraph:
    """Power-law hypergraph with unit net weights.

    Net sizes ``clip(rng.zipf(zipf_a), 2, size_hi)``; pins uniform without
    replacement inside each net (sorted per net); net weights 1; vertex
    weights U{1..vertex_weight_hi}; S / T by :func:`hash_terminals`.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.clip(rng.zipf(zipf_a, num_nets), 2, size_hi).astype(np.int64)
    pins = _distinct_pins(rng, num_vertices, sizes)
    off = np.zeros(num_nets + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    if vertex_weight_hi > 1:
        vw = rng.integers(1, vertex_weight_hi + 1, num_vertices)
    else:
        vw = np.ones(num_vertices, dtype=np.int64)
    src, snk = hash_terminals(seed, num_vertices, terminal_fraction)
    return Hypergraph(int(num_vertices), _i32(off), _i32(pins),
                      np.ones(num_nets, dtype=np.int32), _i32(vw), src, snk,
                      dict(kind="zipf", seed=seed, V=num_vertices, E=num_nets,
                           a=zipf_a, hi=size_hi))


def tiny_hypergraph(seed: int, max_vertices: int = 12, max_nets: int = 10,
                    max_weight: int = 5) -> Hypergraph:
    """Tiny random instance for exhaustive checks, with adversarial shapes.

    The seed selects one of several shapes (plain random; a hub vertex in
    every net; one net holding all vertices; weights near the int32 guard;
    single terminals), and the remaining draws fill in pins and weights.
    Single-pin nets, nets inside S or T and nets with both S and T pins
    occur naturally.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V = int(rng.integers(2, max_vertices + 1))
    E = int(rng.integers(1, max_nets + 1))
    shape = seed % 6
    nets = []
    for _ in range(E):
        s = int(rng.integers(1, min(V, 6) + 1))
        nets.append(rng.choice(V, s, replace=False))
    if shape == 1:                              # hub vertex in every net
        hub = int(rng.integers(0, V))
        nets = [np.unique(np.append(n, hub)) for n in nets]
    elif shape == 2:                            # one net holding everything
        nets.append(np.arange(V))
    w = rng.integers(1, max_weight + 1, len(nets))
    if shape == 3:                              # weights near the int32 guard
        big = (2**31 - 1) // (len(nets) + 1)
        w = rng.integers(big // 2, big + 1, len(nets))
    perm = rng.permutation(V)
    if shape == 4 or V == 2:                    # single terminals
        ns, nt = 1, 1
    else:
        ns = int(rng.integers(1, max(2, V // 3) + 1))
        nt = int(rng.integers(1, max(2, (V - ns) // 2) + 1))
        nt = min(nt, V - ns)
    src = np.sort(perm[:ns])
    snk = np.sort(perm[ns:ns + nt])
    if shape == 5:                              # a net inside S and one inside T
        nets.append(src.copy())
        nets.append(snk.copy())
        w = np.append(w, rng.integers(1, max_weight + 1, 2))
    return hypergraph_from_nets(V, nets, w, src, snk,
                                meta=dict(kind="tiny", seed=seed, shape=shape))


# ---------------------------------------------------------------------------
# block-pair flow problems of a k-way partition
# ---------------------------------------------------------------------------

_REGIONS_LIB = None


def _regions_lib():
    """Load (building on first use) the host C region builder."""
    global _REGIONS_LIB
    if _REGIONS_LIB is not None:
        return _REGIONS_LIB
    import ctypes
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    lib = os.path.join(here, "libhfregions.so")
    src = os.path.join(here, "regions.c")
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        build_regions_lib()
    L = ctypes.CDLL(lib)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.hfr_new.restype = P
    L.hfr_new.argtypes = [I32, I32, P, P, P, P, I32, P]
    L.hfr_free.argtypes = [P]
    L.hfr_free.restype = None
    L.hfr_objective.argtypes = [P]
    L.hfr_objective.restype = I64
    L.hfr_lp.argtypes = [P, I32, I64]
    L.hfr_lp.restype = I64
    L.hfr_blocks.argtypes = [P, P, P]
    L.hfr_blocks.restype = None
    L.hfr_pairs.argtypes = [P, I64, I32, P, P, P]
    L.hfr_pairs.restype = I32
    L.hfr_regions.argtypes = [P, I32, P, P, P, I64, I64, I64, I32]
    L.hfr_regions.restype = I32
    L.hfr_region_info.argtypes = [P, I32, P]
    L.hfr_region_info.restype = None
    L.hfr_region_take.argtypes = [P, I32, P, P, P, P, P]
    L.hfr_region_take.restype = None
    _REGIONS_LIB = L
    return L


def build_regions_lib() -> str:
    """Compile ``regions.c`` (host code) into ``libhfregions.so``."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    lib = os.path.join(here, "libhfregions.so")
    tmp = lib + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-fvisibility=hidden", "-o", tmp,
                    os.path.join(here, "regions.c")], check=True)
    os.replace(tmp, lib)
    return lib


def zipf_sizes_until(rng, target_pins: int, zipf_a: float = 2.2, size_hi: int = 2000,
                     chunk: int = 1 << 20) -> np.ndarray:
    """Net sizes ``clip(zipf(a), 2, hi)`` drawn in chunks of ``chunk`` until
    their sum reaches ``target_pins``; the prefix up to (and including) the
    net that reaches it is returned."""
    parts, total = [], 0
    while total < target_pins:
        s = np.clip(rng.zipf(zipf_a, chunk), 2, size_hi).astype(np.int64)
        parts.append(s)
        total += int(s.sum())
    sizes = np.concatenate(parts)
    cs = np.cumsum(sizes)
    n = int(np.searchsorted(cs, target_pins)) + 1
    return sizes[:n]


@dataclass
class BlockPairSet:
    """Flow problems of one partitioned hypergraph.

    ``problems[i]`` is a :class:`Hypergraph` whose last two vertices are the
    contracted source (``S = [n]``) and sink (``T = [n + 1]``); its ``meta``
    holds the block pair, the pair's cut weight, ``cut_before`` (weight of
    the problem's nets cut by the current partition) and ``features`` (12
    ints: cut weight, region pins, boundary vertices, 7 net-size bins of the
    problem, c(Vi), c(Vj)).
    """

    hypergraph: Hypergraph
    block: np.ndarray
    block_weights: np.ndarray
    lmax: int
    lp_moves: int
    objective_before: int
    objective_after: int
    problems: list


def block_pair_problems(seed: int, num_vertices: int = 2_000_000,
                        target_pins: int = 10_000_000, size_hi: int = 2000,
                        zipf_a: float = 2.2, k: int = 64, lp_rounds: int = 3,
                        eps: float = 0.03, alpha: int = 16, min_cut: int = 10,
                        max_problems: int = 500, threads: int = 0) -> BlockPairSet:
    """Block-pair flow problems of a partitioned power-law hypergraph.

    Draw order: net sizes (:func:`zipf_sizes_until`), pins uniform without
    replacement (sorted per net), then ``perm = rng.permutation(V)`` and the
    balanced random partition ``block[v] = perm[v] % k``.  Unit net and
    vertex weights.  Label propagation (``lp_rounds`` sweeps) with
    ``Lmax = floor((100 + 100 eps) * ceil(c(V) / k) / 100)``; pairs with cut
    weight >= ``min_cut``, heaviest ``max_problems``; regions with side bound
    ``min(alpha / 2 * cut, (1 + alpha eps) * ceil((c(Vi)+c(Vj))/2) - c(other))``.
    Regions are built on ``threads`` host threads (0: OpenMP default); the
    result does not depend on the thread count.
    """
    import ctypes
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = zipf_sizes_until(rng, target_pins, zipf_a, size_hi)
    pins = _distinct_pins(rng, num_vertices, sizes)
    E = int(sizes.shape[0])
    off = np.zeros(E + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    perm = rng.permutation(num_vertices)
    block0 = _i32(perm % k)
    hg = Hypergraph(int(num_vertices), _i32(off), _i32(pins), np.ones(E, dtype=np.int32),
                    np.ones(num_vertices, dtype=np.int32), _i32([]), _i32([]),
                    dict(kind="block_pairs", seed=seed, V=num_vertices, E=E, k=k))
    return _pair_problems(hg, block0, seed, k, lp_rounds, eps, alpha, min_cut, max_problems,
                          threads)


def region_caps(block_weights, pairs, cuts, alpha: int = 16, eps: float = 0.03) -> np.ndarray:
    """Side weight caps of the regions of block pairs (count x 2), the bound
    the region builders use: ``min(alpha / 2 * cut, (1 + alpha eps) *
    ceil((c(Vi) + c(Vj)) / 2) - c(other block))``, at least 0, in integer
    arithmetic (eps in whole percent)."""
    bw = np.asarray(block_weights, dtype=np.int64)
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    cut = np.asarray(cuts, dtype=np.int64).reshape(-1)
    eps_pct = int(round(eps * 100))
    scale_num = 100 + alpha * eps_pct
    out = np.zeros((pr.shape[0], 2), dtype=np.int64)
    for t, (i, j) in enumerate(pr):
        cvi, cvj = int(bw[i]), int(bw[j])
        lim = scale_num * ((cvi + cvj + 1) // 2) // 100
        out[t, 0] = max(0, min((alpha // 2) * int(cut[t]), lim - cvj))
        out[t, 1] = max(0, min((alpha // 2) * int(cut[t]), lim - cvi))
    return out


def _pair_problems(hg, block0, seed, k, lp_rounds, eps, alpha, min_cut, max_problems, threads,
                   kind="block_pair"):
    """Label propagation from ``block0``, the heaviest block pairs and their
    region flow problems (host C builder, ``regions.c``)."""
    import ctypes
    num_vertices = hg.num_vertices
    E = hg.num_nets
    L = _regions_lib()

    def ptr(a):
        return a.ctypes.data_as(ctypes.c_void_p)

    ctx = L.hfr_new(num_vertices, E, ptr(hg.net_offsets), ptr(hg.pins), ptr(hg.net_weights),
                    ptr(hg.vertex_weights), k, ptr(block0))
    if not ctx:
        raise ValueError("region builder rejected the input")
    try:
        cV = int(hg.vertex_weights.sum())
        eps_pct = int(round(eps * 100))
        lmax = (100 + eps_pct) * (-(-cV // k)) // 100
        obj0 = int(L.hfr_objective(ctx))
        moves = int(L.hfr_lp(ctx, lp_rounds, lmax))
        obj1 = int(L.hfr_objective(ctx))
        block = np.empty(num_vertices, dtype=np.int32)
        bw = np.empty(k, dtype=np.int64)
        L.hfr_blocks(ctx, ptr(block), ptr(bw))
        pi = np.empty(max_problems, dtype=np.int32)
        pj = np.empty(max_problems, dtype=np.int32)
        pc = np.empty(max_problems, dtype=np.int64)
        npairs = int(L.hfr_pairs(ctx, min_cut, max_problems, ptr(pi), ptr(pj), ptr(pc)))
        if npairs < 0:
            raise MemoryError("region builder: out of memory")
        info = np.zeros(14, dtype=np.int64)
        scale_num = 100 + alpha * eps_pct
        if L.hfr_regions(ctx, npairs, ptr(pi), ptr(pj), ptr(pc), alpha // 2, scale_num, 100,
                         threads) != 0:
            raise MemoryError("region builder: out of memory")
        problems = []
        for t in range(npairs):
            i, j, cut = int(pi[t]), int(pj[t]), int(pc[t])
            L.hfr_region_info(ctx, t, ptr(info))
            nv, ne, npins = int(info[0]), int(info[1]), int(info[2])
            roff = np.empty(ne + 1, dtype=np.int32)
            rpins = np.empty(npins, dtype=np.int32)
            rw = np.empty(ne, dtype=np.int32)
            rvw = np.empty(nv, dtype=np.int32)
            gid = np.empty(nv - 2, dtype=np.int32)
            L.hfr_region_take(ctx, t, ptr(roff), ptr(rpins), ptr(rw), ptr(rvw), ptr(gid))
            n = nv - 2
            feats = np.array([cut, npins, int(info[4]), *[int(x) for x in info[7:14]],
                              int(bw[i]), int(bw[j])], dtype=np.int64)
            problems.append(Hypergraph(
                nv, roff, rpins, rw, rvw, _i32([n]), _i32([n + 1]),
                dict(kind=kind, seed=seed, pair=(i, j), cut=cut,
                     cut_before=int(info[3]), boundary=int(info[4]),
                     side_weights=(int(info[5]), int(info[6])),
                     features=feats, gid=gid)))
    finally:
        L.hfr_free(ctx)
    return BlockPairSet(hg, block, bw, lmax, moves, obj0, obj1, problems)



def planted_block_pair_problems(seed: int, num_vertices: int = 2_000_000,
                                target_pins: int = 10_000_000, size_hi: int = 2000,
                                zipf_a: float = 2.2, k: int = 64, local_fraction: float = 0.98,
                                noisy_pairs: int = 150, swap_fraction: float = 0.02,
                                lp_rounds: int = 3, eps: float = 0.03, alpha: int = 16,
                                min_cut: int = 10, max_problems: int = 500,
                                threads: int = 0) -> BlockPairSet:
    """Block-pair flow problems of a hypergraph with planted blocks, for a
    partition that is good except around a few block pairs.

    Draw order: net sizes (:func:`zipf_sizes_until`); ``perm =
    rng.permutation(V)`` and planted blocks ``perm[v] % k``; per net a home
    block ``U{0..k-1}``; per net a uniform draw deciding whether it is local
    (probability ``local_fraction``: pins uniform without replacement from
    the home block) or global (pins uniform over all vertices); the pins of
    the local nets, then of the global nets; ``noisy_pairs`` pairs of
    blocks; for each such pair ``swap_fraction`` of a block's vertices
    (``rng.choice`` without
    replacement, among vertices not swapped before) swap blocks; the pairs
    are distinct, drawn by ``rng.choice`` over the k(k-1)/2 pair indices
    (pair index t of a < b in row-major order).  Unit weights.  Then, as
    :func:`block_pair_problems`: label propagation, the heaviest pairs and
    their regions.  The clean pairs' current cut is (nearly always) already
    a minimum cut of their region; the perturbed pairs can recover most of
    the swapped vertices.
    """
    if num_vertices % k:
        raise ValueError("num_vertices must be a multiple of k")
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = zipf_sizes_until(rng, target_pins, zipf_a, size_hi)
    E = int(sizes.shape[0])
    bs = num_vertices // k
    if int(sizes.max()) > bs:
        raise ValueError("a net is larger than a block")
    perm = rng.permutation(num_vertices)
    planted = (perm % k).astype(np.int64)
    members = np.argsort(planted, kind="stable").reshape(k, bs)  # increasing ids per block
    home = rng.integers(0, k, E)
    local = rng.random(E) < local_fraction
    off = np.zeros(E + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    pins = np.empty(int(off[-1]), dtype=np.int64)

    def positions(mask):
        sz = sizes[mask]
        starts = np.repeat(off[:-1][mask], sz)
        within = np.arange(int(sz.sum()), dtype=np.int64) - np.repeat(np.cumsum(sz) - sz, sz)
        return starts + within, sz

    pos, sz = positions(local)
    loc = _distinct_pins(rng, bs, sz)                          # sorted per net
    pins[pos] = members[np.repeat(home[local], sz), loc]       # stays sorted per net
    pos, sz = positions(~local)
    pins[pos] = _distinct_pins(rng, num_vertices, sz)
    block0 = planted.copy()
    npairs = k * (k - 1) // 2
    if noisy_pairs > npairs:
        raise ValueError("more noisy pairs than block pairs")
    m = int(swap_fraction * bs)
    noisy = []
    for t in np.sort(rng.choice(npairs, noisy_pairs, replace=False)):
        a = int(np.searchsorted(np.cumsum(np.arange(k - 1, 0, -1)), t, side="right"))
        b = int(t - (a * (2 * k - a - 1)) // 2 + a + 1)
        ea = members[a][block0[members[a]] == a]  # not swapped yet
        eb = members[b][block0[members[b]] == b]
        va = rng.choice(ea, min(m, ea.size), replace=False)
        vb = rng.choice(eb, min(m, eb.size), replace=False)
        block0[va] = b
        block0[vb] = a
        noisy.append((a, b))
    hg = Hypergraph(int(num_vertices), _i32(off), _i32(pins), np.ones(E, dtype=np.int32),
                    np.ones(num_vertices, dtype=np.int32), _i32([]), _i32([]),
                    dict(kind="planted_block_pairs", seed=seed, V=num_vertices, E=E, k=k,
                         noisy_pairs=noisy))
    return _pair_problems(hg, _i32(block0), seed, k, lp_rounds, eps, alpha, min_cut,
                          max_problems, threads, kind="planted_block_pair")


def scorer_init_params(seed: int) -> np.ndarray:
    """Initial parameters of the 12 -> 64 -> 64 -> 1 scorer (5,057 float32,
    layout W1, b1, W2, b2, W3, b3): every weight and bias of a layer with
    fan-in f drawn uniformly from [-1/sqrt(f), 1/sqrt(f)] (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shape, fan_in in (((64, 12), 12), ((64,), 12), ((64, 64), 64), ((64,), 64),
                          ((1, 64), 64), ((1,), 64)):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, size=shape).ravel())
    return np.concatenate(parts).astype(np.float32)


def scorer_features(problems) -> np.ndarray:
    """The 12 integer features of each block-pair problem (int64 [n x 12]):
    pair cut weight, region pins, boundary vertices, 7 net-size bins, c(Vi),
    c(Vj)."""
    return np.stack([np.asarray(p.meta["features"], dtype=np.int64) for p in problems])
