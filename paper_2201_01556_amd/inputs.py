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
