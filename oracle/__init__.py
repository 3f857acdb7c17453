"""CPU oracle for the hypergraph max-flow / min-cut hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2201_01556_amd``) and never imports it.

Contents
--------
``maxflow``            plain C FIFO push-relabel on the explicit Lawler
                       expansion (``lawler_pr.c``), excess-seeded source-side
                       BFS; optional preflow-to-flow self check; optional
                       maximal sink side by reverse residual BFS.
``flowcutter``         the FlowCutter loop (section "Flow-Based Refinement",
                       algorithm "FlowCutter Core") with one piercing node
                       per iteration, every max flow solved from scratch.
``brute_force``        enumerate every source side X with S <= X <= V \\ T
                       (<= 16 free vertices): F = min cut, minimal X =
                       intersection of all minimisers (min cuts form a
                       lattice, so the intersection is itself a minimiser);
                       ``brute_force_sides`` also gives the union (the
                       maximal minimiser).
``edmonds_karp``       shortest augmenting paths on a separately built
                       explicit graph (pure Python; small inputs).
``scipy_maxflow``      the same network through
                       ``scipy.sparse.csgraph.maximum_flow`` (int32).
``cut_weight``         hypergraph cut weight of a source side X (plain
                       definition from the section "Preliminaries").
``net_side_from_x``    per-net membership bits implied by X.
``check_preflow``      feasibility of an exported preflow of the capped
                       network (capacities, non-negative excess, value).
``residual_labels``    exact residual distances to the sink in the capped
                       network for a given flow state (plain BFS).
``maxflow_many``       ``maxflow`` of many hypergraphs on a process pool.
``maxflow_pinned``     ``maxflow`` timed in a process pinned to one core.

The paper prints no worked example for this path (its two illustrative
figures are not part of the text), so the pins of this oracle are
mathematical: brute force, a second max-flow algorithm, a library routine,
closed forms and hand-checked fixtures (``tests/golden``).
"""
from __future__ import annotations

import ctypes
import os
from collections import deque

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {
    -1: "allocation failed",
    -2: "sink reachable from the source side (not a maximum preflow)",
    -3: "preflow-to-flow self check failed",
    -4: "invalid input",
    -5: "flow conservation violated after conversion",
}


def build(force: bool = False) -> str:
    """Compile ``lawler_pr.c`` with gcc into ``oracle/liboracle.so``."""
    import subprocess
    src = os.path.join(_HERE, "lawler_pr.c")
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_maxflow.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p,
                                       i32p, i32p, ctypes.c_int32, i32p,
                                       ctypes.c_int32, ctypes.c_int32, i64p, u8p,
                                       u8p, i64p]
        lib.oracle_maxflow.restype = ctypes.c_int
        lib.oracle_maxflow_sides.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p,
                                             i32p, i32p, ctypes.c_int32, i32p,
                                             ctypes.c_int32, ctypes.c_int32, i64p, u8p,
                                             u8p, u8p, i64p]
        lib.oracle_maxflow_sides.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleResult:
    def __init__(self, F, vside, nside, stats, tside=None):
        self.flow = int(F)
        self.vertex_side = vside
        self.net_side = nside
        self.sink_side = tside
        self.stats = dict(relabels=int(stats[0]), pushes=int(stats[1]),
                          global_relabels=int(stats[2]), nodes=int(stats[3]),
                          arcs=int(stats[4]), inf=int(stats[5]))


def maxflow(hg, selfcheck: bool = False, sink_side: bool = False) -> OracleResult:
    """Maximum flow value and minimal source side of ``hg`` (C oracle);
    with ``sink_side`` also the maximal sink side (vertices that reach a sink
    in the residual network), as ``result.sink_side``."""
    lib = _load()
    V, E = hg.num_vertices, hg.num_nets
    off = np.ascontiguousarray(hg.net_offsets, dtype=np.int32)
    pins = np.ascontiguousarray(hg.pins, dtype=np.int32)
    w = np.ascontiguousarray(hg.net_weights, dtype=np.int32)
    S = np.ascontiguousarray(hg.sources, dtype=np.int32)
    T = np.ascontiguousarray(hg.sinks, dtype=np.int32)
    F = np.zeros(1, dtype=np.int64)
    vside = np.zeros(max(V, 1), dtype=np.uint8)
    nside = np.zeros(max(E, 1), dtype=np.uint8)
    stats = np.zeros(8, dtype=np.int64)
    if sink_side:
        tside = np.zeros(max(V, 1), dtype=np.uint8)
        rc = lib.oracle_maxflow_sides(V, E, _p(off, ctypes.c_int32), _p(pins, ctypes.c_int32),
                                      _p(w, ctypes.c_int32), _p(S, ctypes.c_int32), len(S),
                                      _p(T, ctypes.c_int32), len(T), 1 if selfcheck else 0,
                                      _p(F, ctypes.c_int64), _p(vside, ctypes.c_uint8),
                                      _p(nside, ctypes.c_uint8), _p(tside, ctypes.c_uint8),
                                      _p(stats, ctypes.c_int64))
    else:
        tside = None
        rc = lib.oracle_maxflow(V, E, _p(off, ctypes.c_int32), _p(pins, ctypes.c_int32),
                                _p(w, ctypes.c_int32), _p(S, ctypes.c_int32), len(S),
                                _p(T, ctypes.c_int32), len(T), 1 if selfcheck else 0,
                                _p(F, ctypes.c_int64), _p(vside, ctypes.c_uint8),
                                _p(nside, ctypes.c_uint8), _p(stats, ctypes.c_int64))
    if rc != 0:
        raise RuntimeError(f"oracle_maxflow failed: {ERRORS.get(rc, rc)}")
    return OracleResult(F[0], vside[:V].copy(), nside[:E].copy(), stats,
                        None if tside is None else tside[:V].copy())


# ---------------------------------------------------------------------------
# plain definitions
# ---------------------------------------------------------------------------

class _Plain:
    """Minimal hypergraph record passed to worker processes."""

    def __init__(self, t):
        (self.num_vertices, self.net_offsets, self.pins, self.net_weights, self.sources,
         self.sinks) = t

    @property
    def num_nets(self):
        return int(self.net_offsets.shape[0] - 1)


def _maxflow_worker(t):
    r = maxflow(_Plain(t))
    return r.flow, r.vertex_side, r.net_side


def _pin_to(cpu):
    os.sched_setaffinity(0, {cpu})


def _maxflow_timed_worker(t):
    import time
    h = _Plain(t)
    t0 = time.perf_counter()
    r = maxflow(h)
    dt = time.perf_counter() - t0
    return r.flow, r.vertex_side, r.net_side, dt


def maxflow_pinned(hg, cpu=None):
    """``maxflow`` of one hypergraph in a fresh process pinned to one core
    (``cpu``, default the last core this process may use), timed there
    around the solve and the source-side BFS only.  Returns (F, vertex_side,
    net_side, seconds, cpu)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    if cpu is None:
        cpu = max(os.sched_getaffinity(0))
    t = (int(hg.num_vertices), np.ascontiguousarray(hg.net_offsets), np.ascontiguousarray(hg.pins),
         np.ascontiguousarray(hg.net_weights), np.ascontiguousarray(hg.sources),
         np.ascontiguousarray(hg.sinks))
    with cf.ProcessPoolExecutor(max_workers=1, mp_context=mp.get_context("spawn"),
                                initializer=_pin_to, initargs=(cpu,)) as ex:
        F, vs, ns, dt = ex.submit(_maxflow_timed_worker, t).result()
    return F, vs, ns, dt, cpu


def maxflow_many(hgs, workers=None):
    """``maxflow`` of every hypergraph in ``hgs`` on a pool of ``workers``
    processes (started fresh, so a parent that holds a GPU context shares
    nothing with them).  Returns a list of (F, vertex_side, net_side)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    args = [(int(h.num_vertices), np.ascontiguousarray(h.net_offsets), np.ascontiguousarray(h.pins),
             np.ascontiguousarray(h.net_weights), np.ascontiguousarray(h.sources),
             np.ascontiguousarray(h.sinks)) for h in hgs]
    if workers <= 1 or len(args) <= 1:
        return [_maxflow_worker(a) for a in args]
    with cf.ProcessPoolExecutor(max_workers=workers,
                                mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_maxflow_worker, args, chunksize=max(1, len(args) // (4 * workers))))


def _pins_inside(hg, x):
    """Number of pins of each net that lie in x."""
    E = hg.num_nets
    net_of = np.repeat(np.arange(E), np.diff(hg.net_offsets))
    return np.bincount(net_of, weights=x[hg.pins].astype(np.float64),
                       minlength=E).astype(np.int64)


def cut_weight(hg, x) -> int:
    """Weight of the nets cut by source side ``x`` (bool per vertex): a net
    counts when it has a pin inside x and a pin outside x."""
    x = np.asarray(x, dtype=bool)
    inside = _pins_inside(hg, x)
    sizes = np.diff(hg.net_offsets)
    cut = (inside > 0) & (inside < sizes)
    return int(hg.net_weights[cut].astype(np.int64).sum())


def net_side_from_x(hg, x) -> np.ndarray:
    """bit 0 = net has a pin in x; bit 1 = all pins of the net lie in x
    (nets with at least one pin).  Empty nets get 0."""
    x = np.asarray(x, dtype=bool)
    inside = _pins_inside(hg, x)
    sizes = np.diff(hg.net_offsets)
    b0 = inside > 0
    b1 = (inside == sizes) & (sizes > 0)
    return (b0.astype(np.uint8) | (b1.astype(np.uint8) << 1)).astype(np.uint8)


def brute_force(hg):
    """(F, minimal source side) by enumerating all feasible source sides.

    Only for hypergraphs whose free vertices number at most 16.
    Returns (F, x_min bool array, number of minimisers).
    """
    V = hg.num_vertices
    S = set(int(v) for v in hg.sources)
    T = set(int(v) for v in hg.sinks)
    free = [v for v in range(V) if v not in S and v not in T]
    if len(free) > 16:
        raise ValueError("brute force limited to 16 free vertices")
    nets = [set(int(v) for v in n) for n in hg.nets()]
    w = [int(c) for c in hg.net_weights]
    best = None
    x_min = None
    count = 0
    for mask in range(1 << len(free)):
        X = set(S)
        for i, v in enumerate(free):
            if mask >> i & 1:
                X.add(v)
        c = 0
        for n, we in zip(nets, w):
            k = len(n & X)
            if 0 < k < len(n):
                c += we
        if best is None or c < best:
            best, x_min, count = c, set(X), 1
        elif c == best:
            x_min &= X
            count += 1
    x = np.zeros(V, dtype=bool)
    for v in x_min:
        x[v] = True
    return best, x, count


def brute_force_sides(hg):
    """(F, minimal minimiser, maximal minimiser) by enumeration (<= 16 free
    vertices).  The maximal minimiser is the union of all minimisers; its
    complement is the maximal sink side."""
    V = hg.num_vertices
    S = set(int(v) for v in hg.sources)
    T = set(int(v) for v in hg.sinks)
    free = [v for v in range(V) if v not in S and v not in T]
    if len(free) > 16:
        raise ValueError("brute force limited to 16 free vertices")
    nets = [set(int(v) for v in n) for n in hg.nets()]
    w = [int(c) for c in hg.net_weights]
    best, lo, hi = None, None, None
    for mask in range(1 << len(free)):
        X = set(S) | {v for i, v in enumerate(free) if mask >> i & 1}
        c = sum(we for n, we in zip(nets, w) if 0 < len(n & X) < len(n))
        if best is None or c < best:
            best, lo, hi = c, set(X), set(X)
        elif c == best:
            lo &= X
            hi |= X
    xl = np.zeros(V, dtype=bool)
    xh = np.zeros(V, dtype=bool)
    xl[list(lo)] = True
    xh[list(hi)] = True
    return best, xl, xh


def _lawler_arcs(hg):
    """Explicit Lawler arcs (tail, head, capacity) with super terminals."""
    V, E = hg.num_vertices, hg.num_nets
    inf = 1 + int(hg.net_weights.astype(np.int64).sum())
    sig, tau = V + 2 * E, V + 2 * E + 1
    arcs = []
    for e, n in enumerate(hg.nets()):
        for v in n:
            arcs.append((int(v), V + e, inf))
            arcs.append((V + E + e, int(v), inf))
        arcs.append((V + e, V + E + e, int(hg.net_weights[e])))
    for v in hg.sources:
        arcs.append((sig, int(v), inf))
    for v in hg.sinks:
        arcs.append((int(v), tau, inf))
    return arcs, V + 2 * E + 2, sig, tau, inf


def _sides_from_reached(hg, reached):
    V, E = hg.num_vertices, hg.num_nets
    x = np.array([bool(reached[v]) for v in range(V)], dtype=bool)
    nside = np.array([int(reached[V + e]) | (int(reached[V + E + e]) << 1)
                      for e in range(E)], dtype=np.uint8)
    return x, nside


def edmonds_karp(hg):
    """Shortest-augmenting-path max flow (Edmonds & Karp) on the explicit
    Lawler graph; source side by BFS from the super source in the residual
    graph of the final flow.  Returns (F, x bool[V], net_side uint8[E])."""
    arcs, n, sig, tau, inf = _lawler_arcs(hg)
    res = {}
    adj = [set() for _ in range(n)]
    for a, b, c in arcs:
        res[(a, b)] = res.get((a, b), 0) + c
        res.setdefault((b, a), 0)
        adj[a].add(b)
        adj[b].add(a)
    adj = [sorted(s) for s in adj]
    F = 0
    while True:
        parent = [-1] * n
        parent[sig] = sig
        q = deque([sig])
        while q and parent[tau] < 0:
            u = q.popleft()
            for v in adj[u]:
                if parent[v] < 0 and res[(u, v)] > 0:
                    parent[v] = u
                    q.append(v)
        if parent[tau] < 0:
            break
        b, v = None, tau
        while v != sig:
            u = parent[v]
            b = res[(u, v)] if b is None else min(b, res[(u, v)])
            v = u
        v = tau
        while v != sig:
            u = parent[v]
            res[(u, v)] -= b
            res[(v, u)] += b
            v = u
        F += b
    reached = [False] * n
    reached[sig] = True
    q = deque([sig])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if not reached[v] and res[(u, v)] > 0:
                reached[v] = True
                q.append(v)
    x, nside = _sides_from_reached(hg, reached)
    return F, x, nside


def scipy_maxflow(hg, method: str = "dinic"):
    """Max flow through ``scipy.sparse.csgraph.maximum_flow`` on the explicit
    Lawler graph (int32 capacities), then BFS from the super source over the
    residual graph.  Returns (F, x bool[V], net_side uint8[E])."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_flow
    arcs, n, sig, tau, inf = _lawler_arcs(hg)
    if inf >= 2**31:
        raise ValueError("capacities exceed int32")
    a = np.array(arcs, dtype=np.int64).reshape(-1, 3)
    cap = sp.csr_matrix((a[:, 2].astype(np.int32), (a[:, 0], a[:, 1])), shape=(n, n))
    r = maximum_flow(cap, sig, tau, method=method)
    flow = r.flow.tocsr()
    resid = (cap.astype(np.int64) - flow.astype(np.int64)).tocsr()
    resid.eliminate_zeros()
    reached = np.zeros(n, dtype=bool)
    reached[sig] = True
    q = deque([sig])
    while q:
        u = q.popleft()
        lo, hi = resid.indptr[u], resid.indptr[u + 1]
        for v, c in zip(resid.indices[lo:hi], resid.data[lo:hi]):
            if c > 0 and not reached[v]:
                reached[v] = True
                q.append(v)
    x, nside = _sides_from_reached(hg, reached)
    return int(r.flow_value), x, nside


# ---------------------------------------------------------------------------
# checks of an exported flow state of the capped network
#
# State per pin slot p of net e with vertex u:
#   f_in[p]  = flow on (u, e_in)    0 <= f_in <= w(e)   (capacity restricted)
#   f_out[p] = flow on (e_out, u)   >= 0
# per net: f_b[e] = flow on (e_in, e_out), 0 <= f_b <= w(e); a net with a
# source pin receives w(e) from the contracted source, sinks absorb
# everything pushed into them.
# ---------------------------------------------------------------------------

def check_preflow(hg, f_in, f_out, f_b, flow_value):
    """Return a list of violated preflow conditions (empty if feasible)."""
    V, E = hg.num_vertices, hg.num_nets
    off = hg.net_offsets
    w = hg.net_weights.astype(np.int64)
    f_in = np.asarray(f_in, dtype=np.int64)
    f_out = np.asarray(f_out, dtype=np.int64)
    f_b = np.asarray(f_b, dtype=np.int64)
    role = np.zeros(V, dtype=np.int8)
    role[hg.sources] = 1
    role[hg.sinks] = 2
    net_of = np.repeat(np.arange(E), np.diff(off))
    errs = []
    if (f_in < 0).any() or (f_in > w[net_of]).any():
        errs.append("f_in outside [0, w]")
    if (f_out < 0).any():
        errs.append("negative f_out")
    if (f_b < 0).any() or (f_b > w).any():
        errs.append("f_b outside [0, w]")
    term_pin = role[hg.pins] != 0
    if (f_in[term_pin] != 0).any():
        errs.append("flow leaves a terminal through a pin arc")
    if (f_out[role[hg.pins] == 1] != 0).any():
        errs.append("flow enters a source vertex")
    has_s = np.zeros(E, dtype=bool)
    if len(net_of):
        has_s = np.bincount(net_of, weights=(role[hg.pins] == 1), minlength=E) > 0
    ex_in = np.bincount(net_of, weights=f_in, minlength=E) + np.where(has_s, w, 0) - f_b
    ex_out = f_b - np.bincount(net_of, weights=f_out, minlength=E)
    ex_v = np.bincount(hg.pins, weights=f_out - f_in, minlength=V)
    if (ex_in < 0).any() or (ex_out < 0).any():
        errs.append("negative excess at a net node")
    if (ex_v[role == 0] < 0).any():
        errs.append("negative excess at a vertex")
    into_t = int(f_out[role[hg.pins] == 2].sum())
    if into_t != int(flow_value):
        errs.append(f"flow value {flow_value} != flow into sinks {into_t}")
    return errs


def residual_labels(hg, f_in, f_out, f_b):
    """Exact distance to the sink set in the residual graph of the capped
    network, as three arrays (vertices, e_in, e_out).  Unreachable nodes get
    -1, source vertices -2 (never labelled), sinks 0."""
    V, E = hg.num_vertices, hg.num_nets
    off = hg.net_offsets
    w = hg.net_weights.astype(np.int64)
    role = np.zeros(V, dtype=np.int8)
    role[hg.sources] = 1
    role[hg.sinks] = 2
    dv = np.full(V, -1, dtype=np.int64)
    din = np.full(E, -1, dtype=np.int64)
    dout = np.full(E, -1, dtype=np.int64)
    dv[role == 1] = -2
    inc = [[] for _ in range(V)]
    for e in range(E):
        for p in range(off[e], off[e + 1]):
            inc[hg.pins[p]].append((e, p))
    q = deque()
    for t in np.nonzero(role == 2)[0]:
        dv[t] = 0
        q.append(("v", int(t)))
    while q:
        kind, a = q.popleft()
        if kind == "v":
            lvl = dv[a]
            for e, p in inc[a]:
                if dout[e] == -1:                     # (e_out, u) infinite
                    dout[e] = lvl + 1
                    q.append(("o", e))
                if din[e] == -1 and f_in[p] > 0:      # reverse of (u, e_in)
                    din[e] = lvl + 1
                    q.append(("i", e))
        elif kind == "i":
            lvl = din[a]
            for p in range(off[a], off[a + 1]):
                u = hg.pins[p]
                if dv[u] == -1 and f_in[p] < w[a]:    # (u, e_in) capped at w
                    dv[u] = lvl + 1
                    q.append(("v", int(u)))
            if dout[a] == -1 and f_b[a] > 0:          # reverse bridge
                dout[a] = lvl + 1
                q.append(("o", a))
        else:
            lvl = dout[a]
            if din[a] == -1 and f_b[a] < w[a]:        # bridge
                din[a] = lvl + 1
                q.append(("i", a))
            for p in range(off[a], off[a + 1]):
                u = hg.pins[p]
                if dv[u] == -1 and f_out[p] > 0:      # reverse of (e_out, u)
                    dv[u] = lvl + 1
                    q.append(("v", int(u)))
    return dv, din, dout


# ---------------------------------------------------------------------------
# FlowCutter (section "Flow-Based Refinement", algorithm "FlowCutter Core",
# paragraph "Piercing")
# ---------------------------------------------------------------------------

class _WithTerminals:
    """The hypergraph of ``hg`` with the terminal sets S, T (bool masks)."""

    def __init__(self, hg, S, T):
        self.num_vertices = hg.num_vertices
        self.num_nets = hg.num_nets
        self.net_offsets = hg.net_offsets
        self.pins = hg.pins
        self.net_weights = hg.net_weights
        self.sources = np.nonzero(S)[0].astype(np.int32)
        self.sinks = np.nonzero(T)[0].astype(np.int32)


class FlowCutterResult:
    def __init__(self, status, flow, x, iterations, trace, S, T, counts=None, first_balanced=0):
        self.status = status          # "balanced", "infeasible" or "cap"
        self.flow = int(flow)         # cut weight of the returned bipartition
        self.vertex_side = x          # bool per vertex: the returned source side
        self.iterations = iterations  # max-flow computations
        self.trace = trace            # per iteration (side, node, F, c(S_r), c(T_r))
        self.counts = counts          # per iteration: vertices pierced (0 at the end)
        self.sources = S
        self.sinks = T
        self.first_balanced = first_balanced  # iteration of the first balanced cut (0: none)


def _cut_nets(hg, side):
    """Nets with a pin inside ``side`` and a pin outside (bool per net)."""
    inside = _pins_inside(hg, side)
    sizes = np.diff(hg.net_offsets)
    return (inside > 0) & (inside < sizes)


def _piercing_node(hg, cut, sr, tr, own_terminals_side):
    """Piercing vertex, in order of preference: the smallest-id pin outside
    S_r and T_r of a net cut by the pierced side's bipartition (a boundary
    vertex that avoids an augmenting path); the smallest-id vertex outside
    S_r and T_r anywhere (still no augmenting path); the smallest-id pin of
    such a cut net on the opposite side that is not yet a terminal (creates
    an augmenting path).  (-1, False) if there is none."""
    E = hg.num_nets
    net_of = np.repeat(np.arange(E), np.diff(hg.net_offsets))
    on_cut = cut[net_of]
    pins = hg.pins[on_cut]
    free = pins[~sr[pins] & ~tr[pins]]
    if free.size:
        return int(free.min()), False
    anywhere = np.nonzero(~sr & ~tr)[0]
    if anywhere.size:
        return int(anywhere[0]), False
    aug = pins[own_terminals_side[pins]]
    if aug.size:
        return int(aug.min()), True
    return -1, False


# Pierces of a side made one vertex at a time before bulk piercing starts
# measuring (paragraph "Bulk Piercing": one node for the first few rounds).
BULK_WARMUP = 3


def _augmenting_candidates(hg, cut, own_terminals_side):
    """Sorted distinct pins of cut nets that lie on the other side and are
    not terminals yet (each creates an augmenting path)."""
    net_of = np.repeat(np.arange(hg.num_nets), np.diff(hg.net_offsets))
    pins = hg.pins[cut[net_of]]
    return np.unique(pins[own_terminals_side[pins]])


def flowcutter(hg, vertex_weights, max_source_weight, max_sink_weight,
               max_iterations=100000, bulk_percent=0, most_balanced=False):
    """FlowCutter, one piercing node per iteration or, with bulk_percent > 0,
    bulk piercing (paragraph "Bulk Piercing" of the section "Flow-Based
    Refinement").

    Each iteration solves the max flow of the current (S, T) from scratch
    (warm starting changes only the work, not F, S_r or T_r, which the
    current terminal sets determine), derives the minimal source side S_r
    and the maximal sink side T_r, and returns the first balanced
    bipartition, trying (S_r, V \\ S_r) before (V \\ T_r, T_r).  Otherwise the
    lighter of S_r and T_r (source side on ties) becomes the new terminal
    set plus one piercing node: the smallest-id pin, outside S_r and T_r, of
    a net cut by that side's bipartition; if there is none, the smallest-id
    vertex outside S_r and T_r anywhere; if there is none, the smallest-id
    such cut-net pin on the other side that is not yet a terminal (it
    creates an augmenting path).  Balanced: c(X) <= max_source_weight and
    c(V \\ X) <= max_sink_weight.

    Bulk piercing, in integer arithmetic (beta = bulk_percent / 100): only
    when the pierced side has no candidate that avoids an augmenting path,
    and after that side's first BULK_WARMUP pierces.  Each side keeps its
    own measurement -- weight its reachable set gained per pierced vertex,
    the gain taken at the next iteration -- and its own goal: the term
    starts at c(V) // 2 - c(side) when the side first bulk-pierces and is
    multiplied by beta every bulk iteration; the goal is the term plus what
    the previous goal missed.  The side then takes the
    max(1, goal * pierced // gained) smallest-id augmenting candidates (all
    of them if fewer).  The trace names the smallest one.

    Most balanced cut (paragraph "Most Balanced Cut"), with most_balanced:
    from the first balanced iteration on, the run keeps piercing while no
    augmenting path is created -- the lighter side takes its free boundary
    pin, else any free vertex, by the rule above -- and stops when neither
    side has a vertex outside S_r and T_r left (or at the iteration cap).
    Every iteration offers (S_r, V \\ S_r) and (V \\ T_r, T_r); among the
    balanced ones seen, the one with the lightest heavier side max(c(X),
    c(V \\ X)) is returned (the first one found on ties).  The cut weight
    stays the flow value of the first balanced iteration.  The paper repeats
    this with randomized choices; here one pass follows the deterministic
    smallest-id rule.
    """
    V = hg.num_vertices
    c = np.asarray(vertex_weights, dtype=np.int64)
    total = int(c.sum())
    S = np.zeros(V, dtype=bool)
    T = np.zeros(V, dtype=bool)
    S[hg.sources] = True
    T[hg.sinks] = True
    trace, counts = [], []
    pierces = [0, 0]   # pierces made per side
    gained = [0, 0]    # measured weight gained per side ...
    pierced = [0, 0]   # ... by this many pierced vertices
    term = [None, None]
    missed = [0, 0]
    pending = None     # (side, c(side) before its pierce, vertices, goal)
    best = None        # most balanced cut so far: (heavier side, X, F)
    first_balanced = 0
    for it in range(1, max_iterations + 1):
        r = maxflow(_WithTerminals(hg, S, T), sink_side=True)
        sr = r.vertex_side.astype(bool)
        tr = r.sink_side.astype(bool)
        cs, ct = int(c[sr].sum()), int(c[tr].sum())
        if pending is not None:
            s, before, k, goal = pending
            gain = max(0, (cs if s == 0 else ct) - before)
            gained[s] += gain
            pierced[s] += k
            if goal is not None:
                missed[s] = max(0, goal - gain)
            pending = None
        balanced = []
        if cs <= max_source_weight and total - cs <= max_sink_weight:
            balanced.append(sr)
        if total - ct <= max_source_weight and ct <= max_sink_weight:
            balanced.append(~tr)
        if balanced and not most_balanced:
            trace.append((-1, -1, r.flow, cs, ct))
            counts.append(0)
            return FlowCutterResult("balanced", r.flow, balanced[0], it, trace, S, T, counts,
                                    it)
        side = 0 if cs <= ct else 1
        own, mine = (sr, tr & ~T) if side == 0 else (tr, sr & ~S)
        cut = _cut_nets(hg, own)
        p, aug = _piercing_node(hg, cut, sr, tr, mine)
        if balanced or best is not None:
            if best is None:
                first_balanced = it
            for x in balanced:
                cx = int(c[x].sum())
                heavier = max(cx, total - cx)
                if best is None or heavier < best[0]:
                    best = (heavier, x.copy(), r.flow)
            if p < 0 or aug:
                trace.append((-1, -1, r.flow, cs, ct))
                counts.append(0)
                return FlowCutterResult("balanced", best[2], best[1], it, trace, S, T, counts,
                                        first_balanced)
            trace.append((side, p, r.flow, cs, ct))
            counts.append(1)
            if side == 0:
                S = sr.copy()
                S[p] = True
            else:
                T = tr.copy()
                T[p] = True
            continue
        trace.append((side, p, r.flow, cs, ct))
        if p < 0:
            counts.append(0)
            x = sr if side == 0 else ~tr
            return FlowCutterResult("infeasible", r.flow, x, it, trace, S, T, counts)
        nodes = np.array([p])
        goal = None
        weight = cs if side == 0 else ct
        if (aug and bulk_percent > 0 and pierces[side] >= BULK_WARMUP
                and gained[side] > 0):
            if term[side] is None:
                term[side] = max(0, total // 2 - weight)
            term[side] = term[side] * bulk_percent // 100
            goal = term[side] + missed[side]
            k = max(1, goal * pierced[side] // gained[side])
            nodes = _augmenting_candidates(hg, cut, mine)[:k]
        counts.append(int(nodes.size))
        pierces[side] += 1
        pending = (side, weight, int(nodes.size), goal)
        if side == 0:
            S = sr.copy()
            S[nodes] = True
        else:
            T = tr.copy()
            T[nodes] = True
    if best is not None:
        return FlowCutterResult("balanced", best[2], best[1], max_iterations, trace, S, T,
                                counts, first_balanced)
    return FlowCutterResult("cap", trace[-1][2], sr, max_iterations, trace, S, T, counts)
