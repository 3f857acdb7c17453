"""Pins of the oracle's two flow-state checkers, ``check_preflow`` and
``residual_labels``, against things other than themselves.

The GPU parity test of exact global-relabel labels and preflow feasibility
uses these two functions as its only judges, so they are pinned here:

* random preflows of the capped Lawler network (every arc u -> e_in carries
  at most w(e); a net with a source pin starts with w(e) in e_in), made by
  random feasible pushes on an explicitly built arc list, must pass
  ``check_preflow``; states with one planted violation of each preflow
  condition must be reported with that condition;
* ``residual_labels`` must equal the shortest-path distances to the sink set
  computed by ``scipy.sparse.csgraph.dijkstra`` (unit weights) on the
  explicit residual graph of the same state, with source vertices removed
  (they are contracted into the source, whose label is never lowered);
* plausible mistakes planted into copies of both functions must each fail
  one of these pins.

Definitions: section "Preliminaries", paragraphs "Flows" and "Flows on
Hypergraphs" (Lawler expansion, residual network, preflow); section
"Parallel Maximum Flow Algorithm", paragraph "Restricting Capacities" (the
cap w(e) on u -> e_in) and the global relabeling (exact residual distance
to the sink).
"""
import inspect

import numpy as np
import pytest

from paper_2201_01556_amd import inputs

INF = 1 << 40


class _State:
    """A preflow of the capped network as the oracle's checkers take it."""

    def __init__(self, hg):
        V, E = hg.num_vertices, hg.num_nets
        self.hg = hg
        self.f_in = np.zeros(hg.num_pins, dtype=np.int64)
        self.f_out = np.zeros(hg.num_pins, dtype=np.int64)
        self.f_b = np.zeros(E, dtype=np.int64)
        self.role = np.zeros(V, dtype=np.int8)
        self.role[hg.sources] = 1
        self.role[hg.sinks] = 2
        self.net_of = np.repeat(np.arange(E), np.diff(hg.net_offsets))
        self.w = hg.net_weights.astype(np.int64)
        # node ids of the explicit graph: v, e_in = V + e, e_out = V + E + e
        self.exc = np.zeros(V + 2 * E, dtype=np.int64)
        for e in range(E):
            p0, p1 = hg.net_offsets[e], hg.net_offsets[e + 1]
            if (self.role[hg.pins[p0:p1]] == 1).any():
                self.exc[V + e] += self.w[e]   # saturated contracted source arc
        self.flow_value = 0

    def arcs(self):
        """Every arc of the capped network as (tail, head, residual, kind,
        index): kind 'in' = (u, e_in) / reverse, 'out' = (e_out, u) /
        reverse, 'b' = bridge / reverse; ``index`` is the pin slot or net,
        ``sign`` +1 for the arc's own direction, -1 for its reverse."""
        hg, V, E = self.hg, self.hg.num_vertices, self.hg.num_nets
        out = []
        for p in range(hg.num_pins):
            e, u = int(self.net_of[p]), int(hg.pins[p])
            ein, eout = V + e, V + E + e
            out.append((u, ein, self.w[e] - self.f_in[p], "in", p, +1))
            out.append((ein, u, self.f_in[p], "in", p, -1))
            out.append((eout, u, INF - self.f_out[p], "out", p, +1))
            out.append((u, eout, self.f_out[p], "out", p, -1))
        for e in range(E):
            out.append((V + e, V + E + e, self.w[e] - self.f_b[e], "b", e, +1))
            out.append((V + E + e, V + e, self.f_b[e], "b", e, -1))
        return out

    def push(self, rng):
        """One random feasible push from a random non-terminal node with
        excess; returns False when no such push exists."""
        V = self.hg.num_vertices
        term = lambda x: x < V and self.role[x] != 0  # noqa: E731
        cands = [a for a in self.arcs()
                 if a[2] > 0 and self.exc[a[0]] > 0 and not term(a[0])
                 and not (a[1] < V and self.role[a[1]] == 1)]
        if not cands:
            return False
        tail, head, res, kind, idx, sign = cands[int(rng.integers(len(cands)))]
        amt = int(rng.integers(1, min(int(self.exc[tail]), int(res)) + 1))
        arr = {"in": self.f_in, "out": self.f_out, "b": self.f_b}[kind]
        arr[idx] += sign * amt
        self.exc[tail] -= amt
        self.exc[head] += amt
        if head < V and self.role[head] == 2:
            self.flow_value += amt
        return True


def _random_preflow(hg, seed, pushes):
    rng = np.random.Generator(np.random.PCG64(seed))
    st = _State(hg)
    for _ in range(pushes):
        if not st.push(rng):
            break
    return st


def _scipy_distances(st):
    """Residual distance of every node to the sink set by dijkstra with unit
    weights on the explicit residual graph (source vertices removed)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    hg, V, E = st.hg, st.hg.num_vertices, st.hg.num_nets
    n = V + 2 * E
    src = lambda x: x < V and st.role[x] == 1  # noqa: E731
    rows, cols = [], []
    for tail, head, res, *_ in st.arcs():
        if res > 0 and not src(tail) and not src(head):
            rows.append(head)      # reversed: distances *to* the sinks
            cols.append(tail)
    g = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    sinks = np.nonzero(st.role == 2)[0]
    d = dijkstra(g, directed=True, indices=sinks, unweighted=True, min_only=True)
    d = np.where(np.isinf(d), -1, d).astype(np.int64)
    d[:V][st.role == 1] = -2
    return d[:V], d[V:V + E], d[V + E:]


def _cases():
    cases = [(inputs.tiny_hypergraph(s), s, 40) for s in range(120)]
    cases += [(inputs.uniform_hypergraph(s, num_vertices=60, num_nets=90, num_sources=6,
                                         num_sinks=6), 1000 + s, 400)
              for s in range(6)]
    return cases


_STATES = None


def _states():
    global _STATES
    if _STATES is None:
        _STATES = [_random_preflow(hg, seed, k) for hg, seed, k in _cases()]
    return _STATES


def test_random_preflows_are_nontrivial():
    """The generated states exercise every arc kind (otherwise the pins
    below would not see a wrong residual condition)."""
    sts = _states()
    assert sum(int((s.f_in > 0).sum()) for s in sts) > 200
    assert sum(int((s.f_out > 0).sum()) for s in sts) > 200
    assert sum(int(((s.f_b > 0) & (s.f_b < s.w)).sum()) for s in sts) > 20
    assert sum(int((s.f_b == s.w).sum()) for s in sts) > 50
    assert sum(int((s.f_in == s.w[s.net_of]).sum()) for s in sts) > 50
    assert sum(s.flow_value > 0 for s in sts) > 30
    # some states keep excess in the middle of the network (a preflow, not a flow)
    V = [s.hg.num_vertices for s in sts]
    assert sum(int((s.exc[v:] > 0).sum()) for s, v in zip(sts, V)) > 20


def _violations(st):
    """(name, state arrays, flow value, expected message) with one planted
    violation each; every name is produced for some state of the set."""
    hg, V = st.hg, st.hg.num_vertices
    out = []
    base = (st.f_in, st.f_out, st.f_b)

    def mod(i, idx, delta):
        arrs = [a.copy() for a in base]
        arrs[i][idx] += delta
        return arrs

    w_pin = st.w[st.net_of]
    free_pin = st.role[hg.pins] == 0
    # f_in above the cap (the vertex then also loses excess)
    p = np.nonzero(free_pin)[0]
    if len(p):
        arrs = [a.copy() for a in base]
        arrs[0][p[0]] = w_pin[p[0]] + 1
        out.append(("cap", arrs, st.flow_value, "f_in outside [0, w]"))
    if hg.num_pins:
        out.append(("neg f_out", mod(1, 0, -(int(st.f_out[0]) + 1)), st.flow_value,
                    "negative f_out"))
    if hg.num_nets:
        arrs = [a.copy() for a in base]
        arrs[2][0] = st.w[0] + 1
        out.append(("bridge", arrs, st.flow_value, "f_b outside [0, w]"))
    sp = np.nonzero(st.role[hg.pins] == 2)[0]
    sp = [q for q in sp if st.f_in[q] < w_pin[q]]
    if sp:
        out.append(("sink pin", mod(0, sp[0], 1), st.flow_value,
                    "flow leaves a terminal through a pin arc"))
    sp = np.nonzero(st.role[hg.pins] == 1)[0]
    if len(sp):
        out.append(("source in", mod(1, sp[0], 1), st.flow_value, "flow enters a source vertex"))
    # a net node that would hold negative excess
    ex_in = st.exc[V:V + hg.num_nets]
    e0 = np.nonzero((ex_in == 0) & (st.f_b < st.w))[0]
    if len(e0):
        out.append(("e_in", mod(2, e0[0], 1), st.flow_value, "negative excess at a net node"))
    ex_out = st.exc[V + hg.num_nets:]
    for e in np.nonzero(ex_out == 0)[0]:
        q = [q for q in range(hg.net_offsets[e], hg.net_offsets[e + 1])
             if st.role[hg.pins[q]] == 0]
        if q:
            out.append(("e_out", mod(1, q[0], 1), st.flow_value,
                        "negative excess at a net node"))
            break
    vz = [q for q in np.nonzero(free_pin)[0]
          if st.exc[hg.pins[q]] == 0 and st.f_in[q] < w_pin[q]]
    if vz:
        out.append(("vertex", mod(0, vz[0], 1), st.flow_value, "negative excess at a vertex"))
    out.append(("value", list(base), st.flow_value + 1, "flow value"))
    return out


def _check_all(check_preflow):
    """True when every valid state passes and every planted violation is
    reported with its message."""
    seen = set()
    for st in _states():
        if check_preflow(st.hg, st.f_in, st.f_out, st.f_b, st.flow_value):
            return False
        for name, (fi, fo, fb), fv, msg in _violations(st):
            errs = check_preflow(st.hg, fi, fo, fb, fv)
            if not any(e.startswith(msg) for e in errs):
                return False
            seen.add(name)
    return len(seen) == 9


def test_check_preflow_pinned(oracle_mod):
    assert _check_all(oracle_mod.check_preflow)


def _labels_agree(residual_labels):
    for st in _states():
        got = residual_labels(st.hg, st.f_in, st.f_out, st.f_b)
        exp = _scipy_distances(st)
        for a, b in zip(got, exp):
            if not np.array_equal(np.asarray(a, dtype=np.int64), b):
                return False
    return True


def test_residual_labels_vs_scipy(oracle_mod):
    assert _labels_agree(oracle_mod.residual_labels)


def _uncapped_reach(st):
    """Nodes that reach the sink set in the residual graph of the uncapped
    network (the pin arcs u -> e_in without the cap w(e)), source vertices
    removed: one bool per node of the explicit graph."""
    hg, V, E = st.hg, st.hg.num_vertices, st.hg.num_nets
    n = V + 2 * E
    src = lambda x: x < V and st.role[x] == 1  # noqa: E731
    into = [[] for _ in range(n)]
    for tail, head, res, kind, _, sign in st.arcs():
        if kind == "in" and sign == +1:
            res = INF  # uncapped
        if res > 0 and not src(tail) and not src(head):
            into[head].append(tail)
    seen = np.zeros(n, dtype=bool)
    stack = [int(t) for t in np.nonzero(st.role == 2)[0]]
    seen[stack] = True
    while stack:
        x = stack.pop()
        for y in into[x]:
            if not seen[y]:
                seen[y] = True
                stack.append(y)
    return seen


def test_sink_side_from_capped_labels():
    """The reading behind the sink side derived from exact labels: the nodes
    with a finite residual distance in the capped network (set D) all reach
    the sinks in the uncapped network, and the uncapped network's sink side
    is D plus what reaches a seed through its residual arcs, a seed being a
    non-source vertex outside D with a saturated arc u -> e_in into an e_in
    of D (the only arcs the two networks differ in).  Distances by scipy on
    the explicit graph, the uncapped side by search on the explicit graph,
    over random preflows."""
    # a state where they differ: the source 0 sends one unit through net 0
    # to vertex 1, which pushes it into net 1 (its arc into e_in saturated);
    # net 1's e_in reaches the sink 2 over the bridge, vertex 1 only through
    # that saturated arc
    hand = _State(inputs.hypergraph_from_nets(3, [[0, 1], [1, 2]], [1, 1], [0], [2]))
    hand.f_b[0] = 1
    hand.f_out[1] = 1     # slot 1 = (net 0, vertex 1)
    hand.f_in[2] = 1      # slot 2 = (net 1, vertex 1)
    grew = 0
    for k, st in enumerate([hand] + _states()):
        hg, V, E = st.hg, st.hg.num_vertices, st.hg.num_nets
        dv, din, dout = _scipy_distances(st)
        D = np.concatenate([dv >= 0, din >= 0, dout >= 0])
        T = _uncapped_reach(st)
        assert not (D & ~T).any()
        seeds = set()
        for p in range(hg.num_pins):
            e, u = int(st.net_of[p]), int(hg.pins[p])
            if st.f_in[p] == st.w[e] and D[V + e] and not D[u] and st.role[u] != 1:
                seeds.add(u)
        # reverse search of the uncapped residual graph from the seeds
        into = [[] for _ in range(V + 2 * E)]
        src = lambda x: x < V and st.role[x] == 1  # noqa: E731
        for tail, head, res, kind, _, sign in st.arcs():
            if kind == "in" and sign == +1:
                res = INF
            if res > 0 and not src(tail) and not src(head):
                into[head].append(tail)
        got = D.copy()
        stack = sorted(seeds)
        got[stack] = True
        while stack:
            x = stack.pop()
            for y in into[x]:
                if not got[y]:
                    got[y] = True
                    stack.append(y)
        assert (got == T).all()
        if k == 0:  # vertex 1 and net 0's e_out (node 5), which reaches it
            assert np.nonzero(T & ~D)[0].tolist() == [1, 5] and seeds == {1}
        grew += int((T & ~D).sum() > 0)
    assert grew >= 1


CHECK_MUTANTS = {
    "contracted source arc ignored": ("+ np.where(has_s, w, 0) - f_b", "- f_b"),
    "cap off by one": ("(f_in > w[net_of]).any()", "(f_in > w[net_of] + 1).any()"),
    "e_out excess unchecked": ("if (ex_in < 0).any() or (ex_out < 0).any():",
                               "if (ex_in < 0).any():"),
    "vertex excess of sinks": ("(ex_v[role == 0] < 0)", "(ex_v[role == 2] < 0)"),
    "value counted at sources": ("into_t = int(f_out[role[hg.pins] == 2].sum())",
                                 "into_t = int(f_out[role[hg.pins] == 1].sum())"),
    "terminal pin arcs unchecked": ("if (f_in[term_pin] != 0).any():", "if False:"),
    "source inflow checked at sinks": ("if (f_out[role[hg.pins] == 1] != 0).any():",
                                       "if (f_out[role[hg.pins] == 2] != 0).any():"),
}

LABEL_MUTANTS = {
    "reverse pin arc always residual": ("if din[e] == -1 and f_in[p] > 0:",
                                        "if din[e] == -1 and f_in[p] >= 0:"),
    "pin arc uncapped": ("if dv[u] == -1 and f_in[p] < w[a]:", "if dv[u] == -1:"),
    # (the reverse bridge e_out -> e_in never decides a label: e_in is
    # labelled from e_out or from a pin u, and in the second case e_out
    # gets the same label from u through the infinite arc e_out -> u, so a
    # mistake in that condition cannot change a distance)
    "bridge reads the reverse residual": ("if din[a] == -1 and f_b[a] < w[a]:",
                                          "if din[a] == -1 and f_b[a] > 0:"),
    "bridge ignores its flow": ("if din[a] == -1 and f_b[a] < w[a]:",
                                "if din[a] == -1 and f_b[a] <= w[a]:"),
    "e_out pins read the wrong flow": ("if dv[u] == -1 and f_out[p] > 0:",
                                       "if dv[u] == -1 and f_in[p] > 0:"),
    "e_out one level too far": ("dout[e] = lvl + 1", "dout[e] = lvl + 2"),
    "sources relabelled": ("dv[role == 1] = -2", "dv[role == 1] = -1"),
}


def _mutant(oracle_mod, fn, old, new):
    src = inspect.getsource(fn)
    assert old in src, old
    ns = dict(vars(oracle_mod))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns[fn.__name__]


@pytest.mark.parametrize("name", sorted(CHECK_MUTANTS))
def test_check_preflow_catches_planted_mistakes(oracle_mod, name):
    old, new = CHECK_MUTANTS[name]
    m = _mutant(oracle_mod, oracle_mod.check_preflow, old, new)
    try:
        ok = _check_all(m)
    except Exception:
        ok = False
    assert not ok, f"mutant '{name}' passes the preflow pins"


@pytest.mark.parametrize("name", sorted(LABEL_MUTANTS))
def test_residual_labels_catch_planted_mistakes(oracle_mod, name):
    old, new = LABEL_MUTANTS[name]
    m = _mutant(oracle_mod, oracle_mod.residual_labels, old, new)
    try:
        ok = _labels_agree(m)
    except Exception:
        ok = False
    assert not ok, f"mutant '{name}' passes the label pins"
