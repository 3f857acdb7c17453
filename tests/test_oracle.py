"""Pins of the CPU oracle against things other than itself.

* hand-checked fixtures (tests/golden/fixtures.json);
* brute force over all source sides on tiny hypergraphs (max-flow = min-cut,
  minimal minimiser = intersection of all minimisers);
* a second max-flow algorithm (Edmonds-Karp on a separately built graph);
* library routines (scipy maximum_flow; networkx on the graph special case);
* closed forms (a net holding a source and a sink pin is always cut; S and T
  in different components give F = 0);
* the excess-seeded BFS against BFS from the source after returning all
  excess (the claim of the paragraph "Source-Side Cut").
* mutation check: plausible mistakes planted into a copy of the oracle's C
  source are caught by these pins.
"""
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2201_01556_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixtures():
    with open(os.path.join(HERE, "golden", "fixtures.json")) as f:
        return json.load(f)["cases"]


def _fixture_hg(c):
    return inputs.hypergraph_from_nets(c["V"], c["nets"], c["w"], c["S"], c["T"])


@pytest.mark.parametrize("case", _fixtures(), ids=lambda c: c["name"])
def test_fixture(oracle_mod, case):
    hg = _fixture_hg(case)
    x_exp = np.zeros(case["V"], dtype=bool)
    x_exp[case["x"]] = True
    # brute force agrees with the hand-derived value (pins the enumerator)
    F_bf, x_bf, _ = oracle_mod.brute_force(hg)
    assert F_bf == case["F"]
    assert (x_bf == x_exp).all()
    # the C oracle
    r = oracle_mod.maxflow(hg, selfcheck=True)
    assert r.flow == case["F"]
    assert (r.vertex_side.astype(bool) == x_exp).all()
    assert list(r.net_side) == case["net_side"]
    # Edmonds-Karp
    F_ek, x_ek, n_ek = oracle_mod.edmonds_karp(hg)
    assert F_ek == case["F"] and (x_ek == x_exp).all()
    assert list(n_ek) == case["net_side"]


@pytest.mark.parametrize("block", range(6))
def test_tiny_vs_brute_force_and_ek(oracle_mod, block):
    for seed in range(block * 100, block * 100 + 100):
        hg = inputs.tiny_hypergraph(seed)
        r = oracle_mod.maxflow(hg, selfcheck=True)
        F, x, _ = oracle_mod.brute_force(hg)
        assert r.flow == F, seed
        assert (r.vertex_side.astype(bool) == x).all(), seed
        assert (r.net_side == oracle_mod.net_side_from_x(hg, x)).all(), seed
        F_ek, x_ek, n_ek = oracle_mod.edmonds_karp(hg)
        assert F_ek == F and (x_ek == x).all() and (n_ek == r.net_side).all(), seed
        assert oracle_mod.cut_weight(hg, x) == F


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("method", ["dinic", "edmonds_karp"])
def test_scipy_crosscheck_uniform(oracle_mod, seed, method):
    hg = inputs.uniform_hypergraph(seed)
    r = oracle_mod.maxflow(hg, selfcheck=True)
    F, x, nside = oracle_mod.scipy_maxflow(hg, method=method)
    assert r.flow == F
    assert (r.vertex_side.astype(bool) == x).all()
    assert (r.net_side == nside).all()
    assert oracle_mod.cut_weight(hg, x) == F


def test_scipy_crosscheck_zipf_small(oracle_mod):
    hg = inputs.zipf_hypergraph(5, num_vertices=20000, num_nets=40000, size_hi=200)
    r = oracle_mod.maxflow(hg, selfcheck=True)
    F, x, nside = oracle_mod.scipy_maxflow(hg)
    assert r.flow == F and (r.vertex_side.astype(bool) == x).all()
    assert (r.net_side == nside).all()


def test_graph_special_case_networkx(oracle_mod):
    """All nets of size 2: the hypergraph cut is the undirected graph cut."""
    nx = pytest.importorskip("networkx")
    for seed in range(5):
        rng = np.random.Generator(np.random.PCG64(1000 + seed))
        V = 60
        nets, w = [], []
        for _ in range(150):
            a, b = rng.choice(V, 2, replace=False)
            nets.append([int(a), int(b)])
            w.append(int(rng.integers(1, 10)))
        perm = rng.permutation(V)
        hg = inputs.hypergraph_from_nets(V, nets, w, np.sort(perm[:5]), np.sort(perm[5:10]))
        G = nx.DiGraph()
        for (a, b), c in zip(nets, w):
            for u, v in ((a, b), (b, a)):
                G.add_edge(u, v, capacity=G.get_edge_data(u, v, {"capacity": 0})["capacity"] + c)
        for s in hg.sources:
            G.add_edge("s", int(s))          # no capacity attribute = infinite
        for t in hg.sinks:
            G.add_edge(int(t), "t")
        val, flow = nx.maximum_flow(G, "s", "t")
        # minimal source side: BFS from s over the residual of networkx's flow
        seen = {"s"}
        stack = ["s"]
        while stack:
            u = stack.pop()
            for v in list(G.successors(u)) + list(G.predecessors(u)):
                cap = G[u][v].get("capacity", float("inf")) if G.has_edge(u, v) else 0
                r = cap - flow[u].get(v, 0) + (flow[v].get(u, 0) if G.has_edge(v, u) else 0)
                if v not in seen and r > 0:
                    seen.add(v)
                    stack.append(v)
        x_nx = np.array([v in seen for v in range(V)])
        r = oracle_mod.maxflow(hg, selfcheck=True)
        assert r.flow == val
        assert (r.vertex_side.astype(bool) == x_nx).all()


def test_closed_form_st_net(oracle_mod):
    """A net with a source pin and a sink pin is cut by every feasible side."""
    for w in (1, 7, 2**30):
        hg = inputs.hypergraph_from_nets(4, [[0, 3], [1, 2]], [w, 1], [0], [3])
        r = oracle_mod.maxflow(hg, selfcheck=True)
        assert r.flow == w
        assert list(r.vertex_side) == [1, 0, 0, 0]


def test_closed_form_components(oracle_mod):
    """S and T in different components: F = 0 and x = the union of the
    components that touch S."""
    rng = np.random.Generator(np.random.PCG64(7))
    nets = []
    for _ in range(40):
        nets.append(sorted(rng.choice(20, 3, replace=False).tolist()))
    for _ in range(40):
        nets.append(sorted((20 + rng.choice(20, 3, replace=False)).tolist()))
    hg = inputs.hypergraph_from_nets(45, nets, np.ones(len(nets), int), [0, 1], [21, 22])
    r = oracle_mod.maxflow(hg, selfcheck=True)
    assert r.flow == 0
    # vertices connected to S through nets (plain graph search)
    reach = {0, 1}
    frontier = [0, 1]
    while frontier:
        u = frontier.pop()
        for n in nets:
            if u in n:
                for v in n:
                    if v not in reach:
                        reach.add(v)
                        frontier.append(v)
    x = np.zeros(45, dtype=bool)
    x[sorted(reach)] = True
    assert (r.vertex_side.astype(bool) == x).all()


def test_certificate_and_selfcheck_uniform(oracle_mod):
    for seed in range(10):
        hg = inputs.uniform_hypergraph(seed)
        r = oracle_mod.maxflow(hg, selfcheck=True)
        x = r.vertex_side.astype(bool)
        assert oracle_mod.cut_weight(hg, x) == r.flow
        assert (r.net_side == oracle_mod.net_side_from_x(hg, x)).all()
        assert x[hg.sources].all() and not x[hg.sinks].any()


def test_invalid_inputs(oracle_mod):
    hg = inputs.hypergraph_from_nets(3, [[0, 5]], [1], [0], [2])
    with pytest.raises(RuntimeError):
        oracle_mod.maxflow(hg)
    hg = inputs.hypergraph_from_nets(3, [[0, 1]], [0], [0], [2])
    with pytest.raises(RuntimeError):
        oracle_mod.maxflow(hg)


def test_generators_deterministic():
    a = inputs.uniform_hypergraph(3)
    b = inputs.uniform_hypergraph(3)
    c = inputs.uniform_hypergraph(4)
    assert a.sha256() == b.sha256() != c.sha256()
    z1 = inputs.zipf_hypergraph(1, num_vertices=5000, num_nets=10000, size_hi=100)
    z2 = inputs.zipf_hypergraph(1, num_vertices=5000, num_nets=10000, size_hi=100)
    assert z1.sha256() == z2.sha256()
    # pins distinct inside every net, terminals disjoint and of 1 % size
    off = z1.net_offsets
    for e in range(z1.num_nets):
        p = z1.pins[off[e]:off[e + 1]]
        assert len(np.unique(p)) == len(p)
    assert len(np.intersect1d(z1.sources, z1.sinks)) == 0
    assert len(z1.sources) == 50 == len(z1.sinks)
    sizes = np.diff(off)
    assert sizes.min() >= 2 and sizes.max() <= 100


def test_splitmix64_reference_values():
    """Published first outputs of splitmix64 seeded with 0: the generator's
    state advances by the golden-gamma constant and each output is the
    finaliser of the new state."""
    gamma = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        states = np.array([0, 1, 2], dtype=np.uint64) * gamma
    out = inputs.splitmix64(states)
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4
    assert int(out[2]) == 0x06C45D188009454F


# ---------------------------------------------------------------------------
# mutation check of the pins
# ---------------------------------------------------------------------------

def _cutter_cases():
    with open(os.path.join(HERE, "golden", "flowcutter.json")) as f:
        return json.load(f)["cases"]


def _run_cutter_case(fn, case):
    hg = inputs.hypergraph_from_nets(case["V"], case["nets"], case["w"], case["S"], case["T"])
    c = np.asarray(case.get("c", np.ones(case["V"])))
    kw = dict(bulk_percent=case.get("bulk_percent", 0))
    if case.get("most_balanced"):
        kw["most_balanced"] = True
    return fn(hg, c, case["max_source"], case["max_sink"], **kw)


def _counts_of(case):
    """Vertices pierced per iteration: as listed, else one per iteration."""
    if "counts" in case:
        return case["counts"]
    return [1] * (case["iterations"] - 1) + [0]


@pytest.mark.parametrize("case", _cutter_cases(), ids=lambda c: c["name"])
def test_flowcutter_fixture(oracle_mod, case):
    r = _run_cutter_case(oracle_mod.flowcutter, case)
    assert r.status == case["status"]
    assert r.flow == case["F"]
    assert np.nonzero(r.vertex_side)[0].tolist() == case["x"]
    assert r.iterations == case["iterations"]
    assert [list(t) for t in r.trace] == case["trace"]
    assert r.counts == _counts_of(case)
    if "first_balanced" in case:
        assert r.first_balanced == case["first_balanced"]


@pytest.mark.parametrize("block", range(3))
def test_sink_side_vs_brute_force(oracle_mod, block):
    """Maximal sink side = complement of the union of all minimisers."""
    for seed in range(block * 100, block * 100 + 100):
        hg = inputs.tiny_hypergraph(seed)
        F, xl, xh = oracle_mod.brute_force_sides(hg)
        r = oracle_mod.maxflow(hg, sink_side=True)
        assert r.flow == F, seed
        assert (r.vertex_side.astype(bool) == xl).all(), seed
        assert (r.sink_side.astype(bool) == ~xh).all(), seed


def test_flowcutter_tiny_invariants(oracle_mod):
    """On tiny inputs: every returned cut is a minimum cut of the final
    terminal sets (brute force), respects them and the balance bounds when
    balanced; flows never decrease; at most |V| iterations."""
    rng = np.random.default_rng(7)
    seen = set()
    for seed in range(300):
        hg = inputs.tiny_hypergraph(seed)
        V = hg.num_vertices
        c = rng.integers(1, 4, V)
        total = int(c.sum())
        L = (total + 1) // 2 + int(rng.integers(0, 3))
        r = oracle_mod.flowcutter(hg, c, L, L)
        seen.add(r.status)
        assert r.iterations <= V
        flows = [t[2] for t in r.trace]
        assert flows == sorted(flows), seed
        x = r.vertex_side.astype(bool)
        assert r.flow == oracle_mod.cut_weight(hg, x), seed
        assert x[r.sources].all() and not x[r.sinks].any(), seed
        fin = inputs.hypergraph_from_nets(V, [list(n) for n in hg.nets()], hg.net_weights,
                                          np.nonzero(r.sources)[0], np.nonzero(r.sinks)[0])
        assert oracle_mod.brute_force(fin)[0] == r.flow, seed
        if r.status == "balanced":
            assert int(c[x].sum()) <= L and total - int(c[x].sum()) <= L, seed
    assert seen >= {"balanced", "infeasible"}


def test_most_balanced_tiny_invariants(oracle_mod):
    """On tiny inputs the balance phase only adds pierces after the first
    balanced iteration: the run agrees with the plain run up to it, keeps
    its flow value (the plain run's, itself pinned by brute force), returns
    a cut of that weight that respects the original terminals and the
    bounds, and whose heavier side is no heavier than the plain run's."""
    rng = np.random.default_rng(17)
    improved = 0
    for seed in range(300):
        hg = inputs.tiny_hypergraph(seed)
        V = hg.num_vertices
        c = rng.integers(1, 4, V)
        total = int(c.sum())
        L = (total + 1) // 2 + int(rng.integers(0, 4))
        r0 = oracle_mod.flowcutter(hg, c, L, L)
        r = oracle_mod.flowcutter(hg, c, L, L, most_balanced=True)
        assert r.status == r0.status, seed
        if r0.status != "balanced":
            assert r.trace == r0.trace and r.first_balanced == 0, seed
            continue
        k = r0.iterations
        assert r.first_balanced == r0.first_balanced == k, seed
        assert r.trace[:k - 1] == r0.trace[:k - 1], seed
        assert r.iterations <= k + V, seed
        assert all(t[2] == r0.flow for t in r.trace[k - 1:]), seed
        assert all(n <= 1 for n in r.counts[k - 1:]), seed
        x = r.vertex_side.astype(bool)
        assert r.flow == r0.flow == oracle_mod.cut_weight(hg, x), seed
        assert x[hg.sources].all() and not x[hg.sinks].any(), seed
        cx = int(c[x].sum())
        assert cx <= L and total - cx <= L, seed
        x0 = r0.vertex_side.astype(bool)
        h0 = max(int(c[x0].sum()), total - int(c[x0].sum()))
        assert max(cx, total - cx) <= h0, seed
        improved += max(cx, total - cx) < h0
    assert improved >= 5


CUTTER_MUTANTS = {
    "pierce heavier side": ("side = 0 if cs <= ct else 1", "side = 0 if cs > ct else 1"),
    "largest id": ("return int(free.min()), False", "return int(free.max()), False"),
    "skip sink-side balance": ("if total - ct <= max_source_weight and ct <= max_sink_weight:",
                               "if False:"),
    "sink side = complement": ("tr = r.sink_side.astype(bool)", "tr = ~sr"),
    "no augmenting fallback": ("aug = pins[own_terminals_side[pins]]", "aug = pins[:0]"),
    "no free-vertex fallback": ("anywhere = np.nonzero(~sr & ~tr)[0]", "anywhere = pins[:0]"),
    "bulk without warm-up": ("pierces[side] >= BULK_WARMUP", "pierces[side] >= 0"),
    "bulk on free vertices": ("if (aug and bulk_percent > 0", "if (bulk_percent > 0"),
    "bulk ratio inverted": ("k = max(1, goal * pierced[side] // gained[side])",
                            "k = max(1, goal * gained[side] // pierced[side])"),
    "bulk term from c(V)": ("term[side] = max(0, total // 2 - weight)",
                            "term[side] = max(0, total - weight)"),
    "bulk forgets the missed goal": ("goal = term[side] + missed[side]", "goal = term[side]"),
    "balance ties take the later cut": ("if best is None or heavier < best[0]:",
                                        "if best is None or heavier <= best[0]:"),
    "balance phase pierces augmenting": ("if p < 0 or aug:", "if p < 0:"),
    "balance phase ignores the sink side": ("            for x in balanced:\n",
                                            "            for x in balanced[:1]:\n"),
    "balance phase keeps the first cut": ("                    best = (heavier, x.copy(), r.flow)",
                                          "                    best = best or (heavier, x.copy(), r.flow)"),
    "balance phase starts late": ("                first_balanced = it", "                first_balanced = it + 1"),
}


@pytest.mark.parametrize("name", sorted(CUTTER_MUTANTS))
def test_flowcutter_pins_catch_planted_mistakes(oracle_mod, name):
    """A copy of the oracle's FlowCutter with one planted mistake must fail
    at least one hand-derived fixture."""
    import inspect
    old, new = CUTTER_MUTANTS[name]
    src = inspect.getsource(oracle_mod._piercing_node) + "\n" + inspect.getsource(
        oracle_mod.flowcutter)
    assert old in src
    ns = dict(vars(oracle_mod))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    failed = False
    for case in _cutter_cases():
        try:
            r = _run_cutter_case(ns["flowcutter"], case)
            ok = (r.status == case["status"] and r.flow == case["F"] and
                  [list(t) for t in r.trace] == case["trace"] and
                  r.counts == _counts_of(case) and
                  np.nonzero(r.vertex_side)[0].tolist() == case["x"] and
                  r.first_balanced == case.get("first_balanced", r.first_balanced))
        except Exception:
            ok = False
        failed |= not ok
    assert failed, f"mutant '{name}' passes every FlowCutter fixture"


MUTANTS = {
    "bridge capacity off by one": ("ADD_ARC(ein, eout, (int64_t)w[e]);",
                                   "ADD_ARC(ein, eout, (int64_t)w[e] + 1);"),
    "pin arc transposed": ("ADD_ARC(eout, pins[p], inf);",
                           "ADD_ARC(pins[p], eout, inf);"),
    "source side not seeded with excess": ("forward_bfs(&s, reached, 1);",
                                           "forward_bfs(&s, reached, 0);"),
    "reverse BFS reads the forward arc": ("g->cap[g->rev[a]] > 0) {",
                                          "g->cap[a] > 0) {"),
    "sink arcs with zero capacity": ("for (int32_t i = 0; i < nT; ++i) ADD_ARC(T[i], tau, inf);",
                                     "for (int32_t i = 0; i < nT; ++i) ADD_ARC(T[i], tau, 0);"),
    "net-side bits swapped": ("(reached[V + e] | (reached[V + E + e] << 1))",
                              "(reached[V + E + e] | (reached[V + e] << 1))"),
    "source arcs start unsaturated": ("    g.cap[a] = 0;\n    g.cap[g.rev[a]] += c;\n    s.exc[g.head[a]] += c;",
                                      "    (void)c;"),
}


def _build_mutant(tmp, old, new):
    src = open(os.path.join(os.path.dirname(HERE), "oracle", "lawler_pr.c")).read()
    assert old in src, old
    path = os.path.join(tmp, "m.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmp, "liboracle.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, path])
    return so


_MUTANT_RUNNER = r"""
import importlib.util, json, os, sys
import numpy as np
root, so = sys.argv[1], sys.argv[2]
sys.path.insert(0, root)
from paper_2201_01556_amd import inputs
import oracle as good
spec = importlib.util.spec_from_file_location("oracle_mutant", os.path.join(root, "oracle", "__init__.py"))
mod = importlib.util.module_from_spec(spec)
spec.loader.exec_module(mod)
mod._LIB_PATH = so
mod._lib = None
cases = [inputs.hypergraph_from_nets(c["V"], c["nets"], c["w"], c["S"], c["T"])
         for c in json.load(open(os.path.join(root, "tests", "golden", "fixtures.json")))["cases"]]
cases += [inputs.tiny_hypergraph(s) for s in range(60)]
for hg in cases:
    try:
        r = mod.maxflow(hg)
    except RuntimeError:
        sys.exit(3)
    F, x, _ = good.brute_force(hg)
    if r.flow != F or (r.vertex_side.astype(bool) != x).any():
        sys.exit(3)
    if (r.net_side != good.net_side_from_x(hg, x)).any():
        sys.exit(3)
sys.exit(0)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(oracle_mod, name):
    """Each mutant must fail a pin: a wrong answer, an error code, or a
    crash of the child process that runs it all count as caught."""
    import sys
    old, new = MUTANTS[name]
    tmp = tempfile.mkdtemp()
    try:
        so = _build_mutant(tmp, old, new)
        root = os.path.dirname(HERE)
        rc = subprocess.run([sys.executable, "-c", _MUTANT_RUNNER, root, so],
                            capture_output=True, timeout=300).returncode
        assert rc != 0, f"mutant '{name}' survived the pins"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
