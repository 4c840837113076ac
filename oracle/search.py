"""Monte-Carlo tree search over the SpMV design space -- TEST INFRASTRUCTURE.

A plain, slow restatement of Sec. III-C of the paper, used only by the tests
to check the library's search.  It shares no code with the library: the DAG,
the Table III tokens and the plan space come from this package
(:data:`oracle.DAG_EDGES`, :func:`oracle.required_syncs`).

A node of the tree is a program prefix P_k (Sec. III-B), kept as the tuple
of its steps; a step is ``(token, stream)`` with ``stream`` the canonical
stream of a GPU vertex (streams labelled by first use: two prefixes equal
under a bijection of streams are one node) and ``None`` otherwise.

The random choices the method makes are inputs: ``draws`` is a sequence of
non-negative integers, and the k-th random choice among m candidates takes
candidate ``draws[k] % m``.  ``key(token, stream)`` orders the candidates of
a node; the first of equal scores in creation order is selected.
"""
from __future__ import annotations

import math

from . import DAG_EDGES, GPU_VERTICES, required_syncs, plan_tokens


class Dag:
    """A program DAG as the search sees it: the tokens of an order, what
    must precede each token (DAG predecessors and the Table III pairs), and
    which tokens are GPU vertices."""

    def __init__(self, tokens, need, gpu):
        self.tokens = list(tokens)
        self.need = {t: set(need.get(t, ())) for t in self.tokens}
        self.gpu = set(gpu)


def coarse_dag() -> Dag:
    """The SpMV DAG of Sec. III-A with the Table III tokens its GPU -> CPU
    edges need (Unpack implied before yR)."""
    toks = ["start"] + plan_tokens() + ["end"]
    need = {t: set() for t in toks}
    for u, v in DAG_EDGES:
        need[v].add(u)
    for u, v, rec, wait in required_syncs():
        need[rec].add(u)
        need[wait].add(rec)
        need[v].add(wait)
    need["end"] = set(toks) - {"end"}
    return Dag(toks, need, [g for g in GPU_VERTICES])


def _default_key(token, stream):
    names = ["start"] + plan_tokens() + ["end"]
    return (names.index(token), -1 if stream is None else stream)


def children(prefix, n_streams: int, key=_default_key, dag: Dag | None = None):
    """Next steps of a prefix (Sec. III-C, Expansion): every DAG vertex not
    yet placed whose predecessors are placed, and every Table III token whose
    operand is placed -- a record after its GPU vertex, a host wait after its
    record; a CPU vertex needing a wait also needs the wait placed.  GPU
    vertices are bound to each stream already used and to one new stream
    while fewer than ``n_streams`` are used.  ``end`` comes last."""
    dag = dag or _COARSE
    placed = {t for t, _ in prefix}
    used = len({s for _, s in prefix if s is not None})
    out = []
    for t in dag.tokens:
        if t in placed or not dag.need[t] <= placed:
            continue
        if t in dag.gpu:
            out += [(t, s) for s in range(min(used + 1, n_streams))]
        else:
            out.append((t, None))
    return sorted(out, key=lambda st: key(*st))


_COARSE = coarse_dag()


def plan_of(prefix):
    """(order of token names, canonical streams of (Pack, yL, yR)) of a
    complete prefix: the form :func:`oracle.plan_space` uses."""
    streams = {t: s for t, s in prefix if s is not None}
    return tuple(t for t, _ in prefix), tuple(streams[g] for g in GPU_VERTICES)


class Node:
    def __init__(self, prefix, n_streams, key, dag):
        self.prefix = prefix
        self.untried = children(prefix, n_streams, key, dag)
        self.complete = not self.untried
        self.children = []              # created children, in creation order
        self.n = 0                      # rollouts through this node
        self.t_min = math.inf
        self.t_max = -math.inf
        self.full = False               # every plan below has been benchmarked


def exploitation(parent: Node, child: Node) -> float:
    """V of Sec. III-C (Selection): the child's observed time range over the
    parent's when both have at least two rollouts, else 1.  Where the
    parent's range is zero (all its times equal) the ratio is undefined and
    V is 1, as when there is no basis for comparison."""
    if child.n >= 2 and parent.n >= 2 and parent.t_max > parent.t_min:
        return (child.t_max - child.t_min) / (parent.t_max - parent.t_min)
    return 1.0


def exploration(parent: Node, child: Node, c: float) -> float:
    """c * sqrt(ln N / n), or -inf when the child's subtree is fully
    explored (Sec. III-C, Selection)."""
    if child.full:
        return -math.inf
    return c * math.sqrt(math.log(parent.n) / child.n)


def mcts(cost, n_streams: int = 2, iterations: int = 0, draws=(), c: float = math.sqrt(2.0),
         key=_default_key, trace=None, dag: Dag | None = None):
    """Run the search.  ``cost(plan)`` gives the time of a complete plan (in
    :func:`plan_of` form for the coarse DAG, the prefix tuple itself for any
    other ``dag``).  Stops after ``iterations`` rollouts (0: until the
    root is fully explored).  Returns (list of (plan, time) per rollout, root
    node).  ``trace``, when given, is called as trace(event, data) with
    events "select" (parent, child, V, score), "path" (the nodes of a
    rollout, root first, before their statistics are updated)."""
    root = Node((), n_streams, key, dag)
    draws = iter(draws)
    log = []
    while not root.full and (iterations == 0 or len(log) < iterations):
        # Selection: descend by the largest combined value; stop at a node
        # that has a child without rollouts (one not created yet)
        node, path = root, [root]
        while not node.untried and not node.complete:
            best, best_score = None, None
            for ch in node.children:
                V = exploitation(node, ch)
                score = exploration(node, ch, c) + V
                if trace:
                    trace("select", (node, ch, V, score))
                if best is None or score > best_score:
                    best, best_score = ch, score
            node = best
            path.append(node)
        # Expansion (one zero-rollout child) and rollout (random children
        # until the program is complete; every node stays in the tree)
        while not node.complete:
            k = next(draws) % len(node.untried)
            step = node.untried.pop(k)
            child = Node(node.prefix + (step,), n_streams, key, dag)
            node.children.append(child)
            node = child
            path.append(node)
        plan = plan_of(node.prefix) if dag is None else node.prefix
        t = cost(plan)
        log.append((plan, t))
        if trace:
            trace("path", list(path))
        # Backpropagation: rollout count and the time range of every node on
        # the path; a node is fully explored when it is complete or all its
        # children exist and are fully explored
        for nd in path:
            nd.n += 1
            nd.t_min = min(nd.t_min, t)
            nd.t_max = max(nd.t_max, t)
        for nd in reversed(path):
            nd.full = nd.complete or (not nd.untried and all(ch.full for ch in nd.children))
    return log, root


def walk(root):
    """Every node of the tree, parents before children."""
    out, stack = [], [root]
    while stack:
        nd = stack.pop()
        out.append(nd)
        stack.extend(reversed(nd.children))
    return out
