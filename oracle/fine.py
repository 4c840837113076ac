"""The fine-grained SpMV program of Sec. III-A -- TEST INFRASTRUCTURE.

The paper notes that the single Pack and PostSends vertices could instead be
one independent vertex per destination (and likewise the receives), which
removes false dependencies at the price of a larger space.  This module
builds that DAG for one rank from the oracle's split and counts its
programs, plainly, for the tests to check the library against.  Token names
carry the peer rank in brackets ("Pack[2]", "CER-after-Pack[2]").

* :func:`fine_dag` -- per destination q: Pack[q] -> PostSend[q] ->
  WaitSend[q] -> end, with the Table III pair CER-after-Pack[q],
  CES-b4-PostSend[q] for the GPU -> CPU edge; per source q: PostRecv[q] ->
  WaitRecv[q] -> yR (yR needs every source; Unpack runs implied before it);
  start -> Pack[q], yL, PostRecv[q]; yL -> end.
* :func:`count_orders` -- topological orders by plain recursion over the
  set of placed tokens (memoised).
* :func:`count_stream_maps` -- canonical stream maps by brute force over
  every assignment of the GPU vertices to streams, relabelled by first use.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

from .search import Dag


def peers(split: dict, rank: int):
    """(destinations, sources): ranks with a non-empty send list, ranks that
    own halo entries, ascending."""
    so, ro = list(split["send_off"]), list(split["recv_off"])
    P = len(so) - 1
    dests = [q for q in range(P) if q != rank and so[q + 1] > so[q]]
    srcs = [q for q in range(P) if q != rank and ro[q + 1] > ro[q]]
    return dests, srcs


def fine_dag(split: dict, rank: int) -> Dag:
    dests, srcs = peers(split, rank)
    toks = ["start", "yL", "yR", "end"]
    need = {"yL": {"start"}, "yR": {"start"}}
    gpu = ["yL", "yR"]
    for q in dests:
        pk, cer, ces = f"Pack[{q}]", f"CER-after-Pack[{q}]", f"CES-b4-PostSend[{q}]"
        ps, ws = f"PostSend[{q}]", f"WaitSend[{q}]"
        toks += [pk, cer, ces, ps, ws]
        need[pk] = {"start"}
        need[cer] = {pk}
        need[ces] = {cer}
        need[ps] = {pk, ces}
        need[ws] = {ps}
        gpu.append(pk)
    for q in srcs:
        pr, wr = f"PostRecv[{q}]", f"WaitRecv[{q}]"
        toks += [pr, wr]
        need[pr] = {"start"}
        need[wr] = {pr}
        need["yR"].add(wr)
    need["end"] = set(toks) - {"end"}
    return Dag(toks, need, gpu)


def count_orders(dag: Dag) -> int:
    toks = tuple(dag.tokens)

    @lru_cache(maxsize=None)
    def rec(placed: frozenset) -> int:
        if len(placed) == len(toks):
            return 1
        total = 0
        for t in toks:
            if t not in placed and dag.need[t] <= placed:
                total += rec(placed | {t})
        return total
    return rec(frozenset())


def count_stream_maps(n_gpu: int, n_streams: int) -> int:
    maps = set()
    for a in itertools.product(range(n_streams), repeat=n_gpu):
        relabel = {}
        for s in a:
            relabel.setdefault(s, len(relabel))
        maps.add(tuple(relabel[s] for s in a))
    return len(maps)


def count_programs(dag: Dag, n_streams: int = 2) -> int:
    return count_orders(dag) * count_stream_maps(len(dag.gpu), n_streams)
