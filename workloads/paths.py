"""Contraction paths and slice choices for tensor networks (label bookkeeping).

The paper takes its contraction order from a hyper-optimised path search and
its sliced bonds from a slice finder (Section V); neither tool is available
here, so this module supplies seeded stand-ins:

* ``greedy_path``: repeatedly contract the pair of tensors sharing a bond whose
  contraction shrinks memory the most (cost = size(out) - size(a) - size(b)),
  with seeded random perturbations over several restarts; the restart with the
  smallest (largest intermediate rank, total flops) wins.
* ``greedy_slices``: on a fixed path, repeatedly slice the bond whose removal
  lowers the largest intermediate rank the most (ties: total flops over all
  slices, then a seeded random key).

Paths use the single-static-assignment form: tensors 0..n-1 are the inputs and
step s creates tensor n + s from the pair path[s].  Only label sets are
handled here; no tensor values are touched.
"""
from __future__ import annotations

import heapq
import math

from .rng import SplitMix64


def _out_labels(la: frozenset, lb: frozenset) -> frozenset:
    # A label carried by both operands is a bond and is summed over (Section
    # II.A); every other label survives.  Open labels occur once in a network.
    return la ^ lb


def path_stats(labels, path, sliced=()):
    """(max rank over all tensors, flops of one slice, per-step ranks).

    flops counts 8 real operations per complex multiply-add, M*N*K of them.
    """
    sl = frozenset(sliced)
    live = [frozenset(l) - sl for l in labels]
    max_rank = max((len(l) for l in live), default=0)
    flops = 0
    steps = []
    for a, b in path:
        la, lb = live[a], live[b]
        out = _out_labels(la, lb)
        flops += 8 * (1 << len(la | lb))
        max_rank = max(max_rank, len(out))
        steps.append((len(la), len(lb), len(out)))
        live.append(out)
    return max_rank, flops, steps


def _greedy_once(labels, rng: SplitMix64, temperature: float):
    n = len(labels)
    live = {i: frozenset(l) for i, l in enumerate(labels)}
    holders: dict[int, set] = {}
    for i, l in live.items():
        for x in l:
            holders.setdefault(x, set()).add(i)

    heap = []

    def push(i, j):
        la, lb = live[i], live[j]
        out = _out_labels(la, lb)
        cost = (1 << len(out)) - (1 << len(la)) - (1 << len(lb))
        if temperature > 0.0:
            cost = cost * math.exp(temperature * rng.normal())
        heapq.heappush(heap, (cost, rng.uniform(), min(i, j), max(i, j)))

    seen = set()
    for x, hs in holders.items():
        hs = sorted(hs)
        for u in range(len(hs)):
            for v in range(u + 1, len(hs)):
                if (hs[u], hs[v]) not in seen:
                    seen.add((hs[u], hs[v]))
                    push(hs[u], hs[v])

    path = []
    nxt = n
    while heap:
        _, _, i, j = heapq.heappop(heap)
        if i not in live or j not in live:
            continue
        la, lb = live.pop(i), live.pop(j)
        out = _out_labels(la, lb)
        for x in la:
            holders[x].discard(i)
        for x in lb:
            holders[x].discard(j)
        path.append((i, j))
        k = nxt
        nxt += 1
        live[k] = out
        nbrs = set()
        for x in out:
            nbrs |= holders.setdefault(x, set())
            holders[x].add(k)
        for m in sorted(nbrs - {k}):
            push(m, k)
    # Disconnected pieces (none for circuits): join them by outer products,
    # smallest first.
    while len(live) > 1:
        ids = sorted(live, key=lambda t: (len(live[t]), t))
        i, j = ids[0], ids[1]
        la, lb = live.pop(i), live.pop(j)
        path.append((min(i, j), max(i, j)))
        live[nxt] = _out_labels(la, lb)
        nxt += 1
    return path


def greedy_path(labels, seed: int, restarts: int = 8, temperature: float = 0.3):
    best, best_key = None, None
    for r in range(restarts):
        rng = SplitMix64(seed * 7919 + r)
        path = _greedy_once(labels, rng, 0.0 if r == 0 else temperature)
        mr, fl, _ = path_stats(labels, path)
        key = (mr, fl)
        if best_key is None or key < best_key:
            best, best_key = path, key
    return best


def bond_labels(labels):
    count: dict[int, int] = {}
    for l in labels:
        for x in l:
            count[x] = count.get(x, 0) + 1
    return sorted(x for x, c in count.items() if c == 2)


def greedy_slices(labels, path, seed: int, n_slices: int | None = None,
                  max_rank: int | None = None, max_sliced: int = 64):
    """Choose bonds to slice on a fixed path.

    Stops after exactly ``n_slices`` bonds, or once the largest intermediate
    rank is <= ``max_rank`` (whichever is given), or at ``max_sliced`` bonds.
    Each round scores every unsliced bond x by (largest rank with x sliced
    too, total flops over all slices, seeded random key) and takes the least.
    Scores come from per-bond tallies: slicing x lowers the rank of exactly
    the tensors carrying x, so the largest rank drops by one iff x is carried
    by every tensor of the current largest rank, and a step's flops halve iff
    x is among its operands' labels.
    """
    rng = SplitMix64(seed * 104729 + 17)
    sliced: list[int] = []
    cands = bond_labels(labels)
    base = [frozenset(l) for l in labels]
    # Label sets of every operand pair and every result on the path.
    sets = list(base)
    unions = []
    for a, b in path:
        unions.append(sets[a] | sets[b])
        sets.append(_out_labels(sets[a], sets[b]))

    def done():
        if n_slices is not None:
            return len(sliced) >= n_slices
        mr, _, _ = path_stats(labels, path, sliced)
        return max_rank is not None and mr <= max_rank

    while not done() and len(sliced) < max_sliced:
        cur = frozenset(sliced)
        ranks = [len(t - cur) for t in sets]
        top = max(ranks)
        n_top = sum(1 for r in ranks if r == top)
        in_top: dict[int, int] = {}
        for t, r in zip(sets, ranks):
            if r == top:
                for x in t:
                    in_top[x] = in_top.get(x, 0) + 1
        weights = [1 << len(u - cur) for u in unions]
        total = sum(weights)
        with_x: dict[int, int] = {}
        for u, wgt in zip(unions, weights):
            for x in u:
                with_x[x] = with_x.get(x, 0) + wgt
        best, best_key = None, None
        for x in cands:
            if x in cur:
                continue
            mr = top - 1 if in_top.get(x, 0) == n_top else top
            # Flops over all 2^(|S|+1) slices; halves for steps carrying x.
            fl = (2 * total - with_x.get(x, 0)) << len(cur)
            key = (mr, fl, rng.uniform())
            if best_key is None or key < best_key:
                best, best_key = x, key
        if best is None:
            break
        sliced.append(best)
    return sliced
