"""Seeded synthetic workloads for block tensordot and sliced networks.

Seeds: workload c, trial t uses seed 1000*c + t.  Operand buffers are drawn
directly in their stored (block-major) layout: the entries are i.i.d., so the
dense tensor is simply whatever that buffer denotes.

  1. one block tensordot, complex128: rank-16 operands, every dim 2, contract
     A's last 8 axes with B's first 8 taken in a seeded random order; each
     operand blocked by splitting its first 3 axes in two.
  2. one amplitude of a 20-qubit random circuit on a 4x5 grid, 12 cycles,
     greedy path, 4 sliced bonds (16 slices).
  3. rank-28 operands, 14 contracted axes: a random 14-subset of A's axes and
     one of B's, paired in random order; unblocked (a blocked variant splits
     the first 3 axes of each operand).
  4. 256 independent block tensordots, operand ranks uniform in [8, 24],
     contracted counts uniform in [2, 10]; a draw is redone until
     k <= min(rA, rB) and rA + rB - 2k <= 24; blocked like workload 1.
  5. amplitude requests for random circuits on 30-53 sites, 8-14 cycles,
     each carrying 1-64 slices (2^0 .. 2^6, uniform exponent) and sliced
     further while its largest intermediate has rank above 30; a circuit
     needing more than 6 sliced bonds, or more than 2e13 flops over all its
     slices, is redrawn.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import circuits, paths
from .rng import (SplitMix64, complex_normal, gaussian_integers, substream_seed,
                  unit_values, wide_odd_integers)


def seed_of(config: int, trial: int = 0) -> int:
    return 1000 * config + trial


@dataclass
class Operand:
    dims: list
    grid: list
    data: np.ndarray  # flat complex128, stored block-major


@dataclass
class Problem:
    a: Operand
    b: Operand
    axes_a: list
    axes_b: list
    seed: int = 0

    @property
    def k(self) -> int:
        return len(self.axes_a)


# Value distributions of operand entries: complex normals (re, im ~ N(0, 1/2)),
# Gaussian integers in [-8, 8], odd integers of nine significant bits
# (257..511 with signs: a bfloat16 split of each has a nonzero low part), and
# units {0, +-1, +-i}.
VALUE_KINDS = ("normal", "integer", "wide", "unit")


def _fill(seed: int, tag: int, n: int, kind) -> np.ndarray:
    s = substream_seed(seed, tag)
    if kind is True or kind == "integer":
        return gaussian_integers(s, n)
    if kind == "wide":
        return wide_odd_integers(s, n)
    if kind == "unit":
        return unit_values(s, n)
    return complex_normal(s, n)


def make_problem(rank_a, rank_b, axes_a, axes_b, grid_a, grid_b, seed,
                 integer=False, values=None) -> Problem:
    """values: (kind of A, kind of B) from VALUE_KINDS; overrides integer."""
    ka, kb = values if values is not None else (integer, integer)
    da, db = [2] * rank_a, [2] * rank_b
    a = Operand(da, list(grid_a), _fill(seed, 1, 1 << rank_a, ka))
    b = Operand(db, list(grid_b), _fill(seed, 2, 1 << rank_b, kb))
    return Problem(a, b, list(axes_a), list(axes_b), seed)


def split_first(rank: int, nsplit: int = 3) -> list:
    return [2 if j < nsplit else 1 for j in range(rank)]


def config1(trial: int = 0, integer: bool = False) -> Problem:
    seed = seed_of(1, trial)
    rng = SplitMix64(substream_seed(seed, 0))
    axes_a = list(range(8, 16))
    axes_b = rng.permutation(8)
    return make_problem(16, 16, axes_a, axes_b, split_first(16), split_first(16),
                        seed, integer)


def random_axes(rng: SplitMix64, rank_a: int, rank_b: int, k: int):
    return rng.sample(rank_a, k), rng.sample(rank_b, k)


def config3(trial: int = 0, rank: int = 28, k: int = 14, blocked: bool = False,
            integer: bool = False, values=None) -> Problem:
    seed = seed_of(3, trial)
    rng = SplitMix64(substream_seed(seed, 0))
    axes_a, axes_b = random_axes(rng, rank, rank, k)
    ga = split_first(rank) if blocked else [1] * rank
    gb = split_first(rank) if blocked else [1] * rank
    return make_problem(rank, rank, axes_a, axes_b, ga, gb, seed, integer, values)


def config4_shapes(trial: int = 0, count: int = 256, max_out_rank: int = 24):
    """(rank_a, rank_b, axes_a, axes_b) for each problem of workload 4."""
    seed = seed_of(4, trial)
    rng = SplitMix64(substream_seed(seed, 0))
    shapes = []
    while len(shapes) < count:
        ra, rb, k = rng.randint(8, 24), rng.randint(8, 24), rng.randint(2, 10)
        if k > min(ra, rb) or ra + rb - 2 * k > max_out_rank:
            continue
        axa, axb = random_axes(rng, ra, rb, k)
        shapes.append((ra, rb, axa, axb))
    return shapes


def config4(trial: int = 0, count: int = 256, integer: bool = False,
            max_out_rank: int = 24):
    seed = seed_of(4, trial)
    probs = []
    for i, (ra, rb, axa, axb) in enumerate(config4_shapes(trial, count, max_out_rank)):
        probs.append(make_problem(ra, rb, axa, axb, split_first(ra), split_first(rb),
                                  substream_seed(seed, 100 + i), integer))
    return probs


@dataclass
class NetworkWorkload:
    network: circuits.Network
    path: list
    sliced: list
    bitstring: list | None
    circuit: circuits.Circuit
    seed: int = 0
    meta: dict = field(default_factory=dict)


def circuit_workload(rows, cols, cycles, seed, n_slices=None, max_rank=None,
                     open_legs=False, n_sites=None, restarts=8) -> NetworkWorkload:
    circ = circuits.random_circuit(rows, cols, cycles, substream_seed(seed, 10), n_sites)
    bits = None if open_legs else circuits.random_bitstring(circ.n, substream_seed(seed, 11))
    net = circuits.circuit_network(circ, bits)
    path = paths.greedy_path(net.labels, substream_seed(seed, 12) & 0xFFFFFFFF, restarts)
    sliced = []
    if n_slices or max_rank is not None:
        sliced = paths.greedy_slices(net.labels, path, substream_seed(seed, 13) & 0xFFFFFFFF,
                                     n_slices=n_slices, max_rank=max_rank)
    mr, fl, _ = paths.path_stats(net.labels, path, sliced)
    meta = {"max_rank": mr, "flops_per_slice": fl, "n_sliced": len(sliced)}
    return NetworkWorkload(net, path, sliced, bits, circ, seed, meta)


def config2(trial: int = 0, n_slices: int = 4) -> NetworkWorkload:
    return circuit_workload(4, 5, 12, seed_of(2, trial), n_slices=n_slices)


def config5_request(trial: int, index: int, max_rank: int = 30, max_sliced: int = 6,
                    flops_cap: float = 2e13, sites=(30, 53), cycles=(8, 14)):
    """One serving request: draws (sites, cycles) and a slice count of 2^0 ..
    2^max_sliced (uniform exponent), slices that many bonds greedily, slices
    more while the largest intermediate is above max_rank, and redraws while
    that needs more than max_sliced bonds or the request's total flops (all
    slices) exceed flops_cap."""
    seed = substream_seed(seed_of(5, trial), 1000 + index)
    rng = SplitMix64(seed)
    for attempt in range(64):
        n = rng.randint(*sites)
        cyc = rng.randint(*cycles)
        n_target = rng.randint(0, max_sliced)
        rows, cols = circuits.grid_shape(n)
        wl = circuit_workload(rows, cols, cyc, substream_seed(seed, attempt), n_sites=n,
                              restarts=2)
        lab, path = wl.network.labels, wl.path
        sl_seed = substream_seed(seed, 100 + attempt) & 0xFFFFFFFF
        sliced = paths.greedy_slices(lab, path, sl_seed, n_slices=n_target) if n_target else []
        if paths.path_stats(lab, path, sliced)[0] > max_rank:
            sliced = paths.greedy_slices(lab, path, sl_seed, max_rank=max_rank,
                                         max_sliced=max_sliced + 1)
        mr, fl, _ = paths.path_stats(lab, path, sliced)
        total = fl * (1 << len(sliced))
        if len(sliced) <= max_sliced and mr <= max_rank and total <= flops_cap:
            wl.sliced = sliced
            wl.meta.update({"sites": n, "cycles": cyc, "attempt": attempt, "max_rank": mr,
                            "flops_per_slice": fl, "n_sliced": len(sliced),
                            "total_flops": total})
            return wl
    raise RuntimeError("no feasible circuit drawn")
