"""The Lite distribution scheme and its metrics (oracle; test infrastructure only).

Section 6 ("Distribution Scheme Lite") and its pseudocode figure assign the
elements of mode-n slices to P bins (processors in the paper; workgroups in
the GPU library) in two stages:

  * sort the slices by cardinality (ascending) and set limit = ceil(|E| / P);
  * stage 1 walks the sorted slices, giving each whole slice to bin
    p = 0, 1, ..., P-1, 0, 1, ... (round robin) and stops at the first slice
    that would push its bin above limit;
  * stage 2 walks the remaining slices and the bins 0..P-1 together: a slice
    that fits the current bin's gap (limit - load) goes there whole and the
    walk moves to the next slice; otherwise the bin is filled to the limit
    with elements of the slice and the walk moves to the next bin.

Readings where the paper is silent or garbled (stated once here, used below):
  * empty slices are left out (they are shared by no bin);
  * ties in the size sort are broken by ascending slice id;
  * the round-robin receiver of the t-th sorted slice (t = 0, 1, ...) is t mod P;
  * "select any g elements" takes the first g remaining elements of the slice
    in canonical (lexicographic, l_1 most significant) order;
  * a bin with gap 0 receives nothing and the walk moves to the next bin;
  * stage 2 ends when the slices run out (or the bins do).

Layout order of the elements of one mode (what the GPU's mode-sorted copy must
reproduce bit for bit): bins in order 0..P-1; inside a bin, its stage-1 slices
in sorted order, then its stage-2 pieces in the order stage 2 assigned them;
inside a slice piece, canonical element order.

Metrics (Section 4): E_max = max_p |E^p| (metric 1), R_sum = sum_p R^p
(metric 2), R_max = max_p R^p (metric 3), where R^p counts the slices bin p
shares.  A slice is bad when more than one bin shares it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


@dataclass
class LiteResult:
    P: int
    limit: int
    m: int
    L_nonempty: int
    n_stage1: int                       # slices placed whole by stage 1 (the paper's t-hat minus one)
    order: list                         # nonempty slice ids in sorted order
    pieces: dict                        # slice id -> list of (bin, count), in assignment order
    bin_slices: list                    # per bin: list of (slice id, count), in layout order
    load: list                          # final |E^p|
    stats: dict = field(default_factory=dict)


def lite(slice_sizes, P: int) -> LiteResult:
    """Run Lite on per-slice cardinalities (index = slice id, 0 allowed)."""
    sizes = [int(s) for s in slice_sizes]
    m = sum(sizes)
    if P < 1:
        raise ValueError("P must be >= 1")
    limit = ceil_div(m, P) if m > 0 else 0
    # Sort slices by cardinality (ties by id), empty slices excluded.
    order = sorted((l for l in range(len(sizes)) if sizes[l] > 0), key=lambda l: (sizes[l], l))
    load = [0] * P
    pieces = {}
    bin_slices = [[] for _ in range(P)]

    # Stage 1: whole slices, round robin, until one would exceed the limit.
    t = 0
    p = 0
    while t < len(order):
        S = order[t]
        if load[p] + sizes[S] > limit:
            break
        load[p] += sizes[S]
        pieces[S] = [(p, sizes[S])]
        bin_slices[p].append((S, sizes[S]))
        p = (p + 1) % P
        t += 1
    n_stage1 = t

    # Stage 2: fill bins 0..P-1 to the limit, splitting slices over contiguous bins.
    p = 0
    remaining = sizes[order[t]] if t < len(order) else 0
    while p < P and t < len(order):
        S = order[t]
        g = limit - load[p]
        if remaining <= g:
            load[p] += remaining
            pieces.setdefault(S, []).append((p, remaining))
            bin_slices[p].append((S, remaining))
            t += 1
            remaining = sizes[order[t]] if t < len(order) else 0
        else:
            if g > 0:
                load[p] += g
                pieces.setdefault(S, []).append((p, g))
                bin_slices[p].append((S, g))
                remaining -= g
            p += 1
    if t < len(order):
        raise AssertionError("stage 2 ran out of bins; impossible when limit = ceil(m/P)")

    res = LiteResult(P=P, limit=limit, m=m, L_nonempty=len(order), n_stage1=n_stage1, order=order,
                     pieces=pieces, bin_slices=bin_slices, load=load)
    res.stats = metrics_from_bins(bin_slices, load)
    res.stats.update(P=P, limit=limit, m=m, L_nonempty=len(order), n_stage1=n_stage1)
    return res


def metrics_from_bins(bin_slices, load) -> dict:
    """Section 4 metrics of any assignment given as per-bin (slice, count) lists."""
    R = [len({s for s, c in b if c > 0}) for b in bin_slices]
    sharers = {}
    for p, b in enumerate(bin_slices):
        for s, c in b:
            if c > 0:
                sharers.setdefault(s, set()).add(p)
    n_bad = sum(1 for v in sharers.values() if len(v) > 1)
    return dict(E_max=max(load) if load else 0, R_sum=sum(R), R_max=max(R) if R else 0, n_bad=n_bad,
                R_per_bin=R)


def metrics_from_policy(slice_of_elem, owner_of_elem, P: int) -> dict:
    """Metrics 1-3 (Section 4) of an element -> processor policy."""
    E = [0] * P
    shares = [set() for _ in range(P)]
    for s, p in zip(slice_of_elem, owner_of_elem):
        E[p] += 1
        shares[p].add(s)
    R = [len(x) for x in shares]
    return dict(E_max=max(E), R_sum=sum(R), R_max=max(R), R_per_bin=R)


def choose_bins(m: int, L_nonempty: int, wg_nnz: int, rows_cap: int) -> int:
    """Number of bins: enough that no bin exceeds wg_nnz elements on average and,
    by Theorem 6.1 part 3 (R_max <= ceil(L/P) + 2), no bin holds more than
    rows_cap slices."""
    if rows_cap < 3:
        raise ValueError("rows_cap must be >= 3")
    return max(1, ceil_div(m, wg_nnz), ceil_div(L_nonempty, rows_cap - 2))


@dataclass
class Partition:
    """One mode's partition in the form the GPU library exports."""
    bin_ptr: np.ndarray       # int64[P+1]: layout offsets of the bins
    elem_order: np.ndarray    # int64[m]: canonical element index at each layout position
    seg_bin: np.ndarray       # int32[S]: bin of each segment (a slice piece), layout order
    seg_slice: np.ndarray     # int32[S]: slice id of each segment
    seg_begin: np.ndarray     # int64[S]: first layout position
    seg_end: np.ndarray       # int64[S]: one past the last layout position
    seg_bad: np.ndarray       # uint8[S]: 1 when the slice is shared by more than one bin
    stats: dict
    lite: LiteResult


def partition_mode(idx_n, L_n: int, P: int, coarse_order=None) -> Partition:
    """Lite (or, given a random slice order, CoarseG) along one mode for
    coalesced elements in canonical order.

    idx_n: the mode-n coordinate of every element (canonical order)."""
    idx_n = np.asarray(idx_n, dtype=np.int64)
    m = idx_n.shape[0]
    sizes = np.bincount(idx_n, minlength=L_n) if m else np.zeros(L_n, np.int64)
    res = lite(sizes.tolist(), P) if coarse_order is None else coarse_g(sizes.tolist(), P, coarse_order)
    # Elements of each slice in canonical order (stable sort by slice id).
    by_slice = np.argsort(idx_n, kind="stable")
    start = np.zeros(L_n + 1, np.int64)
    np.cumsum(sizes, out=start[1:])
    taken = np.zeros(L_n, np.int64)   # elements of each slice already placed
    elem_order = np.empty(m, np.int64)
    bin_ptr = np.zeros(P + 1, np.int64)
    segs = []
    pos = 0
    for p in range(P):
        bin_ptr[p] = pos
        for s, c in res.bin_slices[p]:
            a = start[s] + taken[s]
            elem_order[pos:pos + c] = by_slice[a:a + c]
            taken[s] += c
            bad = 1 if len(res.pieces[s]) > 1 else 0
            segs.append((p, s, pos, pos + c, bad))
            pos += c
    bin_ptr[P] = pos
    assert pos == m
    S = len(segs)
    arr = np.array(segs, dtype=np.int64).reshape(S, 5)
    return Partition(bin_ptr=bin_ptr, elem_order=elem_order,
                     seg_bin=arr[:, 0].astype(np.int32), seg_slice=arr[:, 1].astype(np.int32),
                     seg_begin=arr[:, 2].copy(), seg_end=arr[:, 3].copy(),
                     seg_bad=arr[:, 4].astype(np.uint8), stats=res.stats, lite=res)


# ---------------------------------------------------------------------------------------------
# CoarseG (Section 5, "Coarse Grained Schemes"): a prior scheme, kept as the
# baseline Lite is compared with.  Along mode n each slice goes whole to one
# processor: the slices are arranged in a random order and contiguous blocks
# of them are allocated to the processors.  Reading (the paper does not say
# where the blocks end): the block boundaries balance elements, the slice whose
# elements start at prefix x (in the random order) going to bin
# min(P - 1, floor(x P / m)).  Empty slices are left out.  The random order is
# an input (the caller draws it).
# ---------------------------------------------------------------------------------------------

def coarse_g(slice_sizes, P: int, order) -> LiteResult:
    sizes = [int(s) for s in slice_sizes]
    m = sum(sizes)
    if P < 1:
        raise ValueError("P must be >= 1")
    if sorted(int(l) for l in order) != list(range(len(sizes))):
        raise ValueError("order must be a permutation of the slice ids")
    load = [0] * P
    pieces = {}
    bin_slices = [[] for _ in range(P)]
    x = 0
    for l in order:
        l = int(l)
        if sizes[l] == 0:
            continue
        p = min(P - 1, x * P // m)
        load[p] += sizes[l]
        pieces[l] = [(p, sizes[l])]
        bin_slices[p].append((l, sizes[l]))
        x += sizes[l]
    nonempty = [int(l) for l in order if sizes[int(l)] > 0]
    res = LiteResult(P=P, limit=ceil_div(m, P) if m > 0 else 0, m=m, L_nonempty=len(nonempty),
                     n_stage1=len(nonempty), order=nonempty, pieces=pieces, bin_slices=bin_slices, load=load)
    res.stats = metrics_from_bins(bin_slices, load)
    res.stats.update(P=P, limit=res.limit, m=m, L_nonempty=len(nonempty), n_stage1=len(nonempty))
    return res
