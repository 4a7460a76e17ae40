"""Seeded subdomain partitions of a mesh's elements (input generation only).

The Schwarz preconditioner of Section 4 needs a partition of the fine elements
into N non-overlapping subdomains, aligned with coefficient jumps, and a coarse
agglomeration.  Here both are given as plain integer labels per element.

* :func:`quadrants` -- 2-D: subdomain by the quadrant of the element centroid.
* :func:`rcb` -- recursive coordinate bisection with prescribed (possibly uneven)
  target sizes, run separately inside each tissue region so that no subdomain
  crosses a region interface.
"""
from __future__ import annotations

import numpy as np


def quadrants(centroids: np.ndarray) -> np.ndarray:
    c = np.asarray(centroids)
    return ((c[:, 0] >= 0.5).astype(np.int32) + 2 * (c[:, 1] >= 0.5).astype(np.int32))


def _rcb(ids, cen, weights, out, base):
    if len(weights) == 1:
        out[ids] = base
        return
    half = len(weights) // 2
    wl, wr = weights[:half], weights[half:]
    frac = wl.sum() / weights.sum()
    span = cen[ids].max(0) - cen[ids].min(0)
    ax = int(np.argmax(span))
    order = ids[np.lexsort((ids, cen[ids, ax]))]
    cut = int(round(frac * len(ids)))
    cut = min(max(cut, half), len(ids) - (len(weights) - half))
    _rcb(order[:cut], cen, wl, out, base)
    _rcb(order[cut:], cen, wr, out, base + half)


def rcb(centroids, n_parts, region=None, spread=0.0, seed=0):
    """Partition elements into ``n_parts`` parts by recursive coordinate bisection.

    Parts are split evenly over regions (proportionally to region size) and
    never cross a region boundary.  Part target sizes are drawn uniformly from
    [1 - spread, 1 + spread] x mean with ``numpy.random.default_rng(seed)``.
    Returns an int32 label per element.
    """
    cen = np.asarray(centroids, dtype=np.float64)
    n = len(cen)
    region = np.zeros(n, dtype=np.int64) if region is None else np.asarray(region)
    regs = np.unique(region)
    sizes = np.array([(region == r).sum() for r in regs], dtype=np.float64)
    parts_per = np.maximum(1, np.round(n_parts * sizes / sizes.sum()).astype(int))
    parts_per[-1] = n_parts - parts_per[:-1].sum()
    rng = np.random.default_rng(seed)
    out = -np.ones(n, dtype=np.int64)
    base = 0
    for r, k in zip(regs, parts_per):
        ids = np.nonzero(region == r)[0]
        w = 1.0 + spread * (2.0 * rng.random(k) - 1.0) if spread > 0 else np.ones(k)
        _rcb(ids, cen, w, out, base)
        base += k
    return out.astype(np.int32)


def order_by_part(part, centroids):
    """Element permutation that makes every part contiguous (stable inside a
    part by a lexicographic order of the centroid)."""
    c = np.asarray(centroids)
    keys = [c[:, d] for d in range(c.shape[1] - 1, -1, -1)] + [np.asarray(part)]
    return np.lexsort(keys)
