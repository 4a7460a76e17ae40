"""Seeded 3-D polyhedral meshes by greedy agglomeration of a hexahedral grid.

Input generation only.  An ``n x n x n`` grid of cubes over ``[0, L]^3`` is
agglomerated into polyhedral elements (unions of cubes) of about ``target``
cubes each:

* cubes are visited in a seeded random order; every still-free cube seeds a new
  element, which grows by repeatedly taking the free face-neighbour cube of the
  same tissue region that lies closest to the element's current centroid
  (ties broken by a seeded random key) until it holds ``target`` cubes or has
  no free neighbour left;
* elements that end up with fewer than ``min_keep`` cubes are merged into the
  smallest face-adjacent element of the same region.

Elements never cross a region interface, so the subdomain and coarse partitions
built from them can be aligned with conductivity jumps.  Facets are the unit
squares between cubes of different elements (interior) or on the cube's
boundary; an interface between two elements consists of several such facets.
"""
from __future__ import annotations

import heapq

import numpy as np

from .meshdata import Mesh


def _cube_neighbours(n):
    idx = np.arange(n ** 3).reshape(n, n, n)
    nb = -np.ones((n ** 3, 6), dtype=np.int64)
    nb[idx[1:, :, :].ravel(), 0] = idx[:-1, :, :].ravel()
    nb[idx[:-1, :, :].ravel(), 1] = idx[1:, :, :].ravel()
    nb[idx[:, 1:, :].ravel(), 2] = idx[:, :-1, :].ravel()
    nb[idx[:, :-1, :].ravel(), 3] = idx[:, 1:, :].ravel()
    nb[idx[:, :, 1:].ravel(), 4] = idx[:, :, :-1].ravel()
    nb[idx[:, :, :-1].ravel(), 5] = idx[:, :, 1:].ravel()
    return nb


def agglomerate_grid(n: int, seed: int, target: int = 8, region=None, min_keep: int = 3):
    """Element id per cube (C order over (i, j, k)) of an agglomerated n^3 grid."""
    rng = np.random.default_rng(seed)
    nc = n ** 3
    ijk = np.stack(np.unravel_index(np.arange(nc), (n, n, n)), 1).astype(np.float64)
    region = np.zeros(nc, dtype=np.int64) if region is None else np.asarray(region)
    nb = _cube_neighbours(n)
    tie = rng.random(nc)
    owner = -np.ones(nc, dtype=np.int64)
    n_el = 0
    for s in rng.permutation(nc):
        if owner[s] >= 0:
            continue
        el = n_el
        n_el += 1
        owner[s] = el
        members = [s]
        csum = ijk[s].copy()
        heap = []
        for t in nb[s]:
            if t >= 0 and owner[t] < 0 and region[t] == region[s]:
                heapq.heappush(heap, (0.0, tie[t], int(t)))
        while len(members) < target and heap:
            # re-rank the frontier by the distance to the current centroid
            cen = csum / len(members)
            cand = {t for _, _, t in heap if owner[t] < 0}
            if not cand:
                break
            best = min(cand, key=lambda t: (((ijk[t] - cen) ** 2).sum(), tie[t]))
            owner[best] = el
            members.append(best)
            csum += ijk[best]
            heap = [(0.0, tie[t], t) for t in cand if t != best]
            for t in nb[best]:
                if t >= 0 and owner[t] < 0 and region[t] == region[s]:
                    heap.append((0.0, tie[t], int(t)))
    # merge small fragments into the smallest adjacent element of the same region
    size = np.bincount(owner, minlength=n_el)
    for el in np.argsort(size, kind="stable"):
        if size[el] == 0 or size[el] >= min_keep:
            continue
        cubes = np.nonzero(owner == el)[0]
        cands = {}
        for c in cubes:
            for t in nb[c]:
                if t >= 0 and owner[t] != el and region[t] == region[c]:
                    cands[owner[t]] = size[owner[t]]
        if not cands:
            continue
        tgt = min(cands, key=lambda e: (cands[e], e))
        owner[cubes] = tgt
        size[tgt] += size[el]
        size[el] = 0
    # relabel densely in order of first cube
    _, first = np.unique(owner, return_index=True)
    order = np.argsort(first)
    remap = -np.ones(owner.max() + 1, dtype=np.int64)
    remap[np.unique(owner)[order]] = np.arange(len(order))
    return remap[owner]


def agglomerated_cube_mesh(n: int, length: float, seed: int, target: int = 8,
                           region_of_cube=None, elem_order=None, min_keep: int = 3) -> Mesh:
    """Polyhedral mesh of [0, length]^3 from an agglomerated n^3 cube grid.

    ``region_of_cube``: optional int array over cubes (C order); elements never
    cross region boundaries.  ``elem_order``: optional callable(owner, centroids)
    returning a permutation that renumbers elements (used to make subdomains
    contiguous in memory).
    """
    owner = agglomerate_grid(n, seed, target, region_of_cube, min_keep=min(min_keep, target))
    return cube_mesh_from_owner(owner, n, length, region_of_cube, elem_order)


def cube_mesh_from_owner(owner, n: int, length: float, region_of_cube=None, elem_order=None) -> Mesh:
    """Polyhedral mesh of [0, length]^3 whose element e is the union of the
    cubes c of an n^3 grid (C order) with ``owner[c] == e`` (ids 0..n_el-1)."""
    owner = np.asarray(owner, dtype=np.int64)
    h = length / n
    nc = n ** 3
    i, j, k = np.unravel_index(np.arange(nc), (n, n, n))
    lo = np.stack([i, j, k], 1) * h
    n_el = owner.max() + 1
    cube_order = np.lexsort((np.arange(nc), owner))  # group cubes by element
    counts = np.bincount(owner, minlength=n_el)
    cell_ptr = np.concatenate([[0], np.cumsum(counts)])
    cell_geom = np.stack([lo[cube_order], lo[cube_order] + h], 1)

    idx = np.arange(nc).reshape(n, n, n)
    f_elem, f_geom, f_norm = [], [], []
    for ax in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, n - 1)
        sl_hi[ax] = slice(1, n)
        a = idx[tuple(sl_lo)].ravel()
        b = idx[tuple(sl_hi)].ravel()
        diff = owner[a] != owner[b]
        a, b = a[diff], b[diff]
        flo = lo[b].copy()
        fhi = lo[b] + h
        fhi[:, ax] = flo[:, ax]
        nrm = np.zeros((len(a), 3))
        nrm[:, ax] = 1.0
        f_elem.append(np.stack([owner[a], owner[b]], 1))
        f_geom.append(np.stack([flo, fhi], 1))
        f_norm.append(nrm)
        # boundary faces on both sides of this axis
        for side, sgn in ((0, -1.0), (n - 1, 1.0)):
            sl = [slice(None)] * 3
            sl[ax] = side
            c = idx[tuple(sl)].ravel()
            blo = lo[c].copy()
            if sgn > 0:
                blo[:, ax] += h
            bhi = blo + h
            bhi[:, ax] = blo[:, ax]
            nrm = np.zeros((len(c), 3))
            nrm[:, ax] = sgn
            f_elem.append(np.stack([owner[c], -np.ones(len(c), dtype=np.int64)], 1))
            f_geom.append(np.stack([blo, bhi], 1))
            f_norm.append(nrm)
    mesh = Mesh(
        dim=3,
        cell_ptr=cell_ptr.astype(np.int64),
        cell_geom=np.ascontiguousarray(cell_geom),
        facet_elem=np.concatenate(f_elem).astype(np.int64),
        facet_geom=np.ascontiguousarray(np.concatenate(f_geom)),
        facet_normal=np.ascontiguousarray(np.concatenate(f_norm)),
    )
    mesh.extra["cube_owner"] = owner
    mesh.extra["grid_n"] = n
    mesh.extra["grid_h"] = h
    if region_of_cube is not None:
        reg = np.zeros(n_el, dtype=np.int32)
        reg[owner] = np.asarray(region_of_cube)
        mesh.region = reg
    if elem_order is not None:
        mesh = renumber_elements(mesh, elem_order(mesh))
    return mesh


def renumber_elements(mesh: Mesh, perm) -> Mesh:
    """New mesh whose element e is old element ``perm[e]``; facet minus/plus
    ordering and normals are preserved."""
    perm = np.asarray(perm)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    counts = np.diff(mesh.cell_ptr)[perm]
    cell_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cells = np.concatenate([np.arange(mesh.cell_ptr[p], mesh.cell_ptr[p + 1]) for p in perm])
    fe = mesh.facet_elem.copy()
    fe[:, 0] = inv[fe[:, 0]]
    m = fe[:, 1] >= 0
    fe[m, 1] = inv[fe[m, 1]]
    out = Mesh(dim=mesh.dim, cell_ptr=cell_ptr, cell_geom=mesh.cell_geom[cells],
               facet_elem=fe, facet_geom=mesh.facet_geom, facet_normal=mesh.facet_normal)
    if mesh.region is not None:
        out.region = mesh.region[perm]
    if mesh.sigma is not None:
        out.sigma = mesh.sigma[perm]
    out.extra = dict(mesh.extra)
    if "cube_owner" in out.extra:
        out.extra["cube_owner"] = inv[out.extra["cube_owner"]]
    return out
