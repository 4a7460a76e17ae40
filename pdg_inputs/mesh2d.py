"""Seeded 2-D polygonal meshes: clipped Voronoi tessellations of the unit square.

Input generation only: geometry of the polytopal mesh (Section 3 of the paper
uses general polygonal meshes; Section 5 uses Voronoi-like polygonal grids).
Nothing here evaluates a basis, a quadrature rule or any discrete operator.

Construction
------------
* ``n`` seeds drawn uniformly in the square from ``numpy.random.default_rng(seed)``.
* Each Voronoi cell is the square clipped by the bisector half-planes of the
  other seeds (Sutherland-Hodgman on a convex polygon, with every edge labelled
  by the constraint that produced it).
* ``lloyd`` Lloyd iterations move every seed to its cell's centroid.
* Each polygon is split into a fan of triangles around its vertex average
  (these triangles are the sub-cells both implementations integrate over).
* Every polygon edge that lies on a bisector is an interior facet between the
  two cells; edges on the square's sides are boundary facets.
"""
from __future__ import annotations

import numpy as np

from .meshdata import Mesh


def _clip(poly, labels, a, b, lab):
    """Clip convex polygon ``poly`` to the half-plane a.x <= b.

    ``labels[k]`` names the constraint that produced edge poly[k] -> poly[k+1].
    """
    out_p, out_l = [], []
    m = len(poly)
    s = poly @ a - b
    for k in range(m):
        k1 = (k + 1) % m
        pk, pk1 = poly[k], poly[k1]
        ink, ink1 = s[k] <= 0.0, s[k1] <= 0.0
        if ink:
            out_p.append(pk)
            out_l.append(labels[k])
            if not ink1:
                t = s[k] / (s[k] - s[k1])
                out_p.append(pk + t * (pk1 - pk))
                out_l.append(lab)
        elif ink1:
            t = s[k] / (s[k] - s[k1])
            out_p.append(pk + t * (pk1 - pk))
            out_l.append(labels[k])
    if not out_p:
        return np.zeros((0, 2)), []
    return np.array(out_p), out_l


def _dedup(poly, labels, tol=1e-13):
    """Drop zero-length edges (coincident consecutive vertices)."""
    keep_p, keep_l = [], []
    m = len(poly)
    for k in range(m):
        nxt = poly[(k + 1) % m]
        if np.linalg.norm(nxt - poly[k]) > tol:
            keep_p.append(poly[k])
            keep_l.append(labels[k])
    return np.array(keep_p), keep_l


def voronoi_cells(points, n_cand=48):
    """Clipped Voronoi cells of ``points`` in [0,1]^2.

    Each cell is the square clipped by the bisector half-planes of its nearest
    seeds (nearest first); the candidate set grows until every seed left out
    is provably too far to cut the cell (farther than twice the cell's
    radius).  Returns a list of (vertices[m,2] counter-clockwise,
    edge_labels[m]) where a label j >= 0 is the neighbouring seed and
    -1..-4 are the square's sides.
    """
    from scipy.spatial import cKDTree

    points = np.asarray(points, dtype=np.float64)
    n = len(points)
    square = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    sq_labels = [-1, -2, -3, -4]  # bottom, right, top, left
    tree = cKDTree(points)
    cells = []
    for i in range(n):
        nc = n_cand
        while True:
            k = min(n, nc + 2)
            dist, idx = tree.query(points[i], k=k)
            order = idx[np.argsort(dist, kind="stable")]
            order = order[order != i]
            use = order if k >= n else order[:nc]
            poly, labels = square.copy(), list(sq_labels)
            for j in use:
                a = points[j] - points[i]
                b = 0.5 * (points[j] @ points[j] - points[i] @ points[i])
                # skip half-planes that cannot cut the current cell
                if np.max(poly @ a - b) <= 0.0:
                    continue
                poly, labels = _clip(poly, labels, a, b, int(j))
            poly, labels = _dedup(poly, labels)
            if k >= n:
                break
            # every seed left out must be too far to cut the cell
            rmax = np.sqrt(((poly - points[i]) ** 2).sum(1).max())
            if ((points[order[nc]] - points[i]) ** 2).sum() > (2.0 * rmax) ** 2:
                break
            nc *= 2
        cells.append((poly, labels))
    return cells


def _polygon_area_centroid(poly):
    x, y = poly[:, 0], poly[:, 1]
    x1, y1 = np.roll(x, -1), np.roll(y, -1)
    cr = x * y1 - x1 * y
    area = 0.5 * cr.sum()
    cx = ((x + x1) * cr).sum() / (6.0 * area)
    cy = ((y + y1) * cr).sum() / (6.0 * area)
    return area, np.array([cx, cy])


def voronoi_mesh(n: int, seed: int, lloyd: int = 10) -> Mesh:
    """Polygonal mesh of the unit square with ``n`` Lloyd-relaxed Voronoi cells."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    for _ in range(lloyd):
        cells = voronoi_cells(pts)
        pts = np.array([_polygon_area_centroid(p)[1] for p, _ in cells])
    cells = voronoi_cells(pts)

    tri_list, cell_ptr = [], [0]
    polys = []
    for poly, _ in cells:
        c = poly.mean(axis=0)  # vertex average: fan centre
        m = len(poly)
        for k in range(m):
            tri_list.append([c, poly[k], poly[(k + 1) % m]])
        cell_ptr.append(len(tri_list))
        polys.append(poly)

    f_elem, f_geom, f_norm = [], [], []
    for i, (poly, labels) in enumerate(cells):
        m = len(poly)
        for k in range(m):
            j = labels[k]
            a, b = poly[k], poly[(k + 1) % m]
            t = b - a
            nrm = np.array([t[1], -t[0]]) / np.linalg.norm(t)  # outward for CCW polygon
            if j >= 0:
                if i < j:
                    f_elem.append([i, j])
                    f_geom.append([a, b])
                    f_norm.append(nrm)
            else:
                f_elem.append([i, -1])
                f_geom.append([a, b])
                f_norm.append(nrm)

    mesh = Mesh(
        dim=2,
        cell_ptr=np.asarray(cell_ptr, dtype=np.int64),
        cell_geom=np.asarray(tri_list, dtype=np.float64),
        facet_elem=np.asarray(f_elem, dtype=np.int64),
        facet_geom=np.asarray(f_geom, dtype=np.float64),
        facet_normal=np.asarray(f_norm, dtype=np.float64),
    )
    mesh.polygons = polys
    mesh.seeds = pts
    return mesh
