"""Quadrature on polytopal elements and their facets (Section 3).

The paper does not state its quadrature.  Reading used on both sides:

* 2-D elements are split into a fan of sub-triangles (given by the mesh).  On a
  triangle (v0, v1, v2) the collapsed map x(s, t) = (1-s) v0 + s((1-t) v1 + t v2),
  (s, t) in [0, 1]^2, with (p+2) Gauss-Legendre points in s and in t; Jacobian
  s |det(v1 - v0, v2 - v1)|.  Exact for polynomials of degree 2p + 2.
* 3-D elements are unions of boxes: (p+1)^3 tensor Gauss-Legendre points per box.
* Facets: (p+2) Gauss-Legendre points per 2-D segment; (p+1)^2 tensor points per
  3-D rectangle.

Pinned by: closed-form polygon and box moments (Green's theorem / exact sums).
"""
from __future__ import annotations

import numpy as np


def gauss01(n):
    """n-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def element_rule(mesh, p):
    """Quadrature points of every element.

    Returns (x [Q, d], w [Q], elem [Q]); points are grouped by element in
    element order (contiguous), sub-cell by sub-cell.
    """
    own = mesh.cell_owner()
    g = mesh.cell_geom
    if mesh.dim == 2:
        s, ws = gauss01(p + 2)
        S, T = np.meshgrid(s, s, indexing="ij")
        W = np.outer(ws, ws)
        S, T, W = S.ravel(), T.ravel(), W.ravel()
        v0, v1, v2 = g[:, 0], g[:, 1], g[:, 2]
        x = ((1.0 - S)[None, :, None] * v0[:, None, :]
             + S[None, :, None] * ((1.0 - T)[None, :, None] * v1[:, None, :] + T[None, :, None] * v2[:, None, :]))
        e1, e2 = v1 - v0, v2 - v1
        det = np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        w = W[None, :] * S[None, :] * det[:, None]
    else:
        s, ws = gauss01(p + 1)
        P = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1).reshape(-1, 3)
        W = np.einsum("i,j,k->ijk", ws, ws, ws).ravel()
        lo, hi = g[:, 0], g[:, 1]
        x = lo[:, None, :] + P[None, :, :] * (hi - lo)[:, None, :]
        w = W[None, :] * np.prod(hi - lo, axis=1)[:, None]
    nq = x.shape[1]
    return x.reshape(-1, mesh.dim), w.ravel(), np.repeat(own, nq)


def facet_rule(mesh, p, facets=None):
    """Quadrature points on facets.  Returns (x [Fq, d], w [Fq], facet [Fq])."""
    idx = np.arange(mesh.n_facet) if facets is None else np.asarray(facets)
    g = mesh.facet_geom[idx]
    if mesh.dim == 2:
        s, ws = gauss01(p + 2)
        a, b = g[:, 0], g[:, 1]
        x = a[:, None, :] + s[None, :, None] * (b - a)[:, None, :]
        w = ws[None, :] * np.linalg.norm(b - a, axis=1)[:, None]
    else:
        s, ws = gauss01(p + 1)
        lo, hi = g[:, 0], g[:, 1]
        ext = hi - lo
        flat = ext == 0.0
        assert np.all(flat.sum(1) == 1), "3-D facets must be axis-aligned rectangles"
        ax = np.argmax(flat, axis=1)
        t1 = np.where(ax == 0, 1, 0)
        t2 = np.where(ax == 2, 1, 2)
        U, V = np.meshgrid(s, s, indexing="ij")
        U, V = U.ravel(), V.ravel()
        WW = np.outer(ws, ws).ravel()
        rows = np.arange(len(idx))
        x = np.empty((len(idx), len(U), 3))
        x[rows, :, ax] = lo[rows, ax][:, None]
        x[rows, :, t1] = lo[rows, t1][:, None] + U[None, :] * ext[rows, t1][:, None]
        x[rows, :, t2] = lo[rows, t2][:, None] + V[None, :] * ext[rows, t2][:, None]
        w = WW[None, :] * (ext[rows, t1] * ext[rows, t2])[:, None]
    nq = x.shape[1]
    return x.reshape(-1, mesh.dim), w.ravel(), np.repeat(idx, nq)


def element_bbox(mesh):
    """Bounding box (lo, hi) [n_elem, d] of every element's sub-cell vertices."""
    own = mesh.cell_owner()
    g = mesh.cell_geom
    lo = np.full((mesh.n_elem, mesh.dim), np.inf)
    hi = np.full((mesh.n_elem, mesh.dim), -np.inf)
    np.minimum.at(lo, own, g.min(axis=1))
    np.maximum.at(hi, own, g.max(axis=1))
    return lo, hi


def element_diameter(mesh):
    """h_K: largest distance between two sub-cell vertices of K (Section 3)."""
    h = np.zeros(mesh.n_elem)
    for e in range(mesh.n_elem):
        g = mesh.cell_geom[mesh.cell_ptr[e]:mesh.cell_ptr[e + 1]]
        if mesh.dim == 2:
            v = g.reshape(-1, 2)
        else:
            lo, hi = g[:, 0], g[:, 1]
            corners = []
            for m in range(8):
                sel = [(m >> d) & 1 for d in range(3)]
                corners.append(np.where(np.array(sel)[None, :] == 1, hi, lo))
            v = np.concatenate(corners)
        v = np.unique(v, axis=0)
        d2 = ((v[:, None, :] - v[None, :, :]) ** 2).sum(-1)
        h[e] = np.sqrt(d2.max())
    return h
