"""Plain-array description of a polytopal mesh, shared as *data* by both sides.

Each element K is a union of sub-cells (triangles in 2-D, axis-aligned boxes in
3-D).  Facets are the pieces of element boundaries: a segment (2-D) or an
axis-aligned rectangle (3-D), each with the element on its minus side, the
element on its plus side (-1 on the domain boundary) and the unit normal that
points from minus to plus.  An interface between two agglomerates may consist
of several facets (each integrated separately).

Array layout (all C-contiguous)::

    cell_ptr     int64 [n_elem+1]          CSR over sub-cells
    cell_geom    f64   [n_cell,3,2]        2-D: triangle vertices
                 f64   [n_cell,2,3]        3-D: box (lo corner, hi corner)
    facet_elem   int64 [n_facet,2]         (minus, plus); plus = -1 on the boundary
    facet_geom   f64   [n_facet,2,2]       2-D: segment end points
                 f64   [n_facet,2,3]       3-D: rectangle (lo, hi); one coordinate equal
    facet_normal f64   [n_facet,dim]       unit normal, minus -> plus
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    cell_ptr: np.ndarray
    cell_geom: np.ndarray
    facet_elem: np.ndarray
    facet_geom: np.ndarray
    facet_normal: np.ndarray
    region: np.ndarray | None = None
    sigma: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return len(self.cell_ptr) - 1

    @property
    def n_cell(self) -> int:
        return len(self.cell_geom)

    @property
    def n_facet(self) -> int:
        return len(self.facet_elem)

    def cell_owner(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_elem), np.diff(self.cell_ptr))

    def cell_measure(self) -> np.ndarray:
        g = self.cell_geom
        if self.dim == 2:
            e1, e2 = g[:, 1] - g[:, 0], g[:, 2] - g[:, 0]
            return 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        return np.prod(g[:, 1] - g[:, 0], axis=1)

    def cell_center(self) -> np.ndarray:
        g = self.cell_geom
        return g.mean(axis=1)

    def element_measure(self) -> np.ndarray:
        return np.bincount(self.cell_owner(), weights=self.cell_measure(), minlength=self.n_elem)

    def element_centroid(self) -> np.ndarray:
        own, vol, c = self.cell_owner(), self.cell_measure(), self.cell_center()
        tot = np.bincount(own, weights=vol, minlength=self.n_elem)
        return np.stack([np.bincount(own, weights=vol * c[:, d], minlength=self.n_elem) / tot
                         for d in range(self.dim)], axis=1)

    def interior_facets(self) -> np.ndarray:
        return np.nonzero(self.facet_elem[:, 1] >= 0)[0]

    def element_adjacency(self):
        """Sorted unique (a, b), a < b, element pairs sharing at least one facet."""
        f = self.facet_elem[self.facet_elem[:, 1] >= 0]
        a, b = np.minimum(f[:, 0], f[:, 1]), np.maximum(f[:, 0], f[:, 1])
        return np.unique(np.stack([a, b], 1), axis=0)

    def as_abi_arrays(self):
        """Contiguous arrays in the layout the C-ABI mesh descriptor expects."""
        sig = self.sigma
        if sig is None:
            sig = np.broadcast_to(np.eye(self.dim), (self.n_elem, self.dim, self.dim))
        return dict(
            cell_ptr=np.ascontiguousarray(self.cell_ptr, dtype=np.int64),
            cell_geom=np.ascontiguousarray(self.cell_geom, dtype=np.float64),
            facet_elem=np.ascontiguousarray(self.facet_elem, dtype=np.int64),
            facet_geom=np.ascontiguousarray(self.facet_geom, dtype=np.float64),
            facet_normal=np.ascontiguousarray(self.facet_normal, dtype=np.float64),
            sigma=np.ascontiguousarray(sig, dtype=np.float64),
        )


def concat_meshes(meshes):
    """Disjoint union of meshes of one dimension: elements, sub-cells and
    facets of mesh k follow those of meshes 0..k-1 (element indices shifted).
    Returns the union and elem_ptr, the element range of every input mesh."""
    dim = meshes[0].dim
    assert all(m.dim == dim for m in meshes)
    n_el = np.array([m.n_elem for m in meshes], dtype=np.int64)
    elem_ptr = np.concatenate([[0], np.cumsum(n_el)]).astype(np.int64)
    n_cell = np.array([m.n_cell for m in meshes], dtype=np.int64)
    cell_off = np.concatenate([[0], np.cumsum(n_cell)])[:-1]
    cell_ptr = np.concatenate([[0]] + [m.cell_ptr[1:] + o for m, o in zip(meshes, cell_off)]).astype(np.int64)
    facet_elem = np.concatenate([np.where(m.facet_elem >= 0, m.facet_elem + o, -1)
                                 for m, o in zip(meshes, elem_ptr[:-1])]).astype(np.int64)
    sig = [m.sigma if m.sigma is not None else np.broadcast_to(np.eye(dim), (m.n_elem, dim, dim)) for m in meshes]
    reg = [m.region if m.region is not None else np.zeros(m.n_elem, np.int32) for m in meshes]
    out = Mesh(dim=dim, cell_ptr=cell_ptr,
               cell_geom=np.concatenate([m.cell_geom for m in meshes]),
               facet_elem=facet_elem,
               facet_geom=np.concatenate([m.facet_geom for m in meshes]),
               facet_normal=np.concatenate([m.facet_normal for m in meshes]),
               region=np.concatenate(reg), sigma=np.concatenate(sig))
    return out, elem_ptr
