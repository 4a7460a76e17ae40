"""Modal basis of the broken space V_h = P^p(T_h) (Section 3).

The paper does not fix a basis.  Reading used here: on each element K with
bounding box [a, b], the tensor Legendre polynomials of total degree <= p,

    phi_alpha(x) = prod_j sqrt((2 alpha_j + 1) / (b_j - a_j)) L_{alpha_j}(xi_j),
    xi_j = 2 (x_j - a_j) / (b_j - a_j) - 1,

which are orthonormal in L^2 of the box (so the element mass matrix is the
identity on box-shaped elements).  Ordering: total degree ascending, then
alpha_1 descending, then alpha_2 descending.

Pinned by: orthonormality on boxes (closed form), reproduction of polynomials
of degree <= p by the L^2 projection.
"""
from __future__ import annotations

import itertools

import numpy as np
from numpy.polynomial import legendre as npleg


def multi_indices(dim: int, p: int) -> np.ndarray:
    out = []
    for deg in range(p + 1):
        block = [a for a in itertools.product(range(deg + 1), repeat=dim) if sum(a) == deg]
        block.sort(key=lambda a: tuple(-x for x in a))
        out.extend(block)
    return np.array(out, dtype=np.int64)


def n_dofs(dim: int, p: int) -> int:
    return len(multi_indices(dim, p))


def _legendre_table(xi, p):
    """L_k(xi) and L_k'(xi) for k = 0..p (via numpy's Legendre series)."""
    vals = np.empty((p + 1,) + xi.shape)
    ders = np.empty((p + 1,) + xi.shape)
    for k in range(p + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        vals[k] = npleg.legval(xi, c)
        ders[k] = npleg.legval(xi, npleg.legder(c)) if k > 0 else 0.0
    return vals, ders


def eval_basis(x, lo, hi, p, grad=False):
    """Basis values (and gradients) at points ``x`` [Q, d] of boxes [lo, hi]
    given per point ([Q, d] each).  Returns phi [Q, nd] (and dphi [Q, nd, d])."""
    x, lo, hi = np.asarray(x), np.asarray(lo), np.asarray(hi)
    dim = x.shape[1]
    mi = multi_indices(dim, p)
    ext = hi - lo
    xi = 2.0 * (x - lo) / ext - 1.0
    tabs = [_legendre_table(xi[:, j], p) for j in range(dim)]
    scale = [np.sqrt((2.0 * np.arange(p + 1)[:, None] + 1.0) / ext[None, :, j]) for j in range(dim)]
    Q = x.shape[0]
    phi = np.ones((Q, len(mi)))
    for k, a in enumerate(mi):
        for j in range(dim):
            phi[:, k] *= scale[j][a[j]] * tabs[j][0][a[j]]
    if not grad:
        return phi
    dphi = np.ones((Q, len(mi), dim))
    for k, a in enumerate(mi):
        for g in range(dim):
            for j in range(dim):
                if j == g:
                    dphi[:, k, g] *= scale[j][a[j]] * tabs[j][1][a[j]] * (2.0 / ext[:, j])
                else:
                    dphi[:, k, g] *= scale[j][a[j]] * tabs[j][0][a[j]]
    return phi, dphi
