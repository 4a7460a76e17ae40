"""Two-level additive Schwarz preconditioner (Section 4, eq. (5)).

    B^{-1} = sum_{i=0}^{N} R_i^T K_i^{-1} R_i,   K_i = R_i K R_i^T.

* Local level (i = 1..N): R_i^T extends by zero the dofs of the elements of
  subdomain i, so K_i is the principal submatrix of K on those dofs; it is
  factorised with a dense Cholesky factorisation (scipy.linalg.cho_factor).
* Coarse level (i = 0): V_0 = P^q on every coarse element (an agglomerate of
  fine elements), with the same modal Legendre basis taken on the coarse
  element's bounding box.  R_0^T is the L^2 projection V_0 -> V_h; since V_0 is
  contained in V_h it is exact: the matrix P with blocks
  P_K = M_K^{-1} int_K phi_K psi_c^T.  Reading of the "L^2 adjoint" R_0 in matrix
  form: R_0 = P^T (the residual is a dual vector), which keeps B symmetric as
  PCG requires.  K_0 = P^T K P, factorised with dense Cholesky.

Pinned by: special cases (one subdomain without coarse level is the exact
inverse; element-sized subdomains give block-Jacobi; one subdomain plus the
coarse level gives P_ad eigenvalues in {1, 2}), symmetry and positive
definiteness of B, and exactness of the coarse transfer (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import eval_basis, n_dofs


class Schwarz:
    def __init__(self, disc, K, elem_sub, elem_coarse=None, coarse_q=1):
        self.disc = disc
        nd = disc.nd
        elem_sub = np.asarray(elem_sub)
        self.n_sub = int(elem_sub.max()) + 1
        self.dofs = []
        self.chol = []
        Kc = K.tocsr()
        for i in range(self.n_sub):
            els = np.nonzero(elem_sub == i)[0]
            if len(els) == 0:
                raise ValueError(f"subdomain {i} is empty")
            d = (els[:, None] * nd + np.arange(nd)[None, :]).ravel()
            Ki = Kc[d][:, d].toarray()
            self.dofs.append(d)
            self.chol.append(sla.cho_factor(Ki, lower=True))
        self.coarse_q = int(coarse_q)
        self.P = None
        if self.coarse_q > 0:
            ec = elem_sub if elem_coarse is None else np.asarray(elem_coarse)
            self.P = coarse_prolongation(disc, ec, self.coarse_q)
            self.K0 = (self.P.T @ (Kc @ self.P)).toarray()
            self.K0 = 0.5 * (self.K0 + self.K0.T)
            self.chol0 = sla.cho_factor(self.K0, lower=True)

    def local_factors(self):
        """The scipy cho_factor storage of every K_i (for tests): its lower
        triangle is the Cholesky factor L_i with L_i L_i^T = K_i; the entries
        above the diagonal are left over from K_i and carry no meaning."""
        return [c[0] for c in self.chol]

    def apply(self, r):
        """z = B^{-1} r (eq. (5))."""
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        for d, c in zip(self.dofs, self.chol):
            z[d] += sla.cho_solve(c, r[d])
        if self.P is not None:
            z += self.P @ sla.cho_solve(self.chol0, self.P.T @ r)
        return z

    def apply_local(self, r):
        z = np.zeros_like(r)
        for d, c in zip(self.dofs, self.chol):
            z[d] += sla.cho_solve(c, r[d])
        return z


def coarse_prolongation(disc, elem_coarse, q):
    """P: coefficients of the coarse basis psi_c (degree q on each coarse
    element's bounding box) in the fine basis, P_K = M_K^{-1} int_K phi psi^T."""
    mesh = disc.mesh
    ec = np.asarray(elem_coarse)
    n0 = int(ec.max()) + 1
    nq0 = n_dofs(mesh.dim, q)
    clo = np.full((n0, mesh.dim), np.inf)
    chi = np.full((n0, mesh.dim), -np.inf)
    np.minimum.at(clo, ec, disc.lo)
    np.maximum.at(chi, ec, disc.hi)
    qc = ec[disc.qe]
    phi = disc.basis_at(disc.qx, disc.qe)
    psi = eval_basis(disc.qx, clo[qc], chi[qc], q)
    G = np.zeros((disc.n_elem, disc.nd, nq0))
    np.add.at(G, disc.qe, disc.qw[:, None, None] * phi[:, :, None] * psi[:, None, :])
    PK = np.linalg.solve(disc.M, G)                    # [n_elem, nd, nq0]
    rows = (np.arange(disc.n_elem)[:, None, None] * disc.nd + np.arange(disc.nd)[None, :, None]
            + 0 * np.arange(nq0)[None, None, :])
    cols = ec[:, None, None] * nq0 + np.arange(nq0)[None, None, :] + 0 * rows
    return sp.csr_matrix((PK.ravel(), (rows.ravel(), cols.ravel())), shape=(disc.n_dof, n0 * nq0))
