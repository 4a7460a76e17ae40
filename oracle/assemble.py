"""Mass matrix, SIPG matrix and system matrix of the PolyDG discretisation.

Follows Section 3 of the paper:

* the penalty of eq. (2):  eta = eta0 {Sigma_K}_A p^2 / {h_K}_H on every interior
  facet, with the arithmetic average of Sigma_K and the harmonic average of the
  element diameters.  The paper's definition of Sigma_K is garbled (it writes
  the squared L^2(K) norm of sqrt(Sigma)); reading used: Sigma_K = largest
  eigenvalue of the (piecewise constant) tensor on K;
* the SIPG form of eq. (3): volume term (Sigma grad u, grad v)_K, the two
  consistency/symmetry terms with the average {Sigma grad .} and the vector jump
  [v] = v^- n^- + v^+ n^+ of Arnold et al., and the penalty term, all on interior
  facets only (homogeneous Neumann condition: no boundary-facet terms);
* the system matrix K = (chi_m C_m / dt) M + 1/2 A, i.e. the paper's
  K_h = C_m chi_m M_h + dt/2 A_h divided by dt (this rescaling changes neither
  the PCG iterates nor the relative residual).

Pinned by: symmetry, A 1 = 0, positive definiteness (brute force on small
meshes), consistency for global linear functions, polynomial reproduction and
manufactured-solution convergence rates (tests/test_oracle_discretisation.py);
the penalty of eq. (2) and the diameter h_K by the closed form of the SIPG form
on indicator functions of hand-built elements (tests/test_oracle_penalty.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .basis import eval_basis, n_dofs
from .quadrature import element_bbox, element_diameter, element_rule, facet_rule


@dataclass
class Discretisation:
    mesh: object
    p: int
    nd: int
    lo: np.ndarray
    hi: np.ndarray
    h: np.ndarray
    qx: np.ndarray          # element quadrature points
    qw: np.ndarray
    qe: np.ndarray
    qptr: np.ndarray        # [n_elem+1] offsets of each element's points
    M: np.ndarray           # [n_elem, nd, nd] element mass blocks
    A: sp.csr_matrix        # SIPG matrix (dof level)

    @property
    def n_elem(self):
        return self.mesh.n_elem

    @property
    def n_dof(self):
        return self.n_elem * self.nd

    def basis_at(self, x, elems, grad=False):
        return eval_basis(x, self.lo[elems], self.hi[elems], self.p, grad=grad)

    def mass_matrix(self) -> sp.csr_matrix:
        return sp.block_diag(list(self.M), format="csr")

    def system_matrix(self, chi_m, c_m, dt) -> sp.csr_matrix:
        c = chi_m * c_m / dt
        return (c * self.mass_matrix() + 0.5 * self.A).tocsr()


def _segments(qe, n_elem):
    counts = np.bincount(qe, minlength=n_elem)
    return np.concatenate([[0], np.cumsum(counts)])


def lambda_max(sigma):
    return np.linalg.eigvalsh(sigma)[:, -1]


def discretise(mesh, p, eta0, chunk=512) -> Discretisation:
    """Assemble the element mass blocks and the SIPG matrix A (eq. (3))."""
    nd = n_dofs(mesh.dim, p)
    lo, hi = element_bbox(mesh)
    h = element_diameter(mesh)
    qx, qw, qe = element_rule(mesh, p)
    qptr = _segments(qe, mesh.n_elem)
    sigma = mesh.sigma if mesh.sigma is not None else np.broadcast_to(np.eye(mesh.dim), (mesh.n_elem, mesh.dim, mesh.dim))
    n = mesh.n_elem

    M = np.zeros((n, nd, nd))
    Avol = np.zeros((n, nd, nd))
    for e0 in range(0, n, chunk):
        e1 = min(n, e0 + chunk)
        q0, q1 = qptr[e0], qptr[e1]
        el = qe[q0:q1]
        phi, dphi = eval_basis(qx[q0:q1], lo[el], hi[el], p, grad=True)
        w = qw[q0:q1]
        sg = np.einsum("qab,qjb->qja", sigma[el], dphi)          # Sigma grad phi_j
        mq = np.einsum("q,qi,qj->qij", w, phi, phi)
        aq = np.einsum("q,qia,qja->qij", w, dphi, sg)
        starts = qptr[e0:e1] - q0
        M[e0:e1] = np.add.reduceat(mq, starts, axis=0)
        Avol[e0:e1] = np.add.reduceat(aq, starts, axis=0)

    rows, cols, vals = [], [], []
    loc = np.arange(nd)
    for e in range(n):
        rows.append(np.repeat(e * nd + loc, nd))
        cols.append(np.tile(e * nd + loc, nd))
        vals.append(Avol[e].ravel())

    fint = mesh.interior_facets()
    lam = lambda_max(np.asarray(sigma))
    fe = mesh.facet_elem
    for f0 in range(0, len(fint), 4 * chunk):
        fs = fint[f0:f0 + 4 * chunk]
        fx, fw, ff = facet_rule(mesh, p, fs)
        a, b = fe[ff, 0], fe[ff, 1]
        nrm = mesh.facet_normal[ff]
        pa, da = eval_basis(fx, lo[a], hi[a], p, grad=True)
        pb, db = eval_basis(fx, lo[b], hi[b], p, grad=True)
        ga = np.einsum("qja,qa->qj", da, np.einsum("qab,qb->qa", sigma[a], nrm))  # (Sigma^- grad phi^-) . n
        gb = np.einsum("qja,qa->qj", db, np.einsum("qab,qb->qa", sigma[b], nrm))  # (Sigma^+ grad phi^+) . n
        ha, hb = h[a], h[b]
        eta = eta0 * 0.5 * (lam[a] + lam[b]) * p * p / (2.0 * ha * hb / (ha + hb))
        # test index i (rows), trial index j (cols)
        aa = -0.5 * np.einsum("qj,qi->qij", ga, pa) - 0.5 * np.einsum("qj,qi->qij", pa, ga) \
            + eta[:, None, None] * np.einsum("qj,qi->qij", pa, pa)
        ab = -0.5 * np.einsum("qj,qi->qij", gb, pa) + 0.5 * np.einsum("qj,qi->qij", pb, ga) \
            - eta[:, None, None] * np.einsum("qj,qi->qij", pb, pa)
        ba = 0.5 * np.einsum("qj,qi->qij", ga, pb) - 0.5 * np.einsum("qj,qi->qij", pa, gb) \
            - eta[:, None, None] * np.einsum("qj,qi->qij", pa, pb)
        bb = 0.5 * np.einsum("qj,qi->qij", gb, pb) + 0.5 * np.einsum("qj,qi->qij", pb, gb) \
            + eta[:, None, None] * np.einsum("qj,qi->qij", pb, pb)
        nq = len(ff) // len(fs)
        sh = (len(fs), nq, nd, nd)
        blocks = [(aa, fe[fs, 0], fe[fs, 0]), (ab, fe[fs, 0], fe[fs, 1]),
                  (ba, fe[fs, 1], fe[fs, 0]), (bb, fe[fs, 1], fe[fs, 1])]
        for arr, re, ce in blocks:
            blk = (arr * fw[:, None, None]).reshape(sh).sum(axis=1)
            rows.append((re[:, None, None] * nd + loc[None, :, None] + 0 * loc[None, None, :]).ravel())
            cols.append((ce[:, None, None] * nd + 0 * loc[None, :, None] + loc[None, None, :]).ravel())
            vals.append(blk.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n * nd, n * nd)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return Discretisation(mesh, p, nd, lo, hi, h, qx, qw, qe, qptr, M, A)


def project_elementwise(disc: Discretisation, values_at_points):
    """L^2 projection onto V_h of a function given by its values at the element
    quadrature points: U_K = M_K^{-1} int_K f phi."""
    phi = disc.basis_at(disc.qx, disc.qe)
    rhs = np.zeros((disc.n_elem, disc.nd))
    np.add.at(rhs, disc.qe, (disc.qw * values_at_points)[:, None] * phi)
    return np.linalg.solve(disc.M, rhs[..., None])[..., 0]


def project_piecewise_constant(disc: Discretisation, elem_values):
    """L^2 projection of a per-element constant function (initial data)."""
    v = np.asarray(elem_values, dtype=np.float64)
    return project_elementwise(disc, v[disc.qe])


def evaluate(disc: Discretisation, U, x, elems):
    """u_h(x) for points x inside the given elements."""
    phi = disc.basis_at(x, elems)
    Ue = np.asarray(U).reshape(disc.n_elem, disc.nd)[elems]
    return np.einsum("qi,qi->q", phi, Ue)
