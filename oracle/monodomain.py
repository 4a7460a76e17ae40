"""One fully discrete time step of the monodomain / ionic system (eq. (4)).

Per step k (Section 3):

1. ionic update (second line of eq. (4)):
   M Y_l^(k+1) = M Y_l^(k) - dt G_l^(k),  G_l,i = int_K m_l(u_h^k, y_h^k) phi_i,
   element by element (M is block diagonal);
2. extrapolated ion term: I^(k+1)_i = int_K f(u~, y_h^(k+1)) phi_i with the
   second-order explicit extrapolation of the potential to t^(k+1),
   u~ = 2 u_h^k - u_h^(k-1), as eq. (4) writes the term (default,
   ``problem.ion_extrap = "endpoint"``).  The extrapolation to the
   Crank-Nicolson mid-point, u~ = (3 u_h^k - u_h^(k-1)) / 2
   (``"midpoint"``), is the reading taken at dt = 0.05 ms, where the
   extrapolation to t^(k+1) diverges with this ionic model;
   at k = 0, U^(-1) := U^(0);
3. right-hand side of the first line of eq. (4) divided by dt:
   b = (c M - 1/2 A) U^k - chi_m I + F = 2 c M U^k - K U^k - chi_m I + F,
   c = chi_m C_m / dt, F = 0 in every workload here (no applied current);
4. PCG on K U^(k+1) = b with x0 = U^k and B_ad^{-1} of eq. (5).

All integrals use the element quadrature of :mod:`oracle.quadrature`.
"""
from __future__ import annotations

import numpy as np

from . import ionic
from .assemble import discretise, project_piecewise_constant
from .pcg import pcg
from .schwarz import Schwarz


class Monodomain:
    def __init__(self, problem, with_schwarz=True, cache_basis=True):
        self.pr = problem
        self.disc = discretise(problem.mesh, problem.p, problem.eta0)
        d = self.disc
        self.c = problem.chi_m * problem.c_m / problem.dt
        self.K = d.system_matrix(problem.chi_m, problem.c_m, problem.dt)
        self.Mmat = d.mass_matrix()
        self.Minv = np.linalg.inv(d.M)
        self.prm = np.asarray(problem.ionic, dtype=np.float64)
        # u~ of the ion term: 2u^k - u^(k-1) at t^(k+1), or (3u^k - u^(k-1))/2 at the mid-point
        mode = getattr(problem, "ion_extrap", "endpoint")
        self.ext = {"midpoint": (1.5, -0.5), "endpoint": (2.0, -1.0)}[mode]
        self.schwarz = None
        if with_schwarz:
            self.schwarz = Schwarz(d, self.K, problem.elem_sub, problem.elem_coarse, problem.coarse_q)
        self._phi = d.basis_at(d.qx, d.qe) if cache_basis else None

    # -- initial data -------------------------------------------------------
    def initial_state(self):
        d = self.disc
        U0 = project_piecewise_constant(d, self.pr.u0_elem).ravel()
        Y0 = np.stack([project_piecewise_constant(d, self.pr.y0_elem[l]).ravel()
                       for l in range(self.pr.y0_elem.shape[0])])
        return U0, U0.copy(), Y0

    # -- pieces of one step ---------------------------------------------------
    def _chunks(self, chunk=2048):
        d = self.disc
        for e0 in range(0, d.n_elem, chunk):
            e1 = min(d.n_elem, e0 + chunk)
            q0, q1 = d.qptr[e0], d.qptr[e1]
            phi = self._phi[q0:q1] if self._phi is not None else d.basis_at(d.qx[q0:q1], d.qe[q0:q1])
            yield e0, e1, q0, q1, phi

    def ionic_update(self, U, Uprev, Y):
        """Returns (Y^(k+1), I^(k+1)) (eq. (4), second line, and the ion term)."""
        d, dt, nd = self.disc, self.pr.dt, self.disc.nd
        n = d.n_elem
        Ue, Upe = U.reshape(n, nd), Uprev.reshape(n, nd)
        Ye = Y.reshape(Y.shape[0], n, nd)
        Ynew = np.empty_like(Ye)
        I = np.zeros((n, nd))
        for e0, e1, q0, q1, phi in self._chunks():
            el = d.qe[q0:q1]
            w = d.qw[q0:q1]
            uq = np.einsum("qi,qi->q", phi, Ue[el])
            yq = np.einsum("qi,lqi->lq", phi, Ye[:, el])
            mq = ionic.m_ion(uq, yq, self.prm)                      # [5, Q]
            G = np.zeros((Ye.shape[0], e1 - e0, nd))
            for l in range(Ye.shape[0]):
                np.add.at(G[l], el - e0, (w * mq[l])[:, None] * phi)
            Ynew[:, e0:e1] = Ye[:, e0:e1] - dt * np.einsum("eij,lej->lei", self.Minv[e0:e1], G)
            ut = self.ext[0] * uq + self.ext[1] * np.einsum("qi,qi->q", phi, Upe[el])
            yn = np.einsum("qi,lqi->lq", phi, Ynew[:, el])
            fq = ionic.f_ion(ut, yn, self.prm)
            np.add.at(I, el, (w * fq)[:, None] * phi)
        return Ynew.reshape(Y.shape), I.ravel()

    def rhs(self, U, I, F=None):
        b = 2.0 * self.c * (self.Mmat @ U) - self.K @ U - self.pr.chi_m * I
        if F is not None:
            b = b + F
        return b

    def solve(self, b, x0, tol=None, maxit=None, precond=True):
        tol = self.pr.tol if tol is None else tol
        maxit = self.pr.maxit if maxit is None else maxit
        B = self.schwarz.apply if (precond and self.schwarz is not None) else (lambda r: r.copy())
        return pcg(lambda v: self.K @ v, b, x0, B, tol, maxit)

    def step(self, U, Uprev, Y, tol=None, maxit=None, precond=True, F=None, ionic_on=True):
        if ionic_on:
            Ynew, I = self.ionic_update(U, Uprev, Y)
        else:  # pure diffusion (f = 0, m = 0): used by the time-order and conservation pins
            Ynew, I = Y.copy(), np.zeros_like(U)
        b = self.rhs(U, I, F)
        Unew, info = self.solve(b, U, tol, maxit, precond)
        return Unew, U.copy(), Ynew, info

    def run(self, n_steps=None, **kw):
        n_steps = self.pr.n_steps if n_steps is None else n_steps
        U, Up, Y = self.initial_state()
        out = []
        for _ in range(n_steps):
            U, Up, Y, info = self.step(U, Up, Y, **kw)
            out.append((U.copy(), Y.copy(), info))
        return out
