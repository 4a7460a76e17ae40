"""Preconditioned conjugate gradient and the Lanczos condition-number estimate.

* PCG (Section 4: the system of eq. (4) is solved at every step by PCG with
  B_ad^{-1} of eq. (5)).  Plain Hestenes-Stiefel recurrences; stop when the
  Euclidean norm of the recurrence residual satisfies ||r_j|| <= tol ||b||
  (Section 5 uses the Euclidean relative residual).  x0 is given by the caller
  (the time stepper passes U^(k)).
* Lanczos estimate (Section 5: a tridiagonal matrix built from the PCG
  coefficients has extreme eigenvalues that approximate those of P_ad):
  T_11 = 1/alpha_1, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
  T_{j,j+1} = sqrt(beta_j)/alpha_j; kappa = lambda_max(T) / lambda_min(T).

Pinned by: dense direct solves, scipy.sparse.linalg.cg with the same stopping
rule, and brute-force generalized eigenvalues of (K, B) on small meshes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class PCGInfo:
    iters: int = 0
    relres: float = 0.0
    true_relres: float = 0.0
    converged: bool = True
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    resnorms: list = field(default_factory=list)


class PCGBreakdown(ArithmeticError):
    pass


def pcg(apply_K, b, x0, apply_B, tol, maxit):
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    info = PCGInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), info
    r = b - apply_K(x)
    rn = np.linalg.norm(r)
    info.resnorms.append(rn)
    if rn <= tol * bnorm:
        info.relres = info.true_relres = rn / bnorm
        return x, info
    z = apply_B(r)
    p = z.copy()
    rho = r @ z
    if not rho > 0:
        raise PCGBreakdown("(r, z) <= 0")
    info.converged = False
    for j in range(1, maxit + 1):
        q = apply_K(p)
        pq = p @ q
        if not pq > 0:
            raise PCGBreakdown("(p, Kp) <= 0")
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        info.alphas.append(alpha)
        rn = np.linalg.norm(r)
        info.resnorms.append(rn)
        if not np.isfinite(rn):
            raise FloatingPointError("non-finite residual")
        if rn <= tol * bnorm:
            info.iters = j
            info.converged = True
            break
        z = apply_B(r)
        rho_new = r @ z
        if not rho_new > 0:
            raise PCGBreakdown("(r, z) <= 0")
        beta = rho_new / rho
        info.betas.append(beta)
        p = z + beta * p
        rho = rho_new
    else:
        info.iters = maxit
    info.relres = rn / bnorm
    info.true_relres = np.linalg.norm(b - apply_K(x)) / bnorm
    return x, info


def lanczos_tridiagonal(alphas, betas):
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return T


def lanczos_kappa(alphas, betas):
    if len(alphas) == 0:
        return 1.0
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(alphas, betas))
    return ev[-1] / ev[0]
