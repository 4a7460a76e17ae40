"""Pins of the oracle's Schwarz preconditioner, PCG, time stepping and ionic
model against library routines, brute force, closed forms and exact special
cases."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy.integrate import solve_ivp

from oracle import ionic
from oracle.assemble import evaluate
from oracle.basis import eval_basis
from oracle.monodomain import Monodomain
from oracle.pcg import lanczos_kappa, pcg
from oracle.schwarz import Schwarz, coarse_prolongation
from pdg_inputs import params, problems

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_B(sch, n):
    return np.stack([sch.apply(e) for e in np.eye(n)], 1)


@pytest.fixture(scope="module")
def small2d():
    pr = problems.small2d(n=20, p=2)
    return pr, Monodomain(pr)


def test_pcg_matches_dense_solve_and_scipy_cg(small2d):
    pr, md = small2d
    rng = np.random.default_rng(1)
    b = rng.standard_normal(pr.n_dof)
    x0 = rng.standard_normal(pr.n_dof)
    x, info = md.solve(b, x0, tol=1e-10)
    K = md.K.toarray()
    xd = np.linalg.solve(K, b)
    kappaK = np.linalg.cond(K)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= kappaK * 1e-10
    # scipy's cg with the same preconditioner and the same ||r|| <= rtol ||b|| rule
    count = [0]

    def cb(_):
        count[0] += 1
    Bop = spla.LinearOperator(K.shape, matvec=md.schwarz.apply)
    xs, flag = spla.cg(md.K, b, x0=x0, rtol=1e-10, atol=0.0, M=Bop, callback=cb, maxiter=1000)
    assert flag == 0
    assert abs(count[0] - info.iters) <= 1
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-8 * np.abs(xd).max())


def test_schwarz_one_subdomain_no_coarse_is_exact(small2d):
    pr, md = small2d
    sch = Schwarz(md.disc, md.K, np.zeros(pr.n_elem, int), coarse_q=0)
    b = np.random.default_rng(2).standard_normal(pr.n_dof)
    x, info = pcg(lambda v: md.K @ v, b, np.zeros_like(b), sch.apply, 1e-10, 50)
    assert info.iters == 1


def test_schwarz_one_subdomain_plus_coarse_spectrum(small2d):
    pr, md = small2d
    sch = Schwarz(md.disc, md.K, np.zeros(pr.n_elem, int), np.zeros(pr.n_elem, int), coarse_q=1)
    B = _dense_B(sch, pr.n_dof)
    ev = np.sort(np.linalg.eigvals(B @ md.K.toarray()).real)
    assert np.all(np.minimum(abs(ev - 1), abs(ev - 2)) < 1e-9)
    assert np.sum(abs(ev - 2) < 1e-9) == 3  # dim P^1 on one coarse element in 2-D
    b = np.random.default_rng(3).standard_normal(pr.n_dof)
    _, info = pcg(lambda v: md.K @ v, b, np.zeros_like(b), sch.apply, 1e-10, 50)
    assert info.iters <= 2


def test_schwarz_element_blocks_is_block_jacobi(small2d):
    pr, md = small2d
    nd = pr.nd
    sch = Schwarz(md.disc, md.K, np.arange(pr.n_elem), coarse_q=0)
    K = md.K.toarray()
    Bj = np.zeros_like(K)
    for e in range(pr.n_elem):
        s = slice(e * nd, (e + 1) * nd)
        Bj[s, s] = np.linalg.inv(K[s, s])
    np.testing.assert_allclose(_dense_B(sch, pr.n_dof), Bj, rtol=0, atol=1e-12 * abs(Bj).max())


def test_schwarz_symmetric_positive_definite(small2d):
    pr, md = small2d
    B = _dense_B(md.schwarz, pr.n_dof)
    assert abs(B - B.T).max() <= 1e-13 * abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    # local part: restriction of K to each subdomain is the principal submatrix
    K = md.K.toarray()
    for d, Ki in zip(md.schwarz.dofs, md.schwarz.local_factors()):
        L = np.tril(Ki)
        np.testing.assert_allclose(L @ L.T, K[np.ix_(d, d)], rtol=0, atol=1e-11 * abs(K).max())


@pytest.mark.parametrize("q", [1, 2])
def test_coarse_transfer_reproduces_coarse_basis(small2d, q):
    pr, md = small2d
    d = md.disc
    P = coarse_prolongation(d, pr.elem_coarse, q).toarray()
    nq0 = (q + 1) * (q + 2) // 2
    ec = pr.elem_coarse
    n0 = ec.max() + 1
    clo = np.array([d.lo[ec == c].min(0) for c in range(n0)])
    chi = np.array([d.hi[ec == c].max(0) for c in range(n0)])
    rng = np.random.default_rng(4)
    for e in range(pr.n_elem):
        # random points inside the element's first sub-triangle
        tri = pr.mesh.cell_geom[pr.mesh.cell_ptr[e]]
        ab = rng.random((4, 2))
        ab = np.where(ab.sum(1, keepdims=True) > 1, 1 - ab, ab)
        x = tri[0] + ab[:, :1] * (tri[1] - tri[0]) + ab[:, 1:] * (tri[2] - tri[0])
        phi = eval_basis(x, np.repeat(d.lo[e:e + 1], 4, 0), np.repeat(d.hi[e:e + 1], 4, 0), pr.p)
        c = ec[e]
        psi = eval_basis(x, np.repeat(clo[c:c + 1], 4, 0), np.repeat(chi[c:c + 1], 4, 0), q)
        PK = P[e * pr.nd:(e + 1) * pr.nd, c * nq0:(c + 1) * nq0]
        np.testing.assert_allclose(phi @ PK, psi, rtol=0, atol=1e-12 * abs(psi).max())


def test_lanczos_kappa_matches_generalized_eigenvalues(small2d):
    pr, md = small2d
    b = np.random.default_rng(5).standard_normal(pr.n_dof)
    _, info = md.solve(b, np.zeros_like(b), tol=1e-12)
    B = _dense_B(md.schwarz, pr.n_dof)
    ev = sla.eigh(md.K.toarray(), np.linalg.inv(B), eigvals_only=True)
    kappa = ev[-1] / ev[0]
    est = lanczos_kappa(info.alphas, info.betas)
    assert est <= kappa * (1 + 1e-8)
    assert est >= 0.99 * kappa


def test_crank_nicolson_second_order_in_time():
    """Pure diffusion (ionic terms off) started from a generalized eigenvector
    A v = lam M v: the semi-discrete solution is exp(-lam t / (chi C)) v, and
    the time stepper's error at T decays like dt^2."""
    pr = problems.small2d(n=16, p=2)
    T = 0.05
    md0 = Monodomain(pr, with_schwarz=False)
    lam, V = sla.eigh(md0.disc.A.toarray(), md0.disc.mass_matrix().toarray())
    k = 3
    v = V[:, k]
    errs = []
    for nsteps in (4, 8, 16, 32):
        pr.dt = T / nsteps
        md = Monodomain(pr, with_schwarz=False)
        U, Up, Y = v.copy(), v.copy(), np.zeros((5, pr.n_dof))
        for _ in range(nsteps):
            U, Up, Y, _ = md.step(U, Up, Y, tol=1e-14, precond=False, ionic_on=False)
        errs.append(np.linalg.norm(U - np.exp(-lam[k] * T / (pr.chi_m * pr.c_m)) * v))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(abs(r - 2.0) < 0.1 for r in rates), (lam[k], errs, rates)


def test_mass_conservation_without_ionic_terms(cfg1_oracle):
    md = cfg1_oracle
    U, Up, Y = md.initial_state()
    one = np.zeros(md.disc.n_dof)
    from oracle.assemble import project_piecewise_constant
    one = project_piecewise_constant(md.disc, np.ones(md.disc.n_elem)).ravel()
    m0 = one @ (md.Mmat @ U)
    for _ in range(3):
        U, Up, Y, info = md.step(U, Up, Y, ionic_on=False)
        mk = one @ (md.Mmat @ U)
        # K U^(k+1) = b holds to the PCG tolerance, so the mass moves by at most
        # |1^T r| / c with ||r|| <= tol ||b||
        b = 2 * md.c * (md.Mmat @ Up) - md.K @ Up
        assert abs(mk - m0) <= np.linalg.norm(one) * 1e-10 * np.linalg.norm(b) / md.c * 1.01
        m0 = mk


@pytest.mark.parametrize("reading", ["midpoint", "endpoint"])
def test_uniform_state_reduces_to_single_cell_recurrence(reading):
    """Spatially uniform data: every element follows the 0-D recurrence
    y^(k+1) = y^k + dt dy/dt(u^k, y^k); C_m (u^(k+1) - u^k) = -dt f(u~, y^(k+1)),
    with u~ = (3u^k - u^(k-1))/2 (mid-point reading) or 2u^k - u^(k-1)."""
    pr = problems.small2d(n=12, p=1)
    pr.u0_elem[:] = -52.0
    pr.ion_extrap = reading
    md = Monodomain(pr)
    U, Up, Y = md.initial_state()
    u, up, y = -52.0, -52.0, params.Y_REST.copy()
    prm = pr.ionic
    for _ in range(5):
        U, Up, Y, info = md.step(U, Up, Y, tol=1e-13)
        ynew = y + pr.dt * ionic.dydt(np.array(u), y, prm)
        ut = (3.0 * u - up) / 2.0 if reading == "midpoint" else 2.0 * u - up
        unew = u - pr.dt / pr.c_m * ionic.f_ion(np.array(ut), ynew, prm)
        up, u, y = u, float(unew), ynew
        d = md.disc
        np.testing.assert_allclose(evaluate(d, U, d.qx, d.qe), u, rtol=1e-9)
        for l in range(5):
            np.testing.assert_allclose(evaluate(d, Y[l], d.qx, d.qe), y[l], rtol=1e-9, atol=1e-12)


def test_ionic_forward_euler_converges_to_adaptive_ode_solution():
    prm = params.IONIC_DEFAULT
    T = 2.0

    def rhs(t, s):
        V, y = s[0], s[1:]
        return np.concatenate([[-ionic.f_ion(np.array(V), y, prm) / 1.0], ionic.dydt(np.array(V), y, prm)])
    s0 = np.concatenate([[-50.0], params.Y_REST])
    ref = solve_ivp(rhs, (0, T), s0, method="LSODA", rtol=1e-11, atol=1e-12).y[:, -1]
    errs = []
    for n in (2000, 4000, 8000):
        dt = T / n
        s = s0.copy()
        for _ in range(n):
            s = s + dt * rhs(0, s)
        errs.append(np.abs(s - ref).max())
    rate = np.log2(errs[1] / errs[2])
    assert 0.8 < rate < 1.3, errs


def test_rest_gates_and_firing():
    n_inf, h_inf = ionic.gate_steady_state(params.U_REST)
    assert abs(n_inf - params.Y_REST[0]) < 1e-3 and abs(h_inf - params.Y_REST[1]) < 1e-3
    prm = params.IONIC_DEFAULT
    # a suprathreshold depolarisation fires an action potential (V crosses 0 mV)
    V, y, dt = -45.0, params.Y_REST.copy(), 1e-3
    vmax = V
    for _ in range(5000):
        dv = -ionic.f_ion(np.array(V), y, prm)
        y = y + dt * ionic.dydt(np.array(V), y, prm)
        V = V + dt * dv
        vmax = max(vmax, V)
    assert vmax > 0.0
    # the xexp series branch agrees with the closed form next to the switch point
    x = np.array([0.99e-4, 1.01e-4, -0.99e-4, -1.01e-4])
    np.testing.assert_allclose(ionic._xexp(x), x / (1 - np.exp(-x)), rtol=1e-12)


def test_paper_claim_preconditioner_cuts_iterations(cfg1_oracle):
    """Section 5 / Table 1: the two-level preconditioner reduces kappa and the
    iteration count by large factors compared with plain CG (the paper's
    smallest CG/PCG iteration ratio is 596/69 ~ 8.6)."""
    with open(os.path.join(GOLDEN, "table1_paper.json")) as f:
        t1 = json.load(f)
    ratio_paper = min(cg[1] / pc[1] for cg, pc in zip(t1["p1"]["CG"], t1["p1"]["H=2h"]))
    assert ratio_paper > 8
    md = cfg1_oracle
    U, Up, Y = md.initial_state()
    Yn, I = md.ionic_update(U, Up, Y)
    b = md.rhs(U, I)
    _, pc = md.solve(b, U, precond=True)
    _, cg = md.solve(b, U, precond=False)
    assert cg.iters / pc.iters > 3
    assert lanczos_kappa(cg.alphas, cg.betas) / lanczos_kappa(pc.alphas, pc.betas) > 10
