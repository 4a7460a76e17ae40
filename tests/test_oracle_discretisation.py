"""Pins of the oracle's basis, quadrature and assembly against closed forms and
exact special cases (not against the oracle's own formulas)."""
import numpy as np
import pytest

from oracle.assemble import discretise, evaluate, project_elementwise
from oracle.basis import eval_basis, multi_indices
from oracle.quadrature import element_rule, facet_rule
from pdg_inputs import problems
from pdg_inputs.mesh2d import voronoi_mesh
from pdg_inputs.mesh3d import agglomerated_cube_mesh
from pdg_inputs.problems import isotropic_sigma


def _polygon_moment(poly, a, b):
    """int_P x^a y^b by Green's theorem: int x^a y^b = oint x^(a+1) y^b / (a+1) dy,
    evaluated exactly on each edge with a high-order 1-D Gauss rule."""
    xg, wg = np.polynomial.legendre.leggauss(a + b + 3)
    xg, wg = 0.5 * (xg + 1), 0.5 * wg
    tot = 0.0
    for k in range(len(poly)):
        p0, p1 = poly[k], poly[(k + 1) % len(poly)]
        x = p0[0] + xg * (p1[0] - p0[0])
        y = p0[1] + xg * (p1[1] - p0[1])
        tot += np.sum(wg * x ** (a + 1) * y ** b) * (p1[1] - p0[1]) / (a + 1)
    return tot


@pytest.mark.parametrize("p", [1, 2, 4])
def test_quadrature_polygon_moments(p):
    mesh = voronoi_mesh(16, seed=7, lloyd=3)
    x, w, e = element_rule(mesh, p)
    for a in range(2 * p + 3):
        for b in range(2 * p + 3 - a):
            got = np.bincount(e, weights=w * x[:, 0] ** a * x[:, 1] ** b, minlength=mesh.n_elem)
            want = np.array([_polygon_moment(poly, a, b) for poly in mesh.polygons])
            np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def test_quadrature_box_moments():
    pr = problems.small3d(n_grid=4, p=2)
    x, w, e = element_rule(pr.mesh, 2)
    g = pr.mesh.cell_geom
    own = pr.mesh.cell_owner()
    for a, b, c in [(0, 0, 0), (2, 1, 2), (5, 0, 1), (3, 3, 0)]:
        got = np.bincount(e, weights=w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c, minlength=pr.n_elem)
        cellm = ((g[:, 1, 0] ** (a + 1) - g[:, 0, 0] ** (a + 1)) / (a + 1)
                 * (g[:, 1, 1] ** (b + 1) - g[:, 0, 1] ** (b + 1)) / (b + 1)
                 * (g[:, 1, 2] ** (c + 1) - g[:, 0, 2] ** (c + 1)) / (c + 1))
        want = np.bincount(own, weights=cellm, minlength=pr.n_elem)
        np.testing.assert_allclose(got, want, rtol=1e-13)


def test_facet_rule_lengths(cfg1_problem):
    m = cfg1_problem.mesh
    x, w, f = facet_rule(m, 2)
    L = np.bincount(f, weights=w, minlength=m.n_facet)
    np.testing.assert_allclose(L, np.linalg.norm(m.facet_geom[:, 1] - m.facet_geom[:, 0], axis=1), rtol=1e-14)


def test_basis_ordering():
    assert multi_indices(2, 2).tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]
    assert multi_indices(3, 1).tolist() == [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    assert len(multi_indices(3, 4)) == 35 and len(multi_indices(2, 4)) == 15


def test_mass_is_identity_on_box_elements():
    mesh = agglomerated_cube_mesh(3, 2.0, seed=1, target=1)
    mesh.sigma = isotropic_sigma(mesh.n_elem, 3, 1.0)
    d = discretise(mesh, 3, eta0=10.0)
    for M in d.M:
        np.testing.assert_allclose(M, np.eye(d.nd), atol=1e-13)


def test_basis_gradient_matches_finite_difference():
    rng = np.random.default_rng(0)
    x = rng.random((5, 3))
    lo, hi = np.zeros((5, 3)) - 0.3, np.ones((5, 3)) * 1.7
    phi, dphi = eval_basis(x, lo, hi, 3, grad=True)
    for g in range(3):
        e = np.zeros(3)
        e[g] = 1e-6
        fd = (eval_basis(x + e, lo, hi, 3) - eval_basis(x - e, lo, hi, 3)) / 2e-6
        np.testing.assert_allclose(dphi[:, :, g], fd, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_projection_reproduces_polynomials(which):
    pr = problems.small2d(p=3) if which == "2d" else problems.small3d(p=3)
    d = discretise(pr.mesh, pr.p, pr.eta0)
    x = d.qx
    f = 0.3 + x[:, 0] ** 2 * x[:, 1] - 2 * x[:, 1] ** 3 + x[:, 0] * x[:, -1]
    U = project_elementwise(d, f)
    np.testing.assert_allclose(evaluate(d, U.ravel(), x, d.qe), f, rtol=0, atol=1e-12)


@pytest.fixture(scope="module", params=["2d", "3d"])
def disc_and_problem(request):
    pr = problems.small2d(p=2) if request.param == "2d" else problems.small3d(p=2)
    return pr, discretise(pr.mesh, pr.p, pr.eta0)


def test_A_symmetric_and_kills_constants(disc_and_problem):
    pr, d = disc_and_problem
    A = d.A
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    one = project_elementwise(d, np.ones(len(d.qw))).ravel()
    assert np.abs(A @ one).max() <= 1e-12 * abs(A).max()


def test_K_spd_bruteforce(disc_and_problem):
    pr, d = disc_and_problem
    K = d.system_matrix(pr.chi_m, pr.c_m, pr.dt).toarray()
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev[0] > 0
    np.linalg.cholesky(K)


def _boundary_load(mesh, d, flux):
    """int_{dOmega} flux(x, n) phi_i over boundary facets."""
    bf = np.nonzero(mesh.facet_elem[:, 1] < 0)[0]
    x, w, f = facet_rule(mesh, d.p + 2, bf)
    el = mesh.facet_elem[f, 0]
    phi = d.basis_at(x, el)
    vals = flux(x, mesh.facet_normal[f])
    load = np.zeros((mesh.n_elem, d.nd))
    np.add.at(load, el, (w * vals)[:, None] * phi)
    return load.ravel()


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_consistency_for_global_linear_functions(which):
    """For u linear and Sigma constant, A U = int_{dOmega} (Sigma grad u . n) phi."""
    pr = problems.small2d(p=2) if which == "2d" else problems.small3d(p=2)
    mesh = pr.mesh
    S = np.array([[2.0, 0.3], [0.3, 1.0]]) if which == "2d" else np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 1.5]])
    mesh.sigma = np.broadcast_to(S, (mesh.n_elem,) + S.shape).copy()
    d = discretise(mesh, pr.p, 10.0)
    gvec = np.arange(1, mesh.dim + 1, dtype=float) * 0.7
    U = project_elementwise(d, 0.4 + d.qx @ gvec).ravel()
    load = _boundary_load(mesh, d, lambda x, n: n @ (S @ gvec))
    np.testing.assert_allclose(d.A @ U, load, rtol=0, atol=1e-11 * np.abs(load).max())


def test_polynomial_reproduction_steady_problem():
    """(cM + A) U = F with u in P^p(Omega) and its exact load (volume source plus
    boundary flux) gives U = u exactly (the DG solution is exact for u in V_h)."""
    pr = problems.small2d(p=3)
    mesh = pr.mesh
    d = discretise(mesh, 3, 10.0)
    c = 2.5
    u = lambda x: x[:, 0] ** 2 * (3 - 2 * x[:, 0]) + x[:, 1] ** 2 * (1 - x[:, 1]) + 0.5 * x[:, 0] * x[:, 1]
    lap = lambda x: (6 - 12 * x[:, 0]) + (2 - 6 * x[:, 1])
    grad = lambda x: np.stack([6 * x[:, 0] - 6 * x[:, 0] ** 2 + 0.5 * x[:, 1],
                               2 * x[:, 1] - 3 * x[:, 1] ** 2 + 0.5 * x[:, 0]], 1)
    src = c * u(d.qx) - lap(d.qx)
    phi = d.basis_at(d.qx, d.qe)
    F = np.zeros((mesh.n_elem, d.nd))
    np.add.at(F, d.qe, (d.qw * src)[:, None] * phi)
    F = F.ravel() + _boundary_load(mesh, d, lambda x, n: (grad(x) * n).sum(1))
    Kss = (c * d.mass_matrix() + d.A).toarray()
    U = np.linalg.solve(Kss, F)
    np.testing.assert_allclose(evaluate(d, U, d.qx, d.qe), u(d.qx), rtol=0, atol=1e-10)


def _mms_error(n, p, seed=3):
    mesh = voronoi_mesh(n, seed=seed, lloyd=10)
    mesh.sigma = isotropic_sigma(mesh.n_elem, 2, 1.0)
    d = discretise(mesh, p, 10.0)
    c = 1.0
    u = lambda x: np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    src = (c + 2 * np.pi ** 2) * u(d.qx)
    phi = d.basis_at(d.qx, d.qe)
    F = np.zeros((mesh.n_elem, d.nd))
    np.add.at(F, d.qe, (d.qw * src)[:, None] * phi)
    Kss = (c * d.mass_matrix() + d.A).tocsc()
    import scipy.sparse.linalg as spla
    U = spla.spsolve(Kss, F.ravel())
    err = evaluate(d, U, d.qx, d.qe) - u(d.qx)
    return np.sqrt(np.sum(d.qw * err ** 2))


@pytest.mark.parametrize("p", [1, 2])
def test_mms_convergence_rate(p):
    """L2 error of the SIPG solution of c u - div grad u = f decays like h^(p+1)."""
    ns = [64, 256, 1024]
    errs = [_mms_error(n, p) for n in ns]
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(np.sqrt(ns[i + 1] / ns[i])) for i in range(2)]
    assert abs(rates[-1] - (p + 1)) < 0.35, (errs, rates)


@pytest.mark.parametrize("p,grids", [(1, (16, 24)), (2, (8, 16))])
def test_mms_convergence_rate_3d(p, grids):
    """Same manufactured solution on agglomerated polyhedra (about 8 cubes per
    element); the observed rate between two grids approaches p + 1."""
    import scipy.sparse.linalg as spla
    errs = []
    for n in grids:
        mesh = agglomerated_cube_mesh(n, 1.0, seed=5, target=8)
        mesh.sigma = isotropic_sigma(mesh.n_elem, 3, 1.0)
        d = discretise(mesh, p, 10.0)
        u = lambda x: np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]) * np.cos(np.pi * x[:, 2])
        src = (1.0 + 3 * np.pi ** 2) * u(d.qx)
        phi = d.basis_at(d.qx, d.qe)
        F = np.zeros((mesh.n_elem, d.nd))
        np.add.at(F, d.qe, (d.qw * src)[:, None] * phi)
        U = spla.spsolve((d.mass_matrix() + d.A).tocsc(), F.ravel())
        err = evaluate(d, U, d.qx, d.qe) - u(d.qx)
        errs.append(np.sqrt(np.sum(d.qw * err ** 2)))
    rate = np.log(errs[0] / errs[1]) / np.log(grids[1] / grids[0])
    assert abs(rate - (p + 1)) < 0.5, (errs, rate)
