"""Closed-form pin of the SIPG penalty of eq. (2) and of the element diameter
h_K (Section 3), for the oracle and for the host assembly of the library.

For u = the indicator function of element a (piecewise constant, so every
gradient term of eq. (3) vanishes) the SIPG form reduces to its penalty term:

    u_a^T A u_a = sum over interior facets F of a of  eta_F |F|,
    u_a^T A u_b = - sum over facets F shared by a and b of  eta_F |F|,

with eta_F = eta0 * (lmax(Sigma^-) + lmax(Sigma^+)) / 2 * p^2 * (h^- + h^+) / (2 h^- h^+)
(arithmetic average of Sigma_K, harmonic average of h_K).  The meshes are
hand-built so that each of these plausible mistakes changes the result:
the arithmetic mean of h instead of the harmonic one, the trace or the
smallest eigenvalue of Sigma instead of the largest, p instead of p^2, and the
bounding-box diagonal instead of the diameter (the cross-shaped and obtuse
elements have a diameter shorter than their box diagonal).  Every expected
value below is computed by hand from the geometry, not by the code under test.
"""
import numpy as np
import pytest

from oracle.assemble import discretise, project_piecewise_constant
from oracle.quadrature import element_diameter
from pdg_inputs.meshdata import Mesh

ETA0 = 10.0
S2 = np.sqrt(2.0)


def _mesh3d():
    """A: plus-shaped union of three unit-height boxes; B and C: boxes glued to
    A's +x arm and to A's +y arm.  Only the two A-B and A-C facets are interior."""
    boxes = [
        ([1, 0, 0], [2, 3, 1]), ([0, 1, 0], [1, 2, 1]), ([2, 1, 0], [3, 2, 1]),  # A
        ([3, 1, 0], [5, 2, 1]),                                                   # B
        ([1, 3, 0], [2, 4, 1]),                                                   # C
    ]
    cell_geom = np.array([[lo, hi] for lo, hi in boxes], dtype=np.float64)
    facet_geom = np.array([[[3, 1, 0], [3, 2, 1]],      # A | B, area 1
                           [[1, 3, 0], [2, 3, 1]]],     # A | C, area 1
                          dtype=np.float64)
    sigma = np.array([
        [[3, 1, 0], [1, 3, 0], [0, 0, 1]],   # eigenvalues 4, 2, 1 (trace 7)
        [[2, 0, 0], [0, 5, 0], [0, 0, 1]],   # eigenvalues 5, 2, 1 (trace 8)
        [[3, 0, 0], [0, 3, 0], [0, 0, 3]],   # isotropic 3
    ], dtype=np.float64)
    return Mesh(dim=3, cell_ptr=np.array([0, 3, 4, 5], np.int64), cell_geom=cell_geom,
                facet_elem=np.array([[0, 1], [0, 2]], np.int64), facet_geom=facet_geom,
                facet_normal=np.array([[1, 0, 0], [0, 1, 0]], np.float64), sigma=sigma)


def _mesh2d():
    """A: the obtuse triangle (0,0), (2,0), (1,1) (diameter 2, box diagonal
    sqrt 5); B: (0,0), (1,1), (0,1) across the edge y = x; C: (2,0), (2,1),
    (1,1) across the edge x + y = 2."""
    cell_geom = np.array([[[0, 0], [2, 0], [1, 1]],
                          [[0, 0], [1, 1], [0, 1]],
                          [[2, 0], [2, 1], [1, 1]]], dtype=np.float64)
    facet_geom = np.array([[[0, 0], [1, 1]], [[2, 0], [1, 1]]], dtype=np.float64)
    sigma = np.array([[[3, 1], [1, 3]],      # eigenvalues 4, 2
                      [[1, 0], [0, 5]],      # eigenvalues 5, 1
                      [[2, 0], [0, 2]]],     # isotropic 2
                     dtype=np.float64)
    return Mesh(dim=2, cell_ptr=np.array([0, 1, 2, 3], np.int64), cell_geom=cell_geom,
                facet_elem=np.array([[0, 1], [0, 2]], np.int64), facet_geom=facet_geom,
                facet_normal=np.array([[-1, 1], [1, 1]], np.float64) / S2, sigma=sigma)


# Hand-computed data per mesh: diameters, largest eigenvalues, interior
# facets (minus, plus, measure).
HAND = {
    3: dict(mesh=_mesh3d,
            # A: (0,1,0)-(3,2,1) -> sqrt(9+1+1); box diagonal would be sqrt(19)
            h=[np.sqrt(11.0), np.sqrt(6.0), np.sqrt(3.0)],
            lmax=[4.0, 5.0, 3.0],
            facets=[(0, 1, 1.0), (0, 2, 1.0)]),
    2: dict(mesh=_mesh2d,
            # A: longest edge 2; box [0,2]x[0,1] diagonal would be sqrt(5)
            h=[2.0, S2, S2],
            lmax=[4.0, 5.0, 2.0],
            facets=[(0, 1, S2), (0, 2, S2)]),
}


def _eta(hd, a, b, p):
    ha, hb = hd["h"][a], hd["h"][b]
    return ETA0 * 0.5 * (hd["lmax"][a] + hd["lmax"][b]) * p * p * (ha + hb) / (2.0 * ha * hb)


def _expected_gram(hd, p):
    """G[a, b] = u_a^T A u_b for the indicator functions, by hand."""
    G = np.zeros((3, 3))
    for a, b, meas in hd["facets"]:
        w = _eta(hd, a, b, p) * meas
        G[a, a] += w
        G[b, b] += w
        G[a, b] -= w
        G[b, a] -= w
    return G


def _indicators(mesh, nd):
    """Coefficient vectors of the indicator functions: the basis is orthonormal
    on each element's bounding box, so its constant member is 1 / sqrt(|box|)
    and the constant 1 has coefficient sqrt(|box|) on it."""
    n = mesh.n_elem
    out = np.zeros((n, n * nd))
    for a in range(n):
        v = mesh.cell_geom[mesh.cell_ptr[a]:mesh.cell_ptr[a + 1]].reshape(-1, mesh.dim)
        out[a, a * nd] = np.sqrt(np.prod(v.max(axis=0) - v.min(axis=0)))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_diameter_is_the_largest_vertex_distance(dim):
    hd = HAND[dim]
    np.testing.assert_allclose(element_diameter(hd["mesh"]()), hd["h"], rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [2, 3])
def test_oracle_penalty_on_indicator_functions(dim, p):
    hd = HAND[dim]
    mesh = hd["mesh"]()
    disc = discretise(mesh, p, ETA0)
    U = _indicators(mesh, disc.nd)
    # the indicators are what the oracle's own projection gives
    for a in range(mesh.n_elem):
        v = np.zeros(mesh.n_elem)
        v[a] = 1.0
        np.testing.assert_allclose(project_piecewise_constant(disc, v).ravel(), U[a], atol=1e-13)
    G = U @ (disc.A @ U.T)
    np.testing.assert_allclose(G, _expected_gram(hd, p), rtol=1e-12, atol=1e-9)


def test_the_pin_separates_the_plausible_mistakes():
    """Each mutation of eq. (2) moves at least one Gram entry by far more than
    the 1e-12 tolerance used above (checked on the hand formulas)."""
    for dim, hd in HAND.items():
        p = 2
        base = _expected_gram(hd, p)
        ha, hb = hd["h"][0], hd["h"][1]
        mutations = {
            "arithmetic mean of h": 0.5 * (ha + hb) / (2.0 * ha * hb / (ha + hb)),
            "p instead of p^2": 1.0 / p,
        }
        for name, factor in mutations.items():
            assert abs(factor - 1.0) > 1e-3, (dim, name)
        # trace / smallest eigenvalue instead of the largest, box diagonal for h_K
        trace = {3: [7.0, 8.0, 9.0], 2: [6.0, 6.0, 4.0]}[dim]
        lmin = {3: [1.0, 1.0, 3.0], 2: [2.0, 1.0, 2.0]}[dim]
        boxdiag = {3: [np.sqrt(19.0), np.sqrt(6.0), np.sqrt(3.0)], 2: [np.sqrt(5.0), S2, S2]}[dim]
        for name, key, val in [("trace", "lmax", trace), ("lambda_min", "lmax", lmin), ("box diagonal", "h", boxdiag)]:
            alt = dict(hd)
            alt[key] = val
            assert np.abs(_expected_gram(alt, p) - base).max() > 1e-3 * np.abs(base).max(), (dim, name)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [2, 3])
def test_library_penalty_on_indicator_functions(dim, p):
    """The same closed form for the host assembly of the library:
    A = 2 (K - c M) with the library's K = c M + A / 2."""
    from paper_2512_19536_amd import solver
    hd = HAND[dim]
    mesh = hd["mesh"]()
    ctx = solver.Context(None)
    ctx.set_mesh(mesh, p)
    chi, cm, dt = 1.0, 1.0, 0.5
    ctx.assemble(chi, cm, dt, ETA0)
    row_ptr, col, val, mass = ctx.get_matrix()
    n, nd = mesh.n_elem, val.shape[1]
    K = np.zeros((n * nd, n * nd))
    for e in range(n):
        for k in range(row_ptr[e], row_ptr[e + 1]):
            K[e * nd:(e + 1) * nd, col[k] * nd:(col[k] + 1) * nd] = val[k]
    Mm = np.zeros_like(K)
    for e in range(n):
        Mm[e * nd:(e + 1) * nd, e * nd:(e + 1) * nd] = mass[e]
    A = 2.0 * (K - (chi * cm / dt) * Mm)
    U = _indicators(mesh, nd)
    G = U @ A @ U.T
    np.testing.assert_allclose(G, _expected_gram(hd, p), rtol=1e-12, atol=1e-9)
