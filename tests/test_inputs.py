"""Sanity of the seeded input generators (geometry only)."""
import numpy as np

from pdg_inputs import mesh2d, problems
from pdg_inputs.mesh3d import agglomerate_grid


def test_voronoi_partition_of_unity(cfg1_problem):
    m = cfg1_problem.mesh
    assert m.n_elem == 64
    np.testing.assert_allclose(m.element_measure().sum(), 1.0, rtol=0, atol=1e-13)
    assert np.all(m.element_measure() > 0)


def test_voronoi_facets_shared_by_two_cells():
    pts = np.random.default_rng(3).random((40, 2))
    cells = mesh2d.voronoi_cells(pts)
    for i, (poly, lab) in enumerate(cells):
        for k, j in enumerate(lab):
            if j < 0:
                continue
            a, b = poly[k], poly[(k + 1) % len(poly)]
            pj, lj = cells[j]
            # cell j has the same segment (reversed) labelled i
            ks = [kk for kk, l in enumerate(lj) if l == i]
            assert len(ks) == 1
            c, d = pj[ks[0]], pj[(ks[0] + 1) % len(pj)]
            assert np.allclose(a, d, atol=1e-12) and np.allclose(b, c, atol=1e-12)


def test_closed_elements_normals_sum_to_zero(cfg1_problem, small3d_problem):
    for m in (cfg1_problem.mesh, small3d_problem.mesh):
        acc = np.zeros((m.n_elem, m.dim))
        g = m.facet_geom
        if m.dim == 2:
            area = np.linalg.norm(g[:, 1] - g[:, 0], axis=1)
        else:
            ext = g[:, 1] - g[:, 0]
            area = np.prod(np.where(ext == 0, 1.0, ext), axis=1)
        fe = m.facet_elem
        np.add.at(acc, fe[:, 0], area[:, None] * m.facet_normal)
        inner = fe[:, 1] >= 0
        np.add.at(acc, fe[inner, 1], -area[inner, None] * m.facet_normal[inner])
        assert np.abs(acc).max() < 1e-12


def test_agglomerates_connected_and_region_pure():
    n = 8
    k = np.unravel_index(np.arange(n ** 3), (n,) * 3)[2]
    region = (k < n // 2).astype(int)
    own = agglomerate_grid(n, seed=5, target=8, region=region)
    idx = np.arange(n ** 3).reshape(n, n, n)
    for e in np.unique(own):
        cubes = set(np.nonzero(own == e)[0].tolist())
        assert len({region[c] for c in cubes}) == 1
        # BFS connectivity through face neighbours
        start = next(iter(cubes))
        seen, todo = {start}, [start]
        while todo:
            c = todo.pop()
            i, j, kk = np.unravel_index(c, (n,) * 3)
            for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                a, b, cc = i + di, j + dj, kk + dk
                if 0 <= a < n and 0 <= b < n and 0 <= cc < n:
                    t = int(idx[a, b, cc])
                    if t in cubes and t not in seen:
                        seen.add(t)
                        todo.append(t)
        assert seen == cubes


def test_subdomains_uneven_and_aligned():
    pr = problems.small3d(n_grid=8, n_sub=8)
    sizes = np.bincount(pr.elem_sub)
    assert sizes.min() > 0 and len(sizes) == 8
    for s in range(8):
        assert len(np.unique(pr.mesh.region[pr.elem_sub == s])) == 1
