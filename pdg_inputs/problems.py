"""Seeded synthetic workloads (data only): meshes, tissue, partitions, initial data.

Every workload is a :class:`Problem`: a mesh with per-element conductivity
tensors, the polynomial degree, the time-step constants, a subdomain label and
a coarse-element label per element, and piecewise-constant (per element)
initial values of the potential and of the five ionic states.  Both the oracle
and the HIP library turn the per-element initial values into coefficient
vectors themselves.

Workloads
---------
``cfg1``  2-D unit square, 64 Lloyd-relaxed Voronoi polygons (seed 1), p = 2,
          isotropic sigma = 1, dt = 0.05 ms, eta0 = 10, 4 quadrant subdomains,
          P1 coarse space on the subdomains, 10 steps; u = -70 mV with +30 mV in
          the elements whose centroid lies in the corner disk |x| < 0.1.
``cfg2``  3-D cube [0, 10 mm]^3, 40^3 cubes agglomerated to ~8 cubes per element
          (seed 2), p = 2; dt = 2.5 us (the paper's time step); grey
          conductivity 20, white region z < 5 mm with 3x the grey conductivity;
          64 subdomains with sizes spread +/-40 % (seed 3) that do not cross the
          region interface; P1 coarse space on the subdomains; planar stimulus
          (+30 mV) in the elements touching the x = 0 face; 20 steps.
``cfg3``  64^3 cubes (seed 4), p = 3, dt = 2.5 us, fibre-aligned conductivity
          10:1 along a smooth seeded random fibre field (seed 5), 512
          subdomains (seed 6), FP32 Schwarz solves.
``small3d`` a tiny 3-D problem (6^3 cubes) for quick tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import params
from .mesh2d import voronoi_mesh
from .mesh3d import agglomerated_cube_mesh, renumber_elements
from .meshdata import Mesh
from .partition import order_by_part, quadrants, rcb


@dataclass
class Problem:
    name: str
    mesh: Mesh
    p: int
    chi_m: float
    c_m: float
    dt: float
    eta0: float
    elem_sub: np.ndarray
    elem_coarse: np.ndarray
    coarse_q: int
    n_steps: int
    tol: float
    u0_elem: np.ndarray                  # [n_elem]
    y0_elem: np.ndarray                  # [5, n_elem]
    ionic: np.ndarray = field(default_factory=lambda: params.IONIC_DEFAULT.copy())
    local_prec: str = "f64"
    coarse_prec: str = "f64"
    maxit: int = 5000

    @property
    def n_elem(self):
        return self.mesh.n_elem

    @property
    def nd(self):
        d, p = self.mesh.dim, self.p
        return (p + 1) * (p + 2) // 2 if d == 2 else (p + 1) * (p + 2) * (p + 3) // 6

    @property
    def n_dof(self):
        return self.n_elem * self.nd

    @property
    def n_sub(self):
        return int(self.elem_sub.max()) + 1


def _rest_state(n_elem):
    y = np.repeat(params.Y_REST[:, None], n_elem, axis=1)
    return np.ascontiguousarray(y)


def isotropic_sigma(n_elem, dim, values):
    s = np.zeros((n_elem, dim, dim))
    for d in range(dim):
        s[:, d, d] = values
    return s


def fibre_field(points, seed, n_modes=8):
    """Smooth unit vector field: normalised sum of seeded low-frequency Fourier
    modes evaluated at ``points`` (rows), scaled to the unit cube."""
    rng = np.random.default_rng(seed)
    pts = np.asarray(points)
    span = pts.max(0) - pts.min(0)
    x = (pts - pts.min(0)) / np.where(span > 0, span, 1.0)
    v = np.zeros_like(x)
    base = rng.normal(size=x.shape[1])
    v += base
    for _ in range(n_modes):
        k = rng.integers(1, 3, size=x.shape[1]) * np.pi
        ph = rng.random() * 2 * np.pi
        amp = rng.normal(size=x.shape[1])
        v += np.cos(x @ k + ph)[:, None] * amp[None, :]
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def fibre_sigma(directions, sigma_l, sigma_n):
    """Sigma = sigma_n I + (sigma_l - sigma_n) l (x) l for fibre direction l."""
    d = directions.shape[1]
    return sigma_n * np.eye(d)[None] + (sigma_l - sigma_n) * np.einsum("ei,ej->eij", directions, directions)


def cfg1() -> Problem:
    mesh = voronoi_mesh(64, seed=1, lloyd=10)
    n = mesh.n_elem
    mesh.sigma = isotropic_sigma(n, 2, 1.0)
    mesh.region = np.zeros(n, dtype=np.int32)
    cen = mesh.element_centroid()
    sub = quadrants(cen)
    u0 = np.full(n, params.U_REST)
    u0[np.linalg.norm(cen, axis=1) < 0.1] += 30.0
    return Problem("cfg1", mesh, p=2, chi_m=1.0, c_m=1.0, dt=0.05, eta0=10.0,
                   elem_sub=sub.astype(np.int32), elem_coarse=sub.astype(np.int32), coarse_q=1,
                   n_steps=10, tol=1e-10, u0_elem=u0, y0_elem=_rest_state(n))


def _cube_problem(name, n_grid, length, seed_mesh, seed_part, n_sub, p, spread,
                  sigma_kind, n_steps, seed_fibre=None, white_ratio=3.0, sigma0=1.0,
                  sigma_ratio=10.0, dt=0.05, target=8) -> Problem:
    nc = n_grid ** 3
    k = np.unravel_index(np.arange(nc), (n_grid,) * 3)[2]
    region_cube = (k < n_grid // 2).astype(np.int64) if sigma_kind == "two_region" else np.zeros(nc, np.int64)
    mesh = agglomerated_cube_mesh(n_grid, length, seed_mesh, target=target, region_of_cube=region_cube)
    cen = mesh.element_centroid()
    part = rcb(cen, n_sub, region=mesh.region, spread=spread, seed=seed_part)
    perm = order_by_part(part, cen)
    mesh = renumber_elements(mesh, perm)
    part = part[perm]
    cen = cen[perm]
    n = mesh.n_elem
    if sigma_kind == "two_region":
        vals = np.where(mesh.region == 1, white_ratio * sigma0, sigma0)
        mesh.sigma = isotropic_sigma(n, 3, vals)
    else:
        fib = fibre_field(cen, seed_fibre)
        mesh.sigma = fibre_sigma(fib, sigma_ratio * sigma0, sigma0)
        mesh.extra["fibre"] = fib
    # planar stimulus: elements owning a cube of the first layer x < h
    h = mesh.extra["grid_h"]
    first = np.zeros(n, dtype=bool)
    lo_x = mesh.cell_geom[:, 0, 0]
    owner = mesh.cell_owner()
    first[owner[lo_x < 0.5 * h]] = True
    u0 = np.full(n, params.U_REST)
    u0[first] += 30.0
    return Problem(name, mesh, p=p, chi_m=1.0, c_m=1.0, dt=dt, eta0=10.0,
                   elem_sub=part.astype(np.int32), elem_coarse=part.astype(np.int32), coarse_q=1,
                   n_steps=n_steps, tol=1e-10, u0_elem=u0, y0_elem=_rest_state(n))


# 3-D workloads use the paper's time step (2.5 us).  With the explicit ion term
# a step of 0.05 ms is unstable once the stimulated elements fire; the
# conductivity scale 20 keeps the system matrix equal (up to a factor) to the
# one of dt = 0.05 ms with conductivity 1, so the solver sees the same
# stiffness-dominated operator.
DT_3D = 0.0025
SIGMA_3D = 20.0


def cfg2() -> Problem:
    return _cube_problem("cfg2", 40, 10.0, seed_mesh=2, seed_part=3, n_sub=64, p=2, spread=0.4,
                         sigma_kind="two_region", n_steps=20, sigma0=SIGMA_3D, dt=DT_3D)


def cfg3() -> Problem:
    pr = _cube_problem("cfg3", 64, 10.0, seed_mesh=4, seed_part=6, n_sub=512, p=3, spread=0.0,
                       sigma_kind="fibre", n_steps=50, seed_fibre=5, sigma0=SIGMA_3D, dt=DT_3D)
    pr.local_prec, pr.coarse_prec = "f32", "f32"
    return pr


def small3d(n_grid=6, p=2, n_sub=4, seed=11) -> Problem:
    return _cube_problem(f"small3d_{n_grid}_p{p}", n_grid, 1.0, seed_mesh=seed, seed_part=seed + 1,
                         n_sub=n_sub, p=p, spread=0.3, sigma_kind="two_region", n_steps=3)


def small2d(n=24, p=2, seed=5) -> Problem:
    mesh = voronoi_mesh(n, seed=seed, lloyd=4)
    ne = mesh.n_elem
    mesh.sigma = isotropic_sigma(ne, 2, 1.0)
    mesh.region = np.zeros(ne, dtype=np.int32)
    cen = mesh.element_centroid()
    sub = quadrants(cen)
    u0 = np.full(ne, params.U_REST)
    u0[np.linalg.norm(cen, axis=1) < 0.25] += 30.0
    return Problem(f"small2d_{n}_p{p}", mesh, p=p, chi_m=1.0, c_m=1.0, dt=0.05, eta0=10.0,
                   elem_sub=sub.astype(np.int32), elem_coarse=sub.astype(np.int32), coarse_q=1,
                   n_steps=3, tol=1e-10, u0_elem=u0, y0_elem=_rest_state(ne))


BUILDERS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3}
