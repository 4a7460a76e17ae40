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
``cfg4``  a batch of 64 independent 3-D problems: target sizes N log-uniform
          in [2k, 60k] dofs and degrees p uniform in {1..4} (seed 7); each a
          cube of n^3 cubes of 0.25 mm agglomerated to ~8 cubes per element with
          n = round((8 N / nd)^(1/3)), the physics of cfg2 (two regions,
          dt = 2.5 us, planar stimulus), clamp(round(N / 250), 8, 256)
          subdomains of equal target size (so about 250 dofs each) with the P1
          coarse space on them, FP32 Schwarz solves.  Systems of one degree are
          concatenated into one problem (``elem_ptr`` gives the systems).
``cfg5``  trajectories for the learned initial guess on the cfg2 mesh, partition
          and time step: trajectory s has a +30 mV stimulus in the ball of
          radius 1.5 mm around a seeded random centre and, in the white region,
          conductivity 3 sigma0 along a seeded random fibre field and sigma0
          across it (grey: sigma0, isotropic); FP32 Schwarz solves.  Training
          seeds 100..119, held-out seeds 200..204, 100 steps each.
``small3d`` a tiny 3-D problem (6^3 cubes) for quick tests.
``table1_problem(N_h, p, k)`` one cell of the paper's Table 1 (2-D grey/white
          square, one subdomain per element, coarse degree q = p on
          agglomerates of about k^2 elements, i.e. H = k h).
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field, replace

import numpy as np

from . import params
from .mesh2d import voronoi_mesh
from .mesh3d import agglomerated_cube_mesh, cube_mesh_from_owner, renumber_elements
from .meshdata import Mesh, concat_meshes
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
    elem_ptr: np.ndarray | None = None   # batch of independent systems: element range of each
    # potential in the explicit ion term of eq. (4): "endpoint" = 2u^k - u^(k-1)
    # (extrapolated to t^(k+1), as the equation writes it) or "midpoint" =
    # (3u^k - u^(k-1))/2; the workloads at dt = 0.05 ms take "midpoint", where
    # the extrapolation to t^(k+1) diverges
    ion_extrap: str = "endpoint"

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
                   n_steps=10, tol=1e-10, u0_elem=u0, y0_elem=_rest_state(n), ion_extrap="midpoint")


def _cube_problem(name, n_grid, length, seed_mesh, seed_part, n_sub, p, spread,
                  sigma_kind, n_steps, seed_fibre=None, white_ratio=3.0, sigma0=1.0,
                  sigma_ratio=10.0, dt=0.05, target=8) -> Problem:
    nc = n_grid ** 3
    k = np.unravel_index(np.arange(nc), (n_grid,) * 3)[2]
    region_cube = (k < n_grid // 2).astype(np.int64) if sigma_kind == "two_region" else np.zeros(nc, np.int64)
    mesh = agglomerated_cube_mesh(n_grid, length, seed_mesh, target=target, region_of_cube=region_cube)
    return _problem_on_cube_mesh(name, mesh, seed_part, n_sub, p, spread, sigma_kind, n_steps,
                                 seed_fibre, white_ratio, sigma0, sigma_ratio, dt)


def _problem_on_cube_mesh(name, mesh, seed_part, n_sub, p, spread, sigma_kind, n_steps, seed_fibre,
                          white_ratio, sigma0, sigma_ratio, dt) -> Problem:
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
                   n_steps=n_steps, tol=1e-10, u0_elem=u0, y0_elem=_rest_state(n),
                   ion_extrap="endpoint" if dt <= DT_3D else "midpoint")


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


def slab3d(n_grid=4, p=4, n_sub=3, seed=21) -> Problem:
    """A 3-D test mesh with one element of many neighbours: the cubes of the
    grid's second x-layer form one plate element, every other cube is an
    element of its own, so the plate borders 2 n_grid^2 elements (33 blocks in
    its matrix row at n_grid = 4)."""
    nc = n_grid ** 3
    i = np.unravel_index(np.arange(nc), (n_grid,) * 3)[0]
    plate = i == 1
    owner = np.empty(nc, dtype=np.int64)
    owner[plate] = 0
    owner[~plate] = 1 + np.arange(int((~plate).sum()))
    k = np.unravel_index(np.arange(nc), (n_grid,) * 3)[2]
    region_cube = np.where(plate, 0, (k >= n_grid // 2).astype(np.int64))
    mesh = cube_mesh_from_owner(owner, n_grid, 1.0, region_of_cube=region_cube)
    return _problem_on_cube_mesh(f"slab3d_{n_grid}_p{p}", mesh, seed, n_sub, p, 0.3, "two_region", 3,
                                 None, 3.0, 1.0, 10.0, 0.05)


def one_element3d(p=2) -> Problem:
    """The degenerate 3-D case: a single element (2 x 2 x 2 cubes), one
    subdomain and a coarse space on it; every facet is a boundary facet."""
    mesh = cube_mesh_from_owner(np.zeros(8, dtype=np.int64), 2, 1.0, region_of_cube=np.zeros(8, dtype=np.int64))
    return _problem_on_cube_mesh(f"one_element3d_p{p}", mesh, 1, 1, p, 0.0, "two_region", 3,
                                 None, 3.0, 1.0, 10.0, 0.05)


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
                   n_steps=3, tol=1e-10, u0_elem=u0, y0_elem=_rest_state(ne), ion_extrap="midpoint")


def trajectory_problem(base: Problem, seed, radius=None, white_ratio=3.0, prec="f32") -> Problem:
    """A variant of `base` (same mesh, partition and constants) with a seeded
    ball stimulus and a seeded fibre field in the white region (region 1)."""
    rng = np.random.default_rng(seed)
    mesh = base.mesh
    cen = mesh.element_centroid()
    lo, hi = cen.min(0), cen.max(0)
    if radius is None:
        radius = 0.15 * float(np.max(hi - lo))
    sigma0 = float(base.mesh.sigma[:, 0, 0].min())
    fib = fibre_field(cen, seed)
    sig = isotropic_sigma(mesh.n_elem, mesh.dim, sigma0)
    white = np.asarray(mesh.region) == 1
    sig[white] = fibre_sigma(fib[white], white_ratio * sigma0, sigma0)
    centre = lo + rng.random(mesh.dim) * (hi - lo)
    dist = np.linalg.norm(cen - centre, axis=1)
    inside = dist < radius
    if not inside.any():
        inside[np.argmin(dist)] = True
    u0 = np.full(mesh.n_elem, params.U_REST)
    u0[inside] += 30.0
    m2 = replace(mesh, sigma=sig, extra=dict(mesh.extra, fibre=fib))
    return replace(base, name=f"{base.name}_traj{seed}", mesh=m2, u0_elem=u0,
                   y0_elem=_rest_state(mesh.n_elem), local_prec=prec, coarse_prec=prec)


def learned_small(n_grid=12, p=2, n_sub=8, seed=31) -> Problem:
    """A small cube (n_grid^3 cubes of 0.25 mm) with the 3-D physics of cfg2,
    the base of quick trajectory sets for the learned form."""
    return _cube_problem(f"learned_small_{n_grid}", n_grid, 0.25 * n_grid, seed_mesh=seed, seed_part=seed + 1,
                         n_sub=n_sub, p=p, spread=0.3, sigma_kind="two_region", n_steps=40,
                         sigma0=SIGMA_3D, dt=DT_3D)


# Table 1 of the paper (Section 5): 2-D square, grey matter on top (sigma = 0.63,
# isotropic), white matter below (sigma_l = 0.69, sigma_n = 2.571 with the
# anisotropy along the vertical), initial potential -50 mV in the disk
# (x - 0.5)^2 + (y - 1)^2 < 0.016 and -67 mV elsewhere, dt = 2.5 us, one
# element per subdomain, coarse space of degree q = p on agglomerates with
# H = 2h .. 16h, stopping tolerance 1e-9.  chi_m C_m is not given; TABLE1_CHI_CM
# is the value for which the condition number of the unpreconditioned system
# at p = 1, N_h = 512 equals the paper's 1.34e4 (dense eigenvalues of that
# matrix), used for every cell.
TABLE1_CHI_CM = 0.014319
TABLE1_NH = (512, 1024, 2048, 4096)
TABLE1_H = (2, 4, 8, 16)


@functools.lru_cache(maxsize=8)
def _table1_mesh(n_h, seed):
    return voronoi_mesh(n_h, seed=seed, lloyd=10)


def table1_problem(n_h, p, h_ratio, chi_cm=None, seed=None, n_steps=10) -> Problem:
    """One cell of Table 1: N_h Voronoi cells, degree p, coarse agglomerates of
    about h_ratio^2 cells (H = h_ratio h), one subdomain per element."""
    mesh = replace(_table1_mesh(n_h, 1000 + n_h if seed is None else seed))
    n = mesh.n_elem
    cen = mesh.element_centroid()
    region = (cen[:, 1] < 0.5).astype(np.int32)  # 1 = white matter (bottom)
    mesh.region = region
    sig = isotropic_sigma(n, 2, 0.63)
    sig[region == 1] = np.diag([0.69, 2.571])
    mesh.sigma = sig
    u0 = np.full(n, -67.0)
    u0[(cen[:, 0] - 0.5) ** 2 + (cen[:, 1] - 1.0) ** 2 < 0.016] = -50.0
    n_coarse = max(1, int(round(n_h / h_ratio ** 2)))
    coarse = rcb(cen, n_coarse, region=region, spread=0.0, seed=n_h + h_ratio)
    # number the elements agglomerate by agglomerate (the numbering is free)
    perm = order_by_part(coarse, cen)
    mesh = renumber_elements(mesh, perm)
    coarse, u0 = coarse[perm], u0[perm]
    chi = TABLE1_CHI_CM if chi_cm is None else chi_cm
    return Problem(f"table1_N{n_h}_p{p}_H{h_ratio}h", mesh, p=p, chi_m=chi, c_m=1.0, dt=0.0025, eta0=10.0,
                   elem_sub=np.arange(n, dtype=np.int32), elem_coarse=coarse.astype(np.int32), coarse_q=p,
                   n_steps=n_steps, tol=1e-9, u0_elem=u0, y0_elem=_rest_state(n))


CFG5_TRAIN_SEEDS = tuple(range(100, 120))
CFG5_TEST_SEEDS = tuple(range(200, 205))


def cfg5(n_steps=100):
    """(training problems, held-out problems) of the learned form on the cfg2 mesh."""
    base = cfg2()
    base.n_steps = n_steps
    return ([trajectory_problem(base, s) for s in CFG5_TRAIN_SEEDS],
            [trajectory_problem(base, s) for s in CFG5_TEST_SEEDS])


def concat_problems(name, probs) -> Problem:
    """One problem holding independent systems of one degree side by side
    (meshes, labels and initial data concatenated; ``elem_ptr`` set)."""
    p0 = probs[0]
    for q in probs:
        assert (q.p, q.dt, q.chi_m, q.c_m, q.eta0, q.coarse_q, q.tol, q.local_prec, q.coarse_prec, q.ion_extrap) == \
            (p0.p, p0.dt, p0.chi_m, p0.c_m, p0.eta0, p0.coarse_q, p0.tol, p0.local_prec, p0.coarse_prec, p0.ion_extrap)
        assert np.array_equal(q.ionic, p0.ionic)
    mesh, elem_ptr = concat_meshes([q.mesh for q in probs])
    sub_off = np.cumsum([0] + [int(q.elem_sub.max()) + 1 for q in probs])
    crs_off = np.cumsum([0] + [int(q.elem_coarse.max()) + 1 for q in probs])
    sub = np.concatenate([q.elem_sub + o for q, o in zip(probs, sub_off)]).astype(np.int32)
    crs = np.concatenate([q.elem_coarse + o for q, o in zip(probs, crs_off)]).astype(np.int32)
    return Problem(name, mesh, p=p0.p, chi_m=p0.chi_m, c_m=p0.c_m, dt=p0.dt, eta0=p0.eta0,
                   elem_sub=sub, elem_coarse=crs, coarse_q=p0.coarse_q, n_steps=p0.n_steps, tol=p0.tol,
                   u0_elem=np.concatenate([q.u0_elem for q in probs]),
                   y0_elem=np.ascontiguousarray(np.concatenate([q.y0_elem for q in probs], axis=1)),
                   ionic=p0.ionic.copy(), local_prec=p0.local_prec, coarse_prec=p0.coarse_prec,
                   maxit=p0.maxit, elem_ptr=elem_ptr, ion_extrap=p0.ion_extrap)


@dataclass
class Batch:
    """Independent systems and their grouping by degree (one concatenated
    problem per degree, systems in generation order inside a group)."""
    name: str
    systems: list
    groups: dict      # p -> (concatenated Problem, [system indices])

    @property
    def n_dof(self):
        return sum(q.n_dof for q in self.systems)


def nd3(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def cfg4_sizes(n_sys=64, seed=7):
    """Target dofs and degree of every system of the batch workload."""
    rng = np.random.default_rng(seed)
    N = np.exp(rng.uniform(np.log(2000.0), np.log(60000.0), n_sys))
    ps = rng.integers(1, 5, n_sys)
    return N, ps


def batch_system(i, N, p, n_steps=10, prec="f32") -> Problem:
    nd = nd3(p)
    n_grid = max(4, int(round((8.0 * N / nd) ** (1.0 / 3.0))))
    n_sub = int(np.clip(round(N / 250.0), 8, 256))
    pr = _cube_problem(f"cfg4_s{i}", n_grid, 0.25 * n_grid, seed_mesh=700 + i, seed_part=800 + i,
                       n_sub=n_sub, p=p, spread=0.0, sigma_kind="two_region", n_steps=n_steps,
                       sigma0=SIGMA_3D, dt=DT_3D)
    pr.local_prec = pr.coarse_prec = prec
    return pr


def make_batch(name, systems) -> Batch:
    groups = {}
    for p in sorted({q.p for q in systems}):
        idx = [i for i, q in enumerate(systems) if q.p == p]
        groups[p] = (concat_problems(f"{name}_p{p}", [systems[i] for i in idx]), idx)
    return Batch(name, systems, groups)


def cfg4(n_sys=64, seed=7) -> Batch:
    N, ps = cfg4_sizes(n_sys, seed)
    return make_batch("cfg4", [batch_system(i, N[i], int(ps[i])) for i in range(n_sys)])


BUILDERS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4}
