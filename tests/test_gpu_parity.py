"""GPU parity of the HIP path (through the C-ABI) against the FP64 oracle.

Bars: SpMV, Schwarz apply, ionic update and right-hand side agree with the
oracle to rounding (relative 1e-12 in the max norm); PCG solves and time steps
agree to relative L2 1e-8 on the solution with equal iteration counts.  A
difference of one iteration is accepted only when the oracle's deciding
residual lies within a factor 1.2 of the stopping threshold on the side that
makes the difference: late PCG residual norms move by 6-14 % under relative
perturbations of b of 1e-15..1e-11 in the oracle itself, so such a count is
decided by rounding.
"""
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.monodomain import Monodomain  # noqa: E402
from oracle.pcg import lanczos_kappa  # noqa: E402
from paper_2512_19536_amd import _lib, solver  # noqa: E402
from paper_2512_19536_amd._lib import PdgError  # noqa: E402
from pdg_inputs import problems  # noqa: E402
from parity_rules import iters_agree  # noqa: E402

DEV = "cuda:0"


def _gpu_ok():
    return torch.cuda.is_available()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not _gpu_ok():
        pytest.skip("no GPU")


CASES = {
    "cfg1": problems.cfg1,
    "2d_p1": lambda: problems.small2d(n=30, p=1),
    "2d_p3": lambda: problems.small2d(n=30, p=3),
    "2d_p4": lambda: problems.small2d(n=30, p=4),
    "3d_p1": lambda: problems.small3d(n_grid=8, p=1, n_sub=6),
    "3d_p2": lambda: problems.small3d(n_grid=8, p=2, n_sub=6),
    "3d_p3": lambda: problems.small3d(n_grid=8, p=3, n_sub=6),
    "3d_p4": lambda: problems.small3d(n_grid=6, p=4, n_sub=3),
    # coarse degree q = p (Section 4: V_0 = P^q on the agglomerates, q <= p)
    "3d_p2_q2": lambda: replace(problems.small3d(n_grid=8, p=2, n_sub=6), coarse_q=2),
    # the Table-1 mode: one subdomain per element (block Jacobi) plus a
    # q = p coarse space on agglomerates of ~4 elements (H = 2h); 375 coarse
    # dofs for p = 4 span six tiles
    "t1_p1": lambda: problems.table1_problem(64, 1, 2),
    "t1_p3": lambda: problems.table1_problem(80, 3, 2),
    "t1_p4": lambda: problems.table1_problem(100, 4, 2),
    # coarse variants: q < p, and a coarse mesh distinct from (and coarser
    # than) the subdomains
    "t1_p4_q2": lambda: replace(problems.table1_problem(100, 4, 2), coarse_q=2),
    "3d_p3_q2_own_coarse": lambda: _own_coarse(problems.small3d(n_grid=8, p=3, n_sub=6), 3, q=2),
    # a plate element with 32 neighbours: its matrix row spans three chunks
    # (16 + 16 + 1 blocks) of the layout for blocks of more than 32 rows
    "3d_p4_slab": lambda: problems.slab3d(n_grid=4, p=4, n_sub=3),
    # one element: one subdomain of 10 dofs (one tile, mostly padding) and a
    # 4-dof coarse system on it
    "3d_one_element": lambda: problems.one_element3d(p=2),
    # subdomains of exactly 64 dofs (one full tile, no padding) and of 128 dofs
    "3d_p1_tile64": lambda: _blocks_of(problems.small3d(n_grid=8, p=1, n_sub=4), (16, 32)),
    # both readings of the ion-term extrapolation at the paper's time step:
    # to t^(k+1) (eq. (4), the default there) and to the mid-point
    "3d_p2_endpoint": lambda: replace(problems.small3d(n_grid=8, p=2, n_sub=6), dt=0.0025, ion_extrap="endpoint"),
    "3d_p2_midpoint": lambda: replace(problems.small3d(n_grid=8, p=2, n_sub=6), dt=0.0025, ion_extrap="midpoint"),
    # p = 1 at the paper's time step on the 3-D physics (k_ionic<3,1>)
    "3d_p1_dt": lambda: problems.learned_small(n_grid=8, p=1, n_sub=6),
}


def _blocks_of(pr, sizes):
    """The problem with subdomains of consecutive elements, cycling through the
    given element counts (the last one takes the rest)."""
    n = pr.n_elem
    sub = np.zeros(n, dtype=np.int32)
    e, k = 0, 0
    while e < n:
        m = sizes[k % len(sizes)]
        sub[e:e + m] = k
        e += m
        k += 1
    return replace(pr, elem_sub=sub, elem_coarse=sub.copy())


def _own_coarse(pr, n_coarse, q):
    """The problem with coarse agglomerates of its own (RCB, not the subdomains)."""
    from pdg_inputs.partition import rcb
    ec = rcb(pr.mesh.element_centroid(), n_coarse, seed=77)
    assert len(np.unique(ec)) == n_coarse and not np.array_equal(ec, pr.elem_sub)
    return replace(pr, elem_coarse=ec.astype(np.int32), coarse_q=q)

_cache = {}


def _setup(case):
    if case not in _cache:
        print(f"[setup] {case}", flush=True)
        pr = CASES[case]()
        md = Monodomain(pr)
        ctx = solver.from_problem(pr, device=DEV, options={_lib.PDG_OPT_LANCZOS_CAP: 1 << 15})
        _cache[case] = (pr, md, ctx)
    return _cache[case]


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("case", sorted(CASES))
def test_spmv(case):
    pr, md, ctx = _setup(case)
    x = np.random.default_rng(1).standard_normal(pr.n_dof)
    y = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
    ctx.spmv(T(x), y)
    assert rel_max(N(y), md.K @ x) < 1e-13


@pytest.mark.parametrize("case", sorted(CASES))
def test_schwarz_apply(case):
    pr, md, ctx = _setup(case)
    r = np.random.default_rng(2).standard_normal(pr.n_dof)
    z = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
    ctx.precond_apply(T(r), z)
    assert rel_max(N(z), md.schwarz.apply(r)) < 1e-11


@pytest.mark.parametrize("period", [1, 3, 8])
def test_kernel_timing_samples_the_launches_that_did_work(period):
    """One Schwarz launch in `period` of a solve is timed: the init apply and
    iterations 1..iters did work (launches queued past convergence do not
    count), so ceil((iters + 1) / period) launches are reported."""
    pr, md, ctx = _setup("3d_p2")
    b = T(np.random.default_rng(5).standard_normal(pr.n_dof))
    x = torch.zeros_like(b)
    ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, period)
    ctx.kernel_timing()
    info = ctx.solve(b, x, 1e-10, 5000)
    n, ms, by = ctx.kernel_timing()
    ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, 0)
    assert info["iters"] > 2 * period
    assert n == (info["iters"] + period) // period
    assert ms > 0 and by > 0


@pytest.mark.parametrize("case", ["cfg1", "2d_p1", "2d_p4", "3d_p1", "3d_p1_dt", "3d_p2", "3d_p4",
                                  "3d_p2_endpoint", "3d_p2_midpoint", "t1_p1"])
def test_project_ionic_rhs(case):
    pr, md, ctx = _setup(case)
    U0, _, Y0 = md.initial_state()
    Ug, Upg, Yg = solver.initial_state(ctx, pr)
    # the oracle projects through M_K^{-1} by quadrature (rounding ~ cond(M_K) eps)
    assert rel_max(N(Ug), U0) < 1e-11 and rel_max(N(Yg), Y0.ravel()) < 1e-11
    rng = np.random.default_rng(3)
    U = U0 + 2.0 * rng.standard_normal(U0.shape)
    Up = U0 + 2.0 * rng.standard_normal(U0.shape)
    Yn, I = md.ionic_update(U, Up, Y0)
    Yd = T(Y0.ravel())
    Id = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
    ctx.ionic(T(U), T(Up), Yd, Id)
    assert rel_max(N(Id), I) < 1e-11
    # Y^(k+1) applies M_K^{-1}: both sides round at the level cond(M_K) * eps
    # (cond(M_K) reaches ~2e4 on p = 4 agglomerates)
    kappa = np.linalg.cond(md.disc.M).max()
    tol = max(1e-12, 100.0 * kappa * np.finfo(float).eps)
    for l in range(5):
        got = N(Yd).reshape(5, -1)[l]
        assert np.abs(got - Yn[l]).max() <= tol * max(np.abs(Yn[l]).max(), 1e-3), (l, kappa)
    b = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
    ctx.rhs(T(U), T(I), None, b)
    assert rel_max(N(b), md.rhs(U, I)) < 1e-12


@pytest.mark.parametrize("case", sorted(CASES))
def test_solve(case):
    pr, md, ctx = _setup(case)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(pr.n_dof)
    x0 = rng.standard_normal(pr.n_dof)
    xo, oinfo = md.solve(b, x0, tol=1e-10)
    x = T(x0)
    info = ctx.solve(T(b), x, 1e-10, 2000)
    print(case, "iters gpu", info["iters"], "oracle", oinfo.iters, flush=True)
    assert iters_agree(info["iters"], oinfo, 1e-10, np.linalg.norm(b))
    assert rel_l2(N(x), xo) < 1e-8
    assert info["relres"] <= 1e-10


@pytest.mark.parametrize("case", ["cfg1", "2d_p1", "3d_p1", "3d_p1_dt", "3d_p2", "3d_p3", "t1_p1", "t1_p3",
                                  "3d_p2_endpoint", "3d_p2_midpoint"])
def test_time_steps(case):
    pr, md, ctx = _setup(case)
    nsteps = pr.n_steps if case == "cfg1" else 3
    U, Up, Y = md.initial_state()
    Ug, Upg, Yg = solver.initial_state(ctx, pr)
    for k in range(nsteps):
        Yn_o, I_o = md.ionic_update(U, Up, Y)
        b_o = md.rhs(U, I_o)
        U, Up, Y, oinfo = md.step(U, Up, Y)
        info = ctx.step(Ug, Upg, Yg, None, pr.tol, pr.maxit)
        err = rel_l2(N(Ug), U)
        print(f"{case} step {k}: iters gpu {info['iters']} oracle {oinfo.iters} relL2 {err:.2e}", flush=True)
        assert iters_agree(info["iters"], oinfo, pr.tol, np.linalg.norm(b_o))
        assert err < 1e-8
        assert rel_l2(N(Upg), Up) < 1e-8
        assert rel_l2(N(Yg), Y.ravel()) < 1e-8


def test_determinism_bitwise():
    pr, md, ctx = _setup("3d_p2")
    b = T(np.random.default_rng(5).standard_normal(pr.n_dof))
    outs = []
    for _ in range(2):
        x = torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV)
        ctx.solve(b, x, 1e-10, 1000)
        outs.append(N(x))
    assert np.array_equal(outs[0], outs[1])


def test_zero_rhs_and_noconv():
    pr, md, ctx = _setup("2d_p1")
    x = T(np.ones(pr.n_dof))
    info = ctx.solve(torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV), x, 1e-10, 100)
    assert info["iters"] == 0 and float(N(x).max()) == 0.0 and float(N(x).min()) == 0.0
    b = T(np.random.default_rng(6).standard_normal(pr.n_dof))
    x = torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV)
    with pytest.raises(PdgError) as ei:
        ctx.solve(b, x, 1e-12, 2)
    assert ei.value.status == _lib.PDG_ENOCONV
    # the context still works after an error
    info = ctx.solve(b, x, 1e-10, 1000)
    assert info["relres"] <= 1e-10


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_reduced_precision_schwarz_still_meets_fp64_tolerance(prec):
    """Precision form: FP32 / BF16-stored local inverses with FP32 accumulation
    and an FP32 coarse solve; outer recurrences, dots and SpMV in FP64.  The
    solution still satisfies the FP64 relative residual 1e-10 and lies within
    1e-8 (relative L2) of the FP64 oracle; iterations are reported."""
    pr = problems.small3d(n_grid=8, p=2, n_sub=6)
    md = Monodomain(pr)
    ctx = solver.from_problem(pr, device=DEV, local_prec=prec, coarse_prec="f32")
    ctx.set_option(_lib.PDG_OPT_TRUE_RESIDUAL, 1)
    b = np.random.default_rng(7).standard_normal(pr.n_dof)
    xo, oinfo = md.solve(b, np.zeros(pr.n_dof), tol=1e-10)
    x = torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV)
    info = ctx.solve(T(b), x, 1e-10, 2000)
    print(prec, "iters", info["iters"], "fp64 oracle", oinfo.iters, "true relres", info["true_relres"], flush=True)
    assert info["true_relres"] < 2e-10
    assert rel_l2(N(x), xo) < 1e-8
    assert info["iters"] <= oinfo.iters + 5


@pytest.mark.parametrize("k", [0, 1, 2, 10])
def test_bf16_scaled_store_and_fp32_fallback(k):
    """BF16 local store: K_i^{-1} = D C D with C (unit diagonal) in BF16; a
    subdomain whose rounded C minus 2^-k I fails the Cholesky check is stored
    in FP32 instead.  k = 0 sends every subdomain to FP32 (the rounded C has a
    unit diagonal), which must reproduce the FP32 store bit for bit; every k
    meets the FP64 tolerance and the oracle's solution to 1e-8."""
    pr = problems.small3d(n_grid=8, p=2, n_sub=6)
    md = Monodomain(pr)
    opts = {_lib.PDG_OPT_TRUE_RESIDUAL: 1, _lib.PDG_OPT_BF16_MARGIN: k}
    ctx = solver.from_problem(pr, device=DEV, local_prec="bf16", coarse_prec="f32", options=opts)
    b = np.random.default_rng(7).standard_normal(pr.n_dof)
    xo, oinfo = md.solve(b, np.zeros(pr.n_dof), tol=1e-10)
    x = torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV)
    info = ctx.solve(T(b), x, 1e-10, 2000)
    print(f"bf16 margin 2^-{k}: {info['local_fp32']} of 6 subdomains in FP32, iters {info['iters']} "
          f"(fp64 oracle {oinfo.iters}), true relres {info['true_relres']:.2e}", flush=True)
    assert info["true_relres"] < 2e-10
    assert rel_l2(N(x), xo) < 1e-8
    if k == 0:
        assert info["local_fp32"] == 6
        c32 = solver.from_problem(pr, device=DEV, local_prec="f32", coarse_prec="f32", options=opts)
        x32 = torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV)
        i32 = c32.solve(T(b), x32, 1e-10, 2000)
        assert i32["iters"] == info["iters"] and i32["local_fp32"] == 0
        assert np.array_equal(N(x32), N(x))
        c32.close()
    if k == 10:
        assert info["local_fp32"] == 0
    ctx.close()


@pytest.mark.parametrize("case", ["2d_p3", "t1_p1", "t1_p4"])
def test_unpreconditioned_cg(case):
    """B = I (the CG reference rows of Table 1): z = r exactly; a CG solve
    meets the tolerance, lies within kappa * tol of the direct solution (the
    bound for any iterate with that residual), takes the oracle's number of
    iterations up to 2 % (CG run past n iterations in floating point, as here,
    loses orthogonality at a rate set by rounding, so the count is not fixed
    by the arithmetic alone), and its recorded (alpha, beta) give the oracle's
    Lanczos kappa (t1_p4 takes ~2900 iterations: the long-history path).
    Switching the preconditioner back on gives the bits of the earlier
    preconditioned solve."""
    pr, md, ctx = _setup(case)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(pr.n_dof)
    x0 = rng.standard_normal(pr.n_dof)
    xp_before = T(x0)
    ctx.solve(T(b), xp_before, 1e-10, 2000)
    ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 0)
    try:
        z = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
        ctx.precond_apply(T(b), z)
        assert np.array_equal(N(z), b)
        xo, oinfo = md.solve(b, x0, tol=1e-10, maxit=20000, precond=False)
        x = T(x0)
        info = ctx.solve(T(b), x, 1e-10, 20000)
        kappa, _, _ = ctx.lanczos()
        k_o = lanczos_kappa(oinfo.alphas, oinfo.betas)
        print(case, "CG iters gpu", info["iters"], "oracle", oinfo.iters, "kappa", kappa, k_o, flush=True)
        assert abs(info["iters"] - oinfo.iters) <= max(1, 0.02 * oinfo.iters)
        assert info["relres"] <= 1e-10
        xd = np.linalg.solve(md.K.toarray(), b)
        assert rel_l2(N(x), xd) <= 2.0 * k_o * 1e-10
        assert abs(kappa - k_o) <= 1e-3 * k_o
    finally:
        ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 1)
    xp_after = T(x0)
    ctx.solve(T(b), xp_after, 1e-10, 2000)
    assert np.array_equal(N(xp_after), N(xp_before))


# ---------------------------------------------------------------------------
# The pre-summed dot products: a single-block reduction kernel sums the
# per-workgroup partials of (p, q), (r, z) and (r, r) once (switched on by
# itself only for systems of cfg3's size).  Forced on small systems, the solves
# and time steps must match the oracle and be bitwise equal to the default path
# (both sum in the same order).
@pytest.mark.parametrize("case", ["cfg1", "3d_p2", "3d_p3", "t1_p1", "3d_p2_endpoint"])
def test_presummed_reductions(case):
    pr, md, ctx = _setup(case)
    ctx_f = solver.from_problem(pr, device=DEV, options={_lib.PDG_OPT_PRESUM: 1})
    rng = np.random.default_rng(41)
    b = rng.standard_normal(pr.n_dof)
    x0 = rng.standard_normal(pr.n_dof)
    xo, oinfo = md.solve(b, x0, tol=1e-10)
    xd, xf = T(x0), T(x0)
    info_d = ctx.solve(T(b), xd, 1e-10, 2000)
    info_f = ctx_f.solve(T(b), xf, 1e-10, 2000)
    assert info_f["iters"] == info_d["iters"]
    assert np.array_equal(N(xf), N(xd))
    assert iters_agree(info_f["iters"], oinfo, 1e-10, np.linalg.norm(b))
    assert rel_l2(N(xf), xo) < 1e-8
    # plain CG (B = I) pre-sums (r, r) instead of (r, z)
    ctx_f.set_option(_lib.PDG_OPT_PRECONDITIONER, 0)
    ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 0)
    try:
        xd, xf = T(x0), T(x0)
        info_d = ctx.solve(T(b), xd, 1e-10, 20000)
        info_f = ctx_f.solve(T(b), xf, 1e-10, 20000)
        assert info_f["iters"] == info_d["iters"] and np.array_equal(N(xf), N(xd))
    finally:
        ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 1)
        ctx_f.set_option(_lib.PDG_OPT_PRECONDITIONER, 1)
    # time steps
    U, Up, Y = md.initial_state()
    Ug, Upg, Yg = solver.initial_state(ctx_f, pr)
    for k in range(2):
        Yn_o, I_o = md.ionic_update(U, Up, Y)
        b_o = md.rhs(U, I_o)
        U, Up, Y, oinfo = md.step(U, Up, Y)
        info = ctx_f.step(Ug, Upg, Yg, None, pr.tol, pr.maxit)
        err = rel_l2(N(Ug), U)
        print(f"{case} presum step {k}: iters gpu {info['iters']} oracle {oinfo.iters} relL2 {err:.2e}", flush=True)
        assert iters_agree(info["iters"], oinfo, pr.tol, np.linalg.norm(b_o))
        assert err < 1e-8
    ctx_f.close()


# ---------------------------------------------------------------------------
# Device error statuses: each is detected on the device and returned by the call.
def test_nan_rhs_gives_nonfinite():
    pr, md, ctx = _setup("3d_p2")
    b = np.random.default_rng(8).standard_normal(pr.n_dof)
    b[pr.n_dof // 3] = np.nan
    x = torch.zeros(pr.n_dof, dtype=torch.float64, device=DEV)
    with pytest.raises(PdgError) as ei:
        ctx.solve(T(b), x, 1e-10, 100)
    assert ei.value.status == _lib.PDG_ENONFINITE
    # the context still works afterwards
    b[pr.n_dof // 3] = 1.0
    info = ctx.solve(T(b), x, 1e-10, 1000)
    assert info["relres"] <= 1e-10


@pytest.mark.parametrize("call", ["ionic", "step"])
def test_nonpositive_concentration_gives_nonfinite(call):
    """A non-positive extracellular potassium [K]_o (ionic state 2) before its
    logarithm is an error (the model is not evaluated there), not clamped."""
    pr, md, ctx = _setup("3d_p2_endpoint")
    U, Up, Y = md.initial_state()
    Y = Y.reshape(5, pr.n_elem, pr.nd).copy()
    e = pr.n_elem // 2
    Y[2, e, :] = 0.0
    Y[2, e, 0] = -1.0  # a negative constant on element e
    Yd, Ud, Upd = T(Y.ravel()), T(U), T(Up)
    with pytest.raises(PdgError) as ei:
        if call == "ionic":
            ctx.ionic(Ud, Upd, Yd, torch.empty(pr.n_dof, dtype=torch.float64, device=DEV))
        else:
            ctx.step(Ud, Upd, Yd, None, pr.tol, pr.maxit)
    assert ei.value.status == _lib.PDG_ENONFINITE
    # a valid state steps normally afterwards
    U, Up, Y = md.initial_state()
    info = ctx.step(T(U), T(Up), T(Y.ravel()), None, pr.tol, pr.maxit)
    assert info["relres"] <= pr.tol


def test_large_item_size_is_cut_to_the_lds_limit():
    """PDG_OPT_SCHWARZ_ITEM_KB = 8192 asks for items of up to 256 FP64 tiles.
    The plan cuts them to what one workgroup's LDS holds (here for the coarse
    system of 3,840 dofs, 60 tile rows), and the solve agrees with the default
    plan's."""
    pr = problems.table1_problem(1024, 4, 2, n_steps=2)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(pr.n_dof)
    res = {}
    for kb in (128, 8192):
        ctx = solver.from_problem(pr, device=DEV, options={_lib.PDG_OPT_SCHWARZ_ITEM_KB: kb})
        x = T(np.zeros(pr.n_dof))
        info = ctx.solve(T(b), x, 1e-10, 5000)
        print(f"[item kb {kb}] iters {info['iters']} relres {info['relres']:.2e}", flush=True)
        assert info["relres"] <= 1e-10
        res[kb] = (info["iters"], N(x))
    assert abs(res[128][0] - res[8192][0]) <= 1
    assert rel_l2(res[8192][1], res[128][1]) < 1e-8
