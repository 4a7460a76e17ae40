"""GPU parity at the benchmarked sizes, in the launch configuration bench.py times.

* cfg2 (80,610 dofs, 64 subdomains + P1 coarse, FP64): SpMV and Schwarz apply
  against the oracle element by element; two time steps against the oracle
  (equal iteration counts under the rule of test_gpu_parity, relative L2 1e-8).
* cfg3 (~660k dofs, p = 3, 512 subdomains): too large for the oracle in a
  test, so its first step is stored (tests/golden/cfg3_step1.json, sampled
  entries): FP64, FP32 and BF16 Schwarz solves against it, then a second step
  of each against the FP64 form, every one meeting the FP64 true relative
  residual 1e-10.
* cfg4 (64 systems, ~1.05M dofs, p = 1..4, one context per degree, graphs on,
  as benchmarked): every system converges with a true relative residual below
  2e-10; one system of each degree gives in its own context the same bits and
  iteration count; the two smallest systems agree with the FP64 oracle (which
  uses FP64 Schwarz solves) to 1e-8.
* the long run of Section 5 (Fig. 2: p = q = 4, N_h = 4096, H = 4h, one
  subdomain per element, 61,440 dofs and 3,840 coarse dofs): its first two
  time steps against the oracle (equal iterations under the rule of
  test_gpu_parity, relative L2 1e-8 on U and on the ionic state).
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2512_19536_amd import _lib, solver  # noqa: E402
from pdg_inputs import problems  # noqa: E402
from parity_rules import iters_agree  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_cfg2_full_size_against_oracle():
    from oracle.monodomain import Monodomain
    pr = problems.cfg2()
    print("[cfg2] oracle setup", flush=True)
    md = Monodomain(pr)
    ctx = solver.from_problem(pr, device=DEV)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(pr.n_dof)
    y = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
    ctx.spmv(T(x), y)
    yo = md.K @ x
    assert np.abs(N(y) - yo).max() <= 1e-13 * np.abs(yo).max()
    z = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
    ctx.precond_apply(T(x), z)
    zo = md.schwarz.apply(x)
    assert np.abs(N(z) - zo).max() <= 1e-11 * np.abs(zo).max()
    U, Up, Y = md.initial_state()
    Ug, Upg, Yg = solver.initial_state(ctx, pr)
    for k in range(2):
        Yn, I = md.ionic_update(U, Up, Y)
        bnorm = np.linalg.norm(md.rhs(U, I))
        U, Up, Y, oinfo = md.step(U, Up, Y)
        info = ctx.step(Ug, Upg, Yg, None, pr.tol, pr.maxit)
        err = rel_l2(N(Ug), U)
        print(f"[cfg2] step {k}: iters gpu {info['iters']} oracle {oinfo.iters} rel L2 {err:.2e}", flush=True)
        assert iters_agree(info["iters"], oinfo, pr.tol, bnorm)
        assert err < 1e-8
        assert rel_l2(N(Yg), Y.ravel()) < 1e-8


CFG3_FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_step1.json")


@pytest.mark.timeout(900)
def test_cfg3_precision_forms_against_oracle():
    """cfg3 with FP64, FP32 and BF16-stored Schwarz solves (FP32 coarse for the
    reduced forms; outer CG, dots and SpMV in FP64): the first step from the
    initial state against the FP64 oracle's, stored by
    tests/golden/make_cfg3_fixture.py (sampled entries; equal iterations for
    FP64 under the rule of test_gpu_parity); the second step of each form
    meets the FP64 true relative residual and agrees with the FP64 form."""
    with open(CFG3_FIXTURE) as f:
        fx = json.load(f)
    idx = np.asarray(fx["idx"])
    U1o, U0o = np.asarray(fx["U1"]), np.asarray(fx["U0"])
    pr = problems.cfg3()
    assert pr.n_dof == fx["n_dof"]
    opts = {_lib.PDG_OPT_TRUE_RESIDUAL: 1}
    second = {}
    for prec in ("f64", "f32", "bf16"):
        print(f"[cfg3] {prec} setup", flush=True)
        c = solver.from_problem(pr, device=DEV, local_prec=prec, coarse_prec="f64" if prec == "f64" else "f32",
                                options=opts)
        U, Up, Y = solver.initial_state(c, pr)
        # the same per-element constants projected by each side's own code
        assert np.abs(N(U)[idx] - U0o).max() <= 1e-12 * np.abs(U0o).max()
        info = c.step(U, Up, Y, None, pr.tol, pr.maxit)
        u1 = N(U)[idx]
        err = np.linalg.norm(u1 - U1o) / np.linalg.norm(U1o)
        derr = np.linalg.norm(u1 - U1o) / np.linalg.norm(U1o - U0o)
        print(f"[cfg3] {prec} step 0: iters {info['iters']} (oracle {fx['iters']}), {info['local_fp32']} "
              f"subdomains in FP32, true relres {info['true_relres']:.2e}, sampled rel L2 vs oracle {err:.2e} "
              f"(of the change {derr:.2e})", flush=True)
        assert info["true_relres"] < 2e-10
        assert err < 1e-8
        if prec == "f64":
            thr = pr.tol * fx["bnorm"]
            g, o = info["iters"], fx["iters"]
            assert g == o or (g == o - 1 and fx["resnorm_last"][0] <= 1.2 * thr) or \
                (g == o + 1 and fx["resnorm_last"][1] >= thr / 1.2)
        info = c.step(U, Up, Y, None, pr.tol, pr.maxit)
        print(f"[cfg3] {prec} step 1: iters {info['iters']}, true relres {info['true_relres']:.2e}", flush=True)
        assert info["true_relres"] < 2e-10
        second[prec] = N(U)
        c.close()
        del c
        torch.cuda.empty_cache()
    for prec in ("f32", "bf16"):
        err = rel_l2(second[prec], second["f64"])
        print(f"[cfg3] step 1: {prec} vs f64 rel L2 {err:.2e}", flush=True)
        assert err < 1e-8


@pytest.mark.timeout(600)
def test_cfg4_batch_full_size():
    batch = problems.cfg4()
    print(f"[cfg4] {len(batch.systems)} systems, {batch.n_dof} dofs; setup", flush=True)
    opts = {_lib.PDG_OPT_GRAPH: 1, _lib.PDG_OPT_TRUE_RESIDUAL: 1}
    bs = solver.BatchSolver(batch, device=DEV, options=opts)
    U, Up, Y = bs.initial_state()
    U0 = [u.clone() for u in U]
    bs.step(U, Up, Y, 1e-10, 5000)
    worst = 0.0
    for i in range(len(batch.systems)):
        si = bs.system_info(i)
        assert si["status"] == _lib.PDG_OK
        worst = max(worst, si["true_relres"])
    print(f"[cfg4] step 0: worst true relres {worst:.2e}", flush=True)
    assert worst < 2e-10
    # one system of each degree in its own context
    for p, (_, idx) in sorted(batch.groups.items()):
        i = idx[len(idx) // 2]
        q = batch.systems[i]
        c1 = solver.from_problem(q, device=DEV)
        u, up, y = solver.initial_state(c1, q)
        info = c1.step(u, up, y, None, q.tol, q.maxit)
        ci, sl = bs.system_slice(i)
        print(f"[cfg4] system {i} (p={p}, {q.n_dof} dofs): iters batch {bs.system_info(i)['iters']} "
              f"single {info['iters']}", flush=True)
        assert info["iters"] == bs.system_info(i)["iters"]
        assert np.array_equal(N(u), N(U[ci])[sl])
        del c1
    # the two smallest systems against the oracle
    from oracle.monodomain import Monodomain
    for i in np.argsort([q.n_dof for q in batch.systems])[:2]:
        q = batch.systems[int(i)]
        md = Monodomain(q)
        Uo, Upo, Yo = md.initial_state()
        Uo, Upo, Yo, oinfo = md.step(Uo, Upo, Yo)
        ci, sl = bs.system_slice(int(i))
        err = rel_l2(N(U[ci])[sl], Uo)
        print(f"[cfg4] system {int(i)} vs oracle: iters gpu {bs.system_info(int(i))['iters']} "
              f"oracle {oinfo.iters}, rel L2 {err:.2e}", flush=True)
        assert err < 1e-8


def test_fig2_long_run_configuration_against_oracle():
    from oracle.monodomain import Monodomain
    pr = problems.table1_problem(4096, 4, 4)
    print(f"[fig2] {pr.name}: {pr.n_dof} dofs; oracle setup", flush=True)
    md = Monodomain(pr)
    ctx = solver.from_problem(pr, device=DEV)
    U, Up, Y = md.initial_state()
    Ug, Upg, Yg = solver.initial_state(ctx, pr)
    for k in range(2):
        Yn, I = md.ionic_update(U, Up, Y)
        bnorm = np.linalg.norm(md.rhs(U, I))
        U, Up, Y, oinfo = md.step(U, Up, Y)
        info = ctx.step(Ug, Upg, Yg, None, pr.tol, pr.maxit)
        err = rel_l2(N(Ug), U)
        derr = rel_l2(N(Ug) - Up, U - Up)
        print(f"[fig2] step {k}: iters gpu {info['iters']} oracle {oinfo.iters} rel L2 {err:.2e} "
              f"(of the change {derr:.2e})", flush=True)
        assert iters_agree(info["iters"], oinfo, pr.tol, bnorm)
        assert err < 1e-8
        assert rel_l2(N(Yg), Y.ravel()) < 1e-8
