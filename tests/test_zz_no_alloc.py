"""The allocation-free preconditioner apply (pdg_precond_apply_noalloc).

It runs the kernels of pdg_precond_apply with their scratch in a static
device array, so its output must equal pdg_precond_apply's bit for bit, and
both must match the oracle's B^{-1} r (eq. (5)) to rounding.  Two calls in a
row, the second on a smaller system (a stale tail of the larger call's
scratch must not leak into it), then the larger system again.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.monodomain import Monodomain  # noqa: E402
from paper_2512_19536_amd import _lib, solver  # noqa: E402
from pdg_inputs import problems  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _check(name, pr, md, ctx, seed):
    print(f"[noalloc] {name}: {pr.n_dof} dofs, seed {seed}", flush=True)
    r = np.random.default_rng(seed).standard_normal(pr.n_dof)
    rd = _T(r)
    z_ref = torch.full((pr.n_dof,), np.nan, dtype=torch.float64, device=DEV)
    z_na = torch.full((pr.n_dof,), np.nan, dtype=torch.float64, device=DEV)
    ctx.precond_apply(rd, z_ref)
    ctx.precond_apply_noalloc(rd, z_na)
    a, b = _N(z_na), _N(z_ref)
    assert np.array_equal(a, b), f"{name}: max diff {np.abs(a - b).max():.3e}"
    assert _rel_max(a, md.schwarz.apply(r)) < 1e-11


def test_noalloc_apply_matches_precond_apply():
    big = problems.small3d(n_grid=8, p=3, n_sub=6)       # 10,240 dofs, coarse level
    small = problems.cfg1()                              # 384 dofs
    md_big, md_small = Monodomain(big), Monodomain(small)
    ctx_big = solver.from_problem(big, device=DEV)
    ctx_small = solver.from_problem(small, device=DEV)
    try:
        _check("larger", big, md_big, ctx_big, 11)
        _check("larger, again", big, md_big, ctx_big, 12)
        _check("smaller", small, md_small, ctx_small, 13)
        _check("larger after smaller", big, md_big, ctx_big, 14)
    finally:
        ctx_big.close()
        ctx_small.close()


def test_noalloc_apply_fp32_tiles_and_plain_cg():
    pr = problems.small3d(n_grid=8, p=2, n_sub=6)
    md = Monodomain(pr)
    ctx = solver.from_problem(pr, device=DEV, local_prec="f32", coarse_prec="f32")
    try:
        r = np.random.default_rng(21).standard_normal(pr.n_dof)
        rd = _T(r)
        z_ref = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
        z_na = torch.empty(pr.n_dof, dtype=torch.float64, device=DEV)
        ctx.precond_apply(rd, z_ref)
        ctx.precond_apply_noalloc(rd, z_na)
        assert np.array_equal(_N(z_na), _N(z_ref))
        assert _rel_max(_N(z_na), md.schwarz.apply(r)) < 1e-4
        # B = I: the apply copies r
        ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 0)
        ctx.precond_apply_noalloc(rd, z_na)
        assert np.array_equal(_N(z_na), r)
    finally:
        ctx.close()
