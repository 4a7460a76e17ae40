"""The paper's Table-1 experiment mode on the GPU (Section 5): one subdomain
per element (block Jacobi) plus a coarse space of degree q = p on nested
agglomerates, grey/white square, dt = 2.5 us, relative residual 1e-9.

Checks the claims the paper draws from Table 1 (trend only; its meshes and
ionic parameters are not available, so magnitudes are not pinned):
* at fixed H/h the iteration count and the condition-number estimate stay
  about constant as the fine mesh is refined (scalability);
* they grow with H/h;
* the preconditioned solver needs far fewer iterations than plain CG, whose
  condition number grows like h^-2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2512_19536_amd import _lib, solver  # noqa: E402
from pdg_inputs import problems  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cell(n_h, p, k, precond=True, n_steps=3):
    pr = problems.table1_problem(n_h, p, k)
    ctx = solver.from_problem(pr, device=DEV, options={_lib.PDG_OPT_LANCZOS_CAP: 1 << 14})
    if not precond:
        ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 0)
    U, Up, Y = solver.initial_state(ctx, pr)
    iters = []
    for _ in range(n_steps):
        info = ctx.step(U, Up, Y, None, pr.tol, 20000)
        assert info["relres"] <= pr.tol
        iters.append(info["iters"])
    kappa = ctx.lanczos()[0]
    print(f"[table1] N_h={n_h} p={p} {'H=%dh' % k if precond else 'CG'}: iters {iters} kappa {kappa:.4g}",
          flush=True)
    return float(np.mean(iters)), kappa


def test_table1_trends_p1():
    res = {(nh, k): _cell(nh, 1, k) for nh in (256, 1024) for k in (2, 4)}
    cg = {nh: _cell(nh, 1, 2, precond=False) for nh in (256, 1024)}
    for k in (2, 4):
        (i0, k0), (i1, k1) = res[(256, k)], res[(1024, k)]
        assert abs(i1 - i0) <= 0.25 * i0 and 0.5 <= k1 / k0 <= 2.0
    for nh in (256, 1024):
        assert res[(nh, 4)][0] > res[(nh, 2)][0] and res[(nh, 4)][1] > res[(nh, 2)][1]
        assert cg[nh][0] > 4 * res[(nh, 2)][0]
    # kappa(K) ~ h^-2: four times the elements, about four times the condition number
    assert 2.5 <= cg[1024][1] / cg[256][1] <= 6.0
