"""GPU Lanczos estimate of the condition number (Section 5's diagnostic).

* The coefficients the library records during a step equal the oracle's for
  the same step in the early iterations (1e-9 relative from identical inputs at
  the first step; 1e-6 at the next, whose inputs already differ at the PCG
  tolerance); later ones drift apart
  with rounding, as CG coefficients do (the sensitivity behind the iteration
  rule), so the two runs' estimates agree only to about 1e-3.
* The device's bisection gives the extreme eigenvalues of the tridiagonal
  matrix built from the recorded coefficients to 1e-10 relative (numpy eigvalsh
  of the same matrix, built by the oracle's routine)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.monodomain import Monodomain  # noqa: E402
from oracle.pcg import lanczos_tridiagonal  # noqa: E402
from paper_2512_19536_amd import _lib, solver  # noqa: E402
from paper_2512_19536_amd._lib import PdgError  # noqa: E402
from pdg_inputs import problems  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = {"cfg1": problems.cfg1, "3d_p3": lambda: problems.small3d(p=3), "2d_p4": lambda: problems.small2d(n=20, p=4)}


@pytest.mark.parametrize("case", sorted(CASES))
def test_lanczos_kappa_matches_oracle(case):
    pr = CASES[case]()
    md = Monodomain(pr)
    ctx = solver.from_problem(pr, device=DEV)
    U, Up, Y = md.initial_state()
    Ug, Upg, Yg = solver.initial_state(ctx, pr)
    for k in range(2):
        U, Up, Y, oinfo = md.step(U, Up, Y)
        info = ctx.step(Ug, Upg, Yg, None, pr.tol, pr.maxit)
        if info["iters"] != oinfo.iters:
            continue  # a count decided by rounding (see the iteration rule): matrices differ in size
        kappa, lo, hi = ctx.lanczos(0)
        a, b = ctx.pcg_coefficients(0)
        n_early = min(10, len(a) - 1)
        rt = 1e-9 if k == 0 else 1e-6
        assert np.allclose(a[:n_early], oinfo.alphas[:n_early], rtol=rt, atol=0)
        assert np.allclose(b[:n_early], oinfo.betas[:n_early], rtol=rt, atol=0)
        ev = np.linalg.eigvalsh(lanczos_tridiagonal(list(a), list(b[:-1])))
        evo = np.linalg.eigvalsh(lanczos_tridiagonal(oinfo.alphas, oinfo.betas))
        print(f"[lanczos] {case} step {k}: iters {info['iters']} kappa gpu {kappa:.8f} (same coefficients "
              f"{ev[-1] / ev[0]:.8f}; oracle run {evo[-1] / evo[0]:.8f})", flush=True)
        assert abs(lo - ev[0]) <= 1e-10 * abs(ev[0])
        assert abs(hi - ev[-1]) <= 1e-10 * abs(ev[-1])
        assert abs(kappa - evo[-1] / evo[0]) <= 1e-3 * (evo[-1] / evo[0])
    # other compute calls make the estimate stale
    ctx.ionic(Ug, Upg, Yg.clone(), torch.empty_like(Ug))
    with pytest.raises(PdgError) as e:
        ctx.lanczos(0)
    assert e.value.status == _lib.PDG_ESTATE
