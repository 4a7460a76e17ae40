"""C-ABI library on the host (no GPU): symbol exports, host-side setup parity
against the oracle (independent implementations), and error codes."""
import os
import re

import numpy as np
import pytest

from oracle.monodomain import Monodomain
from paper_2512_19536_amd import _lib, solver
from paper_2512_19536_amd._lib import PdgError
from pdg_inputs import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "pdg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pdg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared


def _dense_from_bsr(row_ptr, col, val, n_elem, nd):
    K = np.zeros((n_elem * nd, n_elem * nd))
    for e in range(n_elem):
        for k in range(row_ptr[e], row_ptr[e + 1]):
            c = col[k]
            K[e * nd:(e + 1) * nd, c * nd:(c + 1) * nd] = val[k]
    return K


CASES = {
    "cfg1": problems.cfg1,
    "2d_p1": lambda: problems.small2d(n=20, p=1),
    "2d_p4": lambda: problems.small2d(n=20, p=4),
    "3d_p1": lambda: problems.small3d(p=1),
    "3d_p3": lambda: problems.small3d(p=3),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_host_setup_matches_oracle(case):
    pr = CASES[case]()
    md = Monodomain(pr)
    ctx = solver.from_problem(pr, device=None)
    row_ptr, col, val, mass = ctx.get_matrix()
    nd = pr.nd
    assert np.all(col[row_ptr[:-1]] == np.arange(pr.n_elem))  # diagonal block first
    K = _dense_from_bsr(row_ptr, col, val, pr.n_elem, nd)
    Ko = md.K.toarray()
    assert abs(K - Ko).max() <= 1e-13 * abs(Ko).max()
    assert abs(mass - md.disc.M).max() <= 1e-13 * abs(md.disc.M).max()
    for s in range(pr.n_sub):
        Kinv = ctx.get_local_inverse(s)
        d = md.schwarz.dofs[s]
        ref = np.linalg.inv(Ko[np.ix_(d, d)])
        assert abs(Kinv - ref).max() <= 1e-11 * abs(ref).max()
    P, K0 = ctx.get_coarse()
    nq0 = P.shape[2]
    Pl = np.zeros(md.schwarz.P.shape)
    for e in range(pr.n_elem):
        c = pr.elem_coarse[e]
        Pl[e * nd:(e + 1) * nd, c * nq0:(c + 1) * nq0] = P[e]
    Po = md.schwarz.P.toarray()
    assert abs(Pl - Po).max() <= 1e-12 * abs(Po).max()
    assert abs(K0 - md.schwarz.K0).max() <= 1e-12 * abs(K0).max()


def _expect(status, fn, *a, **k):
    with pytest.raises(PdgError) as ei:
        fn(*a, **k)
    assert ei.value.status == status, str(ei.value)


def test_error_codes_from_the_host():
    pr = problems.small2d(n=12, p=2)
    ctx = solver.Context(None)
    # out of order
    _expect(_lib.PDG_ESTATE, ctx.assemble, 1.0, 1.0, 0.05, 10.0)
    # bad degree
    _expect(_lib.PDG_EINVAL, ctx.set_mesh, pr.mesh, 7)
    ctx.set_mesh(pr.mesh, 2)
    _expect(_lib.PDG_EINVAL, ctx.assemble, 1.0, 1.0, -0.05, 10.0)
    ctx.assemble(1.0, 1.0, 0.05, 10.0)
    _expect(_lib.PDG_EINVAL, ctx.set_ionic, np.zeros(5))
    bad = pr.elem_sub.copy()
    bad[0] = 99
    d = solver.Context.setup_preconditioner
    _expect(_lib.PDG_EINVAL, d, ctx, bad, None, 1)
    # compute calls on a host-only context
    _expect(_lib.PDG_ESTATE, ctx.workspace_query)
    ctx.setup_preconditioner(pr.elem_sub, None, 1)
    assert ctx.workspace_query() > 0
    _expect(_lib.PDG_ESTATE, ctx._call, "pdg_bind_workspace", None, 0)


def test_indefinite_system_reports_not_spd():
    """Without penalty (eta0 = 0) and a negligible mass term the SIPG matrix is
    indefinite, so a subdomain's Cholesky factorisation meets a pivot <= 0."""
    pr = problems.small2d(n=16, p=2)
    ctx = solver.Context(None)
    ctx.set_mesh(pr.mesh, 2)
    ctx.assemble(1.0, 1.0, 1e9, 0.0)
    _expect(_lib.PDG_ENOTSPD, ctx.setup_preconditioner, np.zeros(pr.n_elem, np.int32), None, 0)


def test_non_spd_conductivity_rejected():
    pr = problems.small2d(n=12, p=1)
    pr.mesh.sigma = pr.mesh.sigma.copy()
    pr.mesh.sigma[3] = np.array([[1.0, 2.0], [2.0, 1.0]])
    ctx = solver.Context(None)
    _expect(_lib.PDG_EINVAL, ctx.set_mesh, pr.mesh, 1)
