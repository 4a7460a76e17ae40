"""C-ABI library on the host (no GPU): symbol exports, host-side setup parity
against the oracle (independent implementations), and error codes."""
import copy
import os
import re
from dataclasses import replace

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
    "3d_p2_q2": lambda: replace(problems.small3d(p=2), coarse_q=2),
    "t1_p2": lambda: problems.table1_problem(48, 2, 2),
    "t1_p4": lambda: problems.table1_problem(40, 4, 2),
    "t1_p4_q2": lambda: replace(problems.table1_problem(40, 4, 2), coarse_q=2),
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
    # empty mesh
    empty = copy.deepcopy(pr.mesh)
    empty.cell_ptr = np.zeros(1, np.int64)
    for f in ("cell_geom", "facet_elem", "facet_geom", "facet_normal", "sigma"):
        setattr(empty, f, getattr(pr.mesh, f)[:0])
    _expect(_lib.PDG_EINVAL, ctx.set_mesh, empty, 2)
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


def test_option_and_coarse_errors_from_the_host():
    """Option values out of range, the coarse degree above p, and the workspace
    growing with the Lanczos history; all on a host-only context."""
    pr = problems.small2d(n=12, p=2)
    ctx = solver.Context(None)
    for opt, val in ((_lib.PDG_OPT_PRECONDITIONER, 2), (_lib.PDG_OPT_LANCZOS_CAP, 0),
                     (_lib.PDG_OPT_LANCZOS_CAP, (1 << 20) + 1), (_lib.PDG_OPT_ION_EXTRAPOLATION, 2),
                     (_lib.PDG_OPT_SCHWARZ_ITEM_KB, 16), (_lib.PDG_OPT_SPMV_WAVES, 3),
                     (_lib.PDG_OPT_KERNEL_TIMING, -1), (_lib.PDG_OPT_KERNEL_TIMING, (1 << 20) + 1), (99, 1)):
        _expect(_lib.PDG_EINVAL, ctx.set_option, opt, val)
    for opt in (_lib.PDG_OPT_PRECONDITIONER, _lib.PDG_OPT_ION_EXTRAPOLATION, _lib.PDG_OPT_KERNEL_TIMING):
        ctx.set_option(opt, 0)
        ctx.set_option(opt, 1)
    ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, 8)
    ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, 0)
    ctx.set_mesh(pr.mesh, 2)
    ctx.assemble(1.0, 1.0, 0.05, 10.0)
    _expect(_lib.PDG_EINVAL, ctx.setup_preconditioner, pr.elem_sub, None, 3)  # q > p
    ctx.setup_preconditioner(pr.elem_sub, None, 2)
    w0 = ctx.workspace_query()
    ctx.set_option(_lib.PDG_OPT_LANCZOS_CAP, 4096)
    assert ctx.workspace_query() == w0 + 2048 * 16


def test_coarse_system_size_limit():
    """A coarse system above 16,384 dofs is refused at setup (PDG_EINVAL); the
    largest Table-1 cell (15,360) is below it."""
    big = problems.table1_problem(1100, 4, 1)  # 1100 one-element agglomerates x 15 = 16,500 coarse dofs
    c2 = solver.Context(None)
    c2.set_mesh(big.mesh, 4)
    c2.assemble(big.chi_m, big.c_m, big.dt, big.eta0)
    with pytest.raises(PdgError) as ei:
        c2.setup_preconditioner(big.elem_sub, big.elem_coarse, 4)
    assert ei.value.status == _lib.PDG_EINVAL and "16384" in str(ei.value)


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


def _small_batch():
    """Three independent 3-D problems of one degree (different meshes, sizes,
    partitions) concatenated into one batch problem."""
    systems = [problems.small3d(n_grid=g, p=2, n_sub=ns, seed=sd) for g, ns, sd in ((5, 3, 21), (6, 4, 22), (4, 2, 23))]
    return systems, problems.concat_problems("batch", systems)


def test_batch_host_setup_is_block_diagonal():
    """A batch context holds exactly the matrices, local inverses and coarse
    operators of its systems' own contexts (block diagonal over systems)."""
    systems, bp = _small_batch()
    cb = solver.from_problem(bp, device=None)
    row_ptr, col, val, _ = cb.get_matrix()
    Kb = _dense_from_bsr(row_ptr, col, val, bp.n_elem, bp.nd)
    Pb, K0b = cb.get_coarse()
    e0, s0, c0 = 0, 0, 0
    for q in systems:
        cq = solver.from_problem(q, device=None)
        rp, cl, vl, _ = cq.get_matrix()
        Kq = _dense_from_bsr(rp, cl, vl, q.n_elem, q.nd)
        d0, d1 = e0 * bp.nd, (e0 + q.n_elem) * bp.nd
        assert np.array_equal(Kb[d0:d1, d0:d1], Kq)
        assert not np.any(Kb[d0:d1, :d0]) and not np.any(Kb[d0:d1, d1:])
        for s in range(q.n_sub):
            assert np.array_equal(cb.get_local_inverse(s0 + s), cq.get_local_inverse(s))
        Pq, K0q = cq.get_coarse()
        assert np.array_equal(Pb[e0:e0 + q.n_elem], Pq)
        nq = K0q.shape[0]
        assert np.allclose(K0b[c0:c0 + nq, c0:c0 + nq], K0q, rtol=0, atol=1e-12 * abs(K0q).max())
        assert not np.any(K0b[c0:c0 + nq, :c0]) and not np.any(K0b[c0:c0 + nq, c0 + nq:])
        e0 += q.n_elem
        s0 += q.n_sub
        c0 += nq


def test_batch_validation_errors():
    systems, bp = _small_batch()
    ctx = solver.Context(None)
    ctx.set_mesh(bp.mesh, bp.p)
    n = bp.n_elem
    for bad in ([0, n + 1], [1, n], [0, 10, 10, n]):
        with pytest.raises(PdgError) as e:
            ctx.set_systems(bad)
        assert e.value.status == _lib.PDG_EINVAL
    # a cut through one system leaves facets between the two parts
    with pytest.raises(PdgError) as e:
        ctx.set_systems([0, systems[0].n_elem // 2, n])
    assert e.value.status == _lib.PDG_EINVAL
    # a subdomain spanning two systems
    ctx.set_systems(bp.elem_ptr)
    ctx.assemble(bp.chi_m, bp.c_m, bp.dt, bp.eta0)
    sub = bp.elem_sub.copy()
    sub[systems[0].n_elem] = sub[0]
    with pytest.raises(PdgError) as e:
        ctx.setup_preconditioner(sub, None, 1)
    assert e.value.status == _lib.PDG_EINVAL
    # after setup the system split is fixed
    ctx.setup_preconditioner(bp.elem_sub, bp.elem_coarse, 1)
    with pytest.raises(PdgError) as e:
        ctx.set_systems(bp.elem_ptr)
    assert e.value.status == _lib.PDG_ESTATE


def test_concat_meshes_keeps_systems_apart():
    systems, bp = _small_batch()
    m = bp.mesh
    f = m.facet_elem
    sys_of = np.searchsorted(bp.elem_ptr, np.arange(m.n_elem), side="right") - 1
    inner = f[:, 1] >= 0
    assert np.array_equal(sys_of[f[inner, 0]], sys_of[f[inner, 1]])
    assert m.n_facet == sum(q.mesh.n_facet for q in systems)
    assert np.allclose(m.element_measure(), np.concatenate([q.mesh.element_measure() for q in systems]))
