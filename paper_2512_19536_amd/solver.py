"""Python face of libpdg: one :class:`Context` per problem, methods named after
the C entry points (pdg_<name>).  Arguments are marshalled to the C-ABI; all
compute runs in the library's HIP kernels.  PyTorch provides the device memory
(the workspace and the state vectors) and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import PdgMesh, PdgPrecondDesc, PdgSolveInfo, PdgTuneResult, check


def _ptr(a):
    """Address of a contiguous numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


class Context:
    """Owns a pdg_ctx.  ``device`` is a torch CUDA/HIP device or None for a
    host-only context (setup calls only)."""

    def __init__(self, device=None, stream=None):
        self.lib = _lib.load()
        self._ctx = ctypes.c_void_p()
        self.device = device
        self.torch = None
        dev_index, s = -1, None
        if device is not None:
            import torch
            self.torch = torch
            dev = torch.device(device)
            dev_index = dev.index if dev.index is not None else torch.cuda.current_device()
            self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
            s = ctypes.c_void_p(self.stream.cuda_stream)
        st = self.lib.pdg_create(ctypes.byref(self._ctx), dev_index, s)
        check(None, st)
        self._keep = []
        self.ws = None

    def close(self):
        if self._ctx:
            self.lib.pdg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        check(self._ctx, getattr(self.lib, name)(self._ctx, *args))

    # ---- setup ---------------------------------------------------------------
    def set_mesh(self, mesh, p):
        arr = mesh.as_abi_arrays()
        self._mesh_arrays = arr
        m = PdgMesh(dim=mesh.dim, n_elem=mesh.n_elem, cell_ptr=_ptr(arr["cell_ptr"]),
                    cell_geom=_ptr(arr["cell_geom"]), n_facet=len(arr["facet_elem"]),
                    facet_elem=_ptr(arr["facet_elem"]), facet_geom=_ptr(arr["facet_geom"]),
                    facet_normal=_ptr(arr["facet_normal"]), sigma=_ptr(arr["sigma"]))
        self._call("pdg_set_mesh", ctypes.byref(m), int(p))

    def set_systems(self, elem_ptr):
        ep = np.ascontiguousarray(elem_ptr, dtype=np.int64)
        self._call("pdg_set_systems", len(ep) - 1, _ptr(ep))

    def get_sizes(self):
        n_elem, nd, n_dof, nnzb = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        self._call("pdg_get_sizes", ctypes.byref(n_elem), ctypes.byref(nd), ctypes.byref(n_dof), ctypes.byref(nnzb))
        return n_elem.value, nd.value, n_dof.value, nnzb.value

    def assemble(self, chi_m, c_m, dt, eta0):
        self._call("pdg_assemble", float(chi_m), float(c_m), float(dt), float(eta0))

    def get_matrix(self):
        n_elem, nd, _, nnzb = self.get_sizes()
        row_ptr = np.zeros(n_elem + 1, np.int64)
        col = np.zeros(nnzb, np.int32)
        val = np.zeros((nnzb, nd, nd))
        mass = np.zeros((n_elem, nd, nd))
        self._call("pdg_get_matrix", _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(mass))
        return row_ptr, col, val, mass

    def set_ionic(self, params):
        prm = np.ascontiguousarray(params, dtype=np.float64)
        self._call("pdg_set_ionic", _ptr(prm), len(prm))

    def setup_preconditioner(self, elem_sub, elem_coarse=None, coarse_q=1, local_prec="f64", coarse_prec="f64"):
        es = np.ascontiguousarray(elem_sub, dtype=np.int32)
        ec = None if elem_coarse is None else np.ascontiguousarray(elem_coarse, dtype=np.int32)
        d = PdgPrecondDesc(n_sub=int(es.max()) + 1, elem_sub=_ptr(es),
                           n_coarse=0 if ec is None else int(ec.max()) + 1, elem_coarse=_ptr(ec),
                           coarse_q=int(coarse_q), local_prec=_lib.PRECISIONS[local_prec],
                           coarse_prec=_lib.PRECISIONS[coarse_prec])
        self._call("pdg_setup_preconditioner", ctypes.byref(d))

    def get_precond_sizes(self, sub=0):
        n_i, n0, nq0 = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self._call("pdg_get_precond_sizes", int(sub), ctypes.byref(n_i), ctypes.byref(n0), ctypes.byref(nq0))
        return n_i.value, n0.value, nq0.value

    def get_local_inverse(self, sub):
        n_i, _, _ = self.get_precond_sizes(sub)
        out = np.zeros((n_i, n_i))
        self._call("pdg_get_local_inverse", int(sub), _ptr(out))
        return out

    def get_coarse(self):
        n_elem, nd, _, _ = self.get_sizes()
        _, n0, nq0 = self.get_precond_sizes(0)
        P = np.zeros((n_elem, nd, nq0))
        K0 = np.zeros((n0, n0))
        self._call("pdg_get_coarse", _ptr(P), _ptr(K0))
        return P, K0

    def workspace_query(self):
        b = ctypes.c_size_t()
        self._call("pdg_workspace_query", ctypes.byref(b))
        return b.value

    def bind_workspace(self, buf=None):
        """Bind a device buffer (a torch uint8 tensor; allocated here if None)."""
        nbytes = self.workspace_query()
        if buf is None:
            buf = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        base = buf.data_ptr()
        off = (-base) % 256
        self.ws = buf
        self._call("pdg_bind_workspace", ctypes.c_void_p(base + off), ctypes.c_size_t(nbytes))

    def set_option(self, option, value):
        self._call("pdg_set_option", int(option), int(value))

    def autotune(self, reps=20):
        res = PdgTuneResult()
        self._call("pdg_autotune", int(reps), ctypes.byref(res))
        return res.as_dict()

    def kernel_timing(self):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        self._call("pdg_kernel_timing", ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by))
        return n.value, ms.value, by.value

    # ---- compute (device tensors) ----------------------------------------------
    def project_p0(self, vals, coeff):
        ncomp = vals.shape[0] if vals.dim() == 2 else 1
        self._call("pdg_project_p0", _ptr(vals), int(ncomp), _ptr(coeff))

    def spmv(self, x, y):
        self._call("pdg_spmv", _ptr(x), _ptr(y))

    def precond_apply(self, r, z):
        self._call("pdg_precond_apply", _ptr(r), _ptr(z))

    def precond_apply_noalloc(self, r, z):
        self._call("pdg_precond_apply_noalloc", _ptr(r), _ptr(z))

    def ionic(self, u, u_prev, ions, I):
        self._call("pdg_ionic", _ptr(u), _ptr(u_prev), _ptr(ions), _ptr(I))

    def rhs(self, u, I, f_ext, b):
        self._call("pdg_rhs", _ptr(u), _ptr(I), _ptr(f_ext), _ptr(b))

    def solve(self, rhs, x, tol, maxit):
        info = PdgSolveInfo()
        st = self.lib.pdg_solve(self._ctx, _ptr(rhs), _ptr(x), float(tol), int(maxit), ctypes.byref(info))
        check(self._ctx, st)
        return info.as_dict()

    def step(self, u, u_prev, ions, f_ext, tol, maxit):
        info = PdgSolveInfo()
        st = self.lib.pdg_step(self._ctx, _ptr(u), _ptr(u_prev), _ptr(ions), _ptr(f_ext), float(tol), int(maxit),
                               ctypes.byref(info))
        check(self._ctx, st)
        return info.as_dict()

    def step_guess(self, u, u_prev, ions, f_ext, guess, tol, maxit):
        info = PdgSolveInfo()
        st = self.lib.pdg_step_guess(self._ctx, _ptr(u), _ptr(u_prev), _ptr(ions), _ptr(f_ext), _ptr(guess),
                                     float(tol), int(maxit), ctypes.byref(info))
        check(self._ctx, st)
        return info.as_dict()

    def guess_extrapolate(self, u, u1, u2, order, guess):
        self._call("pdg_guess_extrapolate", _ptr(u), _ptr(u1), _ptr(u2), int(order), _ptr(guess))

    def lanczos(self, sys=0):
        """(kappa, lambda_min, lambda_max) of the last solve's Lanczos matrix."""
        k, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._call("pdg_lanczos", int(sys), ctypes.byref(k), ctypes.byref(lo), ctypes.byref(hi))
        return k.value, lo.value, hi.value

    def pcg_coefficients(self, sys=0, n=2048):
        """(alpha_1..alpha_m, beta_1..beta_m) recorded during the last solve."""
        a, b = np.zeros(n), np.zeros(n)
        self._call("pdg_get_pcg_coefficients", int(sys), _ptr(a), _ptr(b), int(n))
        m = self.system_info(sys)["iters"]
        return a[:min(m, n)], b[:min(m, n)]

    def system_info(self, sys):
        info, st = PdgSolveInfo(), ctypes.c_int32()
        self._call("pdg_get_system_info", int(sys), ctypes.byref(info), ctypes.byref(st))
        d = info.as_dict()
        d["status"] = st.value
        return d


def step_batch(ctxs, us, u_prevs, ions, tol, maxit, f_ext=None):
    """pdg_step_batch over several contexts (each on its own stream)."""
    n = len(ctxs)
    lib = ctxs[0].lib
    arr = lambda xs: (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])  # noqa: E731
    cs = (ctypes.c_void_p * n)(*[c._ctx.value for c in ctxs])
    infos = (PdgSolveInfo * n)()
    st = lib.pdg_step_batch(cs, n, arr(us), arr(u_prevs), arr(ions), None if f_ext is None else arr(f_ext),
                            float(tol), int(maxit), infos)
    check(ctxs[0]._ctx, st)
    return [i.as_dict() for i in infos]


def from_problem(problem, device="cuda:0", local_prec=None, coarse_prec=None, bind=True, options=None,
                 stream=None):
    """Context set up for a workload object with the attributes of
    ``pdg_inputs.problems.Problem`` (mesh, p, constants, partitions, ionic;
    optionally ``elem_ptr`` for a batch of independent systems).
    ``options``: {pdg option id: value} applied right after creation."""
    ctx = Context(device, stream)
    for k, v in (options or {}).items():
        ctx.set_option(k, v)
    ctx.set_option(_lib.PDG_OPT_ION_EXTRAPOLATION,
                   {"endpoint": 1, "midpoint": 0}[getattr(problem, "ion_extrap", "endpoint")])
    ctx.set_mesh(problem.mesh, problem.p)
    if getattr(problem, "elem_ptr", None) is not None:
        ctx.set_systems(problem.elem_ptr)
    ctx.assemble(problem.chi_m, problem.c_m, problem.dt, problem.eta0)
    ctx.set_ionic(problem.ionic)
    ctx.setup_preconditioner(problem.elem_sub, problem.elem_coarse, problem.coarse_q,
                             local_prec or problem.local_prec, coarse_prec or problem.coarse_prec)
    if bind and device is not None:
        ctx.bind_workspace()
    return ctx


def initial_state(ctx, problem):
    """(U^0, U^-1 = U^0, Y^0) on the context's device from the workload's
    per-element initial values (projected by the library)."""
    torch = ctx.torch
    dev = ctx.device
    n, nd = problem.n_elem, problem.nd
    with torch.cuda.stream(ctx.stream):
        u_vals = torch.tensor(np.asarray(problem.u0_elem, dtype=np.float64), device=dev)
        y_vals = torch.tensor(np.ascontiguousarray(problem.y0_elem, dtype=np.float64), device=dev)
        U = torch.empty(n * nd, dtype=torch.float64, device=dev)
        Y = torch.empty(y_vals.shape[0] * n * nd, dtype=torch.float64, device=dev)
        ctx.project_p0(u_vals.unsqueeze(0), U)
        ctx.project_p0(y_vals, Y)
        Up = U.clone()
    ctx.stream.synchronize()
    return U, Up, Y


class BatchSolver:
    """A batch of independent systems (``pdg_inputs.problems.Batch``): one
    context per polynomial degree holding that degree's systems, each context
    on its own stream (or all on the current stream), stepped together by
    pdg_step_batch."""

    def __init__(self, batch, device="cuda:0", options=None, separate_streams=True):
        import torch
        self.batch = batch
        self.ctxs, self.problems, self.members = [], [], []
        for p, (pr, idx) in sorted(batch.groups.items()):
            st = torch.cuda.Stream(device=device) if separate_streams else None
            self.ctxs.append(from_problem(pr, device=device, options=options, stream=st))
            self.problems.append(pr)
            self.members.append(idx)
        # system k -> (context index, system index inside the context)
        self.where = {}
        for ci, idx in enumerate(self.members):
            for s, k in enumerate(idx):
                self.where[k] = (ci, s)

    def set_option(self, option, value):
        for c in self.ctxs:
            c.set_option(option, value)

    def initial_state(self):
        st = [initial_state(c, pr) for c, pr in zip(self.ctxs, self.problems)]
        return [list(x) for x in zip(*st)]  # [U list, Up list, Y list]

    def step(self, U, Up, Y, tol, maxit):
        return step_batch(self.ctxs, U, Up, Y, tol, maxit)

    def system_slice(self, k):
        """(context index, dof slice) of system k inside its context's vectors."""
        ci, s = self.where[k]
        ep = self.problems[ci].elem_ptr
        nd = self.problems[ci].nd
        return ci, slice(int(ep[s]) * nd, int(ep[s + 1]) * nd)

    def system_info(self, k):
        ci, s = self.where[k]
        return self.ctxs[ci].system_info(s)
