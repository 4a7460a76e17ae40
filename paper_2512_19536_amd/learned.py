"""Learned initial guess (not part of the paper): a per-element network,
trained on trajectories the method itself generates, predicts U^(k+1) - U^k;
pdg_step_guess starts PCG from U^k + prediction wherever that lowers the
initial residual, and from U^k elsewhere.

Everything numeric runs in libpdg's kernels (feature and target kernels, BF16
matrix-core products, Adam, guess); this module only marshals arguments,
keeps the trajectory store (torch device memory) and holds the training loop.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import _lib
from ._lib import PdgMlpDesc, check_mlp
from .solver import _ptr, from_problem, initial_state

N_IN, WIDTH, N_OUT = 96, 256, 32


def row_block(n_elem):
    """Rows of one time step's elements in a batch (padded to 32)."""
    return (n_elem + 31) // 32 * 32


class Mlp:
    """A pdg_mlp with its workspace (a torch uint8 tensor)."""

    def __init__(self, nd, max_rows, device="cuda:0", stream=None, n_in=N_IN, width=WIDTH, n_out=N_OUT):
        import torch
        self.torch = torch
        self.lib = _lib.load()
        self.nd = nd
        self.device = device
        dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._m = ctypes.c_void_p()
        desc = PdgMlpDesc(n_in=n_in, width=width, n_out=n_out, n_out_valid=nd, max_rows=max_rows)
        check_mlp(None, self.lib.pdg_mlp_create(ctypes.byref(self._m), dev.index or 0,
                                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(desc)))
        self.desc = desc
        n, b = ctypes.c_int64(), ctypes.c_size_t()
        self._call("pdg_mlp_get_sizes", ctypes.byref(n), ctypes.byref(b))
        self.n_params = n.value
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self._call("pdg_mlp_bind_workspace", ctypes.c_void_p(base + (-base) % 256), ctypes.c_size_t(b.value))

    def _call(self, name, *args):
        check_mlp(self._m, getattr(self.lib, name)(self._m, *args))

    def close(self):
        if self._m:
            self.lib.pdg_mlp_destroy(self._m)
            self._m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- parameters ---------------------------------------------------------
    def init_params(self, seed):
        """He-uniform weights, zero biases (seeded numpy draw)."""
        rng = np.random.default_rng(seed)
        d = self.desc
        dims = [d.n_in, d.width, d.width, d.width, d.n_out]
        parts = []
        for k, n in zip(dims[:-1], dims[1:]):
            lim = np.sqrt(6.0 / k)
            parts += [rng.uniform(-lim, lim, n * k), np.zeros(n)]
        self.set_params(np.concatenate(parts))

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        self._call("pdg_mlp_set_params", _ptr(t), len(t))

    def get_params(self):
        t = np.zeros(self.n_params, dtype=np.float32)
        self._call("pdg_mlp_get_params", _ptr(t), len(t))
        return t

    def set_normalisation(self, xs, xk, ts, tk):
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (xs, xk, ts, tk)]
        self._call("pdg_mlp_set_normalisation", *[_ptr(v) for v in a])
        self.norm = a

    def set_batch(self, X_bits, T, w):
        X_bits = np.ascontiguousarray(X_bits, dtype=np.uint16)
        T = np.ascontiguousarray(T, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._call("pdg_mlp_set_batch", len(w), _ptr(X_bits), _ptr(T), _ptr(w))

    # ---- data ---------------------------------------------------------------
    def features(self, row0, n_elem, n_rows, u0, u1, u2, u3, ions, raw=None):
        self._call("pdg_mlp_features", int(row0), int(n_elem), int(n_rows), self.nd, _ptr(u0), _ptr(u1), _ptr(u2),
                   _ptr(u3), _ptr(ions), _ptr(raw))

    def targets(self, row0, n_elem, n_rows, u_next, u0, raw=None):
        self._call("pdg_mlp_targets", int(row0), int(n_elem), int(n_rows), self.nd, _ptr(u_next), _ptr(u0),
                   _ptr(raw))

    # ---- compute ------------------------------------------------------------
    def forward(self, rows, y_out=None):
        self._call("pdg_mlp_forward", int(rows), _ptr(y_out))

    def guess(self, row0, n_elem, u0, out):
        self._call("pdg_mlp_guess", int(row0), int(n_elem), self.nd, _ptr(u0), _ptr(out))

    def gradients(self, rows, n_valid):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        self._call("pdg_mlp_gradients", int(rows), int(n_valid), _ptr(g), ctypes.byref(loss))
        return loss.value, g

    def train_step(self, rows, n_valid, lr, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        loss = ctypes.c_double()
        self._call("pdg_mlp_train_step", int(rows), int(n_valid), ctypes.c_float(lr), ctypes.c_float(beta1),
                   ctypes.c_float(beta2), ctypes.c_float(eps), ctypes.byref(loss) if want_loss else None)
        return loss.value if want_loss else None


class Trajectory:
    """States of one run of the method: U^0..U^n and Y^0..Y^(n-1) (device)."""

    def __init__(self, problem, U, Y, iters, seconds):
        self.problem, self.U, self.Y, self.iters, self.seconds = problem, U, Y, iters, seconds

    @property
    def n_steps(self):
        return self.U.shape[0] - 1

    def history(self, k):
        """(u^k, u^(k-1), u^(k-2), u^(k-3), y^k), with u^(j) = u^0 for j < 0."""
        U = self.U
        return U[k], U[max(k - 1, 0)], U[max(k - 2, 0)], U[max(k - 3, 0)], self.Y[k]


def generate(problem, n_steps, device="cuda:0", options=None, log=None):
    """Runs the method for n_steps and stores its states on the device."""
    torch = __import__("torch")
    t0 = time.perf_counter()
    ctx = from_problem(problem, device=device, options=options)
    t_setup = time.perf_counter() - t0
    U, Up, Y = initial_state(ctx, problem)
    Us = torch.empty((n_steps + 1, U.numel()), dtype=torch.float64, device=device)
    Ys = torch.empty((n_steps, Y.numel()), dtype=torch.float64, device=device)
    Us[0].copy_(U)
    iters = []
    t0 = time.perf_counter()
    for k in range(n_steps):
        Ys[k].copy_(Y)
        info = ctx.step(U, Up, Y, None, problem.tol, problem.maxit)
        Us[k + 1].copy_(U)
        iters.append(info["iters"])
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    if log:
        log(f"[learned] {problem.name}: setup {t_setup:.1f} s, {n_steps} steps {t_run:.2f} s, "
            f"iters mean {np.mean(iters):.1f}")
    ctx.close()
    return Trajectory(problem, Us, Ys, iters, t_run)


def fit_normalisation(mlp, trajs, n_samples=64, seed=0):
    """Per-feature and per-target shift (mean) and scale (1 / std) from the
    raw values of a seeded sample of steps (computed by the library's feature
    and target kernels, reduced on the host)."""
    torch = mlp.torch
    rng = np.random.default_rng(seed)
    nd = mlp.nd
    n_in, n_out = mlp.desc.n_in, mlp.desc.n_out
    n_elem = trajs[0].problem.n_elem
    raw_x = torch.empty((n_elem, n_in), dtype=torch.float32, device=mlp.device)
    raw_t = torch.empty((n_elem, nd), dtype=torch.float32, device=mlp.device)
    xs, ts = [], []
    for _ in range(n_samples):
        tr = trajs[rng.integers(len(trajs))]
        k = int(rng.integers(tr.n_steps))
        mlp.features(0, n_elem, n_elem, *tr.history(k), raw=raw_x)
        mlp.targets(0, n_elem, n_elem, tr.U[k + 1], tr.U[k], raw=raw_t)
        mlp.stream.synchronize()
        xs.append(raw_x.cpu().numpy().astype(np.float64))
        ts.append(raw_t.cpu().numpy().astype(np.float64))
    X, T = np.concatenate(xs), np.concatenate(ts)

    def shift_scale(A, n):
        mu, sd = A.mean(0), A.std(0)
        floor = 1e-6 * max(float(sd.max()), 1e-30)
        sd = np.where(sd > floor, sd, 1.0)
        s = np.zeros(n, np.float32)
        k = np.ones(n, np.float32)
        s[:A.shape[1]] = mu
        k[:A.shape[1]] = 1.0 / sd
        return s, k

    x_shift, x_scale = shift_scale(X, n_in)
    t_shift, t_scale = shift_scale(T, n_out)
    mlp.set_normalisation(x_shift, x_scale, t_shift, t_scale)
    return x_shift, x_scale, t_shift, t_scale


def load_batch(mlp, trajs, pairs):
    """Features and targets of (trajectory, step) pairs into consecutive row
    blocks; returns (rows, valid rows)."""
    n_elem = trajs[0].problem.n_elem
    blk = row_block(n_elem)
    for b, (ti, k) in enumerate(pairs):
        tr = trajs[ti]
        mlp.features(b * blk, n_elem, blk, *tr.history(k))
        mlp.targets(b * blk, n_elem, blk, tr.U[k + 1], tr.U[k])
    return len(pairs) * blk, len(pairs) * n_elem


def train(mlp, trajs, epochs, batch_steps=4, lr=1e-3, lr_min=1e-5, seed=0, log=None):
    """Adam over all (trajectory, step) pairs in seeded random order, cosine
    learning-rate decay; returns per-epoch mean loss and the wall time."""
    rng = np.random.default_rng(seed)
    pairs = [(ti, k) for ti, tr in enumerate(trajs) for k in range(tr.n_steps)]
    n_batches = len(pairs) // batch_steps
    total = epochs * n_batches
    hist = []
    t0 = time.perf_counter()
    it = 0
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        losses = []
        for bi in range(n_batches):
            sel = [pairs[j] for j in order[bi * batch_steps:(bi + 1) * batch_steps]]
            rows, n_valid = load_batch(mlp, trajs, sel)
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * it / max(total - 1, 1)))
            want = bi == n_batches - 1 or bi % 16 == 0
            l = mlp.train_step(rows, n_valid, lr_t, want_loss=want)
            if want:
                losses.append(l)
            it += 1
        hist.append(float(np.mean(losses)))
        if log:
            log(f"[learned] epoch {ep}: loss {hist[-1]:.4e}")
    mlp.torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def evaluate(mlp, problem, n_steps, device="cuda:0", options=None, extrapolate_order=1, log=None):
    """Held-out evaluation along the method's own trajectory: at every step the
    same state is advanced three ways -- from U^k, from the extrapolated guess
    and from the learned guess -- and iterations and times are recorded; the
    trajectory continues with the plain result."""
    torch = mlp.torch
    opts = dict(options or {})
    # one Schwarz launch in eight timed: timing each launch would slow every
    # iteration by a few microseconds in all three variants
    opts[_lib.PDG_OPT_KERNEL_TIMING] = 8
    ctx = from_problem(problem, device=device, options=opts)
    U, Up, Y = initial_state(ctx, problem)
    n_elem, nd = problem.n_elem, problem.nd
    hist = [U.clone()]
    u, up, y = (torch.empty_like(v) for v in (U, Up, Y))
    g = torch.empty_like(U)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rec = {"plain": [], "extrap": [], "learned": [], "t_plain": [], "t_extrap": [], "t_learned": [],
           "used": [], "diff": []}

    def timed(fn):
        ev[0].record(ctx.stream)
        out = fn()
        ev[1].record(ctx.stream)
        ev[1].synchronize()
        return out, ev[0].elapsed_time(ev[1])

    for k in range(n_steps):
        h = [hist[max(k - j, 0)] for j in range(4)]
        # plain
        for a, b in ((u, U), (up, Up), (y, Y)):
            a.copy_(b)
        ctx.stream.synchronize()
        info, ms = timed(lambda: ctx.step(u, up, y, None, problem.tol, problem.maxit))
        rec["plain"].append(info["iters"])
        rec["t_plain"].append(ms)
        u_plain, y_plain = u.clone(), y.clone()
        # extrapolation
        for a, b in ((u, U), (up, Up), (y, Y)):
            a.copy_(b)
        ctx.stream.synchronize()

        def run_extrap():
            ctx.guess_extrapolate(h[0], h[1], h[2], extrapolate_order, g)
            return ctx.step_guess(u, up, y, None, g, problem.tol, problem.maxit)
        info, ms = timed(run_extrap)
        rec["extrap"].append(info["iters"])
        rec["t_extrap"].append(ms)
        # learned
        for a, b in ((u, U), (up, Up), (y, Y)):
            a.copy_(b)
        ctx.stream.synchronize()

        def run_learned():
            mlp.features(0, n_elem, row_block(n_elem), h[0], h[1], h[2], h[3], Y)
            mlp.forward(row_block(n_elem))
            mlp.guess(0, n_elem, h[0], g)
            return ctx.step_guess(u, up, y, None, g, problem.tol, problem.maxit)
        info, ms = timed(run_learned)
        rec["learned"].append(info["iters"])
        rec["t_learned"].append(ms)
        rec["used"].append(info["guess_used"])
        rec["diff"].append(float((u - u_plain).norm() / u_plain.norm()))
        # the trajectory continues with the plain result
        Up.copy_(U)
        U.copy_(u_plain)
        Y.copy_(y_plain)
        hist.append(U.clone())
        if log and (k % 20 == 0 or k == n_steps - 1):
            log(f"[learned] {problem.name} step {k}: iters plain {rec['plain'][-1]} extrap {rec['extrap'][-1]} "
                f"learned {rec['learned'][-1]} (guess used {rec['used'][-1]})")
    rec["schwarz_timing"] = ctx.kernel_timing()  # (launches, total ms, bytes per launch)
    ctx.close()
    return rec
