"""GPU tests of the learned initial guess.

* The BF16 matrix-core network against the FP64 oracle network (oracle.mlp):
  forward outputs (hidden activations rounded to BF16 on both sides), loss and
  gradients of every parameter tensor (relative error <= 2e-2, cosine >= 0.999:
  the GPU keeps activations and back-propagated gradients in BF16), and two Adam
  steps (FP32 on the GPU, FP64 in the oracle, same gradients).
* Feature, target and guess kernels against plain numpy constructions.
* pdg_step_guess: a guess equal to U^k or a useless guess falls back and gives
  the plain step's bits; the converged solution as guess needs at most one
  iteration; extrapolated guesses reach the plain solution.
* End to end on a small cube: a network trained on the method's own
  trajectories lowers the mean iteration count on held-out steps.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import mlp as omlp  # noqa: E402
from paper_2512_19536_amd import _lib, learned, solver  # noqa: E402
from pdg_inputs import problems  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_layers(theta):
    layers = omlp.unpack(theta.astype(np.float64), learned.N_IN, learned.WIDTH, learned.N_OUT)
    return [(omlp.round_bf16(W), b) for W, b in layers]


def random_batch(rng, rows, nd, n_pad=7):
    X = rng.standard_normal((rows, learned.N_IN))
    X[:, 9 * nd:] = 0.0
    bits = omlp.bf16_bits(X)
    T = np.zeros((rows, learned.N_OUT), np.float32)
    T[:, :nd] = rng.standard_normal((rows, nd))
    w = np.ones(rows, np.float32)
    w[-n_pad:] = 0.0
    T[-n_pad:] = 0.0
    return bits, omlp.from_bf16_bits(bits), T, w


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def cosine(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.fixture
def net():
    m = learned.Mlp(nd=10, max_rows=1024, device=DEV)
    m.init_params(5)
    return m


def test_forward_matches_oracle(net):
    rng = np.random.default_rng(1)
    rows = 256
    bits, Xr, T, w = random_batch(rng, rows, 10)
    net.set_batch(bits, T, w)
    y = torch.empty((rows, learned.N_OUT), dtype=torch.float32, device=DEV)
    net.forward(rows, y)
    torch.cuda.synchronize()
    Yg = y.cpu().numpy().astype(np.float64)
    Yo, _ = omlp.forward(oracle_layers(net.get_params()), Xr, bf16_activations=True)
    err = rel(Yg, Yo)
    print(f"[mlp] forward rel err {err:.2e}", flush=True)
    assert err < 2e-3


def test_gradients_match_oracle(net):
    rng = np.random.default_rng(2)
    rows, nd = 512, 10
    bits, Xr, T, w = random_batch(rng, rows, nd)
    net.set_batch(bits, T, w)
    n_valid = int(np.count_nonzero(w))
    loss, g = net.gradients(rows, n_valid)
    theta = net.get_params()
    lo, go = omlp.loss_and_grads(oracle_layers(theta), Xr, T.astype(np.float64), w, nd, bf16_activations=True)
    print(f"[mlp] loss gpu {loss:.6e} oracle {lo:.6e}", flush=True)
    assert abs(loss - lo) <= 1e-3 * lo
    gl = omlp.unpack(g.astype(np.float64), learned.N_IN, learned.WIDTH, learned.N_OUT)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(gl, go)):
        for name, a, b in (("W", gW, oW), ("b", gb, ob)):
            if np.linalg.norm(b) == 0:
                assert np.linalg.norm(a) == 0
                continue
            e, c = rel(a, b), cosine(a, b)
            print(f"[mlp] layer {l} d{name}: rel {e:.2e} cos {c:.6f}", flush=True)
            assert e <= 2e-2 and c >= 0.999, (l, name)


def test_adam_steps_match_oracle(net):
    rng = np.random.default_rng(3)
    rows, nd = 256, 10
    bits, _, T, w = random_batch(rng, rows, nd)
    net.set_batch(bits, T, w)
    n_valid = int(np.count_nonzero(w))
    th = net.get_params().astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in (1, 2):
        _, g = net.gradients(rows, n_valid)
        net.train_step(rows, n_valid, lr=1e-3)
        th, m, v = omlp.adam(th, g.astype(np.float64), m, v, t, lr=1e-3)
        got = net.get_params().astype(np.float64)
        err = np.abs(got - th).max()
        print(f"[mlp] adam step {t}: max abs err {err:.2e}", flush=True)
        assert err <= 1e-6 * np.abs(th).max() + 1e-8
        th = got  # continue from the GPU's FP32 parameters


def test_feature_target_guess_kernels(net):
    rng = np.random.default_rng(4)
    n_elem, nd = 77, 10
    blk = learned.row_block(n_elem)
    us = [rng.standard_normal(n_elem * nd) * 10 - 70 for _ in range(5)]
    ions = rng.standard_normal(5 * n_elem * nd)
    T_ = lambda a: torch.tensor(a, device=DEV)  # noqa: E731
    u0, u1, u2, u3, un = (T_(a) for a in us)
    y = T_(ions)
    raw = torch.empty((n_elem, learned.N_IN), dtype=torch.float32, device=DEV)
    net.features(0, n_elem, blk, u0, u1, u2, u3, y, raw=raw)
    rawt = torch.empty((n_elem, nd), dtype=torch.float32, device=DEV)
    net.targets(0, n_elem, blk, un, u0, raw=rawt)
    torch.cuda.synchronize()
    U = [a.reshape(n_elem, nd) for a in us]
    F = np.zeros((n_elem, learned.N_IN))
    F[:, :9 * nd] = np.concatenate([U[0], U[0] - U[1], U[1] - U[2], U[2] - U[3]]
                                   + [ions.reshape(5, n_elem, nd)[k] for k in range(5)], axis=1)
    assert np.array_equal(raw.cpu().numpy(), F.astype(np.float32))
    assert np.array_equal(rawt.cpu().numpy(), (U[4] - U[0]).astype(np.float32))
    # normalised features and targets equal a host-built batch, bit for bit
    xs = rng.standard_normal(learned.N_IN).astype(np.float32)
    xk = (0.5 + rng.random(learned.N_IN)).astype(np.float32)
    ts = rng.standard_normal(learned.N_OUT).astype(np.float32)
    tk = (0.5 + rng.random(learned.N_OUT)).astype(np.float32)
    net.set_normalisation(xs, xk, ts, tk)
    net.features(0, n_elem, blk, u0, u1, u2, u3, y)
    net.targets(0, n_elem, blk, un, u0)
    l1, g1 = net.gradients(blk, n_elem)
    ya = torch.empty((blk, learned.N_OUT), dtype=torch.float32, device=DEV)
    net.forward(blk, ya)
    Xh = np.zeros((blk, learned.N_IN))
    Xh[:n_elem] = ((F - xs.astype(np.float64)) * xk.astype(np.float64)).astype(np.float32)
    Xh[:n_elem, 9 * nd:] = 0.0
    Th = np.zeros((blk, learned.N_OUT), np.float32)
    Th[:n_elem, :nd] = ((U[4] - U[0] - ts[:nd].astype(np.float64)) * tk[:nd].astype(np.float64)).astype(np.float32)
    wh = np.zeros(blk, np.float32)
    wh[:n_elem] = 1.0
    net.set_batch(omlp.bf16_bits(Xh), Th, wh)
    l2, g2 = net.gradients(blk, n_elem)
    yb = torch.empty_like(ya)
    net.forward(blk, yb)
    torch.cuda.synchronize()
    assert np.array_equal(ya.cpu().numpy(), yb.cpu().numpy())
    assert l1 == l2 and np.array_equal(g1, g2)
    # guess = u0 + de-normalised prediction
    gs = torch.empty_like(u0)
    net.guess(0, n_elem, u0, gs)
    torch.cuda.synchronize()
    Y = ya.cpu().numpy()[:n_elem, :nd].astype(np.float64)
    ref = U[0] + Y / tk[:nd].astype(np.float64) + ts[:nd].astype(np.float64)
    assert np.abs(gs.cpu().numpy().reshape(n_elem, nd) - ref).max() <= 1e-13 * np.abs(ref).max()


def _state_after(ctx, pr, n):
    U, Up, Y = solver.initial_state(ctx, pr)
    for _ in range(n):
        ctx.step(U, Up, Y, None, pr.tol, pr.maxit)
    return U, Up, Y


def test_step_guess_fallback_and_use():
    pr = problems.learned_small(n_grid=8)
    ctx = solver.from_problem(pr, device=DEV)
    U, Up, Y = _state_after(ctx, pr, 3)
    Uh = [U.clone(), Up.clone()]

    def run(guess=None):
        u, up, y = U.clone(), Up.clone(), Y.clone()
        if guess is None:
            info = ctx.step(u, up, y, None, pr.tol, pr.maxit)
        else:
            info = ctx.step_guess(u, up, y, None, guess, pr.tol, pr.maxit)
        torch.cuda.synchronize()
        return info, u.cpu().numpy(), up.cpu().numpy(), y.cpu().numpy()

    i0, u0, up0, y0 = run()
    assert i0["guess_used"] == -1
    for g in (U.clone(), U + 1e3 * torch.randn_like(U)):
        i1, u1, up1, y1 = run(g)
        assert i1["guess_used"] == 0
        assert i1["iters"] == i0["iters"]
        assert np.array_equal(u1, u0) and np.array_equal(up1, up0) and np.array_equal(y1, y0)
    i2, u2, _, _ = run(torch.tensor(u0, device=DEV))
    assert i2["guess_used"] == 1 and i2["iters"] <= 1
    assert rel(u2, u0) < 1e-12
    for order in (1, 2):
        g = torch.empty_like(U)
        u_1 = Uh[1]
        ctx.guess_extrapolate(Uh[0], u_1, u_1, order, g)
        i3, u3, _, _ = run(g)
        print(f"[guess] extrapolation order {order}: iters {i3['iters']} (plain {i0['iters']}), "
              f"used {i3['guess_used']}", flush=True)
        assert rel(u3, u0) < 1e-8


def test_trained_network_lowers_iterations():
    base = problems.learned_small(n_grid=12)
    train_p = [problems.trajectory_problem(base, s) for s in range(300, 306)]
    test_p = problems.trajectory_problem(base, 400)
    n_steps = 40
    trajs = [learned.generate(q, n_steps, device=DEV) for q in train_p]
    n_elem = base.n_elem
    net = learned.Mlp(nd=base.nd, max_rows=4 * learned.row_block(n_elem), device=DEV)
    learned.fit_normalisation(net, trajs, n_samples=32, seed=0)
    net.init_params(0)
    hist, secs = learned.train(net, trajs, epochs=40, batch_steps=4, lr=2e-3, seed=0)
    print(f"[learned] training: loss {hist[0]:.3e} -> {hist[-1]:.3e} in {secs:.1f} s", flush=True)
    assert hist[-1] < 0.5 * hist[0]
    rec = learned.evaluate(net, test_p, 30, device=DEV)
    mp, me, ml = (float(np.mean(rec[k])) for k in ("plain", "extrap", "learned"))
    print(f"[learned] held-out mean iters: plain {mp:.2f} extrapolated {me:.2f} learned {ml:.2f}; "
          f"guess used {np.mean(np.array(rec['used']) > 0):.2f}; max rel diff {max(rec['diff']):.1e}", flush=True)
    assert max(rec["diff"]) < 1e-8
    assert ml < mp
    # and against the non-learned guess (linear extrapolation of the last two
    # iterates, used wherever it lowers the initial residual)
    assert ml < me
