"""GPU parity of the learned per-cell smoother against the FP64 oracle
(oracle.mlp, oracle.learned): network forward, training gradient and Adam
steps, training pairs, the learned V-cycle, the two fallbacks, and what the
trained network gains over plain block Jacobi inside FGMRES.

Tolerances (FP32 network against the FP64 oracle):
  * forward: a K-term FP32 dot product errs by at most gamma_K sum |w h|
    with gamma_K = K u32 (u32 = 2^-24); K <= 64 per layer, three layers:
    1e-5 relative to the output scale covers it with margin;
  * gradient: the same bound through the backward pass, 1e-5 normwise
    relative (the network's gradient pin);
  * pairs: the features and targets are FP64 values rounded once to FP32:
    relative 2^-23 plus the FP64 summation-order differences;
  * learned V-cycle: the FP32 network output enters scaled by the Jacobi
    step norm: relative 1e-5;
  * bf16 learned V-cycle against the oracle's bf16 emulation: relative 5e-6
    and at most a tenth of its distance from the FP64 network.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


_STATE = {}


def _problem(seed, n=16):
    key = ("prob", seed, n)
    if key not in _STATE:
        from xdg_inputs import features, problems
        _log(f"[gpu-learned] generating c4 seed={seed} n={n} p=3")
        pr = problems.c4(seed=seed, n=n, p=3, nrhs=1)
        pr.b = np.asarray(pr.b).reshape(-1)
        rs, g = features.cell_features(pr)
        _STATE[key] = (pr, rs, g)
    return _STATE[key]


def _solver(seed, torch, **kw):
    from paper_2003_02431_amd import binding as B
    pr, rs, g = _problem(seed)
    # rtol 1e-9: the solution error against x* must be <= 1e-8
    o = dict(krylov=B.XDG_FGMRES, restart=30, rtol=1e-9, maxit=300, smoother=B.XDG_LEARNED)
    o.update(kw)
    S = B.Solver(pr, B.options(**o))
    B.xdg_set_cell_features(S.h, rs, g)
    return pr, rs, g, S


def _params(seed, out_scale):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    th = mlp.init_params(rng) + 0.02 * rng.standard_normal(mlp.N_PARAM)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    W3 *= out_scale
    b3 *= out_scale
    return th.astype(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev32(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def net(torch):
    """A handle whose network the kernel-level tests drive."""
    return _solver(41, torch)[3]


@pytest.mark.parametrize("n", [1, 5, 1000, 4099])
def test_forward(n, torch, net):
    from oracle import mlp
    from paper_2003_02431_amd import binding as B
    th = _params(1, 1.0)
    B.xdg_mlp_set(net.h, th)
    X = np.random.default_rng(n).standard_normal((n, 45)).astype(np.float32).astype(np.float64)
    Y = torch.empty((n, 40), dtype=torch.float32, device="cuda")
    B.xdg_mlp_forward(net.h, _dev32(torch, X), Y)
    ref, _ = mlp.forward(th, X)
    y = Y.cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
    _log(f"  forward n={n}: max err / max |y| = {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("n", [1, 257, 3000])
def test_gradient(n, torch, net):
    from oracle import mlp
    from paper_2003_02431_amd import binding as B
    th = _params(2, 0.5)
    B.xdg_mlp_set(net.h, th)
    rng = np.random.default_rng(100 + n)
    X = rng.standard_normal((n, 45)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((n, 40)).astype(np.float32).astype(np.float64)
    G = torch.empty(B.xdg_mlp_param_count(), dtype=torch.float32, device="cuda")
    loss = B.xdg_mlp_gradient(net.h, _dev32(torch, X), _dev32(torch, T), G)
    g = G.cpu().numpy().astype(np.float64)
    gref = mlp.grad(th, X, T)
    lref = mlp.loss(th, X, T)
    eg, el = _rel(g, gref), abs(loss - lref) / lref
    _log(f"  gradient n={n}: rel err {eg:.2e}, loss rel err {el:.2e}")
    assert eg <= 1e-5 and el <= 1e-5
    # reproducible: the same call gives the same bits
    G2 = torch.empty_like(G)
    assert B.xdg_mlp_gradient(net.h, _dev32(torch, X), _dev32(torch, T), G2) == loss
    assert torch.equal(G, G2)


def test_adam_steps(torch, net):
    """Three full-batch Adam steps against oracle.mlp.adam_step in FP64.  The
    first steps move each weight by about lr * sign(g): entries whose
    gradient is large enough for FP32 to get its sign right must agree to a
    small fraction of lr, all others stay within Adam's bound (|step| <= lr
    per step, up to eps)."""
    from oracle import mlp
    from paper_2003_02431_amd import binding as B
    th0 = _params(3, 0.5)
    B.xdg_mlp_set(net.h, th0)
    rng = np.random.default_rng(7)
    n, lr, steps = 512, 1e-3, 3
    X = rng.standard_normal((n, 45)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((n, 40)).astype(np.float32).astype(np.float64)
    hist = B.xdg_mlp_train(net.h, _dev32(torch, X), _dev32(torch, T), n, steps, lr)
    got = B.xdg_mlp_get(net.h).astype(np.float64)
    th, m, v = th0.copy(), np.zeros_like(th0), np.zeros_like(th0)
    gmin = np.full_like(th0, np.inf)
    for t in range(1, steps + 1):
        g = mlp.grad(th, X, T)
        assert abs(hist[t - 1] - mlp.loss(th, X, T)) <= 1e-5 * mlp.loss(th, X, T)
        gmin = np.minimum(gmin, np.abs(g))
        th, m, v = mlp.adam_step(th, g, m, v, t, lr)
    d = np.abs(got - th)
    sure = gmin > 1e-3 * np.max(gmin)
    _log(f"  adam: max |dtheta| on well-determined entries {d[sure].max():.2e} "
         f"({sure.sum()} of {sure.size}), overall {d.max():.2e}")
    assert d[sure].max() <= 1e-2 * lr
    assert d.max() <= 2 * steps * lr


def test_pairs(torch):
    from oracle import learned, mg
    from paper_2003_02431_amd import binding as B
    pr, rs, g, S = _solver(41, torch)
    H = mg.hierarchy_of(pr)
    rng = np.random.default_rng(5)
    L = pr.b.size
    xk, xs = rng.uniform(-1, 1, L), rng.uniform(-1, 1, L)
    for cell0, step, clip in ((0, 1, 0.0), (2, 7, 0.0), (1, 3, 0.5)):
        Xr, Tr = learned.pairs(H, rs, g.astype(np.float64), pr.b, xk, xs, clip)
        sel = np.arange(cell0, S.n_cells, step)
        X = torch.empty((sel.size, 45), dtype=torch.float32, device="cuda")
        T = torch.empty((sel.size, 40), dtype=torch.float32, device="cuda")
        n = B.xdg_learned_pairs(S.h, S.vec(0, pr.b), S.vec(0, xk), S.vec(0, xs), cell0, step, X, T,
                                clip)
        assert n == sel.size
        x, t = X.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
        # relative per entry, with a floor at 1e-9 of the sample's norm for
        # entries that cancel (FP64 summation order differs)
        def err(a, ref):
            floor = 1e-9 * np.linalg.norm(ref, axis=1, keepdims=True) + 1e-300
            return float(np.max(np.abs(a - ref) / (np.abs(ref) + floor)))
        ex, et = err(x, Xr[sel]), err(t, Tr[sel])
        _log(f"  pairs cell0={cell0} step={step} clip={clip}: n={n} max rel err X {ex:.2e} "
             f"T {et:.2e}")
        assert ex <= 2.5e-7 and et <= 2.5e-7
    S.close()


def test_learned_vcycle_and_guard(torch):
    from oracle import learned, mg
    from paper_2003_02431_amd import binding as B
    pr, rs, g, S = _solver(41, torch)
    H = mg.hierarchy_of(pr)
    r = np.random.default_rng(8).uniform(-1, 1, pr.b.size)
    th = _params(4, 0.05)
    B.xdg_mlp_set(S.h, th)
    # every cell's proposal inside the guard, far from it
    F, _, _ = learned.features(H, rs, g.astype(np.float64), r)
    from oracle import mlp
    ny = np.linalg.norm(mlp.forward(th, F)[0], axis=1)
    assert ny.max() < 0.5 * S.guard
    z = S.vec(0)
    g0 = B.xdg_learned_stats(S.h)[0]
    B.xdg_vcycle(S.h, S.vec(0, r), z)
    ref = learned.vcycle(H, rs, g.astype(np.float64), th, r, S.guard)
    plain = H.vcycle(r)
    e, d = _rel(z.cpu().numpy(), ref), _rel(ref, plain)
    _log(f"  learned V-cycle rel err {e:.2e} (learned vs plain differ by {d:.2e})")
    assert e <= 1e-5 and d >= 1e-3
    assert B.xdg_learned_stats(S.h)[0] == g0
    # oversized proposals: every cell keeps the plain step -> the plain V-cycle
    B.xdg_mlp_set(S.h, _params(4, 1e4))
    B.xdg_vcycle(S.h, S.vec(0, r), z)
    e = _rel(z.cpu().numpy(), plain)
    guarded = B.xdg_learned_stats(S.h)[0] - g0
    _log(f"  all-guarded V-cycle vs plain rel err {e:.2e}, guarded cells {guarded}")
    assert e <= 1e-11 and guarded == S.n_cells
    S.close()


def test_bf16_learned_vcycle(torch):
    """The bf16 matrix-core network inside the V-cycle against the oracle's
    bf16 emulation (bf16 operands, FP64 sums): both round the same values to
    bf16, so they differ only where an FP32 sum lands on the other side of a
    bf16 rounding boundary -- far below the distance of either from the
    FP64 network (about 5e-5 here).  A parameter change repacks the weights:
    oversized proposals then give the plain V-cycle with every cell guarded."""
    from oracle import learned, mg
    from paper_2003_02431_amd import binding as B
    pr, rs, g, S = _solver(41, torch, smoother=B.XDG_LEARNED_BF16)
    H = mg.hierarchy_of(pr)
    r = np.random.default_rng(8).uniform(-1, 1, pr.b.size)
    th = _params(4, 0.05)
    B.xdg_mlp_set(S.h, th)
    z = S.vec(0)
    g0 = B.xdg_learned_stats(S.h)[0]
    B.xdg_vcycle(S.h, S.vec(0, r), z)
    G = g.astype(np.float64)
    ref = learned.vcycle(H, rs, G, th, r, S.guard, bf16=True)
    ref64 = learned.vcycle(H, rs, G, th, r, S.guard)
    e, d = _rel(z.cpu().numpy(), ref), _rel(ref, ref64)
    _log(f"  bf16 learned V-cycle rel err {e:.2e} (bf16 vs FP64 network {d:.2e})")
    assert e <= 5e-6 and d >= 1e-5 and e <= 0.1 * d
    assert B.xdg_learned_stats(S.h)[0] == g0
    plain = H.vcycle(r)
    B.xdg_mlp_set(S.h, _params(4, 1e4))
    B.xdg_vcycle(S.h, S.vec(0, r), z)
    e = _rel(z.cpu().numpy(), plain)
    guarded = B.xdg_learned_stats(S.h)[0] - g0
    _log(f"  bf16 all-guarded V-cycle vs plain rel err {e:.2e}, guarded cells {guarded}")
    assert e <= 1e-11 and guarded == S.n_cells
    S.close()


def test_ragged_tail_learned_vcycle(torch):
    """4,068 cells (not a multiple of the 16-cell bf16 batch or the 8-cell
    FP32 chunk): a residual supported on the last 8 cells only, so that the
    V-cycle differs from the plain one only through the tail's corrections;
    both networks against the oracle."""
    from oracle import learned, mg
    from paper_2003_02431_amd import binding as B
    pr, rs, g, S = _solver(47, torch)
    assert S.n_cells % 16 == 4 and S.n_cells % 8 == 4
    H = mg.hierarchy_of(pr)
    cp = np.asarray(pr.cell_ptr)
    r = np.zeros(pr.b.size)
    tail = slice(cp[-9] * pr.np, cp[-1] * pr.np)
    r[tail] = np.random.default_rng(9).uniform(-1, 1, r[tail].size)
    th = _params(4, 0.05)
    B.xdg_mlp_set(S.h, th)
    G = g.astype(np.float64)
    plain = H.vcycle(r)
    for sm, bf, tol in ((B.XDG_LEARNED, False, 1e-5), (B.XDG_LEARNED_BF16, True, 5e-6)):
        S.set_smoother(sm)
        z = S.vec(0)
        g0 = B.xdg_learned_stats(S.h)[0]
        B.xdg_vcycle(S.h, S.vec(0, r), z)
        ref = learned.vcycle(H, rs, G, th, r, S.guard, bf16=bf)
        e, d = _rel(z.cpu().numpy(), ref), _rel(ref, plain)
        _log(f"  ragged tail ({S.n_cells} cells), smoother {sm}: rel err {e:.2e} "
             f"(learned vs plain {d:.2e})")
        assert e <= tol and d >= 1e-3 and B.xdg_learned_stats(S.h)[0] == g0
    S.close()


def _xstar(pr):
    from oracle import mg
    H = mg.hierarchy_of(pr)
    return mg.pcg(H.A[0], pr.b, H.vcycle, rtol=1e-13, maxit=1000)[0]


def test_nan_weights_fall_back_to_plain(torch):
    from paper_2003_02431_amd import binding as B
    pr, rs, g, S = _solver(41, torch)
    b = S.vec(0, pr.b)
    S.set_smoother(B.XDG_JACOBI)
    x0 = S.vec(0)
    _, it0, _, _ = B.xdg_solve(S.h, b, x0)
    th = _params(5, 1.0)
    th[7] = np.nan
    B.xdg_mlp_set(S.h, th)
    S.set_smoother(B.XDG_LEARNED)
    x1 = S.vec(0)
    rc, it1, fr, _ = B.xdg_solve(S.h, b, x1)
    guarded, fb = B.xdg_learned_stats(S.h)
    e = _rel(x1.cpu().numpy(), x0.cpu().numpy())
    _log(f"  NaN weights: plain it={it0}, learned it={it1}, guarded cells={guarded}, "
         f"x diff {e:.1e}")
    assert rc == 0 and it1 == it0 and guarded >= S.n_cells and e <= 1e-10
    S.close()


def test_stall_fallback(torch):
    """Corrupted weights whose proposals pass a (disabled) guard: the V-cycle
    output is noise, FGMRES's residual-decrease test switches the network off
    and the solve still reaches the oracle's solution."""
    from paper_2003_02431_amd import binding as B
    pr, rs, g, S = _solver(41, torch)
    th = _params(6, 0.0)
    from oracle import mlp
    W3 = mlp.unpack(th)[4]
    W3[:] = np.random.default_rng(0).standard_normal(W3.shape) * 3.0
    B.xdg_mlp_set(S.h, th.astype(np.float32))
    S.set_smoother(B.XDG_LEARNED, guard=1e30)
    x = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, pr.b), x)
    guarded, fb = B.xdg_learned_stats(S.h)
    err = _rel(x.cpu().numpy(), _xstar(pr))
    _log(f"  random-output network: it={it} fallbacks={fb} guarded={guarded} err={err:.2e}")
    assert rc == 0 and fb >= 1 and err <= 1e-8
    S.close()


CLIP, GUARD = 0.25, 0.5


def test_training_and_gain(torch):
    """Pairs from plain solves on two training interfaces (targets clipped to
    norm CLIP), full-batch Adam on the GPU, then FGMRES with and without the
    network (guard GUARD) on a third interface: both must reach 1e-8 relative
    error against the oracle's x*; iterations and times are reported, and the
    held-out loss must fall below that of plain Jacobi (the zero network)."""
    from paper_2003_02431_amd import binding as B, learned as LS
    Xs, Ts = [], []
    for seed in (31, 32):
        pr, rs, g, S = _solver(seed, torch, smoother=B.XDG_JACOBI)
        xs = S.vec(0, _xstar(pr))
        X, T = LS.plain_pairs(S, S.vec(0, pr.b), xs, iterates=range(0, 12), clip=CLIP)
        Xs.append(X)
        Ts.append(T)
        S.close()
    X, T = torch.cat(Xs), torch.cat(Ts)
    pr, rs, g, S = _solver(33, torch)
    B.xdg_mlp_set(S.h, LS.init_params(0))
    xs_np = _xstar(pr)
    xs = S.vec(0, xs_np)
    Xv, Tv = LS.plain_pairs(S, S.vec(0, pr.b), xs, iterates=range(0, 12, 3), clip=CLIP)
    G = torch.empty(B.xdg_mlp_param_count(), dtype=torch.float32, device="cuda")
    l0 = B.xdg_mlp_gradient(S.h, Xv, Tv, G)
    t0 = time.time()
    hist = LS.train(S, X, T, steps=600, lr=1e-3)
    torch.cuda.synchronize()
    ttrain = time.time() - t0
    l1 = B.xdg_mlp_gradient(S.h, Xv, Tv, G)
    _log(f"  training: {X.shape[0]} pairs, loss {hist[0]:.4f} -> {hist[-1]:.4f} in {ttrain:.2f}s; "
         f"held-out loss {l0:.4f} (plain Jacobi) -> {l1:.4f}")
    assert hist[-1] < hist[0] and l1 < l0
    S.set_smoother(B.XDG_LEARNED, guard=GUARD)
    b = S.vec(0, pr.b)
    res = {}
    for name, sm in (("plain", B.XDG_JACOBI), ("learned", B.XDG_LEARNED),
                     ("learned_bf16", B.XDG_LEARNED_BF16)):
        S.set_smoother(sm)
        x = S.vec(0)
        torch.cuda.synchronize()
        t = time.time()
        rc, it, fr, _ = B.xdg_solve(S.h, b, x)
        dt = time.time() - t
        err = _rel(x.cpu().numpy(), xs_np)
        res[name] = (it, dt, err)
        _log(f"  {name}: rc={rc} it={it} time={dt * 1e3:.1f} ms relres={fr:.2e} err={err:.2e}")
        assert rc == 0 and err <= 1e-8
    # checkpoint: the trained parameters survive a save / load round trip
    import tempfile, os
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "mlp.npy")
        before = B.xdg_mlp_get(S.h)
        LS.save_params(S, f)
        B.xdg_mlp_set(S.h, LS.init_params(1))
        LS.load_params(S, f)
        assert np.array_equal(B.xdg_mlp_get(S.h), before)
    gd, fb = B.xdg_learned_stats(S.h)
    _log(f"  gain: iterations {res['plain'][0]} -> {res['learned'][0]}, time "
         f"{res['plain'][1] * 1e3:.1f} -> {res['learned'][1] * 1e3:.1f} ms, guarded cells {gd}, "
         f"solver fallbacks {fb}")
    S.close()
