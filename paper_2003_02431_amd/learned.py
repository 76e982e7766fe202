"""Learned per-cell smoother: host orchestration over the C-ABI (training
pairs from plain solves, training, switching the smoother).  Every numerical
step runs in libxdg's kernels; this module only sequences the calls and
allocates the device buffers."""
import numpy as np

from . import binding as B

N_IN, N_OUT = 45, 40


def init_params(seed=0):
    """Seeded initial parameters: uniform fan-in/fan-out scaled hidden layers,
    zero biases and a zero output layer, so that the untrained network
    proposes no correction (the smoother starts as plain block Jacobi)."""
    g = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, N_IN), (64, 64)):
        lim = np.sqrt(6.0 / (rows + cols))
        parts += [g.uniform(-lim, lim, rows * cols), np.zeros(rows)]
    parts += [np.zeros(N_OUT * 64), np.zeros(N_OUT)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == B.xdg_mlp_param_count()
    return p


def plain_pairs(S, b, xs, iterates, cell_step=1, clip=0.0, restart_rtol=1e-300):
    """Training pairs from iterates of the handle's plain solver.

    For every k in `iterates`, x_k is the k-th iterate of the plain
    (block-Jacobi) solve of M x = b from x = 0; the pairs of x_k are taken on
    the cells k mod cell_step, k mod cell_step + cell_step, ...; targets
    longer than `clip` (> 0) are scaled to that length.  Returns
    float32 device tensors X [n, 45], T [n, 40].  The handle's smoother and
    stopping rule are restored afterwards."""
    torch = S.torch
    opt = S.opt
    h = S.h
    n_cells = S.n_cells
    counts = [len(range(k % cell_step, n_cells, cell_step)) for k in iterates]
    X = torch.empty((sum(counts), N_IN), dtype=torch.float32, device=S.device)
    T = torch.empty((sum(counts), N_OUT), dtype=torch.float32, device=S.device)
    B.xdg_set_smoother(h, B.XDG_JACOBI, S.guard)
    off = 0
    try:
        for k, cnt in zip(iterates, counts):
            x = S.vec(0)
            if k > 0:
                B.xdg_set_tolerance(h, restart_rtol, int(k))
                B.xdg_solve(h, b, x)
            n = B.xdg_learned_pairs(h, b, x, xs, k % cell_step, cell_step, X[off:off + cnt],
                                    T[off:off + cnt], clip)
            assert n == cnt
            off += cnt
    finally:
        B.xdg_set_tolerance(h, opt.rtol, opt.maxit)
        B.xdg_set_smoother(h, S.smoother, S.guard)
    return X, T


def train(S, X, T, steps, lr=1e-3, batch=None):
    """Adam on the handle's network; batch None = full batch.  Returns the
    loss history (numpy)."""
    return B.xdg_mlp_train(S.h, X, T, batch or X.shape[0], steps, lr)


def save_params(S, path):
    """Write the handle's network parameters to a .npy file (plain array, no
    pickling)."""
    np.save(path, B.xdg_mlp_get(S.h), allow_pickle=False)


def load_params(S, path):
    """Load parameters written by save_params into the handle (resets the
    Adam state)."""
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.size != B.xdg_mlp_param_count():
        raise ValueError(f"{path}: expected {B.xdg_mlp_param_count()} float32 parameters")
    B.xdg_mlp_set(S.h, p)
