"""Pins of the moving-interface inputs (Section 2.3): the agglomeration map of
the new time level and the L2 re-projection between the two agglomerated
spaces (xdg_inputs.moving), applied by the oracle as a rectangular block
operator (oracle.mg.block_operator).

* every cut part that is new at t1 or below the volume-fraction threshold is
  agglomerated (its t1 aggregate holds another part), and no aggregate mixes
  species;
* a polynomial of degree <= p in each species lies in both spaces, so its
  coefficients at t0 (L2 projection onto the t0 bases) are mapped by the
  re-projection exactly onto its coefficients at t1;
* cells that are uncut and not agglomerated at both times keep their
  coefficients (identity blocks);
* the re-projection does not increase the L2 norm beyond the t0 norm of the
  polynomial extension it projects (checked on the exact polynomial).
"""
import numpy as np
import pytest

from oracle import mg
from xdg_inputs.moving import moving_pair


@pytest.fixture(scope="module", params=[2, 3])
def pair(request):
    return moving_pair(n=8, p=request.param, c0=(0.01, -0.02, 0.015), shift=(0.3, 0.2, -0.1))


def _coeffs(pr, u, q):
    """L2 projection of u(X, s) onto the orthonormal level-0 bases of pr."""
    L0, g = pr.levels[0], pr.geom
    c = np.zeros((L0.n_rows, L0.np))
    for r in range(L0.n_rows):
        s = int(L0.species[r])
        for j in L0.pieces(r):
            X, W = g.volume_rule(j, s, q)
            if len(W):
                c[r] += (L0.bases[r].eval(X, grad=False) * W[:, None]).T @ u(X, s)
    return c.reshape(-1)


def test_new_and_small_parts_are_agglomerated(pair):
    pr0, pr1, _ = pair
    g0, g1, L1 = pr0.geom, pr1.geom, pr1.levels[0]
    pieces = np.diff(L1.piece_ptr)
    n_new = 0
    for j in g1.cut:
        for s in range(2):
            if not g1.present[j, s]:
                continue
            new = not g0.present[j, s]
            n_new += new
            if new or g1.frac[j, s] <= pr1.alpha:
                assert pieces[L1.part_of[2 * j + s]] >= 2, (j, s)
    assert n_new > 0            # the shift moves the interface across cells
    for r in range(L1.n_rows):
        s = int(L1.species[r])
        assert all(g1.present[j, s] for j in L1.pieces(r))


def test_polynomials_are_reprojected_exactly(pair):
    pr0, pr1, Pi = pair
    p = pr0.p
    rng = np.random.default_rng(7)
    coef = rng.uniform(-1, 1, (2, p + 1, p + 1, p + 1))

    def u(X, s):
        out = np.zeros(len(X))
        for a in range(p + 1):
            for b in range(p + 1 - a):
                for c in range(p + 1 - a - b):
                    out += coef[s, a, b, c] * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c
        return out

    q = p + 3
    c0, c1 = _coeffs(pr0, u, q), _coeffs(pr1, u, q)
    P = mg.block_operator(Pi["row_ptr"], Pi["col_idx"], Pi["val"], Pi["n_cols"])
    got = P @ c0
    err = np.linalg.norm(got - c1) / np.linalg.norm(c1)
    assert err <= 1e-12, err
    # the L2 norm of the t1 coefficients is the norm of u on the t1 domain
    assert np.linalg.norm(got) <= np.linalg.norm(c1) * (1 + 1e-12)


def test_unchanged_cells_keep_their_coefficients(pair):
    pr0, pr1, Pi = pair
    L0, L1 = pr0.levels[0], pr1.levels[0]
    Np = L1.np
    P = mg.block_operator(Pi["row_ptr"], Pi["col_idx"], Pi["val"], Pi["n_cols"]).tocsr()
    x0 = np.random.default_rng(8).uniform(-1, 1, L0.n_rows * Np)
    x1 = P @ x0
    g0, g1 = pr0.geom, pr1.geom
    checked = 0
    for r in range(L1.n_rows):
        cells = L1.pieces(r)
        j = int(cells[0])
        if len(cells) != 1 or j in g0.cut or j in g1.cut or not L1.standard[r]:
            continue
        s = int(L1.species[r])
        q = int(L0.part_of[2 * j + s])
        if len(L0.pieces(q)) != 1:
            continue
        assert np.array_equal(x1[r * Np:(r + 1) * Np], x0[q * Np:(q + 1) * Np])
        checked += 1
    assert checked > 100
