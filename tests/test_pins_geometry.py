"""Pins of the problem generator's geometry: paper Table tab:DOFs (Section 4),
closed-form moments of the cut-cell quadrature, and the divergence theorem
on every cut cell."""
import os

import numpy as np
import pytest

from xdg_inputs.geometry import Geometry
from xdg_inputs.levelset import Quadric
from xdg_inputs.problems import paper_sphere_fractions
from xdg_inputs.quadrature import partition_rule, surface_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tab_dofs.txt")


def _table():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if line:
            rows.append((int(line[0]), [None if v == "-" else int(v) for v in line[1:]]))
    return rows


@pytest.mark.parametrize("n,dofs", _table())
def test_tab_dofs(n, dofs):
    """DOFs = N_k * (agglomerated block rows) reproduce Table tab:DOFs exactly
    (sphere read as x^2+y^2+z^2 = 0.49, alpha = 0.1 for every row)."""
    _, rows = paper_sphere_fractions(n)
    for k, Nk, want in zip((2, 3, 5), (10, 20, 56), dofs):
        if want is not None:
            assert rows * Nk == want, (n, k)


@pytest.mark.parametrize("D,n,r,ctr", [(2, 16, 0.7, (0.0, 0.0)), (2, 13, 0.55, (0.031, -0.07)),
                                       (3, 8, 0.6, (0.02, -0.03, 0.045)), (3, 12, 0.7, (0, 0, 0))])
def test_sphere_moments(D, n, r, ctr):
    """Species volumes and interface measure equal the closed forms."""
    g = Geometry(D, n, Quadric.sphere(np.array(ctr, float), r), q_cut=12)
    if D == 2:
        vol, area = np.pi * r * r, 2 * np.pi * r
    else:
        vol, area = 4.0 / 3.0 * np.pi * r ** 3, 4 * np.pi * r * r
    assert abs(g.vol[:, 0].sum() - vol) <= 1e-13 * vol * 10
    assert abs(g.vol[:, 1].sum() - (2.0 ** D - vol)) <= 1e-12
    ia = sum(g.interface_area(j) for j in g.cut)
    assert abs(ia - area) <= 1e-12 * area


def test_ellipse_area_and_perimeter_free_check():
    """Ellipse area pi*a*b (2D) and ellipsoid volume 4/3 pi a b c (3D)."""
    g2 = Geometry(2, 10, Quadric.ellipsoid([0.01, -0.02], [0.6, 0.45]), q_cut=12)
    assert abs(g2.vol[:, 0].sum() - np.pi * 0.6 * 0.45) < 1e-13
    g3 = Geometry(3, 8, Quadric.ellipsoid([0, 0, 0], [0.62, 0.47, 0.55]), q_cut=12)
    assert abs(g3.vol[:, 0].sum() - 4 / 3 * np.pi * 0.62 * 0.47 * 0.55) < 1e-12


@pytest.mark.parametrize("D", [2, 3])
def test_divergence_theorem_per_cut_cell(D):
    """int_{K cap A} div F = oint F.n over the species-A faces and the
    interface (normal pointing out of A), for a polynomial field F."""
    phi = Quadric.sphere(np.array([0.03, -0.05, 0.02][:D]), 0.57)
    g = Geometry(D, 6, phi, q_cut=12)

    def F(X):
        return np.stack([X[:, 0] ** 3 + X[:, 1] * X[:, 0], X[:, 1] ** 2 * X[:, 0] + 1.0]
                        + ([X[:, 2] ** 3 - X[:, 0] * X[:, 1] * X[:, 2]] if D == 3 else []), axis=1)

    def divF(X):
        d = 3 * X[:, 0] ** 2 + X[:, 1] + 2 * X[:, 1] * X[:, 0]
        if D == 3:
            d = d + 3 * X[:, 2] ** 2 - X[:, 0] * X[:, 1]
        return d

    worst = 0.0
    for j in g.cut:
        P, W = g.volume_rule(j, 0, 4)
        lhs = W @ divF(P)
        rhs = 0.0
        for d, plane, t, sg in g.cell_faces(j):
            Pf, Wf = g.face_rule(d, plane, t, 0, 6)
            if len(Wf):
                rhs += sg * (Wf @ F(Pf)[:, d])
        Pi, Wi, Ni = g.interface_rule(j)
        rhs += Wi @ np.sum(F(Pi) * Ni, axis=1)
        worst = max(worst, abs(lhs - rhs))
    assert worst < 1e-13


def test_plane_cut_is_exact():
    """A planar cut of the unit square: area of {x + y < 0.3} in [0,1]^2."""
    phi = Quadric.plane([1.0, 1.0], 0.3)
    P, W, S = partition_rule([phi], np.zeros(2), np.ones(2), 4)
    assert abs(W[S[:, 0] < 0].sum() - 0.045) < 1e-16
    Ps, Ws, Ns = surface_rule(phi, np.zeros(2), np.ones(2), 4)
    assert abs(Ws.sum() - 0.3 * np.sqrt(2)) < 1e-15
    assert np.allclose(Ns, 1 / np.sqrt(2))
