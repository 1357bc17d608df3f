"""Pins of the oracle's optimiser-side prelude: the density filter and the
Heaviside projection (Sec. 3.1), their chain rule, and the constraint
functionals G1, G2, G3 (Sec. 2.6).

The filter is pinned by what a normalised symmetric cone filter must do
(constants and, away from the edges, linear fields pass unchanged; a point
source spreads symmetrically).  The projection is pinned by its fixed points
and limits.  Each chain rule is checked against central differences of the
oracle's own forward maps.  The constraints are pinned by closed forms.
"""
import math

import numpy as np
import pytest

from test_oracle_pins import small2d, small3d


def design_problem(d):
    if d == 2:
        return small2d(m=(13, 11, 1), xg_min=(9.0, 8.0, 0.0), xg_max=(11.0, 10.0, 0.0),
                       n=(24, 22, 1))
    return small3d(m=(9, 8, 7), n=(20, 20, 16), xg_min=(9.5, 9.5, 7.5),
                   xg_max=(10.5, 10.5, 8.5))


def grid_coords(p):
    m0, m1 = p.m[0], p.m[1]
    m2 = p.m[2] if p.d == 3 else 1
    k = np.arange(m0 * m1 * m2)
    return k % m0, (k // m0) % m1, k // (m0 * m1)


@pytest.mark.parametrize("d", [2, 3])
def test_filter_keeps_constant_and_interior_linear_fields(orc, d):
    """Normalised weights keep a constant field everywhere.  Symmetric
    weights keep a linear field wherever the stencil is whole.  beta = 0
    means no projection."""
    p = design_problem(d)
    R = 2.5
    x, y, z = grid_coords(p)
    c = orc.design_prelude(p, np.full(p.M, 0.37), R, 0.0, 0.5)
    assert np.allclose(c, 0.37, rtol=0, atol=1e-15)
    lin = 0.1 + 0.02 * x - 0.015 * y + (0.01 * z if d == 3 else 0.0)
    f = orc.design_prelude(p, lin, R, 0.0, 0.5)
    r = int(math.floor(R))
    inner = (x >= r) & (x < p.m[0] - r) & (y >= r) & (y < p.m[1] - r)
    if d == 3:
        inner &= (z >= r) & (z < p.m[2] - r)
    assert inner.sum() > 0
    assert np.allclose(f[inner], lin[inner], rtol=0, atol=1e-15)
    # at the edges the truncated stencil is one-sided: the field changes
    assert np.abs(f[~inner] - lin[~inner]).max() > 1e-4


def test_filter_point_source_is_symmetric(orc):
    """A unit value at an interior point spreads into a pattern symmetric
    under the reflections of the grid, and vanishes at distance >= R."""
    p = design_problem(2)
    R = 3.2
    g = np.zeros(p.M)
    c0, c1 = 6, 5
    g[c0 + p.m[0] * c1] = 1.0
    f = orc.design_prelude(p, g, R, 0.0, 0.5).reshape(p.m[1], p.m[0])
    for dx in range(-3, 4):
        for dy in range(-3, 4):
            v = f[c1 + dy, c0 + dx]
            assert abs(v - f[c1 - dy, c0 - dx]) < 1e-16
            assert abs(v - f[c1 + dy, c0 - dx]) < 1e-16
            if math.hypot(dx, dy) >= R:
                assert v == 0.0
            else:
                assert v > 0.0
    # weights fall off with distance
    assert f[c1, c0] > f[c1, c0 + 1] > f[c1, c0 + 2] > f[c1, c0 + 3]


def test_projection_fixed_points_and_limits(orc):
    """Eq. projection maps 0 -> 0 and 1 -> 1 for any beta and eta, eta to
    tanh(b eta) / (tanh(b eta) + tanh(b (1 - eta))), is nearly the identity
    for small beta, and nearly a step at eta for large beta."""
    p = design_problem(2)
    R = 0.5  # stencil of the point itself: the filter is the identity
    rng = np.random.default_rng(3)
    g = rng.uniform(0.0, 1.0, p.M)
    g[0], g[1], g[2] = 0.0, 1.0, 0.3
    for beta, eta in ((1.0, 0.5), (8.0, 0.3), (32.0, 0.6)):
        out = orc.design_prelude(p, g, R, beta, eta)
        assert abs(out[0]) < 1e-15 and abs(out[1] - 1.0) < 1e-15
        gg = g.copy()
        gg[2] = eta
        o2 = orc.design_prelude(p, gg, R, beta, eta)
        want = math.tanh(beta * eta) / (math.tanh(beta * eta) + math.tanh(beta * (1 - eta)))
        assert abs(o2[2] - want) < 1e-15
        assert np.all(np.diff(out[np.argsort(g)]) >= 0)  # monotone
    small = orc.design_prelude(p, g, R, 1e-4, 0.5)
    assert np.allclose(small, g, rtol=0, atol=1e-8)
    step = orc.design_prelude(p, g, R, 400.0, 0.5)
    far = np.abs(g - 0.5) > 0.05
    assert np.allclose(step[far], (g[far] > 0.5).astype(float), rtol=0, atol=1e-8)


@pytest.mark.parametrize("d", [2, 3])
def test_prelude_chain_rule_against_central_differences(orc, d):
    """The chain rule through projection and filter is the transpose of their
    Jacobian: <dJ/dphys, J_prelude v> equals <dJ/dgamma, v>, the left side
    by central differences of the forward prelude."""
    p = design_problem(d)
    rng = np.random.default_rng(10 + d)
    g = rng.uniform(0.1, 0.9, p.M)
    gbar = rng.standard_normal(p.M)
    R, beta, eta = 2.2, 6.0, 0.45
    back = orc.design_prelude_adjoint(p, g, R, beta, eta, gbar)
    for s in range(3):
        v = np.random.default_rng(20 + s).standard_normal(p.M)
        h = 1e-6
        jv = (orc.design_prelude(p, g + h * v, R, beta, eta)
              - orc.design_prelude(p, g - h * v, R, beta, eta)) / (2 * h)
        lhs, rhs = gbar @ jv, back @ v
        assert abs(lhs - rhs) < 1e-8 * max(abs(lhs), 1e-3), (lhs, rhs)


def test_volume_constraints_closed_form(orc):
    """G1 = mean(phys) / vmax - 1, G2 = mean(1 - phys) / vmax - 1, so
    G1 + G2 = 1 / vmax - 2 for any field; the gradients are +-1 / (vmax M)."""
    p = design_problem(2)
    chi = np.full((p.nt, 3), 0.5)
    psi = np.full(p.nt, 0.5)
    G, d1, d2, _ = orc.constraints(p, np.full(p.M, 0.6), chi, psi, 0.8, 1e-3, 16.0)
    assert abs(G[0] - (0.6 / 0.8 - 1)) < 1e-13 and abs(G[1] - (0.4 / 0.8 - 1)) < 1e-13
    rng = np.random.default_rng(5)
    G, d1, d2, _ = orc.constraints(p, rng.uniform(0, 1, p.M), chi, psi, 0.7, 1e-3, 16.0)
    assert abs(G[0] + G[1] - (1 / 0.7 - 2)) < 1e-14
    assert np.allclose(d1, 1 / (0.7 * p.M), rtol=1e-15, atol=0)
    assert np.allclose(d2, -1 / (0.7 * p.M), rtol=1e-15, atol=0)


def test_angular_velocity_constraint_closed_form_and_gradient(orc):
    """psi linear in time with the identity filter (R_w = 1) makes omega
    constant: omega = (th_max - th_min) b for psi_n = a + b n, so
    G3 = nt^(1/p) |omega| / omega_max - 1.  dG3/dpsi matches central
    differences of G3 for a random psi with a real filter."""
    p = design_problem(2).replace(nt=20, r_w=1)
    chi = np.full((p.nt, 3), 0.5)
    b = 0.01
    psi = 0.3 + b * np.arange(p.nt)
    om = (p.th_max - p.th_min) * b
    for pw in (2.0, 16.0):
        G, _, _, _ = orc.constraints(p, np.full(p.M, 0.5), chi, psi, 0.8, 2e-3, pw)
        assert abs(G[2] - (p.nt ** (1 / pw) * om / 2e-3 - 1)) < 1e-12
    p = p.replace(r_w=4)
    rng = np.random.default_rng(8)
    psi = rng.uniform(0.3, 0.7, p.nt)
    phys = np.full(p.M, 0.5)
    G, _, _, d3 = orc.constraints(p, phys, chi, psi, 0.8, 5e-3, 8.0)
    h = 1e-6
    for t in (0, 7, 19):
        pp, pm = psi.copy(), psi.copy()
        pp[t] += h
        pm[t] -= h
        fd = (orc.constraints(p, phys, chi, pp, 0.8, 5e-3, 8.0)[0][2]
              - orc.constraints(p, phys, chi, pm, 0.8, 5e-3, 8.0)[0][2]) / (2 * h)
        assert abs(fd - d3[t]) < 1e-7 * max(abs(fd), 1e-3), (t, fd, d3[t])


def test_angular_velocity_constraint_without_rotation(orc):
    """psi constant with the identity filter (R_w = 1): theta is constant,
    omega is exactly 0 at every step, G3 = -1, and the gradient (the p-norm
    has none at 0) is taken as 0."""
    p = design_problem(2).replace(nt=15, r_w=1)
    chi = np.full((p.nt, 3), 0.5)
    G, _, _, d3 = orc.constraints(p, np.full(p.M, 0.5), chi, np.full(p.nt, 0.4), 0.8, 1e-3, 16.0)
    assert G[2] == -1.0
    assert np.array_equal(d3, np.zeros(p.nt))
