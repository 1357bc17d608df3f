"""Pins of the oracle's second objective J2 (Eq. objective2, Sec. 2.6): the
weighted propulsive force, drag work and torque work on the body, from the
force density kappa_ref (u_ref - u_S_ref) at the design points.

- A body translating with a uniform flow feels no force: J2 and its shape
  gradient vanish (the kernel is a partition of unity, so u_ref = u = u_S).
- The reverse sweep's J2 terms (the seed on the fluid velocity and the
  direct dependence on kappa_ref, position, velocity, angle and angular
  velocity) give the derivatives complex step takes through the whole
  forward march.
- Over a single step the ALKS, fed the same J2 terms, equals the exact
  adjoint.
"""
import math

import numpy as np
import pytest

from test_oracle_pins import rand_inputs, rest_state, small2d


def oar(**kw):
    base = dict(objective=1, w_d=0.3, w_t=0.5, l_m=4.0, phi=0.0)
    base.update(kw)
    return small2d(**base)


def test_j2_vanishes_for_a_body_moving_with_the_flow(orc):
    U = np.array([0.03, -0.02])
    p = oar(bc=(0, 0, 0), n=(24, 22, 1), m=(5, 5, 1), margin=4, nt=8, r_t=1, r_w=1,
            xg_min=(0.0, 0.0, 0.0), xg_max=(40.0, 40.0, 0.0))
    t = np.arange(p.nt) + 1
    chi = np.zeros((p.nt, 3))
    chi[:, 0] = (10.0 + U[0] * t) / 40.0
    chi[:, 1] = (11.0 + U[1] * t) / 40.0
    psi = np.full(p.nt, 0.5)
    gamma = np.random.default_rng(5).uniform(0.1, 0.9, size=p.M)
    s0 = rest_state(p, u=(U[0], U[1], 0))
    f = orc.forward(p, gamma, chi, psi, state0=s0)
    assert abs(f["J"]) < 1e-15 and abs(f["E"]) < 1e-15 and abs(f["V"]) < 1e-15
    a = orc.adjoint(p, gamma, chi, psi, state0=s0)
    assert np.abs(a["dgamma"]).max() < 1e-13


def test_j2_parts_add_up(orc):
    """J_out = (J2, F_L, F_D); J2 = F_L + w_D F_D + w_T T, and with both
    weights 0 it is F_L alone."""
    p = oar()
    gamma, chi, psi = rand_inputs(p, 3)
    f = orc.forward(p, gamma, chi, psi)
    f0 = orc.forward(p.replace(w_d=0.0, w_t=0.0), gamma, chi, psi)
    fd = orc.forward(p.replace(w_t=0.0), gamma, chi, psi)
    assert abs(f0["J"] - f0["E"]) < 1e-18
    assert abs(f0["E"] - f["E"]) < 1e-18 and abs(f0["V"] - f["V"]) < 1e-18
    assert abs(fd["J"] - (f["E"] + p.w_d * f["V"])) < 1e-15 * max(abs(fd["J"]), 1e-12)
    assert abs(f["J"]) > 0 and abs(f["V"]) > 0 and abs(f["J"] - fd["J"]) > 0


def test_j2_adjoint_against_complex_step(orc):
    """Directional derivatives of J2 by complex step through the motion
    prelude, map, LKS march and J2, against the reverse sweep."""
    p = oar(nt=10)
    gamma, chi, psi = rand_inputs(p, 21)
    a = orc.adjoint(p, gamma, chi, psi)
    rng = np.random.default_rng(22)
    for _ in range(3):
        dg = rng.standard_normal(p.M)
        dc = rng.standard_normal((p.nt, 3))
        dc[:, 2] = 0
        dp = rng.standard_normal(p.nt)
        _, dJ = orc.forward_cs(p, gamma, chi, psi, dgamma=dg, dchi=dc, dpsi=dp)
        adj = a["dgamma"] @ dg + (a["dchi"] * dc).sum() + a["dpsi"] @ dp
        assert abs(dJ[0] - adj) < 1e-10 * max(abs(dJ[0]), 1e-14), (dJ[0], adj)
    # each motion variable separately (rotation drives the torque term)
    for comp in (0, 1):
        dc = np.zeros((p.nt, 3))
        dc[:, comp] = rng.standard_normal(p.nt)
        _, dJ = orc.forward_cs(p, gamma, chi, psi, dchi=dc)
        assert abs(dJ[0] - (a["dchi"] * dc).sum()) < 1e-10 * max(abs(dJ[0]), 1e-14), comp
    dp = rng.standard_normal(p.nt)
    _, dJ = orc.forward_cs(p, gamma, chi, psi, dpsi=dp)
    assert abs(dJ[0] - a["dpsi"] @ dp) < 1e-10 * max(abs(dJ[0]), 1e-14)


def test_j2_alks_single_step_equals_exact(orc):
    p = oar(nt=1, r_t=1, r_w=1)
    gamma, chi, psi = rand_inputs(p, 31)
    rng = np.random.default_rng(32)
    s0 = rest_state(p) + 2e-2 * rng.standard_normal((p.d + 1) * p.N)
    a = orc.adjoint(p, gamma, chi, psi, state0=s0)
    b = orc.alks_adjoint(p, gamma, chi, psi, state0=s0)
    assert np.linalg.norm(a["dgamma"]) > 0
    for k in ("dgamma", "dchi", "dpsi"):
        assert np.allclose(b[k], a[k], rtol=1e-12, atol=1e-14 * np.abs(a[k]).max()), k
