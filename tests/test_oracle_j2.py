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
- Closed forms of one step's sums, written out here from the geometry of the
  rigid motion: fluid at rest under a pure rotation (the torque sum is
  -omega^2 sum kappa_ref |r|^2) and under a pure translation (the drag sum
  is -(u^G_2)^2 sum kappa_ref), a uniform flow past a still or a rotating
  body (the force sum is U_1 sum kappa_ref), and the general combination.
  A flipped torque orientation, a missing u^G_2 factor or a sign error in
  the force density each fails one of them.
- The normalisations of Eq. objective2 (1/(N_t M), 1/((x2max - x2min) M),
  1/(2 pi l_m M)) and the sum over the steps, from a whole march whose body
  is so weak that the fluid stays at rest to first order.
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


# ------------------------------------------------------------ closed forms
def _geometry(p, motion8):
    """Design points' offsets v = R(theta) r from the centre and the rigid
    velocity omega (-v_2, v_1) + u^G, written out from Sec. 2.3."""
    D0, D1 = p.m[0] + 2 * p.margin, p.m[1] + 2 * p.margin
    xi0, xi1 = np.meshgrid(np.arange(D0), np.arange(D1))  # [D1][D0], x fastest
    r1 = (xi0 - 0.5 * (D0 - 1)).ravel()
    r2 = (xi1 - 0.5 * (D1 - 1)).ravel()
    th, om = motion8[6], motion8[7]
    c, s = math.cos(th), math.sin(th)
    v1, v2 = c * r1 - s * r2, s * r1 + c * r2
    U1 = -om * v2 + motion8[3]
    U2 = om * v1 + motion8[4]
    return r1, r2, v1, v2, U1, U2


def _sums_closed_form(p, kref, motion8, Uflow):
    """Step sums for a uniform fluid velocity Uflow (zero: at rest) whose
    kernel average at every design point is Uflow itself."""
    _, _, v1, v2, U1, U2 = _geometry(p, motion8)
    f1 = kref * (Uflow[0] - U1)
    f2 = kref * (Uflow[1] - U2)
    return np.array([f1.sum(), motion8[4] * f2.sum(), motion8[7] * (v1 * f2 - v2 * f1).sum()])


def _kref(orc, p, seed):
    gamma = np.random.default_rng(seed).uniform(0.05, 0.95, size=p.M)
    return orc.kappa_ref(p, gamma)


def test_j2_step_sums_fluid_at_rest_pure_rotation(orc):
    p = oar()
    kref = _kref(orc, p, 40)
    om = 0.013
    m8 = np.array([9.3, 8.1, 0.0, 0.0, 0.0, 0.0, 0.37, om])
    u = np.zeros(2 * p.N)
    got = orc.j2_sums(p, kref, m8, u)
    r1, r2, _, _, _, _ = _geometry(p, m8)
    torque = -om * om * (kref * (r1 * r1 + r2 * r2)).sum()
    assert torque < 0
    assert abs(got[2] - torque) < 1e-13 * abs(torque), (got[2], torque)
    assert abs(got[1]) < 1e-30  # u^G_2 = 0: no drag work
    # F_L: -sum kappa_ref U_1 = omega sum kappa_ref v_2
    assert abs(got[0] - _sums_closed_form(p, kref, m8, (0.0, 0.0))[0]) < 1e-13 * abs(got[0])


def test_j2_step_sums_fluid_at_rest_pure_translation(orc):
    p = oar()
    kref = _kref(orc, p, 41)
    ug = np.array([0.021, -0.034])
    m8 = np.array([9.3, 8.1, 0.0, ug[0], ug[1], 0.0, -0.21, 0.0])
    got = orc.j2_sums(p, kref, m8, np.zeros(2 * p.N))
    K = kref.sum()
    assert abs(got[0] - (-ug[0] * K)) < 1e-13 * abs(ug[0] * K)
    assert abs(got[1] - (-ug[1] * ug[1] * K)) < 1e-13 * abs(ug[1] * ug[1] * K)
    assert abs(got[2]) < 1e-30  # omega = 0: no torque work


@pytest.mark.parametrize("om", [0.0, 0.02])
def test_j2_step_sums_uniform_flow(orc, om):
    """A uniform flow U on a periodic grid: the kernel transfers U to every
    design point unchanged (partition of unity), so a still body feels
    f = kappa_ref U and F_L's sum is U_1 sum kappa_ref; with a rotating body
    the torque sum gains omega (U_2 sum kappa v_1 - U_1 sum kappa v_2) and
    -omega^2 sum kappa |v|^2."""
    p = oar(bc=(0, 0, 0), n=(24, 22, 1), m=(5, 5, 1), margin=4)
    kref = _kref(orc, p, 42)
    U = np.array([0.031, -0.017])
    u = np.concatenate([np.full(p.N, U[0]), np.full(p.N, U[1])])
    m8 = np.array([11.4, 10.7, 0.0, 0.0, 0.0, 0.0, 0.29, om])
    got = orc.j2_sums(p, kref, m8, u)
    want = _sums_closed_form(p, kref, m8, U)
    if om == 0.0:
        assert abs(want[0] - U[0] * kref.sum()) < 1e-15
        assert abs(got[2]) < 1e-30
    for k in range(3):
        assert abs(got[k] - want[k]) < 1e-13 * max(abs(want[k]), 1e-20), (k, got, want)


def test_j2_step_sums_general_motion_fluid_at_rest(orc):
    """Translation and rotation together, fluid at rest: every sum, with
    the cross terms u^G omega of the drag and torque work."""
    p = oar()
    kref = _kref(orc, p, 43)
    m8 = np.array([9.6, 8.4, 0.0, -0.012, 0.027, 0.0, 1.1, -0.008])
    got = orc.j2_sums(p, kref, m8, np.zeros(2 * p.N))
    want = _sums_closed_form(p, kref, m8, (0.0, 0.0))
    _, _, v1, v2, _, _ = _geometry(p, m8)
    ug1, om = m8[4], m8[7]
    # the drag sum written out: -u^G_2 (omega sum kappa v_1 + u^G_2 sum kappa)
    drag = -ug1 * (om * (kref * v1).sum() + ug1 * kref.sum())
    assert abs(want[1] - drag) < 1e-15
    for k in range(3):
        assert abs(got[k] - want[k]) < 1e-13 * abs(want[k]), (k, got, want)


def test_j2_normalisations_over_a_march(orc):
    """A body too weak to set the fluid moving (kappa_max = 1e-7): the fluid
    stays at rest to first order, so every step's sums are the closed forms
    above at that step's motion, and J_out = (J2, F_L, F_D) must be their
    sums over the steps times 1/(N_t M), 1/((x2max - x2min) M) and, for
    the torque work T = (J2 - F_L - w_D F_D) / w_T, 1/(2 pi l_m M)."""
    p = oar(nt=10, kappa_max=1e-7, l_m=3.5, w_d=0.4, w_t=0.7)
    gamma, chi, psi = rand_inputs(p, 44)
    mot = orc.motion(p, chi, psi)
    kref = orc.kappa_ref(p, gamma)
    sums = np.zeros(3)
    for t in range(p.nt):
        sums += _sums_closed_form(p, kref, mot[t], (0.0, 0.0))
    M = p.m[0] * p.m[1]
    FL = sums[0] / (p.nt * M)
    FD = sums[1] / ((p.xg_max[1] - p.xg_min[1]) * M)
    T = sums[2] / (2.0 * math.pi * p.l_m * M)
    f = orc.forward(p, gamma, chi, psi)
    assert abs(FL) > 0 and abs(FD) > 0 and abs(T) > 0
    assert abs(f["E"] - FL) < 1e-5 * abs(FL), (f["E"], FL)
    assert abs(f["V"] - FD) < 1e-5 * abs(FD), (f["V"], FD)
    Tg = (f["J"] - f["E"] - p.w_d * f["V"]) / p.w_t
    assert abs(Tg - T) < 1e-5 * abs(T), (Tg, T)
    assert abs(f["J"] - (FL + p.w_d * FD + p.w_t * T)) < 1e-5 * abs(f["J"])
