"""Pins of the oracle's paper-literal ALKS backward (Sec. 2.5).

The ALKS discretises the continuous adjoint on the lattice.  It is not the
exact transpose of the forward march, so nothing computes the same numbers by
another route.  It is pinned instead by:

- closed forms of one source-free level for uniform fields and for a single
  Fourier mode of the adjoint stress (the coupling factors and the
  divergence term of the adjoint equilibrium);
- two regimes in which it must coincide with the exact discrete adjoint,
  which is itself pinned by complex step and finite differences:
  - with no body (kappa = 0) its multipliers evolve exactly as the discrete
    adjoint's;
  - over a single step no coupling has formed yet, so every gradient agrees;
- the size of its departure from the exact gradient on the 64x64 workload.
  The paper's own check against finite differences shows slight
  differences, App. A.
"""
import math

import numpy as np
import pytest

from paper_2608_01071_amd import workloads as W

from test_oracle_pins import rand_inputs, rest_state, small2d, small3d


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cosine(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def periodic(d, n):
    if d == 2:
        return small2d(n=(n, n, 1), bc=(0, 0, 0), tgt_lo=(0, 0, 0), tgt_hi=(1, n, 1))
    return small3d(n=(n, n, n), bc=(0, 0, 0), tgt_lo=(0, 0, 0), tgt_hi=(1, 1, 1))


@pytest.mark.parametrize("d", [2, 3])
def test_alks_uniform_level_closed_form(orc, d):
    """Uniform multipliers and velocity, no divergence: the adjoint
    equilibrium is p~ + 3 c_i.(u~ + 3 s~ u - p~ u), and its lattice moments
    (sum w = 1, sum w c_a c_b = delta_ab / 3, odd moments 0) give
    p~* = p~, u~* = u~ + 3 s~ u - p~ u, s~* = (p~ / 3) I."""
    p = periodic(d, 6)
    N = p.N
    rng = np.random.default_rng(20 + d)
    pt = 0.7
    ut = np.array([0.3, -0.2, 0.1])[:d]
    st = rng.standard_normal((d, d))  # need not be symmetric
    u = np.array([0.05, -0.03, 0.02])[:d]
    f = np.zeros((1 + d + 9) * N)
    f[:N] = pt
    for a in range(d):
        f[(1 + a) * N:(2 + a) * N] = ut[a]
        for b in range(d):
            k = 1 + d + 3 * a + b
            f[k * N:(k + 1) * N] = st[a, b]
    uf = np.repeat(u, N)
    out = orc.alks_gather(p, f, uf).reshape(1 + d + 9, N)
    assert np.allclose(out[0], pt, rtol=0, atol=1e-15)
    want_u = ut + 3.0 * st @ u - pt * u
    for a in range(d):
        assert np.allclose(out[1 + a], want_u[a], rtol=0, atol=1e-15)
        for b in range(d):
            want = pt / 3.0 if a == b else 0.0
            assert np.allclose(out[1 + d + 3 * a + b], want, rtol=0, atol=1e-15)


def test_alks_divergence_term_single_mode(orc):
    """s~_xy = s~_yx = cos(t y) on a periodic D2Q9 grid, all else zero.  The
    divergence term -A d_b(s~_ab + s~_ba), with d read as minus the transpose
    of the central difference, is V = (2 A sin t sin(t y), 0), and the gather
    gives u~*_x = (2 + cos t) / 9 * V_x, u~*_y = 0, p~* = 0."""
    n = 12
    p = periodic(2, n)
    N = p.N
    A = 0.75 - 4.5 * p.nu
    th = 2.0 * math.pi / n
    y = np.repeat(np.arange(n), n)  # node index x + n y
    f = np.zeros((1 + 2 + 9) * N)
    mode = np.cos(th * y)
    f[(3 + 1) * N:(3 + 2) * N] = mode  # s~_xy (plane 3*0 + 1)
    f[(3 + 3) * N:(3 + 4) * N] = mode  # s~_yx (plane 3*1 + 0)
    out = orc.alks_gather(p, f, np.zeros(2 * N)).reshape(12, N)
    V = 2.0 * A * math.sin(th) * np.sin(th * y)
    assert np.allclose(out[1], (2.0 + math.cos(th)) / 9.0 * V, rtol=0, atol=1e-15)
    assert np.allclose(out[2], 0.0, rtol=0, atol=1e-15)
    assert np.allclose(out[0], 0.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_alks_equals_discrete_adjoint_without_body(orc, d):
    """gamma = 0 makes kappa = 0 at every step.  The ALKS multipliers then
    evolve exactly as the discrete adjoint's (f~ = -F), so its estimate of
    dJ/d(state0) equals the exact one.  The flow is not trivial: a random
    initial state and, in 2D, a moving wall."""
    if d == 2:
        uw = np.zeros((3, 2, 3))
        uw[1, 1, 0] = 0.05
        p = small2d(phi=0.3, u_wall=uw)
    else:
        p = small3d()
    _, chi, psi = rand_inputs(p, 50 + d)
    rng = np.random.default_rng(60 + d)
    s0 = rest_state(p) + 2e-2 * rng.standard_normal((p.d + 1) * p.N)
    g0 = np.zeros(p.M)
    a = orc.adjoint(p, g0, chi, psi, state0=s0)
    b = orc.alks_adjoint(p, g0, chi, psi, state0=s0)
    S = (p.d + 1) * p.N
    assert np.linalg.norm(a["adj_initial"]) > 0
    assert rel(b["adj_initial"][:S], a["adj_initial"]) < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_alks_single_step_equals_discrete_adjoint(orc, d):
    """Over one step the ALKS has formed no coupling yet: the Brinkman and
    objective sources act on u~ alone in both schemes, and
    3 (u - u^S).u~ equals the discrete dJ/dkappa.  Every gradient agrees,
    with a body present (the target box covers it)."""
    if d == 2:
        p = small2d(phi=0.3, nt=1, r_t=1, r_w=1, tgt_lo=(5, 3, 0), tgt_hi=(15, 15, 1))
    else:
        p = small3d(nt=1, r_t=1, r_w=1, tgt_lo=(5, 5, 3), tgt_hi=(13, 13, 9))
    gamma, chi, psi = rand_inputs(p, 70 + d)
    rng = np.random.default_rng(80 + d)
    s0 = rest_state(p) + 2e-2 * rng.standard_normal((p.d + 1) * p.N)
    a = orc.adjoint(p, gamma, chi, psi, state0=s0)
    b = orc.alks_adjoint(p, gamma, chi, psi, state0=s0)
    assert np.linalg.norm(a["dgamma"]) > 0
    b["adj_initial"] = b["adj_initial"][:(p.d + 1) * p.N]
    for k in ("dgamma", "dchi", "dpsi", "adj_initial"):
        assert np.allclose(b[k], a[k], rtol=1e-12, atol=1e-14 * np.abs(a[k]).max()), k


def test_alks_departure_from_exact_gradient_c1(orc):
    """The 64x64 workload (200 steps, kappa_max = 300): the ALKS gradient
    points the way of the exact one (cosine >= 0.995) and differs from it by
    a few percent.  The measured values are 5.0 % (gamma), 5.4 % (chi) and
    7.6 % (psi); the bound here is 10 %.  The difference is not zero: inside
    the body the ALKS leaves the u-coupling of the adjoint equilibrium
    undivided by 1 + kappa."""
    p, gamma, chi, psi = W.c1(precision=1)
    a = orc.adjoint(p, gamma, chi, psi)
    b = orc.alks_adjoint(p, gamma, chi, psi)
    for k in ("dgamma", "dchi", "dpsi"):
        r = rel(b[k], a[k])
        assert 1e-3 < r < 0.10, (k, r)
        assert cosine(b[k], a[k]) > 0.995, k


def test_alks_is_linear_in_the_seed(orc):
    """The ALKS is linear in its multipliers: scaling the objective seed
    scales every output (by a power of two, so exactly)."""
    p = small2d(phi=0.2, nt=6)
    gamma, chi, psi = rand_inputs(p, 90)
    a = orc.alks_adjoint(p, gamma, chi, psi)
    b = orc.alks_adjoint(p, gamma, chi, psi, dJ=-2.0)
    for k in ("dgamma", "dchi", "dpsi", "adj_initial"):
        assert np.array_equal(b[k], -2.0 * a[k]), k


def ncarry(p):
    """Planes of the ALKS state p~, u~ and the symmetric s~."""
    return 1 + p.d + p.d * (p.d + 1) // 2


def random_terminal(p, seed, ptilde=True, stilde=True):
    """A carried ALKS state of plausible size in the adj_terminal layout:
    d+1 planes that are not read, then (p~, u~, s~)."""
    rng = np.random.default_rng(seed)
    S = (p.d + 1) * p.N
    term = np.zeros(S + ncarry(p) * p.N)
    term[S:] = 1e-3 * rng.standard_normal(ncarry(p) * p.N)
    if not ptilde:
        term[S:S + p.N] = 0.0
    if not stilde:
        term[S + (1 + p.d) * p.N:] = 0.0
    return term


def exact_terminal(orc, p, term, u_last):
    """The exact adjoint's terminal state (pbar, ubar) = (-3 p~, -V) that
    the carried ALKS state stands for at the last level, V formed with that
    level's velocity."""
    S = (p.d + 1) * p.N
    carry = term[S:]
    return np.concatenate([-3.0 * carry[:p.N], -orc.alks_vector(p, carry, u_last)])


@pytest.mark.parametrize("d", [2, 3])
def test_alks_terminal_state_without_body_equals_exact_adjoint(orc, d):
    """Periodic approximation (Sec. 3.3) with gamma = 0: an ALKS run from a
    carried state (p~, u~, s~) at t1 gives the exact adjoint's dJ/d(state0)
    for the terminal adjoint (-3 p~, -V), V formed with this run's own
    velocity at t1 (Algorithm 1 forms the adjoint equilibrium of every level
    from that level's flow)."""
    p = small2d(phi=0.3) if d == 2 else small3d()
    _, chi, psi = rand_inputs(p, 90 + d)
    rng = np.random.default_rng(91 + d)
    s0 = rest_state(p) + 2e-2 * rng.standard_normal((p.d + 1) * p.N)
    g0 = np.zeros(p.M)
    S = (p.d + 1) * p.N
    term = random_terminal(p, 92 + d)
    fwd = orc.forward(p, g0, chi, psi, state0=s0)
    u_last = fwd["final"][p.N:S]
    a = orc.adjoint(p, g0, chi, psi, state0=s0, adj_terminal=exact_terminal(orc, p, term, u_last))
    b = orc.alks_adjoint(p, g0, chi, psi, state0=s0, adj_terminal=term)
    assert rel(b["adj_initial"][:S], a["adj_initial"]) < 1e-12
    # the velocity the coupling is formed with matters: another run's
    # velocity (here the start state's) gives a different answer
    wrong = orc.adjoint(p, g0, chi, psi, state0=s0,
                        adj_terminal=exact_terminal(orc, p, term, s0[p.N:S]))
    assert rel(b["adj_initial"][:S], wrong["adj_initial"]) > 1e-6


def test_alks_terminal_state_single_step(orc):
    """One step from a carried state with p~ = 0 and s~ = 0, whose adjoint
    equilibrium has no coupling part (V = 3 u~): the sources act on the same
    vector in both schemes, so every gradient and dJ/d(state0) equal the
    exact adjoint's from (0, -3 u~), with a body."""
    p = small2d(phi=0.3, nt=1, r_t=1, r_w=1, tgt_lo=(5, 3, 0), tgt_hi=(15, 15, 1))
    gamma, chi, psi = rand_inputs(p, 95)
    rng = np.random.default_rng(96)
    s0 = rest_state(p) + 2e-2 * rng.standard_normal((p.d + 1) * p.N)
    S = (p.d + 1) * p.N
    term = random_terminal(p, 97, ptilde=False, stilde=False)
    ex = np.concatenate([np.zeros(p.N), -3.0 * term[S + p.N:S + (1 + p.d) * p.N]])
    a = orc.adjoint(p, gamma, chi, psi, state0=s0, adj_terminal=ex)
    b = orc.alks_adjoint(p, gamma, chi, psi, state0=s0, adj_terminal=term)
    b["adj_initial"] = b["adj_initial"][:S]
    for k in ("dgamma", "dchi", "dpsi", "adj_initial"):
        assert np.allclose(b[k], a[k], rtol=1e-12, atol=1e-14 * np.abs(a[k]).max()), k


def test_alks_is_linear_in_the_terminal_state(orc):
    """Seed and carried state enter linearly: the run with both is the sum
    of the run with the seed alone and the run with the state alone."""
    p = small2d(phi=0.2, nt=6)
    gamma, chi, psi = rand_inputs(p, 98)
    term = random_terminal(p, 99)
    both = orc.alks_adjoint(p, gamma, chi, psi, adj_terminal=term)
    seed = orc.alks_adjoint(p, gamma, chi, psi)
    state = orc.alks_adjoint(p, gamma, chi, psi, dJ=0.0, adj_terminal=term)
    for k in ("dgamma", "dchi", "dpsi", "adj_initial"):
        assert rel(both[k], seed[k] + state[k]) < 1e-12, k


def test_alks_terminal_planes_before_the_carry_are_not_read(orc):
    p = small2d(phi=0.2, nt=4)
    gamma, chi, psi = rand_inputs(p, 100)
    term = random_terminal(p, 101)
    S = (p.d + 1) * p.N
    a = orc.alks_adjoint(p, gamma, chi, psi, adj_terminal=term)
    term[:S] = np.random.default_rng(102).standard_normal(S)
    b = orc.alks_adjoint(p, gamma, chi, psi, adj_terminal=term)
    for k in ("dgamma", "dchi", "dpsi", "adj_initial"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("nt", [1, 3])
def test_alks_carry_multistep_uniform_closed_form(orc, nt):
    """A body that fills a periodic box: the design grid covers every node
    (margin 0, m = n) with a uniform density at rest, so kappa is the
    uniform kappa_ref = k everywhere (the kernel is a partition of unity),
    and a uniform start velocity u0 decays as u_t = u0 / (1 + k)^t with p
    fixed.  J1 averages n.u over the whole box (phi = 0), so each level's
    seed is -(dJ / N_T) n / 3 on u~.  From a carried uniform state
    (p~c, u~c, s~c) the ALKS, written out level by level, is:
      level N_t: u~ = (u~c - g n / 3) / (1 + k), s~ = s~c;
      gather:    p~* = p~c, u~* = u~ + 3 s~ u - p~c u (u of the level
                 gathered from), s~* = p~c I / 3, after which the coupling
                 cancels: u~* = u~;
      level t:   u~ = (u~* - g n / 3) / (1 + k);
    dJ/dkappa per node per level is 3 u_t . u~_t and, the kernel summing to
    1 over the nodes, dJ/dkappa_ref = sum_t 3 u_t . u~_t at every design
    point; the motion gradient vanishes.  This fixes where the carry enters,
    that its coupling takes this run's velocity u_{N_t}, the seed's factor
    and the division of the raw moment by 1 + kappa at every level."""
    n = 8
    p = small2d(n=(n, n, 1), bc=(0, 0, 0), m=(n, n, 1), margin=0, nt=nt, r_t=1, r_w=1,
                xg_min=(3.5, 3.5, 0.0), xg_max=(3.5, 3.5, 0.0), th_min=0.0, th_max=0.0,
                tgt_lo=(0, 0, 0), tgt_hi=(n, n, 1), ndir=(1.0, 0.0, 0.0), phi=0.0,
                kappa_max=0.9, q=0.1)
    N = p.N
    gam = 0.6
    gamma = np.full(p.M, gam)
    chi = np.full((nt, 3), 0.5)
    psi = np.full(nt, 0.5)
    k = p.kappa_max * p.q * gam / ((1.0 - gam) + p.q)
    u0 = np.array([0.02, -0.013])
    s0 = rest_state(p, u=(u0[0], u0[1], 0.0))
    pc = 0.37
    uc = np.array([0.11, -0.23])
    sc = np.array([[0.05, -0.08], [-0.08, 0.21]])  # not p~c I / 3
    term = np.zeros((p.d + 1) * N + ncarry(p) * N)
    S = (p.d + 1) * N
    term[S:S + N] = pc
    term[S + N:S + 2 * N] = uc[0]
    term[S + 2 * N:S + 3 * N] = uc[1]
    term[S + 3 * N:S + 4 * N] = sc[0, 0]
    term[S + 4 * N:S + 5 * N] = sc[1, 1]
    term[S + 5 * N:S + 6 * N] = sc[0, 1]
    dJ = 1.7
    g = dJ / (nt * N)
    nvec = np.array([1.0, 0.0])
    u = [u0 / (1.0 + k) ** t for t in range(nt + 1)]
    # closed form, level by level
    ut = {}
    ut[nt] = (uc - g * nvec / 3.0) / (1.0 + k)
    s_lvl = sc
    for t in range(nt - 1, -1, -1):
        ustar = ut[t + 1] + 3.0 * s_lvl @ u[t + 1] - pc * u[t + 1]
        s_lvl = pc * np.eye(2) / 3.0
        ut[t] = ustar if t == 0 else (ustar - g * nvec / 3.0) / (1.0 + k)
    kbar = sum(3.0 * u[t] @ ut[t] for t in range(1, nt + 1))
    dgam = kbar * p.kappa_max * p.q * (1.0 + p.q) / ((1.0 - gam) + p.q) ** 2

    r = orc.alks_adjoint(p, gamma, chi, psi, state0=s0, dJ=dJ, adj_terminal=term)
    c = r["adj_initial"][S:].reshape(ncarry(p), N)
    assert np.allclose(c[0], pc, rtol=1e-13, atol=0)
    assert np.allclose(c[1], ut[0][0], rtol=1e-12, atol=1e-16)
    assert np.allclose(c[2], ut[0][1], rtol=1e-12, atol=1e-16)
    assert np.allclose(c[3], pc / 3.0, rtol=1e-13, atol=0)
    assert np.allclose(c[4], pc / 3.0, rtol=1e-13, atol=0)
    assert np.allclose(c[5], 0.0, rtol=0, atol=1e-16)
    assert np.allclose(r["dgamma"], dgam, rtol=1e-11, atol=0), (r["dgamma"][:3], dgam)
    assert np.abs(r["dchi"]).max() < 1e-12 * abs(dgam) * N
    # the estimate of dJ/d(state0): (-3 p~, -V), V = 3 u~ once s~ = p~ I / 3
    est = r["adj_initial"][:S].reshape(3, N)
    assert np.allclose(est[0], -3.0 * pc, rtol=1e-13, atol=0)
    if nt > 1:
        assert np.allclose(est[1], -3.0 * ut[0][0], rtol=1e-12, atol=1e-16)
