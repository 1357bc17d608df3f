"""GPU parity: every stage of the HIP path against the CPU oracle.

All calls go through the C ABI (ctypes binding).  Inputs are seeded; the
oracle works in FP64 on the same arrays.  Tolerances:
  * FP64 state: relative 1e-11 of the field's max magnitude per stage, 1e-10
    for whole runs (only the summation order differs);
  * FP32 state with FP64 sums: objective relative error <= 1e-5, gradient
    relative L2 error <= 1e-3 (the targets of the precision extension);
    single stages <= 2e-5 of the field's max magnitude.
Grids are ragged (not multiples of the 32x8 tile) and include the sizes
n = 2 (mod tile) on wall axes, where the tile grid is shifted by one node.
"""
import math

import numpy as np
import pytest
import torch

from paper_2608_01071_amd import workloads as W

pytestmark = pytest.mark.gpu

THIRD = 1.0 / 3.0


def lk():
    from paper_2608_01071_amd import lks
    return lks


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def l2err(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def prob2d(n=(45, 21), prec=1, **kw):
    base = dict(d=2, n=(n[0], n[1], 1), bc=(0, 1, 0), nu=0.08, kappa_max=60.0, q=0.1,
                m=(8, 6, 1), margin=4, xg_min=(n[0] / 2 - 1.5, n[1] / 2 - 1.0, 0.0),
                xg_max=(n[0] / 2 + 1.5, n[1] / 2 + 1.0, 0.0), th_min=-0.3, th_max=0.3,
                nt=12, r_t=3, r_w=3, tgt_lo=(n[0] // 2 - 2, 1, 0),
                tgt_hi=(n[0] // 2 + 2, n[1] - 1, 1),
                ndir=(1.0, 0.0, 0.0), phi=0.2, precision=prec, ckpt_k=5)
    base.update(kw)
    return W.Problem(**base)


def prob3d(n=(34, 18, 20), prec=1, **kw):
    base = dict(d=3, n=n, bc=(1, 1, 0), nu=0.08, kappa_max=40.0, q=0.1, m=(6, 4, 5), margin=3,
                xg_min=(n[0] / 2 - 1.0, n[1] / 2 - 0.5, n[2] / 2 - 1.0),
                xg_max=(n[0] / 2 + 1.0, n[1] / 2 + 0.5, n[2] / 2 + 1.0), th_min=-0.3,
                th_max=0.3, nt=6, r_t=2, r_w=2, tgt_lo=(4, 4, 2), tgt_hi=(30, 14, 5),
                ndir=(0.0, 0.0, 1.0), phi=0.1, precision=prec, ckpt_k=4)
    base.update(kw)
    return W.Problem(**base)


def rand_state(p, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    s = np.zeros((p.d + 1) * p.N)
    s[: p.N] = THIRD + 0.01 * rng.standard_normal(p.N)
    s[p.N:] = amp * rng.standard_normal(p.d * p.N)
    return s


def gpu_state(s, p):
    g = s.copy()
    g[: p.N] -= THIRD
    return g


def oracle_state(g, p):
    s = np.asarray(g, dtype=np.float64).copy()
    s[: p.N] += THIRD
    return s


def rand_inputs(p, seed):
    rng = np.random.default_rng(seed)
    gamma = rng.uniform(0.05, 0.95, size=p.M)
    chi = rng.uniform(0.3, 0.7, size=(p.nt, 3))
    psi = rng.uniform(0.3, 0.7, size=p.nt)
    return gamma, chi, psi


PROBS = {
    "2d_walls_y": lambda prec: prob2d((45, 21), prec),
    "2d_shift_y": lambda prec: prob2d((37, 18), prec),
    "2d_walls_xy_shift_x": lambda prec: prob2d((34, 19), prec, bc=(1, 1, 0), tgt_lo=(14, 0, 0),
                                                tgt_hi=(20, 19, 1)),
    "3d_shift_xy": lambda prec: prob3d((34, 18, 20), prec),
    "3d_plain": lambda prec: prob3d((29, 23, 17), prec, tgt_lo=(3, 3, 1), tgt_hi=(26, 20, 3)),
}


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_motion_and_kappa_ref(orc, name, prec):
    p = PROBS[name](prec)
    plan = lk().Plan(p)
    gamma, chi, psi = rand_inputs(p, 1)
    m = cpu(plan.motion(chi, psi))
    assert relerr(m, orc.motion(p, chi, psi)) < 1e-14
    k = cpu(plan.kappa_ref(gamma))
    tol = 1e-15 if prec == 1 else 1e-7
    assert relerr(k, orc.kappa_ref(p, gamma)) < tol


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_map(orc, name, prec):
    p = PROBS[name](prec)
    plan = lk().Plan(p)
    rng = np.random.default_rng(2)
    kref = rng.uniform(0, 50, size=p.Mtot)
    tol = 1e-12 if prec == 1 else 2e-6
    for th in (0.0, 0.31, -1.2, math.pi / 2):
        mot = np.array([p.n[0] / 2 + 0.37, p.n[1] / 2 - 0.21, (p.n[2] / 2 + 0.13) if p.d == 3 else 0,
                        0.02, -0.01, 0.005 if p.d == 3 else 0, th, 0.003])
        k, us = plan.map(kref, mot)
        ko, uo = orc.map_fields(p, kref, mot)
        assert relerr(cpu(k), ko) < tol, th
        assert relerr(cpu(us), uo) < tol, th


def test_map_wraps_periodic_seam(orc):
    """A body straddling the periodic seam maps its support across it."""
    p = prob2d((45, 21), 1)
    plan = lk().Plan(p)
    kref = np.random.default_rng(3).uniform(0, 5, size=p.Mtot)
    mot = np.array([1.3, 10.2, 0, 0.01, 0.0, 0, 0.4, 0.002])
    k, us = plan.map(kref, mot)
    ko, uo = orc.map_fields(p, kref, mot)
    assert relerr(cpu(k), ko) < 1e-12 and relerr(cpu(us), uo) < 1e-12
    assert np.abs(ko.reshape(21, 45)[:, -3:]).max() > 0


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_step(orc, name, prec):
    p = PROBS[name](prec)
    plan = lk().Plan(p)
    rng = np.random.default_rng(4)
    s = rand_state(p, 5)
    kap = rng.uniform(0, 30, size=p.N)
    us = 0.05 * rng.standard_normal(p.d * p.N)
    out = cpu(plan.step(gpu_state(s, p), kap, us))
    ref = orc.step(p, s, kap, us)
    tol = 1e-13 if prec == 1 else 2e-6
    # pressure offset compared as p - 1/3, velocity as is
    assert relerr(out[: p.N], ref[: p.N] - THIRD) < (1e-11 if prec == 1 else 2e-5)
    assert relerr(out[p.N:], ref[p.N:]) < tol


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_step_adjoint(orc, name, prec):
    p = PROBS[name](prec)
    plan = lk().Plan(p)
    rng = np.random.default_rng(6)
    s_in = rand_state(p, 7)
    kap = rng.uniform(0, 30, size=p.N)
    us = 0.05 * rng.standard_normal(p.d * p.N)
    s_out = orc.step(p, s_in, kap, us)
    lam = rng.standard_normal((p.d + 1) * p.N)
    lp, kb, ub = plan.step_adjoint(gpu_state(s_in, p), gpu_state(s_out, p), kap, us, lam)
    rlp, rkb, rub = orc.step_adjoint(p, s_in, s_out, kap, us, lam)
    tol = 1e-12 if prec == 1 else 2e-5
    assert relerr(cpu(lp), rlp) < tol
    assert relerr(cpu(kb), rkb) < tol
    assert relerr(cpu(ub), rub) < tol


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_map_adjoint(orc, name, prec):
    p = PROBS[name](prec)
    plan = lk().Plan(p)
    rng = np.random.default_rng(8)
    kref = rng.uniform(0, 50, size=p.Mtot)
    kbar = rng.standard_normal(p.N)
    usbar = rng.standard_normal(p.d * p.N)
    # wall nodes carry no body adjoint (the step transpose zeroes them)
    n = p.n
    idx = np.arange(p.N)
    x, y, z = idx % n[0], (idx // n[0]) % n[1], idx // (n[0] * n[1])
    wall = np.zeros(p.N, bool)
    for a, c in enumerate((x, y, z)[: p.d]):
        if p.bc[a] == 1:
            wall |= (c == 0) | (c == n[a] - 1)
    kbar[wall] = 0
    usbar.reshape(p.d, p.N)[:, wall] = 0
    tol = 1e-12 if prec == 1 else 2e-5
    for th in (0.0, 0.41):
        mot = np.array([p.n[0] / 2 - 0.3, p.n[1] / 2 + 0.2, (p.n[2] / 2 - 0.4) if p.d == 3 else 0,
                        0.01, 0.02, 0.01 if p.d == 3 else 0, th, 0.004])
        kb, mb = plan.map_adjoint(kref, mot, kbar, usbar)
        rkb, rmb = orc.map_adjoint(p, kref, mot, kbar, usbar)
        assert relerr(cpu(kb), rkb) < tol
        assert relerr(cpu(mb), rmb) < (1e-11 if prec == 1 else 1e-4)


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_forward_adjoint_run(orc, name, prec):
    """Whole runs (checkpoint K < nt, ragged segment) vs the oracle."""
    p = PROBS[name](prec)
    plan = lk().Plan(p)
    gamma, chi, psi = rand_inputs(p, 9)
    J3, fin = plan.forward(gamma, chi, psi, want_final=True)
    g = plan.adjoint(gamma, chi, psi, want_initial=True)
    ref = orc.forward(p, gamma, chi, psi)
    adj = orc.adjoint(p, gamma, chi, psi)
    J = cpu(J3)
    if prec == 1:
        assert abs(J[0] - ref["J"]) <= 1e-10 * abs(ref["J"])
        assert relerr(oracle_state(cpu(fin), p), ref["final"]) < 1e-10
        for k in ("dgamma", "dchi", "dpsi"):
            assert l2err(cpu(g[k]), adj[k]) < 1e-9, k
        assert relerr(cpu(g["adj_initial"]), adj["adj_initial"]) < 1e-9
    else:
        assert abs(J[0] - ref["J"]) <= 1e-5 * abs(ref["J"])
        for k in ("dgamma", "dchi", "dpsi"):
            assert l2err(cpu(g[k]), adj[k]) < 1e-3, k


@pytest.mark.parametrize("prec", [1, 0])
def test_c1_forward_adjoint(orc, prec):
    """The 64x64 / 200-step workload (D2Q9, design 32x32, x/y/theta motion)."""
    p, gamma, chi, psi = W.c1(precision=prec)
    p = p.replace(ckpt_k=50)
    plan = lk().Plan(p)
    J3, _ = plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi)
    ref = orc.forward(p, gamma, chi, psi)
    adj = orc.adjoint(p, gamma, chi, psi)
    J = cpu(J3)[0]
    if prec == 1:
        assert abs(J - ref["J"]) <= 1e-10 * abs(ref["J"])
        tol = 1e-8
    else:
        assert abs(J - ref["J"]) <= 1e-5 * abs(ref["J"])
        tol = 1e-3
    for k in ("dgamma", "dchi", "dpsi"):
        assert l2err(cpu(g[k]), adj[k]) < tol, k


def test_checkpoint_interval_does_not_change_gradients(orc):
    """K in {1, 3, 7, nt} and full tape give bit-identical gradients, with the
    body fields of every step kept or re-mapped per segment."""
    p0 = prob2d((45, 21), 0, nt=14)
    gamma, chi, psi = rand_inputs(p0, 10)
    outs = []
    for K in (1, 3, 7, 14):
        for tape in (-1, 1):
            plan = lk().Plan(p0.replace(ckpt_k=K, body_tape=tape))
            J3, _ = plan.forward(gamma, chi, psi)
            g = plan.adjoint(gamma, chi, psi)
            outs.append((cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1])
def test_body_tape_modes_agree_3d(orc, prec):
    """3D: keeping every step's body fields (no map in the recompute) and
    re-mapping them per segment give bit-identical objective and gradients,
    and both match the oracle."""
    p0 = prob3d(prec=prec)
    gamma, chi, psi = rand_inputs(p0, 21)
    outs = []
    for tape in (-1, 1):
        plan = lk().Plan(p0.replace(body_tape=tape))
        J3, _ = plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi)
        outs.append((cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    ref = orc.forward(p0, gamma, chi, psi)
    adj = orc.adjoint(p0, gamma, chi, psi)
    assert abs(outs[1][0][0] - ref["J"]) <= (1e-10 if prec == 1 else 1e-5) * abs(ref["J"])
    for k, key in enumerate(("dgamma", "dchi", "dpsi")):
        assert l2err(outs[1][1 + k], adj[key]) < (1e-9 if prec == 1 else 1e-3), key


def test_periodic_approximation_state_carry(orc):
    """state0 / state_final and adj_terminal / adj_initial round trip
    (Sec. 3.3): a second run started from the first run's final state
    matches the oracle started from the same state."""
    p = prob2d((45, 21), 1)
    plan = lk().Plan(p)
    gamma, chi, psi = rand_inputs(p, 11)
    _, fin = plan.forward(gamma, chi, psi, want_final=True)
    s1 = oracle_state(cpu(fin), p)
    J3, fin2 = plan.forward(gamma, chi, psi, state0=fin, want_final=True)
    rng = np.random.default_rng(12)
    aterm = 0.01 * rng.standard_normal((p.d + 1) * p.N)
    g = plan.adjoint(gamma, chi, psi, adj_terminal=aterm, want_initial=True)
    ref = orc.forward(p, gamma, chi, psi, state0=s1)
    adj = orc.adjoint(p, gamma, chi, psi, state0=s1, adj_terminal=aterm)
    assert abs(cpu(J3)[0] - ref["J"]) <= 1e-10 * abs(ref["J"])
    assert relerr(oracle_state(cpu(fin2), p), ref["final"]) < 1e-10
    assert relerr(cpu(g["adj_initial"]), adj["adj_initial"]) < 1e-9
    assert l2err(cpu(g["dgamma"]), adj["dgamma"]) < 1e-9


def test_edge_cases(orc):
    """Empty target (J = 0, zero gradients), no body (kappa_max = 0),
    a single step, and seed scaling."""
    lks = lk()
    p = prob2d((45, 21), 1, tgt_lo=(0, 0, 0), tgt_hi=(0, 21, 1))
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 13)
    J3, _ = plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi)
    assert np.all(cpu(J3) == 0) and np.all(cpu(g["dgamma"]) == 0) and np.all(cpu(g["dpsi"]) == 0)
    p = prob2d((45, 21), 1, kappa_max=0.0)
    plan = lks.Plan(p)
    J3, _ = plan.forward(gamma, chi, psi)
    assert abs(cpu(J3)[0]) == 0.0
    p = prob2d((45, 21), 1, nt=1, ckpt_k=1)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 14)
    s0 = rand_state(p, 15)
    J3, _ = plan.forward(gamma, chi, psi, state0=gpu_state(s0, p))
    g = plan.adjoint(gamma, chi, psi, dJ=[-3.0])
    ref = orc.forward(p, gamma, chi, psi, state0=s0)
    adj = orc.adjoint(p, gamma, chi, psi, state0=s0, dJ=-3.0)
    assert abs(cpu(J3)[0] - ref["J"]) <= 1e-11 * abs(ref["J"])
    assert l2err(cpu(g["dgamma"]), adj["dgamma"]) < 1e-10


def test_edge_cases_3d(orc):
    """D3Q15: an empty target (J = 0, zero gradients), no body (kappa_max = 0,
    a moving start state: J as the oracle's, every gradient exactly zero), and
    a single step from a given state with K = 1 and a scaled seed, against the
    oracle."""
    lks = lk()
    p = prob3d(prec=1, tgt_lo=(0, 0, 0), tgt_hi=(0, 18, 1))
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 23)
    J3, _ = plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi)
    assert np.all(cpu(J3) == 0)
    assert np.all(cpu(g["dgamma"]) == 0) and np.all(cpu(g["dpsi"]) == 0)
    p = prob3d(prec=1, kappa_max=0.0)
    plan = lks.Plan(p)
    s0 = rand_state(p, 26)  # a moving start state: at rest nothing would drive the flow
    J3, _ = plan.forward(gamma, chi, psi, state0=gpu_state(s0, p))
    g = plan.adjoint(gamma, chi, psi)
    ref = orc.forward(p, gamma, chi, psi, state0=s0, want_final=False)
    assert abs(ref["J"]) > 1e-8
    assert abs(cpu(J3)[0] - ref["J"]) <= 1e-10 * abs(ref["J"])
    for k in ("dgamma", "dchi", "dpsi"):
        assert np.all(cpu(g[k]) == 0), k
    p = prob3d(prec=1, nt=1, ckpt_k=1)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 24)
    s0 = rand_state(p, 25)
    J3, _ = plan.forward(gamma, chi, psi, state0=gpu_state(s0, p))
    g = plan.adjoint(gamma, chi, psi, dJ=[-3.0])
    ref = orc.forward(p, gamma, chi, psi, state0=s0)
    adj = orc.adjoint(p, gamma, chi, psi, state0=s0, dJ=-3.0)
    assert abs(cpu(J3)[0] - ref["J"]) <= 1e-11 * abs(ref["J"])
    for k in ("dgamma", "dchi", "dpsi"):
        assert l2err(cpu(g[k]), adj[k]) < 1e-10, k


@pytest.mark.parametrize("prec", [0, 1])
def test_step_results_do_not_depend_on_the_plane(prec):
    """D3Q15 in a periodic box: one forward step and one adjoint step of a
    z-invariant state, body and adjoint state give bitwise identical planes.
    (The plane loops are unrolled, so a plane's arithmetic must not depend on
    the parity of its place in a segment.)"""
    lks = lk()
    n = (40, 24, 20)
    p = prob3d(n=n, prec=prec, bc=(0, 0, 0), tgt_lo=(0, 0, 0), tgt_hi=(1, 1, 1))
    plan = lks.Plan(p)
    P = n[0] * n[1]
    rng = np.random.default_rng(77)
    tile = lambda a, f: np.repeat(a.reshape(f, 1, P), n[2], axis=1).ravel()
    st = tile(np.concatenate([0.01 * rng.standard_normal(P), 0.03 * rng.standard_normal(3 * P)]), 4)
    so = tile(np.concatenate([0.01 * rng.standard_normal(P), 0.03 * rng.standard_normal(3 * P)]), 4)
    kap = tile(np.abs(rng.standard_normal(P)), 1)
    us = tile(0.01 * rng.standard_normal(3 * P), 3)
    lam = tile(0.1 * rng.standard_normal(4 * P), 4)
    out = cpu(plan.step(st, kap, us)).reshape(4, n[2], P)
    assert np.array_equal(out, np.broadcast_to(out[:, :1], out.shape))
    lp, kb, ub = (cpu(t) for t in plan.step_adjoint(st, so, kap, us, lam))
    for v, f in ((lp, 4), (kb, 1), (ub, 3)):
        v = v.reshape(f, n[2], P)
        assert np.array_equal(v, np.broadcast_to(v[:, :1], v.shape)), f


@pytest.mark.parametrize("prec", [0, 1])
def test_zsegment_length_does_not_change_the_fields(prec):
    """D3Q15: the z-segment length (how the column tiles cut the march) does
    not change the final state or the gradients, bitwise (phi = 0, so the
    adjoint seed does not depend on the summed mean); J differs only by the
    grouping of its FP64 sums."""
    lks = lk()
    p = prob3d(prec=prec, phi=0.0)
    gamma, chi, psi = rand_inputs(p, 31)
    outs = []
    for zseg in (0, 4, 7):
        plan = lks.Plan(p)
        if zseg:
            plan.set_zseg(zseg)
        J3, fin = plan.forward(gamma, chi, psi, want_final=True)
        g = plan.adjoint(gamma, chi, psi)
        outs.append((cpu(J3)[0], cpu(fin), [cpu(g[k]) for k in ("dgamma", "dchi", "dpsi")]))
    for J, fin, gr in outs[1:]:
        assert abs(J - outs[0][0]) <= 1e-13 * abs(outs[0][0])
        assert np.array_equal(fin, outs[0][1])
        for a, b in zip(gr, outs[0][2]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_translation_moves_the_fields_bitwise(prec, scheme):
    """D3Q15 in a periodic box: moving the body, the target and the start
    state by whole nodes (3, 2, 2) puts every node at another place in its
    tile and segment; in FP32 the final state moves with them bitwise and
    the gradients are bitwise unchanged (phi = 0; J differs only by the
    grouping of its FP64 sums); in FP64, whose transfer weights come from
    absolute positions, they agree to rounding.  Both reverse sweeps (the
    exact adjoint and the ALKS)."""
    lks = lk()
    n = (34, 18, 20)
    d = (3, 2, 2)  # the target box stays inside the grid (it is clipped, not wrapped)
    base = prob3d(n=n, prec=prec, bc=(0, 0, 0), phi=0.0, scheme=scheme)
    moved = base.replace(
        xg_min=tuple(a + b for a, b in zip(base.xg_min, d)),
        xg_max=tuple(a + b for a, b in zip(base.xg_max, d)),
        tgt_lo=tuple(a + b for a, b in zip(base.tgt_lo, d)),
        tgt_hi=tuple(a + b for a, b in zip(base.tgt_hi, d)))
    gamma, chi, psi = rand_inputs(base, 41)
    s0 = gpu_state(rand_state(base, 42), base)
    roll = lambda v: np.roll(v.reshape(4, n[2], n[1], n[0]), shift=(d[2], d[1], d[0]),
                             axis=(1, 2, 3)).ravel()
    outs = []
    for p, st in ((base, s0), (moved, roll(s0))):
        plan = lks.Plan(p)
        J3, fin = plan.forward(gamma, chi, psi, state0=st, want_final=True)
        g = plan.adjoint(gamma, chi, psi)
        outs.append((cpu(J3)[0], cpu(fin), [cpu(g[k]) for k in ("dgamma", "dchi", "dpsi")]))
    (J0, f0, g0), (J1, f1, g1) = outs
    assert abs(J1 - J0) <= 1e-12 * abs(J0)
    if prec == 0:
        assert np.array_equal(f1, roll(f0))
        for a, b in zip(g1, g0):
            assert np.array_equal(a, b)
    else:
        # FP64 forms the transfer weights from absolute positions, so the
        # moved body's weights differ in their last bits
        assert relerr(f1, roll(f0)) < 1e-13
        for a, b in zip(g1, g0):
            assert relerr(a, b) < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_translation_moves_the_fields_bitwise_2d(prec):
    """D2Q9 in a periodic box, moved by whole nodes (5, 3): as the 3D check,
    every node sits elsewhere in its 32 x 8 (forward) and 32 x 16 (adjoint)
    tile; FP32 bitwise, FP64 to rounding."""
    lks = lk()
    n = (45, 21)
    d = (5, 3)
    base = prob2d(n, prec, bc=(0, 0, 0), phi=0.0, tgt_lo=(20, 2, 0), tgt_hi=(24, 17, 1))
    moved = base.replace(
        xg_min=(base.xg_min[0] + d[0], base.xg_min[1] + d[1], 0.0),
        xg_max=(base.xg_max[0] + d[0], base.xg_max[1] + d[1], 0.0),
        tgt_lo=(20 + d[0], 2 + d[1], 0), tgt_hi=(24 + d[0], 17 + d[1], 1))
    gamma, chi, psi = rand_inputs(base, 43)
    s0 = gpu_state(rand_state(base, 44), base)
    roll = lambda v: np.roll(v.reshape(3, n[1], n[0]), shift=(d[1], d[0]), axis=(1, 2)).ravel()
    outs = []
    for p, st in ((base, s0), (moved, roll(s0))):
        plan = lks.Plan(p)
        J3, fin = plan.forward(gamma, chi, psi, state0=st, want_final=True)
        g = plan.adjoint(gamma, chi, psi)
        outs.append((cpu(J3)[0], cpu(fin), [cpu(g[k]) for k in ("dgamma", "dchi", "dpsi")]))
    (J0, f0, g0), (J1, f1, g1) = outs
    assert abs(J1 - J0) <= 1e-12 * abs(J0)
    if prec == 0:
        assert np.array_equal(f1, roll(f0))
        for a, b in zip(g1, g0):
            assert np.array_equal(a, b)
    else:
        assert relerr(f1, roll(f0)) < 1e-13
        for a, b in zip(g1, g0):
            assert relerr(a, b) < 1e-12


def test_domain_error_before_march():
    """A body whose support reaches a wall node is rejected (LKS_EDOMAIN)."""
    lks = lk()
    p = prob2d((45, 21), 1, xg_min=(22.0, 2.0, 0.0), xg_max=(23.0, 3.0, 0.0))
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 16)
    with pytest.raises(lks.LksError) as e:
        plan.forward(gamma, chi, psi)
    assert e.value.status == lks.LKS_EDOMAIN


def test_instability_reported():
    """|u| >= 0.5 (or a non-finite value) anywhere in the march is reported as
    LKS_EUNSTABLE.  Forced from the host: a uniform initial flow at 0.6 is an
    exact solution, so every step carries it and trips the check."""
    lks = lk()
    p = prob2d((45, 21), 1, bc=(0, 0, 0), kappa_max=0.0, nt=3, ckpt_k=3)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 16)
    s0 = np.zeros((p.d + 1) * p.N)
    s0[p.N:2 * p.N] = 0.6
    with pytest.raises(lks.LksError) as e:
        plan.forward(gamma, chi, psi, state0=s0)
    assert e.value.status == lks.LKS_EUNSTABLE


def test_autograd_function(orc):
    """LKSObjective: torch.autograd backward equals the oracle adjoint."""
    lks = lk()
    p = prob2d((45, 21), 1)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 17)
    tg = torch.tensor(gamma, device="cuda", requires_grad=True)
    tc = torch.tensor(chi, device="cuda", requires_grad=True)
    tp = torch.tensor(psi, device="cuda", requires_grad=True)
    J = lks.LKSObjective.apply(tg, tc, tp, plan)
    (2.0 * J).backward()
    adj = orc.adjoint(p, gamma, chi, psi, dJ=2.0)
    assert l2err(cpu(tg.grad), adj["dgamma"]) < 1e-9
    assert l2err(cpu(tc.grad), adj["dchi"]) < 1e-9
    assert l2err(cpu(tp.grad), adj["dpsi"]) < 1e-9


def test_autograd_two_applies_on_one_plan(orc):
    """(J(x) - J(y)).backward() with both applies on one plan: the second
    march overwrites the first one's checkpoints, so the first backward
    marches again for its own inputs.  Both gradients match the oracle."""
    lks = lk()
    p = prob2d((45, 21), 1)
    plan = lks.Plan(p)
    gx, cx, px = rand_inputs(p, 41)
    gy, cy, py = rand_inputs(p, 42)
    t = [torch.tensor(v, device="cuda", requires_grad=True) for v in (gx, cx, px, gy, cy, py)]
    Jx = lks.LKSObjective.apply(t[0], t[1], t[2], plan)
    Jy = lks.LKSObjective.apply(t[3], t[4], t[5], plan)
    (Jx - Jy).backward()
    ax = orc.adjoint(p, gx, cx, px)
    ay = orc.adjoint(p, gy, cy, py, dJ=-1.0)
    for k, key in enumerate(("dgamma", "dchi", "dpsi")):
        assert l2err(cpu(t[k].grad), ax[key]) < 1e-9, key
        assert l2err(cpu(t[3 + k].grad), ay[key]) < 1e-9, key
    # a plain forward in between is caught the same way
    t2 = [torch.tensor(v, device="cuda", requires_grad=True) for v in (gx, cx, px)]
    J = lks.LKSObjective.apply(t2[0], t2[1], t2[2], plan)
    plan.forward(gy, cy, py)
    J.backward()
    assert l2err(cpu(t2[0].grad), ax["dgamma"]) < 1e-9


def test_adjoint_refuses_other_inputs():
    """lks_adjoint reverses the last forward march: called with a gamma, chi
    or psi that differs from that march's, it returns LKS_EINVAL and
    launches nothing."""
    lks = lk()
    p = prob2d((45, 21), 1)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 43)
    plan.forward(gamma, chi, psi)
    for k in range(3):
        args = [gamma.copy(), chi.copy(), psi.copy()]
        args[k].flat[0] += 1e-3
        with pytest.raises(lks.LksError) as e:
            plan.adjoint(*args)
        assert e.value.status == lks.LKS_EINVAL
    g = plan.adjoint(gamma, chi, psi)
    assert np.abs(cpu(g["dgamma"])).max() > 0


def test_long_segment_transposes_in_chunks():
    """A segment longer than the 256 steps whose map transposes share one
    launch is reversed in chunks; one segment (K = nt) keeps every state, so
    the reverse sweep recomputes nothing.  Both give the gradients of a
    short-segment run bit for bit, alone and batched."""
    lks = lk()
    p0 = prob2d((45, 21), 0, nt=600, r_t=20, r_w=20)
    gamma, chi, psi = rand_inputs(p0, 44)
    outs = []
    for K in (77, 300, 600):
        plan = lks.Plan(p0.replace(ckpt_k=K))
        J3, _ = plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi)
        outs.append((cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
        del plan
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    specs = [p0.replace(ckpt_k=600), p0.replace(ckpt_k=600, n=(37, 21, 1), tgt_lo=(16, 1, 0),
                                                  tgt_hi=(20, 20, 1))]
    b = lks.Batch([lks.Plan(q) for q in specs])
    out = b.run([gamma] * 2, [chi] * 2, [psi] * 2)
    assert np.array_equal(cpu(out[0][0]), outs[0][0])
    assert np.array_equal(cpu(out[0][1]["dgamma"]), outs[0][1])
    solo = lks.Plan(specs[1])
    J3, _ = solo.forward(gamma, chi, psi)
    g = solo.adjoint(gamma, chi, psi)
    assert np.array_equal(cpu(out[1][0]), cpu(J3))
    assert np.array_equal(cpu(out[1][1]["dpsi"]), cpu(g["dpsi"]))


def test_reproducible_bitwise():
    """Two identical runs give bit-identical objective and gradients."""
    lks = lk()
    p = prob3d((34, 18, 20), 0)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 18)
    res = []
    for _ in range(2):
        J3, _ = plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi)
        res.append((cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"])))
    for a, b in zip(*res):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["2d_walls_y", "3d_shift_xy"])
def test_graph_replay_matches_eager(name):
    """Time loops replayed from captured hipGraphs equal eager launches bit for
    bit, on repeated replays with eager work in between and after the inputs
    change (per-step data come from device tables, not baked arguments)."""
    lks = lk()
    p = PROBS[name](0)
    eager = lks.Plan(p)
    eager.set_graphs(False)
    graph = lks.Plan(p)
    inputs = [rand_inputs(p, 21), rand_inputs(p, 22), rand_inputs(p, 21)]
    for k, (gamma, chi, psi) in enumerate(inputs):
        J_e, fin_e = eager.forward(gamma, chi, psi, want_final=True)
        g_e = eager.adjoint(gamma, chi, psi, want_initial=True)
        ref = [cpu(J_e), cpu(fin_e), cpu(g_e["dgamma"]), cpu(g_e["dchi"]), cpu(g_e["dpsi"]),
               cpu(g_e["adj_initial"])]
        for rep in range(2):
            J_g, fin_g = graph.forward(gamma, chi, psi, want_final=True)
            torch.zeros(1000, device="cuda").sum().item()  # eager work between replays
            g_g = graph.adjoint(gamma, chi, psi, want_initial=True)
            got = [cpu(J_g), cpu(fin_g), cpu(g_g["dgamma"]), cpu(g_g["dchi"]), cpu(g_g["dpsi"]),
                   cpu(g_g["adj_initial"])]
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (k, rep)


def test_batch_run_matches_solo_runs(orc):
    """Uneven independent instances in one captured graph give the solo results
    bitwise (same kernels, same order per instance), and the first instance
    also matches the oracle; a second call replays the graph."""
    lks = lk()
    specs = [
        W.make_2d(40, 12, 24, 3, nu=0.1, seed=11, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=7),
        W.make_2d(53, 16, 24, 5, nu=0.08, seed=12, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=7),
        W.make_2d(37, 10, 24, 1, nu=0.12, seed=13, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=7, ny=29),
    ]
    solo = []
    for p, g, c, s in specs:
        pl = lks.Plan(p)
        J3, _ = pl.forward(g, c, s)
        gr = pl.adjoint(g, c, s)
        solo.append((cpu(J3), {k: cpu(gr[k]) for k in ("dgamma", "dchi", "dpsi")}))
    plans = [lks.Plan(p) for p, *_ in specs]
    b = lks.Batch(plans)
    for call in range(2):
        out = b.run([x[1] for x in specs], [x[2] for x in specs], [x[3] for x in specs])
        for k, (J3, gr) in enumerate(out):
            assert np.array_equal(cpu(J3), solo[k][0]), (call, k)
            for key in ("dgamma", "dchi", "dpsi"):
                assert np.array_equal(cpu(gr[key]), solo[k][1][key]), (call, k, key)
    p, g, c, s = specs[0]
    ref = orc.forward(p, g, c, s, want_final=False)
    assert abs(solo[0][0][0] - ref["J"]) <= 1e-5 * abs(ref["J"])
    adj = orc.adjoint(p, g, c, s)
    assert l2err(solo[0][1]["dgamma"], adj["dgamma"]) < 1e-3


def test_batch_run_unequal_instances_use_graph_branches():
    """Instances with different step counts (or a 3D one) cannot share
    launches; they run as graph branches and still match their solo runs."""
    lks = lk()
    specs = [
        W.make_2d(40, 12, 20, 3, nu=0.1, seed=21, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=6),
        W.make_2d(45, 12, 26, 3, nu=0.1, seed=22, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=6),
    ]
    p3 = prob3d(prec=0)
    rng = np.random.default_rng(5)
    specs.append((p3, rng.uniform(0.2, 0.8, size=p3.M), rng.uniform(0.3, 0.7, size=(p3.nt, 3)),
                  rng.uniform(0.3, 0.7, size=p3.nt)))
    solo = []
    for p, g, c, s in specs:
        pl = lks.Plan(p)
        J3, _ = pl.forward(g, c, s)
        gr = pl.adjoint(g, c, s)
        solo.append((cpu(J3), cpu(gr["dgamma"]), cpu(gr["dpsi"])))
    b = lks.Batch([lks.Plan(p) for p, *_ in specs])
    out = b.run([x[1] for x in specs], [x[2] for x in specs], [x[3] for x in specs])
    for k, (J3, gr) in enumerate(out):
        assert np.array_equal(cpu(J3), solo[k][0]), k
        assert np.array_equal(cpu(gr["dgamma"]), solo[k][1]), k
        assert np.array_equal(cpu(gr["dpsi"]), solo[k][2]), k


# ----------------------------------------------------------------------------
# The benchmark workload at full size: D3Q15 128^3, design 64^3 + margin 4,
# FP32 state, the plan the benchmark builds (z segments, tile origin, body box
# sized over all 5000 steps).  The oracle finishes single full-grid stages in
# seconds, so these compare every node.

@pytest.fixture(scope="module")
def c4_full(orc):
    p, gamma, chi, psi = W.c4()
    mot = orc.motion(p, chi, psi)
    kref = orc.kappa_ref(p, gamma)
    return p, gamma, chi, psi, mot, kref


def test_c4_full_size_map_and_step(orc, c4_full):
    p, gamma, chi, psi, mot, kref = c4_full
    plan = lk().Plan(p)
    for n in (1, 1250, 2500):  # rotation 0, about pi/2 and about pi
        m8 = mot[n - 1]
        k, us = plan.map(kref, m8)
        ko, uo = orc.map_fields(p, kref, m8)
        assert relerr(cpu(k), ko) < 2e-6, n
        assert relerr(cpu(us), uo) < 2e-6, n
    rng = np.random.default_rng(41)
    s = rand_state(p, 42, amp=0.03)
    out = cpu(plan.step(gpu_state(s, p), ko, uo))
    ref = orc.step(p, s, ko, uo)
    assert relerr(out[: p.N], ref[: p.N] - THIRD) < 2e-5
    assert relerr(out[p.N:], ref[p.N:]) < 2e-6
    lam = rng.standard_normal((p.d + 1) * p.N)
    lp, kb, ub = plan.step_adjoint(gpu_state(s, p), gpu_state(ref, p), ko, uo, lam)
    rlp, rkb, rub = orc.step_adjoint(p, s, ref, ko, uo, lam)
    assert relerr(cpu(lp), rlp) < 2e-5
    assert relerr(cpu(kb), rkb) < 2e-5
    assert relerr(cpu(ub), rub) < 2e-5
    kbm, mbm = plan.map_adjoint(kref, m8, rkb, rub)
    rkbm, rmbm = orc.map_adjoint(p, kref, m8, rkb, rub)
    assert relerr(cpu(kbm), rkbm) < 2e-5
    assert relerr(cpu(mbm), rmbm) < 1e-4


@pytest.mark.parametrize("scheme", [0, 1])
def test_c4_full_size_forward_adjoint_first_steps(orc, c4_full, scheme):
    """Forward + reverse sweep (exact adjoint, and the ALKS) through
    lks_forward / lks_adjoint on the full FP32 grid for the run's first two
    steps (checkpoint every step), against the oracle.  A random start state
    and a target over the whole interior make J and all three gradients
    depend on the body within two steps."""
    p, gamma, chi, psi, _, _ = c4_full
    p2 = p.replace(nt=2, ckpt_k=1, scheme=scheme, tgt_lo=(1, 1, 0), tgt_hi=(127, 127, 128))
    s0 = rand_state(p2, 61, amp=0.02)
    plan = lk().Plan(p2)
    J3, _ = plan.forward(gamma, chi[:2], psi[:2], state0=gpu_state(s0, p2))
    g = plan.adjoint(gamma, chi[:2], psi[:2])
    ref = orc.forward(p2, gamma, chi[:2], psi[:2], state0=s0, want_final=False)
    if scheme == 0:
        adj = orc.adjoint(p2, gamma, chi[:2], psi[:2], state0=s0)
    else:
        adj = orc.alks_adjoint(p2, gamma, chi[:2], psi[:2], state0=s0)
    assert abs(cpu(J3)[0] - ref["J"]) <= 1e-5 * abs(ref["J"])
    for k in ("dgamma", "dchi", "dpsi"):
        assert np.linalg.norm(adj[k]) > 0, k
        assert l2err(cpu(g[k]), adj[k]) < 1e-3, k


def test_fp32_objective_over_a_long_horizon():
    """FP32 state with FP64 sums keeps J1 within 1e-5 of the FP64 path over
    thousands of steps: the FP32 lattice constants make the pressure and
    velocity pass-through sums exactly 1, so no per-step gain compounds."""
    lks = lk()
    Js = []
    for prec in (1, 0):
        p, g, c, s = W.make_2d(64, 32, 3000, 200, nu=0.06, seed=31, precision=prec, ckpt_k=300)
        plan = lks.Plan(p)
        J3, _ = plan.forward(g, c, s)
        Js.append(cpu(J3)[0])
    assert abs(Js[1] - Js[0]) <= 1e-5 * abs(Js[0]), Js


# ----------------------------------------------------------------------------
# The D2Q9 workloads at full size: 512^2 (256^2 design, 20000 steps) and
# 1024^2 (512^2 design, 10000 steps), in the plans their own problem
# statements build (checkpoint interval, body box, motion bounds).

@pytest.mark.parametrize("cfg", ["c2", "c3"])
def test_d2q9_full_size_first_steps(orc, cfg):
    """The first two steps of the workload's motion through lks_forward /
    lks_adjoint on every node, FP64 and FP32, against the oracle.  A random
    start state and a target over the whole interior make the objective and
    all three gradients depend on the body within two steps."""
    p, gamma, chi, psi = getattr(W, cfg)()
    nx, ny = p.n[0], p.n[1]
    p2 = p.replace(nt=2, ckpt_k=1, precision=1, tgt_lo=(0, 1, 0), tgt_hi=(nx, ny - 1, 1),
                   phi=0.1)
    s0 = rand_state(p2, 51, amp=0.02)
    ref = orc.forward(p2, gamma, chi[:2], psi[:2], state0=s0, want_final=False)
    adj = orc.adjoint(p2, gamma, chi[:2], psi[:2], state0=s0)
    for prec in (1, 0):
        pp = p2.replace(precision=prec)
        plan = lk().Plan(pp)
        J3, _ = plan.forward(gamma, chi[:2], psi[:2], state0=gpu_state(s0, pp))
        g = plan.adjoint(gamma, chi[:2], psi[:2])
        tj, tg = (1e-10, 1e-9) if prec == 1 else (1e-5, 1e-3)
        assert abs(cpu(J3)[0] - ref["J"]) <= tj * abs(ref["J"]), prec
        for k in ("dgamma", "dchi", "dpsi"):
            assert np.linalg.norm(adj[k]) > 0, k
            assert l2err(cpu(g[k]), adj[k]) < tg, (prec, k)


def test_c2_fp32_against_fp64_full_horizon():
    """512^2, 20000 steps from rest, forward + adjoint: the FP32 state with
    FP64 sums against the FP64 plain form (objective within 1e-5, gradients
    within 1e-3)."""
    out = {}
    for prec in (1, 0):
        p, gamma, chi, psi = W.c2(precision=prec)
        plan = lk().Plan(p)
        J3, _ = plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi)
        out[prec] = (cpu(J3)[0], {k: cpu(g[k]) for k in ("dgamma", "dchi", "dpsi")})
        del plan
    J64, g64 = out[1]
    J32, g32 = out[0]
    assert abs(J32 - J64) <= 1e-5 * abs(J64), (J32, J64)
    for k in g64:
        assert l2err(g32[k], g64[k]) < 1e-3, k


@pytest.mark.timeout(900)  # the oracle's 10000-step adjoint takes about 90 s
def test_c3_crop_gradient_through_autograd(orc):
    """The 1024^2 workload's gradient check: a 64^2 crop (the centre 32^2 of its
    generated design field, the same chi, psi, nu and kappa_max, 10000 steps)
    through torch.autograd with checkpoints every K in {50, 100, 200}, FP32
    state, against the oracle."""
    lks = lk()
    p3, gamma3, chi, psi = W.c3()
    g2 = gamma3.reshape(p3.m[1], p3.m[0])
    c0 = p3.m[0] // 2 - 16
    gamma = g2[c0:c0 + 32, c0:c0 + 32].ravel().copy()
    p, *_ = W.make_2d(64, 32, p3.nt, p3.r_t, nu=p3.nu, seed=2, kappa_max=p3.kappa_max,
                      precision=0)
    ref = orc.forward(p.replace(precision=1), gamma, chi, psi, want_final=False)
    adj = orc.adjoint(p.replace(precision=1), gamma, chi, psi)
    grads = []
    for K in (50, 100, 200):
        plan = lks.Plan(p.replace(ckpt_k=K))
        tg = torch.tensor(gamma, device="cuda", requires_grad=True)
        tc = torch.tensor(chi, device="cuda", requires_grad=True)
        tp = torch.tensor(psi, device="cuda", requires_grad=True)
        J = lks.LKSObjective.apply(tg, tc, tp, plan)
        J.backward()
        assert abs(float(J.detach()) - ref["J"]) <= 1e-5 * abs(ref["J"]), K
        grads.append([cpu(tg.grad), cpu(tc.grad), cpu(tp.grad)])
        for a, k in zip(grads[-1], ("dgamma", "dchi", "dpsi")):
            assert l2err(a, adj[k]) < 1e-3, (K, k)
    for gk in grads[1:]:
        for a, b in zip(gk, grads[0]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("d", [2, 3])
def test_gpu_gradient_against_central_differences(d):
    """On the GPU alone, FP64: central differences (h = 1e-6) of J from
    lks_forward on 8 design entries and 8 motion entries agree with
    lks_adjoint's gradient (the paper's verification method, Appendix A)."""
    lks = lk()
    p = prob2d((45, 21), 1, nt=12) if d == 2 else prob3d(prec=1)
    plan = lks.Plan(p)
    gamma, chi, psi = rand_inputs(p, 61)
    plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi)
    dg, dc, dp = cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])
    J = lambda ga, ch, ps: cpu(plan.forward(ga, ch, ps)[0])[0]
    rng = np.random.default_rng(62)
    h = 1e-6
    gmax = max(np.abs(dg).max(), 1e-300)
    for j in rng.choice(p.M, 8, replace=False):
        gp, gm = gamma.copy(), gamma.copy()
        gp[j] += h
        gm[j] -= h
        fd = (J(gp, chi, psi) - J(gm, chi, psi)) / (2 * h)
        assert abs(fd - dg[j]) < 1e-6 * max(abs(fd), 1e-2 * gmax), (j, fd, dg[j])
    cmax = max(np.abs(dc).max(), np.abs(dp).max())
    for j in range(8):
        t = int(rng.integers(p.nt))
        comp = j % 4 if d == 3 else (0, 1, 3)[j % 3]
        if comp < 3:
            cp, cm = chi.copy(), chi.copy()
            cp[t, comp] += h
            cm[t, comp] -= h
            fd = (J(gamma, cp, psi) - J(gamma, cm, psi)) / (2 * h)
            ad = dc[t, comp]
        else:
            pp, pm = psi.copy(), psi.copy()
            pp[t] += h
            pm[t] -= h
            fd = (J(gamma, chi, pp) - J(gamma, chi, pm)) / (2 * h)
            ad = dp[t]
        assert abs(fd - ad) < 1e-6 * max(abs(fd), 1e-2 * cmax), (t, comp, fd, ad)


def test_c1_gradient_against_central_differences():
    """The paper's verification (Appendix A) on the 64x64 / 200-step workload
    itself, FP64 on the GPU: central differences of J (h = 1e-6) on 8 random
    design entries and 8 random motion entries (x, y, theta at random steps)
    agree with lks_adjoint's gradient to 1e-6, with checkpoints every 50 steps."""
    lks = lk()
    p, gamma, chi, psi = W.c1(precision=1)
    gamma = gamma.ravel().copy()
    plan = lks.Plan(p.replace(ckpt_k=50))
    plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi)
    dg, dc, dp = cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])
    J = lambda ga, ch, ps: cpu(plan.forward(ga, ch, ps)[0])[0]
    rng = np.random.default_rng(2026)
    h = 1e-6
    gmax = np.abs(dg).max()
    assert gmax > 0
    for j in rng.choice(p.M, 8, replace=False):
        gp, gm = gamma.copy(), gamma.copy()
        gp[j] += h
        gm[j] -= h
        fd = (J(gp, chi, psi) - J(gm, chi, psi)) / (2 * h)
        assert abs(fd - dg[j]) < 1e-6 * max(abs(fd), 1e-2 * gmax), (j, fd, dg[j])
    cmax = max(np.abs(dc).max(), np.abs(dp).max())
    assert cmax > 0
    for j in range(8):
        t = int(rng.integers(p.nt))
        comp = (0, 1, 3)[j % 3]
        if comp < 3:
            cp, cm = chi.copy(), chi.copy()
            cp[t, comp] += h
            cm[t, comp] -= h
            fd = (J(gamma, cp, psi) - J(gamma, cm, psi)) / (2 * h)
            ad = dc[t, comp]
        else:
            pp, pm = psi.copy(), psi.copy()
            pp[t] += h
            pm[t] -= h
            fd = (J(gamma, chi, pp) - J(gamma, chi, pm)) / (2 * h)
            ad = dp[t]
        assert abs(fd - ad) < 1e-6 * max(abs(fd), 1e-2 * cmax), (t, comp, fd, ad)
