"""GPU parity of the general 3D rotation (three Euler angles, lks_problem.rot
= LKS_ROT_EULER) against the oracle (pinned in test_oracle_rot3.py), through
the C ABI: the motion prelude, the transfer and its transpose at several
angle sets (quarter turns included), whole forward + adjoint runs (both
reverse sweeps), the reduction to the rotation about z, checkpoint and
body-tape invariance, and the constraints.  FP64: 1e-12 per stage, 1e-10 on
J and 1e-9 on gradients per run; FP32 state with FP64 sums: 2e-5 per stage,
J within 1e-5 and gradients within 1e-3."""
import math

import numpy as np
import pytest

from test_gpu_parity import cpu, l2err, lk, oracle_state, prob3d, relerr

pytestmark = pytest.mark.gpu


def rot3(n=(36, 34, 30), prec=1, **kw):
    base = dict(rot=1, tilt_min=(-0.35, -0.3), tilt_max=(0.3, 0.4), m=(6, 5, 5), margin=3,
                xg_min=(n[0] / 2 - 1.0, n[1] / 2 - 0.5, n[2] / 2 - 1.0),
                xg_max=(n[0] / 2 + 1.0, n[1] / 2 + 0.5, n[2] / 2 + 1.0),
                tgt_lo=(4, 4, 2), tgt_hi=(n[0] - 4, n[1] - 4, 6))
    base.update(kw)
    return prob3d(n, prec, **base)


# z extents fit any rotation of the design block (its support must not
# exceed a periodic extent), x and y keep it clear of the walls
PROBS3 = {
    "walls_xy": lambda prec: rot3((36, 34, 30), prec),
    "ragged": lambda prec: rot3((33, 31, 29), prec, m=(5, 4, 6), tgt_lo=(3, 3, 1),
                                tgt_hi=(30, 28, 4), ckpt_k=5),
}


def inputs3(p, seed):
    rng = np.random.default_rng(seed)
    gamma = rng.uniform(0.05, 0.95, size=p.M)
    chi = rng.uniform(0.3, 0.7, size=(p.nt, 3))
    psi = rng.uniform(0.2, 0.8, size=(p.nt, 3))
    return gamma, chi, psi


ANGLES = [(0.0, 0.0, 0.0), (0.31, -0.22, 0.77), (-0.9, 0.4, 2.1), (math.pi / 2, 0.0, 0.0),
          (0.0, -math.pi / 2, 0.3)]


@pytest.mark.parametrize("prec", [1, 0])
def test_rot3_motion_and_transfer(orc, prec):
    p = PROBS3["walls_xy"](prec)
    plan = lk().Plan(p)
    gamma, chi, psi = inputs3(p, 1)
    m = cpu(plan.motion(chi, psi))
    assert m.shape == (p.nt, 12)
    assert relerr(m, orc.motion(p, chi, psi)) < 1e-14
    rng = np.random.default_rng(2)
    kref = rng.uniform(0, 50, size=p.Mtot)
    tol = 1e-12 if prec == 1 else 2e-6
    for th in ANGLES:
        mot = np.array([p.n[0] / 2 + 0.37, p.n[1] / 2 - 0.21, p.n[2] / 2 + 0.13,
                        0.02, -0.01, 0.005, *th, 0.003, -0.002, 0.004])
        k, us = plan.map(kref, mot)
        ko, uo = orc.map_fields(p, kref, mot)
        assert relerr(cpu(k), ko) < tol, th
        assert relerr(cpu(us), uo) < tol, th


@pytest.mark.parametrize("prec", [1, 0])
def test_rot3_transfer_transpose(orc, prec):
    p = PROBS3["walls_xy"](prec)
    plan = lk().Plan(p)
    rng = np.random.default_rng(8)
    kref = rng.uniform(0, 50, size=p.Mtot)
    kbar = rng.standard_normal(p.N)
    usbar = rng.standard_normal(p.d * p.N)
    n = p.n
    idx = np.arange(p.N)
    x, y = idx % n[0], (idx // n[0]) % n[1]
    wall = (x == 0) | (x == n[0] - 1) | (y == 0) | (y == n[1] - 1)
    kbar[wall] = 0
    usbar.reshape(3, p.N)[:, wall] = 0
    tol = 1e-12 if prec == 1 else 2e-5
    for th in ANGLES:
        mot = np.array([p.n[0] / 2 - 0.3, p.n[1] / 2 + 0.2, p.n[2] / 2 - 0.4,
                        0.01, 0.02, 0.01, *th, 0.004, -0.003, 0.002])
        kb, mb = plan.map_adjoint(kref, mot, kbar, usbar)
        rkb, rmb = orc.map_adjoint(p, kref, mot, kbar, usbar)
        assert mb.numel() == 12
        assert relerr(cpu(kb), rkb) < tol, th
        assert relerr(cpu(mb), rmb) < (1e-11 if prec == 1 else 1e-4), th


@pytest.mark.parametrize("name", sorted(PROBS3))
@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("scheme", [0, 1])
def test_rot3_forward_adjoint_run(orc, name, prec, scheme):
    p = PROBS3[name](prec).replace(scheme=scheme)
    print(f"rot3 run {name} prec={prec} scheme={scheme} n={p.n}", flush=True)
    plan = lk().Plan(p)
    gamma, chi, psi = inputs3(p, 9)
    J3, fin = plan.forward(gamma, chi, psi, want_final=True)
    g = plan.adjoint(gamma, chi, psi)
    ref = orc.forward(p, gamma, chi, psi)
    adj = (orc.alks_adjoint if scheme else orc.adjoint)(p, gamma, chi, psi)
    J = cpu(J3)
    assert cpu(g["dpsi"]).shape == (p.nt, 3)
    for k in ("dgamma", "dchi", "dpsi"):
        assert np.linalg.norm(adj[k]) > 0, k
    if prec == 1:
        assert abs(J[0] - ref["J"]) <= 1e-10 * abs(ref["J"])
        assert relerr(oracle_state(cpu(fin), p), ref["final"]) < 1e-10
        for k in ("dgamma", "dchi", "dpsi"):
            assert l2err(cpu(g[k]), adj[k]) < 1e-9, k
    else:
        assert abs(J[0] - ref["J"]) <= 1e-5 * abs(ref["J"])
        for k in ("dgamma", "dchi", "dpsi"):
            assert l2err(cpu(g[k]), adj[k]) < 1e-3, k


def test_rot3_reduces_to_rotation_about_z():
    """Zero tilt ranges: the three-angle path (its own map, transpose and
    epilogue) gives the rotation-about-z path's objective and gradients."""
    lks = lk()
    pz = prob3d((34, 18, 20), 1)
    p3 = pz.replace(rot=1, tilt_min=(0.0, 0.0), tilt_max=(0.0, 0.0))
    gamma, chi, psi3 = inputs3(p3, 4)
    outs = []
    for p, psi in ((pz, psi3[:, 2].copy()), (p3, psi3)):
        plan = lks.Plan(p)
        J3, _ = plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi)
        outs.append((cpu(J3)[0], cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
    (Jz, gz, cz, pzv), (J3v, g3, c3, p3v) = outs
    assert abs(J3v - Jz) <= 1e-12 * abs(Jz)
    assert l2err(g3, gz) < 1e-11 and l2err(c3, cz) < 1e-11
    assert l2err(p3v[:, 2], pzv) < 1e-11
    assert np.all(p3v[:, :2] == 0)


def test_rot3_checkpoint_and_body_tape_do_not_change_gradients():
    p0 = PROBS3["walls_xy"](0).replace(nt=9)
    gamma, chi, psi = inputs3(p0, 10)
    outs = []
    for K in (2, 4, 9):
        for tape in (-1, 1):
            plan = lk().Plan(p0.replace(ckpt_k=K, body_tape=tape))
            J3, _ = plan.forward(gamma, chi, psi)
            g = plan.adjoint(gamma, chi, psi)
            outs.append((cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_rot3_constraints(orc):
    p = PROBS3["walls_xy"](1)
    plan = lk().Plan(p)
    rng = np.random.default_rng(5)
    phys = rng.uniform(0.0, 1.0, p.M)
    _, chi, psi = inputs3(p, 6)
    G, d1, d2, d3 = plan.constraints(phys, chi, psi, 0.7, 2e-2, 4.0)
    Gr, r1, r2, r3 = orc.constraints(p, phys, chi, psi, 0.7, 2e-2, 4.0)
    assert np.allclose(cpu(G), Gr, rtol=1e-13, atol=1e-15)
    assert cpu(d3).size == 3 * p.nt
    assert relerr(cpu(d3).ravel(), np.ravel(r3)) < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_rot3_translation_moves_the_fields(prec):
    """Three-angle rotation in a periodic box: body, target and start state
    moved by whole nodes (3, 2, 2) move the final state bitwise in FP32 and
    leave the design gradient bitwise unchanged (phi = 0).  The motion
    gradients are sums of per-block FP64 partials over grid tiles, which the
    move regroups, so they agree to FP64 rounding; FP64 state, whose transfer
    weights come from absolute positions, agrees to rounding throughout."""
    lks = lk()
    n = (36, 34, 30)
    d = (3, 2, 2)
    base = rot3(n, prec, bc=(0, 0, 0), phi=0.0)
    moved = base.replace(
        xg_min=tuple(a + b for a, b in zip(base.xg_min, d)),
        xg_max=tuple(a + b for a, b in zip(base.xg_max, d)),
        tgt_lo=tuple(a + b for a, b in zip(base.tgt_lo, d)),
        tgt_hi=tuple(a + b for a, b in zip(base.tgt_hi, d)))
    gamma, chi, psi = inputs3(base, 51)
    # halve the motion about the range midpoints: with the noisy start state
    # the full ranges carry this seed past the march's |u| < 0.5 limit
    chi, psi = 0.5 + 0.5 * (chi - 0.5), 0.5 + 0.5 * (psi - 0.5)
    rng = np.random.default_rng(52)
    s0 = np.concatenate([0.01 * rng.standard_normal(base.N), 0.03 * rng.standard_normal(3 * base.N)])
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
        assert np.array_equal(g1[0], g0[0])
        for a, b in zip(g1[1:], g0[1:]):
            assert relerr(a, b) < 1e-12
    else:
        assert relerr(f1, roll(f0)) < 1e-13
        for a, b in zip(g1, g0):
            assert relerr(a, b) < 1e-12
