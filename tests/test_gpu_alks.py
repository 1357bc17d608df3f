"""GPU parity of the paper-literal ALKS reverse sweep (Sec. 2.5, scheme = 1).

Every call goes through the C ABI.  The reference is the oracle's own ALKS
(pinned in test_oracle_alks.py), on the same seeded inputs.  Tolerances are
those of the exact adjoint: FP64 state to 1e-9 relative (summation order
only), FP32 state with FP64 sums to 1e-3 relative L2 on every gradient.
"""
import numpy as np
import pytest

from paper_2608_01071_amd import workloads as W

from test_gpu_parity import PROBS, cpu, l2err, lk, prob2d, rand_inputs, relerr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_alks_run_matches_oracle(orc, name, prec):
    """Whole ALKS runs (checkpoint K < nt, ragged segment, walls on one or
    two axes, 2D and 3D) against the oracle's ALKS."""
    p = PROBS[name](prec).replace(scheme=1)
    plan = lk().Plan(p)
    gamma, chi, psi = rand_inputs(p, 9)
    plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi, want_initial=True)
    ref = orc.alks_adjoint(p, gamma, chi, psi)
    tol = 1e-9 if prec == 1 else 1e-3
    for k in ("dgamma", "dchi", "dpsi"):
        assert l2err(cpu(g[k]), ref[k]) < tol, k
    if prec == 1:
        assert relerr(cpu(g["adj_initial"]), ref["adj_initial"]) < 1e-9


@pytest.mark.parametrize("prec", [1, 0])
def test_alks_c1_matches_oracle_and_departs_from_exact(orc, prec):
    """The 64x64 / 200-step workload: the GPU ALKS matches the oracle's ALKS,
    and like it departs from the exact gradient by a few percent."""
    p, gamma, chi, psi = W.c1(precision=prec)
    p = p.replace(ckpt_k=50, scheme=1)
    plan = lk().Plan(p)
    plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi)
    ref = orc.alks_adjoint(p, gamma, chi, psi)
    exact = orc.adjoint(p, gamma, chi, psi)
    tol = 1e-8 if prec == 1 else 1e-3
    for k in ("dgamma", "dchi", "dpsi"):
        assert l2err(cpu(g[k]), ref[k]) < tol, k
        assert 1e-3 < l2err(cpu(g[k]), exact[k]) < 0.1, k


def test_alks_without_body_equals_exact_adjoint():
    """gamma = 0 (kappa = 0 everywhere): on the GPU too the ALKS estimate of
    dJ/d(state0) equals the exact adjoint's."""
    p = prob2d((45, 21), 1)
    gamma, chi, psi = rand_inputs(p, 31)
    gamma[:] = 0.0
    out = []
    for scheme in (0, 1):
        plan = lk().Plan(p.replace(scheme=scheme))
        plan.forward(gamma, chi, psi)
        out.append(cpu(plan.adjoint(gamma, chi, psi, want_initial=True)["adj_initial"]))
    assert np.abs(out[0]).max() > 0
    assert relerr(out[1][: out[0].size], out[0]) < 1e-12


def test_alks_checkpoint_interval_does_not_change_gradients():
    """The raw-moment slots follow the adjoint state across segments: K in
    {1, 3, 7, nt} and both body-tape modes give bit-identical gradients."""
    p0 = prob2d((45, 21), 0, nt=14, scheme=1)
    gamma, chi, psi = rand_inputs(p0, 10)
    outs = []
    for K in (1, 3, 7, 14):
        for tape in (-1, 1):
            plan = lk().Plan(p0.replace(ckpt_k=K, body_tape=tape))
            plan.forward(gamma, chi, psi)
            g = plan.adjoint(gamma, chi, psi)
            outs.append((cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_alks_batch_matches_solo_runs(orc):
    """ALKS instances share the batched launches and give their solo results
    bitwise; the first matches the oracle's ALKS."""
    lks = lk()
    specs = [
        W.make_2d(40, 12, 24, 3, nu=0.1, seed=11, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=7),
        W.make_2d(53, 16, 24, 5, nu=0.08, seed=12, amp=0.5, sigma_n=0.05, th_amp=0.05,
                  precision=0, ckpt_k=7),
    ]
    specs = [(p.replace(scheme=1), g, c, s) for p, g, c, s in specs]
    solo = []
    for p, g, c, s in specs:
        pl = lks.Plan(p)
        pl.forward(g, c, s)
        gr = pl.adjoint(g, c, s)
        solo.append({k: cpu(gr[k]) for k in ("dgamma", "dchi", "dpsi")})
    b = lks.Batch([lks.Plan(p) for p, *_ in specs])
    out = b.run([x[1] for x in specs], [x[2] for x in specs], [x[3] for x in specs])
    for k, (_, gr) in enumerate(out):
        for key in ("dgamma", "dchi", "dpsi"):
            assert np.array_equal(cpu(gr[key]), solo[k][key]), (k, key)
    p, g, c, s = specs[0]
    ref = orc.alks_adjoint(p, g, c, s)
    for key in ("dgamma", "dchi", "dpsi"):
        assert l2err(solo[0][key], ref[key]) < 1e-3, key


@pytest.mark.parametrize("name", ["2d_walls_y", "2d_walls_xy_shift_x", "3d_shift_xy"])
@pytest.mark.parametrize("prec", [1, 0])
def test_alks_terminal_state_matches_oracle(orc, name, prec):
    """Periodic approximation with the ALKS (Algorithm 1): a run from a
    carried state (p~, u~, s~) at t1, whose adjoint equilibrium is formed
    with this run's velocity there, and its output: the dJ/d(state0)
    estimate and the ALKS state of level 0, against the oracle's ALKS from
    the same state.  The planes before the carried state are not read."""
    p = PROBS[name](prec).replace(scheme=1)
    plan = lk().Plan(p)
    gamma, chi, psi = rand_inputs(p, 13)
    size = orc.alks_state_size(p)
    assert plan.adj_state_size == size
    term = 1e-3 * np.random.default_rng(14).standard_normal(size)
    plan.forward(gamma, chi, psi)
    g = plan.adjoint(gamma, chi, psi, adj_terminal=term, want_initial=True)
    ref = orc.alks_adjoint(p, gamma, chi, psi, adj_terminal=term)
    tol = 1e-9 if prec == 1 else 1e-3
    for k in ("dgamma", "dchi", "dpsi"):
        assert l2err(cpu(g[k]), ref[k]) < tol, k
    ai = cpu(g["adj_initial"])
    assert ai.size == size
    if prec == 1:
        assert relerr(ai, ref["adj_initial"]) < 1e-9
    else:
        S = (p.d + 1) * p.N
        assert l2err(ai[S:], ref["adj_initial"][S:]) < 1e-4
    S = (p.d + 1) * p.N
    term[:S] = 0.0
    plan.forward(gamma, chi, psi)
    g2 = plan.adjoint(gamma, chi, psi, adj_terminal=term, want_initial=True)
    assert np.array_equal(cpu(g2["dgamma"]), cpu(g["dgamma"]))


def test_alks_periodic_carry_over_two_runs(orc):
    """Two design iterations of the periodic approximation: the second run
    starts from the first one's final state and carries its adj_initial
    into adj_terminal, on the GPU and in the oracle."""
    p = PROBS["2d_walls_y"](1).replace(scheme=1)
    gamma, chi, psi = rand_inputs(p, 15)
    plan = lk().Plan(p)
    _, fin = plan.forward(gamma, chi, psi, want_final=True)
    a1 = plan.adjoint(gamma, chi, psi, want_initial=True)
    s1 = cpu(fin)
    _ = plan.forward(gamma, chi, psi, state0=s1)
    a2 = plan.adjoint(gamma, chi, psi, adj_terminal=cpu(a1["adj_initial"]), want_initial=True)
    r1 = orc.alks_adjoint(p, gamma, chi, psi)
    f1 = orc.forward(p, gamma, chi, psi)["final"]
    r2 = orc.alks_adjoint(p, gamma, chi, psi, state0=f1, adj_terminal=r1["adj_initial"])
    assert relerr(cpu(a2["adj_initial"]), r2["adj_initial"]) < 1e-9
    for k in ("dgamma", "dchi", "dpsi"):
        assert l2err(cpu(a2[k]), r2[k]) < 1e-9, k
