"""The Algorithm 1 driver (lks_optimize) against the same sequence run on
the oracle: continuation over beta, the density filter and projection
(Sec. 3.1), the periodic approximation's carry of the final state into the
next march and of the adjoint's initial state into the next reverse sweep
(Sec. 3.3), J and G1-G3 (Sec. 2.6), the chain rule back to the design
variables, and a fixed-step projected-gradient update standing in for MMA
(the caller's optimiser).  FP64: J and G per iteration within 1e-10, the
design variables after the last update within 1e-8."""
import numpy as np
import pytest
import torch

from test_gpu_parity import cpu, lk, prob2d, prob3d

pytestmark = pytest.mark.gpu

STEP = {"gamma": 0.05, "chi": 0.02, "psi": 0.02}


def step(x, g, a):
    """Projected gradient ascent with a step normalised by the largest entry."""
    m = np.abs(g).max()
    return np.clip(x + (a / m) * g if m > 0 else x, 0.0, 1.0)


def oracle_sequence(orc, p, gamma, chi, psi, betas, n_opt, R, eta, cons, periodic, alks):
    """Algorithm 1 on the oracle, iteration by iteration."""
    hist, st, adj = [], None, None
    adjoint = orc.alks_adjoint if alks else orc.adjoint
    for beta in betas:
        Jp = None
        for k in range(n_opt):
            phys = orc.design_prelude(p, gamma, R, beta, eta)
            f = orc.forward(p, phys, chi, psi, state0=st if periodic else None)
            G, d1, d2, d3 = orc.constraints(p, phys, chi, psi, *cons)
            hist.append((f["J"], *G))
            a = adjoint(p, phys, chi, psi, state0=st if periodic else None,
                        adj_terminal=adj if periodic else None)
            st = f["final"]
            adj = a["adj_initial"]
            dg = orc.design_prelude_adjoint(p, gamma, R, beta, eta, a["dgamma"])
            gamma = step(gamma, dg, STEP["gamma"])
            chi = step(chi, a["dchi"], STEP["chi"])
            psi = step(psi, a["dpsi"], STEP["psi"])
    return gamma, chi, psi, hist


def gpu_update(state):
    for key, gkey in (("gamma", "dJ_dgamma"), ("chi", "dJ_dchi"), ("psi", "dJ_dpsi")):
        x, g = state[key], state[gkey]
        m = g.abs().max()
        if m > 0:
            x.add_(g, alpha=STEP[key] / float(m)).clamp_(0.0, 1.0)
    return False


@pytest.mark.parametrize("case", ["2d_exact", "2d_alks", "3d_exact"])
def test_optimize_matches_oracle_sequence(orc, case):
    lks = lk()
    if case.startswith("2d"):
        p = prob2d((45, 21), 1, m=(9, 7, 1), nt=10)
    else:
        p = prob3d((34, 18, 20), 1, nt=5)
    p = p.replace(scheme=1 if case.endswith("alks") else 0)
    rng = np.random.default_rng(31)
    gamma = rng.uniform(0.2, 0.8, size=p.M)
    chi = rng.uniform(0.4, 0.6, size=(p.nt, 3))
    psi = rng.uniform(0.4, 0.6, size=p.nt)
    betas, n_opt, R, eta = (1.0, 8.0), 2, 2.5, 0.5
    cons = (0.6, 0.01, 4.0)
    print(f"optimize {case}: {p.n}, {len(betas)} x {n_opt} iterations", flush=True)
    plan = lks.Plan(p)
    g, c, s, hist, res = lks.optimize(plan, gamma, chi, psi, gpu_update, beta=betas, n_opt=n_opt,
                                      radius=R, eta=eta, tol=0.0, vmax=cons[0],
                                      omega_max=cons[1], p_omega=cons[2], periodic=True)
    assert res["iterations"] == 4 and res["levels"] == 2 and res["stopped"] == 0
    og, oc, ops, ohist = oracle_sequence(orc, p, gamma, chi, psi, betas, n_opt, R, eta, cons,
                                         True, case.endswith("alks"))
    for (J, *G), (oJ, *oG) in zip(hist, ohist):
        assert abs(J - oJ) <= 1e-10 * abs(oJ), (J, oJ)
        assert np.allclose(G, oG, rtol=1e-12, atol=1e-14)
    # the iterations moved the design (the updates were not all clipped away)
    assert np.abs(og - gamma).max() > 1e-3
    assert np.abs(cpu(g) - og).max() < 1e-8
    assert np.abs(cpu(c) - oc).max() < 1e-8
    assert np.abs(cpu(s) - ops).max() < 1e-8


def test_optimize_stopping_criterion_and_callback_stop():
    """With a tolerance no change of J exceeds, every level stops at its
    second iteration (Sec. 3.2 compares J of two consecutive iterations); an
    active constraint that is violated keeps the level running to n_opt; a
    callback returning True stops the loop."""
    lks = lk()
    p = prob2d((45, 21), 1, m=(9, 7, 1), nt=8)
    rng = np.random.default_rng(32)
    gamma = rng.uniform(0.2, 0.8, size=p.M)
    chi = rng.uniform(0.4, 0.6, size=(p.nt, 3))
    psi = rng.uniform(0.4, 0.6, size=p.nt)
    plan = lks.Plan(p)
    kw = dict(radius=2.5, eta=0.5, vmax=0.6, omega_max=0.01, p_omega=4.0)
    *_, hist, res = lks.optimize(plan, gamma, chi, psi, gpu_update, beta=(1.0, 2.0, 4.0),
                                 n_opt=5, tol=1e30, **kw)
    assert res["iterations"] == 6 and res["levels"] == 3 and res["stopped"] == 0
    # G1 <= 0 required: vmax = 0.01 makes G1 > 0 at every iteration
    *_, hist, res = lks.optimize(plan, gamma, chi, psi, gpu_update, beta=(1.0,), n_opt=3,
                                 tol=1e30, g_active=1, **dict(kw, vmax=0.01))
    assert res["iterations"] == 3 and all(h[1] > 0 for h in hist)
    calls = []

    def stop_second(state):
        calls.append(state["total"])
        gpu_update(state)
        return len(calls) == 2

    *_, hist, res = lks.optimize(plan, gamma, chi, psi, stop_second, beta=(1.0, 2.0), n_opt=5,
                                 tol=0.0, **kw)
    assert res["stopped"] == 1 and res["iterations"] == 2 and calls == [1, 2]
