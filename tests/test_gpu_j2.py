"""GPU parity of the second objective J2 (Eq. objective2, Sec. 2.6; 2D),
through the C ABI, against the oracle's J2 (pinned in test_oracle_j2.py) on
the same seeded inputs.

The forward returns (J2, F_L, F_D); the reverse sweep, exact or ALKS, takes
J2's seed on the fluid velocity and its direct terms (dJ/dkappa_ref and the
motion partials).  Tolerances: FP64 state to 1e-10 relative on J and 1e-9
relative L2 on every gradient (summation order only); FP32 state with FP64
sums to 1e-5 relative on J and 1e-3 relative L2 on the gradients, the bars of
the J1 parity tests.
"""
import numpy as np
import pytest

from paper_2608_01071_amd import workloads as W

from test_gpu_parity import cpu, l2err, lk, prob2d, rand_inputs

pytestmark = pytest.mark.gpu


def oar(n=(45, 21), prec=1, **kw):
    base = dict(objective=1, w_d=0.3, w_t=0.5, l_m=4.0, phi=0.0)
    base.update(kw)
    return prob2d(n, prec, **base)


J2_PROBS = {
    "walls_y": lambda prec: oar((45, 21), prec),
    "ragged_shift_y": lambda prec: oar((37, 18), prec, ckpt_k=7, nt=15),
    "walls_xy": lambda prec: oar((34, 19), prec, bc=(1, 1, 0)),
}


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("name", sorted(J2_PROBS))
@pytest.mark.parametrize("prec", [1, 0])
def test_j2_run_matches_oracle(orc, name, prec, scheme):
    p = J2_PROBS[name](prec).replace(scheme=scheme)
    gamma, chi, psi = rand_inputs(p, 41)
    plan = lk().Plan(p)
    J3, _ = plan.forward(gamma, chi, psi)
    J3 = cpu(J3)
    ref = orc.forward(p, gamma, chi, psi)
    tj = 1e-10 if prec == 1 else 1e-5
    for k, key in enumerate(("J", "E", "V")):
        assert abs(J3[k] - ref[key]) <= tj * abs(ref[key]), (key, J3[k], ref[key])
    g = plan.adjoint(gamma, chi, psi)
    gr = (orc.adjoint if scheme == 0 else orc.alks_adjoint)(p, gamma, chi, psi)
    tol = 1e-9 if prec == 1 else 1e-3
    for key in ("dgamma", "dchi", "dpsi"):
        assert np.linalg.norm(gr[key]) > 0
        assert l2err(cpu(g[key]), gr[key]) < tol, key


def test_j2_weights_split_the_objective(orc):
    """With w_D = w_T = 0 the GPU's J2 is F_L alone; switching the weights on
    changes J2 but not F_L or F_D."""
    p = oar((45, 21), 1)
    gamma, chi, psi = rand_inputs(p, 42)
    a = cpu(lk().Plan(p.replace(w_d=0.0, w_t=0.0)).forward(gamma, chi, psi)[0])
    b = cpu(lk().Plan(p).forward(gamma, chi, psi)[0])
    assert a[0] == a[1]
    assert a[1] == b[1] and a[2] == b[2]
    assert a[0] != b[0]


def test_j2_checkpoint_interval_does_not_change_gradients():
    """The direct terms go into the per-step rows of the segment sums: K in
    {1, 4, nt} and both body-tape modes give bit-identical gradients, exact
    and ALKS alike."""
    for scheme in (0, 1):
        p0 = oar((37, 18), 0, nt=13, scheme=scheme)
        gamma, chi, psi = rand_inputs(p0, 43)
        outs = []
        for K in (1, 4, 13):
            for tape in (-1, 1):
                plan = lk().Plan(p0.replace(ckpt_k=K, body_tape=tape))
                plan.forward(gamma, chi, psi)
                g = plan.adjoint(gamma, chi, psi)
                outs.append((cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
        for o in outs[1:]:
            for x, y in zip(o, outs[0]):
                assert np.array_equal(x, y)


def test_j2_in_a_batch_matches_solo_runs(orc):
    """J2 instances in lks_batch_run run as graph branches beside a J1
    instance; each gives its solo result bitwise."""
    lks = lk()
    specs = [oar((45, 21), 0), prob2d((45, 21), 0), oar((37, 18), 0, scheme=1, nt=15, ckpt_k=7)]
    inputs = [rand_inputs(p, 44 + k) for k, p in enumerate(specs)]
    solo = []
    for p, (g, c, s) in zip(specs, inputs):
        pl = lks.Plan(p)
        J3, _ = pl.forward(g, c, s)
        gr = pl.adjoint(g, c, s)
        solo.append((cpu(J3), {k: cpu(gr[k]) for k in ("dgamma", "dchi", "dpsi")}))
    b = lks.Batch([lks.Plan(p) for p in specs])
    out = b.run([x[0] for x in inputs], [x[1] for x in inputs], [x[2] for x in inputs])
    for k, (J3, gr) in enumerate(out):
        assert np.array_equal(cpu(J3), solo[k][0]), k
        for key in ("dgamma", "dchi", "dpsi"):
            assert np.array_equal(cpu(gr[key]), solo[k][1][key]), (k, key)


@pytest.mark.parametrize("scheme", [0, 1])
def test_oar_full_size_first_steps(orc, scheme):
    """The 2D oar workload at the size the benchmark runs (512^2, 256^2
    design) in the plan its problem statement builds: the first three steps
    of its motion (two checkpoint segments, the second ragged) from a random
    start state with a mean flow, J2 and all three gradients on every point
    against the oracle, FP64 and FP32.  (Without the mean flow the forces of
    a random field nearly cancel: J2 is then some 1e-3 of its terms, and the
    FP32 state's rounding moves it by about 5e-5 of itself.)"""
    from test_gpu_parity import gpu_state, rand_state
    p, gamma, chi, psi = W.oar()
    p3 = p.replace(nt=3, ckpt_k=2, precision=1, scheme=scheme)
    s0 = rand_state(p3, 61, amp=0.02)
    s0[p3.N: 2 * p3.N] += 0.03
    ref = orc.forward(p3, gamma, chi[:3], psi[:3], state0=s0, want_final=False)
    adj = (orc.adjoint if scheme == 0 else orc.alks_adjoint)(p3, gamma, chi[:3], psi[:3],
                                                            state0=s0)
    for prec in (1, 0):
        pp = p3.replace(precision=prec)
        plan = lk().Plan(pp)
        J3, _ = plan.forward(gamma, chi[:3], psi[:3], state0=gpu_state(s0, pp))
        g = plan.adjoint(gamma, chi[:3], psi[:3])
        tj, tg = (1e-10, 1e-9) if prec == 1 else (1e-5, 1e-3)
        for k, key in enumerate(("J", "E", "V")):
            assert abs(cpu(J3)[k] - ref[key]) <= tj * abs(ref[key]), (prec, key)
        for k in ("dgamma", "dchi", "dpsi"):
            assert np.linalg.norm(adj[k]) > 0, k
            assert l2err(cpu(g[k]), adj[k]) < tg, (prec, k)
        del plan


def test_j2_graph_replay_matches_eager():
    """The captured forward and adjoint graphs (accumulators cleared inside
    them) give on every replay what an eager run gives, bitwise."""
    p = oar((37, 18), 0, nt=11, ckpt_k=4, scheme=1)
    gamma, chi, psi = rand_inputs(p, 47)
    plan = lk().Plan(p)
    runs = []
    for _ in range(3):
        J3, _ = plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi)
        runs.append((cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"])))
    eager = lk().Plan(p)
    eager.set_graphs(False)
    J3, _ = eager.forward(gamma, chi, psi)
    g = eager.adjoint(gamma, chi, psi)
    ref = (cpu(J3), cpu(g["dgamma"]), cpu(g["dchi"]), cpu(g["dpsi"]))
    for r in runs:
        for a, b in zip(r, ref):
            assert np.array_equal(a, b)
