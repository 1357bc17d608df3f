"""GPU parity of the optimiser-side prelude (Sec. 3.1) and the constraint
functionals (Sec. 2.6) against the oracle (pinned in test_oracle_design.py),
through the C ABI.  FP64 on both sides, only the summation order differs:
1e-13 of the field's magnitude per stage, 1e-9 through a whole
forward/adjoint chain.
"""
import numpy as np
import pytest


from test_gpu_parity import cpu, l2err, lk, prob2d, prob3d, rand_inputs, relerr

pytestmark = pytest.mark.gpu


def design_probs():
    return {
        "2d": prob2d((96, 64), 1, m=(37, 29, 1), xg_min=(47.0, 31.0, 0.0),
                     xg_max=(49.0, 33.0, 0.0), tgt_lo=(30, 10, 0), tgt_hi=(66, 54, 1)),
        "3d": prob3d((40, 36, 24), 1, m=(13, 11, 9), xg_min=(19.5, 17.5, 11.5),
                     xg_max=(20.5, 18.5, 12.5)),
    }


@pytest.mark.parametrize("name", ["2d", "3d"])
@pytest.mark.parametrize("R,beta,eta", [(2.2, 0.0, 0.5), (4.8, 8.0, 0.45), (1.0, 32.0, 0.6)])
def test_design_filter_and_chain_rule_match_oracle(orc, name, R, beta, eta):
    p = design_probs()[name]
    plan = lk().Plan(p)
    rng = np.random.default_rng(3)
    g = rng.uniform(0.0, 1.0, p.M)
    gb = rng.standard_normal(p.M)
    phys = cpu(plan.design_filter(g, R, beta, eta))
    ref = orc.design_prelude(p, g, R, beta, eta)
    assert np.abs(phys - ref).max() < 1e-13
    back = cpu(plan.design_filter_adjoint(g, R, beta, eta, gb))
    refb = orc.design_prelude_adjoint(p, g, R, beta, eta, gb)
    assert relerr(back, refb) < 1e-13


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_constraints_match_oracle(orc, name):
    p = design_probs()[name]
    plan = lk().Plan(p)
    rng = np.random.default_rng(4)
    phys = rng.uniform(0.0, 1.0, p.M)
    _, chi, psi = rand_inputs(p, 5)
    for vmax, omax, pw in ((0.8, 1e-3, 16.0), (0.5, 2e-2, 2.0)):
        G, d1, d2, d3 = plan.constraints(phys, chi, psi, vmax, omax, pw)
        Gr, r1, r2, r3 = orc.constraints(p, phys, chi, psi, vmax, omax, pw)
        assert np.allclose(cpu(G), Gr, rtol=1e-13, atol=1e-15)
        assert np.allclose(cpu(d1), r1, rtol=1e-15, atol=0)
        assert np.allclose(cpu(d2), r2, rtol=1e-15, atol=0)
        assert relerr(cpu(d3), r3) < 1e-12


def test_constraints_without_rotation(orc):
    """psi constant with the identity filter: omega = 0 exactly, G3 = -1
    and dG3/dpsi = 0 on both sides."""
    p = design_probs()["2d"].replace(r_w=1)
    plan = lk().Plan(p)
    _, chi, _ = rand_inputs(p, 5)
    psi = np.full(p.nt, 0.4)
    phys = np.full(p.M, 0.5)
    G, _, _, d3 = plan.constraints(phys, chi, psi, 0.8, 1e-3, 16.0)
    Gr, _, _, r3 = orc.constraints(p, phys, chi, psi, 0.8, 1e-3, 16.0)
    assert cpu(G)[2] == -1.0 and Gr[2] == -1.0
    assert np.array_equal(cpu(d3), r3)


def test_constraints_leave_the_forward_data_intact():
    """lks_constraints between lks_forward and lks_adjoint, with another
    motion, changes nothing the adjoint reads."""
    p = prob2d((45, 21), 1)
    gamma, chi, psi = rand_inputs(p, 6)
    plan = lk().Plan(p)
    plan.forward(gamma, chi, psi)
    a = {k: cpu(v) for k, v in plan.adjoint(gamma, chi, psi).items() if v is not None}
    plan.forward(gamma, chi, psi)
    plan.constraints(np.full(p.M, 0.3), chi[::-1].copy(), psi[::-1].copy(), 0.8, 1e-3, 16.0)
    b = {k: cpu(v) for k, v in plan.adjoint(gamma, chi, psi).items() if v is not None}
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_design_chain_end_to_end(orc, name):
    """One iteration of the loop's differentiable part on the GPU: design
    variables -> filter and projection -> forward -> adjoint -> chain rule,
    against the same chain in the oracle."""
    p = design_probs()[name].replace(nt=6, ckpt_k=4)
    plan = lk().Plan(p)
    rng = np.random.default_rng(7)
    g = rng.uniform(0.1, 0.9, p.M)
    _, chi, psi = rand_inputs(p, 8)
    R, beta, eta = 2.5, 4.0, 0.5
    phys = plan.design_filter(g, R, beta, eta)
    plan.forward(phys, chi, psi)
    gr = plan.adjoint(phys, chi, psi)
    dg = cpu(plan.design_filter_adjoint(g, R, beta, eta, gr["dgamma"]))
    ophys = orc.design_prelude(p, g, R, beta, eta)
    oadj = orc.adjoint(p, ophys, chi, psi)
    odg = orc.design_prelude_adjoint(p, g, R, beta, eta, oadj["dgamma"])
    assert l2err(dg, odg) < 1e-9


def test_design_argument_checks():
    lks = lk()
    p = prob2d((45, 21), 1)
    plan = lks.Plan(p)
    g = np.full(p.M, 0.5)
    for R, beta, eta in ((0.0, 1.0, 0.5), (100.0, 1.0, 0.5), (2.0, 1.0, 1.5)):
        with pytest.raises(lks.LksError) as e:
            plan.design_filter(g, R, beta, eta)
        assert e.value.status == lks.LKS_EINVAL
    _, chi, psi = rand_inputs(p, 1)
    for vmax, omax, pw in ((0.0, 1e-3, 16.0), (0.8, 0.0, 16.0), (0.8, 1e-3, 0.5)):
        with pytest.raises(lks.LksError) as e:
            plan.constraints(g, chi, psi, vmax, omax, pw)
        assert e.value.status == lks.LKS_EINVAL
