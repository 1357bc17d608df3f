"""The allocation-free design chain rule (lks_design_filter_adjoint_noalloc)
against the entry point it varies, lks_design_filter_adjoint, through the C
ABI: the same kernels, so the results must be bit-identical; and against the
oracle's chain rule (Sec. 3.1, Eqs. filtering, projection) to 1e-13.  Two
calls in a row, the second with a smaller design grid, so the second reads
only what it wrote into the shared device scratch."""
import numpy as np
import pytest

from test_gpu_parity import cpu, lk, prob2d, prob3d, relerr

pytestmark = pytest.mark.gpu


def test_noalloc_chain_rule_matches_allocating_entry_point(orc):
    lks = lk()
    big = prob3d((40, 36, 24), 1, m=(13, 11, 9), xg_min=(19.5, 17.5, 11.5),
                 xg_max=(20.5, 18.5, 12.5))
    small = prob2d((96, 64), 1, m=(37, 29, 1), xg_min=(47.0, 31.0, 0.0),
                   xg_max=(49.0, 33.0, 0.0), tgt_lo=(30, 10, 0), tgt_hi=(66, 54, 1))
    assert small.M < big.M
    rng = np.random.default_rng(7)
    for p, (R, beta, eta) in ((big, (4.8, 8.0, 0.45)), (small, (2.2, 16.0, 0.5))):
        print(f"noalloc chain rule: M = {p.M}, R = {R}", flush=True)
        plan = lks.Plan(p)
        g = rng.uniform(0.0, 1.0, p.M)
        gb = rng.standard_normal(p.M)
        want = cpu(plan.design_filter_adjoint(g, R, beta, eta, gb))
        got = cpu(plan.design_filter_adjoint_noalloc(g, R, beta, eta, gb))
        assert np.array_equal(got, want)
        ref = orc.design_prelude_adjoint(p, g, R, beta, eta, gb)
        assert relerr(got, ref) < 1e-13
