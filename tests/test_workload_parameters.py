"""The synthetic oar workload uses the parameters the paper prints for its 2D
oar example (Sec. 4.2), stored with their citation in
tests/golden/paper_example_parameters.json.  The geometry of that example is
shown only in figures, so the domain and design grid sizes are this build's
stand-ins (documented with the generator)."""
import json
import os

from paper_2608_01071_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example_parameters.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_file_lists_the_three_examples():
    g = load()
    for key in ("2d_pump", "2d_oar", "3d_pump"):
        assert g[key]["cite"].startswith("Sec. 4."), key
        assert g[key]["nu"] > 0 and g[key]["q"] > 0 and g[key]["N_t"] > 0, key


def test_oar_workload_uses_the_printed_parameters():
    o = load()["2d_oar"]
    p, gamma, chi, psi = W.oar()
    assert p.nt == o["N_t"]
    assert p.nu == o["nu"]
    assert p.kappa_max == o["kappa_max"]
    assert p.q == o["q"]
    assert p.r_t == o["R_t"]
    assert p.r_w == o["R_omega"]
    assert p.w_d == o["w_D"] and p.w_t == o["w_T"]
    assert p.objective == 1  # J2
