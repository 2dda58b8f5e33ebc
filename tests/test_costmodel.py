"""The report's cost formula reproduces the paper's printed table."""
import os

from paper_1901_04200_amd import costmodel

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cost_formula_matches_paper_table():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "paper_cost_table.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for isa, kf, kr, g in rows:
        assert abs(costmodel.gradient_cost_over_paths_costF(float(kf), float(kr)) - float(g)) < 5e-3, isa


def test_kr_over_kf_from_times():
    # pass 2 = K_F + K_R: a pass 2 that takes 1.5 x the forward means K_R/K_F = 0.5
    assert abs(costmodel.kr_over_kf(2.0, 3.0) - 0.5) < 1e-15
    assert abs(costmodel.gradient_over_forward(0.5) - 2.5) < 1e-15
