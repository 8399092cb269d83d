"""The parity allowances of the GPU tests come from this CPU study: the
oracle against copies of itself that differ by one rounding, per workload
(see tests/parity_budget.py).  Every committed figure must be reproduced, and
every cell a perturbation flags must meet the bar again when both copies run
at rtol 1e-11 / atol 1e-14."""
import pytest

import parity_budget as pb


@pytest.mark.parametrize("workload", pb.WORKLOADS)
def test_study_reproduces(workload):
    n, flagged, umax, tight_ok = pb.measure(workload)
    print(f"[budget] {workload}: {n} cells, {flagged} flagged, max {umax} units; "
          f"{pb.allowed_flags(workload, n)} allowed per {n}, bound {pb.unit_bound(workload)} units",
          flush=True)
    assert (n, flagged) == pb.STUDY[workload][:2]
    assert umax == pytest.approx(pb.STUDY[workload][2], abs=0.05)
    assert tight_ok


def test_allowance_formula():
    """The stated margin: a quarter over the study's rate, three standard
    deviations of counting noise and two cells; twice the study's distance,
    at least 10 units."""
    assert pb.allowed_flags("front_hot", 1000) == 2
    n, f, u = pb.STUDY["stress32"]
    mu = 1.25 * f / n * 2000
    assert pb.allowed_flags("stress32", 2000) == int(mu + 3 * mu ** 0.5 + 2)
    assert pb.unit_bound("stress32") == 2 * u
    assert pb.unit_bound("cells") == 10.0
