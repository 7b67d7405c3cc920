"""Pins of the reference TT interior-point method (oracle, CPU).

At full TT rank (no truncation binds at n = 8) the reference TT-IPM must
reach the closed-form SDP values: MaxCut of K_8 is n^2/4 = 16, MaxCut of
C_7 + K_1 is (7/2)(1 + cos(pi/7)) (odd cycle, Sec. 4.1), and the Lovasz theta
of C_5 + 3 K_1 is sqrt(5) + 3 (Sec. 4.2).  Each solve starts from the
scaled identity, takes XZ warm-up then AHO directions, and runs block AMEn,
rounding with the Cor. 1 shift and the eta schedule, so a sign, index or
coefficient mistake anywhere in that chain keeps it from the closed form (the
odd cycle has a non-uniform optimum, the theta instance an inequality-free
but non-vertex-transitive one).  Both objectives are checked to 1e-7, with the
local systems solved by the block elimination of Sec. 3.3 and by a dense LU of
the reduced system.  (On the theta instance the elimination's Cholesky of the
local L_Z meets a numerically indefinite block near the optimum and raises;
the GPU path falls back to the LU there, the reference leaves that choice to
the caller.)
"""
import math

import pytest

import instances as I
from oracle import problems as OP, ttipm_ref as R

CASES = {
    "K8_maxcut": (lambda: OP.maxcut(I.complete(3).cores), 16.0, ("elim", "dense")),
    "C7+K1_maxcut": (lambda: OP.maxcut(I.odd_cycle_plus_isolated(3).cores), 3.5 * (1 + math.cos(math.pi / 7)),
                     ("elim", "dense")),
    "C5+3K1_theta": (lambda: OP.theta(I.c5_plus_3k1().cores), 3 + math.sqrt(5), ("dense",)),
}


@pytest.mark.parametrize("name,local", [(n, l) for n, c in CASES.items() for l in c[2]])
def test_reference_ttipm_reaches_closed_form(name, local):
    make, value, _ = CASES[name]
    # stop at 1e-8: the feasibility measures settle near 1e-8 (rounding of the
    # local solves), and far past that mu the iterates lose definiteness
    res = R.solve(make(), rank_cap=64, stop_gap=1e-8, delta=1e-12, max_iter=40, local=local)
    assert res["status"] == "converged"
    for key in ("pobj", "dobj"):
        assert abs(res[key] - value) / (1 + value) < 1e-7, (key, res[key], value)
