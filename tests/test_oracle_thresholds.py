"""Pins of the acceptance threshold table T[a] (Sec. 2 Metropolis rule).

T[a] must equal floor(exp(-beta*dE) * 2^32) for dE > 0 and 2^32 otherwise,
with dE = 2*J*(2a-4).  The reference here is exp evaluated to 60 significant
digits with Python's decimal module, independent of libm."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import workloads

getcontext().prec = 60
TWO32 = 1 << 32


def exact_threshold(beta: float, J: float, a: int) -> int:
    dE = Decimal(J) * 2 * (2 * a - 4)
    if dE <= 0:
        return TWO32
    x = (-(Decimal(beta) * dE)).exp() * TWO32
    return int(x.to_integral_value(rounding="ROUND_FLOOR"))


BETAS = [0.0, 1e-9, 0.1, 0.3, 0.40, workloads.BETA_CRIT_CONFIG, 0.44, 0.46, 0.48, 0.50, 0.6,
         1.0, 2.77, 5.5, 5.6, 10.0] + list(np.linspace(0.30, 0.60, 32))


@pytest.mark.parametrize("J", [1.0, 0.5, -1.0, 0.0, 1.7])
def test_thresholds_exact_floor(orc, J):
    for beta in BETAS:
        T = orc.thresholds(beta, J)
        for a in range(5):
            exact = exact_threshold(beta, J, a)
            # libm exp is within 1 ulp; the floor can differ from the exact one only
            # when exp*2^32 lies within ~1e-6 of an integer, which never happens here.
            assert int(T[a]) == exact, (beta, J, a, int(T[a]), exact)


def test_special_values(orc):
    # ferromagnet: dE <= 0 for a <= 2 -> always accepted
    T = orc.thresholds(0.44, 1.0)
    assert list(T[:3]) == [TWO32] * 3
    assert 0 < T[4] < T[3] < TWO32
    # beta = 0: every move accepted
    assert list(orc.thresholds(0.0, 1.0)) == [TWO32] * 5
    # J = 0: dE = 0 everywhere
    assert list(orc.thresholds(0.7, 0.0)) == [TWO32] * 5
    # zero-temperature limit: exp(-4 beta J) * 2^32 < 1 once 4 beta J > 32 ln 2
    b0 = 32 * math.log(2) / 4
    assert list(orc.thresholds(b0 * 1.001, 1.0)[3:]) == [0, 0]
    assert orc.thresholds(b0 * 0.999, 1.0)[3] >= 1
    # antiferromagnet mirrors the classes: a <-> 4 - a
    Tf, Ta = orc.thresholds(0.37, 1.0), orc.thresholds(0.37, -1.0)
    assert list(Tf) == list(Ta[::-1])
