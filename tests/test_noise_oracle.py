"""Pins of the oracle's noise model (CPU): Philox4x32-10 against its
published known-answer vectors, Poisson variates against the moments and the
probability mass function of the Poisson law, the negative-log transform
against its definition's limits, Box-Muller against the normal moments."""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers(oracle):
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.parametrize("lam", [0.3, 4.0, 9.9, 10.0, 37.5, 1234.0, 1e5])
def test_poisson_moments(oracle, lam):
    n = 40000
    ks = np.array([oracle.poisson(lam, 12345, 7, i) for i in range(n)], dtype=np.float64)
    se = math.sqrt(lam / n)
    assert abs(ks.mean() - lam) < 5 * se
    # variance of the sample variance of a Poisson law: (lam + 2 lam^2) / n
    assert abs(ks.var() - lam) < 5 * math.sqrt((lam + 2 * lam * lam) / n)
    assert ks.min() >= 0


@pytest.mark.parametrize("lam", [2.5, 14.0])
def test_poisson_pmf(oracle, lam):
    n = 60000
    ks = np.array([oracle.poisson(lam, 99, 1, i) for i in range(n)])
    kmax = int(lam + 6 * math.sqrt(lam)) + 1
    obs = np.bincount(np.minimum(ks, kmax), minlength=kmax + 1)
    pmf = np.array([math.exp(-lam + k * math.log(lam) - math.lgamma(k + 1)) for k in range(kmax)])
    exp_ = np.append(pmf, 1 - pmf.sum()) * n
    keep = exp_ > 20
    chi2 = float(((obs[keep] - exp_[keep]) ** 2 / exp_[keep]).sum())
    dof = int(keep.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_poisson_streams_are_independent_of_order(oracle):
    a = [oracle.poisson(50.0, 5, 3, i) for i in range(200)]
    b = [oracle.poisson(50.0, 5, 3, i) for i in reversed(range(200))][::-1]
    assert a == b
    c = [oracle.poisson(50.0, 5, 4, i) for i in range(200)]
    assert a != c


def test_log_transform_limits(oracle):
    p = np.array([0.0, 1e-9, 0.5, 3.0, 40.0])
    y, c = oracle.sim_poisson_log(p, 1e5, 7, 0)
    assert np.all(y >= 0)
    # a count at or above the air count clamps to zero attenuation
    assert y[0] == -math.log(min(max(c[0], 1) / 1e5, 1.0))
    # zero counts are floored at one count
    assert c[4] == 0 and abs(y[4] - math.log(1e5)) < 1e-12
    # noise scale: std of y ~ 1/sqrt(I0 exp(-p)) for large counts
    pp = np.full(20000, 2.0)
    yy, _ = oracle.sim_poisson_log(pp, 1e5, 11, 0)
    assert abs(yy.mean() - 2.0) < 1e-3
    assert abs(yy.std() - 1 / math.sqrt(1e5 * math.exp(-2.0))) < 0.05 / math.sqrt(1e5 * math.exp(-2))


def test_gaussian_moments(oracle):
    z = oracle.sim_gaussian(np.zeros(100000), 1.0, 3, 0)
    assert abs(z.mean()) < 5 / math.sqrt(1e5)
    assert abs(z.std() - 1) < 5 / math.sqrt(2e5)
    assert abs(np.mean(z ** 4) - 3) < 0.1
