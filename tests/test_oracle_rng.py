"""Pins of the oracle's random numbers (counter-based generator of Sec. 3.9's role).

Philox4x32-10 is pinned to its published known-answer vectors; the uniform,
Gaussian and Gamma maps are pinned to their distributions (moments within CLT
bounds and Kolmogorov-Smirnov tests against scipy's reference CDFs).
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert O.philox(ctr, key) == out


def test_u01_open_interval_and_exact():
    assert O.u01(0) == 0.5 / 2 ** 32
    assert O.u01(0xFFFFFFFF) == (2 ** 32 - 0.5) / 2 ** 32
    assert 0.0 < O.u01(0) < O.u01(1) < O.u01(0xFFFFFFFF) < 1.0


def test_box_muller_special_values():
    # u2 = (2^30 + 0.5)/2^32 is a hair above 1/4: angle ~ pi/2, so z0 ~ 0 and z1 ~ r
    z0, z1 = O.box_muller(0x7FFFFFFF, 0x40000000)
    r = np.sqrt(-2.0 * np.log((0x7FFFFFFF + 0.5) / 2 ** 32))
    assert abs(z0) < 1e-8 and abs(z1 - r) < 1e-12


def test_gaussian_moments_and_ks():
    n_pid = 50000
    z = np.concatenate([O.normals(1234, 0, pid, 7, 2, 8) for pid in range(n_pid)])
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # pairs from one Box-Muller transform are uncorrelated
    zz = z.reshape(-1, 2)
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 5 / np.sqrt(zz.shape[0])


def test_streams_differ_by_every_counter_word():
    base = O.normals(99, 0, 12345, 3, 2, 8)
    for args in [(99, 1, 12345, 3, 2), (98, 0, 12345, 3, 2), (99, 0, 12346, 3, 2),
                 (99, 0, 12345, 4, 2), (99, 0, 12345, 3, 3), (99, 0, 12345 + (1 << 32), 3, 2)]:
        assert not np.allclose(O.normals(*args, 8), base)


@pytest.mark.parametrize("shape,mean", [(4.0, 1.0), (4.0, 37.5), (1.5, 2.0)])
def test_gamma_distribution(shape, mean):
    n = 40000
    g = np.array([O.gamma(shape, mean, 77, 0, pid, 5, 3) for pid in range(n)])
    theta = mean / shape
    var = shape * theta ** 2
    assert abs(g.mean() - mean) < 5 * np.sqrt(var / n)
    # variance of the sample variance for Gamma: (mu4 - var^2)/n, mu4 = 3 k (k+2) theta^4
    mu4 = 3 * shape * (shape + 2) * theta ** 4
    assert abs(g.var() - var) < 5 * np.sqrt((mu4 - var ** 2) / n)
    assert stats.kstest(g, "gamma", args=(shape, 0, theta)).pvalue > 1e-4
    assert (g > 0).all()
