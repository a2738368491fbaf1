"""Pins of the oracle's counter-based generator (Philox4x32-10)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox(tuple(v[0:4]), tuple(v[4:6])) == tuple(v[6:10])


def test_uniform_is_dyadic_and_in_range():
    u = np.array([oracle.uniform(7, 3, s, 0, i) for s in range(3) for i in range(500)])
    assert np.all((u >= 0) & (u < 1))
    assert np.all(np.ldexp(u, 53) == np.floor(np.ldexp(u, 53)))
    # 1500 iid U(0,1): mean within 5 sigma
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))


def test_normal_moments():
    z = np.array([oracle.normal(11, 4, 0, m, i) for m in range(4) for i in range(2000)])
    n = len(z)
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    # kurtosis of a normal is 3
    assert abs((z ** 4).mean() / z.var() ** 2 - 3) < 0.3


def test_streams_are_distinct():
    a = [oracle.uniform(1, 3, 0, 0, i) for i in range(64)]
    b = [oracle.uniform(1, 4, 0, 0, i) for i in range(64)]
    c = [oracle.uniform(2, 3, 0, 0, i) for i in range(64)]
    assert len(set(a) & set(b)) == 0 and len(set(a) & set(c)) == 0
