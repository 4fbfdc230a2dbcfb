"""Pins of the oracle's SBX and polynomial mutation (Appendix B).

SBX is pinned by its defining distribution (the spread factor
beta = |c1-c2|/|x1-x2| has CDF b^(eta+1)/2 below 1 and 1 - b^-(eta+1)/2
above, Deb & Agrawal 1995), by the mean-preserving identity c1 + c2 = x1 + x2,
and by the fair exchange and sign decisions.  Polynomial mutation is pinned
by its special values (u=0 -> lower bound, u=1 -> upper bound, u=1/2 -> no
change), monotonicity, boundedness, and its reduction at the box edge to the
unbounded form (2u)^(1/(eta+1)) - 1, which ties it to the SBX spread factor.
"""
import numpy as np
import pytest
from scipy import stats


def _pairs(ora, K, d, N, seed=0, lo=0.3, hi=0.7):
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, size=(K, d)).astype(np.float32)
    valid = np.ones(K, np.uint8)
    parents, _ = ora.mate(seed=seed, t=1, valid=valid, N=N)
    return X, parents


def test_sbx_spread_factor_distribution(ora):
    K, d, N = 64, 40, 2000
    X, parents = _pairs(ora, K, d, N)
    prm = ora.params(p_m=0.0)
    Xoff, pre = ora.reproduce(prm, seed=9, t=4, X=X, parents=parents, N=N, with_pre=True)
    P = (N + 1) // 2
    x1 = X[parents[:, 0]].astype(np.float64)
    x2 = X[parents[:, 1]].astype(np.float64)
    c1, c2 = pre[:P], pre[P:2 * P]
    diff = np.abs(x1 - x2)
    ok = diff > 1e-3
    # mean preserving (children stay inside the box here, so no clipping)
    assert np.allclose((c1 + c2)[ok], (x1 + x2)[ok], rtol=0, atol=1e-15)
    beta = np.abs(c1 - c2)[ok] / diff[ok]
    copies = np.abs(beta - 1.0) < 1e-9
    frac = copies.mean()
    assert abs(frac - 0.5) < 5 * np.sqrt(0.25 / copies.size)
    b = beta[~copies]
    eta = 20.0

    def cdf(x):
        x = np.asarray(x, dtype=np.float64)
        return np.where(x <= 1.0, 0.5 * x ** (eta + 1), 1.0 - 0.5 * x ** (-(eta + 1)))

    assert stats.kstest(b, cdf).pvalue > 1e-4
    # sign of B: child1 is the child nearer parent 1 with probability 1/2
    bb = np.abs(c1 - x1)[ok][~copies] < np.abs(c2 - x1)[ok][~copies]
    sel = b < 0.999
    assert abs(bb[sel].mean() - 0.5) < 5 * np.sqrt(0.25 / sel.sum())
    assert Xoff.dtype == np.float32 and np.array_equal(Xoff, pre.astype(np.float32))


def test_sbx_identical_parents_reproduce_the_parent(ora):
    K, d, N = 4, 33, 8
    rng = np.random.default_rng(1)
    row = rng.uniform(0, 1, size=d).astype(np.float32)
    X = np.tile(row, (K, 1))
    parents = np.zeros(((N + 1) // 2, 2), np.int32)
    parents[:, 1] = 1
    Xoff = ora.reproduce(ora.params(p_m=0.0), seed=3, t=2, X=X, parents=parents, N=N)
    assert np.array_equal(Xoff, np.tile(row, (N, 1)))


def test_odd_population_pairs_children(ora):
    K, d, N = 10, 16, 5
    X, parents = _pairs(ora, K, d, N, seed=4)
    Xoff, pre = ora.reproduce(ora.params(p_m=0.0), seed=4, t=1, X=X, parents=parents, N=N,
                              with_pre=True)
    P = 3
    for p in range(2):  # offspring p and p + P come from pair p
        s = X[parents[p, 0]].astype(np.float64) + X[parents[p, 1]]
        assert np.allclose(pre[p] + pre[p + P], s, atol=1e-15)
    assert Xoff.shape == (5, 16)


def test_children_stay_in_box(ora):
    K, d, N = 50, 30, 400
    rng = np.random.default_rng(8)
    X = rng.choice(np.array([0.0, 1.0, 0.5, 1e-6], np.float32), size=(K, d))
    parents, _ = ora.mate(seed=8, t=1, valid=np.ones(K, np.uint8), N=N)
    Xoff = ora.reproduce(ora.params(p_m=5.0), seed=8, t=1, X=X, parents=parents, N=N)
    assert Xoff.min() >= 0.0 and Xoff.max() <= 1.0 and np.all(np.isfinite(Xoff))
    Xoff = ora.reproduce(ora.params(p_m=5.0, lb=-3.0, ub=2.0), seed=8, t=1, X=X * 5 - 3,
                         parents=parents, N=N)
    assert Xoff.min() >= -3.0 and Xoff.max() <= 2.0


def test_sbx_beta_special_values(ora):
    assert ora.sbx_beta(0.0) == 0.0
    assert ora.sbx_beta(0.5) == 1.0
    assert ora.sbx_beta(0.5 - 2**-24) == pytest.approx(1.0, abs=1e-7)
    # CDF relation of the spread factor (inverse-transform sampling)
    for mc in [0.01, 0.1, 0.3, 0.49]:
        b = ora.sbx_beta(mc, 20.0)
        assert 0.5 * b**21 == pytest.approx(mc, rel=1e-13)
    for mc in [0.51, 0.7, 0.9, 1 - 2**-24]:
        b = ora.sbx_beta(mc, 20.0)
        assert 1.0 - 0.5 * b ** (-21) == pytest.approx(mc, rel=1e-13)
        assert b > 1.0


def test_pm_special_values_and_monotone(ora):
    for x in [0.0, 0.2, 0.5, 0.93, 1.0]:
        assert x + ora.pm_delta(x, 0.0) == pytest.approx(0.0, abs=1e-15)
        assert x + ora.pm_delta(x, 1.0) == pytest.approx(1.0, abs=1e-15)
        assert ora.pm_delta(x, 0.5) == 0.0
        us = np.linspace(0, 1, 201)
        vals = np.array([x + ora.pm_delta(x, u) for u in us])
        assert np.all(np.diff(vals) >= -1e-15)
        assert vals.min() >= -1e-15 and vals.max() <= 1 + 1e-15
    # other boxes
    assert -2.0 + ora.pm_delta(-2.0, 0.0, lb=-5, ub=3) == pytest.approx(-5.0)
    assert -2.0 + ora.pm_delta(-2.0, 1.0, lb=-5, ub=3) == pytest.approx(3.0)


def test_pm_reduces_to_unbounded_form_at_the_box_edges(ora):
    # x = ub (delta_1 = 1), u < 1/2: Delta/(ub-lb) = (2u)^(1/(xi+1)) - 1 = beta_sbx(u) - 1
    for u in [0.01, 0.2, 0.45]:
        assert ora.pm_delta(1.0, u) == pytest.approx(ora.sbx_beta(u) - 1.0, rel=1e-13)
    # x = lb (delta_2 = 1), u > 1/2: Delta/(ub-lb) = 1 - (2(1-u))^(1/(xi+1))
    for u in [0.55, 0.8, 0.99]:
        assert ora.pm_delta(0.0, u) == pytest.approx(1.0 - ora.sbx_beta(1.0 - u), rel=1e-13)


def test_mutation_applies_at_the_drawn_sites_only(ora):
    d = 40
    c = np.linspace(0.05, 0.95, d)
    out = ora.mutate_child(seed=2, t=7, o=3, c=c, p_m=3.0)
    sites, mags = ora.mutation_sites(seed=2, t=7, o=3, d=d, p_m=3.0)
    changed = np.nonzero(out != c)[0]
    assert set(changed.tolist()) <= set(sites.tolist())
    for s, u in zip(sites, mags):
        assert out[s] == pytest.approx(min(max(c[s] + ora.pm_delta(c[s], u), 0.0), 1.0))
    # no mutation at p_m = 0
    assert np.array_equal(ora.mutate_child(seed=2, t=7, o=3, c=c, p_m=0.0), c)
