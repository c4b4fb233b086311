"""The genetic-algorithm driver on the CPU: budget, bounds, determinism,
elitism and convergence on objectives with a known minimiser, failed
evaluations, and a GA fit driven by the oracle's -2logL."""
import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import ga, inputs


def _bowl(center):
    c = np.log(np.asarray(center))

    def f(theta):
        return np.sum((np.log(theta) - c) ** 2, axis=1)
    return f


def test_budget_bounds_and_batches():
    seen = []

    def f(theta):
        seen.append(theta.copy())
        return np.sum(theta, axis=1)
    r = ga.ga_minimise(f, 3, lo=0.05, hi=20.0, pop=100, gens=20, seed=1)
    assert r.evaluations == 2000 and r.generations == 20 and len(seen) == 20
    for th in seen:
        assert th.shape == (100, 3)
        assert np.all(th >= 0.05 * (1 - 1e-12)) and np.all(th <= 20.0 * (1 + 1e-12))
    # generation 0 is a Latin-hypercube sample of the log box
    u = (np.log(seen[0]) - np.log(0.05)) / (np.log(20.0) - np.log(0.05))
    for k in range(3):
        assert np.array_equal(np.sort(np.floor(u[:, k] * 100)), np.arange(100))


def test_deterministic_given_the_seed():
    a = ga.ga_minimise(_bowl([0.3, 4.0]), 2, seed=5, keep_history=True)
    b = ga.ga_minimise(_bowl([0.3, 4.0]), 2, seed=5, keep_history=True)
    c = ga.ga_minimise(_bowl([0.3, 4.0]), 2, seed=6)
    assert np.array_equal(a.theta, b.theta) and a.nll == b.nll
    assert all(np.array_equal(x, y) for x, y in zip(a.all_theta, b.all_theta))
    assert not np.array_equal(a.theta, c.theta)


def test_elitism_and_survivors():
    r = ga.ga_minimise(_bowl([1.0, 1.0, 1.0]), 3, seed=2, keep_history=True)
    h = np.array(r.best_history)
    assert np.all(np.diff(h) <= 0)                     # best never gets worse
    allv = np.concatenate(r.all_values)
    assert r.nll == allv.min()                         # the best ever evaluated
    # survivors are the pop best of everything evaluated so far ((mu + lambda))
    assert np.allclose(np.sort(r.values), np.sort(allv)[:100])


@pytest.mark.parametrize("center", [[0.3, 4.0], [0.05, 1.0, 25.0, 2.0]])
def test_converges_on_a_bowl(center):
    d = len(center)
    r = ga.ga_minimise(_bowl(center), d, lo=0.01, hi=100.0, seed=3)
    assert np.max(np.abs(np.log(r.theta) - np.log(center))) < 0.05 * d, r.theta


def test_failed_evaluations_never_win():
    """Half of the box fails (NaN, as a failed factorisation gives): the
    best theta is in the other half and is the bowl's constrained minimum."""
    f0 = _bowl([0.5, 0.5])

    def f(theta):
        v = f0(theta)
        return np.where(theta[:, 0] < 1.0, np.nan, v)
    r = ga.ga_minimise(f, 2, seed=4, keep_history=True)
    assert np.isfinite(r.nll) and r.theta[0] >= 1.0
    assert np.any(~np.isfinite(np.concatenate(r.all_values)))
    assert abs(np.log(r.theta[0])) < 0.05 and abs(np.log(r.theta[1]) - np.log(0.5)) < 0.05


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        ga.ga_minimise(_bowl([1.0]), 1, lo=0.0)
    with pytest.raises(ValueError):
        ga.ga_minimise(_bowl([1.0]), 1, pop=1)
    with pytest.raises(ValueError):
        ga.ga_minimise(lambda th: np.zeros(3), 1)


def test_ga_fit_with_the_oracle_objective():
    """A small fit (n=40, d=2, the paper's p=1.95 and no nugget) at the
    paper's budget (100 x 20) driven by the FP64 oracle: the reported value
    is the oracle's at the reported theta, and it is no worse than a 40 x 40
    grid search over the same box."""
    w = inputs.ga_workload(40, 2, seed=11, N=10)

    def f(theta):
        r = oracle.nll_batch(w.X, w.y, theta, w.p, w.delta)
        return np.where(r.info == 0, r.nll, np.inf)
    res = ga.ga_minimise(f, 2, lo=0.01, hi=100.0, seed=0)
    assert res.evaluations == 2000
    again = oracle.nll_batch(w.X, w.y, res.theta[None, :], w.p, w.delta)
    assert again.info[0] == 0 and again.nll[0] == res.nll
    g = np.exp(np.linspace(np.log(0.01), np.log(100.0), 40))
    grid = np.array([[a, b] for a in g for b in g])
    assert res.nll <= np.min(f(grid)) + 1e-9 * abs(res.nll)
