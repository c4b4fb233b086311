"""Genetic-algorithm fit of the correlation parameters, one batched
likelihood call per generation.

The paper minimises -2logL with a genetic algorithm at a fixed budget of
2000 evaluations: a population of 100 over 20 generations (Sec. 3-4).  Its
operators are not given, so this is a real-coded GA of our own design:

* search space: phi = log(theta) in the box [log lo, log hi]^d;
* generation 0: a Latin-hypercube sample of the box (one point per stratum in
  every coordinate);
* each later generation: `pop` children, each from two parents picked by
  tournament (size `tour`, lowest -2logL wins), blend crossover (BLX-alpha:
  child coordinate uniform on the parents' interval widened by alpha times its
  length on each side) with probability `pc` (else a copy of the first
  parent), then Gaussian mutation of each coordinate with probability `pm`
  (standard deviation `sigma` times the box width), reflected into the box;
* survivors: the best `pop` of parents and children together ((mu + lambda)
  selection, so the best value never gets worse); ties keep the earlier
  individual (stable sort);
* a theta whose factorisation fails (info != 0) or whose value is not finite
  has fitness +inf.

Every generation's population is evaluated by one call of `objective`
(B x d thetas -> B values), so with the GPU objective a generation is one
gp_nll_batch launch sequence; the operators are host arithmetic on a
pop x d array.  All randomness comes from one seeded numpy Generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GAResult:
    theta: np.ndarray            # d, best theta found
    nll: float                   # its -2logL
    evaluations: int             # objective values computed
    generations: int
    best_history: list = field(default_factory=list)   # best nll after each generation
    population: np.ndarray | None = None                # final population (theta), pop x d
    values: np.ndarray | None = None                    # their -2logL
    all_theta: list = field(default_factory=list)       # every evaluated batch (theta)
    all_values: list = field(default_factory=list)      # and its values


def _lhs(pop, d, rng):
    u = np.empty((pop, d))
    for k in range(d):
        u[:, k] = (rng.permutation(pop) + rng.random(pop)) / pop
    return u


def _reflect(phi, a, b):
    w = b - a
    z = np.mod(phi - a, 2 * w)
    return a + np.where(z > w, 2 * w - z, z)


def _tournament(vals, rng, count, tour):
    idx = rng.integers(0, vals.shape[0], size=(count, tour))
    # lowest value wins; ties go to the lower index within the draw order
    return idx[np.arange(count), np.argmin(vals[idx], axis=1)]


def ga_minimise(objective, d: int, lo: float = 0.01, hi: float = 100.0, pop: int = 100,
                gens: int = 20, seed: int = 0, tour: int = 3, pc: float = 0.9,
                alpha: float = 0.5, pm: float = 0.2, sigma: float = 0.1,
                keep_history: bool = False) -> GAResult:
    """Minimise objective(theta) over theta in [lo, hi]^d with pop x gens
    evaluations.  objective: (B x d float64 array) -> B float64 values
    (+inf or NaN for failed evaluations)."""
    if pop < 2 or gens < 1 or d < 1 or not (0 < lo < hi):
        raise ValueError("ga_minimise: need pop >= 2, gens >= 1, d >= 1, 0 < lo < hi")
    rng = np.random.default_rng(seed)
    a, b = np.log(lo), np.log(hi)
    res = GAResult(theta=np.empty(d), nll=np.inf, evaluations=0, generations=0)

    def evaluate(phi):
        th = np.exp(phi)
        v = np.asarray(objective(th), dtype=np.float64).reshape(-1)
        if v.shape[0] != phi.shape[0]:
            raise ValueError("objective returned the wrong number of values")
        v = np.where(np.isfinite(v), v, np.inf)
        if keep_history:
            res.all_theta.append(th)
            res.all_values.append(v.copy())
        return v

    phi = a + (b - a) * _lhs(pop, d, rng)
    vals = evaluate(phi)
    res.evaluations += pop
    res.best_history.append(float(vals.min()))
    for _ in range(1, gens):
        p1 = _tournament(vals, rng, pop, tour)
        p2 = _tournament(vals, rng, pop, tour)
        x1, x2 = phi[p1], phi[p2]
        lo_k, hi_k = np.minimum(x1, x2), np.maximum(x1, x2)
        span = hi_k - lo_k
        blend = lo_k - alpha * span + (1 + 2 * alpha) * span * rng.random((pop, d))
        cross = rng.random(pop) < pc
        child = np.where(cross[:, None], blend, x1)
        mutate = rng.random((pop, d)) < pm
        child = child + mutate * rng.standard_normal((pop, d)) * sigma * (b - a)
        child = _reflect(child, a, b)
        cvals = evaluate(child)
        res.evaluations += pop
        both = np.concatenate([phi, child])
        bvals = np.concatenate([vals, cvals])
        keep = np.argsort(bvals, kind="stable")[:pop]
        phi, vals = both[keep], bvals[keep]
        res.best_history.append(float(vals[0]))
    res.generations = gens
    best = int(np.argmin(vals))
    res.theta = np.exp(phi[best])
    res.nll = float(vals[best])
    res.population = np.exp(phi)
    res.values = vals
    return res


def gpu_objective(ds, prec: str = "fp64", max_batch: int = 100):
    """-2logL of a theta batch on the GPU (gp_nll_batch); +inf where info != 0.
    The workspace is allocated once for `max_batch` thetas."""
    import torch

    from . import binding
    ws = binding.alloc_workspace(binding.workspace_bytes(ds.n, ds.d, max_batch, prec), ds.device)
    out = torch.empty((max_batch, 5), dtype=torch.float64, device=ds.device)

    def f(theta):
        th = torch.as_tensor(np.ascontiguousarray(theta), dtype=torch.float64).to(ds.device)
        B = th.shape[0]
        if B > max_batch:
            raise ValueError(f"batch {B} above the objective's max_batch {max_batch}")
        binding.nll_batch_raw(ds, th, ws, out[:B], prec=prec)
        r = binding.unpack_results(out[:B].cpu())   # one copy back per generation
        v, info = r["nll"].numpy(), r["info"].numpy()
        return np.where((info == 0) & np.isfinite(v), v, np.inf)
    return f


def fit_ga(ds, lo: float = 0.01, hi: float = 100.0, pop: int = 100, gens: int = 20,
           seed: int = 0, prec: str = "fp64", **kw) -> GAResult:
    """GA fit of a GPU-resident dataset: pop x gens gp_nll_batch evaluations."""
    return ga_minimise(gpu_objective(ds, prec, pop), ds.d, lo, hi, pop, gens, seed, **kw)
