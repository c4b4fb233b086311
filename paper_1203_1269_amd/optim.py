"""Batched multi-start L-BFGS on the profile likelihood.

The paper notes that the likelihood surface is multimodal near theta = 0 and
that a multi-start gradient-based optimiser is the alternative to its genetic
algorithm (Sec. 2).  This driver runs S independent L-BFGS fits at once
through gp_lbfgs: every value+gradient evaluation of the starts still
searching (and every line-search trial) is one batched gp_nll_grad call on
the GPU, and the two-loop recursion, the trial points, the Armijo test and
the history updates run as kernels on the S x d search state on the device.

Parametrisation: phi = log(theta), so theta stays positive; the gradient is
chained as d nll/d phi = theta * d nll/d theta.  Line search: backtracking
with the Armijo condition (c1 = 1e-4), halving the step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import binding


@dataclass
class FitResult:
    theta: np.ndarray          # S x d, final iterates
    nll: np.ndarray            # S, final values
    grad_norm: np.ndarray      # S, inf-norm of d nll / d log(theta)
    iterations: np.ndarray     # S, accepted steps
    evaluations: int           # batched gp_nll_grad calls
    history: list = field(default_factory=list)   # best nll after each iteration
    start_history: np.ndarray = None                 # (iterations + 1) x S, each start's nll


def lbfgs_multistart(ds: "binding.Dataset", theta0, iters: int = 50, m: int = 10,
                     c1: float = 1e-4, max_ls: int = 20, gtol: float = 1e-6,
                     theta_bounds=(1e-4, 1e4)) -> FitResult:
    """S = len(theta0) fits at once through gp_lbfgs (search state and
    bookkeeping on the device)."""
    r = binding.lbfgs(ds, theta0, iters=iters, m=m, c1=c1, max_ls=max_ls, gtol=gtol,
                      theta_bounds=theta_bounds)
    trace = r["trace"].cpu().numpy()
    return FitResult(r["theta"].cpu().numpy(), r["nll"].cpu().numpy(), r["gnorm"].cpu().numpy(),
                     r["iters"].cpu().numpy().astype(int), r["evaluations"],
                     [float(np.min(row)) for row in trace], trace)
