"""Host (NumPy) reference of the batched multi-start L-BFGS that the library
runs on the device (gp_lbfgs): the same algorithm, step rules and
parametrisation, the bookkeeping in NumPy on the host and one batched
gp_nll_grad call per evaluation.  Test infrastructure: the GPU tests compare
the device fit with it."""
from __future__ import annotations

import numpy as np

from paper_1203_1269_amd import binding
from paper_1203_1269_amd.optim import FitResult


def _eval(ds, phi, ws):
    res, g = binding.nll_grad(ds, np.exp(phi), ws=ws)
    f = res["nll"].cpu().numpy()
    info = res["info"].cpu().numpy()
    g = g.cpu().numpy() * np.exp(phi)
    bad = (info != 0) | ~np.isfinite(f)
    f = np.where(bad, np.inf, f)
    return f, g


def _two_loop(g, S_hist, Y_hist):
    q = g.copy()
    alphas = []
    for s, y in reversed(list(zip(S_hist, Y_hist))):
        rho = 1.0 / (y @ s)
        a = rho * (s @ q)
        alphas.append((a, rho, s, y))
        q -= a * y
    if S_hist:
        s, y = S_hist[-1], Y_hist[-1]
        q *= (s @ y) / (y @ y)
    for a, rho, s, y in reversed(alphas):
        b = rho * (y @ q)
        q += (a - b) * s
    return -q


def lbfgs_multistart_host(ds: "binding.Dataset", theta0, iters: int = 50, m: int = 10,
                     c1: float = 1e-4, max_ls: int = 20, gtol: float = 1e-6,
                     theta_bounds=(1e-4, 1e4)) -> FitResult:
    phi = np.log(np.asarray(theta0, dtype=np.float64)).copy()
    S, d = phi.shape
    lo, hi = np.log(theta_bounds[0]), np.log(theta_bounds[1])
    need = binding.grad_workspace_bytes(ds.n, ds.d, S)
    ws = binding.alloc_workspace(need, ds.device)
    f, g = _eval(ds, phi, ws)
    nevals = 1
    hist_s = [[] for _ in range(S)]
    hist_y = [[] for _ in range(S)]
    active = np.isfinite(f) & (np.max(np.abs(g), axis=1) > gtol)
    its = np.zeros(S, dtype=int)
    history = [float(np.min(f))]
    per_start = [f.copy()]
    for _ in range(iters):
        if not active.any():
            break
        dirs = np.zeros_like(phi)
        for s in np.nonzero(active)[0]:
            p = _two_loop(g[s], hist_s[s], hist_y[s])
            if p @ g[s] >= 0:          # not a descent direction: restart
                hist_s[s].clear(); hist_y[s].clear()
                p = -g[s]
            dirs[s] = p
        # unit step once curvature pairs exist; a step of at most 1 in log(theta)
        # before that
        first = np.array([len(h) == 0 for h in hist_s])
        step = np.where(first, np.minimum(1.0, 1.0 / np.maximum(np.abs(dirs).max(axis=1), 1e-300)), 1.0)
        step = np.where(active, step, 0.0)
        pending = active.copy()
        new_phi, new_f, new_g = phi.copy(), f.copy(), g.copy()
        slope = np.sum(g * dirs, axis=1)
        for _ls in range(max_ls):
            if not pending.any():
                break
            idx = np.nonzero(pending)[0]
            trial = np.clip(phi[idx] + step[idx, None] * dirs[idx], lo, hi)
            ft, gt = _eval(ds, trial, ws)      # only the starts still searching
            nevals += 1
            ok = ft <= f[idx] + c1 * step[idx] * slope[idx]
            acc = idx[ok]
            new_phi[acc], new_f[acc], new_g[acc] = trial[ok], ft[ok], gt[ok]
            pending[acc] = False
            step = np.where(pending, step * 0.5, step)
        moved = active & ~pending
        for s in np.nonzero(moved)[0]:
            sv, yv = new_phi[s] - phi[s], new_g[s] - g[s]
            if sv @ yv > 1e-12 * np.sqrt((sv @ sv) * (yv @ yv)):
                hist_s[s].append(sv); hist_y[s].append(yv)
                if len(hist_s[s]) > m:
                    hist_s[s].pop(0); hist_y[s].pop(0)
        phi, f, g = new_phi, new_f, new_g
        its += moved
        active = moved & (np.max(np.abs(g), axis=1) > gtol)
        history.append(float(np.min(f)))
        per_start.append(f.copy())
    return FitResult(np.exp(phi), f, np.max(np.abs(g), axis=1), its, nevals, history,
                     np.array(per_start))
