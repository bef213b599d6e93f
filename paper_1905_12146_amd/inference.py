"""Gradient consumers on the GPU log-likelihood (Section 4 of the paper uses
the gradient for maximum likelihood by L-BFGS and for Hamiltonian Monte
Carlo on a random-effects clock).

* ``lbfgs_maximize(f, x0)``: L-BFGS maximisation of any f(x) -> (value,
  gradient); ``mle_branch_lengths(ctx, t0)`` applies it to the branch
  lengths in log space (x = log t, d/dx = t * dlogL/dt).
* ``RandomEffectsClock``: t_b = exp(theta_b) tau_b with theta_b ~ N(0,
  sigma^2) i.i.d.; log posterior and gradient in theta from one
  logL-and-gradient call, and a diagonal preconditioner from the Hessian
  diagonal (-d2/dtheta2 of the log posterior at a point, floored).
* ``hmc(f, x0, ...)``: leapfrog HMC with a diagonal mass matrix (identity:
  vanilla HMC; a fixed preconditioner).
* ``adaptive_hmc(f, neg_hess_diag, x0, ...)``: preconditioned HMC whose
  diagonal mass matrix is the running average of -d2 log p / dx_i^2 over
  the states visited every k-th iteration, clamped to [m_min, m_max]
  (Section 3.2.1).
* ``ess(x)``: effective sample size of a chain (initial monotone sequence
  of autocorrelation pairs).
* ``served_chains(server, ...)``: several HMC chains whose gradient calls go
  through the continuous-batching server, one session per chain.

The samplers only need f, so they are exercised on analytic targets without
a GPU; the phylogenetic adapters call the library.
"""
from __future__ import annotations

import threading
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np

Target = Callable[[np.ndarray], Tuple[float, np.ndarray]]


# ---------------------------------------------------------------- maximisation

@dataclass
class MaxResult:
    x: np.ndarray
    value: float
    grad: np.ndarray
    n_evals: int
    success: bool
    message: str


def lbfgs_maximize(f: Target, x0: np.ndarray, gtol: float = 1e-6, maxiter: int = 500,
                   bounds=None, ftol: float = 1e-15) -> MaxResult:
    """Maximise f with scipy's L-BFGS-B on -f (f returns value, gradient)."""
    from scipy.optimize import minimize

    n = [0]

    def neg(x):
        v, g = f(x)
        n[0] += 1
        return -v, -np.asarray(g, dtype=np.float64)

    r = minimize(neg, np.asarray(x0, dtype=np.float64), jac=True, method="L-BFGS-B", bounds=bounds,
                 options={"gtol": gtol, "ftol": ftol, "maxiter": maxiter, "maxcor": 20})
    v, g = f(r.x)
    return MaxResult(x=r.x, value=float(v), grad=np.asarray(g), n_evals=n[0] + 1, success=bool(r.success),
                     message=str(r.message))


def mle_branch_lengths(ctx, t0: np.ndarray, gtol: float = 1e-6, maxiter: int = 500,
                       t_min: float = 1e-8) -> MaxResult:
    """Maximum-likelihood branch lengths by L-BFGS in x = log t.

    ``ctx`` is a binding.Context with tree, patterns and model set.
    Returns the result in x (``result.x``); t = exp(x)."""
    def f(x):
        t = np.exp(x)
        logL, g = ctx.logL_and_grad(t)
        return logL, g * t

    x0 = np.log(np.maximum(np.asarray(t0, dtype=np.float64), t_min))
    return lbfgs_maximize(f, x0, gtol=gtol, maxiter=maxiter)


# ---------------------------------------------------------------- random-effects clock

@dataclass
class RandomEffectsClock:
    """log p(theta | data) = logL(exp(theta) tau) - |theta|^2 / (2 sigma^2) + c."""
    ctx: object
    tau: np.ndarray
    sigma: float = 0.5
    calls: int = 0

    def lengths(self, theta: np.ndarray) -> np.ndarray:
        return np.exp(theta) * self.tau

    def __call__(self, theta: np.ndarray) -> Tuple[float, np.ndarray]:
        t = self.lengths(theta)
        logL, g = self.ctx.logL_and_grad(t)
        self.calls += 1
        return logL - 0.5 * float(theta @ theta) / self.sigma ** 2, g * t - theta / self.sigma ** 2

    def neg_hess_diag(self, theta: np.ndarray) -> np.ndarray:
        """-d2 log p / dtheta_b^2 from the Hessian diagonal (Section 2.7):
        d2/dtheta2 logL(e^theta tau) = t^2 H_bb + t g_b."""
        t = self.lengths(theta)
        self.ctx.logL(t)
        g, h = self.ctx.hessian_diag()
        self.calls += 1
        return -(t * t * h + t * g) + 1.0 / self.sigma ** 2

    def precision_diag(self, theta: np.ndarray, floor: float = 1e-3) -> np.ndarray:
        """neg_hess_diag at one point, floored (a fixed preconditioner)."""
        return np.maximum(self.neg_hess_diag(theta), floor)


# ---------------------------------------------------------------- HMC

@dataclass
class HMCResult:
    samples: np.ndarray           # [n_samples, dim]
    log_p: np.ndarray             # [n_samples]
    accept_rate: float
    energy_error: np.ndarray      # H(end) - H(start) of every trajectory
    n_grad: int
    accepted: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=bool))


def leapfrog(f: Target, x: np.ndarray, p: np.ndarray, g: np.ndarray, step: float, n_steps: int,
             inv_mass: np.ndarray):
    """n_steps leapfrog steps of H(x, p) = -log p(x) + p^T M^-1 p / 2 from
    (x, p) with gradient g = d log p / dx at x; returns (x, p, log p, g)."""
    x = x.copy()
    p = p + 0.5 * step * g
    lp = None
    for i in range(n_steps):
        x = x + step * inv_mass * p
        lp, g = f(x)
        if i + 1 < n_steps:
            p = p + step * g
    p = p + 0.5 * step * g
    return x, p, lp, g


def hmc(f: Target, x0: np.ndarray, n_samples: int, step: float, n_leapfrog: int,
        mass_diag: Optional[np.ndarray] = None, seed: int = 0) -> HMCResult:
    """Hamiltonian Monte Carlo with a diagonal mass matrix."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x0, dtype=np.float64).copy()
    d = x.size
    mass = np.ones(d) if mass_diag is None else np.asarray(mass_diag, dtype=np.float64)
    inv_mass = 1.0 / mass
    lp, g = f(x)
    n_grad = 1
    out = np.empty((n_samples, d))
    lps = np.empty(n_samples)
    dH = np.empty(n_samples)
    acc = np.zeros(n_samples, dtype=bool)
    for k in range(n_samples):
        p0 = rng.normal(size=d) * np.sqrt(mass)
        H0 = -lp + 0.5 * float(p0 @ (inv_mass * p0))
        x1, p1, lp1, g1 = leapfrog(f, x, p0, g, step, n_leapfrog, inv_mass)
        n_grad += n_leapfrog
        H1 = -lp1 + 0.5 * float(p1 @ (inv_mass * p1)) if np.isfinite(lp1) else np.inf
        dH[k] = H1 - H0
        if np.log(rng.uniform()) < -(H1 - H0):
            x, lp, g = x1, lp1, g1
            acc[k] = True
        out[k] = x
        lps[k] = lp
    return HMCResult(samples=out, log_p=lps, accept_rate=float(acc.mean()), energy_error=dH, n_grad=n_grad,
                     accepted=acc)


def adaptive_hmc(f: Target, neg_hess_diag: Callable[[np.ndarray], np.ndarray], x0: np.ndarray, n_samples: int,
                 step: float, n_leapfrog: int, k: int = 10, m_min: float = 1e-2, m_max: float = 1e4,
                 seed: int = 0, init: Optional[Tuple[np.ndarray, int]] = None) -> HMCResult:
    """HMC with the adaptive diagonal mass matrix of Section 3.2.1.

    After every k-th iteration s, the negative Hessian diagonal of log p at
    the current state joins a running average H^(s) (the mean over the
    states x^(k), x^(2k), ..., x^(s)); the following iterations use
    M_ii = min(max(H_ii^(s), m_min), m_max).  Until the first update the
    mass matrix is the identity.  The change of H between updates is
    O(1/s) (vanishing adaptation).  The result's ``mass_history`` holds the
    mass matrix after each update; ``h_sum`` and ``n_updates`` the running
    sum and count, which ``init`` takes to continue an earlier run's
    adaptation."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x0, dtype=np.float64).copy()
    d = x.size
    h_sum = np.zeros(d) if init is None else np.asarray(init[0], dtype=np.float64).copy()
    n_upd = 0 if init is None else int(init[1])
    mass = np.clip(h_sum / n_upd, m_min, m_max) if n_upd else np.ones(d)
    lp, g = f(x)
    n_grad = 1
    out = np.empty((n_samples, d))
    lps = np.empty(n_samples)
    dH = np.empty(n_samples)
    acc = np.zeros(n_samples, dtype=bool)
    history = []
    for it in range(n_samples):
        inv_mass = 1.0 / mass
        p0 = rng.normal(size=d) * np.sqrt(mass)
        H0 = -lp + 0.5 * float(p0 @ (inv_mass * p0))
        x1, p1, lp1, g1 = leapfrog(f, x, p0, g, step, n_leapfrog, inv_mass)
        n_grad += n_leapfrog
        H1 = -lp1 + 0.5 * float(p1 @ (inv_mass * p1)) if np.isfinite(lp1) else np.inf
        dH[it] = H1 - H0
        if np.log(rng.uniform()) < -(H1 - H0):
            x, lp, g = x1, lp1, g1
            acc[it] = True
        out[it] = x
        lps[it] = lp
        if (it + 1) % k == 0:
            h_sum += neg_hess_diag(x)
            n_upd += 1
            mass = np.clip(h_sum / n_upd, m_min, m_max)
            history.append(mass.copy())
    r = HMCResult(samples=out, log_p=lps, accept_rate=float(acc.mean()), energy_error=dH, n_grad=n_grad,
                  accepted=acc)
    r.mass_history = np.array(history)
    r.h_sum, r.n_updates = h_sum, n_upd
    return r


def ess(x: np.ndarray) -> float:
    """Effective sample size of one chain x[n]: n / (1 + 2 sum_t rho_t), the
    autocorrelation sum truncated by Geyer's initial monotone sequence (sums
    of adjacent pairs, kept while positive and made non-increasing)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 4:
        return float(n)
    xc = x - x.mean()
    var = float(xc @ xc) / n
    if var == 0.0:
        return float(n)
    f = np.fft.rfft(xc, 2 * n)
    acov = np.fft.irfft(f * np.conj(f))[:n] / n
    rho = acov / var
    pairs = []
    for t in range(0, n - 1, 2):
        gsum = rho[t] + rho[t + 1]
        if gsum <= 0.0:
            break
        pairs.append(min(gsum, pairs[-1]) if pairs else gsum)
    tau = -1.0 + 2.0 * float(np.sum(pairs)) if pairs else 1.0
    return float(n / max(tau, 1e-12))


# ---------------------------------------------------------------- chains through the server

class ServedClock:
    """RandomEffectsClock whose logL-and-gradient calls go through a serving
    session (binding-compatible ``logL_and_grad``)."""

    def __init__(self, server, workload):
        self.server = server
        self.session = server.open(workload)
        self.n_branches = len(workload.t)

    def logL_and_grad(self, t):
        from . import binding as B
        status, logL, grad, _ = self.server.wait(self.server.submit(self.session, t), self.n_branches)
        if status != B.PG_OK:
            raise B.PhyloGradError(status, "served call")
        return logL, grad

    def close(self):
        self.server.close(self.session)


def served_chains(server, workloads: List[object], taus: List[np.ndarray], n_samples: int, step: float,
                  n_leapfrog: int, sigma: float = 0.5, seeds: Optional[List[int]] = None) -> List[HMCResult]:
    """One HMC chain per workload, run concurrently; every gradient call of
    every chain goes through the server, which batches them."""
    seeds = list(range(len(workloads))) if seeds is None else seeds
    results: List[Optional[HMCResult]] = [None] * len(workloads)
    errors: List[BaseException] = []

    def run(i):
        try:
            ctx = ServedClock(server, workloads[i])
            try:
                model = RandomEffectsClock(ctx, taus[i], sigma)
                results[i] = hmc(model, np.zeros(len(taus[i])), n_samples, step, n_leapfrog, seed=seeds[i])
            finally:
                ctx.close()
        except BaseException as e:  # reported to the caller
            errors.append(e)

    threads = [threading.Thread(target=run, args=(i,), daemon=True) for i in range(len(workloads))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    if errors:
        raise errors[0]
    return results  # type: ignore[return-value]
