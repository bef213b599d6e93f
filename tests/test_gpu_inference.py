"""Gradient consumers on the GPU path: maximum-likelihood branch lengths by
L-BFGS (against the same optimiser driven by the CPU oracle's gradient),
HMC on a random-effects clock (leapfrog reversibility with the GPU
gradient, acceptance, a Hessian-diagonal preconditioner), and HMC chains
served through the continuous-batching server (bitwise the same samples as
the chains run on their own contexts)."""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from paper_1905_12146_amd.inference import (RandomEffectsClock, adaptive_hmc, hmc, lbfgs_maximize,
                                            leapfrog, mle_branch_lengths, served_chains)
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu


def _work(n=12, s=150, k=2, seed=4):
    return small(n_tips=n, n_patterns=s, n_cats=k, ambiguous=0.05, seed=seed, tips="simulate")


def test_lbfgs_mle_matches_oracle_driven_lbfgs(gpu):
    w = _work()
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        l0, _ = ctx.logL_and_grad(w.t)
        r = mle_branch_lengths(ctx, w.t, gtol=1e-9)
    args = list(args_of(w))

    def f_oracle(x):
        args[1] = np.exp(x)
        out = O.linear_gradient(*args)
        return out["logL"], out["grad"] * np.exp(x)
    ref = lbfgs_maximize(f_oracle, np.log(w.t), gtol=1e-9)
    print("MLE logL gpu", r.value, "oracle-driven", ref.value, "start", l0, "evals", r.n_evals, flush=True)
    assert r.value >= l0
    assert abs(r.value - ref.value) <= 1e-8 * abs(ref.value)
    assert np.max(np.abs(r.grad)) <= 1e-3


def test_clock_hmc_reversible_and_accepting(gpu):
    w = _work(n=10, s=120, k=1, seed=6)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        model = RandomEffectsClock(ctx, w.t.copy(), sigma=0.5)
        theta0 = np.zeros(len(w.t))
        lp0, g0 = model(theta0)
        p0 = np.random.default_rng(0).normal(size=theta0.size)
        x1, p1, _, g1 = leapfrog(model, theta0, p0, g0, 0.01, 10, np.ones(theta0.size))
        x2, p2, _, _ = leapfrog(model, x1, -p1, g1, 0.01, 10, np.ones(theta0.size))
        assert np.allclose(x2, theta0, atol=1e-9) and np.allclose(-p2, p0, atol=1e-8)
        r = hmc(model, theta0, 40, step=0.01, n_leapfrog=10, seed=3)
        prec = model.precision_diag(r.samples[-1])
        rp = hmc(model, r.samples[-1], 20, step=0.1, n_leapfrog=10, mass_diag=prec, seed=4)
    print("vHMC accept", r.accept_rate, "pHMC accept", rp.accept_rate, flush=True)
    assert r.accept_rate >= 0.5 and np.all(np.isfinite(r.samples))
    assert np.all(prec > 0) and rp.accept_rate >= 0.5


def test_served_chains_equal_direct_chains(gpu):
    from paper_1905_12146_amd.serving import Server
    ws = [_work(n=8 + 3 * i, s=90 + 20 * i, k=2, seed=20 + i) for i in range(3)]
    taus = [w.t.copy() for w in ws]
    with Server(0, B.PG_FP64, 4 << 30, 8) as srv:
        served = served_chains(srv, ws, taus, n_samples=6, step=0.02, n_leapfrog=5, seeds=[1, 2, 3])
        stats = srv.stats()
    for w, tau, seed, rs in zip(ws, taus, [1, 2, 3], served):
        with B.Context(0, B.PG_FP64) as ctx:
            ctx.set_workload(w)
            rd = hmc(RandomEffectsClock(ctx, tau, 0.5), np.zeros(len(tau)), 6, 0.02, 5, seed=seed)
        assert np.array_equal(rs.samples, rd.samples) and np.array_equal(rs.log_p, rd.log_p)
    assert stats["calls"] == 3 * (1 + 6 * 5)



class _OracleCtx:
    """logL_and_grad / logL / hessian_diag of a workload from the CPU oracle."""

    def __init__(self, w):
        self.args = list(args_of(w))
        self.t = None

    def logL_and_grad(self, t):
        self.args[1] = np.asarray(t, dtype=np.float64)
        r = O.linear_gradient(*self.args)
        return r["logL"], r["grad"]

    def logL(self, t):
        self.t = np.asarray(t, dtype=np.float64)
        return self.logL_and_grad(t)[0]

    def hessian_diag(self):
        self.args[1] = self.t
        r = O.linear_gradient(*self.args)
        return r["grad"], r["hess"]


def test_hmc_with_gpu_gradients_follows_the_oracle_driven_chain(gpu):
    """Same seed, same model: vanilla HMC and adaptive pHMC (Section 3.2.1,
    mass matrix from the GPU Hessian diagonal) driven by the GPU path take the
    same accept decisions and the same states as when driven by the oracle's
    gradient and Hessian, to rounding."""
    w = _work(n=10, s=120, k=2, seed=8)
    oracle_model = RandomEffectsClock(_OracleCtx(w), w.t.copy(), sigma=0.5)
    theta0 = np.zeros(len(w.t))
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        gpu_model = RandomEffectsClock(ctx, w.t.copy(), sigma=0.5)
        rv = hmc(gpu_model, theta0, 12, step=0.02, n_leapfrog=6, seed=11)
        ra = adaptive_hmc(gpu_model, gpu_model.neg_hess_diag, theta0, 12, step=0.05, n_leapfrog=6, k=3,
                          m_min=1e-2, m_max=1e4, seed=12)
    ov = hmc(oracle_model, theta0, 12, step=0.02, n_leapfrog=6, seed=11)
    oa = adaptive_hmc(oracle_model, oracle_model.neg_hess_diag, theta0, 12, step=0.05, n_leapfrog=6, k=3,
                      m_min=1e-2, m_max=1e4, seed=12)
    print("vHMC accepted", rv.accepted.sum(), "pHMC accepted", ra.accepted.sum(), flush=True)
    assert np.array_equal(rv.accepted, ov.accepted) and np.array_equal(ra.accepted, oa.accepted)
    assert np.allclose(rv.samples, ov.samples, rtol=1e-8, atol=1e-10)
    assert np.allclose(ra.samples, oa.samples, rtol=1e-8, atol=1e-10)
    assert np.allclose(ra.mass_history, oa.mass_history, rtol=1e-7)
