"""Gradient consumers (L-BFGS, leapfrog HMC) on analytic targets: the
sampler and optimiser logic, without a GPU."""
import numpy as np

from paper_1905_12146_amd.inference import hmc, lbfgs_maximize, leapfrog


def gaussian(prec):
    prec = np.asarray(prec, dtype=np.float64)

    def f(x):
        return -0.5 * float(x @ (prec * x)), -prec * x
    return f


def test_hmc_standard_normal_moments():
    f = gaussian(np.ones(5))
    r = hmc(f, np.zeros(5), 4000, step=0.25, n_leapfrog=8, seed=1)
    assert r.accept_rate > 0.9
    assert np.all(np.abs(r.samples.mean(axis=0)) < 0.1)
    assert np.all(np.abs(r.samples.var(axis=0) - 1.0) < 0.15)


def test_leapfrog_is_reversible():
    f = gaussian([1.0, 4.0, 0.25])
    x0 = np.array([0.3, -0.2, 1.1])
    p0 = np.array([0.5, 0.1, -0.7])
    _, g0 = f(x0)
    inv_m = np.ones(3)
    x1, p1, _, g1 = leapfrog(f, x0, p0, g0, 0.1, 17, inv_m)
    x2, p2, _, _ = leapfrog(f, x1, -p1, g1, 0.1, 17, inv_m)
    assert np.allclose(x2, x0, atol=1e-12) and np.allclose(-p2, p0, atol=1e-12)


def test_energy_error_is_second_order():
    f = gaussian([1.0, 3.0])
    x0 = np.array([0.8, -0.4])
    p0 = np.array([0.3, 0.9])
    _, g0 = f(x0)

    def dh(step, n):
        x1, p1, lp1, _ = leapfrog(f, x0, p0, g0, step, n, np.ones(2))
        return abs((-lp1 + 0.5 * p1 @ p1) - (-f(x0)[0] + 0.5 * p0 @ p0))
    ratio = dh(0.1, 10) / dh(0.05, 20)
    assert 3.0 < ratio < 5.0


def test_preconditioning_helps_anisotropic_target():
    prec = np.array([1e-2, 1.0, 1e2])
    f = gaussian(prec)
    plain = hmc(f, np.zeros(3), 300, step=0.15, n_leapfrog=10, seed=2)
    pre = hmc(f, np.zeros(3), 300, step=0.15, n_leapfrog=10, mass_diag=prec, seed=2)
    assert pre.accept_rate > plain.accept_rate
    assert pre.accept_rate > 0.8


def test_lbfgs_quadratic():
    c = np.array([1.0, -2.0, 0.5])
    a = np.array([2.0, 0.5, 10.0])

    def f(x):
        d = x - c
        return -float(d @ (a * d)), -2 * a * d
    r = lbfgs_maximize(f, np.zeros(3), gtol=1e-10)
    assert r.success and np.allclose(r.x, c, atol=1e-7)
