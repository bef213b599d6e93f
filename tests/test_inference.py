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


def test_ess_of_known_chains():
    from paper_1905_12146_amd.inference import ess
    rng = np.random.default_rng(3)
    n = 20000
    iid = rng.normal(size=n)
    assert 0.9 * n < ess(iid) < 1.1 * n
    phi = 0.8                                    # AR(1): ESS = n (1 - phi) / (1 + phi)
    x = np.empty(n)
    x[0] = rng.normal()
    for i in range(1, n):
        x[i] = phi * x[i - 1] + rng.normal() * np.sqrt(1 - phi * phi)
    expect = n * (1 - phi) / (1 + phi)
    assert 0.85 * expect < ess(x) < 1.15 * expect


def test_adaptive_mass_is_the_running_mean_of_the_negative_hessian():
    """Section 3.2.1: M_ii = clamp(mean of -d2 log p / dx_i^2 over every k-th
    state, m_min, m_max).  On log p = sum -(x^4/4 + a x^2/2) the negative
    Hessian diagonal 3 x^2 + a varies with x: the mass matrix must equal the
    mean of it over the recorded states, stay within the bounds, and change
    by O(1/s) between updates."""
    from paper_1905_12146_amd.inference import adaptive_hmc
    a = np.array([0.01, 1.0, 50.0, 1e5])

    def f(x):
        return -float(np.sum(x ** 4 / 4 + a * x * x / 2)), -(x ** 3 + a * x)

    seen = []

    def nh(x):
        seen.append(x.copy())
        return 3 * x * x + a

    k = 5
    r = adaptive_hmc(f, nh, np.full(4, 0.1), 400, step=0.1, n_leapfrog=8, k=k, m_min=0.05, m_max=1e3, seed=4)
    assert len(seen) == 400 // k == len(r.mass_history)
    for j in range(len(seen)):
        # recorded states are the chain's states at iterations k-1, 2k-1, ...
        assert np.array_equal(seen[j], r.samples[(j + 1) * k - 1])
        mean = np.mean([3 * x * x + a for x in seen[: j + 1]], axis=0)
        assert np.allclose(r.mass_history[j], np.clip(mean, 0.05, 1e3), rtol=1e-12)
    assert r.mass_history[:, 0].min() >= 0.05 and r.mass_history[:, 3].max() == 1e3
    step = np.abs(np.diff(r.mass_history[:, 1:3], axis=0)).max(axis=1)
    s = np.arange(2, len(r.mass_history) + 1)
    assert np.all(step * s <= 50.0 * r.mass_history[1:, 1:3].max(axis=1))   # O(1/s)


def test_adaptive_preconditioning_raises_the_worst_ess():
    from paper_1905_12146_amd.inference import adaptive_hmc, ess
    prec = np.array([1e-2, 1.0, 1e2])
    f = gaussian(prec)
    vanilla = hmc(f, np.zeros(3), 1500, step=0.15, n_leapfrog=10, seed=5)
    adapt = adaptive_hmc(f, lambda x: prec.copy(), np.zeros(3), 1500, step=0.15, n_leapfrog=10, k=10, seed=5)
    burn = 100
    e_v = min(ess(vanilla.samples[burn:, i]) for i in range(3))
    e_a = min(ess(adapt.samples[burn:, i]) for i in range(3))
    assert e_a > 3 * e_v, (e_a, e_v)
