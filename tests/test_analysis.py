"""Static-potential analysis on synthetic Wilson loops with known answers."""
import numpy as np
import pytest

from paper_1010_4834_amd import analysis as an


def test_bin_series():
    x = np.arange(10.0)
    b = an.bin_series(x, 3)          # 3 bins of 3, tail dropped
    assert np.array_equal(b, [1.0, 4.0, 7.0])
    with pytest.raises(ValueError):
        an.bin_series(x, 1)


def test_jackknife_of_mean_is_standard_error():
    rng = np.random.default_rng(3)
    bins = rng.normal(size=(25, 4))
    est, err, _ = an.jackknife(bins)
    assert np.allclose(est, bins.mean(axis=0))
    assert np.allclose(err, bins.std(axis=0, ddof=1) / np.sqrt(25))


def test_jackknife_nonlinear_matches_delta_method():
    rng = np.random.default_rng(4)
    a = 2.0 + 0.01 * rng.normal(size=400)
    b = 1.0 + 0.01 * rng.normal(size=400)
    bins = np.stack([a, b], axis=1)
    est, err, _ = an.jackknife(bins, lambda m: np.log(m[0] / m[1]))
    # delta method for independent a, b: var = (sa/a)^2 + (sb/b)^2
    sa, sb = a.std(ddof=1) / np.sqrt(400), b.std(ddof=1) / np.sqrt(400)
    expect = np.sqrt((sa / a.mean()) ** 2 + (sb / b.mean()) ** 2)
    assert abs(err - expect) < 0.05 * expect
    assert abs(est - np.log(a.mean() / b.mean())) < 1e-15


def cornell(R, A=0.55, B=-0.26, sigma=0.0366):
    return A + B / R + sigma * R


def test_effective_potential_of_pure_exponentials():
    R = np.arange(1, 9, dtype=float)[:, None]
    T = np.arange(1, 11, dtype=float)[None, :]
    C = 0.8 - 0.02 * R
    W = C * np.exp(-cornell(R) * T)
    V = an.effective_potential(W)
    assert V.shape == (8, 9)
    assert np.allclose(V, np.broadcast_to(cornell(R), V.shape), rtol=0, atol=1e-13)


def test_cornell_fit_exact():
    R = np.arange(2, 10, dtype=float)
    A, B, s = an.cornell_fit(R, cornell(R))
    assert abs(A - 0.55) < 1e-12 and abs(B + 0.26) < 1e-12 and abs(s - 0.0366) < 1e-13


def test_static_potential_recovers_string_tension():
    rng = np.random.default_rng(5)
    nconf, Rmax, Tmax = 400, 8, 8
    R = np.arange(1, Rmax + 1, dtype=float)[:, None]
    T = np.arange(1, Tmax + 1, dtype=float)[None, :]
    W0 = 0.9 * np.exp(-cornell(R) * T)
    # multiplicative noise, correlated within a configuration
    noise = 1.0 + 0.02 * rng.normal(size=(nconf, Rmax, 1)) + 0.01 * rng.normal(size=(nconf, Rmax, Tmax))
    res = an.static_potential(W0[None] * noise, t0=3, rmin=2, rmax=8, nbins=40)
    assert res["dsigma"] > 0
    assert abs(res["sigma"] - 0.0366) < 4 * res["dsigma"]
    assert abs(res["sigma"] - 0.0366) < 0.004
    assert np.all(np.abs(res["V"] - cornell(R[:, 0])) < 5 * res["dV"] + 1e-12)


def test_static_potential_rejects_bad_ranges():
    W = np.ones((10, 4, 4))
    with pytest.raises(ValueError):
        an.static_potential(W, t0=4, rmin=1, rmax=4, nbins=5)
    with pytest.raises(ValueError):
        an.static_potential(W, t0=1, rmin=3, rmax=3, nbins=5)


def test_stable_t0_waits_for_the_excited_state():
    """W = c0 e^{-V T} + c1 e^{-(V + gap) T} with an excited-state weight c1
    growing with R (as ground-state overlaps fall with R): the effective
    potential approaches V from above, most at large R, which biases sigma
    upwards at small t0; the chosen t0 is where the excited state has decayed
    below the noise, and the fit there recovers sigma."""
    rng = np.random.default_rng(6)
    nconf, Rmax, Tmax = 400, 8, 14
    R = np.arange(1, Rmax + 1, dtype=float)[:, None]
    T = np.arange(1, Tmax + 1, dtype=float)[None, :]
    V = cornell(R)
    c1 = 0.05 * R
    W0 = (1 - c1) * np.exp(-V * T) + c1 * np.exp(-(V + 0.5) * T)
    noise = 1.0 + 0.003 * rng.normal(size=(nconf, Rmax, 1)) + 0.002 * rng.normal(size=(nconf, Rmax, Tmax))
    Wc = W0[None] * noise
    t0 = an.stable_t0(Wc, 2, 8, 40)
    assert t0 is not None and t0 >= 4
    res = an.static_potential(Wc, t0, 2, 8, 40)
    assert abs(res["sigma"] - 0.0366) < 4 * res["dsigma"] + 5e-4
    # at t0 = 1 the excited state biases sigma upwards
    assert an.static_potential(Wc, 1, 2, 8, 40)["sigma"] > res["sigma"] + 3 * res["dsigma"]
