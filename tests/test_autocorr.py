"""Pins of the autocorrelation estimator used by the double-checkerboard
study: AR(1) series x_t = phi x_{t-1} + noise have rho(t) = phi^t, so
tau_int = 1/2 + phi / (1 - phi) exactly; white noise has tau_int = 1/2."""
import numpy as np
import pytest

import bench


def _ar1(phi, R, n, rng):
    x = np.empty((R, n))
    x[:, 0] = rng.standard_normal(R) / np.sqrt(1 - phi * phi)  # stationary start
    eps = rng.standard_normal((R, n))
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + eps[:, t]
    return x


@pytest.mark.parametrize("phi", [0.5, 0.9, 0.97])
def test_ar1_tau(phi):
    rng = np.random.default_rng(1234)
    x = _ar1(phi, 64, 20000, rng)
    tau, W, err = bench.tau_int(x)
    exact = 0.5 + phi / (1 - phi)
    assert abs(tau - exact) < 4 * err + 0.02 * exact  # window truncation bias ~ e^{-W/tau}
    assert W >= 6 * tau - 1


def test_white_noise_tau_is_one_half():
    rng = np.random.default_rng(99)
    tau, W, err = bench.tau_int(rng.standard_normal((32, 8000)))
    assert abs(tau - 0.5) < 4 * err + 0.01


def test_units_scale_with_the_measurement_interval():
    """Measuring every m-th value of an AR(1) chain gives phi^m per step."""
    rng = np.random.default_rng(7)
    x = _ar1(0.95, 32, 40000, rng)
    t1, _, _ = bench.tau_int(x)
    t4, _, e4 = bench.tau_int(x[:, ::4])
    exact4 = 0.5 + 0.95 ** 4 / (1 - 0.95 ** 4)
    assert abs(t4 - exact4) < 4 * e4 + 0.02 * exact4
    assert t4 < t1
