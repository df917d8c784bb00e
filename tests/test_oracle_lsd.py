"""The least-squares misfit the paper compares the EMD with (Section 2.1) and its
adjoint source (Section 2.3), pinned to closed forms.

For a Ricker wavelet r(t) = (1 - 2at^2) exp(-at^2), a = (pi f)^2, and its copy
shifted by tau, 1/2 int (r(t - tau) - r(t))^2 dt = C(0) - C(tau) with the
autocorrelation C(tau) = sqrt(pi / 2a) (a^2 tau^4 - 6 a tau^2 + 3) / 4 exp(-a tau^2 / 2)
(r is -(1/2a) times the second derivative of exp(-at^2), so C is (1/4a^2) times the
fourth derivative of the Gaussian's autocorrelation sqrt(pi/2a) exp(-a tau^2/2)).  At
1 ms sampling the wavelet's spectrum is zero to double precision beyond 500 Hz, so the
cell sum equals the integral up to rounding."""
import numpy as np
import pytest

from synth import config1_pairs, random_small_pair


def ricker_autocorrelation(tau, f):
    a = (np.pi * f) ** 2
    return np.sqrt(np.pi / (2 * a)) * (a * a * tau ** 4 - 6 * a * tau ** 2 + 3) / 4 * np.exp(-a * tau ** 2 / 2)


@pytest.mark.parametrize("f", [8.0, 10.0])
def test_lsd_of_shifted_rickers_matches_the_autocorrelation(oracle_mod, f):
    shifts = np.arange(-200, 201, 10)
    gs = config1_pairs(shifts, f_peak=f)
    got = np.array([oracle_mod.lsd(g.pcal, g.pobs, g.dx, g.dt)[0] for g in gs])
    want = ricker_autocorrelation(0.0, f) - ricker_autocorrelation(1e-3 * shifts, f)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-15 * want.max())


def test_lsd_curve_skips_cycles_at_8hz(oracle_mod):
    # Section 3.1: two local minima beside the global one at zero shift, where the
    # autocorrelation has its side maxima: C'(tau) is proportional to -x^2 + 10x - 15
    # with x = a tau^2, so tau* = sqrt(5 + sqrt(10)) / (pi f)  (113.7 ms at 8 Hz)
    f = 8.0
    shifts = np.arange(-200, 201, 1)
    gs = config1_pairs(shifts, f_peak=f)
    v = np.array([oracle_mod.lsd(g.pcal, g.pobs, g.dx, g.dt)[0] for g in gs])
    mins = [int(shifts[k]) for k in range(1, len(v) - 1) if v[k] < v[k - 1] and v[k] < v[k + 1]]
    assert shifts[int(np.argmin(v))] == 0
    tau = 1e3 * np.sqrt(5 + np.sqrt(10)) / (np.pi * f)
    assert len(mins) == 3 and mins[1] == 0
    assert abs(-mins[0] - tau) <= 0.5 and abs(mins[2] - tau) <= 0.5


def test_lsd_gradient_and_symmetry(oracle_mod):
    g = random_small_pair(9, 37, 4)
    f, grad = oracle_mod.lsd(g.pcal, g.pobs, g.dx, g.dt)
    f2, grad2 = oracle_mod.lsd(g.pobs, g.pcal, g.dx, g.dt)
    assert f == f2
    np.testing.assert_array_equal(grad, -grad2)
    assert oracle_mod.lsd(g.pcal, g.pcal, g.dx, g.dt)[0] == 0.0
    # the misfit is quadratic: the central difference is exact up to rounding
    rng = np.random.default_rng(0)
    d = rng.normal(size=g.pcal.shape)
    h = 1e-3
    fd = (oracle_mod.lsd(g.pcal + h * d, g.pobs, g.dx, g.dt)[0] -
          oracle_mod.lsd(g.pcal - h * d, g.pobs, g.dx, g.dt)[0]) / (2 * h)
    assert fd == pytest.approx(float((grad * d).sum()), rel=1e-9)
