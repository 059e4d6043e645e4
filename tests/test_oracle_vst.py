"""Pins of the FP64 variance-stabilising oracle (no GPU).

The forward transform against its algebraic inverse and its scale
invariance; variance stabilisation from exact Poisson sums (scipy's pmf);
the closed-form inverse against the exact expectation of the transform
under Poisson and Poisson-Gaussian noise (pmf sums and Gauss-Hermite
quadrature), where it must beat the algebraic and asymptotic inverses at
low counts; the 8-bit FP32 map against the FP64 transform."""
import math

import numpy as np
import pytest
from scipy.stats import poisson

from oracle import vst as V


def pois_expect(fn, lam):
    k = np.arange(0, int(lam + 40 * math.sqrt(lam) + 60))
    return float((poisson.pmf(k, lam) * fn(k)).sum())


def test_algebraic_inverse_and_scale_invariance():
    rng = np.random.default_rng(0)
    for alpha, sigma, mu in ((1.0, 0.0, 0.0), (2.5, 3.0, 1.5), (0.3, 0.7, -2.0)):
        z = rng.uniform(0, 500, 1000)
        D = V.forward(z, alpha, sigma, mu)
        np.testing.assert_allclose(V.algebraic_inverse(D, alpha, sigma, mu), z, rtol=1e-12, atol=1e-9)
        # f(z; alpha, sigma, mu) = f((z - mu) / alpha; 1, sigma / alpha, 0)
        np.testing.assert_allclose(D, V.forward((z - mu) / alpha, 1.0, sigma / alpha), rtol=1e-12)
        # so is the unbiased inverse: alpha I(D; sigma / alpha) + mu
        np.testing.assert_allclose(V.unbiased_inverse(D, alpha, sigma, mu),
                                   alpha * V.unbiased_inverse(D, 1.0, sigma / alpha) + mu, rtol=1e-12, atol=1e-12)
    # the argument is clamped at zero
    assert V.forward(-10.0, 1.0, 0.0) == 0.0


@pytest.mark.parametrize("lam", [20.0, 50.0, 200.0])
def test_stabilises_poisson_variance(lam):
    m1 = pois_expect(lambda k: V.forward(k, 1.0, 0.0), lam)
    m2 = pois_expect(lambda k: V.forward(k, 1.0, 0.0) ** 2, lam)
    assert abs(m2 - m1 * m1 - 1.0) < 0.01
    # the untransformed variance is lam
    assert abs(pois_expect(lambda k: k * k, lam) - pois_expect(lambda k: k, lam) ** 2 - lam) < 1e-6 * lam


def test_stabilises_poisson_gaussian_variance():
    rng = np.random.default_rng(1)
    alpha, sigma, lam = 2.0, 6.0, 40.0
    z = alpha * rng.poisson(lam, 400_000) + rng.normal(0.0, sigma, 400_000)
    assert abs(V.forward(z, alpha, sigma).var() - 1.0) < 0.02


@pytest.mark.parametrize("lam", [0.05, 0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0, 30.0, 100.0])
def test_closed_form_inverts_the_poisson_expectation(lam):
    Ef = pois_expect(lambda k: V.forward(k, 1.0, 0.0), lam)
    err = float(V.unbiased_inverse(Ef, 1.0, 0.0)) - lam
    assert abs(err) < 0.02
    if 0.2 <= lam <= 1.0:
        # the plain inverses are biased by a tenth or more at low counts
        assert abs(float(V.algebraic_inverse(Ef, 1.0, 0.0)) - lam) > 10 * abs(err) + 0.02
        assert abs(Ef * Ef / 4 - 0.125 - lam) > 5 * abs(err) + 0.02


@pytest.mark.parametrize("s", [0.5, 1.0, 2.0])
def test_closed_form_inverts_the_poisson_gaussian_expectation(s):
    x, w = np.polynomial.hermite_e.hermegauss(80)
    w = w / w.sum()
    for lam, tol in ((1.0, 0.04), (2.0, 0.015), (5.0, 3e-3), (10.0, 3e-3), (100.0, 3e-4)):
        k = np.arange(0, int(lam + 40 * math.sqrt(lam) + 60))
        Ef = float((poisson.pmf(k, lam)[:, None] * w[None, :] * V.forward(k[:, None] + s * x[None, :], 1.0, s)).sum())
        assert abs(float(V.unbiased_inverse(Ef, 1.0, s)) - lam) / lam < tol, (s, lam)


def test_zero_count_maps_to_zero():
    assert float(V.unbiased_inverse(V.D0, 1.0, 0.0)) == pytest.approx(0.0, abs=1e-12)
    assert float(V.unbiased_inverse(0.5, 3.0, 1.0, 7.0)) == 7.0  # below f(0): the estimate is mu


def test_u8_map_rounds_the_fp64_transform():
    rng = np.random.default_rng(2)
    alpha, sigma, mu, scale, offset = 1.7, 2.0, 0.5, 6.0, 3.0
    z = np.concatenate([rng.uniform(-20, 400, 20000), [-1e9, 1e9]]).astype(np.float32)
    u = V.forward_u8_f32(z, alpha, sigma, mu, scale, offset).astype(np.float64)
    ref = np.clip(scale * V.forward(z.astype(np.float64), alpha, sigma, mu) + offset, 0, 255)
    assert np.abs(u - ref).max() <= 0.5 + 1e-3
    assert u[-2] == 3.0 and u[-1] == 255.0
    assert V.noise_level(6.0) == pytest.approx(math.sqrt(36 + 1 / 12))
