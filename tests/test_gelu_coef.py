"""CPU pins of the network kernels' GELU polynomial (gelu_coef.h).

The kernels compute GELU(x) = max(x, 0) - |x t| 2^(P(t) - z^2 log2 e) with
z = |x| / sqrt 2 and t = 1 / (1 + kGeluT |x|), which is x/2 (1 + erf(x/sqrt 2))
when 2^P(t) = t^-1 erfc(z) e^(z^2) / 2.  The checks compute that exponent
from scipy's scaled complementary error function, independently of the
script that fitted the coefficients, and replay the kernels' FP32 operation
order to bound the result's error.  A perturbed coefficient must fail.
"""
import math
import os
import re

import numpy as np
from scipy.special import erfc, erfcx

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2510_07672_amd", "csrc", "gelu_coef.h")
LOG2E = 1.0 / math.log(2.0)


def read_header():
    text = open(HDR).read()
    kt = float(re.search(r"kGeluT = ([-0-9.e+]+)f", text).group(1))
    deg = int(re.search(r"kGeluDeg = (\d+);", text).group(1))
    body = text[text.index("kGeluP[kGeluDeg + 1] = {"):]
    coef = [float(v) for v in re.findall(r"([-0-9.e+]+)f,", body[:body.index("};")])]
    assert len(coef) == deg + 1
    return np.float32(kt), np.array(coef, dtype=np.float32)


def exponent_exact(x):
    """log2(erfc(z) e^(z^2) / (2 t)) for z = |x| / sqrt 2, in float64."""
    kt, _ = read_header()
    t = 1.0 / (1.0 + float(kt) * np.abs(x))
    return np.log(erfcx(np.abs(x) / math.sqrt(2.0)) / t) * LOG2E - 1.0, t


def horner(coef, t):
    p = np.zeros_like(t) + float(coef[0])
    for c in coef[1:]:
        p = p * t + float(c)
    return p


def gelu_exact(x):
    return 0.5 * x * erfc(-x / math.sqrt(2.0))


def fit_error(coef):
    x = np.linspace(0.0, 6.5 * math.sqrt(2.0), 200001)
    ex, t = exponent_exact(x)
    return float(np.max(np.abs(horner(coef, t) - ex)))


def test_fit_error_on_the_fitted_range():
    _, coef = read_header()
    assert fit_error(coef) < 2.5e-7


def test_perturbed_coefficient_fails():
    _, coef = read_header()
    bad = coef.copy()
    bad[3] = np.float32(bad[3] * (1 + 1e-4))
    assert fit_error(bad) > 2.5e-7


def test_tail_beyond_the_fit_decays():
    """Past z = 6.5 the polynomial is extrapolated; the result must stay a
    tiny fraction of x (exact GELU is below 1e-19 |x| there)."""
    _, coef = read_header()
    x = -np.linspace(6.5 * math.sqrt(2.0), 60.0, 20001)
    ex, t = exponent_exact(x)
    p = horner(coef, t)
    assert np.all(np.isfinite(p)) and np.max(np.abs(p - ex)) < 1.0
    h = np.abs(x * t) * np.exp2(p - 0.5 * x * x * LOG2E)
    assert np.max(h / np.abs(x)) < 1e-18


def _fma32(a, b, c):
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def gelu_fp32(x, kt, coef):
    """The kernel's operation order in FP32 (reciprocal and exp2 rounded
    once, FMAs rounded once)."""
    x = np.float32(x)
    t = np.float32(1.0 / np.float64(_fma32(abs(x), kt, np.float32(1.0))))
    p = coef[0]
    for c in coef[1:]:
        p = _fma32(p, t, c)
    q = np.float32(x * np.float32(-0.5 * LOG2E))
    e = np.float32(2.0 ** np.float64(_fma32(q, x, p)))
    return _fma32(-abs(np.float32(x * t)), e, max(x, np.float32(0.0)))


def test_fp32_result_error():
    kt, coef = read_header()
    xs = np.concatenate([np.linspace(-8.0, 8.0, 16001), np.geomspace(1e-6, 8.0, 3000),
                         -np.geomspace(1e-6, 8.0, 3000)])
    bounds = [(-8.0, -5.0, 5e-6), (-5.0, -2.0, 2e-6), (-2.0, 2.0, 8e-7), (2.0, 8.01, 2e-7)]
    for lo, hi, tol in bounds:
        sel = xs[(xs >= lo) & (xs < hi)]
        err = max(abs(float(gelu_fp32(x, kt, coef)) - gelu_exact(float(np.float32(x))))
                  / abs(gelu_exact(float(np.float32(x)))) for x in sel if x != 0.0)
        assert err < tol, (lo, hi, err)
