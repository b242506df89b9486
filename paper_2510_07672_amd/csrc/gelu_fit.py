"""Coefficients of the network kernels' GELU (gelu_f32 in cnn_kernels.hip).

GELU(x) = x/2 (1 + erf(x / sqrt 2)).  With z = |x| / sqrt 2 the kernels use
the form erfc(z) = t exp(-z^2 + Q(t)), t = 1 / (1 + C z), and evaluate
h = x erfc(z) / 2 as x t 2^(P(t) - z^2 log2 e) with P = log2(e) Q - 1.  P is a
polynomial of degree DEG fitted here to

    log2(erfc(z) / t) + z^2 log2 e - 1,   z in [0, ZMAX],

by weighted least squares in t (sampled at Chebyshev points), the weights
multiplied each round by the square root of the relative residual, which
drives the fit toward the smallest maximum error.  Beyond ZMAX the form
still decays like exp(-z^2) (P stays bounded on 0 < t <= 1), and erfc(ZMAX)
is below 1e-19.

Run from the repository root to rewrite gelu_coef.h beside this file:

    python3 paper_2510_07672_amd/csrc/gelu_fit.py
"""
import os

import numpy as np
from scipy.special import log_ndtr

DEG, C, ZMAX = 7, 0.3, 6.5
LOG2E = 1.0 / np.log(2.0)


def target(z):
    """log2(erfc(z) / t) + z^2 log2 e - 1 for t = 1 / (1 + C z)."""
    t = 1.0 / (1.0 + C * z)
    log_erfc = np.log(2.0) + log_ndtr(-z * np.sqrt(2.0))
    return (log_erfc - np.log(t) + z * z) * LOG2E - 1.0


def fit():
    """Monomial coefficients of P, highest degree first, in float64."""
    tmin = 1.0 / (1.0 + C * ZMAX)
    t = tmin + (1.0 - tmin) * (0.5 + 0.5 * np.cos(np.linspace(0.0, np.pi, 40001)))
    z = (1.0 / t - 1.0) / C
    f = target(z)
    V = np.vander(t, DEG + 1)
    w = np.ones_like(t)
    for _ in range(80):
        coef, *_ = np.linalg.lstsq(V * w[:, None], f * w, rcond=None)
        r = np.abs(V @ coef - f)
        w = w * np.sqrt(r / r.max() + 1e-4)
        w /= w.max()
    return coef


def main():
    coef = fit().astype(np.float32)
    kt = np.float32(C / np.sqrt(2.0))
    lines = [
        "// Written by gelu_fit.py (same folder): the polynomial of the network",
        "// kernels' GELU, P(t) ~ log2(erfc(z) / t) + z^2 log2(e) - 1 with",
        f"// t = 1 / (1 + {C} z), z = |x| / sqrt 2, degree {DEG}, fitted on z in [0, {ZMAX}].",
        "#pragma once",
        "",
        "namespace pr {",
        "",
        f"constexpr float kGeluT = {float(kt):.9g}f;  // {C} / sqrt 2: t = 1 / (1 + kGeluT |x|)",
        f"constexpr int kGeluDeg = {DEG};",
        "// coefficients of P, highest degree first",
        "constexpr float kGeluP[kGeluDeg + 1] = {",
    ]
    lines += [f"    {float(c):.9g}f," for c in coef]
    lines += ["};", "", "}  // namespace pr", ""]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gelu_coef.h")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print("wrote", out)


if __name__ == "__main__":
    main()
