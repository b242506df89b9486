// Written by gelu_fit.py (same folder): the polynomial of the network
// kernels' GELU, P(t) ~ log2(erfc(z) / t) + z^2 log2(e) - 1 with
// t = 1 / (1 + 0.3 z), z = |x| / sqrt 2, degree 7, fitted on z in [0, 6.5].
#pragma once

namespace pr {

constexpr float kGeluT = 0.212132037f;  // 0.3 / sqrt 2: t = 1 / (1 + kGeluT |x|)
constexpr int kGeluDeg = 7;
// coefficients of P, highest degree first
constexpr float kGeluP[kGeluDeg + 1] = {
    0.763559401f,
    -3.1534512f,
    4.7543292f,
    -3.64550114f,
    2.1981976f,
    0.123973601f,
    1.52731931f,
    -3.56842661f,
};

}  // namespace pr
