// Rotation lists of Alg. 2's Euler parameterisation (host code, no device use).
//
// Alg. 2 loops over three angles (theta, phi, xi), each from -K delta_r to
// +K delta_r in steps of delta_r, theta outermost.  The paper does not fix the
// Euler convention; this library reads R(theta, phi, xi) = Rz(theta) Ry(phi) Rx(xi)
// (intrinsic z-y-x), applied after an optional centre rotation C (the initial
// guess of a local registration): R = C R(theta, phi, xi).  Computed in double,
// stored as float32 row-major 3x3.
#include <cmath>

#include "host.h"

using namespace dses;

extern "C" dses_status dses_rotations_euler(const float *center, int32_t K, float step,
                                            float *out)
{
    set_error("");
    if (!out || K < 0 || K > 200 || !(step > 0.0f) || !std::isfinite(step)) {
        set_error("need an output buffer, 0 <= K <= 200 and a positive finite step");
        return DSES_E_INVAL;
    }
    double C[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (center)
        for (int e = 0; e < 9; ++e) C[e] = center[e];
    const int side = 2 * K + 1;
    size_t o = 0;
    for (int a = 0; a < side; ++a)
        for (int b = 0; b < side; ++b)
            for (int c = 0; c < side; ++c) {
                const double th = (a - K) * (double)step, ph = (b - K) * (double)step,
                             xi = (c - K) * (double)step;
                const double ct = std::cos(th), st = std::sin(th), cp = std::cos(ph),
                             sp = std::sin(ph), cx = std::cos(xi), sx = std::sin(xi);
                // Rz(theta) Ry(phi) Rx(xi)
                const double E[9] = {ct * cp, ct * sp * sx - st * cx, ct * sp * cx + st * sx,
                                     st * cp, st * sp * sx + ct * cx, st * sp * cx - ct * sx,
                                     -sp,     cp * sx,                cp * cx};
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double v = 0.0;
                        for (int l = 0; l < 3; ++l) v += C[3 * i + l] * E[3 * l + j];
                        out[o + 3 * i + j] = (float)v;
                    }
                o += 9;
            }
    return DSES_OK;
}
