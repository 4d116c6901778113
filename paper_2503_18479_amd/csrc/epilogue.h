// Loss epilogue shared by the fused kernels and the large-loop-count path:
// for one complex field value B = (x, y) and its target t, the loss term of
// Eq. 1 and, in place of B, the weight w = dL/d conj(B) of the adjoint.
//   MAG:     term (|B| - t)^2, w = (1 - t/|B|) B;
//   COMPLEX: term |B - t|^2,   w = B - t;
//   RATIO:   MAG of the total field B + inc (inc: the incident field, real),
//            w = (1 - t/|B + inc|) (B + inc); with t = beta |inc| and the
//            caller's scale 1/inc^2 this is the enhancement-factor loss
//            (beta_hat - beta)^2, beta_hat = |B + inc| / |inc| (Sec. IV-B).
#pragma once
#include "internal.h"

namespace cosim {

// Per-element loss epilogue.  MAG: e = |B| - T, w = e B/|B| (0 where B = 0).
// COMPLEX: e = B - T, w = e.  Returns e^2 (|e|^2) and overwrites (x, y) by w.
// FP32 form: with s = 1/sqrt(|B|^2) (hardware rsq, ~1 ulp), |B| = |B|^2 s and
// e/|B| = 1 - T s, which needs neither a square root nor a division.
template <int LOSS>
__device__ inline float epilogue_f(float &x, float &y, float t, float inc = 0.0f) {
    if (LOSS == COSIM_LOSS_RATIO) x += inc;
    if (LOSS == COSIM_LOSS_MAG || LOSS == COSIM_LOSS_RATIO) {
        // A normal floor of 1e-36 is added to |B|^2 (inside the products, at
        // no extra instruction): at B = 0 this gives e = -t (loss t^2) and
        // w = c B = 0 without a branch; above |B| ~ 1e-12 it is far below the
        // rounding of |B|^2, and below |B| ~ 1e-18 the magnitude's derivative
        // is singular anyway.
        const float m2 = fmaf(x, x, fmaf(y, y, 1e-36f));
        const float rs = __builtin_amdgcn_rsqf(m2);
        const float e = fmaf(m2, rs, -t);
        const float c = fmaf(-t, rs, 1.0f);
        x *= c;
        y *= c;
        return e * e;
    } else {
        const float ex = x - t;
        x = ex;
        return fmaf(ex, ex, y * y);
    }
}

template <int LOSS, typename T>
__device__ inline double epilogue(T &x, T &y, T t, T inc = T(0)) {
    if constexpr (sizeof(T) == 4) {
        return (double)epilogue_f<LOSS>(x, y, t, inc);
    } else if (LOSS == COSIM_LOSS_MAG || LOSS == COSIM_LOSS_RATIO) {
        if (LOSS == COSIM_LOSS_RATIO) x += inc;
        const T mag = sqrt(x * x + y * y);
        const T e = mag - t;
        const T c = mag > T(0) ? e / mag : T(0);
        x *= c;
        y *= c;
        return (double)e * (double)e;
    } else {
        const T ex = x - t;
        const double v = (double)ex * ex + (double)y * y;
        x = ex;
        return v;
    }
}


}  // namespace cosim
