// Kernel power |x-y|^{-d-2s} = (r^2)^pe for r^2 > 0 finite and |pe| <= 2,
// in FP64 without the special-case handling of a general pow:
//   ln(r^2): r^2 = m 2^e with m in [1/sqrt2, sqrt2); ln m = 2 atanh(t),
//            t = (m-1)/(m+1), |t| <= 0.1716, by its Taylor series
//            2t (1 + t^2/3 + t^4/5 + ...) to t^22 (remainder < 3e-18);
//   exp(P):  Cody-Waite reduction P = k ln2 + r (ln2 split in a 32-bit head
//            and a tail, |r| <= ln2/2) and the Taylor series of exp(r) to r^12
//            (remainder < 2e-16), scaled by 2^k.
// Relative error about 2e-15 for |pe ln r^2| <= 40, dominated by the rounding
// of pe * ln r^2.
#pragma once

#include <hip/hip_runtime.h>

namespace fl {

__host__ __device__ inline double kpow(double r2, double pe) {
#if defined(__HIP_DEVICE_COMPILE__)
    double m = __builtin_amdgcn_frexp_mant(r2);  // r2 = m 2^e, m in [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(r2);
#else
    int e;
    double m = frexp(r2, &e);
#endif
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
#if defined(__HIP_DEVICE_COMPILE__)
    // t = (m-1)/(m+1): hardware reciprocal refined by one Newton step
    const double den = m + 1.0;
    double y = __builtin_amdgcn_rcp(den);
    y = fma(y, fma(-den, y, 1.0), y);
    const double t = (m - 1.0) * y;
#else
    const double t = (m - 1.0) / (m + 1.0);
#endif
    const double t2 = t * t;
    double q = 2.0 / 23.0;
    q = fma(q, t2, 2.0 / 21.0);
    q = fma(q, t2, 2.0 / 19.0);
    q = fma(q, t2, 2.0 / 17.0);
    q = fma(q, t2, 2.0 / 15.0);
    q = fma(q, t2, 2.0 / 13.0);
    q = fma(q, t2, 2.0 / 11.0);
    q = fma(q, t2, 2.0 / 9.0);
    q = fma(q, t2, 2.0 / 7.0);
    q = fma(q, t2, 2.0 / 5.0);
    q = fma(q, t2, 2.0 / 3.0);
    q = fma(q, t2, 2.0);
    const double lnm = t * q;
    const double LN2_HI = 6.93147180369123816490e-01;  // 32 significant bits
    const double LN2_LO = 1.90821492927058770002e-10;
    const double de = (double)e;
    const double P = pe * fma(de, LN2_HI, fma(de, LN2_LO, lnm));
    const double kf = rint(P * 1.44269504088896340736);
    double r = fma(-kf, LN2_HI, P);
    r = fma(-kf, LN2_LO, r);
    double p = 1.0 / 479001600.0;  // 1/12!
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)kf);
}

// Kernel power r2^pe by tables held in LDS (pw: pairs (2/m_i, m_i^pe), m_i = 1 + (i +
// 1/2)/256, then 2^(pe n), n = -128..127; 768 doubles) with the
// coefficients C(pe, k): r2 = 2^n m with m in [1, 2) (n from the exponent
// field, i = the top 8 mantissa bits, m / 2 from v_frexp_mant_f64), the
// remaining factor m / m_i = 1 + t (|t| <= 1/512) is raised to pe by its degree-5
// Taylor polynomial.  No transcendental and ~9 FP64 operations instead of
// ~38; relative error below 1e-15 for r2 in [2^-128, 2^128) (callers keep
// their squared distances inside).
struct KPowTab {
    const double* pw;
    double c1, c2, c3, c4, c5;
    __device__ __forceinline__ double operator()(double r2) const {
        const long long bits = __double_as_longlong(r2);
        const int hi = (int)(bits >> 32);
        const int n = (hi >> 20) - 895;  // biased exponent - 1023 + 128
        const int i = (hi >> 12) & 255;
        const double mh = __builtin_amdgcn_frexp_mant(r2);  // mantissa / 2, in [1/2, 1)
        const double2 f = ((const double2*)pw)[i];          // 2/m_i, m_i^pe
        const double t = fma(mh, f.x, -1.0);                 // = m / m_i - 1 exactly as with m, 1/m_i
        double p = fma(c5, t, c4);
        p = fma(p, t, c3);
        p = fma(p, t, c2);
        p = fma(p, t, c1);
        p = fma(p, t, 1.0);
        return (p * f.y) * pw[512 + n];
    }
};

}  // namespace fl
