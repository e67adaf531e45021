// Learned correction of the order-2 rule for separated element pairs in
// the closest distance classes (Sec. 5 pair decomposition, App. B orders):
// canonical pair form, features and the 9-64-64-21 tanh network on the
// FP16 matrix cores (v_mfma_f32_16x16x32_f16, FP32 accumulation).
//
// Canonical form of a pair (K, Kt) (invariant under similarity maps and
// vertex relabelling; every quantity it compares is computed the same way
// whatever the input order, so ties resolve identically everywhere):
//   * the triangle with the larger squared longest edge comes first
//     (equal: the one whose lexicographically smallest vertex is smaller);
//   * each triangle is ordered (a, b, c) with ab a longest edge (several:
//     the one whose opposite vertex is lexicographically smallest) and c
//     to the left of a -> b.
// Features: c of the first triangle and the canonical vertices of the
// second in the first's frame (origin a, x axis b - a, unit |b - a|), and
// s.  Outputs: relative errors t = I / Q2 - 1 of the order-2 rule for the
// 21 integrals SK (a <= b), ST (a <= b), X (row-major) in canonical order;
// the corrected values Q2 (1 + t) are then made consistent with the sum
// rules (sur_sum_rules).
#pragma once

#include <hip/hip_runtime.h>

namespace fl {

constexpr int SUR_NIN = 9, SUR_NH = 64, SUR_NOUT = 21, SUR_KIN = 32, SUR_KOUT = 32;
constexpr int SUR_OW1 = 0;
constexpr int SUR_OB1 = SUR_OW1 + SUR_NH * SUR_KIN;
constexpr int SUR_OW2 = SUR_OB1 + SUR_NH;
constexpr int SUR_OB2 = SUR_OW2 + SUR_NH * SUR_NH;
constexpr int SUR_OW3 = SUR_OB2 + SUR_NH;
constexpr int SUR_OB3 = SUR_OW3 + SUR_KOUT * SUR_NH;
constexpr int SUR_NPARAM = SUR_OB3 + SUR_KOUT;  // 8352
constexpr int SUR_NRB = 6, SUR_NSB = 4;         // distance bins x s bins

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Network views for inference: FP16 weights (row-major W1 64x32, W2 64x64,
// W3 32x64), FP32 biases, FP32 standardisation (feature means mx and
// reciprocal deviations isx; target means mt and deviations st).
struct SurNet {
    const _Float16* W1;
    const _Float16* W2;
    const _Float16* W3;
    const float* b1;
    const float* b2;
    const float* b3;
    const float* mx;
    const float* isx;
    const float* mt;
    const float* st;
};

// ------------------------------------------------------ canonical form --

__device__ __forceinline__ double sur_sq(double px, double py, double qx, double qy) {
#pragma clang fp contract(off)
    const double dx = px - qx, dy = py - qy;
    const double a = dx * dx, b = dy * dy;
    return a + b;
}

__device__ __forceinline__ bool sur_lexless(double px, double py, double qx, double qy) {
    return px < qx || (px == qx && py < qy);
}

// vertex order (o[0], o[1], o[2]) of triangle P (x0 y0 x1 y1 x2 y2)
__device__ __forceinline__ void sur_canon_tri(const double* P, int* o) {
#pragma clang fp contract(off)
    double L[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = (i + 1) % 3;
        L[i] = sur_sq(P[2 * j], P[2 * j + 1], P[2 * i], P[2 * i + 1]);
    }
    const double mx = fmax(fmax(L[0], L[1]), L[2]);
    int best = -1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (L[i] != mx) continue;
        const int c = (i + 2) % 3;
        if (best < 0) {
            best = i;
        } else {
            const int cb = (best + 2) % 3;
            if (sur_lexless(P[2 * c], P[2 * c + 1], P[2 * cb], P[2 * cb + 1])) best = i;
        }
    }
    int ia = best, ib = (best + 1) % 3;
    const int ic = (best + 2) % 3;
    const double ax = P[2 * ia], ay = P[2 * ia + 1];
    const double u0 = P[2 * ib] - ax, u1 = P[2 * ib + 1] - ay;
    const double w0 = P[2 * ic] - ax, w1 = P[2 * ic + 1] - ay;
    const double p = u0 * w1, q = u1 * w0;
    if (p - q < 0.0) {
        const int t = ia;
        ia = ib;
        ib = t;
    }
    o[0] = ia;
    o[1] = ib;
    o[2] = ic;
}

__device__ __forceinline__ double sur_h2(const double* P) {
    const double a = sur_sq(P[2], P[3], P[0], P[1]);
    const double b = sur_sq(P[4], P[5], P[2], P[3]);
    const double c = sur_sq(P[0], P[1], P[4], P[5]);
    return fmax(fmax(a, b), c);
}

__device__ __forceinline__ void sur_lexmin(const double* P, double& x, double& y) {
    x = P[0];
    y = P[1];
#pragma unroll
    for (int i = 1; i < 3; ++i)
        if (sur_lexless(P[2 * i], P[2 * i + 1], x, y)) {
            x = P[2 * i];
            y = P[2 * i + 1];
        }
}

// Canonical form of (X, Y).  Returns swap (1: Y first); o1 / o2: vertex
// orders of the first / second triangle; C1 / C2 their canonical
// coordinates.
__device__ __forceinline__ int sur_canon(const double* X, const double* Y, int* o1, int* o2, double* C1,
                                         double* C2) {
    const double hX = sur_h2(X), hY = sur_h2(Y);
    int swap = 0;
    if (hY > hX) {
        swap = 1;
    } else if (hY == hX) {
        double xx, xy, yx, yy;
        sur_lexmin(X, xx, xy);
        sur_lexmin(Y, yx, yy);
        swap = sur_lexless(yx, yy, xx, xy) ? 1 : 0;
    }
    const double* F = swap ? Y : X;
    const double* S = swap ? X : Y;
    sur_canon_tri(F, o1);
    sur_canon_tri(S, o2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        C1[2 * i] = F[2 * o1[i]];
        C1[2 * i + 1] = F[2 * o1[i] + 1];
        C2[2 * i] = S[2 * o2[i]];
        C2[2 * i + 1] = S[2 * o2[i] + 1];
    }
    return swap;
}

// features (9) of a pair in canonical form
__device__ __forceinline__ void sur_features(const double* C1, const double* C2, double s, double* f) {
#pragma clang fp contract(off)
    const double ax = C1[0], ay = C1[1];
    const double ex = C1[2] - ax, ey = C1[3] - ay;
    const double L2 = ex * ex + ey * ey;
    auto frame = [&](double px, double py, double& u, double& v) {
        const double dx = px - ax, dy = py - ay;
        const double p1 = dx * ex, p2 = dy * ey, q1 = ex * dy, q2 = ey * dx;
        u = (p1 + p2) / L2;
        v = (q1 - q2) / L2;
    };
    frame(C1[4], C1[5], f[0], f[1]);
    frame(C2[0], C2[1], f[2], f[3]);
    frame(C2[2], C2[3], f[4], f[5]);
    frame(C2[4], C2[5], f[6], f[7]);
    f[8] = s;
}

// distance bin from the features: centroid distance in the first
// triangle's frame against the edges 1, 1.5, 2, 2.5, 3
__device__ __forceinline__ int sur_rbin_features(const double* f) {
#pragma clang fp contract(off)
    const double cx = (1.0 + f[0]) / 3.0, cy = f[1] / 3.0;
    const double tx = ((f[2] + f[4]) + f[6]) / 3.0, ty = ((f[3] + f[5]) + f[7]) / 3.0;
    const double dx = tx - cx, dy = ty - cy;
    const double a = dx * dx, b = dy * dy;
    const double d2 = a + b;
    const double e2[5] = {1.0, 2.25, 4.0, 6.25, 9.0};
    int c = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
        if (d2 >= e2[i]) c = i + 1;
    return c;
}

__device__ __forceinline__ int sur_sbin(double s) {
    return (s >= 0.25) + (s >= 0.5) + (s >= 0.75);
}

// The barycentric coordinates sum to 1 on each element, so every
// quadrature of a separated pair satisfies sum_b SK_ab = sum_b X_ab and
// sum_a ST_ab = sum_a X_ab; the network's corrections do not.  Recomputing
// the six diagonal values from the others restores both, so the assembled
// matrix keeps the zero row sums of its Omega x Omega part (constants stay
// in its kernel).  SK, ST: symmetric slots 00 01 02 11 12 22; O row-major.
__device__ __forceinline__ void sur_sum_rules(double* SK, double* ST, const double* O) {
    SK[0] = (O[0] + O[1] + O[2]) - SK[1] - SK[2];
    SK[3] = (O[3] + O[4] + O[5]) - SK[1] - SK[4];
    SK[5] = (O[6] + O[7] + O[8]) - SK[2] - SK[4];
    ST[0] = (O[0] + O[3] + O[6]) - ST[1] - ST[2];
    ST[3] = (O[1] + O[4] + O[7]) - ST[1] - ST[4];
    ST[5] = (O[2] + O[5] + O[8]) - ST[2] - ST[4];
}

// ------------------------------------------------------------- network --

// standardised FP32 features
__device__ __forceinline__ void sur_std_features(const SurNet& N, const double* F, float* xn) {
#pragma unroll
    for (int k = 0; k < SUR_NIN; ++k) xn[k] = (float)(F[k] - (double)N.mx[k]) * N.isx[k];
}

// tanh in FP32: odd Taylor polynomial below |z| = 0.5 (error < 2e-6
// relative), (1 - e) / (1 + e) with e = exp(-2|z|) above.
__device__ __forceinline__ float sur_tanh(float z) {
    const float a = fabsf(z);
    float r;
    if (a < 0.5f) {
        const float z2 = a * a;
        float p = 62.f / 2835.f;
        p = p * z2 - 17.f / 315.f;
        p = p * z2 + 2.f / 15.f;
        p = p * z2 - 1.f / 3.f;
        p = p * z2 + 1.f;
        r = a * p;
    } else {
        const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * a);  // exp(-2a)
        r = (1.f - e) * __builtin_amdgcn_rcpf(1.f + e);
    }
    return copysignf(r, z);
}

__device__ __forceinline__ f4 sur_mma(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ h8 sur_cat(h4 lo, h4 hi) {
    return h8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

__device__ __forceinline__ h4 sur_h4(f4 v) {
    return h4{(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]};
}

// Register layout of one wave working on 16 samples.  Lane l = 16 g + r
// (r = l & 15, g = l >> 4).  The products are computed transposed
// (Z^T = W X^T): the matrix-core A operand is a weight tile, B the
// activations; the f32 result of a 16-unit tile t leaves lane (r, g)
// holding units 16 t + 4 g + v (v = 0..3) of sample r.  The next layer's
// B operand for K chunk c (units 32 c .. 32 c + 31) is then the lane's own
// values of tiles 2c and 2c+1 (K slots e = 0..3 -> unit 32c + 4g + e,
// e = 4..7 -> unit 32c + 16 + 4g + e - 4), and the weight operand is read
// with the same slot map, so no data moves between lanes.
struct SurAct {
    f4 z1[4], z2[4];  // pre-activations (kept for the backward pass)
    h4 h1[4], h2[4];  // FP16 activations
    f4 out[2];        // outputs, units 0..31
};

// Forward pass of 16 samples.  xb: the lane's B operand of layer 1,
// standardised features of sample r in K slots 8g..8g+7 (inputs 8g..8g+7;
// slots >= 9 zero).
__device__ __forceinline__ void sur_forward16(const SurNet& N, h8 xb, SurAct& a) {
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const h8 w = *(const h8*)(N.W1 + (16 * t + r) * SUR_KIN + 8 * g);
        a.z1[t] = sur_mma(w, xb, zero);
        f4 h;
#pragma unroll
        for (int v = 0; v < 4; ++v) h[v] = sur_tanh(a.z1[t][v] + N.b1[16 * t + 4 * g + v]);
        a.h1[t] = sur_h4(h);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f4 z = zero;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const _Float16* wr = N.W2 + (16 * t + r) * SUR_NH + 32 * c + 4 * g;
            const h8 w = sur_cat(*(const h4*)wr, *(const h4*)(wr + 16));
            z = sur_mma(w, sur_cat(a.h1[2 * c], a.h1[2 * c + 1]), z);
        }
        a.z2[t] = z;
        f4 h;
#pragma unroll
        for (int v = 0; v < 4; ++v) h[v] = sur_tanh(z[v] + N.b2[16 * t + 4 * g + v]);
        a.h2[t] = sur_h4(h);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f4 z = zero;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const _Float16* wr = N.W3 + (16 * t + r) * SUR_NH + 32 * c + 4 * g;
            const h8 w = sur_cat(*(const h4*)wr, *(const h4*)(wr + 16));
            z = sur_mma(w, sur_cat(a.h2[2 * c], a.h2[2 * c + 1]), z);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) z[v] += N.b3[16 * t + 4 * g + v];
        a.out[t] = z;
    }
}

// Layer-1 operand of sample r of group q (lanes 16 q .. 16 q + 15 own the
// samples; each holds its 9 standardised features as 5 packed FP16 pairs
// p[0..4], feature 2i in the low half of p[i]).  Every lane of the wave
// must call this (it uses cross-lane reads).
__device__ __forceinline__ h8 sur_gather_x(const unsigned int* p, int q) {
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int src = 16 * q + r;
    unsigned int w[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) w[i] = (unsigned int)__shfl((int)p[i], src, 64);
    unsigned int o[4] = {0u, 0u, 0u, 0u};
    if (g == 0) {
        o[0] = w[0];
        o[1] = w[1];
        o[2] = w[2];
        o[3] = w[3];
    } else if (g == 1) {
        o[0] = w[4];
    }
    h8 x;
    __builtin_memcpy(&x, o, sizeof(x));
    return x;
}

// pack standardised features (float) into FP16 pairs
__device__ __forceinline__ void sur_pack_x(const float* xn, unsigned int* p) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const _Float16 lo = (_Float16)xn[2 * i];
        const _Float16 hi = (2 * i + 1 < SUR_NIN) ? (_Float16)xn[2 * i + 1] : (_Float16)0.f;
        unsigned short a, b;
        __builtin_memcpy(&a, &lo, 2);
        __builtin_memcpy(&b, &hi, 2);
        p[i] = (unsigned int)a | ((unsigned int)b << 16);
    }
}

}  // namespace fl
