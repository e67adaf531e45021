// Device kernels for the dense P1 stiffness matrix of the integral
// fractional Laplacian (Ainsworth & Glusa, arXiv:1708.03912), gfx950.
//
// Assembly follows the element-pair decomposition of Sec. 5:
//   separated pairs  -> far_kernel   (tensor Gauss, order by distance class,
//                                     App. B), tiled 64 x 64 elements,
//                                     LDS-accumulated, FP64
//   identical pairs  -> self_kernel  (regularised, 1D integrals over the
//                                     difference hexagon)
//   boundary facets  -> self_kernel  (a^{Kxe}, Sec. 2 / Sec. 5)
//   edge / vertex    -> touch kernels (regularised, analytic radial factor)
//   diagonal blocks  -> scatter_self (gather per DOF row, deterministic)
// The product and CG kernels are in fl_solve.hip.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "fl_internal.hpp"
#include "fl_math.hpp"

namespace fl {

__constant__ RuleTables c_R;

hipError_t upload_rules(const RuleTables& R, hipStream_t st) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_R), &R, sizeof(RuleTables), 0,
                                  hipMemcpyHostToDevice, st);
}

// Dense assembly accumulates the upper triangle only (entry (min, max) of
// every contribution to (i, j) and (j, i): one FP64 atomic where a
// symmetric pair of atomics would go, which halves the traffic that limits
// the tile flush); mirror_lower_kernel copies it to the lower triangle.
__device__ __forceinline__ long long upper_index(int i, int j, long long lda) {
    return i <= j ? (long long)i * lda + j : (long long)j * lda + i;
}

// an off-diagonal contribution v to (i, j) and to (j, i): once in the upper
// triangle, twice when i = j (two vertices folded onto one DOF)
__device__ __forceinline__ void add_pair_upper(const FarParams& P, int i, int j, double v) {
    acc_add(P.fa, P.A, upper_index(i, j, P.lda), i == j ? 2.0 * v : v);
}

__device__ __forceinline__ int sym3(int a, int b) {
    // upper-triangular slot of (a,b), a <= b, in a 3x3 symmetric block
    return a <= b ? a * 3 - a * (a + 1) / 2 + b : b * 3 - b * (b + 1) / 2 + a;
}

// Weight of the cell pair (K, Kt) in a symmetry-reduced assembly (1
// without one): sector pairs 1, image pairs 0; a sector cell S (internal
// index = its caller index) with an image L of the sector cell p under
// B^i: 1/2 without preimage data (both members of each couple
// (S, B^i p) ~ (p, B^-i S) are present), with it 1 for p > S, 0 for p < S,
// and for p = S 1 if 2 i < K, 1/2 if 2 i = K, 0 else.
__device__ __forceinline__ double pair_w(const ElemDev& E, int K, int Kt) {
    if (!E.w) return 1.0;
    const double wK = E.w[K], wT = E.w[Kt];
    if (!E.spre) return 0.5 * (wK + wT);
    if (wK == wT) return wK;
    const int S = wK > wT ? K : Kt, L = wK > wT ? Kt : K;
    const int p = E.spre[L];
    if (p != S) return p > S ? 1.0 : 0.0;
    const int r2 = 2 * E.srot[L];
    return r2 < E.sorder ? 1.0 : (r2 == E.sorder ? 0.5 : 0.0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sums over the wave of four values at once (halving exchange): after the
// xor-32 and xor-16 steps lane l holds a partial sum of value
// m = 2 b5 + b4 (b: lane bits), the xor-8 .. 1 steps finish it; lane 16 m
// returns the sum of v[m].  7 exchanges instead of 24.
__device__ __forceinline__ double wave_sum4(const double* v, int lane) {
    const int h5 = (lane >> 5) & 1, h4 = (lane >> 4) & 1;
    double w[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double mine = h5 ? v[2 + j] : v[j];
        const double give = h5 ? v[j] : v[2 + j];
        w[j] = mine + __shfl_xor(give, 32, 64);
    }
    double x = (h4 ? w[1] : w[0]) + __shfl_xor(h4 ? w[0] : w[1], 16, 64);
    x += __shfl_xor(x, 8, 64);
    x += __shfl_xor(x, 4, 64);
    x += __shfl_xor(x, 2, 64);
    x += __shfl_xor(x, 1, 64);
    return x;
}

// The same four sums by cross-lane VALU operations instead of LDS
// permutes: v_permlane32_swap(x, y) exchanges the upper 32 lanes of x with
// the lower 32 lanes of y, so the sum of its two results holds, in the
// lower half, x summed over the lane pairs (l, l + 32) and, in the upper
// half, y summed over them; v_permlane16_swap does the same for the 16-lane
// rows (rows 0, 2 take x, rows 1, 3 take y); four DPP row rotations (by 8,
// 4, 2, 1) complete the sums within each row.  Every lane of row m returns
// the sum of v[m].
__device__ __forceinline__ double dsum_pl32(double x, double y) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double dsum_pl16(double x, double y) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// (a row rotation reads a valid lane for every lane, so the moves need no
// initialised destination)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum4_lanes(const double* v) {
    const double w0 = dsum_pl32(v[0], v[2]), w1 = dsum_pl32(v[1], v[3]);
    double x = dsum_pl16(w0, w1);
    x += dpp_d<0x128>(x);  // row_ror:8
    x += dpp_d<0x124>(x);  // row_ror:4
    x += dpp_d<0x122>(x);  // row_ror:2
    x += dpp_d<0x121>(x);  // row_ror:1
    return x;
}

// Sums over the wave of six values at once (halving exchange): after the
// xor-32 / 16 / 8 steps each lane holds a partial sum of one slot
// m = 4 b5 + 2 b4 + b3 (b: lane bits), the xor-4 / 2 / 1 steps finish it;
// lane 8 m returns the sum of v[m] (m < 6).  10 exchanges instead of 36.
__device__ __forceinline__ double wave_sum6(const double* v, int lane) {
    const int h5 = (lane >> 5) & 1, h4 = (lane >> 4) & 1, h3 = (lane >> 3) & 1;
    double w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double mine = (4 * h5 + j) < 6 ? v[4 * h5 + j] : 0.0;
        const double give = (4 * (1 - h5) + j) < 6 ? v[4 * (1 - h5) + j] : 0.0;
        w[j] = mine + __shfl_xor(give, 32, 64);
    }
    double x[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) x[j] = w[2 * h4 + j] + __shfl_xor(w[2 * (1 - h4) + j], 16, 64);
    double y = x[h3] + __shfl_xor(x[1 - h3], 8, 64);
    y += __shfl_xor(y, 4, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 1, 64);
    return y;
}

// Calls f(rr, cc) for the entries i = tid, tid + 256, ... of an nr x nc
// block (i = rr nc + cc; 256 threads), the pair advanced by the fixed step
// (256 / nc, 256 mod nc) instead of a division per entry.
template <class F>
__device__ __forceinline__ void for_block_entries(int nr, int nc, int tid, F&& f) {
    if (nr <= 0 || nc <= 0) return;
    const int dr = 256 / nc, dc = 256 - dr * nc;
    int rr = tid / nc, cc = tid - rr * nc;
    while (rr < nr) {
        f(rr, cc);
        rr += dr;
        cc += dc;
        if (cc >= nc) {
            cc -= nc;
            ++rr;
        }
    }
}

// ----------------------------------------------------------- separated --

// Separated triangles with the order-k collapsed rule on both.  X, Y:
// vertex coordinates.  Outputs raw sums without area / C factors:
//   SK[sym] = sum_pq w_p w_q l_a l_b(x_p) k,  ST likewise with y_q,
//   O[3a+b] = sum_pq w_p w_q l_a(x_p) l_b(y_q) k.
// Loop order q (points of Kt) outside, p (points of K) inside; the inner
// loop carries only scalar accumulators, every rule-dependent factor
// (w, w l_a, w l_a l_b) comes from the constant table.  k is uniform across
// the wave, so the table reads are scalar loads.  KO > 0 fixes k = KO at
// compile time (inner loop unrolled: its KO^2 kernel evaluations are
// independent); KO = 0 takes k at run time.
// Kernel power r2^pe: the series routine of fl_math.hpp ...
struct KPow {
    double pe;
    __device__ __forceinline__ double operator()(double r2) const { return kpow(r2, pe); }
};

// ... or by the tables of KPowTab (fl_math.hpp) held in LDS.
__device__ __forceinline__ KPowTab make_kpow_tab(const double* pw_lds) {
    return KPowTab{pw_lds, c_R.pw_c[1], c_R.pw_c[2], c_R.pw_c[3], c_R.pw_c[4], c_R.pw_c[5]};
}

// copy the table part of c_R into LDS (768 doubles; caller synchronises)
__device__ __forceinline__ void load_pow_tables(double* pw) {
    for (int i = threadIdx.x; i < 768; i += blockDim.x)
        pw[i] = i < 512 ? ((i & 1) ? c_R.pw_fr[i >> 1] : c_R.pw_inv[i >> 1]) : c_R.pw_ex[i - 512];
}

// N kernel powers from the LDS tables in three phases -- squared-distance
// bits and table offsets, the table reads, the polynomials -- with
// scheduling barriers between them, so that the N pairs of reads are in
// flight together instead of one pair at a time.
template <int N>
__device__ __forceinline__ void kpow_tab_batch(const KPowTab& kp, const double (&r2)[N], double (&kv)[N]) {
    int hi[N];
    double m[N];
#pragma unroll
    for (int p = 0; p < N; ++p) {
        hi[p] = __double2hiint(r2[p]);
        m[p] = __builtin_amdgcn_frexp_mant(r2[p]);  // mantissa / 2 (the table holds 2 / m_i)
    }
    double2 fr[N];
    double ex[N];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < N; ++p) {
        fr[p] = ((const double2*)kp.pw)[(hi[p] >> 12) & 255];
        ex[p] = kp.pw[512 + (hi[p] >> 20) - 895];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < N; ++p) {
        const double t = fma(m[p], fr[p].x, -1.0);
        double pp = fma(kp.c5, t, kp.c4);
        pp = fma(pp, t, kp.c3);
        pp = fma(pp, t, kp.c2);
        pp = fma(pp, t, kp.c1);
        pp = fma(pp, t, 1.0);
        kv[p] = (pp * fr[p].y) * ex[p];
    }
}

// The same in two stages, for software pipelining: the first computes the
// table offsets and issues the reads of a batch, the second (after other
// work) finishes the powers.
template <int N>
struct KPowStage {
    double m[N];
    double2 fr[N];
    double ex[N];
};

template <int N>
__device__ __forceinline__ void kpow_tab_issue(const KPowTab& kp, const double (&r2)[N], KPowStage<N>& st) {
    int hi[N];
#pragma unroll
    for (int p = 0; p < N; ++p) {
        hi[p] = __double2hiint(r2[p]);
        st.m[p] = __builtin_amdgcn_frexp_mant(r2[p]);  // mantissa / 2 (the table holds 2 / m_i)
    }
#pragma unroll
    for (int p = 0; p < N; ++p) {
        st.fr[p] = ((const double2*)kp.pw)[(hi[p] >> 12) & 255];
        st.ex[p] = kp.pw[512 + (hi[p] >> 20) - 895];
    }
}

template <int N>
__device__ __forceinline__ void kpow_tab_finish(const KPowTab& kp, const KPowStage<N>& st, double (&kv)[N]) {
    // the N Horner chains advance together, one step at a time
    double t[N], pp[N];
#pragma unroll
    for (int p = 0; p < N; ++p) t[p] = fma(st.m[p], st.fr[p].x, -1.0);
#pragma unroll
    for (int p = 0; p < N; ++p) pp[p] = fma(kp.c5, t[p], kp.c4);
#pragma unroll
    for (int p = 0; p < N; ++p) pp[p] = fma(pp[p], t[p], kp.c3);
#pragma unroll
    for (int p = 0; p < N; ++p) pp[p] = fma(pp[p], t[p], kp.c2);
#pragma unroll
    for (int p = 0; p < N; ++p) pp[p] = fma(pp[p], t[p], kp.c1);
#pragma unroll
    for (int p = 0; p < N; ++p) pp[p] = fma(pp[p], t[p], 1.0);
#pragma unroll
    for (int p = 0; p < N; ++p) kv[p] = (pp[p] * st.fr[p].y) * st.ex[p];
}

// Fixed order KO: factorised sums.  With k_pq = k(x_p, y_q) and the rule's
// weights w and barycentric values l:
//   G_p = sum_q w_q k_pq,  H_q = sum_p w_p k_pq,  M_pb = sum_q w_q l_b(y_q) k_pq,
//   SK_ab = sum_p w_p l_a l_b(x_p) G_p,  ST_ab = sum_q w_q l_a l_b(y_q) H_q,
//   O_ab = sum_p w_p l_a(x_p) M_pb.
// Five accumulations per kernel evaluation, and the loop over Kt's points
// needs only the current point's constants plus the KO^2 weights w_p.
template <int KO, class KP>
__device__ __forceinline__ void far_pair2_fixed(const double* X, const double* Y, const KP& kp, double* SK,
                                                double* ST, double* O) {
    constexpr int Q = KO * KO;
    // the rule's offset is opaque to the optimiser, so its constants are
    // fetched by scalar loads on each call instead of being kept live (and
    // spilled) across the caller's loop over pairs
    int off = tri_off(KO);
    asm volatile("" : "+s"(off));
    const double ex0 = X[2] - X[0], ey0 = X[3] - X[1], ex1 = X[4] - X[0], ey1 = X[5] - X[1];
    const double fx0 = Y[2] - Y[0], fy0 = Y[3] - Y[1], fx1 = Y[4] - Y[0], fy1 = Y[5] - Y[1];
    double px[Q], py[Q], G[Q], M[Q][3];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const double* cp = c_R.tri[off + p];
        px[p] = X[0] + cp[0] * ex0 + cp[1] * ex1;
        py[p] = X[1] + cp[0] * ey0 + cp[1] * ey1;
        G[p] = 0.0;
        M[p][0] = M[p][1] = M[p][2] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) ST[m] = 0.0;
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const double* cq = c_R.tri[off + q];
        const double yx = Y[0] + cq[0] * fx0 + cq[1] * fx1;
        const double yy = Y[1] + cq[0] * fy0 + cq[1] * fy1;
        const double wq = cq[2], v0 = cq[3], v1 = cq[4], v2 = cq[5];
        double H = 0.0;
        double kvs[Q];
        if constexpr (std::is_same<KP, KPowTab>::value) {
            double r2[Q];
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const double dx = px[p] - yx, dy = py[p] - yy;
                r2[p] = dx * dx + dy * dy;
            }
            kpow_tab_batch<Q>(kp, r2, kvs);
        } else {
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const double dx = px[p] - yx, dy = py[p] - yy;
                kvs[p] = kp(dx * dx + dy * dy);
            }
        }
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const double kv = kvs[p];
            G[p] += wq * kv;
            H += c_R.tri[off + p][2] * kv;
            M[p][0] += v0 * kv;
            M[p][1] += v1 * kv;
            M[p][2] += v2 * kv;
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) ST[m] += cq[6 + m] * H;
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) SK[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) O[m] = 0.0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const double* cp = c_R.tri[off + p];
#pragma unroll
        for (int m = 0; m < 6; ++m) SK[m] += cp[6 + m] * G[p];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) O[3 * a + b] += cp[3 + a] * M[p][b];
    }
}

// KO = 0: order k at run time; KO = 2: the factorised form above; KO = 3, 4
// (the orders of the closest separated pairs): the loop below with the
// inner loop over K's points unrolled, its kernel evaluations independent.
template <int KO, class KP>
__device__ __forceinline__ void far_pair2(int k, const double* X, const double* Y, const KP& kp,
                                          double* SK, double* ST, double* O) {
    if constexpr (KO > 0 && KO <= 2) {
        far_pair2_fixed<KO>(X, Y, kp, SK, ST, O);
        return;
    }
    if (KO > 0) k = KO;
    const int Q = k * k;
    const int off = tri_off(k);
#pragma unroll
    for (int m = 0; m < 6; ++m) { SK[m] = 0.0; ST[m] = 0.0; }
#pragma unroll
    for (int m = 0; m < 9; ++m) O[m] = 0.0;
    const double ex0 = X[2] - X[0], ey0 = X[3] - X[1], ex1 = X[4] - X[0], ey1 = X[5] - X[1];
    const double fx0 = Y[2] - Y[0], fy0 = Y[3] - Y[1], fx1 = Y[4] - Y[0], fy1 = Y[5] - Y[1];
    // fixed order: K's points once, outside the loop over Kt's points
    constexpr int QP = KO > 0 ? KO * KO : 1;
    double px[QP], py[QP];
    if constexpr (KO > 0) {
#pragma unroll
        for (int p = 0; p < QP; ++p) {
            const double* cp = c_R.tri[off + p];
            px[p] = X[0] + cp[0] * ex0 + cp[1] * ex1;
            py[p] = X[1] + cp[0] * ey0 + cp[1] * ey1;
        }
    }
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const double* cq = c_R.tri[off + q];
        const double yx = Y[0] + cq[0] * fx0 + cq[1] * fx1;
        const double yy = Y[1] + cq[0] * fy0 + cq[1] * fy1;
        double gy = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0;
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0, t5 = 0.0;
        // opaque per iteration: the unrolled loop's factors are fetched by
        // scalar loads on each pass rather than kept live (and spilled)
        auto body = [&](int p, int offp) {
            const double* cp = c_R.tri[offp + p];
            double dx, dy;
            if constexpr (KO > 0) {
                dx = px[p] - yx;
                dy = py[p] - yy;
            } else {
                dx = (X[0] + cp[0] * ex0 + cp[1] * ex1) - yx;
                dy = (X[1] + cp[0] * ey0 + cp[1] * ey1) - yy;
            }
            const double kv = kp(dx * dx + dy * dy);
            gy += cp[2] * kv;
            n0 += cp[3] * kv;
            n1 += cp[4] * kv;
            n2 += cp[5] * kv;
            t0 += cp[6] * kv;
            t1 += cp[7] * kv;
            t2 += cp[8] * kv;
            t3 += cp[9] * kv;
            t4 += cp[10] * kv;
            t5 += cp[11] * kv;
        };
        if constexpr (KO > 0) {
            // chunks of at most 9 points, each behind an opaque offset: the
            // factors are fetched by scalar loads per chunk and pass rather
            // than kept live (and spilled) across the loops
            constexpr int CH = KO * KO <= 9 ? KO * KO : 4;
#pragma unroll
            for (int p0 = 0; p0 < KO * KO; p0 += CH) {
                int offp = off;
                asm volatile("" : "+s"(offp));
#pragma unroll
                for (int j = 0; j < CH; ++j)
                    if (p0 + j < KO * KO) body(p0 + j, offp);
            }
        } else {
#pragma unroll 1
            for (int p = 0; p < Q; ++p) body(p, off);
        }
        const double wq = cq[2];
        SK[0] += wq * t0; SK[1] += wq * t1; SK[2] += wq * t2;
        SK[3] += wq * t3; SK[4] += wq * t4; SK[5] += wq * t5;
#pragma unroll
        for (int m = 0; m < 6; ++m) ST[m] += cq[6 + m] * gy;
        const double na[3] = {n0, n1, n2};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) O[3 * a + b] += cq[3 + b] * na[a];
    }
}

template <int KO>
__device__ __forceinline__ void far_pair2(int k, const double* X, const double* Y, double pe, double* SK,
                                          double* ST, double* O) {
    far_pair2<KO>(k, X, Y, KPow{pe}, SK, ST, O);
}

// Separated segments, k-point Gauss-Legendre on both (same outputs, slots
// 0,1,3 of the symmetric blocks and 0,1,3,4 of O).
__device__ __forceinline__ void far_pair1(int k, const double* X, const double* Y, double pe,
                                          double* SK, double* ST, double* O) {
    const int off = gl_off(k);
#pragma unroll
    for (int m = 0; m < 6; ++m) { SK[m] = 0.0; ST[m] = 0.0; }
#pragma unroll
    for (int m = 0; m < 9; ++m) O[m] = 0.0;
    const double ex = X[1] - X[0], fx = Y[1] - Y[0];
#pragma unroll 1
    for (int q = 0; q < k; ++q) {
        const double* cq = c_R.seg[off + q];
        const double yv = Y[0] + cq[0] * fx;
        double gy = 0.0, n0 = 0.0, n1 = 0.0, t0 = 0.0, t1 = 0.0, t3 = 0.0;
#pragma unroll 1
        for (int p = 0; p < k; ++p) {
            const double* cp = c_R.seg[off + p];
            const double d = (X[0] + cp[0] * ex) - yv;
            const double kv = kpow(d * d, pe);
            gy += cp[1] * kv;
            n0 += cp[2] * kv;
            n1 += cp[3] * kv;
            t0 += cp[4] * kv;
            t1 += cp[5] * kv;
            t3 += cp[6] * kv;
        }
        const double wq = cq[1];
        SK[0] += wq * t0; SK[1] += wq * t1; SK[3] += wq * t3;
        ST[0] += cq[4] * gy; ST[1] += cq[5] * gy; ST[3] += cq[6] * gy;
        O[0] += cq[2] * n0; O[1] += cq[3] * n0;
        O[3] += cq[2] * n1; O[4] += cq[3] * n1;
    }
}

// FP32 variants for the mixed-precision assembly: kernel power with the
// hardware base-2 log / exp (v_log_f32, v_exp_f32), FP32 sums within the
// pair.  The offset between the two elements' first vertices is formed in
// FP64 before rounding, so coordinates far from the origin lose nothing.
__device__ __forceinline__ float kpow32(float r2, float pe) {
    return __builtin_amdgcn_exp2f(pe * __builtin_amdgcn_logf(r2));
}

// FP32 counterpart of far_pair2_fixed (sums within the pair in FP32)
template <int KO>
__device__ __forceinline__ void far_pair2_f32_fixed(const double* X, const double* Y, double pe64, double* SK,
                                                    double* ST, double* O) {
    constexpr int Q = KO * KO;
    const int off = tri_off(KO);
    const float pe = (float)pe64;
    const float ox = (float)(X[0] - Y[0]), oy = (float)(X[1] - Y[1]);
    const float ex0 = (float)(X[2] - X[0]), ey0 = (float)(X[3] - X[1]);
    const float ex1 = (float)(X[4] - X[0]), ey1 = (float)(X[5] - X[1]);
    const float fx0 = (float)(Y[2] - Y[0]), fy0 = (float)(Y[3] - Y[1]);
    const float fx1 = (float)(Y[4] - Y[0]), fy1 = (float)(Y[5] - Y[1]);
    float px[Q], py[Q], G[Q], M[Q][3], st[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float* cp = c_R.trif[off + p];
        px[p] = cp[0] * ex0 + cp[1] * ex1;
        py[p] = cp[0] * ey0 + cp[1] * ey1;
        G[p] = 0.f;
        M[p][0] = M[p][1] = M[p][2] = 0.f;
    }
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const float* cq = c_R.trif[off + q];
        const float yx = cq[0] * fx0 + cq[1] * fx1 - ox;
        const float yy = cq[0] * fy0 + cq[1] * fy1 - oy;
        const float wq = cq[2], v0 = cq[3], v1 = cq[4], v2 = cq[5];
        float H = 0.f;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float dx = px[p] - yx, dy = py[p] - yy;
            const float kv = kpow32(dx * dx + dy * dy, pe);
            G[p] += wq * kv;
            H += c_R.trif[off + p][2] * kv;
            M[p][0] += v0 * kv;
            M[p][1] += v1 * kv;
            M[p][2] += v2 * kv;
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) st[m] += cq[6 + m] * H;
    }
    float sk[6] = {0, 0, 0, 0, 0, 0}, oo[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float* cp = c_R.trif[off + p];
#pragma unroll
        for (int m = 0; m < 6; ++m) sk[m] += cp[6 + m] * G[p];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) oo[3 * a + b] += cp[3 + a] * M[p][b];
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) { SK[m] = sk[m]; ST[m] = st[m]; }
#pragma unroll
    for (int m = 0; m < 9; ++m) O[m] = oo[m];
}

template <int KO>
__device__ __forceinline__ void far_pair2_f32(int k, const double* X, const double* Y, double pe64,
                                              double* SK, double* ST, double* O) {
    if constexpr (KO > 0) {
        far_pair2_f32_fixed<KO>(X, Y, pe64, SK, ST, O);
        return;
    }
    if (KO > 0) k = KO;
    const int Q = k * k;
    const int off = tri_off(k);
    const float pe = (float)pe64;
    const float ox = (float)(X[0] - Y[0]), oy = (float)(X[1] - Y[1]);
    const float ex0 = (float)(X[2] - X[0]), ey0 = (float)(X[3] - X[1]);
    const float ex1 = (float)(X[4] - X[0]), ey1 = (float)(X[5] - X[1]);
    const float fx0 = (float)(Y[2] - Y[0]), fy0 = (float)(Y[3] - Y[1]);
    const float fx1 = (float)(Y[4] - Y[0]), fy1 = (float)(Y[5] - Y[1]);
    float sk[6] = {0, 0, 0, 0, 0, 0}, st[6] = {0, 0, 0, 0, 0, 0}, oo[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const float* cq = c_R.trif[off + q];
        const float yx = cq[0] * fx0 + cq[1] * fx1 - ox;
        const float yy = cq[0] * fy0 + cq[1] * fy1 - oy;
        float gy = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f, t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f, t4 = 0.f,
              t5 = 0.f;
        auto body = [&](int p) {
            const float* cp = c_R.trif[off + p];
            const float dx = (cp[0] * ex0 + cp[1] * ex1) - yx;
            const float dy = (cp[0] * ey0 + cp[1] * ey1) - yy;
            const float kv = kpow32(dx * dx + dy * dy, pe);
            gy += cp[2] * kv;
            n0 += cp[3] * kv;
            n1 += cp[4] * kv;
            n2 += cp[5] * kv;
            t0 += cp[6] * kv;
            t1 += cp[7] * kv;
            t2 += cp[8] * kv;
            t3 += cp[9] * kv;
            t4 += cp[10] * kv;
            t5 += cp[11] * kv;
        };
        if constexpr (KO > 0) {
#pragma unroll
            for (int p = 0; p < KO * KO; ++p) body(p);
        } else {
#pragma unroll 1
            for (int p = 0; p < Q; ++p) body(p);
        }
        const float wq = cq[2];
        sk[0] += wq * t0; sk[1] += wq * t1; sk[2] += wq * t2;
        sk[3] += wq * t3; sk[4] += wq * t4; sk[5] += wq * t5;
#pragma unroll
        for (int m = 0; m < 6; ++m) st[m] += cq[6 + m] * gy;
        const float na[3] = {n0, n1, n2};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) oo[3 * a + b] += cq[3 + b] * na[a];
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) { SK[m] = sk[m]; ST[m] = st[m]; }
#pragma unroll
    for (int m = 0; m < 9; ++m) O[m] = oo[m];
}

__device__ __forceinline__ void far_pair1_f32(int k, const double* X, const double* Y, double pe64,
                                              double* SK, double* ST, double* O) {
    const int off = gl_off(k);
    const float pe = (float)pe64;
    const float ox = (float)(X[0] - Y[0]);
    const float ex = (float)(X[1] - X[0]), fx = (float)(Y[1] - Y[0]);
    float sk0 = 0.f, sk1 = 0.f, sk3 = 0.f, st0 = 0.f, st1 = 0.f, st3 = 0.f, o0 = 0.f, o1 = 0.f, o3 = 0.f,
          o4 = 0.f;
#pragma unroll 1
    for (int q = 0; q < k; ++q) {
        const float* cq = c_R.segf[off + q];
        const float yv = cq[0] * fx - ox;
        float gy = 0.f, n0 = 0.f, n1 = 0.f, t0 = 0.f, t1 = 0.f, t3 = 0.f;
#pragma unroll 1
        for (int p = 0; p < k; ++p) {
            const float* cp = c_R.segf[off + p];
            const float d = cp[0] * ex - yv;
            const float kv = kpow32(d * d, pe);
            gy += cp[1] * kv;
            n0 += cp[2] * kv;
            n1 += cp[3] * kv;
            t0 += cp[4] * kv;
            t1 += cp[5] * kv;
            t3 += cp[6] * kv;
        }
        const float wq = cq[1];
        sk0 += wq * t0; sk1 += wq * t1; sk3 += wq * t3;
        st0 += cq[4] * gy; st1 += cq[5] * gy; st3 += cq[6] * gy;
        o0 += cq[2] * n0; o1 += cq[3] * n0; o3 += cq[2] * n1; o4 += cq[3] * n1;
    }
    for (int m = 0; m < 6; ++m) { SK[m] = 0.0; ST[m] = 0.0; }
    for (int m = 0; m < 9; ++m) O[m] = 0.0;
    SK[0] = sk0; SK[1] = sk1; SK[3] = sk3;
    ST[0] = st0; ST[1] = st1; ST[3] = st3;
    O[0] = o0; O[1] = o1; O[3] = o3; O[4] = o4;
}

// runtime order k; kp evaluates the FP64 kernel power of 2D pairs
template <int DIM, int MIX, class KP>
__device__ __forceinline__ void far_pair(int k, const double* X, const double* Y, double pe, const KP& kp,
                                         double* SK, double* ST, double* O) {
    if (DIM == 2) {
        if (MIX) far_pair2_f32<0>(k, X, Y, pe, SK, ST, O);
        else far_pair2<0>(k, X, Y, kp, SK, ST, O);
    } else {
        if (MIX) far_pair1_f32(k, X, Y, pe, SK, ST, O);
        else far_pair1(k, X, Y, pe, SK, ST, O);
    }
}

template <int DIM, int MIX>
__device__ __forceinline__ void far_pair(int k, const double* X, const double* Y, double pe, double* SK,
                                         double* ST, double* O) {
    far_pair<DIM, MIX>(k, X, Y, pe, KPow{pe}, SK, ST, O);
}

// Order class: #{m : d2 >= theta_m^2 * max(h2K, h2Kt)}.  Every product and
// sum is rounded on its own (contraction into FMA is switched off here), so
// the class of every pair, ties included, is reproducible bit for bit by an
// independent implementation of the same formula.
__device__ __forceinline__ int order_class(double d2, double hmax2, int ncls, const double* th2) {
#pragma clang fp contract(off)
    int c = 0;
    for (int m = 0; m < ncls; ++m) {
        double t = th2[m] * hmax2;
        if (d2 >= t) c = m + 1;
    }
    return c;
}

// squared distance of two points in DIM dimensions, no contraction
__device__ __forceinline__ double dist2_nc(double x0, double y0, double x1, double y1, int dim) {
#pragma clang fp contract(off)
    double dx = x0 - x1;
    double d2 = dx * dx;
    if (dim == 2) {
        double dy = y0 - y1;
        double t = dy * dy;
        d2 = d2 + t;
    }
    return d2;
}

// Cluster near field: bit l % 16 of nb[r][l / 16] is set when the anchor
// leaves of the row element I0 + r and the column element J0 + l are a near
// pair (the pair's diagonal-block parts are then assembled here, otherwise
// they come from the far field).  256 threads: row tid / 4, 16 columns each.
__device__ void nm_tile_bits(const NearMap& M, int I0, int J0, int T, unsigned short (*nb)[4], int tid) {
    const int r = tid >> 2, q = tid & 3;
    unsigned bits = 0;
    const int K = I0 + r;
    if (K < T) {
        const int a = M.aleaf[K];
        for (int u = 0; u < 16; ++u) {
            const int Kt = J0 + q * 16 + u;
            if (Kt < T && nm_block(M, a, M.aleaf[Kt]) >= 0) bits |= 1u << u;
        }
    }
    nb[r][q] = (unsigned short)bits;
}

__device__ __forceinline__ bool nm_bit(const unsigned short (*nb)[4], int r, int l) {
    return (nb[r][l >> 4] >> (l & 15)) & 1;
}

// add v to near-field entry (i, j) if (i, j) lies in the near field
__device__ __forceinline__ void nm_add(const NearMap& M, int i, int j, double v) {
    double* q = nm_slot(M, i, j);
    if (q) atomicAdd(q, v);
}

// One workgroup per tile (bi <= bj) of BE x BE element pairs.  Wave w takes
// rows K = I0 + w, w+4, ...; lane l takes Kt = J0 + l.  Off-diagonal blocks
// are accumulated in LDS over the block's local DOF numbering and flushed
// to A (and its mirror) with one global atomic per touched entry; the
// diagonal-block increments go to per-element accumulators S.  CL = 1: the
// cluster near field (P.nm): diagonal-block parts only for pairs of near
// anchor leaves, off-diagonal entries only in near blocks.
template <int DIM, int FARK, int MIX, int CL>
__global__ __launch_bounds__(256) void far_kernel(ElemDev E, FarParams P) {
    constexpr int NV = DIM + 1;
    constexpr int NC = NV * DIM;
    constexpr bool TAB = DIM == 2 && !MIX;  // FP64 kernel power by LDS tables
    __shared__ __align__(16) double pw[TAB ? 768 : 1];
    __shared__ double L[MAXV * MAXV];
    __shared__ double SI[BE * 6];
    __shared__ double SJ[BE * 6];
    __shared__ int vI[MAXV], vJ[MAXV];
    __shared__ unsigned char locI[BE * 3], locJ[BE * 3];
    __shared__ unsigned long long ccount[FL_MAX_CLASSES + 1];
    __shared__ double sI[10][BE];  // row elements: coordinates, centroid, h^2, |K|
    __shared__ int sV[3][BE];      // row elements: vertex ids
    __shared__ unsigned short nbits[CL ? BE : 1][4];

    const long long t = blockIdx.x;
    const int2 tb = P.tiles[t];
    const int bi = tb.x, bj = tb.y;
    const int I0 = bi * BE, J0 = bj * BE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nVI = P.blk_ndof[bi], nVJ = P.blk_ndof[bj];
    const bool det = P.fa.lo != nullptr;  // repeatable: off-diagonal entries straight to the words
    const bool direct = (nVI > MAXV) || (nVJ > MAXV) || det;
    const int T = P.T;

    for (int i = tid; i < BE * 3; i += 256) {
        int K = I0 + i / 3, Kt = J0 + i / 3;
        locI[i] = (K < T) ? P.loc[(long long)K * 3 + i % 3] : 255;
        locJ[i] = (Kt < T) ? P.loc[(long long)Kt * 3 + i % 3] : 255;
    }
    if (!direct) {
        for (int i = tid; i < MAXV; i += 256) {
            vI[i] = P.blk_dofs[(long long)bi * MAXV + i];
            vJ[i] = P.blk_dofs[(long long)bj * MAXV + i];
        }
        for (int i = tid; i < nVI * nVJ; i += 256) L[i] = 0.0;
    }
    for (int i = tid; i < BE * 6; i += 256) { SI[i] = 0.0; SJ[i] = 0.0; }
    if (tid <= FL_MAX_CLASSES) ccount[tid] = 0;
    if constexpr (TAB) load_pow_tables(pw);
    for (int i = tid; i < 13 * BE; i += 256) {
        const int f = i / BE, r = i - f * BE, K = I0 + r;
        if (f < 10) {
            double v = 0.0;
            if (K < T) {
                if (f < NC) v = E.x[f][K];
                else if (f == 6) v = E.cen[0][K];
                else if (f == 7 && DIM == 2) v = E.cen[1][K];
                else if (f == 8) v = E.h2[K];
                else if (f == 9) v = E.meas[K];
            }
            sI[f][r] = v;
        } else {
            const int a = f - 10;
            sV[a][r] = (K < T && a < NV) ? E.vid[a][K] : -2;
        }
    }
    if constexpr (CL) nm_tile_bits(P.nm, I0, J0, T, nbits, tid);
    __syncthreads();

    const int Kt = J0 + lane;
    const bool okt = Kt < T;
    double Y[6] = {0, 0, 0, 0, 0, 0}, cyt[2] = {0, 0}, h2t = 0, mt = 0;
    int vt[3] = {-1, -1, -1};
    if (okt) {
#pragma unroll
        for (int c = 0; c < NC; ++c) Y[c] = E.x[c][Kt];
        for (int c = 0; c < DIM; ++c) cyt[c] = E.cen[c][Kt];
        h2t = E.h2[Kt];
        mt = E.meas[Kt];
#pragma unroll
        for (int a = 0; a < NV; ++a) vt[a] = E.vid[a][Kt];
    }
    double STacc[6] = {0, 0, 0, 0, 0, 0};

    for (int r = wave; r < BE; r += 4) {
        const int K = I0 + r;
        if (K >= T) break;
        double X[6] = {0, 0, 0, 0, 0, 0};
        int vk[3] = {-2, -2, -2};
#pragma unroll
        for (int c = 0; c < NC; ++c) X[c] = sI[c][r];
        const double cx[2] = {sI[6][r], sI[7][r]};
        const double h2k = sI[8][r], mk = sI[9][r];
#pragma unroll
        for (int a = 0; a < NV; ++a) vk[a] = sV[a][r];

        bool valid = okt && (bi != bj || K < Kt);
        int cls = -1;
        if (FARK > 0) {
            // far tile: the host proved every pair separated and in the last class
            if (valid) cls = P.ncls;
        } else {
#pragma unroll
            for (int a = 0; a < NV; ++a)
#pragma unroll
                for (int b = 0; b < NV; ++b) valid = valid && (vk[a] != vt[b]);
            if (valid) {
                const double d2 = dist2_nc(cx[0], cx[1], cyt[0], cyt[1], DIM);
                double hm = h2k > h2t ? h2k : h2t;
                cls = order_class(d2, hm, P.ncls, P.th2);
            }
        }
        if constexpr (FARK == 0) {
#pragma unroll
            for (int c = 0; c <= FL_MAX_CLASSES; ++c) {
                if (c <= P.ncls) {
                    unsigned long long bal = __ballot(cls == c);
                    if (lane == 0 && bal) atomicAdd(&ccount[c], (unsigned long long)__popcll(bal));
                }
            }
        }
        double SK[6] = {0, 0, 0, 0, 0, 0}, ST[6] = {0, 0, 0, 0, 0, 0};
        double O[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (FARK > 0) {
            if (valid) {
                if (DIM == 2) {
                    if constexpr (MIX) far_pair2_f32<FARK>(FARK, X, Y, P.pe, SK, ST, O);
                    else far_pair2<FARK>(FARK, X, Y, make_kpow_tab(pw), SK, ST, O);
                } else {
                    if (MIX) far_pair1_f32(FARK, X, Y, P.pe, SK, ST, O);
                    else far_pair1(FARK, X, Y, P.pe, SK, ST, O);
                }
            }
        } else {
            // one pass per distinct order present in the wave
            int myk = 0;
#pragma unroll
            for (int m = 0; m <= FL_MAX_CLASSES; ++m)
                if (m <= P.ncls && cls == m) myk = P.kf[m];
            for (int c = 0; c <= P.ncls; ++c) {
                if (!P.kfirst[c]) continue;
                const int kc = P.kf[c];
                if (__any(myk == kc)) {
                    if (myk == kc) {
                        if constexpr (TAB) far_pair<DIM, MIX>(kc, X, Y, P.pe, make_kpow_tab(pw), SK, ST, O);
                        else far_pair<DIM, MIX>(kc, X, Y, P.pe, SK, ST, O);
                    }
                }
            }
        }
        const double f = valid ? P.C * mk * mt * pair_w(E, K, Kt) : 0.0;
        const double fs = (CL && !nm_bit(nbits, r, lane)) ? 0.0 : f;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            SK[m] *= fs;
            STacc[m] += ST[m] * fs;
        }
        // diagonal block of K: reduce over the wave (this wave owns row r);
        // the six sums end in lanes 0, 8, ..., 40
        {
            const double v = wave_sum6(SK, lane);
            if ((lane & 7) == 0 && (lane >> 3) < 6) SI[r * 6 + (lane >> 3)] += v;
        }
        if (valid) {
            if (!direct) {
#pragma unroll
                for (int a = 0; a < NV; ++a) {
                    int ra = locI[r * 3 + a];
                    if (ra == 255) continue;
#pragma unroll
                    for (int b = 0; b < NV; ++b) {
                        int cb = locJ[lane * 3 + b];
                        if (cb == 255) continue;
                        double v = -f * O[3 * a + b];
                        atomicAdd(&L[ra * nVJ + cb], v);
                        if (bi == bj) atomicAdd(&L[cb * nVJ + ra], v);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < NV; ++a) {
                    int ga = E.dof[a][K];
                    if (ga < 0) continue;
#pragma unroll
                    for (int b = 0; b < NV; ++b) {
                        int gb = E.dof[b][Kt];
                        if (gb < 0) continue;
                        double v = -f * O[3 * a + b];
                        if constexpr (CL) {
                            nm_add(P.nm, ga, gb, v);
                            nm_add(P.nm, gb, ga, v);
                        } else {
                            add_pair_upper(P, ga, gb, v);
                        }
                    }
                }
            }
        }
    }
    if (okt) {
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            if (STacc[m] == 0.0) continue;
            // four waves add into the same column sums: in LDS their order varies
            if (det) fix_add(P.fs, (long long)Kt * 6 + m, STacc[m]);
            else atomicAdd(&SJ[lane * 6 + m], STacc[m]);
        }
    }
    __syncthreads();
    if (!direct) {
        for_block_entries(nVI, nVJ, tid, [&](int rr, int cc) {
            const double v = L[rr * nVJ + cc];
            if (v == 0.0) return;
            if constexpr (CL) {
                nm_add(P.nm, vI[rr], vJ[cc], v);
                if (bi != bj) nm_add(P.nm, vJ[cc], vI[rr], v);
            } else if (bi != bj) {
                add_pair_upper(P, vI[rr], vJ[cc], v);
            } else if (vI[rr] <= vJ[cc]) {
                // a diagonal tile's block holds both orientations already
                acc_add(P.fa, P.A, (long long)vI[rr] * P.lda + vJ[cc], v);
            }
        });
    }
    for (int i = tid; i < BE * 6; i += 256) {
        int K = I0 + i / 6, Kt2 = J0 + i / 6;
        if (K < T && SI[i] != 0.0) acc_add(P.fs, P.S, (long long)K * 6 + i % 6, SI[i]);
        if (Kt2 < T && SJ[i] != 0.0) acc_add(P.fs, P.S, (long long)Kt2 * 6 + i % 6, SJ[i]);
    }
    if constexpr (FARK > 0) {
        // far tile (bi != bj): every pair of its rows and columns, last class
        if (tid == 0)
            atomicAdd(&P.cls_count[P.ncls],
                      (unsigned long long)(min(BE, T - I0) * (long long)min(BE, T - J0)));
    } else {
        if (tid <= P.ncls && ccount[tid]) atomicAdd(&P.cls_count[tid], ccount[tid]);
    }
}

// Near tiles: the pairs of the tile are classified first and bucketed by
// class (counting sort in LDS), then every thread takes one pair of a
// bucket at a time, so all lanes of a wave run the same order.  Diagonal
// blocks, self terms and off-diagonal blocks are accumulated in LDS as in
// far_kernel and flushed once per tile.
template <int DIM, int MIX, int SUR, int CL>
__global__ __launch_bounds__(256) void near_kernel(ElemDev E, FarParams P) {
    static_assert(!(CL && SUR), "the cluster near field takes the exact rules");
    constexpr int NV = DIM + 1;
    constexpr int NC = NV * DIM;
    __shared__ double L[MAXV * MAXV];
    __shared__ double SI[BE * 6];
    __shared__ double SJ[BE * 6];
    __shared__ double sI[10][BE], sJ[10][BE];
    __shared__ int sVI[3][BE], sVJ[3][BE];
    __shared__ int vI[MAXV], vJ[MAXV];
    __shared__ unsigned char locI[BE * 3], locJ[BE * 3];
    __shared__ unsigned char pcls[BE * BE];
    __shared__ unsigned short plist[BE * BE];
    __shared__ int ccnt[FL_MAX_CLASSES + 1], coff[FL_MAX_CLASSES + 2], cfill[FL_MAX_CLASSES + 1];
    __shared__ float souts[SUR ? 4 * 16 * 24 : 1];  // network outputs, 16 samples per wave
    constexpr bool TAB = DIM == 2 && !MIX;   // FP64 kernel power by LDS tables
    __shared__ __align__(16) double pw[TAB ? 768 : 1];
    __shared__ unsigned short nbits[CL ? BE : 1][4];

    const long long t = blockIdx.x;
    const int2 tb = P.tiles[t];
    const int bi = tb.x, bj = tb.y;
    const int I0 = bi * BE, J0 = bj * BE;
    const int tid = threadIdx.x;
    const int nVI = P.blk_ndof[bi], nVJ = P.blk_ndof[bj];
    // repeatable assembly: every pair straight into the global words (the
    // LDS sums would depend on the order of their FP64 atomics)
    const bool det = P.fa.lo != nullptr;
    const bool direct = (nVI > MAXV) || (nVJ > MAXV) || det;
    const int T = P.T;

    for (int i = tid; i < BE * 3; i += 256) {
        int K = I0 + i / 3, Kt = J0 + i / 3;
        locI[i] = (K < T) ? P.loc[(long long)K * 3 + i % 3] : 255;
        locJ[i] = (Kt < T) ? P.loc[(long long)Kt * 3 + i % 3] : 255;
    }
    if (!direct) {
        for (int i = tid; i < MAXV; i += 256) {
            vI[i] = P.blk_dofs[(long long)bi * MAXV + i];
            vJ[i] = P.blk_dofs[(long long)bj * MAXV + i];
        }
        for (int i = tid; i < nVI * nVJ; i += 256) L[i] = 0.0;
    }
    for (int i = tid; i < BE * 6; i += 256) { SI[i] = 0.0; SJ[i] = 0.0; }
    if (tid <= FL_MAX_CLASSES) { ccnt[tid] = 0; cfill[tid] = 0; }
    if constexpr (TAB) load_pow_tables(pw);
    for (int i = tid; i < 13 * BE; i += 256) {
        const int f = i / BE, r = i - f * BE;
        const int K = I0 + r, Kt = J0 + r;
        if (f < 10) {
            double a = 0.0, b = 0.0;
            if (f < NC) {
                if (K < T) a = E.x[f][K];
                if (Kt < T) b = E.x[f][Kt];
            } else if (f == 6) {
                if (K < T) a = E.cen[0][K];
                if (Kt < T) b = E.cen[0][Kt];
            } else if (f == 7 && DIM == 2) {
                if (K < T) a = E.cen[1][K];
                if (Kt < T) b = E.cen[1][Kt];
            } else if (f == 8) {
                if (K < T) a = E.h2[K];
                if (Kt < T) b = E.h2[Kt];
            } else if (f == 9) {
                if (K < T) a = E.meas[K];
                if (Kt < T) b = E.meas[Kt];
            }
            sI[f][r] = a;
            sJ[f][r] = b;
        } else {
            const int a = f - 10;
            sVI[a][r] = (K < T && a < NV) ? E.vid[a][K] : -2;
            sVJ[a][r] = (Kt < T && a < NV) ? E.vid[a][Kt] : -3;
        }
    }
    if constexpr (CL) nm_tile_bits(P.nm, I0, J0, T, nbits, tid);
    __syncthreads();
    // classify
    for (int pidx = tid; pidx < BE * BE; pidx += 256) {
        const int r = pidx / BE, l = pidx - r * BE;
        const int K = I0 + r, Kt = J0 + l;
        bool valid = K < T && Kt < T && (bi != bj || K < Kt);
#pragma unroll
        for (int a = 0; a < NV; ++a)
#pragma unroll
            for (int b = 0; b < NV; ++b) valid = valid && (sVI[a][r] != sVJ[b][l]);
        unsigned char c = 255;
        if (valid) {
            const double d2 = dist2_nc(sI[6][r], sI[7][r], sJ[6][l], sJ[7][l], DIM);
            const double hm = sI[8][r] > sJ[8][l] ? sI[8][r] : sJ[8][l];
            c = (unsigned char)order_class(d2, hm, P.ncls, P.th2);
            atomicAdd(&ccnt[c], 1);
        }
        pcls[pidx] = c;
    }
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int c = 0; c <= P.ncls; ++c) { coff[c] = acc; acc += ccnt[c]; }
        coff[P.ncls + 1] = acc;
    }
    __syncthreads();
    for (int pidx = tid; pidx < BE * BE; pidx += 256) {
        const unsigned char c = pcls[pidx];
        if (c == 255) continue;
        const int slot = coff[c] + atomicAdd(&cfill[c], 1);
        plist[slot] = (unsigned short)pidx;
    }
    __syncthreads();
    // classes below nsur: the learned surrogate where certified (order-2
    // rule on the canonical pair times 1 + t), the exact rule otherwise
    int c0 = 0;
    if constexpr (SUR) {
        const SurParams& SP = P.sur;
        c0 = SP.nsur < P.ncls + 1 ? SP.nsur : P.ncls + 1;
        const int nb = coff[c0];
        const int lane = tid & 63, wave = tid >> 6, r16 = lane & 15, g = lane >> 4;
        const double rb_e2[5] = {1.0, 2.25, 4.0, 6.25, 9.0};
        unsigned long long n_sur = 0, n_fb = 0;
        for (int base = 0; base < nb; base += 256) {
            const int slot = base + tid;
            const bool valid = slot < nb;
            int r = 0, l = 0, cls = 0;
            // phase 1: canonical form, features, certification.  o1 / o2:
            // vertex slots, in the order of the computed blocks, of the first /
            // second element (canonical for the network, stored order for the
            // exact rule); swap: the first element is Kt
            int o1[3] = {0, 1, 2}, o2[3] = {0, 1, 2}, swap = 0;
            bool sur = false;
            float xn[SUR_NIN];
#pragma unroll
            for (int k = 0; k < SUR_NIN; ++k) xn[k] = 0.f;
            if (valid) {
                const int pidx = plist[slot];
                r = pidx / BE;
                l = pidx - r * BE;
                cls = pcls[pidx];
                double X[6], Y[6], C1[6], C2[6], f[SUR_NIN];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    X[q] = sI[q][r];
                    Y[q] = sJ[q][l];
                }
                const double d2 = dist2_nc(sI[6][r], sI[7][r], sJ[6][l], sJ[7][l], 2);
                const double hm = sI[8][r] > sJ[8][l] ? sI[8][r] : sJ[8][l];
                const int rb = order_class(d2, hm, 5, rb_e2);
                int c1[3], c2[3];
                const int sw = sur_canon(X, Y, c1, c2, C1, C2);
                sur_features(C1, C2, SP.s, f);
                bool in = true;
#pragma unroll
                for (int k = 0; k < SUR_NIN; ++k) in = in && f[k] >= SP.lo[k] && f[k] <= SP.hi[k];
                sur = in && SP.use_rbin[rb];
                if (sur) {
                    swap = sw;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        o1[a] = c1[a];
                        o2[a] = c2[a];
                    }
                    sur_std_features(SP.N, f, xn);
                }
            }
            // phase 2: the network for the wave's 64 pairs, 16 at a time
            float tv[SUR_NOUT];
            const bool any_sur = __any(sur);
            if (any_sur) {
                unsigned int pk[5];
                sur_pack_x(xn, pk);
                float* ow = souts + wave * 16 * 24;
                for (int q = 0; q < 4; ++q) {
                    const h8 xb = sur_gather_x(pk, q);
                    SurAct a;
                    sur_forward16(SP.N, xb, a);
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (16 * t + 4 * g + v < 24) ow[r16 * 24 + 16 * t + 4 * g + v] = a.out[t][v];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (g == q) {
#pragma unroll
                        for (int j = 0; j < SUR_NOUT; ++j) tv[j] = ow[r16 * 24 + j];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
            // phase 3: the pair's blocks
            double SK[6], ST[6], O[9];
            if (valid) {
                double X[6], Y[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    X[q] = sI[q][r];
                    Y[q] = sJ[q][l];
                }
                if (sur) {
                    const double* Fp = swap ? Y : X;
                    const double* Sp = swap ? X : Y;
                    double C1[6], C2[6];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        C1[2 * a] = Fp[2 * o1[a]];
                        C1[2 * a + 1] = Fp[2 * o1[a] + 1];
                        C2[2 * a] = Sp[2 * o2[a]];
                        C2[2 * a + 1] = Sp[2 * o2[a] + 1];
                    }
                    if constexpr (MIX) far_pair2_f32<2>(2, C1, C2, P.pe, SK, ST, O);
                    else if constexpr (TAB) far_pair2<2>(2, C1, C2, make_kpow_tab(pw), SK, ST, O);
                    else far_pair2<2>(2, C1, C2, P.pe, SK, ST, O);
#pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        SK[j] *= 1.0 + ((double)tv[j] * (double)SP.N.st[j] + (double)SP.N.mt[j]);
                        ST[j] *= 1.0 + ((double)tv[6 + j] * (double)SP.N.st[6 + j] + (double)SP.N.mt[6 + j]);
                    }
#pragma unroll
                    for (int j = 0; j < 9; ++j)
                        O[j] *= 1.0 + ((double)tv[12 + j] * (double)SP.N.st[12 + j] + (double)SP.N.mt[12 + j]);
                    sur_sum_rules(SK, ST, O);
                } else {
                    if constexpr (TAB) far_pair<2, MIX>(P.kf[cls], X, Y, P.pe, make_kpow_tab(pw), SK, ST, O);
                    else far_pair<2, MIX>(P.kf[cls], X, Y, P.pe, SK, ST, O);
                }
            }
            for (int c = 0; c < c0; ++c) {
                const unsigned long long bal = __ballot(valid && !sur && cls == c);
                if ((tid & 63) == 0 && bal) atomicAdd(SP.counters + 4 + c, (unsigned long long)__popcll(bal));
            }
            if (!valid) continue;
            if (sur) ++n_sur;
            else ++n_fb;
            // blocks of the row element K (r) and the column element Kt (l)
            const double* BK = swap ? ST : SK;
            const double* BT = swap ? SK : ST;
            const int* pK = swap ? o2 : o1;
            const int* pT = swap ? o1 : o2;
            const double fct = P.C * sI[9][r] * sJ[9][l] * pair_w(E, I0 + r, J0 + l);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a; b < 3; ++b) {
                    const int q = sym3(a, b);
                    atomicAdd(&SI[r * 6 + sym3(pK[a], pK[b])], fct * BK[q]);
                    atomicAdd(&SJ[l * 6 + sym3(pT[a], pT[b])], fct * BT[q]);
                }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    // O[3a+b]: vertex a of the first element, b of the second
                    const int sk = swap ? o2[b] : o1[a], sl = swap ? o1[a] : o2[b];
                    const double v = -fct * O[3 * a + b];
                    if (!direct) {
                        const int ra = locI[r * 3 + sk], cb = locJ[l * 3 + sl];
                        if (ra == 255 || cb == 255) continue;
                        atomicAdd(&L[ra * nVJ + cb], v);
                        if (bi == bj) atomicAdd(&L[cb * nVJ + ra], v);
                    } else {
                        const int ga = E.dof[sk][I0 + r], gb = E.dof[sl][J0 + l];
                        if (ga < 0 || gb < 0) continue;
                        add_pair_upper(P, ga, gb, v);
                    }
                }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            n_sur += __shfl_xor(n_sur, m, 64);
            n_fb += __shfl_xor(n_fb, m, 64);
        }
        if ((tid & 63) == 0) {
            if (n_sur) atomicAdd(SP.counters, n_sur);
            if (n_fb) atomicAdd(SP.counters + 1, n_fb);
        }
    }
    // one class at a time, one pair per thread
    for (int c = c0; c <= P.ncls; ++c) {
        const int k = P.kf[c];
        for (int base = coff[c]; base < coff[c + 1]; base += 256) {
            const int slot = base + tid;
            if (slot >= coff[c + 1]) continue;
            const int pidx = plist[slot];
            const int r = pidx / BE, l = pidx - r * BE;
            double X[6] = {0, 0, 0, 0, 0, 0}, Y[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < NC; ++q) { X[q] = sI[q][r]; Y[q] = sJ[q][l]; }
            double SK[6], ST[6], O[9];
            if (DIM == 2 && k == 2) {
                // the commonest order in near tiles: the unrolled fixed-order rule
                if constexpr (MIX) far_pair2_f32<2>(2, X, Y, P.pe, SK, ST, O);
                else if constexpr (TAB) far_pair2<2>(2, X, Y, make_kpow_tab(pw), SK, ST, O);
                else far_pair2<2>(2, X, Y, P.pe, SK, ST, O);
            } else if (TAB && k == 3) {
                if constexpr (TAB) far_pair2<3>(3, X, Y, make_kpow_tab(pw), SK, ST, O);
            } else if (TAB && k == 4) {
                if constexpr (TAB) far_pair2<4>(4, X, Y, make_kpow_tab(pw), SK, ST, O);
            } else {
                if constexpr (TAB) far_pair<DIM, MIX>(k, X, Y, P.pe, make_kpow_tab(pw), SK, ST, O);
                else far_pair<DIM, MIX>(k, X, Y, P.pe, SK, ST, O);
            }
            const double f = P.C * sI[9][r] * sJ[9][l] * pair_w(E, I0 + r, J0 + l);
            const double fs = (CL && !nm_bit(nbits, r, l)) ? 0.0 : f;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                if (SK[m] == 0.0 && ST[m] == 0.0) continue;
                if (det) {
                    if (SK[m] != 0.0) fix_add(P.fs, (long long)(I0 + r) * 6 + m, fs * SK[m]);
                    if (ST[m] != 0.0) fix_add(P.fs, (long long)(J0 + l) * 6 + m, fs * ST[m]);
                } else if (fs != 0.0) {
                    if (SK[m] != 0.0) atomicAdd(&SI[r * 6 + m], fs * SK[m]);
                    if (ST[m] != 0.0) atomicAdd(&SJ[l * 6 + m], fs * ST[m]);
                }
            }
            if (!direct) {
#pragma unroll
                for (int a = 0; a < NV; ++a) {
                    int ra = locI[r * 3 + a];
                    if (ra == 255) continue;
#pragma unroll
                    for (int b = 0; b < NV; ++b) {
                        int cb = locJ[l * 3 + b];
                        if (cb == 255) continue;
                        double v = -f * O[3 * a + b];
                        atomicAdd(&L[ra * nVJ + cb], v);
                        if (bi == bj) atomicAdd(&L[cb * nVJ + ra], v);
                    }
                }
            } else {
                const int K = I0 + r, Kt = J0 + l;
#pragma unroll
                for (int a = 0; a < NV; ++a) {
                    int ga = E.dof[a][K];
                    if (ga < 0) continue;
#pragma unroll
                    for (int b = 0; b < NV; ++b) {
                        int gb = E.dof[b][Kt];
                        if (gb < 0) continue;
                        double v = -f * O[3 * a + b];
                        if constexpr (CL) {
                            nm_add(P.nm, ga, gb, v);
                            nm_add(P.nm, gb, ga, v);
                        } else {
                            add_pair_upper(P, ga, gb, v);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    if (!direct) {
        for_block_entries(nVI, nVJ, tid, [&](int rr, int cc) {
            const double v = L[rr * nVJ + cc];
            if (v == 0.0) return;
            if constexpr (CL) {
                nm_add(P.nm, vI[rr], vJ[cc], v);
                if (bi != bj) nm_add(P.nm, vJ[cc], vI[rr], v);
            } else if (bi != bj) {
                add_pair_upper(P, vI[rr], vJ[cc], v);
            } else if (vI[rr] <= vJ[cc]) {
                // a diagonal tile's block holds both orientations already
                acc_add(P.fa, P.A, (long long)vI[rr] * P.lda + vJ[cc], v);
            }
        });
    }
    for (int i = tid; i < BE * 6; i += 256) {
        int K = I0 + i / 6, Kt2 = J0 + i / 6;
        if (K < T && SI[i] != 0.0) acc_add(P.fs, P.S, (long long)K * 6 + i % 6, SI[i]);
        if (Kt2 < T && SJ[i] != 0.0) acc_add(P.fs, P.S, (long long)Kt2 * 6 + i % 6, SJ[i]);
    }
    if (tid <= P.ncls && ccnt[tid]) atomicAdd(&P.cls_count[tid], (unsigned long long)ccnt[tid]);
}

// ------------------------------------------- far tiles, 2D, FP64, KO <= 2 --
//
// Every pair of a far tile (bi < bj) is separated and in the last distance
// class (proved on the host from the blocks' centroid boxes), so all its
// pairs take the same order-KO rule.  With the rule's points x_p of K and
// y_q of Kt, weights w, barycentric values l and k_pq = |x_p - y_q|^{-2-2s}:
//   M_pb = sum_q w_q l_b(y_q) k_pq,   H_q = sum_p w_p k_pq,
//   off-diagonal block   O_ab = sum_p w_p l_a(x_p) M_pb,
//   diagonal block of K:  sum_p w_p l_a l_b(x_p) G_p,  G_p = sum_b M_pb
//                         (= sum_q w_q k_pq: the l_b sum to 1),
//   diagonal block of Kt: sum_q w_q l_a l_b(y_q) H_q,
// four accumulations per kernel evaluation.  The diagonal blocks are linear
// in G and H, so the tile sums the scaled potentials
//   Phi_p(K)  = sum_Kt C |K| |Kt| G_p   (over the lanes, once per row),
//   Psi_q(Kt) = sum_K  C |K| |Kt| H_q   (in the lane's registers),
// and applies the l_a l_b weights once per element and tile.  Wave w takes
// rows K = I0 + w, w + 4, ...; lane l takes Kt = J0 + l, whose mapped points
// stay in registers; the rows' mapped points are staged in LDS.  The
// off-diagonal blocks are summed in LDS over the two blocks' local DOF
// numbering; a spare row and column take the vertices without a DOF, so the
// adds are branch-free.  The Psi partials of the four waves are added in
// wave order.
// MIX = 1 (FL_MIXED): the evaluations in FP32 (hardware log2 / exp2), the
// points relative to an origin in the row block (the first row's first
// vertex), so that their rounding error stays relative to the pair's
// distance; the sums of a pair are formed in FP32 and added in FP64.
// CL = 1: the cluster near field, as in far_kernel (the potentials take only
// the pairs of near anchor leaves).  DET = 1 (repeatable assembly): the
// block is summed in LDS as the fixed-point words of the global
// accumulation (integer atomics: any order gives the same words) and its
// words are added to A's words; the other sums of the kernel are fixed-order
// reductions already.
template <int KO, int MIX, int W, int CL, int DET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void far2_kernel(ElemDev E, FarParams P) {
    constexpr int Q = KO * KO;
    constexpr int LS = MAXV + 1;  // row stride of L; row / column MAXV: vertices without a DOF
    __shared__ __align__(16) double pw[MIX ? 2 : 768];
    __shared__ __align__(16) double L[LS * LS];      // DET: the int64 remainder words
    __shared__ int Lhi[DET ? LS * LS : 1];            // DET: the int32 coarse words
    using XT = std::conditional_t<MIX, float, double>;
    __shared__ __align__(16) XT sX[BE][2 * Q];       // rows' mapped points, (x, y) per point
    __shared__ double sMK[BE];                      // |K| of the rows (0 past T)
    __shared__ int sRO[BE][3];                      // byte offsets of the rows' L rows
    __shared__ double sPhi[BE][Q];
    __shared__ int vI[MAXV], vJ[MAXV];
    __shared__ unsigned short nbits[CL ? BE : 1][4];

    const int2 tb = P.tiles[blockIdx.x];
    const int bi = tb.x, bj = tb.y;
    const int I0 = bi * BE, J0 = bj * BE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nVI = P.blk_ndof[bi], nVJ = P.blk_ndof[bj];
    const bool direct = (nVI > MAXV) || (nVJ > MAXV);
    const int T = P.T;
    constexpr int off = (KO - 1) * KO * (2 * KO - 1) / 6;  // tri_off(KO)
    // origin of the FP32 coordinates (unused in FP64)
    const double o0 = MIX ? E.x[0][I0] : 0.0, o1 = MIX ? E.x[1][I0] : 0.0;

    if constexpr (!MIX) load_pow_tables(pw);
    for (int i = tid; i < LS * LS; i += 256) L[i] = 0.0;
    if constexpr (DET)
        for (int i = tid; i < LS * LS; i += 256) Lhi[i] = 0;
    if (!direct)
        for (int i = tid; i < MAXV; i += 256) {
            vI[i] = P.blk_dofs[(long long)bi * MAXV + i];
            vJ[i] = P.blk_dofs[(long long)bj * MAXV + i];
        }
    if (tid < BE) {
        const int r = tid, K = I0 + r;
        const bool ok = K < T;
        const int Kc = ok ? K : T - 1;
        double X[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) X[c] = E.x[c][Kc];
        const double ex0 = X[2] - X[0], ey0 = X[3] - X[1], ex1 = X[4] - X[0], ey1 = X[5] - X[1];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const double* cp = c_R.tri[off + p];
            sX[r][2 * p] = (XT)((X[0] - o0) + cp[0] * ex0 + cp[1] * ex1);
            sX[r][2 * p + 1] = (XT)((X[1] - o1) + cp[0] * ey0 + cp[1] * ey1);
        }
        sMK[r] = ok ? E.meas[Kc] : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int la = ok ? P.loc[(long long)Kc * 3 + a] : 255;
            sRO[r][a] = (la == 255 ? MAXV : la) * LS * 8;
        }
    }

    // the lane's column element: lanes 16 g .. 16 g + 15 take the columns
    // g, g + 4, .., g + 60, so that the elements a 16-lane group adds into
    // the LDS block at once are spread over the tile and seldom share a
    // vertex (fewer lanes on one LDS address in the atomic adds)
    const int col = 4 * (lane & 15) + (lane >> 4);
    const int Kt = J0 + col;
    const bool okt = Kt < T;
    const int Ktc = okt ? Kt : T - 1;
    double yq[2 * Q];
    {
        double Y[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) Y[c] = E.x[c][Ktc];
        const double fx0 = Y[2] - Y[0], fy0 = Y[3] - Y[1], fx1 = Y[4] - Y[0], fy1 = Y[5] - Y[1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double* cq = c_R.tri[off + q];
            yq[2 * q] = (Y[0] - o0) + cq[0] * fx0 + cq[1] * fx1;
            yq[2 * q + 1] = (Y[1] - o1) + cq[0] * fy0 + cq[1] * fy1;
        }
    }
    const double ct = okt ? P.C * E.meas[Ktc] : 0.0;
    int cbo[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int lb = okt ? P.loc[(long long)Ktc * 3 + b] : 255;
        cbo[b] = (lb == 255 ? MAXV : lb) * 8;
    }
    // rule constants: w_q l_b(y_q) and w_p
    double cw[Q][3], wq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        wq[q] = c_R.tri[off + q][2];
#pragma unroll
        for (int b = 0; b < 3; ++b) cw[q][b] = c_R.tri[off + q][3 + b];
    }
    const KPowTab kp = make_kpow_tab(pw);
    float yqf[2 * Q];
#pragma unroll
    for (int c = 0; c < 2 * Q; ++c) yqf[c] = (float)yq[c];
    const float pef = (float)P.pe;
    double Psi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) Psi[q] = 0.0;
    if constexpr (CL) nm_tile_bits(P.nm, I0, J0, T, nbits, tid);
    __syncthreads();

    for (int r = wave; r < BE; r += 4) {
        if (I0 + r >= T) break;  // (rows past T have |K| = 0 in sMK)
        double xp[2 * Q];
#pragma unroll
        for (int c = 0; c < 2 * Q; ++c) xp[c] = sX[r][c];
        double f = sMK[r] * ct;
        if constexpr (W) f *= okt ? pair_w(E, I0 + r, Kt) : 0.0;
        const double fs = (CL && !nm_bit(nbits, r, col)) ? 0.0 : f;
        double M[Q][3];
        if constexpr (MIX) {
            float xf[2 * Q], Mf[Q][3];
#pragma unroll
            for (int c = 0; c < 2 * Q; ++c) xf[c] = sX[r][c];
#pragma unroll
            for (int p = 0; p < Q; ++p) Mf[p][0] = Mf[p][1] = Mf[p][2] = 0.f;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                float h = 0.f;
#pragma unroll
                for (int p = 0; p < Q; ++p) {
                    const float dx = xf[2 * p] - yqf[2 * q], dy = xf[2 * p + 1] - yqf[2 * q + 1];
                    const float kv = kpow32(dx * dx + dy * dy, pef);
                    Mf[p][0] += (float)cw[q][0] * kv;
                    Mf[p][1] += (float)cw[q][1] * kv;
                    Mf[p][2] += (float)cw[q][2] * kv;
                    h += (float)wq[p] * kv;
                }
                Psi[q] += fs * (double)h;
            }
#pragma unroll
            for (int p = 0; p < Q; ++p)
#pragma unroll
                for (int b = 0; b < 3; ++b) M[p][b] = Mf[p][b];
        } else {
#pragma unroll
        for (int p = 0; p < Q; ++p) M[p][0] = M[p][1] = M[p][2] = 0.0;
        // the Q evaluations of each point y_q of Kt form a batch; the table
        // reads of batch q + 1 are issued before the powers of batch q are
        // finished (two stages in turn), so their latency is covered by
        // this wave's own arithmetic
        KPowStage<Q> stg[2];
        auto issue = [&](int q, KPowStage<Q>& st) {
            double r2[Q];
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const double dx = xp[2 * p] - yq[2 * q], dy = xp[2 * p + 1] - yq[2 * q + 1];
                r2[p] = dx * dx + dy * dy;
            }
            kpow_tab_issue<Q>(kp, r2, st);
        };
        issue(0, stg[0]);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q + 1 < Q) issue(q + 1, stg[(q + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            double kvs[Q];
            kpow_tab_finish<Q>(kp, stg[q & 1], kvs);
            double h = 0.0;
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const double kv = kvs[p];
                M[p][0] += cw[q][0] * kv;
                M[p][1] += cw[q][1] * kv;
                M[p][2] += cw[q][2] * kv;
                h += wq[p] * kv;
            }
            Psi[q] += fs * h;
            __builtin_amdgcn_sched_barrier(0);
        }
        }
        // Phi_p of row r: the sum over the lanes of f G_p
        {
            double g[Q];
#pragma unroll
            for (int p = 0; p < Q; ++p) g[p] = fs * ((M[p][0] + M[p][1]) + M[p][2]);
            if constexpr (Q == 4) {
                const double v = wave_sum4_lanes(g);
                if ((lane & 15) == 0) sPhi[r][lane >> 4] = v;
            } else {
                const double v = wave_sum(g[0]);
                if (lane == 0) sPhi[r][0] = v;
            }
        }
        // off-diagonal block, scaled by -f
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double o[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int p = 0; p < Q; ++p)
#pragma unroll
                for (int b = 0; b < 3; ++b) o[b] += cw[p][a] * M[p][b];
            if (!direct) {
                const int ro = sRO[r][a];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    if constexpr (DET) {
                        const int idx = (ro + cbo[b]) >> 3;
                        const double th = -f * o[b] * P.fa.to_hi;
                        if (!(fabs(th) < 1073741824.0)) {
                            *P.fa.flag = 1;
                            continue;
                        }
                        const double fh = floor(th);
                        const long long lo = __double2ll_rn((th - fh) * P.fa.lo_per_hi);
                        if (fh != 0.0) atomicAdd(&Lhi[idx], (int)fh);
                        if (lo) atomicAdd((unsigned long long*)&L[idx], (unsigned long long)lo);
                    } else {
                        atomicAdd((double*)((char*)L + ro + cbo[b]), -f * o[b]);
                    }
                }
            } else if (okt) {
                const int ga = E.dof[a][I0 + r];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const int gb = E.dof[b][Kt];
                    if (ga < 0 || gb < 0) continue;
                    const double v = -f * o[b];
                    if constexpr (CL) {
                        nm_add(P.nm, ga, gb, v);
                        nm_add(P.nm, gb, ga, v);
                    } else {
                        add_pair_upper(P, ga, gb, v);
                    }
                }
            }
        }
    }
    __syncthreads();
    // diagonal blocks of the rows
    for (int i = tid; i < BE * 6; i += 256) {
        const int r = i / 6, m = i - r * 6, K = I0 + r;
        if (K >= T) continue;
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < Q; ++p) v += c_R.tri[off + p][6 + m] * sPhi[r][p];
        if (v != 0.0) acc_add(P.fs, P.S, (long long)K * 6 + m, v);
    }
    // off-diagonal block and its mirror into A
    if (DET && !direct) {
        // the words go to A's words (same scale), doubled on a folded diagonal
        const long long* Llo = (const long long*)L;
        for_block_entries(nVI, nVJ, tid, [&](int rr, int cc) {
            const long long lo = Llo[rr * LS + cc];
            const int hi = Lhi[rr * LS + cc];
            if (lo == 0 && hi == 0) return;
            const int gi = vI[rr], gj = vJ[cc];
            const long long k = gi == gj ? 2 : 1;
            const long long at = upper_index(gi, gj, P.lda);
            if (hi) atomicAdd(&P.fa.hi[at], (int)(k * hi));
            if (lo) atomicAdd((unsigned long long*)&P.fa.lo[at], (unsigned long long)(k * lo));
        });
    } else if (!direct) {
        for_block_entries(nVI, nVJ, tid, [&](int rr, int cc) {
            const double v = L[rr * LS + cc];
            if (v == 0.0) return;
            if constexpr (CL) {
                nm_add(P.nm, vI[rr], vJ[cc], v);
                nm_add(P.nm, vJ[cc], vI[rr], v);
            } else {
                add_pair_upper(P, vI[rr], vJ[cc], v);
            }
        });
    }
    __syncthreads();
    // diagonal blocks of the columns: each wave's part, added in wave order
    {
        double st[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) v += c_R.tri[off + q][6 + m] * Psi[q];
            st[m] = v;
        }
        double* stage = L;  // 4 x 64 x 6 doubles
#pragma unroll
        for (int m = 0; m < 6; ++m) stage[(wave * 64 + col) * 6 + m] = st[m];
    }
    __syncthreads();
    for (int i = tid; i < BE * 6; i += 256) {
        const int l = i / 6, m = i - l * 6, Ktt = J0 + l;
        if (Ktt >= T) continue;
        const double* stage = L;
        const double v = ((stage[(0 * 64 + l) * 6 + m] + stage[(1 * 64 + l) * 6 + m]) +
                          stage[(2 * 64 + l) * 6 + m]) + stage[(3 * 64 + l) * 6 + m];
        if (v != 0.0) acc_add(P.fs, P.S, (long long)Ktt * 6 + m, v);
    }
    if (tid == 0)
        atomicAdd(&P.cls_count[P.ncls], (unsigned long long)(min(BE, T - I0) * (long long)min(BE, T - J0)));
}

void launch_far(const ElemDev& E, const FarParams& P, hipStream_t st) {
    if (P.ntiles == 0) return;
    dim3 grid((unsigned)P.ntiles), block(256);
    if (P.nm.An) {
        // cluster near field: FP64, exact rules (the host refuses the rest)
        if (P.dim == 2) hipLaunchKernelGGL((near_kernel<2, 0, 0, 1>), grid, block, 0, st, E, P);
        else hipLaunchKernelGGL((near_kernel<1, 0, 0, 1>), grid, block, 0, st, E, P);
        return;
    }
    if (P.dim == 2) {
        if (P.sur.nsur > 0) {
            if (P.mixed) hipLaunchKernelGGL((near_kernel<2, 1, 1, 0>), grid, block, 0, st, E, P);
            else hipLaunchKernelGGL((near_kernel<2, 0, 1, 0>), grid, block, 0, st, E, P);
        } else {
            if (P.mixed) hipLaunchKernelGGL((near_kernel<2, 1, 0, 0>), grid, block, 0, st, E, P);
            else hipLaunchKernelGGL((near_kernel<2, 0, 0, 0>), grid, block, 0, st, E, P);
        }
    } else {
        if (P.mixed) hipLaunchKernelGGL((near_kernel<1, 1, 0, 0>), grid, block, 0, st, E, P);
        else hipLaunchKernelGGL((near_kernel<1, 0, 0, 0>), grid, block, 0, st, E, P);
    }
}

void launch_far_tiles(const ElemDev& E, const FarParams& P, int fark, hipStream_t st) {
    if (P.ntiles == 0) return;
    dim3 grid((unsigned)P.ntiles), block(256);
#define FL_FAR_CASE(D, K)                                                                    \
    do {                                                                                     \
        if (P.nm.An) hipLaunchKernelGGL((far_kernel<D, K, 0, 1>), grid, block, 0, st, E, P);      \
        else if (P.mixed) hipLaunchKernelGGL((far_kernel<D, K, 1, 0>), grid, block, 0, st, E, P); \
        else hipLaunchKernelGGL((far_kernel<D, K, 0, 0>), grid, block, 0, st, E, P);              \
    } while (0)
    if (P.dim == 2 && fark <= 2) {
        const bool w = E.w != nullptr;
#define FL_FAR2(K, MX, W) hipLaunchKernelGGL((far2_kernel<K, MX, W, 0, 0>), grid, block, 0, st, E, P)
#define FL_FAR2D(K, MX, W) hipLaunchKernelGGL((far2_kernel<K, MX, W, 0, 1>), grid, block, 0, st, E, P)
        if (P.nm.An) {
            if (fark == 1) hipLaunchKernelGGL((far2_kernel<1, 0, 0, 1, 0>), grid, block, 0, st, E, P);
            else hipLaunchKernelGGL((far2_kernel<2, 0, 0, 1, 0>), grid, block, 0, st, E, P);
        } else if (P.fa.lo) {
            if (fark == 1) {
                if (P.mixed) { if (w) FL_FAR2D(1, 1, 1); else FL_FAR2D(1, 1, 0); }
                else { if (w) FL_FAR2D(1, 0, 1); else FL_FAR2D(1, 0, 0); }
            } else {
                if (P.mixed) { if (w) FL_FAR2D(2, 1, 1); else FL_FAR2D(2, 1, 0); }
                else { if (w) FL_FAR2D(2, 0, 1); else FL_FAR2D(2, 0, 0); }
            }
        } else if (fark == 1) {
            if (P.mixed) { if (w) FL_FAR2(1, 1, 1); else FL_FAR2(1, 1, 0); }
            else { if (w) FL_FAR2(1, 0, 1); else FL_FAR2(1, 0, 0); }
        } else {
            if (P.mixed) { if (w) FL_FAR2(2, 1, 1); else FL_FAR2(2, 1, 0); }
            else { if (w) FL_FAR2(2, 0, 1); else FL_FAR2(2, 0, 0); }
        }
#undef FL_FAR2
#undef FL_FAR2D
    } else if (P.dim == 2) {
        switch (fark) {
            case 1: FL_FAR_CASE(2, 1); break;
            case 2: FL_FAR_CASE(2, 2); break;
            case 3: FL_FAR_CASE(2, 3); break;
            default: FL_FAR_CASE(2, 4); break;
        }
    } else {
        switch (fark) {
            case 1: FL_FAR_CASE(1, 1); break;
            case 2: FL_FAR_CASE(1, 2); break;
            case 3: FL_FAR_CASE(1, 3); break;
            default: FL_FAR_CASE(1, 4); break;
        }
    }
#undef FL_FAR_CASE
}

// ------------------------------------------------ identical + boundary --

// Identical triangle (regularised): I_ab = 4|K|^2 B_id sum over the half
// boundary of the difference hexagon of int_0^1 D_a D_b |z|^{-2-2s} dt,
// B_id = 2/((2-2s)(3-2s)(4-2s)).  Returns the 6 symmetric entries.
__device__ void ident2(const double* X, double s, double pe, int k, double* M6) {
    const double HX[4][3] = {{-1, 1, 0}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 0}};
    for (int m = 0; m < 6; ++m) M6[m] = 0.0;
    const int off = gl_off(k);
    for (int e = 0; e < 3; ++e)
        for (int i = 0; i < k; ++i) {
            double t = c_R.gl_x[off + i];
            double D[3];
            for (int a = 0; a < 3; ++a) D[a] = HX[e][a] + t * (HX[e + 1][a] - HX[e][a]);
            double z0 = D[0] * X[0] + D[1] * X[2] + D[2] * X[4];
            double z1 = D[0] * X[1] + D[1] * X[3] + D[2] * X[5];
            double kv = kpow(z0 * z0 + z1 * z1, pe) * c_R.gl_w[off + i];
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b) M6[sym3(a, b)] += kv * D[a] * D[b];
        }
    double area = 0.5 * fabs((X[2] - X[0]) * (X[5] - X[1]) - (X[4] - X[0]) * (X[3] - X[1]));
    double Bid = 2.0 / ((2.0 - 2.0 * s) * (3.0 - 2.0 * s) * (4.0 - 2.0 * s));
    double f = 4.0 * area * area * Bid;
    for (int m = 0; m < 6; ++m) M6[m] *= f;
}

// Boundary facet e = [p0,p1] (inward normal n) separated from triangle K:
// order-k triangle rule on K times k-point Gauss-Legendre on e.
template <class KP>
__device__ void bnd_far2(const double* X, const double* fe, const KP& kp, int k, double* M6) {
    const int to = tri_off(k), go = gl_off(k);
    const int Q = k * k;
    double area = 0.5 * fabs((X[2] - X[0]) * (X[5] - X[1]) - (X[4] - X[0]) * (X[3] - X[1]));
    double e0 = fe[2] - fe[0], e1 = fe[3] - fe[1];
    double Le = sqrt(e0 * e0 + e1 * e1);
    for (int p = 0; p < Q; ++p) {
        double l1 = c_R.tl1[to + p], l2 = c_R.tl2[to + p];
        double l0 = 1.0 - l1 - l2;
        double xx = l0 * X[0] + l1 * X[2] + l2 * X[4];
        double xy = l0 * X[1] + l1 * X[3] + l2 * X[5];
        double g = 0.0;
        for (int q = 0; q < k; ++q) {
            double t = c_R.gl_x[go + q];
            double d0 = xx - (fe[0] + t * e0), d1 = xy - (fe[1] + t * e1);
            g += c_R.gl_w[go + q] * (fe[4] * d0 + fe[5] * d1) * kp(d0 * d0 + d1 * d1);
        }
        g *= area * Le * c_R.tw[to + p];
        double lam[3] = {l0, l1, l2};
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) M6[sym3(a, b)] += g * lam[a] * lam[b];
    }
}

// e = [p0,p1] is an edge of K = (p0,p1,a) (local order p0,p1,a).  Polar
// form in (w,beta) about the edge with the gauge max(0,beta+w)+max(0,-w):
// unit polyline (1,0)->(0,1)->(-1,1)->(-1,0); radial weight r^{1-2s}
// (entries carrying the factor beta) or r^{-2s} (entries among p0,p1,
// finite only for s < 1/2), 2-point rules exact in r and in the foot
// variable, k-point Gauss-Legendre along the polyline.  Output in local
// order; entries among p0,p1 are NaN for s >= 1/2.
__device__ void bnd_edge2(const double* p0, const double* p1, const double* pa, const double* n,
                          double s, double pe, int k, double* M) {
    const double SEG[4][2] = {{1, 0}, {0, 1}, {-1, 1}, {-1, 0}};
    const int go = gl_off(k), g2 = gl_off(2);
    double E0 = p1[0] - p0[0], E1 = p1[1] - p0[1];
    double a0 = pa[0] - p0[0], a1 = pa[1] - p0[1];
    double na = n[0] * a0 + n[1] * a1;
    double Le = sqrt(E0 * E0 + E1 * E1);
    double area = 0.5 * fabs(E0 * a1 - a0 * E1);
    double acc[9];
    for (int m = 0; m < 9; ++m) acc[m] = 0.0;
    const bool lows = s < 0.5;
    for (int sg = 0; sg < 3; ++sg)
        for (int i = 0; i < k; ++i) {
            double t = c_R.gl_x[go + i];
            double pw = SEG[sg][0] + t * (SEG[sg + 1][0] - SEG[sg][0]);
            double pb = SEG[sg][1] + t * (SEG[sg + 1][1] - SEG[sg][1]);
            double z0 = pw * E0 + pb * a0, z1 = pw * E1 + pb * a1;
            double ang = c_R.gl_w[go + i] * pb * kpow(z0 * z0 + z1 * z1, pe);
            double lo = pw < 0.0 ? -pw : 0.0;
            for (int il = 0; il < 2; ++il) {
                double lx = c_R.gl_x[g2 + il], lw = c_R.gl_w[g2 + il];
                for (int ir = 0; ir < 2; ++ir) {
                    {
                        double r = c_R.r1_x[ir];
                        double tau = r * lo + lx * (1.0 - r);
                        double sig = tau + r * pw, beta = r * pb;
                        double lam[3] = {1.0 - sig - beta, sig, beta};
                        double wt = ang * lw * c_R.r1_w[ir] * (1.0 - r) * pb;
                        acc[6] += wt * lam[0];
                        acc[7] += wt * lam[1];
                        acc[8] += wt * lam[2];
                    }
                    if (lows) {
                        double r = c_R.r0_x[ir];
                        double tau = r * lo + lx * (1.0 - r);
                        double sig = tau + r * pw, beta = r * pb;
                        double l0 = 1.0 - sig - beta, l1 = sig;
                        double wt = ang * lw * c_R.r0_w[ir] * (1.0 - r);
                        acc[0] += wt * l0 * l0;
                        acc[1] += wt * l0 * l1;
                        acc[4] += wt * l1 * l1;
                    }
                }
            }
        }
    double f = 2.0 * area * Le * na;
    double nan = __longlong_as_double(0x7ff8000000000000ULL);
    M[0] = lows ? f * acc[0] : nan;
    M[1] = lows ? f * acc[1] : nan;
    M[3] = M[1];
    M[4] = lows ? f * acc[4] : nan;
    M[2] = M[6] = f * acc[6];
    M[5] = M[7] = f * acc[7];
    M[8] = f * acc[8];
}

// e = [q,p] shares only the vertex q with K = (q,b1,b2) (local order
// q,b1,b2).  Polar form in (u,v) with the gauge max(u,v); radial weight
// r^{1-2s}, 2-point rule exact; k-point Gauss-Legendre in the other two
// directions.
__device__ void bnd_vert2(const double* q, const double* b1, const double* b2, const double* pp,
                          const double* n, double pe, int k, double* M) {
    const int go = gl_off(k);
    double E0 = pp[0] - q[0], E1 = pp[1] - q[1];
    double Le = sqrt(E0 * E0 + E1 * E1);
    double area = 0.5 * fabs((b1[0] - q[0]) * (b2[1] - q[1]) - (b2[0] - q[0]) * (b1[1] - q[1]));
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int face = 0; face < 2; ++face)
        for (int i = 0; i < k; ++i) {
            double ti = c_R.gl_x[go + i];
            double pu = face == 0 ? 1.0 : ti;
            double pv = face == 0 ? ti : 1.0;
            for (int j = 0; j < k; ++j) {
                double tj = c_R.gl_x[go + j];
                double A0 = (b1[0] - q[0]) + tj * (b2[0] - b1[0]);
                double A1 = (b1[1] - q[1]) + tj * (b2[1] - b1[1]);
                double z0 = pu * A0 - pv * E0, z1 = pu * A1 - pv * E1;
                double ang = c_R.gl_w[go + i] * c_R.gl_w[go + j] * pu * pu * (n[0] * A0 + n[1] * A1) *
                             kpow(z0 * z0 + z1 * z1, pe);
                for (int ir = 0; ir < 2; ++ir) {
                    double uu = c_R.r1_x[ir] * pu;
                    double lam[3] = {1.0 - uu, uu * (1.0 - tj), uu * tj};
                    double wt = ang * c_R.r1_w[ir];
                    for (int a = 0; a < 3; ++a)
                        for (int b = a; b < 3; ++b) acc[sym3(a, b)] += wt * lam[a] * lam[b];
                }
            }
        }
    double f = 2.0 * area * Le;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = f * acc[sym3(a, b)];
}

// One thread per (element, chunk of P.fchunk boundary facets): the
// boundary term sum_e a^{Kxe} over the chunk (weight C/(2s)); the thread of
// chunk 0 adds the identical-pair term (weight C/2).  The partial 3x3 block
// is added to the element's diagonal-block accumulator S atomically, the
// pair counts once per wave.
template <int DIM>
__global__ __launch_bounds__(256) void self_kernel(ElemDev E, BndParams P) {
    // 2D: the kernel power of the separated element-edge pairs by the LDS
    // tables (same exponent as the separated element pairs)
    __shared__ __align__(16) double pw[DIM == 2 ? 768 : 1];
    if constexpr (DIM == 2) {
        load_pow_tables(pw);
        __syncthreads();
    }
    const int K0 = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = K0 < P.T;
    const int K = live ? K0 : P.T - 1;  // (threads past T count nothing and add nothing)
    const int e_lo = blockIdx.y * P.fchunk;
    const int e_hi = live ? min(P.nb, e_lo + P.fchunk) : e_lo;
    constexpr int NV = DIM + 1;
    double X[6] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < NV * DIM; ++c) X[c] = E.x[c][K];
    int vk[3] = {-1, -1, -1};
    for (int a = 0; a < NV; ++a) vk[a] = E.vid[a][K];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    // identical pair
    if (blockIdx.y != 0) {
    } else if (DIM == 1) {
        double h = fabs(X[1] - X[0]);
        double v = 2.0 * pow(h, 1.0 - 2.0 * P.s) / ((2.0 - 2.0 * P.s) * (3.0 - 2.0 * P.s));
        acc[0] = 0.5 * P.C * v;
        acc[1] = -0.5 * P.C * v;
        acc[3] = 0.5 * P.C * v;
    } else {
        double M6[6];
        ident2(X, P.s, P.pe, P.k_touch, M6);
        for (int m = 0; m < 6; ++m) acc[m] = 0.5 * P.C * M6[m];
    }
    if (P.with_boundary) {
        const double fb = P.C / (2.0 * P.s);
        double cx = E.cen[0][K], cy = DIM == 2 ? E.cen[1][K] : 0.0, h2k = E.h2[K];
        unsigned long long ntouch = 0, nfar = 0;
        for (int e = e_lo; e < e_hi; ++e) {
            const double* fe = P.fac + 6 * (long long)e;
            if (DIM == 1) {
                int fv = P.fvid[2 * e];
                double ye = fe[0];
                bool touching = (vk[0] == fv || vk[1] == fv);
                double h = fabs(X[1] - X[0]);
                double m00, m01, m11;
                if (touching) {
                    ++ntouch;
                    double hp = pow(h, 1.0 - 2.0 * P.s);
                    m00 = P.s < 0.5 ? hp * (1.0 / (1.0 - 2.0 * P.s) - 2.0 / (2.0 - 2.0 * P.s) +
                                            1.0 / (3.0 - 2.0 * P.s))
                                    : __longlong_as_double(0x7ff8000000000000ULL);
                    m01 = hp * (1.0 / (2.0 - 2.0 * P.s) - 1.0 / (3.0 - 2.0 * P.s));
                    m11 = hp / (3.0 - 2.0 * P.s);
                    if (vk[0] == fv) {
                        acc[0] += fb * m00; acc[1] += fb * m01; acc[3] += fb * m11;
                    } else {
                        acc[3] += fb * m00; acc[1] += fb * m01; acc[0] += fb * m11;
                    }
                } else {
                    ++nfar;
                    int cls = order_class(dist2_nc(cx, 0.0, ye, 0.0, 1), h2k, P.ncls, P.th2);
                    int k = P.kfb[cls];
                    const int go = gl_off(k);
                    for (int i = 0; i < k; ++i) {
                        double t = c_R.gl_x[go + i];
                        double x = X[0] + t * (X[1] - X[0]);
                        double kv = pow(fabs(x - ye), -2.0 * P.s) * h * c_R.gl_w[go + i];
                        double l0 = 1.0 - t, l1 = t;
                        acc[0] += fb * kv * l0 * l0;
                        acc[1] += fb * kv * l0 * l1;
                        acc[3] += fb * kv * l1 * l1;
                    }
                }
                continue;
            }
            int f0 = P.fvid[2 * e], f1 = P.fvid[2 * e + 1];
            int sh0 = -1, sh1 = -1;
            for (int a = 0; a < 3; ++a) {
                if (vk[a] == f0) sh0 = a;
                if (vk[a] == f1) sh1 = a;
            }
            const double p0[2] = {fe[0], fe[1]}, p1[2] = {fe[2], fe[3]}, nn[2] = {fe[4], fe[5]};
            if (sh0 >= 0 && sh1 >= 0) {
                ++ntouch;
                int ia = 3 - sh0 - sh1;
                double pa[2] = {X[2 * ia], X[2 * ia + 1]};
                double M[9];
                bnd_edge2(p0, p1, pa, nn, P.s, P.pe, P.k_touch_bnd, M);
                int g[3] = {sh0, sh1, ia};
                for (int a = 0; a < 3; ++a)
                    for (int b = a; b < 3; ++b) {
                        // local (p0,p1,a) -> element slots
                        int ea = g[a], eb = g[b];
                        acc[sym3(ea, eb)] += fb * M[3 * a + b];
                    }
            } else if (sh0 >= 0 || sh1 >= 0) {
                ++ntouch;
                int a = sh0 >= 0 ? sh0 : sh1;
                const double* pother = sh0 >= 0 ? p1 : p0;
                int i1 = (a + 1) % 3, i2 = (a + 2) % 3;
                if (vk[i1] > vk[i2]) { int tt = i1; i1 = i2; i2 = tt; }
                double q[2] = {X[2 * a], X[2 * a + 1]};
                double b1[2] = {X[2 * i1], X[2 * i1 + 1]}, b2[2] = {X[2 * i2], X[2 * i2 + 1]};
                double M[9];
                bnd_vert2(q, b1, b2, pother, nn, P.pe, P.k_touch_bnd, M);
                int g[3] = {a, i1, i2};
                for (int aa = 0; aa < 3; ++aa)
                    for (int bb = aa; bb < 3; ++bb) acc[sym3(g[aa], g[bb])] += fb * M[3 * aa + bb];
            } else {
                ++nfar;
                double m0 = (p0[0] + p1[0]) / 2.0, m1 = (p0[1] + p1[1]) / 2.0;
                double le2 = dist2_nc(p1[0], p1[1], p0[0], p0[1], 2);
                double hm = h2k > le2 ? h2k : le2;
                int cls = order_class(dist2_nc(cx, cy, m0, m1, 2), hm, P.ncls, P.th2);
                double M6[6] = {0, 0, 0, 0, 0, 0};
                bnd_far2(X, fe, make_kpow_tab(pw), P.kfb[cls], M6);
                for (int m = 0; m < 6; ++m) acc[m] += fb * M6[m];
            }
        }
        // (every lane of the wave takes part in the sums)
        for (int o = 32; o >= 1; o >>= 1) {
            ntouch += __shfl_xor(ntouch, o, 64);
            nfar += __shfl_xor(nfar, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            if (ntouch) atomicAdd(&P.counters[0], ntouch);
            if (nfar) atomicAdd(&P.counters[1], nfar);
        }
    }
    if (!live) return;
    const double wk = E.w ? E.w[K] : 1.0;
    for (int m = 0; m < 6; ++m)
        // (for s >= 1/2 the boundary term of a boundary vertex diverges; those
        // entries never reach A, and the words of the repeatable assembly
        // take finite values only)
        if (acc[m] != 0.0 && wk != 0.0 && (!P.fs.lo || isfinite(acc[m])))
            acc_add(P.fs, P.S, (long long)K * 6 + m, wk * acc[m]);
}

void launch_self(const ElemDev& E, const BndParams& P, hipStream_t st) {
    // facets per thread: doubled from 4 while the grid keeps about 2048
    // workgroups or more (fewer partial blocks added into S), at most 256
    BndParams Q = P;
    const long long wgx = (P.T + 255) / 256;
    int fc = 4;
    if (P.with_boundary)
        while (fc < 256 && wgx * ((P.nb + 2 * fc - 1) / (2 * fc)) >= 2048) fc *= 2;
    Q.fchunk = fc;
    const int chunks = P.with_boundary ? max(1, (P.nb + fc - 1) / fc) : 1;
    dim3 grid((unsigned)wgx, chunks), block(256);
    if (P.dim == 2)
        hipLaunchKernelGGL(self_kernel<2>, grid, block, 0, st, E, Q);
    else
        hipLaunchKernelGGL(self_kernel<1>, grid, block, 0, st, E, Q);
}

// ----------------------------------------------------- edge and vertex --

__device__ __forceinline__ void edge_acc(const double* E, const double* ap, const double* bp,
                                         double u, double v, double w, double wt, double pe,
                                         double* M6) {
    double z0 = w * E[0] + u * ap[0] - v * bp[0];
    double z1 = w * E[1] + u * ap[1] - v * bp[1];
    double kv = kpow(z0 * z0 + z1 * z1, pe) * wt;
    double P[3] = {u, v, w};
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) M6[sym3(a, b)] += kv * P[a] * P[b];
}

// output of the touching-pair kernels: the dense matrix, or the cluster
// near field (every touching pair lies in a near block)
__device__ __forceinline__ void touch_add(const TouchParams& P, int i, int j, double v) {
    if (P.nm.An) nm_add(P.nm, i, j, v);
    else if (i <= j) acc_add(P.fa, P.A, (long long)i * P.lda + j, v);  // (j, i) visits the same value
}

// Triangles sharing an edge: K = (q0,q1,a), Kt = (q0,q1,b), q0 < q1 by
// vertex id.  Coordinates (u,v,w) relative to the edge, analytic radial
// factor 1/((3-2s)(4-2s)), faces of the unit gauge surface: triangles F1,
// F4 (order-k collapsed rule) and parallelograms F2, F3 (k x k Gauss).
__global__ __launch_bounds__(256) void touch_edge2_kernel(ElemDev E, TouchParams P) {
    const long long pid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pid >= P.npairs) return;
    const int K = P.pairs[2 * pid], Kt = P.pairs[2 * pid + 1];
    int vk[3], vt[3];
    double X[6], Y[6];
    for (int a = 0; a < 3; ++a) { vk[a] = E.vid[a][K]; vt[a] = E.vid[a][Kt]; }
    for (int c = 0; c < 6; ++c) { X[c] = E.x[c][K]; Y[c] = E.x[c][Kt]; }
    int sk[2], st[2], ns = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (vk[a] == vt[b]) { sk[ns] = a; st[ns] = b; ++ns; }
    if (ns != 2) return;
    // order shared vertices by id
    if (vk[sk[0]] > vk[sk[1]]) {
        int t1 = sk[0]; sk[0] = sk[1]; sk[1] = t1;
        int t2 = st[0]; st[0] = st[1]; st[1] = t2;
    }
    const int ia = 3 - sk[0] - sk[1], ib = 3 - st[0] - st[1];
    const double q0[2] = {X[2 * sk[0]], X[2 * sk[0] + 1]};
    const double q1[2] = {X[2 * sk[1]], X[2 * sk[1] + 1]};
    const double Ev[2] = {q1[0] - q0[0], q1[1] - q0[1]};
    const double ap[2] = {X[2 * ia] - q0[0], X[2 * ia + 1] - q0[1]};
    const double bp[2] = {Y[2 * ib] - q0[0], Y[2 * ib + 1] - q0[1]};
    const int k = P.k;
    const int go = gl_off(k);
    double M6[6] = {0, 0, 0, 0, 0, 0};
    const double T1[3][3] = {{0, 1, 0}, {1, 1, 0}, {0, 1, 1}};
    const double T4[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 0, -1}};
    for (int f = 0; f < 2; ++f) {
        const double(*T)[3] = f == 0 ? T1 : T4;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                double u1 = c_R.gj_x[go + i];
                double l1 = u1, l2 = (1.0 - u1) * c_R.gl_x[go + j];
                double wt = 2.0 * c_R.gj_w[go + i] * c_R.gl_w[go + j];
                double Pp[3];
                for (int c = 0; c < 3; ++c) Pp[c] = T[0][c] + l1 * (T[1][c] - T[0][c]) + l2 * (T[2][c] - T[0][c]);
                edge_acc(Ev, ap, bp, Pp[0], Pp[1], Pp[2], 0.5 * wt, P.pe, M6);
            }
    }
    const double P2[3][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 1}};
    const double P3[3][3] = {{0, 1, 0}, {1, 0, 0}, {0, -1, -1}};
    for (int f = 0; f < 2; ++f) {
        const double(*T)[3] = f == 0 ? P2 : P3;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                double ti = c_R.gl_x[go + i], tj = c_R.gl_x[go + j];
                double Pp[3];
                for (int c = 0; c < 3; ++c) Pp[c] = T[0][c] + ti * T[1][c] + tj * T[2][c];
                edge_acc(Ev, ap, bp, Pp[0], Pp[1], Pp[2], c_R.gl_w[go + i] * c_R.gl_w[go + j], P.pe, M6);
            }
    }
    const double Cm[4][3] = {{-1, 1, -1}, {0, 0, 1}, {1, 0, 0}, {0, -1, 0}};
    double aK = E.meas[K], aT = E.meas[Kt];
    double f = P.C * 4.0 * aK * aT / ((3.0 - 2.0 * P.s) * (4.0 - 2.0 * P.s)) * pair_w(E, K, Kt);
    int g[4] = {E.dof[sk[0]][K], E.dof[sk[1]][K], E.dof[ia][K], E.dof[ib][Kt]};
    for (int i = 0; i < 4; ++i) {
        if (g[i] < 0) continue;
        for (int j = 0; j < 4; ++j) {
            if (g[j] < 0) continue;
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc += Cm[i][a] * M6[sym3(a, b)] * Cm[j][b];
            touch_add(P, g[i], g[j], f * acc);
        }
    }
}

// Elements sharing one vertex.  2D: K = (q,b1,b2), Kt = (q,c1,c2), b1 < b2,
// c1 < c2 by id; two prisms of the gauge max(X1+X2, X3+X4), analytic
// radial factor 1/(4-2s).  1D: K = [l,q], Kt = [q,r], faces u = 1, v = 1,
// radial factor 1/(3-2s).
template <int DIM>
__global__ __launch_bounds__(256) void touch_vert_kernel(ElemDev E, TouchParams P) {
    const long long pid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pid >= P.npairs) return;
    const int K = P.pairs[2 * pid], Kt = P.pairs[2 * pid + 1];
    const int k = P.k, go = gl_off(k);
    if (DIM == 1) {
        int vk[2] = {E.vid[0][K], E.vid[1][K]}, vt[2] = {E.vid[0][Kt], E.vid[1][Kt]};
        double X[2] = {E.x[0][K], E.x[1][K]}, Y[2] = {E.x[0][Kt], E.x[1][Kt]};
        int a = -1, b = -1;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                if (vk[i] == vt[j]) { a = i; b = j; }
        if (a < 0) return;
        double xq = X[a], xl = X[1 - a], xr = Y[1 - b];
        double h1 = fabs(xl - xq), h2 = fabs(xr - xq);
        double M[6] = {0, 0, 0, 0, 0, 0};
        for (int face = 0; face < 2; ++face)
            for (int i = 0; i < k; ++i) {
                double t = c_R.gl_x[go + i];
                double u = face == 0 ? 1.0 : t, v = face == 0 ? t : 1.0;
                double N[3] = {u, v - u, -v};
                double dd = h1 * u + h2 * v;
                double kv = kpow(dd * dd, P.pe) * c_R.gl_w[go + i];
                for (int p = 0; p < 3; ++p)
                    for (int q = p; q < 3; ++q) M[sym3(p, q)] += kv * N[p] * N[q];
            }
        double f = P.C * h1 * h2 / (3.0 - 2.0 * P.s) * pair_w(E, K, Kt);
        int g[3] = {E.dof[1 - a][K], E.dof[a][K], E.dof[1 - b][Kt]};
        for (int i = 0; i < 3; ++i) {
            if (g[i] < 0) continue;
            for (int j = 0; j < 3; ++j) {
                if (g[j] < 0) continue;
                touch_add(P, g[i], g[j], f * M[sym3(i, j)]);
            }
        }
        return;
    }
    int vk[3], vt[3];
    double X[6], Y[6];
    for (int a = 0; a < 3; ++a) { vk[a] = E.vid[a][K]; vt[a] = E.vid[a][Kt]; }
    for (int c = 0; c < 6; ++c) { X[c] = E.x[c][K]; Y[c] = E.x[c][Kt]; }
    int a = -1, b = -1;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (vk[i] == vt[j]) { a = i; b = j; }
    if (a < 0) return;
    int i1 = (a + 1) % 3, i2 = (a + 2) % 3, j1 = (b + 1) % 3, j2 = (b + 2) % 3;
    if (vk[i1] > vk[i2]) { int t = i1; i1 = i2; i2 = t; }
    if (vt[j1] > vt[j2]) { int t = j1; j1 = j2; j2 = t; }
    const double qx = X[2 * a], qy = X[2 * a + 1];
    const double g0[4] = {X[2 * i1] - qx, X[2 * i2] - qx, -(Y[2 * j1] - qx), -(Y[2 * j2] - qx)};
    const double g1[4] = {X[2 * i1 + 1] - qy, X[2 * i2 + 1] - qy, -(Y[2 * j1 + 1] - qy), -(Y[2 * j2 + 1] - qy)};
    double M[10];
    for (int m = 0; m < 10; ++m) M[m] = 0.0;
    for (int reg = 0; reg < 2; ++reg)
        for (int i = 0; i < k; ++i)
            for (int ii = 0; ii < k; ++ii)
                for (int jj = 0; jj < k; ++jj) {
                    double t = c_R.gl_x[go + i];
                    double u1 = c_R.gj_x[go + ii];
                    double l1 = u1, l2 = (1.0 - u1) * c_R.gl_x[go + jj];
                    double tw = 2.0 * c_R.gj_w[go + ii] * c_R.gl_w[go + jj];
                    double Xv[4];
                    if (reg == 0) { Xv[0] = 1.0 - t; Xv[1] = t; Xv[2] = l1; Xv[3] = l2; }
                    else { Xv[0] = l1; Xv[1] = l2; Xv[2] = 1.0 - t; Xv[3] = t; }
                    double z0 = 0.0, z1 = 0.0;
                    for (int c = 0; c < 4; ++c) { z0 += Xv[c] * g0[c]; z1 += Xv[c] * g1[c]; }
                    double kv = kpow(z0 * z0 + z1 * z1, P.pe) * c_R.gl_w[go + i] * 0.5 * tw;
                    int m = 0;
                    for (int p = 0; p < 4; ++p)
                        for (int q = p; q < 4; ++q) M[m++] += kv * Xv[p] * Xv[q];
                }
    // full 4x4 from packed
    double F[4][4];
    {
        int m = 0;
        for (int p = 0; p < 4; ++p)
            for (int q = p; q < 4; ++q) { F[p][q] = M[m]; F[q][p] = M[m]; ++m; }
    }
    const double Cm[5][4] = {{-1, -1, 1, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, -1}};
    double f = P.C * 4.0 * E.meas[K] * E.meas[Kt] / (4.0 - 2.0 * P.s) * pair_w(E, K, Kt);
    int g[5] = {E.dof[a][K], E.dof[i1][K], E.dof[i2][K], E.dof[j1][Kt], E.dof[j2][Kt]};
    for (int i = 0; i < 5; ++i) {
        if (g[i] < 0) continue;
        for (int j = 0; j < 5; ++j) {
            if (g[j] < 0) continue;
            double acc = 0.0;
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q) acc += Cm[i][p] * F[p][q] * Cm[j][q];
            touch_add(P, g[i], g[j], f * acc);
        }
    }
}

void launch_touch_edge2(const ElemDev& E, const TouchParams& P, hipStream_t st) {
    if (P.npairs == 0) return;
    dim3 grid((unsigned)((P.npairs + 255) / 256)), block(256);
    hipLaunchKernelGGL(touch_edge2_kernel, grid, block, 0, st, E, P);
}

void launch_touch_vert(const ElemDev& E, const TouchParams& P, hipStream_t st) {
    if (P.npairs == 0) return;
    dim3 grid((unsigned)((P.npairs + 255) / 256)), block(256);
    if (P.dim == 2)
        hipLaunchKernelGGL(touch_vert_kernel<2>, grid, block, 0, st, E, P);
    else
        hipLaunchKernelGGL(touch_vert_kernel<1>, grid, block, 0, st, E, P);
}

// --------------------------------------------------- diagonal blocks --

// P1 mass matrix entry of element K: integral of lambda_a lambda_b over K =
// |K| (1 + delta_ab) / ((d + 1)(d + 2))
__device__ __forceinline__ double mass_entry(double meas, int a, int b, int dim) {
    return meas * (a == b ? 2.0 : 1.0) / (double)((dim + 1) * (dim + 2));
}

// One thread per vertex: for every element K containing it, add the row
// of K's diagonal-block accumulator (and mass times K's mass matrix row)
// into A (only this thread writes the row, so the result is deterministic).
__global__ __launch_bounds__(256) void scatter_self_kernel(ElemDev E, const int* v2c_ptr,
                                                           const int* v2c_idx, const int* node2dof,
                                                           const unsigned char* vloc, int nv, int dim,
                                                           const double* S, double mass, double* A,
                                                           long long lda) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = node2dof[v];
    if (i < 0) return;
    double* row = A + (long long)i * lda;
    for (int e = v2c_ptr[v]; e < v2c_ptr[v + 1]; ++e) {
        const int K = v2c_idx[e];
        const int a = vloc[e];
        const double mk = mass * E.meas[K] * (E.w ? E.w[K] : 1.0);
        for (int b = 0; b <= dim; ++b) {
            int j = E.dof[b][K];
            if (j < 0) continue;
            if (j < i) continue;  // the lower triangle is the mirror of the upper
            double add = S[(long long)K * 6 + sym3(a, b)];
            if (mass != 0.0) add += mass_entry(mk, a, b, dim);
            row[j] += add;
        }
    }
}

void launch_scatter_self(const ElemDev& E, const int* v2c_ptr, const int* v2c_idx,
                         const int* node2dof, const unsigned char* vloc, int nv, int dim,
                         const double* S, double mass, double* A, long long lda, hipStream_t st) {
    dim3 grid((nv + 255) / 256), block(256);
    hipLaunchKernelGGL(scatter_self_kernel, grid, block, 0, st, E, v2c_ptr, v2c_idx, node2dof, vloc,
                       nv, dim, S, mass, A, lda);
}

__global__ __launch_bounds__(256) void fix_to_double_kernel(const long long* lo, const int* hi, double from_hi,
                                                            double from_lo, long long n, double* D) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long l = lo[i];
        const int h = hi[i];
        D[i] = (double)h * from_hi + (double)l * from_lo;
    }
}

void launch_fix_to_double(const long long* lo, const int* hi, double from_hi, double from_lo, long long n, double* D,
                          hipStream_t st) {
    if (n <= 0) return;
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fix_to_double_kernel, dim3((unsigned)blocks), dim3(256), 0, st, lo, hi, from_hi, from_lo, n, D);
}

// Lower triangle from the upper one: workgroup (J, I), I <= J, copies the
// transpose of the 64 x 64 tile (I, J) through LDS into tile (J, I)
// (diagonal tiles: their strictly lower part); workgroups with I > J exit.
// part 0: every tile I <= J (grid nt x nt); 1: the diagonal tiles only
// (grid nt x 1, I = J); 2: the tiles I < J only
__global__ __launch_bounds__(256) void mirror_lower_kernel(double* A, long long lda, int n, int part) {
    __shared__ double t[64][65];
    const int J = blockIdx.x, I = part == 1 ? J : (int)blockIdx.y;
    if (I > J || (part == 2 && I == J)) return;
    const int r0 = I * 64, c0 = J * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int gr = r0 + r, gc = c0 + tx;
        t[r][tx] = (gr < n && gc < n) ? A[(long long)gr * lda + gc] : 0.0;
    }
    __syncthreads();
    // row c0 + r of the lower tile = column r of the upper tile
    for (int r = ty; r < 64; r += 4) {
        const int gr = c0 + r, gc = r0 + tx;
        if (gr < n && gc < n && (I != J || tx < r)) A[(long long)gr * lda + gc] = t[tx][r];
    }
}

// zero the upper triangle and the padding columns of every row (row i:
// columns i .. lda-1; one workgroup per row at a time); the transpose writes
// the strictly lower triangle
__global__ __launch_bounds__(256) void zero_upper_kernel(double* A, long long lda, int n) {
    for (long long i = blockIdx.x; i < n; i += gridDim.x) {
        double* row = A + i * lda;
        for (long long j = i + threadIdx.x; j < lda; j += 256) row[j] = 0.0;
    }
}

void launch_zero_upper(double* A, long long lda, long long n, hipStream_t st) {
    if (n <= 0) return;
    const unsigned blocks = (unsigned)(n < 65536 ? n : 65536);
    hipLaunchKernelGGL(zero_upper_kernel, dim3(blocks), dim3(256), 0, st, A, lda, (int)n);
}

void launch_mirror_lower(double* A, long long lda, long long n, int part, hipStream_t st) {
    if (n <= 1) return;
    const unsigned nt = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(mirror_lower_kernel, dim3(nt, part == 1 ? 1u : nt), dim3(256), 0, st, A, lda, (int)n, part);
}

// The same into the cluster near field (entries (i, j) of elements around
// DOF i: near blocks; one thread per vertex owns row i, so no atomics).
__global__ __launch_bounds__(256) void scatter_self_near_kernel(ElemDev E, const int* v2c_ptr,
                                                                const int* v2c_idx, const int* node2dof,
                                                                const unsigned char* vloc, int nv, int dim,
                                                                const double* S, double mass, NearMap nm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = node2dof[v];
    if (i < 0) return;
    for (int e = v2c_ptr[v]; e < v2c_ptr[v + 1]; ++e) {
        const int K = v2c_idx[e];
        const int a = vloc[e];
        const double mk = mass * E.meas[K];
        for (int b = 0; b <= dim; ++b) {
            int j = E.dof[b][K];
            if (j < 0) continue;
            double add = S[(long long)K * 6 + sym3(a, b)];
            if (mass != 0.0) add += mass_entry(mk, a, b, dim);
            double* q = nm_slot(nm, i, j);
            if (q) *q += add;
        }
    }
}

void launch_scatter_self_near(const ElemDev& E, const int* v2c_ptr, const int* v2c_idx, const int* node2dof,
                              const unsigned char* vloc, int nv, int dim, const double* S, double mass,
                              const NearMap& nm, hipStream_t st) {
    if (nv == 0) return;
    hipLaunchKernelGGL(scatter_self_near_kernel, dim3((nv + 255) / 256), dim3(256), 0, st, E, v2c_ptr, v2c_idx,
                       node2dof, vloc, nv, dim, S, mass, nm);
}

__global__ __launch_bounds__(256) void near_diag_kernel(NearMap nm, long long n, double* d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* q = nm_slot(nm, (int)i, (int)i);
    d[i] = q ? *q : 0.0;
}

void launch_near_diag(const NearMap& nm, long long n, double* d, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(near_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nm, n, d);
}

// y_i = sum over the elements K of DOF i's vertex of K's mass matrix row
// times x (one thread per DOF, fixed order)
__global__ __launch_bounds__(256) void mass_matvec_kernel(ElemDev E, const int* dof_node, const int* v2c_ptr,
                                                          const int* v2c_idx, const unsigned char* vloc,
                                                          int dim, long long n, const double* x, double* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int v = dof_node[i];
    double acc = 0.0;
    for (int e = v2c_ptr[v]; e < v2c_ptr[v + 1]; ++e) {
        const int K = v2c_idx[e];
        const int a = vloc[e];
        for (int b = 0; b <= dim; ++b) {
            const int j = E.dof[b][K];
            if (j >= 0) acc += mass_entry(E.meas[K], a, b, dim) * x[j];
        }
    }
    y[i] = acc;
}

void launch_mass_matvec(const ElemDev& E, const int* dof_node, const int* v2c_ptr, const int* v2c_idx,
                        const unsigned char* vloc, int dim, long long n, const double* x, double* y,
                        hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(mass_matvec_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, E, dof_node,
                       v2c_ptr, v2c_idx, vloc, dim, n, x, y);
}

__global__ void zero_kernel(double* p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

void launch_zero(double* p, long long n, hipStream_t st) {
    if (n <= 0) return;
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}

// b_i = sum_{K containing i} |K| / (d+1)  (f = 1)
__global__ void load_one_kernel(const int* dof_node, const int* v2c_ptr, const int* v2c_idx,
                                const double* meas, int dim, long long n, double* b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int v = dof_node[i];
    double acc = 0.0;
    for (int e = v2c_ptr[v]; e < v2c_ptr[v + 1]; ++e) acc += meas[v2c_idx[e]];
    b[i] = acc / (double)(dim + 1);
}

void launch_load_one(const int* dof_node, const int* v2c_ptr, const int* v2c_idx,
                     const double* meas, int dim, long long n, double* b, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(load_one_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dof_node,
                       v2c_ptr, v2c_idx, meas, dim, n, b);
}

// Pair integrals of m separated triangle pairs with the order-k rule.
// canonical = 0: the 21 integrals (areas included) in the given vertex
// order; canonical = 1: features of the canonical form (feats) and the
// relative error t = I_k / Q2 - 1 of the order-2 rule (out), both on the
// canonical pair.
__global__ __launch_bounds__(256) void pair_integrals_kernel(const double* X, const double* Y,
                                                             const double* s, long long m, int k,
                                                             int canonical, double* out, double* feats) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double x[6], y[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        x[c] = X[i * 6 + c];
        y[c] = Y[i * 6 + c];
    }
    const double sv = s[i], pe = -(1.0 + sv);
    double SK[6], ST[6], O[9];
    double* o = out + i * 21;
    if (!canonical) {
        far_pair2<0>(k, x, y, pe, SK, ST, O);
        auto area = [](const double* P) {
            return 0.5 * fabs((P[2] - P[0]) * (P[5] - P[1]) - (P[3] - P[1]) * (P[4] - P[0]));
        };
        const double f = area(x) * area(y);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            o[j] = f * SK[j];
            o[6 + j] = f * ST[j];
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) o[12 + j] = f * O[j];
        return;
    }
    int o1[3], o2[3];
    double C1[6], C2[6], fe[SUR_NIN];
    sur_canon(x, y, o1, o2, C1, C2);
    sur_features(C1, C2, sv, fe);
#pragma unroll
    for (int j = 0; j < SUR_NIN; ++j) feats[i * SUR_NIN + j] = fe[j];
    double SK2[6], ST2[6], O2[9];
    far_pair2<0>(k, C1, C2, pe, SK, ST, O);
    far_pair2<2>(2, C1, C2, pe, SK2, ST2, O2);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        o[j] = SK[j] / SK2[j] - 1.0;
        o[6 + j] = ST[j] / ST2[j] - 1.0;
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) o[12 + j] = O[j] / O2[j] - 1.0;
}

void launch_pair_integrals(const double* X, const double* Y, const double* s, long long m, int k,
                           int canonical, double* out, double* feats, hipStream_t st) {
    if (m <= 0) return;
    hipLaunchKernelGGL(pair_integrals_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, X, Y, s,
                       m, k, canonical, out, feats);
}

}  // namespace fl
