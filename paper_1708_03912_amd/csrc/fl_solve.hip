// Device kernels of the solve (Sec. 5): the symmetric product that reads
// the upper triangle of the dense matrix, Jacobi-preconditioned CG (one
// launch pair per iteration, the scalars on the device), its FP32 variant
// with FP64 residual replacement, and the small helpers around them
// (diagonal, dot products, casts).  gfx950.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fl_internal.hpp"

namespace fl {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
// ---------------------------------------------------------------- solve --

__global__ void diag_kernel(const double* A, long long lda, long long n, double* d) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = A[i * lda + i];
}

void launch_diag(const double* A, long long lda, long long n, double* d, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, lda, n, d);
}

// deterministic block reduction (256 threads)
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// sum of the first m partials, same order in every block
__device__ __forceinline__ double sum_partials(const double* part, int m, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) v += part[i];
    return block_sum(v, sh);
}

// this lane's share of the sum of the first m partials (lane stride 256,
// four accumulators): the same order in every block
__device__ __forceinline__ double load_partials(const double* part, int m) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = threadIdx.x;
    for (; i + 768 < m; i += 1024) {
        s0 += part[i];
        s1 += part[i + 256];
        s2 += part[i + 512];
        s3 += part[i + 768];
    }
    for (; i < m; i += 256) s0 += part[i];
    return (s0 + s1) + (s2 + s3);
}

// three block sums with one pair of barriers (256 threads, sh: 12 doubles)
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[w] = a;
        sh[4 + w] = b;
        sh[8 + w] = c;
    }
    __syncthreads();
    a = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    b = (sh[4] + sh[5]) + (sh[6] + sh[7]);
    c = (sh[8] + sh[9]) + (sh[10] + sh[11]);
    __syncthreads();
}

// Symmetric dense product from the upper triangle.  The stiffness matrix is
// symmetric (Sec. 5: every pair adds a block and its transpose), so a
// product reads only its 64 x 64 tiles (bi <= bj): half of the n^2 entries.
// Workgroup (J, I) of an (nJ, nI) grid takes the tiles of block rows
// I R .. I R + R - 1 and block columns J m .. J m + m - 1 on or above the
// diagonal, row by row, with the next tile's loads in flight while the
// current one is used.  It forms the row sums A_IJ v_J of each of its block
// rows, summed over its tiles in registers, and the column sums A_IJ^T v_I
// of its tiles with bi < bj, summed over its rows in LDS.  Partial sums go
// to slots that exactly one workgroup writes (no atomics):
//   prow[J n + i]  row sums of workgroup column J in the block row of i,
//                  for J = b / m .. nJ - 1 (b the block of i),
//   pcol[I n + j]  column sums of workgroup row I for j in block b,
//                  for I = 0 .. b / R (zero where no tile lies above),
// and (A v)_i is their sum in that order (fixed order).  Grouping R rows
// makes an element's column slots one per R block rows instead of one per
// tile, which keeps the slots' traffic a few percent of the matrix's.
// Small systems (R = 1) take strips of m tiles from each block row's
// diagonal instead (every strip but a row's last full, the column sums
// stored per tile), which suits their few, latency-bound workgroups.
// Thread (wave w, lane l) holds columns 16 w + 2 (l & 7) + {0, 1} and rows
// (l >> 3) + 8 k, k = 0..7, of each tile: one load of a wave covers eight
// contiguous row segments of 16 entries.  A column sum is complete after
// three exchanges inside the wave; the row sums are reduced once per block
// row (three exchanges, then the four waves in order through LDS).
typedef double sym_d2 __attribute__((ext_vector_type(2)));
typedef float sym_f2 __attribute__((ext_vector_type(2)));
template <class T>
struct Pair2;
template <>
struct Pair2<double> {
    using type = sym_d2;
};
template <>
struct Pair2<float> {
    using type = sym_f2;
};

// the thread's 8 x 2 entries of tile (bi, bj).  Branch-free: indices
// outside n x n are clamped into the matrix (rows to n - 1, columns to
// lda - 2); sym_unpack zeroes those entries.
// live = false: the loads still issue (so that the waits of the caller
// count the same loads on every path) but all read row I0 of the tile just
// loaded, which is in the cache; the values are not used.
template <class T>
__device__ __forceinline__ void sym_load(const T* __restrict__ A, long long lda, long long n, long long I0,
                                         long long j, typename Pair2<T>::type (&raw)[8], bool live = true) {
    using V2 = typename Pair2<T>::type;
    const int rg = (threadIdx.x & 63) >> 3;
    const long long jc = min(j, lda - 2);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const long long i = live ? min(I0 + rg + 8 * k, n - 1) : min(I0, n - 1);
        raw[k] = __builtin_nontemporal_load((const V2*)(A + i * lda + jc));
    }
}

template <class T>
__device__ __forceinline__ void sym_unpack(const typename Pair2<T>::type (&raw)[8], long long n, long long I0,
                                           long long j, double (&a0)[8], double (&a1)[8]) {
    const int rg = (threadIdx.x & 63) >> 3;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool in = I0 + rg + 8 * k < n && j < n;
        a0[k] = in ? (double)raw[k].x : 0.0;
        a1[k] = (in && j + 1 < n) ? (double)raw[k].y : 0.0;
    }
}

// Vectors of the product, read as raw loads (issued early, with the tiles)
// and turned into FP64 values afterwards: the vector x itself, or the CG
// direction p_it = z + beta p_{it-1} formed on the fly.
template <class T>
struct SymVecX {
    const T* x;
    struct L {
        T a;
    };
    __device__ __forceinline__ L load(long long i) const { return {x[i]}; }
    __device__ __forceinline__ double val(const L& l) const { return (double)l.a; }
};
template <class T>
struct SymVecP {
    const T* z;
    const T* pp;
    T beta;
    struct L {
        T a, b;
    };
    __device__ __forceinline__ L load(long long i) const { return {z[i], pp[i]}; }
    __device__ __forceinline__ double val(const L& l) const { return (double)(T)(l.a + beta * l.b); }
};

// One block row of a workgroup's tiles: tiles bj = b0 .. b1 - 1 of block
// row bi with the vector V.  The row sums go to the slot prow[J n + i] (the
// caller's workgroup column J); the column sums of every tile with bj > bi
// are added to cacc[(bj - J0) 64 + column in the tile] (LDS, one thread per
// entry within a row; the barrier at the end of the row orders the rows'
// additions), or with direct (one block row per workgroup) stored to their
// slot pcol[bi n + j] at once.  Returns this thread's share of the row's
// part of v^T A v (with direct, the column sums' part too).
// red: 256 doubles of LDS.  Loads of the next tile and of its vector entries
// (indices clamped into the arrays, so the loads are unconditional and the
// waits count only older ones) are issued before the current tile is used.
template <class T, class VF>
__device__ __forceinline__ double sym_row(const T* __restrict__ A, long long lda, const SymPlan& P, int bi, int b0,
                                          int b1, int J, int J0, bool direct, const VF& V, double* red,
                                          double* cacc) {
    using V2 = typename Pair2<T>::type;
    using VL = typename VF::L;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, cp = lane & 7, rg = lane >> 3;
    const long long n = P.n, I0 = (long long)bi * SYM_TB;
    const int coff = 16 * w + 2 * cp;
    double vi[8], racc[8];
    {
        VL li[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) li[k] = V.load(min(I0 + rg + 8 * k, n - 1));
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            vi[k] = I0 + rg + 8 * k < n ? V.val(li[k]) : 0.0;
            racc[k] = 0.0;
        }
    }
    double vcol = 0.0;  // (direct) the column sums' part of v^T A v
    // tile bj (its entries raw, its vector entries l0, l1) into the row and
    // column sums
    auto tile = [&](int bj, long long j, const V2 (&raw)[8], const VL& l0, const VL& l1) {
        const double x0 = j < n ? V.val(l0) : 0.0, x1 = j + 1 < n ? V.val(l1) : 0.0;
        double a0[8], a1[8];
        sym_unpack<T>(raw, n, I0, j, a0, a1);
        double c0 = 0.0, c1 = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            racc[k] += a0[k] * x0 + a1[k] * x1;
            c0 += a0[k] * vi[k];
            c1 += a1[k] * vi[k];
        }
        if (bj > bi) {
            // column sums over the 8 row groups (lane bits 3..5); lanes 0..7
            // end with column j, lanes 32..39 with column j + 1
            const int h5 = (lane >> 5) & 1;
            double y = (h5 ? c1 : c0) + __shfl_xor(h5 ? c0 : c1, 32, 64);
            y += __shfl_xor(y, 16, 64);
            y += __shfl_xor(y, 8, 64);
            if ((lane & 0x18) == 0) {
                if (!direct) {
                    cacc[(bj - J0) * SYM_TB + coff + h5] += y;
                } else if (j + h5 < n) {
                    P.pcol[(long long)bi * n + j + h5] = y;
                    vcol += y * (h5 ? x1 : x0);
                }
            }
        }
    };
    // two buffers in turn: the next tile's loads (and its vector entries)
    // are issued before the current tile is used, with no copy between the
    // buffers and no branch around the loads (past the end of the row they
    // read the current tile's first row again), so the waits count only the
    // older loads
    V2 ra[8], rb[8];
    VL a0, a1, c0, c1;
    long long j = (long long)b0 * SYM_TB + coff;
    sym_load<T>(A, lda, n, I0, j, ra);
    a0 = V.load(min(j, n - 1));
    a1 = V.load(min(j + 1, n - 1));
    for (int bj = b0;; bj += 2, j += 2 * SYM_TB) {
        const bool lb = bj + 1 < b1;
        const long long jb = lb ? j + SYM_TB : j;
        sym_load<T>(A, lda, n, I0, jb, rb, lb);
        c0 = V.load(min(jb, n - 1));
        c1 = V.load(min(jb + 1, n - 1));
        __builtin_amdgcn_sched_barrier(0);  // no use of rb, c0, c1 moves above here
        tile(bj, j, ra, a0, a1);
        if (!lb) break;
        const bool la = bj + 2 < b1;
        const long long ja = la ? j + 2 * SYM_TB : j + SYM_TB;
        sym_load<T>(A, lda, n, I0, ja, ra, la);
        a0 = V.load(min(ja, n - 1));
        a1 = V.load(min(ja + 1, n - 1));
        __builtin_amdgcn_sched_barrier(0);
        tile(bj + 1, j + SYM_TB, rb, c0, c1);
        if (!la) break;
    }
    // row sums: over the column pairs (lane bits 0..2, halving exchange:
    // lane cp ends with row rg + 8 cp), then over the waves in order
    {
        const int q2 = (cp >> 2) & 1, q1 = (cp >> 1) & 1, q0 = cp & 1;
        double w4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            w4[u] = (q2 ? racc[4 + u] : racc[u]) + __shfl_xor(q2 ? racc[u] : racc[4 + u], 4, 64);
        double w2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) w2[u] = (q1 ? w4[2 + u] : w4[u]) + __shfl_xor(q1 ? w4[u] : w4[2 + u], 2, 64);
        const double y = (q0 ? w2[1] : w2[0]) + __shfl_xor(q0 ? w2[0] : w2[1], 1, 64);
        red[w * 64 + rg + 8 * cp] = y;
    }
    __syncthreads();
    double vd = vcol;
    if (t < 64) {
        const double s = ((red[t] + red[64 + t]) + red[128 + t]) + red[192 + t];
        const long long i = I0 + t;
        if (i < n) {
            P.prow[(long long)J * n + i] = s;
            vd += s * V.val(V.load(i));
        }
    }
    __syncthreads();  // red is rewritten by the next row
    return vd;
}

// FP32 matrix: the same row with 16-byte loads.  Thread (wave w, lane l)
// holds columns 32 (w & 1) + 4 (l & 7) .. + 3 of tile b + (w >> 1) and rows
// (l >> 3) + 8 k, so one step of the workgroup covers two tiles (waves 0, 1
// the first, waves 2, 3 the second) with eight loads per thread.  Column
// sums: a four-value halving exchange over the row groups (lanes with
// (l >> 3) = 0, 2, 4, 6 end with columns +0..+3); row sums as above.
typedef float sym_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void sym_load4(const float* __restrict__ A, long long lda, long long n, long long I0,
                                          long long j, sym_f4 (&raw)[8], bool live) {
    const int rg = (threadIdx.x & 63) >> 3;
    const long long jc = min(j, lda - 4);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const long long i = live ? min(I0 + rg + 8 * k, n - 1) : min(I0, n - 1);
        raw[k] = __builtin_nontemporal_load((const sym_f4*)(A + i * lda + jc));
    }
}

template <class VF>
__device__ __forceinline__ double sym_row4(const float* __restrict__ A, long long lda, const SymPlan& P, int bi,
                                           int b0, int b1, int J, int J0, bool direct, const VF& V, double* red,
                                           double* cacc) {
    using VL = typename VF::L;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, cq = lane & 7, rg = lane >> 3;
    const long long n = P.n, I0 = (long long)bi * SYM_TB;
    const int half = w >> 1, coff = 32 * (w & 1) + 4 * cq;
    double vi[8], racc[8];
    {
        VL li[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) li[k] = V.load(min(I0 + rg + 8 * k, n - 1));
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            vi[k] = I0 + rg + 8 * k < n ? V.val(li[k]) : 0.0;
            racc[k] = 0.0;
        }
    }
    double vcol = 0.0;  // (direct) the column sums' part of v^T A v
    // this wave's tile of step s (tile b0 + 2 s + half), its first column,
    // and whether it lies in the row's range
    auto col = [&](int s) { return (long long)(b0 + 2 * s + half) * SYM_TB + coff; };
    auto live = [&](int s) { return b0 + 2 * s + half < b1; };
    auto step = [&](int s, const sym_f4 (&raw)[8], const VL (&lx)[4]) {
        const int bj = b0 + 2 * s + half;
        const bool lv = bj < b1;
        const long long j = (long long)bj * SYM_TB + coff;
        double x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = (lv && j + m < n) ? V.val(lx[m]) : 0.0;
        double cs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool in = lv && I0 + rg + 8 * k < n;
            const double a[4] = {(in && j < n) ? (double)raw[k].x : 0.0, (in && j + 1 < n) ? (double)raw[k].y : 0.0,
                                 (in && j + 2 < n) ? (double)raw[k].z : 0.0,
                                 (in && j + 3 < n) ? (double)raw[k].w : 0.0};
            racc[k] += (a[0] * x[0] + a[1] * x[1]) + (a[2] * x[2] + a[3] * x[3]);
#pragma unroll
            for (int m = 0; m < 4; ++m) cs[m] += a[m] * vi[k];
        }
        if (lv && bj > bi) {
            const int h5 = (lane >> 5) & 1, h4 = (lane >> 4) & 1;
            double u[2];
#pragma unroll
            for (int q = 0; q < 2; ++q)
                u[q] = (h5 ? cs[2 + q] : cs[q]) + __shfl_xor(h5 ? cs[q] : cs[2 + q], 32, 64);
            double y = (h4 ? u[1] : u[0]) + __shfl_xor(h4 ? u[0] : u[1], 16, 64);
            y += __shfl_xor(y, 8, 64);
            if ((lane & 8) == 0) {
                const int m = 2 * h5 + h4;
                if (!direct) {
                    cacc[(bj - J0) * SYM_TB + coff + m] += y;
                } else if (j + m < n) {
                    P.pcol[(long long)bi * n + j + m] = y;
                    vcol += y * x[m];
                }
            }
        }
    };
    const int ns = (b1 - b0 + 1) / 2;  // steps of two tiles
    sym_f4 ra[8], rb[8];
    VL la[4], lb[4];
    {
        const bool l0 = live(0);
        const long long j = l0 ? col(0) : (long long)b0 * SYM_TB + coff;
        sym_load4(A, lda, n, I0, j, ra, l0);
#pragma unroll
        for (int m = 0; m < 4; ++m) la[m] = V.load(min(j + m, n - 1));
    }
    for (int s = 0;; s += 2) {
        {
            const bool ln = s + 1 < ns && live(s + 1);
            const long long j = ln ? col(s + 1) : (long long)b0 * SYM_TB + coff;
            sym_load4(A, lda, n, I0, j, rb, ln);
#pragma unroll
            for (int m = 0; m < 4; ++m) lb[m] = V.load(min(j + m, n - 1));
        }
        __builtin_amdgcn_sched_barrier(0);
        step(s, ra, la);
        if (s + 1 >= ns) break;
        {
            const bool ln = s + 2 < ns && live(s + 2);
            const long long j = ln ? col(s + 2) : (long long)b0 * SYM_TB + coff;
            sym_load4(A, lda, n, I0, j, ra, ln);
#pragma unroll
            for (int m = 0; m < 4; ++m) la[m] = V.load(min(j + m, n - 1));
        }
        __builtin_amdgcn_sched_barrier(0);
        step(s + 1, rb, lb);
        if (s + 2 >= ns) break;
    }
    // row sums: over the column quads (lane bits 0..2), then the waves
    {
        const int q2 = (cq >> 2) & 1, q1 = (cq >> 1) & 1, q0 = cq & 1;
        double w4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            w4[u] = (q2 ? racc[4 + u] : racc[u]) + __shfl_xor(q2 ? racc[u] : racc[4 + u], 4, 64);
        double w2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) w2[u] = (q1 ? w4[2 + u] : w4[u]) + __shfl_xor(q1 ? w4[u] : w4[2 + u], 2, 64);
        const double y = (q0 ? w2[1] : w2[0]) + __shfl_xor(q0 ? w2[0] : w2[1], 1, 64);
        red[w * 64 + rg + 8 * cq] = y;
    }
    __syncthreads();
    double vd = vcol;
    if (t < 64) {
        const double s = ((red[t] + red[64 + t]) + red[128 + t]) + red[192 + t];
        const long long i = I0 + t;
        if (i < n) {
            P.prow[(long long)J * n + i] = s;
            vd += s * V.val(V.load(i));
        }
    }
    __syncthreads();  // red is rewritten by the next row
    return vd;
}

// Workgroup (J, I) holds the tiles (bi, bj), bi <= bj, of block rows
// bi = I R .. I R + R - 1 and block columns bj = J m .. J m + m - 1 (those
// past the end or below the diagonal excepted; a workgroup whose columns
// all lie left of its first row has none).  R = 1 (small systems): block
// row I and the strip bj = I + J m .. I + J m + m - 1 from its diagonal
// instead, so that every strip but a row's last is full.
__device__ __forceinline__ bool sym_group_live(const SymPlan& P, int I, int J) {
    if (P.R == 1) return I + J * P.m < P.nb;
    return J * P.m + P.m - 1 >= I * P.R && J * P.m < P.nb;
}

// The workgroup's part of the product, block row by block row: row sums to
// prow[J n + i] for its rows, column sums accumulated in LDS (cacc: m x 64
// doubles) over its rows and written to pcol[I n + j] for every column j of
// its block columns bj >= I R (zero where no tile of the workgroup lies
// above the diagonal in that column).  Returns this thread's share of the
// workgroup's part of v^T A v (diagonal tiles once, the others twice).
template <class T, class VF>
__device__ __forceinline__ double sym_group_any(const T* __restrict__ A, long long lda, const SymPlan& P, int I,
                                                int J, const VF& V, double* red, double* cacc) {
    const int t = threadIdx.x;
    const long long n = P.n;
    if (P.R == 1) {
        const int b0 = I + J * P.m, b1 = min(P.nb, b0 + P.m);
        if constexpr (std::is_same<T, float>::value) return sym_row4(A, lda, P, I, b0, b1, J, b0, true, V, red, cacc);
        else return sym_row<T>(A, lda, P, I, b0, b1, J, b0, true, V, red, cacc);
    }
    const int J0 = J * P.m, J1 = min(P.nb, J0 + P.m);
    for (int q = t; q < P.m * SYM_TB; q += 256) cacc[q] = 0.0;
    __syncthreads();
    double vd = 0.0;
    for (int r = 0; r < P.R; ++r) {
        const int bi = I * P.R + r;
        const int b0 = max(J0, bi);
        if (bi >= P.nb || b0 >= J1) break;  // (the rows below start further right still)
        if constexpr (std::is_same<T, float>::value) vd += sym_row4(A, lda, P, bi, b0, J1, J, J0, false, V, red, cacc);
        else vd += sym_row<T>(A, lda, P, bi, b0, J1, J, J0, false, V, red, cacc);
    }
    const int c0 = max(J0, I * P.R + 1);  // (columns with a row of the workgroup above them)
    for (int q = (c0 - J0) * SYM_TB + t; q < (J1 - J0) * SYM_TB; q += 256) {
        const long long j = (long long)J0 * SYM_TB + q;
        if (j < n) {
            const double y = cacc[q];
            P.pcol[(long long)I * n + j] = y;
            vd += y * V.val(V.load(j));
        }
    }
    return vd;
}

// this lane's share of (A v)_i from the slots (lane g of an aligned group
// of P.G takes every G-th slot); group_sum completes it
__device__ __forceinline__ double sym_gather_share(const SymPlan& P, long long i, int g) {
    const int G = P.G;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < P.n) {
        // row slots of the workgroup columns J = b / m .. nJ - 1 (R = 1: the
        // strips J = 0 .. of block row b), then the column slots of the
        // workgroup rows I with I R < b
        const int b = (int)(i / SYM_TB);
        const int jr0 = P.R == 1 ? 0 : b / P.m;
        const int nrow = P.R == 1 ? (P.nb - b + P.m - 1) / P.m : P.nJ - jr0;
        const int ns = nrow + (b + P.R - 1) / P.R;
        auto slot = [&](int u) -> double {
            return u < nrow ? P.prow[(long long)(jr0 + u) * P.n + i] : P.pcol[(long long)(u - nrow) * P.n + i];
        };
        int u = g;
        for (; u + 3 * G < ns; u += 4 * G) {
            const double v0 = slot(u), v1 = slot(u + G), v2 = slot(u + 2 * G), v3 = slot(u + 3 * G);
            s0 += v0;
            s1 += v1;
            s2 += v2;
            s3 += v3;
        }
        for (; u < ns; u += G) s0 += slot(u);
    }
    return (s0 + s1) + (s2 + s3);
}

// sum over an aligned group of G lanes (all lanes must call it)
__device__ __forceinline__ double group_sum(double s, int G) {
    for (int o = 1; o < G; o <<= 1) s += __shfl_xor(s, o);
    return s;
}

// slots of A x (plain product)
template <class T>
__global__ __launch_bounds__(256) void symv_kernel(const T* __restrict__ A, long long lda, SymPlan P,
                                                   const T* __restrict__ x) {
    __shared__ double red[256];
    __shared__ double cacc[SYM_M * SYM_TB];
    const int I = blockIdx.y, J = blockIdx.x;
    if (!sym_group_live(P, I, J)) return;
    (void)sym_group_any<T>(A, lda, P, I, J, SymVecX<T>{x}, red, cacc);
}

// y = A x from the slots
__global__ __launch_bounds__(256) void sym_reduce_kernel(SymPlan P, double* y) {
    const long long i = (long long)blockIdx.x * (256 / P.G) + threadIdx.x / P.G;
    const int g = threadIdx.x & (P.G - 1);
    const double s = group_sum(sym_gather_share(P, i, g), P.G);
    if (g == 0 && i < P.n) y[i] = s;
}

// r = b - A x in FP64 from the slots, also r32 = (float) r
__global__ __launch_bounds__(256) void sym_residual_kernel(SymPlan P, const double* b, double* r, float* r32) {
    const long long i = (long long)blockIdx.x * (256 / P.G) + threadIdx.x / P.G;
    const int g = threadIdx.x & (P.G - 1);
    const double s = group_sum(sym_gather_share(P, i, g), P.G);
    if (g == 0 && i < P.n) {
        const double ri = b[i] - s;
        r[i] = ri;
        r32[i] = (float)ri;
    }
}

// Jacobi step x += omega (b - A x) / d (mode 0) or residual r = b - A x
// (mode 1) from the slots of A x
__global__ __launch_bounds__(256) void sym_smooth_kernel(SymPlan P, double* x, const double* b, const double* d,
                                                         double omega, int mode, double* r) {
    const long long i = (long long)blockIdx.x * (256 / P.G) + threadIdx.x / P.G;
    const int g = threadIdx.x & (P.G - 1);
    const double s = group_sum(sym_gather_share(P, i, g), P.G);
    if (g == 0 && i < P.n) {
        if (mode == 0) x[i] += omega * (b[i] - s) / d[i];
        else r[i] = b[i] - s;
    }
}

void sym_plan_geometry(long long n, SymPlan* P) {
    P->n = n;
    P->nb = (int)((n + SYM_TB - 1) / SYM_TB);
    // block columns per workgroup: up to SYM_M while the triangle still holds
    // about 2048 workgroups (the chip stays filled), at least 3 (the fixed
    // cost of a workgroup is spread over several tiles); block rows: doubled
    // up to SYM_R while about 2048 workgroups remain.  Each doubling of R
    // halves the column slots an element sums (one per workgroup row above
    // it instead of one per tile); on the 1e5-DOF disk (R = 16) a CG
    // iteration took 6% less time than with R = 4, 3% less than with R = 8
    // and 0.7% less than with R = 32
    const long long tiles = (long long)P->nb * (P->nb + 1) / 2;
    P->m = (int)std::max<long long>(3, std::min<long long>(SYM_M, tiles / 2048));
    P->R = 1;
    while (P->R < SYM_R && tiles / ((long long)P->m * 2 * P->R) >= 2048) P->R *= 2;
    P->nJ = (P->nb + P->m - 1) / P->m;
    P->nI = (P->nb + P->R - 1) / P->R;
    P->nwg = (long long)P->nJ * P->nI;
    // large systems: CG scalars by a one-workgroup kernel, and 4 lanes per
    // element in the reductions (a load instruction then reads 4 runs of 16
    // consecutive entries of the slot arrays, 128 B each); otherwise every
    // workgroup of the product reduces the partials itself and their count
    // stays below 1024
    P->sk = n > SYM_SK_N ? 1 : 0;
    int G = P->sk ? 4 : 16;
    if (!P->sk)
        while (G > 1 && (n * G + 255) / 256 > 1024) G >>= 1;
    P->G = G;
    P->nred = (int)std::max<long long>(1, (n * G + 255) / 256);
}

size_t sym_plan_doubles(const SymPlan& P) {
    return (size_t)(P.nJ + P.nI) * (size_t)P.n + (size_t)P.nwg + SYM_PQ_BLOCKS + 8;
}

void sym_plan_bind(SymPlan* P, double* buf) {
    P->prow = buf;
    P->pcol = buf + (long long)P->nJ * P->n;
    P->wpart = buf + (long long)(P->nJ + P->nI) * P->n;
    P->wpart2 = P->wpart + P->nwg;
    // many workgroups: one pre-reduction pass so that every block of the
    // update sums SYM_PQ_BLOCKS partials instead of nwg
    P->pre = P->nwg > 8192;
    P->pq = P->pre ? P->wpart2 : P->wpart;
    P->npq = P->pre ? SYM_PQ_BLOCKS : (int)P->nwg;
}

// wpart (nwg) -> wpart2 (SYM_PQ_BLOCKS), fixed assignment
__global__ __launch_bounds__(256) void sym_pq_reduce_kernel(SymPlan P) {
    __shared__ double sh[12];
    double s = 0.0, u1 = 0.0, u2 = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < P.nwg; i += (long long)SYM_PQ_BLOCKS * 256)
        s += P.wpart[i];
    block_sum3(s, u1, u2, sh);
    if (threadIdx.x == 0) P.wpart2[blockIdx.x] = s;
}

void launch_sym_pq_reduce(const SymPlan& P, hipStream_t st) {
    if (P.pre) hipLaunchKernelGGL(sym_pq_reduce_kernel, dim3(SYM_PQ_BLOCKS), dim3(256), 0, st, P);
}

template <class T>
void symv_launch(const SymPlan& P, const T* A, long long lda, const T* x, hipStream_t st) {
    hipLaunchKernelGGL(symv_kernel<T>, dim3(P.nJ, P.nI), dim3(256), 0, st, A, lda, P, x);
}

void launch_symv(const SymPlan& P, const double* A, long long lda, const double* x, double* y, hipStream_t st) {
    if (P.n == 0) return;
    symv_launch(P, A, lda, x, st);
    hipLaunchKernelGGL(sym_reduce_kernel, dim3(P.nred), dim3(256), 0, st, P, y);
}

void launch_sym_smooth(const SymPlan& P, const double* A, long long lda, double* x, const double* b,
                       const double* d, double omega, int mode, double* r, hipStream_t st) {
    if (P.n == 0) return;
    symv_launch(P, A, lda, (const double*)x, st);
    hipLaunchKernelGGL(sym_smooth_kernel, dim3(P.nred), dim3(256), 0, st, P, x, b, d, omega, mode, r);
}

void launch_residual(const SymPlan& P, const double* A, long long lda, const double* x, const double* b,
                     double* r, float* r32, hipStream_t st) {
    if (P.n == 0) return;
    symv_launch(P, A, lda, x, st);
    hipLaunchKernelGGL(sym_residual_kernel, dim3(P.nred), dim3(256), 0, st, P, b, r, r32);
}

// Jacobi-PCG (Sec. 5), two kernels per iteration, for the FP64 state
// (CgState) and the FP32 one (CgState32: FP32 matrix and vectors, products
// and dot products accumulated in FP64).  Partial sums are kept per block
// and reduced in a fixed order by every block that needs them
// (deterministic); r.z and r.r partials are double-buffered by iteration
// parity, the search direction p too.
//   cg_symv(it):    check ||r_it|| against rtol ||b||; beta = rz_it/rz_{it-1};
//                   p_it = z + beta p_{it-1} (computed on the fly for the
//                   product, stored by the workgroup holding the diagonal
//                   tile); slots of A p_it and workgroup partials of
//                   p_it.A p_it
//   cg_update(it):  alpha = rz_it / p.Ap; q = A p from the slots;
//                   x += alpha p; r -= alpha q; z = r/d; partials of r.z
//                   and r.r for iteration it+1
// The update and the initialisation run G = sp.G lanes per element (nblk =
// sp.nred blocks).  status: flag[0] stop, flag[1] iterations done, flag[2]
// 1 breakdown / 2 non-finite; scal[0] = b.b, scal[1] = last r.r.
template <class ST>
using cg_elem_t = std::remove_const_t<std::remove_pointer_t<decltype(ST::b)>>;

template <class ST>
__global__ __launch_bounds__(256) void cg_init_kernel(ST S) {
    using T = cg_elem_t<ST>;
    __shared__ double sh[12];
    const long long i = (long long)blockIdx.x * (256 / S.sp.G) + threadIdx.x / S.sp.G;
    const bool lead = (threadIdx.x & (S.sp.G - 1)) == 0;
    double rz = 0.0, rr = 0.0, unused = 0.0;
    if (lead && i < S.n) {
        const T bi = S.b[i];
        S.x[i] = T(0);
        S.r[i] = bi;
        const T zi = bi / S.d[i];
        S.z[i] = zi;
        S.p[S.n + i] = T(0);  // p_{-1}
        rz = (double)bi * zi;
        rr = (double)bi * bi;
    }
    block_sum3(rz, rr, unused, sh);
    if (threadIdx.x == 0) {
        S.part[blockIdx.x] = rz;              // rz, parity 0
        S.part[2 * S.nblk + blockIdx.x] = rr; // rr, parity 0
    }
}

template <class ST>
__global__ __launch_bounds__(256) void cg_init_reduce_kernel(ST S) {
    __shared__ double sh[12];
    double bb = load_partials(S.part + 2 * S.nblk, S.nblk), rz = load_partials(S.part, S.nblk), u2 = 0.0;
    block_sum3(bb, rz, u2, sh);
    if (threadIdx.x == 0) {
        S.scal[0] = bb;
        S.scal[1] = bb;
        S.flag[0] = (bb == 0.0) ? 1 : 0;
        S.flag[1] = 0;
        S.flag[2] = 0;
        if (!(bb == bb) || bb > 1.79e308) { S.flag[0] = 1; S.flag[2] = 2; }
        if (S.sp.sk) {
            // the scalar kernel's state for iteration 0 and its stop test
            S.scal[2] = 0.0;
            S.scal[3] = rz;
            S.hist[0] = bb;
            if (!S.flag[0] && (sqrt(bb) <= S.rtol * sqrt(bb) || S.maxit <= 0)) S.flag[0] = 1;
        }
    }
}

// Large systems: after cg_update(it), one workgroup reduces the r.z and r.r
// partials of iteration it + 1 (fixed order), records r.r, applies the stop
// test and leaves beta_{it+1} = rz_{it+1} / rz_it and rz_{it+1} for the
// next cg_symv and cg_update, which then read two scalars instead of
// reducing the partials in every workgroup.
template <class ST>
__global__ __launch_bounds__(256) void cg_scalar_kernel(ST S, int it) {
    __shared__ double sh[12];
    if (*(volatile int*)&S.flag[0]) return;
    const int par1 = (it + 1) & 1;
    double rz = load_partials(S.part + par1 * S.nblk, S.nblk);
    double rr = load_partials(S.part + 2 * S.nblk + par1 * S.nblk, S.nblk), u = 0.0;
    block_sum3(rz, rr, u, sh);
    if (threadIdx.x == 0) {
        S.hist[(it + 1) & 63] = rr;
        const double bb = S.scal[0];
        if (sqrt(rr) <= S.rtol * sqrt(bb) || it + 1 >= S.maxit || !(rr == rr)) {
            S.flag[0] = 1;
            S.flag[1] = it + 1;
            S.scal[1] = rr;
            if (!(rr == rr)) S.flag[2] = 2;
        } else {
            S.scal[2] = rz / S.scal[3];
            S.scal[3] = rz;
        }
    }
}

template <class ST>
__global__ __launch_bounds__(256) void cg_symv_kernel(ST S, int it) {
    using T = cg_elem_t<ST>;
    __shared__ double sh[12];
    __shared__ double red[256];
    __shared__ double cacc[SYM_M * SYM_TB];
    const SymPlan& P = S.sp;
    const int I = blockIdx.y, J = blockIdx.x, t = threadIdx.x;
    const long long wg = (long long)I * gridDim.x + J;
    if (!sym_group_live(P, I, J)) {  // below the diagonal: an empty partial
        if (t == 0) P.wpart[wg] = 0.0;
        return;
    }
    const long long n = S.n;
    const int par = it & 1;
    const T* pprev = S.p + (long long)(1 - par) * n;
    T* pcur = S.p + (long long)par * n;
    double beta64;
    if (P.sk) {
        // stop test and beta from the scalar kernel of the last iteration
        if (*(volatile int*)&S.flag[0]) return;
        beta64 = it > 0 ? S.scal[2] : 0.0;
    } else {
        double rz = load_partials(S.part + par * S.nblk, S.nblk);
        double rr = load_partials(S.part + 2 * S.nblk + par * S.nblk, S.nblk);
        double rzp = it > 0 ? load_partials(S.part + (1 - par) * S.nblk, S.nblk) : 0.0;
        if (*(volatile int*)&S.flag[0]) return;
        block_sum3(rz, rr, rzp, sh);
        if (I == 0 && J == 0 && t == 0) S.hist[it & 63] = rr;
        const double bb = S.scal[0];
        if (sqrt(rr) <= S.rtol * sqrt(bb) || it >= S.maxit || !(rr == rr)) {
            if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
                S.flag[0] = 1;
                S.flag[1] = it;
                S.scal[1] = rr;
                if (!(rr == rr)) S.flag[2] = 2;
            }
            return;
        }
        beta64 = it > 0 ? rz / rzp : 0.0;
    }
    const T beta = (T)beta64;
    // p_it = z + beta p_{it-1}, formed where the product needs it; the
    // workgroup holding a block row's diagonal tile stores it
    double vd = sym_group_any<T>(S.A, S.lda, P, I, J, SymVecP<T>{S.z, pprev, beta}, red, cacc), u1 = 0.0,
           u2 = 0.0;
    for (int r = 0; r < P.R; ++r) {
        const int bi = I * P.R + r;
        const long long i = (long long)bi * SYM_TB + t;
        const bool diag = P.R == 1 ? J == 0 : (bi >= J * P.m && bi < J * P.m + P.m);
        if (bi < P.nb && diag && t < SYM_TB && i < n)
            pcur[i] = S.z[i] + beta * pprev[i];
    }
    block_sum3(vd, u1, u2, sh);
    if (t == 0) P.wpart[wg] = vd;
}

template <class ST>
__global__ __launch_bounds__(256) void cg_update_kernel(ST S, int it) {
    using T = cg_elem_t<ST>;
    __shared__ double sh[12];
    const SymPlan& P = S.sp;
    const int par = it & 1;
    const long long n = S.n;
    const long long i = (long long)blockIdx.x * (256 / P.G) + threadIdx.x / P.G;
    const int g = threadIdx.x & (P.G - 1);
    const bool own = g == 0 && i < n;
    const T* pcur = S.p + (long long)par * n;
    // every load first: partials, slots of A p, the element's vectors
    double pq = load_partials(P.pq, P.npq);
    double rz = P.sk ? 0.0 : load_partials(S.part + par * S.nblk, S.nblk);
    double q = sym_gather_share(P, i, g);
    T pi = T(0), xi = T(0), ri = T(0), di = T(1);
    if (own) {
        pi = pcur[i];
        xi = S.x[i];
        ri = S.r[i];
        di = S.d[i];
    }
    if (*(volatile int*)&S.flag[0]) return;
    double u = 0.0;
    block_sum3(pq, rz, u, sh);
    if (P.sk) rz = S.scal[3];
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S.flag[0] = 1;
            S.flag[1] = it;
            S.flag[2] = 1;
        }
        return;
    }
    q = group_sum(q, P.G);
    const T alpha = (T)(rz / pq);
    double a = 0.0, b = 0.0;
    if (own) {
        S.x[i] = xi + alpha * pi;
        const T rn = ri - alpha * (T)q;
        S.r[i] = rn;
        const T zi = rn / di;
        S.z[i] = zi;
        a = (double)rn * zi;
        b = (double)rn * rn;
    }
    u = 0.0;
    block_sum3(a, b, u, sh);
    if (threadIdx.x == 0) {
        S.part[(1 - par) * S.nblk + blockIdx.x] = a;
        S.part[2 * S.nblk + (1 - par) * S.nblk + blockIdx.x] = b;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) S.flag[1] = it + 1;
}

// after the last launched iteration: residual of iteration `it`
template <class ST>
__global__ __launch_bounds__(256) void cg_final_kernel(ST S, int it) {
    __shared__ double sh[12];
    double rr = load_partials(S.part + 2 * S.nblk + (it & 1) * S.nblk, S.nblk), u1 = 0.0, u2 = 0.0;
    block_sum3(rr, u1, u2, sh);
    if (threadIdx.x == 0 && !S.flag[0]) S.scal[1] = rr;
}

// Residual replacement for iteration it of a running CG (the FP32 inner
// solve of the mixed-precision path): the correction x restarts from zero,
// the recursive residual is replaced by S.b (the true residual, computed in
// FP64 by the caller and rounded), z = r / d, and the r.z, r.r partials of
// iteration it are rewritten; p_{it-1} is kept, so the next iteration
// continues the same sequence of search directions (beta from the new r.z
// and the last one) instead of restarting.
template <class ST>
__global__ __launch_bounds__(256) void cg_replace_kernel(ST S, int it) {
    using T = cg_elem_t<ST>;
    __shared__ double sh[12];
    const long long i = (long long)blockIdx.x * (256 / S.sp.G) + threadIdx.x / S.sp.G;
    const bool lead = (threadIdx.x & (S.sp.G - 1)) == 0;
    double rz = 0.0, rr = 0.0, unused = 0.0;
    if (lead && i < S.n) {
        const T ri = S.b[i];
        S.x[i] = T(0);
        S.r[i] = ri;
        const T zi = ri / S.d[i];
        S.z[i] = zi;
        rz = (double)ri * zi;
        rr = (double)ri * ri;
    }
    block_sum3(rz, rr, unused, sh);
    const int par = it & 1;
    if (threadIdx.x == 0) {
        S.part[par * S.nblk + blockIdx.x] = rz;
        S.part[2 * S.nblk + par * S.nblk + blockIdx.x] = rr;
    }
}

// after cg_replace: the new reference norm (the stop test of the segment
// compares with it) and, for the scalar-kernel mode, beta_it and rz_it;
// clears the stop flag (flag[1] keeps the iteration count)
template <class ST>
__global__ __launch_bounds__(256) void cg_replace_reduce_kernel(ST S, int it) {
    __shared__ double sh[12];
    const int par = it & 1;
    double rr = load_partials(S.part + 2 * S.nblk + par * S.nblk, S.nblk);
    double rz = load_partials(S.part + par * S.nblk, S.nblk), u = 0.0;
    block_sum3(rr, rz, u, sh);
    if (threadIdx.x == 0) {
        S.scal[0] = rr;
        S.scal[1] = rr;
        S.flag[0] = 0;
        S.flag[2] = 0;
        if (S.sp.sk) {
            S.hist[it & 63] = rr;
            S.scal[2] = it > 0 ? rz / S.scal[3] : 0.0;
            S.scal[3] = rz;
        }
    }
}

template <class ST>
void cg_init_launch(const ST& s, hipStream_t st) {
    hipLaunchKernelGGL(cg_init_kernel<ST>, dim3(s.nblk), dim3(256), 0, st, s);
    hipLaunchKernelGGL(cg_init_reduce_kernel<ST>, dim3(1), dim3(256), 0, st, s);
}

template <class ST>
void cg_iter_launch(const ST& s, int it, hipStream_t st) {
    hipLaunchKernelGGL(cg_symv_kernel<ST>, dim3(s.sp.nJ, s.sp.nI), dim3(256), 0, st, s, it);
    launch_sym_pq_reduce(s.sp, st);
    hipLaunchKernelGGL(cg_update_kernel<ST>, dim3(s.nblk), dim3(256), 0, st, s, it);
    if (s.sp.sk) hipLaunchKernelGGL(cg_scalar_kernel<ST>, dim3(1), dim3(256), 0, st, s, it);
}

template <class ST>
void cg_final_launch(const ST& s, int it, hipStream_t st) {
    hipLaunchKernelGGL(cg_final_kernel<ST>, dim3(1), dim3(256), 0, st, s, it);
}

void launch_cg_init(const CgState& s, hipStream_t st) { cg_init_launch(s, st); }
void launch_cg_iter_at(const CgState& s, int it, hipStream_t st) { cg_iter_launch(s, it, st); }
void launch_cg_final(const CgState& s, int it, hipStream_t st) { cg_final_launch(s, it, st); }
void launch_cg32_init(const CgState32& s, hipStream_t st) { cg_init_launch(s, st); }
void launch_cg32_iter_at(const CgState32& s, int it, hipStream_t st) { cg_iter_launch(s, it, st); }
void launch_cg32_final(const CgState32& s, int it, hipStream_t st) { cg_final_launch(s, it, st); }
void launch_cg32_replace(const CgState32& s, int it, hipStream_t st) {
    hipLaunchKernelGGL(cg_replace_kernel<CgState32>, dim3(s.nblk), dim3(256), 0, st, s, it);
    hipLaunchKernelGGL(cg_replace_reduce_kernel<CgState32>, dim3(1), dim3(256), 0, st, s, it);
}

// out[0] = a.b, out[1] = a.c (deterministic two-pass)
__global__ __launch_bounds__(256) void dot2_kernel(const double* a, const double* b, const double* c,
                                                   long long n, double* part, int nblk) {
    __shared__ double sh[4];
    double s1 = 0.0, s2 = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)nblk * 256) {
        s1 += a[i] * b[i];
        s2 += a[i] * c[i];
    }
    double t1 = block_sum(s1, sh), t2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t1;
        part[nblk + blockIdx.x] = t2;
    }
}

__global__ __launch_bounds__(256) void dot2_reduce_kernel(const double* part, int nblk, double* out) {
    __shared__ double sh[4];
    double t1 = sum_partials(part, nblk, sh);
    double t2 = sum_partials(part + nblk, nblk, sh);
    if (threadIdx.x == 0) { out[0] = t1; out[1] = t2; }
}

void launch_dot2(const double* a, const double* b, const double* c, long long n, double* part,
                 int nblk, double* out, hipStream_t st) {
    hipLaunchKernelGGL(dot2_kernel, dim3(nblk), dim3(256), 0, st, a, b, c, n, part, nblk);
    hipLaunchKernelGGL(dot2_reduce_kernel, dim3(1), dim3(256), 0, st, part, nblk, out);
}

// ------------------------------------------------ mixed precision --

// The FP32 copy drives only the symmetric product, which reads the 64 x 64
// tiles on and above the diagonal: row i is converted from the first column
// of its block (64 floor(i / 64)) to n - 1, about half the matrix.  One
// workgroup per row at a time, two entries per thread and step (16-byte
// reads, 8-byte writes; lda is a multiple of 32, so the pairs are aligned).
__global__ __launch_bounds__(256) void to_f32_kernel(const double* A, long long lda, long long n, float* A32) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    for (long long i = blockIdx.x; i < n; i += gridDim.x) {
        const long long j0 = (i / SYM_TB) * SYM_TB;
        const double* a = A + i * lda;
        float* b = A32 + i * lda;
        for (long long j = j0 + 2 * (long long)threadIdx.x; j < n; j += 512) {
            if (j + 1 < n) {
                const d2 v = *(const d2*)(a + j);
                *(f2*)(b + j) = f2{(float)v.x, (float)v.y};
            } else {
                b[j] = (float)a[j];
            }
        }
    }
}

void launch_to_f32(const double* A, long long lda, long long n, float* A32, hipStream_t st) {
    if (n == 0) return;
    const long long blocks = n < 65536 ? n : 65536;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, lda, n, A32);
}

__global__ void diag32_kernel(const float* A, long long lda, long long n, float* d) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = A[i * lda + i];
}

void launch_diag32(const float* A, long long lda, long long n, float* d, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(diag32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, lda, n, d);
}


__global__ void add_correction_kernel(double* u, const float* e, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] += (double)e[i];
}

__global__ void cast_f32_kernel(const double* a, float* b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

void launch_cast_f32(const double* a, float* b, long long n, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(cast_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

void launch_add_correction(double* u, const float* e, long long n, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(add_correction_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, u, e, n);
}

}  // namespace fl
