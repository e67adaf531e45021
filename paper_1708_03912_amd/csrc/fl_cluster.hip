// Cluster (H-matrix) approximation of the stiffness matrix (Sec. 6):
// tensor Chebyshev interpolation of the kernel on admissible pairs of
// cluster boxes, nested bases through the shift coefficients, the near
// field as dense leaf blocks.  Set-up kernels (basis coefficients, shift
// coefficients, kernel blocks, near blocks) and the product (upward pass,
// far field, downward pass, leaves); the tree and the block lists come from
// fl_cluster_api.hip.  All FP64, fixed summation orders.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fl_internal.hpp"
#include "fl_math.hpp"

namespace fl {

namespace {

// Lagrange polynomial a of the m reference nodes t at xi (product over b != a
// in increasing b)
__device__ __forceinline__ double lag(const double* t, int m, int a, double xi) {
    double p = 1.0;
    for (int b = 0; b < m; ++b)
        if (b != a) p *= (xi - t[b]) / (t[a] - t[b]);
    return p;
}

// tensor Lagrange basis function a (first coordinate slowest) of cluster c
// at the point (x, y)
__device__ __forceinline__ double lag_box(const HDev& H, int c, int a, double x, double y) {
    const double* bx = H.box + 3 * c;
    if (H.dim == 1) return lag(H.tnode, H.m, a, (x - bx[0]) / bx[2]);
    const int a0 = a / H.m, a1 = a - a0 * H.m;
    return lag(H.tnode, H.m, a0, (x - bx[0]) / bx[2]) * lag(H.tnode, H.m, a1, (y - bx[1]) / bx[2]);
}

// Chebyshev point b of cluster c
__device__ __forceinline__ void cheb_pt(const HDev& H, int c, int b, double& x, double& y) {
    const double* bx = H.box + 3 * c;
    if (H.dim == 1) {
        x = bx[0] + bx[2] * H.tnode[b];
        y = 0.0;
        return;
    }
    const int b0 = b / H.m, b1 = b - b0 * H.m;
    x = bx[0] + bx[2] * H.tnode[b0];
    y = bx[1] + bx[2] * H.tnode[b1];
}

// V[r][a] = int phi_i L_a^leaf(r) over the cells around DOF i = perm[r], by
// the (m+1)-point rule of every cell.  One thread per (r, a).
__global__ __launch_bounds__(256) void h_basis_kernel(HDev H) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= H.n * H.M) return;
    const long long r = id / H.M;
    const int a = (int)(id - r * H.M);
    const int v = H.node[r];
    const int c = H.rleaf[r];
    const int nper = H.dim + 1;
    double acc = 0.0;
    for (int e = H.vptr[v]; e < H.vptr[v + 1]; ++e) {
        const int K = H.vidx[e];
        const int* cv = H.cells + (long long)K * nper;
        double P[3][2];
        int loc = 0;
        for (int b = 0; b < nper; ++b) {
            P[b][0] = H.verts[(long long)cv[b] * H.dim];
            P[b][1] = H.dim == 2 ? H.verts[(long long)cv[b] * H.dim + 1] : 0.0;
            if (cv[b] == v) loc = b;
        }
        double meas;
        if (H.dim == 1) {
            meas = fabs(P[1][0] - P[0][0]);
        } else {
            meas = 0.5 * fabs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]));
        }
        for (int q = 0; q < H.nq; ++q) {
            const double* l = H.qlam + q * nper;
            double x = 0.0, y = 0.0;
            for (int b = 0; b < nper; ++b) {
                x += l[b] * P[b][0];
                y += l[b] * P[b][1];
            }
            acc += (meas * H.qw[q] * l[loc]) * lag_box(H, c, a, x, y);
        }
    }
    H.V[id] = acc;
}

// V in 2D with MC points per direction known at compile time: one thread
// per r forms the whole row (MC^2 entries); at each quadrature point the 2 MC
// one-dimensional Lagrange values are formed once (by lag, with the nodes in
// registers) and their products taken: the same numbers and the same sums
// (cells, then points, in order) as h_basis_kernel.
template <int MC>
__global__ __launch_bounds__(256) void h_basis_row_kernel(HDev H) {
    constexpr int MM = MC * MC;
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= H.n) return;
    double t[MC];
#pragma unroll
    for (int k = 0; k < MC; ++k) t[k] = H.tnode[k];
    const int v = H.node[r];
    const double* bx = H.box + 3 * H.rleaf[r];
    const double bx0 = bx[0], bx1 = bx[1], bs = bx[2];
    double acc[MM];
#pragma unroll
    for (int a = 0; a < MM; ++a) acc[a] = 0.0;
    for (int e = H.vptr[v]; e < H.vptr[v + 1]; ++e) {
        const int K = H.vidx[e];
        const int* cv = H.cells + (long long)K * 3;
        double P[3][2];
        int loc = 0;
        for (int b = 0; b < 3; ++b) {
            P[b][0] = H.verts[(long long)cv[b] * 2];
            P[b][1] = H.verts[(long long)cv[b] * 2 + 1];
            if (cv[b] == v) loc = b;
        }
        const double meas = 0.5 * fabs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]));
        for (int q = 0; q < H.nq; ++q) {
            const double* l = H.qlam + q * 3;
            double x = 0.0, y = 0.0;
            for (int b = 0; b < 3; ++b) {
                x += l[b] * P[b][0];
                y += l[b] * P[b][1];
            }
            const double w = meas * H.qw[q] * l[loc];
            const double xi = (x - bx0) / bs, eta = (y - bx1) / bs;
            double l0[MC], l1[MC];
#pragma unroll
            for (int k = 0; k < MC; ++k) {
                l0[k] = lag(t, MC, k, xi);
                l1[k] = lag(t, MC, k, eta);
            }
#pragma unroll
            for (int a0 = 0; a0 < MC; ++a0)
#pragma unroll
                for (int a1 = 0; a1 < MC; ++a1) acc[a0 * MC + a1] += w * (l0[a0] * l1[a1]);
        }
    }
#pragma unroll
    for (int a = 0; a < MM; ++a) H.V[r * MM + a] = acc[a];
}

// T_c[b][a] = L_a^parent(xi_b^c), clusters c >= 1.  One thread per entry.
__global__ __launch_bounds__(256) void h_transfer_kernel(HDev H) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long MM = (long long)H.M * H.M;
    if (id >= (long long)H.nc * MM) return;
    const int c = (int)(id / MM);
    if (c == 0) return;
    const int rem = (int)(id - (long long)c * MM);
    const int b = rem / H.M, a = rem - b * H.M;
    double x, y;
    cheb_pt(H, c, b, x, y);
    const double v = lag_box(H, H.cpar[c], a, x, y);
    H.T[id] = v;
    H.Tt[(long long)c * MM + (long long)a * H.M + b] = v;
}

// Kernel blocks of the admissible pairs, stored column by column:
// Kb[p][b][a] = k(xi_a^sigma, xi_b^tau).  One thread per entry.
__global__ __launch_bounds__(256) void h_kblock_kernel(HDev H, double pe) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long MM = (long long)H.M * H.M;
    if (id >= H.nfar * MM) return;
    const long long p = id / MM;
    const int rem = (int)(id - p * MM);
    const int b = rem / H.M, a = rem - b * H.M;
    double xs, ys, xt, yt;
    cheb_pt(H, H.fsrc[p], a, xs, ys);
    cheb_pt(H, H.fdst[p], b, xt, yt);
    const double dx = xs - xt, dy = ys - yt;
    H.Kb[id] = kpow(dx * dx + dy * dy, pe);
}

// Near blocks copied from the dense matrix (column by column per block,
// tree order).
__global__ __launch_bounds__(256) void h_near_kernel(HDev H, const double* __restrict__ A, long long lda) {
    for (long long p = blockIdx.y; p < H.nnear; p += gridDim.y) {
        const int s = H.nsrc[p], t = H.ndst[p];
        const int rs = H.clo[s], ns = H.chi[s] - rs, rt = H.clo[t], nt = H.chi[t] - rt;
        for (int id = threadIdx.x + blockIdx.x * blockDim.x; id < ns * nt; id += blockDim.x * gridDim.x) {
            const int j = id / ns, i = id - j * ns;
            H.An[H.noff[p] + id] = A[(long long)H.perm[rs + i] * lda + H.perm[rt + j]];
        }
    }
}

// ---------------------------------------------------------------- product

// xp[r] = x[perm[r]]
__global__ __launch_bounds__(256) void h_gather_kernel(HDev H, const double* __restrict__ x) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < H.n) H.xp[r] = x[H.perm[r]];
}

// leaves: xh[c][a] = sum_r V[r][a] xp[r] (r in increasing order); one
// workgroup per leaf, eight rows' loads in flight
__global__ __launch_bounds__(64) void h_up_leaf_kernel(HDev H) {
    const int c = H.leaf[blockIdx.x];
    const int M = H.M, hi = H.chi[c];
    for (int a = threadIdx.x; a < M; a += blockDim.x) {
        double acc = 0.0;
        int r = H.clo[c];
        for (; r + 8 <= hi; r += 8) {
            double v[8], x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                v[j] = H.V[(long long)(r + j) * M + a];
                x[j] = H.xp[r + j];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) acc = fma(v[j], x[j], acc);
        }
        for (; r < hi; ++r) acc = fma(H.V[(long long)r * M + a], H.xp[r], acc);
        H.xh[(long long)c * M + a] = acc;
    }
}

// lane l's value of v, broadcast through two scalar registers (l uniform)
__device__ __forceinline__ double lane_bcast(double v, int l) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// internal clusters of one level: xh[c][a] = sum_sons sum_b T_son[b][a] xh[son][b]
// (son 0 first, b increasing).  M <= MB <= 64: lane a loads its column of
// both sons' shift coefficients into registers (for each b the lanes read
// one contiguous row; every load issued before the first is used) and the
// sons' coefficients are broadcast from the lanes that hold them; no LDS.
// Larger M: one lane per output reads its column directly.
template <int MB, bool EX>
__global__ __launch_bounds__(64) void h_up_kernel(HDev H, const int4* __restrict__ list) {
    const int4 e = list[blockIdx.x];  // {c, son 0, son 1, -}
    const int c = e.x, M = EX ? MB : H.M, MM = M * M;
    if (M <= MB) {
        const int a = threadIdx.x, ac = min(a, M - 1);
        const double* T0 = H.T + (long long)e.y * MM + ac;
        const double* T1 = H.T + (long long)e.z * MM + ac;
        // rows b >= M are loaded clamped and zeroed: their terms add exact zeros
        const double x0 = H.xh[(long long)e.y * M + ac];
        const double x1 = H.xh[(long long)e.z * M + ac];
        double t0[MB], t1[MB];
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            const int bc = min(b, M - 1);
            const double u0 = T0[bc * M], u1 = T1[bc * M];
            t0[b] = b < M ? u0 : 0.0;
            t1[b] = b < M ? u1 : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the products
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < MB; ++b) acc = fma(t0[b], lane_bcast(x0, b), acc);
#pragma unroll
        for (int b = 0; b < MB; ++b) acc = fma(t1[b], lane_bcast(x1, b), acc);
        if (a < M) H.xh[(long long)c * M + a] = acc;
        return;
    }
    for (int a = threadIdx.x; a < M; a += blockDim.x) {
        double acc = 0.0;
        for (int sn : {e.y, e.z}) {
            const double* Ts = H.T + (long long)sn * MM;
            const double* xs = H.xh + (long long)sn * M;
            for (int b = 0; b < M; ++b) acc = fma(Ts[b * M + a], xs[b], acc);
        }
        H.xh[(long long)c * M + a] = acc;
    }
}

// far field: yh[s][a] = sum over admissible (s, t) of sum_b K[a][b] xh[t][b];
// one workgroup per cluster, four groups of 64 lanes take every fourth pair
// (pairs in increasing order, b increasing within a pair), their partial
// sums are added in group order.  M <= MB <= 64: per pair, lane a loads its
// block column (K[a][b] for every b; the lanes of a wave read consecutive
// entries) and the partner's cluster vector, every load issued before the
// first product; the partner index of the next pair is fetched with them,
// so a pair waits for one memory latency; the cluster vector is broadcast
// from the lanes that hold it.  Larger M: 16 loads of the block column in
// flight before their products.
template <int MB, typename KT>
__device__ __forceinline__ void far_fetch(const HDev& H, const KT* __restrict__ Kb, int M, long long p, int t, int ac,
                                          double (&k)[MB], double& x) {
    const KT* Kp = Kb + p * M * M + ac;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const double u = Kp[min(b, M - 1) * M];
        k[b] = b < M ? u : 0.0;  // rows b >= M add exact zeros
    }
    x = H.xh[(long long)t * M + ac];
    __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the products that follow
}

template <int MB, bool EX, typename KT>
__device__ __forceinline__ void far_body(const HDev& H, const KT* __restrict__ Kb) {
    __shared__ double red[4][64];
    const int c = blockIdx.x;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int M = EX ? MB : H.M;
    if (M <= MB) {
        const int ac = min(lane, M - 1);
        const long long pb = H.fptr[c] + g, pe = H.fptr[c + 1];
        double acc = 0.0;
        if (pb < pe) {
            double k[MB], x;
            int t = H.fdst[pb];
            for (long long p = pb; p < pe; p += 4) {
                const int tn = H.fdst[min(p + 4, pe - 1)];
                far_fetch<MB>(H, Kb, M, p, t, ac, k, x);
#pragma unroll
                for (int b = 0; b < MB; ++b) acc = fma(k[b], lane_bcast(x, b), acc);
                t = tn;
            }
        }
        red[g][lane] = acc;
        __syncthreads();
        if (g == 0 && lane < M) H.yh[(long long)c * M + lane] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        return;
    }
    for (int a0 = 0; a0 < M; a0 += 64) {
        const int a = a0 + lane;
        double acc = 0.0;
        if (a < M) {
            // the sum keeps the order b = 0, 1, ...
            for (long long p = H.fptr[c] + g; p < H.fptr[c + 1]; p += 4) {
                const KT* Kp = Kb + p * M * M;
                const double* xt = H.xh + (long long)H.fdst[p] * M;
                int b = 0;
                for (; b + 16 <= M; b += 16) {
                    double kr[16], xr[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        kr[k] = Kp[(b + k) * M + a];
                        xr[k] = xt[b + k];
                    }
#pragma unroll
                    for (int k = 0; k < 16; ++k) acc = fma(kr[k], xr[k], acc);
                }
                for (; b < M; ++b) acc = fma(Kp[b * M + a], xt[b], acc);
            }
        }
        red[g][lane] = acc;
        __syncthreads();
        if (g == 0 && a < M) H.yh[(long long)c * M + a] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        __syncthreads();
    }
}

// the far field with the kernel blocks in FP64 or (FP32 representation) in
// FP32, products and sums in FP64
template <int MB, bool EX>
__global__ __launch_bounds__(256) void h_far_kernel(HDev H) {
    far_body<MB, EX, double>(H, H.Kb);
}
template <int MB, bool EX>
__global__ __launch_bounds__(256) void h_far32_kernel(HDev H) {
    far_body<MB, EX, float>(H, H.Kbf);
}

// clusters of one level (>= 1): yh[c][b] += sum_a T_c[b][a] yh[parent][a]
// (a increasing).  M <= MB <= 64: lane b loads row b of T_c from the
// transposed copy (for each a the lanes read one contiguous row of it) into
// registers and the parent's coefficients are broadcast; no LDS.  Larger M:
// one lane per output reads its row directly.
template <int MB, bool EX>
__global__ __launch_bounds__(64) void h_down_kernel(HDev H, const int4* __restrict__ list) {
    const int4 e = list[blockIdx.x];  // {c, parent, -, -}
    const int c = e.x, M = EX ? MB : H.M, MM = M * M;
    const double* yp = H.yh + (long long)e.y * M;
    if (M <= MB) {
        const int b = threadIdx.x, bc = min(b, M - 1);
        const double* Tc = H.Tt + (long long)c * MM + bc;
        const double yv = yp[bc];
        double t[MB];
#pragma unroll
        for (int a = 0; a < MB; ++a) {
            const double u = Tc[min(a, M - 1) * M];
            t[a] = a < M ? u : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the products
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < MB; ++a) acc = fma(t[a], lane_bcast(yv, a), acc);
        if (b < M) H.yh[(long long)c * M + b] += acc;
        return;
    }
    const double* Tc = H.T + (long long)c * MM;
    for (int b = threadIdx.x; b < M; b += blockDim.x) {
        double acc = 0.0;
        for (int a = 0; a < M; ++a) acc = fma(Tc[b * M + a], yp[a], acc);
        H.yh[(long long)c * M + b] += acc;
    }
}

// a pass kernel for M: M itself as a compile-time constant for the
// squares 4, 9, ..., 64 (2D with m = 2 to 8), else MB = the next of 4, 9,
// 16 above M (1D, and m = 1) or 64 (M > 64, 2D with m >= 9: the kernels
// take their direct form)
#define FL_MB_LAUNCH(KER, GRID, BLOCK, ...)                                              \
    do {                                                                                 \
        const dim3 g_((unsigned)(GRID)), b_(BLOCK);                                      \
        switch (H.M) {                                                                   \
            case 4: hipLaunchKernelGGL((KER<4, true>), g_, b_, 0, st, __VA_ARGS__); break;   \
            case 9: hipLaunchKernelGGL((KER<9, true>), g_, b_, 0, st, __VA_ARGS__); break;   \
            case 16: hipLaunchKernelGGL((KER<16, true>), g_, b_, 0, st, __VA_ARGS__); break; \
            case 25: hipLaunchKernelGGL((KER<25, true>), g_, b_, 0, st, __VA_ARGS__); break; \
            case 36: hipLaunchKernelGGL((KER<36, true>), g_, b_, 0, st, __VA_ARGS__); break; \
            case 49: hipLaunchKernelGGL((KER<49, true>), g_, b_, 0, st, __VA_ARGS__); break; \
            case 64: hipLaunchKernelGGL((KER<64, true>), g_, b_, 0, st, __VA_ARGS__); break; \
            default:                                                                     \
                if (H.M < 4)                                                             \
                    hipLaunchKernelGGL((KER<4, false>), g_, b_, 0, st, __VA_ARGS__);     \
                else if (H.M < 9)                                                        \
                    hipLaunchKernelGGL((KER<9, false>), g_, b_, 0, st, __VA_ARGS__);     \
                else if (H.M < 16)                                                       \
                    hipLaunchKernelGGL((KER<16, false>), g_, b_, 0, st, __VA_ARGS__);    \
                else                                                                     \
                    hipLaunchKernelGGL((KER<64, false>), g_, b_, 0, st, __VA_ARGS__);    \
        }                                                                                \
    } while (0)


// leaves: y[perm[r]] = -C sum_a V[r][a] yh[c][a] + sum over near (c, t) of
// the block row times xp[t]; one workgroup per leaf, eight groups of 32
// lanes take every eighth near block (column-major blocks: the lanes of a
// group read consecutive entries), group partials added in group order.
// Leaves of at most 32 DOFs: lane i loads its whole block row (every load
// issued before the first product) and the partner's x, broadcast within
// the group; the next block's range and offset are fetched with them, so a
// block waits for one memory latency; the row sum runs over the columns in
// order.  Larger leaves: rows in chunks of 32, four partial sums over the
// columns.
template <int MB, bool EX, typename KT>
__device__ __forceinline__ void leaf_body(const HDev& H, const KT* __restrict__ An, double C, double* __restrict__ y) {
    __shared__ double red[8][32];
    const int li = blockIdx.x;
    const int c = H.leaf[li];
    const int lo = H.clo[c], nr = H.chi[c] - lo;
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    const int M = EX ? MB : H.M;
    if (H.lmax <= 32 && M <= MB) {
        const int ic = min(lane, nr - 1);  // lanes >= nr repeat the last row and store nothing
        double acc = 0.0;
        if (g == 0) {
            // sum over a in order, every load issued before the first product
            const double* Vr = H.V + (long long)(lo + ic) * M;
            const double* yc = H.yh + (long long)c * M;
            double v[MB], w[MB];
#pragma unroll
            for (int a = 0; a < MB; ++a) {
                const int ac = min(a, M - 1);
                const double u = Vr[ac];
                v[a] = a < M ? u : 0.0;
                w[a] = yc[ac];
            }
            double f = 0.0;
#pragma unroll
            for (int a = 0; a < MB; ++a) f = fma(v[a], w[a], f);
            acc = -C * f;
        }
        const int eb = H.lnptr[li] + g, ee = H.lnptr[li + 1];
        if (eb < ee) {
            int2 rg = H.nrng[eb];
            long long off = H.noff[eb];
            for (int e = eb; e < ee; e += 8) {
                const int en = min(e + 8, ee - 1);
                const int2 rgn = H.nrng[en];
                const long long offn = H.noff[en];
                const KT* blk = An + off + ic;
                double b[32];
#pragma unroll
                for (int j = 0; j < 32; ++j) {
                    const double u = blk[(long long)min(j, rg.y - 1) * nr];
                    b[j] = j < rg.y ? u : 0.0;  // columns j >= nt add exact zeros
                }
                const double xv = H.xp[rg.x + min(lane, rg.y - 1)];
                __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the products
                double sr = 0.0;
#pragma unroll
                for (int j = 0; j < 32; ++j) sr = fma(b[j], __shfl(xv, j, 32), sr);
                acc += sr;
                rg = rgn;
                off = offn;
            }
        }
        red[g][lane] = acc;
        __syncthreads();
        if (g == 0 && lane < nr) {
            double tot = red[0][lane];
            for (int k = 1; k < 8; ++k) tot += red[k][lane];
            y[H.perm[lo + lane]] = tot;
        }
        return;
    }
    for (int r0 = 0; r0 < nr; r0 += 32) {
        const int i = r0 + lane;
        double acc = 0.0;
        if (i < nr) {
            if (g == 0) {
                const long long r = lo + i;
                double f = 0.0;
                for (int a = 0; a < M; ++a) f = fma(H.V[r * M + a], H.yh[(long long)c * M + a], f);
                acc = -C * f;
            }
            for (int e = H.lnptr[li] + g; e < H.lnptr[li + 1]; e += 8) {
                const int t = H.ndst[e];
                const int rt = H.clo[t], nt = H.chi[t] - rt;
                const KT* blk = An + H.noff[e] + i;
                const double* xt = H.xp + rt;
                // four partial sums over columns j mod 4: four loads in flight
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                int j = 0;
                for (; j + 4 <= nt; j += 4) {
                    const double b0 = blk[(long long)j * nr], b1 = blk[(long long)(j + 1) * nr];
                    const double b2 = blk[(long long)(j + 2) * nr], b3 = blk[(long long)(j + 3) * nr];
                    s0 = fma(b0, xt[j], s0);
                    s1 = fma(b1, xt[j + 1], s1);
                    s2 = fma(b2, xt[j + 2], s2);
                    s3 = fma(b3, xt[j + 3], s3);
                }
                for (; j < nt; ++j) s0 = fma(blk[(long long)j * nr], xt[j], s0);
                acc += (s0 + s1) + (s2 + s3);
            }
        }
        red[g][lane] = acc;
        __syncthreads();
        if (g == 0 && i < nr) {
            double tot = red[0][lane];
            for (int k = 1; k < 8; ++k) tot += red[k][lane];
            y[H.perm[lo + i]] = tot;
        }
        __syncthreads();
    }
}

// the leaves with the near blocks in FP64 or (FP32 representation) in FP32,
// products and sums in FP64
template <int MB, bool EX>
__global__ __launch_bounds__(256) void h_leaf_out_kernel(HDev H, double C, double* __restrict__ y) {
    leaf_body<MB, EX, double>(H, H.An, C, y);
}
template <int MB, bool EX>
__global__ __launch_bounds__(256) void h_leaf_out32_kernel(HDev H, double C, double* __restrict__ y) {
    leaf_body<MB, EX, float>(H, H.Anf, C, y);
}

// ------------------------------------------- far part of the self terms

// Leaf coefficients of the density 1 on the elements anchored in each leaf:
// xh[c][a] = sum over those elements K of int_K L_a^c, by the (m+1)-point
// rule.  One workgroup per leaf.
__global__ __launch_bounds__(64) void h_density_kernel(HDev H, ElemDev E, const int* __restrict__ lc_ptr,
                                                       const int* __restrict__ lc_idx) {
    const int li = blockIdx.x;
    const int c = H.leaf[li];
    const int nper = H.dim + 1;
    for (int a = threadIdx.x; a < H.M; a += blockDim.x) {
        double acc = 0.0;
        for (int e = lc_ptr[li]; e < lc_ptr[li + 1]; ++e) {
            const int K = lc_idx[e];
            double P[3][2];
            for (int b = 0; b < nper; ++b) {
                P[b][0] = E.x[H.dim * b][K];
                P[b][1] = H.dim == 2 ? E.x[H.dim * b + 1][K] : 0.0;
            }
            const double meas = E.meas[K];
            for (int q = 0; q < H.nq; ++q) {
                const double* l = H.qlam + q * nper;
                double x = 0.0, y = 0.0;
                for (int b = 0; b < nper; ++b) {
                    x += l[b] * P[b][0];
                    y += l[b] * P[b][1];
                }
                acc += (meas * H.qw[q]) * lag_box(H, c, a, x, y);
            }
        }
        H.xh[(long long)c * H.M + a] = acc;
    }
}

// The same in 2D with MC points per direction known at compile time: the
// leaf's quadrature points (elements in order, then points) in chunks of
// 64; lane p of a chunk forms point p's weight and its 2 MC one-dimensional
// Lagrange values in LDS, then lane a sums the chunk's terms in order --
// the same numbers and sums as h_density_kernel.
template <int MC>
__global__ __launch_bounds__(64) void h_density_tab_kernel(HDev H, ElemDev E, const int* __restrict__ lc_ptr,
                                                           const int* __restrict__ lc_idx) {
    constexpr int MM = MC * MC;
    __shared__ double Wp[64], L0[64][MC], L1[64][MC];
    const int li = blockIdx.x;
    const int c = H.leaf[li];
    const int tid = threadIdx.x, a0 = tid / MC, a1 = tid - a0 * MC;
    const int e0 = lc_ptr[li], nq = H.nq;
    const int np = (lc_ptr[li + 1] - e0) * nq;
    const double* bx = H.box + 3 * c;
    double acc = 0.0;
    for (int p0 = 0; p0 < np; p0 += 64) {
        const int p = p0 + tid;
        if (p < np) {
            const int e = p / nq, q = p - e * nq;
            const int K = lc_idx[e0 + e];
            double P[3][2];
            for (int b = 0; b < 3; ++b) {
                P[b][0] = E.x[2 * b][K];
                P[b][1] = E.x[2 * b + 1][K];
            }
            const double* l = H.qlam + q * 3;
            double x = 0.0, y = 0.0;
            for (int b = 0; b < 3; ++b) {
                x += l[b] * P[b][0];
                y += l[b] * P[b][1];
            }
            Wp[tid] = E.meas[K] * H.qw[q];
            const double xi = (x - bx[0]) / bx[2], eta = (y - bx[1]) / bx[2];
            for (int k = 0; k < MC; ++k) {
                L0[tid][k] = lag(H.tnode, MC, k, xi);
                L1[tid][k] = lag(H.tnode, MC, k, eta);
            }
        }
        __syncthreads();
        const int cnt = min(64, np - p0);
        if (tid < MM)
            for (int j = 0; j < cnt; ++j) acc += Wp[j] * (L0[j][a0] * L1[j][a1]);
        __syncthreads();
    }
    if (tid < MM) H.xh[(long long)c * MM + tid] = acc;
}

// S[K][ab] += C int_K l_a l_b g, g(x) = sum_a L_a^c(x) yh[c][a] (c: the leaf
// of K's anchor), by the (m+1)-point rule; one thread per element.  The
// tensor basis is evaluated as sum_a0 L_a0(x) sum_a1 L_a1(y) yh[a0 m + a1].
__global__ __launch_bounds__(256) void h_self_far_kernel(HDev H, ElemDev E, int T, const int* __restrict__ aleafc,
                                                        double C, double* __restrict__ S) {
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= T) return;
    const int c = aleafc[K];
    if (c < 0) return;
    const int nper = H.dim + 1, m = H.m;
    double P[3][2];
    for (int b = 0; b < nper; ++b) {
        P[b][0] = E.x[H.dim * b][K];
        P[b][1] = H.dim == 2 ? E.x[H.dim * b + 1][K] : 0.0;
    }
    const double meas = E.meas[K];
    const double* yh = H.yh + (long long)c * H.M;
    const double* bx = H.box + 3 * c;
    double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < H.nq; ++q) {
        const double* l = H.qlam + q * nper;
        double x = 0.0, y = 0.0;
        for (int b = 0; b < nper; ++b) {
            x += l[b] * P[b][0];
            y += l[b] * P[b][1];
        }
        const double xi = (x - bx[0]) / bx[2];
        double g = 0.0;
        if (H.dim == 1) {
            for (int a = 0; a < m; ++a) g += lag(H.tnode, m, a, xi) * yh[a];
        } else {
            const double eta = (y - bx[1]) / bx[2];
            double l1[15];
            for (int b = 0; b < m; ++b) l1[b] = lag(H.tnode, m, b, eta);
            for (int a = 0; a < m; ++a) {
                double t = 0.0;
                for (int b = 0; b < m; ++b) t += l1[b] * yh[a * m + b];
                g += lag(H.tnode, m, a, xi) * t;
            }
        }
        const double w = meas * H.qw[q] * g;
        for (int a = 0; a < nper; ++a)
            for (int b = a; b < nper; ++b) acc[a][b] += w * l[a] * l[b];
    }
    // packed symmetric 3 x 3: (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
    const int pk[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    for (int a = 0; a < nper; ++a)
        for (int b = a; b < nper; ++b) S[(long long)K * 6 + pk[a][b]] += C * acc[a][b];
}

inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

// leaf coefficients (unless leaf_done), upward pass (one launch per level,
// deepest first), far field, downward pass (one launch per level, shallowest
// first); the lists hold four ints per cluster (device allocations: 256-byte
// aligned)
void h_passes(const HDev& H, const int* const* up_lists, const int* up_counts, int n_up,
              const int* const* down_lists, const int* down_counts, int n_down, int leaf_done, hipStream_t st) {
    if (!leaf_done) hipLaunchKernelGGL(h_up_leaf_kernel, dim3((unsigned)H.nleaf), dim3(64), 0, st, H);
    for (int l = 0; l < n_up; ++l)
        if (up_counts[l] > 0) FL_MB_LAUNCH(h_up_kernel, up_counts[l], 64, H, (const int4*)up_lists[l]);
    if (H.Kbf)
        FL_MB_LAUNCH(h_far32_kernel, H.nc, 256, H);
    else
        FL_MB_LAUNCH(h_far_kernel, H.nc, 256, H);
    for (int l = 0; l < n_down; ++l)
        if (down_counts[l] > 0) FL_MB_LAUNCH(h_down_kernel, down_counts[l], 64, H, (const int4*)down_lists[l]);
}

}  // namespace

void launch_h_self_far(const HDev& H, const ElemDev& E, int T, const int* lc_ptr, const int* lc_idx,
                       const int* aleafc, const int* const* up_lists, const int* up_counts, int n_up,
                       const int* const* down_lists, const int* down_counts, int n_down, double C, double* S,
                       hipStream_t st) {
    if (H.n == 0 || T == 0) return;
    {
        const dim3 g((unsigned)H.nleaf), b(64);
        switch (H.dim == 2 ? H.M : 0) {
            case 4: hipLaunchKernelGGL(h_density_tab_kernel<2>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            case 9: hipLaunchKernelGGL(h_density_tab_kernel<3>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            case 16: hipLaunchKernelGGL(h_density_tab_kernel<4>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            case 25: hipLaunchKernelGGL(h_density_tab_kernel<5>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            case 36: hipLaunchKernelGGL(h_density_tab_kernel<6>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            case 49: hipLaunchKernelGGL(h_density_tab_kernel<7>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            case 64: hipLaunchKernelGGL(h_density_tab_kernel<8>, g, b, 0, st, H, E, lc_ptr, lc_idx); break;
            default: hipLaunchKernelGGL(h_density_kernel, g, b, 0, st, H, E, lc_ptr, lc_idx);
        }
    }
    h_passes(H, up_lists, up_counts, n_up, down_lists, down_counts, n_down, 1, st);
    hipLaunchKernelGGL(h_self_far_kernel, dim3(nb256(T)), dim3(256), 0, st, H, E, T, aleafc, C, S);
}

void launch_h_setup(const HDev& H, const double* A, long long lda, double pe, hipStream_t st) {
    if (H.n > 0) {
        const dim3 g(nb256(H.n)), b(256);
        switch (H.dim == 2 ? H.M : 0) {
            case 4: hipLaunchKernelGGL(h_basis_row_kernel<2>, g, b, 0, st, H); break;
            case 9: hipLaunchKernelGGL(h_basis_row_kernel<3>, g, b, 0, st, H); break;
            case 16: hipLaunchKernelGGL(h_basis_row_kernel<4>, g, b, 0, st, H); break;
            case 25: hipLaunchKernelGGL(h_basis_row_kernel<5>, g, b, 0, st, H); break;
            case 36: hipLaunchKernelGGL(h_basis_row_kernel<6>, g, b, 0, st, H); break;
            case 49: hipLaunchKernelGGL(h_basis_row_kernel<7>, g, b, 0, st, H); break;
            case 64: hipLaunchKernelGGL(h_basis_row_kernel<8>, g, b, 0, st, H); break;
            default: hipLaunchKernelGGL(h_basis_kernel, dim3(nb256(H.n * H.M)), b, 0, st, H);
        }
    }
    if (H.nc > 1)
        hipLaunchKernelGGL(h_transfer_kernel, dim3(nb256((long long)H.nc * H.M * H.M)), dim3(256), 0, st, H);
    if (H.nfar > 0)
        hipLaunchKernelGGL(h_kblock_kernel, dim3(nb256(H.nfar * H.M * H.M)), dim3(256), 0, st, H, pe);
    if (H.nnear > 0 && A)
        hipLaunchKernelGGL(h_near_kernel, dim3(4, (unsigned)(H.nnear < 32768 ? H.nnear : 32768)), dim3(256), 0, st,
                           H, A, lda);
}

void launch_h_matvec(const HDev& H, const int* const* up_lists, const int* up_counts, int n_up,
                     const int* const* down_lists, const int* down_counts, int n_down, double C, const double* x,
                     double* y, hipStream_t st) {
    if (H.n == 0) return;
    hipLaunchKernelGGL(h_gather_kernel, dim3(nb256(H.n)), dim3(256), 0, st, H, x);
    h_passes(H, up_lists, up_counts, n_up, down_lists, down_counts, n_down, 0, st);
    if (H.Anf)
        FL_MB_LAUNCH(h_leaf_out32_kernel, H.nleaf, 256, H, C, y);
    else
        FL_MB_LAUNCH(h_leaf_out_kernel, H.nleaf, 256, H, C, y);
}
#undef FL_MB_LAUNCH

}  // namespace fl

namespace fl {
namespace {
__global__ __launch_bounds__(256) void h_to_f32_kernel(const double* __restrict__ a, float* __restrict__ b,
                                                       long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}
}  // namespace

void launch_h_to_f32(const double* a, float* b, long long n, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(h_to_f32_kernel, dim3((unsigned)std::min<long long>((n + 255) / 256, 1 << 20)), dim3(256), 0,
                           st, a, b, n);
}

namespace {
__global__ __launch_bounds__(256) void h_diag_kernel(const double* __restrict__ A, long long lda, long long n,
                                                     double* __restrict__ d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = A[i * lda + i];
}
}  // namespace

void launch_h_diag(const double* A, long long lda, long long n, double* d, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(h_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, lda, n, d);
}
}  // namespace fl
