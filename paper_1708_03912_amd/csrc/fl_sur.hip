// Training, inference and certification kernels of the pair-integral
// surrogate (network and canonical form in fl_sur.hpp).  The forward and
// backward passes run on the FP16 matrix cores with FP32 accumulation;
// master weights, Adam moments and all reductions are FP32 / FP64.
#include <hip/hip_runtime.h>

#include "fl_internal.hpp"
#include "fl_sur.hpp"

namespace fl {

namespace {

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

constexpr int TS = 72;  // LDS row stride (halfs) of the [unit][sample] arrays
constexpr int XS = 40;  // LDS row stride (halfs) of the [sample][input] array

// FP16 copy of parameter p (biases stay FP32 in the master vector)
__device__ __forceinline__ void write_half_param(const SurHalves& H, int p, float v) {
    const _Float16 h = (_Float16)v;
    if (p < SUR_OB1) {
        H.W1[p] = h;
    } else if (p >= SUR_OW2 && p < SUR_OB2) {
        const int q = p - SUR_OW2, j = q / SUR_NH, k = q % SUR_NH;
        H.W2[q] = h;
        H.W2T[k * SUR_NH + j] = h;
    } else if (p >= SUR_OW3 && p < SUR_OB3) {
        const int q = p - SUR_OW3, j = q / SUR_NH, k = q % SUR_NH;
        H.W3[q] = h;
        H.W3T[k * SUR_KOUT + j] = h;
    }
}

}  // namespace

// One training step's forward + backward pass over 64 samples per
// workgroup (wave w: samples 16 w .. 16 w + 15).  Writes the workgroup's
// gradient of 1/2 sum_samples sum_outputs (out - y)^2 (standardised units)
// and its sum of squared errors.
__global__ __launch_bounds__(256) void sur_train_kernel(SurTrain A) {
    __shared__ __align__(16) _Float16 xs[64 * XS];
    __shared__ float yn[64 * 33];
    __shared__ int ok[64];
    __shared__ __align__(16) _Float16 XT[SUR_KIN * TS];
    __shared__ __align__(16) _Float16 H1T[SUR_NH * TS];
    __shared__ __align__(16) _Float16 H2T[SUR_NH * TS];
    __shared__ __align__(16) _Float16 D3T[SUR_KOUT * TS];
    __shared__ __align__(16) _Float16 G2T[SUR_NH * TS];
    __shared__ __align__(16) _Float16 G1T[SUR_NH * TS];
    __shared__ double lsum[4];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const SurNet& N = A.N;
    if (tid < 64) {
        long long idx;
        int valid = 1;
        if (A.mode == 0) {
            const unsigned long long key =
                splitmix64(A.seed ^ splitmix64((unsigned long long)(A.step * A.batch + blockIdx.x * 64 + tid)));
            idx = (long long)(key % (unsigned long long)A.m);
        } else {
            idx = A.base + (long long)blockIdx.x * 64 + tid;
            valid = idx < A.m;
            if (!valid) idx = 0;
        }
        ok[tid] = valid;
        float xn[SUR_NIN];
        sur_std_features(N, A.F + idx * SUR_NIN, xn);
        for (int k = 0; k < XS; ++k) xs[tid * XS + k] = (_Float16)(k < SUR_NIN && valid ? xn[k] : 0.f);
        for (int j = 0; j < 33; ++j) {
            float y = 0.f;
            if (j < SUR_NOUT && valid) y = (float)(A.T[idx * SUR_NOUT + j] - (double)N.mt[j]) / N.st[j];
            yn[tid * 33 + j] = y;
        }
    }
    __syncthreads();

    // forward, 16 samples per wave
    const int sr = 16 * wave + r;  // this lane's sample in the workgroup
    const h8 xb = *(const h8*)(xs + sr * XS + 8 * g);
    SurAct a;
    sur_forward16(N, xb, a);
    f4 d3[2];
    float l2 = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int u = 16 * t + 4 * g + v;
            const float d = ok[sr] && u < SUR_NOUT ? a.out[t][v] - yn[sr * 33 + u] : 0.f;
            d3[t][v] = d;
            l2 += d * d;
        }
    // backward: g_h2^T = W3^T d3^T (K = 32 outputs), g_h1^T = W2^T g_z2^T
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    h4 gz2[4], gz1[4];
    const h8 db = sur_cat(sur_h4(d3[0]), sur_h4(d3[1]));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const _Float16* wr = A.W3T + (16 * t + r) * SUR_KOUT + 4 * g;
        const f4 gh = sur_mma(sur_cat(*(const h4*)wr, *(const h4*)(wr + 16)), db, zero);
        f4 gz;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float h = (float)a.h2[t][v];
            gz[v] = gh[v] * (1.f - h * h);
        }
        gz2[t] = sur_h4(gz);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f4 gh = zero;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const _Float16* wr = A.W2T + (16 * t + r) * SUR_NH + 32 * c + 4 * g;
            gh = sur_mma(sur_cat(*(const h4*)wr, *(const h4*)(wr + 16)), sur_cat(gz2[2 * c], gz2[2 * c + 1]), gh);
        }
        f4 gz;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float h = (float)a.h1[t][v];
            gz[v] = gh[v] * (1.f - h * h);
        }
        gz1[t] = sur_h4(gz);
    }
    // transposed copies [unit][sample] for the weight-gradient products
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int u = 16 * t + 4 * g + v;
            H1T[u * TS + sr] = a.h1[t][v];
            H2T[u * TS + sr] = a.h2[t][v];
            G2T[u * TS + sr] = gz2[t][v];
            G1T[u * TS + sr] = gz1[t][v];
        }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) D3T[(16 * t + 4 * g + v) * TS + sr] = (_Float16)d3[t][v];
    for (int i = tid; i < SUR_KIN * 64; i += 256) {
        const int k = i / 64, b = i % 64;
        XT[k * TS + b] = xs[b * XS + k];
    }
    // squared error of the workgroup
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) l2 += __shfl_xor(l2, m, 64);
    if (lane == 0) lsum[wave] = l2;
    __syncthreads();

    // weight gradients dW[j][k] = sum_b G[b][j] In[b][k]: 32 tiles of 16x16
    float* out = A.part + (long long)blockIdx.x * SUR_NPARAM;
    for (int tile = wave; tile < 32; tile += 4) {
        const _Float16 *GT, *IT;
        int j0, k0, off, ncol;
        if (tile < 8) {            // W1: 4 x 2 tiles
            GT = G1T; IT = XT; j0 = 16 * (tile >> 1); k0 = 16 * (tile & 1); off = SUR_OW1; ncol = SUR_KIN;
        } else if (tile < 24) {    // W2: 4 x 4 tiles
            const int q = tile - 8;
            GT = G2T; IT = H1T; j0 = 16 * (q >> 2); k0 = 16 * (q & 3); off = SUR_OW2; ncol = SUR_NH;
        } else {                   // W3: 2 x 4 tiles
            const int q = tile - 24;
            GT = D3T; IT = H2T; j0 = 16 * (q >> 2); k0 = 16 * (q & 3); off = SUR_OW3; ncol = SUR_NH;
        }
        f4 acc = zero;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const h8 ga = *(const h8*)(GT + (j0 + r) * TS + 32 * c + 8 * g);
            const h8 ib = *(const h8*)(IT + (k0 + r) * TS + 32 * c + 8 * g);
            acc = sur_mma(ga, ib, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) out[off + (j0 + 4 * g + v) * ncol + k0 + r] = acc[v];
    }
    // bias gradients
    if (tid < 2 * SUR_NH + SUR_KOUT) {
        const _Float16* row;
        int o;
        if (tid < SUR_NH) { row = G1T + tid * TS; o = SUR_OB1 + tid; }
        else if (tid < 2 * SUR_NH) { row = G2T + (tid - SUR_NH) * TS; o = SUR_OB2 + tid - SUR_NH; }
        else { row = D3T + (tid - 2 * SUR_NH) * TS; o = SUR_OB3 + tid - 2 * SUR_NH; }
        float sacc = 0.f;
        for (int b = 0; b < 64; ++b) sacc += (float)row[b];
        out[o] = sacc;
    }
    if (tid == 0) A.loss[blockIdx.x] = (double)lsum[0] + lsum[1] + lsum[2] + lsum[3];
}

// Sum of the workgroup partial gradients, times gscale (-> FP32 gradient);
// with update: one Adam step on the FP32 master weights and fresh FP16
// copies (row-major and the transposes of W2 and W3).
__global__ __launch_bounds__(256) void sur_adam_kernel(SurAdam S) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= SUR_NPARAM) return;
    float gsum = 0.f;
    for (int w = 0; w < S.nwg; ++w) gsum += S.part[(long long)w * SUR_NPARAM + p];
    const float gr = gsum * S.gscale;
    if (S.grad_out) S.grad_out[p] = gr;
    if (!S.update) return;
    const float m = S.b1 * S.m[p] + (1.f - S.b1) * gr;
    const float v = S.b2 * S.v[p] + (1.f - S.b2) * gr * gr;
    S.m[p] = m;
    S.v[p] = v;
    const float th = S.theta[p] - S.lr * (m / S.bc1) / (sqrtf(v / S.bc2) + S.eps);
    S.theta[p] = th;
    write_half_param(S.H, p, th);
}

// FP16 copies of every parameter
__global__ __launch_bounds__(256) void sur_halves_kernel(const float* theta, SurHalves H) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= SUR_NPARAM) return;
    write_half_param(H, p, theta[p]);
}

// Inference: t = out * st + mt for m samples (64 per wave, 4 groups of 16).
// With T: per-bin maximum over the 21 outputs of |t - T| (atomicMax on the
// float bits, all values non-negative) and bin populations.
__global__ __launch_bounds__(256) void sur_predict_kernel(SurPredict P) {
    __shared__ float outs[4][64 * 33];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const long long i = (long long)blockIdx.x * 256 + tid;
    const bool valid = i < P.m;
    const SurNet& N = P.N;
    float xn[SUR_NIN];
    for (int k = 0; k < SUR_NIN; ++k) xn[k] = 0.f;
    if (valid) sur_std_features(N, P.F + i * SUR_NIN, xn);
    unsigned int pk[5];
    sur_pack_x(xn, pk);
    float* ow = outs[wave];
    for (int q = 0; q < 4; ++q) {
        const h8 xb = sur_gather_x(pk, q);
        SurAct a;
        sur_forward16(N, xb, a);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) ow[(16 * q + r) * 33 + 16 * t + 4 * g + v] = a.out[t][v];
    }
    __syncthreads();
    if (!valid) return;
    float emax = 0.f;
    for (int j = 0; j < SUR_NOUT; ++j) {
        const double t = (double)ow[lane * 33 + j] * (double)N.st[j] + (double)N.mt[j];
        if (P.out) P.out[i * SUR_NOUT + j] = t;
        if (P.T) emax = fmaxf(emax, (float)fabs(t - P.T[i * SUR_NOUT + j]));
    }
    if (P.T) {
        const double* f = P.F + i * SUR_NIN;
        const int b = sur_rbin_features(f) * SUR_NSB + sur_sbin(f[8]);
        atomicMax(P.emax_bits + b, __float_as_uint(emax));
        atomicAdd(P.count + b, 1u);
    }
}

// Column statistics of a row-major m x ncol FP64 array, pass 1: partial
// sums, minima and maxima per workgroup (grid-stride over rows).
__global__ __launch_bounds__(256) void sur_colstat_kernel(const double* X, long long m, int ncol,
                                                          const double* mean, double* part) {
    __shared__ double sh[256];
    for (int c = 0; c < ncol; ++c) {
        double s = 0.0, lo = INFINITY, hi = -INFINITY;
        for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < m; i += (long long)gridDim.x * 256) {
            double v = X[i * ncol + c];
            if (mean) {
                v -= mean[c];
                s += v * v;
            } else {
                s += v;
                lo = fmin(lo, v);
                hi = fmax(hi, v);
            }
        }
        double* o = part + ((long long)blockIdx.x * ncol + c) * 3;
        for (int k = 0; k < 3; ++k) {
            double v = k == 0 ? s : (k == 1 ? lo : hi);
            sh[threadIdx.x] = v;
            __syncthreads();
            for (int w = 128; w >= 1; w >>= 1) {
                if ((int)threadIdx.x < w) {
                    const double x = sh[threadIdx.x], y = sh[threadIdx.x + w];
                    sh[threadIdx.x] = k == 0 ? x + y : (k == 1 ? fmin(x, y) : fmax(x, y));
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) o[k] = sh[0];
            __syncthreads();
        }
    }
}

// pass 2: combine the workgroup partials (one thread per column)
__global__ void sur_colstat_reduce_kernel(const double* part, int nblk, int ncol, double* out) {
    const int c = threadIdx.x;
    if (c >= ncol) return;
    double s = 0.0, lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
        const double* o = part + ((long long)b * ncol + c) * 3;
        s += o[0];
        lo = fmin(lo, o[1]);
        hi = fmax(hi, o[2]);
    }
    out[3 * c] = s;
    out[3 * c + 1] = lo;
    out[3 * c + 2] = hi;
}

// ---------------------------------------------------------------- launch --

void launch_sur_train(const SurTrain& A, int nwg, hipStream_t st) {
    hipLaunchKernelGGL(sur_train_kernel, dim3(nwg), dim3(256), 0, st, A);
}

void launch_sur_adam(const SurAdam& S, hipStream_t st) {
    hipLaunchKernelGGL(sur_adam_kernel, dim3((SUR_NPARAM + 255) / 256), dim3(256), 0, st, S);
}

void launch_sur_halves(const float* theta, const SurHalves& H, hipStream_t st) {
    hipLaunchKernelGGL(sur_halves_kernel, dim3((SUR_NPARAM + 255) / 256), dim3(256), 0, st, theta, H);
}

void launch_sur_predict(const SurPredict& P, hipStream_t st) {
    if (P.m <= 0) return;
    hipLaunchKernelGGL(sur_predict_kernel, dim3((unsigned)((P.m + 255) / 256)), dim3(256), 0, st, P);
}

void launch_sur_colstat(const double* X, long long m, int ncol, const double* mean, double* part, int nblk,
                        double* out, hipStream_t st) {
    hipLaunchKernelGGL(sur_colstat_kernel, dim3(nblk), dim3(256), 0, st, X, m, ncol, mean, part);
    hipLaunchKernelGGL(sur_colstat_reduce_kernel, dim3(1), dim3(64), 0, st, (const double*)part, nblk, ncol,
                       out);
}

}  // namespace fl
