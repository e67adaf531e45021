// Batched dense products and batched Jacobi-PCG for many right-hand sides
// and several fractional orders s at once (Sec. 5: the solve is driven by
// dense matrix-vector products; with 64 right-hand sides per matrix the
// product becomes a GEMM, which runs on the matrix cores).
//
// Layouts (all internal buffers are padded and zero-filled):
//   matrices   ns blocks of n_pad x lda, row-major (A is symmetric, so a row
//              is also a column), block j at j * sA elements;
//   vectors    ns blocks of 64 columns, column-major with leading dimension
//              n_pad, block j at j * 64 * n_pad;  n_pad is a multiple of 256.
//
// GEMM Y_j = A_j X_j (one launch for every system j whose columns are still
// active).  A workgroup owns BM = WM x WAVES rows of one system and all 64
// columns.  Each wave streams its WM rows of A straight from HBM into
// registers (each lane a 32-byte run along K per step, non-temporal: A is
// read once per product), the 64-column X tile is staged through
// double-buffered LDS and shared by the waves.  The K order inside one MFMA
// step is permuted identically for A and X (lane group g takes the g-th
// run), which leaves the product unchanged and lets every lane load
// contiguous memory.  Tiles are ordered so that one XCD works through the
// row blocks of one system, which keeps X_j in that XCD's L2.
#include <hip/hip_runtime.h>

#include "fl_internal.hpp"

namespace fl {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int DT>
struct GT;
template <>
struct GT<GD_F64> {
    typedef double acc_t;
    typedef v4d accv;
    enum { SZ = 8, EPL = 4, KSTEP = 16 };
};
template <>
struct GT<GD_F32> {
    typedef float acc_t;
    typedef v4f accv;
    enum { SZ = 4, EPL = 8, KSTEP = 32 };
};
template <>
struct GT<GD_BF16> {
    typedef float acc_t;
    typedef v4f accv;
    enum { SZ = 2, EPL = 16, KSTEP = 64 };
};

// 32 bytes of one operand held by a lane: EPL consecutive K elements
struct Seg {
    u32x4 a, b;
};

__device__ __forceinline__ Seg ld_seg_nt(const char* p) {
    Seg s;
    s.a = __builtin_nontemporal_load((const u32x4*)p);
    s.b = __builtin_nontemporal_load((const u32x4*)p + 1);
    return s;
}
__device__ __forceinline__ Seg ld_seg_lds(const char* p) {
    Seg s;
    s.a = *(const u32x4*)p;
    s.b = *((const u32x4*)p + 1);
    return s;
}

template <int DT>
__device__ __forceinline__ void mma(const Seg& x, const Seg& y, typename GT<DT>::accv& c);

template <>
__device__ __forceinline__ void mma<GD_F64>(const Seg& x, const Seg& y, v4d& c) {
    const double* a = (const double*)&x;
    const double* b = (const double*)&y;
#pragma unroll
    for (int e = 0; e < 4; ++e) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], b[e], c, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<GD_F32>(const Seg& x, const Seg& y, v4f& c) {
    const float* a = (const float*)&x;
    const float* b = (const float*)&y;
#pragma unroll
    for (int e = 0; e < 8; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], c, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<GD_BF16>(const Seg& x, const Seg& y, v4f& c) {
    v8bf a0 = __builtin_bit_cast(v8bf, x.a), a1 = __builtin_bit_cast(v8bf, x.b);
    v8bf b0 = __builtin_bit_cast(v8bf, y.a), b1 = __builtin_bit_cast(v8bf, y.b);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, c, 0, 0, 0);
}

// DT: element type of A and X; NPA: A planes (bf16 only: 1 = hi, 2 = hi+lo);
// WM rows per wave; WAVES per workgroup; BK: K extent of one LDS stage.
template <int DT, int NPA, int WM, int WAVES, int BK>
__global__ __launch_bounds__(WAVES * 64) void gemm_kernel(GemmArgs g) {
    typedef GT<DT> G;
    typedef typename G::acc_t acc_t;
    typedef typename G::accv accv;
    constexpr int SZ = G::SZ, EPL = G::EPL, KSTEP = G::KSTEP;
    constexpr int BM = WM * WAVES, NT = WAVES * 64, MB = WM / 16, NKS = BK / KSTEP;
    constexpr int NPX = DT == GD_BF16 ? 2 : 1;  // X planes: bf16 hi + lo
    constexpr int COLB = BK * SZ + 16;          // LDS bytes per column (16-byte pad)
    constexpr int PLANEB = 64 * COLB;
    constexpr int CPC = BK * SZ / 16;           // 16-byte chunks per column and stage
    constexpr int NCH = 64 * CPC * NPX;
    constexpr int CPT = NCH / NT;
    static_assert(NCH % NT == 0, "stage size must be a multiple of the workgroup");
    static_assert(BK % KSTEP == 0 && WM % 16 == 0, "tile shape");
    static_assert(DT == GD_BF16 || NPA == 1, "two A planes only for bf16");
    __shared__ __align__(16) char lds[2][NPX * PLANEB];
    __shared__ double red[WAVES][64];

    // work item w = (tile, split); tiles = (active system, row block); a
    // contiguous range of work items per XCD (workgroups are dealt to the
    // XCDs round-robin)
    const long long nrb = g.n_pad / BM;
    const long long nwork = (long long)g.nsys * nrb * g.ksplit;
    const long long per = (nwork + 7) / 8;
    const long long L = blockIdx.x;
    const long long w = (L & 7) * per + (L >> 3);
    if (w >= nwork) return;
    const int split = (int)(w % g.ksplit);
    const long long t = w / g.ksplit;
    const int j = g.sys[t / nrb];
    const long long rb = t % nrb;
    if (g.act) {
        const int a = g.act[j * 64 + (threadIdx.x & 63)];
        if (!__syncthreads_or(a)) return;
    }
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r16 = lane & 15, gq = lane >> 4;
    const long long row0 = rb * BM + wave * WM;

    const char* Ap[NPA];
    Ap[0] = (const char*)g.A + ((long long)j * g.sA + (row0 + r16) * g.lda + gq * EPL) * SZ;
    if (NPA == 2) Ap[NPA - 1] = (const char*)g.A2 + ((long long)j * g.sA + (row0 + r16) * g.lda + gq * EPL) * SZ;
    const char* Xp[NPX];
    Xp[0] = (const char*)g.X + (long long)j * g.sX * SZ;
    if (NPX == 2) Xp[NPX - 1] = (const char*)g.X2 + (long long)j * g.sX * SZ;

    accv acc[MB][4];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[m][c] = accv{0, 0, 0, 0};

    u32x4 stg[CPT];
    auto gload = [&](long long k0) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = tid + c * NT;
            const int pl = ch / (64 * CPC), cc = ch % (64 * CPC), col = cc / CPC, q = cc % CPC;
            stg[c] = *(const u32x4*)(Xp[pl] + ((long long)col * g.n_pad + k0) * SZ + q * 16);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = tid + c * NT;
            const int pl = ch / (64 * CPC), cc = ch % (64 * CPC), col = cc / CPC, q = cc % CPC;
            *(u32x4*)(&lds[buf][pl * PLANEB + col * COLB + q * 16]) = stg[c];
        }
    };

    const long long nkt = g.n_pad / BK, kchunk = (nkt + g.ksplit - 1) / g.ksplit;
    const long long kb = split * kchunk, nk = kb + kchunk < nkt ? kb + kchunk : nkt;
    if (kb < nk) {
        gload(kb * BK);
        lstore((int)(kb & 1));
    }
    __syncthreads();
    for (long long kc = kb; kc < nk; ++kc) {
        const int buf = (int)(kc & 1);
        if (kc + 1 < nk) gload((kc + 1) * BK);
        Seg a[NKS][MB][NPA];
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int p = 0; p < NPA; ++p)
                    a[ks][m][p] = ld_seg_nt(Ap[p] + ((long long)m * 16 * g.lda + kc * BK + ks * KSTEP) * SZ);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int off = (cb * 16 + r16) * COLB + (ks * KSTEP + gq * EPL) * SZ;
                const Seg bh = ld_seg_lds(&lds[buf][off]);
                if (DT == GD_BF16) {
                    const Seg bl = ld_seg_lds(&lds[buf][PLANEB * (NPX - 1) + off]);
#pragma unroll
                    for (int m = 0; m < MB; ++m) {
                        mma<DT>(a[ks][m][0], bh, acc[m][cb]);
                        mma<DT>(a[ks][m][0], bl, acc[m][cb]);
                        if (NPA == 2) mma<DT>(a[ks][m][NPA - 1], bh, acc[m][cb]);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < MB; ++m) mma<DT>(a[ks][m][0], bh, acc[m][cb]);
                }
            }
        }
        if (kc + 1 < nk) lstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue.  Lane (r16, gq) holds column cb*16 + r16 of the 16-row block
    // m; item v is row 4*gq + v (f32 / bf16 MFMA) or row gq + 4*v (f64 MFMA).
    acc_t* Y = (acc_t*)g.Y + (long long)split * g.ysplit + (long long)j * g.sX;
    const acc_t* V = (const acc_t*)g.V + (long long)j * g.sX;
    double dsum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const long long cbase = (long long)(cb * 16 + r16) * g.n_pad + row0 + m * 16;
            accv v = acc[m][cb];
            if (DT == GD_F64) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const long long off = cbase + gq + 4 * i;
                    acc_t y = v[i];
                    if (g.epi == 2) y = V[off] - y;
                    Y[off] = y;
                    if (g.epi == 1) dsum[cb] += (double)V[off] * (double)y;
                    else if (g.epi == 2) dsum[cb] += (double)y * (double)y;
                }
            } else {
                const long long off = cbase + 4 * gq;
                if (g.epi == 2) {
                    const accv b = *(const accv*)(V + off);
                    v = b - v;
                }
                *(accv*)(Y + off) = v;
                if (g.epi == 1) {
                    const accv pv = *(const accv*)(V + off);
#pragma unroll
                    for (int i = 0; i < 4; ++i) dsum[cb] += (double)pv[i] * (double)v[i];
                } else if (g.epi == 2) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) dsum[cb] += (double)v[i] * (double)v[i];
                }
            }
        }
    if (g.epi != 0) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            dsum[cb] += __shfl_xor(dsum[cb], 16);
            dsum[cb] += __shfl_xor(dsum[cb], 32);
            if (gq == 0) red[wave][cb * 16 + r16] = dsum[cb];
        }
        __syncthreads();
        if (tid < 64) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) s += red[w][tid];
            g.part[((long long)j * nrb + rb) * 64 + tid] = s;
        }
    }
}

// ------------------------------------------------------------------------
// Kernel table for the autotuner.  Every entry is a complete kernel; the
// tuner times the entries of one element type on the actual sizes and
// keeps the fastest.
typedef void (*GemmFn)(GemmArgs);
struct GemmEntry {
    int dt, npa, wm, waves, bk;
    GemmFn fn;
};

#define GE(DT, NPA, WM, WV, BK) {DT, NPA, WM, WV, BK, gemm_kernel<DT, NPA, WM, WV, BK>}
static const GemmEntry kGemm[] = {
    GE(GD_F64, 1, 16, 4, 32),   GE(GD_F64, 1, 32, 4, 32),   GE(GD_F64, 1, 32, 4, 64),
    GE(GD_F64, 1, 16, 8, 64),   GE(GD_F64, 1, 32, 8, 32),
    GE(GD_F32, 1, 32, 4, 64),   GE(GD_F32, 1, 64, 4, 32),   GE(GD_F32, 1, 32, 8, 64),
    GE(GD_F32, 1, 16, 8, 128),  GE(GD_F32, 1, 64, 4, 64),
    GE(GD_BF16, 1, 32, 4, 128), GE(GD_BF16, 1, 64, 4, 64),  GE(GD_BF16, 1, 32, 8, 128),
    GE(GD_BF16, 1, 16, 8, 256), GE(GD_BF16, 1, 64, 4, 128),
    GE(GD_BF16, 2, 32, 4, 64),  GE(GD_BF16, 2, 16, 8, 128), GE(GD_BF16, 2, 32, 8, 64),
    GE(GD_BF16, 2, 32, 4, 128),
};
#undef GE

int gemm_count() { return (int)(sizeof(kGemm) / sizeof(kGemm[0])); }

GemmInfo gemm_info(int id) {
    GemmInfo i{};
    if (id < 0 || id >= gemm_count()) return i;
    const GemmEntry& e = kGemm[id];
    i.dt = e.dt;
    i.npa = e.npa;
    i.wm = e.wm;
    i.waves = e.waves;
    i.bk = e.bk;
    i.bm = e.wm * e.waves;
    return i;
}

hipError_t launch_gemm(int id, const GemmArgs& g, hipStream_t st) {
    if (id < 0 || id >= gemm_count()) return hipErrorInvalidValue;
    const GemmEntry& e = kGemm[id];
    const long long bm = (long long)e.wm * e.waves;
    if (g.n_pad % 256 != 0 || g.n_pad % e.bk != 0 || g.nsys <= 0 || g.nsys > FL_MAX_BATCH || g.ksplit < 1 ||
        (g.ksplit > 1 && g.epi != 0))
        return hipErrorInvalidValue;
    const long long ntiles = (g.n_pad / bm) * g.nsys * g.ksplit;
    const long long per = (ntiles + 7) / 8;
    hipLaunchKernelGGL(e.fn, dim3((unsigned)(8 * per)), dim3(e.waves * 64), 0, st, g);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// conversions into the padded batch layouts

// FP64 matrix block (n x n used, ld ld64) -> FP32 or bf16 planes (ld ldl,
// n_pad rows; padding written as zero).  bf16: hi = RNE(a), lo = RNE(a - hi).
__global__ void mat_lo_kernel(const double* A, long long ld64, long long n, long long n_pad,
                              long long ldl, int dt, int npa, void* P0, void* P1) {
    for (long long row = blockIdx.y; row < n_pad; row += gridDim.y)
        for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ldl;
             c += (long long)gridDim.x * blockDim.x) {
            const double a = (row < n && c < n) ? A[row * ld64 + c] : 0.0;
            const long long o = row * ldl + c;
            if (dt == GD_F32) {
                ((float*)P0)[o] = (float)a;
            } else {
                const __bf16 hi = (__bf16)(float)a;
                ((__bf16*)P0)[o] = hi;
                if (npa == 2) ((__bf16*)P1)[o] = (__bf16)(float)(a - (double)(float)hi);
            }
        }
}

void launch_mat_lo(const double* A, long long ld64, long long n, long long n_pad, long long ldl, int dt,
                   int npa, void* P0, void* P1, hipStream_t st) {
    if (n_pad <= 0) return;
    const unsigned gx = (unsigned)std::min<long long>((ldl + 255) / 256, 64);
    hipLaunchKernelGGL(mat_lo_kernel, dim3(gx, (unsigned)std::min<long long>(n_pad, 32768)), dim3(256), 0, st, A, ld64, n, n_pad, ldl,
                       dt, npa, P0, P1);
}

// diagonal of every matrix block -> FP64 and FP32 reciprocals (0 in padding)
__global__ void bdiag_kernel(const double* A, long long lda, long long sA, long long n, long long n_pad,
                             int ns, double* dinv64, float* dinv32) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n_pad || j >= ns) return;
    double v = 0.0;
    if (i < n) {
        const double d = A[(long long)j * sA + i * lda + i];
        v = d != 0.0 ? 1.0 / d : 0.0;
    }
    dinv64[(long long)j * n_pad + i] = v;
    if (dinv32) dinv32[(long long)j * n_pad + i] = (float)v;
}

void launch_bdiag(const double* A, long long lda, long long sA, long long n, long long n_pad, int ns,
                  double* dinv64, float* dinv32, hipStream_t st) {
    if (n_pad <= 0 || ns <= 0) return;
    hipLaunchKernelGGL(bdiag_kernel, dim3((unsigned)((n_pad + 255) / 256), (unsigned)ns), dim3(256), 0, st,
                       A, lda, sA, n, n_pad, ns, dinv64, dinv32);
}

// user column-major (n x nrhs, ld, block stride) <-> padded internal
// (64 columns of n_pad per system).  Padding rows / columns are zero.
template <class S, class D>
__global__ void pack_kernel(const S* src, long long ld, long long sstride, long long n, int nrhs,
                            long long n_pad, D* dst) {
    const int j = blockIdx.z, c = blockIdx.y;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (long long)gridDim.x * blockDim.x) {
        D v = (D)0;
        if (i < n && c < nrhs) v = (D)src[(long long)j * sstride + (long long)c * ld + i];
        dst[((long long)j * 64 + c) * n_pad + i] = v;
    }
}
template <class S, class D>
__global__ void unpack_kernel(const S* src, long long n_pad, long long n, int nrhs, D* dst, long long ld,
                              long long dstride) {
    const int j = blockIdx.z, c = blockIdx.y;
    if (c >= nrhs) return;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[(long long)j * dstride + (long long)c * ld + i] = (D)src[((long long)j * 64 + c) * n_pad + i];
}

static dim3 pack_grid(long long n_pad, int ns) {
    return dim3((unsigned)std::min<long long>((n_pad + 255) / 256, 32), 64, (unsigned)ns);
}

void launch_pack_f64(const double* src, long long ld, long long sstride, long long n, int nrhs,
                     long long n_pad, int ns, double* dst, hipStream_t st) {
    hipLaunchKernelGGL((pack_kernel<double, double>), pack_grid(n_pad, ns), dim3(256), 0, st, src, ld, sstride,
                       n, nrhs, n_pad, dst);
}
void launch_pack_f32(const float* src, long long ld, long long sstride, long long n, int nrhs,
                     long long n_pad, int ns, float* dst, hipStream_t st) {
    hipLaunchKernelGGL((pack_kernel<float, float>), pack_grid(n_pad, ns), dim3(256), 0, st, src, ld, sstride, n,
                       nrhs, n_pad, dst);
}
void launch_unpack_f64(const double* src, long long n_pad, long long n, int nrhs, int ns, double* dst,
                       long long ld, long long dstride, hipStream_t st) {
    hipLaunchKernelGGL((unpack_kernel<double, double>), pack_grid(n_pad, ns), dim3(256), 0, st, src, n_pad, n,
                       nrhs, dst, ld, dstride);
}
void launch_unpack_f32(const float* src, long long n_pad, long long n, int nrhs, int ns, float* dst,
                       long long ld, long long dstride, hipStream_t st) {
    hipLaunchKernelGGL((unpack_kernel<float, float>), pack_grid(n_pad, ns), dim3(256), 0, st, src, n_pad, n,
                       nrhs, dst, ld, dstride);
}

// deterministic non-trivial fill (autotuner operands): v_i = 1 + (i mod 7) / 8
template <class T>
__global__ void fill_kernel(T* x, long long m) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = (T)(1.0 + (double)(i % 7) * 0.125);
}
void launch_fill_f64(double* x, long long m, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(fill_kernel<double>, dim3(2048), dim3(256), 0, st, x, m);
}
void launch_fill_f32(float* x, long long m, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(fill_kernel<float>, dim3(2048), dim3(256), 0, st, x, m);
}

// FP32 vectors -> bf16 hi / lo planes (same layout)
__global__ void split_bf16_kernel(const float* x, long long m, __bf16* hi, __bf16* lo) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const float v = x[i];
        const __bf16 h = (__bf16)v;
        hi[i] = h;
        lo[i] = (__bf16)(v - (float)h);
    }
}
void launch_split_bf16(const float* x, long long m, void* hi, void* lo, hipStream_t st) {
    if (m <= 0) return;
    const unsigned g = (unsigned)std::min<long long>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(split_bf16_kernel, dim3(g), dim3(256), 0, st, x, m, (__bf16*)hi, (__bf16*)lo);
}

// ------------------------------------------------------------------------
// Batched Jacobi-PCG (Sec. 5), one workgroup per (system j, column c).
// Per iteration: Q = A P with p.q partials from the GEMM epilogue, then one
// step kernel: alpha = rz / p.q; r -= alpha q; z = D^{-1} r; rz', rr';
// convergence test ||r|| <= rtol ||b||; beta = rz'/rz; x += alpha p;
// p = z + beta p (x uses the old p, so both updates share one pass).
constexpr int BCG_T = 512;

template <class T>
__device__ __forceinline__ double block_sum2(double& a, double& b, double* sh) {
    // sum a and b over the workgroup (BCG_T threads); result in a, b on all threads
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        sh[2 * w] = a;
        sh[2 * w + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int i = 0; i < BCG_T / 64; ++i) {
        a += sh[2 * i];
        b += sh[2 * i + 1];
    }
    return a;
}

template <class T>
__device__ __forceinline__ void write_planes(const BcgState<T>& S, long long o, T v) {
    if (S.ph) {
        const float f = (float)v;
        const __bf16 h = (__bf16)f;
        ((__bf16*)S.ph)[o] = h;
        ((__bf16*)S.pl)[o] = (__bf16)(f - (float)h);
    }
}

// r = b, x = 0, z = D^{-1} r, p = z; rz, bb; activity
template <class T>
__global__ __launch_bounds__(BCG_T) void bcg_init_kernel(BcgState<T> S) {
    __shared__ double sh[2 * BCG_T / 64];
    const int c = blockIdx.x, j = blockIdx.y;
    const long long col = ((long long)j * 64 + c) * S.n_pad;
    const T* dinv = S.dinv + (long long)j * S.n_pad;
    const int idx = j * 64 + c;
    if (!S.want[idx]) {
        for (long long i = threadIdx.x; i < S.n_pad; i += BCG_T) {
            S.x[col + i] = (T)0;
            S.r[col + i] = (T)0;
            S.p[col + i] = (T)0;
            write_planes(S, col + i, (T)0);
        }
        if (threadIdx.x == 0) {
            S.act[idx] = 0;
            S.iters[idx] = 0;
            S.status[idx] = 0;
            S.rz[idx] = 0.0;
            S.bb[idx] = 0.0;
            S.rel[idx] = 0.0;
            if (S.upd) S.upd[idx] = 0;
            if (S.lsf) S.lsf[idx] = 0;
        }
        return;
    }
    double rz = 0.0, bb = 0.0;
    for (long long i = threadIdx.x; i < S.n_pad; i += BCG_T) {
        const T b = S.b[col + i];
        const T z = b * dinv[i];
        S.x[col + i] = (T)0;
        S.r[col + i] = b;
        S.p[col + i] = z;
        write_planes(S, col + i, z);
        rz += (double)b * (double)z;
        bb += (double)b * (double)b;
    }
    block_sum2<T>(rz, bb, sh);
    if (threadIdx.x == 0) {
        const bool fin = bb == bb && bb < 1.79e308;
        S.rz[idx] = rz;
        S.bb[idx] = bb;
        S.iters[idx] = 0;
        S.status[idx] = fin ? 0 : 2;
        S.act[idx] = (fin && bb > 0.0 && S.maxit > 0) ? 1 : 0;
        S.rel[idx] = bb > 0.0 ? 1.0 : 0.0;
        if (S.upd) {
            S.upd[idx] = 0;
            S.rupd2[idx] = bb;
        }
        if (S.lsf) S.lsf[idx] = 0;
    }
}

template <class T>
__global__ __launch_bounds__(BCG_T) void bcg_step_kernel(BcgState<T> S) {
    __shared__ double sh[2 * BCG_T / 64];
    const int c = blockIdx.x, j = blockIdx.y;
    const int idx = j * 64 + c;
    if (!S.act[idx]) return;
    const long long col = ((long long)j * 64 + c) * S.n_pad;
    const T* dinv = S.dinv + (long long)j * S.n_pad;
    // p.q from the GEMM epilogue partials, or q = sum of the K-split partial
    // products and p.q formed here
    double pq = 0.0, dummy = 0.0;
    if (S.ksplit == 1) {
        for (int rb = threadIdx.x; rb < S.nrbq; rb += BCG_T) pq += S.partq[((long long)j * S.nrbq + rb) * 64 + c];
    } else {
        for (long long i = threadIdx.x; i < S.n_pad; i += BCG_T) {
            T qs = S.q[col + i];
            for (int k = 1; k < S.ksplit; ++k) qs += S.q[k * S.ysplit + col + i];
            S.q[col + i] = qs;
            pq += (double)S.p[col + i] * (double)qs;
        }
    }
    block_sum2<T>(pq, dummy, sh);
    const double rz_old = S.rz[idx];
    const double num = (S.lsf && S.lsf[idx]) ? S.pr[idx] : rz_old;
    if (!(pq > 0.0) || !(pq < 1.79e308)) {
        if (threadIdx.x == 0) {
            S.status[idx] = (pq == pq) ? 1 : 2;
            S.act[idx] = 0;
        }
        return;
    }
    const double alpha = num / pq;
    const T a = (T)alpha;
    double rz = 0.0, rr = 0.0;
    for (long long i = threadIdx.x; i < S.n_pad; i += BCG_T) {
        const T r = S.r[col + i] - a * S.q[col + i];
        S.r[col + i] = r;
        const T z = r * dinv[i];
        rz += (double)r * (double)z;
        rr += (double)r * (double)r;
    }
    block_sum2<T>(rz, rr, sh);
    const int it = S.iters[idx] + 1;
    const double bb = S.bb[idx];
    const bool fin = rr == rr && rr < 1.79e308;
    const bool conv = rr <= S.rtol2 * bb;
    const bool stop = conv || !fin || it >= S.maxit;
    // with residual replacement p stays current even at a stop: the
    // replacement may find the column unconverged and resume it
    const bool newp = !stop || (S.upd && fin);
    const T beta = (T)(rz_old > 0.0 ? rz / rz_old : 0.0);
    for (long long i = threadIdx.x; i < S.n_pad; i += BCG_T) {
        const T p = S.p[col + i];
        S.x[col + i] += a * p;
        if (newp) {
            const T pn = S.r[col + i] * dinv[i] + beta * p;
            S.p[col + i] = pn;
            write_planes(S, col + i, pn);
        }
    }
    if (threadIdx.x == 0) {
        S.iters[idx] = it;
        S.rz[idx] = rz;
        S.rel[idx] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        if (!fin) S.status[idx] = 2;
        if (stop) S.act[idx] = 0;
        if (S.upd && fin && (stop || rr < S.delta2 * S.rupd2[idx])) {
            S.upd[idx] = 1;
            S.act[idx] = 0;
        }
        if (S.lsf) S.lsf[idx] = 0;
    }
}

template <class T>
void launch_bcg_init(const BcgState<T>& S, int ns, hipStream_t st) {
    hipLaunchKernelGGL(bcg_init_kernel<T>, dim3(64, ns), dim3(BCG_T), 0, st, S);
}
template <class T>
void launch_bcg_step(const BcgState<T>& S, int ns, hipStream_t st) {
    hipLaunchKernelGGL(bcg_step_kernel<T>, dim3(64, ns), dim3(BCG_T), 0, st, S);
}
template void launch_bcg_init<float>(const BcgState<float>&, int, hipStream_t);
template void launch_bcg_init<double>(const BcgState<double>&, int, hipStream_t);
template void launch_bcg_step<float>(const BcgState<float>&, int, hipStream_t);
template void launch_bcg_step<double>(const BcgState<double>&, int, hipStream_t);

// active columns: out[0] total, out[1 + j] of system j (one wave per system)
__global__ __launch_bounds__(1024) void count_kernel(const int* act, int ns, int* out) {
    __shared__ int sh[16];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int c = 0;
    if (w < ns) c = __popcll(__ballot(act[w * 64 + l] != 0));
    if (l == 0) sh[w] = w < ns ? c : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int i = 0; i < 16; ++i) tot += sh[i];
        out[0] = tot;
    }
    if (l == 0 && w < ns) out[1 + w] = c;
}
void launch_count(const int* act, int ns, int* out, hipStream_t st) {
    hipLaunchKernelGGL(count_kernel, dim3(1), dim3(1024), 0, st, act, ns, out);
}

// ------------------------------------------------------------------------
// Mixed-precision batched CG: FP64 solution and true residuals around the
// FP32-arithmetic CG recurrence on the low-precision matrix.

// u += x, x = 0 on the columns with upd set
__global__ void corr_masked_kernel(double* u, float* x, const int* upd, long long n_pad) {
    const int c = blockIdx.y, j = blockIdx.z;
    if (!upd[j * 64 + c]) return;
    const long long col = ((long long)j * 64 + c) * n_pad;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (long long)gridDim.x * blockDim.x) {
        u[col + i] += (double)x[col + i];
        x[col + i] = 0.f;
    }
}
void launch_corr_masked(double* u, float* x, const int* upd, long long n_pad, int ns, hipStream_t st) {
    const unsigned gx = (unsigned)std::min<long long>((n_pad + 255) / 256, 16);
    hipLaunchKernelGGL(corr_masked_kernel, dim3(gx, 64, ns), dim3(256), 0, st, u, x, upd, n_pad);
}

__global__ __launch_bounds__(256) void reliable_kernel(ReliableState R) {
    __shared__ double sh[12];
    const int c = blockIdx.x, j = blockIdx.y;
    const int idx = j * 64 + c;
    if (!R.upd[idx]) return;
    const long long col = ((long long)j * 64 + c) * R.n_pad;
    const float* dinv = R.dinv + (long long)j * R.n_pad;
    // r64 = b - sum of the partial products; rr, and (used only if the
    // column goes on) r, rz, p.r
    double rr = 0.0, rz = 0.0, pr = 0.0;
    for (long long i = threadIdx.x; i < R.n_pad; i += 256) {
        double y = R.y64[col + i];
        for (int k = 1; k < R.ksplit; ++k) y += R.y64[k * R.ysplit + col + i];
        const double r64 = R.b64[col + i] - y;
        rr += r64 * r64;
        const float r = (float)r64;
        R.r[col + i] = r;
        rz += (double)r * (double)(r * dinv[i]);
        pr += (double)R.p[col + i] * (double)r;
    }
    for (int o = 32; o > 0; o >>= 1) {
        rr += __shfl_xor(rr, o);
        rz += __shfl_xor(rz, o);
        pr += __shfl_xor(pr, o);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = rr;
        sh[4 + (threadIdx.x >> 6)] = rz;
        sh[8 + (threadIdx.x >> 6)] = pr;
    }
    __syncthreads();
    rr = sh[0] + sh[1] + sh[2] + sh[3];
    rz = sh[4] + sh[5] + sh[6] + sh[7];
    pr = sh[8] + sh[9] + sh[10] + sh[11];
    const double bb = R.bb[idx];
    const bool fin = rr == rr && rr < 1.79e308;
    const bool done = !fin || rr <= R.rtol2 * bb || R.iters[idx] >= R.maxit;
    if (threadIdx.x == 0) {
        R.rel[idx] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        if (!fin) R.status[idx] = 2;
        if (done) {
            R.act[idx] = 0;
        } else {
            R.rz[idx] = rz;
            R.rupd2[idx] = rr;
            R.pr[idx] = pr;
            R.lsf[idx] = 1;
            R.act[idx] = 1;
        }
        R.upd[idx] = 0;
    }
}
void launch_reliable(const ReliableState& R, int ns, hipStream_t st) {
    hipLaunchKernelGGL(reliable_kernel, dim3(64, ns), dim3(256), 0, st, R);
}

// b.b per column of the padded FP64 right-hand sides; activity (columns
// c < nrhs with a finite, nonzero b); u = 0; r32 = fp32(b) for the
// low-precision CG
__global__ __launch_bounds__(256) void refine_init_kernel(RefineState R, int nrhs) {
    __shared__ double sh[8];
    const int c = blockIdx.x, j = blockIdx.y;
    const int idx = j * 64 + c;
    const long long col = ((long long)j * 64 + c) * R.n_pad;
    double bb = 0.0;
    for (long long i = threadIdx.x; i < R.n_pad; i += 256) {
        const double b = R.b64[col + i];
        bb += b * b;
        R.u64[col + i] = 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) bb += __shfl_xor(bb, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = bb;
    __syncthreads();
    bb = sh[0] + sh[1] + sh[2] + sh[3];
    const bool fin = bb == bb && bb < 1.79e308;
    const bool on = c < nrhs && fin && bb > 0.0;
    if (R.r32)
        for (long long i = threadIdx.x; i < R.n_pad; i += 256) R.r32[col + i] = on ? (float)R.b64[col + i] : 0.f;
    if (threadIdx.x == 0) {
        R.bb[idx] = bb;
        R.status[idx] = fin ? 0 : 2;
        R.oact[idx] = on ? 1 : 0;
        if (R.want) R.want[idx] = on ? 1 : 0;
        R.rel[idx] = bb > 0.0 ? 1.0 : 0.0;
    }
}
void launch_refine_init(const RefineState& R, int ns, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(refine_init_kernel, dim3(64, ns), dim3(256), 0, st, R, nrhs);
}

// ------------------------------------------------------------------------
// Load vectors (Sec. 2: <f, phi_i>) for many right-hand sides, gathered per
// DOF over its cells (deterministic).
//   FOURIER: f_c = sum_m coef[c][m] psi_m, 2D psi_m(x) = cos(pi (k1 x1 + k2 x2))
//   with m = 4 k1 + k2, k1, k2 in 0..3; 1D psi_m(x) = cos(pi m x), m < 16.
//   Order-4 collapsed Gauss rule per triangle (4-point Gauss-Legendre per
//   segment); the 16 mode integrals g_m = int psi_m phi_i are formed first.
//   NODAL: f = P1 interpolant of nodal values; b = M f exactly
//   (M^K_ab = |K| (1 + delta_ab) / ((d+1)(d+2))).
__global__ void load_fourier_kernel(LoadArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int v = a.dof_node[i];
    double g[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) g[m] = 0.0;
    const int nper = a.dim + 1;
    for (int e = a.v2c_ptr[v]; e < a.v2c_ptr[v + 1]; ++e) {
        const int K = a.v2c_idx[e];
        const int loc = a.vloc[e];
        const double meas = a.meas[K];
        if (a.dim == 2) {
            const double x0 = a.E.x[0][K], y0 = a.E.x[1][K], x1 = a.E.x[2][K], y1 = a.E.x[3][K],
                         x2 = a.E.x[4][K], y2 = a.E.x[5][K];
            for (int q = 0; q < a.nq; ++q) {
                const double l1 = a.q[4 * q], l2 = a.q[4 * q + 1], w = a.q[4 * q + 2];
                const double l0 = 1.0 - l1 - l2;
                const double lam = loc == 0 ? l0 : (loc == 1 ? l1 : l2);
                const double px = l0 * x0 + l1 * x1 + l2 * x2, py = l0 * y0 + l1 * y1 + l2 * y2;
                const double wt = w * meas * lam;
#pragma unroll
                for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
                    for (int k2 = 0; k2 < 4; ++k2) g[4 * k1 + k2] += wt * cos(M_PI * (k1 * px + k2 * py));
            }
        } else {
            const double x0 = a.E.x[0][K], x1 = a.E.x[1][K];
            for (int q = 0; q < a.nq; ++q) {
                const double t = a.q[4 * q], w = a.q[4 * q + 2];
                const double lam = loc == 0 ? 1.0 - t : t;
                const double px = x0 + t * (x1 - x0);
                const double wt = w * meas * lam;
#pragma unroll
                for (int m = 0; m < 16; ++m) g[m] += wt * cos(M_PI * m * px);
            }
        }
        (void)nper;
    }
    for (int c = 0; c < a.nrhs; ++c) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < 16; ++m) s += a.coef[16 * c + m] * g[m];
        a.b[(long long)c * a.n + i] = s;
    }
}

__global__ void load_nodal_kernel(LoadArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int v = a.dof_node[i];  // owner of the (cell, local vertex) list
    const int nper = a.dim + 1;
    const double den = a.dim == 2 ? 12.0 : 6.0;
    for (int c = 0; c < a.nrhs; ++c) {
        const double* f = a.coef + (long long)c * a.nv;
        double s = 0.0;
        for (int e = a.v2c_ptr[v]; e < a.v2c_ptr[v + 1]; ++e) {
            const int K = a.v2c_idx[e];
            double sum = 0.0;
            for (int b = 0; b < nper; ++b) sum += f[a.E.vid[b][K]];
            // the hat function's own vertex (v itself, or its image under a
            // symmetry reduction)
            s += a.meas[K] / den * (sum + f[a.E.vid[a.vloc[e]][K]]);
        }
        a.b[(long long)c * a.n + i] = s;
    }
}

void launch_load(const LoadArgs& a, int kind, hipStream_t st) {
    if (a.n <= 0) return;
    const unsigned g = (unsigned)((a.n + 127) / 128);
    if (kind == FL_RHS_FOURIER16) hipLaunchKernelGGL(load_fourier_kernel, dim3(g), dim3(128), 0, st, a);
    else hipLaunchKernelGGL(load_nodal_kernel, dim3(g), dim3(128), 0, st, a);
}

}  // namespace fl
