// Host side of the batched calls in include/fraclap.h: several fractional
// orders and many right-hand sides at once (load vectors, MFMA products,
// batched Jacobi-PCG with FP64 iterative refinement, GEMM autotuner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fl_handle.hpp"
#include "fl_internal.hpp"
#include "fl_quad.hpp"

using namespace fl;

namespace {

int bfail(fl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return bfail(h, FL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
int grow(fl_handle* h, T** p, size_t* cap, size_t bytes) {
    if (*cap >= bytes && *p) return FL_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) return bfail(h, FL_ENOMEM, std::string("device allocation: ") + hipGetErrorString(e));
    *p = (T*)q;
    *cap = std::max<size_t>(bytes, 256);
    return FL_OK;
}

constexpr int KSPLIT_MAX = 8;

// bump allocator over the batch workspace (256-byte aligned parts)
struct Bump {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += ((bytes + 255) / 256) * 256;
        return o;
    }
};

int gd_of(int dtype) { return dtype == FL_F64 ? GD_F64 : (dtype == FL_F32 ? GD_F32 : GD_BF16); }
int npa_of(int dtype) { return dtype == FL_BF16X2 ? 2 : 1; }
bool valid_dtype(int d) { return d == FL_F64 || d == FL_F32 || d == FL_BF16 || d == FL_BF16X2; }

// FP32 / bf16 copies of the batch matrices, made once per assembly
int ensure_planes(fl_handle* h, int dtype) {
    fl_batch& B = h->B;
    const size_t el = (size_t)B.ns * B.n_pad * B.ld;
    int rc = FL_OK;
    if (dtype == FL_F32 && !B.have32) {
        if ((rc = grow(h, &B.A32, &B.A32_cap, el * sizeof(float)))) return rc;
        for (int j = 0; j < B.ns; ++j)
            launch_mat_lo(B.A64 + (size_t)j * B.n_pad * B.ld, B.ld, B.n, B.n_pad, B.ld, GD_F32, 1,
                          B.A32 + (size_t)j * B.n_pad * B.ld, nullptr, h->stream);
        HIPCHK(hipGetLastError());
        B.have32 = true;
    }
    const bool need_hi = (dtype == FL_BF16 || dtype == FL_BF16X2) && !B.havehi;
    const bool need_lo = dtype == FL_BF16X2 && !B.havelo;
    if (need_hi || need_lo) {
        if ((rc = grow(h, &B.Ahi, &B.Ahi_cap, el * 2))) return rc;
        if (need_lo && (rc = grow(h, &B.Alo, &B.Alo_cap, el * 2))) return rc;
        for (int j = 0; j < B.ns; ++j) {
            const size_t o = (size_t)j * B.n_pad * B.ld;
            launch_mat_lo(B.A64 + o, B.ld, B.n, B.n_pad, B.ld, GD_BF16, need_lo ? 2 : 1,
                          (char*)B.Ahi + 2 * o, need_lo ? (char*)B.Alo + 2 * o : nullptr, h->stream);
        }
        HIPCHK(hipGetLastError());
        B.havehi = true;
        if (need_lo) B.havelo = true;
    }
    return FL_OK;
}

// GEMM arguments for systems j0 .. j0+nsys-1 of the batch in `dtype`
GemmArgs gemm_args(const fl_batch& B, int dtype, int j0, int nsys) {
    GemmArgs g{};
    g.nsys = nsys;
    for (int i = 0; i < nsys; ++i) g.sys[i] = i;
    g.ksplit = 1;
    g.n_pad = B.n_pad;
    g.lda = B.ld;
    g.sA = B.n_pad * B.ld;
    const size_t o = (size_t)j0 * B.n_pad * B.ld;
    if (dtype == FL_F64) g.A = B.A64 + o;
    else if (dtype == FL_F32) g.A = B.A32 + o;
    else {
        g.A = (const char*)B.Ahi + 2 * o;
        if (dtype == FL_BF16X2) g.A2 = (const char*)B.Alo + 2 * o;
    }
    g.sX = 64 * B.n_pad;
    return g;
}

// workspace of the tuner / product: X (and bf16 planes), Y for all systems
struct MatWs {
    void* X;
    void* Xh;
    void* Xl;
    void* Y;
};
int ensure_ws(fl_handle* h, size_t bytes) {
    return grow(h, &h->B.ws, &h->B.ws_cap, bytes);
}
int product_ws(fl_handle* h, int dtype, int nsys, MatWs* W) {
    fl_batch& B = h->B;
    const size_t V = (size_t)nsys * 64 * B.n_pad;
    const size_t xs = dtype == FL_F64 ? 8 : 4;
    Bump b;
    const size_t oX = b.take(V * xs), oH = b.take(dtype >= FL_BF16 ? V * 2 : 0),
                 oL = b.take(dtype >= FL_BF16 ? V * 2 : 0), oY = b.take(V * xs);
    int rc = ensure_ws(h, b.off);
    if (rc) return rc;
    W->X = B.ws + oX;
    W->Xh = B.ws + oH;
    W->Xl = B.ws + oL;
    W->Y = B.ws + oY;
    return FL_OK;
}

// time every configuration of dtype on the whole batch, keep the fastest
int tune(fl_handle* h, int dtype, std::vector<fl_tune_entry>* table) {
    fl_batch& B = h->B;
    int rc = ensure_planes(h, dtype);
    if (rc) return rc;
    MatWs W;
    if ((rc = product_ws(h, dtype, B.ns, &W))) return rc;
    const long long V = (long long)B.ns * 64 * B.n_pad;
    if (dtype == FL_F64) launch_fill_f64((double*)W.X, V, h->stream);
    else launch_fill_f32((float*)W.X, V, h->stream);
    if (dtype >= FL_BF16) launch_split_bf16((const float*)W.X, V, W.Xh, W.Xl, h->stream);
    GemmArgs g = gemm_args(B, dtype, 0, B.ns);
    g.X = dtype >= FL_BF16 ? W.Xh : W.X;
    g.X2 = W.Xl;
    g.Y = W.Y;
    g.epi = 0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const double n = (double)B.n;
    const double abytes = (double)B.ns * n * n * (dtype == FL_F64 ? 8.0 : dtype == FL_F32 ? 4.0 : 2.0 * npa_of(dtype));
    const double flops = 2.0 * n * n * 64.0 * B.ns;
    int best = -1;
    double best_ms = 1e300;
    for (int id = 0; id < gemm_count(); ++id) {
        GemmInfo gi = gemm_info(id);
        if (gi.dt != gd_of(dtype) || gi.npa != npa_of(dtype)) continue;
        HIPCHK(launch_gemm(id, g, h->stream));
        const int reps = 3;
        HIPCHK(hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) HIPCHK(launch_gemm(id, g, h->stream));
        HIPCHK(hipEventRecord(e1, h->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const double t = ms / reps;
        if (table) {
            fl_tune_entry te{};
            te.wm = gi.wm;
            te.waves = gi.waves;
            te.bk = gi.bk;
            te.planes = gi.npa;
            te.ms = t;
            te.tflops = flops / (t * 1e-3) / 1e12;
            te.gbps = abytes / (t * 1e-3) / 1e9;
            table->push_back(te);
        }
        if (t < best_ms) {
            best_ms = t;
            best = id;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return bfail(h, FL_EINVAL, "no GEMM configuration for this element type");
    B.best[dtype] = best;
    return FL_OK;
}

int ensure_tuned(fl_handle* h, int dtype) {
    if (h->B.best[dtype] >= 0) return FL_OK;
    return tune(h, dtype, nullptr);
}

int need_batch(fl_handle* h) {
    if (h->B.ns <= 0) return bfail(h, FL_ESTATE, "fl_assemble_batch must be called first");
    return FL_OK;
}

// active columns in total (*out) and the systems that still have one
// (written as the launch list of g, if given)
int count_active(fl_handle* h, const int* act, int ns, int* out, GemmArgs* g = nullptr) {
    fl_batch& B = h->B;
    if (!B.hflag) HIPCHK(hipHostMalloc((void**)&B.hflag, 256, 0));
    int* dcount = (int*)(B.ws + B.ws_cap - 256);  // last 256 bytes of the workspace
    launch_count(act, ns, dcount, h->stream);
    HIPCHK(hipMemcpyAsync(B.hflag, dcount, sizeof(int) * (1 + ns), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *out = B.hflag[0];
    if (g) {
        g->nsys = 0;
        for (int j = 0; j < ns; ++j)
            if (B.hflag[1 + j] > 0) g->sys[g->nsys++] = j;
    }
    return FL_OK;
}

// K split for a CG product over the active systems of g: aim at >= 1024
// workgroups, keep >= 4 K stages per split, at most `cap` splits
int choose_ksplit(const fl_batch& B, int id, int nsys, int cap) {
    const GemmInfo gi = gemm_info(id);
    const long long work = (long long)nsys * (B.n_pad / gi.bm);
    const long long nk = B.n_pad / gi.bk;
    int k = 1;
    while (k < cap && work * k < 1024 && nk / (2 * k) >= 4) k *= 2;
    return k;
}

}  // namespace

extern "C" {

int fl_load_vector(fl_handle* h, int kind, const double* coeffs, int64_t nrhs, double* b) {
    if (!h) return FL_EINVAL;
    if (!h->planned) return bfail(h, FL_ESTATE, "no assembly");
    if (kind != FL_RHS_ONE && kind != FL_RHS_FOURIER16 && kind != FL_RHS_P1_NODAL)
        return bfail(h, FL_EINVAL, "unknown right-hand-side kind");
    if (nrhs < 0) return bfail(h, FL_EINVAL, "nrhs < 0");
    const int64_t n = h->n;
    if (n == 0 || nrhs == 0) return FL_OK;
    if (!b) return bfail(h, FL_EINVAL, "null output");
    if (kind != FL_RHS_ONE && !coeffs) return bfail(h, FL_EINVAL, "null coefficients");
    if (nrhs > (int64_t)1 << 20) return bfail(h, FL_EINVAL, "nrhs too large");
    HIPCHK(hipSetDevice(h->device));
    if (kind == FL_RHS_ONE) {
        for (int64_t c = 0; c < nrhs; ++c)
            launch_load_one(h->d_dof_node, h->d_v2c_ptr, h->d_v2c_idx, h->d_meas, h->dim, n, b + c * n, h->stream);
        HIPCHK(hipGetLastError());
        return FL_OK;
    }
    // rule: order-4 collapsed Gauss (2D) / 4-point Gauss-Legendre (1D)
    std::vector<double> q;
    if (h->dim == 2) {
        double ux[4], uw[4], vx[4], vw[4];
        gauss_jacobi01(4, 1.0, 0.0, ux, uw);
        gauss_jacobi01(4, 0.0, 0.0, vx, vw);
        for (int i = 0; i < 4; ++i)
            for (int jj = 0; jj < 4; ++jj) {
                q.push_back(ux[i]);
                q.push_back((1.0 - ux[i]) * vx[jj]);
                q.push_back(2.0 * uw[i] * vw[jj]);
                q.push_back(0.0);
            }
    } else {
        double tx[4], tw[4];
        gauss_jacobi01(4, 0.0, 0.0, tx, tw);
        for (int i = 0; i < 4; ++i) {
            q.push_back(tx[i]);
            q.push_back(0.0);
            q.push_back(tw[i]);
            q.push_back(0.0);
        }
    }
    const size_t ncoef = kind == FL_RHS_FOURIER16 ? (size_t)nrhs * 16 : (size_t)h->nv * nrhs;
    for (size_t i = 0; i < ncoef; ++i)
        if (!std::isfinite(coeffs[i])) return bfail(h, FL_ENONFINITE, "non-finite coefficient");
    void* dq = nullptr;
    HIPCHK(hipMalloc(&dq, sizeof(double) * (q.size() + ncoef)));
    hipError_t e = hipMemcpyAsync(dq, q.data(), sizeof(double) * q.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((double*)dq + q.size(), coeffs, sizeof(double) * ncoef, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
        (void)hipFree(dq);
        return bfail(h, FL_EDEVICE, std::string("copy: ") + hipGetErrorString(e));
    }
    LoadArgs a{};
    a.E = h->E;
    a.dim = h->dim;
    a.n = n;
    a.nv = h->nv;
    a.dof_node = h->d_dof_node;
    a.v2c_ptr = h->d_v2c_ptr;
    a.v2c_idx = h->d_v2c_idx;
    a.vloc = h->d_vloc;
    a.meas = h->d_meas;
    a.nq = (int)(q.size() / 4);
    a.q = (const double*)dq;
    a.coef = (const double*)dq + q.size();
    a.nrhs = (int)nrhs;
    a.b = b;
    launch_load(a, kind, h->stream);
    e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(dq);
    if (e != hipSuccess || e2 != hipSuccess)
        return bfail(h, FL_EDEVICE, std::string("load vector: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    return FL_OK;
}

int fl_export_batch_matrix(fl_handle* h, int j, double* dst, int64_t ld, int on_device) {
    if (!h) return FL_EINVAL;
    int rc = need_batch(h);
    if (rc) return rc;
    fl_batch& B = h->B;
    if (j < 0 || j >= B.ns) return bfail(h, FL_EINVAL, "matrix index out of range");
    if (B.n == 0) return FL_OK;
    if (!dst) return bfail(h, FL_EINVAL, "null destination");
    if (ld < B.n) return bfail(h, FL_EINVAL, "ld < n");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipMemcpy2DAsync(dst, ld * sizeof(double), B.A64 + (size_t)j * B.n_pad * B.ld, B.ld * sizeof(double),
                            B.n * sizeof(double), B.n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            h->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

int fl_autotune(fl_handle* h, int dtype, fl_tune_entry* out, int max_out, int* n_out, int* best) {
    if (!h) return FL_EINVAL;
    int rc = need_batch(h);
    if (rc) return rc;
    if (!valid_dtype(dtype)) return bfail(h, FL_EINVAL, "unknown element type");
    if (h->B.n == 0) {
        if (n_out) *n_out = 0;
        if (best) *best = -1;
        return FL_OK;
    }
    HIPCHK(hipSetDevice(h->device));
    std::vector<fl_tune_entry> t;
    if ((rc = tune(h, dtype, &t))) return rc;
    int k = 0, bi = -1;
    for (int id = 0, m = 0; id < gemm_count(); ++id) {
        GemmInfo gi = gemm_info(id);
        if (gi.dt != gd_of(dtype) || gi.npa != npa_of(dtype)) continue;
        if (id == h->B.best[dtype]) bi = m;
        ++m;
    }
    if (out)
        for (; k < (int)t.size() && k < max_out; ++k) out[k] = t[k];
    if (n_out) *n_out = (int)t.size();
    if (best) *best = bi;
    return FL_OK;
}

int fl_matmul(fl_handle* h, int s_index, int dtype, const void* X, int64_t ldx, void* Y, int64_t ldy,
              int64_t nrhs) {
    if (!h) return FL_EINVAL;
    int rc = need_batch(h);
    if (rc) return rc;
    fl_batch& B = h->B;
    if (!valid_dtype(dtype)) return bfail(h, FL_EINVAL, "unknown element type");
    if (s_index < -1 || s_index >= B.ns) return bfail(h, FL_EINVAL, "s_index out of range");
    if (nrhs < 0) return bfail(h, FL_EINVAL, "nrhs < 0");
    if (B.n == 0 || nrhs == 0) return FL_OK;
    if (!X || !Y) return bfail(h, FL_EINVAL, "null operand");
    if (X == Y) return bfail(h, FL_EINVAL, "X and Y must not alias");
    if (ldx < B.n || ldy < B.n) return bfail(h, FL_EINVAL, "leading dimension < n");
    HIPCHK(hipSetDevice(h->device));
    if ((rc = ensure_planes(h, dtype))) return rc;
    if ((rc = ensure_tuned(h, dtype))) return rc;
    const int j0 = s_index < 0 ? 0 : s_index, nsys = s_index < 0 ? B.ns : 1;
    MatWs W;
    if ((rc = product_ws(h, dtype, nsys, &W))) return rc;
    const long long V = (long long)nsys * 64 * B.n_pad;
    GemmArgs g = gemm_args(B, dtype, j0, nsys);
    g.X = dtype >= FL_BF16 ? W.Xh : W.X;
    g.X2 = W.Xl;
    g.Y = W.Y;
    g.epi = 0;
    const long long sx = s_index < 0 ? ldx * nrhs : 0, sy = s_index < 0 ? ldy * nrhs : 0;
    for (int64_t c0 = 0; c0 < nrhs; c0 += 64) {
        const int nc = (int)std::min<int64_t>(64, nrhs - c0);
        if (dtype == FL_F64) {
            launch_pack_f64((const double*)X + c0 * ldx, ldx, sx, B.n, nc, B.n_pad, nsys, (double*)W.X, h->stream);
        } else {
            launch_pack_f32((const float*)X + c0 * ldx, ldx, sx, B.n, nc, B.n_pad, nsys, (float*)W.X, h->stream);
            if (dtype >= FL_BF16) launch_split_bf16((const float*)W.X, V, W.Xh, W.Xl, h->stream);
        }
        HIPCHK(launch_gemm(B.best[dtype], g, h->stream));
        if (dtype == FL_F64)
            launch_unpack_f64((const double*)W.Y, B.n_pad, B.n, nc, nsys, (double*)Y + c0 * ldy, ldy, sy, h->stream);
        else
            launch_unpack_f32((const float*)W.Y, B.n_pad, B.n, nc, nsys, (float*)Y + c0 * ldy, ldy, sy, h->stream);
        HIPCHK(hipGetLastError());
    }
    return FL_OK;
}

int fl_solve_batch(fl_handle* h, const double* Bm, int64_t ldb, int64_t strideB, double* U, int64_t ldu,
                   int64_t strideU, int64_t nrhs, double rtol, int32_t maxit, int inner, int32_t* iters,
                   double* relres) {
    if (!h) return FL_EINVAL;
    int rc = need_batch(h);
    if (rc) return rc;
    fl_batch& B = h->B;
    const int ns = B.ns;
    if (!valid_dtype(inner)) return bfail(h, FL_EINVAL, "unknown inner element type");
    if (nrhs < 0 || !(rtol >= 0.0) || maxit < 0) return bfail(h, FL_EINVAL, "nrhs, rtol, maxit must be >= 0");
    if (B.n == 0 || nrhs == 0) {
        for (int64_t i = 0; i < (int64_t)ns * nrhs; ++i) {
            if (iters) iters[i] = 0;
            if (relres) relres[i] = 0.0;
        }
        return FL_OK;
    }
    if (!Bm || !U) return bfail(h, FL_EINVAL, "null vector");
    if (ldb < B.n || ldu < B.n) return bfail(h, FL_EINVAL, "leading dimension < n");
    if (strideB < 0 || strideU < 0 || (ns > 1 && strideU < ldu * nrhs) || (strideB > 0 && strideB < ldb * nrhs))
        return bfail(h, FL_EINVAL, "block strides overlap");
    HIPCHK(hipSetDevice(h->device));
    const bool mixed = inner != FL_F64;
    if (mixed && (rc = ensure_planes(h, inner))) return rc;
    if ((rc = ensure_tuned(h, FL_F64))) return rc;
    if (mixed && (rc = ensure_tuned(h, inner))) return rc;
    const int id64 = B.best[FL_F64], idin = B.best[inner];
    const int nrb64 = (int)(B.n_pad / gemm_info(id64).bm);
    const int nrbin = (int)(B.n_pad / gemm_info(idin).bm);

    // workspace
    const size_t V = (size_t)ns * 64 * B.n_pad, NS = (size_t)ns * 64;
    Bump bp;
    const size_t o_b64 = bp.take(V * 8), o_u64 = bp.take(V * 8), o_r64 = bp.take(V * 8 * (mixed ? KSPLIT_MAX : 1)),
                 o_p64 = bp.take(V * 8),
                 o_q64 = bp.take(mixed ? 0 : V * 8 * KSPLIT_MAX), o_d64 = bp.take((size_t)ns * B.n_pad * 8),
                 o_d32 = bp.take((size_t)ns * B.n_pad * 4), o_r32 = bp.take(mixed ? V * 4 : 0),
                 o_x32 = bp.take(mixed ? V * 4 : 0), o_rr32 = bp.take(mixed ? V * 4 : 0),
                 o_p32 = bp.take(mixed ? V * 4 : 0), o_q32 = bp.take(mixed ? V * 4 * KSPLIT_MAX : 0),
                 o_ph = bp.take(mixed && inner >= FL_BF16 ? V * 2 : 0),
                 o_pl = bp.take(mixed && inner >= FL_BF16 ? V * 2 : 0),
                 o_part = bp.take(NS * (size_t)std::max(nrb64, nrbin) * 8),
                 o_ints = bp.take(NS * 8 * 4), o_dbl = bp.take(NS * 8 * 8), o_tail = bp.take(256);
    (void)o_tail;
    if ((rc = ensure_ws(h, bp.off))) return rc;
    char* ws = B.ws;
    double* b64 = (double*)(ws + o_b64);
    double* u64 = (double*)(ws + o_u64);
    double* r64 = (double*)(ws + o_r64);
    double* p64 = (double*)(ws + o_p64);
    double* q64 = (double*)(ws + o_q64);
    double* d64 = (double*)(ws + o_d64);
    float* d32 = (float*)(ws + o_d32);
    int* I = (int*)(ws + o_ints);
    int *oact = I, *want = I + NS, *act = I + 2 * NS, *its = I + 3 * NS, *st_in = I + 4 * NS,
        *st_out = I + 5 * NS, *upd = I + 6 * NS, *lsf = I + 7 * NS;
    double* D = (double*)(ws + o_dbl);
    double *bb = D, *rel = D + NS, *rz = D + 2 * NS, *ibb = D + 3 * NS, *irel = D + 4 * NS,
           *rupd2 = D + 5 * NS, *prv = D + 6 * NS;

    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, h->stream));
    launch_bdiag(B.A64, B.ld, B.n_pad * B.ld, B.n, B.n_pad, ns, d64, d32, h->stream);

    std::vector<int> h_its((size_t)ns * 64), h_tot((size_t)ns * 64), h_st((size_t)ns * 64), h_st2((size_t)ns * 64);
    std::vector<double> h_rel((size_t)ns * 64);
    int status = FL_OK, outer_max = 0;
    const int chunk = 8;
    for (int64_t c0 = 0; c0 < nrhs && status == FL_OK; c0 += 64) {
        const int nc = (int)std::min<int64_t>(64, nrhs - c0);
        launch_pack_f64(Bm + c0 * ldb, ldb, strideB, B.n, nc, B.n_pad, ns, b64, h->stream);
        RefineState R{};
        R.n_pad = B.n_pad;
        R.b64 = b64;
        R.u64 = u64;
        R.r32 = mixed ? (float*)(ws + o_r32) : nullptr;
        R.bb = bb;
        R.oact = oact;
        R.want = want;
        R.status = st_out;
        R.rel = rel;
        launch_refine_init(R, ns, nc, h->stream);  // b.b, outer activity, u = 0
        HIPCHK(hipGetLastError());
        std::fill(h_tot.begin(), h_tot.end(), 0);
        std::fill(h_st.begin(), h_st.end(), 0);
        if (!mixed) {
            BcgState<double> S{};
            S.n_pad = B.n_pad;
            S.x = u64;
            S.r = r64;
            S.p = p64;
            S.q = q64;
            S.b = b64;
            S.dinv = d64;
            S.want = oact;
            S.act = act;
            S.iters = its;
            S.status = st_in;
            S.rz = rz;
            S.bb = ibb;
            S.rel = irel;
            S.partq = (double*)(ws + o_part);
            S.nrbq = nrb64;
            S.rtol2 = rtol * rtol;
            S.maxit = maxit;
            launch_bcg_init(S, ns, h->stream);
            GemmArgs g = gemm_args(B, FL_F64, 0, ns);
            g.X = p64;
            g.Y = q64;
            g.V = p64;
            g.part = (double*)(ws + o_part);
            g.act = act;
            g.epi = 1;
            int nact = 1;
            if ((rc = count_active(h, act, ns, &nact, &g))) return rc;
            for (int it = 0; nact > 0 && it < maxit; it += chunk) {
                const int ks = choose_ksplit(B, id64, g.nsys, KSPLIT_MAX);
                g.ksplit = ks;
                g.epi = ks > 1 ? 0 : 1;
                g.ysplit = (long long)V;
                S.ksplit = ks;
                S.ysplit = (long long)V;
                for (int k = 0; k < chunk; ++k) {
                    HIPCHK(launch_gemm(id64, g, h->stream));
                    launch_bcg_step(S, ns, h->stream);
                }
                HIPCHK(hipGetLastError());
                if ((rc = count_active(h, act, ns, &nact, &g))) return rc;
            }
            HIPCHK(hipMemcpy(h_its.data(), its, sizeof(int) * NS, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(h_st.data(), st_in, sizeof(int) * NS, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(h_rel.data(), irel, sizeof(double) * NS, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < NS; ++i) h_tot[i] = h_its[i];
        } else {
            BcgState<float> S{};
            S.n_pad = B.n_pad;
            S.x = (float*)(ws + o_x32);
            S.r = (float*)(ws + o_rr32);
            S.p = (float*)(ws + o_p32);
            S.q = (float*)(ws + o_q32);
            S.ph = inner >= FL_BF16 ? (void*)(ws + o_ph) : nullptr;
            S.pl = inner >= FL_BF16 ? (void*)(ws + o_pl) : nullptr;
            S.b = R.r32;
            S.dinv = d32;
            S.want = want;
            S.act = act;
            S.iters = its;
            S.status = st_in;
            S.rz = rz;
            S.bb = ibb;
            S.rel = irel;
            S.partq = (double*)(ws + o_part);
            S.nrbq = nrbin;
            S.rtol2 = rtol * rtol;
            S.maxit = maxit;
            S.upd = upd;
            S.rupd2 = rupd2;
            S.lsf = lsf;
            S.pr = prv;
            // replace when |r| fell 100x (10x for the one-plane bf16 matrix,
            // whose products drift faster)
            S.delta2 = inner == FL_BF16 ? 1e-2 : 1e-4;
            GemmArgs gr = gemm_args(B, FL_F64, 0, ns);  // A u (K-split partial products)
            gr.X = u64;
            gr.Y = r64;
            gr.act = upd;
            gr.epi = 0;
            gr.ysplit = (long long)V;
            GemmArgs gi = gemm_args(B, inner, 0, ns);   // q = A p, p.q partials
            gi.X = inner >= FL_BF16 ? S.ph : (const void*)S.p;
            gi.X2 = S.pl;
            gi.Y = S.q;
            gi.V = S.p;
            gi.part = (double*)(ws + o_part);
            gi.act = act;
            gi.epi = 1;
            ReliableState RS{};
            RS.n_pad = B.n_pad;
            RS.b64 = b64;
            RS.y64 = r64;
            RS.ysplit = (long long)V;
            RS.r = S.r;
            RS.dinv = d32;
            RS.rz = rz;
            RS.rupd2 = rupd2;
            RS.bb = bb;
            RS.p = S.p;
            RS.pr = prv;
            RS.lsf = lsf;
            RS.act = act;
            RS.upd = upd;
            RS.iters = its;
            RS.status = st_out;
            RS.rel = rel;
            RS.rtol2 = rtol * rtol;
            RS.maxit = maxit;
            launch_bcg_init(S, ns, h->stream);       // r = fp32(b), x = 0, p = D^-1 r
            int nact = 0, nupd = 0, replacements = 0;
            if ((rc = count_active(h, act, ns, &nact, &gi))) return rc;
            for (long long guard = 0; (nact > 0 || nupd > 0) && guard <= (long long)maxit + 64; guard += chunk) {
                if (nact > 0) {
                    const int ks = choose_ksplit(B, idin, gi.nsys, KSPLIT_MAX);
                    gi.ksplit = ks;
                    gi.epi = ks > 1 ? 0 : 1;
                    gi.ysplit = (long long)V;
                    S.ksplit = ks;
                    S.ysplit = (long long)V;
                    for (int k = 0; k < chunk; ++k) {
                        HIPCHK(launch_gemm(idin, gi, h->stream));
                        launch_bcg_step(S, ns, h->stream);
                    }
                    HIPCHK(hipGetLastError());
                }
                if ((rc = count_active(h, upd, ns, &nupd, &gr))) return rc;
                if (nupd > 0) {
                    // u += x in FP64, r = b - A u with the FP64 matrix
                    launch_corr_masked(u64, S.x, upd, B.n_pad, ns, h->stream);
                    gr.ksplit = RS.ksplit = choose_ksplit(B, id64, gr.nsys, KSPLIT_MAX);
                    HIPCHK(launch_gemm(id64, gr, h->stream));
                    launch_reliable(RS, ns, h->stream);
                    HIPCHK(hipGetLastError());
                    ++replacements;
                    nupd = 0;
                }
                if ((rc = count_active(h, act, ns, &nact, &gi))) return rc;
            }
            outer_max = std::max(outer_max, replacements);
            HIPCHK(hipMemcpy(h_its.data(), its, sizeof(int) * NS, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(h_rel.data(), rel, sizeof(double) * NS, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(h_st.data(), st_in, sizeof(int) * NS, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(h_st2.data(), st_out, sizeof(int) * NS, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < NS; ++i) {
                h_tot[i] = h_its[i];
                if (h_st2[i]) h_st[i] = h_st2[i];
            }
        }
        launch_unpack_f64(u64, B.n_pad, B.n, nc, ns, U + c0 * ldu, ldu, strideU, h->stream);
        HIPCHK(hipGetLastError());
        for (int j = 0; j < ns; ++j)
            for (int c = 0; c < nc; ++c) {
                const size_t i = (size_t)j * 64 + c, o = (size_t)j * nrhs + c0 + c;
                if (iters) iters[o] = h_tot[i];
                if (relres) relres[o] = h_rel[i];
                if (h_st[i] == 2) status = FL_ENONFINITE;
                else if (h_st[i] == 1 && status != FL_ENONFINITE) status = FL_EBREAKDOWN;
                else if (!(h_rel[i] <= rtol) && status == FL_OK) status = FL_ENOCONV;
            }
    }
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->st.t_solve_ms = ms;
    h->st.last_outer = outer_max;
    if (status == FL_EBREAKDOWN) return bfail(h, FL_EBREAKDOWN, "CG breakdown: p.Ap <= 0");
    if (status == FL_ENONFINITE) return bfail(h, FL_ENONFINITE, "non-finite data in the solve");
    return status;
}

}  // extern "C"
