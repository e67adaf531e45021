// Host side of the learned pair-integral surrogate (include/fraclap.h):
// data generation, initialisation, scaling, training, inference,
// certification and the surrogate parameters of an assembly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fl_handle.hpp"
#include "fl_internal.hpp"

using namespace fl;

namespace {

int sfail(fl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return sfail(h, FL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int NHALF = SUR_NH * SUR_KIN + SUR_NH * SUR_NH + SUR_KOUT * SUR_NH + SUR_NH * SUR_NH + SUR_NH * SUR_KOUT;
constexpr int NSCAL = 2 * SUR_NIN + 2 * SUR_NOUT;
constexpr int NSTAT_BLK = 256;
constexpr size_t WS_DOUBLES = (size_t)NSTAT_BLK * SUR_NOUT * 3 + 4096;
constexpr double SAFETY = 1.25;
constexpr unsigned MIN_BIN = 32;

template <class T>
int grow(fl_handle* h, T** p, size_t* cap, size_t bytes) {
    if (*p && *cap >= bytes) return FL_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    void* q = nullptr;
    if (hipMalloc(&q, bytes < 256 ? 256 : bytes) != hipSuccess) return sfail(h, FL_ENOMEM, "device allocation failed");
    *p = (T*)q;
    *cap = bytes < 256 ? 256 : bytes;
    return FL_OK;
}

int alloc_net(fl_handle* h) {
    fl_sur& S = h->sur;
    if (S.theta) return FL_OK;
    HIPCHK(hipMalloc((void**)&S.theta, sizeof(float) * SUR_NPARAM));
    HIPCHK(hipMalloc((void**)&S.m, sizeof(float) * SUR_NPARAM));
    HIPCHK(hipMalloc((void**)&S.v, sizeof(float) * SUR_NPARAM));
    HIPCHK(hipMalloc((void**)&S.half, sizeof(_Float16) * NHALF));
    HIPCHK(hipMalloc((void**)&S.scal, sizeof(float) * NSCAL));
    HIPCHK(hipMalloc((void**)&S.ws, sizeof(double) * WS_DOUBLES));
    return FL_OK;
}

SurHalves halves(fl_handle* h) {
    _Float16* p = h->sur.half;
    SurHalves H;
    H.W1 = p;
    H.W2 = H.W1 + SUR_NH * SUR_KIN;
    H.W3 = H.W2 + SUR_NH * SUR_NH;
    H.W2T = H.W3 + SUR_KOUT * SUR_NH;
    H.W3T = H.W2T + SUR_NH * SUR_NH;
    return H;
}

SurNet net(fl_handle* h) {
    const SurHalves H = halves(h);
    SurNet N;
    N.W1 = H.W1;
    N.W2 = H.W2;
    N.W3 = H.W3;
    N.b1 = h->sur.theta + SUR_OB1;
    N.b2 = h->sur.theta + SUR_OB2;
    N.b3 = h->sur.theta + SUR_OB3;
    N.mx = h->sur.scal;
    N.isx = N.mx + SUR_NIN;
    N.mt = N.isx + SUR_NIN;
    N.st = N.mt + SUR_NOUT;
    return N;
}

int upload_scaling(fl_handle* h) {
    fl_sur& S = h->sur;
    float sc[NSCAL];
    for (int k = 0; k < SUR_NIN; ++k) {
        sc[k] = (float)S.mx[k];
        sc[SUR_NIN + k] = (float)(1.0 / S.sx[k]);
    }
    for (int j = 0; j < SUR_NOUT; ++j) {
        sc[2 * SUR_NIN + j] = (float)S.mt[j];
        sc[2 * SUR_NIN + SUR_NOUT + j] = (float)S.st[j];
    }
    HIPCHK(hipMemcpyAsync(S.scal, sc, sizeof(sc), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

int reset_adam(fl_handle* h) {
    HIPCHK(hipMemsetAsync(h->sur.m, 0, sizeof(float) * SUR_NPARAM, h->stream));
    HIPCHK(hipMemsetAsync(h->sur.v, 0, sizeof(float) * SUR_NPARAM, h->stream));
    h->sur.adam_t = 0;
    return FL_OK;
}

int upload_theta(fl_handle* h, const std::vector<float>& th) {
    HIPCHK(hipMemcpyAsync(h->sur.theta, th.data(), sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice,
                          h->stream));
    launch_sur_halves(h->sur.theta, halves(h), h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

unsigned long long splitmix64(unsigned long long& x) {
    unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int check_pairs(fl_handle* h, int64_t m, const void* X, const void* Y, const void* s, const void* out) {
    if (!h) return FL_EINVAL;
    if (m < 0) return sfail(h, FL_EINVAL, "m must be >= 0");
    if (m > 0 && (!X || !Y || !s || !out)) return sfail(h, FL_EINVAL, "null device pointer");
    return FL_OK;
}

int need_net(fl_handle* h, bool scaling) {
    if (!h->sur.have) return sfail(h, FL_ESTATE, "no surrogate network (fl_surrogate_init / set_params)");
    if (scaling && !h->sur.have_scaling)
        return sfail(h, FL_ESTATE, "no surrogate scaling (fl_surrogate_fit_scaling / set_params)");
    return FL_OK;
}

}  // namespace

int fl_sur_params(fl_handle* h, double s, const fl_opts& o, SurParams* sp) {
    fl_sur& S = h->sur;
    if (!S.have || !S.have_scaling)
        return sfail(h, FL_ESTATE, "surrogate assembly needs a network with scaling (fl_surrogate_*)");
    SurParams& B = *sp;
    B.nsur = o.surrogate;
    B.s = s;
    B.N = net(h);
    for (int k = 0; k < SUR_NIN; ++k) {
        B.lo[k] = S.lo[k];
        B.hi[k] = S.hi[k];
    }
    const int sb = (s >= 0.25) + (s >= 0.5) + (s >= 0.75);
    for (int rb = 0; rb < SUR_NRB; ++rb) B.use_rbin[rb] = S.bound[rb * SUR_NSB + sb] <= o.sur_tol ? 1 : 0;
    return FL_OK;
}

void fl_sur_free(fl_handle* h) {
    fl_sur& S = h->sur;
    for (void* p : {(void*)S.theta, (void*)S.m, (void*)S.v, (void*)S.half, (void*)S.scal, (void*)S.part,
                    (void*)S.loss, (void*)S.ws})
        if (p) (void)hipFree(p);
    S = fl_sur{};
}

extern "C" {

int fl_default_train_opts(fl_train_opts* out) {
    if (!out) return FL_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->steps = 20000;
    out->batch = 1024;
    out->lr = 3e-3;
    out->lr_min = 1e-5;
    out->beta1 = 0.9;
    out->beta2 = 0.999;
    out->eps = 1e-8;
    out->seed = 1;
    return FL_OK;
}

int fl_pair_integrals(fl_handle* h, int64_t m, const double* X, const double* Y, const double* s, int k,
                      double* out) {
    int rc = check_pairs(h, m, X, Y, s, out);
    if (rc) return rc;
    if (k < 1 || k > FL_MAX_ORDER_FAR) return sfail(h, FL_EINVAL, "k must lie in 1..8");
    if (m == 0) return FL_OK;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(upload_rules(fl_base_rules(), h->stream));
    launch_pair_integrals(X, Y, s, m, k, 0, out, nullptr, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_surrogate_dataset(fl_handle* h, int64_t m, const double* X, const double* Y, const double* s,
                         int k_exact, double* feats, double* targets) {
    int rc = check_pairs(h, m, X, Y, s, targets);
    if (rc) return rc;
    if (m > 0 && !feats) return sfail(h, FL_EINVAL, "null device pointer");
    if (k_exact < 3 || k_exact > FL_MAX_ORDER_FAR) return sfail(h, FL_EINVAL, "k_exact must lie in 3..8");
    if (m == 0) return FL_OK;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(upload_rules(fl_base_rules(), h->stream));
    launch_pair_integrals(X, Y, s, m, k_exact, 1, targets, feats, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_surrogate_init(fl_handle* h, uint64_t seed) {
    if (!h) return FL_EINVAL;
    HIPCHK(hipSetDevice(h->device));
    int rc = alloc_net(h);
    if (rc) return rc;
    std::vector<float> th(SUR_NPARAM, 0.f);
    unsigned long long x = seed;
    auto fill = [&](int off, int rows, int cols, int ld, int fan_in, int fan_out) {
        const double lim = std::sqrt(6.0 / (fan_in + fan_out));
        for (int i = 0; i < rows; ++i)
            for (int j = 0; j < cols; ++j) {
                const double u = (double)(splitmix64(x) >> 11) * (1.0 / 9007199254740992.0);
                th[off + i * ld + j] = (float)(lim * (2.0 * u - 1.0));
            }
    };
    fill(SUR_OW1, SUR_NH, SUR_NIN, SUR_KIN, SUR_NIN, SUR_NH);
    fill(SUR_OW2, SUR_NH, SUR_NH, SUR_NH, SUR_NH, SUR_NH);
    fill(SUR_OW3, SUR_NOUT, SUR_NH, SUR_NH, SUR_NH, SUR_NOUT);
    rc = upload_theta(h, th);
    if (rc) return rc;
    rc = reset_adam(h);
    if (rc) return rc;
    h->sur.have = true;
    h->sur.have_scaling = false;
    for (double& b : h->sur.bound) b = INFINITY;
    return FL_OK;
}

int fl_surrogate_fit_scaling(fl_handle* h, const double* feats, const double* targets, int64_t m) {
    if (!h) return FL_EINVAL;
    int rc = need_net(h, false);
    if (rc) return rc;
    if (m < 1 || !feats || !targets) return sfail(h, FL_EINVAL, "need m >= 1 samples");
    HIPCHK(hipSetDevice(h->device));
    fl_sur& S = h->sur;
    double* part = S.ws;
    double* res = S.ws + (size_t)NSTAT_BLK * SUR_NOUT * 3;  // 3 x 21
    double* mean_d = res + 3 * SUR_NOUT;                       // 21
    double hr[3 * SUR_NOUT];
    for (int pass = 0; pass < 2; ++pass) {
        const double* X = pass ? targets : feats;
        const int nc = pass ? SUR_NOUT : SUR_NIN;
        double mean[SUR_NOUT];
        launch_sur_colstat(X, m, nc, nullptr, part, NSTAT_BLK, res, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hr, res, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int c = 0; c < nc; ++c) mean[c] = hr[3 * c] / (double)m;
        if (!pass)
            for (int c = 0; c < nc; ++c) {
                S.lo[c] = hr[3 * c + 1];
                S.hi[c] = hr[3 * c + 2];
            }
        HIPCHK(hipMemcpyAsync(mean_d, mean, sizeof(double) * nc, hipMemcpyHostToDevice, h->stream));
        launch_sur_colstat(X, m, nc, mean_d, part, NSTAT_BLK, res, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hr, res, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int c = 0; c < nc; ++c) {
            const double sd = std::max(std::sqrt(hr[3 * c] / (double)m), 1e-12);
            if (pass) {
                S.mt[c] = mean[c];
                S.st[c] = sd;
            } else {
                S.mx[c] = mean[c];
                S.sx[c] = sd;
            }
        }
    }
    rc = upload_scaling(h);
    if (rc) return rc;
    S.have_scaling = true;
    return FL_OK;
}

int fl_surrogate_set_params(fl_handle* h, const double* blob) {
    if (!h) return FL_EINVAL;
    if (!blob) return sfail(h, FL_EINVAL, "null blob");
    HIPCHK(hipSetDevice(h->device));
    int rc = alloc_net(h);
    if (rc) return rc;
    fl_sur& S = h->sur;
    std::vector<float> th(SUR_NPARAM);
    for (int p = 0; p < SUR_NPARAM; ++p) th[p] = (float)blob[p];
    const double* q = blob + SUR_NPARAM;
    for (int k = 0; k < SUR_NIN; ++k) {
        S.mx[k] = q[k];
        S.sx[k] = q[SUR_NIN + k];
        if (!(S.sx[k] > 0.0)) return sfail(h, FL_EINVAL, "feature deviations must be positive");
    }
    q += 2 * SUR_NIN;
    for (int j = 0; j < SUR_NOUT; ++j) {
        S.mt[j] = q[j];
        S.st[j] = q[SUR_NOUT + j];
    }
    q += 2 * SUR_NOUT;
    for (int k = 0; k < SUR_NIN; ++k) {
        S.lo[k] = q[k];
        S.hi[k] = q[SUR_NIN + k];
    }
    q += 2 * SUR_NIN;
    for (int b = 0; b < SUR_NRB * SUR_NSB; ++b) S.bound[b] = q[b];
    rc = upload_theta(h, th);
    if (rc) return rc;
    rc = upload_scaling(h);
    if (rc) return rc;
    rc = reset_adam(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    S.have = S.have_scaling = true;
    return FL_OK;
}

int fl_surrogate_get_params(fl_handle* h, double* blob) {
    if (!h) return FL_EINVAL;
    if (!blob) return sfail(h, FL_EINVAL, "null blob");
    int rc = need_net(h, false);
    if (rc) return rc;
    fl_sur& S = h->sur;
    std::vector<float> th(SUR_NPARAM);
    HIPCHK(hipMemcpyAsync(th.data(), S.theta, sizeof(float) * SUR_NPARAM, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int p = 0; p < SUR_NPARAM; ++p) blob[p] = th[p];
    double* q = blob + SUR_NPARAM;
    for (int k = 0; k < SUR_NIN; ++k) {
        q[k] = S.mx[k];
        q[SUR_NIN + k] = S.sx[k];
    }
    q += 2 * SUR_NIN;
    for (int j = 0; j < SUR_NOUT; ++j) {
        q[j] = S.mt[j];
        q[SUR_NOUT + j] = S.st[j];
    }
    q += 2 * SUR_NOUT;
    for (int k = 0; k < SUR_NIN; ++k) {
        q[k] = S.lo[k];
        q[SUR_NIN + k] = S.hi[k];
    }
    q += 2 * SUR_NIN;
    for (int b = 0; b < SUR_NRB * SUR_NSB; ++b) q[b] = S.bound[b];
    return FL_OK;
}

int fl_surrogate_grad(fl_handle* h, const double* feats, const double* targets, int64_t m, float* grad,
                      double* loss) {
    if (!h) return FL_EINVAL;
    int rc = need_net(h, true);
    if (rc) return rc;
    if (m < 1 || !feats || !targets) return sfail(h, FL_EINVAL, "need m >= 1 samples");
    HIPCHK(hipSetDevice(h->device));
    fl_sur& S = h->sur;
    const long long nwg = (m + 63) / 64;
    if (nwg > (1LL << 24)) return sfail(h, FL_EINVAL, "too many samples");
    rc = grow(h, &S.part, &S.part_cap, sizeof(float) * SUR_NPARAM * nwg);
    if (rc) return rc;
    rc = grow(h, &S.loss, &S.loss_cap, sizeof(double) * nwg);
    if (rc) return rc;
    SurTrain A{};
    A.F = feats;
    A.T = targets;
    A.m = m;
    A.mode = 1;
    A.base = 0;
    A.N = net(h);
    const SurHalves H = halves(h);
    A.W2T = H.W2T;
    A.W3T = H.W3T;
    A.part = S.part;
    A.loss = S.loss;
    launch_sur_train(A, (int)nwg, h->stream);
    HIPCHK(hipGetLastError());
    SurAdam U{};
    U.part = S.part;
    U.nwg = (int)nwg;
    U.gscale = (float)(2.0 / ((double)m * SUR_NOUT));
    U.update = 0;
    U.grad_out = (float*)S.ws;
    launch_sur_adam(U, h->stream);
    HIPCHK(hipGetLastError());
    std::vector<double> lp(nwg);
    if (grad)
        HIPCHK(hipMemcpyAsync(grad, S.ws, sizeof(float) * SUR_NPARAM, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(lp.data(), S.loss, sizeof(double) * nwg, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double L = 0.0;
    for (double v : lp) L += v;
    if (loss) *loss = L / ((double)m * SUR_NOUT);
    return FL_OK;
}

int fl_surrogate_train(fl_handle* h, const double* feats, const double* targets, int64_t m,
                       const fl_train_opts* opts, double* loss_hist) {
    if (!h) return FL_EINVAL;
    int rc = need_net(h, true);
    if (rc) return rc;
    fl_train_opts o;
    if (opts) o = *opts;
    else fl_default_train_opts(&o);
    if (m < 1 || !feats || !targets) return sfail(h, FL_EINVAL, "need m >= 1 samples");
    if (o.steps < 0 || o.batch < 64 || o.batch % 64 || o.batch > 65536)
        return sfail(h, FL_EINVAL, "steps >= 0, batch a multiple of 64 in 64..65536");
    if (!(o.lr > 0.0) || o.lr_min < 0.0 || !(o.beta1 >= 0.0 && o.beta1 < 1.0) ||
        !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps > 0.0))
        return sfail(h, FL_EINVAL, "bad Adam parameters");
    if (o.steps == 0) return FL_OK;
    HIPCHK(hipSetDevice(h->device));
    fl_sur& S = h->sur;
    const int nwg = o.batch / 64;
    rc = grow(h, &S.part, &S.part_cap, sizeof(float) * SUR_NPARAM * nwg);
    if (rc) return rc;
    rc = grow(h, &S.loss, &S.loss_cap, sizeof(double) * nwg * (size_t)o.steps);
    if (rc) return rc;
    SurTrain A{};
    A.F = feats;
    A.T = targets;
    A.m = m;
    A.mode = 0;
    A.batch = o.batch;
    A.seed = o.seed;
    A.N = net(h);
    const SurHalves H = halves(h);
    A.W2T = H.W2T;
    A.W3T = H.W3T;
    A.part = S.part;
    SurAdam U{};
    U.theta = S.theta;
    U.m = S.m;
    U.v = S.v;
    U.part = S.part;
    U.nwg = nwg;
    U.gscale = (float)(2.0 / ((double)o.batch * SUR_NOUT));
    U.update = 1;
    U.b1 = (float)o.beta1;
    U.b2 = (float)o.beta2;
    U.eps = (float)o.eps;
    U.H = H;
    for (int it = 0; it < o.steps; ++it) {
        const long long t = ++S.adam_t;
        A.step = t;
        A.loss = S.loss + (size_t)it * nwg;
        launch_sur_train(A, nwg, h->stream);
        U.lr = (float)(o.lr_min + 0.5 * (o.lr - o.lr_min) * (1.0 + std::cos(M_PI * it / (double)o.steps)));
        U.bc1 = (float)(1.0 - std::pow(o.beta1, (double)t));
        U.bc2 = (float)(1.0 - std::pow(o.beta2, (double)t));
        launch_sur_adam(U, h->stream);
    }
    HIPCHK(hipGetLastError());
    std::vector<double> lp((size_t)nwg * o.steps);
    HIPCHK(hipMemcpyAsync(lp.data(), S.loss, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (loss_hist)
        for (int it = 0; it < o.steps; ++it) {
            double L = 0.0;
            for (int w = 0; w < nwg; ++w) L += lp[(size_t)it * nwg + w];
            loss_hist[it] = L / ((double)o.batch * SUR_NOUT);
        }
    return FL_OK;
}

int fl_surrogate_predict(fl_handle* h, const double* feats, int64_t m, double* out) {
    if (!h) return FL_EINVAL;
    int rc = need_net(h, true);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!feats || !out))) return sfail(h, FL_EINVAL, "bad arguments");
    if (m == 0) return FL_OK;
    HIPCHK(hipSetDevice(h->device));
    SurPredict P{};
    P.F = feats;
    P.m = m;
    P.N = net(h);
    P.out = out;
    launch_sur_predict(P, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_surrogate_certify(fl_handle* h, const double* feats, const double* targets, int64_t m,
                         double* bound) {
    if (!h) return FL_EINVAL;
    int rc = need_net(h, true);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!feats || !targets))) return sfail(h, FL_EINVAL, "bad arguments");
    HIPCHK(hipSetDevice(h->device));
    fl_sur& S = h->sur;
    unsigned int* bins = (unsigned int*)S.ws;  // emax bits, then counts
    const int NB = SUR_NRB * SUR_NSB;
    HIPCHK(hipMemsetAsync(bins, 0, sizeof(unsigned int) * 2 * NB, h->stream));
    SurPredict P{};
    P.F = feats;
    P.m = m;
    P.N = net(h);
    P.T = targets;
    P.emax_bits = bins;
    P.count = bins + NB;
    launch_sur_predict(P, h->stream);
    HIPCHK(hipGetLastError());
    unsigned int hb[2 * NB];
    HIPCHK(hipMemcpyAsync(hb, bins, sizeof(hb), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int b = 0; b < NB; ++b) {
        float e;
        std::memcpy(&e, &hb[b], sizeof(e));
        S.bound[b] = hb[NB + b] >= MIN_BIN ? SAFETY * (double)e : INFINITY;
        if (bound) bound[b] = S.bound[b];
    }
    return FL_OK;
}

}  // extern "C"
