// Host side of the C ABI in include/fraclap.h: mesh validation, DOF map
// (Sec. 3), element-pair planning (Sec. 5 decomposition into identical /
// common-edge / common-vertex / separated pairs and element/facet pairs),
// quadrature tables (App. B orders), device buffers and kernel launches.
//
// Compiled with -ffp-contract=off: the centroids, squared diameters and
// facet data computed here feed the per-pair order classes, which must be
// reproducible bit for bit from the same formulas.
//
// Every per-assembly input of the kernels is packed into one pinned host
// staging buffer and sent with a single asynchronous copy into one device
// "plan" buffer; device buffers (plan, matrix, scratch) grow on demand and
// are reused by later assemblies on the same handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fl_handle.hpp"
#include "fl_internal.hpp"
#include "fl_quad.hpp"

using namespace fl;

static double* noalloc_scratch(fl_handle* h);

namespace {

int fail(fl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(h, FL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void reset_assembly(fl_handle* h) {
    h->assembled = false;
    h->lower_pending = false;
    h->mg.ready = false;  // the hierarchy belongs to the previous matrix
    h->sf.ready = false;  // so does the strong-form geometry (DOF map)
    h->hm.ready = false;  // and the cluster approximation
    h->planned = false;
    h->B.ns = 0;
    h->n = h->lda = 0;
    h->E = ElemDev{};
    h->d_v2c_ptr = h->d_v2c_idx = h->d_node2dof = h->d_dof_node = nullptr;
    h->d_vloc = nullptr;
    h->d_meas = nullptr;
}

void free_buffers(fl_handle* h) {
    reset_assembly(h);
    if (h->plan) (void)hipFree(h->plan);
    if (h->pin) (void)hipHostFree(h->pin);
    if (h->dA) (void)hipFree(h->dA);
    if (h->dS) (void)hipFree(h->dS);
    if (h->dcnt) (void)hipFree(h->dcnt);
    if (h->dA32) (void)hipFree(h->dA32);
    h->dA32 = nullptr;
    h->A32_cap = 0;
    if (h->dAhi) (void)hipFree(h->dAhi);
    if (h->dSfix) (void)hipFree(h->dSfix);
    h->dAhi = nullptr;
    h->dSfix = nullptr;
    h->Ahi_cap = h->Sfix_cap = 0;
    fl_batch& B = h->B;
    if (B.A64) (void)hipFree(B.A64);
    if (B.A32) (void)hipFree(B.A32);
    if (B.Ahi) (void)hipFree(B.Ahi);
    if (B.Alo) (void)hipFree(B.Alo);
    if (B.ws) (void)hipFree(B.ws);
    if (B.hflag) (void)hipHostFree(B.hflag);
    h->B = fl_batch{};
    h->pc.valid = false;
    h->plan = h->pin = nullptr;
    h->dA = h->dS = nullptr;
    h->dcnt = nullptr;
    h->plan_cap = h->pin_cap = h->A_cap = h->S_cap = 0;
}

void free_solver(fl_handle* h) {
    if (h->w) (void)hipFree(h->w);
    if (h->w_part) (void)hipFree(h->w_part);
    if (h->w_stat) (void)hipFree(h->w_stat);
    if (h->w_hstat) (void)hipHostFree(h->w_hstat);
    if (h->w32) (void)hipFree(h->w32);
    if (h->w_sym) (void)hipFree(h->w_sym);
    h->w32 = nullptr;
    h->w_sym = nullptr;
    h->sym = SymPlan{};
    h->w = h->w_part = nullptr;
    h->w_stat = h->w_hstat = nullptr;
    h->w_n = -1;
}

// grow a device buffer (contents are not preserved)
template <class T>
int ensure_dev(fl_handle* h, T** p, size_t* cap, size_t bytes) {
    if (*cap >= bytes && *p) return FL_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) return fail(h, FL_ENOMEM, std::string("device allocation: ") + hipGetErrorString(e));
    *p = (T*)q;
    *cap = std::max<size_t>(bytes, 256);
    return FL_OK;
}

// Layout of the packed plan: each part is 256-byte aligned.
struct Packer {
    struct Part {
        const void* src;
        size_t bytes, off;
    };
    std::vector<Part> parts;
    size_t total = 0;
    template <class T>
    size_t add(const std::vector<T>& v) {
        size_t off = total;
        parts.push_back({v.data(), v.size() * sizeof(T), off});
        total += ((v.size() * sizeof(T) + 255) / 256) * 256;
        return off;
    }
};

uint64_t morton2(double x, double y, double x0, double y0, double span) {
    auto q = [&](double v, double lo) {
        double t = (v - lo) / span;
        if (t < 0) t = 0;
        if (t > 1) t = 1;
        return (uint64_t)(t * 65535.0);
    };
    // interleave the 16-bit codes (bits spread by shift-and-mask steps)
    auto spread = [](uint64_t v) {
        v = (v | (v << 8)) & 0x00ff00ffull;
        v = (v | (v << 4)) & 0x0f0f0f0full;
        v = (v | (v << 2)) & 0x33333333ull;
        v = (v | (v << 1)) & 0x55555555ull;
        return v;
    };
    return spread(q(x, x0)) | (spread(q(y, y0)) << 1);
}

int check_opts(fl_handle* h, const fl_opts& o) {
    if (o.dof_mode != FL_DOF_PAPER && o.dof_mode != FL_DOF_INTERIOR)
        return fail(h, FL_EINVAL, "dof_mode must be FL_DOF_PAPER or FL_DOF_INTERIOR");
    if (o.n_classes < 0 || o.n_classes > FL_MAX_CLASSES)
        return fail(h, FL_EINVAL, "n_classes out of range");
    if (o.precision != FL_FP64 && o.precision != FL_MIXED)
        return fail(h, FL_EINVAL, "precision must be FL_FP64 or FL_MIXED");
    if (o.k_touch < 1 || o.k_touch > FL_MAX_ORDER_TOUCH || o.k_touch_bnd < 1 ||
        o.k_touch_bnd > FL_MAX_ORDER_TOUCH)
        return fail(h, FL_EINVAL, "touching orders must lie in 1..16");
    for (int m = 0; m <= o.n_classes; ++m)
        if (o.k_far[m] < 1 || o.k_far[m] > FL_MAX_ORDER_FAR || o.k_far_bnd[m] < 1 ||
            o.k_far_bnd[m] > FL_MAX_ORDER_FAR)
            return fail(h, FL_EINVAL, "separated-pair orders must lie in 1..8");
    if (o.surrogate < 0 || o.surrogate > o.n_classes)
        return fail(h, FL_EINVAL, "surrogate must lie in 0..n_classes (the last class stays exact)");
    if (o.surrogate > 0 && h->dim != 2) return fail(h, FL_EINVAL, "the surrogate is for triangle meshes (dim 2)");
    if (!(o.sur_tol >= 0.0)) return fail(h, FL_EINVAL, "sur_tol must be >= 0");
    if (!(o.mass_shift >= 0.0) || !std::isfinite(o.mass_shift))
        return fail(h, FL_EINVAL, "mass_shift must be finite and >= 0");
    if (o.deterministic != 0 && o.deterministic != 1) return fail(h, FL_EINVAL, "deterministic must be 0 or 1");
    if (o.deterministic && o.surrogate > 0)
        return fail(h, FL_EINVAL, "the repeatable assembly takes the exact rules (surrogate = 0)");
    for (int m = 0; m < o.n_classes; ++m) {
        if (!(o.theta[m] > 0.0) || !std::isfinite(o.theta[m]))
            return fail(h, FL_EINVAL, "theta must be positive and finite");
        if (m > 0 && !(o.theta[m] > o.theta[m - 1]))
            return fail(h, FL_EINVAL, "theta must be strictly increasing");
    }
    return FL_OK;
}

double cdn(int d, double s) {
    return std::pow(2.0, 2.0 * s) * s * std::tgamma(s + 0.5 * d) /
           (std::pow(M_PI, 0.5 * d) * std::tgamma(1.0 - s));
}

// Gauss-Legendre / Gauss-Jacobi(1,0) tables (k = 1..16), collapsed triangle
// rules and segment rules (k = 1..8); independent of s, built once.
const RuleTables& base_rules() {
    static RuleTables R = [] {
        RuleTables T;
        std::memset(&T, 0, sizeof(T));
        // kernel-power tables: 2 / m_i with m_i = 1 + (i + 1/2) / 256, the
        // midpoint of the mantissas whose top 8 bits are i (the kernels take
        // the mantissa as m / 2 in [1/2, 1), v_frexp_mant_f64, so that
        // (m / 2)(2 / m_i) is exactly m / m_i)
        for (int i = 0; i < 256; ++i) T.pw_inv[i] = (double)(2.0L / (1.0L + ((long double)i + 0.5L) / 256.0L));
        for (int k = 1; k <= 16; ++k) {
            gauss_jacobi01(k, 0.0, 0.0, T.gl_x + gl_off(k), T.gl_w + gl_off(k));
            gauss_jacobi01(k, 1.0, 0.0, T.gj_x + gl_off(k), T.gj_w + gl_off(k));
        }
        for (int k = 1; k <= 8; ++k) {
            int m = tri_off(k);
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) {
                    double u = T.gj_x[gl_off(k) + i];
                    T.tl1[m] = u;
                    T.tl2[m] = (1.0 - u) * T.gl_x[gl_off(k) + j];
                    T.tw[m] = 2.0 * T.gj_w[gl_off(k) + i] * T.gl_w[gl_off(k) + j];
                    double l1 = T.tl1[m], l2 = T.tl2[m], w = T.tw[m];
                    double lam[3] = {1.0 - l1 - l2, l1, l2};
                    double* c = T.tri[m];
                    c[0] = l1;
                    c[1] = l2;
                    c[2] = w;
                    for (int a = 0; a < 3; ++a) c[3 + a] = w * lam[a];
                    int slot = 6;
                    for (int a = 0; a < 3; ++a)
                        for (int b = a; b < 3; ++b) c[slot++] = w * lam[a] * lam[b];
                    ++m;
                }
        }
        for (int k = 1; k <= 8; ++k)
            for (int i = 0; i < k; ++i) {
                double t = T.gl_x[gl_off(k) + i], w = T.gl_w[gl_off(k) + i];
                double* c = T.seg[gl_off(k) + i];
                c[0] = t;
                c[1] = w;
                c[2] = w * (1.0 - t);
                c[3] = w * t;
                c[4] = w * (1.0 - t) * (1.0 - t);
                c[5] = w * (1.0 - t) * t;
                c[6] = w * t * t;
                c[7] = 0.0;
            }
        for (int m = 0; m < TRI_TAB; ++m)
            for (int c = 0; c < 12; ++c) T.trif[m][c] = (float)T.tri[m][c];
        for (int m = 0; m < 36; ++m)
            for (int c = 0; c < 8; ++c) T.segf[m][c] = (float)T.seg[m][c];
        return T;
    }();
    return R;
}

}  // namespace

extern "C" {

int fl_default_opts(fl_opts* out) {
    if (!out) return FL_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->dof_mode = FL_DOF_PAPER;
    out->with_boundary = 1;
    out->k_touch = 6;
    out->k_touch_bnd = 6;
    out->sur_tol = 1e-2;
    out->n_classes = 3;
    out->theta[0] = 1.5;
    out->theta[1] = 3.0;
    out->theta[2] = 6.0;
    const int kf[4] = {4, 3, 2, 2};
    for (int m = 0; m < 4; ++m) out->k_far[m] = out->k_far_bnd[m] = kf[m];
    return FL_OK;
}

int fl_create(fl_handle** out, int device, void* hip_stream) {
    if (!out) return FL_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FL_EDEVICE;
    if (device < 0 || device >= ndev) return FL_EINVAL;
    fl_handle* h = new fl_handle();
    h->device = device;
    h->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return FL_EDEVICE;
    }
    if (!noalloc_scratch(h)) {
        delete h;
        return FL_EDEVICE;
    }
    *out = h;
    return FL_OK;
}

void fl_destroy(fl_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    free_buffers(h);
    free_solver(h);
    fl_sur_free(h);
    fl_mg_free(h);
    fl_sf_free(h);
    fl_hm_free(h);
    delete h;
}

const char* fl_last_error(const fl_handle* h) {
    if (!h) return "null handle";
    return h->err.c_str();
}

int fl_set_mesh(fl_handle* h, int dim, int64_t nv, const double* verts, int64_t nc,
                const int32_t* cells, int64_t nb, const int32_t* bfacets) {
    if (!h) return FL_EINVAL;
    if (dim != 1 && dim != 2) return fail(h, FL_EINVAL, "dim must be 1 or 2");
    if (nv <= 0 || nc <= 0 || nb < 0 || !verts || !cells || (nb > 0 && !bfacets))
        return fail(h, FL_EINVAL, "empty mesh or null array");
    if (nc > (int64_t)1 << 30 || nv > (int64_t)1 << 30) return fail(h, FL_EINVAL, "mesh too large");
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    reset_assembly(h);
    h->pc.valid = false;
    h->dim = 0;
    h->sym_T = 0;
    h->sym_order = 1;
    h->vfold.clear();
    h->sym_pre.clear();
    h->sym_rot.clear();
    const int nper = dim + 1;
    for (int64_t i = 0; i < nv * dim; ++i)
        if (!std::isfinite(verts[i])) return fail(h, FL_EMESH, "non-finite vertex coordinate");
    for (int64_t i = 0; i < nc * nper; ++i)
        if (cells[i] < 0 || cells[i] >= nv) return fail(h, FL_EMESH, "cell vertex index out of range");
    for (int64_t i = 0; i < nb * dim; ++i)
        if (bfacets[i] < 0 || bfacets[i] >= nv) return fail(h, FL_EMESH, "facet vertex index out of range");
    if (dim == 2) {  // (before the per-cell checks: their squares stay finite)
        double lo[2] = {verts[0], verts[1]}, hi[2] = {verts[0], verts[1]};
        for (int64_t v = 0; v < nv; ++v)
            for (int j = 0; j < 2; ++j) {
                lo[j] = std::min(lo[j], verts[2 * v + j]);
                hi[j] = std::max(hi[j], verts[2 * v + j]);
            }
        if (!(std::hypot(hi[0] - lo[0], hi[1] - lo[1]) < 0x1p60))
            return fail(h, FL_EMESH, "mesh extent above the supported scale (2^60)");
    }
    for (int64_t K = 0; K < nc; ++K) {
        const int32_t* c = cells + nper * K;
        double meas;
        if (dim == 1) {
            meas = std::fabs(verts[c[1]] - verts[c[0]]);
        } else {
            const double* a = verts + 2 * c[0];
            const double* b = verts + 2 * c[1];
            const double* d = verts + 2 * c[2];
            meas = 0.5 * std::fabs((b[0] - a[0]) * (d[1] - a[1]) - (d[0] - a[0]) * (b[1] - a[1]));
        }
        if (!(meas > 0.0)) return fail(h, FL_EMESH, "degenerate cell " + std::to_string(K));
        if (dim == 2) {
            // The FP64 kernel power of the separated-pair kernels covers
            // squared distances in [2^-128, 2^128).  A quadrature point of a
            // triangle lies at least (smallest barycentric coordinate) x
            // (smallest height) from its boundary: above 2^-11 x 2 x inradius
            // for the rules of order <= 8, so separated pairs stay above
            // 2^-114 for inradii >= 2^-48; no two points are further apart
            // than the coordinate extent.
            const double* a = verts + 2 * c[0];
            const double* b = verts + 2 * c[1];
            const double* d = verts + 2 * c[2];
            auto len = [](const double* p, const double* q) {
                const double u = q[0] - p[0], w = q[1] - p[1];
                return std::sqrt(u * u + w * w);
            };
            const double per = len(a, b) + len(b, d) + len(d, a);
            if (!(2.0 * meas / per >= 0x1p-48))
                return fail(h, FL_EMESH, "cell " + std::to_string(K) + " below the supported scale (inradius < 2^-48)");
        }
    }
    // vertex -> cells (CSR) to find the cell owning each boundary facet
    std::vector<int32_t> ptr(nv + 1, 0), idx(nc * nper);
    for (int64_t i = 0; i < nc * nper; ++i) ptr[cells[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) ptr[v + 1] += ptr[v];
    {
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t K = 0; K < nc; ++K)
            for (int a = 0; a < nper; ++a) idx[fill[cells[nper * K + a]]++] = (int32_t)K;
    }
    h->facet_opp.assign(nb, -1);
    h->on_boundary.assign(nv, 0);
    for (int64_t e = 0; e < nb; ++e) {
        const int32_t* f = bfacets + dim * e;
        int owners = 0, opp = -1;
        for (int32_t j = ptr[f[0]]; j < ptr[f[0] + 1]; ++j) {
            const int32_t* c = cells + nper * idx[j];
            bool has = true;
            if (dim == 2) has = (c[0] == f[1] || c[1] == f[1] || c[2] == f[1]) && f[0] != f[1];
            if (!has) continue;
            ++owners;
            for (int a = 0; a < nper; ++a)
                if (c[a] != f[0] && (dim == 1 || c[a] != f[1])) opp = c[a];
        }
        if (owners != 1)
            return fail(h, FL_EMESH, "boundary facet " + std::to_string(e) + " does not lie on exactly one cell");
        h->facet_opp[e] = opp;
        for (int a = 0; a < dim; ++a) h->on_boundary[f[a]] = 1;
    }
    h->dim = dim;
    h->nv = nv;
    h->nc = nc;
    h->nb = nb;
    h->verts.assign(verts, verts + nv * dim);
    h->cells.assign(cells, cells + nc * nper);
    h->bfacets.assign(bfacets, bfacets + nb * dim);
    return FL_OK;
}

int fl_set_symmetry(fl_handle* h, int32_t order, int64_t ncells_sector, const int32_t* vfold,
                    const int32_t* cell_pre, const int32_t* cell_rot) {
    if (!h) return FL_EINVAL;
    if (h->dim == 0) return fail(h, FL_ESTATE, "fl_set_mesh must be called first");
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    reset_assembly(h);
    h->pc.valid = false;
    h->sym_pre.clear();
    h->sym_rot.clear();
    if (order == 1 && ncells_sector == 0) {
        h->sym_T = 0;
        h->sym_order = 1;
        h->vfold.clear();
        return FL_OK;
    }
    if (order < 2) return fail(h, FL_EINVAL, "order must be >= 2 (or 1 with 0 sector cells to switch off)");
    if (ncells_sector < 1 || ncells_sector > h->nc) return fail(h, FL_EINVAL, "sector cell count out of range");
    if (!vfold) return fail(h, FL_EINVAL, "null vfold");
    std::vector<char> in_sector(h->nv, 0);
    const int nper = h->dim + 1;
    for (int64_t i = 0; i < ncells_sector * nper; ++i) in_sector[h->cells[i]] = 1;
    for (int64_t v = 0; v < h->nv; ++v) {
        const int32_t r = vfold[v];
        if (r < 0 || r >= h->nv) return fail(h, FL_EMESH, "vfold entry out of range");
        if (vfold[r] != r) return fail(h, FL_EMESH, "vfold must map onto representatives (vfold[vfold[v]] = vfold[v])");
        if (!in_sector[r]) return fail(h, FL_EMESH, "a representative is not a vertex of the sector's cells");
        if (h->on_boundary[v] != h->on_boundary[r])
            return fail(h, FL_EMESH, "a vertex and its representative differ in boundary status");
    }
    if ((cell_pre == nullptr) != (cell_rot == nullptr)) return fail(h, FL_EINVAL, "cell_pre and cell_rot go together");
    if (cell_pre) {
        for (int64_t K = 0; K < h->nc; ++K) {
            const int32_t p = cell_pre[K], r = cell_rot[K];
            if (p < 0 || p >= ncells_sector || r < 0 || r >= order)
                return fail(h, FL_EMESH, "cell_pre / cell_rot entry out of range");
            if ((K < ncells_sector) != (r == 0) || (K < ncells_sector && p != K))
                return fail(h, FL_EMESH, "sector cells must be their own preimage with rotation 0, images not");
            // an image and its preimage fold onto the same vertices
            int a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
            for (int j = 0; j <= h->dim; ++j) {
                a[j] = vfold[h->cells[(h->dim + 1) * K + j]];
                b[j] = vfold[h->cells[(h->dim + 1) * (int64_t)p + j]];
            }
            std::sort(a, a + h->dim + 1);
            std::sort(b, b + h->dim + 1);
            for (int j = 0; j <= h->dim; ++j)
                if (a[j] != b[j]) return fail(h, FL_EMESH, "a cell and its preimage fold onto different vertices");
        }
        h->sym_pre.assign(cell_pre, cell_pre + h->nc);
        h->sym_rot.assign(cell_rot, cell_rot + h->nc);
    }
    h->vfold.assign(vfold, vfold + h->nv);
    h->sym_T = ncells_sector;
    h->sym_order = order;
    return FL_OK;
}

int64_t fl_matrix_ld(const fl_handle* h) { return (h && h->assembled) ? h->lda : 0; }

const double* fl_matrix_ptr(const fl_handle* h) {
    if (!h || !h->assembled) return nullptr;
    // the caller may read the whole matrix: its lower tiles are written first
    if (fl_complete_lower(const_cast<fl_handle*>(h)) != FL_OK) return nullptr;
    return h->dA;
}

}  // extern "C"

namespace fl {

// DOF map (Sec. 3): all nodes, or the interior ones; with a symmetry
// reduction the representatives only, images taking their DOF.
void set_dof_map(fl_handle* h, bool all_nodes) {
    const bool symm = h->sym_T > 0;
    h->node2dof.assign(h->nv, -1);
    h->dof_node.clear();
    for (int64_t v = 0; v < h->nv; ++v)
        if ((!symm || h->vfold[v] == v) && (all_nodes || !h->on_boundary[v])) {
            h->node2dof[v] = (int32_t)h->dof_node.size();
            h->dof_node.push_back((int32_t)v);
        }
    if (symm)  // images take the DOF of their representative
        for (int64_t v = 0; v < h->nv; ++v) h->node2dof[v] = h->node2dof[h->vfold[v]];
}

// Element order, touching-pair lists, tiles, facet data after the DOF map;
// everything packed and sent to the device plan buffer.  sel: the element
// block pairs to tile (all pairs bi <= bj when null).
int plan_assembly(fl_handle* h, bool all_nodes, const fl_opts& o, Plan& P, const TileSelect* sel) {
    auto t0 = std::chrono::steady_clock::now();
    h->pc.valid = false;  // the plan buffer is rewritten
    int rc = FL_OK;
    const int dim = h->dim, nper = dim + 1;
    const int64_t T = h->nc, nv = h->nv;
    const bool symm = h->sym_T > 0;
    const int64_t Tw = symm ? h->sym_T : T;
    set_dof_map(h, all_nodes);
    const int64_t n = (int64_t)h->dof_node.size();
    P.T = T;
    P.nv = nv;
    P.n = n;
    P.dim = dim;
    P.nper = nper;

    // internal element order: Morton order of centroids (2D), by x (1D)
    std::vector<int32_t> perm(T);
    {
        std::vector<double> cx(T), cy(T, 0.0);
        double lo0 = 1e300, lo1 = 1e300, hi0 = -1e300, hi1 = -1e300;
        for (int64_t K = 0; K < T; ++K) {
            const int32_t* c = &h->cells[nper * K];
            double sx = 0, sy = 0;
            for (int a = 0; a < nper; ++a) {
                sx += h->verts[dim * c[a]];
                if (dim == 2) sy += h->verts[dim * c[a] + 1];
            }
            cx[K] = sx / nper;
            cy[K] = sy / nper;
            lo0 = std::min(lo0, cx[K]); hi0 = std::max(hi0, cx[K]);
            lo1 = std::min(lo1, cy[K]); hi1 = std::max(hi1, cy[K]);
        }
        std::vector<uint64_t> key(T);
        if (dim == 2) {
            double span = std::max(hi0 - lo0, hi1 - lo1);
            if (!(span > 0)) span = 1;
            for (int64_t K = 0; K < T; ++K) key[K] = (morton2(cx[K], cy[K], lo0, lo1, span) << 32) | (uint64_t)K;
        } else {
            double span = hi0 - lo0;
            if (!(span > 0)) span = 1;
            for (int64_t K = 0; K < T; ++K)
                key[K] = ((uint64_t)((cx[K] - lo0) / span * 4294967295.0) << 32) | (uint64_t)K;
        }
        // with a symmetry reduction the sector's cells come first: the top
        // bit of the position code marks an image cell (the code keeps 31 bits)
        if (symm)
            for (int64_t K = 0; K < T; ++K)
                key[K] = ((((key[K] >> 33) | (K >= Tw ? 0x80000000ull : 0ull))) << 32) | (key[K] & 0xffffffffull);
        // stable LSD radix sort on the 32-bit position code (upper half of
        // the key): equal codes keep increasing K, as a sort of the key would
        std::vector<uint64_t> tmp(T);
        for (int pass = 0; pass < 4; ++pass) {
            const int sh = 32 + 8 * pass;
            size_t cnt[257] = {0};
            for (int64_t K = 0; K < T; ++K) cnt[((key[K] >> sh) & 0xff) + 1]++;
            if (cnt[((key[0] >> sh) & 0xff) + 1] == (size_t)T) continue;  // one bucket: nothing to do
            for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
            for (int64_t K = 0; K < T; ++K) tmp[cnt[(key[K] >> sh) & 0xff]++] = key[K];
            key.swap(tmp);
        }
        for (int64_t K = 0; K < T; ++K) perm[K] = (int32_t)(key[K] & 0xffffffffu);
        if (symm && !h->sym_pre.empty()) {
            // the sector in the caller's order (internal index = caller
            // index, which the pair weights compare), then the images by
            // (rotation, preimage): the cross pairs that count sit on one
            // side of the block diagonal of each image copy
            for (int64_t K = 0; K < Tw; ++K) perm[K] = (int32_t)K;
            std::vector<int32_t> img;
            for (int64_t K = Tw; K < T; ++K) img.push_back((int32_t)K);
            std::stable_sort(img.begin(), img.end(), [&](int32_t a, int32_t b) {
                return h->sym_rot[a] != h->sym_rot[b] ? h->sym_rot[a] < h->sym_rot[b] : h->sym_pre[a] < h->sym_pre[b];
            });
            for (size_t k = 0; k < img.size(); ++k) perm[Tw + k] = img[k];
        }
    }
    // element SoA in internal order
    const int NC = nper * dim;
    std::vector<std::vector<double>> X(NC, std::vector<double>(T));
    std::vector<double> cen0(T), cen1(T, 0.0), h2(T), meas(T);
    std::vector<std::vector<int>> vid(nper, std::vector<int>(T, -1)), dof(nper, std::vector<int>(T, -1));
    for (int64_t Ki = 0; Ki < T; ++Ki) {
        const int32_t* c = &h->cells[nper * perm[Ki]];
        for (int a = 0; a < nper; ++a) {
            vid[a][Ki] = c[a];
            dof[a][Ki] = h->node2dof[c[a]];
            for (int d = 0; d < dim; ++d) X[dim * a + d][Ki] = h->verts[dim * c[a] + d];
        }
        if (dim == 1) {
            double x0 = X[0][Ki], x1 = X[1][Ki];
            cen0[Ki] = (x0 + x1) / 2.0;
            double e = x1 - x0;
            h2[Ki] = e * e;
            meas[Ki] = std::fabs(x1 - x0);
        } else {
            double ax = X[0][Ki], ay = X[1][Ki], bx = X[2][Ki], by = X[3][Ki], dx = X[4][Ki], dy = X[5][Ki];
            cen0[Ki] = ((ax + bx) + dx) / 3.0;
            cen1[Ki] = ((ay + by) + dy) / 3.0;
            double P[3][2] = {{ax, ay}, {bx, by}, {dx, dy}};
            double m = 0.0;
            for (int i = 0; i < 3; ++i) {
                double e0 = P[(i + 1) % 3][0] - P[i][0], e1 = P[(i + 1) % 3][1] - P[i][1];
                double l = e0 * e0 + e1 * e1;
                if (l > m) m = l;
            }
            h2[Ki] = m;
            meas[Ki] = 0.5 * std::fabs((bx - ax) * (dy - ay) - (dx - ax) * (by - ay));
        }
    }
    // vertex -> internal elements (CSR, increasing element order) with the
    // local index of the vertex; lpos: position of each (element, vertex)
    // in its vertex's list
    std::vector<int> v2c_ptr(nv + 1, 0), v2c_idx(T * nper), lpos(T * nper);
    std::vector<unsigned char> vloc(T * nper);
    for (int64_t Ki = 0; Ki < T; ++Ki)
        for (int a = 0; a < nper; ++a) v2c_ptr[vid[a][Ki] + 1]++;
    for (int64_t v = 0; v < nv; ++v) v2c_ptr[v + 1] += v2c_ptr[v];
    {
        std::vector<int> fill(v2c_ptr.begin(), v2c_ptr.end() - 1);
        for (int64_t Ki = 0; Ki < T; ++Ki)
            for (int a = 0; a < nper; ++a) {
                int v = vid[a][Ki];
                lpos[Ki * nper + a] = fill[v];
                v2c_idx[fill[v]] = (int)Ki;
                vloc[fill[v]] = (unsigned char)a;
                fill[v]++;
            }
    }
    // touching pairs (Sec. 5): K < Kt sharing dim vertices (common edge, 2D)
    // or one vertex.  The elements after Ki in a vertex's list are the Kt >
    // Ki at that vertex; shared-vertex counts through a marker array.
    std::vector<int> edge_pairs, vert_pairs;
    bool touch_ok = true;
    auto find_touching = [&]() {
        edge_pairs.reserve((size_t)T * 4);
        vert_pairs.reserve((size_t)T * 12);
        std::vector<int> mark(T, -1), cnt(T, 0);
        int seen[256];
        for (int64_t Ki = 0; Ki < T; ++Ki) {
            int ns = 0;
            for (int a = 0; a < nper; ++a) {
                const int v = vid[a][Ki];
                const int e1 = v2c_ptr[v + 1];
                for (int e = lpos[Ki * nper + a] + 1; e < e1; ++e) {
                    const int Kt = v2c_idx[e];
                    if (mark[Kt] != (int)Ki) {
                        mark[Kt] = (int)Ki;
                        cnt[Kt] = 0;
                        if (ns == 256) { touch_ok = false; return; }
                        seen[ns++] = Kt;
                    }
                    cnt[Kt]++;
                }
            }
            // (first-seen order: deterministic; the touching kernels add into A)
            for (int q = 0; q < ns; ++q) {
                const int Kt = seen[q], sh = cnt[Kt];
                if (!(dim == 2 && sh == 2) && sh != 1) { touch_ok = false; return; }
                if (symm && Ki >= Tw && Kt >= Tw) continue;  // two images: weight 0
                if (dim == 2 && sh == 2) { edge_pairs.push_back((int)Ki); edge_pairs.push_back(Kt); }
                else { vert_pairs.push_back((int)Ki); vert_pairs.push_back(Kt); }
            }
        }
    };
    find_touching();
    if (!touch_ok) return fail(h, FL_EMESH, "duplicate cells or a vertex shared by more than 256 cells");
    // far-field tiles, see launch_far_tiles
    const int nblk = (int)((T + BE - 1) / BE);
    P.nblk = nblk;
    std::vector<int2> tiles, far_tiles;
    {
        std::vector<double> bx0(nblk, 1e300), bx1(nblk, -1e300), by0(nblk, 1e300), by1(nblk, -1e300),
            bh(nblk, 0.0);
        for (int64_t Ki = 0; Ki < T; ++Ki) {
            int b = (int)(Ki / BE);
            bx0[b] = std::min(bx0[b], cen0[Ki]);
            bx1[b] = std::max(bx1[b], cen0[Ki]);
            by0[b] = std::min(by0[b], cen1[Ki]);
            by1[b] = std::max(by1[b], cen1[Ki]);
            bh[b] = std::max(bh[b], h2[Ki]);
        }
        // a tile is "far" when the centroid boxes of the two blocks are so
        // far apart that every pair is separated (centroid distance > 2 h
        // excludes a common vertex) and falls in the last distance class
        double th_last2 = 4.0;
        if (o.n_classes > 0) th_last2 = std::max(4.0, o.theta[o.n_classes - 1] * o.theta[o.n_classes - 1]);
        const bool use_far = o.k_far[o.n_classes] <= 4;
        // with preimage data: the largest preimage among a block's image
        // cells; a tile of sector cells against image cells whose preimages
        // all come before the sector cells has weight 0 throughout
        std::vector<int> bmaxpre(nblk, -1);
        if (symm && !h->sym_pre.empty())
            for (int64_t Ki = Tw; Ki < T; ++Ki)
                bmaxpre[Ki / BE] = std::max(bmaxpre[Ki / BE], (int)h->sym_pre[perm[Ki]]);
        // 0: no tile, 1: tile, 2: far tile
        auto classify = [&](int bi, int bj) -> int {
            if (symm && (int64_t)bi * BE >= Tw) return 0;  // image blocks only: weight 0
            if (symm && !h->sym_pre.empty() && (int64_t)(bi + 1) * BE <= Tw && (int64_t)bj * BE >= Tw &&
                bmaxpre[bj] < bi * BE)
                return 0;
            bool far = false;
            if (use_far && bi != bj) {
                double dx = std::max(0.0, std::max(bx0[bj] - bx1[bi], bx0[bi] - bx1[bj]));
                double dy = std::max(0.0, std::max(by0[bj] - by1[bi], by0[bi] - by1[bj]));
                double d2 = dx * dx + dy * dy;
                far = d2 > th_last2 * std::max(bh[bi], bh[bj]) * (1.0 + 1e-9);
            }
            return far ? 2 : 1;
        };
        if (!sel) {
            // all pairs bi <= bj: block rows split over host threads in ranges
            // of about equal pair counts, each range into lists of its own,
            // joined in row order (the order of one sequential pass)
            const long long npairs = (long long)nblk * (nblk + 1) / 2;
            const int nth = (int)std::max<long long>(
                1, std::min<long long>({(long long)std::max(1u, std::thread::hardware_concurrency()), 16LL,
                                        npairs / 65536 + 1}));
            std::vector<int> row0(nth + 1, nblk);
            {
                long long acc = 0;
                int k = 1;
                row0[0] = 0;
                for (int bi = 0; bi < nblk && k < nth; ++bi) {
                    acc += nblk - bi;
                    if (acc * nth >= npairs * k) row0[k++] = bi + 1;
                }
            }
            std::vector<std::vector<int2>> part_near(nth), part_far(nth);
            auto work = [&](int k) {
                for (int bi = row0[k]; bi < row0[k + 1]; ++bi)
                    for (int bj = bi; bj < nblk; ++bj) {
                        const int c = classify(bi, bj);
                        if (c) (c == 2 ? part_far[k] : part_near[k]).push_back(make_int2(bi, bj));
                    }
            };
            std::vector<std::thread> pool;
            for (int k = 1; k < nth; ++k) pool.emplace_back(work, k);
            work(0);
            for (std::thread& t : pool) t.join();
            size_t nn = 0, nf = 0;
            for (int k = 0; k < nth; ++k) {
                nn += part_near[k].size();
                nf += part_far[k].size();
            }
            tiles.reserve(nn);
            far_tiles.reserve(nf);
            for (int k = 0; k < nth; ++k) {
                tiles.insert(tiles.end(), part_near[k].begin(), part_near[k].end());
                far_tiles.insert(far_tiles.end(), part_far[k].begin(), part_far[k].end());
            }
        } else {
            std::vector<int2> pairs;
            (*sel)(perm, dof, nblk, pairs);
            for (const int2& t : pairs) {
                const int c = classify(t.x, t.y);
                if (c) (c == 2 ? far_tiles : tiles).push_back(t);
            }
        }
    }
    std::vector<int> blk_ndof(nblk), blk_dofs((size_t)nblk * MAXV, -1);
    std::vector<unsigned char> loc(T * 3, 255);
    {
        // distinct DOFs of each block (marker array, first-seen order) and
        // each element vertex's index among them
        std::vector<int> ds, mark(n, -1), pos(n, 0);
        for (int b = 0; b < nblk; ++b) {
            ds.clear();
            const int64_t k0 = (int64_t)b * BE, k1 = std::min<int64_t>(T, (int64_t)(b + 1) * BE);
            for (int64_t Ki = k0; Ki < k1; ++Ki)
                for (int a = 0; a < nper; ++a) {
                    const int d = dof[a][Ki];
                    if (d >= 0 && mark[d] != b) {
                        mark[d] = b;
                        ds.push_back(d);
                    }
                }
            blk_ndof[b] = (int)ds.size();
            if ((int)ds.size() > MAXV) continue;  // tile falls back to global atomics
            for (size_t i = 0; i < ds.size(); ++i) {
                blk_dofs[(size_t)b * MAXV + i] = ds[i];
                pos[ds[i]] = (int)i;
            }
            for (int64_t Ki = k0; Ki < k1; ++Ki)
                for (int a = 0; a < nper; ++a)
                    if (dof[a][Ki] >= 0) loc[Ki * 3 + a] = (unsigned char)pos[dof[a][Ki]];
        }
    }
    // boundary facets: coordinates, inward unit normal (Sec. 2)
    std::vector<double> fac(std::max<int64_t>(h->nb, 1) * 6, 0.0);
    std::vector<int> fvid(std::max<int64_t>(h->nb, 1) * 2, -1);
    for (int64_t e = 0; e < h->nb; ++e) {
        const int32_t* f = &h->bfacets[dim * e];
        int opp = h->facet_opp[e];
        if (dim == 1) {
            double y = h->verts[f[0]], xo = h->verts[opp];
            fac[6 * e] = y;
            fac[6 * e + 4] = xo > y ? 1.0 : -1.0;
            fvid[2 * e] = f[0];
        } else {
            double p0x = h->verts[2 * f[0]], p0y = h->verts[2 * f[0] + 1];
            double p1x = h->verts[2 * f[1]], p1y = h->verts[2 * f[1] + 1];
            double tx = p1x - p0x, ty = p1y - p0y;
            double L = std::sqrt(tx * tx + ty * ty);
            double nx = -ty / L, ny = tx / L;
            double ox = h->verts[2 * opp] - p0x, oy = h->verts[2 * opp + 1] - p0y;
            if (nx * ox + ny * oy < 0) { nx = -nx; ny = -ny; }
            double* F = &fac[6 * e];
            F[0] = p0x; F[1] = p0y; F[2] = p1x; F[3] = p1y; F[4] = nx; F[5] = ny;
            fvid[2 * e] = f[0];
            fvid[2 * e + 1] = f[1];
        }
    }
    // symmetry reduction: cell weights (the sector's cells are the first Tw
    // internal ones), and per-DOF (cell, local vertex) lists: over all cells
    // for the diagonal-block scatter, over the sector for load and mass
    std::vector<double> wcell;
    std::vector<int> sc_ptr, sc_idx, sw_ptr, sw_idx, ident;
    std::vector<unsigned char> sc_vloc, sw_vloc;
    if (symm) {
        wcell.assign(T, 0.0);
        for (int64_t Ki = 0; Ki < Tw; ++Ki) wcell[Ki] = 1.0;
        sc_ptr.assign(n + 1, 0);
        sw_ptr.assign(n + 1, 0);
        for (int64_t Ki = 0; Ki < T; ++Ki)
            for (int a = 0; a < nper; ++a)
                if (dof[a][Ki] >= 0) {
                    sc_ptr[dof[a][Ki] + 1]++;
                    if (Ki < Tw) sw_ptr[dof[a][Ki] + 1]++;
                }
        for (int64_t i = 0; i < n; ++i) {
            sc_ptr[i + 1] += sc_ptr[i];
            sw_ptr[i + 1] += sw_ptr[i];
        }
        sc_idx.resize(sc_ptr[n]);
        sc_vloc.resize(sc_ptr[n]);
        sw_idx.resize(sw_ptr[n]);
        sw_vloc.resize(sw_ptr[n]);
        std::vector<int> fc(sc_ptr.begin(), sc_ptr.end() - 1), fw(sw_ptr.begin(), sw_ptr.end() - 1);
        for (int64_t Ki = 0; Ki < T; ++Ki)
            for (int a = 0; a < nper; ++a) {
                const int d = dof[a][Ki];
                if (d < 0) continue;
                sc_idx[fc[d]] = (int)Ki;
                sc_vloc[fc[d]++] = (unsigned char)a;
                if (Ki < Tw) {
                    sw_idx[fw[d]] = (int)Ki;
                    sw_vloc[fw[d]++] = (unsigned char)a;
                }
            }
        ident.resize(n);
        for (int64_t i = 0; i < n; ++i) ident[i] = (int)i;
    }
    // pack everything into the pinned staging buffer, one copy to the device
    Packer pk;
    std::vector<size_t> offX(NC);
    for (int c = 0; c < NC; ++c) offX[c] = pk.add(X[c]);
    const size_t o_c0 = pk.add(cen0), o_c1 = pk.add(cen1), o_h2 = pk.add(h2), o_me = pk.add(meas);
    std::vector<size_t> o_vid(nper), o_dof(nper);
    for (int a = 0; a < nper; ++a) { o_vid[a] = pk.add(vid[a]); o_dof[a] = pk.add(dof[a]); }
    size_t o_ft = pk.add(far_tiles), o_nt = pk.add(tiles), o_bnd = pk.add(blk_ndof),
                 o_bdofs = pk.add(blk_dofs), o_loc = pk.add(loc), o_v2cp = pk.add(v2c_ptr),
                 o_v2ci = pk.add(v2c_idx), o_vloc = pk.add(vloc), o_n2d = pk.add(h->node2dof),
                 o_dn = pk.add(h->dof_node), o_ep = pk.add(edge_pairs), o_vp = pk.add(vert_pairs),
                 o_fac = pk.add(fac), o_fvid = pk.add(fvid);
    std::vector<int> spre, srot;
    if (symm && !h->sym_pre.empty()) {
        spre.resize(T);
        srot.resize(T);
        for (int64_t Ki = 0; Ki < T; ++Ki) {
            spre[Ki] = Ki < Tw ? -1 : h->sym_pre[perm[Ki]];
            srot[Ki] = Ki < Tw ? 0 : h->sym_rot[perm[Ki]];
        }
    }
    const size_t o_spre = pk.add(spre), o_srot = pk.add(srot);
    const size_t o_w = pk.add(wcell), o_scp = pk.add(sc_ptr), o_sci = pk.add(sc_idx), o_scv = pk.add(sc_vloc),
                 o_swp = pk.add(sw_ptr), o_swi = pk.add(sw_idx), o_swv = pk.add(sw_vloc), o_id = pk.add(ident);
    if (pk.total > h->pin_cap) {
        if (h->pin) (void)hipHostFree(h->pin);
        h->pin = nullptr;
        h->pin_cap = 0;
        HIPCHK(hipHostMalloc((void**)&h->pin, pk.total, 0));
        h->pin_cap = pk.total;
    }
    for (const auto& p : pk.parts)
        if (p.bytes) std::memcpy(h->pin + p.off, p.src, p.bytes);
    if ((rc = ensure_dev(h, &h->plan, &h->plan_cap, pk.total))) return rc;
    if ((rc = ensure_dev(h, &h->dS, &h->S_cap, sizeof(double) * (size_t)T * 6))) return rc;
    if (!h->dcnt) HIPCHK(hipMalloc((void**)&h->dcnt, sizeof(unsigned long long) * 32));
    HIPCHK(hipMemcpyAsync(h->plan, h->pin, pk.total, hipMemcpyHostToDevice, h->stream));
    char* base = h->plan;
    auto dv = [&](size_t off) { return (void*)(base + off); };
    ElemDev E{};
    for (int c = 0; c < NC; ++c) E.x[c] = (const double*)dv(offX[c]);
    E.cen[0] = (const double*)dv(o_c0);
    E.cen[1] = dim == 2 ? (const double*)dv(o_c1) : nullptr;
    E.h2 = (const double*)dv(o_h2);
    E.meas = (const double*)dv(o_me);
    for (int a = 0; a < nper; ++a) {
        E.vid[a] = (const int*)dv(o_vid[a]);
        E.dof[a] = (const int*)dv(o_dof[a]);
    }
    E.w = symm ? (const double*)dv(o_w) : nullptr;
    E.spre = (symm && !h->sym_pre.empty()) ? (const int*)dv(o_spre) : nullptr;
    E.srot = (symm && !h->sym_pre.empty()) ? (const int*)dv(o_srot) : nullptr;
    E.sorder = h->sym_order;
    h->E = E;
    h->d_meas = (double*)dv(o_me);
    h->d_v2c_ptr = (int*)dv(o_v2cp);
    h->d_v2c_idx = (int*)dv(o_v2ci);
    h->d_node2dof = (int*)dv(o_n2d);
    h->d_dof_node = (int*)dv(o_dn);
    h->d_vloc = (const unsigned char*)dv(o_vloc);
    h->d_sc_ptr = h->d_v2c_ptr;
    h->d_sc_idx = h->d_v2c_idx;
    h->d_sc_map = h->d_node2dof;
    h->d_sc_vloc = h->d_vloc;
    h->sc_rows = (int)nv;
    if (symm) {
        // DOF-indexed lists: the scatter owns DOF rows, load and mass sum over
        // the sector's cells of every vertex folded onto the DOF
        h->d_sc_ptr = (int*)dv(o_scp);
        h->d_sc_idx = (int*)dv(o_sci);
        h->d_sc_vloc = (const unsigned char*)dv(o_scv);
        h->d_sc_map = (int*)dv(o_id);
        h->sc_rows = (int)n;
        h->d_v2c_ptr = (int*)dv(o_swp);
        h->d_v2c_idx = (int*)dv(o_swi);
        h->d_vloc = (const unsigned char*)dv(o_swv);
        h->d_dof_node = (int*)dv(o_id);
    }
    P.o_ft = o_ft; P.o_nt = o_nt; P.o_bnd = o_bnd; P.o_bdofs = o_bdofs; P.o_loc = o_loc;
    P.o_vloc = o_vloc; P.o_ep = o_ep; P.o_vp = o_vp; P.o_fac = o_fac; P.o_fvid = o_fvid;
    P.n_tiles = (long long)tiles.size();
    P.n_far_tiles = (long long)far_tiles.size();
    P.n_edge = (long long)edge_pairs.size() / 2;
    P.n_vert = (long long)vert_pairs.size() / 2;
    P.t_plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return FL_OK;
}

// Bound on every partial sum the assembly accumulates.  For the hat
// function of vertex v, with L_v its largest gradient on its cells and
// |supp_v| their total measure, (phi(x) - phi(y))^2 <= min(L_v^2 |x-y|^2, 1)
// on {x in supp} or {y in supp}, so
//   a(phi_v, phi_v) <= C |supp_v| |S^{d-1}| L_v^{2s} (1/(2-2s) + 1/(2s));
// every pair contribution to a diagonal entry is >= 0, and the absolute
// contributions to an off-diagonal entry sum to at most the geometric mean
// of two such bounds (Cauchy-Schwarz), and so do those to the cells'
// diagonal blocks.  Times 2 for the quadrature, times K^2 with a K-fold
// symmetry reduction (a DOF collects its orbit).
double entry_bound(const fl_handle* h, double s) {
    const int dim = h->dim, nper = dim + 1;
    std::vector<double> supp(h->nv, 0.0), L(h->nv, 0.0);
    for (int64_t K = 0; K < h->nc; ++K) {
        const int32_t* c = &h->cells[nper * K];
        if (dim == 1) {
            const double len = std::fabs(h->verts[c[1]] - h->verts[c[0]]);
            for (int a = 0; a < 2; ++a) {
                supp[c[a]] += len;
                L[c[a]] = std::max(L[c[a]], 1.0 / len);
            }
        } else {
            double P[3][2];
            for (int a = 0; a < 3; ++a)
                for (int j = 0; j < 2; ++j) P[a][j] = h->verts[2 * c[a] + j];
            const double area =
                0.5 * std::fabs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]));
            for (int a = 0; a < 3; ++a) {
                const double* p = P[(a + 1) % 3];
                const double* q = P[(a + 2) % 3];
                const double edge = std::hypot(q[0] - p[0], q[1] - p[1]);  // opposite vertex a
                supp[c[a]] += area;
                L[c[a]] = std::max(L[c[a]], edge / (2.0 * area));
            }
        }
    }
    const double sphere = dim == 1 ? 2.0 : 2.0 * M_PI;
    const double rad = 1.0 / (2.0 - 2.0 * s) + 1.0 / (2.0 * s);
    double m = 0.0;
    for (int64_t v = 0; v < h->nv; ++v)
        m = std::max(m, supp[v] * std::pow(L[v], 2.0 * s));
    double k2 = h->sym_T > 0 ? (double)h->sym_order * h->sym_order : 1.0;
    return 2.0 * k2 * cdn(dim, s) * sphere * rad * m;
}

// One assembly of A^s (Sec. 5 pair decomposition) into A (row-major, lda;
// a_elems elements zeroed first), optional FP32 copy A32 (same lda).
// Adds the phase times to *st and fills its pair counts.
int run_assembly(fl_handle* h, const Plan& P, double s, const fl_opts& o, double* A, int64_t lda,
                 long long a_elems, float* A32, fl_stats_t* st, const NearMap* nm,
                 const std::function<int()>* before_scatter) {
    int rc = FL_OK;
    const int dim = P.dim;
    const int64_t T = P.T, nv = P.nv, n = P.n;
    const int nblk = P.nblk;
    char* base = h->plan;
    auto dv = [&](size_t off) { return (void*)(base + off); };
    const ElemDev E = h->E;
    double* dS = h->dS;
    unsigned long long* dcnt = h->dcnt;
    const size_t o_ft = P.o_ft, o_nt = P.o_nt, o_bnd = P.o_bnd, o_bdofs = P.o_bdofs, o_loc = P.o_loc,
                 o_vloc = P.o_vloc, o_ep = P.o_ep, o_vp = P.o_vp, o_fac = P.o_fac, o_fvid = P.o_fvid;
    (void)nblk;
    (void)rc;
    // quadrature tables: cached base rules + the two s-dependent radial rules
    RuleTables R = base_rules();
    if (s < 0.5) gauss_jacobi01(2, 0.0, -2.0 * s, R.r0_x, R.r0_w);
    gauss_jacobi01(2, 0.0, 1.0 - 2.0 * s, R.r1_x, R.r1_w);
    set_pow_tables(R, -(0.5 * dim + s));
    HIPCHK(upload_rules(R, h->stream));
    // the upper triangle only (the transpose writes the lower one at the end),
    // unless the buffer has padding rows past n (the batched matrices)
    if (A && a_elems == n * lda) launch_zero_upper(A, lda, n, h->stream);
    else launch_zero(A, a_elems, h->stream);
    launch_zero(dS, T * 6, h->stream);
    launch_zero((double*)dcnt, 32, h->stream);
    // repeatable accumulation: A's FP64 buffer holds the int64 remainders
    // (zero bits are zero in both), an int32 plane the coarse words; the
    // scale puts the entry bound just below 2^16 coarse units
    const bool det = o.deterministic && A;
    FixAcc fa{}, fsx{};
    double from_hi = 0.0, from_lo = 0.0;
    int* dflag = nullptr;
    if (det) {
        const size_t hi_words = ((size_t)a_elems + 1) / 2;  // int32 pairs as doubles
        if ((rc = ensure_dev(h, &h->dAhi, &h->Ahi_cap, hi_words * 8))) return rc;
        const size_t s_lo = (size_t)T * 6 * 8, s_hi = ((size_t)T * 6 * 4 + 7) / 8 * 8;
        if ((rc = ensure_dev(h, &h->dSfix, &h->Sfix_cap, s_lo + s_hi + 8))) return rc;
        launch_zero((double*)h->dAhi, (long long)hi_words, h->stream);
        launch_zero((double*)h->dSfix, (long long)((s_lo + s_hi + 8) / 8), h->stream);
        int e = 0;
        (void)std::frexp(entry_bound(h, s), &e);  // bound < 2^e
        fa.to_hi = std::ldexp(1.0, 16 - e);
        fa.lo_per_hi = 4503599627370496.0;  // 2^52
        from_hi = std::ldexp(1.0, e - 16);
        from_lo = std::ldexp(1.0, e - 68);
        dflag = (int*)(h->dSfix + s_lo + s_hi);
        fa.flag = dflag;
        fsx = fa;
        fa.lo = (long long*)A;
        fa.hi = h->dAhi;
        fsx.lo = (long long*)h->dSfix;
        fsx.hi = (int*)(h->dSfix + s_lo);
    }

    hipEvent_t ev[5];
    for (int i = 0; i < 5; ++i) HIPCHK(hipEventCreate(&ev[i]));
    HIPCHK(hipEventRecord(ev[0], h->stream));

    const double C = cdn(dim, s);
    const double pe = -(0.5 * dim + s);
    FarParams FP{};
    FP.dim = dim;
    FP.T = (int)T;
    FP.pe = pe;
    FP.C = C;
    FP.ncls = o.n_classes;
    for (int m = 0; m < o.n_classes; ++m) FP.th2[m] = o.theta[m] * o.theta[m];
    for (int m = 0; m <= o.n_classes; ++m) FP.kf[m] = o.k_far[m];
    for (int m = 0; m <= o.n_classes; ++m) {
        FP.kfirst[m] = 1;
        for (int j = 0; j < m; ++j)
            if (o.k_far[j] == o.k_far[m]) FP.kfirst[m] = 0;
    }
    FP.nblk = nblk;
    FP.tiles = (const int2*)dv(o_nt);
    FP.ntiles = P.n_tiles;
    FP.blk_ndof = (const int*)dv(o_bnd);
    FP.blk_dofs = (const int*)dv(o_bdofs);
    FP.loc = (const unsigned char*)dv(o_loc);
    FP.A = A;
    FP.lda = lda;
    FP.S = dS;
    FP.cls_count = dcnt;
    FP.mixed = o.precision == FL_MIXED ? 1 : 0;
    if (nm) FP.nm = *nm;
    FP.fa = fa;
    FP.fs = fsx;
    if (o.surrogate > 0) {
        if ((rc = fl_sur_params(h, s, o, &FP.sur))) return rc;
        FP.sur.counters = dcnt + 12;
    }
    launch_far(E, FP, h->stream);
    HIPCHK(hipGetLastError());
    {
        FarParams FF = FP;
        FF.tiles = (const int2*)dv(o_ft);
        FF.ntiles = P.n_far_tiles;
        launch_far_tiles(E, FF, o.k_far[o.n_classes], h->stream);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipEventRecord(ev[1], h->stream));

    BndParams BP{};
    BP.dim = dim;
    BP.s = s;
    BP.pe = pe;
    BP.C = C;
    BP.T = (int)(h->sym_T > 0 ? h->sym_T : T);  // identical pairs and boundary terms: the sector's cells
    BP.nb = (int)h->nb;
    BP.fac = (const double*)dv(o_fac);
    BP.fvid = (const int*)dv(o_fvid);
    BP.k_touch_bnd = o.k_touch_bnd;
    BP.ncls = o.n_classes;
    for (int m = 0; m < o.n_classes; ++m) BP.th2[m] = FP.th2[m];
    for (int m = 0; m <= o.n_classes; ++m) BP.kfb[m] = o.k_far_bnd[m];
    BP.k_touch = o.k_touch;
    BP.with_boundary = o.with_boundary;
    BP.S = dS;
    BP.counters = dcnt + 10;
    BP.fs = fsx;
    launch_self(E, BP, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev[2], h->stream));

    TouchParams TP{};
    TP.dim = dim;
    TP.s = s;
    TP.pe = pe;
    TP.C = C;
    TP.k = o.k_touch;
    TP.A = A;
    TP.lda = lda;
    if (nm) TP.nm = *nm;
    TP.fa = fa;
    if (dim == 2) {
        TP.npairs = P.n_edge;
        TP.pairs = (const int*)dv(o_ep);
        launch_touch_edge2(E, TP, h->stream);
        HIPCHK(hipGetLastError());
    }
    TP.npairs = P.n_vert;
    TP.pairs = (const int*)dv(o_vp);
    launch_touch_vert(E, TP, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev[3], h->stream));

    if (det) {
        launch_fix_to_double(fsx.lo, fsx.hi, from_hi, from_lo, T * 6, dS, h->stream);
        launch_fix_to_double(fa.lo, fa.hi, from_hi, from_lo, a_elems, A, h->stream);
        HIPCHK(hipGetLastError());
    }
    if (before_scatter) {
        if ((rc = (*before_scatter)())) return rc;
        HIPCHK(hipGetLastError());
    }
    if (nm)
        launch_scatter_self_near(E, h->d_sc_ptr, h->d_sc_idx, h->d_sc_map, h->d_sc_vloc, h->sc_rows, dim, dS,
                                 o.mass_shift, *nm, h->stream);
    else
        launch_scatter_self(E, h->d_sc_ptr, h->d_sc_idx, h->d_sc_map, h->d_sc_vloc, h->sc_rows, dim, dS,
                            o.mass_shift, A, lda, h->stream);
    HIPCHK(hipGetLastError());
    if (A) {
        // the handle's own matrix: the diagonal tiles now (the symmetric
        // product reads them whole), the rest when a reader of the full
        // matrix asks (fl_complete_lower); other matrices: everything
        const bool own = A == h->dA;
        launch_mirror_lower(A, lda, n, own ? 1 : 0, h->stream);
        HIPCHK(hipGetLastError());
        if (own) h->lower_pending = true;
    }
    if (A32) {
        launch_to_f32(A, lda, n, A32, h->stream);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipEventRecord(ev[4], h->stream));
    unsigned long long cnt[16];
    HIPCHK(hipMemcpyAsync(cnt, dcnt, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    int out_of_range = 0;
    if (det) HIPCHK(hipMemcpyAsync(&out_of_range, dflag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipEventSynchronize(ev[4]));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (out_of_range)
        return fail(h, FL_ENONFINITE, "repeatable assembly: a contribution outside the range of its fixed-point scale");
    float ms = 0.f, ph[4] = {0, 0, 0, 0};
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[4]));
    for (int i = 0; i < 4; ++i) HIPCHK(hipEventElapsedTime(&ph[i], ev[i], ev[i + 1]));
    for (int i = 0; i < 5; ++i) (void)hipEventDestroy(ev[i]);
    unsigned long long cnt2[16];
    HIPCHK(hipMemcpy(cnt2, dcnt + 16, sizeof(cnt2), hipMemcpyDeviceToHost));

    fl_stats_t& S = *st;
    S.n = n;
    S.n_cells = T;
    S.n_verts = nv;
    S.n_bfacets = h->nb;
    S.pairs_identical = T;
    S.pairs_edge = P.n_edge;
    S.pairs_vertex = P.n_vert;
    for (int m = 0; m <= FL_MAX_CLASSES; ++m) S.pairs_far[m] = m <= o.n_classes ? (int64_t)cnt[m] : 0;
    S.pairs_bnd_touch = (int64_t)cnt[10];
    S.pairs_bnd_far = (int64_t)cnt[11];
    S.pairs_surrogate = o.surrogate > 0 ? (int64_t)cnt[12] : 0;
    S.pairs_fallback = o.surrogate > 0 ? (int64_t)cnt[13] : 0;
    // kernel evaluations by the rules in use
    {
        int64_t ev2 = 0;
        const int kT = o.k_touch, kB = o.k_touch_bnd;
        for (int m = 0; m <= o.n_classes; ++m) {
            int64_t q = dim == 2 ? (int64_t)o.k_far[m] * o.k_far[m] : o.k_far[m];
            // band classes: order 2 for the surrogate pairs, the class order
            // for the fallbacks (counted per class by the near-tile kernel)
            int64_t np = m < o.surrogate ? (int64_t)cnt2[m] : S.pairs_far[m];
            ev2 += np * q * q;
        }
        if (o.surrogate > 0) ev2 += S.pairs_surrogate * 16;  // order 2: 4 x 4 points
        if (dim == 2) {
            ev2 += T * 3 * kT + S.pairs_edge * 4 * kT * kT + S.pairs_vertex * 2 * kT * kT * kT;
            ev2 += S.pairs_bnd_touch * 6 * kB * 2;  // upper bound per touching facet pair
        } else {
            ev2 += S.pairs_vertex * 2 * kT;
        }
        S.kernel_evals = ev2;
    }
    S.t_plan_ms = P.t_plan_ms;
    S.t_assemble_ms += ms;
    S.t_far_ms += ph[0];
    S.t_self_ms += ph[1];
    S.t_touch_ms += ph[2];
    S.t_scatter_ms += ph[3];
    return FL_OK;
}

}  // namespace fl

namespace {

int check_s_opts(fl_handle* h, double s, const fl_opts* opts_in, fl_opts* o) {
    if (!(s > 0.0 && s < 1.0)) return fail(h, FL_EINVAL, "s must lie in (0,1)");
    if (opts_in) *o = *opts_in;
    else fl_default_opts(o);
    return check_opts(h, *o);
}

bool fits(fl_handle* h, double bytes) {
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) != hipSuccess) return false;
    return bytes + (double)h->nc * 512.0 <= (double)freeb * 0.98;
}

}  // namespace

const fl::RuleTables& fl_base_rules() { return base_rules(); }

int fl_complete_lower(fl_handle* h) {
    if (!h->lower_pending || !h->dA || h->n <= 1) {
        h->lower_pending = false;
        return FL_OK;
    }
    HIPCHK(hipSetDevice(h->device));
    launch_mirror_lower(h->dA, h->lda, h->n, 2, h->stream);
    HIPCHK(hipGetLastError());
    h->lower_pending = false;
    return FL_OK;
}

void fl_release_dense(fl_handle* h) {
    reset_assembly(h);
    if (h->dA) (void)hipFree(h->dA);
    if (h->dA32) (void)hipFree(h->dA32);
    h->dA = nullptr;
    h->dA32 = nullptr;
    h->A_cap = h->A32_cap = 0;
    free_solver(h);
}
double fl_cdn(int d, double s) { return cdn(d, s); }

namespace fl {
// r2^pe = 2^(pe (n + i/256)) (1 + t)^pe with 2^(n + i/256) the nearest
// multiple of 1/256 in the exponent: tables of 2^(pe i/256) and 2^(pe n)
// (long double, rounded once) and the Taylor coefficients C(pe, k) of
// (1 + t)^pe, |t| < 1.4e-3 (degree 5: truncation below 5e-17).
void set_pow_tables(RuleTables& R, double pe) {
    const long double P = pe;
    for (int i = 0; i < 256; ++i) R.pw_fr[i] = (double)powl(1.0L + ((long double)i + 0.5L) / 256.0L, P);
    for (int n = -128; n < 128; ++n) R.pw_ex[n + 128] = (double)exp2l(P * (long double)n);
    long double c = 1.0L;
    R.pw_c[0] = 1.0;
    for (int k = 1; k < 8; ++k) {
        c = c * (P - (long double)(k - 1)) / (long double)k;
        R.pw_c[k] = (double)c;
    }
}
}  // namespace fl

extern "C" {

namespace {
// The plan inputs besides the mesh: the DOF set and the distance classes
// (the tiles' far / near split); the orders enter only the assembly runs.
bool plan_key_equal(const fl_plan_cache& c, bool all_nodes, const fl_opts& o) {
    if (c.all_nodes != all_nodes || c.n_classes != o.n_classes) return false;
    if (c.use_far != (o.k_far[o.n_classes] <= 4)) return false;
    for (int m = 0; m < o.n_classes; ++m)
        if (c.theta[m] != o.theta[m]) return false;
    return true;
}

void plan_store(fl_handle* h, bool all_nodes, const fl_opts& o, const Plan& P) {
    fl_plan_cache& c = h->pc;
    c.all_nodes = all_nodes;
    c.n_classes = o.n_classes;
    for (int m = 0; m < FL_MAX_CLASSES; ++m) c.theta[m] = m < o.n_classes ? o.theta[m] : 0.0;
    c.use_far = o.k_far[o.n_classes] <= 4;
    c.P = P;
    c.E = h->E;
    c.v2c_ptr = h->d_v2c_ptr;
    c.v2c_idx = h->d_v2c_idx;
    c.node2dof = h->d_node2dof;
    c.dof_node = h->d_dof_node;
    c.vloc = h->d_vloc;
    c.sc_ptr = h->d_sc_ptr;
    c.sc_idx = h->d_sc_idx;
    c.sc_map = h->d_sc_map;
    c.sc_vloc = h->d_sc_vloc;
    c.sc_rows = h->sc_rows;
    c.meas = h->d_meas;
    c.valid = true;
}

// The kept plan when its inputs match (the handle's views restored,
// t_plan_ms = 0), else a new one, kept for the next call.
int plan_or_reuse(fl_handle* h, bool all_nodes, const fl_opts& o, Plan& P) {
    const fl_plan_cache& c = h->pc;
    if (c.valid && plan_key_equal(c, all_nodes, o)) {
        set_dof_map(h, all_nodes);  // (host copy; other calls may have set another)
        P = c.P;
        P.t_plan_ms = 0.0;
        h->E = c.E;
        h->d_v2c_ptr = c.v2c_ptr;
        h->d_v2c_idx = c.v2c_idx;
        h->d_node2dof = c.node2dof;
        h->d_dof_node = c.dof_node;
        h->d_vloc = c.vloc;
        h->d_sc_ptr = c.sc_ptr;
        h->d_sc_idx = c.sc_idx;
        h->d_sc_map = c.sc_map;
        h->d_sc_vloc = c.sc_vloc;
        h->sc_rows = c.sc_rows;
        h->d_meas = c.meas;
        return FL_OK;
    }
    const int rc = plan_assembly(h, all_nodes, o, P, nullptr);
    if (rc == FL_OK) plan_store(h, all_nodes, o, P);
    return rc;
}
}  // namespace

int fl_assemble(fl_handle* h, double s, const fl_opts* opts_in, int64_t* n_out) {
    if (!h) return FL_EINVAL;
    if (h->dim == 0) return fail(h, FL_ESTATE, "fl_set_mesh must be called first");
    fl_opts o;
    int rc = check_s_opts(h, s, opts_in, &o);
    if (rc) return rc;
    HIPCHK(hipSetDevice(h->device));
    if (h->stream) HIPCHK(hipStreamSynchronize(h->stream));
    reset_assembly(h);
    // DOF map (Sec. 3): all nodes if s < 1/2 (paper rule), else interior
    const bool all_nodes = (o.dof_mode == FL_DOF_PAPER) && (s < 0.5);
    int64_t n = 0;
    for (int64_t v = 0; v < h->nv; ++v)
        n += ((h->sym_T == 0 || h->vfold[v] == v) && (all_nodes || !h->on_boundary[v])) ? 1 : 0;
    const int64_t lda = ((n + 31) / 32) * 32;
    const size_t A_bytes = sizeof(double) * (size_t)n * (size_t)lda + 8;
    if (A_bytes > h->A_cap) {
        if (h->dA) (void)hipFree(h->dA);
        h->dA = nullptr;
        h->A_cap = 0;
        const double extra = o.deterministic ? 0.5 * (double)A_bytes : 0.0;  // coarse words
        if (!fits(h, (double)A_bytes + extra))
            return fail(h, FL_ENOMEM, "matrix of " + std::to_string(n) + " DOFs does not fit in device memory");
    }
    Plan P;
    if ((rc = plan_or_reuse(h, all_nodes, o, P))) return rc;
    if ((rc = ensure_dev(h, &h->dA, &h->A_cap, A_bytes))) return rc;
    float* A32 = nullptr;
    if (o.precision == FL_MIXED) {
        if ((rc = ensure_dev(h, &h->dA32, &h->A32_cap, sizeof(float) * (size_t)n * (size_t)lda + 16))) return rc;
        A32 = h->dA32;
    }
    fl_stats_t S{};
    if ((rc = run_assembly(h, P, s, o, h->dA, lda, (long long)n * lda, A32, &S))) return rc;
    h->st = S;
    h->s = s;
    h->opts = o;
    h->n = n;
    h->lda = lda;
    h->assembled = true;
    h->planned = true;
    if (n_out) *n_out = n;
    return FL_OK;
}

int fl_assemble_batch(fl_handle* h, const double* s, int ns, const fl_opts* opts_in, int64_t* n_out) {
    if (!h) return FL_EINVAL;
    if (h->dim == 0) return fail(h, FL_ESTATE, "fl_set_mesh must be called first");
    if (!s || ns < 1 || ns > FL_MAX_BATCH) return fail(h, FL_EINVAL, "need 1 <= ns <= FL_MAX_BATCH values of s");
    fl_opts o;
    int rc = FL_OK;
    for (int j = 0; j < ns; ++j)
        if ((rc = check_s_opts(h, s[j], opts_in, &o))) return rc;
    if (o.deterministic) return fail(h, FL_EINVAL, "the repeatable assembly is for fl_assemble");
    bool all_nodes = (o.dof_mode == FL_DOF_PAPER) && (s[0] < 0.5);
    for (int j = 1; j < ns; ++j)
        if (((o.dof_mode == FL_DOF_PAPER) && (s[j] < 0.5)) != all_nodes)
            return fail(h, FL_EINVAL, "the s values give different DOF sets; use FL_DOF_INTERIOR");
    HIPCHK(hipSetDevice(h->device));
    if (h->stream) HIPCHK(hipStreamSynchronize(h->stream));
    reset_assembly(h);
    fl_batch& B = h->B;
    B.ns = 0;
    B.have32 = B.havehi = B.havelo = false;
    int64_t n = 0;
    for (int64_t v = 0; v < h->nv; ++v)
        n += ((h->sym_T == 0 || h->vfold[v] == v) && (all_nodes || !h->on_boundary[v])) ? 1 : 0;
    const int64_t n_pad = std::max<int64_t>(256, ((n + 255) / 256) * 256);
    const size_t bytes = sizeof(double) * (size_t)ns * (size_t)n_pad * (size_t)n_pad;
    if (bytes > B.A64_cap) {
        if (B.A64) (void)hipFree(B.A64);
        B.A64 = nullptr;
        B.A64_cap = 0;
        if (!fits(h, (double)bytes))
            return fail(h, FL_ENOMEM, "batch of " + std::to_string(ns) + " matrices does not fit in device memory");
    }
    Plan P;
    if ((rc = plan_or_reuse(h, all_nodes, o, P))) return rc;
    if ((rc = ensure_dev(h, &B.A64, &B.A64_cap, bytes))) return rc;
    fl_stats_t S{};
    for (int j = 0; j < ns; ++j) {
        double* Aj = B.A64 + (size_t)j * n_pad * n_pad;
        if ((rc = run_assembly(h, P, s[j], o, Aj, n_pad, (long long)n_pad * n_pad, nullptr, &S))) return rc;
        B.s[j] = s[j];
    }
    B.ns = ns;
    B.n = n;
    B.n_pad = n_pad;
    B.ld = n_pad;
    for (int d = 0; d < 4; ++d) B.best[d] = -1;
    h->st = S;
    h->opts = o;
    h->s = s[0];
    h->n = n;
    h->planned = true;
    if (n_out) *n_out = n;
    return FL_OK;
}

int fl_dofs(const fl_handle* h, int32_t* node_of_dof) {
    if (!h) return FL_EINVAL;
    if (!h->planned) return FL_ESTATE;
    if (h->n == 0) return FL_OK;
    if (!node_of_dof) return FL_EINVAL;
    std::memcpy(node_of_dof, h->dof_node.data(), sizeof(int32_t) * h->n);
    return FL_OK;
}

int fl_export_matrix(fl_handle* h, double* dst, int64_t ld, int on_device) {
    if (!h) return FL_EINVAL;
    if (!h->assembled) return fail(h, FL_ESTATE, "no assembled matrix");
    if (h->n == 0) return FL_OK;
    if (!dst) return fail(h, FL_EINVAL, "null destination");
    if (ld < h->n) return fail(h, FL_EINVAL, "ld < n");
    HIPCHK(hipSetDevice(h->device));
    if (h->n == 0) return FL_OK;
    if (int rc = fl_complete_lower(h)) return rc;
    HIPCHK(hipMemcpy2DAsync(dst, ld * sizeof(double), h->dA, h->lda * sizeof(double),
                            h->n * sizeof(double), h->n,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

int fl_import_matrix(fl_handle* h, const double* src, int64_t ld, int on_device) {
    if (!h) return FL_EINVAL;
    if (!h->assembled) return fail(h, FL_ESTATE, "no assembled matrix to replace");
    if (h->n == 0) return FL_OK;
    if (!src) return fail(h, FL_EINVAL, "null source");
    if (ld < h->n) return fail(h, FL_EINVAL, "ld < n");
    HIPCHK(hipSetDevice(h->device));
    h->mg.ready = false;  // the hierarchy's coarse operators came from the old matrix
    h->hm.ready = false;  // so did the cluster approximation
    h->lower_pending = false;  // the imported matrix is whole
    HIPCHK(hipMemcpy2DAsync(h->dA, h->lda * sizeof(double), src, ld * sizeof(double), h->n * sizeof(double),
                            h->n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
    if (h->opts.precision == FL_MIXED && h->dA32) launch_to_f32(h->dA, h->lda, h->n, h->dA32, h->stream);
    if (!on_device) HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

int fl_load_vector_one(fl_handle* h, double* b) {
    if (!h) return FL_EINVAL;
    if (!h->planned) return fail(h, FL_ESTATE, "no assembly");
    if (h->n == 0) return FL_OK;
    if (!b) return fail(h, FL_EINVAL, "null vector");
    HIPCHK(hipSetDevice(h->device));
    launch_load_one(h->d_dof_node, h->d_v2c_ptr, h->d_v2c_idx, h->d_meas, h->dim, h->n, b, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

static int ensure_solver(fl_handle* h);

int fl_mass_matvec(fl_handle* h, const double* x, double* y) {
    if (!h) return FL_EINVAL;
    if (!h->planned) return fail(h, FL_ESTATE, "no assembly");
    if (h->n == 0) return FL_OK;
    if (!x || !y) return fail(h, FL_EINVAL, "null vector");
    if (x == y) return fail(h, FL_EINVAL, "x and y must not alias");
    HIPCHK(hipSetDevice(h->device));
    launch_mass_matvec(h->E, h->d_dof_node, h->d_v2c_ptr, h->d_v2c_idx, h->d_vloc, h->dim, h->n, x, y, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

extern "C++" {
int fl_solver_workspace(fl_handle* h) { return ensure_solver(h); }

// Scratch of fl_matvec_noalloc, for callers that cannot allocate (code
// under graph capture, serving loops): the slots and partials of the
// symmetric product in a file-scope device array (each device the library
// runs on holds its own copy until the process ends).  Host code uses only
// the per-device address that hipGetSymbolAddress returns (the array's name
// is not a device address on the host); it is resolved once per device by
// fl_create, with that device current.
static constexpr size_t FL_NOALLOC_DOUBLES = (size_t)6 << 20;  // 48 MiB
static __device__ __align__(256) double scratch[FL_NOALLOC_DOUBLES];
static constexpr int FL_NOALLOC_MAXDEV = 64;
static double* g_scratch_dev[FL_NOALLOC_MAXDEV];
static std::mutex g_scratch_mu;

// the scratch address on h->device (the device must be current)
static double* noalloc_scratch(fl_handle* h) {
    if (h->device < 0 || h->device >= FL_NOALLOC_MAXDEV) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[h->device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_dev[h->device] = (double*)ptr;
    }
    return g_scratch_dev[h->device];
}

static int* stat_flag(char* b) { return (int*)b; }
static double* stat_scal(char* b) { return (double*)(b + FL_STAT_SCAL); }
static double* stat_hist(char* b) { return (double*)(b + FL_STAT_HIST); }

// Copy the whole status block to its pinned mirror and wait.
static int pull_status(fl_handle* h) {
    HIPCHK(hipMemcpyAsync(h->w_hstat, h->w_stat, FL_STAT_BYTES, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

// Runs CG iterations (launch(it) enqueues iteration it) in chunks until the
// device status says stop or maxit iterations were launched.  After each
// chunk the status block comes back in one copy; the next chunk covers the
// iterations that the last chunk's convergence rate predicts (r.r history,
// plus a margin), so that few host round trips are needed and few launched
// iterations find the solver already stopped.  first: length of the first
// chunk.  Leaves the status block in the pinned mirror; *launched: the
// number of iterations launched.
template <class F>
static int cg_run_chunks(fl_handle* h, double rtol, int maxit, const F& launch, int* launched, int first = 16,
                         int start = 0) {
    const int* hf = stat_flag(h->w_hstat);
    const double* hs = stat_scal(h->w_hstat);
    const double* hh = stat_hist(h->w_hstat);
    int it = start, m = first;
    *launched = start;
    // device time of the launched iterations alone (events around each
    // chunk), summed into the handle's statistics
    hipEvent_t c0, c1;
    HIPCHK(hipEventCreate(&c0));
    HIPCHK(hipEventCreate(&c1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{c0, c1};
    while (!hf[0] && it < maxit) {
        m = std::max(1, std::min(m, maxit - it));
        HIPCHK(hipEventRecord(c0, h->stream));
        for (int j = 0; j < m; ++j) launch(it + j);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(c1, h->stream));
        it += m;
        *launched = it;
        int rc = pull_status(h);
        if (rc) return rc;
        float cms = 0.f;
        HIPCHK(hipEventElapsedTime(&cms, c0, c1));
        h->st.t_cg_kernels_ms += cms;
        h->st.cg_launched += m;
        if (hf[0]) break;
        // geometric rate over the last (up to 8) iterations of this chunk
        const int q = std::min(8, m - 1);
        const double ra = hh[(it - 1 - q) & 63], rb = hh[(it - 1) & 63], target = rtol * rtol * hs[0];
        int next = 16;
        if (q >= 1 && ra > 0 && rb > 0 && rb < ra && target > 0) {
            const double per = std::log(rb / ra) / q;              // log of the rate per iteration
            const double need = std::log(target / rb) / per;       // iterations still needed
            if (need > 0 && need < 1e6) next = (int)std::ceil(1.1 * need) + 1;
            else if (need <= 0) next = 2;
        }
        m = std::max(2, std::min(64, next));
    }
    return FL_OK;
}
}  // extern "C++"

int fl_matvec(fl_handle* h, const double* x, double* y) {
    if (!h) return FL_EINVAL;
    if (!h->assembled) return fail(h, FL_ESTATE, "no assembled matrix");
    if (h->n == 0) return FL_OK;
    if (!x || !y) return fail(h, FL_EINVAL, "null vector");
    if (x == y) return fail(h, FL_EINVAL, "x and y must not alias");
    HIPCHK(hipSetDevice(h->device));
    int rc = ensure_solver(h);
    if (rc) return rc;
    launch_symv(h->sym, h->dA, h->lda, x, y, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_matvec_noalloc(fl_handle* h, const double* x, double* y) {
    if (!h) return FL_EINVAL;
    if (!h->assembled) return fail(h, FL_ESTATE, "no assembled matrix");
    if (h->n == 0) return FL_OK;
    if (!x || !y) return fail(h, FL_EINVAL, "null vector");
    if (x == y) return fail(h, FL_EINVAL, "x and y must not alias");
    HIPCHK(hipSetDevice(h->device));
    SymPlan sp{};
    sym_plan_geometry(h->n, &sp);
    const size_t need = sym_plan_doubles(sp);
    if (need > FL_NOALLOC_DOUBLES) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "fl_matvec_noalloc: n = %lld needs %zu MiB of scratch, more than its %zu MiB; use fl_matvec",
                      (long long)h->n, (need * sizeof(double) + (1 << 20) - 1) >> 20,
                      (FL_NOALLOC_DOUBLES * sizeof(double)) >> 20);
        return fail(h, FL_EINVAL, msg);
    }
    double* buf = noalloc_scratch(h);
    if (!buf) return fail(h, FL_EDEVICE, "fl_matvec_noalloc: no scratch address on this device");
    sym_plan_bind(&sp, buf);
    launch_symv(sp, h->dA, h->lda, x, y, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

// Solver workspace for the current n: vectors, partial sums, status words
// and the slots of the symmetric product.
static int ensure_solver(fl_handle* h) {
    if (h->w_n == h->n && (h->opts.precision != FL_MIXED || h->w32)) return FL_OK;
    free_solver(h);
    const int64_t n = h->n;
    SymPlan sp{};
    sym_plan_geometry(n, &sp);
    const int64_t ndot = (n + 255) / 256;
    HIPCHK(hipMalloc((void**)&h->w, sizeof(double) * (size_t)(7 * n + 8)));
    // CG partials (4 per reduction block), then the dot products of the
    // mixed-precision refinement (which must not touch the CG partials)
    HIPCHK(hipMalloc((void**)&h->w_part, sizeof(double) * (size_t)(6 * std::max<int64_t>(sp.nred, ndot) + 8)));
    HIPCHK(hipMalloc((void**)&h->w_stat, FL_STAT_BYTES));
    HIPCHK(hipHostMalloc((void**)&h->w_hstat, FL_STAT_BYTES, 0));
    if (h->opts.precision == FL_MIXED) HIPCHK(hipMalloc((void**)&h->w32, sizeof(float) * (size_t)(9 * n + 16)));
    HIPCHK(hipMalloc((void**)&h->w_sym, sizeof(double) * sym_plan_doubles(sp)));
    sym_plan_bind(&sp, h->w_sym);
    h->sym = sp;
    h->w_n = n;
    return FL_OK;
}

// FL_MIXED: Jacobi-PCG whose products read the FP32 matrix (half the bytes
// of the FP64 one) with FP32 vectors, and FP64 residual replacement: when
// the recursive residual has dropped by DELTA (or reached what the
// tolerance needs), the FP32 correction is added to u in FP64, the true
// residual b - A u is formed with the FP64 matrix and replaces the
// recursive one, and the iteration continues with the same search
// direction (no restart), so the iteration count stays close to that of
// the FP64 solver.  Stops on the FP64 residual.
static int solve_mixed(fl_handle* h, const double* b, double* u, double rtol, int32_t maxit, int32_t* iters,
                       double* relres) {
    int rc = FL_OK;
    const int64_t n = h->n;
    const int nblk = (int)((n + 255) / 256);
    double* r = h->w;                 // FP64 residual
    float* W = h->w32;
    double* dpart = h->w_part + 4 * std::max<int64_t>(h->sym.nred, nblk);
    CgState32 S{};
    S.n = n;
    S.A = h->dA32;
    S.lda = h->lda;
    S.d = W;
    S.b = W + n;                      // FP32 copy of the true residual
    S.x = W + 2 * n;                  // FP32 correction since the last replacement
    S.r = W + 3 * n;
    S.z = W + 4 * n;
    S.p = W + 5 * n;                  // 2 n
    S.part = h->w_part;
    S.scal = stat_scal(h->w_stat);
    S.flag = stat_flag(h->w_stat);
    S.hist = stat_hist(h->w_stat);
    S.sp = h->sym;
    S.nblk = h->sym.nred;
    S.maxit = maxit;
    const double DELTA = 1e-2;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, h->stream));
    launch_diag32(h->dA32, h->lda, n, (float*)S.d, h->stream);
    launch_zero(u, n, h->stream);
    // u = 0: the residual is b
    launch_cast_f32(b, (float*)S.b, n, h->stream);
    launch_dot2(b, b, b, n, dpart, nblk, stat_scal(h->w_stat) + 8, h->stream);
    HIPCHK(hipGetLastError());
    if ((rc = pull_status(h))) return rc;
    const double bb = stat_scal(h->w_hstat)[8];
    double rr = bb;
    int it = 0, outer = 0, status = FL_OK, seg_len = 16;
    if (!(bb == bb) || bb > 1.79e308) status = FL_ENONFINITE;
    bool first = true;
    while (status == FL_OK && bb > 0.0 && !(std::sqrt(rr) <= rtol * std::sqrt(bb)) && it < maxit && outer < 400) {
        // segment: FP32 iterations until the recursive residual has dropped
        // by DELTA, or by what the tolerance still needs (with a margin)
        S.rtol = std::max(DELTA, 0.5 * rtol * std::sqrt(bb / rr));
        if (first) launch_cg32_init(S, h->stream);
        else launch_cg32_replace(S, it, h->stream);
        first = false;
        if ((rc = pull_status(h))) return rc;
        int launched = 0;
        if ((rc = cg_run_chunks(h, S.rtol, maxit, [&](int k) { launch_cg32_iter_at(S, k, h->stream); }, &launched,
                                seg_len + 2, it)))
            return rc;
        const int* flag = stat_flag(h->w_hstat);
        if (flag[2] == 1) { status = FL_EBREAKDOWN; break; }
        seg_len = std::max(2, flag[1] - it);
        it = flag[1];
        // u += correction; true residual in FP64 (and its FP32 copy)
        launch_add_correction(u, S.x, n, h->stream);
        launch_residual(h->sym, h->dA, h->lda, u, b, r, (float*)S.b, h->stream);
        launch_dot2(r, r, r, n, dpart, nblk, stat_scal(h->w_stat) + 8, h->stream);
        HIPCHK(hipGetLastError());
        if ((rc = pull_status(h))) return rc;
        rr = stat_scal(h->w_hstat)[8];
        if (!(rr == rr) || rr > 1.79e308) { status = FL_ENONFINITE; break; }
        ++outer;
    }
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    double rel = bb > 0 ? std::sqrt(rr) / std::sqrt(bb) : 0.0;
    h->st.t_solve_ms = ms;
    h->st.last_iters = it;
    h->st.last_relres = rel;
    h->st.last_outer = outer;
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (status == FL_EBREAKDOWN) return fail(h, FL_EBREAKDOWN, "CG breakdown: p.Ap <= 0");
    if (status == FL_ENONFINITE) return fail(h, FL_ENONFINITE, "non-finite residual");
    if (!(rel <= rtol)) return FL_ENOCONV;
    return FL_OK;
}

int fl_solve(fl_handle* h, const double* b, double* u, double rtol, int32_t maxit, int32_t* iters,
             double* relres) {
    if (!h) return FL_EINVAL;
    if (!h->assembled) return fail(h, FL_ESTATE, "no assembled matrix");
    if (!(rtol >= 0.0) || maxit < 0) return fail(h, FL_EINVAL, "rtol >= 0 and maxit >= 0 required");
    if (h->n == 0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return FL_OK;
    }
    if (!b || !u) return fail(h, FL_EINVAL, "null vector");
    HIPCHK(hipSetDevice(h->device));
    int rc = ensure_solver(h);
    if (rc) return rc;
    h->st.t_cg_kernels_ms = 0.0;
    h->st.cg_launched = 0;
    if (h->opts.precision == FL_MIXED) return solve_mixed(h, b, u, rtol, maxit, iters, relres);
    const int64_t n = h->n;
    CgState S{};
    S.n = n;
    S.A = h->dA;
    S.lda = h->lda;
    S.r = h->w;
    S.z = h->w + n;
    S.p = h->w + 2 * n;  // two buffers
    double* dd = h->w + 5 * n;
    S.d = dd;
    S.b = b;
    S.x = u;
    S.part = h->w_part;
    S.scal = stat_scal(h->w_stat);
    S.flag = stat_flag(h->w_stat);
    S.hist = stat_hist(h->w_stat);
    S.rtol = rtol;
    S.maxit = maxit;
    S.sp = h->sym;
    S.nblk = h->sym.nred;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, h->stream));
    launch_diag(h->dA, h->lda, n, dd, h->stream);
    launch_cg_init(S, h->stream);
    HIPCHK(hipGetLastError());
    if ((rc = pull_status(h))) return rc;
    if (stat_flag(h->w_hstat)[2] == 2) return fail(h, FL_ENONFINITE, "right-hand side is not finite");
    int it = 0;
    if ((rc = cg_run_chunks(h, rtol, maxit, [&](int k) { launch_cg_iter_at(S, k, h->stream); }, &it))) return rc;
    // residual of the final iterate (when the loop ended at maxit)
    launch_cg_final(S, it, h->stream);
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if ((rc = pull_status(h))) return rc;
    const int* flag = stat_flag(h->w_hstat);
    const double* sc = stat_scal(h->w_hstat);
    int iterations = flag[1];
    double rel = sc[0] > 0 ? std::sqrt(sc[1]) / std::sqrt(sc[0]) : 0.0;
    h->st.t_solve_ms = ms;
    h->st.last_iters = iterations;
    h->st.last_relres = rel;
    h->st.last_outer = 0;
    if (iters) *iters = iterations;
    if (relres) *relres = rel;
    if (flag[2] == 1) return fail(h, FL_EBREAKDOWN, "CG breakdown: p.Ap <= 0");
    if (flag[2] == 2) return fail(h, FL_ENONFINITE, "non-finite residual");
    if (!(rel <= rtol)) return FL_ENOCONV;
    return FL_OK;
}

int fl_energy_error2(fl_handle* h, double fu, const double* b, const double* uh, double* e2_out) {
    if (!h || !e2_out) return FL_EINVAL;
    if (!h->assembled) return fail(h, FL_ESTATE, "no assembled matrix");
    if (h->n == 0) {
        *e2_out = fu;
        return FL_OK;
    }
    if (!b || !uh) return fail(h, FL_EINVAL, "null vector");
    HIPCHK(hipSetDevice(h->device));
    int rc = ensure_solver(h);
    if (rc) return rc;
    const int64_t n = h->n;
    double* y = h->w + 6 * n;
    launch_symv(h->sym, h->dA, h->lda, uh, y, h->stream);
    const int nblk = (int)std::min<int64_t>((n + 255) / 256, 1024);
    launch_dot2(uh, b, y, n, h->w_part, nblk, stat_scal(h->w_stat) + 8, h->stream);
    HIPCHK(hipGetLastError());
    if ((rc = pull_status(h))) return rc;
    const double* r = stat_scal(h->w_hstat) + 8;
    *e2_out = fu - 2.0 * r[0] + r[1];
    return FL_OK;
}

int fl_stats(const fl_handle* h, fl_stats_t* out) {
    if (!h || !out) return FL_EINVAL;
    *out = h->st;
    return FL_OK;
}

}  // extern "C"
