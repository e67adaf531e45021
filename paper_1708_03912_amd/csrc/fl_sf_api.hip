// Host side of the strong-form evaluation and the error indicators
// (include/fraclap.h: fl_eval_points, fl_strong_form, fl_indicators).
// Sec. 4: the indicators eta-hat_i need the L2 norms of the residual
// f - (-Delta)^s u_h on every cell, and the lemma on the strong form turns
// the pointwise values into regular boundary integrals (eq. 8; eq. 9 for
// d = 1, s = 1/2).  The plan holds the geometry (evaluation points,
// facets, Gauss points on the facets, touching-cell lists); the kernels
// (fl_sf.hip) take the coefficients of u.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "fl_handle.hpp"
#include "fl_internal.hpp"

using namespace fl;

namespace {

constexpr int SF_WG_TARGETS = 512;   // targets per far-kernel workgroup
constexpr int SF_MAX_CHUNKS = 64;

int sfail(fl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return sfail(h, FL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
int sf_upload(fl_handle* h, T** p, const std::vector<T>& v) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(v.size(), 1)) != hipSuccess)
        return sfail(h, FL_ENOMEM, "strong form: device allocation failed");
    h->sf.bufs.push_back(q);
    *p = (T*)q;
    if (!v.empty()) HIPCHK(hipMemcpy(q, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return FL_OK;
}

template <class T>
int sf_alloc(fl_handle* h, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
        return sfail(h, FL_ENOMEM, "strong form: device allocation failed");
    h->sf.bufs.push_back(q);
    *p = (T*)q;
    return FL_OK;
}

void sf_cl_release(fl_handle* h) {
    for (void* p : h->sf.clbufs) (void)hipFree(p);
    h->sf.clbufs.clear();
    h->sf.cl_ready = false;
    h->sf.cl_up.clear();
    h->sf.cl_down.clear();
    h->sf.cl_upc.clear();
    h->sf.cl_downc.clear();
    h->sf.C = SfClDev{};
}

void sf_release(fl_handle* h) {
    sf_cl_release(h);
    for (void* p : h->sf.bufs) (void)hipFree(p);
    h->sf = fl_sf{};
}

template <class T>
int cl_upload(fl_handle* h, T** p, const std::vector<T>& v) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(v.size(), 1)) != hipSuccess)
        return sfail(h, FL_ENOMEM, "strong form: device allocation failed");
    h->sf.clbufs.push_back(q);
    *p = (T*)q;
    if (!v.empty()) HIPCHK(hipMemcpy(q, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return FL_OK;
}

struct SfCl {
    int lo, hi, level, parent;
    double blo[2], side;
    std::vector<int> sons;
};

bool sf_admissible(const SfCl& a, const SfCl& b, double eta) {
    double g2 = 0.0;
    for (int j = 0; j < 2; ++j) {
        const double g = std::max(0.0, std::max(b.blo[j] - (a.blo[j] + a.side), a.blo[j] - (b.blo[j] + b.side)));
        g2 += g * g;
    }
    return eta * std::sqrt(g2) >= std::max(a.side * std::sqrt(2.0), b.side * std::sqrt(2.0));
}

// Evaluation rule of a cell with k points per direction: barycentric
// coordinates (Q x (d+1)) and weights on the reference cell summing to 1.
// d = 2: the collapsed Gauss rule (Gauss-Jacobi(1,0) x Gauss-Legendre);
// d = 1: Gauss-Legendre.
void eval_rule(int dim, int k, std::vector<double>& lam, std::vector<double>& w) {
    const RuleTables& R = fl_base_rules();
    lam.clear();
    w.clear();
    if (dim == 1) {
        for (int i = 0; i < k; ++i) {
            const double t = R.gl_x[gl_off(k) + i];
            lam.push_back(1.0 - t);
            lam.push_back(t);
            w.push_back(R.gl_w[gl_off(k) + i]);
        }
    } else {
        for (int m = tri_off(k); m < tri_off(k) + k * k; ++m) {
            const double l1 = R.tl1[m], l2 = R.tl2[m];
            lam.push_back(1.0 - l1 - l2);
            lam.push_back(l1);
            lam.push_back(l2);
            w.push_back(R.tw[m]);
        }
    }
}

// Points (nc x Q x dim) and weights times |K| (nc x Q), cells in the
// caller's order.
void eval_points_host(const fl_handle* h, int k, std::vector<double>& X, std::vector<double>& W) {
    const int dim = h->dim, nper = dim + 1;
    std::vector<double> lam, w;
    eval_rule(dim, k, lam, w);
    const int Q = (int)w.size();
    X.assign((size_t)h->nc * Q * dim, 0.0);
    W.assign((size_t)h->nc * Q, 0.0);
    for (int64_t K = 0; K < h->nc; ++K) {
        const int32_t* c = &h->cells[nper * K];
        double meas;
        if (dim == 1) {
            meas = std::fabs(h->verts[c[1]] - h->verts[c[0]]);
        } else {
            const double* a = &h->verts[2 * c[0]];
            const double* b = &h->verts[2 * c[1]];
            const double* d = &h->verts[2 * c[2]];
            meas = 0.5 * std::fabs((b[0] - a[0]) * (d[1] - a[1]) - (d[0] - a[0]) * (b[1] - a[1]));
        }
        for (int q = 0; q < Q; ++q) {
            for (int j = 0; j < dim; ++j) {
                double x = 0.0;
                for (int a = 0; a < nper; ++a) x += lam[q * nper + a] * h->verts[dim * c[a] + j];
                X[((size_t)K * Q + q) * dim + j] = x;
            }
            W[(size_t)K * Q + q] = meas * w[q];
        }
    }
}

int check_rules(fl_handle* h, int k, int qf, int qn) {
    if (k < 1 || k > 8) return sfail(h, FL_EINVAL, "k_eval must lie in 1..8");
    if (qf < 1 || qf > 16 || qn < 1 || qn > 16) return sfail(h, FL_EINVAL, "q_far and q_near must lie in 1..16");
    return FL_OK;
}

// Geometry of the evaluation for (mesh, DOF map, k, qf, qn).
int sf_plan(fl_handle* h, int k, int qf, int qn) {
    fl_sf& S = h->sf;
    if (S.ready && S.k == k && S.qf == qf && S.qn == qn && S.n == h->n) return FL_OK;
    HIPCHK(hipStreamSynchronize(h->stream));  // earlier launches may still read the old plan
    sf_release(h);
    const int dim = h->dim, nper = dim + 1;
    const int64_t T = h->nc, nv = h->nv;
    if (dim == 1) {
        // the kernel-power tables cover r^2 in [2^-128, 2^128): points lie
        // at least 0.0198 h_K from the vertices for k <= 8
        double lo = h->verts[0], hi = h->verts[0], hmin = INFINITY;
        for (int64_t v = 0; v < nv; ++v) lo = std::min(lo, h->verts[v]), hi = std::max(hi, h->verts[v]);
        for (int64_t K = 0; K < T; ++K)
            hmin = std::min(hmin, std::fabs(h->verts[h->cells[2 * K + 1]] - h->verts[h->cells[2 * K]]));
        if (!(hi - lo < 0x1p60) || !(hmin >= 0x1p-56))
            return sfail(h, FL_EMESH, "interval mesh outside the supported scale (cells >= 2^-56, extent < 2^60)");
    }
    std::vector<double> lam, wq, X, W;
    eval_rule(dim, k, lam, wq);
    const int Q = (int)wq.size();
    eval_points_host(h, k, X, W);
    const long long nt = (long long)T * Q;
    std::vector<double> tx(nt), ty(nt, 0.0), h2(T), cx((size_t)T * nper * dim);
    std::vector<int> cdof((size_t)T * nper);
    for (long long t = 0; t < nt; ++t) {
        tx[t] = X[(size_t)t * dim];
        if (dim == 2) ty[t] = X[(size_t)t * dim + 1];
    }
    for (int64_t K = 0; K < T; ++K) {
        const int32_t* c = &h->cells[nper * K];
        for (int a = 0; a < nper; ++a) {
            cdof[K * nper + a] = h->node2dof[c[a]];
            for (int j = 0; j < dim; ++j) cx[(K * nper + a) * dim + j] = h->verts[dim * c[a] + j];
        }
        double m = 0.0;
        for (int a = 0; a < nper; ++a)
            for (int b = a + 1; b < nper; ++b) {
                double l = 0.0;
                for (int j = 0; j < dim; ++j) {
                    const double e = h->verts[dim * c[b] + j] - h->verts[dim * c[a] + j];
                    l += e * e;
                }
                m = std::max(m, l);
            }
        h2[K] = m;
    }
    // vertex -> cells (increasing)
    std::vector<int> vptr(nv + 1, 0), vidx((size_t)T * nper);
    for (int64_t i = 0; i < T * nper; ++i) vptr[h->cells[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    {
        std::vector<int> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t K = 0; K < T; ++K)
            for (int a = 0; a < nper; ++a) vidx[fill[h->cells[nper * K + a]]++] = (int)K;
    }
    // facets: (K1, local index e1) and (K2, e2) or K2 = -1
    std::vector<int> fK;
    std::vector<int> fE;
    if (dim == 1) {
        for (int64_t v = 0; v < nv; ++v) {
            const int n = vptr[v + 1] - vptr[v];
            if (n == 0) continue;
            const int K1 = vidx[vptr[v]];
            fK.push_back(K1);
            fK.push_back(n > 1 ? vidx[vptr[v] + 1] : -1);
            fE.push_back(h->cells[2 * K1] == v ? 0 : 1);
        }
    } else {
        std::vector<unsigned long long> key((size_t)T * 3);
        for (int64_t K = 0; K < T; ++K)
            for (int e = 0; e < 3; ++e) {
                const unsigned a = (unsigned)h->cells[3 * K + e], b = (unsigned)h->cells[3 * K + (e + 1) % 3];
                const unsigned long long lo = std::min(a, b), hi = std::max(a, b);
                key[K * 3 + e] = (lo << 32) | hi;
            }
        std::vector<int64_t> ord((size_t)T * 3);
        for (int64_t i = 0; i < T * 3; ++i) ord[i] = i;
        std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return key[x] < key[y] || (key[x] == key[y] && x < y); });
        for (size_t i = 0; i < ord.size();) {
            size_t j = i + 1;
            while (j < ord.size() && key[ord[j]] == key[ord[i]]) ++j;
            if (j - i > 2) return sfail(h, FL_EMESH, "an edge lies on more than two cells");
            fK.push_back((int)(ord[i] / 3));
            fK.push_back(j - i == 2 ? (int)(ord[i + 1] / 3) : -1);
            fE.push_back((int)(ord[i] % 3));
            i = j;
        }
    }
    const long long nf = (long long)fE.size();
    const RuleTables& R = fl_base_rules();
    const int qsrc = dim == 1 ? 1 : qf;
    const long long ns = nf * qsrc;
    std::vector<double> fN(nf * dim), sx(ns), sy(ns, 0.0);
    std::vector<int2> bf;
    for (long long f = 0; f < nf; ++f) {
        const int K1 = fK[2 * f], e = fE[f];
        const int32_t* c = &h->cells[nper * K1];
        if (dim == 1) {
            const double p = h->verts[c[e]], o = h->verts[c[1 - e]];
            fN[f] = p > o ? 1.0 : -1.0;
            sx[f] = p;
        } else {
            const double* A = &h->verts[2 * c[e]];
            const double* B = &h->verts[2 * c[(e + 1) % 3]];
            const double* Cc = &h->verts[2 * c[(e + 2) % 3]];
            const double E0 = B[0] - A[0], E1 = B[1] - A[1];
            const double det = E0 * (Cc[1] - A[1]) - (Cc[0] - A[0]) * E1;
            const double sg = det > 0.0 ? 1.0 : -1.0;
            fN[2 * f] = sg * E1;
            fN[2 * f + 1] = -sg * E0;
            for (int j = 0; j < qf; ++j) {
                const double t = R.gl_x[gl_off(qf) + j];
                sx[f * qf + j] = std::fma(t, E0, A[0]);
                sy[f * qf + j] = std::fma(t, E1, A[1]);
            }
        }
        if (fK[2 * f + 1] < 0) bf.push_back(make_int2(K1, e));
    }
    // boundary sources (value terms, only if boundary vertices carry DOFs):
    // the q_far points of each boundary facet in its cell's orientation
    int bnd_u = 0;
    for (int64_t v = 0; v < nv; ++v)
        if (h->on_boundary[v] && h->node2dof[v] >= 0) bnd_u = 1;
    std::vector<double> bsx, bsy;
    if (bnd_u)
        for (const int2& kb : bf) {
            const int32_t* c = &h->cells[nper * kb.x];
            if (dim == 1) {
                bsx.push_back(h->verts[c[kb.y]]);
                bsy.push_back(0.0);
            } else {
                const double* A = &h->verts[2 * c[kb.y]];
                const double* B = &h->verts[2 * c[(kb.y + 1) % 3]];
                for (int j = 0; j < qf; ++j) {
                    const double t = R.gl_x[gl_off(qf) + j];
                    bsx.push_back(std::fma(t, B[0] - A[0], A[0]));
                    bsy.push_back(std::fma(t, B[1] - A[1], A[1]));
                }
            }
        }
    const long long nbs = (long long)bsx.size();
    // touching cells: sharing a vertex (d = 2), the cell itself (d = 1)
    std::vector<int> nptr(T + 1, 0), nidx;
    {
        std::vector<int> tmp;
        for (int64_t K = 0; K < T; ++K) {
            if (dim == 1) {
                nidx.push_back((int)K);
            } else {
                tmp.clear();
                for (int a = 0; a < 3; ++a) {
                    const int v = h->cells[3 * K + a];
                    tmp.insert(tmp.end(), vidx.begin() + vptr[v], vidx.begin() + vptr[v + 1]);
                }
                std::sort(tmp.begin(), tmp.end());
                tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
                nidx.insert(nidx.end(), tmp.begin(), tmp.end());
            }
            nptr[K + 1] = (int)nidx.size();
        }
    }
    // far-kernel grid: enough workgroups for the chip, sources split in chunks
    const long long ntb = (nt + SF_WG_TARGETS - 1) / SF_WG_TARGETS;
    int nch = (int)std::min<long long>(SF_MAX_CHUNKS, std::max<long long>(1, (2048 + ntb - 1) / std::max<long long>(ntb, 1)));
    long long chunk = (ns + nch - 1) / nch;
    chunk = std::max<long long>(256, (chunk + 255) / 256 * 256);
    nch = (int)std::max<long long>(1, (ns + chunk - 1) / chunk);
    const int nchb = (int)((nbs + chunk - 1) / chunk);

    std::vector<double> gx(R.gl_x, R.gl_x + GL_TAB), gw(R.gl_w, R.gl_w + GL_TAB);
    SfDev D{};
    D.dim = dim;
    D.Q = Q;
    D.T = T;
    D.nt = nt;
    D.nf = nf;
    D.qf = dim == 1 ? 1 : qf;
    D.qn = dim == 1 ? 1 : qn;
    D.ns = ns;
    D.nbf = (long long)bf.size();
    D.bnd_u = bnd_u;
    D.nbs = nbs;
    int rc;
    double *p_cx, *p_lam, *p_tx, *p_ty, *p_fN, *p_gx, *p_gw, *p_sc, *p_bc;
    int *p_cdof, *p_fK, *p_nptr, *p_nidx;
    int2* p_bf;
    if ((rc = sf_upload(h, &p_cx, cx)) || (rc = sf_upload(h, &p_cdof, cdof)) || (rc = sf_upload(h, &p_lam, lam)) ||
        (rc = sf_upload(h, &p_tx, tx)) || (rc = sf_upload(h, &p_ty, ty)) || (rc = sf_upload(h, &p_fK, fK)) ||
        (rc = sf_upload(h, &p_fN, fN)) || (rc = sf_upload(h, &p_gx, gx)) || (rc = sf_upload(h, &p_gw, gw)) ||
        (rc = sf_upload(h, &p_nptr, nptr)) || (rc = sf_upload(h, &p_nidx, nidx)) || (rc = sf_upload(h, &p_bf, bf)) ||
        (rc = sf_upload(h, &S.sx, sx)) || (rc = sf_upload(h, &S.sy, sy)) || (rc = sf_upload(h, &S.W, W)) ||
        (rc = sf_upload(h, &S.h2, h2)) || (rc = sf_upload(h, &S.vptr, vptr)) || (rc = sf_upload(h, &S.vidx, vidx)) ||
        (rc = sf_upload(h, &S.bsx, bsx)) || (rc = sf_upload(h, &S.bsy, bsy)) ||
        (rc = sf_alloc(h, &p_bc, (size_t)2 * nbs)) ||
        (rc = sf_alloc(h, &p_sc, (size_t)ns)) || (rc = sf_alloc(h, &S.part, (size_t)(nch + nchb) * nt)) ||
        (rc = sf_alloc(h, &S.tab, 776))) {
        sf_release(h);
        return rc;
    }
    D.cx = p_cx;
    D.cdof = p_cdof;
    D.lam = p_lam;
    D.tx = p_tx;
    D.ty = p_ty;
    D.fK = p_fK;
    D.fN = p_fN;
    D.gx = p_gx;
    D.gw = p_gw;
    D.sc = p_sc;
    D.bc = p_bc;
    D.nptr = p_nptr;
    D.nidx = p_nidx;
    D.bf = p_bf;
    S.D = D;
    S.k = k;
    S.qf = qf;
    S.qn = qn;
    S.n = h->n;
    S.nch = nch;
    S.nchb = nchb;
    S.chunk = chunk;
    S.tab_s = -1.0;
    S.ready = true;
    return FL_OK;
}

// Cell tree, block lists and source ownership of the cluster evaluation
// (d = 2): the same construction as the oracle's (median split of the
// centroids along their longest extent, cube boxes of the cells' vertex
// bounding boxes, admissibility eta dist >= max diam).
int sf_cl_plan(fl_handle* h, int m, double eta, int leaf) {
    fl_sf& S = h->sf;
    if (S.cl_ready && S.cl_m == m && S.cl_eta == eta && S.cl_leaf == leaf) return FL_OK;
    HIPCHK(hipStreamSynchronize(h->stream));
    sf_cl_release(h);
    const int64_t T = h->nc;
    std::vector<double> cx(T), cy(T), lo0(T), lo1(T), hi0(T), hi1(T);
    for (int64_t K = 0; K < T; ++K) {
        const int32_t* c = &h->cells[3 * K];
        const double* a = &h->verts[2 * c[0]];
        const double* b = &h->verts[2 * c[1]];
        const double* d = &h->verts[2 * c[2]];
        cx[K] = ((a[0] + b[0]) + d[0]) / 3.0;
        cy[K] = ((a[1] + b[1]) + d[1]) / 3.0;
        lo0[K] = std::min(std::min(a[0], b[0]), d[0]);
        lo1[K] = std::min(std::min(a[1], b[1]), d[1]);
        hi0[K] = std::max(std::max(a[0], b[0]), d[0]);
        hi1[K] = std::max(std::max(a[1], b[1]), d[1]);
    }
    std::vector<SfCl> cl;
    std::vector<int> perm(T);
    std::function<int(std::vector<int>&, int, int, int)> make = [&](std::vector<int>& idx, int lo, int level,
                                                                    int parent) -> int {
        SfCl c;
        c.lo = lo;
        c.hi = lo + (int)idx.size();
        c.level = level;
        c.parent = parent;
        double bl[2] = {INFINITY, INFINITY}, bh[2] = {-INFINITY, -INFINITY};
        for (int K : idx) {
            bl[0] = std::min(bl[0], lo0[K]);
            bl[1] = std::min(bl[1], lo1[K]);
            bh[0] = std::max(bh[0], hi0[K]);
            bh[1] = std::max(bh[1], hi1[K]);
        }
        const double side = std::max(bh[0] - bl[0], bh[1] - bl[1]);
        c.side = side;
        for (int j = 0; j < 2; ++j) c.blo[j] = 0.5 * (bl[j] + bh[j]) - 0.5 * side;
        const int cid = (int)cl.size();
        cl.push_back(c);
        for (size_t k = 0; k < idx.size(); ++k) perm[lo + k] = idx[k];
        if ((int)idx.size() > leaf) {
            double e0l = INFINITY, e0h = -INFINITY, e1l = INFINITY, e1h = -INFINITY;
            for (int K : idx) {
                e0l = std::min(e0l, cx[K]);
                e0h = std::max(e0h, cx[K]);
                e1l = std::min(e1l, cy[K]);
                e1h = std::max(e1h, cy[K]);
            }
            const int ax = (e1h - e1l > e0h - e0l) ? 1 : 0;
            const std::vector<double>& key = ax == 0 ? cx : cy;
            std::vector<int> order(idx);
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
            const size_t half = order.size() / 2;
            std::vector<int> p1(order.begin(), order.begin() + half), p2(order.begin() + half, order.end());
            const int s1 = make(p1, lo, level + 1, cid);
            cl[cid].sons.push_back(s1);
            const int s2 = make(p2, lo + (int)half, level + 1, cid);
            cl[cid].sons.push_back(s2);
        }
        return cid;
    };
    {
        std::vector<int> all(T);
        for (int64_t K = 0; K < T; ++K) all[K] = (int)K;
        make(all, 0, 0, -1);
    }
    const int nc = (int)cl.size();
    std::vector<std::pair<int, int>> far, near;
    std::function<void(int, int)> rec = [&](int a, int b) {
        if (sf_admissible(cl[a], cl[b], eta)) {
            far.push_back({a, b});
            return;
        }
        const bool la = cl[a].sons.empty(), lb = cl[b].sons.empty();
        if (la && lb) near.push_back({a, b});
        else if (la) for (int t : cl[b].sons) rec(a, t);
        else if (lb) for (int t : cl[a].sons) rec(t, b);
        else for (int u : cl[a].sons) for (int t : cl[b].sons) rec(u, t);
    };
    rec(0, 0);
    std::stable_sort(far.begin(), far.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        return a.first < b.first;
    });
    std::vector<int> leaf_ids, leaf_of(nc, -1);
    for (int c = 0; c < nc; ++c)
        if (cl[c].sons.empty()) {
            leaf_of[c] = (int)leaf_ids.size();
            leaf_ids.push_back(c);
        }
    std::stable_sort(near.begin(), near.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        return leaf_of[a.first] < leaf_of[b.first];
    });
    std::vector<int> clo(nc), chi(nc), cpar(nc), sptr(nc + 1, 0), sidx;
    std::vector<double> box(3 * (size_t)nc);
    int depth = 0;
    for (int c = 0; c < nc; ++c) {
        clo[c] = cl[c].lo;
        chi[c] = cl[c].hi;
        cpar[c] = cl[c].parent;
        box[3 * c] = cl[c].blo[0];
        box[3 * c + 1] = cl[c].blo[1];
        box[3 * c + 2] = cl[c].side;
        for (int sn : cl[c].sons) sidx.push_back(sn);
        sptr[c + 1] = (int)sidx.size();
        depth = std::max(depth, cl[c].level);
    }
    std::vector<long long> fptr(nc + 1, 0);
    std::vector<int> fdst;
    for (auto& p : far) {
        fdst.push_back(p.second);
        fptr[p.first + 1]++;
    }
    for (int c = 0; c < nc; ++c) fptr[c + 1] += fptr[c];
    const int nleaf = (int)leaf_ids.size();
    std::vector<int> lnptr(nleaf + 1, 0), ndst;
    for (auto& p : near) {
        ndst.push_back(p.second);
        lnptr[leaf_of[p.first] + 1]++;
    }
    for (int l = 0; l < nleaf; ++l) lnptr[l + 1] += lnptr[l];
    // edges owned by each tree position (the edge's first cell)
    std::vector<int> pos(T);
    for (int64_t k = 0; k < T; ++k) pos[perm[k]] = (int)k;
    std::vector<int> fK(2 * S.D.nf);
    HIPCHK(hipMemcpy(fK.data(), S.D.fK, sizeof(int) * fK.size(), hipMemcpyDeviceToHost));
    std::vector<int> optr(T + 1, 0), oidx(S.D.nf);
    for (long long f = 0; f < S.D.nf; ++f) optr[pos[fK[2 * f]] + 1]++;
    for (int64_t k = 0; k < T; ++k) optr[k + 1] += optr[k];
    {
        std::vector<int> fill(optr.begin(), optr.end() - 1);
        for (long long f = 0; f < S.D.nf; ++f) oidx[fill[pos[fK[2 * f]]]++] = (int)f;
    }
    std::vector<double> tnode(m);
    for (int k = 0; k < m; ++k) tnode[k] = 0.5 - 0.5 * std::cos((2.0 * k + 1.0) * M_PI / (2.0 * m));
    // per-level lists, four ints per entry: upward {c, son 0, son 1, 0},
    // downward {c, parent, 0, 0} (the bisection gives two sons)
    std::vector<std::vector<int>> up(depth + 1), down(depth + 1);
    for (int c = 0; c < nc; ++c) {
        if (!cl[c].sons.empty()) {
            if (cl[c].sons.size() != 2) return sfail(h, FL_EINVAL, "cell tree: internal cluster without two sons");
            for (int v : {c, cl[c].sons[0], cl[c].sons[1], 0}) up[cl[c].level].push_back(v);
        }
        if (c > 0)
            for (int v : {c, cpar[c], 0, 0}) down[cl[c].level].push_back(v);
    }
    SfClDev C{};
    C.m = m;
    C.M = m * m;
    C.nc = nc;
    C.nleaf = nleaf;
    int rc;
    int *p_clo, *p_chi, *p_cpar, *p_sptr, *p_sidx, *p_perm, *p_leaf, *p_optr, *p_oidx, *p_fdst, *p_lnptr, *p_ndst;
    double *p_box, *p_tnode;
    long long* p_fptr;
    if ((rc = cl_upload(h, &p_clo, clo)) || (rc = cl_upload(h, &p_chi, chi)) || (rc = cl_upload(h, &p_cpar, cpar)) ||
        (rc = cl_upload(h, &p_sptr, sptr)) || (rc = cl_upload(h, &p_sidx, sidx)) || (rc = cl_upload(h, &p_perm, perm)) ||
        (rc = cl_upload(h, &p_leaf, leaf_ids)) || (rc = cl_upload(h, &p_optr, optr)) ||
        (rc = cl_upload(h, &p_oidx, oidx)) || (rc = cl_upload(h, &p_fdst, fdst)) ||
        (rc = cl_upload(h, &p_lnptr, lnptr)) || (rc = cl_upload(h, &p_ndst, ndst)) || (rc = cl_upload(h, &p_box, box)) ||
        (rc = cl_upload(h, &p_tnode, tnode)) || (rc = cl_upload(h, &p_fptr, fptr))) {
        sf_cl_release(h);
        return rc;
    }
    C.clo = p_clo;
    C.chi = p_chi;
    C.cpar = p_cpar;
    C.sptr = p_sptr;
    C.sidx = p_sidx;
    C.perm = p_perm;
    C.leaf = p_leaf;
    C.optr = p_optr;
    C.oidx = p_oidx;
    C.fdst = p_fdst;
    C.lnptr = p_lnptr;
    C.ndst = p_ndst;
    C.box = p_box;
    C.tnode = p_tnode;
    C.fptr = p_fptr;
    std::vector<double> zT((size_t)nc * C.M * C.M, 0.0), zc((size_t)nc * C.M, 0.0);
    if ((rc = cl_upload(h, &C.T, zT)) || (rc = cl_upload(h, &C.mom, zc)) || (rc = cl_upload(h, &C.loc, zc))) {
        sf_cl_release(h);
        return rc;
    }
    for (int l = depth; l >= 0; --l) {
        int* q = nullptr;
        if ((rc = cl_upload(h, &q, up[l]))) {
            sf_cl_release(h);
            return rc;
        }
        S.cl_up.push_back(q);
        S.cl_upc.push_back((int)up[l].size() / 4);
    }
    for (int l = 1; l <= depth; ++l) {
        int* q = nullptr;
        if ((rc = cl_upload(h, &q, down[l]))) {
            sf_cl_release(h);
            return rc;
        }
        S.cl_down.push_back(q);
        S.cl_downc.push_back((int)down[l].size() / 4);
    }
    launch_sfc_transfer(C, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    S.C = C;
    S.cl_m = m;
    S.cl_eta = eta;
    S.cl_leaf = leaf;
    S.cl_ready = true;
    return FL_OK;
}

bool log_form(int dim, double s) { return dim == 1 && std::fabs(s - 0.5) < 1e-15; }

// kernel-power tables of r2^pe, pe = -(d + 2s - 2)/2: pairs (1/m_i,
// m_i^pe), 2^(pe n), the Taylor coefficients (776 doubles)
int sf_tables(fl_handle* h, double s) {
    fl_sf& S = h->sf;
    if (S.tab_s == s) return FL_OK;
    std::unique_ptr<RuleTables> R(new RuleTables(fl_base_rules()));
    set_pow_tables(*R, -0.5 * (h->dim + 2.0 * s - 2.0));
    std::vector<double> t(776, 0.0);
    for (int i = 0; i < 256; ++i) {
        t[2 * i] = R->pw_inv[i];
        t[2 * i + 1] = R->pw_fr[i];
        t[512 + i] = R->pw_ex[i];
    }
    for (int i = 0; i < 8; ++i) t[768 + i] = R->pw_c[i];
    HIPCHK(hipStreamSynchronize(h->stream));  // earlier launches may still read the old tables
    HIPCHK(hipMemcpy(S.tab, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
    S.tab_s = s;
    return FL_OK;
}

}  // namespace

void fl_sf_free(fl_handle* h) { sf_release(h); }

extern "C" {

int fl_eval_points(fl_handle* h, int32_t k_eval, double* x, double* w) {
    if (!h) return FL_EINVAL;
    if (h->dim == 0) return sfail(h, FL_ESTATE, "fl_set_mesh must be called first");
    if (k_eval < 1 || k_eval > 8) return sfail(h, FL_EINVAL, "k_eval must lie in 1..8");
    if (!x || !w) return sfail(h, FL_EINVAL, "null output");
    HIPCHK(hipSetDevice(h->device));
    std::vector<double> X, W;
    eval_points_host(h, k_eval, X, W);
    HIPCHK(hipMemcpyAsync(x, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(w, W.data(), sizeof(double) * W.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FL_OK;
}

int fl_strong_form(fl_handle* h, double s, const double* u, int32_t k_eval, int32_t q_far, int32_t q_near,
                   double* Lu) {
    if (!h) return FL_EINVAL;
    if (!h->planned) return sfail(h, FL_ESTATE, "no DOF map: call fl_assemble first");
    if (!(s > 0.0 && s < 1.0)) return sfail(h, FL_EINVAL, "s must lie in (0,1)");
    if (!Lu || (!u && h->n > 0)) return sfail(h, FL_EINVAL, "null vector");
    int rc = check_rules(h, k_eval, q_far, q_near);
    if (rc) return rc;
    HIPCHK(hipSetDevice(h->device));
    if ((rc = sf_plan(h, k_eval, q_far, q_near))) return rc;
    const bool logk = log_form(h->dim, s);
    if (!logk && (rc = sf_tables(h, s))) return rc;
    fl_sf& S = h->sf;
    SfDev D = S.D;
    const double d2 = h->dim + 2.0 * s - 2.0;
    D.pe = -0.5 * d2;
    D.inv2s = 1.0 / (2.0 * s);
    D.cg = logk ? 1.0 / (2.0 * s) : 1.0 / (2.0 * s * d2);
    D.cg_own = logk ? 1.0 : 1.0 / d2;
    D.C = fl_cdn(h->dim, s);
    launch_sf_sources(D, u, h->stream);
    launch_sf_far(D, S.sx, S.sy, S.bsx, S.bsy, S.chunk, S.nch, S.nchb, S.tab, S.part, logk, h->stream);
    launch_sf_near(D, u, S.part, S.nch + S.nchb, S.tab, Lu, logk, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_strong_form_cluster(fl_handle* h, double s, const double* u, int32_t k_eval, int32_t q_far, int32_t q_near,
                           int32_t m, double eta, int32_t leaf, double* Lu) {
    if (!h) return FL_EINVAL;
    if (!h->planned) return sfail(h, FL_ESTATE, "no DOF map: call fl_assemble first");
    if (h->dim != 2) return sfail(h, FL_EINVAL, "the cluster evaluation is for triangle meshes (dim 2)");
    if (!(s > 0.0 && s < 1.0)) return sfail(h, FL_EINVAL, "s must lie in (0,1)");
    if (!Lu || (!u && h->n > 0)) return sfail(h, FL_EINVAL, "null vector");
    if (m < 1 || m > 15) return sfail(h, FL_EINVAL, "m must lie in 1..15");
    if (!(eta > 0.0) || !std::isfinite(eta)) return sfail(h, FL_EINVAL, "eta must be positive and finite");
    if (leaf < 1 || leaf > 1024) return sfail(h, FL_EINVAL, "leaf must lie in 1..1024");
    int rc = check_rules(h, k_eval, q_far, q_near);
    if (rc) return rc;
    HIPCHK(hipSetDevice(h->device));
    if ((rc = sf_plan(h, k_eval, q_far, q_near))) return rc;
    if ((rc = sf_tables(h, s))) return rc;
    if ((rc = sf_cl_plan(h, m, eta, leaf))) return rc;
    fl_sf& S = h->sf;
    SfDev D = S.D;
    const double d2 = 2.0 * s;
    D.pe = -0.5 * d2;
    D.inv2s = 1.0 / (2.0 * s);
    D.cg = 1.0 / (2.0 * s * d2);
    D.cg_own = 1.0 / d2;
    D.C = fl_cdn(2, s);
    launch_sf_sources(D, u, h->stream);
    // row 0: no direct sources (zeros), rows 1..nchb: the boundary value terms
    SfDev Dz = D;
    Dz.ns = 0;
    launch_sf_far(Dz, S.sx, S.sy, S.bsx, S.bsy, S.chunk, 1, S.nchb, S.tab, S.part, false, h->stream);
    launch_sfc_eval(S.C, D, S.sx, S.sy, S.cl_up.data(), S.cl_upc.data(), (int)S.cl_up.size(), S.cl_down.data(),
                    S.cl_downc.data(), (int)S.cl_down.size(), S.tab, S.part, h->stream);
    launch_sf_near(D, u, S.part, 1 + S.nchb, S.tab, Lu, false, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_indicators(fl_handle* h, double s, const double* Lu, const double* f, int32_t k_eval, double* eta_cell,
                  double* eta_node) {
    if (!h) return FL_EINVAL;
    if (!(s > 0.0 && s < 1.0)) return sfail(h, FL_EINVAL, "s must lie in (0,1)");
    if (!Lu || !eta_cell) return sfail(h, FL_EINVAL, "null vector");
    if (!h->sf.ready || h->sf.k != k_eval)
        return sfail(h, FL_ESTATE, "no strong-form evaluation with this k_eval: call fl_strong_form first");
    HIPCHK(hipSetDevice(h->device));
    const fl_sf& S = h->sf;
    launch_sf_indicators(S.D, Lu, f, S.W, S.h2, s, h->nv, S.vptr, S.vidx, eta_cell, eta_node, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

}  // extern "C"
