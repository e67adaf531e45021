// Host side of the cluster (H-matrix) approximation (include/fraclap.h:
// fl_cluster_build, fl_cluster_assemble, fl_cluster_matvec,
// fl_solve_cluster, fl_cluster_info).  Sec. 6: a cluster tree over the DOFs,
// cluster boxes (cubes containing the supports), admissible pairs
// eta dist >= max diam approximated by the tensor Chebyshev interpolation of
// the kernel with nested bases, the rest (leaf pairs) kept exactly.
// Readings: leaves of at most `leaf` DOFs (the paper's leaves are single
// DOFs); a cluster is split at the median of its DOF coordinates along the
// longest extent (stable order); its box is the cube of the largest extent
// of the supports' bounding box, centred on it.  The near blocks are copied
// from the assembled dense matrix (fl_cluster_build) or assembled from the
// element pairs of the element tiles that hold near pairs
// (fl_cluster_assemble): off-diagonal parts of every pair, diagonal-block
// parts of the pairs whose cells' anchor leaves are near, the rest of every
// cell's diagonal block through the far field (the kernel integrated over
// the far cells as the far field of the density 1).  Built without
// floating-point contraction so that the boxes, and with them the
// admissibility decisions, are those of an independent implementation of
// the same formulas.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "fl_handle.hpp"
#include "fl_internal.hpp"

using namespace fl;

namespace {

int cfail(fl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return cfail(h, FL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
int hm_upload(fl_handle* h, T** p, const std::vector<T>& v) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(v.size(), 1)) != hipSuccess)
        return cfail(h, FL_ENOMEM, "cluster approximation: device allocation failed");
    h->hm.bufs.push_back(q);
    h->hm.bytes += sizeof(T) * v.size();
    *p = (T*)q;
    if (!v.empty()) HIPCHK(hipMemcpy(q, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return FL_OK;
}

template <class T>
int hm_alloc(fl_handle* h, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
        return cfail(h, FL_ENOMEM, "cluster approximation: device allocation failed");
    h->hm.bufs.push_back(q);
    h->hm.bytes += sizeof(T) * count;
    *p = (T*)q;
    return FL_OK;
}

// frees one device allocation of the representation before the others
void hm_free(fl_handle* h, void* p, size_t bytes) {
    auto& b = h->hm.bufs;
    for (size_t i = 0; i < b.size(); ++i)
        if (b[i] == p) {
            (void)hipFree(p);
            b.erase(b.begin() + (long)i);
            h->hm.bytes -= bytes;
            return;
        }
}

void hm_release(fl_handle* h) {
    for (void* p : h->hm.bufs) (void)hipFree(p);
    if (h->hm.hsc) (void)hipHostFree(h->hm.hsc);
    h->hm = fl_hm{};
}

struct HCl {
    int lo, hi, level, parent;
    double blo[2], side;
    std::vector<int> sons;
};

bool admissible(const HCl& a, const HCl& b, double eta, int dim) {
    double g2 = 0.0;
    for (int j = 0; j < dim; ++j) {
        const double g = std::max(0.0, std::max(b.blo[j] - (a.blo[j] + a.side), a.blo[j] - (b.blo[j] + b.side)));
        g2 += g * g;
    }
    const double dist = std::sqrt(g2);
    const double sq = std::sqrt((double)dim);
    return eta * dist >= std::max(a.side * sq, b.side * sq);
}

// Tree, boxes and block partition of the current DOF map (host side).
struct HostTree {
    int dim = 0, depth = 0;
    std::vector<HCl> cl;
    std::vector<int> perm;                        // tree position -> DOF
    std::vector<std::pair<int, int>> far, near;   // near: by (leaf index, leaf index)
    std::vector<int> leaf_ids, leaf_of;           // leaf index -> cluster, cluster -> leaf index
    std::vector<int> anchor;                      // caller cell -> anchor DOF (-1: none)
};

// Cluster tree by median bisection of the DOF coordinates, the anchor DOF
// of every cell (its DOF vertex first in tree order; a cell without one
// takes the anchor of its facet neighbour of smallest index that has one,
// repeated until nothing changes), the boxes (cube of the largest extent of
// the supports' bounding box, centred on it; a cell without DOF widens its
// anchor's support box), and the block partition from (root, root).
void build_host_tree(const fl_handle* h, double eta, int leaf, HostTree& t) {
    const int dim = h->dim, nper = dim + 1;
    const int64_t n = (int64_t)h->dof_node.size(), nv = h->nv, T = h->nc;
    t = HostTree{};
    t.dim = dim;
    // supports: bounding box of the cells around every vertex
    std::vector<double> vlo(nv * 2, INFINITY), vhi(nv * 2, -INFINITY);
    auto cell_box = [&](int64_t K, double* clo, double* chi) {
        clo[0] = clo[1] = INFINITY;
        chi[0] = chi[1] = -INFINITY;
        for (int a = 0; a < nper; ++a)
            for (int j = 0; j < dim; ++j) {
                const double x = h->verts[dim * h->cells[nper * K + a] + j];
                clo[j] = std::min(clo[j], x);
                chi[j] = std::max(chi[j], x);
            }
    };
    for (int64_t K = 0; K < T; ++K) {
        double clo[2], chi[2];
        cell_box(K, clo, chi);
        for (int a = 0; a < nper; ++a) {
            const int v = h->cells[nper * K + a];
            for (int j = 0; j < dim; ++j) {
                vlo[2 * v + j] = std::min(vlo[2 * v + j], clo[j]);
                vhi[2 * v + j] = std::max(vhi[2 * v + j], chi[j]);
            }
        }
    }
    // tree structure (pre-order ids), perm: tree position -> DOF.  A
    // cluster's DOFs, in the order it received them, are stably sorted along
    // the axis of largest extent and split at the middle; the shape depends
    // on the sizes alone, so the pre-order id of every son is known before
    // the sorts (nodes(s) clusters under one of s DOFs) and the subtrees of
    // large clusters are built on host threads, with the same result as one
    // recursion
    t.perm.assign(n, 0);
    std::vector<double> cxy((size_t)n * dim);
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < dim; ++j) cxy[(size_t)i * dim + j] = h->verts[dim * h->dof_node[i] + j];
    std::function<int64_t(int64_t)> nodes = [&](int64_t sz) -> int64_t {
        return sz > leaf ? 1 + nodes(sz / 2) + nodes(sz - sz / 2) : 1;
    };
    if (n > 0) {
        t.cl.assign((size_t)nodes(n), HCl{});
        for (int64_t i = 0; i < n; ++i) t.perm[i] = (int)i;
        std::function<void(int, int, int, int, int)> make = [&](int lo, int hi, int level, int parent, int cid) {
            HCl& c = t.cl[cid];
            c.lo = lo;
            c.hi = hi;
            c.level = level;
            c.parent = parent;
            c.blo[0] = c.blo[1] = 0.0;
            c.side = 0.0;
            const int sz = hi - lo;
            if (sz <= leaf) return;
            int ax = 0;
            double best = -1.0;
            for (int j = 0; j < dim; ++j) {
                double lo_ = INFINITY, hi_ = -INFINITY;
                for (int r = lo; r < hi; ++r) {
                    const double x = cxy[(size_t)t.perm[r] * dim + j];
                    lo_ = std::min(lo_, x);
                    hi_ = std::max(hi_, x);
                }
                if (hi_ - lo_ > best) {
                    best = hi_ - lo_;
                    ax = j;
                }
            }
            std::vector<std::pair<double, int>> key(sz);
            for (int r = lo; r < hi; ++r) key[r - lo] = {cxy[(size_t)t.perm[r] * dim + ax], t.perm[r]};
            std::stable_sort(key.begin(), key.end(),
                             [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                                 return a.first < b.first;
                             });
            for (int r = lo; r < hi; ++r) t.perm[r] = key[r - lo].second;
            const int half = sz / 2;
            const int s1 = cid + 1, s2 = cid + 1 + (int)nodes(half);
            c.sons = {s1, s2};
            if (sz >= 8192) {
                std::thread left(make, lo, lo + half, level + 1, cid, s1);
                make(lo + half, hi, level + 1, cid, s2);
                left.join();
            } else {
                make(lo, lo + half, level + 1, cid, s1);
                make(lo + half, hi, level + 1, cid, s2);
            }
        };
        make(0, (int)n, 0, -1, 0);
    }
    // anchors
    std::vector<int> pos(n);
    for (int64_t r = 0; r < n; ++r) pos[t.perm[r]] = (int)r;
    t.anchor.assign(T, -1);
    bool dofless = false;
    for (int64_t K = 0; K < T; ++K) {
        int best = -1;
        for (int a = 0; a < nper; ++a) {
            const int i = h->node2dof[h->cells[nper * K + a]];
            if (i >= 0 && (best < 0 || pos[i] < pos[best])) best = i;
        }
        t.anchor[K] = best;
        dofless = dofless || best < 0;
    }
    if (dofless && n > 0) {
        // facet neighbours: cells sharing dim vertices (sorted facet keys)
        std::vector<std::pair<std::pair<int, int>, int>> fk;
        fk.reserve(T * nper);
        for (int64_t K = 0; K < T; ++K)
            for (int a = 0; a < nper; ++a) {
                int v0 = -1, v1 = -1;
                for (int b = 0; b < nper; ++b) {
                    if (b == a) continue;
                    const int v = h->cells[nper * K + b];
                    if (v0 < 0) v0 = v;
                    else v1 = v;
                }
                if (dim == 2 && v0 > v1) std::swap(v0, v1);
                fk.push_back({{v0, v1}, (int)K});
            }
        std::sort(fk.begin(), fk.end());
        std::vector<std::vector<int>> nbr(T);
        for (size_t i = 0; i < fk.size();) {
            size_t j = i;
            while (j < fk.size() && fk[j].first == fk[i].first) ++j;
            for (size_t a = i; a < j; ++a)
                for (size_t b = i; b < j; ++b)
                    if (a != b) nbr[fk[a].second].push_back(fk[b].second);
            i = j;
        }
        for (auto& v : nbr) std::sort(v.begin(), v.end());
        bool changed = true;
        while (changed) {
            changed = false;
            for (int64_t K = 0; K < T; ++K) {
                if (t.anchor[K] >= 0) continue;
                for (int k : nbr[K])
                    if (t.anchor[k] >= 0) {
                        t.anchor[K] = t.anchor[k];
                        changed = true;
                        break;
                    }
            }
        }
        for (int64_t K = 0; K < T; ++K) {
            bool has = false;
            for (int a = 0; a < nper; ++a) has = has || h->node2dof[h->cells[nper * K + a]] >= 0;
            if (has || t.anchor[K] < 0) continue;
            double clo[2], chi[2];
            cell_box(K, clo, chi);
            const int v = h->dof_node[t.anchor[K]];
            for (int j = 0; j < dim; ++j) {
                vlo[2 * v + j] = std::min(vlo[2 * v + j], clo[j]);
                vhi[2 * v + j] = std::max(vhi[2 * v + j], chi[j]);
            }
        }
    }
    // boxes
    for (HCl& c : t.cl) {
        double blo[2] = {INFINITY, INFINITY}, bhi[2] = {-INFINITY, -INFINITY};
        for (int r = c.lo; r < c.hi; ++r) {
            const int v = h->dof_node[t.perm[r]];
            for (int j = 0; j < dim; ++j) {
                blo[j] = std::min(blo[j], vlo[2 * v + j]);
                bhi[j] = std::max(bhi[j], vhi[2 * v + j]);
            }
        }
        double side = 0.0;
        for (int j = 0; j < dim; ++j) side = std::max(side, bhi[j] - blo[j]);
        c.side = side;
        c.blo[1] = 0.0;
        for (int j = 0; j < dim; ++j) {
            const double cen = 0.5 * (blo[j] + bhi[j]);
            c.blo[j] = cen - 0.5 * side;
        }
        t.depth = std::max(t.depth, c.level);
    }
    // admissible pairs and near leaf pairs (recursion from (root, root))
    std::function<void(int, int)> rec = [&](int s, int u) {
        if (admissible(t.cl[s], t.cl[u], eta, dim)) {
            t.far.push_back({s, u});
            return;
        }
        const bool ls = t.cl[s].sons.empty(), lt = t.cl[u].sons.empty();
        if (ls && lt) {
            t.near.push_back({s, u});
        } else if (ls) {
            for (int tt : t.cl[u].sons) rec(s, tt);
        } else if (lt) {
            for (int ss : t.cl[s].sons) rec(ss, u);
        } else {
            for (int ss : t.cl[s].sons)
                for (int tt : t.cl[u].sons) rec(ss, tt);
        }
    };
    const int nc = (int)t.cl.size();
    if (nc > 0) rec(0, 0);
    std::stable_sort(t.far.begin(), t.far.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
    t.leaf_of.assign(nc, -1);
    for (int c = 0; c < nc; ++c)
        if (t.cl[c].sons.empty()) {
            t.leaf_of[c] = (int)t.leaf_ids.size();
            t.leaf_ids.push_back(c);
        }
    std::stable_sort(t.near.begin(), t.near.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        const int la = t.leaf_of[a.first], lb = t.leaf_of[b.first];
        return la != lb ? la < lb : t.leaf_of[a.second] < t.leaf_of[b.second];
    });
}

// Device copy of the tree and block lists, the workspaces and the near
// blocks (An, allocated, not filled).  Fills H and the handle's lists.
int upload_tree(fl_handle* h, const HostTree& t, int m, HDev& H) {
    const int dim = t.dim, nper = dim + 1;
    const int64_t n = h->n, nv = h->nv, T = h->nc;
    int M = 1;
    for (int j = 0; j < dim; ++j) M *= m;
    const int nc = (int)t.cl.size();
    std::vector<int> clo(nc), chi(nc), cpar(nc), sptr(nc + 1, 0), sidx, node(n), rleaf(n);
    std::vector<double> box(3 * (size_t)nc);
    for (int c = 0; c < nc; ++c) {
        clo[c] = t.cl[c].lo;
        chi[c] = t.cl[c].hi;
        cpar[c] = t.cl[c].parent;
        box[3 * c] = t.cl[c].blo[0];
        box[3 * c + 1] = t.cl[c].blo[1];
        box[3 * c + 2] = t.cl[c].side;
        for (int sn : t.cl[c].sons) sidx.push_back(sn);
        sptr[c + 1] = (int)sidx.size();
        if (t.cl[c].sons.empty())
            for (int r = t.cl[c].lo; r < t.cl[c].hi; ++r) rleaf[r] = c;
    }
    for (int64_t r = 0; r < n; ++r) node[r] = h->dof_node[t.perm[r]];
    std::vector<long long> fptr(nc + 1, 0);
    std::vector<int> fsrc, fdst;
    for (auto& p : t.far) {
        fsrc.push_back(p.first);
        fdst.push_back(p.second);
        fptr[p.first + 1]++;
    }
    for (int c = 0; c < nc; ++c) fptr[c + 1] += fptr[c];
    const int nleaf = (int)t.leaf_ids.size();
    std::vector<int> lnptr(nleaf + 1, 0), nsrc, ndst, nrng;
    std::vector<long long> noff;
    long long near_entries = 0;
    for (auto& p : t.near) {
        nsrc.push_back(p.first);
        ndst.push_back(p.second);
        nrng.push_back(clo[p.second]);
        nrng.push_back(chi[p.second] - clo[p.second]);
        noff.push_back(near_entries);
        near_entries += (long long)(chi[p.first] - clo[p.first]) * (chi[p.second] - clo[p.second]);
        lnptr[t.leaf_of[p.first] + 1]++;
    }
    for (int l = 0; l < nleaf; ++l) lnptr[l + 1] += lnptr[l];
    int lmax = 0;
    for (int c : t.leaf_ids) lmax = std::max(lmax, chi[c] - clo[c]);
    // Chebyshev points of the first kind on [0, 1] (increasing) and the
    // (m+1)-point cell rule
    std::vector<double> tnode(m);
    for (int k = 0; k < m; ++k) tnode[k] = 0.5 - 0.5 * std::cos((2.0 * k + 1.0) * M_PI / (2.0 * m));
    const RuleTables& R = fl_base_rules();
    const int kq = m + 1;
    std::vector<double> qlam, qw;
    if (dim == 1) {
        for (int i = 0; i < kq; ++i) {
            const double x = R.gl_x[gl_off(kq) + i];
            qlam.push_back(1.0 - x);
            qlam.push_back(x);
            qw.push_back(R.gl_w[gl_off(kq) + i]);
        }
    } else {
        for (int i = 0; i < kq; ++i)
            for (int j = 0; j < kq; ++j) {
                const double l1 = R.gj_x[gl_off(kq) + i], l2 = (1.0 - l1) * R.gl_x[gl_off(kq) + j];
                qlam.push_back(1.0 - l1 - l2);
                qlam.push_back(l1);
                qlam.push_back(l2);
                qw.push_back(2.0 * R.gj_w[gl_off(kq) + i] * R.gl_w[gl_off(kq) + j]);
            }
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
    // per-level cluster lists, four ints per entry so that a workgroup has
    // every index it needs after one load: upward (internal clusters,
    // deepest level first) {c, son 0, son 1, 0}, downward (every cluster
    // below the root, shallowest first) {c, parent, 0, 0}.  The bisection
    // gives every internal cluster exactly two sons.
    const int depth = t.depth;
    std::vector<std::vector<int>> up(depth + 1), down(depth + 1);
    for (int c = 0; c < nc; ++c) {
        if (!t.cl[c].sons.empty()) {
            if (t.cl[c].sons.size() != 2) return cfail(h, FL_EINVAL, "cluster tree: internal cluster without two sons");
            for (int v : {c, t.cl[c].sons[0], t.cl[c].sons[1], 0}) up[t.cl[c].level].push_back(v);
        }
        if (c > 0)
            for (int v : {c, cpar[c], 0, 0}) down[t.cl[c].level].push_back(v);
    }
    fl_hm& Hm = h->hm;
    H = HDev{};
    H.dim = dim;
    H.m = m;
    H.M = M;
    H.n = n;
    H.nc = nc;
    H.nleaf = nleaf;
    H.nfar = (long long)t.far.size();
    H.nnear = (long long)t.near.size();
    H.nq = (int)qw.size();
    int rc;
    const int *p_clo, *p_chi, *p_cpar, *p_sptr, *p_sidx, *p_perm, *p_node, *p_rleaf, *p_leaf, *p_cells, *p_vptr,
        *p_vidx, *p_fsrc, *p_fdst, *p_lnptr, *p_nsrc, *p_ndst, *p_nrng;
    const double *p_box, *p_tnode, *p_verts, *p_qlam, *p_qw;
    const long long *p_fptr, *p_noff;
    std::vector<int> cells(h->cells.begin(), h->cells.end());
    std::vector<double> verts(h->verts.begin(), h->verts.end());
#define UP(ptr, vec)                                                         \
    do {                                                                     \
        using E_ = std::remove_const_t<std::remove_pointer_t<decltype(ptr)>>; \
        E_* q_ = nullptr;                                                    \
        if ((rc = hm_upload(h, &q_, vec))) {                                 \
            hm_release(h);                                                   \
            return rc;                                                       \
        }                                                                    \
        ptr = q_;                                                            \
    } while (0)
    UP(p_clo, clo);
    UP(p_chi, chi);
    UP(p_cpar, cpar);
    UP(p_sptr, sptr);
    UP(p_sidx, sidx);
    UP(p_perm, t.perm);
    UP(p_node, node);
    UP(p_rleaf, rleaf);
    UP(p_leaf, t.leaf_ids);
    UP(p_cells, cells);
    UP(p_vptr, vptr);
    UP(p_vidx, vidx);
    UP(p_fsrc, fsrc);
    UP(p_fdst, fdst);
    UP(p_lnptr, lnptr);
    UP(p_nsrc, nsrc);
    UP(p_ndst, ndst);
    UP(p_nrng, nrng);
    UP(p_box, box);
    UP(p_tnode, tnode);
    UP(p_verts, verts);
    UP(p_qlam, qlam);
    UP(p_qw, qw);
    UP(p_fptr, fptr);
    UP(p_noff, noff);
#undef UP
    H.clo = p_clo;
    H.chi = p_chi;
    H.cpar = p_cpar;
    H.sptr = p_sptr;
    H.sidx = p_sidx;
    H.box = p_box;
    H.tnode = p_tnode;
    H.perm = p_perm;
    H.node = p_node;
    H.rleaf = p_rleaf;
    H.leaf = p_leaf;
    H.verts = p_verts;
    H.cells = p_cells;
    H.vptr = p_vptr;
    H.vidx = p_vidx;
    H.qlam = p_qlam;
    H.qw = p_qw;
    H.fptr = p_fptr;
    H.fsrc = p_fsrc;
    H.fdst = p_fdst;
    H.lnptr = p_lnptr;
    H.nsrc = p_nsrc;
    H.ndst = p_ndst;
    H.noff = p_noff;
    H.nrng = (const int2*)p_nrng;
    H.lmax = lmax;
    if ((rc = hm_alloc(h, &H.V, (size_t)n * M)) || (rc = hm_alloc(h, &H.T, (size_t)nc * M * M)) ||
        (rc = hm_alloc(h, &H.Tt, (size_t)nc * M * M)) ||
        (rc = hm_alloc(h, &H.Kb, (size_t)H.nfar * M * M)) || (rc = hm_alloc(h, &H.An, (size_t)near_entries)) ||
        (rc = hm_alloc(h, &H.xp, (size_t)n)) || (rc = hm_alloc(h, &H.xh, (size_t)nc * M)) ||
        (rc = hm_alloc(h, &H.yh, (size_t)nc * M)) || (rc = hm_alloc(h, &Hm.d, (size_t)n)) ||
        (rc = hm_alloc(h, &Hm.cg, (size_t)4 * n)) || (rc = hm_alloc(h, &Hm.sc, 16))) {
        hm_release(h);
        return rc;
    }
    if (hipHostMalloc((void**)&Hm.hsc, 16 * sizeof(double)) != hipSuccess) {
        hm_release(h);
        return cfail(h, FL_ENOMEM, "cluster approximation: pinned allocation failed");
    }
    for (int l = depth; l >= 0; --l) {
        int* q = nullptr;
        if ((rc = hm_upload(h, &q, up[l]))) {
            hm_release(h);
            return rc;
        }
        Hm.up_lists.push_back(q);
        Hm.up_counts.push_back((int)up[l].size() / 4);
    }
    for (int l = 1; l <= depth; ++l) {
        int* q = nullptr;
        if ((rc = hm_upload(h, &q, down[l]))) {
            hm_release(h);
            return rc;
        }
        Hm.down_lists.push_back(q);
        Hm.down_counts.push_back((int)down[l].size() / 4);
    }
    Hm.m = m;
    Hm.depth = depth;
    Hm.near_entries = near_entries;
    return FL_OK;
}

int check_cluster_args(fl_handle* h, int32_t m, double eta, int32_t leaf) {
    if (h->sym_T > 0) return cfail(h, FL_EINVAL, "the cluster approximation does not take a symmetry reduction");
    if (m < 1 || m > 15) return cfail(h, FL_EINVAL, "m must lie in 1..15");
    if (!(eta > 0.0) || !std::isfinite(eta)) return cfail(h, FL_EINVAL, "eta must be positive and finite");
    if (leaf < 1 || leaf > 1024) return cfail(h, FL_EINVAL, "leaf must lie in 1..1024");
    return FL_OK;
}

}  // namespace

void fl_hm_free(fl_handle* h) { hm_release(h); }

extern "C" {

int fl_cluster_build(fl_handle* h, int32_t m, double eta, int32_t leaf) {
    if (!h) return FL_EINVAL;
    if (!h->assembled) return cfail(h, FL_ESTATE, "no assembled matrix (fl_assemble)");
    int rc = check_cluster_args(h, m, eta, leaf);
    if (rc) return rc;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    hm_release(h);
    HostTree t;
    build_host_tree(h, eta, leaf, t);
    HDev H{};
    if ((rc = upload_tree(h, t, m, H))) return rc;
    fl_hm& Hm = h->hm;
    if ((rc = fl_complete_lower(h))) return rc;  // the near blocks are copied from the whole matrix
    launch_h_setup(H, h->dA, h->lda, -0.5 * (h->dim + 2.0 * h->s), h->stream);
    launch_h_diag(h->dA, h->lda, h->n, Hm.d, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    Hm.H = H;
    Hm.leaf = leaf;
    Hm.eta = eta;
    Hm.C = fl_cdn(h->dim, h->s);
    Hm.direct = false;
    Hm.ready = true;
    return FL_OK;
}

int fl_cluster_assemble(fl_handle* h, double s, const fl_opts* opts_in, int32_t m, double eta, int32_t leaf,
                        int64_t* n_out) {
    if (!h) return FL_EINVAL;
    if (h->dim == 0) return cfail(h, FL_ESTATE, "fl_set_mesh must be called first");
    if (!(s > 0.0 && s < 1.0)) return cfail(h, FL_EINVAL, "s must lie in (0,1)");
    fl_opts o;
    if (opts_in) o = *opts_in;
    else fl_default_opts(&o);
    int rc = check_cluster_args(h, m, eta, leaf);
    if (rc) return rc;
    if (o.precision != FL_FP64 && o.precision != FL_MIXED)
        return cfail(h, FL_EINVAL, "precision must be FL_FP64 or FL_MIXED");
    // FL_MIXED: the blocks are assembled in FP64 and kept in FP32
    const bool f32 = o.precision == FL_MIXED;
    o.precision = FL_FP64;
    if (o.surrogate != 0) return cfail(h, FL_EINVAL, "the cluster near field takes the exact rules (surrogate = 0)");
    if (o.deterministic) return cfail(h, FL_EINVAL, "the repeatable assembly is for fl_assemble");
    HIPCHK(hipSetDevice(h->device));
    if (h->stream) HIPCHK(hipStreamSynchronize(h->stream));
    hm_release(h);
    // the dense matrix of an earlier assembly is released: this path exists
    // for problems whose dense matrix does not fit
    fl_release_dense(h);
    const bool all_nodes = (o.dof_mode == FL_DOF_PAPER) && (s < 0.5);
    set_dof_map(h, all_nodes);
    const int64_t n = (int64_t)h->dof_node.size(), T = h->nc;
    const int nper = h->dim + 1;
    HostTree t;
    build_host_tree(h, eta, leaf, t);
    for (int64_t K = 0; K < T && n > 0; ++K)
        if (t.anchor[K] < 0)
            return cfail(h, FL_EMESH, "a mesh component without DOF (cell " + std::to_string(K) + ")");
    const int nleaf = (int)t.leaf_ids.size();
    // DOF -> leaf index and position in the leaf
    std::vector<int> dleaf(n), drow(n), lsize(nleaf), lpart;
    for (int l = 0; l < nleaf; ++l) {
        const HCl& c = t.cl[t.leaf_ids[l]];
        lsize[l] = c.hi - c.lo;
        for (int r = c.lo; r < c.hi; ++r) {
            dleaf[t.perm[r]] = l;
            drow[t.perm[r]] = r - c.lo;
        }
    }
    std::vector<int> aleaf_cell(T, 0);
    for (int64_t K = 0; K < T; ++K) aleaf_cell[K] = n > 0 ? dleaf[t.anchor[K]] : 0;
    std::vector<std::vector<int>> partners(nleaf);
    for (auto& p : t.near) {
        partners[t.leaf_of[p.first]].push_back(t.leaf_of[p.second]);
        lpart.push_back(t.leaf_of[p.second]);
    }
    // element tiles: the block pairs holding a DOF pair or an anchor pair
    // of near leaves; also the internal order's anchor leaves and the
    // leaf -> anchored elements lists
    std::vector<int> aleaf_int(T), lc_ptr(nleaf + 1, 0), lc_idx(T), aleafc(T);
    TileSelect sel = [&](const std::vector<int32_t>& perm, const std::vector<std::vector<int>>& dof, int nblk,
                         std::vector<int2>& pairs) {
        std::vector<std::vector<int>> bl(nleaf);   // leaf -> blocks (increasing)
        std::vector<int> seen(nleaf, -1);
        for (int b = 0; b < nblk; ++b) {
            const int64_t k0 = (int64_t)b * BE, k1 = std::min<int64_t>(T, (int64_t)(b + 1) * BE);
            auto note = [&](int l) {
                if (seen[l] != b) {
                    seen[l] = b;
                    bl[l].push_back(b);
                }
            };
            for (int64_t Ki = k0; Ki < k1; ++Ki) {
                note(aleaf_cell[perm[Ki]]);
                for (int a = 0; a < nper; ++a)
                    if (dof[a][Ki] >= 0) note(dleaf[dof[a][Ki]]);
            }
        }
        // the block pairs (lo <= hi) as bits of an nblk x nblk map, read out
        // row by row: the pairs in increasing (lo, hi) order, each once
        std::vector<uint64_t> bits(((size_t)nblk * nblk + 63) / 64, 0);
        for (int l = 0; l < nleaf; ++l)
            for (int u : partners[l]) {
                if (u < l) continue;
                for (int b1 : bl[l])
                    for (int b2 : bl[u]) {
                        const size_t k = (size_t)std::min(b1, b2) * nblk + std::max(b1, b2);
                        bits[k >> 6] |= 1ull << (k & 63);
                    }
            }
        pairs.clear();
        for (int lo = 0; lo < nblk; ++lo) {
            const size_t k0 = (size_t)lo * nblk + lo, k1 = (size_t)(lo + 1) * nblk;
            for (size_t w = k0 >> 6; w <= (k1 - 1) >> 6; ++w) {
                uint64_t m = bits[w];
                if (w == (k0 >> 6)) m &= ~0ull << (k0 & 63);
                if (w == ((k1 - 1) >> 6) && (k1 & 63)) m &= ~0ull >> (64 - (k1 & 63));
                while (m) {
                    const size_t k = (w << 6) + (size_t)__builtin_ctzll(m);
                    m &= m - 1;
                    pairs.push_back(make_int2(lo, (int)(k - (size_t)lo * nblk)));
                }
            }
        }
        for (int64_t Ki = 0; Ki < T; ++Ki) aleaf_int[Ki] = aleaf_cell[perm[Ki]];
        for (int64_t Ki = 0; Ki < T; ++Ki) lc_ptr[aleaf_int[Ki] + 1]++;
        for (int l = 0; l < nleaf; ++l) lc_ptr[l + 1] += lc_ptr[l];
        std::vector<int> fill(lc_ptr.begin(), lc_ptr.end() - 1);
        for (int64_t Ki = 0; Ki < T; ++Ki) lc_idx[fill[aleaf_int[Ki]]++] = (int)Ki;
        for (int64_t Ki = 0; Ki < T; ++Ki) aleafc[Ki] = t.leaf_ids.empty() ? -1 : t.leaf_ids[aleaf_int[Ki]];
    };
    Plan P;
    h->n = n;
    if (n > 0 && (rc = plan_assembly(h, all_nodes, o, P, &sel))) return rc;
    HDev H{};
    if ((rc = upload_tree(h, t, m, H))) return rc;
    fl_hm& Hm = h->hm;
    const double C = fl_cdn(h->dim, s);
    fl_stats_t st{};
    if (n > 0) {
        NearMap nm{};
        int *p_dleaf = nullptr, *p_drow = nullptr, *p_lsize = nullptr, *p_lpart = nullptr, *p_aleaf = nullptr,
            *p_lcp = nullptr, *p_lci = nullptr, *p_aleafc = nullptr;
        if ((rc = hm_upload(h, &p_dleaf, dleaf)) || (rc = hm_upload(h, &p_drow, drow)) ||
            (rc = hm_upload(h, &p_lsize, lsize)) || (rc = hm_upload(h, &p_lpart, lpart)) ||
            (rc = hm_upload(h, &p_aleaf, aleaf_int)) || (rc = hm_upload(h, &p_lcp, lc_ptr)) ||
            (rc = hm_upload(h, &p_lci, lc_idx)) || (rc = hm_upload(h, &p_aleafc, aleafc))) {
            hm_release(h);
            return rc;
        }
        nm.An = H.An;
        nm.dleaf = p_dleaf;
        nm.drow = p_drow;
        nm.lsize = p_lsize;
        nm.lptr = H.lnptr;
        nm.lpart = p_lpart;
        nm.lpoff = H.noff;
        nm.aleaf = p_aleaf;
        launch_zero(H.An, Hm.near_entries, h->stream);
        // far field first: the self terms' far part runs through it
        const double pe = -0.5 * (h->dim + 2.0 * s);
        launch_h_setup(H, nullptr, 0, pe, h->stream);
        HIPCHK(hipGetLastError());
        std::function<int()> far_self = [&]() -> int {
            launch_h_self_far(H, h->E, (int)T, p_lcp, p_lci, p_aleafc, Hm.up_lists.data(), Hm.up_counts.data(),
                              (int)Hm.up_lists.size(), Hm.down_lists.data(), Hm.down_counts.data(),
                              (int)Hm.down_lists.size(), C, h->dS, h->stream);
            return FL_OK;
        };
        if ((rc = run_assembly(h, P, s, o, nullptr, 0, 0, nullptr, &st, &nm, &far_self))) {
            hm_release(h);
            return rc;
        }
        launch_near_diag(nm, n, Hm.d, h->stream);
        HIPCHK(hipGetLastError());
        Hm.nm = nm;
        if (f32) {
            // FP32 representation: the kernel and near blocks rounded once
            // from their FP64 assembly; the FP64 copies are released
            float *kbf = nullptr, *anf = nullptr;
            const long long kb_n = H.nfar * H.M * H.M;
            if ((rc = hm_alloc(h, &kbf, (size_t)kb_n)) || (rc = hm_alloc(h, &anf, (size_t)Hm.near_entries))) {
                hm_release(h);
                return rc;
            }
            launch_h_to_f32(H.Kb, kbf, kb_n, h->stream);
            launch_h_to_f32(H.An, anf, Hm.near_entries, h->stream);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(h->stream));
            hm_free(h, H.Kb, sizeof(double) * (size_t)kb_n);
            hm_free(h, H.An, sizeof(double) * (size_t)Hm.near_entries);
            H.Kb = nullptr;
            H.An = nullptr;
            Hm.nm.An = nullptr;  // the map's FP64 target is gone
            H.Kbf = kbf;
            H.Anf = anf;
        }
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->st = st;
    h->s = s;
    h->opts = o;
    h->n = n;
    h->lda = 0;
    h->assembled = false;
    h->planned = n > 0;
    Hm.H = H;
    Hm.leaf = leaf;
    Hm.eta = eta;
    Hm.C = C;
    Hm.direct = true;
    Hm.ready = true;
    if (n_out) *n_out = n;
    return FL_OK;
}

int fl_cluster_matvec(fl_handle* h, const double* x, double* y) {
    if (!h) return FL_EINVAL;
    if (!h->hm.ready) return cfail(h, FL_ESTATE, "no cluster approximation of the current matrix (fl_cluster_build)");
    if (h->n == 0) return FL_OK;
    if (!x || !y) return cfail(h, FL_EINVAL, "null vector");
    HIPCHK(hipSetDevice(h->device));
    const fl_hm& Hm = h->hm;
    launch_h_matvec(Hm.H, Hm.up_lists.data(), Hm.up_counts.data(), (int)Hm.up_lists.size(), Hm.down_lists.data(),
                    Hm.down_counts.data(), (int)Hm.down_lists.size(), Hm.C, x, y, h->stream);
    HIPCHK(hipGetLastError());
    return FL_OK;
}

int fl_cluster_info(const fl_handle* h, int64_t* out) {
    if (!h || !out) return FL_EINVAL;
    if (!h->hm.ready) return FL_ESTATE;
    const fl_hm& Hm = h->hm;
    out[0] = Hm.H.nc;
    out[1] = Hm.H.nleaf;
    out[2] = Hm.H.nfar;
    out[3] = Hm.H.nnear;
    out[4] = Hm.near_entries;
    out[5] = (int64_t)Hm.bytes;
    out[6] = Hm.depth;
    return FL_OK;
}

int fl_solve_cluster(fl_handle* h, const double* b, double* u, double rtol, int32_t maxit, int32_t* iters,
                     double* relres) {
    if (!h) return FL_EINVAL;
    if (!h->hm.ready) return cfail(h, FL_ESTATE, "no cluster approximation of the current matrix (fl_cluster_build)");
    if (!(rtol >= 0.0) || maxit < 0) return cfail(h, FL_EINVAL, "rtol >= 0 and maxit >= 0 required");
    if (h->n == 0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return FL_OK;
    }
    if (!b || !u) return cfail(h, FL_EINVAL, "null vector");
    HIPCHK(hipSetDevice(h->device));
    int rc = fl_solver_workspace(h);
    if (rc) return rc;
    fl_hm& Hm = h->hm;
    const int64_t n = h->n;
    double *r = Hm.cg, *z = Hm.cg + n, *p = Hm.cg + 2 * n, *q = Hm.cg + 3 * n;
    const int nblk = (int)std::min<int64_t>((n + 255) / 256, 1024);
    auto Hmul = [&](const double* x, double* y) {
        launch_h_matvec(Hm.H, Hm.up_lists.data(), Hm.up_counts.data(), (int)Hm.up_lists.size(),
                        Hm.down_lists.data(), Hm.down_counts.data(), (int)Hm.down_lists.size(), Hm.C, x, y,
                        h->stream);
    };
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, h->stream));
    launch_zero(u, n, h->stream);
    HIPCHK(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    launch_mg_scale(z, r, Hm.d, 1.0, n, h->stream);
    launch_dot2(r, z, r, n, h->w_part, nblk, Hm.sc, h->stream);
    HIPCHK(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(Hm.hsc, Hm.sc, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const double bb = Hm.hsc[1];
    int status = FL_OK, it = 0;
    double rr = bb;
    if (!std::isfinite(bb)) status = FL_ENONFINITE;
    // iteration k: rz_k, rr_k at sc[2 (k & 1)], sc[2 (k & 1) + 1]; p.Ap at sc[4]
    while (status == FL_OK && bb > 0.0 && !(std::sqrt(rr) <= rtol * std::sqrt(bb)) && it < maxit) {
        const int cur = 2 * (it & 1), nxt = 2 * ((it + 1) & 1);
        Hmul(p, q);
        launch_dot2(p, q, q, n, h->w_part, nblk, Hm.sc + 4, h->stream);
        launch_mg_axpy(u, r, p, q, n, Hm.sc, cur, 4, h->stream);
        launch_mg_scale(z, r, Hm.d, 1.0, n, h->stream);
        launch_dot2(r, z, r, n, h->w_part, nblk, Hm.sc + nxt, h->stream);
        launch_mg_pupdate(p, z, n, Hm.sc, nxt, cur, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(Hm.hsc, Hm.sc, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        ++it;
        rr = Hm.hsc[nxt + 1];
        const double pq = Hm.hsc[4], rz = Hm.hsc[nxt];
        if (!std::isfinite(rr) || !std::isfinite(pq) || !std::isfinite(rz)) {
            status = FL_ENONFINITE;
            break;
        }
        if (!(pq > 0.0) || (!(rz > 0.0) && rr > 0.0)) {
            status = FL_EBREAKDOWN;
            break;
        }
    }
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double rel = bb > 0 ? std::sqrt(rr) / std::sqrt(bb) : 0.0;
    h->st.t_solve_ms = ms;
    h->st.last_iters = it;
    h->st.last_relres = rel;
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (status == FL_EBREAKDOWN) return cfail(h, FL_EBREAKDOWN, "CG breakdown: p.Ap <= 0 or r.z <= 0");
    if (status == FL_ENONFINITE) return cfail(h, FL_ENONFINITE, "non-finite residual");
    if (!(rel <= rtol)) return FL_ENOCONV;
    return FL_OK;
}

}  // extern "C"
