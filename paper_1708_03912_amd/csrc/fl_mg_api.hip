// Host side of geometric multigrid (include/fraclap.h: fl_mg_setup,
// fl_solve_mg).  Sec. 5 proposes multigrid on nested meshes as the solver
// whose iteration count stays bounded under refinement; the cycle used here
// (the paper gives none): Galerkin coarse operators P^T A P, a V(2,2) cycle
// with damped Jacobi smoothing (omega = 2/3) through the symmetric product,
// the coarsest level solved by its explicit inverse, one cycle from a zero
// guess as the preconditioner of CG.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fl_handle.hpp"
#include "fl_internal.hpp"

using namespace fl;

namespace {

constexpr double OMEGA = 2.0 / 3.0;
constexpr int64_t MAX_COARSE = 2048;   // DOFs of the coarsest level (inverted in one workgroup)

int mfail(fl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return mfail(h, FL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dalloc(fl_handle* h, T** p, size_t count) {
    HIPCHK(hipMalloc((void**)p, sizeof(T) * (count ? count : 1)));
    return FL_OK;
}

template <class T>
int upload(fl_handle* h, T** p, const std::vector<T>& v) {
    int rc = dalloc(h, p, v.size());
    if (rc) return rc;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, h->stream));
    return FL_OK;
}

int64_t ld_of(int64_t n) { return ((n + 31) / 32) * 32; }

void hm_product(fl_handle* h, const double* x, double* y) {
    const fl_hm& Hm = h->hm;
    launch_h_matvec(Hm.H, Hm.up_lists.data(), Hm.up_counts.data(), (int)Hm.up_lists.size(), Hm.down_lists.data(),
                    Hm.down_counts.data(), (int)Hm.down_lists.size(), Hm.C, x, y, h->stream);
}

// One V(2,2) cycle on level l from x = 0 for the right-hand side b; the
// finest level is the handle's matrix, or its cluster approximation when
// `hfine` (then the smoother's products go through the cluster product into
// the finest level's spare vector; its diagonal blocks are exact, so the
// diagonal is A's).
void vcycle(fl_handle* h, int l, const double* b, double* x, bool hfine) {
    fl_mg& G = h->mg;
    const int L = (int)G.lev.size();
    fl_mg_level& V = G.lev[l];
    if (l == 0) {
        launch_symv(V.sp, G.Ainv, V.lda, b, x, h->stream);
        return;
    }
    const bool fine = l == L - 1;
    if (fine && hfine) {
        fl_mg_level& C = G.lev[l - 1];
        double* y = V.x;
        launch_mg_scale(x, b, V.d, OMEGA, V.n, h->stream);
        hm_product(h, x, y);
        launch_mg_jacobi(x, b, y, V.d, OMEGA, 0, nullptr, V.n, h->stream);
        hm_product(h, x, y);
        launch_mg_jacobi(x, b, y, V.d, OMEGA, 1, V.r, V.n, h->stream);
        launch_mg_restrict(C.n, V.cptr, V.cidx, V.cw, V.r, C.b, h->stream);
        vcycle(h, l - 1, C.b, C.x, hfine);
        launch_mg_prolong_add(V.n, V.par, V.pw, C.x, x, h->stream);
        for (int k = 0; k < 2; ++k) {
            hm_product(h, x, y);
            launch_mg_jacobi(x, b, y, V.d, OMEGA, 0, nullptr, V.n, h->stream);
        }
        return;
    }
    const double* A = fine ? h->dA : V.A;
    const int64_t lda = fine ? h->lda : V.lda;
    const SymPlan& sp = fine ? h->sym : V.sp;
    fl_mg_level& C = G.lev[l - 1];
    launch_mg_scale(x, b, V.d, OMEGA, V.n, h->stream);
    launch_sym_smooth(sp, A, lda, x, b, V.d, OMEGA, 0, nullptr, h->stream);
    launch_sym_smooth(sp, A, lda, x, b, V.d, OMEGA, 1, V.r, h->stream);
    launch_mg_restrict(C.n, V.cptr, V.cidx, V.cw, V.r, C.b, h->stream);
    vcycle(h, l - 1, C.b, C.x, hfine);
    launch_mg_prolong_add(V.n, V.par, V.pw, C.x, x, h->stream);
    launch_sym_smooth(sp, A, lda, x, b, V.d, OMEGA, 0, nullptr, h->stream);
    launch_sym_smooth(sp, A, lda, x, b, V.d, OMEGA, 0, nullptr, h->stream);
}

}  // namespace

void fl_mg_free(fl_handle* h) {
    fl_mg& G = h->mg;
    for (auto& V : G.lev) {
        for (void* p : {(void*)V.A, (void*)V.d, (void*)V.x, (void*)V.b, (void*)V.r, (void*)V.slots, (void*)V.par,
                        (void*)V.pw, (void*)V.cptr, (void*)V.cidx, (void*)V.cw})
            if (p) (void)hipFree(p);
    }
    G.lev.clear();
    for (void* p : {(void*)G.Ainv, (void*)G.B, (void*)G.cg, (void*)G.sc, (void*)G.dflag})
        if (p) (void)hipFree(p);
    if (G.hsc) (void)hipHostFree(G.hsc);
    G = fl_mg{};
}

extern "C" {

int fl_mg_setup(fl_handle* h, int nlevels, const int64_t* nv, const int32_t* parents) {
    if (h && h->sym_T > 0) return mfail(h, FL_EINVAL, "multigrid does not take a symmetry reduction");
    if (!h) return FL_EINVAL;
    if (!h->assembled || h->B.ns > 0) return mfail(h, FL_ESTATE, "fl_mg_setup needs a matrix from fl_assemble");
    if (nlevels < 2 || nlevels > 16 || !nv || !parents) return mfail(h, FL_EINVAL, "2..16 levels and arrays required");
    if (nv[nlevels - 1] != h->nv) return mfail(h, FL_EINVAL, "nv of the finest level differs from the mesh");
    for (int l = 0; l < nlevels; ++l)
        if (nv[l] <= 0 || nv[l] > ((int64_t)1 << 30)) return mfail(h, FL_EINVAL, "vertex counts out of range");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    fl_mg_free(h);
    const int L = nlevels;
    // parents of level l (l >= 1) start at off[l]
    std::vector<int64_t> off(L + 1, 0);
    for (int l = 1; l < L; ++l) off[l + 1] = off[l] + 2 * nv[l];
    // boundary flags per level from the finest mesh through the inherited vertices
    std::vector<std::vector<char>> bnd(L);
    bnd[L - 1].assign(h->on_boundary.begin(), h->on_boundary.end());
    for (int l = L - 1; l >= 1; --l) {
        const int32_t* par = parents + off[l];
        std::vector<int64_t> inh(nv[l - 1], -1);
        for (int64_t v = 0; v < nv[l]; ++v) {
            const int32_t a = par[2 * v], b = par[2 * v + 1];
            if (a < 0 || b < 0 || a >= nv[l - 1] || b >= nv[l - 1])
                return mfail(h, FL_EMESH, "parent vertex out of range at level " + std::to_string(l));
            if (a == b) {
                if (inh[a] >= 0) return mfail(h, FL_EMESH, "coarse vertex inherited twice at level " + std::to_string(l));
                inh[a] = v;
            }
        }
        bnd[l - 1].assign(nv[l - 1], 0);
        for (int64_t c = 0; c < nv[l - 1]; ++c) {
            if (inh[c] < 0) return mfail(h, FL_EMESH, "coarse vertex without a fine copy at level " + std::to_string(l));
            bnd[l - 1][c] = bnd[l][inh[c]];
        }
    }
    // DOF maps (the rule of the assembly: all nodes for s < 1/2 in the paper's mode)
    const bool all_nodes = (h->opts.dof_mode == FL_DOF_PAPER) && (h->s < 0.5);
    std::vector<std::vector<int32_t>> dof(L);
    std::vector<int64_t> n(L, 0);
    for (int l = 0; l < L; ++l) {
        dof[l].assign(nv[l], -1);
        for (int64_t v = 0; v < nv[l]; ++v)
            if (all_nodes || !bnd[l][v]) dof[l][v] = (int32_t)n[l]++;
    }
    if (n[L - 1] != h->n) return mfail(h, FL_EMESH, "finest DOF count differs from the assembly");
    if (n[0] > MAX_COARSE) return mfail(h, FL_EINVAL, "coarsest level has more than 2048 DOFs");
    for (int l = 0; l < L; ++l)
        if (n[l] == 0) return mfail(h, FL_EINVAL, "a level without DOFs");
    int rc = FL_OK;
    fl_mg& G = h->mg;
    G.lev.resize(L);
    for (int l = 0; l < L; ++l) {
        fl_mg_level& V = G.lev[l];
        V.n = n[l];
        V.lda = l == L - 1 ? h->lda : ld_of(n[l]);
        if ((rc = dalloc(h, &V.d, V.n)) || (rc = dalloc(h, &V.x, V.n)) || (rc = dalloc(h, &V.b, V.n)) ||
            (rc = dalloc(h, &V.r, V.n)))
            return rc;
        if (l < L - 1) {
            if ((rc = dalloc(h, &V.A, (size_t)V.n * V.lda + 8))) return rc;
            sym_plan_geometry(V.n, &V.sp);
            if ((rc = dalloc(h, &V.slots, sym_plan_doubles(V.sp)))) return rc;
            sym_plan_bind(&V.sp, V.slots);
        }
    }
    // transfer operators (host build, fixed orders)
    size_t bmax = 0;
    for (int l = 1; l < L; ++l) {
        const int32_t* par = parents + off[l];
        std::vector<int2> pr(n[l]);
        std::vector<double2> pw(n[l]);
        std::vector<std::vector<std::pair<int, double>>> ch(n[l - 1]);
        for (int64_t v = 0; v < nv[l]; ++v) {
            const int32_t i = dof[l][v];
            if (i < 0) continue;
            const int32_t a = par[2 * v], b = par[2 * v + 1];
            int2 p = make_int2(-1, -1);
            double2 w = make_double2(0.0, 0.0);
            if (a == b) {
                if (dof[l - 1][a] >= 0) {
                    p.x = dof[l - 1][a];
                    w.x = 1.0;
                }
            } else {
                if (dof[l - 1][a] >= 0) {
                    p.x = dof[l - 1][a];
                    w.x = 0.5;
                }
                if (dof[l - 1][b] >= 0) {
                    p.y = dof[l - 1][b];
                    w.y = 0.5;
                }
            }
            pr[i] = p;
            pw[i] = w;
            if (p.x >= 0) ch[p.x].push_back({i, w.x});
            if (p.y >= 0) ch[p.y].push_back({i, w.y});
        }
        std::vector<int> cptr(n[l - 1] + 1, 0), cidx;
        std::vector<double> cw;
        for (int64_t c = 0; c < n[l - 1]; ++c) {
            for (auto& e : ch[c]) {
                cidx.push_back(e.first);
                cw.push_back(e.second);
            }
            cptr[c + 1] = (int)cidx.size();
        }
        fl_mg_level& V = G.lev[l];
        if ((rc = upload(h, &V.par, pr)) || (rc = upload(h, &V.pw, pw)) || (rc = upload(h, &V.cptr, cptr)) ||
            (rc = upload(h, &V.cidx, cidx)) || (rc = upload(h, &V.cw, cw)))
            return rc;
        bmax = std::max(bmax, (size_t)n[l] * (size_t)ld_of(n[l - 1]));
    }
    // Galerkin operators, finest to coarsest, and the diagonals (the finest
    // operator is read whole)
    if ((rc = dalloc(h, &G.B, bmax))) return rc;
    if ((rc = fl_complete_lower(h))) return rc;
    for (int l = L - 1; l >= 1; --l) {
        const fl_mg_level& V = G.lev[l];
        fl_mg_level& C = G.lev[l - 1];
        const double* A = l == L - 1 ? h->dA : V.A;
        launch_mg_galerkin(A, V.lda, V.n, C.n, V.cptr, V.cidx, V.cw, G.B, C.lda, C.A, C.lda, h->stream);
        HIPCHK(hipGetLastError());
    }
    for (int l = 0; l < L; ++l) {
        const fl_mg_level& V = G.lev[l];
        launch_diag(l == L - 1 ? h->dA : V.A, V.lda, V.n, V.d, h->stream);
    }
    // the coarsest inverse
    const fl_mg_level& C0 = G.lev[0];
    if ((rc = dalloc(h, &G.Ainv, (size_t)C0.n * C0.lda + 8)) || (rc = dalloc(h, &G.dflag, 4)) ||
        (rc = dalloc(h, &G.sc, 16)) || (rc = dalloc(h, &G.cg, 4 * (size_t)h->n)))
        return rc;
    HIPCHK(hipHostMalloc((void**)&G.hsc, 64 * sizeof(double), 0));
    HIPCHK(hipMemcpyAsync(G.Ainv, C0.A, sizeof(double) * (size_t)C0.n * C0.lda, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemsetAsync(G.dflag, 0, sizeof(int) * 4, h->stream));
    launch_mg_invert(G.Ainv, C0.n, C0.lda, G.dflag, h->stream);
    HIPCHK(hipGetLastError());
    int flag[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(flag, G.dflag, sizeof(flag), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (flag[0]) return mfail(h, FL_EBREAKDOWN, "coarsest operator is not positive definite");
    G.ready = true;
    return FL_OK;
}

}  // extern "C"

namespace {

// CG preconditioned by one V-cycle; the operator (of CG and of the finest
// level of the cycle) is the handle's matrix or, with `hfine`, its cluster
// approximation.
int mg_pcg(fl_handle* h, const double* b, double* u, double rtol, int32_t maxit, int32_t* iters, double* relres,
           bool hfine) {
    HIPCHK(hipSetDevice(h->device));
    int rc = fl_solver_workspace(h);
    if (rc) return rc;
    fl_mg& G = h->mg;
    const int L = (int)G.lev.size();
    const int64_t n = h->n;
    double *r = G.cg, *z = G.cg + n, *p = G.cg + 2 * n, *q = G.cg + 3 * n;
    const int nblk = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, h->stream));
    launch_zero(u, n, h->stream);
    HIPCHK(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    vcycle(h, L - 1, r, z, hfine);
    launch_dot2(r, z, r, n, h->w_part, nblk, G.sc, h->stream);  // rz_0, rr_0
    HIPCHK(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(G.hsc, G.sc, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const double bb = G.hsc[1];
    int status = FL_OK, it = 0;
    double rr = bb;
    if (!std::isfinite(bb)) status = FL_ENONFINITE;
    // iteration k: rz_k, rr_k at sc[2 (k & 1)], sc[2 (k & 1) + 1]; p.Ap at sc[4]
    while (status == FL_OK && bb > 0.0 && !(std::sqrt(rr) <= rtol * std::sqrt(bb)) && it < maxit) {
        const int cur = 2 * (it & 1), nxt = 2 * ((it + 1) & 1);
        if (hfine) hm_product(h, p, q);
        else launch_symv(h->sym, h->dA, h->lda, p, q, h->stream);
        launch_dot2(p, q, q, n, h->w_part, nblk, G.sc + 4, h->stream);
        launch_mg_axpy(u, r, p, q, n, G.sc, cur, 4, h->stream);
        vcycle(h, L - 1, r, z, hfine);
        launch_dot2(r, z, r, n, h->w_part, nblk, G.sc + nxt, h->stream);
        launch_mg_pupdate(p, z, n, G.sc, nxt, cur, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(G.hsc, G.sc, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        ++it;
        rr = G.hsc[nxt + 1];
        const double pq = G.hsc[4], rz = G.hsc[nxt];
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
    h->st.last_outer = L;
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (status == FL_EBREAKDOWN) return mfail(h, FL_EBREAKDOWN, "CG breakdown: p.Ap <= 0 or r.z <= 0");
    if (status == FL_ENONFINITE) return mfail(h, FL_ENONFINITE, "non-finite residual");
    if (!(rel <= rtol)) return FL_ENOCONV;
    return FL_OK;
}

}  // namespace

extern "C" {

int fl_solve_mg(fl_handle* h, const double* b, double* u, double rtol, int32_t maxit, int32_t* iters,
                double* relres) {
    if (!h) return FL_EINVAL;
    if (!h->mg.ready) return mfail(h, FL_ESTATE, "no multigrid hierarchy for the current matrix (fl_mg_setup)");
    if (!(rtol >= 0.0) || maxit < 0) return mfail(h, FL_EINVAL, "rtol >= 0 and maxit >= 0 required");
    if (!b || !u) return mfail(h, FL_EINVAL, "null vector");
    return mg_pcg(h, b, u, rtol, maxit, iters, relres, false);
}

int fl_solve_cluster_mg(fl_handle* h, const double* b, double* u, double rtol, int32_t maxit, int32_t* iters,
                        double* relres) {
    if (!h) return FL_EINVAL;
    if (!h->mg.ready) return mfail(h, FL_ESTATE, "no multigrid hierarchy for the current matrix (fl_mg_setup)");
    if (!h->hm.ready)
        return mfail(h, FL_ESTATE, "no cluster approximation of the current matrix (fl_cluster_build)");
    if (!(rtol >= 0.0) || maxit < 0) return mfail(h, FL_EINVAL, "rtol >= 0 and maxit >= 0 required");
    if (!b || !u) return mfail(h, FL_EINVAL, "null vector");
    return mg_pcg(h, b, u, rtol, maxit, iters, relres, true);
}

}  // extern "C"
