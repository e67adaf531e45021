// Internal declarations shared by the host planner (fl_api.hip) and the
// device kernels (fl_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fraclap.h"
#include "fl_sur.hpp"

namespace fl {

constexpr int BE = 64;      // elements per far-field tile side
constexpr int MAXV = 64;    // DOFs per element block kept in LDS
constexpr int TRI_TAB = 204;  // sum_{k=1..8} k^2 triangle-rule points
constexpr int GL_TAB = 136;   // sum_{k=1..16} k Gauss points

// Device tables of Gauss rules, filled once per assembly.
struct RuleTables {
    double gl_x[GL_TAB], gl_w[GL_TAB];  // Gauss-Legendre on [0,1], k = 1..16
    double gj_x[GL_TAB], gj_w[GL_TAB];  // Gauss-Jacobi weight (1-u) on [0,1]
    double tl1[TRI_TAB], tl2[TRI_TAB], tw[TRI_TAB];  // collapsed triangle rules, k = 1..8
    // per triangle-rule point: l1, l2, w, w l0, w l1, w l2, w l_a l_b (a<=b)
    double tri[TRI_TAB][12];
    // per Gauss-Legendre point (k = 1..8): t, w, w l0, w l1, w l0 l0, w l0 l1, w l1 l1
    double seg[36][8];
    double r0_x[2], r0_w[2];            // 2-point rule, weight r^{-2s} on [0,1]
    double r1_x[2], r1_w[2];            // 2-point rule, weight r^{1-2s} on [0,1]
    float trif[TRI_TAB][12];            // FP32 copies for the mixed-precision path
    float segf[36][8];
    // kernel power r2^pe by tables (kpow_tab): 2 / m_i and m_i^pe for the
    // 256 mantissa bins (m_i their midpoints), 2^(pe n) for n = -128..127,
    // and the binomial coefficients C(pe, k), k = 0..5 (pe of the current
    // assembly)
    double pw_inv[256], pw_fr[256], pw_ex[256], pw_c[8];
};
// fill the pe-dependent parts of the kernel-power tables
void set_pow_tables(RuleTables& R, double pe);

__host__ __device__ inline int gl_off(int k) { return k * (k - 1) / 2; }
__host__ __device__ inline int tri_off(int k) { return (k - 1) * k * (2 * k - 1) / 6; }

// Element data, structure of arrays, in the library's internal element order.
struct ElemDev {
    const double* x[6];     // vertex coordinates: 2D x0,y0,x1,y1,x2,y2; 1D x0,x1
    const double* cen[2];   // centroid
    const double* h2;       // squared longest edge
    const double* meas;     // |K|
    const int* vid[3];      // vertex ids
    const int* dof[3];      // DOF ids, -1 if the vertex is not a DOF
    const double* w;        // weight per cell (symmetry reduction: 1 on the sector, 0 on its
                            // images; a pair counts with the mean of its two cells), or null
    const int* spre;        // with w: null, or per cell the preimage sector cell (-1 on the
    const int* srot;        // sector) and the rotation index: one member of each equal couple
    int sorder;             // of cross pairs counts (weight 1); sorder = K
};

// Learned surrogate for the separated pairs of the closest classes: the
// near-tile kernel gives pairs of class < nsur whose features lie in the
// training box and whose distance bin is certified at this s the order-2
// rule times the network's correction, the others the exact rule.
struct SurParams {
    int nsur;               // 0: off
    double s;
    SurNet N;
    double lo[SUR_NIN], hi[SUR_NIN];  // box of the training features
    int use_rbin[SUR_NRB];  // distance bins certified at this s
    unsigned long long* counters;  // [0] surrogate pairs, [1] fallback pairs, [4 + c] fallback of class c
};

// Where the pair kernels put their output when the cluster method's near
// field is assembled instead of the dense matrix: the near blocks (leaf
// pairs that are not admissible), each stored column by column, found from
// the two DOFs' leaves by a binary search of the first leaf's partners
// (increasing leaf index).  An == nullptr: dense mode.
struct NearMap {
    double* An = nullptr;
    const int* dleaf = nullptr;     // DOF -> leaf index
    const int* drow = nullptr;      // DOF -> position in its leaf
    const int* lsize = nullptr;     // leaf -> DOFs
    const int* lptr = nullptr;      // leaf -> first partner (nleaf + 1)
    const int* lpart = nullptr;     // partner leaf indices
    const long long* lpoff = nullptr;  // offset of each (leaf, partner) block in An
    const int* aleaf = nullptr;     // internal element -> leaf index of its anchor DOF
};

// index of the block (leaf a, leaf b) among a's partners, -1 if not near
__device__ __forceinline__ int nm_block(const NearMap& M, int a, int b) {
    int lo = M.lptr[a], hi = M.lptr[a + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (M.lpart[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    return (lo < M.lptr[a + 1] && M.lpart[lo] == b) ? lo : -1;
}

// entry (i, j) of the near field, nullptr when (i, j) lies in the far field
__device__ __forceinline__ double* nm_slot(const NearMap& M, int i, int j) {
    const int a = M.dleaf[i];
    const int p = nm_block(M, a, M.dleaf[j]);
    if (p < 0) return nullptr;
    return M.An + M.lpoff[p] + M.drow[i] + (long long)M.drow[j] * M.lsize[a];
}

// Repeatable accumulation (fl_opts.deterministic): a value v shared by
// several kernels or workgroups is split exactly into v = hi 2^-F1 +
// lo 2^-F2 (F2 = F1 + 52, hi = floor(v 2^F1), lo the rounded remainder)
// and both parts are added with integer atomics, which do not depend on
// order.  lo == nullptr: plain FP64 atomics.  flag[0] is set when a value
// falls outside the range the scale was chosen for (never, given the
// bound the host derives it from).
struct FixAcc {
    long long* lo = nullptr;   // same indexing as the FP64 target
    int* hi = nullptr;
    double to_hi = 0.0;        // 2^F1
    double lo_per_hi = 0.0;    // 2^52
    int* flag = nullptr;
};

__device__ __forceinline__ void fix_add(const FixAcc& F, long long idx, double v) {
    const double th = v * F.to_hi;  // exact: a power of two
    if (!(fabs(th) < 1073741824.0)) {
        *F.flag = 1;
        return;
    }
    const double fh = floor(th);
    const long long lo = __double2ll_rn((th - fh) * F.lo_per_hi);  // th - fh exact, in [0, 1)
    const int hi = (int)fh;
    if (hi) atomicAdd(&F.hi[idx], hi);
    if (lo) atomicAdd((unsigned long long*)&F.lo[idx], (unsigned long long)lo);
}

// v added to an FP64 accumulator, or to its fixed-point words
__device__ __forceinline__ void acc_add(const FixAcc& F, double* D, long long idx, double v) {
    if (F.lo) fix_add(F, idx, v);
    else atomicAdd(&D[idx], v);
}

struct FarParams {
    int dim;
    int T;
    double pe;              // exponent of r^2 in the kernel: -(d/2 + s)
    double C;               // C(d,s)
    int ncls;
    double th2[FL_MAX_CLASSES];
    int kf[FL_MAX_CLASSES + 1];
    int kfirst[FL_MAX_CLASSES + 1];  // 1 if no lower class has the same order
    int nblk;
    const int2* tiles;      // (bi, bj), bi <= bj
    long long ntiles;
    const int* blk_ndof;    // DOFs per element block
    const int* blk_dofs;    // nblk x MAXV DOF ids (first blk_ndof valid)
    const unsigned char* loc;  // T x 3 local DOF index in its block (255: none)
    double* A;
    long long lda;
    double* S;              // T x 6 per-element diagonal-block accumulators
    unsigned long long* cls_count;  // ncls+1 counters
    int mixed;              // 1: separated pairs evaluated in FP32
    SurParams sur;          // learned surrogate for the closest classes
    NearMap nm;             // cluster near field (nm.An set): output map, self-part mask
    FixAcc fa, fs;          // repeatable accumulation of A and of S
};

struct TouchParams {
    int dim;
    double s, pe, C;
    int k;
    long long npairs;
    const int* pairs;       // npairs x 2 element ids (K < Kt)
    double* A;
    long long lda;
    NearMap nm;             // cluster near field (nm.An set): output map
    FixAcc fa;              // repeatable accumulation of A
};

struct BndParams {
    int dim;
    double s, pe, C;
    int T;
    int nb;
    const double* fac;      // nb x 6: p0x p0y p1x p1y nx ny (1D: y, n)
    const int* fvid;        // nb x 2 vertex ids (1D: one)
    int k_touch_bnd;
    int ncls;
    double th2[FL_MAX_CLASSES];
    int kfb[FL_MAX_CLASSES + 1];
    int k_touch;
    int with_boundary;
    int fchunk;             // facets per thread (set by launch_self)
    double* S;
    unsigned long long* counters;  // [0] touching, [1] separated
    FixAcc fs;              // repeatable accumulation of S
};

// launch wrappers (fl_kernels.hip)
hipError_t upload_rules(const RuleTables& R, hipStream_t st);
// General tiles (per-pair classification) and far tiles (every pair of the
// block pair provably in the last class: fixed order fark, no touching).
void launch_far(const ElemDev& E, const FarParams& P, hipStream_t st);
void launch_far_tiles(const ElemDev& E, const FarParams& P, int fark, hipStream_t st);
void launch_self(const ElemDev& E, const BndParams& P, hipStream_t st);
void launch_touch_edge2(const ElemDev& E, const TouchParams& P, hipStream_t st);
void launch_touch_vert(const ElemDev& E, const TouchParams& P, hipStream_t st);
// diagonal-block accumulators S into A, plus mass * (P1 mass matrix)
void launch_scatter_self(const ElemDev& E, const int* v2c_ptr, const int* v2c_idx,
                         const int* node2dof, const unsigned char* vloc, int nv, int dim,
                         const double* S, double mass, double* A, long long lda, hipStream_t st);
// y = M x, M the P1 mass matrix on the DOFs
// D[i] = hi[i] 2^-F1 + lo[i] 2^-F2 for i < n (D may alias lo: in place)
void launch_fix_to_double(const long long* lo, const int* hi, double from_hi, double from_lo, long long n, double* D,
                          hipStream_t st);
// zero row i from column i on, i < n (the upper triangle and the padding)
void launch_zero_upper(double* A, long long lda, long long n, hipStream_t st);
// A[j][i] = A[i][j] for j > i (the assembly writes the upper triangle), in
// the 64 x 64 tiles: part 0 all, 1 the diagonal tiles, 2 the others
void launch_mirror_lower(double* A, long long lda, long long n, int part, hipStream_t st);
// the same into the cluster near field; mass as above
void launch_scatter_self_near(const ElemDev& E, const int* v2c_ptr, const int* v2c_idx, const int* node2dof,
                              const unsigned char* vloc, int nv, int dim, const double* S, double mass,
                              const NearMap& nm, hipStream_t st);
// d[i] = near-field entry (i, i)
void launch_near_diag(const NearMap& nm, long long n, double* d, hipStream_t st);
void launch_mass_matvec(const ElemDev& E, const int* dof_node, const int* v2c_ptr, const int* v2c_idx,
                        const unsigned char* vloc, int dim, long long n, const double* x, double* y,
                        hipStream_t st);
void launch_zero(double* p, long long n, hipStream_t st);
// FP32 copy of the tiles on and above the diagonal (what the symmetric product reads)
void launch_to_f32(const double* A, long long lda, long long n, float* A32, hipStream_t st);
void launch_load_one(const int* dof_node, const int* v2c_ptr, const int* v2c_idx,
                     const double* meas, int dim, long long n, double* b, hipStream_t st);

// solver kernels
void launch_diag(const double* A, long long lda, long long n, double* d, hipStream_t st);

// Symmetric dense product from the upper triangle (fl_solve.hip): 64 x 64
// tiles (bi <= bj); workgroup (J, I) of an (nJ, nI) grid takes the tiles of
// block rows I R .. I R + R - 1 and block columns J m .. J m + m - 1;
// partial sums in slot arrays (no atomics), reduced with G lanes per
// element.
constexpr int SYM_TB = 64;
constexpr int SYM_M = 16;            // most block columns per workgroup
constexpr int SYM_R = 16;            // most block rows per workgroup
constexpr long long SYM_SK_N = 16384;  // larger systems: CG scalars by their own kernel
constexpr int SYM_PQ_BLOCKS = 256;   // pre-reduction of the v.Av partials
struct SymPlan {
    long long n;
    int nb;          // block rows, ceil(n / 64)
    int m;           // block columns per workgroup (<= SYM_M)
    int R;           // block rows per workgroup (<= SYM_R)
    int sk;          // 1: CG scalars by cg_scalar_kernel (large n)
    int nJ;          // workgroup columns, ceil(nb / m)
    int nI;          // workgroup rows, ceil(nb / R)
    long long nwg;   // workgroups of a product, nJ x nI (those below the diagonal empty)
    int G;           // lanes per element in the reductions (power of two <= 16)
    int nred;        // blocks of the reductions, ceil(n G / 256)
    double* prow;    // nJ x n row-sum slots
    double* pcol;    // nI x n column-sum slots
    double* wpart;   // nwg workgroup partials of v.Av
    double* wpart2;  // SYM_PQ_BLOCKS pre-reduced partials
    bool pre;        // pre-reduction in use
    const double* pq;  // partials the CG update sums: wpart or wpart2
    int npq;
};
void sym_plan_geometry(long long n, SymPlan* P);           // everything but the pointers
size_t sym_plan_doubles(const SymPlan& P);                  // slot + partial storage
void sym_plan_bind(SymPlan* P, double* buf);
// y = A x; A symmetric, only its upper triangle is read
void launch_symv(const SymPlan& P, const double* A, long long lda, const double* x, double* y, hipStream_t st);
// r = b - A x (FP64), r32 = (float) r
void launch_residual(const SymPlan& P, const double* A, long long lda, const double* x, const double* b,
                     double* r, float* r32, hipStream_t st);
// mode 0: x += omega (b - A x) / d;  mode 1: r = b - A x
void launch_sym_smooth(const SymPlan& P, const double* A, long long lda, double* x, const double* b,
                       const double* d, double omega, int mode, double* r, hipStream_t st);

// ------------------------------------------------------------ multigrid --
// (fl_mg.hip) transfer operators between nested levels, Galerkin products,
// coarsest-level inverse and the vector kernels of MG-preconditioned CG.
void launch_mg_scale(double* x, const double* b, const double* d, double omega, long long n, hipStream_t st);
void launch_mg_jacobi(double* x, const double* b, const double* y, const double* d, double omega, int mode,
                      double* r, long long n, hipStream_t st);
// b_c[c] = sum over the children (f, w) of c of w r_f[f]   (P^T r)
void launch_mg_restrict(long long nc, const int* cptr, const int* cidx, const double* cw, const double* rf,
                        double* bc, hipStream_t st);
// x_f[i] += sum over the (<= 2) parents (c, w) of i of w x_c[c]   (x += P x_c)
void launch_mg_prolong_add(long long nf, const int2* par, const double2* pw, const double* xc, double* xf,
                           hipStream_t st);
// B = A P (nf x nc, ld ldb), then Ac = P^T B (nc x nc, ld ldc)
void launch_mg_galerkin(const double* A, long long lda, long long nf, long long nc, const int* cptr,
                        const int* cidx, const double* cw, double* B, long long ldb, double* Ac, long long ldc,
                        hipStream_t st);
// in-place inverse of an SPD n x n matrix (ld), Gauss-Jordan without
// pivoting in one workgroup; flag[0] = 1 if a pivot is not positive
void launch_mg_invert(double* M, long long n, long long ld, int* flag, hipStream_t st);
// x += (sc[ia] / sc[ib]) p;  r -= (sc[ia] / sc[ib]) q
void launch_mg_axpy(double* x, double* r, const double* p, const double* q, long long n, const double* sc, int ia,
                    int ib, hipStream_t st);
// p = z + (sc[ia] / sc[ib]) p
void launch_mg_pupdate(double* p, const double* z, long long n, const double* sc, int ia, int ib, hipStream_t st);

// Strong form of the fractional Laplacian of a P1 function (Sec. 4, lemma
// on the strong form) at the evaluation points of every cell, and the
// error indicators built on it.  Cells in the caller's order.
struct SfDev {
    int dim, Q;             // space dimension, evaluation points per cell
    long long T, nt;        // cells, targets T * Q
    const double* cx;       // vertex coordinates of each cell, (dim + 1) * dim per cell
    const int* cdof;        // DOF of each cell vertex, -1 if none
    const double* lam;      // Q x (dim + 1) barycentric coordinates of the points
    const double* tx;       // target coordinates (ty: zeros in d = 1)
    const double* ty;
    long long nf;           // facets: edges (d = 2), vertices (d = 1)
    const int* fK;          // per facet: cell K1, cell K2 (-1 on the boundary)
    const double* fN;       // outward normal of K1 times the facet measure (dim per facet)
    int qf, qn;             // edge rules of the separated and the touching cells (d = 2)
    const double* gx;       // Gauss-Legendre nodes / weights on [0,1], k = 1..16
    const double* gw;
    long long ns;           // sources: facets x qf (d = 2), facets (d = 1)
    double* sc;             // source coefficients (per call)
    const int* nptr;        // cells sharing a vertex with each cell, itself included (d = 1: itself)
    const int* nidx;
    long long nbf;          // boundary facets: owner cell, local facet index
    const int2* bf;
    int bnd_u;              // boundary vertices carry DOFs (value terms of boundary facets)
    long long nbs;          // boundary sources: boundary facets x qf (d = 2), boundary facets (d = 1)
    double* bc;             // their value-term coefficients, 2 per source (per call)
    double pe;              // exponent of r^2 in |x-y|^{-(d+2s-2)}: -(d + 2s - 2)/2
    double cg, cg_own;      // 1/(2s(d+2s-2)) and 1/(d+2s-2); 1/(2s) and 1 in the log form
    double inv2s, C;        // 1/(2s), C(d,s)
};
// Cluster (H-matrix) approximation of A (Sec. 6): tree in DOF ranges
// (tree order), Chebyshev boxes, nested bases, admissible and near pairs.
struct HDev {
    int dim, m, M;          // space dimension, points per direction, M = m^dim
    long long n;            // DOFs
    int nc, nleaf;          // clusters (pre-order, root 0), leaves
    const int* clo;         // DOF range [clo, chi) of each cluster in tree order
    const int* chi;
    const int* cpar;        // parent (-1 at the root)
    const int* sptr;        // sons (CSR)
    const int* sidx;
    const double* box;      // per cluster: corner x, corner y, side
    const double* tnode;    // m Chebyshev points on [0, 1]
    const int* perm;        // tree position -> DOF
    const int* node;        // tree position -> vertex
    const int* rleaf;       // tree position -> leaf cluster
    const int* leaf;        // leaf cluster ids
    // mesh (caller's order) for the basis coefficients
    const double* verts;
    const int* cells;
    const int* vptr;        // vertex -> cells (CSR, increasing)
    const int* vidx;
    int nq;                 // (m+1)-point cell rule: barycentric coordinates, weights
    const double* qlam;
    const double* qw;
    double* V;              // n x M basis coefficients (tree order)
    double* T;              // nc x M x M shift coefficients T_c[b][a]
    double* Tt;             // the same transposed, Tt_c[a][b] = T_c[b][a]
    long long nfar;         // admissible pairs, grouped by the first cluster
    const long long* fptr;  // nc + 1
    const int* fsrc;
    const int* fdst;
    double* Kb;             // nfar x M x M kernel blocks, column by column
    const float* Kbf;       // FP32 representation: the kernel blocks and
    const float* Anf;       // the near blocks rounded to FP32 (else null)
    long long nnear;        // near leaf pairs, grouped by the first leaf
    const int* lnptr;       // nleaf + 1 (by leaf index)
    const int* nsrc;
    const int* ndst;
    const long long* noff;  // offset of each block in An
    const int2* nrng;       // per near pair: first tree position and size of its second leaf
    int lmax;               // largest leaf (DOFs)
    double* An;             // near blocks, column by column
    double* xp;             // product workspace: x and y in tree order, cluster vectors
    double* xh;
    double* yh;
};
void launch_h_setup(const HDev& H, const double* A, long long lda, double pe, hipStream_t st);
// Far part of the elements' diagonal blocks (cluster method): the density 1
// on the elements anchored in each leaf, its leaf coefficients, the upward,
// far and downward passes, and S[K] += C int_K l_a l_b sum_a L_a P_a.
// lc_ptr / lc_idx: leaf index -> internal elements anchored there;
// aleafc: internal element -> leaf cluster id.
void launch_h_self_far(const HDev& H, const ElemDev& E, int T, const int* lc_ptr, const int* lc_idx,
                       const int* aleafc, const int* const* up_lists, const int* up_counts, int n_up,
                       const int* const* down_lists, const int* down_counts, int n_down, double C, double* S,
                       hipStream_t st);
void launch_h_diag(const double* A, long long lda, long long n, double* d, hipStream_t st);
// b[i] = (float)a[i], i < n (round to nearest)
void launch_h_to_f32(const double* a, float* b, long long n, hipStream_t st);
void launch_h_matvec(const HDev& H, const int* const* up_lists, const int* up_counts, int n_up,
                     const int* const* down_lists, const int* down_counts, int n_down, double C, const double* x,
                     double* y, hipStream_t st);

// Cluster evaluation of the strong form's all-pairs part (Sec. 6): a tree
// over the cells (tree positions), Chebyshev moments of the edge sources
// owned by a cluster's cells, local expansions, near leaf pairs directly.
struct SfClDev {
    int m, M, nc, nleaf;
    const int* clo;         // tree-position range [clo, chi) of each cluster
    const int* chi;
    const int* cpar;
    const int* sptr;        // sons (CSR)
    const int* sidx;
    const double* box;      // corner x, corner y, side
    const double* tnode;    // m Chebyshev points on [0, 1]
    const int* perm;        // tree position -> cell
    const int* leaf;        // leaf cluster ids
    const int* optr;        // tree position -> edges it owns (CSR)
    const int* oidx;
    const long long* fptr;  // admissible pairs by first cluster
    const int* fdst;
    const int* lnptr;       // near leaf pairs by leaf index
    const int* ndst;
    double* T;              // nc x M x M shift coefficients
    double* mom;            // nc x M moments
    double* loc;            // nc x M local expansions
};
void launch_sfc_transfer(const SfClDev& Cl, hipStream_t st);
void launch_sfc_eval(const SfClDev& Cl, const SfDev& D, const double* sx, const double* sy,
                     const int* const* up_lists, const int* up_counts, int n_up, const int* const* down_lists,
                     const int* down_counts, int n_down, const double* tab, double* part0, hipStream_t st);
void launch_sf_sources(const SfDev& D, const double* u, hipStream_t st);
void launch_sf_far(const SfDev& D, const double* sx, const double* sy, const double* bsx, const double* bsy,
                   long long chunk, int nch, int nchb, const double* tab, double* part, bool logk,
                   hipStream_t st);
void launch_sf_near(const SfDev& D, const double* u, const double* part, int nch, const double* tab,
                    double* Lu, bool logk, hipStream_t st);
void launch_sf_indicators(const SfDev& D, const double* Lu, const double* f, const double* W,
                          const double* h2, double s, long long nv, const int* vptr, const int* vidx,
                          double* eta_cell, double* eta_node, hipStream_t st);

// CG building blocks
struct CgState {
    long long n;
    const double* A;
    long long lda;
    const double* d;    // diagonal
    const double* b;
    double* x;
    double* r;
    double* z;
    double* p;          // 2 x n (double-buffered by iteration parity)
    double* part;       // 4 x nblk: r.z, r.r by parity
    double* scal;       // [0] b.b, [1] last r.r
    int* flag;          // [0] stop, [1] iterations, [2] 1 breakdown / 2 non-finite
    double* hist;       // r.r at the start of iteration it, at hist[it % 64]
    double rtol;
    int maxit;
    int nblk;           // = sp.nred
    SymPlan sp;         // product slots; sp.wpart holds the p.Ap partials
};
void launch_cg_init(const CgState& s, hipStream_t st);
void launch_cg_iter_at(const CgState& s, int it, hipStream_t st);
void launch_cg_final(const CgState& s, int it, hipStream_t st);

// FP32 Jacobi-PCG (inner solver of the mixed-precision refinement); same
// algorithm and status layout as CgState, vectors and matrix in FP32,
// products and dot products accumulated in FP64.
struct CgState32 {
    long long n;
    const float* A;
    long long lda;
    const float* d;
    const float* b;
    float* x;
    float* r;
    float* z;
    float* p;           // 2 x n
    double* part;
    double* scal;
    int* flag;
    double* hist;
    double rtol;
    int maxit;
    int nblk;
    SymPlan sp;
};
void launch_cg32_init(const CgState32& s, hipStream_t st);
void launch_cg32_iter_at(const CgState32& s, int it, hipStream_t st);
void launch_cg32_final(const CgState32& s, int it, hipStream_t st);
// replace the residual of iteration it by s.b, keep p (mixed-precision
// refinement without restarts)
void launch_cg32_replace(const CgState32& s, int it, hipStream_t st);
// x += e (FP32 correction)
void launch_diag32(const float* A, long long lda, long long n, float* d, hipStream_t st);
void launch_add_correction(double* u, const float* e, long long n, hipStream_t st);
void launch_cast_f32(const double* a, float* b, long long n, hipStream_t st);  // b = (float) a
void launch_dot2(const double* a, const double* b, const double* c, long long n, double* part,
                 int nblk, double* out, hipStream_t st);

// ---------------------------------------------------------------- batch --
// Element types of the batched GEMM (fl_batch.hip).
enum { GD_F64 = 0, GD_F32 = 1, GD_BF16 = 2 };

struct GemmArgs {
    int nsys;               // systems in this launch
    int sys[FL_MAX_BATCH];  // their indices in the batch
    int ksplit;             // K split: split k writes Y + k * ysplit (epi 0 only)
    long long ysplit;
    long long n_pad;        // rows = K extent; multiple of 256
    const void* A;          // plane 0: ns blocks of n_pad x lda (row-major), block stride sA
    const void* A2;         // bf16 low plane (two-plane variants)
    long long lda, sA;
    const void* X;          // plane 0 of X: ns blocks of 64 columns x n_pad (column-major)
    const void* X2;         // bf16 low plane of X
    long long sX;           // elements between systems (64 n_pad)
    void* Y;                // accumulator type (double for GD_F64, else float), layout of X
    const void* V;          // epilogue vector, accumulator type, layout of X
    double* part;           // ns x nrb x 64 epilogue partial sums
    const int* act;         // ns x 64 activity (null: every system)
    int epi;                // 0: Y = A X; 1: also part = sum V.Y; 2: Y = V - A X, part = sum Y.Y
};

struct GemmInfo {
    int dt, npa, wm, waves, bk, bm;
};
int gemm_count();
GemmInfo gemm_info(int id);
hipError_t launch_gemm(int id, const GemmArgs& g, hipStream_t st);

void launch_mat_lo(const double* A, long long ld64, long long n, long long n_pad, long long ldl, int dt,
                   int npa, void* P0, void* P1, hipStream_t st);
void launch_bdiag(const double* A, long long lda, long long sA, long long n, long long n_pad, int ns,
                  double* dinv64, float* dinv32, hipStream_t st);
void launch_pack_f64(const double* src, long long ld, long long sstride, long long n, int nrhs,
                     long long n_pad, int ns, double* dst, hipStream_t st);
void launch_pack_f32(const float* src, long long ld, long long sstride, long long n, int nrhs,
                     long long n_pad, int ns, float* dst, hipStream_t st);
void launch_unpack_f64(const double* src, long long n_pad, long long n, int nrhs, int ns, double* dst,
                       long long ld, long long dstride, hipStream_t st);
void launch_unpack_f32(const float* src, long long n_pad, long long n, int nrhs, int ns, float* dst,
                       long long ld, long long dstride, hipStream_t st);
void launch_split_bf16(const float* x, long long m, void* hi, void* lo, hipStream_t st);
void launch_fill_f64(double* x, long long m, hipStream_t st);
void launch_fill_f32(float* x, long long m, hipStream_t st);

// Batched Jacobi-PCG state; vectors in the padded batch layout, per-system
// scalars indexed j * 64 + c.
template <class T>
struct BcgState {
    long long n_pad;
    T* x;
    T* r;
    T* p;
    T* q;                   // GEMM output A p
    void* ph;               // bf16 hi / lo planes of p (null: not needed)
    void* pl;
    const T* b;
    const T* dinv;          // ns x n_pad reciprocal diagonal (0 in padding)
    const int* want;        // columns that take part
    int* act;
    int* iters;
    int* status;            // 0 ok, 1 breakdown (p.Ap <= 0), 2 non-finite
    double* rz;
    double* bb;
    double* rel;            // ||r|| / ||b|| of the last iterate
    const double* partq;    // GEMM epilogue partials of p.q (ksplit == 1)
    int nrbq;
    int ksplit;             // > 1: q is the sum of ksplit partial products
    long long ysplit;       // elements between the partial products
    double rtol2;
    int maxit;
    // reliable updates (mixed precision): a column asks for a residual
    // replacement (upd = 1) and pauses (act = 0) when rr < delta2 * rupd2 or
    // when it claims convergence / reaches maxit; p is kept up to date so it
    // can go on.  The first step after a replacement takes the exact line
    // search alpha = p.r / p.Ap (lsf set, numerator in pr).
    int* upd;               // null: plain CG
    double* rupd2;          // |r|^2 at the last replacement
    double delta2;
    int* lsf;
    const double* pr;
};
template <class T>
void launch_bcg_init(const BcgState<T>& S, int ns, hipStream_t st);
template <class T>
void launch_bcg_step(const BcgState<T>& S, int ns, hipStream_t st);
// out[0] = active columns, out[1 + j] = active columns of system j
void launch_count(const int* act, int ns, int* out, hipStream_t st);

// Right-hand-side set-up of the batched solve: |b|^2, activity, u = 0,
// r32 = fp32(b) for mixed precision.
struct RefineState {
    long long n_pad;
    const double* b64;
    double* u64;
    float* r32;             // null: not needed
    double* bb;
    int* oact;              // columns with a finite nonzero b
    int* want;              // CG participation (may be null)
    int* status;
    double* rel;
};
void launch_refine_init(const RefineState& R, int ns, int nrhs, hipStream_t st);


// Residual replacement of the mixed-precision CG: after u += x (x = 0) and the
// FP64 product A u (possibly as K-split partial products) on the columns
// with upd set, r64 = b - A u; either the column has converged (act = 0,
// final relres) or r = fp32(r64), rz, rupd2 are refreshed and the column
// goes on (act = 1).
struct ReliableState {
    long long n_pad;
    const double* b64;
    const double* y64;      // partial products of A u (ksplit of them)
    int ksplit;
    long long ysplit;
    float* r;
    const float* dinv;
    double* rz;
    double* rupd2;
    const double* bb;       // |b|^2 of the FP64 right-hand side
    const float* p;         // current search directions
    double* pr;             // p.r after the replacement
    int* lsf;
    int* act;
    int* upd;
    const int* iters;
    int* status;
    double* rel;
    double rtol2;
    int maxit;
};
void launch_corr_masked(double* u, float* x, const int* upd, long long n_pad, int ns, hipStream_t st);
void launch_reliable(const ReliableState& R, int ns, hipStream_t st);

struct LoadArgs {
    ElemDev E;
    int dim;
    long long n, nv;
    const int* dof_node;
    const int* v2c_ptr;
    const int* v2c_idx;
    const unsigned char* vloc;
    const double* meas;
    int nq;
    const double* q;        // nq x 4: l1 (1D: t), l2, w
    const double* coef;     // FOURIER: nrhs x 16; NODAL: nv x nrhs (column-major)
    int nrhs;
    double* b;              // n x nrhs column-major
};
void launch_load(const LoadArgs& a, int kind, hipStream_t st);

// ------------------------------------------------------------ surrogate --
// FP16 weight copies written after every update
struct SurHalves {
    _Float16* W1;   // 64 x 32
    _Float16* W2;   // 64 x 64
    _Float16* W3;   // 32 x 64
    _Float16* W2T;  // 64 x 64, W2T[j][k] = W2[k][j]
    _Float16* W3T;  // 64 x 32, W3T[j][k] = W3[k][j]
};

struct SurTrain {
    const double* F;        // m x 9 features
    const double* T;        // m x 21 targets
    long long m;
    int mode;               // 0: 64 random samples per workgroup (seed, step); 1: samples base + ...
    int batch;              // samples per step (mode 0)
    unsigned long long seed;
    long long step;
    long long base;
    SurNet N;
    const _Float16* W2T;
    const _Float16* W3T;
    float* part;            // gridDim x SUR_NPARAM gradient partials
    double* loss;           // gridDim partial sums of squared errors
};
void launch_sur_train(const SurTrain& A, int nwg, hipStream_t st);

struct SurAdam {
    float* theta;           // FP32 master parameters
    float* m;
    float* v;
    const float* part;
    int nwg;
    float gscale;           // factor from the partial sums to dL/dtheta
    int update;             // 0: only the gradient
    float lr, b1, b2, eps, bc1, bc2;  // bc: 1 - beta^t
    float* grad_out;        // optional FP32 gradient
    SurHalves H;
};
void launch_sur_adam(const SurAdam& S, hipStream_t st);
void launch_sur_halves(const float* theta, const SurHalves& H, hipStream_t st);

struct SurPredict {
    const double* F;
    long long m;
    SurNet N;
    double* out;            // m x 21 predicted t (optional)
    const double* T;        // optional targets: per-bin error maxima
    unsigned int* emax_bits;  // SUR_NRB x SUR_NSB
    unsigned int* count;
};
void launch_sur_predict(const SurPredict& P, hipStream_t st);
// column sums (or, with mean, sums of squared deviations), minima, maxima
void launch_sur_colstat(const double* X, long long m, int ncol, const double* mean, double* part, int nblk,
                        double* out, hipStream_t st);

// pair integrals (21 values, order k, vertex order as given) and the
// training set (canonical features, t = I_k / Q2 - 1) of m separated pairs
void launch_pair_integrals(const double* X, const double* Y, const double* s, long long m, int k,
                           int canonical, double* out, double* feats, hipStream_t st);


}  // namespace fl
