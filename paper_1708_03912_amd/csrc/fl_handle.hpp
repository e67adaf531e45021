// Private definition of the library handle (shared by the host units).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "fl_internal.hpp"

// Matrices of one fl_assemble_batch call and the buffers of the batched
// products / solves.
struct fl_batch {
    int ns = 0;
    double s[FL_MAX_BATCH] = {};
    int64_t n = 0, n_pad = 0, ld = 0;       // FP64 and low-precision planes share ld = n_pad
    double* A64 = nullptr;                  // ns x n_pad x ld
    size_t A64_cap = 0;
    float* A32 = nullptr;
    size_t A32_cap = 0;
    void* Ahi = nullptr;                    // bf16 planes
    size_t Ahi_cap = 0;
    void* Alo = nullptr;
    size_t Alo_cap = 0;
    bool have32 = false, havehi = false, havelo = false;
    int best[4] = {-1, -1, -1, -1};         // tuned GEMM entry per element type
    char* ws = nullptr;                     // solver / product workspace
    size_t ws_cap = 0;
    int* hflag = nullptr;                   // pinned host word (active count)
};

// Pair-integral surrogate: network, scaling and certification table.
struct fl_sur {
    bool have = false;                      // parameters present
    bool have_scaling = false;              // standardisation and box present
    float* theta = nullptr;                 // FP32 master parameters (device)
    float* m = nullptr;                     // Adam moments
    float* v = nullptr;
    long long adam_t = 0;
    _Float16* half = nullptr;               // W1, W2, W3, W2T, W3T (device)
    float* scal = nullptr;                  // mx, isx (9 each), mt, st (21 each) (device)
    double mx[fl::SUR_NIN] = {}, sx[fl::SUR_NIN] = {}, mt[fl::SUR_NOUT] = {}, st[fl::SUR_NOUT] = {};
    double lo[fl::SUR_NIN] = {}, hi[fl::SUR_NIN] = {};
    double bound[fl::SUR_NRB * fl::SUR_NSB] = {};
    float* part = nullptr;                  // training partial gradients
    size_t part_cap = 0;
    double* loss = nullptr;                 // per-step workgroup squared errors
    size_t loss_cap = 0;
    double* ws = nullptr;                   // statistics / certification scratch
};

// Layout of the solver status block.
constexpr size_t FL_STAT_SCAL = 64, FL_STAT_HIST = 192, FL_STAT_BYTES = 1024;

// Multigrid hierarchy (fl_mg_setup): levels coarsest first; the finest
// level is the handle's assembled matrix.
struct fl_mg_level {
    int64_t n = 0, lda = 0;
    double* A = nullptr;            // Galerkin operator (below the finest level)
    double* d = nullptr;            // its diagonal
    double* x = nullptr;            // cycle vectors: correction, right-hand side, residual
    double* b = nullptr;
    double* r = nullptr;
    fl::SymPlan sp{};               // symmetric product (below the finest level)
    double* slots = nullptr;
    // prolongation from the next coarser level: parents of each DOF (-1:
    // none) and weights; restriction: children of each coarser DOF (CSR)
    int2* par = nullptr;
    double2* pw = nullptr;
    int* cptr = nullptr;
    int* cidx = nullptr;
    double* cw = nullptr;
};

struct fl_mg {
    bool ready = false;
    std::vector<fl_mg_level> lev;
    double* Ainv = nullptr;         // inverse of the coarsest operator (ld lev[0].lda)
    double* B = nullptr;            // Galerkin workspace
    double* cg = nullptr;           // fine CG vectors r, z, p, q
    double* sc = nullptr;           // device scalars
    double* hsc = nullptr;          // pinned mirror
    int* dflag = nullptr;
};

// Strong-form evaluation (fl_strong_form): geometry of one (mesh, DOF map,
// k_eval, edge rules) combination, rebuilt when any of them changes.
struct fl_sf {
    bool ready = false;
    int k = 0, qf = 0, qn = 0, nch = 0, nchb = 0;   // far chunks: facet sources, boundary sources
    int64_t n = -1;                 // DOF count the plan was built for
    fl::SfDev D{};
    long long chunk = 0;
    double* sx = nullptr;           // source coordinates
    double* sy = nullptr;
    double* bsx = nullptr;          // boundary-source coordinates
    double* bsy = nullptr;
    double* W = nullptr;            // evaluation weights times |K|
    double* h2 = nullptr;           // squared cell diameters
    int* vptr = nullptr;            // vertex -> cells (CSR) for the nodal indicators
    int* vidx = nullptr;
    double* part = nullptr;         // far-field partial sums, (nch + nchb) x nt
    double* tab = nullptr;          // kernel-power tables of tab_s
    double tab_s = -1.0;
    std::vector<void*> bufs;        // every allocation above
    // cluster evaluation of the all-pairs part (fl_strong_form_cluster)
    bool cl_ready = false;
    int cl_m = 0, cl_leaf = 0;
    double cl_eta = 0.0;
    fl::SfClDev C{};
    std::vector<const int*> cl_up, cl_down;
    std::vector<int> cl_upc, cl_downc;
    std::vector<void*> clbufs;
};

// Cluster approximation: of the assembled matrix (fl_cluster_build), or
// assembled directly from the mesh (fl_cluster_assemble, direct = true).
struct fl_hm {
    bool ready = false;
    bool direct = false;
    fl::NearMap nm{};               // direct: the near blocks' map
    int m = 0, leaf = 0, depth = 0;
    double eta = 0.0, C = 0.0;
    fl::HDev H{};
    std::vector<const int*> up_lists, down_lists;
    std::vector<int> up_counts, down_counts;
    double* d = nullptr;            // diagonal of A (Jacobi)
    double* cg = nullptr;           // r, z, p, q
    double* sc = nullptr;           // device scalars and their pinned mirror
    double* hsc = nullptr;
    long long near_entries = 0;
    size_t bytes = 0;               // device bytes of the representation
    std::vector<void*> bufs;        // every device allocation above
};

namespace fl {
// Result of the s-independent planning of an assembly: device views live in
// the handle (plan buffer), the offsets of the per-launch lists here.
struct Plan {
    int64_t T = 0, nv = 0, n = 0;
    int dim = 0, nper = 0, nblk = 0;
    size_t o_ft = 0, o_nt = 0, o_bnd = 0, o_bdofs = 0, o_loc = 0, o_vloc = 0, o_ep = 0, o_vp = 0,
           o_fac = 0, o_fvid = 0;
    long long n_tiles = 0, n_far_tiles = 0, n_edge = 0, n_vert = 0;
    double t_plan_ms = 0.0;
};
}  // namespace fl

// The plan of the last fl_assemble / fl_assemble_batch over all element
// pairs and the handle's views into it, kept for the next such call while
// the mesh, the DOF set and the distance classes stay the same.  Any other
// planning (which rewrites the plan buffer), fl_set_mesh, fl_set_symmetry
// and the release of the buffers drop it.
struct fl_plan_cache {
    bool valid = false;
    bool all_nodes = false;
    int n_classes = 0;
    double theta[FL_MAX_CLASSES] = {};
    bool use_far = false;
    fl::Plan P{};
    fl::ElemDev E{};
    int* v2c_ptr = nullptr;
    int* v2c_idx = nullptr;
    int* node2dof = nullptr;
    int* dof_node = nullptr;
    const unsigned char* vloc = nullptr;
    const int* sc_ptr = nullptr;
    const int* sc_idx = nullptr;
    const int* sc_map = nullptr;
    const unsigned char* sc_vloc = nullptr;
    int sc_rows = 0;
    double* meas = nullptr;
};

struct fl_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // mesh (host copy)
    int dim = 0;
    int64_t nv = 0, nc = 0, nb = 0;
    std::vector<double> verts;
    std::vector<int32_t> cells, bfacets;
    std::vector<int32_t> facet_opp;     // vertex of the owning cell opposite the facet
    std::vector<char> on_boundary;
    // symmetry reduction (fl_set_symmetry): cells [0, sym_T) form the sector,
    // vfold maps every vertex to its representative; sym_T = 0: none
    int64_t sym_T = 0;
    int sym_order = 1;
    std::vector<int32_t> vfold;
    std::vector<int32_t> sym_pre, sym_rot;  // preimage sector cell and rotation of every cell, or empty

    // assembly
    bool assembled = false;   // single matrix (fl_assemble) present
    // the single matrix's strictly lower tiles (below the diagonal tiles) are
    // still to be written from the upper ones (fl_complete_lower)
    bool lower_pending = false;
    bool planned = false;     // DOF map and device geometry present
    double s = 0.0;
    fl_opts opts{};
    int64_t n = 0, lda = 0;
    std::vector<int32_t> dof_node, node2dof;

    // device / pinned buffers, grown on demand and reused
    char* plan = nullptr;
    size_t plan_cap = 0;
    char* pin = nullptr;
    size_t pin_cap = 0;
    double* dA = nullptr;
    size_t A_cap = 0;
    double* dS = nullptr;
    size_t S_cap = 0;
    float* dA32 = nullptr;
    size_t A32_cap = 0;
    unsigned long long* dcnt = nullptr;
    // repeatable assembly: coarse words of A (int32, n x lda), both words of
    // S (T x 6), the out-of-range flag
    int* dAhi = nullptr;
    size_t Ahi_cap = 0;
    char* dSfix = nullptr;
    size_t Sfix_cap = 0;

    // views into the plan buffer used after assembly
    fl::ElemDev E{};
    int* d_v2c_ptr = nullptr;
    int* d_v2c_idx = nullptr;
    int* d_node2dof = nullptr;
    int* d_dof_node = nullptr;
    const unsigned char* d_vloc = nullptr;  // local index of the vertex in each v2c entry
    // rows of the diagonal-block scatter: per row owner (vertex, or DOF with a
    // symmetry reduction) its (cell, local vertex) entries and its DOF
    const int* d_sc_ptr = nullptr;
    const int* d_sc_idx = nullptr;
    const int* d_sc_map = nullptr;
    const unsigned char* d_sc_vloc = nullptr;
    int sc_rows = 0;
    double* d_meas = nullptr;

    // solver workspace
    double* w = nullptr;   // r, z, p (2n), q, d, tmp (7 n)
    float* w32 = nullptr;  // FP32 refinement workspace (8 n)
    double* w_part = nullptr;
    char* w_stat = nullptr;   // solver status block (device): int flags[16], double scal[16], double hist[64]
    char* w_hstat = nullptr;  // its pinned host mirror
    int64_t w_n = -1;
    fl::SymPlan sym{};     // symmetric product of the n x n matrix (slots in w_sym)
    double* w_sym = nullptr;

    fl_stats_t st{};
    fl_plan_cache pc;
    fl_batch B;
    fl_sur sur;
    fl_mg mg;
    fl_sf sf;
    fl_hm hm;
};

namespace fl {
// Chooses the element-block pairs (bi <= bj) to tile, from the internal
// element order (perm: internal -> caller index) and the DOF of every
// internal element's vertices (dof[a][Ki], -1: none).
using TileSelect = std::function<void(const std::vector<int32_t>& perm, const std::vector<std::vector<int>>& dof,
                                      int nblk, std::vector<int2>& pairs)>;
// Planning and one assembly run (defined with the assembly driver).  With nm
// the pair kernels write the cluster near field instead of A (A may be
// null), and before_scatter runs just before the diagonal blocks are
// scattered (on the handle's stream).
int plan_assembly(fl_handle* h, bool all_nodes, const fl_opts& o, Plan& P, const TileSelect* sel);
int run_assembly(fl_handle* h, const Plan& P, double s, const fl_opts& o, double* A, int64_t lda,
                 long long a_elems, float* A32, fl_stats_t* st, const NearMap* nm = nullptr,
                 const std::function<int()>* before_scatter = nullptr);
// DOF map for the current mesh (Sec. 3: all nodes, or the interior ones)
void set_dof_map(fl_handle* h, bool all_nodes);
}  // namespace fl

// Drop the dense matrix of the last assembly (and everything built on it)
// and free its device memory.
void fl_release_dense(fl_handle* h);
// Write the single matrix's tiles below the diagonal tiles from the upper
// ones if an assembly left them out (every reader of the full matrix calls
// it first; the symmetric product reads only the tiles on and above the
// diagonal).  Asynchronous on the handle's stream.
int fl_complete_lower(fl_handle* h);

// Quadrature tables independent of s (defined with the assembly driver).
const fl::RuleTables& fl_base_rules();
// C(d,s), the constant of the operator (Sec. 2)
double fl_cdn(int d, double s);
void fl_sf_free(fl_handle* h);
void fl_hm_free(fl_handle* h);
// Surrogate parameters of an assembly at s with options o (classes below
// o.surrogate); FL_ESTATE without a network and scaling.  Defined with the
// surrogate calls.
int fl_sur_params(fl_handle* h, double s, const fl_opts& o, fl::SurParams* sp);
void fl_sur_free(fl_handle* h);
// Release the multigrid hierarchy (defined with the multigrid calls).
void fl_mg_free(fl_handle* h);
// Solver workspace of the current matrix, incl. its symmetric-product plan
// (defined with the single-system solver).
int fl_solver_workspace(fl_handle* h);
