/*
 * fraclap.h -- C ABI of the MI355X (gfx950) library that assembles, applies
 * and solves the dense P1 Galerkin system of the integral fractional
 * Laplacian, following Ainsworth & Glusa, arXiv:1708.03912.
 *
 * Problem (Sec. 2, fractional Poisson problem and its variational form):
 *   find u in H~^s(Omega) with a(u,v) = <f,v> for all v, where
 *   a(u,v) = C(d,s)/2 int_Omega int_Omega (u(x)-u(y))(v(x)-v(y)) / |x-y|^{d+2s}
 *          + C(d,s)/(2s) int_Omega u v(x) int_dOmega n_y.(x-y) / |x-y|^{d+2s},
 *   n_y the inward unit normal, C(d,s) = 2^{2s} s Gamma(s+d/2) /
 *   (pi^{d/2} Gamma(1-s)).
 * Discretisation (Sec. 3): continuous P1 on a conforming simplicial mesh of
 * a polygonal Omega (d = 1, 2); degrees of freedom are all vertices when
 * s < 1/2 and the interior vertices when s >= 1/2 (FL_DOF_PAPER), or always
 * the interior vertices (FL_DOF_INTERIOR).  DOF order: increasing vertex
 * index.  Stiffness matrix A^s_ij = a(phi_i, phi_j) (Sec. 3).
 * Assembly (Sec. 5): a = sum_{K,Kt} a^{KxKt} + sum_{K,e} a^{Kxe} over
 * element pairs and element/boundary-facet pairs; separated pairs use
 * tensor Gauss rules whose order falls with distance (App. B), touching
 * pairs (identical / common edge / common vertex) regularised rules.
 * Solve (Sec. 5): Jacobi-preconditioned CG driven by the dense matvec.
 *
 * Conventions for every call:
 *   - all functions return an int status: FL_OK (0), a negative error code,
 *     or FL_ENOCONV (+1, a warning);
 *   - fl_last_error(h) gives a message for the last failure on h (the
 *     string lives until the next call on h);
 *   - "device" pointers are HIP device allocations on the handle's device,
 *     owned by the caller unless stated otherwise; all device work is
 *     enqueued on the stream given to fl_create (in order, asynchronous
 *     unless a host output is returned, in which case the call
 *     synchronises that stream);
 *   - one handle per stream; a handle is not thread safe;
 *   - when the assembly has no degrees of freedom (n = 0) every vector /
 *     matrix argument may be NULL and the calls succeed without work.
 */
#ifndef FRACLAP_H
#define FRACLAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FL_OK 0
#define FL_EINVAL (-1)      /* bad argument (s outside (0,1), bad order...) */
#define FL_EMESH (-2)       /* invalid mesh                                  */
#define FL_ENOMEM (-3)      /* device allocation refused or failed            */
#define FL_EDEVICE (-4)     /* HIP runtime error (message attached)           */
#define FL_ESTATE (-5)      /* call out of order (e.g. matvec before assemble)*/
#define FL_ENONFINITE (-6)  /* NaN / Inf in an input vector                   */
#define FL_EBREAKDOWN (-7)  /* CG breakdown: p.Ap <= 0                        */
#define FL_ENOCONV 1        /* CG hit maxit; best iterate returned            */

#define FL_DOF_PAPER 0      /* Sec. 3 rule: all nodes if s < 1/2             */
#define FL_DOF_INTERIOR 1   /* interior nodes only                           */

#define FL_FP64 0           /* every step in FP64                            */
#define FL_MIXED 1          /* separated pairs and the inner CG in FP32      */

#define FL_F64 0            /* element types of fl_matmul / fl_solve_batch    */
#define FL_F32 1            /* FP32 matrix copy, FP32 vectors                 */
#define FL_BF16 2           /* bf16 matrix (one plane), FP32 vectors split
                               into bf16 hi + lo, FP32 accumulation         */
#define FL_BF16X2 3         /* bf16 hi + lo matrix planes, as FL_BF16 else   */

#define FL_RHS_ONE 0        /* f = 1                                          */
#define FL_RHS_FOURIER16 1  /* f = sum of 16 cosine modes (coefficients)      */
#define FL_RHS_P1_NODAL 2   /* f = P1 interpolant of nodal values             */

#define FL_MAX_BATCH 16     /* s values per fl_assemble_batch                 */
#define FL_MAX_CLASSES 8    /* distance classes for separated pairs          */
#define FL_MAX_ORDER_FAR 8  /* largest order for separated pairs             */
#define FL_MAX_ORDER_TOUCH 16 /* largest order for touching pairs            */

#define FL_SUR_NIN 9        /* surrogate features                             */
#define FL_SUR_NOUT 21      /* surrogate outputs (pair integrals)             */
#define FL_SUR_NPARAM 8352  /* packed network parameters                      */
#define FL_SUR_NRB 6        /* certification distance bins                    */
#define FL_SUR_NSB 4        /* certification s bins                           */
#define FL_SUR_BLOB 8454    /* doubles in a parameter blob                    */

typedef struct fl_handle fl_handle;

/* Quadrature orders (App. B).  A separated pair (K,Kt) -- no common vertex --
 * is put in class m = #{i : d2 >= theta_i^2 * max(hK^2, hKt^2)}, with d2 the
 * squared distance of the centroids and h the longest edge; it uses the
 * order k_far[m] on both elements (segment: k-point Gauss-Legendre;
 * triangle: k Gauss-Jacobi(1,0) x k Gauss-Legendre collapsed points).
 * Element/facet pairs use k_far_bnd[m] with the facet midpoint in place of
 * the second centroid.  Touching element pairs use k_touch and touching
 * element/facet pairs k_touch_bnd in every regularised direction.
 * theta must be strictly increasing and positive. */
typedef struct {
    int dof_mode;                        /* FL_DOF_PAPER / FL_DOF_INTERIOR  */
    int with_boundary;                   /* 1: integral operator (default);
                                            0: regional operator (drops the
                                            a^{Kxe} term, Sec. 2)          */
    int k_touch;                         /* 1..FL_MAX_ORDER_TOUCH           */
    int k_touch_bnd;                     /* 1..FL_MAX_ORDER_TOUCH           */
    int n_classes;                       /* number of thresholds, 0..8      */
    double theta[FL_MAX_CLASSES];        /* centroid-distance thresholds    */
    int k_far[FL_MAX_CLASSES + 1];       /* 1..FL_MAX_ORDER_FAR             */
    int k_far_bnd[FL_MAX_CLASSES + 1];   /* 1..FL_MAX_ORDER_FAR             */
    int precision;                       /* FL_FP64 (default) or FL_MIXED:
                                            separated pairs evaluated in
                                            FP32 (hardware log2/exp2, FP32
                                            sums within a pair; tile and
                                            cross-tile sums, touching pairs
                                            and the boundary term in FP64);
                                            an FP32 copy of A drives an
                                            inner FP32 Jacobi-PCG inside
                                            FP64 iterative refinement     */
    int surrogate;                       /* 0 (default): off.  0 < c <=
                                            n_classes (2D only): separated
                                            pairs of the classes
                                            0 .. c-1 go to the learned
                                            surrogate (fl_surrogate_*):
                                            order-2 rule times the
                                            network's correction where the
                                            pair is certified, the exact
                                            rule of its class elsewhere  */
    double sur_tol;                      /* certified bound (relative error
                                            of each pair integral) a
                                            distance bin must meet to use
                                            the network (default 1e-2)     */
    double mass_shift;                   /* mu >= 0: the assembled matrix is
                                            A^s + mu M, M the P1 mass matrix
                                            (M_ij = integral of phi_i phi_j)
                                            on the DOFs.  Sec. 5: a backward
                                            Euler step of the fractional
                                            heat equation solves
                                            (M + dt A^s) u = b, i.e.
                                            (A^s + M/dt) u = b/dt.  0
                                            (default): A^s alone           */
    int deterministic;                   /* 0 (default): contributions are
                                            added with FP64 atomics (the
                                            order, and with it the last
                                            bits, vary from run to run).
                                            1 (fl_assemble only): bitwise
                                            repeatable -- every contribution
                                            that a kernel shares with others
                                            is split exactly into two
                                            fixed-point words (a coarse
                                            int32 and an int64 remainder at
                                            2^-68 of a bound on the entries,
                                            a(phi_i, phi_i) <= C |supp_i|
                                            |S^{d-1}| L_i^{2s} (1/(2-2s) +
                                            1/(2s)), L_i the largest
                                            gradient of phi_i) and summed
                                            with integer atomics, which do
                                            not depend on order; one pass
                                            turns them back into FP64.
                                            Needs n x ld x 4 more bytes of
                                            device memory.  FL_EINVAL for
                                            fl_assemble_batch,
                                            fl_cluster_assemble and with
                                            surrogate > 0               */
} fl_opts;

typedef struct {
    int64_t n;                /* number of DOFs of the last assembly        */
    int64_t n_cells, n_verts, n_bfacets;
    int64_t pairs_identical, pairs_edge, pairs_vertex; /* touching pairs    */
    int64_t pairs_far[FL_MAX_CLASSES + 1];             /* separated, per class */
    int64_t pairs_bnd_touch, pairs_bnd_far;
    int64_t kernel_evals;     /* kernel evaluations of the last assembly    */
    double t_plan_ms;         /* host planning time of the last assembly    */
    double t_assemble_ms;     /* device time of the last assembly           */
    double t_far_ms;          /* ... of which separated element pairs       */
    double t_self_ms;         /* ... identical pairs + boundary facets      */
    double t_touch_ms;        /* ... common-edge / common-vertex pairs      */
    double t_scatter_ms;      /* ... diagonal blocks into A                 */
    double t_solve_ms;        /* device time of the last solve              */
    int32_t last_iters;       /* iterations of the last solve (mixed: the
                                 FP32 iterations)                          */
    double last_relres;
    int32_t last_outer;       /* FP64 residual replacements of the last
                                 solve (mixed fl_solve, fl_solve_batch)    */
    int64_t pairs_surrogate;  /* band pairs done by the network             */
    int64_t pairs_fallback;   /* band pairs that kept the exact rule        */
    double t_cg_kernels_ms;   /* device time of the CG iteration kernels of
                                 the last fl_solve (events around each
                                 chunk of launched iterations; host round
                                 trips excluded)                           */
    int64_t cg_launched;      /* CG iterations launched by the last fl_solve
                                 (>= iterations done: launched iterations
                                 after the stop test exit at once)         */
} fl_stats_t;

/* Default orders (the calibrated table: k_touch = k_touch_bnd = 6,
 * theta = {1.5, 3, 6}, k_far = k_far_bnd = {4, 3, 2, 2}) and dof_mode =
 * FL_DOF_PAPER, with_boundary = 1.  out: host struct owned by the caller. */
int fl_default_opts(fl_opts *out);

/* Create a handle on HIP device `device`; all work goes on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  The handle owns every
 * device buffer it allocates.  *out receives the handle. */
int fl_create(fl_handle **out, int device, void *hip_stream);

/* Release the handle and all device memory it owns.  NULL is ignored. */
void fl_destroy(fl_handle *h);

/* Message for the last failure on h (never NULL). */
const char *fl_last_error(const fl_handle *h);

/* Mesh (Sec. 3: conforming triangulation P_h of a polygon, boundary trace
 * dP_h).  Host arrays, copied (caller keeps ownership):
 *   dim      1 or 2
 *   verts    nv x dim row-major vertex coordinates (finite)
 *   cells    nc x (dim+1) vertex indices, either orientation, |K| > 0
 *   bfacets  nb x dim boundary facets (2D: the two end vertices of a
 *            boundary edge; 1D: the boundary vertex); each must lie on
 *            exactly one cell, whose interior fixes the inward normal.
 * Errors: FL_EINVAL (dim, sizes), FL_EMESH (indices out of range, non-finite
 * or degenerate cells, facet not on exactly one cell).  Invalidates any
 * previous assembly. */
int fl_set_mesh(fl_handle *h, int dim, int64_t nv, const double *verts, int64_t nc,
                const int32_t *cells, int64_t nb, const int32_t *bfacets);

/* Assemble A^s (Sec. 3 definition, Sec. 5 pair decomposition, App. B
 * orders) in FP64 into a device matrix owned by the handle: n x n,
 * row-major with leading dimension fl_matrix_ld(h) (n rounded up to a
 * multiple of 32 doubles).  s in (0,1) else FL_EINVAL.  opts may be NULL
 * (defaults).  *n_out receives n.  Synchronises the stream.  FL_ENOMEM if
 * the matrix does not fit (checked before allocating). */
int fl_assemble(fl_handle *h, double s, const fl_opts *opts, int64_t *n_out);

/* Leading dimension (in elements) of the assembled matrix; 0 before
 * fl_assemble. */
int64_t fl_matrix_ld(const fl_handle *h);

/* Device pointer to the assembled FP64 matrix (owned by the handle, valid
 * until the next fl_set_mesh / fl_assemble / fl_destroy); NULL before.
 * The assembly itself writes the tiles on and above the 64 x 64 diagonal
 * tiles (all that the product and the solvers read); the first call after
 * an assembly enqueues, on the handle's stream, the copy of the rest of the
 * lower triangle from the upper one, so read the matrix after that stream
 * (fl_export_matrix, fl_mg_setup and fl_cluster_build do the same). */
const double *fl_matrix_ptr(const fl_handle *h);

/* node_of_dof: host int32 array of length n receiving the vertex index of
 * each DOF (increasing).  FL_ESTATE before fl_assemble. */
int fl_dofs(const fl_handle *h, int32_t *node_of_dof);

/* Copy A (n x n) to dst with leading dimension ld >= n; dst is a device
 * pointer if on_device, else a host pointer (then the stream is
 * synchronised). */
int fl_export_matrix(fl_handle *h, double *dst, int64_t ld, int on_device);

/* Load vector (Sec. 2: <f, phi_i>) for f = 1 on Omega, exactly:
 * b_i = sum_{K containing i} |K| / (d+1).  b: device, length n. */
int fl_load_vector_one(fl_handle *h, double *b);

/* Geometric multigrid on nested meshes (Sec. 5: a solver whose iteration
 * count stays bounded under refinement).  The handle's mesh (fl_set_mesh)
 * is the finest of nlevels nested meshes and fl_assemble has built its
 * matrix.  nv[l]: vertex count of level l (l = 0 coarsest, nv[nlevels-1] =
 * the mesh's).  parents: host, levels l = 1 .. nlevels-1 concatenated, each
 * nv[l] x 2 int32: the two coarse (level l-1) vertices of which vertex v is
 * the edge midpoint, or (p, p) for the copy of coarse vertex p (every
 * coarse vertex exactly once).  Each level uses the assembly's DOF rule
 * (boundary status inherited through the copies).  Builds the
 * prolongations of P1 functions, the Galerkin operators P^T A P on the
 * device and the inverse of the coarsest one (at most 2048 DOFs).  A new
 * fl_assemble / fl_import_matrix discards the hierarchy.  FL_EMESH for an
 * inconsistent hierarchy, FL_EBREAKDOWN if the coarsest operator is not
 * positive definite.  Synchronises the stream. */
int fl_mg_setup(fl_handle *h, int nlevels, const int64_t *nv, const int32_t *parents);

/* CG on A u = b preconditioned by one multigrid V(2,2) cycle (damped
 * Jacobi, omega = 2/3, through the symmetric product on every level;
 * coarsest level solved exactly).  b, u: device, length n; u is
 * overwritten (initial guess 0).  Stops when ||r||_2 <= rtol ||b||_2 or
 * after maxit iterations (then FL_ENOCONV).  FL_ESTATE without a current
 * hierarchy; FL_EBREAKDOWN, FL_ENONFINITE as fl_solve.  Host iters /
 * relres may be NULL.  Synchronises the stream. */
int fl_solve_mg(fl_handle *h, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                double *relres);

/* Cluster (H-matrix) approximation of the assembled matrix (Sec. 6): a
 * cluster tree over the DOFs (median bisection; leaves of at most `leaf`
 * DOFs), cluster boxes = cubes containing the supports, admissible pairs
 * eta dist >= max(diam) approximated by -C V_s K_st V_t^T with the tensor
 * Chebyshev interpolation of order m (1..15 points per direction) of the
 * kernel and nested bases (shift coefficients); the other leaf pairs are
 * copied from the assembled matrix.  Requires fl_assemble; a new
 * fl_assemble / fl_import_matrix discards it.  Synchronises the stream. */
int fl_cluster_build(fl_handle *h, int32_t m, double eta, int32_t leaf);

/* The cluster approximation of A^s assembled from the mesh alone, without
 * the dense matrix (Sec. 6: the near field from the pair contributions of
 * Sec. 5, assembly and memory growing like the near field, not like n^2).
 * Tree, boxes, admissibility and far blocks as fl_cluster_build.  Near
 * blocks: every touching pair, boundary term and off-diagonal pair block
 * of the element pairs whose DOFs meet in a near leaf pair, in full; the
 * diagonal-block parts of a separated pair (K, Kt) -- the terms
 * phi_i phi_j(x) int_Kt k and phi_i phi_j(y) int_K k of the pair integrand
 * -- only when the anchor leaves of K and Kt are a near pair; for the other
 * cells the same integral is the far field of the density 1 on them,
 * evaluated through the cluster tree (upward pass of its leaf
 * coefficients, kernel blocks, downward pass) and integrated over K with
 * the (m+1)-point rule.  A cell's anchor is its DOF vertex first in tree
 * order; a cell without one takes the anchor of its facet neighbour of
 * smallest index that has one and widens that DOF's support box.
 * opts: as fl_assemble, but surrogate 0 only (FL_EINVAL otherwise);
 * precision FL_FP64, or FL_MIXED: the kernel and near blocks are assembled
 * in FP64, rounded once to FP32 and kept so (the FP64 copies freed), the
 * product multiplies and sums in FP64 -- half the bytes per product, the
 * operator still symmetric; the Jacobi diagonal stays FP64.  No symmetry
 * reduction (FL_EINVAL).  FL_EMESH for a
 * mesh component without any DOF.  Replaces (and frees) a dense matrix of
 * an earlier fl_assemble; afterwards fl_cluster_matvec, fl_solve_cluster,
 * fl_load_vector_one and fl_dofs work, the dense-matrix calls return
 * FL_ESTATE.  Host *n_out (may be NULL): the number of DOFs.  The phase
 * times and pair counts of fl_stats cover the near-field tiles.
 * Synchronises the stream. */
int fl_cluster_assemble(fl_handle *h, double s, const fl_opts *opts, int32_t m, double eta, int32_t leaf,
                        int64_t *n_out);

/* y = A_H x with the cluster approximation: upward pass, kernel blocks,
 * downward pass, near blocks.  x, y: device, length n, not aliased.
 * FL_ESTATE without fl_cluster_build.  Asynchronous. */
int fl_cluster_matvec(fl_handle *h, const double *x, double *y);

/* Jacobi-preconditioned CG (Sec. 5) on A_H u = b (the preconditioner is the
 * diagonal of the assembled matrix, or of the near blocks after
 * fl_cluster_assemble: the same entries).  Arguments and results as fl_solve.
 * Synchronises the stream. */
int fl_solve_cluster(fl_handle *h, const double *b, double *u, double rtol, int32_t maxit,
                     int32_t *iters, double *relres);

/* Multigrid-preconditioned CG (Sec. 5 multigrid, Sec. 6 operator) on
 * A_H u = b: the operator of CG and of the finest level of the V(2,2) cycle
 * is the cluster approximation (its diagonal blocks are exact, so the
 * smoother divides by the diagonal of the assembled matrix); the coarser
 * levels are the Galerkin operators of fl_mg_setup.  Requires both
 * fl_mg_setup and fl_cluster_build on the current matrix (FL_ESTATE
 * otherwise).  Arguments and results as fl_solve_mg.  Synchronises the
 * stream. */
int fl_solve_cluster_mg(fl_handle *h, const double *b, double *u, double rtol, int32_t maxit,
                        int32_t *iters, double *relres);

/* Sizes of the cluster approximation, host out[7]: clusters, leaves,
 * admissible pairs, near pairs, near entries, device bytes, depth.
 * FL_ESTATE without one. */
int fl_cluster_info(const fl_handle *h, int64_t *out);

/* Symmetry reduction (Sec. 7: a rotation B with B^K = Id mapping the domain
 * and the data to themselves).  The mesh given to fl_set_mesh is the whole
 * symmetric mesh with the cells of the sector omega first
 * (ncells_sector of them); vfold (host, nv int32) maps every vertex to its
 * representative, the vertex of the sector it is an image of (vfold[r] = r
 * for representatives; the sector's second radial edge folds onto the
 * first).  The following assemblies then form the reduced system of the
 * symmetric functions: DOFs are the representatives (increasing vertex
 * order, the DOF rule of Sec. 3), every cell pair counts with the mean of
 * its cells' weights (1 on the sector, 0 on the images: each sector cell
 * meets every image of the other cells once, which is the effective
 * kernel k_eff = sum_i |x - B^i y|^{-d-2s}), identical pairs and the
 * boundary term (against the whole boundary) come from the sector's cells,
 * and load vectors and the mass matrix integrate over the sector.  This is
 * P^T A P / K of the full system (P: orbit sums), so a symmetric solution
 * has the full solution's values, and the energy identity of
 * fl_energy_error2 takes (f,u)/K.  Image-image pairs are never computed.
 * cell_pre / cell_rot (host, nc int32 each, or both NULL): the sector cell
 * every cell is an image of and the rotation index i with cell = B^i pre
 * (sector cells: themselves, 0).  With them the two equal cross pairs
 * (S, B^i T) and (T, B^-i S) are formed once with weight 1 (about 1/K of
 * the full mesh's pairs instead of 2/K), and the sector is kept in the
 * caller's order.
 * order = 1 with ncells_sector = 0 switches the reduction off.  The cluster
 * approximation and multigrid refuse a reduced system (FL_EINVAL).
 * FL_EMESH for an inconsistent vfold (out of range, not idempotent, a
 * representative outside the sector, boundary status not shared). */
int fl_set_symmetry(fl_handle *h, int32_t order, int64_t ncells_sector, const int32_t *vfold,
                    const int32_t *cell_pre, const int32_t *cell_rot);

/* Evaluation points of the a posteriori indicators (Sec. 4: local L2
 * norms by quadrature): k_eval in 1..8 points per direction in every cell
 * (d = 2: the collapsed Gauss rule, Gauss-Jacobi(1,0) in the first
 * barycentric coordinate l1 times Gauss-Legendre in l2 / (1 - l1), point q
 * = i k_eval + j; d = 1: Gauss-Legendre), cells in the order given to
 * fl_set_mesh.  x: device, nc x Q x d doubles (Q = k_eval^d); w: device,
 * nc x Q weights times |K|.  Synchronises the stream. */
int fl_eval_points(fl_handle *h, int32_t k_eval, double *x, double *w);

/* Strong form (-Delta)^s u_h at the evaluation points of every cell, by
 * the lemma of Sec. 4 (eq. 8: regular integrals over the cell boundaries;
 * eq. 9, the logarithmic form, for d = 1 and s = 1/2).  u: device, the n
 * DOF values of the last assembly's DOF map (zero at the other vertices);
 * Lu: device, nc x Q doubles (layout of fl_eval_points).  Edge integrals
 * (d = 2): q_far Gauss-Legendre points on the edges of cells sharing no
 * vertex with the evaluation cell, q_near (both 1..16) on the others and on
 * the cell itself; in d = 1 they are point values (q_far, q_near are
 * checked but unused).  The geometry is prepared on the first call for a
 * (mesh, DOF map, k_eval, q_far, q_near) and kept.  FL_ESTATE before
 * fl_assemble; FL_EMESH for an interval mesh with cells below 2^-56 or an
 * extent of 2^60 or more.  Asynchronous on the handle's stream. */
int fl_strong_form(fl_handle *h, double s, const double *u, int32_t k_eval, int32_t q_far,
                   int32_t q_near, double *Lu);

/* fl_strong_form with the all-pairs part evaluated by the cluster method
 * (Sec. 6: the strong form at the indicator points reuses the cluster
 * machinery): a tree over the cells (median bisection of the centroids,
 * leaves of at most `leaf` cells, cube boxes), admissible pairs eta dist >=
 * max diam through Chebyshev moments of the edge sources (m points per
 * direction, nested by shift coefficients) and local expansions, the other
 * leaf pairs summed directly; the touching-cell terms and the boundary
 * value terms as in fl_strong_form.  d = 2 only (FL_EINVAL otherwise).
 * The tree is kept for the next call with the same (m, eta, leaf).
 * Arguments and results otherwise as fl_strong_form.  Asynchronous. */
int fl_strong_form_cluster(fl_handle *h, double s, const double *u, int32_t k_eval, int32_t q_far,
                           int32_t q_near, int32_t m, double eta, int32_t leaf, double *Lu);

/* Babuska-Rheinboldt type indicators of Sec. 4 from the strong form Lu of
 * the last fl_strong_form call with this k_eval:
 *   eta_cell[K] = h_K^{2s} ||f - Lu||^2_{L2(K)}   (h_K: longest edge),
 *   eta_node[i] = sum of eta_cell over the cells containing vertex i
 *                 (the squared eta-hat_i; every vertex, nv values).
 * f: device, nc x Q values at the evaluation points, or NULL for f = 1.
 * eta_cell: device, nc doubles; eta_node: device, nv doubles, or NULL.
 * FL_ESTATE without a strong-form plan for k_eval.  Asynchronous. */
int fl_indicators(fl_handle *h, double s, const double *Lu, const double *f, int32_t k_eval,
                  double *eta_cell, double *eta_node);

/* y = M x with the P1 mass matrix on the DOFs of the last assembly
 * (M_ij = integral of phi_i phi_j, exactly: |K| (1 + delta_ab) /
 * ((d+1)(d+2)) per element), e.g. the right-hand side M u^n of an implicit
 * heat step (Sec. 5).  x, y: device, length n, not aliased.  FL_ESTATE
 * before fl_assemble. */
int fl_mass_matvec(fl_handle *h, const double *x, double *y);

/* y = A x with the FP64 matrix.  x, y: device, length n, not aliased.
 * Sec. 5: the dense product costs n^2 and drives the iterative solve.  A is
 * symmetric; this product, the solver and fl_energy_error2 read only its
 * upper triangle (64 x 64 tiles on and above the diagonal). */
int fl_matvec(fl_handle *h, const double *x, double *y);

/* fl_matvec without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same result,
 * bit for bit, with the product's slots and partials in a scratch array of
 * 48 MiB that the library holds on each device (resolved by fl_create).
 * x, y: device, length n, not aliased.  FL_EINVAL (nothing launched) when
 * the system needs more scratch than that (n above 19,456: use
 * fl_matvec); FL_ESTATE before fl_assemble.  Every call on one device
 * shares that device's scratch: calls that overlap on one GPU (two streams,
 * two handles at once) race and must be serialised by the caller.
 * Asynchronous on the handle's stream. */
int fl_matvec_noalloc(fl_handle *h, const double *x, double *y);

/* Jacobi-preconditioned CG on A u = b (Sec. 5).  b, u: device, length n;
 * u is overwritten (initial guess 0).  Stops when ||r||_2 <= rtol ||b||_2
 * or after maxit iterations (then FL_ENOCONV with the last iterate).
 * After an FL_MIXED assembly: Jacobi-PCG whose products read the FP32 copy
 * of A (FP32 vectors), with FP64 residual replacement: whenever the
 * recursive residual has dropped by a factor 100 since the last
 * replacement (or by what rtol still needs), the FP32 correction is added
 * to u in FP64 and the recursive residual is replaced by b - A u formed
 * with the FP64 matrix; the search direction is kept (no restart).  The
 * stop test is on the FP64 residual; maxit bounds the FP32 iterations.
 * FL_EBREAKDOWN if p.Ap <= 0; FL_ENONFINITE if b is not finite.  Host
 * outputs iters / relres (may be NULL).  Synchronises the stream. */
int fl_solve(fl_handle *h, const double *b, double *u, double rtol, int32_t maxit,
             int32_t *iters, double *relres);

/* Energy-norm error against an exact solution u with known (f,u)
 * (Sec. 7 identity, valid for any discrete u_h):
 *   e2 = fu - 2 b.u_h + u_h.A u_h.
 * b, uh: device, length n.  *e2_out: host.  Synchronises the stream. */
int fl_energy_error2(fl_handle *h, double fu, const double *b, const double *uh, double *e2_out);

/* Counters and timings of the last assembly / solve (after a batch call:
 * pair counts of one s, times summed over the batch). */
int fl_stats(const fl_handle *h, fl_stats_t *out);

/* Replace the assembled FP64 matrix by src (n x n, leading dimension
 * ld >= n, device pointer if on_device else host), e.g. to restore a saved
 * matrix; n and the DOF map are those of the last fl_assemble.  src must be
 * symmetric: products and solves read its upper triangle only.  FL_ESTATE
 * before fl_assemble.  Synchronises the stream when src is on the host. */
int fl_import_matrix(fl_handle *h, const double *src, int64_t ld, int on_device);

/* Load vectors b_i = <f, phi_i> (Sec. 2) for nrhs right-hand sides, after
 * fl_assemble or fl_assemble_batch (same DOFs).  b: device, n x nrhs,
 * column-major with leading dimension n, owned by the caller.
 *   FL_RHS_ONE        f = 1, exact (coeffs unused, may be NULL);
 *   FL_RHS_FOURIER16  host coeffs[16 c + m], f_c = sum_m coeffs psi_m with
 *                     2D psi_m(x) = cos(pi (k1 x1 + k2 x2)), m = 4 k1 + k2,
 *                     k1, k2 in 0..3 (1D: psi_m(x) = cos(pi m x));
 *                     order-4 collapsed Gauss rule per cell (4-point Gauss
 *                     per segment);
 *   FL_RHS_P1_NODAL   host coeffs, nv x nrhs column-major nodal values of
 *                     f (all vertices); b = mass matrix times f, exact. */
int fl_load_vector(fl_handle *h, int kind, const double *coeffs, int64_t nrhs, double *b);

/* Batch of fractional orders on the current mesh (Sec. 2 operator for each
 * s_j, same pair decomposition and orders as fl_assemble): assembles
 * A^{s_j}, j < ns <= FL_MAX_BATCH, in FP64 into handle-owned device
 * memory.  All s_j must give the same DOF set: dof_mode FL_DOF_INTERIOR,
 * or every s_j on the same side of 1/2 (else FL_EINVAL).  *n_out receives
 * n.  Lower-precision copies (FP32 / bf16 planes) are made on first use by
 * fl_matmul / fl_solve_batch and kept until the next assembly.
 * Synchronises the stream. */
int fl_assemble_batch(fl_handle *h, const double *s, int ns, const fl_opts *opts, int64_t *n_out);

/* Export matrix j of the batch (as fl_export_matrix). */
int fl_export_batch_matrix(fl_handle *h, int j, double *dst, int64_t ld, int on_device);

/* Y = A^{s_j} X for nrhs columns (Sec. 5 dense product; nrhs > 1 runs on
 * the matrix cores).  Needs fl_assemble_batch.  s_index = j, or -1 for
 * every matrix of the batch (then X and Y hold ns blocks, block j at
 * j * ld * nrhs elements).  X: n x nrhs column-major, leading dimension
 * ldx >= n; Y likewise with ldy.  dtype FL_F64: X, Y double, FP64 matrix;
 * FL_F32 / FL_BF16 / FL_BF16X2: X, Y float, the matrix in that storage,
 * FP32 accumulation.  Device pointers owned by the caller, not aliased. */
int fl_matmul(fl_handle *h, int s_index, int dtype, const void *X, int64_t ldx, void *Y, int64_t ldy,
              int64_t nrhs);

/* Solve A^{s_j} U_j = B_j for every j of the batch and nrhs columns
 * (Sec. 5 Jacobi-PCG, x0 = 0, stop at ||r|| <= rtol ||b|| per column).
 * B: device, n x nrhs column-major (leading dimension ldb), block j at
 * B + j * strideB (strideB = 0: the same right-hand sides for every j);
 * U likewise (ldu, strideU > 0 unless ns = 1), overwritten.
 *   inner = FL_F64   plain FP64 batched CG on the FP64 matrices;
 *   inner = FL_F32 / FL_BF16 / FL_BF16X2   mixed-precision CG with
 *           reliable updates: the CG recurrence runs in FP32 arithmetic with
 *           the matrix in that storage and the solution accumulates in FP64;
 *           when a column's residual has fallen 100x (FL_BF16: 10x) since
 *           the last replacement, or it claims convergence, it pauses, u += x is
 *           formed in FP64 and the residual is replaced by the FP64 residual
 *           b - A u (FP64 matrix); the column resumes with its search
 *           direction and an exact line search for that step, and stops
 *           only when the FP64 residual meets rtol (or at maxit).
 * Converged columns drop out of the products.  iters / relres: host
 * arrays of ns x nrhs (index j * nrhs + c; may be NULL): CG iterations and
 * the final relative residual (mixed precision: of the FP64 residual).
 * Returns FL_ENOCONV if a column did not converge, FL_EBREAKDOWN if p.Ap
 * <= 0 occurred, FL_ENONFINITE for non-finite data.  Synchronises the
 * stream. */
int fl_solve_batch(fl_handle *h, const double *B, int64_t ldb, int64_t strideB, double *U, int64_t ldu,
                   int64_t strideU, int64_t nrhs, double rtol, int32_t maxit, int inner, int32_t *iters,
                   double *relres);

/* One timed kernel configuration of the batched product. */
typedef struct {
    int wm, waves, bk, planes; /* rows per wave, waves per workgroup, K stage,
                                  bf16 matrix planes                       */
    double ms;                 /* time of one product over the whole batch */
    double tflops;             /* 2 n^2 * 64 * ns / time                   */
    double gbps;               /* matrix bytes / time                      */
} fl_tune_entry;

/* Autotuner: times every GEMM configuration of `dtype` on the current
 * batch (64 columns per matrix, all matrices) and keeps the fastest for
 * later fl_matmul / fl_solve_batch calls; without this call the tuner runs
 * on first use.  out (host, may be NULL): up to max_out entries in
 * configuration order; *n_out receives the count, *best the index of the
 * chosen one. */
int fl_autotune(fl_handle *h, int dtype, fl_tune_entry *out, int max_out, int *n_out, int *best);

/* ------------------------------------------------------------------------
 * Learned pair-integral surrogate.
 *
 * For a separated pair of triangles (Sec. 5 decomposition, no common
 * vertex) the assembly needs 21 integrals over K x Kt of l_a(x) l_b(x) k,
 * l_a(y) l_b(y) k (a <= b, order 00 01 02 11 12 22) and l_a(x) l_b(y) k
 * (row-major), k = |x - y|^{-2-2s}, l the barycentric coordinates.  App. B
 * raises the Gauss order as pairs get closer; the surrogate keeps the
 * cheapest rule, order 2, and a 9-64-64-21 tanh network predicts its
 * relative error t = I / Q2 - 1 of each integral from the pair's canonical
 * form:
 *   * the triangle with the larger squared longest edge comes first (equal:
 *     the one whose lexicographically smallest vertex is smaller);
 *   * each triangle is ordered (a, b, c) with ab a longest edge (several:
 *     the one whose opposite vertex is lexicographically smallest) and c
 *     to the left of a -> b;
 *   * features: c of the first triangle and the three vertices of the
 *     second in the first's frame (origin a, x axis b - a, unit |b - a|),
 *     then s.
 * Network: inputs and targets standardised (means mx, mt; deviations sx,
 * st); W1 64x32 (columns >= 9 zero), b1, W2 64x64, b2, W3 32x64 (rows >= 21
 * zero), b3 (32, entries >= 21 zero), packed in that order (row-major);
 * tanh after layers 1 and 2.  Inference and training run on the FP16
 * matrix cores with FP32 accumulation; master weights FP32, Adam.
 * Certification: bound[rb][sb] = 1.25 x the largest |t_pred - t| over
 * held-out pairs in distance bin rb (centroid distance over the larger
 * longest edge, edges 1, 1.5, 2, 2.5, 3) and s bin sb (edges 0.25, 0.5,
 * 0.75), infinite below 32 pairs; a pair uses the network only if its
 * features lie in the box of the training features and its bin's bound at
 * the assembly's s is <= fl_opts.sur_tol.
 *
 * Parameter blob (FL_SUR_BLOB doubles): packed parameters, mx[9], sx[9],
 * mt[21], st[21], box lo[9], hi[9], bound[FL_SUR_NRB][FL_SUR_NSB].
 * ---------------------------------------------------------------------- */

typedef struct {
    int steps;            /* Adam steps                                     */
    int batch;            /* samples per step, multiple of 64               */
    double lr, lr_min;    /* cosine schedule from lr to lr_min              */
    double beta1, beta2, eps;
    uint64_t seed;        /* minibatch sampling                             */
} fl_train_opts;

/* steps 20000, batch 1024, lr 3e-3, lr_min 1e-5, beta 0.9 / 0.999, eps
 * 1e-8, seed 1. */
int fl_default_train_opts(fl_train_opts *out);

/* The 21 integrals of m separated triangle pairs with the order-k collapsed
 * Gauss rule on both triangles (k in 1..8), vertex order as given.  X, Y:
 * device m x 6 (x0 y0 x1 y1 x2 y2), s: device m, out: device m x 21.
 * Caller-owned; asynchronous on the handle's stream. */
int fl_pair_integrals(fl_handle *h, int64_t m, const double *X, const double *Y, const double *s, int k,
                      double *out);

/* Training data: canonical features (device m x 9) and targets t = I_k /
 * Q2 - 1 (device m x 21, canonical order, I_k with the order-k rule, k in
 * 3..8) of m separated pairs (device X, Y, s as fl_pair_integrals). */
int fl_surrogate_dataset(fl_handle *h, int64_t m, const double *X, const double *Y, const double *s,
                         int k_exact, double *feats, double *targets);

/* Fresh network: Glorot-uniform weights from a splitmix64 stream seeded by
 * seed, zero biases, zero Adam state; no scaling (fl_surrogate_fit_scaling
 * or fl_surrogate_set_params must follow) and no certified bin. */
int fl_surrogate_init(fl_handle *h, uint64_t seed);

/* Standardisation and box from training data (device feats m x 9, targets
 * m x 21): means, population deviations (floored at 1e-12), feature
 * minima / maxima.  Synchronises the stream. */
int fl_surrogate_fit_scaling(fl_handle *h, const double *feats, const double *targets, int64_t m);

/* Parameter blob in / out (host, FL_SUR_BLOB doubles).  set_params
 * resets the Adam state; parameters are held in FP32. */
int fl_surrogate_set_params(fl_handle *h, const double *blob);
int fl_surrogate_get_params(fl_handle *h, double *blob);

/* Full-batch loss L = mean over the m x 21 standardised entries of
 * (out - y)^2 and its gradient (host grad: FL_SUR_NPARAM floats, may be
 * NULL; host loss, may be NULL), computed by the FP16 forward / backward
 * kernels.  Synchronises the stream. */
int fl_surrogate_grad(fl_handle *h, const double *feats, const double *targets, int64_t m, float *grad,
                      double *loss);

/* Adam training on m samples (device feats / targets) with random
 * minibatches; loss_hist (host, opts->steps doubles, may be NULL) receives
 * each step's minibatch loss.  Needs scaling.  Synchronises the stream. */
int fl_surrogate_train(fl_handle *h, const double *feats, const double *targets, int64_t m,
                       const fl_train_opts *opts, double *loss_hist);

/* Predicted targets t (device out m x 21) for device features m x 9. */
int fl_surrogate_predict(fl_handle *h, const double *feats, int64_t m, double *out);

/* Certification table from held-out data (device feats / targets):
 * replaces the handle's bound table; bound (host, FL_SUR_NRB x FL_SUR_NSB,
 * may be NULL) receives it.  Synchronises the stream. */
int fl_surrogate_certify(fl_handle *h, const double *feats, const double *targets, int64_t m,
                         double *bound);

#ifdef __cplusplus
}
#endif

#endif /* FRACLAP_H */
