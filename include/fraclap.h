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

#define FL_MAX_CLASSES 8    /* distance classes for separated pairs          */
#define FL_MAX_ORDER_FAR 8  /* largest order for separated pairs             */
#define FL_MAX_ORDER_TOUCH 16 /* largest order for touching pairs            */

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
    int32_t last_iters;       /* iterations of the last solve (mixed: inner
                                 FP32 iterations summed over refinements)  */
    double last_relres;
    int32_t last_outer;       /* FP64 refinement steps of the last solve    */
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
 * until the next fl_set_mesh / fl_assemble / fl_destroy); NULL before. */
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

/* y = A x with the FP64 matrix.  x, y: device, length n, not aliased.
 * Sec. 5: the dense product costs n^2 and drives the iterative solve. */
int fl_matvec(fl_handle *h, const double *x, double *y);

/* Jacobi-preconditioned CG on A u = b (Sec. 5).  b, u: device, length n;
 * u is overwritten (initial guess 0).  Stops when ||r||_2 <= rtol ||b||_2
 * or after maxit iterations (then FL_ENOCONV with the last iterate).
 * After an FL_MIXED assembly: FP64 iterative refinement u += e with the
 * residual r = b - A u in FP64, each correction from FP32 Jacobi-PCG on the
 * FP32 copy of A to a relative residual 1e-4 (maxit bounds the total inner
 * iterations).
 * FL_EBREAKDOWN if p.Ap <= 0; FL_ENONFINITE if b is not finite.  Host
 * outputs iters / relres (may be NULL).  Synchronises the stream. */
int fl_solve(fl_handle *h, const double *b, double *u, double rtol, int32_t maxit,
             int32_t *iters, double *relres);

/* Energy-norm error against an exact solution u with known (f,u)
 * (Sec. 7 identity, valid for any discrete u_h):
 *   e2 = fu - 2 b.u_h + u_h.A u_h.
 * b, uh: device, length n.  *e2_out: host.  Synchronises the stream. */
int fl_energy_error2(fl_handle *h, double fu, const double *b, const double *uh, double *e2_out);

/* Counters and timings of the last assembly / solve. */
int fl_stats(const fl_handle *h, fl_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* FRACLAP_H */
