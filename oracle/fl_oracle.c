/*
 * fl_oracle.c -- plain FP64 CPU oracle for the dense P1 Galerkin stiffness
 * matrix of the integral fractional Laplacian (Ainsworth & Glusa,
 * "Towards an efficient finite element method for the integral fractional
 * Laplacian on polygonal domains", arXiv:1708.03912).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code with
 * the HIP library: quadrature nodes come from numpy/scipy (passed in by
 * oracle/oracle.py), the pair integrals below are written from the
 * mathematics, and nothing here is called by the product path.
 *
 * What is computed (paper Sec. 2, bilinear form with the boundary term;
 * Sec. 3, stiffness matrix A^s; Sec. 5, element-pair decomposition):
 *
 *   a(phi_i,phi_j) = sum_K sum_Kt a^{KxKt} + sum_K sum_e a^{Kxe}
 *   a^{KxKt} = C/2 int_K int_Kt (phi_i(x)-phi_i(y))(phi_j(x)-phi_j(y)) k(x,y)
 *   a^{Kxe}  = C/(2s) int_K int_e phi_i phi_j(x) n_e.(x-y) k(x,y)
 *   k(x,y)   = |x-y|^{-d-2s},  n_e the inward unit normal.
 *
 * Every routine below returns the RAW integral (no C factor); the assembly
 * loop applies C/2 (identical pair), C (unordered pair of distinct
 * elements, i.e. both orderings of the double sum) and C/(2s) (boundary).
 *
 * Quadrature (Sec. 5 and App. B: Gauss-type rules with per-pair orders;
 * touching pairs regularised because plain Gauss fails on them):
 *   - separated pairs: tensor rule of order k on each element.  Segment:
 *     k-point Gauss-Legendre.  Triangle: collapsed rule, k Gauss-Jacobi(1,0)
 *     points u_i times k Gauss-Legendre points v_j, barycentric point
 *     (lambda1, lambda2) = (u_i, (1-u_i) v_j), weight 2 WJ_i WL_j (sums to 1).
 *   - touching pairs: the integrand is (degree 2 numerator) x (homogeneous
 *     kernel) in coordinates relative to the shared vertex / edge / whole
 *     element; writing those coordinates in generalised polar form with
 *     respect to a piecewise-linear gauge whose unit sphere is a union of
 *     flat faces makes the radial integral a Beta integral in closed form.
 *     The remaining (angular) integrals are smooth and use Gauss rules of
 *     order k_T.  See each routine.
 *   - boundary pairs touching the boundary facet: same idea; the radial
 *     factor there carries a polynomial and uses 2-point Gauss-Jacobi
 *     rules (exact for the cubic it multiplies).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 32

/* Quadrature tables supplied by the caller (numpy / scipy routines).
 * gl_x/gl_w: Gauss-Legendre on [0,1], k = 1..ORC_MAXK, packed at offset
 * k(k-1)/2.  gj_x/gj_w: Gauss-Jacobi for weight (1-u) on [0,1], same
 * packing.  r0_x/r0_w: 2-point Gauss-Jacobi for weight r^{-2s} on [0,1]
 * (only meaningful for s < 1/2).  r1_x/r1_w: 2-point rule for weight
 * r^{1-2s} on [0,1]. */
typedef struct {
    const double *gl_x, *gl_w, *gj_x, *gj_w;
    double r0_x[2], r0_w[2], r1_x[2], r1_w[2];
} orc_rules;

static int off_k(int k) { return k * (k - 1) / 2; }

/* Triangle rule of order k on the reference triangle: barycentric
 * (lambda1, lambda2) and weights summing to 1.  Returns number of points. */
static int tri_rule(const orc_rules *R, int k, double *l1, double *l2, double *w) {
    const double *ux = R->gj_x + off_k(k), *uw = R->gj_w + off_k(k);
    const double *vx = R->gl_x + off_k(k), *vw = R->gl_w + off_k(k);
    int n = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            l1[n] = ux[i];
            l2[n] = (1.0 - ux[i]) * vx[j];
            w[n] = 2.0 * uw[i] * vw[j];
            ++n;
        }
    return n;
}

static double tri_area(const double *v) {
    /* v = (x0,y0,x1,y1,x2,y2) */
    double det = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
    return 0.5 * fabs(det);
}

/* ---------------------------------------------------------------- 1D ---- */

/* Separated segments K=[X0,X1], Kt=[Y0,Y1], order k.  Outputs (2x2 each,
 * row-major, local order = given endpoint order):
 *   SK[a][b]  = int_K int_Kt l_a l_b(x) k      (diagonal block, x side)
 *   SKt[a][b] = int_K int_Kt l_a l_b(y) k      (diagonal block, y side)
 *   O[a][b]   = -int_K int_Kt l_a(x) l_b(y) k  (off-diagonal block)      */
void orc_far1(const orc_rules *R, double s, int k, const double *X, const double *Y,
              double *SK, double *SKt, double *O) {
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    double hx = fabs(X[1] - X[0]), hy = fabs(Y[1] - Y[0]);
    double p = -(0.5 + s);
    memset(SK, 0, 4 * sizeof(double));
    memset(SKt, 0, 4 * sizeof(double));
    memset(O, 0, 4 * sizeof(double));
    for (int i = 0; i < k; ++i) {
        double x = X[0] + t[i] * (X[1] - X[0]);
        double lx[2] = {1.0 - t[i], t[i]};
        for (int j = 0; j < k; ++j) {
            double y = Y[0] + t[j] * (Y[1] - Y[0]);
            double ly[2] = {1.0 - t[j], t[j]};
            double d = x - y;
            double kv = pow(d * d, p) * (hx * w[i]) * (hy * w[j]);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    SK[2 * a + b] += kv * lx[a] * lx[b];
                    SKt[2 * a + b] += kv * ly[a] * ly[b];
                    O[2 * a + b] -= kv * lx[a] * ly[b];
                }
        }
    }
}

/* Identical segment pair, exact: x-y enters only through
 * lambda(x)-lambda(y) = (x-y)/h * (-1, 1), and
 * int_0^h int_0^h |x-y|^{1-2s} = 2 h^{3-2s} / ((2-2s)(3-2s)). */
void orc_ident1(double s, const double *X, double *I) {
    double h = fabs(X[1] - X[0]);
    double v = 2.0 * pow(h, 1.0 - 2.0 * s) / ((2.0 - 2.0 * s) * (3.0 - 2.0 * s));
    I[0] = v; I[1] = -v; I[2] = -v; I[3] = v;
}

/* Segments sharing the vertex q: K = [l, q], Kt = [q, r] (in any
 * orientation on the line).  Local order (l, q, r).  With x = q + u(l-q),
 * y = q + v(r-q), u, v in [0,1]:
 *   N_l = u, N_q = v - u, N_r = -v,  |x-y| = h1 u + h2 v,  dx dy = h1 h2 du dv.
 * The integrand is homogeneous of degree 1-2s in (u,v); with the gauge
 * max(u,v) the radial part is int_0^1 r^{2-2s} dr = 1/(3-2s) and the
 * angular part is the sum over the faces u=1 and v=1 of the unit square. */
void orc_vert1(const orc_rules *R, double s, int k, double xl, double xq, double xr, double *I) {
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    double h1 = fabs(xl - xq), h2 = fabs(xr - xq);
    double p = -(0.5 + s);
    double M[3][3] = {{0}};
    for (int face = 0; face < 2; ++face)
        for (int i = 0; i < k; ++i) {
            double u = face == 0 ? 1.0 : t[i];
            double v = face == 0 ? t[i] : 1.0;
            double N[3] = {u, v - u, -v};
            double dd = h1 * u + h2 * v;
            double kv = pow(dd * dd, p) * w[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] += kv * N[a] * N[b];
        }
    double f = h1 * h2 / (3.0 - 2.0 * s);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) I[3 * a + b] = f * M[a][b];
}

/* Boundary point y_e (1D "edge"), inward normal n, element K = [X0,X1].
 * n.(x-y_e) |x-y_e|^{-1-2s} = |x-y_e|^{-2s} for x in the domain.
 * touching (y_e is an endpoint of K): exact monomial integrals in
 * t = |x-y_e|; the (y_e,y_e) entry diverges for s >= 1/2 and is returned
 * as NaN (it is never a degree of freedom then).
 * separated: k-point Gauss-Legendre. */
void orc_bnd1(const orc_rules *R, double s, int k, const double *X, double ye, int touching,
              double *I) {
    double h = fabs(X[1] - X[0]);
    if (touching) {
        /* local index of the endpoint at y_e */
        int a0 = (X[0] == ye) ? 0 : 1, a1 = 1 - a0;
        double hp = pow(h, 1.0 - 2.0 * s);
        double m00 = (s < 0.5) ? hp * (1.0 / (1.0 - 2.0 * s) - 2.0 / (2.0 - 2.0 * s) + 1.0 / (3.0 - 2.0 * s))
                               : NAN;
        double m01 = hp * (1.0 / (2.0 - 2.0 * s) - 1.0 / (3.0 - 2.0 * s));
        double m11 = hp / (3.0 - 2.0 * s);
        I[2 * a0 + a0] = m00;
        I[2 * a0 + a1] = m01;
        I[2 * a1 + a0] = m01;
        I[2 * a1 + a1] = m11;
        return;
    }
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    memset(I, 0, 4 * sizeof(double));
    for (int i = 0; i < k; ++i) {
        double x = X[0] + t[i] * (X[1] - X[0]);
        double l[2] = {1.0 - t[i], t[i]};
        double kv = pow(fabs(x - ye), -2.0 * s) * h * w[i];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) I[2 * a + b] += kv * l[a] * l[b];
    }
}

/* ---------------------------------------------------------------- 2D ---- */

/* Separated triangles, order k on both (same outputs as orc_far1, 3x3). */
void orc_far2(const orc_rules *R, double s, int k, const double *X, const double *Y,
              double *SK, double *SKt, double *O) {
    double l1[ORC_MAXK * ORC_MAXK], l2[ORC_MAXK * ORC_MAXK], w[ORC_MAXK * ORC_MAXK];
    int Q = tri_rule(R, k, l1, l2, w);
    double aK = tri_area(X), aKt = tri_area(Y);
    double p = -(1.0 + s);
    memset(SK, 0, 9 * sizeof(double));
    memset(SKt, 0, 9 * sizeof(double));
    memset(O, 0, 9 * sizeof(double));
    for (int i = 0; i < Q; ++i) {
        double lx[3] = {1.0 - l1[i] - l2[i], l1[i], l2[i]};
        double x0 = lx[0] * X[0] + lx[1] * X[2] + lx[2] * X[4];
        double x1 = lx[0] * X[1] + lx[1] * X[3] + lx[2] * X[5];
        for (int j = 0; j < Q; ++j) {
            double ly[3] = {1.0 - l1[j] - l2[j], l1[j], l2[j]};
            double y0 = ly[0] * Y[0] + ly[1] * Y[2] + ly[2] * Y[4];
            double y1 = ly[0] * Y[1] + ly[1] * Y[3] + ly[2] * Y[5];
            double d0 = x0 - y0, d1 = x1 - y1;
            double kv = pow(d0 * d0 + d1 * d1, p) * (aK * w[i]) * (aKt * w[j]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    SK[3 * a + b] += kv * lx[a] * lx[b];
                    SKt[3 * a + b] += kv * ly[a] * ly[b];
                    O[3 * a + b] -= kv * lx[a] * ly[b];
                }
        }
    }
}

/* Many separated triangle pairs at once (OpenMP over the pairs): for pair
 * i the order-k rule of orc_far2 with exponent s[i], written as 21 values:
 * the K block (a <= b: 00 01 02 11 12 22), the Kt block (same order) and
 * the cross block int int l_a(x) l_b(y) k = -O[3a+b], a, b = 0..2.  The
 * tensor rules do not depend on s, so one rule table serves every pair. */
void orc_far2_many(const orc_rules *R, int64_t m, const double *s, int k, const double *X,
                   const double *Y, double *out) {
    static const int sa[6] = {0, 0, 0, 1, 1, 2}, sb[6] = {0, 1, 2, 1, 2, 2};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        double SK[9], ST[9], O[9];
        orc_far2(R, s[i], k, X + 6 * i, Y + 6 * i, SK, ST, O);
        double *o = out + 21 * i;
        for (int t = 0; t < 6; ++t) {
            o[t] = SK[3 * sa[t] + sb[t]];
            o[6 + t] = ST[3 * sa[t] + sb[t]];
        }
        for (int t = 0; t < 9; ++t) o[12 + t] = -O[t];
    }
}

/* Identical triangle K = (v0,v1,v2).  For x, y in K the numerator is
 * D_a D_b with D = lambda(x) - lambda(y) (sums to zero) and
 * x - y = sum_a D_a v_a.  Hence
 *   I_ab = int_{R^2} D_a D_b |z|^{-2-2s} |K cap (K+z)| dz,
 * and |K cap (K+z)| = |K| (1 - c(z))_+^2 where c is the gauge of the
 * difference hexagon K - K, whose vertices are the six vectors
 * +-(v_b - v_a).  In polar form over the hexagon boundary the radial
 * integral is B_id = int_0^1 r^{1-2s} (1-r)^2 dr = 2/((2-2s)(3-2s)(4-2s))
 * and, the hexagon being centrally symmetric with every edge spanning a
 * cone of |det| = 2|K|,
 *   I_ab = 4 |K|^2 B_id sum_{3 edges} int_0^1 D_a D_b |z(t)|^{-2-2s} dt
 * over the half boundary D = (-1,1,0) -> (-1,0,1) -> (0,-1,1) -> (1,-1,0). */
void orc_ident2(const orc_rules *R, double s, int k, const double *V, double *I) {
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    static const double HX[4][3] = {{-1, 1, 0}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 0}};
    double aK = tri_area(V);
    double p = -(1.0 + s);
    double M[3][3] = {{0}};
    for (int e = 0; e < 3; ++e)
        for (int i = 0; i < k; ++i) {
            double D[3];
            for (int a = 0; a < 3; ++a) D[a] = HX[e][a] + t[i] * (HX[e + 1][a] - HX[e][a]);
            double z0 = D[0] * V[0] + D[1] * V[2] + D[2] * V[4];
            double z1 = D[0] * V[1] + D[1] * V[3] + D[2] * V[5];
            double kv = pow(z0 * z0 + z1 * z1, p) * w[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] += kv * D[a] * D[b];
        }
    double Bid = 2.0 / ((2.0 - 2.0 * s) * (3.0 - 2.0 * s) * (4.0 - 2.0 * s));
    double f = 4.0 * aK * aK * Bid;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) I[3 * a + b] = f * M[a][b];
}

/* Triangles sharing the edge q0 q1: K = (q0,q1,a), Kt = (q0,q1,b).
 * Local order (q0, q1, a, b).  Coordinates x = q0 + s1 E + u a',
 * y = q0 + s2 E + v b' (E = q1-q0, a' = a-q0, b' = b-q0), w = s1 - s2:
 *   x - y = w E + u a' - v b',
 *   N = (numerator factors) = Cmat (u,v,w) with rows
 *       q0: (-1, 1,-1), q1: (0,0,1), a: (1,0,0), b: (0,-1,0),
 * both independent of the foot point s2, whose range has length
 * 1 - l(u,v,w), l = max(v, u+w) + max(0,-w) (a gauge on u,v >= 0).
 * Radial factor B_e = int_0^1 r^{2-2s}(1-r) dr = 1/((3-2s)(4-2s)); the
 * unit surface l = 1 consists of two triangles and two parallelograms,
 * each spanning a cone of |det| = 1:
 *   F1 tri  (0,1,0),(1,1,0),(0,1,1)       F4 tri  (1,0,0),(1,1,0),(1,0,-1)
 *   F2 para (1,0,0)+a(0,1,0)+b(-1,0,1)    F3 para (0,1,0)+a(1,0,0)+b(0,-1,-1)
 * (points given as (u,v,w)).  dx dy = 4|K||Kt| ds1 du ds2 dv. */
static void edge_accum(double s, const double *E, const double *ap, const double *bp, double u,
                       double v, double w, double wt, double M[3][3]) {
    double z0 = w * E[0] + u * ap[0] - v * bp[0];
    double z1 = w * E[1] + u * ap[1] - v * bp[1];
    double kv = pow(z0 * z0 + z1 * z1, -(1.0 + s)) * wt;
    double P[3] = {u, v, w};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] += kv * P[a] * P[b];
}

void orc_edge2(const orc_rules *R, double s, int k, const double *q0, const double *q1,
               const double *pa, const double *pb, double *I) {
    double l1[ORC_MAXK * ORC_MAXK], l2[ORC_MAXK * ORC_MAXK], tw[ORC_MAXK * ORC_MAXK];
    int Q = tri_rule(R, k, l1, l2, tw);
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    double E[2] = {q1[0] - q0[0], q1[1] - q0[1]};
    double ap[2] = {pa[0] - q0[0], pa[1] - q0[1]};
    double bp[2] = {pb[0] - q0[0], pb[1] - q0[1]};
    double M[3][3] = {{0}};
    static const double T1[3][3] = {{0, 1, 0}, {1, 1, 0}, {0, 1, 1}};
    static const double T4[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 0, -1}};
    for (int f = 0; f < 2; ++f) {
        const double(*T)[3] = f == 0 ? T1 : T4;
        for (int q = 0; q < Q; ++q) {
            double P[3];
            for (int c = 0; c < 3; ++c)
                P[c] = T[0][c] + l1[q] * (T[1][c] - T[0][c]) + l2[q] * (T[2][c] - T[0][c]);
            edge_accum(s, E, ap, bp, P[0], P[1], P[2], 0.5 * tw[q], M);
        }
    }
    static const double P2[3][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 1}};
    static const double P3[3][3] = {{0, 1, 0}, {1, 0, 0}, {0, -1, -1}};
    for (int f = 0; f < 2; ++f) {
        const double(*T)[3] = f == 0 ? P2 : P3;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                double P[3];
                for (int c = 0; c < 3; ++c) P[c] = T[0][c] + t[i] * T[1][c] + t[j] * T[2][c];
                edge_accum(s, E, ap, bp, P[0], P[1], P[2], w[i] * w[j], M);
            }
    }
    static const double Cm[4][3] = {{-1, 1, -1}, {0, 0, 1}, {1, 0, 0}, {0, -1, 0}};
    double X[6] = {q0[0], q0[1], q1[0], q1[1], pa[0], pa[1]};
    double Y[6] = {q0[0], q0[1], q1[0], q1[1], pb[0], pb[1]};
    double f = 4.0 * tri_area(X) * tri_area(Y) / ((3.0 - 2.0 * s) * (4.0 - 2.0 * s));
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc += Cm[i][a] * M[a][b] * Cm[j][b];
            I[4 * i + j] = f * acc;
        }
}

/* Triangles sharing only the vertex q: K = (q,b1,b2), Kt = (q,c1,c2).
 * Local order (q, b1, b2, c1, c2).  With
 *   x = q + X1 (b1-q) + X2 (b2-q),  y = q + X3 (c1-q) + X4 (c2-q),
 * N = (-X1-X2+X3+X4, X1, X2, -X3, -X4), and the domain is
 * {X >= 0, X1+X2 <= 1, X3+X4 <= 1}: the unit ball of the gauge
 * max(X1+X2, X3+X4).  Radial factor int_0^1 r^{3-2s} dr = 1/(4-2s); the unit
 * surface is two prisms (segment x triangle) each of cone |det| = 1:
 *   A: X = (1-t, t, Y1, Y2),  B: X = (Y1, Y2, 1-t, t),
 * t by k-point Gauss-Legendre, Y by the order-k triangle rule on the
 * reference triangle (area 1/2).  dx dy = 4 |K||Kt| dX. */
void orc_vert2(const orc_rules *R, double s, int k, const double *q, const double *b1,
               const double *b2, const double *c1, const double *c2, double *I) {
    double l1[ORC_MAXK * ORC_MAXK], l2[ORC_MAXK * ORC_MAXK], tw[ORC_MAXK * ORC_MAXK];
    int Q = tri_rule(R, k, l1, l2, tw);
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    double g[4][2] = {{b1[0] - q[0], b1[1] - q[1]},
                      {b2[0] - q[0], b2[1] - q[1]},
                      {-(c1[0] - q[0]), -(c1[1] - q[1])},
                      {-(c2[0] - q[0]), -(c2[1] - q[1])}};
    double M[4][4] = {{0}};
    for (int reg = 0; reg < 2; ++reg)
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < Q; ++j) {
                double X[4];
                if (reg == 0) {
                    X[0] = 1.0 - t[i]; X[1] = t[i]; X[2] = l1[j]; X[3] = l2[j];
                } else {
                    X[0] = l1[j]; X[1] = l2[j]; X[2] = 1.0 - t[i]; X[3] = t[i];
                }
                double z0 = 0.0, z1 = 0.0;
                for (int c = 0; c < 4; ++c) {
                    z0 += X[c] * g[c][0];
                    z1 += X[c] * g[c][1];
                }
                double kv = pow(z0 * z0 + z1 * z1, -(1.0 + s)) * w[i] * 0.5 * tw[j];
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) M[a][b] += kv * X[a] * X[b];
            }
    static const double Cm[5][4] = {
        {-1, -1, 1, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, -1}};
    double X[6] = {q[0], q[1], b1[0], b1[1], b2[0], b2[1]};
    double Y[6] = {q[0], q[1], c1[0], c1[1], c2[0], c2[1]};
    double f = 4.0 * tri_area(X) * tri_area(Y) / (4.0 - 2.0 * s);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) acc += Cm[i][a] * M[a][b] * Cm[j][b];
            I[5 * i + j] = f * acc;
        }
}

/* Boundary edge e = [p0,p1] (inward unit normal n) against triangle K.
 * Raw integral I_ab = int_K l_a l_b(x) int_e n.(x-y) |x-y|^{-2-2s} dy dx.
 *
 * Separated (no shared vertex): order-k triangle rule on K times k-point
 * Gauss-Legendre on e.  Local order = K's vertex order.              */
void orc_bndfar2(const orc_rules *R, double s, int k, const double *V, const double *p0,
                 const double *p1, const double *n, double *I) {
    double l1[ORC_MAXK * ORC_MAXK], l2[ORC_MAXK * ORC_MAXK], tw[ORC_MAXK * ORC_MAXK];
    int Q = tri_rule(R, k, l1, l2, tw);
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    double aK = tri_area(V);
    double Le = hypot(p1[0] - p0[0], p1[1] - p0[1]);
    memset(I, 0, 9 * sizeof(double));
    for (int i = 0; i < Q; ++i) {
        double lx[3] = {1.0 - l1[i] - l2[i], l1[i], l2[i]};
        double x0 = lx[0] * V[0] + lx[1] * V[2] + lx[2] * V[4];
        double x1 = lx[0] * V[1] + lx[1] * V[3] + lx[2] * V[5];
        double g = 0.0;
        for (int j = 0; j < k; ++j) {
            double y0 = p0[0] + t[j] * (p1[0] - p0[0]);
            double y1 = p0[1] + t[j] * (p1[1] - p0[1]);
            double d0 = x0 - y0, d1 = x1 - y1;
            g += w[j] * (n[0] * d0 + n[1] * d1) * pow(d0 * d0 + d1 * d1, -(1.0 + s));
        }
        g *= aK * tw[i] * Le;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) I[3 * a + b] += g * lx[a] * lx[b];
    }
}

/* e = [p0,p1] is an edge of K = (p0,p1,a); local order (p0,p1,a).
 * x = p0 + sig E + beta a', y = p0 + tau E (E = p1-p0, a' = a-p0);
 * n.(x-y) = beta n.a'.  With w = sig - tau the kernel part depends on
 * (w,beta) only, homogeneous of degree -1-2s; the foot tau runs over an
 * interval of length 1 - l(w,beta), l = max(0,beta+w) + max(0,-w).  The unit
 * curve l = 1 (beta >= 0) is the polyline (1,0)->(0,1)->(-1,1)->(-1,0), each
 * segment spanning |det| = 1.  Writing (w,beta) = r p, tau = tau_lo +
 * lam (1-r), the integrand is r^{-2s} (1-r) x (quadratic in r) x smooth(p):
 * 2-point Gauss-Jacobi in r, 2-point Gauss-Legendre in lam (both exact),
 * k-point Gauss-Legendre along each segment.  Entries whose basis product
 * carries the factor beta = r p_beta use weight r^{1-2s}; the entries among
 * (p0,p1) need weight r^{-2s}, integrable only for s < 1/2 (they are NaN
 * otherwise; then p0, p1 are never degrees of freedom).
 * dx dy = 2|K| |E| dsig dbeta dtau.                                        */
void orc_bndedge2(const orc_rules *R, double s, int k, const double *p0, const double *p1,
                  const double *pa, const double *n, double *I) {
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    const double *t2 = R->gl_x + off_k(2), *w2 = R->gl_w + off_k(2);
    static const double SEG[4][2] = {{1, 0}, {0, 1}, {-1, 1}, {-1, 0}};
    double E[2] = {p1[0] - p0[0], p1[1] - p0[1]};
    double ap[2] = {pa[0] - p0[0], pa[1] - p0[1]};
    double na = n[0] * ap[0] + n[1] * ap[1];
    double Le = hypot(E[0], E[1]);
    double X[6] = {p0[0], p0[1], p1[0], p1[1], pa[0], pa[1]};
    double aK = tri_area(X);
    double M[3][3] = {{0}};
    for (int sg = 0; sg < 3; ++sg)
        for (int i = 0; i < k; ++i) {
            double pw = SEG[sg][0] + t[i] * (SEG[sg + 1][0] - SEG[sg][0]);
            double pb = SEG[sg][1] + t[i] * (SEG[sg + 1][1] - SEG[sg][1]);
            double z0 = pw * E[0] + pb * ap[0], z1 = pw * E[1] + pb * ap[1];
            double ang = w[i] * pb * pow(z0 * z0 + z1 * z1, -(1.0 + s));
            double lo = pw < 0.0 ? -pw : 0.0; /* tau_lo / r */
            for (int il = 0; il < 2; ++il)
                for (int ir = 0; ir < 2; ++ir) {
                    /* weight r^{1-2s}: entries with the factor beta */
                    {
                        double r = R->r1_x[ir];
                        double tau = r * lo + t2[il] * (1.0 - r);
                        double sig = tau + r * pw, beta = r * pb;
                        double lam[3] = {1.0 - sig - beta, sig, beta};
                        double wt = ang * w2[il] * R->r1_w[ir] * (1.0 - r);
                        /* beta / r = pb */
                        for (int b = 0; b < 3; ++b) {
                            double v = wt * pb * lam[b];
                            M[2][b] += v;
                            if (b != 2) M[b][2] += v;
                        }
                    }
                    if (s < 0.5) {
                        double r = R->r0_x[ir];
                        double tau = r * lo + t2[il] * (1.0 - r);
                        double sig = tau + r * pw, beta = r * pb;
                        double lam[2] = {1.0 - sig - beta, sig};
                        double wt = ang * w2[il] * R->r0_w[ir] * (1.0 - r);
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b) M[a][b] += wt * lam[a] * lam[b];
                    }
                }
        }
    double f = 2.0 * aK * Le * na;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            int both_edge = (a < 2 && b < 2);
            I[3 * a + b] = (both_edge && !(s < 0.5)) ? NAN : f * M[a][b];
        }
}

/* e = [q,p] shares only the vertex q with K = (q,b1,b2); local order
 * (q,b1,b2).  x = q + u A(t1), A(t1) = (b1-q) + t1 (b2-b1), y = q + v E
 * (E = p-q); dx = 2|K| u du dt1, dy = |E| dv, n.(x-y) = u n.A.  In (u,v)
 * with the gauge max(u,v) (faces u=1 and v=1, each |det| = 1) the
 * integrand is r^{1-2s} x (quadratic in r) x smooth: 2-point Gauss-Jacobi
 * for weight r^{1-2s}, k-point Gauss-Legendre in t1 and along each face. */
void orc_bndvert2(const orc_rules *R, double s, int k, const double *q, const double *b1,
                  const double *b2, const double *pp, const double *n, double *I) {
    const double *t = R->gl_x + off_k(k), *w = R->gl_w + off_k(k);
    double E[2] = {pp[0] - q[0], pp[1] - q[1]};
    double Le = hypot(E[0], E[1]);
    double X[6] = {q[0], q[1], b1[0], b1[1], b2[0], b2[1]};
    double aK = tri_area(X);
    double M[3][3] = {{0}};
    for (int face = 0; face < 2; ++face)
        for (int i = 0; i < k; ++i) {
            double pu = face == 0 ? 1.0 : t[i];
            double pv = face == 0 ? t[i] : 1.0;
            for (int j = 0; j < k; ++j) {
                double A0 = (b1[0] - q[0]) + t[j] * (b2[0] - b1[0]);
                double A1 = (b1[1] - q[1]) + t[j] * (b2[1] - b1[1]);
                double z0 = pu * A0 - pv * E[0], z1 = pu * A1 - pv * E[1];
                double ang = w[i] * w[j] * pu * pu * (n[0] * A0 + n[1] * A1) *
                             pow(z0 * z0 + z1 * z1, -(1.0 + s));
                for (int ir = 0; ir < 2; ++ir) {
                    double r = R->r1_x[ir];
                    double uu = r * pu;
                    double lam[3] = {1.0 - uu, uu * (1.0 - t[j]), uu * t[j]};
                    double wt = ang * R->r1_w[ir];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) M[a][b] += wt * lam[a] * lam[b];
                }
            }
        }
    double f = 2.0 * aK * Le;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) I[3 * a + b] = f * M[a][b];
}

/* --------------------------------------------------------- classification */

/* Order class of a separated pair from the ratio of centroid distance to
 * the larger element diameter (App. B: the required order decreases with
 * dist/h).  Evaluated with a fixed operation order (no contraction) so that
 * an independent implementation reproduces it bit for bit:
 *   class = #{m : d2 >= theta_m^2 * max(h2_K, h2_Kt)}.                     */
static int order_class(double d2, double hmax2, int ncls, const double *theta) {
    int c = 0;
    for (int m = 0; m < ncls; ++m) {
        double th2 = theta[m] * theta[m];
        if (d2 >= th2 * hmax2) c = m + 1;
    }
    return c;
}

static void centroid_h2(int dim, const double *verts, const int32_t *cell, double *c, double *h2) {
    if (dim == 1) {
        double x0 = verts[cell[0]], x1 = verts[cell[1]];
        c[0] = (x0 + x1) / 2.0;
        double e = x1 - x0;
        *h2 = e * e;
        return;
    }
    const double *a = verts + 2 * cell[0], *b = verts + 2 * cell[1], *d = verts + 2 * cell[2];
    c[0] = ((a[0] + b[0]) + d[0]) / 3.0;
    c[1] = ((a[1] + b[1]) + d[1]) / 3.0;
    double m = 0.0;
    const double *P[3] = {a, b, d};
    for (int i = 0; i < 3; ++i) {
        const double *u = P[i], *v = P[(i + 1) % 3];
        double e0 = v[0] - u[0], e1 = v[1] - u[1];
        double l = e0 * e0 + e1 * e1;
        if (l > m) m = l;
    }
    *h2 = m;
}

/* --------------------------------------------------------------- assembly */

typedef struct {
    double s;
    int k_touch, k_touch_bnd;
    int ncls;
    const double *theta;   /* ncls thresholds (increasing) */
    const int *k_far;      /* ncls+1 orders for separated element pairs */
    const int *k_far_bnd;  /* ncls+1 orders for separated element/facet pairs */
    int with_boundary;     /* 0: drop a^{Kxe} (regional operator) */
    int which;             /* bitmask: 1 far, 2 touching, 4 boundary */
    int far_skip_below;    /* separated pairs of class < this are left out
                              (counted only); 0: none */
    const double *cell_w;  /* NULL, or a weight per cell: pair (K, Kt) counts
                              with (w_K + w_Kt) / 2 (identical pairs and the
                              boundary term with w_K), pairs of weight 0 are
                              skipped (symmetry reduction, Sec. 7) */
    const int *cell_pre;   /* with cell_w: NULL, or for every cell the sector
                              cell it is an image of, and ... */
    const int *cell_rot;   /* ... the rotation B^i that maps it there; then
                              of the two equal cross pairs (S, B^i T) and
                              (T, B^-i S) only one counts, with weight 1 */
    int sym_order;         /* K, the order of B */
    const int *cell_leaf;  /* NULL, or a label per cell (a leaf of a cluster
                              tree, 0..nleaf-1) ... */
    int nleaf;
    const unsigned char *leaf_near;  /* ... and an nleaf x nleaf table: the
                              separated pair (K, Kt) adds its diagonal-block
                              parts (the terms phi_i phi_j(x) and
                              phi_i phi_j(y) of Sec. 5's pair integrand) only
                              if leaf_near[label K][label Kt] is nonzero; its
                              off-diagonal block is always added */
} orc_opts;

/* Weight of the cell pair (K, Kt) in a symmetry-reduced assembly: pairs of
 * sector cells 1, pairs of images 0; a sector cell S with an image L of
 * the sector cell p = pre(L) under B^i: without pre/rot 1/2 (both members
 * of each couple (S, B^i p) ~ (p, B^-i S) are present), with them 1 for
 * p > S, 0 for p < S, and for p = S 1 if 2 i < K, 1/2 if 2 i = K, 0 else. */
static double pair_weight(const orc_opts *o, int64_t K, int64_t Kt) {
    if (!o->cell_w) return 1.0;
    const double wK = o->cell_w[K], wT = o->cell_w[Kt];
    if (!o->cell_pre) return 0.5 * (wK + wT);
    if (wK == wT) return wK;
    const int64_t S = wK > wT ? K : Kt, L = wK > wT ? Kt : K;
    const int64_t p = o->cell_pre[L];
    if (p != S) return p > S ? 1.0 : 0.0;
    const int r2 = 2 * o->cell_rot[L];
    return r2 < o->sym_order ? 1.0 : (r2 == o->sym_order ? 0.5 : 0.0);
}

static double cdn(int dim, double s) {
    /* C(d,s) = 2^{2s} s Gamma(s+d/2) / (pi^{d/2} Gamma(1-s)) */
    return pow(2.0, 2.0 * s) * s * tgamma(s + 0.5 * dim) / (pow(M_PI, 0.5 * dim) * tgamma(1.0 - s));
}

double orc_cdn(int dim, double s) { return cdn(dim, s); }

static void add_block(double *A, int64_t nv, const int32_t *rowmask, const int *gi, int na,
                      const int *gj, int nb, const double *B, int ldb, double f) {
    for (int a = 0; a < na; ++a) {
        if (rowmask && rowmask[gi[a]] < 0) continue;
        const int64_t row = rowmask ? rowmask[gi[a]] : gi[a];
        for (int b = 0; b < nb; ++b) {
            double v = f * B[ldb * a + b];
#pragma omp atomic
            A[row * nv + gj[b]] += v;
        }
    }
}

/* Assemble the full-node matrix (nv x nv, row-major, accumulated into A)
 * for the mesh.  rowmask (nv ints, may be NULL) restricts accumulation to
 * the rows of the vertices v with rowmask[v] >= 0, stored as row
 * rowmask[v] of A (then A has that many rows of nv); pairs that cannot
 * reach such a row are skipped.  bnd_normals: nb x dim inward unit normals of the facets.
 * Returns the number of separated pairs per class in cls_count. */
void orc_assemble(const orc_rules *R, const orc_opts *o, int dim, int64_t nv, const double *verts,
                  int64_t nc, const int32_t *cells, int64_t nb, const int32_t *bfacets,
                  const double *bnormals, const int32_t *rowmask, double *A, int64_t *cls_count) {
    const int nper = dim + 1;
    const double s = o->s;
    const double C = cdn(dim, s);
    double *cen = (double *)malloc(sizeof(double) * nc * dim);
    double *h2 = (double *)malloc(sizeof(double) * nc);
    char *hit = (char *)malloc(nc);
    for (int64_t K = 0; K < nc; ++K) {
        centroid_h2(dim, verts, cells + nper * K, cen + dim * K, h2 + K);
        hit[K] = 0;
        for (int a = 0; a < nper; ++a)
            if (!rowmask || rowmask[cells[nper * K + a]] >= 0) hit[K] = 1;
    }
    int64_t cnt[16] = {0};

#pragma omp parallel for schedule(dynamic, 4) reduction(+ : cnt[:16])
    for (int64_t K = 0; K < nc; ++K) {
        const int32_t *cK = cells + nper * K;
        for (int64_t Kt = K; Kt < nc; ++Kt) {
            if (!hit[K] && !hit[Kt]) continue;
            const double wp = pair_weight(o, K, Kt);
            if (wp == 0.0) continue;
            const int32_t *cT = cells + nper * Kt;
            int gK[3], gT[3];
            for (int a = 0; a < nper; ++a) { gK[a] = cK[a]; gT[a] = cT[a]; }
            if (K == Kt) {
                if (!(o->which & 2)) continue;
                double I[9];
                if (dim == 1) {
                    double X[2] = {verts[gK[0]], verts[gK[1]]};
                    orc_ident1(s, X, I);
                } else {
                    double X[6];
                    for (int a = 0; a < 3; ++a) { X[2 * a] = verts[2 * gK[a]]; X[2 * a + 1] = verts[2 * gK[a] + 1]; }
                    orc_ident2(R, s, o->k_touch, X, I);
                }
                add_block(A, nv, rowmask, gK, nper, gK, nper, I, nper, 0.5 * C * wp);
                continue;
            }
            /* shared vertices */
            int nsh = 0, shK[3], shT[3];
            for (int a = 0; a < nper; ++a)
                for (int b = 0; b < nper; ++b)
                    if (gK[a] == gT[b]) { shK[nsh] = a; shT[nsh] = b; ++nsh; }
            if (nsh == 0) {
                if (!(o->which & 1)) continue;
                double d2 = 0.0;
                for (int c = 0; c < dim; ++c) {
                    double dd = cen[dim * K + c] - cen[dim * Kt + c];
                    d2 += dd * dd;
                }
                double hm = h2[K] > h2[Kt] ? h2[K] : h2[Kt];
                int cls = order_class(d2, hm, o->ncls, o->theta);
                cnt[cls] += 1;
                if (cls < o->far_skip_below) continue;
                int k = o->k_far[cls];
                double SK[9], ST[9], O[9];
                if (dim == 1) {
                    double X[2] = {verts[gK[0]], verts[gK[1]]}, Y[2] = {verts[gT[0]], verts[gT[1]]};
                    orc_far1(R, s, k, X, Y, SK, ST, O);
                } else {
                    double X[6], Y[6];
                    for (int a = 0; a < 3; ++a) {
                        X[2 * a] = verts[2 * gK[a]]; X[2 * a + 1] = verts[2 * gK[a] + 1];
                        Y[2 * a] = verts[2 * gT[a]]; Y[2 * a + 1] = verts[2 * gT[a] + 1];
                    }
                    orc_far2(R, s, k, X, Y, SK, ST, O);
                }
                if (!o->cell_leaf || o->leaf_near[(int64_t)o->cell_leaf[K] * o->nleaf + o->cell_leaf[Kt]]) {
                    add_block(A, nv, rowmask, gK, nper, gK, nper, SK, nper, C * wp);
                    add_block(A, nv, rowmask, gT, nper, gT, nper, ST, nper, C * wp);
                }
                add_block(A, nv, rowmask, gK, nper, gT, nper, O, nper, C * wp);
                double OT[9];
                for (int a = 0; a < nper; ++a)
                    for (int b = 0; b < nper; ++b) OT[nper * a + b] = O[nper * b + a];
                add_block(A, nv, rowmask, gT, nper, gK, nper, OT, nper, C * wp);
                continue;
            }
            if (!(o->which & 2)) continue;
            if (dim == 1) {
                /* common vertex: local (l, q, r) */
                int q = gK[shK[0]], l = gK[1 - shK[0]], r = gT[1 - shT[0]];
                double I[9];
                orc_vert1(R, s, o->k_touch, verts[l], verts[q], verts[r], I);
                int g[3] = {l, q, r};
                add_block(A, nv, rowmask, g, 3, g, 3, I, 3, C * wp);
            } else if (nsh == 2) {
                int a0 = gK[shK[0]], a1 = gK[shK[1]];
                int q0 = a0 < a1 ? a0 : a1, q1 = a0 < a1 ? a1 : a0;
                int pa = gK[3 - shK[0] - shK[1]], pb = gT[3 - shT[0] - shT[1]];
                double I[16];
                orc_edge2(R, s, o->k_touch, verts + 2 * q0, verts + 2 * q1, verts + 2 * pa,
                          verts + 2 * pb, I);
                int g[4] = {q0, q1, pa, pb};
                add_block(A, nv, rowmask, g, 4, g, 4, I, 4, C * wp);
            } else {
                int q = gK[shK[0]];
                int b1 = gK[(shK[0] + 1) % 3], b2 = gK[(shK[0] + 2) % 3];
                int c1 = gT[(shT[0] + 1) % 3], c2 = gT[(shT[0] + 2) % 3];
                if (b1 > b2) { int tt = b1; b1 = b2; b2 = tt; }
                if (c1 > c2) { int tt = c1; c1 = c2; c2 = tt; }
                double I[25];
                orc_vert2(R, s, o->k_touch, verts + 2 * q, verts + 2 * b1, verts + 2 * b2,
                          verts + 2 * c1, verts + 2 * c2, I);
                int g[5] = {q, b1, b2, c1, c2};
                add_block(A, nv, rowmask, g, 5, g, 5, I, 5, C * wp);
            }
        }
    }

    if (o->with_boundary && (o->which & 4)) {
        const double fb = C / (2.0 * s);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t K = 0; K < nc; ++K) {
            if (!hit[K]) continue;
            const double fbK = fb * (o->cell_w ? o->cell_w[K] : 1.0);
            if (fbK == 0.0) continue;
            const int32_t *cK = cells + nper * K;
            int gK[3];
            for (int a = 0; a < nper; ++a) gK[a] = cK[a];
            for (int64_t e = 0; e < nb; ++e) {
                const int32_t *fe = bfacets + dim * e;
                const double *n = bnormals + dim * e;
                double I[9];
                if (dim == 1) {
                    int touching = (gK[0] == fe[0] || gK[1] == fe[0]);
                    double X[2] = {verts[gK[0]], verts[gK[1]]};
                    int k = 0;
                    if (!touching) {
                        double c[1], hh;
                        centroid_h2(1, verts, cK, c, &hh);
                        double dd = c[0] - verts[fe[0]];
                        int cls = order_class(dd * dd, hh, o->ncls, o->theta);
                        k = o->k_far_bnd[cls];
                    }
                    orc_bnd1(R, s, k, X, verts[fe[0]], touching, I);
                    add_block(A, nv, rowmask, gK, 2, gK, 2, I, 2, fbK);
                    continue;
                }
                int sh0 = -1, sh1 = -1;
                for (int a = 0; a < 3; ++a) {
                    if (gK[a] == fe[0]) sh0 = a;
                    if (gK[a] == fe[1]) sh1 = a;
                }
                const double *p0 = verts + 2 * fe[0], *p1 = verts + 2 * fe[1];
                if (sh0 >= 0 && sh1 >= 0) {
                    int pa = gK[3 - sh0 - sh1];
                    orc_bndedge2(R, s, o->k_touch_bnd, p0, p1, verts + 2 * pa, n, I);
                    int g[3] = {fe[0], fe[1], pa};
                    add_block(A, nv, rowmask, g, 3, g, 3, I, 3, fbK);
                } else if (sh0 >= 0 || sh1 >= 0) {
                    int a = sh0 >= 0 ? sh0 : sh1;
                    int q = gK[a];
                    int pother = sh0 >= 0 ? fe[1] : fe[0];
                    int b1 = gK[(a + 1) % 3], b2 = gK[(a + 2) % 3];
                    if (b1 > b2) { int tt = b1; b1 = b2; b2 = tt; }
                    orc_bndvert2(R, s, o->k_touch_bnd, verts + 2 * q, verts + 2 * b1,
                                 verts + 2 * b2, verts + 2 * pother, n, I);
                    int g[3] = {q, b1, b2};
                    add_block(A, nv, rowmask, g, 3, g, 3, I, 3, fbK);
                } else {
                    double c[2], hh;
                    centroid_h2(2, verts, cK, c, &hh);
                    double m0 = (p0[0] + p1[0]) / 2.0, m1 = (p0[1] + p1[1]) / 2.0;
                    double e0 = p1[0] - p0[0], e1 = p1[1] - p0[1];
                    double le2 = e0 * e0 + e1 * e1;
                    double d0 = c[0] - m0, d1 = c[1] - m1;
                    double hm = hh > le2 ? hh : le2;
                    int cls = order_class(d0 * d0 + d1 * d1, hm, o->ncls, o->theta);
                    double X[6];
                    for (int b = 0; b < 3; ++b) { X[2 * b] = verts[2 * gK[b]]; X[2 * b + 1] = verts[2 * gK[b] + 1]; }
                    orc_bndfar2(R, s, o->k_far_bnd[cls], X, p0, p1, n, I);
                    add_block(A, nv, rowmask, gK, 3, gK, 3, I, 3, fbK);
                }
            }
        }
    }
    if (cls_count)
        for (int m = 0; m <= o->ncls; ++m) cls_count[m] = cnt[m];
    free(cen);
    free(h2);
    free(hit);
}

/* Dense FP64 matrix-vector product y = A x (row-major n x n), used as the
 * CPU reference for the dense matvec (Sec. 5: n^2 work per product). */
void orc_matvec(int64_t n, const double *A, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        const double *row = A + i * n;
        for (int64_t j = 0; j < n; ++j) acc += row[j] * x[j];
        y[i] = acc;
    }
}

/* Jacobi-preconditioned conjugate gradients (Sec. 5: CG with diagonal
 * scaling converges in O(n^{s/d}) iterations).  x0 = 0; stop when
 * ||r||_2 <= rtol ||b||_2.  Returns the iteration count (or -1 on
 * breakdown p.Ap <= 0); x receives the iterate. */
int orc_pcg(int64_t n, const double *A, const double *b, double *x, double rtol, int maxit,
            double *relres) {
    double *r = (double *)malloc(sizeof(double) * n), *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n), *q = (double *)malloc(sizeof(double) * n);
    double bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        z[i] = r[i] / A[i * n + i];
        p[i] = z[i];
        bb += b[i] * b[i];
    }
    double rz = 0.0, rr = bb;
    for (int64_t i = 0; i < n; ++i) rz += r[i] * z[i];
    double nb = sqrt(bb);
    int it = 0;
    while (sqrt(rr) > rtol * nb && it < maxit) {
        orc_matvec(n, A, p, q);
        double pq = 0.0;
        for (int64_t i = 0; i < n; ++i) pq += p[i] * q[i];
        if (!(pq > 0.0)) { it = -1; break; }
        double alpha = rz / pq;
        double rz2 = 0.0;
        rr = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = r[i] / A[i * n + i];
            rz2 += r[i] * z[i];
            rr += r[i] * r[i];
        }
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        ++it;
    }
    if (relres) *relres = sqrt(rr) / nb;
    free(r); free(z); free(p); free(q);
    return it;
}

/* Separated triangle pairs (K < Kt, no common vertex) whose order class
 * (thresholds theta on centroid distance / larger longest edge, as in
 * orc_assemble) is below nsur.  For each: K, Kt, the class and the bin of
 * the same ratio for the thresholds redges (nr of them).  Writes at most
 * cap entries of 4 int64 each; returns the total count. */
int64_t orc_band_pairs(const double *verts, int64_t nc, const int32_t *cells, int ncls,
                       const double *theta, int nsur, int nr, const double *redges, int64_t cap,
                       int64_t *out) {
    double *cen = (double *)malloc(sizeof(double) * nc * 2);
    double *h2 = (double *)malloc(sizeof(double) * nc);
    for (int64_t K = 0; K < nc; ++K) centroid_h2(2, verts, cells + 3 * K, cen + 2 * K, h2 + K);
    int64_t n = 0;
    for (int64_t K = 0; K < nc; ++K)
        for (int64_t Kt = K + 1; Kt < nc; ++Kt) {
            const int32_t *cK = cells + 3 * K, *cT = cells + 3 * Kt;
            int sh = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) sh += cK[a] == cT[b];
            if (sh) continue;
            double dx = cen[2 * K] - cen[2 * Kt], dy = cen[2 * K + 1] - cen[2 * Kt + 1];
            double d2 = dx * dx + dy * dy;
            double hm = h2[K] > h2[Kt] ? h2[K] : h2[Kt];
            int cls = order_class(d2, hm, ncls, theta);
            if (cls >= nsur) continue;
            if (n < cap) {
                out[4 * n] = K;
                out[4 * n + 1] = Kt;
                out[4 * n + 2] = cls;
                out[4 * n + 3] = order_class(d2, hm, nr, redges);
            }
            ++n;
        }
    free(cen);
    free(h2);
    return n;
}
