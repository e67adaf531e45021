// Strong form of the fractional Laplacian of a P1 function and the
// Babuska-Rheinboldt type error indicators (Sec. 4: the lemma on the strong
// form, eq. 8, and eq. 9 for d = 1, s = 1/2; the indicators eta-hat_i).
//
// Eq. 8 sums, for x in K0, boundary integrals of every cell K: a gradient
// term grad u|K . n |x-y|^{-(d+2s-2)} and a value term u(y) n.(x-y)
// |x-y|^{-(d+2s)}, with other coefficients on K0 itself.  The evaluation is
// split so that the all-pairs part is a plain potential sum:
//   * far (sf_far_kernel): every cell with the separated-cell rule.  On a
//     facet shared by two cells the value terms cancel (u is continuous,
//     the normals are opposite), so each facet carries one coefficient,
//     the jump of the normal derivative: a sum of c_j |x - y_j|^{-(d+2s-2)}
//     over q_far Gauss points y_j per facet.  Boundary facets keep their
//     gradient term here and their value term in the next kernel.
//   * near (sf_near_kernel): for the cells sharing a vertex with K0 the
//     separated-cell terms are replaced by the touching-cell rule (with
//     K0's own coefficients on K0); the value terms of boundary facets
//     (present only when boundary vertices carry DOFs, s < 1/2); the
//     far-field partial sums are reduced in a fixed order.  16 lanes per
//     evaluation point share its touching cells and boundary facets.
// Both kernels are FP64.  In d = 1 a facet is a vertex and its integral a
// point value; only K0 itself needs a correction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fl_internal.hpp"
#include "fl_math.hpp"

namespace fl {

namespace {

constexpr int SF_TILE = 256;  // sources staged in LDS per step
constexpr int SF_TPT = 2;     // targets per thread in the far kernel

// u at vertex a of cell K (0 if the vertex carries no DOF)
__device__ __forceinline__ double uval(const SfDev& D, const double* u, long long K, int a) {
    const int d = D.cdof[K * (D.dim + 1) + a];
    return d >= 0 ? u[d] : 0.0;
}

// Cell K: vertex coordinates, values, gradient of u and orientation sign.
template <int DIM>
struct SfCell {
    double p[DIM + 1][DIM];
    double u[DIM + 1];
    double g[DIM];
    double sgn;
};

template <int DIM>
__device__ __forceinline__ void load_cell(const SfDev& D, const double* u, long long K, SfCell<DIM>& c) {
    const double* x = D.cx + K * (DIM + 1) * DIM;
    for (int a = 0; a <= DIM; ++a) {
        for (int d = 0; d < DIM; ++d) c.p[a][d] = x[a * DIM + d];
        c.u[a] = uval(D, u, K, a);
    }
    if constexpr (DIM == 1) {
        const double h = c.p[1][0] - c.p[0][0];
        c.g[0] = (c.u[1] - c.u[0]) / h;
        c.sgn = h > 0.0 ? 1.0 : -1.0;
    } else {
        // solve [b - a; c - a] g = [u_b - u_a; u_c - u_a]
        const double e1x = c.p[1][0] - c.p[0][0], e1y = c.p[1][1] - c.p[0][1];
        const double e2x = c.p[2][0] - c.p[0][0], e2y = c.p[2][1] - c.p[0][1];
        const double det = e1x * e2y - e2x * e1y;
        const double d1 = c.u[1] - c.u[0], d2 = c.u[2] - c.u[0];
        c.g[0] = (d1 * e2y - d2 * e1y) / det;
        c.g[1] = (e1x * d2 - e2x * d1) / det;
        c.sgn = det > 0.0 ? 1.0 : -1.0;
    }
}

// Facet e of a cell: start point A, direction E (B - A), outward normal N
// times the facet measure, end values.  d = 2: edge from vertex e to vertex
// e + 1; d = 1: vertex e, E = 0, N = +-1.
template <int DIM>
struct SfFacet {
    double A[2], E[2], N[2], ua, ub;
};

template <int DIM>
__device__ __forceinline__ SfFacet<DIM> facet_of(const SfCell<DIM>& c, int e) {
    SfFacet<DIM> f;
    if constexpr (DIM == 1) {
        f.A[0] = c.p[e][0];
        f.A[1] = 0.0;
        f.E[0] = f.E[1] = 0.0;
        f.N[0] = (c.p[e][0] > c.p[1 - e][0]) ? 1.0 : -1.0;
        f.N[1] = 0.0;
        f.ua = f.ub = c.u[e];
    } else {
        const int b = e == 2 ? 0 : e + 1;
        f.A[0] = c.p[e][0];
        f.A[1] = c.p[e][1];
        f.E[0] = c.p[b][0] - c.p[e][0];
        f.E[1] = c.p[b][1] - c.p[e][1];
        f.N[0] = c.sgn * f.E[1];
        f.N[1] = -c.sgn * f.E[0];
        f.ua = c.u[e];
        f.ub = c.u[b];
    }
    return f;
}

// Rule sums over one facet: Ig = sum w g(r2), Iu = sum w kern n.(x-y) u(y),
// Io = sum w kern n.(x-y), with g = |x-y|^{-(d+2s-2)} (log(1/|x-y|) in the
// log form) and kern = |x-y|^{-(d+2s)} = g / r2 (1 / r2 in the log form).
template <int DIM, bool LOGK, class POW>
__device__ __forceinline__ void facet_sums(const SfFacet<DIM>& f, double x, double y, int q, const double* gx,
                                           const double* gw, const POW& P, double& Ig, double& Iu, double& Io) {
    Ig = Iu = Io = 0.0;
    const int nq = DIM == 1 ? 1 : q;
    const int off = gl_off(nq);
    for (int j = 0; j < nq; ++j) {
        const double t = DIM == 1 ? 0.0 : gx[off + j];
        const double w = DIM == 1 ? 1.0 : gw[off + j];
        const double dx = x - fma(t, f.E[0], f.A[0]);
        const double dy = DIM == 1 ? 0.0 : y - fma(t, f.E[1], f.A[1]);
        const double r2 = fma(dx, dx, dy * dy);
        double g, kern;
        if constexpr (LOGK) {
            g = -0.5 * log(r2);
            kern = 1.0 / r2;
        } else {
            g = P(r2);
            kern = g / r2;
        }
        const double nd = fma(dx, f.N[0], dy * f.N[1]);
        const double uy = fma(t, f.ub - f.ua, f.ua);
        Ig = fma(w, g, Ig);
        const double wk = w * kern * nd;
        Iu = fma(wk, uy, Iu);
        Io += wk;
    }
}

__device__ __forceinline__ void load_tab(double* pw, const double* tab) {
    for (int i = threadIdx.x; i < 768; i += blockDim.x) pw[i] = tab[i];
}

__device__ __forceinline__ KPowTab tab_pow(const double* pw, const double* tab) {
    return KPowTab{pw, tab[769], tab[770], tab[771], tab[772], tab[773]};
}

// One thread per facet: coefficients of its q_far sources,
//   c_j = w_j (grad u|K1 . N - grad u|K2 . N) cg   (N: outward of K1).
template <int DIM>
__global__ __launch_bounds__(256) void sf_sources_kernel(SfDev D, const double* __restrict__ u) {
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= D.nf) return;
    const int K1 = D.fK[2 * f], K2 = D.fK[2 * f + 1];
    SfCell<DIM> c;
    load_cell<DIM>(D, u, K1, c);
    const double N0 = D.fN[DIM * f], N1 = DIM == 2 ? D.fN[DIM * f + 1] : 0.0;
    double gN = DIM == 2 ? fma(c.g[0], N0, c.g[DIM - 1] * N1) : c.g[0] * N0;
    if (K2 >= 0) {
        load_cell<DIM>(D, u, K2, c);
        gN -= DIM == 2 ? fma(c.g[0], N0, c.g[DIM - 1] * N1) : c.g[0] * N0;
    }
    gN *= D.cg;
    if constexpr (DIM == 1) {
        D.sc[f] = gN;
    } else {
        const int off = gl_off(D.qf);
        for (int j = 0; j < D.qf; ++j) D.sc[f * D.qf + j] = D.gw[off + j] * gN;
    }
}

// Targets x SF_TPT per thread, a chunk of sources per workgroup row:
//   part[chunk][t] = sum_j c_j g(|x_t - y_j|^2)
// for the rows below nch (jumps of the normal derivative), and for the
// rows from nch on the value terms of the boundary facets,
//   part[nch + chunk][t] = sum_j g(r2) / r2 (b_j . (x_t - y_j)),
// b_j = -w_j u(y_j) N / (2s).  Sources pass through LDS (broadcast reads),
// the kernel power through the LDS tables; no branch in the inner loops.
template <bool LOGK>
__global__ __launch_bounds__(256) void sf_far_kernel(long long nt, const double* __restrict__ tx,
                                                     const double* __restrict__ ty, long long ns,
                                                     const double* __restrict__ sx, const double* __restrict__ sy,
                                                     const double* __restrict__ sc, long long chunk, int nch,
                                                     long long nbs, const double* __restrict__ bsx,
                                                     const double* __restrict__ bsy,
                                                     const double* __restrict__ bc,
                                                     const double* __restrict__ tab, double* __restrict__ part) {
    __shared__ double pw[768];
    __shared__ double4 src[SF_TILE];
    const int tid = threadIdx.x;
    if constexpr (!LOGK) load_tab(pw, tab);
    const KPowTab P = tab_pow(pw, tab);
    double x[SF_TPT], y[SF_TPT], acc[SF_TPT];
#pragma unroll
    for (int i = 0; i < SF_TPT; ++i) {
        long long t = (long long)blockIdx.x * (256 * SF_TPT) + i * 256 + tid;
        t = t < nt ? t : nt - 1;
        x[i] = tx[t];
        y[i] = ty[t];
        acc[i] = 0.0;
    }
    const bool bnd = (int)blockIdx.y >= nch;
    const long long n_src = bnd ? nbs : ns;
    const long long j0 = (long long)(bnd ? blockIdx.y - nch : blockIdx.y) * chunk;
    const long long j1 = j0 + chunk < n_src ? j0 + chunk : n_src;
    for (long long jt = j0; jt < j1; jt += SF_TILE) {
        const int m = (int)(j1 - jt < SF_TILE ? j1 - jt : SF_TILE);
        __syncthreads();
        if (tid < m) {
            const long long j = jt + tid;
            src[tid] = bnd ? make_double4(bsx[j], bsy[j], bc[2 * j], bc[2 * j + 1])
                           : make_double4(sx[j], sy[j], sc[j], 0.0);
        }
        __syncthreads();
        if (!bnd) {
#pragma unroll 2
            for (int j = 0; j < m; ++j) {
                const double4 S = src[j];
#pragma unroll
                for (int i = 0; i < SF_TPT; ++i) {
                    const double dx = x[i] - S.x, dy = y[i] - S.y;
                    const double r2 = fma(dx, dx, dy * dy);
                    const double g = LOGK ? -0.5 * log(r2) : P(r2);
                    acc[i] = fma(S.z, g, acc[i]);
                }
            }
        } else {
            for (int j = 0; j < m; ++j) {
                const double4 S = src[j];
#pragma unroll
                for (int i = 0; i < SF_TPT; ++i) {
                    const double dx = x[i] - S.x, dy = y[i] - S.y;
                    const double r2 = fma(dx, dx, dy * dy);
                    const double kern = LOGK ? 1.0 / r2 : P(r2) / r2;
                    acc[i] = fma(kern, fma(S.z, dx, S.w * dy), acc[i]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < SF_TPT; ++i) {
        const long long t = (long long)blockIdx.x * (256 * SF_TPT) + i * 256 + tid;
        if (t < nt) part[(long long)blockIdx.y * nt + t] = acc[i];
    }
}

// One thread per boundary facet (only when boundary vertices carry DOFs):
// the value-term coefficients b_j = -w_j u(y_j) N / (2s) of its q_far points.
template <int DIM>
__global__ __launch_bounds__(256) void sf_bsources_kernel(SfDev D, const double* __restrict__ u) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= D.nbf) return;
    const int2 kb = D.bf[b];
    SfCell<DIM> c;
    load_cell<DIM>(D, u, kb.x, c);
    const SfFacet<DIM> f = facet_of<DIM>(c, kb.y);
    const int nq = DIM == 1 ? 1 : D.qf;
    const int off = gl_off(nq);
    for (int j = 0; j < nq; ++j) {
        const double t = DIM == 1 ? 0.0 : D.gx[off + j];
        const double w = DIM == 1 ? 1.0 : D.gw[off + j];
        const double c0 = -D.inv2s * w * fma(t, f.ub - f.ua, f.ua);
        D.bc[2 * (b * nq + j)] = c0 * f.N[0];
        D.bc[2 * (b * nq + j) + 1] = c0 * f.N[1];
    }
}

// SF_G lanes per target (cell K0, point q), 64 / SF_G targets per wave: the
// lanes of a group split the touching cells, a fixed-order reduction over
// the group, then the far partial sums (all rows); times C.
constexpr int SF_G = 16;

template <int DIM, bool LOGK>
__global__ __launch_bounds__(256) void sf_near_kernel(SfDev D, const double* __restrict__ u,
                                                      const double* __restrict__ part, int nch,
                                                      const double* __restrict__ tab, double* __restrict__ Lu) {
    __shared__ double pw[768];
    if constexpr (!LOGK) load_tab(pw, tab);
    __syncthreads();
    const KPowTab P = tab_pow(pw, tab);
    const int g = threadIdx.x & (SF_G - 1);
    const long long t0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / SF_G;
    const bool live = t0 < D.nt;
    const long long t = live ? t0 : D.nt - 1;
    const long long K0 = t / D.Q;
    const int q = (int)(t - K0 * D.Q);
    const double x = D.tx[t], y = D.ty[t];
    double ux = 0.0;
    for (int a = 0; a <= DIM; ++a) ux = fma(D.lam[q * (DIM + 1) + a], uval(D, u, K0, a), ux);
    SfCell<DIM> c;
    double corr = 0.0;
    for (int e = D.nptr[K0] + g; e < D.nptr[K0 + 1]; e += SF_G) {
        const int K = D.nidx[e];
        load_cell<DIM>(D, u, K, c);
        const bool own = K == K0;
        for (int fi = 0; fi <= DIM; ++fi) {
            const SfFacet<DIM> f = facet_of<DIM>(c, fi);
            const double gN = fma(c.g[0], f.N[0], DIM == 2 ? c.g[DIM - 1] * f.N[1] : 0.0);
            double Igf, Iuf, Iof, Ign, Iun, Ion;
            facet_sums<DIM, LOGK>(f, x, y, D.qf, D.gx, D.gw, P, Igf, Iuf, Iof);
            facet_sums<DIM, LOGK>(f, x, y, D.qn, D.gx, D.gw, P, Ign, Iun, Ion);
            const double farv = D.cg * gN * Igf - D.inv2s * Iuf;
            const double nearv = own ? D.cg_own * gN * Ign - D.inv2s * ux * Ion : D.cg * gN * Ign - D.inv2s * Iun;
            corr += nearv - farv;
        }
    }
    // lanes g, g^8, g^4 ... of the group: a fixed butterfly order
#pragma unroll
    for (int m = SF_G / 2; m >= 1; m >>= 1) corr += __shfl_xor(corr, m, 64);
    if (g == 0 && live) {
        double acc = 0.0;
        for (int ch = 0; ch < nch; ++ch) acc += part[(long long)ch * D.nt + t];
        Lu[t] = D.C * (acc + corr);
    }
}

// eta_K^2 = h_K^{2s} sum_q W_q (f_q - Lu_q)^2 (f = 1 if null)
__global__ __launch_bounds__(256) void sf_ind_cell_kernel(long long T, int Q, const double* __restrict__ Lu,
                                                          const double* __restrict__ f,
                                                          const double* __restrict__ W,
                                                          const double* __restrict__ h2, double s,
                                                          double* __restrict__ eta) {
    const long long K = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= T) return;
    double acc = 0.0;
    for (int q = 0; q < Q; ++q) {
        const long long i = K * Q + q;
        const double r = (f ? f[i] : 1.0) - Lu[i];
        acc = fma(W[i] * r, r, acc);
    }
    eta[K] = pow(h2[K], s) * acc;
}

// eta_i^2 = sum of eta_K^2 over the cells containing vertex i (fixed order)
__global__ __launch_bounds__(256) void sf_ind_node_kernel(long long nv, const int* __restrict__ vptr,
                                                          const int* __restrict__ vidx,
                                                          const double* __restrict__ eta_c,
                                                          double* __restrict__ eta_n) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double acc = 0.0;
    for (int e = vptr[v]; e < vptr[v + 1]; ++e) acc += eta_c[vidx[e]];
    eta_n[v] = acc;
}


// ------------------------------------------------- cluster evaluation --

__device__ __forceinline__ double sfc_lag(const double* t, int m, int a, double xi) {
    double p = 1.0;
    for (int b = 0; b < m; ++b)
        if (b != a) p *= (xi - t[b]) / (t[a] - t[b]);
    return p;
}

// tensor Lagrange basis function a (first coordinate slowest) of cluster c
__device__ __forceinline__ double sfc_lag_box(const SfClDev& C, int c, int a, double x, double y) {
    const double* bx = C.box + 3 * c;
    const int a0 = a / C.m, a1 = a - a0 * C.m;
    return sfc_lag(C.tnode, C.m, a0, (x - bx[0]) / bx[2]) * sfc_lag(C.tnode, C.m, a1, (y - bx[1]) / bx[2]);
}

__device__ __forceinline__ void sfc_pt(const SfClDev& C, int c, int b, double& x, double& y) {
    const double* bx = C.box + 3 * c;
    const int b0 = b / C.m, b1 = b - b0 * C.m;
    x = bx[0] + bx[2] * C.tnode[b0];
    y = bx[1] + bx[2] * C.tnode[b1];
}

// T_c[b][a] = L_a^parent(xi_b^c), clusters c >= 1
__global__ __launch_bounds__(256) void sfc_transfer_kernel(SfClDev C) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long MM = (long long)C.M * C.M;
    if (id >= (long long)C.nc * MM) return;
    const int c = (int)(id / MM);
    if (c == 0) return;
    const int rem = (int)(id - (long long)c * MM);
    const int b = rem / C.M, a = rem - b * C.M;
    double x, y;
    sfc_pt(C, c, b, x, y);
    C.T[id] = sfc_lag_box(C, C.cpar[c], a, x, y);
}

// leaves: mom[c][b] = sum over the sources of the cells of c of w L_b(y)
__global__ __launch_bounds__(64) void sfc_mom_leaf_kernel(SfClDev C, SfDev D, const double* __restrict__ sx,
                                                          const double* __restrict__ sy) {
    const int c = C.leaf[blockIdx.x];
    for (int b = threadIdx.x; b < C.M; b += blockDim.x) {
        double acc = 0.0;
        for (int p = C.clo[c]; p < C.chi[c]; ++p)
            for (int e = C.optr[p]; e < C.optr[p + 1]; ++e) {
                const long long f = C.oidx[e];
                for (int j = 0; j < D.qf; ++j) {
                    const long long k = f * D.qf + j;
                    acc = fma(D.sc[k], sfc_lag_box(C, c, b, sx[k], sy[k]), acc);
                }
            }
        C.mom[(long long)c * C.M + b] = acc;
    }
}

// internal clusters of one level: mom[c][a] = sum_sons sum_b T_son[b][a] mom[son][b]
__global__ __launch_bounds__(64) void sfc_up_kernel(SfClDev C, const int4* __restrict__ list) {
    const int4 e = list[blockIdx.x];  // {c, son 0, son 1, -}
    const int c = e.x, M = C.M;
    if (M <= 64) {
        // both sons' shift coefficients in dynamic LDS (2 M^2 doubles), all
        // loads issued before the first product; son 0 is summed first
        extern __shared__ double sdyn[];
        const int a = threadIdx.x;
        const double* T0 = C.T + (long long)e.y * M * M;
        const double* T1 = C.T + (long long)e.z * M * M;
        for (int i = a; i < M * M; i += 64) {
            sdyn[i] = T0[i];
            sdyn[M * M + i] = T1[i];
        }
        const double m0 = a < M ? C.mom[(long long)e.y * M + a] : 0.0;
        const double m1 = a < M ? C.mom[(long long)e.z * M + a] : 0.0;
        __syncthreads();
        double acc = 0.0;
        for (int b = 0; b < M; ++b) {
            const double mb = __shfl(m0, b, 64);
            if (a < M) acc = fma(sdyn[b * M + a], mb, acc);
        }
        for (int b = 0; b < M; ++b) {
            const double mb = __shfl(m1, b, 64);
            if (a < M) acc = fma(sdyn[M * M + b * M + a], mb, acc);
        }
        if (a < M) C.mom[(long long)c * M + a] = acc;
        return;
    }
    for (int a = threadIdx.x; a < M; a += blockDim.x) {
        double acc = 0.0;
        for (int sn : {e.y, e.z}) {
            const double* Ts = C.T + (long long)sn * M * M;
            const double* ms = C.mom + (long long)sn * M;
            for (int b = 0; b < M; ++b) acc = fma(Ts[b * M + a], ms[b], acc);
        }
        C.mom[(long long)c * M + a] = acc;
    }
}

// far field: loc[s][a] = sum over admissible (s, t) of sum_b g(xi_a^s, xi_b^t)
// mom[t][b]; four lane groups over the pairs, added in group order
__global__ __launch_bounds__(256) void sfc_far_kernel(SfClDev C, const double* __restrict__ tab) {
    // the kernel power by the LDS tables of the direct far sum (same exponent)
    __shared__ __align__(16) double pw[768];
    load_tab(pw, tab);
    __syncthreads();
    const KPowTab P = tab_pow(pw, tab);
    __shared__ double red[4][64];
    const int c = blockIdx.x;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int a0 = 0; a0 < C.M; a0 += 64) {
        const int a = a0 + lane;
        double acc = 0.0;
        if (a < C.M) {
            double xa, ya;
            sfc_pt(C, c, a, xa, ya);
            for (long long p = C.fptr[c] + g; p < C.fptr[c + 1]; p += 4) {
                const int t = C.fdst[p];
                const double* mt = C.mom + (long long)t * C.M;
                for (int b = 0; b < C.M; ++b) {
                    double xb, yb;
                    sfc_pt(C, t, b, xb, yb);
                    const double dx = xa - xb, dy = ya - yb;
                    acc = fma(P(fma(dx, dx, dy * dy)), mt[b], acc);
                }
            }
        }
        red[g][lane] = acc;
        __syncthreads();
        if (g == 0 && a < C.M) C.loc[(long long)c * C.M + a] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        __syncthreads();
    }
}

// clusters of one level (>= 1): loc[c][b] += sum_a T_c[b][a] loc[parent][a]
__global__ __launch_bounds__(64) void sfc_down_kernel(SfClDev C, const int4* __restrict__ list) {
    const int4 e = list[blockIdx.x];  // {c, parent, -, -}
    const int c = e.x, M = C.M;
    const double* Tc = C.T + (long long)c * M * M;
    const double* lp = C.loc + (long long)e.y * M;
    if (M <= 64) {
        extern __shared__ double sdyn[];  // M^2 doubles of dynamic LDS
        const int b = threadIdx.x;
        for (int i = b; i < M * M; i += 64) sdyn[i] = Tc[i];
        const double lv = b < M ? lp[b] : 0.0;
        __syncthreads();
        double acc = 0.0;
        for (int a = 0; a < M; ++a) {
            const double la = __shfl(lv, a, 64);
            if (b < M) acc = fma(sdyn[b * M + a], la, acc);
        }
        if (b < M) C.loc[(long long)c * M + b] += acc;
        return;
    }
    for (int b = threadIdx.x; b < M; b += blockDim.x) {
        double acc = 0.0;
        for (int a = 0; a < M; ++a) acc = fma(Tc[b * M + a], lp[a], acc);
        C.loc[(long long)c * M + b] += acc;
    }
}

// leaves: every evaluation point of the leaf's cells adds its local
// expansion and the direct sums over the near leaves' sources to part0
__global__ __launch_bounds__(64) void sfc_leaf_eval_kernel(SfClDev C, SfDev D, const double* __restrict__ sx,
                                                           const double* __restrict__ sy,
                                                           const double* __restrict__ tab,
                                                           double* __restrict__ part0) {
    // the kernel power by the LDS tables of the direct far sum (same exponent)
    __shared__ __align__(16) double pw[768];
    load_tab(pw, tab);
    __syncthreads();
    const KPowTab P = tab_pow(pw, tab);
    const int li = blockIdx.x;
    const int c = C.leaf[li];
    const int np = (C.chi[c] - C.clo[c]) * D.Q;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int cell = C.perm[C.clo[c] + i / D.Q];
        const long long t = (long long)cell * D.Q + (i % D.Q);
        const double x = D.tx[t], y = D.ty[t];
        double acc = 0.0;
        for (int a = 0; a < C.M; ++a) acc = fma(sfc_lag_box(C, c, a, x, y), C.loc[(long long)c * C.M + a], acc);
        for (int e = C.lnptr[li]; e < C.lnptr[li + 1]; ++e) {
            const int tc = C.ndst[e];
            for (int p = C.clo[tc]; p < C.chi[tc]; ++p)
                for (int o = C.optr[p]; o < C.optr[p + 1]; ++o) {
                    const long long f = C.oidx[o];
                    for (int j = 0; j < D.qf; ++j) {
                        const long long k = f * D.qf + j;
                        const double dx = x - sx[k], dy = y - sy[k];
                        acc = fma(D.sc[k], P(fma(dx, dx, dy * dy)), acc);
                    }
                }
        }
        part0[t] += acc;
    }
}

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_sf_sources(const SfDev& D, const double* u, hipStream_t st) {
    if (D.nf > 0) {
        if (D.dim == 1)
            hipLaunchKernelGGL(sf_sources_kernel<1>, dim3(nblk(D.nf)), dim3(256), 0, st, D, u);
        else
            hipLaunchKernelGGL(sf_sources_kernel<2>, dim3(nblk(D.nf)), dim3(256), 0, st, D, u);
    }
    if (D.bnd_u && D.nbf > 0) {
        if (D.dim == 1)
            hipLaunchKernelGGL(sf_bsources_kernel<1>, dim3(nblk(D.nbf)), dim3(256), 0, st, D, u);
        else
            hipLaunchKernelGGL(sf_bsources_kernel<2>, dim3(nblk(D.nbf)), dim3(256), 0, st, D, u);
    }
}

void launch_sf_far(const SfDev& D, const double* sx, const double* sy, const double* bsx, const double* bsy,
                   long long chunk, int nch, int nchb, const double* tab, double* part, bool logk,
                   hipStream_t st) {
    if (D.nt == 0 || nch + nchb == 0) return;
    const dim3 grid((unsigned)((D.nt + 256 * SF_TPT - 1) / (256 * SF_TPT)), (unsigned)(nch + nchb));
    const long long nbs = nchb > 0 ? D.nbs : 0;
    if (logk)
        hipLaunchKernelGGL(sf_far_kernel<true>, grid, dim3(256), 0, st, D.nt, D.tx, D.ty, D.ns, sx, sy, D.sc,
                           chunk, nch, nbs, bsx, bsy, D.bc, tab, part);
    else
        hipLaunchKernelGGL(sf_far_kernel<false>, grid, dim3(256), 0, st, D.nt, D.tx, D.ty, D.ns, sx, sy, D.sc,
                           chunk, nch, nbs, bsx, bsy, D.bc, tab, part);
}

void launch_sf_near(const SfDev& D, const double* u, const double* part, int nch, const double* tab,
                    double* Lu, bool logk, hipStream_t st) {
    if (D.nt == 0) return;
    const dim3 grid(nblk(D.nt * SF_G));
    if (D.dim == 1) {
        if (logk)
            hipLaunchKernelGGL((sf_near_kernel<1, true>), grid, dim3(256), 0, st, D, u, part, nch, tab, Lu);
        else
            hipLaunchKernelGGL((sf_near_kernel<1, false>), grid, dim3(256), 0, st, D, u, part, nch, tab, Lu);
    } else {
        hipLaunchKernelGGL((sf_near_kernel<2, false>), grid, dim3(256), 0, st, D, u, part, nch, tab, Lu);
    }
}

void launch_sf_indicators(const SfDev& D, const double* Lu, const double* f, const double* W,
                          const double* h2, double s, long long nv, const int* vptr, const int* vidx,
                          double* eta_cell, double* eta_node, hipStream_t st) {
    if (D.T == 0) return;
    hipLaunchKernelGGL(sf_ind_cell_kernel, dim3(nblk(D.T)), dim3(256), 0, st, D.T, D.Q, Lu, f, W, h2, s,
                       eta_cell);
    if (eta_node && nv > 0)
        hipLaunchKernelGGL(sf_ind_node_kernel, dim3(nblk(nv)), dim3(256), 0, st, nv, vptr, vidx, eta_cell,
                           eta_node);
}

void launch_sfc_transfer(const SfClDev& C, hipStream_t st) {
    if (C.nc > 1)
        hipLaunchKernelGGL(sfc_transfer_kernel, dim3(nblk((long long)C.nc * C.M * C.M)), dim3(256), 0, st, C);
}

void launch_sfc_eval(const SfClDev& C, const SfDev& D, const double* sx, const double* sy,
                     const int* const* up_lists, const int* up_counts, int n_up, const int* const* down_lists,
                     const int* down_counts, int n_down, const double* tab, double* part0, hipStream_t st) {
    if (C.nc == 0) return;
    hipLaunchKernelGGL(sfc_mom_leaf_kernel, dim3((unsigned)C.nleaf), dim3(64), 0, st, C, D, sx, sy);
    // four ints per list entry (device allocations: 256-byte aligned)
    const size_t lds = C.M <= 64 ? sizeof(double) * C.M * C.M : 0;
    for (int l = 0; l < n_up; ++l)
        if (up_counts[l] > 0)
            hipLaunchKernelGGL(sfc_up_kernel, dim3((unsigned)up_counts[l]), dim3(64), 2 * lds, st, C,
                               (const int4*)up_lists[l]);
    hipLaunchKernelGGL(sfc_far_kernel, dim3((unsigned)C.nc), dim3(256), 0, st, C, tab);
    for (int l = 0; l < n_down; ++l)
        if (down_counts[l] > 0)
            hipLaunchKernelGGL(sfc_down_kernel, dim3((unsigned)down_counts[l]), dim3(64), lds, st, C,
                               (const int4*)down_lists[l]);
    hipLaunchKernelGGL(sfc_leaf_eval_kernel, dim3((unsigned)C.nleaf), dim3(64), 0, st, C, D, sx, sy, tab, part0);
}

}  // namespace fl
