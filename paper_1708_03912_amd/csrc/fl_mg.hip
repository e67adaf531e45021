// Geometric multigrid on nested meshes (Sec. 5: multigrid as the solver
// whose iteration count stays bounded under refinement): transfer
// operators, Galerkin coarse operators, the coarsest-level inverse and the
// vector kernels of MG-preconditioned CG.  The cycle itself (damped Jacobi
// smoothing through the symmetric product) is driven by fl_mg_api.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fl_internal.hpp"

namespace fl {

namespace {

__global__ void mg_scale_kernel(double* x, const double* b, const double* d, double omega, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = omega * b[i] / d[i];
}

// Jacobi step from a product y = A x computed elsewhere (the cluster
// product): x += omega (b - y) / d (mode 0) or the residual r = b - y (mode 1)
__global__ void mg_jacobi_kernel(double* x, const double* b, const double* y, const double* d, double omega,
                                 int mode, double* r, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mode == 0) x[i] += omega * (b[i] - y[i]) / d[i];
    else r[i] = b[i] - y[i];
}

// one thread per coarse DOF, children in a fixed order
__global__ void mg_restrict_kernel(long long nc, const int* cptr, const int* cidx, const double* cw,
                                   const double* rf, double* bc) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double s = 0.0;
    for (int e = cptr[c]; e < cptr[c + 1]; ++e) s += cw[e] * rf[cidx[e]];
    bc[c] = s;
}

// one thread per fine DOF; a missing parent has index -1 and weight 0
__global__ void mg_prolong_add_kernel(long long nf, const int2* par, const double2* pw, const double* xc,
                                      double* xf) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int2 p = par[i];
    const double2 w = pw[i];
    double s = 0.0;
    if (p.x >= 0) s += w.x * xc[p.x];
    if (p.y >= 0) s += w.y * xc[p.y];
    xf[i] += s;
}

// B[i][c] = sum_e w_e A[i][f_e]: one thread per (i, c), c fastest; a row of
// A is reused by the whole block from the caches
__global__ void mg_gal_cols_kernel(const double* __restrict__ A, long long lda, long long nf, long long nc,
                                   const int* __restrict__ cptr, const int* __restrict__ cidx,
                                   const double* __restrict__ cw, double* __restrict__ B, long long ldb) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    for (long long i = blockIdx.y; i < nf; i += gridDim.y) {
        const double* row = A + i * lda;
        double s = 0.0;
        for (int e = cptr[c]; e < cptr[c + 1]; ++e) s += cw[e] * row[cidx[e]];
        B[i * ldb + c] = s;
    }
}

// Ac[c][d] = sum_e w_e B[f_e][d]: one thread per (c, d), d fastest (rows of
// B read coalesced)
__global__ void mg_gal_rows_kernel(const double* __restrict__ B, long long ldb, long long nc,
                                   const int* __restrict__ cptr, const int* __restrict__ cidx,
                                   const double* __restrict__ cw, double* __restrict__ Ac, long long ldc) {
    const long long dcol = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (dcol >= nc) return;
    for (long long c = blockIdx.y; c < nc; c += gridDim.y) {
        double s = 0.0;
        for (int e = cptr[c]; e < cptr[c + 1]; ++e) s += cw[e] * B[(long long)cidx[e] * ldb + dcol];
        Ac[c * ldc + dcol] = s;
    }
}

// In-place Gauss-Jordan inversion without pivoting (SPD input), one
// workgroup: for each k the pivot row is scaled, then every other row i
// eliminates column k with its own factor a_ik (rows split over threads).
__global__ __launch_bounds__(256) void mg_invert_kernel(double* M, long long n, long long ld, int* flag) {
    __shared__ double piv;
    for (long long k = 0; k < n; ++k) {
        double* rk = M + k * ld;
        if (threadIdx.x == 0) {
            piv = rk[k];
            if (!(piv > 0.0)) flag[0] = 1;
        }
        __syncthreads();
        const double ip = 1.0 / piv;
        for (long long j = threadIdx.x; j < n; j += blockDim.x) rk[j] = (j == k) ? ip : rk[j] * ip;
        __syncthreads();
        for (long long i = threadIdx.x; i < n; i += blockDim.x) {
            if (i == k) continue;
            double* ri = M + i * ld;
            const double f = ri[k];
            ri[k] = 0.0;
            for (long long j = 0; j < n; ++j) ri[j] -= f * rk[j];
        }
        __syncthreads();
    }
}

__global__ void mg_axpy_kernel(double* x, double* r, const double* p, const double* q, long long n,
                               const double* sc, int ia, int ib) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = sc[ia] / sc[ib];
    x[i] += a * p[i];
    r[i] -= a * q[i];
}

__global__ void mg_pupdate_kernel(double* p, const double* z, long long n, const double* sc, int ia, int ib) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = z[i] + (sc[ia] / sc[ib]) * p[i];
}

inline dim3 grid1(long long n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

void launch_mg_scale(double* x, const double* b, const double* d, double omega, long long n, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(mg_scale_kernel, grid1(n), dim3(256), 0, st, x, b, d, omega, n);
}

void launch_mg_jacobi(double* x, const double* b, const double* y, const double* d, double omega, int mode,
                      double* r, long long n, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(mg_jacobi_kernel, grid1(n), dim3(256), 0, st, x, b, y, d, omega, mode, r, n);
}

void launch_mg_restrict(long long nc, const int* cptr, const int* cidx, const double* cw, const double* rf,
                        double* bc, hipStream_t st) {
    if (nc == 0) return;
    hipLaunchKernelGGL(mg_restrict_kernel, grid1(nc), dim3(256), 0, st, nc, cptr, cidx, cw, rf, bc);
}

void launch_mg_prolong_add(long long nf, const int2* par, const double2* pw, const double* xc, double* xf,
                           hipStream_t st) {
    if (nf == 0) return;
    hipLaunchKernelGGL(mg_prolong_add_kernel, grid1(nf), dim3(256), 0, st, nf, par, pw, xc, xf);
}

void launch_mg_galerkin(const double* A, long long lda, long long nf, long long nc, const int* cptr,
                        const int* cidx, const double* cw, double* B, long long ldb, double* Ac, long long ldc,
                        hipStream_t st) {
    if (nf == 0 || nc == 0) return;
    const unsigned gx = (unsigned)((nc + 255) / 256);
    hipLaunchKernelGGL(mg_gal_cols_kernel, dim3(gx, (unsigned)std::min<long long>(nf, 32768)), dim3(256), 0, st, A,
                       lda, nf, nc, cptr, cidx, cw, B, ldb);
    hipLaunchKernelGGL(mg_gal_rows_kernel, dim3(gx, (unsigned)std::min<long long>(nc, 32768)), dim3(256), 0, st, B,
                       ldb, nc, cptr, cidx, cw, Ac, ldc);
}

void launch_mg_invert(double* M, long long n, long long ld, int* flag, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(mg_invert_kernel, dim3(1), dim3(256), 0, st, M, n, ld, flag);
}

void launch_mg_axpy(double* x, double* r, const double* p, const double* q, long long n, const double* sc, int ia,
                    int ib, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(mg_axpy_kernel, grid1(n), dim3(256), 0, st, x, r, p, q, n, sc, ia, ib);
}

void launch_mg_pupdate(double* p, const double* z, long long n, const double* sc, int ia, int ib, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(mg_pupdate_kernel, grid1(n), dim3(256), 0, st, p, z, n, sc, ia, ib);
}

}  // namespace fl
