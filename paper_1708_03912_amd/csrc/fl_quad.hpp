// Gauss-type quadrature rules generated on the host for the device tables.
//
// Gauss-Jacobi rules for the weight (1-x)^alpha (1+x)^beta on [-1,1] are
// computed with the Golub-Welsch method: the nodes are the eigenvalues of the
// symmetric tridiagonal Jacobi matrix of the monic three-term recurrence, the
// weights mu0 * v_0^2 from the normalised eigenvectors.  The eigenproblem is
// solved with cyclic Jacobi rotations (k <= 32, dense), and every node is then
// polished by Newton steps on the recurrence.  Rules are returned on [0,1]
// (x -> (1+x)/2, weights scaled by 2^{-(alpha+beta+1)}).
#pragma once

#include <cmath>
#include <vector>

namespace fl {

inline void jacobi_recurrence(int k, double a, double b, std::vector<double>& diag,
                              std::vector<double>& off2) {
    diag.assign(k, 0.0);
    off2.assign(k, 0.0);
    for (int n = 0; n < k; ++n) {
        double s = 2.0 * n + a + b;
        if (n == 0)
            diag[n] = (b - a) / (a + b + 2.0);
        else
            diag[n] = (b * b - a * a) / (s * (s + 2.0));
        if (n >= 1) {
            double nn = n;
            off2[n] = 4.0 * nn * (nn + a) * (nn + b) * (nn + a + b) / (s * s * (s + 1.0) * (s - 1.0));
        }
    }
}

// monic Jacobi polynomial p_k, its derivative and p_{k-1} at x
inline void jacobi_eval(int k, const std::vector<double>& diag, const std::vector<double>& off2,
                        double x, double& p, double& dp, double& pkm1) {
    double pm1 = 0.0, p0 = 1.0, dpm1 = 0.0, dp0 = 0.0;
    for (int n = 0; n < k; ++n) {
        double p1 = (x - diag[n]) * p0 - (n >= 1 ? off2[n] * pm1 : 0.0);
        double dp1 = p0 + (x - diag[n]) * dp0 - (n >= 1 ? off2[n] * dpm1 : 0.0);
        pm1 = p0; p0 = p1; dpm1 = dp0; dp0 = dp1;
    }
    p = p0;
    dp = dp0;
    pkm1 = pm1;
}

// k-point rule for int_0^1 (1-u)^alpha u^beta f(u) du; alpha, beta > -1.
inline void gauss_jacobi01(int k, double alpha, double beta, double* x01, double* w01) {
    std::vector<double> diag, off2;
    jacobi_recurrence(k, alpha, beta, diag, off2);
    // dense symmetric tridiagonal matrix
    std::vector<double> M(k * k, 0.0), V(k * k, 0.0);
    for (int i = 0; i < k; ++i) {
        M[i * k + i] = diag[i];
        if (i + 1 < k) M[i * k + i + 1] = M[(i + 1) * k + i] = std::sqrt(off2[i + 1]);
        V[i * k + i] = 1.0;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double offn = 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) offn += M[p * k + q] * M[p * k + q];
        if (offn < 1e-34) break;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                double apq = M[p * k + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = M[p * k + p], aqq = M[q * k + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < k; ++r) {
                    double mrp = M[r * k + p], mrq = M[r * k + q];
                    M[r * k + p] = c * mrp - s * mrq;
                    M[r * k + q] = s * mrp + c * mrq;
                }
                for (int r = 0; r < k; ++r) {
                    double mpr = M[p * k + r], mqr = M[q * k + r];
                    M[p * k + r] = c * mpr - s * mqr;
                    M[q * k + r] = s * mpr + c * mqr;
                }
                for (int r = 0; r < k; ++r) {
                    double vrp = V[r * k + p], vrq = V[r * k + q];
                    V[r * k + p] = c * vrp - s * vrq;
                    V[r * k + q] = s * vrp + c * vrq;
                }
            }
    }
    double mu0 = std::pow(2.0, alpha + beta + 1.0) * std::tgamma(alpha + 1.0) * std::tgamma(beta + 1.0) /
                 std::tgamma(alpha + beta + 2.0);
    // squared norm of p_{k-1}: mu0 * prod_{n=1}^{k-1} off2[n]
    double hk1 = mu0;
    for (int n = 1; n < k; ++n) hk1 *= off2[n];
    std::vector<double> x(k), w(k);
    for (int i = 0; i < k; ++i) {
        double xi = M[i * k + i];
        double p = 0.0, dp = 0.0, pk1 = 0.0;
        for (int it = 0; it < 6; ++it) {
            jacobi_eval(k, diag, off2, xi, p, dp, pk1);
            if (dp == 0.0) break;
            double dx = p / dp;
            xi -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        jacobi_eval(k, diag, off2, xi, p, dp, pk1);
        x[i] = xi;
        // Christoffel numbers of a monic orthogonal family
        w[i] = (k == 1) ? mu0 : hk1 / (pk1 * dp);
    }
    // sort ascending
    for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j)
            if (x[j] < x[i]) { std::swap(x[i], x[j]); std::swap(w[i], w[j]); }
    double scale = std::pow(0.5, alpha + beta + 1.0);
    for (int i = 0; i < k; ++i) {
        x01[i] = 0.5 * (x[i] + 1.0);
        w01[i] = w[i] * scale;
    }
}

}  // namespace fl
