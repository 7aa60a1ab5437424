// Small dense complex linear algebra on the host: Givens rotations for the
// Krylov least-squares problems, a cyclic Jacobi eigensolver for Hermitian
// matrices, a Hessenberg + shifted-QR eigensolver for general complex
// matrices, and LU solves. Matrices are row-major std::vector<cd>.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace mgdd {
namespace la {

using cd = std::complex<double>;
using Mat = std::vector<cd>;

// rotation G = [[c, s], [-conj(s), c]] (c real) with G [a; b] = [rho; 0]
inline void givens(cd a, cd b, double &c, cd &s, cd &rho) {
    double aa = std::abs(a), bb = std::abs(b);
    if (bb == 0.0) { c = 1.0; s = 0.0; rho = a; return; }
    if (aa == 0.0) { c = 0.0; s = 1.0; rho = b; return; }
    double r = std::hypot(aa, bb);
    c = aa / r;
    s = (a / aa) * std::conj(b) / r;
    rho = (a / aa) * r;
}

// Cholesky factor of a Hermitian positive definite G (n x n, row-major):
// G = R^H R with R upper triangular and a positive real diagonal; false when
// a pivot is not positive (then R is incomplete).
inline bool cholesky_upper(int n, const Mat &G, Mat &R) {
    R.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) {
        double d = G[(size_t)i * n + i].real();
        for (int k = 0; k < i; k++) d -= std::norm(R[(size_t)k * n + i]);
        if (!(d > 0.0)) return false;
        const double rii = std::sqrt(d);
        R[(size_t)i * n + i] = rii;
        for (int j = i + 1; j < n; j++) {
            cd sum = G[(size_t)i * n + j];
            for (int k = 0; k < i; k++) sum -= std::conj(R[(size_t)k * n + i]) * R[(size_t)k * n + j];
            R[(size_t)i * n + j] = sum / rii;
        }
    }
    return true;
}

// Inverse of an upper triangular R (n x n, row-major), by back substitution.
inline Mat upper_inverse(int n, const Mat &R) {
    Mat X((size_t)n * n, 0.0);
    for (int j = 0; j < n; j++) {
        X[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
        for (int i = j - 1; i >= 0; i--) {
            cd sum = 0.0;
            for (int k = i + 1; k <= j; k++) sum += R[(size_t)i * n + k] * X[(size_t)k * n + j];
            X[(size_t)i * n + j] = -sum / R[(size_t)i * n + i];
        }
    }
    return X;
}

// Solves A x = b (n x n, row-major) by LU with partial pivoting; false if singular.
inline bool lu_solve(int n, Mat A, std::vector<cd> &b) {
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int i = k + 1; i < n; i++)
            if (std::abs(A[i * n + k]) > std::abs(A[p * n + k])) p = i;
        if (A[p * n + k] == 0.0) return false;
        if (p != k) {
            for (int j = 0; j < n; j++) std::swap(A[k * n + j], A[p * n + j]);
            std::swap(b[k], b[p]);
        }
        for (int i = k + 1; i < n; i++) {
            cd f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; j++) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        cd s = b[i];
        for (int j = i + 1; j < n; j++) s -= A[i * n + j] * b[j];
        b[i] = s / A[i * n + i];
    }
    return true;
}

// Hermitian eigenproblem by cyclic Jacobi rotations. Eigenvalues ascending in
// w, eigenvectors in the columns of Z (row-major n x n).
inline void eigh(int n, Mat A, std::vector<double> &w, Mat &Z) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) Z[i * n + i] = 1.0;
    double fro = 0;
    for (auto &v : A) fro += std::norm(v);
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += std::norm(A[p * n + q]);
        if (std::sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                cd apq = A[p * n + q];
                double m = std::abs(apq);
                if (m <= 1e-300) continue;
                cd ph = apq / m;  // e^{i phi}
                double app = A[p * n + p].real(), aqq = A[q * n + q].real();
                double th = (aqq - app) / (2 * m);
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
                double c = 1 / std::sqrt(t * t + 1), s = t * c;
                // Q = diag(1, conj(ph)) [[c, s], [-s, c]] on rows/cols p, q
                cd Qpp = c, Qpq = s, Qqp = -s * std::conj(ph), Qqq = c * std::conj(ph);
                for (int k = 0; k < n; k++) {  // A <- A Q
                    cd ap = A[k * n + p], aq = A[k * n + q];
                    A[k * n + p] = ap * Qpp + aq * Qqp;
                    A[k * n + q] = ap * Qpq + aq * Qqq;
                }
                for (int k = 0; k < n; k++) {  // A <- Q^H A
                    cd ap = A[p * n + k], aq = A[q * n + k];
                    A[p * n + k] = std::conj(Qpp) * ap + std::conj(Qqp) * aq;
                    A[q * n + k] = std::conj(Qpq) * ap + std::conj(Qqq) * aq;
                }
                A[p * n + q] = A[q * n + p] = 0.0;
                A[p * n + p] = A[p * n + p].real();
                A[q * n + q] = A[q * n + q].real();
                for (int k = 0; k < n; k++) {  // Z <- Z Q
                    cd zp = Z[k * n + p], zq = Z[k * n + q];
                    Z[k * n + p] = zp * Qpp + zq * Qqp;
                    Z[k * n + q] = zp * Qpq + zq * Qqq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; i++) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * n + a].real() < A[b * n + b].real(); });
    w.resize(n);
    Mat Zs((size_t)n * n);
    for (int j = 0; j < n; j++) {
        w[j] = A[idx[j] * n + idx[j]].real();
        for (int k = 0; k < n; k++) Zs[k * n + j] = Z[k * n + idx[j]];
    }
    Z.swap(Zs);
}

// General complex eigenproblem: Householder reduction to Hessenberg form,
// single-shift QR iterations (Wilkinson shift) to the Schur form T = Q^H A Q,
// eigenvectors by back substitution on T. Eigenvalues in lam, unit
// eigenvectors in the columns of X. Returns false if the QR iteration did not
// converge.
inline bool eig(int n, Mat A, std::vector<cd> &lam, Mat &X) {
    Mat Q((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) Q[i * n + i] = 1.0;
    // Hessenberg reduction
    for (int k = 0; k + 2 < n; k++) {
        std::vector<cd> v(n, 0.0);
        double xn = 0;
        for (int i = k + 1; i < n; i++) xn += std::norm(A[i * n + k]);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        cd x0 = A[(k + 1) * n + k];
        cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
        for (int i = k + 1; i < n; i++) v[i] = A[i * n + k];
        v[k + 1] += ph * xn;
        double vn = 0;
        for (int i = k + 1; i < n; i++) vn += std::norm(v[i]);
        if (vn == 0.0) continue;
        // A <- H A, H = I - 2 v v^H / (v^H v)
        for (int j = 0; j < n; j++) {
            cd s = 0;
            for (int i = k + 1; i < n; i++) s += std::conj(v[i]) * A[i * n + j];
            s *= 2.0 / vn;
            for (int i = k + 1; i < n; i++) A[i * n + j] -= v[i] * s;
        }
        // A <- A H, Q <- Q H
        for (int i = 0; i < n; i++) {
            cd s = 0, t = 0;
            for (int j = k + 1; j < n; j++) { s += A[i * n + j] * v[j]; t += Q[i * n + j] * v[j]; }
            s *= 2.0 / vn;
            t *= 2.0 / vn;
            for (int j = k + 1; j < n; j++) { A[i * n + j] -= s * std::conj(v[j]); Q[i * n + j] -= t * std::conj(v[j]); }
        }
        for (int i = k + 2; i < n; i++) A[i * n + k] = 0.0;
    }
    // shifted QR on the Hessenberg matrix
    int hi = n - 1, iter = 0;
    while (hi > 0) {
        if (iter++ > 100 * n) return false;
        int lo = hi;
        while (lo > 0) {
            double s = std::abs(A[(lo - 1) * n + lo - 1]) + std::abs(A[lo * n + lo]);
            if (s == 0.0) s = 1.0;
            if (std::abs(A[lo * n + lo - 1]) <= 1e-16 * s) { A[lo * n + lo - 1] = 0.0; break; }
            lo--;
        }
        if (lo == hi) { hi--; iter = 0; continue; }
        // Wilkinson shift from the trailing 2x2 of the active window
        cd a = A[(hi - 1) * n + hi - 1], b = A[(hi - 1) * n + hi], c = A[hi * n + hi - 1], d = A[hi * n + hi];
        cd tr = a + d, det = a * d - b * c;
        cd disc = std::sqrt(tr * tr / 4.0 - det);
        cd m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
        cd mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        if (iter % 11 == 10) mu = d + cd(std::abs(A[hi * n + hi - 1]), 0.0);  // exceptional shift
        // QR step on rows/cols lo..hi by Givens rotations
        std::vector<double> cs(hi - lo);
        std::vector<cd> ss(hi - lo);
        for (int k = lo; k <= hi; k++) A[k * n + k] -= mu;
        for (int k = lo; k < hi; k++) {
            double cc;
            cd s, rho;
            givens(A[k * n + k], A[(k + 1) * n + k], cc, s, rho);
            cs[k - lo] = cc;
            ss[k - lo] = s;
            for (int j = k; j < n; j++) {
                cd x = A[k * n + j], y = A[(k + 1) * n + j];
                A[k * n + j] = cc * x + s * y;
                A[(k + 1) * n + j] = -std::conj(s) * x + cc * y;
            }
        }
        for (int k = lo; k < hi; k++) {
            double cc = cs[k - lo];
            cd s = ss[k - lo];
            int top = std::min(k + 2, hi);
            for (int i = 0; i <= top; i++) {
                cd x = A[i * n + k], y = A[i * n + k + 1];
                A[i * n + k] = cc * x + std::conj(s) * y;
                A[i * n + k + 1] = -s * x + cc * y;
            }
            for (int i = 0; i < n; i++) {
                cd x = Q[i * n + k], y = Q[i * n + k + 1];
                Q[i * n + k] = cc * x + std::conj(s) * y;
                Q[i * n + k + 1] = -s * x + cc * y;
            }
        }
        for (int k = lo; k <= hi; k++) A[k * n + k] += mu;
    }
    lam.resize(n);
    for (int i = 0; i < n; i++) lam[i] = A[i * n + i];
    // eigenvectors of the triangular T, then back to the original basis
    X.assign((size_t)n * n, 0.0);
    double tnorm = 0;
    for (auto &v : A) tnorm = std::max(tnorm, std::abs(v));
    for (int i = 0; i < n; i++) {
        std::vector<cd> y(n, 0.0);
        y[i] = 1.0;
        for (int j = i - 1; j >= 0; j--) {
            cd s = 0;
            for (int k = j + 1; k <= i; k++) s += A[j * n + k] * y[k];
            cd den = A[j * n + j] - lam[i];
            if (std::abs(den) < 1e-14 * tnorm) den = 1e-14 * tnorm;
            y[j] = -s / den;
        }
        double nn = 0;
        std::vector<cd> x(n, 0.0);
        for (int r = 0; r < n; r++) {
            for (int k = 0; k <= i; k++) x[r] += Q[r * n + k] * y[k];
            nn += std::norm(x[r]);
        }
        nn = std::sqrt(nn);
        for (int r = 0; r < n; r++) X[r * n + i] = x[r] / nn;
    }
    return true;
}

}  // namespace la
}  // namespace mgdd
