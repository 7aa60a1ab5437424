// Host check of the library's small dense linear algebra (run by
// tests/test_linalg.py): Givens rotations, LU solves, the Jacobi Hermitian
// eigensolver, the Hessenberg-QR general eigensolver, the Cholesky factor
// and the triangular inverse, checked by their residuals, orthonormality and
// known spectra.
#include <cstdio>
#include <random>

#include "../paper_1202_2462_amd/csrc/linalg.h"

using namespace mgdd::la;

static Mat rnd(int n, unsigned seed, double diag = 0.0) {
    std::mt19937_64 g(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    Mat A((size_t)n * n);
    for (auto &v : A) v = cd(nd(g), nd(g));
    for (int i = 0; i < n; i++) A[i * n + i] += diag;
    return A;
}

static double nrm(const Mat &A) {
    double s = 0;
    for (auto &v : A) s += std::norm(v);
    return std::sqrt(s);
}

int main() {
    int bad = 0;
    // Givens
    for (int t = 0; t < 20; t++) {
        Mat v = rnd(2, 100 + t);
        double c;
        cd s, rho;
        givens(v[0], v[1], c, s, rho);
        cd r0 = c * v[0] + s * v[1], r1 = -std::conj(s) * v[0] + c * v[1];
        if (std::abs(r1) > 1e-14 || std::abs(r0 - rho) > 1e-14 || std::fabs(c * c + std::norm(s) - 1) > 1e-14) bad++;
    }
    // LU
    for (int n : {1, 5, 17}) {
        Mat A = rnd(n, 7 + n, 3.0);
        std::vector<cd> b(n), x;
        for (int i = 0; i < n; i++) b[i] = cd(i + 1, -i);
        x = b;
        lu_solve(n, A, x);
        double r = 0;
        for (int i = 0; i < n; i++) {
            cd s = -b[i];
            for (int j = 0; j < n; j++) s += A[i * n + j] * x[j];
            r += std::norm(s);
        }
        if (std::sqrt(r) > 1e-12) { printf("lu residual %g\n", std::sqrt(r)); bad++; }
    }
    // Hermitian eigenproblem
    for (int n : {1, 2, 8, 48}) {
        Mat B = rnd(n, 11 + n), A((size_t)n * n);
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) A[i * n + j] = B[i * n + j] + std::conj(B[j * n + i]);
        std::vector<double> w;
        Mat Z;
        eigh(n, A, w, Z);
        double an = nrm(A);
        for (int k = 0; k < n; k++) {
            if (k && w[k] < w[k - 1]) bad++;
            double r = 0;
            for (int i = 0; i < n; i++) {
                cd s = -w[k] * Z[i * n + k];
                for (int j = 0; j < n; j++) s += A[i * n + j] * Z[j * n + k];
                r += std::norm(s);
            }
            if (std::sqrt(r) > 1e-12 * an) { printf("eigh residual n=%d %g\n", n, std::sqrt(r)); bad++; }
            for (int l = 0; l < n; l++) {
                cd g = 0;
                for (int i = 0; i < n; i++) g += std::conj(Z[i * n + k]) * Z[i * n + l];
                if (std::abs(g - (k == l ? 1.0 : 0.0)) > 1e-12) { printf("eigh orthonormality\n"); bad++; }
            }
        }
    }
    // general eigenproblem
    for (int n : {1, 2, 3, 10, 50, 64}) {
        Mat A = rnd(n, 23 + n);
        std::vector<cd> lam;
        Mat X;
        if (!eig(n, A, lam, X)) { printf("eig did not converge n=%d\n", n); bad++; continue; }
        double an = nrm(A);
        cd tr = 0, sl = 0;
        for (int i = 0; i < n; i++) { tr += A[i * n + i]; sl += lam[i]; }
        if (std::abs(tr - sl) > 1e-10 * an) { printf("eig trace n=%d\n", n); bad++; }
        for (int k = 0; k < n; k++) {
            double r = 0;
            for (int i = 0; i < n; i++) {
                cd s = -lam[k] * X[i * n + k];
                for (int j = 0; j < n; j++) s += A[i * n + j] * X[j * n + k];
                r += std::norm(s);
            }
            if (std::sqrt(r) > 1e-9 * an) { printf("eig residual n=%d k=%d %g\n", n, k, std::sqrt(r)); bad++; }
        }
    }
    // triangular matrix: eigenvalues are its diagonal
    {
        int n = 6;
        Mat A = rnd(n, 5);
        for (int i = 0; i < n; i++)
            for (int j = 0; j < i; j++) A[i * n + j] = 0.0;
        std::vector<cd> lam;
        Mat X;
        eig(n, A, lam, X);
        for (int i = 0; i < n; i++) {
            double best = 1e300;
            for (int j = 0; j < n; j++) best = std::min(best, std::abs(lam[j] - A[i * n + i]));
            if (best > 1e-12) { printf("triangular spectrum\n"); bad++; }
        }
    }
    // Cholesky and triangular inverse: G = B^H B + 1, R^H R = G, R upper with
    // a positive diagonal, R R^{-1} = 1; an indefinite matrix is rejected
    for (int n : {1, 3, 20, 40}) {
        Mat B = rnd(n, 31 + n), G((size_t)n * n, 0.0), R;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                for (int k = 0; k < n; k++) G[i * n + j] += std::conj(B[k * n + i]) * B[k * n + j];
                if (i == j) G[i * n + j] += 1.0;
            }
        if (!cholesky_upper(n, G, R)) { printf("cholesky rejected a definite matrix n=%d\n", n); bad++; continue; }
        double gn = nrm(G), err = 0, ierr = 0;
        for (int i = 0; i < n; i++) {
            if (R[i * n + i].imag() != 0.0 || R[i * n + i].real() <= 0.0) bad++;
            for (int j = 0; j < i; j++)
                if (R[i * n + j] != 0.0) bad++;
            for (int j = 0; j < n; j++) {
                cd sum = -G[i * n + j];
                for (int k = 0; k < n; k++) sum += std::conj(R[k * n + i]) * R[k * n + j];
                err += std::norm(sum);
            }
        }
        Mat Ri = upper_inverse(n, R);
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                cd sum = i == j ? -1.0 : 0.0;
                for (int k = 0; k < n; k++) sum += R[i * n + k] * Ri[k * n + j];
                ierr += std::norm(sum);
            }
        if (std::sqrt(err) > 1e-12 * gn || std::sqrt(ierr) > 1e-10) { printf("cholesky n=%d %g %g\n", n, err, ierr); bad++; }
    }
    {
        Mat G = {cd(1, 0), cd(2, 0), cd(2, 0), cd(1, 0)}, R;   // eigenvalues 3 and -1
        if (cholesky_upper(2, G, R)) { printf("cholesky accepted an indefinite matrix\n"); bad++; }
    }
    printf(bad ? "LINALG FAILED %d\n" : "LINALG OK\n", bad);
    return bad ? 1 : 0;
}
