// Small dense complex FP64 linear algebra on the host (Rayleigh-Ritz step of
// the eigensolver): Cholesky factor, triangular inverse, and a cyclic Jacobi
// eigensolver for Hermitian matrices.  Matrices are row-major m x m arrays of
// std::complex<double>.
#pragma once
#include <cmath>
#include <complex>
#include <vector>

namespace dense {
typedef std::complex<double> zc;

// A = R^H R with R upper triangular; returns false if A is not positive definite.
inline bool cholesky_upper(const zc* A, zc* R, int m) {
    for (int i = 0; i < m * m; i++) R[i] = 0;
    for (int j = 0; j < m; j++) {
        double d = std::real(A[j * m + j]);
        for (int k = 0; k < j; k++) d -= std::norm(R[k * m + j]);
        if (!(d > 0)) return false;
        double rjj = std::sqrt(d);
        R[j * m + j] = rjj;
        for (int i = j + 1; i < m; i++) {
            zc s = A[j * m + i];
            for (int k = 0; k < j; k++) s -= std::conj(R[k * m + j]) * R[k * m + i];
            R[j * m + i] = s / rjj;
        }
    }
    return true;
}

// inverse of an upper-triangular matrix
inline void inv_upper(const zc* R, zc* Ri, int m) {
    for (int i = 0; i < m * m; i++) Ri[i] = 0;
    for (int j = 0; j < m; j++) {
        Ri[j * m + j] = 1.0 / R[j * m + j];
        for (int i = j - 1; i >= 0; i--) {
            zc s = 0;
            for (int k = i + 1; k <= j; k++) s += R[i * m + k] * Ri[k * m + j];
            Ri[i * m + j] = -s / R[i * m + i];
        }
    }
}

// C = A B (m x m)
inline void matmul(const zc* A, const zc* B, zc* C, int m) {
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) {
            zc s = 0;
            for (int k = 0; k < m; k++) s += A[i * m + k] * B[k * m + j];
            C[i * m + j] = s;
        }
}

// Hermitian eigensolver (cyclic Jacobi).  On return w holds the eigenvalues in
// ascending order and the columns of Z the eigenvectors (A = Z diag(w) Z^H).
inline void eigh_jacobi(const zc* Ain, double* w, zc* Z, int m) {
    std::vector<zc> A(Ain, Ain + m * m);
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) Z[i * m + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0, tot = 0;
        for (int i = 0; i < m; i++)
            for (int j = 0; j < m; j++) {
                double v = std::norm(A[i * m + j]);
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-32 * tot || off == 0) break;
        for (int p = 0; p < m - 1; p++)
            for (int q = p + 1; q < m; q++) {
                zc apq = A[p * m + q];
                double a = std::abs(apq);
                if (a < 1e-300) continue;
                double app = std::real(A[p * m + p]), aqq = std::real(A[q * m + q]);
                // rotation zeroing A[p][q]: phase e = apq/|apq|, angle from the 2x2 problem
                zc e = apq / a;
                double theta = 0.5 * std::atan2(2 * a, aqq - app);
                double c = std::cos(theta), s = std::sin(theta);
                // columns: new_p = c*col_p - s*conj(e)*col_q ; new_q = s*e*col_p + c*col_q
                for (int k = 0; k < m; k++) {
                    zc akp = A[k * m + p], akq = A[k * m + q];
                    A[k * m + p] = c * akp - s * std::conj(e) * akq;
                    A[k * m + q] = s * e * akp + c * akq;
                }
                for (int k = 0; k < m; k++) {
                    zc apk = A[p * m + k], aqk = A[q * m + k];
                    A[p * m + k] = c * apk - s * e * aqk;
                    A[q * m + k] = s * std::conj(e) * apk + c * aqk;
                }
                A[p * m + q] = 0;
                A[q * m + p] = 0;
                for (int k = 0; k < m; k++) {
                    zc zkp = Z[k * m + p], zkq = Z[k * m + q];
                    Z[k * m + p] = c * zkp - s * std::conj(e) * zkq;
                    Z[k * m + q] = s * e * zkp + c * zkq;
                }
            }
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; i++) idx[i] = i;
    std::vector<double> d(m);
    for (int i = 0; i < m; i++) d[i] = std::real(A[i * m + i]);
    for (int i = 0; i < m; i++)
        for (int j = i + 1; j < m; j++)
            if (d[idx[j]] < d[idx[i]]) std::swap(idx[i], idx[j]);
    std::vector<zc> Zs(m * m);
    for (int j = 0; j < m; j++) {
        w[j] = d[idx[j]];
        for (int k = 0; k < m; k++) Zs[k * m + j] = Z[k * m + idx[j]];
    }
    for (int i = 0; i < m * m; i++) Z[i] = Zs[i];
}
}  // namespace dense
