// Small dense FP64 algebra on the host for the p x p quantities of PCAL:
// Cholesky (Cholesky-based Gram-Schmidt of the starting block, Section 4.2),
// triangular inverse, a cyclic Jacobi symmetric eigensolver and the
// generalized problem A y = lambda S y by Cholesky reduction (Rayleigh-Ritz,
// Section 4.3).  Row-major storage, p <= a few hundred.
#pragma once

#include <cmath>
#include <vector>

namespace ofks {
namespace dense {

// A = L L^T in place (lower triangle holds L, upper zeroed).  false if not SPD.
inline bool cholesky(std::vector<double> &A, int p) {
    for (int j = 0; j < p; ++j) {
        double d = A[j * p + j];
        for (int k = 0; k < j; ++k) d -= A[j * p + k] * A[j * p + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        d = std::sqrt(d);
        A[j * p + j] = d;
        for (int i = j + 1; i < p; ++i) {
            double s = A[i * p + j];
            for (int k = 0; k < j; ++k) s -= A[i * p + k] * A[j * p + k];
            A[i * p + j] = s / d;
        }
        for (int i = 0; i < j; ++i) A[i * p + j] = 0.0;
    }
    return true;
}

// inverse of a lower-triangular L (result lower triangular)
inline std::vector<double> lower_inverse(const std::vector<double> &L, int p) {
    std::vector<double> M(p * p, 0.0);
    for (int j = 0; j < p; ++j) {
        M[j * p + j] = 1.0 / L[j * p + j];
        for (int i = j + 1; i < p; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += L[i * p + k] * M[k * p + j];
            M[i * p + j] = -s / L[i * p + i];
        }
    }
    return M;
}

// Cyclic Jacobi: A symmetric (destroyed), eigenvalues w ascending, V columns
// eigenvectors (row-major, V[i*p + j] = component i of vector j).
inline void sym_eig(std::vector<double> A, int p, std::vector<double> &w, std::vector<double> &V) {
    V.assign(p * p, 0.0);
    for (int i = 0; i < p; ++i) V[i * p + i] = 1.0;
    double fro = 0.0;
    for (double x : A) fro += x * x;
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) off += A[i * p + j] * A[i * p + j];
        if (std::sqrt(off) <= 1e-15 * fro || off == 0.0) break;
        for (int i = 0; i < p; ++i) {
            for (int j = i + 1; j < p; ++j) {
                const double aij = A[i * p + j];
                if (aij == 0.0) continue;
                const double aii = A[i * p + i], ajj = A[j * p + j];
                const double theta = (ajj - aii) / (2.0 * aij);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < p; ++k) {  // rows i, j
                    const double aik = A[i * p + k], ajk = A[j * p + k];
                    A[i * p + k] = c * aik - s * ajk;
                    A[j * p + k] = s * aik + c * ajk;
                }
                for (int k = 0; k < p; ++k) {  // columns i, j
                    const double aki = A[k * p + i], akj = A[k * p + j];
                    A[k * p + i] = c * aki - s * akj;
                    A[k * p + j] = s * aki + c * akj;
                }
                for (int k = 0; k < p; ++k) {
                    const double vki = V[k * p + i], vkj = V[k * p + j];
                    V[k * p + i] = c * vki - s * vkj;
                    V[k * p + j] = s * vki + c * vkj;
                }
            }
        }
    }
    // sort ascending
    std::vector<int> idx(p);
    for (int i = 0; i < p; ++i) idx[i] = i;
    for (int i = 1; i < p; ++i) {
        int k = idx[i], j = i - 1;
        while (j >= 0 && A[idx[j] * p + idx[j]] > A[k * p + k]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = k;
    }
    std::vector<double> V2(p * p);
    w.resize(p);
    for (int j = 0; j < p; ++j) {
        w[j] = A[idx[j] * p + idx[j]];
        for (int i = 0; i < p; ++i) V2[i * p + j] = V[i * p + idx[j]];
    }
    V.swap(V2);
}

// A y = lambda S y with S SPD: S = L L^T, C = L^-1 A L^-T, C = W diag W^T,
// Y = L^-T W (so Y^T S Y = I).  false if S is not SPD.
inline bool sym_gen_eig(const std::vector<double> &A, const std::vector<double> &S, int p,
                        std::vector<double> &w, std::vector<double> &Y) {
    std::vector<double> L = S;
    if (!cholesky(L, p)) return false;
    std::vector<double> Li = lower_inverse(L, p);
    std::vector<double> T(p * p, 0.0), C(p * p, 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            double s = 0.0;
            for (int k = 0; k <= i; ++k) s += Li[i * p + k] * A[k * p + j];
            T[i * p + j] = s;
        }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            double s = 0.0;
            for (int k = 0; k <= j; ++k) s += T[i * p + k] * Li[j * p + k];
            C[i * p + j] = s;
        }
    for (int i = 0; i < p; ++i)
        for (int j = i + 1; j < p; ++j) {
            const double m = 0.5 * (C[i * p + j] + C[j * p + i]);
            C[i * p + j] = C[j * p + i] = m;
        }
    std::vector<double> W;
    sym_eig(C, p, w, W);
    Y.assign(p * p, 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            double s = 0.0;
            for (int k = i; k < p; ++k) s += Li[k * p + i] * W[k * p + j];
            Y[i * p + j] = s;
        }
    return true;
}

// tr(S^-1 A) for S SPD, via S = L L^T: sum_i (L^-1 A L^-T)_ii.
inline bool trace_sinv_a(const std::vector<double> &S, const std::vector<double> &A, int p,
                         double &out) {
    std::vector<double> L = S;
    if (!cholesky(L, p)) return false;
    std::vector<double> Li = lower_inverse(L, p);
    double tr = 0.0;
    std::vector<double> t(p);
    for (int i = 0; i < p; ++i) {
        // t = row i of Li A
        for (int j = 0; j < p; ++j) {
            double s = 0.0;
            for (int k = 0; k <= i; ++k) s += Li[i * p + k] * A[k * p + j];
            t[j] = s;
        }
        double s = 0.0;
        for (int k = 0; k <= i; ++k) s += t[k] * Li[i * p + k];
        tr += s;
    }
    out = tr;
    return true;
}

}  // namespace dense
}  // namespace ofks
