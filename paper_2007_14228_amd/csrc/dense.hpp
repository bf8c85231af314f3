// Small dense FP64 algebra on the host for the p x p quantities of PCAL:
// Cholesky (Cholesky-based Gram-Schmidt of the starting block, Section 4.2),
// triangular inverse, a cyclic Jacobi symmetric eigensolver and the
// generalized problem A y = lambda S y by Cholesky reduction (Rayleigh-Ritz,
// Section 4.3).  Row-major storage, p <= a few hundred.
#pragma once

#include <cmath>
#include <algorithm>
#include <thread>
#include <vector>

namespace ofks {
namespace dense {

// A = L L^T in place (lower triangle holds L, upper zeroed).  false if not SPD.
inline bool cholesky(std::vector<double> &A, int p) {
    // row-oriented dot products with four partial sums (their order is fixed)
    auto dot = [](const double *x, const double *y, int m) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int k = 0;
        for (; k + 4 <= m; k += 4) {
            s0 += x[k] * y[k];
            s1 += x[k + 1] * y[k + 1];
            s2 += x[k + 2] * y[k + 2];
            s3 += x[k + 3] * y[k + 3];
        }
        for (; k < m; ++k) s0 += x[k] * y[k];
        return (s0 + s1) + (s2 + s3);
    };
    for (int j = 0; j < p; ++j) {
        const double *aj = &A[(size_t)j * p];
        double d = A[(size_t)j * p + j] - dot(aj, aj, j);
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        d = std::sqrt(d);
        A[(size_t)j * p + j] = d;
        for (int i = j + 1; i < p; ++i) {
            const double *ai = &A[(size_t)i * p];
            A[(size_t)i * p + j] = (A[(size_t)i * p + j] - dot(ai, aj, j)) / d;
        }
        for (int i = 0; i < j; ++i) A[(size_t)i * p + j] = 0.0;
    }
    return true;
}

// inverse of a lower-triangular L (result lower triangular), by rows:
// row i of L^-1 is (e_i - sum_{k<i} L_ik row k) / L_ii
inline std::vector<double> lower_inverse(const std::vector<double> &L, int p) {
    std::vector<double> M((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) {
        double *mi = &M[(size_t)i * p];
        for (int k = 0; k < i; ++k) {
            const double l = L[(size_t)i * p + k];
            const double *mk = &M[(size_t)k * p];
            for (int j = 0; j <= k; ++j) mi[j] -= l * mk[j];
        }
        const double inv = 1.0 / L[(size_t)i * p + i];
        for (int j = 0; j < i; ++j) mi[j] *= inv;
        mi[i] = inv;
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
    // S = L L^T, S^-1 A = L^-T (L^-1 A): tr(S^-1 A) = sum_i <row i of L^-1, row i of L^-1 A>.
    // The rows are independent; from p = 256 on they are split over host
    // threads, each row's term kept and the terms summed in row order.
    std::vector<double> L = S;
    if (!cholesky(L, p)) return false;
    const std::vector<double> Li = lower_inverse(L, p);
    std::vector<double> term(p);
    auto rows = [&](int i0, int i1) {
        std::vector<double> t(p);
        for (int i = i0; i < i1; ++i) {
            const double *li = &Li[(size_t)i * p];
            for (int j = 0; j < p; ++j) t[j] = 0.0;
            for (int k = 0; k <= i; ++k) {
                const double l = li[k];
                const double *a = &A[(size_t)k * p];
                for (int j = 0; j < p; ++j) t[j] += l * a[j];
            }
            double s = 0.0;
            for (int k = 0; k <= i; ++k) s += t[k] * li[k];
            term[i] = s;
        }
    };
    const int nt = p >= 256 ? std::max(1, std::min(8, (int)std::thread::hardware_concurrency())) : 1;
    if (nt == 1) {
        rows(0, p);
    } else {
        // rows i cost ~ i: cut so that every thread gets about the same work
        std::vector<std::thread> th;
        int lo = 0;
        for (int t = 0; t < nt; ++t) {
            const int hi = t == nt - 1 ? p : (int)std::lround(p * std::sqrt((t + 1.0) / nt));
            if (hi > lo) th.emplace_back(rows, lo, hi);
            lo = std::max(lo, hi);
        }
        for (auto &x : th) x.join();
    }
    double tr = 0.0;
    for (int i = 0; i < p; ++i) tr += term[i];
    out = tr;
    return true;
}

}  // namespace dense
}  // namespace ofks
