// Learned pointwise preconditioner (not in the paper; its Section 6 leaves the
// preconditioner open).  For node i and column l:
//
//   feat_il = [log(L_ii/2), log(B_ii), (H_ii - L_ii/2)/B_ii, g_il / rms(g_l)]
//   x       = (feat - mu) / sigma                         (standardization)
//   h       = tanh(W1 x + b1)        W1: 32 x 4, b1: 32
//   f       = W2 . h + b2            W2: 32,     b2: 1
//   J_il    = 1 / (L_ii/2 - Lambda_ll B_ii) if Lambda_ll < 0, else 1
//             (the Jacobi of the paper's T_l, identity branch as in the paper)
//   P_il    = exp(f) J_il g_il
//
// Parameters: one float vector [W1 (row-major), b1, W2, b2] of 193 values.
// Training minimizes sum_s w_s (exp(f_s) a_s - t_s)^2 over samples
// s = (feat, a = J g, t = (T^-1 g) from the paper preconditioner, w), with
// hand-written forward/backward, per-block gradient partials summed in a
// fixed order, and Adam.  All MLP arithmetic is FP32.
#include "common.hpp"

namespace ofks {

constexpr int LP_H = 32;
constexpr int LP_NPAR = LP_H * 4 + LP_H + LP_H + 1;  // 193
constexpr int LP_SAMPLE = 8;                         // floats per training sample

__device__ __forceinline__ float fast_tanh(float x) {
    // tanh x = 1 - 2 / (exp(2x) + 1); saturates correctly for large |x|
    const float e = __expf(2.0f * x);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// f(x) for standardized x; params in global memory (uniform across lanes)
__device__ __forceinline__ float lp_forward(const float *__restrict__ W, const float x[4]) {
    const float *W1 = W, *b1 = W + 4 * LP_H, *W2 = W + 5 * LP_H;
    const float b2 = W[6 * LP_H];
    float f = b2;
#pragma unroll 8
    for (int k = 0; k < LP_H; ++k) {
        float z = b1[k];
        z = fmaf(W1[4 * k + 0], x[0], z);
        z = fmaf(W1[4 * k + 1], x[1], z);
        z = fmaf(W1[4 * k + 2], x[2], z);
        z = fmaf(W1[4 * k + 3], x[3], z);
        f = fmaf(W2[k], fast_tanh(z), f);
    }
    return f;
}

// In place: P <- exp(f) J G (G is in P).  rms2[c] = sum_i g_ic^2 (FP64), n rows.
// norm = [mu0..mu3, sigma0..sigma3].  Same lane mapping as the block kernels.
template <typename T>
__global__ __launch_bounds__(256) void k_lp_apply(int64_t n, int p, int lpr_log2, T *__restrict__ P,
                                                 const double *__restrict__ lhd, const double *__restrict__ bd,
                                                 const double *__restrict__ hd, const T *__restrict__ lam,
                                                 const uint8_t *__restrict__ negl, const double *__restrict__ g2,
                                                 const float *__restrict__ W, const float *__restrict__ norm) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    const double l2 = lhd[row], b = bd[row];
    float xn[3];
    xn[0] = ((float)log(l2) - norm[0]) / norm[4];
    xn[1] = ((float)log(b) - norm[1]) / norm[5];
    xn[2] = ((float)((hd[row] - l2) / b) - norm[2]) / norm[6];
    for (int c = lane; c < p; c += lpr) {
        const T g = P[row * p + c];
        const float rms = (float)sqrt(g2[c] / (double)n);
        const float x[4] = {xn[0], xn[1], xn[2], (rms > 0.0f ? (float)g / rms - norm[3] : -norm[3]) / norm[7]};
        const float s = __expf(lp_forward(W, x));
        const T J = negl[c] ? T(1) / (T(l2) - lam[c] * T(b)) : T(1);
        P[row * p + c] = (T)s * J * g;
    }
}

// Training samples from rows i = offset + j * stride (all columns), slot
// (j * p + c) after base: raw features, then (a, t, w) of the weighted
// least-squares fit of exp(f) a to t:
//  objective 0 (Euclidean imitation): a = J g, t = P (the paper
//    preconditioner's output T^-1 g), w = tw_c = 1 / mean_i t_ic^2;
//  objective 1 (imitation in the energy norm of T, with the scale taken as
//    locally constant): a = 1, t = g / u, w = tw_c max(J g u, 0), where
//    u = T (J g) (U, active columns; u = g on identity-branch columns) and
//    tw_c = n / <g_c, t_c>.
template <typename T>
__global__ void k_lp_sample(int64_t n, int p, int64_t offset, int64_t stride, int64_t rows, int objective,
                            const T *__restrict__ G, const T *__restrict__ P, const T *__restrict__ U,
                            const double *__restrict__ lhd, const double *__restrict__ bd,
                            const double *__restrict__ hd, const T *__restrict__ lam,
                            const uint8_t *__restrict__ negl, const double *__restrict__ g2,
                            const double *__restrict__ tw, float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * p) return;
    const int64_t j = t / p;
    const int c = (int)(t % p);
    const int64_t i = offset + j * stride;
    if (i >= n) return;
    const double l2 = lhd[i], b = bd[i];
    const T g = G[i * p + c];
    const float rms = (float)sqrt(g2[c] / (double)n);
    const T J = negl[c] ? T(1) / (T(l2) - lam[c] * T(b)) : T(1);
    float *o = out + t * LP_SAMPLE;
    o[0] = (float)log(l2);
    o[1] = (float)log(b);
    o[2] = (float)((hd[i] - l2) / b);
    o[3] = rms > 0.0f ? (float)g / rms : 0.0f;
    if (objective == 0) {
        o[4] = (float)(J * g);
        o[5] = (float)P[i * p + c];
        o[6] = (float)tw[c];
    } else {
        const double a = (double)(J * g);
        const double u = negl[c] ? (double)U[i * p + c] : (double)g;
        const double au = a * u;
        o[4] = 1.0f;
        o[5] = u != 0.0 ? (float)((double)g / u) : 0.0f;
        o[6] = (u != 0.0 && au > 0.0) ? (float)(tw[c] * au) : 0.0f;
    }
    o[7] = 0.0f;
}

// Per-block partials of [loss, dloss/dparam (193)] over samples: each thread
// sums its samples in FP32 (a few hundred at most), the wave and block sums
// are FP64 in a fixed order; part[block][LP_NPAR + 1].
__global__ __launch_bounds__(256) void k_lp_grad(int64_t m, const float *__restrict__ S,
                                                const float *__restrict__ W, const float *__restrict__ norm,
                                                double *__restrict__ part) {
    const float *W1 = W, *b1 = W + 4 * LP_H, *W2 = W + 5 * LP_H;
    float acc[LP_NPAR + 1];
#pragma unroll
    for (int k = 0; k < LP_NPAR + 1; ++k) acc[k] = 0.0f;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
        const float *v = S + s * LP_SAMPLE;
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = (v[j] - norm[j]) / norm[4 + j];
        float h[LP_H];
        float f = W[6 * LP_H];
#pragma unroll
        for (int k = 0; k < LP_H; ++k) {
            float z = b1[k];
#pragma unroll
            for (int j = 0; j < 4; ++j) z = fmaf(W1[4 * k + j], x[j], z);
            h[k] = fast_tanh(z);
            f = fmaf(W2[k], h[k], f);
        }
        const float a = v[4], t = v[5], w = v[6];
        const float pa = __expf(f) * a;
        const float r = pa - t;
        acc[LP_NPAR] += w * r * r;
        const float df = 2.0f * w * r * pa;                // dL/df
        acc[6 * LP_H] += df;                                // b2
#pragma unroll
        for (int k = 0; k < LP_H; ++k) {
            acc[5 * LP_H + k] += df * h[k];                 // W2
            const float dz = df * W2[k] * (1.0f - h[k] * h[k]);
            acc[4 * LP_H + k] += dz;                        // b1
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[4 * k + j] += dz * x[j];   // W1
        }
    }
    // block reduction: fixed order over the 4 waves via LDS, lanes via a tree
    __shared__ double wr[4][LP_NPAR + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < LP_NPAR + 1; ++k) {
        double v = (double)acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) wr[wave][k] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < LP_NPAR + 1; k += blockDim.x)
        part[(int64_t)blockIdx.x * (LP_NPAR + 1) + k] = ((wr[0][k] + wr[1][k]) + wr[2][k]) + wr[3][k];
}

// Adam on the 193 parameters with gradient g = sum / m (FP64 sums).
__global__ void k_lp_adam(const double *__restrict__ gsum, double inv_m, float *__restrict__ W,
                          float *__restrict__ m1, float *__restrict__ m2, float lr, float beta1, float beta2,
                          float eps, int t) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= LP_NPAR) return;
    const float g = (float)(gsum[k] * inv_m);
    m1[k] = beta1 * m1[k] + (1.0f - beta1) * g;
    m2[k] = beta2 * m2[k] + (1.0f - beta2) * g * g;
    const float mh = m1[k] / (1.0f - powf(beta1, (float)t));
    const float vh = m2[k] / (1.0f - powf(beta2, (float)t));
    W[k] -= lr * mh / (sqrtf(vh) + eps);
}

// Feature statistics of the samples: part[block][8] = sums of x_j and x_j^2.
__global__ __launch_bounds__(256) void k_lp_stats(int64_t m, const float *__restrict__ S, double *__restrict__ part) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
        const float *v = S + s * LP_SAMPLE;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[j] += (double)v[j];
            acc[4 + j] += (double)v[j] * (double)v[j];
        }
    }
    __shared__ double wr[4][8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) wr[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8)
        part[(int64_t)blockIdx.x * 8 + threadIdx.x] =
            ((wr[0][threadIdx.x] + wr[1][threadIdx.x]) + wr[2][threadIdx.x]) + wr[3][threadIdx.x];
}

// ---------------------------------------------------------------------------
static inline int lp_ilog2c(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

template <typename T>
hipError_t launch_lp_apply(hipStream_t s, int64_t n, int p, T *P, const double *lhd, const double *bd,
                           const double *hd, const T *lam, const uint8_t *negl, const double *g2, const float *W,
                           const float *norm) {
    int l2 = lp_ilog2c(p);
    if (l2 > 6) l2 = 6;
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
    hipLaunchKernelGGL((k_lp_apply<T>), dim3(grid), dim3(256), 0, s, n, p, l2, P, lhd, bd, hd, lam, negl, g2, W, norm);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lp_sample(hipStream_t s, int64_t n, int p, int64_t offset, int64_t stride, int64_t rows,
                            int objective, const T *G, const T *P, const T *U, const double *lhd, const double *bd,
                            const double *hd, const T *lam, const uint8_t *negl, const double *g2, const double *tw,
                            float *out) {
    const int64_t tot = rows * p;
    if (tot <= 0) return hipSuccess;
    if (objective != 0 && !U) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_lp_sample<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, p, offset, stride,
                       rows, objective, G, P, U, lhd, bd, hd, lam, negl, g2, tw, out);
    return hipGetLastError();
}

hipError_t launch_lp_grad(hipStream_t s, int grid, int64_t m, const float *S, const float *W, const float *norm,
                          double *part) {
    hipLaunchKernelGGL(k_lp_grad, dim3(grid), dim3(256), 0, s, m, S, W, norm, part);
    return hipGetLastError();
}

hipError_t launch_lp_adam(hipStream_t s, const double *gsum, double inv_m, float *W, float *m1, float *m2, float lr,
                          float beta1, float beta2, float eps, int t) {
    hipLaunchKernelGGL(k_lp_adam, dim3(1), dim3(256), 0, s, gsum, inv_m, W, m1, m2, lr, beta1, beta2, eps, t);
    return hipGetLastError();
}

hipError_t launch_lp_stats(hipStream_t s, int grid, int64_t m, const float *S, double *part) {
    hipLaunchKernelGGL(k_lp_stats, dim3(grid), dim3(256), 0, s, m, S, part);
    return hipGetLastError();
}

template hipError_t launch_lp_apply<double>(hipStream_t, int64_t, int, double *, const double *, const double *,
                                            const double *, const double *, const uint8_t *, const double *,
                                            const float *, const float *);
template hipError_t launch_lp_apply<float>(hipStream_t, int64_t, int, float *, const double *, const double *,
                                           const double *, const float *, const uint8_t *, const double *,
                                           const float *, const float *);
template hipError_t launch_lp_sample<double>(hipStream_t, int64_t, int, int64_t, int64_t, int64_t, int,
                                             const double *, const double *, const double *, const double *,
                                             const double *, const double *, const double *, const uint8_t *,
                                             const double *, const double *, float *);
template hipError_t launch_lp_sample<float>(hipStream_t, int64_t, int, int64_t, int64_t, int64_t, int, const float *,
                                            const float *, const float *, const double *, const double *,
                                            const double *, const float *, const uint8_t *, const double *,
                                            const double *, float *);

}  // namespace ofks
