// Graph (message-passing) learned preconditioner (not in the paper; its
// Section 6 leaves the preconditioner open).  A pointwise network gives every
// (row i, column l) a scale and a smoothing weight; one damped Jacobi sweep
// through the paper's operator T_l (eq. precondition-T) over the CSR pattern
// then smooths:
//
//   feat_il  = [log(L_ii/2), log(B_ii), (H_ii - L_ii/2)/B_ii, g_il / rms(g_l)]
//   x        = (feat - mu) / sigma
//   h        = tanh(W1 x + b1)                   W1: 32 x 4, b1: 32
//   (fs, ft) = W2 h + b2                         W2: 2 x 32 (row 0: fs), b2: 2
//   J_il     = 1 / (L_ii/2 - Lambda_ll B_ii) if Lambda_ll < 0, else 1
//   Z        = exp(fs) J G
//   R        = G - T Z            (T = I on identity-branch columns)
//   P        = Z + ft J R
//
// Parameters: one float vector [W1 (row-major), b1, W2 (row-major), b2] of
// 226 values.  Inference is two kernels around one shifted SpMM (Q = T Z,
// the SpMM's MODE 1): k_gl_heads writes Z and ft, k_gl_out forms P from G, Z,
// ft and Q.  Training minimizes the quadratic model of each column's system,
//   loss = sum_l w_l (P_l^T T_l P_l / 2 - G_l^T P_l),  w_l = 1 / (G_l^T J_l G_l),
// by backpropagation through the sweep (T_l is symmetric, so the adjoint of
// the sweep is one more shifted SpMM) and the network, with per-block FP64
// partials summed in a fixed order and Adam.  Network arithmetic is FP32.
#include "common.hpp"

namespace ofks {

constexpr int GL_H = 32;
constexpr int GL_NPAR = 4 * GL_H + GL_H + 2 * GL_H + 2;   // 226

__device__ __forceinline__ float gl_tanh(float x) {
    // tanh x = 1 - 2 / (exp(2x) + 1); saturates correctly for large |x|
    const float e = __expf(2.0f * x);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// Both heads for standardized x; the hidden layer into h when KEEP.
template <bool KEEP>
__device__ __forceinline__ void gl_forward(const float *__restrict__ W, const float x[4], float &fs, float &ft,
                                           float *h) {
    const float *W1 = W, *b1 = W + 4 * GL_H, *W2 = W + 5 * GL_H, *b2 = W + 7 * GL_H;
    fs = b2[0];
    ft = b2[1];
#pragma unroll 8
    for (int k = 0; k < GL_H; ++k) {
        float z = b1[k];
        z = fmaf(W1[4 * k + 0], x[0], z);
        z = fmaf(W1[4 * k + 1], x[1], z);
        z = fmaf(W1[4 * k + 2], x[2], z);
        z = fmaf(W1[4 * k + 3], x[3], z);
        const float t = gl_tanh(z);
        if (KEEP) h[k] = t;
        fs = fmaf(W2[k], t, fs);
        ft = fmaf(W2[GL_H + k], t, ft);
    }
}

// Standardized node features of a row (the first three inputs).
__device__ __forceinline__ void gl_node(double l2, double b, double hdv, const float *__restrict__ norm, float xn[3]) {
    xn[0] = ((float)log(l2) - norm[0]) / norm[4];
    xn[1] = ((float)log(b) - norm[1]) / norm[5];
    xn[2] = ((float)((hdv - l2) / b) - norm[2]) / norm[6];
}

__device__ __forceinline__ float gl_resid_feature(float g, float rms, const float *__restrict__ norm) {
    return ((rms > 0.0f ? g / rms : 0.0f) - norm[3]) / norm[7];
}

// Z = exp(fs) J G and FT = ft for every (row, column); rows handled by
// 2^lpr_log2 lanes that stride over the columns (the block kernels' mapping).
// g2[c] = sum_i g_ic^2 (FP64).
//
// The same arithmetic as gl_forward, arranged for the VALU: the row-only part
// of the first layer is formed once per row (a_k = W1[k,0:3] x_node + b1_k),
// leaving one FMA per hidden unit and column; the hidden pre-activations are
// pre-scaled by 2 log2(e), so tanh z = 1 - 2 / (2^(2 log2(e) z) + 1) takes one
// exp2, one add and one hardware reciprocal; and sum_k W2_k tanh_k is summed
// as sum_k W2_k - 2 sum_k W2_k / (2^(...) + 1).
template <typename T>
__global__ __launch_bounds__(256) void k_gl_heads(int64_t n, int p, int lpr_log2, const T *__restrict__ G,
                                                 const double *__restrict__ lhd, const double *__restrict__ bd,
                                                 const double *__restrict__ hd, const T *__restrict__ lam,
                                                 const uint8_t *__restrict__ negl, const double *__restrict__ g2,
                                                 const float *__restrict__ W, const float *__restrict__ norm,
                                                 T *__restrict__ Z, float *__restrict__ FT) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    const float *W1 = W, *b1 = W + 4 * GL_H, *W2 = W + 5 * GL_H, *b2 = W + 7 * GL_H;
    constexpr float K2 = 2.0f * 1.4426950408889634f;   // 2 log2(e)
    const double l2 = lhd[row], b = bd[row];
    float x[3];
    gl_node(l2, b, hd[row], norm, x);
    float a[GL_H];
    float s0 = b2[0], s1 = b2[1];
#pragma unroll
    for (int k = 0; k < GL_H; ++k) {
        float z = b1[k];
        z = fmaf(W1[4 * k + 0], x[0], z);
        z = fmaf(W1[4 * k + 1], x[1], z);
        z = fmaf(W1[4 * k + 2], x[2], z);
        a[k] = K2 * z;
        s0 += W2[k];
        s1 += W2[GL_H + k];
    }
    for (int c = lane; c < p; c += lpr) {
        const T g = G[row * p + c];
        const float x3 = gl_resid_feature((float)g, (float)sqrt(g2[c] / (double)n), norm);
        float r0 = 0.0f, r1 = 0.0f;
#pragma unroll
        for (int k = 0; k < GL_H; ++k) {
            const float z2 = fmaf(K2 * W1[4 * k + 3], x3, a[k]);
            const float r = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(z2) + 1.0f);
            r0 = fmaf(W2[k], r, r0);
            r1 = fmaf(W2[GL_H + k], r, r1);
        }
        const float fs = fmaf(-2.0f, r0, s0), ft = fmaf(-2.0f, r1, s1);
        const T J = negl[c] ? T(1) / (T(l2) - lam[c] * T(b)) : T(1);
        Z[row * p + c] = (T)__builtin_amdgcn_exp2f(1.4426950408889634f * fs) * J * g;
        FT[row * p + c] = ft;
    }
}

// P = Z + ft J (G - T Z), with Q = T Z on active columns (T = I elsewhere).
// P may be G (in place).
template <typename T>
__global__ __launch_bounds__(256) void k_gl_out(int64_t n, int p, int lpr_log2, const T *G, const T *__restrict__ Z,
                                               const float *__restrict__ FT, const T *__restrict__ Q,
                                               const double *__restrict__ lhd, const double *__restrict__ bd,
                                               const T *__restrict__ lam, const uint8_t *__restrict__ negl,
                                               T *P, T *__restrict__ Rout) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    const T l2 = T(lhd[row]), b = T(bd[row]);
    for (int c = lane; c < p; c += lpr) {
        const int64_t e = row * p + c;
        const bool on = negl[c] != 0;
        const T z = Z[e];
        const T r = G[e] - (on ? Q[e] : z);
        const T J = on ? T(1) / (l2 - lam[c] * b) : T(1);
        if (Rout) Rout[e] = r;
        P[e] = z + (T)FT[e] * J * r;
    }
}

// ---------------------------------------------------------------------------
// Training (FP64 blocks).  Rows are split into gridDim.x chunks; thread c of
// a block owns column c (and c + 256, ...) of its chunk, so every per-column
// partial has a fixed summation order.
// ---------------------------------------------------------------------------

// part[block][0..p) = sum g^2, part[block][p..2p) = sum g J g.
__global__ __launch_bounds__(256) void k_gl_colsums(int64_t n, int p, const double *__restrict__ G,
                                                   const double *__restrict__ lhd, const double *__restrict__ bd,
                                                   const double *__restrict__ lam, const uint8_t *__restrict__ negl,
                                                   double *__restrict__ part) {
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        double gg = 0.0, gjg = 0.0;
        const bool on = negl[c] != 0;
        for (int64_t i = r0; i < r1; ++i) {
            const double g = G[i * p + c];
            const double J = on ? 1.0 / (lhd[i] - lam[c] * bd[i]) : 1.0;
            gg += g * g;
            gjg += g * J * g;
        }
        part[(int64_t)blockIdx.x * 2 * p + c] = gg;
        part[(int64_t)blockIdx.x * 2 * p + p + c] = gjg;
    }
}

// dP = w (T P - G) into TP (in place), dR = ft J dP; loss partials per column:
// part[block][c] = P.TP / 2 - G.P over the chunk (w applied after the sum).
__global__ __launch_bounds__(256) void k_gl_bwd1(int64_t n, int p, const double *__restrict__ G,
                                                const double *__restrict__ P, double *__restrict__ TP,
                                                const float *__restrict__ FT, const double *__restrict__ lhd,
                                                const double *__restrict__ bd, const double *__restrict__ lam,
                                                const uint8_t *__restrict__ negl, const double *__restrict__ w,
                                                double *__restrict__ dR, double *__restrict__ part) {
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        const bool on = negl[c] != 0;
        double acc = 0.0;
        for (int64_t i = r0; i < r1; ++i) {
            const int64_t e = i * p + c;
            const double pv = P[e], g = G[e];
            const double tp = on ? TP[e] : pv;
            acc += 0.5 * pv * tp - g * pv;
            const double dp = w[c] * (tp - g);
            const double J = on ? 1.0 / (lhd[i] - lam[c] * bd[i]) : 1.0;
            TP[e] = dp;
            dR[e] = (double)FT[e] * J * dp;
        }
        part[(int64_t)blockIdx.x * p + c] = acc;
    }
}

// Parameter gradient: with dP (in DP), R, Z, dR and T dR (TDR, active
// columns): dft = dP J R, dZ = dP - T dR, dfs = dZ Z, then backpropagation
// through the heads.  Grid-stride over batches of 256 elements: thread t puts
// element t's inputs x, hidden layer h and (dfs, dft) in LDS; then thread k
// (< 226) adds parameter k's contributions of the whole batch to its own
// FP64 sum, in element order.  part[block][GL_NPAR].
constexpr int GL_LDS = 257;   // padded row of the batch arrays (bank spread)
__global__ __launch_bounds__(256) void k_gl_bwd2(int64_t n, int p, const double *__restrict__ G,
                                                const double *__restrict__ DP, const double *__restrict__ R,
                                                const double *__restrict__ Z, const double *__restrict__ dR,
                                                const double *__restrict__ TDR, const double *__restrict__ lhd,
                                                const double *__restrict__ bd, const double *__restrict__ hd,
                                                const double *__restrict__ lam, const uint8_t *__restrict__ negl,
                                                const double *__restrict__ g2, const float *__restrict__ W,
                                                const float *__restrict__ norm, double *__restrict__ part) {
    __shared__ float sx[4][GL_LDS], sh[GL_H][GL_LDS], sd[2][GL_LDS];
    const float *W2 = W + 5 * GL_H;
    const int t = threadIdx.x;
    double acc = 0.0;
    const int64_t m = n * p;
    for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < m; e0 += (int64_t)gridDim.x * 256) {
        const int64_t e = e0 + t;
        if (e < m) {
            const int64_t i = e / p;
            const int c = (int)(e - i * p);
            const bool on = negl[c] != 0;
            float x[4];
            gl_node(lhd[i], bd[i], hd[i], norm, x);
            x[3] = gl_resid_feature((float)G[e], (float)sqrt(g2[c] / (double)n), norm);
            float h[GL_H], fs, ft;
            gl_forward<true>(W, x, fs, ft, h);
            const double J = on ? 1.0 / (lhd[i] - lam[c] * bd[i]) : 1.0;
            const double dp = DP[e];
            sd[1][t] = (float)(dp * J * R[e]);                         // dft
            sd[0][t] = (float)((dp - (on ? TDR[e] : dR[e])) * Z[e]);   // dfs
#pragma unroll
            for (int j = 0; j < 4; ++j) sx[j][t] = x[j];
#pragma unroll
            for (int k = 0; k < GL_H; ++k) sh[k][t] = h[k];
        } else {
            sd[0][t] = sd[1][t] = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) sx[j][t] = 0.0f;
#pragma unroll
            for (int k = 0; k < GL_H; ++k) sh[k][t] = 0.0f;
        }
        __syncthreads();
        if (t < GL_NPAR) {
            if (t < 5 * GL_H) {          // W1[kk][j] (t < 128) or b1[kk]: through dz_kk
                const int kk = t < 4 * GL_H ? t >> 2 : t - 4 * GL_H;
                const int j = t & 3;
                const float w0 = W2[kk], w1 = W2[GL_H + kk];
                for (int u = 0; u < 256; ++u) {
                    const float hv = sh[kk][u];
                    const float dz = (sd[0][u] * w0 + sd[1][u] * w1) * (1.0f - hv * hv);
                    acc += (double)(t < 4 * GL_H ? dz * sx[j][u] : dz);
                }
            } else if (t < 7 * GL_H) {   // W2[r][kk]
                const int r = (t - 5 * GL_H) >> 5, kk = (t - 5 * GL_H) & (GL_H - 1);
                for (int u = 0; u < 256; ++u) acc += (double)(sd[r][u] * sh[kk][u]);
            } else {                     // b2[r]
                const int r = t - 7 * GL_H;
                for (int u = 0; u < 256; ++u) acc += (double)sd[r][u];
            }
        }
        __syncthreads();
    }
    if (t < GL_NPAR) part[(int64_t)blockIdx.x * GL_NPAR + t] = acc;
}

// Adam on npar parameters with gradient gsum * scale.
__global__ void k_gl_adam(int npar, const double *__restrict__ gsum, double scale, float *__restrict__ W,
                          float *__restrict__ m1, float *__restrict__ m2, float lr, float beta1, float beta2,
                          float eps, int t) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npar) return;
    const float g = (float)(gsum[k] * scale);
    m1[k] = beta1 * m1[k] + (1.0f - beta1) * g;
    m2[k] = beta2 * m2[k] + (1.0f - beta2) * g * g;
    const float mh = m1[k] / (1.0f - powf(beta1, (float)t));
    const float vh = m2[k] / (1.0f - powf(beta2, (float)t));
    W[k] -= lr * mh / (sqrtf(vh) + eps);
}

// Node-feature statistics: part[block][6] = sums of the three node features
// and of their squares over the block's rows.
__global__ __launch_bounds__(256) void k_gl_node_stats(int64_t n, const double *__restrict__ lhd,
                                                      const double *__restrict__ bd, const double *__restrict__ hd,
                                                      double *__restrict__ part) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double f[3] = {log(lhd[i]), log(bd[i]), (hd[i] - lhd[i]) / bd[i]};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            acc[j] += f[j];
            acc[3 + j] += f[j] * f[j];
        }
    }
    __shared__ double wr[4][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) wr[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6)
        part[(int64_t)blockIdx.x * 6 + threadIdx.x] =
            ((wr[0][threadIdx.x] + wr[1][threadIdx.x]) + wr[2][threadIdx.x]) + wr[3][threadIdx.x];
}

// Raw features [n, p, 4] (FP32) of the learned forms for block G.
__global__ __launch_bounds__(256) void k_features(int64_t n, int p, const double *__restrict__ G,
                                                 const double *__restrict__ lhd, const double *__restrict__ bd,
                                                 const double *__restrict__ hd, const double *__restrict__ g2,
                                                 float *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * p) return;
    const int64_t i = e / p;
    const int c = (int)(e - i * p);
    const float rms = (float)sqrt(g2[c] / (double)n);
    float *o = out + e * 4;
    o[0] = (float)log(lhd[i]);
    o[1] = (float)log(bd[i]);
    o[2] = (float)((hd[i] - lhd[i]) / bd[i]);
    o[3] = rms > 0.0f ? (float)G[e] / rms : 0.0f;
}

// ---------------------------------------------------------------------------
static inline int gl_lpr_log2(int p) {
    int l = 0;
    while ((1 << l) < p) ++l;
    return l > 6 ? 6 : l;
}

template <typename T>
hipError_t launch_gl_heads(hipStream_t s, int64_t n, int p, const T *G, const double *lhd, const double *bd,
                           const double *hd, const T *lam, const uint8_t *negl, const double *g2, const float *W,
                           const float *norm, T *Z, float *FT) {
    const int l2 = gl_lpr_log2(p);
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
    hipLaunchKernelGGL((k_gl_heads<T>), dim3(grid), dim3(256), 0, s, n, p, l2, G, lhd, bd, hd, lam, negl, g2, W,
                       norm, Z, FT);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gl_out(hipStream_t s, int64_t n, int p, const T *G, const T *Z, const float *FT, const T *Q,
                         const double *lhd, const double *bd, const T *lam, const uint8_t *negl, T *P, T *Rout) {
    const int l2 = gl_lpr_log2(p);
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
    hipLaunchKernelGGL((k_gl_out<T>), dim3(grid), dim3(256), 0, s, n, p, l2, G, Z, FT, Q, lhd, bd, lam, negl, P,
                       Rout);
    return hipGetLastError();
}

hipError_t launch_gl_colsums(hipStream_t s, int grid, int64_t n, int p, const double *G, const double *lhd,
                             const double *bd, const double *lam, const uint8_t *negl, double *part) {
    hipLaunchKernelGGL(k_gl_colsums, dim3(grid), dim3(256), 0, s, n, p, G, lhd, bd, lam, negl, part);
    return hipGetLastError();
}

hipError_t launch_gl_bwd1(hipStream_t s, int grid, int64_t n, int p, const double *G, const double *P, double *TP,
                          const float *FT, const double *lhd, const double *bd, const double *lam,
                          const uint8_t *negl, const double *w, double *dR, double *part) {
    hipLaunchKernelGGL(k_gl_bwd1, dim3(grid), dim3(256), 0, s, n, p, G, P, TP, FT, lhd, bd, lam, negl, w, dR, part);
    return hipGetLastError();
}

hipError_t launch_gl_bwd2(hipStream_t s, int grid, int64_t n, int p, const double *G, const double *DP,
                          const double *R, const double *Z, const double *dR, const double *TDR, const double *lhd,
                          const double *bd, const double *hd, const double *lam, const uint8_t *negl,
                          const double *g2, const float *W, const float *norm, double *part) {
    hipLaunchKernelGGL(k_gl_bwd2, dim3(grid), dim3(256), 0, s, n, p, G, DP, R, Z, dR, TDR, lhd, bd, hd, lam, negl,
                       g2, W, norm, part);
    return hipGetLastError();
}

hipError_t launch_gl_adam(hipStream_t s, int npar, const double *gsum, double scale, float *W, float *m1, float *m2,
                          float lr, float beta1, float beta2, float eps, int t) {
    hipLaunchKernelGGL(k_gl_adam, dim3((npar + 255) / 256), dim3(256), 0, s, npar, gsum, scale, W, m1, m2, lr,
                       beta1, beta2, eps, t);
    return hipGetLastError();
}

hipError_t launch_gl_node_stats(hipStream_t s, int grid, int64_t n, const double *lhd, const double *bd,
                                const double *hd, double *part) {
    hipLaunchKernelGGL(k_gl_node_stats, dim3(grid), dim3(256), 0, s, n, lhd, bd, hd, part);
    return hipGetLastError();
}

hipError_t launch_features(hipStream_t s, int64_t n, int p, const double *G, const double *lhd, const double *bd,
                           const double *hd, const double *g2, float *out) {
    const int64_t m = n * p;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, n, p, G, lhd, bd, hd, g2, out);
    return hipGetLastError();
}

template hipError_t launch_gl_heads<double>(hipStream_t, int64_t, int, const double *, const double *,
                                            const double *, const double *, const double *, const uint8_t *,
                                            const double *, const float *, const float *, double *, float *);
template hipError_t launch_gl_heads<float>(hipStream_t, int64_t, int, const float *, const double *, const double *,
                                           const double *, const float *, const uint8_t *, const double *,
                                           const float *, const float *, float *, float *);
template hipError_t launch_gl_out<double>(hipStream_t, int64_t, int, const double *, const double *, const float *,
                                          const double *, const double *, const double *, const double *,
                                          const uint8_t *, double *, double *);
template hipError_t launch_gl_out<float>(hipStream_t, int64_t, int, const float *, const float *, const float *,
                                         const float *, const double *, const double *, const float *,
                                         const uint8_t *, float *, float *);

}  // namespace ofks
