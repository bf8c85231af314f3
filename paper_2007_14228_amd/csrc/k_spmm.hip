// Sparse products on the shared P1 CSR pattern.
//
//  k_spmm_pair   : Y1 = A1 X and Y2 = A2 X in one pass (H X and B X, the
//                  "function evaluation" of Algorithm PCAL); values of the
//                  two matrices are interleaved per nonzero so one 16-byte
//                  (f64) or 8-byte (f32) load feeds both products.
//  k_spmm_one    : Y = A X (B X alone: column norms, Cholesky-Gram-Schmidt).
//  k_spmm_shift  : Q[:,l] = (L/2 - lam_l B) D[:,l] (operator of the paper's
//                  preconditioner T_l, eq. precondition-T) with the per-column
//                  dot products <D_l, Q_l> of the CG step fused in.
//  k_spmv_dot    : q = A d and <d, q> for one vector (Hartree CG).
//
// Work mapping (wave64): a row is owned by LPR = 2^lpr_log2 lanes; each lane
// covers V consecutive columns (one vector load of the X row slice), and
// loops over column chunks when p > LPR*V.  A row's p values are contiguous,
// so the LPR lanes of a row read one contiguous X row per nonzero: with
// p = 128 in f64 a wave reads 1 KB per neighbour, fully coalesced.
// Column indices and values are read once per lane group (the same address
// across the group is served by one cache line).
#include "common.hpp"

namespace ofks {

template <typename T> struct pair_t;
template <> struct pair_t<double> { using type = double2; };
template <> struct pair_t<float> { using type = float2; };

template <typename T, int V, int NOUT>
__global__ __launch_bounds__(256) void k_spmm_pair(int64_t n, int p, int lpr_log2,
                                                  const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const typename pair_t<T>::type *__restrict__ ab,
                                                  const T *__restrict__ X, T *__restrict__ Y1,
                                                  T *__restrict__ Y2, int sel) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    const int64_t e0 = rp[row], e1 = rp[row + 1];
    for (int c0 = lane * V; c0 < p; c0 += lpr * V) {
        T a1[V], a2[V];
#pragma unroll
        for (int v = 0; v < V; ++v) { a1[v] = T(0); a2[v] = T(0); }
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t j = col[e];
            const auto w = ab[e];
            T x[V];
            load_vec<T, V>(X + j * p + c0, x);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (NOUT == 2) {
                    a1[v] = fma(w.x, x[v], a1[v]);
                    a2[v] = fma(w.y, x[v], a2[v]);
                } else {
                    a1[v] = fma(sel ? w.y : w.x, x[v], a1[v]);
                }
            }
        }
        store_vec<T, V>(Y1 + row * p + c0, a1);
        if (NOUT == 2) store_vec<T, V>(Y2 + row * p + c0, a2);
    }
}

// Persistent grid: block b handles rows {b*rpb + g + k*gridDim*rpb}; every
// block's share and summation order are fixed by the launch shape, so the
// per-block partial dot products (written to part[b*p + c]) are reproducible.
template <typename T, int V, int CH>
__global__ __launch_bounds__(256) void k_spmm_shift(int64_t n, int p, int lpr_log2,
                                                   const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const typename pair_t<T>::type *__restrict__ lb,
                                                   const T *__restrict__ lam,
                                                   const uint8_t *__restrict__ active,
                                                   const T *__restrict__ D, T *__restrict__ Q,
                                                   double *__restrict__ part) {
    extern __shared__ double red[];  // [groups][p]
    const int lpr = 1 << lpr_log2;
    const int groups = blockDim.x >> lpr_log2;
    const int g = threadIdx.x >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    double dot[CH][V];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < V; ++v) dot[ch][v] = 0.0;

    for (int64_t row = (int64_t)blockIdx.x * groups + g; row < n; row += (int64_t)gridDim.x * groups) {
        const int64_t e0 = rp[row], e1 = rp[row + 1];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = (lane + ch * lpr) * V;
            if (c0 >= p) continue;
            T lm[V], acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) { lm[v] = lam[c0 + v]; acc[v] = T(0); }
            for (int64_t e = e0; e < e1; ++e) {
                const int64_t j = col[e];
                const auto w = lb[e];
                T x[V];
                load_vec<T, V>(D + j * p + c0, x);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = fma(fma(-lm[v], w.y, w.x), x[v], acc[v]);
            }
            T dv[V];
            load_vec<T, V>(D + row * p + c0, dv);
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (!active[c0 + v]) acc[v] = T(0);
            store_vec<T, V>(Q + row * p + c0, acc);
#pragma unroll
            for (int v = 0; v < V; ++v) dot[ch][v] += (double)dv[v] * (double)acc[v];
        }
    }
    // block reduction over row groups, fixed order
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = (lane + ch * lpr) * V;
        if (c0 < p) {
#pragma unroll
            for (int v = 0; v < V; ++v) red[g * p + c0 + v] = dot[ch][v];
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < groups; ++k) s += red[k * p + c];
        part[(int64_t)blockIdx.x * p + c] = s;
    }
}

// Scalar SpMV with the dot <d, A d> fused (Hartree CG); persistent grid,
// one lane per row, per-block partial written to part[block].
__global__ __launch_bounds__(256) void k_spmv_dot(int64_t n, const int64_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ d,
                                                 double *__restrict__ q,
                                                 double *__restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc = fma(a[e], d[col[e]], acc);
        q[i] = acc;
        s = fma(d[i], acc, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int ilog2_ceil(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

template <typename T> static inline int pick_v(int p) {
    if (sizeof(T) == 8) return (p % 2 == 0) ? 2 : 1;
    return (p % 4 == 0) ? 4 : ((p % 2 == 0) ? 2 : 1);
}

// lanes per row: enough lanes to cover p with V-wide accesses, at most 64
static inline int lpr_log2_for(int p, int v) {
    int l = ilog2_ceil((p + v - 1) / v);
    return l > 6 ? 6 : l;
}

template <typename T>
hipError_t launch_spmm_pair(hipStream_t s, int64_t n, int p, const int64_t *rp, const int32_t *col,
                            const void *ab, const T *X, T *Y1, T *Y2, int sel) {
    using P2 = typename pair_t<T>::type;
    const int v = pick_v<T>(p);
    const int l2 = lpr_log2_for(p, v);
    const int64_t threads = n << l2;
    const int bs = 256;
    const unsigned grid = (unsigned)((threads + bs - 1) / bs);
    const P2 *w = (const P2 *)ab;
    const bool two = Y2 != nullptr;
#define OFKS_SPMM_CASE(VV)                                                                   \
    if (v == VV) {                                                                           \
        if (two) hipLaunchKernelGGL((k_spmm_pair<T, VV, 2>), dim3(grid), dim3(bs), 0, s, n, p, l2, rp, col, w, X, Y1, Y2, sel); \
        else hipLaunchKernelGGL((k_spmm_pair<T, VV, 1>), dim3(grid), dim3(bs), 0, s, n, p, l2, rp, col, w, X, Y1, Y2, sel);   \
        return hipGetLastError();                                                            \
    }
    OFKS_SPMM_CASE(1)
    OFKS_SPMM_CASE(2)
    if constexpr (sizeof(T) == 4) { OFKS_SPMM_CASE(4) }
#undef OFKS_SPMM_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_spmm_shift(hipStream_t s, int grid, int64_t n, int p, const int64_t *rp,
                             const int32_t *col, const void *lb, const T *lam, const uint8_t *active,
                             const T *D, T *Q, double *part) {
    using P2 = typename pair_t<T>::type;
    const int v = pick_v<T>(p);
    const int l2 = lpr_log2_for(p, v);
    const int chunks = (p + (v << l2) - 1) / (v << l2);
    const int bs = 256;
    const size_t shm = (size_t)(bs >> l2) * p * sizeof(double);
    const P2 *w = (const P2 *)lb;
#define OFKS_SHIFT_CASE(VV, CC)                                                              \
    if (v == VV && chunks <= CC) {                                                           \
        hipLaunchKernelGGL((k_spmm_shift<T, VV, CC>), dim3(grid), dim3(bs), shm, s, n, p, l2, rp, col, w, lam, active, D, Q, part); \
        return hipGetLastError();                                                            \
    }
    OFKS_SHIFT_CASE(1, 1)
    OFKS_SHIFT_CASE(1, 2)
    OFKS_SHIFT_CASE(1, 4)
    OFKS_SHIFT_CASE(1, 8)
    OFKS_SHIFT_CASE(2, 1)
    OFKS_SHIFT_CASE(2, 2)
    OFKS_SHIFT_CASE(2, 4)
    OFKS_SHIFT_CASE(2, 8)
    if constexpr (sizeof(T) == 4) {
        OFKS_SHIFT_CASE(4, 1)
        OFKS_SHIFT_CASE(4, 2)
        OFKS_SHIFT_CASE(4, 4)
    }
#undef OFKS_SHIFT_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_spmv_dot(hipStream_t s, int grid, int64_t n, const int64_t *rp, const int32_t *col,
                           const double *a, const double *d, double *q, double *part) {
    hipLaunchKernelGGL(k_spmv_dot, dim3(grid), dim3(256), 0, s, n, rp, col, a, d, q, part);
    return hipGetLastError();
}

template hipError_t launch_spmm_pair<double>(hipStream_t, int64_t, int, const int64_t *, const int32_t *,
                                             const void *, const double *, double *, double *, int);
template hipError_t launch_spmm_pair<float>(hipStream_t, int64_t, int, const int64_t *, const int32_t *,
                                            const void *, const float *, float *, float *, int);
template hipError_t launch_spmm_shift<double>(hipStream_t, int, int64_t, int, const int64_t *,
                                              const int32_t *, const void *, const double *,
                                              const uint8_t *, const double *, double *, double *);
template hipError_t launch_spmm_shift<float>(hipStream_t, int, int64_t, int, const int64_t *,
                                             const int32_t *, const void *, const float *,
                                             const uint8_t *, const float *, float *, double *);

}  // namespace ofks
