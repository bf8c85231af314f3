// Sparse products on the shared P1 CSR pattern.
//
//  k_spmm_pair   : Y1 = A1 X and Y2 = A2 X in one pass (H X and B X, the
//                  "function evaluation" of Algorithm PCAL).  The values of the
//                  two matrices are interleaved per nonzero, so one 16-byte
//                  (f64) or 8-byte (f32) load feeds both products; with one
//                  output the caller selects which of the pair is used.
//  k_spmm_shift  : Q[:,l] = (L/2 - lam_l B) D[:,l] (operator of the paper's
//                  preconditioner T_l, eq. precondition-T) with the per-column
//                  dot products <D_l, Q_l> of the CG step fused in.
//  k_spmv_dot    : q = A d and <d, q> for one vector (Hartree CG).
//
// Work mapping (wave64).  A row is owned by a group of LPR = 2^lpr_log2 lanes;
// each lane covers V consecutive columns (one vector load of an X row slice)
// and CH column chunks when p > LPR*V.  A row's p values are contiguous, so a
// group reads one contiguous X row per nonzero (p = 128 in f64: 1 KB per
// neighbour per wave).
//
// Latency: the neighbours of a row are independent, so the group first loads
// up to LPR (column, weight) pairs with one coalesced access, then broadcasts
// them lane to lane and issues U neighbour loads back to back before any
// arithmetic.  Control flow around the broadcasts is uniform across the wave
// (loop bounds use the wave's longest row; rows past n just have no entries).
#include "common.hpp"

// Tuning: neighbour loads in flight per wave for one-column-chunk rows, and
// whether streamed data (CSR entries read once, outputs written once) use
// non-temporal accesses so that they do not evict reused X rows from L2.
#ifndef OFKS_SPMM_U
#define OFKS_SPMM_U 16
#endif
#ifndef OFKS_SPMM_NT
#define OFKS_SPMM_NT 1
#endif

namespace ofks {

template <typename T> __device__ __forceinline__ T stream_load(const T *p) {
#if OFKS_SPMM_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <typename T, int V>
__device__ __forceinline__ void stream_store_vec(T *__restrict__ p, const T (&in)[V]) {
#if OFKS_SPMM_NT
#pragma unroll
    for (int i = 0; i < V; ++i) __builtin_nontemporal_store(in[i], p + i);
#else
    store_vec<T, V>(p, in);
#endif
}

template <typename T> struct pair_t;
template <> struct pair_t<double> { using type = double2; };
template <> struct pair_t<float> { using type = float2; };

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// a1[ch][v] = sum_e w(e).x X[col e][c], a2 likewise with w(e).y, for the row
// owned by this lane group (cnt entries starting at e0; cnt = 0: no row).
// All 64 lanes of the wave must call this together.
template <typename T, int V, int CH, int U>
__device__ __forceinline__ void gather_row(int64_t e0, int cnt, int lpr_log2, int p,
                                           const int32_t *__restrict__ col,
                                           const typename pair_t<T>::type *__restrict__ w,
                                           const T *__restrict__ X, T (&a1)[CH][V], T (&a2)[CH][V]) {
    using P2 = typename pair_t<T>::type;
    const int lpr = 1 << lpr_log2;
    const int glane = threadIdx.x & (lpr - 1);
    const int lane_in_wave = threadIdx.x & 63;
    const int cmax = wave_max(cnt);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < V; ++v) { a1[ch][v] = T(0); a2[ch][v] = T(0); }
    for (int base = 0; base < cmax; base += lpr) {
        int mycol = 0;
        T mwx = T(0), mwy = T(0);
        if (base + glane < cnt) {
            mycol = col[e0 + base + glane];
            const P2 ww = w[e0 + base + glane];
            mwx = ww.x;
            mwy = ww.y;
        }
        const int kend = min(lpr, cmax - base);   // uniform across the wave
        for (int k0 = 0; k0 < kend; k0 += U) {
            int jj[U];
            T wx[U], wy[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int src = (lane_in_wave & ~(lpr - 1)) + ((k0 + u) & (lpr - 1));
                jj[u] = __shfl(mycol, src, 64);
                wx[u] = __shfl(mwx, src, 64);
                wy[u] = __shfl(mwy, src, 64);
                ok[u] = (k0 + u < kend) && (base + k0 + u < cnt);
            }
            T xb[U][CH][V];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch) {
                    const int c0 = (glane + ch * lpr) * V;
                    if (ok[u] && c0 < p) {
                        load_vec<T, V>(X + (int64_t)jj[u] * p + c0, xb[u][ch]);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) xb[u][ch][v] = T(0);
                    }
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        a1[ch][v] = fma(wx[u], xb[u][ch][v], a1[ch][v]);
                        a2[ch][v] = fma(wy[u], xb[u][ch][v], a2[ch][v]);
                    }
        }
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b on XCD b % 8).
// The logical block index gives each XCD a contiguous range of rows, so the
// neighbour rows a row reads were mostly fetched into the same XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb_padded) {
    return (b % 8) * (nb_padded / 8) + b / 8;
}

template <typename T, int V, int CH, int U, int NOUT>
__global__ __launch_bounds__(256) void k_spmm_pair(int64_t n, int p, int lpr_log2,
                                                  const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const typename pair_t<T>::type *__restrict__ ab,
                                                  const T *__restrict__ X, T *__restrict__ Y1,
                                                  T *__restrict__ Y2, int sel) {
    const int lpr = 1 << lpr_log2;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = (lb * blockDim.x + threadIdx.x) >> lpr_log2;
    const int glane = threadIdx.x & (lpr - 1);
    int64_t e0 = 0;
    int cnt = 0;
    if (row < n) {
        e0 = rp[row];
        cnt = (int)(rp[row + 1] - e0);
    }
    T a1[CH][V], a2[CH][V];
    gather_row<T, V, CH, U>(e0, cnt, lpr_log2, p, col, ab, X, a1, a2);
    if (row >= n) return;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = (glane + ch * lpr) * V;
        if (c0 >= p) continue;
        if (NOUT == 2) {
            store_vec<T, V>(Y1 + row * p + c0, a1[ch]);
            store_vec<T, V>(Y2 + row * p + c0, a2[ch]);
        } else {
            store_vec<T, V>(Y1 + row * p + c0, sel ? a2[ch] : a1[ch]);
        }
    }
}

// Persistent grid: each wave owns a fixed sequence of row groups, so every
// block's share and summation order are fixed by the launch shape and the
// per-block partial dot products (part[b*p + c]) are reproducible.
template <typename T, int V, int CH, int U>
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
    const int glane = threadIdx.x & (lpr - 1);
    const int gpw = 64 >> lpr_log2;   // row groups per wave
    double dot[CH][V];
    T lm[CH][V];
    bool on[CH][V];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = (glane + ch * lpr) * V + v;
            dot[ch][v] = 0.0;
            lm[ch][v] = c < p ? lam[c] : T(0);
            on[ch][v] = c < p ? active[c] != 0 : false;
        }
    // XCD x = blockIdx % 8 sweeps the row slab [x S, (x+1) S); its blocks take
    // consecutive row groups of the slab in rounds.  rb is the first row of
    // this wave in a round and is uniform across the wave.
    const int64_t bpx = gridDim.x / 8;
    const int64_t slab = ((n + 7) / 8 + groups - 1) / groups * groups;
    const int64_t s0 = (blockIdx.x % 8) * slab;
    const int64_t s1 = min(n, s0 + slab);
    const int64_t stride = bpx * groups;
    for (int64_t rb = s0 + (int64_t)(blockIdx.x / 8) * groups + (g & ~(gpw - 1)); rb < s1; rb += stride) {
        const int64_t row = rb + (g & (gpw - 1));
        int64_t e0 = 0;
        int cnt = 0;
        if (row < s1) {
            e0 = rp[row];
            cnt = (int)(rp[row + 1] - e0);
        }
        T a1[CH][V], a2[CH][V];
        gather_row<T, V, CH, U>(e0, cnt, lpr_log2, p, col, lb, D, a1, a2);
        if (row < s1) {
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                const int c0 = (glane + ch * lpr) * V;
                if (c0 >= p) continue;
                T q[V], dv[V];
                load_vec<T, V>(D + row * p + c0, dv);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    q[v] = on[ch][v] ? fma(-lm[ch][v], a2[ch][v], a1[ch][v]) : T(0);
                    dot[ch][v] += (double)dv[v] * (double)q[v];
                }
                store_vec<T, V>(Q + row * p + c0, q);
            }
        }
    }
    // block reduction over row groups, fixed order
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = (glane + ch * lpr) * V;
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

// One wave per row (used when a row's p values need all 64 lanes).  The row
// index is wave-uniform, so the row bounds, column indices and weights are
// scalar loads, and all U neighbour loads of a row go out as one batch before
// the arithmetic.
//
// Locality: with a locality-preserving node numbering the neighbours of a
// row have nearby numbers, so the rows in flight on one XCD must be a narrow
// window of consecutive rows for their neighbour rows to stay in that XCD's
// L2.  Rows go to XCDs in contiguous slabs (block b runs on XCD b % 8).
//  MODE 0 (Y1 = A1 X, Y2 = A2 X, or A2 X into Y1 when sel = 1): one row per
//    wave, blocks in slab order, so the dispatcher sweeps each slab forward.
//  MODE 1 (shifted operator, per-block partial dots part[block][p]):
//    persistent; the launcher sizes the grid to the blocks that can be
//    resident at once, and round r of block j takes rows base + 4 (r B + j),
//    so each round sweeps a window of 4 B consecutive rows per XCD.
template <typename T, int V, int CH, int U, int MODE>
__global__ __launch_bounds__(256) void k_spmm_wave(int64_t n, int p, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const typename pair_t<T>::type *__restrict__ w,
                                                  const T *__restrict__ X, T *__restrict__ Y1,
                                                  T *__restrict__ Y2, int sel, const T *__restrict__ lam,
                                                  const uint8_t *__restrict__ active,
                                                  double *__restrict__ part) {
    using P2 = typename pair_t<T>::type;
    __shared__ double red[4][64 * V * CH];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t row, s1, stride;
    if (MODE == 0) {
        row = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
        s1 = n;
        stride = n;   // one row
    } else {
        const int64_t bpx = gridDim.x / 8;
        const int64_t slab = ((n + 7) / 8 + 3) / 4 * 4;
        const int64_t s0 = (blockIdx.x % 8) * slab;
        s1 = min(n, s0 + slab);
        row = s0 + (int64_t)(blockIdx.x / 8) * 4 + wave;
        stride = bpx * 4;
    }
    double dot[CH][V];
    T lm[CH][V];
    bool on[CH][V];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = (lane + ch * 64) * V + v;
            dot[ch][v] = 0.0;
            if (MODE == 1) {
                lm[ch][v] = c < p ? lam[c] : T(0);
                on[ch][v] = c < p ? active[c] != 0 : false;
            }
        }
    for (; row < s1; row += stride) {
        const int64_t e0 = rp[row], e1 = rp[row + 1];
        T a1[CH][V], a2[CH][V];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int v = 0; v < V; ++v) { a1[ch][v] = T(0); a2[ch][v] = T(0); }
        for (int64_t e = e0; e < e1; e += U) {
            const int m = (int)min((int64_t)U, e1 - e);
            int jj[U];
            T wx[U], wy[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (u < m) {
                    jj[u] = stream_load(col + e + u);
                    wx[u] = stream_load(&w[e + u].x);
                    wy[u] = stream_load(&w[e + u].y);
                } else {
                    jj[u] = 0;
                    wx[u] = T(0);
                    wy[u] = T(0);
                }
            }
            T xb[U][CH][V];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch) {
                    const int c0 = (lane + ch * 64) * V;
                    if (u < m && c0 < p) {
                        load_vec<T, V>(X + (int64_t)jj[u] * p + c0, xb[u][ch]);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) xb[u][ch][v] = T(0);
                    }
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        a1[ch][v] = fma(wx[u], xb[u][ch][v], a1[ch][v]);
                        a2[ch][v] = fma(wy[u], xb[u][ch][v], a2[ch][v]);
                    }
        }
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = (lane + ch * 64) * V;
            if (c0 >= p) continue;
            if (MODE == 0) {
                if (Y2) {
                    stream_store_vec<T, V>(Y1 + row * p + c0, a1[ch]);
                    stream_store_vec<T, V>(Y2 + row * p + c0, a2[ch]);
                } else {
                    stream_store_vec<T, V>(Y1 + row * p + c0, sel ? a2[ch] : a1[ch]);
                }
            } else {
                T q[V], dv[V];
                load_vec<T, V>(X + row * p + c0, dv);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    q[v] = on[ch][v] ? fma(-lm[ch][v], a2[ch][v], a1[ch][v]) : T(0);
                    dot[ch][v] += (double)dv[v] * (double)q[v];
                }
                stream_store_vec<T, V>(Y1 + row * p + c0, q);
            }
        }
    }
    if (MODE == 1) {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int v = 0; v < V; ++v) red[wave][(lane + ch * 64) * V + v] = dot[ch][v];
        __syncthreads();
        for (int c = threadIdx.x; c < p; c += blockDim.x)
            part[(int64_t)blockIdx.x * p + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
}

// blocks of the non-persistent mode (one row per wave), whole XCD slabs
int64_t spmm_wave_blocks(int64_t n) { return ((n + 3) / 4 + 7) / 8 * 8; }

// Persistent grid of the shifted mode: the blocks that fit on the device at
// once (occupancy of this kernel instance), a multiple of 8 and at most cap.
template <typename K> int resident_grid(K kernel, int cap) {
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0);
        int g = cus * (per > 0 ? per : 1);
        g = g / 8 * 8;
        cached = g < 8 ? 8 : g;
    }
    return cached < cap ? cached : cap;
}

// SpMV with the dot <d, A d> fused (Hartree CG); persistent grid, 16 lanes
// per row (P1 rows hold about 15 entries): each lane takes every 16th entry
// of the row with coalesced loads, the 16 partial sums are combined by
// shuffles in a fixed order, and the group's first lane writes q_i and
// accumulates d_i q_i.  Per-block partial written to part[block].
__global__ __launch_bounds__(256) void k_spmv_dot(int64_t n, const int64_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ d,
                                                 double *__restrict__ q,
                                                 double *__restrict__ part) {
    __shared__ double red[256];
    const int sub = threadIdx.x & 15;
    double s = 0.0;
    const int64_t rows_per_pass = (int64_t)gridDim.x * (blockDim.x / 16);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 16) + (threadIdx.x >> 4); i - (threadIdx.x >> 4) < n;
         i += rows_per_pass) {
        double acc = 0.0;
        if (i < n) {
            const int64_t e1 = rp[i + 1];
            for (int64_t e = rp[i] + sub; e < e1; e += 16) acc = fma(a[e], d[col[e]], acc);
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
        if (sub == 0 && i < n) {
            q[i] = acc;
            s = fma(d[i], acc, s);
        }
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
// LDS-halo SpMM.  Block b owns the consecutive rows [row0[b], row0[b+1]) (at
// most HALO_RMAX, each with at most 64 entries) and their halo: the distinct
// columns of those rows together with the rows themselves in ascending order,
// hoff[b+1] - hoff[b] <= HALO_MAX rows of X listed at halo[b HALO_STRIDE ...]
// (padded to the stride with the last one), so the block's rows sit at slots
// rbase[b], rbase[b] + 1, ...  brp[b HALO_BRP + k] is the CSR row pointer of
// row row0[b] + k, for k = 0 .. HALO_RMAX (padded with row0[b+1]'s, so rows
// past the block have no entries).  lcol[e] is the halo slot of CSR entry e.
// Every per-block address depends on b alone: the block's metadata loads all
// issue at once instead of one after another.  Wave v of the block takes rows row0[b] + v + HALO_WAVES i; it
// loads their entries (slot, weight pair) once, one entry per lane, and keeps
// them in registers.  For each 512-byte slice of the columns the block stages
// its halo rows of X in LDS; every wave then forms its rows from LDS, reading
// each row's entries back from a per-wave LDS area at uniform addresses (an
// LDS broadcast).  X is gathered from L2 about (halo size / rows) times
// instead of once per nonzero, and consecutive blocks (one XCD's slab, in
// dispatch order) share their halos in that XCD's L2.
//  MODE 0: Y1 = A1 X and Y2 = A2 X (or, Y2 = NULL, A1 X or A2 X by sel).
//  MODE 1: Y1 = Q = (A1 - lam_c A2) D on active columns (0 elsewhere), and
//          part[b][c] = <D_c, Q_c> over the block's rows.
// ---------------------------------------------------------------------------
// Tunables: halo rows (LDS = HALO_MAX x 512 B), rows per block, waves per
// block, and the waves per SIMD the register budget is cut for (set by how
// many blocks the LDS admits per CU).
#ifndef OFKS_HALO_MAX
#define OFKS_HALO_MAX 76   // with the DMA kernel's separate dot area, three blocks still fit a CU's LDS
#endif
#ifndef OFKS_HALO_RMAX
#define OFKS_HALO_RMAX 16   // an 80-row halo holds about 16 Morton-ordered rows' neighbours anyway
#endif
#ifndef OFKS_HALO_WAVES
#define OFKS_HALO_WAVES 8
#endif
#ifndef OFKS_HALO_DMA
#define OFKS_HALO_DMA 1   // 0: stage every slice through registers (the unaligned-row kernel)
#endif
#ifndef OFKS_HALO_WPE
#define OFKS_HALO_WPE 6
#endif
constexpr int HALO_MAX = OFKS_HALO_MAX, HALO_RMAX = OFKS_HALO_RMAX, HALO_WAVES = OFKS_HALO_WAVES, HALO_EMAX = 64;
constexpr int HALO_RPW = HALO_RMAX / HALO_WAVES;   // rows per wave
// Each block's halo row list is padded to HALO_STRIDE entries (repeating its
// last row), so its address depends on the block index alone: the staging
// threads' row lookups need no offset load first.  Both precisions stage
// 32 sixteen-byte segments per slot, HALO_SST slots per pass.
constexpr int HALO_SST = 64 * HALO_WAVES / 32;
constexpr int HALO_STRIDE = (HALO_MAX + HALO_SST - 1) / HALO_SST * HALO_SST;
constexpr int HALO_BRP = HALO_RMAX + 1;            // per-block row pointer stride
static_assert(HALO_RMAX % HALO_WAVES == 0, "whole rows per wave");


// the register cap keeps every block the LDS admits resident
template <typename T, int MODE>
__global__ __launch_bounds__(64 * HALO_WAVES) __attribute__((amdgpu_waves_per_eu(OFKS_HALO_WPE))) void k_spmm_halo(
    int64_t nb, int p, const int64_t *__restrict__ row0, const int64_t *__restrict__ hoff,
    const int32_t *__restrict__ halo, const int32_t *__restrict__ rbase, const int64_t *__restrict__ brp,
    const uint16_t *__restrict__ lcol,
    const typename pair_t<T>::type *__restrict__ w, const T *__restrict__ X, T *__restrict__ Y1,
    T *__restrict__ Y2, int sel, const T *__restrict__ lam, const uint8_t *__restrict__ active,
    double *__restrict__ part) {
    using P2 = typename pair_t<T>::type;
    constexpr int CP = 512 / sizeof(T);   // columns per slice: 64 (f64) or 128 (f32)
    constexpr int VW = 16 / sizeof(T);    // one 16-byte load
    constexpr int LPC = CP / 64;          // columns per lane in a slice
    constexpr int SEG = CP / VW;
    __shared__ T Xs[HALO_MAX * CP];
    // per-wave broadcast area: the current row's entries, read back by every
    // lane at a uniform address (an LDS broadcast instead of VALU readlanes)
    __shared__ int ent_off[HALO_WAVES][64];
    __shared__ P2 ent_w[HALO_WAVES][64];
    // MODE 1 per-wave dot partials reuse the slice's LDS once it is consumed
    static_assert(HALO_WAVES * CP * sizeof(double) <= sizeof(T) * HALO_MAX * CP, "partials fit in the slice");
    double *red = reinterpret_cast<double *>(Xs);
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (b >= nb) {   // padding block of the XCD mapping: a zero partial row
        if (MODE == 1)
            for (int c = threadIdx.x; c < p; c += blockDim.x) part[b * p + c] = 0.0;
        return;
    }
    // 16-byte loads need every row start 16-byte aligned
    const bool vec = p % VW == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
    // staging: thread t always moves 16-byte segment t % SEG of halo slots
    // t / SEG + SST u; the slots' rows of X are looked up once per block
    constexpr int SST = 64 * HALO_WAVES / SEG;
    constexpr int SPT = (HALO_MAX + SST - 1) / SST;
    static_assert((64 * HALO_WAVES) % SEG == 0, "whole slot rows per pass");
    static_assert(SST == HALO_SST && SPT * SST == HALO_STRIDE, "padded halo stride");
    const int sg = threadIdx.x % SEG, ss = threadIdx.x / SEG;
    // (halo is padded per block; slots past the block's halo repeat its last
    // row and are never stored)
    int hrow[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) hrow[u] = halo[b * HALO_STRIDE + ss + SST * u];
    // the halo loads go out first; the block's metadata loads below then all
    // issue together, without the scheduler sinking the halo loads behind them
    __builtin_amdgcn_sched_barrier(0);
    const int64_t r0 = row0[b], r1 = row0[b + 1];
    const int hn = (int)(hoff[b + 1] - hoff[b]);
    const int rb = MODE == 1 ? rbase[b] : 0;   // the block's rows sit at halo slots rb, rb + 1, ...
    // this wave's rows: entry k of row i sits in lane k (lanes past the row
    // re-read entry 0, which every allocation holds, and are never used)
    int len[HALO_RPW], off[HALO_RPW];
    T wa[HALO_RPW], wb[HALO_RPW];
    const int64_t *bp = brp + b * HALO_BRP;
#pragma unroll
    for (int i = 0; i < HALO_RPW; ++i) {
        const int k = wave + HALO_WAVES * i;
        const int64_t e0 = bp[k];
        len[i] = (int)(bp[k + 1] - e0);
        const int64_t e = lane < len[i] ? e0 + lane : 0;
        const P2 ww = w[e];
        off[i] = (int)lcol[e] * CP;
        wa[i] = ww.x;
        wb[i] = ww.y;
    }
    for (int c0 = 0; c0 < p; c0 += CP) {
        const int c = c0 + sg * VW;
        if (vec && c0 + CP <= p) {
            // whole aligned slice: every load of the slice in flight before
            // the first LDS write
            T v[SPT][VW];
#pragma unroll
            for (int u = 0; u < SPT; ++u) load_vec<T, VW>(X + (int64_t)hrow[u] * p + c, v[u]);
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const int sl = ss + SST * u;
                if (sl < hn) {
#pragma unroll
                    for (int j = 0; j < VW; ++j) Xs[sl * CP + sg * VW + j] = v[u][j];
                }
            }
        } else if (vec) {
            // ragged last slice of aligned rows: p is a multiple of VW, so a
            // segment lies wholly inside or wholly past p.  Segments past p
            // load their row's first segment instead (in bounds, no branch)
            // and store zeros.
            const bool in = c < p;
            const int cc = in ? c : 0;
            T v[SPT][VW];
#pragma unroll
            for (int u = 0; u < SPT; ++u) load_vec<T, VW>(X + (int64_t)hrow[u] * p + cc, v[u]);
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const int sl = ss + SST * u;
                if (sl < hn) {
#pragma unroll
                    for (int j = 0; j < VW; ++j) Xs[sl * CP + sg * VW + j] = in ? v[u][j] : T(0);
                }
            }
        } else {
            // unaligned rows: element loads, zeros past p
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const int sl = ss + SST * u;
                const T *src = X + (int64_t)hrow[u] * p + c;
                if (sl < hn) {
#pragma unroll
                    for (int j = 0; j < VW; ++j) Xs[sl * CP + sg * VW + j] = c + j < p ? src[j] : T(0);
                }
            }
        }
        __syncthreads();
        T lm[LPC];
        bool on[LPC];
        double dot[LPC];
#pragma unroll
        for (int j = 0; j < LPC; ++j) {
            const int c = c0 + lane + 64 * j;
            dot[j] = 0.0;
            lm[j] = (MODE == 1 && c < p) ? lam[c] : T(0);
            on[j] = (MODE == 1 && c < p) ? active[c] != 0 : false;
        }
#pragma unroll
        for (int i = 0; i < HALO_RPW; ++i) {
            const int64_t row = r0 + wave + HALO_WAVES * i;
            if (row >= r1) break;
            T dv[LPC];   // D's own row, staged with the halo
            if (MODE == 1) {
#pragma unroll
                for (int j = 0; j < LPC; ++j) dv[j] = Xs[(rb + (int)(row - r0)) * CP + lane + 64 * j];
            }
            T a1[LPC], a2[LPC];
#pragma unroll
            for (int j = 0; j < LPC; ++j) { a1[j] = T(0); a2[j] = T(0); }
            const int m = len[i];
            // the row's entries into this wave's broadcast area (LDS keeps a
            // wave's accesses in order; the wave barriers keep the compiler's)
            __builtin_amdgcn_wave_barrier();
            ent_off[wave][lane] = off[i];
            ent_w[wave][lane] = P2{wa[i], wb[i]};
            __builtin_amdgcn_wave_barrier();
            constexpr int UN = 4;   // entries in flight per step
            int k = 0;
            for (; k + UN <= m; k += UN) {
                T x[UN][LPC];
                P2 ww[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const int o = ent_off[wave][k + u];
                    ww[u] = ent_w[wave][k + u];
#pragma unroll
                    for (int j = 0; j < LPC; ++j) x[u][j] = Xs[o + lane + 64 * j];
                }
#pragma unroll
                for (int u = 0; u < UN; ++u)
#pragma unroll
                    for (int j = 0; j < LPC; ++j) {
                        a1[j] = fma(ww[u].x, x[u][j], a1[j]);
                        a2[j] = fma(ww[u].y, x[u][j], a2[j]);
                    }
            }
            for (; k < m; ++k) {
                const int o = ent_off[wave][k];
                const P2 ww = ent_w[wave][k];
#pragma unroll
                for (int j = 0; j < LPC; ++j) {
                    const T x = Xs[o + lane + 64 * j];
                    a1[j] = fma(ww.x, x, a1[j]);
                    a2[j] = fma(ww.y, x, a2[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < LPC; ++j) {
                const int c = c0 + lane + 64 * j;
                if (c >= p) continue;
                if (MODE == 0) {
                    if (Y2) {
                        Y1[row * p + c] = a1[j];
                        Y2[row * p + c] = a2[j];
                    } else {
                        Y1[row * p + c] = sel ? a2[j] : a1[j];
                    }
                } else {
                    const T q = on[j] ? fma(-lm[j], a2[j], a1[j]) : T(0);
                    dot[j] += (double)dv[j] * (double)q;
                    Y1[row * p + c] = q;
                }
            }
        }
        __syncthreads();   // the slice is consumed
        if (MODE == 1) {
#pragma unroll
            for (int j = 0; j < LPC; ++j) red[wave * CP + lane + 64 * j] = dot[j];
            __syncthreads();
            for (int cl = threadIdx.x; cl < CP; cl += blockDim.x) {
                const int c = c0 + cl;
                if (c >= p) continue;
                double sum = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < HALO_WAVES; ++k2) sum += red[k2 * CP + cl];
                part[b * p + c] = sum;
            }
            __syncthreads();
        }
    }
}

// The same products for blocks whose rows of X are 16-byte aligned, with the
// halo staged by the direct global-to-LDS loads of gfx950
// (global_load_lds_dwordx4): lane t of a wave instruction writes its 16 bytes
// at the wave's LDS base + 16 t, so a wave fills two consecutive 512-byte
// halo slots (lanes 0-31, 32-63) without passing the data through registers.
// The next slice's loads are issued as soon as every wave has consumed the
// current one, before this slice's results are stored, so the stores stay in
// flight while a wave waits only for its own loads (vector memory operations
// complete in issue order).  The shifted product's per-wave dot partials have
// an LDS area of their own.  Per slice: wait for the own loads, barrier,
// compute, barrier, issue the next slice, store, sum the partials.
// Columns at or past p in a ragged last slice stage in-bounds data of the
// row's first segment; no output reads them (each lane's columns are
// independent).
template <typename T, int MODE>
__global__ __launch_bounds__(64 * HALO_WAVES) __attribute__((amdgpu_waves_per_eu(OFKS_HALO_WPE))) void
k_spmm_halo_dma(int64_t nb, int p, const int64_t *__restrict__ row0, const int64_t *__restrict__ hoff,
                const int32_t *__restrict__ halo, const int32_t *__restrict__ rbase, const int64_t *__restrict__ brp,
                const uint16_t *__restrict__ lcol, const typename pair_t<T>::type *__restrict__ w,
                const T *__restrict__ X, T *__restrict__ Y1, T *__restrict__ Y2, int sel, const T *__restrict__ lam,
                const uint8_t *__restrict__ active, double *__restrict__ part) {
    using P2 = typename pair_t<T>::type;
    constexpr int CP = 512 / sizeof(T);   // columns per slice
    constexpr int VW = 16 / sizeof(T);    // one 16-byte segment
    constexpr int LPC = CP / 64;          // columns per lane in a slice
    constexpr int SEG = CP / VW;          // 32 segments per slot
    constexpr int SST = 64 * HALO_WAVES / SEG;
    constexpr int SPT = (HALO_MAX + SST - 1) / SST;
    static_assert(SEG == 32, "a wave instruction fills two slots");
    static_assert(SST == HALO_SST && SPT * SST == HALO_STRIDE, "padded halo stride");
    // an instruction is issued only when its first (even) slot is below the
    // halo size <= HALO_MAX, so with HALO_MAX even it never writes past it
    static_assert(HALO_MAX % 2 == 0, "even halo capacity");
    __shared__ T Xs[HALO_MAX * CP];
    __shared__ int ent_off[HALO_WAVES][64];
    __shared__ P2 ent_w[HALO_WAVES][64];
    __shared__ double red[MODE == 1 ? HALO_WAVES * CP : 1];
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (b >= nb) {
        if (MODE == 1)
            for (int c = threadIdx.x; c < p; c += blockDim.x) part[b * p + c] = 0.0;
        return;
    }
    const int sg = threadIdx.x % SEG, ss = threadIdx.x / SEG;   // ss = 2 wave + lane / 32
    int hrow[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) hrow[u] = halo[b * HALO_STRIDE + ss + SST * u];
    __builtin_amdgcn_sched_barrier(0);
    const int64_t r0 = row0[b], r1 = row0[b + 1];
    const int hn = (int)(hoff[b + 1] - hoff[b]);
    const int rb = MODE == 1 ? rbase[b] : 0;
    // the wave's rows' entries, loaded with the halo rows; both are pinned in
    // registers before the first halo load is issued (empty asm operands: no
    // instruction), so the compiler neither sinks these loads into the slice
    // loop nor waits between the halo loads (a value loaded before an LDS
    // load that is still in flight is otherwise waited for with vmcnt(0))
    int len[HALO_RPW];
    int lc[HALO_RPW];
    P2 we[HALO_RPW];
    const int64_t *bp = brp + b * HALO_BRP;
#pragma unroll
    for (int i = 0; i < HALO_RPW; ++i) {
        const int k = wave + HALO_WAVES * i;
        const int64_t e0 = bp[k];
        len[i] = (int)(bp[k + 1] - e0);
        const int64_t e = lane < len[i] ? e0 + lane : 0;
        we[i] = w[e];
        lc[i] = (int)lcol[e];
    }
    // staging of the slice at columns c0: wave instruction u fills slots
    // SST u + 2 wave and + 1; instructions wholly past the halo are skipped.
    // All addresses are formed before the first load is issued.
    int64_t hoffs[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
        hoffs[u] = (int64_t)hrow[u] * p;
        asm volatile("" : "+v"(hoffs[u]));
    }
#pragma unroll
    for (int i = 0; i < HALO_RPW; ++i) asm volatile("" : "+v"(lc[i]), "+v"(we[i].x), "+v"(we[i].y));
    auto stage = [&](int c0) {
        const int c = c0 + sg * VW;
        const int cc = c < p ? c : 0;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int s0 = SST * u + 2 * wave;
            if (s0 < hn)
                __builtin_amdgcn_global_load_lds((const void *)(X + hoffs[u] + cc),
                                                 (__attribute__((address_space(3))) void *)(Xs + s0 * CP), 16, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    stage(0);
    for (int c0 = 0; c0 < p; c0 += CP) {
        T lm[LPC];
        bool on[LPC];
#pragma unroll
        for (int j = 0; j < LPC; ++j) {
            const int c = c0 + lane + 64 * j;
            lm[j] = (MODE == 1 && c < p) ? lam[c] : T(0);
            on[j] = (MODE == 1 && c < p) ? active[c] != 0 : false;
        }
        __builtin_amdgcn_s_waitcnt(0);   // this thread's loads (and everything before them)
        __builtin_amdgcn_s_barrier();    // every wave's: the slice is in LDS
        __builtin_amdgcn_sched_barrier(0);
        T q1[HALO_RPW][LPC], q2[HALO_RPW][LPC];
        double dot[LPC];
#pragma unroll
        for (int j = 0; j < LPC; ++j) dot[j] = 0.0;
#pragma unroll
        for (int i = 0; i < HALO_RPW; ++i) {
            const int64_t row = r0 + wave + HALO_WAVES * i;
#pragma unroll
            for (int j = 0; j < LPC; ++j) { q1[i][j] = T(0); q2[i][j] = T(0); }
            if (row >= r1) continue;
            T dv[LPC];
            if (MODE == 1) {
#pragma unroll
                for (int j = 0; j < LPC; ++j) dv[j] = Xs[(rb + (int)(row - r0)) * CP + lane + 64 * j];
            }
            T a1[LPC], a2[LPC];
#pragma unroll
            for (int j = 0; j < LPC; ++j) { a1[j] = T(0); a2[j] = T(0); }
            const int m = len[i];
            __builtin_amdgcn_wave_barrier();
            ent_off[wave][lane] = lc[i];
            ent_w[wave][lane] = we[i];
            __builtin_amdgcn_wave_barrier();
            constexpr int UN = 4;
            int k = 0;
            for (; k + UN <= m; k += UN) {
                T x[UN][LPC];
                P2 ww[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const int o = ent_off[wave][k + u] * CP;
                    ww[u] = ent_w[wave][k + u];
#pragma unroll
                    for (int j = 0; j < LPC; ++j) x[u][j] = Xs[o + lane + 64 * j];
                }
#pragma unroll
                for (int u = 0; u < UN; ++u)
#pragma unroll
                    for (int j = 0; j < LPC; ++j) {
                        a1[j] = fma(ww[u].x, x[u][j], a1[j]);
                        a2[j] = fma(ww[u].y, x[u][j], a2[j]);
                    }
            }
            for (; k < m; ++k) {
                const int o = ent_off[wave][k] * CP;
                const P2 ww = ent_w[wave][k];
#pragma unroll
                for (int j = 0; j < LPC; ++j) {
                    const T x = Xs[o + lane + 64 * j];
                    a1[j] = fma(ww.x, x, a1[j]);
                    a2[j] = fma(ww.y, x, a2[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < LPC; ++j) {
                if (MODE == 0) {
                    q1[i][j] = a1[j];
                    q2[i][j] = a2[j];
                } else {
                    const int c = c0 + lane + 64 * j;
                    const T q = on[j] ? fma(-lm[j], a2[j], a1[j]) : T(0);
                    if (c < p) dot[j] += (double)dv[j] * (double)q;
                    q1[i][j] = q;
                }
            }
        }
        if (MODE == 1) {
#pragma unroll
            for (int j = 0; j < LPC; ++j) red[wave * CP + lane + 64 * j] = dot[j];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // LDS done (lgkmcnt 0); vector memory untouched
        __builtin_amdgcn_s_barrier();         // the slice is consumed and the partials written
        __builtin_amdgcn_sched_barrier(0);
        if (c0 + CP < p) stage(c0 + CP);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < HALO_RPW; ++i) {
            const int64_t row = r0 + wave + HALO_WAVES * i;
            if (row >= r1) continue;
#pragma unroll
            for (int j = 0; j < LPC; ++j) {
                const int c = c0 + lane + 64 * j;
                if (c >= p) continue;
                if (MODE == 0) {
                    if (Y2) {
                        Y1[row * p + c] = q1[i][j];
                        Y2[row * p + c] = q2[i][j];
                    } else {
                        Y1[row * p + c] = sel ? q2[i][j] : q1[i][j];
                    }
                } else {
                    Y1[row * p + c] = q1[i][j];
                }
            }
        }
        if (MODE == 1) {
            for (int cl = threadIdx.x; cl < CP; cl += blockDim.x) {
                const int c = c0 + cl;
                if (c >= p) continue;
                double sum = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < HALO_WAVES; ++k2) sum += red[k2 * CP + cl];
                part[b * p + c] = sum;
            }
        }
    }
}

// out[g][c] = sum of rows [g G, (g + 1) G) of an nb x p partial matrix, in row
// order; threads run over columns, so every read is coalesced.
__global__ __launch_bounds__(256) void k_part_rows(int64_t nb, int p, int G, const double *__restrict__ in,
                                                  double *__restrict__ out) {
    const int64_t g = blockIdx.x;
    const int64_t b0 = g * G, b1 = min(nb, b0 + G);
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        double sum = 0.0;
        for (int64_t b = b0; b < b1; ++b) sum += in[b * p + c];
        out[g * p + c] = sum;
    }
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

// Dispatch over (V, CH); U (neighbour loads in flight) shrinks as CH grows to
// bound registers.
#define OFKS_VCH_DISPATCH(LAUNCH)                                 \
    do {                                                          \
        if (v == 1 && ch <= 1) { LAUNCH(1, 1, 8); break; }        \
        if (v == 1 && ch <= 2) { LAUNCH(1, 2, 8); break; }        \
        if (v == 1 && ch <= 4) { LAUNCH(1, 4, 4); break; }        \
        if (v == 1 && ch <= 8) { LAUNCH(1, 8, 2); break; }        \
        if (v == 2 && ch <= 1) { LAUNCH(2, 1, 8); break; }        \
        if (v == 2 && ch <= 2) { LAUNCH(2, 2, 4); break; }        \
        if (v == 2 && ch <= 4) { LAUNCH(2, 4, 2); break; }        \
        if (v == 2 && ch <= 8) { LAUNCH(2, 8, 1); break; }        \
        if constexpr (sizeof(T) == 4) {                           \
            if (v == 4 && ch <= 1) { LAUNCH(4, 1, 8); break; }    \
            if (v == 4 && ch <= 2) { LAUNCH(4, 2, 4); break; }    \
            if (v == 4 && ch <= 4) { LAUNCH(4, 4, 2); break; }    \
        }                                                         \
        return hipErrorInvalidValue;                              \
    } while (0)

template <typename T>
hipError_t launch_spmm_pair(hipStream_t s, int64_t n, int p, const int64_t *rp, const int32_t *col,
                            const void *ab, const T *X, T *Y1, T *Y2, int sel) {
    using P2 = typename pair_t<T>::type;
    const int v = pick_v<T>(p);
    const int l2 = lpr_log2_for(p, v);
    const int ch = (p + (v << l2) - 1) / (v << l2);
    const P2 *w = (const P2 *)ab;
    if (l2 == 6) {
        const unsigned grid = (unsigned)spmm_wave_blocks(n);
#define OFKS_WAVE0(VV, CC)                                                                                   \
    hipLaunchKernelGGL((k_spmm_wave<T, VV, CC, (CC >= 8 ? 2 : OFKS_SPMM_U / CC), 0>), dim3(grid), dim3(256), 0, s, n, p, rp, col, w, X, Y1, Y2, \
                       sel, (const T *)nullptr, (const uint8_t *)nullptr, (double *)nullptr)
        if (v == 1 && ch == 1) OFKS_WAVE0(1, 1);
        else if (v == 1 && ch <= 2) OFKS_WAVE0(1, 2);
        else if (v == 2 && ch == 1) OFKS_WAVE0(2, 1);
        else if (v == 2 && ch <= 2) OFKS_WAVE0(2, 2);
        else if (v == 2 && ch <= 4) OFKS_WAVE0(2, 4);
        else if (v == 2 && ch <= 8) OFKS_WAVE0(2, 8);
        else if constexpr (sizeof(T) == 4) {
            if (v == 4 && ch == 1) OFKS_WAVE0(4, 1);
            else if (v == 4 && ch <= 2) OFKS_WAVE0(4, 2);
            else if (v == 4 && ch <= 4) OFKS_WAVE0(4, 4);
            else return hipErrorInvalidValue;
        } else return hipErrorInvalidValue;
#undef OFKS_WAVE0
        return hipGetLastError();
    }
    const int64_t threads = n << l2;
    const int bs = 256;
    const unsigned grid = (unsigned)((((threads + bs - 1) / bs) + 7) / 8 * 8);   // multiple of the XCD count
    const bool two = Y2 != nullptr;
#define OFKS_PAIR(VV, CC, UU)                                                                                 \
    if (two) hipLaunchKernelGGL((k_spmm_pair<T, VV, CC, UU, 2>), dim3(grid), dim3(bs), 0, s, n, p, l2, rp, col, w, X, Y1, Y2, sel); \
    else hipLaunchKernelGGL((k_spmm_pair<T, VV, CC, UU, 1>), dim3(grid), dim3(bs), 0, s, n, p, l2, rp, col, w, X, Y1, Y2, sel)
    OFKS_VCH_DISPATCH(OFKS_PAIR);
#undef OFKS_PAIR
    return hipGetLastError();
}

// Launches at most `grid` blocks (the caller's partial buffer holds grid * p
// values) and reports the number used in *blocks_used.
template <typename T>
hipError_t launch_spmm_shift(hipStream_t s, int grid, int64_t n, int p, const int64_t *rp,
                             const int32_t *col, const void *lb, const T *lam, const uint8_t *active,
                             const T *D, T *Q, double *part, int *blocks_used) {
    using P2 = typename pair_t<T>::type;
    if (grid % 8 != 0 || grid < 8) return hipErrorInvalidValue;   // whole XCD slabs
    *blocks_used = grid;
    const int v = pick_v<T>(p);
    const int l2 = lpr_log2_for(p, v);
    const int ch = (p + (v << l2) - 1) / (v << l2);
    const int bs = 256;
    const size_t shm = (size_t)(bs >> l2) * p * sizeof(double);
    const P2 *w = (const P2 *)lb;
    if (l2 == 6) {
#define OFKS_WAVE1(VV, CC)                                                                                   \
    do {                                                                                                     \
        auto kfn = k_spmm_wave<T, VV, CC, (CC >= 8 ? 2 : OFKS_SPMM_U / CC), 1>;                                       \
        const int wgrid = resident_grid(kfn, grid);                                                          \
        *blocks_used = wgrid;                                                                                \
        hipLaunchKernelGGL(kfn, dim3(wgrid), dim3(256), 0, s, n, p, rp, col, w, D, Q, (T *)nullptr, 0, lam,   \
                           active, part);                                                                    \
    } while (0)
        if (v == 1 && ch == 1) OFKS_WAVE1(1, 1);
        else if (v == 1 && ch <= 2) OFKS_WAVE1(1, 2);
        else if (v == 2 && ch == 1) OFKS_WAVE1(2, 1);
        else if (v == 2 && ch <= 2) OFKS_WAVE1(2, 2);
        else if (v == 2 && ch <= 4) OFKS_WAVE1(2, 4);
        else if (v == 2 && ch <= 8) OFKS_WAVE1(2, 8);
        else if constexpr (sizeof(T) == 4) {
            if (v == 4 && ch == 1) OFKS_WAVE1(4, 1);
            else if (v == 4 && ch <= 2) OFKS_WAVE1(4, 2);
            else if (v == 4 && ch <= 4) OFKS_WAVE1(4, 4);
            else return hipErrorInvalidValue;
        } else return hipErrorInvalidValue;
#undef OFKS_WAVE1
        return hipGetLastError();
    }
#define OFKS_SHIFT(VV, CC, UU) \
    hipLaunchKernelGGL((k_spmm_shift<T, VV, CC, UU>), dim3(grid), dim3(bs), shm, s, n, p, l2, rp, col, w, lam, active, D, Q, part)
    OFKS_VCH_DISPATCH(OFKS_SHIFT);
#undef OFKS_SHIFT
    return hipGetLastError();
}

hipError_t launch_spmv_dot(hipStream_t s, int grid, int64_t n, const int64_t *rp, const int32_t *col,
                           const double *a, const double *d, double *q, double *part) {
    hipLaunchKernelGGL(k_spmv_dot, dim3(grid), dim3(256), 0, s, n, rp, col, a, d, q, part);
    return hipGetLastError();
}

// Halo-SpMM launch: nb blocks of the plan (grid padded to whole XCD slabs).
// MODE 1 leaves the per-block dots after room for ceil(nbp / HALO_G) group
// sums in part; launch_halo_part_rows then writes the group sums to its start
// and the caller's column sum takes *rows_out rows.  part_capacity in doubles.
constexpr int HALO_G = 64;
static int64_t halo_grid(int64_t nb) { return (nb + 7) / 8 * 8; }

size_t spmm_halo_part_doubles(int64_t nb, int p) {
    const int64_t nbp = halo_grid(nb);
    return (size_t)((nbp + HALO_G - 1) / HALO_G + nbp) * p;
}

template <typename T>
hipError_t launch_spmm_halo(hipStream_t s, int mode, int64_t nb, int p, const int64_t *row0, const int64_t *hoff,
                            const int32_t *halo, const int32_t *rbase, const int64_t *brp, const uint16_t *lcol,
                            const void *wv,
                            const T *X, T *Y1, T *Y2, int sel, const T *lam, const uint8_t *active, double *part,
                            size_t part_capacity, int *rows_out) {
    using P2 = typename pair_t<T>::type;
    const P2 *w = (const P2 *)wv;
    const int64_t nbp = halo_grid(nb);
    if (nbp <= 0 || nbp > 0x7fffffff) return hipErrorInvalidValue;
    // rows of X 16-byte aligned: the DMA-staged kernel
    const bool dma = OFKS_HALO_DMA && p % (16 / (int)sizeof(T)) == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
    if (mode == 0) {
        if (dma)
            hipLaunchKernelGGL((k_spmm_halo_dma<T, 0>), dim3((unsigned)nbp), dim3(64 * HALO_WAVES), 0, s, nb, p, row0,
                               hoff, halo, rbase, brp, lcol, w, X, Y1, Y2, sel, lam, active, part);
        else
            hipLaunchKernelGGL((k_spmm_halo<T, 0>), dim3((unsigned)nbp), dim3(64 * HALO_WAVES), 0, s, nb, p, row0,
                               hoff, halo, rbase, brp, lcol, w, X, Y1, Y2, sel, lam, active, part);
        return hipGetLastError();
    }
    const int64_t ng = (nbp + HALO_G - 1) / HALO_G;
    if ((size_t)(ng + nbp) * p > part_capacity) return hipErrorInvalidValue;
    double *bpart = part + ng * p;
    if (dma)
        hipLaunchKernelGGL((k_spmm_halo_dma<T, 1>), dim3((unsigned)nbp), dim3(64 * HALO_WAVES), 0, s, nb, p, row0, hoff,
                           halo, rbase, brp, lcol, w, X, Y1, (T *)nullptr, 0, lam, active, bpart);
    else
        hipLaunchKernelGGL((k_spmm_halo<T, 1>), dim3((unsigned)nbp), dim3(64 * HALO_WAVES), 0, s, nb, p, row0, hoff,
                           halo, rbase, brp, lcol, w, X, Y1, (T *)nullptr, 0, lam, active, bpart);
    *rows_out = (int)ng;
    return hipGetLastError();
}

// The group sums of a MODE 1 halo launch's per-block dots (fixed order).
hipError_t launch_halo_part_rows(hipStream_t s, int64_t nb, int p, double *part) {
    const int64_t nbp = halo_grid(nb), ng = (nbp + HALO_G - 1) / HALO_G;
    hipLaunchKernelGGL(k_part_rows, dim3((unsigned)ng), dim3(256), 0, s, nbp, p, HALO_G, part + ng * p, part);
    return hipGetLastError();
}

template hipError_t launch_spmm_halo<double>(hipStream_t, int, int64_t, int, const int64_t *, const int64_t *,
                                             const int32_t *, const int32_t *, const int64_t *, const uint16_t *,
                                             const void *,
                                             const double *, double *, double *, int, const double *,
                                             const uint8_t *, double *, size_t, int *);
template hipError_t launch_spmm_halo<float>(hipStream_t, int, int64_t, int, const int64_t *, const int64_t *,
                                            const int32_t *, const int32_t *, const int64_t *, const uint16_t *,
                                            const void *,
                                            const float *, float *, float *, int, const float *, const uint8_t *,
                                            double *, size_t, int *);
int halo_max_rows() { return HALO_MAX; }
int halo_max_block_rows() { return HALO_RMAX; }
int halo_max_row_entries() { return HALO_EMAX; }
int halo_pad_stride() { return HALO_STRIDE; }
int halo_row_ptr_stride() { return HALO_BRP; }

template hipError_t launch_spmm_pair<double>(hipStream_t, int64_t, int, const int64_t *, const int32_t *,
                                             const void *, const double *, double *, double *, int);
template hipError_t launch_spmm_pair<float>(hipStream_t, int64_t, int, const int64_t *, const int32_t *,
                                            const void *, const float *, float *, float *, int);
template hipError_t launch_spmm_shift<double>(hipStream_t, int, int64_t, int, const int64_t *,
                                              const int32_t *, const void *, const double *,
                                              const uint8_t *, const double *, double *, double *, int *);
template hipError_t launch_spmm_shift<float>(hipStream_t, int, int64_t, int, const int64_t *,
                                             const int32_t *, const void *, const float *,
                                             const uint8_t *, const float *, float *, double *, int *);

}  // namespace ofks
