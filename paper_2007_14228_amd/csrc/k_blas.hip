// Block (n x p) kernels of the PCAL iteration.
//
//  k_gram        X^T [BX | HX] as split-K partial tiles (Algorithm PCAL,
//                eq. lambda2 needs S = X^T B X and Lambda0 = X^T H X).
//  k_colsum      fixed-order reduction of per-block partials.
//  k_rowgemm     [G | R] = (BX D^-1) [C | C'] + (HX D^-1) with the update
//                epilogues (gradient of L_beta, residual norm for kkt, the
//                start of the preconditioner's CG or the column norms of G
//                for the learned form), or a plain Y = X M.
//  k_pcg_r       r -= alpha q, <r, J r>                  (inner CG step)
//  k_pcg_dx      x += alpha d and d = J r + beta d
//  k_pcg_scalars alpha / beta per column on the device
//  k_bbdot       <S,Y>, <Y,Y>, <S,S>, ||P||^2, ||X||^2 for the BB step
//  k_update_b    X~ = X - P / eta with X = X~ D^-1; keeps X as X^{k-1}
//  k_coldot      per-column sums of A .* B (column B-norms)
//
// Every reduction writes per-block partials that a fixed-order pass sums, so
// results do not depend on scheduling.
#include "common.hpp"

namespace ofks {

// ---------------------------------------------------------------------------
// Gram: part[split][a][c] = sum_{rows of split} X[r][a] * Y[r][c],
// Y = [BX | HX] (c < p -> BX[:, c], else HX[:, c - p]).
// Tile (16*MT) x (16*NT), 256 threads as 16 x 16, thread (ty, tx) owns rows
// a = a0 + ty + 16 i and columns c = c0 + tx + 16 j.
// ---------------------------------------------------------------------------
template <typename T, typename ACC, int MT, int NT>
__global__ __launch_bounds__(256) void k_gram(int64_t n, int p, int64_t rows_per_split,
                                             const T *__restrict__ X, const T *__restrict__ BX,
                                             const T *__restrict__ HX, double *__restrict__ part) {
    constexpr int TM = 16 * MT, TN = 16 * NT, KC = 16;
    __shared__ T As[KC][TM];
    __shared__ T Bs[KC][TN];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int a0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
    const int64_t r_begin = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r_end = min(n, r_begin + rows_per_split);
    const int p2 = 2 * p;
    ACC acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = ACC(0);

    for (int64_t r0 = r_begin; r0 < r_end; r0 += KC) {
        for (int idx = threadIdx.x; idx < KC * TM; idx += 256) {
            const int kr = idx / TM, cc = idx % TM;
            const int64_t r = r0 + kr;
            const int a = a0 + cc;
            As[kr][cc] = (r < r_end && a < p) ? X[r * p + a] : T(0);
        }
        for (int idx = threadIdx.x; idx < KC * TN; idx += 256) {
            const int kr = idx / TN, cc = idx % TN;
            const int64_t r = r0 + kr;
            const int c = c0 + cc;
            T v = T(0);
            if (r < r_end && c < p2) v = (c < p) ? BX[r * p + c] : HX[r * p + (c - p)];
            Bs[kr][cc] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            ACC av[MT], bv[NT];
#pragma unroll
            for (int i = 0; i < MT; ++i) av[i] = (ACC)As[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < NT; ++j) bv[j] = (ACC)Bs[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
    double *out = part + (int64_t)blockIdx.z * p * p2;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int a = a0 + ty + 16 * i;
        if (a >= p) continue;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int c = c0 + tx + 16 * j;
            if (c < p2) out[(int64_t)a * p2 + c] = (double)acc[i][j];
        }
    }
}

// out[m] = sum_{b < nb} part[b * m_total + m] for m in [0, m_total); one block
// per output, fixed strided partition then a fixed tree.
__global__ __launch_bounds__(256) void k_colsum(int64_t nb, int64_t m_total,
                                               const double *__restrict__ part,
                                               double *__restrict__ out) {
    __shared__ double red[256];
    const int64_t m = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) s += part[b * m_total + m];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[m] = red[0];
}

// ---------------------------------------------------------------------------
// Row GEMM with epilogues.  out[r][c] = sum_k A[r][k] sa[k] M[k][c] (+ addend)
// for c in [0, N).  Tile: 16*MT rows x 16*NT columns; thread (ty, tx) owns
// rows r0 + ty + 16 i, columns c0 + tx + 16 j.  Persistent over row tiles.
// ---------------------------------------------------------------------------
enum { EPI_PLAIN = 0, EPI_GRAD = 1, EPI_GRAD_PCG = 2, EPI_GRAD_NORM = 3 };

// the directions of the inner CG's history form (k_pcg_sum), by value
constexpr int PCG_DIRS_MAX = 16;
struct PcgDirs {
    const void *d[PCG_DIRS_MAX];
};

struct GradArgs {
    const void *HX;       // n x p, unnormalized (scaled by dinv here)
    void *P;              // out: gradient (no CG) / identity-branch columns
    void *R;              // out: CG residual r = G (active columns)
    void *D;              // out: CG direction d = J G (active columns)
    const double *lhd;    // diag(L/2), n
    const double *bd;     // diag(B), n
    const void *lam;      // shift lambda_c of T_c, p
    const uint8_t *active;// column uses the CG preconditioner
    double *part;         // per block: [0] ||R||^2, [1 + c] <r_c, J r_c>
};

template <typename T, int MT, int NT, int EPI>
__global__ __launch_bounds__(256) void k_rowgemm(int64_t n, int p, int N, const T *__restrict__ A,
                                                const T *__restrict__ sa,
                                                const T *__restrict__ M, T *__restrict__ Y,
                                                GradArgs ga) {
    constexpr int TR = 16 * MT, TC = 16 * NT, KC = 16;
    __shared__ T As[TR][KC + 1];
    __shared__ T Ms[KC][TC];
    __shared__ double red[256];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int c0 = blockIdx.y * TC;
    const int64_t ntiles = (n + TR - 1) / TR;
    double r2 = 0.0;
    double rz[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) rz[j] = 0.0;
    const T *HX = (const T *)ga.HX;
    const T *lamv = (const T *)ga.lam;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * TR;
        T acc[MT][NT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = T(0);
        for (int k0 = 0; k0 < p; k0 += KC) {
            for (int idx = threadIdx.x; idx < TR * KC; idx += 256) {
                const int rr = idx / KC, kk = idx % KC;
                const int64_t r = r0 + rr;
                const int k = k0 + kk;
                As[rr][kk] = (r < n && k < p) ? A[r * p + k] * sa[k] : T(0);
            }
            for (int idx = threadIdx.x; idx < KC * TC; idx += 256) {
                const int kk = idx / TC, cc = idx % TC;
                const int k = k0 + kk, c = c0 + cc;
                Ms[kk][cc] = (k < p && c < N) ? M[(int64_t)k * N + c] : T(0);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                T av[MT], mv[NT];
#pragma unroll
                for (int i = 0; i < MT; ++i) av[i] = As[ty + 16 * i][kk];
#pragma unroll
                for (int j = 0; j < NT; ++j) mv[j] = Ms[kk][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j) acc[i][j] = fma(av[i], mv[j], acc[i][j]);
            }
            __syncthreads();
        }
        // epilogue
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int64_t r = r0 + ty + 16 * i;
            if (r >= n) continue;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int c = c0 + tx + 16 * j;
                if (c >= N) continue;
                if (EPI == EPI_PLAIN) {
                    Y[r * N + c] = acc[i][j];
                } else {
                    const int cc = c < p ? c : c - p;
                    const T v = fma(HX[r * p + cc], sa[cc], acc[i][j]);
                    if (c >= p) {
                        r2 += (double)v * (double)v;
                    } else if (EPI == EPI_GRAD) {
                        ((T *)ga.P)[r * p + c] = v;
                    } else if (EPI == EPI_GRAD_NORM) {
                        ((T *)ga.P)[r * p + c] = v;
                        rz[j] += (double)v * (double)v;
                    } else {  // EPI_GRAD_PCG
                        if (ga.active[c]) {
                            const T jinv = T(1) / (T(ga.lhd[r]) - lamv[c] * T(ga.bd[r]));
                            const T z = v * jinv;
                            ((T *)ga.R)[r * p + c] = v;
                            ((T *)ga.D)[r * p + c] = z;
                            rz[j] += (double)v * (double)z;
                        } else {
                            ((T *)ga.P)[r * p + c] = v;
                        }
                    }
                }
            }
        }
    }
    if (EPI == EPI_PLAIN) return;
    // block partials: red over all threads for r2; per column for rz
    double *part = ga.part + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * (1 + p);
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[0] = red[0];
    __syncthreads();
    if (EPI == EPI_GRAD_PCG || EPI == EPI_GRAD_NORM) {
        for (int c = threadIdx.x; c < p; c += 256)
            if (c < c0 || c >= c0 + TC) part[1 + c] = 0.0;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            red[threadIdx.x] = rz[j];
            __syncthreads();
            if (ty == 0) {
                double s = 0.0;
                for (int k = 0; k < 16; ++k) s += red[k * 16 + tx];
                const int c = c0 + tx + 16 * j;
                if (c < p) part[1 + c] = s;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// The same row GEMM on the matrix cores (16x16x4 MFMA, FP64 or FP32).
// Block: 4 waves, 64 rows x TC = 16 NTW columns; wave w owns rows 16w..16w+15
// of the tile and all NTW 16x16 output tiles.  A (scaled by sa) and M are
// staged through LDS in K-chunks of 16 (zero-filled past p, N and n), so any
// shape works; the next chunk's values are loaded into registers while the
// current chunk's MFMAs run.  Operand layout of the 16x16x4 instructions (lane l, measured
// on gfx950): A[l % 16][l / 16], B[l / 16][l % 16]; result slot i < 4 holds
// D[4 (l / 16) + i][l % 16] for f32 and D[l / 16 + 4 i][l % 16] for f64.
// Epilogues and per-block partials as in k_rowgemm.
// ---------------------------------------------------------------------------
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct mfma4;
template <> struct mfma4<double> { using type = mfma_d4; };
template <> struct mfma4<float> { using type = mfma_f4; };
__device__ __forceinline__ mfma_d4 mfma16x16x4(double a, double b, mfma_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfma_f4 mfma16x16x4(float a, float b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// row (within the 16 x 16 tile) of result slot i of lane group lk = l / 16
template <typename T> __device__ __forceinline__ int mfma_row(int lk, int i) {
    return sizeof(T) == 8 ? lk + 4 * i : 4 * lk + i;
}

// Gram on the matrix cores: the same split-K partial tiles as k_gram, tile
// TM x TN = 128 x 128, the 4 waves as 2 x 2, each owning 64 x 64 (4 x 4
// MFMA tiles).  Rows of X and Y are staged through a double-buffered LDS in
// chunks of 16, the next chunk's loads in flight while the current one is
// multiplied (one barrier per chunk).  Here the A operand is X^T (a = column
// of X, k = row) and B is Y.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_mfma(int64_t n, int p, int64_t rows_per_split,
                                                  const T *__restrict__ X, const T *__restrict__ BX,
                                                  const T *__restrict__ HX, double *__restrict__ part) {
    constexpr int TM = 128, TN = 128, KC = 16, PAD = 4;
    constexpr int EX = KC * TM / 256, EY = KC * TN / 256;
    using acc_t = typename mfma4<T>::type;
    __shared__ T Xs[2][KC][TM + PAD];
    __shared__ T Ys[2][KC][TN + PAD];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wy = w >> 1, wx = w & 1;
    const int a0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
    const int64_t r_begin = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r_end = min(n, r_begin + rows_per_split);
    const int p2 = 2 * p;
    acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{T(0), T(0), T(0), T(0)};
    T xr[EX], yr[EY];
    auto gload = [&](int64_t r0) {
#pragma unroll
        for (int j = 0; j < EX; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int kk = e / TM, cc = e % TM;
            const int64_t r = r0 + kk;
            const int a = a0 + cc;
            xr[j] = (r < r_end && a < p) ? X[r * p + a] : T(0);
        }
#pragma unroll
        for (int j = 0; j < EY; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int kk = e / TN, cc = e % TN;
            const int64_t r = r0 + kk;
            const int c = c0 + cc;
            T v = T(0);
            if (r < r_end && c < p2) v = c < p ? BX[r * p + c] : HX[r * p + (c - p)];
            yr[j] = v;
        }
    };
    auto lstore = [&](int b) {
#pragma unroll
        for (int j = 0; j < EX; ++j) {
            const int e = threadIdx.x + 256 * j;
            Xs[b][e / TM][e % TM] = xr[j];
        }
#pragma unroll
        for (int j = 0; j < EY; ++j) {
            const int e = threadIdx.x + 256 * j;
            Ys[b][e / TN][e % TN] = yr[j];
        }
    };
    int buf = 0;
    if (r_begin < r_end) {
        gload(r_begin);
        lstore(0);
    }
    __syncthreads();
    for (int64_t r0 = r_begin; r0 < r_end; r0 += KC) {
        const bool more = r0 + KC < r_end;
        if (more) gload(r0 + KC);
#pragma unroll
        for (int s4 = 0; s4 < KC / 4; ++s4) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Xs[buf][4 * s4 + lk][64 * wy + 16 * i + li];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Ys[buf][4 * s4 + lk][64 * wx + 16 * j + li];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(a[i], b[j], acc[i][j]);
        }
        if (more) lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    double *out = part + (int64_t)blockIdx.z * p * p2;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + 64 * wx + 16 * j + li;
            if (c >= p2) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int a = a0 + 64 * wy + 16 * i + mfma_row<T>(lk, q);
                if (a < p) out[(int64_t)a * p2 + c] = (double)acc[i][j][q];
            }
        }
}

#ifndef OFKS_RG_KC
#define OFKS_RG_KC 16   // K values staged per LDS round
#endif
// Register budget for two waves per SIMD.  Left unconstrained, the compiler
// takes up to 252 registers (FP64) and 184 (FP32), two waves either way;
// with this budget the allocation comes to 187 and 128 (four FP32 waves),
// measured faster at p = 128: FP64 5.33 -> 5.12 ms, FP32 3.08 -> 2.28 ms.
// A three-wave budget spills in FP64 and is slower (5.59 ms).
#ifndef OFKS_RG_WPE
#define OFKS_RG_WPE 2
#endif
// CT column tiles per block: with CT = 2 a 512-thread block computes both
// 16 NTW-column tiles of its row tile (waves 0-3 the first, 4-7 the second),
// so A (and the epilogue's HX) is read once for 2 TC output columns instead
// of once per column tile.
// (FP32 blocks: four waves per SIMD, which the two-tile block needs asked for
// explicitly; the one-tile block reaches it within the two-wave budget.)
template <typename T, int NTW, int EPI, int CT>
__global__ __launch_bounds__(256 * CT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && CT == 2 ? 4 : OFKS_RG_WPE)))
void k_rowgemm_mfma(int64_t n, int p, int N, const T *__restrict__ A, const T *__restrict__ sa,
                    const T *__restrict__ M, T *__restrict__ Y, GradArgs ga) {
    constexpr int TR = 64, TC = 16 * NTW, KC = OFKS_RG_KC, TCB = TC * CT, NTH = 256 * CT;
    using acc_t = typename mfma4<T>::type;
    // two LDS buffers: chunk f + 1 is stored into one while chunk f is read
    // from the other, so a chunk needs one barrier instead of two
    __shared__ T As[2][TR][KC + 1];
    __shared__ T Ms[2][KC][TCB];
    __shared__ double red[NTH];
    // per-column epilogue constants of this block's columns, fixed for the
    // launch (in LDS rather than registers: it keeps more waves resident)
    __shared__ T scl_s[TCB], lmc_s[TCB];
    __shared__ uint8_t act_s[TCB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = w & 3, ct = w >> 2;   // row group and column tile of this wave
    const int li = lane & 15, lk = lane >> 4;
    const int c0 = blockIdx.y * TCB;
    const int cw = ct * TC;              // this wave's first column within the block
    const int64_t ntiles = (n + TR - 1) / TR;
    double r2 = 0.0;
    double rz[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) rz[t] = 0.0;
    for (int cl = threadIdx.x; cl < TCB; cl += NTH) {
        const int c = c0 + cl;
        const int cc = c < p ? c : c - p;
        scl_s[cl] = (EPI != EPI_PLAIN && c < N) ? sa[cc] : T(0);
        lmc_s[cl] = (EPI == EPI_GRAD_PCG && c < p) ? ((const T *)ga.lam)[c] : T(0);
        act_s[cl] = (EPI == EPI_GRAD_PCG && c < p) ? ga.active[c] : 0;
    }
    __syncthreads();
    const T *__restrict__ HX = (const T *)ga.HX;
    T *__restrict__ Pout = (T *)ga.P;
    T *__restrict__ Rout = (T *)ga.R;
    T *__restrict__ Dout = (T *)ga.D;

    // K-chunk staging, software-pipelined: the values of the next chunk (of
    // this tile, or the next tile's first) are loaded into registers before
    // the current chunk's MFMAs and stored to LDS after them.
    // Threads 0-255 move AR consecutive k of one A row; every thread moves MR
    // consecutive columns of one M row (of column tile tid / 256) per chunk
    // (16-byte loads when the chunk is whole and the rows are 16-byte
    // aligned; element loads with bounds otherwise).
    constexpr int AR = TR * KC / 256, MR = KC * TC / 256;
    static_assert(AR * 256 == TR * KC && MR * 256 == KC * TC && KC % AR == 0 && TC % MR == 0, "chunk split");
    constexpr int VWT = 16 / sizeof(T);
    static_assert(AR % VWT == 0 && MR % VWT == 0, "16-byte pieces");
    const int tm = threadIdx.x & 255;
    const bool a_mover = threadIdx.x < 256;
    const int a_rr = tm * AR / KC, a_kk = tm * AR % KC;
    const int m_kk = tm * MR / TC, m_cc = tm * MR % TC + (threadIdx.x >> 8) * TC;
    const bool avec = p % VWT == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0;
    const bool mvec = N % VWT == 0 && reinterpret_cast<uintptr_t>(M) % 16 == 0 && c0 + TCB <= N;
    T ar[AR], mr[MR];
    auto load_chunk = [&](int64_t tile, int k0) {
        const bool kin = k0 + KC <= p;
        if (a_mover) {
            const int64_t r = tile * TR + a_rr;
            if (avec && kin && r < n) {
#pragma unroll
                for (int q = 0; q < AR; q += VWT)
                    load_vec<T, VWT>(A + r * p + k0 + a_kk + q, *reinterpret_cast<T(*)[VWT]>(&ar[q]));
            } else {
#pragma unroll
                for (int j = 0; j < AR; ++j) ar[j] = (r < n && k0 + a_kk + j < p) ? A[r * p + k0 + a_kk + j] : T(0);
            }
#pragma unroll
            for (int j = 0; j < AR; ++j) ar[j] = k0 + a_kk + j < p ? ar[j] * sa[k0 + a_kk + j] : T(0);
        }
        const int k = k0 + m_kk;
        if (mvec && kin) {
#pragma unroll
            for (int q = 0; q < MR; q += VWT)
                load_vec<T, VWT>(M + (int64_t)k * N + c0 + m_cc + q, *reinterpret_cast<T(*)[VWT]>(&mr[q]));
        } else {
#pragma unroll
            for (int j = 0; j < MR; ++j) mr[j] = (k < p && c0 + m_cc + j < N) ? M[(int64_t)k * N + c0 + m_cc + j] : T(0);
        }
    };
    auto store_chunk = [&](int sb) {
        if (a_mover) {
#pragma unroll
            for (int j = 0; j < AR; ++j) As[sb][a_rr][a_kk + j] = ar[j];
        }
#pragma unroll
        for (int j = 0; j < MR; ++j) Ms[sb][m_kk][m_cc + j] = mr[j];
    };
    int buf = 0;
    if ((int64_t)blockIdx.x < ntiles) {
        load_chunk(blockIdx.x, 0);
        store_chunk(0);
    }
    __syncthreads();

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * TR;
        acc_t acc[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) acc[t] = acc_t{T(0), T(0), T(0), T(0)};
        for (int k0 = 0; k0 < p; k0 += KC) {
            const bool last = k0 + KC >= p;
            const int64_t nt = last ? tile + gridDim.x : tile;
            const bool more = nt < ntiles;
            if (more) load_chunk(nt, last ? 0 : k0 + KC);
#pragma unroll
            for (int s4 = 0; s4 < KC / 4; ++s4) {
                const T a = As[buf][16 * wr + li][4 * s4 + lk];
#pragma unroll
                for (int t = 0; t < NTW; ++t) acc[t] = mfma16x16x4(a, Ms[buf][4 * s4 + lk][cw + 16 * t + li], acc[t]);
            }
            if (more) store_chunk(buf ^ 1);   // last read in the previous chunk, before its barrier
            __syncthreads();
            buf ^= 1;
        }
        // epilogue: lane holds rows r0 + 16 wr + mfma_row(lk, i) of column c0 + cw + 16 t + li
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + 16 * wr + mfma_row<T>(lk, i);
            if (r >= n) continue;
            T ld = T(0), bdv = T(0);
            if (EPI == EPI_GRAD_PCG) {
                ld = T(ga.lhd[r]);
                bdv = T(ga.bd[r]);
            }
            T hx[NTW];
            if (EPI != EPI_PLAIN) {
#pragma unroll
                for (int t = 0; t < NTW; ++t) {
                    const int c = c0 + cw + 16 * t + li;
                    hx[t] = c < N ? HX[r * p + (c < p ? c : c - p)] : T(0);
                }
            }
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                const int cl = cw + 16 * t + li;
                const int c = c0 + cl;
                if (c >= N) continue;
                const T val = acc[t][i];
                if (EPI == EPI_PLAIN) {
                    Y[r * N + c] = val;
                    continue;
                }
                const T v = fma(hx[t], scl_s[cl], val);
                if (c >= p) {
                    r2 += (double)v * (double)v;
                } else if (EPI == EPI_GRAD) {
                    Pout[r * p + c] = v;
                } else if (EPI == EPI_GRAD_NORM) {
                    Pout[r * p + c] = v;
                    rz[t] += (double)v * (double)v;
                } else {  // EPI_GRAD_PCG
                    if (act_s[cl]) {
                        const T z = v * (T(1) / (ld - lmc_s[cl] * bdv));
                        Rout[r * p + c] = v;
                        Dout[r * p + c] = z;
                        rz[t] += (double)v * (double)z;
                    } else {
                        Pout[r * p + c] = v;
                    }
                }
            }
        }
    }
    if (EPI == EPI_PLAIN) return;
    double *part = ga.part + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * (1 + p);
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int s = NTH / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[0] = red[0];
    __syncthreads();
    if (EPI == EPI_GRAD_PCG || EPI == EPI_GRAD_NORM) {
        for (int c = threadIdx.x; c < p; c += NTH)
            if (c < c0 || c >= c0 + TCB) part[1 + c] = 0.0;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            red[threadIdx.x] = rz[t];   // [ct][wr][lk][li]
            __syncthreads();
            if (threadIdx.x < 16 * CT) {
                const int tc = threadIdx.x >> 4, l = threadIdx.x & 15;
                double sum = 0.0;
                for (int k = 0; k < 16; ++k) sum += red[tc * 256 + k * 16 + l];
                const int c = c0 + tc * TC + 16 * t + l;
                if (c < p) part[1 + c] = sum;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// The gradient row GEMM with the multiplier resident in LDS (p = 64 or 128,
// N = 2p, K = p).  The block stages its TCB = 16 NT output columns of
// diag(sa) M once, for all K (135 KB for FP64 at p = 128, where each block
// holds one of the two 128-column halves; FP32 and p = 64 hold all N
// columns).  Each wave then owns whole 16-row tiles, with no barrier in its
// loop, so that the two waves of a SIMD drift apart and one's loads and
// epilogue overlap the other's MFMAs.  Per tile, a wave:
//  - issues the tile's HX (and diagonal) loads, which land during its MFMAs;
//  - runs KG x 4 x NT MFMAs on the A rows it holds in registers (16-byte
//    loads, lane (li, lk) holding k = 16 j + 4 lk + m, m < 4), with B read
//    from LDS at the same k;
//  - runs the epilogue, then issues the next tile's A loads.
// Scheduling barriers keep the LDS reads of one (j, m) step from being
// hoisted above the previous step: all in flight at once would not fit the
// registers.  The column sums (PCG start, column norms) are reduced over the
// wave after each tile and kept per wave in LDS, the residual sum per
// thread in LDS, so neither holds registers through the MFMAs.
// With two halves, blocks b and b + 8 (one XCD) take the two halves of the
// same row tiles in the same order; the counters still show A and HX fetched
// from beyond L2 once per half.  The K order inside one MFMA is permuted (any order
// of the 4 k values of an instruction gives the same sum up to rounding).
// LDS layout of the staged multiplier: element (k, c) at
// (k / 4) KS + (k % 4) TCB + c, with the k/4 stride padded by 16 values so
// that the four lane groups lk of one read fall on different banks.
// Partial sums per block as in k_rowgemm_mfma (one grid row).
// ---------------------------------------------------------------------------
template <typename T, int NT, int KG, int HALVES, int EPI>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void k_rowgemm_mres(int64_t n, const T *__restrict__ A, const T *__restrict__ sa, const T *__restrict__ M,
                    GradArgs ga) {
    constexpr int P = 16 * KG, N = 2 * P, TCB = 16 * NT, VW = 16 / (int)sizeof(T), KS = 4 * TCB + 16;
    static_assert(TCB * HALVES == N, "column split");
    using acc_t = typename mfma4<T>::type;
    __shared__ T Ms[4 * KG * KS];
    __shared__ T scl_s[TCB], lmc_s[TCB];
    __shared__ uint8_t act_s[TCB];
    __shared__ double red[512];
    // per wave and column: sum over its tiles of the epilogue's column sums
    __shared__ double rzs[8][NT][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = blockIdx.x;
    const int h = HALVES == 2 ? (b >> 3) & 1 : 0;
    const int64_t q = HALVES == 2 ? (int64_t)(((b >> 4) << 3) | (b & 7)) : (int64_t)b;
    const int64_t nq = HALVES == 2 ? gridDim.x / 2 : gridDim.x;
    const int c0 = h * TCB;

    // diag(sa) M, columns c0 .. c0 + TCB - 1, all P rows
    for (int e = threadIdx.x; e < P * TCB; e += 512) {
        const int k = e / TCB, c = e - k * TCB;
        Ms[(k >> 2) * KS + (k & 3) * TCB + c] = sa[k] * M[k * N + c0 + c];
    }
    for (int cl = threadIdx.x; cl < TCB; cl += 512) {
        const int c = c0 + cl;
        const int cc = c < P ? c : c - P;
        scl_s[cl] = sa[cc];
        lmc_s[cl] = (EPI == EPI_GRAD_PCG && c < P) ? ((const T *)ga.lam)[c] : T(0);
        act_s[cl] = (EPI == EPI_GRAD_PCG && c < P) ? ga.active[c] : 0;
    }
    __syncthreads();
    const T *__restrict__ HX = (const T *)ga.HX;
    T *__restrict__ Pout = (T *)ga.P;
    T *__restrict__ Rout = (T *)ga.R;
    T *__restrict__ Dout = (T *)ga.D;
    // columns of this block below P (gradient) or at and above P (residual):
    // per tile t, known at compile time with one column set, per block with two
    const bool low_half = HALVES == 2 ? h == 0 : true;
    auto is_grad = [&](int t) __attribute__((always_inline)) {
        return HALVES == 2 ? low_half : (16 * t < P);
    };
    // HX column (and output column, below P) of tile t, less li
    auto hcol = [](int t) __attribute__((always_inline)) {
        return HALVES == 2 ? 16 * t : (16 * t < P ? 16 * t : 16 * t - P);
    };

    red[threadIdx.x] = 0.0;   // this thread's running sum of squared residual entries
    if (lk == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t) rzs[w][t][li] = 0.0;
    }
    T a[KG][4];
    // rows past n read row n - 1 (their results are dropped)
    auto load_a = [&](int64_t wt) __attribute__((always_inline)) {
        int64_t r = wt * 16 + li;
        if (r > n - 1) r = n - 1;
        const T *src = A + r * P + 4 * lk;
#pragma unroll
        for (int j = 0; j < KG; ++j)
#pragma unroll
            for (int v = 0; v < 4; v += VW)
                load_vec<T, VW>(src + 16 * j + v, *reinterpret_cast<T(*)[VW]>(&a[j][v]));
    };
    const int64_t nwt = (n + 15) / 16;
    const int64_t stride = nq * 8;
    int64_t wt = q * 8 + w;
    if (wt < nwt) load_a(wt);
    for (; wt < nwt; wt += stride) {
        // this tile's HX values (and diagonals), in flight during the MFMAs
        // (lane l holds the diagonals of row l % 16; the epilogue shuffles)
        T hx[4][NT];
        double ldl = 0.0, bdl = 0.0;
        if (EPI == EPI_GRAD_PCG) {
            int64_t r = wt * 16 + li;
            if (r > n - 1) r = n - 1;
            ldl = ga.lhd[r];
            bdl = ga.bd[r];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int64_t r = wt * 16 + mfma_row<T>(lk, i);
            if (r > n - 1) r = n - 1;
            const T *hrow = HX + r * P + li;
#pragma unroll
            for (int t = 0; t < NT; ++t) hx[i][t] = hrow[hcol(t)];
        }
        __builtin_amdgcn_sched_barrier(0);
        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc_t{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < KG; ++j)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const T *mrow = Ms + (4 * j + lk) * KS + m * TCB + li;
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma16x16x4(a[j][m], mrow[16 * t], acc[t]);
                // keeps the LDS reads of later steps from being hoisted here
                // (all of them in flight at once would not fit the registers)
                __builtin_amdgcn_sched_barrier(0);
            }
        // epilogue: lane holds rows 16 wt + mfma_row(lk, i) of columns c0 + 16 t + li
        double rz[NT], r2 = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) rz[t] = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = wt * 16 + mfma_row<T>(lk, i);
            T ldi = T(0), bdi = T(0);
            if (EPI == EPI_GRAD_PCG) {   // all lanes take part in the shuffles
                ldi = T(__shfl(ldl, mfma_row<T>(lk, i)));
                bdi = T(__shfl(bdl, mfma_row<T>(lk, i)));
            }
            if (r >= n) continue;
            T *prow = Pout + r * P + li;
            T *rrow = Rout + r * P + li;
            T *drow = Dout + r * P + li;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int cl = 16 * t + li;
                const int hc = hcol(t);
                const T v = fma(hx[i][t], scl_s[cl], acc[t][i]);
                if (!is_grad(t)) {
                    r2 += (double)v * (double)v;
                } else if (EPI == EPI_GRAD) {
                    prow[hc] = v;
                } else if (EPI == EPI_GRAD_NORM) {
                    prow[hc] = v;
                    rz[t] += (double)v * (double)v;
                } else {  // EPI_GRAD_PCG
                    if (act_s[cl]) {
                        const T z = v * (T(1) / (ldi - lmc_s[cl] * bdi));
                        rrow[hc] = v;
                        drow[hc] = z;
                        rz[t] += (double)v * (double)z;
                    } else {
                        prow[hc] = v;
                    }
                }
            }
        }
        red[threadIdx.x] += r2;
        if (EPI == EPI_GRAD_PCG || EPI == EPI_GRAD_NORM) {
            // the 4 lane groups' sums of each column, then this wave's running sum
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                double v = rz[t];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (lk == 0) rzs[w][t][li] += v;
            }
        }
        if (wt + stride < nwt) load_a(wt + stride);
    }
    double *part = ga.part + (int64_t)blockIdx.x * (1 + P);
    __syncthreads();
    for (int s = 256; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[0] = red[0];
    __syncthreads();
    if (EPI == EPI_GRAD_PCG || EPI == EPI_GRAD_NORM) {
        for (int c = threadIdx.x; c < P; c += 512)
            if (c < c0 || c >= c0 + TCB) part[1 + c] = 0.0;
        for (int cl = threadIdx.x; cl < TCB; cl += 512) {
            const int c = c0 + cl;
            double sum = 0.0;
            for (int ww = 0; ww < 8; ++ww) sum += rzs[ww][cl >> 4][cl & 15];
            if (c < P) part[1 + c] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Lane-per-column-slice kernels over n x p blocks (same mapping as SpMM).
// ---------------------------------------------------------------------------

// Inner CG of the paper preconditioner, split so that each block pass does
// as much as the reductions allow:
//   k_pcg_r   r -= alpha q, partial <r, J r>                (reads q, r; writes r)
//   k_pcg_dx  x += alpha d, then d = J r + beta d          (reads d, r, x; writes d, x)
//             or, in the last inner iteration, x += alpha d only
// Per-column constants are held in registers; columns that are not active
// (identity branch of eq. precondition-T) keep their stored x.

// r -= alpha q on active columns; per-block partial <r, J r>.  Persistent.
template <typename T, int V, int CH>
__global__ __launch_bounds__(256) void k_pcg_r(int64_t n, int p, int lpr_log2, const T *__restrict__ alpha,
                                              const uint8_t *__restrict__ active,
                                              const double *__restrict__ lhd, const double *__restrict__ bd,
                                              const T *__restrict__ lam, const T *__restrict__ Q,
                                              T *__restrict__ R, double *__restrict__ part) {
    extern __shared__ double red[];
    const int lpr = 1 << lpr_log2;
    const int groups = blockDim.x >> lpr_log2;
    const int g = threadIdx.x >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    double dot[CH][V];
    T al[CH][V], lm[CH][V];
    bool on[CH][V];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = (lane + ch * lpr) * V + v;
            on[ch][v] = c < p && active[c];
            dot[ch][v] = 0.0;
            al[ch][v] = on[ch][v] ? alpha[c] : T(0);   // inactive: r unchanged
            lm[ch][v] = c < p ? lam[c] : T(0);
        }
    for (int64_t row = (int64_t)blockIdx.x * groups + g; row < n; row += (int64_t)gridDim.x * groups) {
        const T ld = (T)lhd[row], bdv = (T)bd[row];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = (lane + ch * lpr) * V;
            if (c0 >= p) continue;
            T q[V], r[V];
            load_vec<T, V>(Q + row * p + c0, q);
            load_vec<T, V>(R + row * p + c0, r);
#pragma unroll
            for (int v = 0; v < V; ++v) {   // selects, not branches, per column
                r[v] = fma(-al[ch][v], q[v], r[v]);
                const double t = (double)r[v] * (double)(r[v] / (ld - lm[ch][v] * bdv));
                dot[ch][v] = on[ch][v] ? dot[ch][v] + t : dot[ch][v];
            }
            store_vec<T, V>(R + row * p + c0, r);
        }
    }
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

// x = (first ? 0 : x) + alpha d on active columns; with DIR also
// d = J r + beta d.  One lane group per row.
template <typename T, int V, int DIR>
__global__ __launch_bounds__(256) void k_pcg_dx(int64_t n, int p, int lpr_log2, int first,
                                               const T *__restrict__ alpha, const T *__restrict__ beta,
                                               const uint8_t *__restrict__ active,
                                               const double *__restrict__ lhd, const double *__restrict__ bd,
                                               const T *__restrict__ lam, const T *__restrict__ R,
                                               T *__restrict__ D, T *__restrict__ X) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    const T ld = (T)lhd[row], bdv = (T)bd[row];
    for (int c0 = lane * V; c0 < p; c0 += lpr * V) {
        bool on[V], all = true, any = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            on[v] = active[c0 + v] != 0;
            all &= on[v];
            any |= on[v];
        }
        if (!any) continue;
        T d[V], x[V], r[V];
        load_vec<T, V>(D + row * p + c0, d);
        if (DIR) load_vec<T, V>(R + row * p + c0, r);
        if (first && all) {
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = T(0);
        } else {
            load_vec<T, V>(X + row * p + c0, x);
        }
        T a[V], bt[V], lm[V];
        load_vec<T, V>(alpha + c0, a);
        if (DIR) {
            load_vec<T, V>(beta + c0, bt);
            load_vec<T, V>(lam + c0, lm);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {   // selects, not branches, per column
            const T nx = first ? a[v] * d[v] : fma(a[v], d[v], x[v]);
            x[v] = on[v] ? nx : x[v];
            if (DIR) {
                const T nd = fma(bt[v], d[v], r[v] / (ld - lm[v] * bdv));
                d[v] = on[v] ? nd : d[v];
            }
        }
        store_vec<T, V>(X + row * p + c0, x);
        if (DIR) store_vec<T, V>(D + row * p + c0, d);
    }
}

// History form of the inner CG (memory permitting): each direction gets a
// block of its own, so no pass reads and rewrites x; P = sum_j alpha_j d_j is
// formed once after the last iteration (the same fmas, in the same order, as
// the running update x += alpha_j d_j of k_pcg_dx, so the same bits).
//   k_pcg_dnext  Dn = J r + beta D on active columns          (reads r, D; writes Dn)
//   k_pcg_sum    X = sum_j alpha_j D_j on active columns      (reads the m D_j; writes X)
template <typename T, int V>
__global__ __launch_bounds__(256) void k_pcg_dnext(int64_t n, int p, int lpr_log2, const T *__restrict__ beta,
                                                  const uint8_t *__restrict__ active,
                                                  const double *__restrict__ lhd, const double *__restrict__ bd,
                                                  const T *__restrict__ lam, const T *__restrict__ R,
                                                  const T *__restrict__ D, T *__restrict__ Dn) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    const T ld = (T)lhd[row], bdv = (T)bd[row];
    for (int c0 = lane * V; c0 < p; c0 += lpr * V) {
        bool on[V], any = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            on[v] = active[c0 + v] != 0;
            any |= on[v];
        }
        if (!any) continue;
        T d[V], r[V];
        load_vec<T, V>(D + row * p + c0, d);
        load_vec<T, V>(R + row * p + c0, r);
        T bt[V], lm[V];
        load_vec<T, V>(beta + c0, bt);
        load_vec<T, V>(lam + c0, lm);
#pragma unroll
        for (int v = 0; v < V; ++v) {   // a select, not a branch, per column
            const T nd = fma(bt[v], d[v], r[v] / (ld - lm[v] * bdv));
            d[v] = on[v] ? nd : d[v];
        }
        store_vec<T, V>(Dn + row * p + c0, d);
    }
}

// G directions j0 .. j0 + G - 1 of one lane's V columns: all G loads issued
// before the first fma (no branch between them), then the fmas in order of j
template <int G, typename T, int V>
__device__ __forceinline__ void pcg_sum_group(int j0, int64_t off, int p, int c0, const T *__restrict__ alpha,
                                              const PcgDirs &dirs, const bool (&on)[V], T (&x)[V]) {
    T d[G][V];
#pragma unroll
    for (int u = 0; u < G; ++u) load_vec<T, V>((const T *)dirs.d[j0 + u] + off, d[u]);
#pragma unroll
    for (int u = 0; u < G; ++u) {
        T al[V];
        load_vec<T, V>(alpha + (int64_t)(j0 + u) * p + c0, al);
        const bool first = j0 + u == 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T nv = first ? al[v] * d[u][v] : fma(al[v], d[u][v], x[v]);
            x[v] = on[v] ? nv : x[v];
        }
    }
}

template <typename T, int V>
__global__ __launch_bounds__(256) void k_pcg_sum(int64_t n, int p, int lpr_log2, int m, const T *__restrict__ alpha,
                                                const uint8_t *__restrict__ active, PcgDirs dirs,
                                                T *__restrict__ X) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    for (int c0 = lane * V; c0 < p; c0 += lpr * V) {
        bool on[V], all = true, any = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            on[v] = active[c0 + v] != 0;
            all &= on[v];
            any |= on[v];
        }
        if (!any) continue;
        T x[V];
        if (all) {
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = T(0);
        } else {
            load_vec<T, V>(X + row * p + c0, x);
        }
        // the directions in groups of 8, then 4, 2, 1 (m = 10: 8 + 2)
        const int64_t off = row * p + c0;
        int j = 0;
        for (; j + 8 <= m; j += 8) pcg_sum_group<8>(j, off, p, c0, alpha, dirs, on, x);
        if (j + 4 <= m) { pcg_sum_group<4>(j, off, p, c0, alpha, dirs, on, x); j += 4; }
        if (j + 2 <= m) { pcg_sum_group<2>(j, off, p, c0, alpha, dirs, on, x); j += 2; }
        if (j < m) pcg_sum_group<1>(j, off, p, c0, alpha, dirs, on, x);
        store_vec<T, V>(X + row * p + c0, x);
    }
}

// alpha_c = rz_c / dq_c (0 when dq_c <= 0);  beta_c = rz_new_c / rz_c (0 when rz_c <= 0).
template <typename T>
__global__ void k_pcg_alpha(int p, const double *__restrict__ dq, const double *__restrict__ rz,
                            T *__restrict__ alpha) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < p) alpha[c] = dq[c] > 0.0 ? (T)(rz[c] / dq[c]) : T(0);
}

template <typename T>
__global__ void k_pcg_beta(int p, const double *__restrict__ rz_new, double *__restrict__ rz,
                           T *__restrict__ beta) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < p) {
        beta[c] = rz[c] > 0.0 ? (T)(rz_new[c] / rz[c]) : T(0);
        rz[c] = rz_new[c];
    }
}

// BB sums.  x = Xt .* dinv; s = x - Xp; y = P - Pp.
// part[block][5] = {<s,y>, <y,y>, <s,s>, <P,P>, <x,x>}; Xp/Pp may be null.
template <typename T, int V, int CH>
__global__ __launch_bounds__(256) void k_bbdot(int64_t n, int p, int lpr_log2,
                                              const T *__restrict__ Xt, const T *__restrict__ dinv,
                                              const T *__restrict__ P, const T *__restrict__ Xp,
                                              const T *__restrict__ Pp, double *__restrict__ part) {
    __shared__ double red[5][256];
    const int lpr = 1 << lpr_log2;
    const int groups = blockDim.x >> lpr_log2;
    const int g = threadIdx.x >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    double s5[5] = {0, 0, 0, 0, 0};
    const bool hist = Xp != nullptr;
    for (int64_t row = (int64_t)blockIdx.x * groups + g; row < n; row += (int64_t)gridDim.x * groups) {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = (lane + ch * lpr) * V;
            if (c0 >= p) continue;
            T xt[V], pv[V];
            load_vec<T, V>(Xt + row * p + c0, xt);
            load_vec<T, V>(P + row * p + c0, pv);
            T xp[V], pp[V];
            if (hist) {
                load_vec<T, V>(Xp + row * p + c0, xp);
                load_vec<T, V>(Pp + row * p + c0, pp);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double x = (double)(xt[v] * dinv[c0 + v]);
                const double pd = (double)pv[v];
                s5[3] += pd * pd;
                s5[4] += x * x;
                if (hist) {
                    const double s = x - (double)xp[v];
                    const double y = pd - (double)pp[v];
                    s5[0] += s * y;
                    s5[1] += y * y;
                    s5[2] += s * s;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s5[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 5) part[(int64_t)blockIdx.x * 5 + threadIdx.x] = red[threadIdx.x][0];
}

// Xp = Xt .* dinv ; Xt = Xp - P / eta
template <typename T, int V>
__global__ __launch_bounds__(256) void k_update_b(int64_t n, int p, int lpr_log2,
                                                 const T *__restrict__ dinv, T eta,
                                                 const T *__restrict__ P, T *__restrict__ Xt,
                                                 T *__restrict__ Xp) {
    const int lpr = 1 << lpr_log2;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lpr_log2;
    const int lane = threadIdx.x & (lpr - 1);
    if (row >= n) return;
    for (int c0 = lane * V; c0 < p; c0 += lpr * V) {
        T xt[V], pv[V], x[V], xn[V];
        load_vec<T, V>(Xt + row * p + c0, xt);
        load_vec<T, V>(P + row * p + c0, pv);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            x[v] = xt[v] * dinv[c0 + v];
            xn[v] = x[v] - pv[v] / eta;
        }
        if (Xp) store_vec<T, V>(Xp + row * p + c0, x);
        store_vec<T, V>(Xt + row * p + c0, xn);
    }
}

// per-column sums of A .* B (and of A .* A when AA is set), persistent;
// part[block][p] (or [block][2p]).
template <typename T, int V, int CH>
__global__ __launch_bounds__(256) void k_coldot(int64_t n, int p, int lpr_log2,
                                               const T *__restrict__ A, const T *__restrict__ B,
                                               double *__restrict__ part) {
    extern __shared__ double red[];
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
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = (lane + ch * lpr) * V;
            if (c0 >= p) continue;
            T a[V], b[V];
            load_vec<T, V>(A + row * p + c0, a);
            load_vec<T, V>(B + row * p + c0, b);
#pragma unroll
            for (int v = 0; v < V; ++v) dot[ch][v] += (double)a[v] * (double)b[v];
        }
    }
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

// Y = X .* s (column scale), optionally converting the element type
template <typename S, typename D>
__global__ void k_scale_copy(int64_t n, int p, const S *__restrict__ X, const S *__restrict__ sc,
                             D *__restrict__ Y) {
    const int64_t m = n * p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        Y[i] = (D)(X[i] * sc[i % p]);
}

// Start of the columnwise CG of the preconditioner from x = 0:
// r = G, d = J G on active columns, P = G on the others; part[block][p] = <r, J r>.
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, int p, const uint8_t *__restrict__ active,
                                                 const double *__restrict__ lhd,
                                                 const double *__restrict__ bd, const T *__restrict__ lam,
                                                 const T *__restrict__ G, T *__restrict__ R,
                                                 T *__restrict__ D, T *__restrict__ P,
                                                 double *__restrict__ part) {
    extern __shared__ double red[];   // [256]
    for (int c = 0; c < p; ++c) {
        double s = 0.0;
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
             r += (int64_t)gridDim.x * blockDim.x) {
            const T g = G[r * p + c];
            if (active[c]) {
                const T z = g / (T(lhd[r]) - lam[c] * T(bd[r]));
                R[r * p + c] = g;
                D[r * p + c] = z;
                s += (double)g * (double)z;
            } else {
                P[r * p + c] = g;
            }
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * p + c] = red[0];
        __syncthreads();
    }
}

// f32 <-> f64 block conversion
template <typename S, typename D>
__global__ void k_convert(int64_t m, const S *__restrict__ a, D *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (D)a[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int ilog2c(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}
template <typename T> static inline int vwidth(int p) {
    if (sizeof(T) == 8) return (p % 2 == 0) ? 2 : 1;
    return (p % 4 == 0) ? 4 : ((p % 2 == 0) ? 2 : 1);
}
static inline int lpr_l2(int p, int v) {
    int l = ilog2c((p + v - 1) / v);
    return l > 6 ? 6 : l;
}

// Split-K plan of k_gram: output tiles (gx x gy) and row splits, so that the
// caller can size the partial buffer (splits * p * 2p doubles) before launch.
struct GramPlan {
    int mt, nt, gx, gy;
    int64_t splits, rows_per_split;
};

GramPlan gram_plan(int64_t n, int p, int target_blocks) {
    GramPlan g{};
    if (p <= 16) { g.mt = 1; g.nt = 2; }
    else if (p <= 32) { g.mt = 2; g.nt = 4; }
    else if (p <= 64) { g.mt = 4; g.nt = 4; }
    else { g.mt = 8; g.nt = 8; }
    const int tm = 16 * g.mt, tn = 16 * g.nt;
    g.gx = (p + tm - 1) / tm;
    g.gy = (2 * p + tn - 1) / tn;
    int64_t splits = target_blocks / (g.gx * g.gy);
    if (splits < 1) splits = 1;
    int64_t rps = (n + splits - 1) / splits;
    rps = ((rps + 15) / 16) * 16;
    if (rps < 16) rps = 16;
    splits = (n + rps - 1) / rps;
    if (splits < 1) splits = 1;
    g.splits = splits;
    g.rows_per_split = rps;
    return g;
}

template <typename T>
hipError_t launch_gram(hipStream_t s, int64_t n, int p, const GramPlan &g, const T *X, const T *BX,
                       const T *HX, double *part, size_t part_capacity) {
    if ((size_t)g.splits * (size_t)p * 2 * p > part_capacity) return hipErrorInvalidValue;
    if (g.splits > 65535) return hipErrorInvalidValue;
    dim3 grid(g.gx, g.gy, (unsigned)g.splits);
    using ACC = T;
    const int64_t rps = g.rows_per_split;
    if (g.mt == 1) hipLaunchKernelGGL((k_gram<T, ACC, 1, 2>), grid, dim3(256), 0, s, n, p, rps, X, BX, HX, part);
    else if (g.mt == 2) hipLaunchKernelGGL((k_gram<T, ACC, 2, 4>), grid, dim3(256), 0, s, n, p, rps, X, BX, HX, part);
    else if (g.mt == 4) hipLaunchKernelGGL((k_gram<T, ACC, 4, 4>), grid, dim3(256), 0, s, n, p, rps, X, BX, HX, part);
    else hipLaunchKernelGGL((k_gram_mfma<T>), grid, dim3(256), 0, s, n, p, rps, X, BX, HX, part);
    return hipGetLastError();
}

hipError_t launch_colsum(hipStream_t s, int64_t nb, int64_t m, const double *part, double *out) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)m), dim3(256), 0, s, nb, m, part, out);
    return hipGetLastError();
}

// Column tile width of k_rowgemm for N output columns (16 * NT).
#ifndef OFKS_RG_TC_MAX
#define OFKS_RG_TC_MAX 128
#endif
int rowgemm_tile_cols(int N) {
    const int tc = N <= 16 ? 16 : (N <= 32 ? 32 : (N <= 64 ? 64 : (N <= 128 ? 128 : 256)));
    return tc < OFKS_RG_TC_MAX ? tc : OFKS_RG_TC_MAX;
}

// Column tiles per block of the MFMA row GEMM: two 128-column tiles in one
// 512-thread block from N = 256 on (A and HX then read once per 256 output
// columns), one otherwise.
#ifndef OFKS_RG_CT
#define OFKS_RG_CT 2
#endif
int rowgemm_col_tiles(int N) { return (OFKS_RG_CT == 2 && rowgemm_tile_cols(N) == 128 && N >= 256) ? 2 : 1; }

// blocks along the output columns of launch_rowgemm (its partial sums are
// gemm_rows x this many blocks)
int rowgemm_grid_y(int N) {
    const int w = rowgemm_tile_cols(N) * rowgemm_col_tiles(N);
    return (N + w - 1) / w;
}

// The LDS-resident-multiplier row GEMM (gradient epilogues, N = 2p, p = 64 or
// 128, 16-byte aligned A).  Off with -DOFKS_RG_MRES=0.
#ifndef OFKS_RG_MRES
#define OFKS_RG_MRES 1
#endif
// FP32 blocks at p = 128: 0 the chunked kernel, 1 all 256 columns per block,
// 2 two 128-column halves
#ifndef OFKS_RG_MRES_F32
#define OFKS_RG_MRES_F32 1
#endif
template <typename T, int NT, int KG, int HALVES, int EPI>
static int mres_grid(int cap) {
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_rowgemm_mres<T, NT, KG, HALVES, EPI>, 512, 0);
        cached = cus * (per > 0 ? per : 1);
    }
    int g = cached < cap ? cached : cap;
    return g / 16 * 16;   // whole pairs of 8-block XCD groups (the two halves)
}

template <typename T, int NT, int KG, int HALVES>
static hipError_t launch_mres(hipStream_t s, int epi, int64_t n, int cap, const T *A, const T *sa, const T *M,
                              GradArgs ga, int *gx_out) {
#define OFKS_MRES(E_)                                                                         \
    if (epi == E_) {                                                                          \
        const int g = mres_grid<T, NT, KG, HALVES, E_>(cap);                                  \
        if (g < 16) return hipErrorInvalidValue;                                              \
        if (gx_out) *gx_out = g;                                                              \
        hipLaunchKernelGGL((k_rowgemm_mres<T, NT, KG, HALVES, E_>), dim3(g), dim3(512), 0, s, n, A, sa, M, ga); \
        return hipGetLastError();                                                             \
    }
    OFKS_MRES(EPI_GRAD)
    OFKS_MRES(EPI_GRAD_NORM)
    OFKS_MRES(EPI_GRAD_PCG)
#undef OFKS_MRES
    return hipErrorInvalidValue;
}

// number of blocks along rows for k_rowgemm epilogues (fixed => deterministic)
template <typename T>
hipError_t launch_rowgemm(hipStream_t s, int epi, int64_t n, int p, int N, int grid_rows, const T *A,
                          const T *sa, const T *M, T *Y, GradArgs ga, int *gx_out) {
    if (OFKS_RG_MRES && epi != EPI_PLAIN && N == 2 * p && (p == 64 || p == 128) && n > 0 &&
        !(sizeof(T) == 4 && p == 128 && OFKS_RG_MRES_F32 == 0) &&
        rowgemm_grid_y(N) == 1 && grid_rows >= 16 && reinterpret_cast<uintptr_t>(A) % 16 == 0) {
        if (p == 128) {
            if constexpr (sizeof(T) == 8) return launch_mres<T, 8, 8, 2>(s, epi, n, grid_rows, A, sa, M, ga, gx_out);
            else if (OFKS_RG_MRES_F32 == 2) return launch_mres<T, 8, 8, 2>(s, epi, n, grid_rows, A, sa, M, ga, gx_out);
            else if (OFKS_RG_MRES_F32 == 1) return launch_mres<T, 16, 8, 1>(s, epi, n, grid_rows, A, sa, M, ga, gx_out);
        }
        return launch_mres<T, 8, 4, 1>(s, epi, n, grid_rows, A, sa, M, ga, gx_out);
    }
    const int tc = rowgemm_tile_cols(N);
    const int nt = tc / 16;
    const int mt = 4;
    const int tr = 16 * mt;
    const int64_t ntiles = (n + tr - 1) / tr;
    int gx = grid_rows;
    if (gx > ntiles) gx = (int)ntiles;
    if (gx < 1) gx = 1;
    const int ct = rowgemm_col_tiles(N);
    const int gy = (N + tc * ct - 1) / (tc * ct);
    if (gx_out) *gx_out = gx;
    dim3 grid(gx, gy);
#define OFKS_RG(MT_, NT_)                                                                     \
    if (nt == NT_ && mt == MT_) {                                                             \
        if (epi == EPI_PLAIN) hipLaunchKernelGGL((k_rowgemm<T, MT_, NT_, EPI_PLAIN>), grid, dim3(256), 0, s, n, p, N, A, sa, M, Y, ga); \
        else if (epi == EPI_GRAD) hipLaunchKernelGGL((k_rowgemm<T, MT_, NT_, EPI_GRAD>), grid, dim3(256), 0, s, n, p, N, A, sa, M, Y, ga); \
        else if (epi == EPI_GRAD_NORM) hipLaunchKernelGGL((k_rowgemm<T, MT_, NT_, EPI_GRAD_NORM>), grid, dim3(256), 0, s, n, p, N, A, sa, M, Y, ga); \
        else hipLaunchKernelGGL((k_rowgemm<T, MT_, NT_, EPI_GRAD_PCG>), grid, dim3(256), 0, s, n, p, N, A, sa, M, Y, ga); \
        return hipGetLastError();                                                             \
    }
    OFKS_RG(4, 1)
    OFKS_RG(4, 2)
#undef OFKS_RG
#define OFKS_RGM(NTW_, CT_)                                                                   \
    if (nt == NTW_ && ct == CT_) {                                                            \
        if (epi == EPI_PLAIN) hipLaunchKernelGGL((k_rowgemm_mfma<T, NTW_, EPI_PLAIN, CT_>), grid, dim3(256 * CT_), 0, s, n, p, N, A, sa, M, Y, ga); \
        else if (epi == EPI_GRAD) hipLaunchKernelGGL((k_rowgemm_mfma<T, NTW_, EPI_GRAD, CT_>), grid, dim3(256 * CT_), 0, s, n, p, N, A, sa, M, Y, ga); \
        else if (epi == EPI_GRAD_NORM) hipLaunchKernelGGL((k_rowgemm_mfma<T, NTW_, EPI_GRAD_NORM, CT_>), grid, dim3(256 * CT_), 0, s, n, p, N, A, sa, M, Y, ga); \
        else hipLaunchKernelGGL((k_rowgemm_mfma<T, NTW_, EPI_GRAD_PCG, CT_>), grid, dim3(256 * CT_), 0, s, n, p, N, A, sa, M, Y, ga); \
        return hipGetLastError();                                                             \
    }
    OFKS_RGM(4, 1)
    OFKS_RGM(8, 1)
    OFKS_RGM(8, 2)
#undef OFKS_RGM
    return hipErrorInvalidValue;
}

#define OFKS_CH_DISPATCH(KERNEL, ...)                                                         \
    do {                                                                                      \
        const int v = vwidth<T>(p);                                                           \
        const int l2 = lpr_l2(p, v);                                                          \
        const int chunks = (p + (v << l2) - 1) / (v << l2);                                   \
        const size_t shm = (size_t)(256 >> l2) * p * sizeof(double);                          \
        (void)shm;                                                                            \
        if (v == 1 && chunks <= 1) { hipLaunchKernelGGL((KERNEL<T, 1, 1>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        if (v == 1 && chunks <= 8) { hipLaunchKernelGGL((KERNEL<T, 1, 8>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        if (v == 2 && chunks <= 1) { hipLaunchKernelGGL((KERNEL<T, 2, 1>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        if (v == 2 && chunks <= 2) { hipLaunchKernelGGL((KERNEL<T, 2, 2>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        if (v == 2 && chunks <= 4) { hipLaunchKernelGGL((KERNEL<T, 2, 4>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        if (v == 2 && chunks <= 8) { hipLaunchKernelGGL((KERNEL<T, 2, 8>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        if constexpr (sizeof(T) == 4) {                                                       \
            if (v == 4 && chunks <= 1) { hipLaunchKernelGGL((KERNEL<T, 4, 1>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
            if (v == 4 && chunks <= 2) { hipLaunchKernelGGL((KERNEL<T, 4, 2>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
            if (v == 4 && chunks <= 4) { hipLaunchKernelGGL((KERNEL<T, 4, 4>), dim3(grid), dim3(256), SHM, s, n, p, l2, __VA_ARGS__); break; } \
        }                                                                                     \
        return hipErrorInvalidValue;                                                          \
    } while (0)

template <typename T>
hipError_t launch_pcg_r(hipStream_t s, int grid, int64_t n, int p, const T *alpha, const uint8_t *active,
                        const double *lhd, const double *bd, const T *lam, const T *Q, T *R, double *part) {
#define SHM shm
    OFKS_CH_DISPATCH(k_pcg_r, alpha, active, lhd, bd, lam, Q, R, part);
#undef SHM
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coldot(hipStream_t s, int grid, int64_t n, int p, const T *A, const T *B,
                         double *part) {
#define SHM shm
    OFKS_CH_DISPATCH(k_coldot, A, B, part);
#undef SHM
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bbdot(hipStream_t s, int grid, int64_t n, int p, const T *Xt, const T *dinv,
                        const T *P, const T *Xp, const T *Pp, double *part) {
#define SHM 0
    OFKS_CH_DISPATCH(k_bbdot, Xt, dinv, P, Xp, Pp, part);
#undef SHM
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_dx(hipStream_t s, int64_t n, int p, int first, int dir, const T *alpha, const T *beta,
                         const uint8_t *active, const double *lhd, const double *bd, const T *lam, const T *R,
                         T *D, T *X) {
    const int v = vwidth<T>(p);
    const int l2 = lpr_l2(p, v);
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
#define OFKS_DX(VV)                                                                                        \
    do {                                                                                                   \
        if (dir)                                                                                           \
            hipLaunchKernelGGL((k_pcg_dx<T, VV, 1>), dim3(grid), dim3(256), 0, s, n, p, l2, first, alpha, beta, \
                               active, lhd, bd, lam, R, D, X);                                             \
        else                                                                                               \
            hipLaunchKernelGGL((k_pcg_dx<T, VV, 0>), dim3(grid), dim3(256), 0, s, n, p, l2, first, alpha, beta, \
                               active, lhd, bd, lam, R, D, X);                                             \
    } while (0)
    if (v == 1) OFKS_DX(1);
    else if (v == 2) OFKS_DX(2);
    else if constexpr (sizeof(T) == 4) OFKS_DX(4);
#undef OFKS_DX
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_dnext(hipStream_t s, int64_t n, int p, const T *beta, const uint8_t *active,
                            const double *lhd, const double *bd, const T *lam, const T *R, const T *D, T *Dn) {
    const int v = vwidth<T>(p);
    const int l2 = lpr_l2(p, v);
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
    if (v == 1) hipLaunchKernelGGL((k_pcg_dnext<T, 1>), dim3(grid), dim3(256), 0, s, n, p, l2, beta, active, lhd, bd, lam, R, D, Dn);
    else if (v == 2) hipLaunchKernelGGL((k_pcg_dnext<T, 2>), dim3(grid), dim3(256), 0, s, n, p, l2, beta, active, lhd, bd, lam, R, D, Dn);
    else if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_pcg_dnext<T, 4>), dim3(grid), dim3(256), 0, s, n, p, l2, beta, active, lhd, bd, lam, R, D, Dn);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_sum(hipStream_t s, int64_t n, int p, int m, const T *alpha, const uint8_t *active,
                          const PcgDirs &dirs, T *X) {
    if (m < 1 || m > PCG_DIRS_MAX) return hipErrorInvalidValue;
    const int v = vwidth<T>(p);
    const int l2 = lpr_l2(p, v);
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
    if (v == 1) hipLaunchKernelGGL((k_pcg_sum<T, 1>), dim3(grid), dim3(256), 0, s, n, p, l2, m, alpha, active, dirs, X);
    else if (v == 2) hipLaunchKernelGGL((k_pcg_sum<T, 2>), dim3(grid), dim3(256), 0, s, n, p, l2, m, alpha, active, dirs, X);
    else if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_pcg_sum<T, 4>), dim3(grid), dim3(256), 0, s, n, p, l2, m, alpha, active, dirs, X);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update_b(hipStream_t s, int64_t n, int p, const T *dinv, T eta, const T *P, T *Xt,
                           T *Xp) {
    const int v = vwidth<T>(p);
    const int l2 = lpr_l2(p, v);
    const unsigned grid = (unsigned)(((n << l2) + 255) / 256);
    if (v == 1) hipLaunchKernelGGL((k_update_b<T, 1>), dim3(grid), dim3(256), 0, s, n, p, l2, dinv, eta, P, Xt, Xp);
    else if (v == 2) hipLaunchKernelGGL((k_update_b<T, 2>), dim3(grid), dim3(256), 0, s, n, p, l2, dinv, eta, P, Xt, Xp);
    else if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_update_b<T, 4>), dim3(grid), dim3(256), 0, s, n, p, l2, dinv, eta, P, Xt, Xp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_scalars(hipStream_t s, int p, int which, const double *a, double *b, T *out) {
    const unsigned grid = (unsigned)((p + 255) / 256);
    if (which == 0) hipLaunchKernelGGL((k_pcg_alpha<T>), dim3(grid), dim3(256), 0, s, p, a, b, out);
    else hipLaunchKernelGGL((k_pcg_beta<T>), dim3(grid), dim3(256), 0, s, p, a, b, out);
    return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_convert(hipStream_t s, int64_t m, const S *a, D *b) {
    hipLaunchKernelGGL((k_convert<S, D>), dim3(2048), dim3(256), 0, s, m, a, b);
    return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_scale_copy(hipStream_t s, int64_t n, int p, const S *X, const S *sc, D *Y) {
    hipLaunchKernelGGL((k_scale_copy<S, D>), dim3(2048), dim3(256), 0, s, n, p, X, sc, Y);
    return hipGetLastError();
}
template hipError_t launch_scale_copy<double, double>(hipStream_t, int64_t, int, const double *, const double *, double *);
template hipError_t launch_scale_copy<float, double>(hipStream_t, int64_t, int, const float *, const float *, double *);
template hipError_t launch_scale_copy<float, float>(hipStream_t, int64_t, int, const float *, const float *, float *);

template <typename T>
hipError_t launch_pcg_init(hipStream_t s, int grid, int64_t n, int p, const uint8_t *active, const double *lhd,
                           const double *bd, const T *lam, const T *G, T *R, T *D, T *P, double *part) {
    hipLaunchKernelGGL((k_pcg_init<T>), dim3(grid), dim3(256), 256 * sizeof(double), s, n, p, active, lhd, bd,
                       lam, G, R, D, P, part);
    return hipGetLastError();
}
template hipError_t launch_pcg_init<double>(hipStream_t, int, int64_t, int, const uint8_t *, const double *,
                                            const double *, const double *, const double *, double *, double *,
                                            double *, double *);
template hipError_t launch_pcg_init<float>(hipStream_t, int, int64_t, int, const uint8_t *, const double *,
                                           const double *, const float *, const float *, float *, float *,
                                           float *, double *);

#define OFKS_INST(T)                                                                                  \
    template hipError_t launch_gram<T>(hipStream_t, int64_t, int, const GramPlan &, const T *, const T *, const T *, double *, size_t); \
    template hipError_t launch_rowgemm<T>(hipStream_t, int, int64_t, int, int, int, const T *, const T *, const T *, T *, GradArgs, int *); \
    template hipError_t launch_pcg_r<T>(hipStream_t, int, int64_t, int, const T *, const uint8_t *, const double *, const double *, const T *, const T *, T *, double *); \
    template hipError_t launch_coldot<T>(hipStream_t, int, int64_t, int, const T *, const T *, double *); \
    template hipError_t launch_bbdot<T>(hipStream_t, int, int64_t, int, const T *, const T *, const T *, const T *, const T *, double *); \
    template hipError_t launch_pcg_dx<T>(hipStream_t, int64_t, int, int, int, const T *, const T *, const uint8_t *, const double *, const double *, const T *, const T *, T *, T *); \
    template hipError_t launch_update_b<T>(hipStream_t, int64_t, int, const T *, T, const T *, T *, T *); \
    template hipError_t launch_pcg_dnext<T>(hipStream_t, int64_t, int, const T *, const uint8_t *, const double *, const double *, const T *, const T *, const T *, T *); \
    template hipError_t launch_pcg_sum<T>(hipStream_t, int64_t, int, int, const T *, const uint8_t *, const PcgDirs &, T *); \
    template hipError_t launch_pcg_scalars<T>(hipStream_t, int, int, const double *, double *, T *);
OFKS_INST(double)
OFKS_INST(float)
template hipError_t launch_convert<double, float>(hipStream_t, int64_t, const double *, float *);
template hipError_t launch_convert<float, double>(hipStream_t, int64_t, const float *, double *);

}  // namespace ofks
