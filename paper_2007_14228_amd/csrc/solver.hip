// Host driver and C ABI of the ofks library.
//
// One PCAL iteration (Algorithm PCAL, Section 3.3) from the stored block
// X~ (the previous step before its column B-normalization):
//   [SCF]  B X~, column norms d, rho, v_xc, Hartree, H(X) re-assembly
//   HX~, BX~                         dual SpMM
//   S~ = X~^T B X~, L~ = X~^T H X~    Gram, reduced in FP64, copied to the host
//   host: D = diag(S~)^(1/2) (deferred normalization of eq. PCAL-main),
//         S = D^-1 S~ D^-1, Lambda0 = D^-1 L~ D^-1, fea, the eq. lambda2
//         multiplier Lambda, C = beta (S - I) - Lambda, C' = -Lambda0
//   G = HX + BX C, R = HX + BX C'     (X = X~ D^-1; R gives kkt)
//   stopping test (Section 4.1)
//   P = T^-1 G by Jacobi-PCG (paper preconditioner) | s .* G (learned) | G
//   BB2 step (Section 4.4) from <S,Y>, <Y,Y>
//   X~ <- X - P / eta ;  X^{k-1} <- X
// The p x p algebra is FP64 on the host; everything n-sized runs in the
// kernels of k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ofks.h"
#include "common.hpp"
#include "dense.hpp"
#include "halo_plan.hpp"

// Persistent grid of the partial-sum block kernels (k_pcg_r, k_bbdot,
// k_coldot, the PCG start), a multiple of the 8 XCDs.  At n = 2e6, p = 128
// (FP64), 1024 blocks beat 2048 and 4096: k_pcg_r 1.26 -> 1.20 ms, k_bbdot
// 1.46 -> 1.35 ms.  The row-gather shifted SpMM keeps its own grid (at most
// its resident block count).
#ifndef OFKS_PART_GRID
#define OFKS_PART_GRID 1024
#endif
#ifndef OFKS_SHIFT_GRID
#define OFKS_SHIFT_GRID 2048
#endif

// Scratch of the allocation-free Gram entry point (ofks_gram_noalloc): the
// split-K partial tiles and, after them, their column sum.  One copy per
// device, alive until the process ends.  Host code never passes the array's
// name to a kernel or a copy: it holds the device address that
// hipGetSymbolAddress returns for each device (noalloc_scratch below).
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace ofks {
// launchers (k_spmm.hip)
template <typename T>
hipError_t launch_spmm_pair(hipStream_t, int64_t, int, const int64_t *, const int32_t *, const void *, const T *,
                            T *, T *, int);
template <typename T>
hipError_t launch_spmm_shift(hipStream_t, int, int64_t, int, const int64_t *, const int32_t *, const void *,
                             const T *, const uint8_t *, const T *, T *, double *, int *);
hipError_t launch_spmv_dot(hipStream_t, int, int64_t, const int64_t *, const int32_t *, const double *,
                           const double *, double *, double *);
template <typename T>
hipError_t launch_spmm_halo(hipStream_t, int, int64_t, int, const int64_t *, const int64_t *, const int32_t *,
                            const int32_t *, const int64_t *, const uint16_t *, const void *, const T *, T *, T *, int,
                            const T *, const uint8_t *, double *, size_t, int *);
size_t spmm_halo_part_doubles(int64_t nb, int p);
hipError_t launch_halo_part_rows(hipStream_t, int64_t, int, double *);
int halo_max_rows();
int halo_max_block_rows();
int halo_max_row_entries();
int halo_pad_stride();
int halo_row_ptr_stride();
// (k_blas.hip)
constexpr int PCG_DIRS_MAX = 16;
struct PcgDirs {
    const void *d[PCG_DIRS_MAX];
};
struct GradArgs {
    const void *HX;
    void *P;
    void *R;
    void *D;
    const double *lhd;
    const double *bd;
    const void *lam;
    const uint8_t *active;
    double *part;
};
enum { EPI_PLAIN = 0, EPI_GRAD = 1, EPI_GRAD_PCG = 2, EPI_GRAD_NORM = 3 };
constexpr int LP_NPAR = 193;
constexpr int LP_SAMPLE = 8;
struct GramPlan {
    int mt, nt, gx, gy;
    int64_t splits, rows_per_split;
};
GramPlan gram_plan(int64_t n, int p, int target_blocks);
template <typename T>
hipError_t launch_gram(hipStream_t, int64_t, int, const GramPlan &, const T *, const T *, const T *, double *, size_t);
hipError_t launch_colsum(hipStream_t, int64_t, int64_t, const double *, double *);
template <typename T>
hipError_t launch_rowgemm(hipStream_t, int, int64_t, int, int, int, const T *, const T *, const T *, T *,
                          GradArgs, int *);
int rowgemm_tile_cols(int N);
int rowgemm_grid_y(int N);
template <typename T>
hipError_t launch_pcg_r(hipStream_t, int, int64_t, int, const T *, const uint8_t *, const double *, const double *,
                        const T *, const T *, T *, double *);
template <typename T>
hipError_t launch_coldot(hipStream_t, int, int64_t, int, const T *, const T *, double *);
template <typename T>
hipError_t launch_bbdot(hipStream_t, int, int64_t, int, const T *, const T *, const T *, const T *, const T *,
                        double *);
template <typename T>
hipError_t launch_pcg_dx(hipStream_t, int64_t, int, int, int, const T *, const T *, const uint8_t *, const double *,
                         const double *, const T *, const T *, T *, T *);
template <typename T>
hipError_t launch_update_b(hipStream_t, int64_t, int, const T *, T, const T *, T *, T *);
template <typename T>
hipError_t launch_pcg_dnext(hipStream_t, int64_t, int, const T *, const uint8_t *, const double *, const double *,
                            const T *, const T *, const T *, T *);
template <typename T>
hipError_t launch_pcg_sum(hipStream_t, int64_t, int, int, const T *, const uint8_t *, const PcgDirs &, T *);
template <typename T>
hipError_t launch_pcg_scalars(hipStream_t, int, int, const double *, double *, T *);
template <typename S, typename D>
hipError_t launch_convert(hipStream_t, int64_t, const S *, D *);
template <typename S, typename D>
hipError_t launch_scale_copy(hipStream_t, int64_t, int, const S *, const S *, D *);
template <typename T>
hipError_t launch_pcg_init(hipStream_t, int, int64_t, int, const uint8_t *, const double *, const double *,
                           const T *, const T *, T *, T *, T *, double *);
// (k_mesh.hip)
hipError_t scan_exclusive(hipStream_t, int64_t, const int32_t *, int64_t *, int64_t *);
hipError_t launch_interior_flags(hipStream_t, int64_t, const uint8_t *, int32_t *);
hipError_t launch_dof(hipStream_t, int64_t, const uint8_t *, const int64_t *, int32_t *);
hipError_t launch_inc_count(hipStream_t, int64_t, const int32_t *, int32_t *);
hipError_t launch_inc_fill(hipStream_t, int64_t, const int32_t *, const int64_t *, int32_t *, int32_t *);
hipError_t launch_inc_sort(hipStream_t, int64_t, const int64_t *, int32_t *, int32_t *);
hipError_t launch_row_pattern(hipStream_t, int64_t, int, const int32_t *, const int64_t *, const int32_t *,
                              const int32_t *, int32_t *, const int64_t *, int32_t *, int32_t *);
hipError_t launch_tet_geom(hipStream_t, int64_t, const double *, const int32_t *, double *, int32_t *);
hipError_t launch_vext(hipStream_t, int64_t, const double *, const int32_t *, int, const double *,
                       const double *, double *);
hipError_t launch_assemble(hipStream_t, int64_t, int, const int32_t *, const int64_t *, const int32_t *,
                           const int32_t *, const double *, const double *, const int64_t *, const int32_t *,
                           double *, double *, double *, double2 *, double2 *, double *, double *, double *);
hipError_t launch_pairs_to_f32(hipStream_t, int64_t, const double2 *, float2 *);
hipError_t launch_split_pairs(hipStream_t, int64_t, const double2 *, double *, double *);
hipError_t launch_make_pairs(hipStream_t, int64_t, const double *, const double *, double2 *);
hipError_t launch_diag(hipStream_t, int64_t, const int64_t *, const int32_t *, const double2 *, double *, double *,
                       int32_t *);
// (k_mlp.hip)
template <typename T>
hipError_t launch_lp_apply(hipStream_t, int64_t, int, T *, const double *, const double *, const double *, const T *,
                           const uint8_t *, const double *, const float *, const float *);
template <typename T>
hipError_t launch_lp_sample(hipStream_t, int64_t, int, int64_t, int64_t, int64_t, int, const T *, const T *,
                            const T *, const double *, const double *, const double *, const T *, const uint8_t *,
                            const double *, const double *, float *);
hipError_t launch_lp_grad(hipStream_t, int, int64_t, const float *, const float *, const float *, double *);
hipError_t launch_lp_adam(hipStream_t, const double *, double, float *, float *, float *, float, float, float, float,
                          int);
hipError_t launch_lp_stats(hipStream_t, int, int64_t, const float *, double *);
// (k_density.hip)
template <typename T>
hipError_t launch_density_xc(hipStream_t, int, int64_t, int, const int32_t *, const int32_t *, const double *,
                             const T *, const T *, double, double *, double *, double *, double *);
hipError_t launch_load_vec(hipStream_t, int64_t, const int32_t *, const int64_t *, const int32_t *,
                           const double *, const double *, double *);
hipError_t launch_veff(hipStream_t, int64_t, const int32_t *, const int32_t *, const double *, const double *,
                       const double *, double *);
hipError_t launch_cg_start(hipStream_t, int, int64_t, double, const double *, const double *, const double *,
                           double *, double *, double *, double *);
hipError_t launch_cg_xr(hipStream_t, int, int64_t, int, double *, int, const double *, const double *,
                        const double *, const double *, double *, double *, double *);
hipError_t launch_cg_dir(hipStream_t, int, int64_t, int, double *, const double *, const double *, const double *,
                         double *);
hipError_t launch_dot(hipStream_t, int, int64_t, const double *, const double *, double *);
// (k_gnn.hip)
constexpr int GL_NPAR_HOST = 226;
template <typename T>
hipError_t launch_gl_heads(hipStream_t, int64_t, int, const T *, const double *, const double *, const double *,
                           const T *, const uint8_t *, const double *, const float *, const float *, T *, float *);
template <typename T>
hipError_t launch_gl_out(hipStream_t, int64_t, int, const T *, const T *, const float *, const T *, const double *,
                         const double *, const T *, const uint8_t *, T *, T *);
hipError_t launch_gl_colsums(hipStream_t, int, int64_t, int, const double *, const double *, const double *,
                             const double *, const uint8_t *, double *);
hipError_t launch_gl_bwd1(hipStream_t, int, int64_t, int, const double *, const double *, double *, const float *,
                          const double *, const double *, const double *, const uint8_t *, const double *, double *,
                          double *);
hipError_t launch_gl_bwd2(hipStream_t, int, int64_t, int, const double *, const double *, const double *,
                          const double *, const double *, const double *, const double *, const double *,
                          const double *, const double *, const uint8_t *, const double *, const float *,
                          const float *, double *);
hipError_t launch_gl_adam(hipStream_t, int, const double *, double, float *, float *, float *, float, float, float,
                          float, int);
hipError_t launch_gl_node_stats(hipStream_t, int, int64_t, const double *, const double *, const double *, double *);
hipError_t launch_features(hipStream_t, int64_t, int, const double *, const double *, const double *,
                           const double *, const double *, float *);
}  // namespace ofks

using namespace ofks;

namespace {

struct ErrorOut {
    int code;
};

template <typename T> struct Blocks {
    T *Xt = nullptr, *Xp = nullptr, *P = nullptr, *Pp = nullptr, *HX = nullptr, *BX = nullptr, *R = nullptr,
      *D = nullptr;
    T *dinv = nullptr, *CC = nullptr, *lam = nullptr, *alpha = nullptr, *beta = nullptr;
};

struct Timer {
    double ms = 0.0;
    int64_t launches = 0;
};

}  // namespace

struct ofks_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    std::vector<void *> allocs;

    // state
    bool has_mesh = false, has_nuclei = false, has_system = false, assembled = false, has_lhalf = false;
    bool has_params = false, has_x = false, done = false;
    ofks_params prm{};

    // mesh
    int64_t n_nodes = 0, n_tets = 0;
    double *xyz = nullptr, *geom = nullptr, *vext_q = nullptr;
    int32_t *tets = nullptr, *dof = nullptr, *inc = nullptr;
    int64_t *iptr = nullptr;
    uint8_t *dir = nullptr;
    int M = 0;
    std::vector<double> Zh, Rh;
    double *Zd = nullptr, *Rd = nullptr;
    double Enuc = 0.0;

    // system
    int64_t n = 0, nnz = 0;
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    double *Lv = nullptr, *Bv = nullptr, *Mv = nullptr, *lhd = nullptr, *bd = nullptr, *hd = nullptr,
           *Ldiag = nullptr;
    double2 *hb = nullptr, *lb = nullptr;
    float2 *hb32 = nullptr, *lb32 = nullptr;
    // LDS-halo SpMM plan: blocks of consecutive rows, their sorted distinct
    // columns (halo) and each entry's slot in its block's halo
    int64_t halo_nb = 0;                  // 0: no plan (a row alone exceeds the halo capacity)
    int64_t *halo_row0 = nullptr, *halo_off = nullptr;
    int32_t *halo_idx = nullptr;          // per block: its halo rows, padded to a fixed stride
    int32_t *halo_rbase = nullptr;        // per block: halo slot of its first row
    int64_t *halo_brp = nullptr;          // per block: its rows' CSR row pointers, padded to a fixed stride
    uint16_t *halo_lcol = nullptr;

    // SCF work
    double *rho_q = nullptr, *eps_q = nullptr, *vxc_q = nullptr, *veff_q = nullptr, *bvec = nullptr,
           *U = nullptr, *cg_r = nullptr, *cg_d = nullptr, *cg_q = nullptr, *cg_sc = nullptr,
           *cg_part = nullptr;   // Hartree CG partial sums (fixed: the captured graph holds the pointer)
    double scf_parts[4] = {0, 0, 0, 0};  // int rho, int eps rho, int vxc rho, U.b/2

    // iteration
    int p = 0;
    int prec = OFKS_F64;
    Blocks<double> b64;
    Blocks<float> b32;
    uint8_t *active = nullptr;
    double *part = nullptr, *red = nullptr, *rz = nullptr;
    size_t part_cap = 0;
    double *hbuf = nullptr;  // pinned host buffer for downloads
    size_t hbuf_cap = 0;
    char *hup = nullptr;     // pinned upload staging, consumed by a cursor reset at each sync
    size_t hup_cap = 0, hup_off = 0;
    int grid = OFKS_PART_GRID;         // persistent grid for partial-sum kernels
    int shift_grid = OFKS_SHIFT_GRID;  // grid cap of the row-gather shifted SpMM
    int gemm_rows = 1024;

    int k = 0;
    double kkt0 = -1.0, eta = 0.0, eta0 = 0.0;
    bool have_prev = false;
    std::vector<double> dinv_h, S, L0;
    double last_kkt = NAN, last_fea = NAN, last_rel = NAN, last_energy = NAN;
    bool dinv_from_scf = false;
    // learned form
    std::vector<double> ehist;   // recent energies (fallback rule)
    float *lp_W = nullptr, *lp_norm = nullptr;
    bool lp_ready = false;
    int lp_hold = 0;             // iterations left on the paper preconditioner after a fallback
    int last_kind = -1;          // preconditioner of the previous step (BB restarts on a change)
    double *g2 = nullptr, *tw = nullptr;
    float *lp_buf = nullptr;     // training-sample collection
    int64_t lp_cap = 0, lp_count = 0, lp_stride = 0;
    hipGraphExec_t cg_graph = nullptr;   // 10 Hartree CG iterations, captured once per system
    double f32_best = 0.0;       // FP32 phase: lowest residual so far and its iteration
    int f32_best_k = 0;
    int lp_objective = 0;        // 0: Euclidean imitation of T^-1 g, 1: energy-norm imitation
    void *lp_u = nullptr;        // T (J G) for the energy-norm samples
    size_t lp_u_bytes = 0;
    // inner CG, history form: directions 1 .. m-1 (direction 0 is the D
    // block) and the m x p step lengths; library memory, taken only while
    // free memory allows (pcg_history)
    void *pcg_dh = nullptr;
    size_t pcg_dh_bytes = 0;
    void *pcg_ah = nullptr;
    size_t pcg_ah_bytes = 0;

    double *scratch_dev = nullptr;   // this device's copy of `scratch` (ofks_gram_noalloc)
    double poisson_tol_now = 0.0;    // > 0: the Hartree CG tolerance of the current iteration
    // caller-owned workspace (ofks_set_workspace): the iteration's device
    // state is carved from it in order while ws_carve is set
    char *ws_base = nullptr;
    size_t ws_size = 0, ws_off = 0;
    size_t ws_f64_base = 0, ws_f64_cap = 0;   // where the FP64 set of an FP32 run's refinement goes
    bool ws_carve = false;
    // graph learned preconditioner
    float *gl_W = nullptr, *gl_norm = nullptr;   // 226 weights, 8 standardization constants (device)
    bool gl_ready = false;
    float *gl_ft = nullptr;                      // smoothing weights ft of the current block (n x p)
    size_t gl_ft_cap = 0;
    double *gl_cap = nullptr;                    // snapshot capture: caller's device buffer of G blocks
    int64_t gl_cap_every = 1;
    int32_t gl_cap_max = 0, gl_cap_count = 0;
    std::vector<double> gl_cap_lam;              // the shifts of each captured block
    double *gl_work = nullptr;                   // training blocks (5 n x p FP64) and ft (n x p FP32)
    size_t gl_work_np = 0;
    std::vector<double> relmin;                  // relmin[j] = lowest rel of X^0..X^j (stall fallback)

    // timing
    bool timing = false;
    std::map<std::string, Timer> timers;
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> evpool;
};

namespace {

int fail(ofks_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(...)                                                                                 \
    do {                                                                                            \
        hipError_t e_ = (__VA_ARGS__);                                                              \
        if (e_ != hipSuccess) return fail(c, OFKS_EHIP, "%s: %s (%s:%d)", #__VA_ARGS__,              \
                                          hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

#define CHK(...)                   \
    do {                           \
        int r_ = (__VA_ARGS__);    \
        if (r_ < 0) return r_;     \
    } while (0)

template <typename T> int dalloc(ofks_ctx *c, T **out, size_t count) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(c, OFKS_EHIP, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    c->allocs.push_back(p);
    *out = (T *)p;
    return OFKS_OK;
}

// Iteration-state allocation: carved from the caller's workspace while one
// is set and ws_carve is on (the entry points that build or advance the
// iteration), else hipMalloc.  Pieces are 256-byte aligned.
template <typename T> int walloc(ofks_ctx *c, T **out, size_t count) {
    if (!(c->ws_base && c->ws_carve)) return dalloc(c, out, count);
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~size_t(255);
    if (c->ws_off + bytes > c->ws_size)
        return fail(c, OFKS_ECAPACITY, "workspace exhausted: %zu of %zu bytes used, %zu more needed (see ofks_workspace_size)",
                    c->ws_off, c->ws_size, bytes);
    *out = (T *)(c->ws_base + c->ws_off);
    c->ws_off += bytes;
    return OFKS_OK;
}

// bytes that walloc takes for a set of nblk blocks of n x p elements of
// `elem` bytes and their five per-column arrays (alloc_blocks' layout)
size_t ws_piece(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~size_t(255); }
size_t ws_block_set(size_t n, size_t p, size_t elem, int nblk) {
    return nblk * ws_piece(n * p * elem) + 3 * ws_piece(p * elem) + ws_piece(2 * p * p * elem) + ws_piece(p * elem);
}
// the region an FP32 run keeps for FP64 blocks: the start block's setup and,
// when a refinement may follow, the whole FP64 set that replaces the FP32 one
size_t ws_f64_region(ofks_ctx *c, int p) {
    return ws_block_set(c->n, p, sizeof(double), c->prm.refine_tol > 0.0 ? 8 : 3);
}

template <typename T> void dfree(ofks_ctx *c, T *&ptr) {
    if (!ptr) return;
    if (c->ws_base && (const char *)ptr >= c->ws_base && (const char *)ptr < c->ws_base + c->ws_size) {
        ptr = nullptr;   // workspace memory is the caller's
        return;
    }
    auto it = std::find(c->allocs.begin(), c->allocs.end(), (void *)ptr);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree((void *)ptr);
    ptr = nullptr;
}

int ensure_host(ofks_ctx *c, size_t doubles) {
    if (c->hbuf_cap >= doubles) return OFKS_OK;
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    c->hbuf = nullptr;
    hipError_t e = hipHostMalloc((void **)&c->hbuf, doubles * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return fail(c, OFKS_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
    c->hbuf_cap = doubles;
    return OFKS_OK;
}

int ensure_part(ofks_ctx *c, size_t doubles);

// Largest per-block partial buffer any kernel of an iteration needs for this
// p, reserved once so that no reallocation happens while kernels that hold
// the pointer are queued.
size_t partials_needed(ofks_ctx *c, int p);

int ensure_part(ofks_ctx *c, size_t doubles) {
    if (c->part_cap >= doubles) return OFKS_OK;
    HIPCHK(hipStreamSynchronize(c->stream));   // kernels in flight may still use the old buffer
    dfree(c, c->part);
    c->part_cap = 0;
    CHK(walloc(c, &c->part, doubles));
    c->part_cap = doubles;
    return OFKS_OK;
}

// --- timing -----------------------------------------------------------------
hipEvent_t get_event(ofks_ctx *c) {
    if (!c->evpool.empty()) {
        hipEvent_t e = c->evpool.back();
        c->evpool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Scope {
    ofks_ctx *c;
    const char *name;
    hipEvent_t a = nullptr;
    Scope(ofks_ctx *c_, const char *n) : c(c_), name(n) {
        if (c->timing) {
            a = get_event(c);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    ~Scope() {
        if (c->timing && a) {
            hipEvent_t b = get_event(c);
            if (b) {
                (void)hipEventRecord(b, c->stream);
                c->pending.push_back({name, a, b});
            }
        }
    }
};

void resolve_timers(ofks_ctx *c) {
    for (auto &pd : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
            auto &t = c->timers[pd.name];
            t.ms += ms;
            t.launches += 1;
        }
        c->evpool.push_back(pd.a);
        c->evpool.push_back(pd.b);
    }
    c->pending.clear();
}

int sync(ofks_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    c->hup_off = 0;
    if (c->timing) resolve_timers(c);
    return OFKS_OK;
}

template <typename T> Blocks<T> &blk(ofks_ctx *c);
template <> Blocks<double> &blk<double>(ofks_ctx *c) { return c->b64; }
template <> Blocks<float> &blk<float>(ofks_ctx *c) { return c->b32; }
template <typename T> const void *hbT(ofks_ctx *c);
template <> const void *hbT<double>(ofks_ctx *c) { return c->hb; }
template <> const void *hbT<float>(ofks_ctx *c) { return c->hb32; }
template <typename T> const void *lbT(ofks_ctx *c);
template <> const void *lbT<double>(ofks_ctx *c) { return c->lb; }
template <> const void *lbT<float>(ofks_ctx *c) { return c->lb32; }

// All iteration blocks, or (setup_only) just those the start block's
// B-orthonormalization uses: X, HX, BX (an FP32 run converts and frees them).
template <typename T> int alloc_blocks(ofks_ctx *c, bool setup_only = false) {
    Blocks<T> &b = blk<T>(c);
    const size_t np = (size_t)c->n * c->p;
    CHK(walloc(c, &b.Xt, np));
    CHK(walloc(c, &b.HX, np));
    CHK(walloc(c, &b.BX, np));
    if (!setup_only) {
        CHK(walloc(c, &b.Xp, np));
        CHK(walloc(c, &b.P, np));
        CHK(walloc(c, &b.Pp, np));
        CHK(walloc(c, &b.R, np));
        CHK(walloc(c, &b.D, np));
    }
    CHK(walloc(c, &b.dinv, c->p));
    CHK(walloc(c, &b.CC, (size_t)c->p * 2 * c->p));
    CHK(walloc(c, &b.lam, c->p));
    CHK(walloc(c, &b.alpha, c->p));
    CHK(walloc(c, &b.beta, c->p));
    return OFKS_OK;
}

template <typename T> void free_blocks(ofks_ctx *c) {
    Blocks<T> &b = blk<T>(c);
    dfree(c, b.Xt);
    dfree(c, b.Xp);
    dfree(c, b.P);
    dfree(c, b.Pp);
    dfree(c, b.HX);
    dfree(c, b.BX);
    dfree(c, b.R);
    dfree(c, b.D);
    dfree(c, b.dinv);
    dfree(c, b.CC);
    dfree(c, b.lam);
    dfree(c, b.alpha);
    dfree(c, b.beta);
}

// stage bytes in pinned memory and enqueue the copy; the staging region is
// not reused before the next sync, so no wait is needed here
int upload_bytes(ofks_ctx *c, void *dst, const void *src, size_t bytes) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (c->hup_off + need > c->hup_cap) {
        CHK(sync(c));
        if (need > c->hup_cap) {
            if (c->hup) (void)hipHostFree(c->hup);
            c->hup = nullptr;
            const size_t cap = std::max<size_t>(need, size_t(1) << 20);
            hipError_t e = hipHostMalloc((void **)&c->hup, cap, hipHostMallocDefault);
            if (e != hipSuccess) return fail(c, OFKS_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
            c->hup_cap = cap;
        }
    }
    char *h = c->hup + c->hup_off;
    std::memcpy(h, src, bytes);
    c->hup_off += need;
    HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, c->stream));
    return OFKS_OK;
}

// upload host doubles as T
template <typename T> int upload(ofks_ctx *c, T *dst, const std::vector<double> &src) {
    std::vector<T> tmp(src.begin(), src.end());
    return upload_bytes(c, dst, tmp.data(), tmp.size() * sizeof(T));
}

int download(ofks_ctx *c, std::vector<double> &dst, const double *src, size_t count) {
    CHK(ensure_host(c, count));
    HIPCHK(hipMemcpyAsync(c->hbuf, src, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CHK(sync(c));
    dst.assign(c->hbuf, c->hbuf + count);
    return OFKS_OK;
}

// ---------------------------------------------------------------------------
// Gram: S~ = X^T BX, L~ = X^T HX (host, FP64, not symmetrized)
// ---------------------------------------------------------------------------
template <typename T>
int gram(ofks_ctx *c, const T *X, const T *BX, const T *HX, std::vector<double> &St, std::vector<double> &Lt) {
    const int p = c->p;
    const size_t pp2 = (size_t)p * 2 * p;
    // size the split-K partials from the launch plan before launching
    const GramPlan plan = gram_plan(c->n, p, 2048);
    CHK(ensure_part(c, (size_t)plan.splits * pp2));
    const int64_t ns = plan.splits;
    {
        Scope sc(c, "gram");
        HIPCHK(launch_gram<T>(c->stream, c->n, p, plan, X, BX, HX, c->part, c->part_cap));
    }
    HIPCHK(launch_colsum(c->stream, ns, (int64_t)pp2, c->part, c->red));
    std::vector<double> G;
    CHK(download(c, G, c->red, pp2));
    St.assign((size_t)p * p, 0.0);
    Lt.assign((size_t)p * p, 0.0);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            St[a * p + b] = G[(size_t)a * 2 * p + b];
            Lt[a * p + b] = G[(size_t)a * 2 * p + p + b];
        }
    return OFKS_OK;
}

size_t partials_needed(ofks_ctx *c, int p) {
    const GramPlan plan = gram_plan(c->n, p, 2048);
    const size_t gy = rowgemm_grid_y(2 * p);
    size_t need = (size_t)plan.splits * p * 2 * p;
    need = std::max(need, (size_t)c->gemm_rows * gy * (1 + p));
    need = std::max(need, (size_t)std::max(c->grid, c->shift_grid) * std::max(p, 5));
    need = std::max(need, (size_t)3 * 1024);
    if (c->halo_nb) need = std::max(need, spmm_halo_part_doubles(c->halo_nb, p));   // either precision
    return need;
}

// SpMM kernel choice (spmm_mode 0), as measured: the LDS-halo kernel for
// FP64 blocks with p >= 64 (faster at p = 64, 96, 128, 160 and 512) and FP32
// blocks with p >= 96 (faster at p = 96, 128, 160, 192 and 512; at p = 64 the
// half-empty 128-column slice loses); the row-gather kernel otherwise.
// spmm_mode 1 (gather) or 2 (halo) forces one.  Returns 1: halo, 0: gather,
// -1: halo forced but no plan exists.
int halo_choice(ofks_ctx *c, int p, size_t elem) {
    const int m = c->prm.spmm_mode;
    if (m == 1) return 0;
    if (m == 2) return c->halo_nb ? 1 : -1;
    return c->halo_nb && (elem == 8 ? p >= 64 : p >= 96) ? 1 : 0;
}

// Y1 = A1 X, Y2 = A2 X (Y2 = NULL: A1 X or A2 X by sel) for the pair matrix w.
template <typename T>
int spmm_pair(ofks_ctx *c, int p, const void *w, const T *X, T *Y1, T *Y2, int sel) {
    const int h = halo_choice(c, p, sizeof(T));
    if (h < 0) return fail(c, OFKS_ESTATE, "spmm_mode halo: no halo plan for this matrix");
    if (h)
        HIPCHK(launch_spmm_halo<T>(c->stream, 0, c->halo_nb, p, c->halo_row0, c->halo_off, c->halo_idx, c->halo_rbase,
                                   c->halo_brp, c->halo_lcol, w, X, Y1, Y2, sel, nullptr, nullptr, nullptr, 0,
                                   nullptr));
    else
        HIPCHK(launch_spmm_pair<T>(c->stream, c->n, p, c->rp, c->col, w, X, Y1, Y2, sel));
    return OFKS_OK;
}

// Q = (L/2 - lam B) D on active columns and per-block <D, Q> partials in
// c->part; *used = partial rows for the column sum.  The product kernel is
// timed as "spmm_shift", the halo kernel's partial-row sums apart from it.
template <typename T>
int spmm_shift(ofks_ctx *c, int p, const void *lb, const T *lam, const uint8_t *act, const T *D, T *Q, int *used) {
    const int h = halo_choice(c, p, sizeof(T));
    if (h < 0) return fail(c, OFKS_ESTATE, "spmm_mode halo: no halo plan for this matrix");
    if (h) {
        CHK(ensure_part(c, spmm_halo_part_doubles(c->halo_nb, p)));
        {
            Scope sc(c, "spmm_shift");
            HIPCHK(launch_spmm_halo<T>(c->stream, 1, c->halo_nb, p, c->halo_row0, c->halo_off, c->halo_idx,
                                       c->halo_rbase, c->halo_brp, c->halo_lcol, lb, D, Q, nullptr, 0, lam, act,
                                       c->part, c->part_cap, used));
        }
        HIPCHK(launch_halo_part_rows(c->stream, c->halo_nb, p, c->part));
        return OFKS_OK;
    }
    CHK(ensure_part(c, (size_t)c->shift_grid * p));
    Scope sc(c, "spmm_shift");
    HIPCHK(launch_spmm_shift<T>(c->stream, c->shift_grid, c->n, p, c->rp, c->col, lb, lam, act, D, Q, c->part,
                                used));
    return OFKS_OK;
}

// column sums of A .* B over rows (FP64)
template <typename T> int coldot(ofks_ctx *c, const T *A, const T *B, std::vector<double> &out) {
    CHK(ensure_part(c, (size_t)c->grid * c->p));
    HIPCHK(launch_coldot<T>(c->stream, c->grid, c->n, c->p, A, B, c->part));
    HIPCHK(launch_colsum(c->stream, c->grid, c->p, c->part, c->red));
    return download(c, out, c->red, c->p);
}

// ---------------------------------------------------------------------------
// SCF: H(X) for X = Xs .* dinv (Section 2.2)
// ---------------------------------------------------------------------------
// Hartree CG grid: enough 256-thread blocks to fill the device (the vectors
// are short, so the kernels are latency-bound); the fused reductions sum one
// partial per block.
#ifndef OFKS_CG_SPMV_BLOCKS
#define OFKS_CG_SPMV_BLOCKS 2048   // the Hartree SpMV's grid
#endif
#ifndef OFKS_CG_UPD_BLOCKS
#define OFKS_CG_UPD_BLOCKS 512     // the CG vector updates' grid: each of their blocks sums all the previous
#endif                             // kernel's partials, so fewer blocks read far fewer (measured at n = 2e5)
constexpr int CG_BLOCKS = OFKS_CG_SPMV_BLOCKS;

void drop_cg_graph(ofks_ctx *c) {
    if (c->cg_graph) (void)hipGraphExecDestroy(c->cg_graph);
    c->cg_graph = nullptr;
}

int poisson(ofks_ctx *c) {
    const int64_t n = c->n;
    const int g = CG_BLOCKS, gu = OFKS_CG_UPD_BLOCKS;   // partials: <d, q> (g), then 3-wide update sums (gu)
    static_assert(OFKS_CG_UPD_BLOCKS <= CG_BLOCKS, "partial buffer sized for CG_BLOCKS");
    double *dqp = c->cg_part, *xrp = c->cg_part + g;
    {
        Scope sc(c, "poisson");
        HIPCHK(launch_spmv_dot(c->stream, g, n, c->rp, c->col, c->Lv, c->U, c->cg_q, dqp));
        // Jacobi preconditioner diag(L/2): a constant multiple of diag(L) leaves the CG iterates unchanged
        HIPCHK(launch_cg_start(c->stream, gu, n, 4.0 * M_PI, c->bvec, c->cg_q, c->lhd, c->cg_r, c->cg_d, xrp,
                               c->cg_sc));
    }
    std::vector<double> sc;
    CHK(download(c, sc, c->cg_sc, 3));
    double rr = sc[1], bb = sc[2];
    const double rt = c->poisson_tol_now > 0.0 ? c->poisson_tol_now : c->prm.poisson_rtol;
    const double tol2 = rt * rt * bb;
    // ten CG iterations (30 launches; an even count, so <r, z> ends in sc[0]
    // again), replayed as one graph when allowed
    auto chunk = [&](hipStream_t s) -> hipError_t {
        for (int j = 0; j < 10; ++j) {
            hipError_t e;
            if ((e = launch_spmv_dot(s, g, n, c->rp, c->col, c->Lv, c->cg_d, c->cg_q, dqp)) != hipSuccess) return e;
            if ((e = launch_cg_xr(s, gu, n, j & 1, c->cg_sc, g, dqp, c->cg_d, c->cg_q, c->lhd, c->U, c->cg_r, xrp)) !=
                hipSuccess)
                return e;
            if ((e = launch_cg_dir(s, gu, n, j & 1, c->cg_sc, xrp, c->cg_r, c->lhd, c->cg_d)) != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (c->prm.use_graphs && !c->cg_graph) {
        // captured on a private stream (the context's stream may be the null
        // stream, which cannot be captured); every node is a kernel launch
        hipStream_t cs = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t el = chunk(cs);
            e = hipStreamEndCapture(cs, &gr);
            if (e == hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->cg_graph, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            c->cg_graph = nullptr;
            return fail(c, OFKS_EHIP, "Hartree CG graph capture: %s", hipGetErrorString(e));
        }
    }
    int it = 0;
    while (rr > tol2 && it < c->prm.poisson_max_iter) {
        {
            Scope s2(c, "poisson");
            if (c->prm.use_graphs) HIPCHK(hipGraphLaunch(c->cg_graph, c->stream));
            else HIPCHK(chunk(c->stream));
        }
        it += 10;
        CHK(download(c, sc, c->cg_sc, 2));
        rr = sc[1];
        if (!std::isfinite(rr)) return fail(c, OFKS_ENONFINITE, "Hartree CG diverged");
    }
    if (rr > tol2) return fail(c, OFKS_NOT_CONVERGED, "Hartree CG did not reach %g", rt);
    return OFKS_OK;
}

// the density's quadrature-point arrays, allocated on the first density
// evaluation (a fixed-H run never needs them)
void free_scf_work(ofks_ctx *c) {
    dfree(c, c->rho_q);
    dfree(c, c->eps_q);
    dfree(c, c->vxc_q);
    dfree(c, c->veff_q);
}

int ensure_scf_work(ofks_ctx *c) {
    if (c->rho_q && c->eps_q && c->vxc_q && c->veff_q) return OFKS_OK;
    free_scf_work(c);   // all four or none
    const int64_t nt = c->n_tets;
    int rc = walloc(c, &c->rho_q, 4 * nt);
    if (rc == OFKS_OK) rc = walloc(c, &c->eps_q, 4 * nt);
    if (rc == OFKS_OK) rc = walloc(c, &c->vxc_q, 4 * nt);
    if (rc == OFKS_OK) rc = walloc(c, &c->veff_q, 4 * nt);
    if (rc != OFKS_OK) free_scf_work(c);
    return rc;
}

template <typename T> int build_h(ofks_ctx *c, const T *X, const T *dinv_dev) {
    CHK(ensure_scf_work(c));
    const int64_t nt = c->n_tets;
    const int g = 1024;
    CHK(ensure_part(c, (size_t)3 * g));
    {
        Scope sc(c, "density");
        HIPCHK(launch_density_xc<T>(c->stream, g, nt, c->p, c->tets, c->dof, c->geom, X, dinv_dev,
                                    c->prm.occupation, c->rho_q, c->eps_q, c->vxc_q, c->part));
    }
    HIPCHK(launch_colsum(c->stream, g, 3, c->part, c->red));
    std::vector<double> s3;
    CHK(download(c, s3, c->red, 3));
    {
        Scope sc(c, "density");
        HIPCHK(launch_load_vec(c->stream, c->n_nodes, c->dof, c->iptr, c->inc, c->geom, c->rho_q, c->bvec));
    }
    int rc = poisson(c);
    if (rc != OFKS_OK) return rc < 0 ? rc : fail(c, OFKS_ENONFINITE, "%s", c->err.c_str());
    HIPCHK(launch_dot(c->stream, 512, c->n, c->U, c->bvec, c->part));
    HIPCHK(launch_colsum(c->stream, 512, 1, c->part, c->red));
    std::vector<double> ub;
    CHK(download(c, ub, c->red, 1));
    c->scf_parts[0] = s3[0];
    c->scf_parts[1] = s3[1];
    c->scf_parts[2] = s3[2];
    c->scf_parts[3] = 0.5 * ub[0];
    {
        Scope sc(c, "assemble_h");
        HIPCHK(launch_veff(c->stream, nt, c->tets, c->dof, c->U, c->vext_q, c->vxc_q, c->veff_q));
        HIPCHK(launch_assemble(c->stream, c->n_nodes, 1, c->dof, c->iptr, c->inc, c->tets, c->geom, c->veff_q,
                               c->rp, c->col, c->Lv, nullptr, nullptr, c->hb, nullptr, nullptr, nullptr, c->hd));
        if (c->hb32) HIPCHK(launch_pairs_to_f32(c->stream, c->nnz, c->hb, c->hb32));
    }
    return OFKS_OK;
}

double bb_eta(int rule, int k, double sy, double yy, double ss, double eta_prev, double eta0) {
    if (rule == OFKS_STEP_FIXED) return eta0;
    double num, den;
    const bool bb1 = rule == OFKS_STEP_BB1 || (rule == OFKS_STEP_ABB1 && k % 2 == 1) ||
                     (rule == OFKS_STEP_ABB2 && k % 2 == 0);
    if (bb1) { num = std::fabs(sy); den = ss; }
    else { num = yy; den = std::fabs(sy); }
    if (!(den > 0.0) || !std::isfinite(num) || !std::isfinite(den)) return eta_prev;
    double e = num / den;
    if (!(e > 0.0) || !std::isfinite(e)) return eta_prev;
    return std::min(std::max(e, 1e-8 * eta0), 1e8 * eta0);
}

// ---------------------------------------------------------------------------
// one PCAL iteration
// ---------------------------------------------------------------------------
// (-DOFKS_PCG_HISTORY=0 keeps the running update of x everywhere)
#ifndef OFKS_PCG_HISTORY
#define OFKS_PCG_HISTORY 1
#endif
// Inner CG, history form: each direction gets a block of its own and
// P = sum_j alpha_j d_j is formed once at the end, which saves the read and
// write of x in every inner iteration (m - 1 extra blocks: 18 GB for FP64
// at n = 2e6, p = 128, m = 10).  Taken only without a caller workspace and
// while free device memory stays above a quarter of the device (or four
// blocks) after the allocation; otherwise pcg_run keeps x up to date as it
// goes.  The two forms give the same bits.
void free_pcg_history(ofks_ctx *c) {
    if (c->pcg_dh || c->pcg_ah) (void)hipStreamSynchronize(c->stream);   // queued work may still use them
    dfree(c, c->pcg_dh);
    dfree(c, c->pcg_ah);
    c->pcg_dh_bytes = c->pcg_ah_bytes = 0;
}

template <typename T> bool pcg_history(ofks_ctx *c, int m, int64_t n, int p) {
    if (c->ws_base || m < 2 || m > PCG_DIRS_MAX) return false;
    const size_t blk = (size_t)n * p * sizeof(T);
    const size_t need = blk * (size_t)(m - 1), need_a = (size_t)m * p * sizeof(T);
    if (c->pcg_dh && c->pcg_dh_bytes == need && c->pcg_ah_bytes >= need_a) return true;
    free_pcg_history(c);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const size_t reserve = std::max(tot / 4, 4 * blk);
    if (fr < need + need_a + reserve) return false;
    void *dh = nullptr, *ah = nullptr;
    if (hipMalloc(&dh, need) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (hipMalloc(&ah, need_a) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(dh);
        return false;
    }
    c->allocs.push_back(dh);
    c->allocs.push_back(ah);
    // defined contents in the columns no iteration writes (inactive ones)
    if (hipMemsetAsync(dh, 0, need, c->stream) != hipSuccess) {
        (void)hipGetLastError();
        free_pcg_history(c);
        return false;
    }
    c->pcg_dh = dh;
    c->pcg_dh_bytes = need;
    c->pcg_ah = ah;
    c->pcg_ah_bytes = need_a;
    return true;
}

// P = T^-1 G columnwise by m Jacobi-PCG iterations from zero (eq. precondition-T).
// On entry R = G and D = J G on active columns, rz = <G, J G>; X holds the
// identity-branch columns already.  Q is scratch for the operator output.
template <typename T>
int pcg_run(ofks_ctx *c, int m, int64_t n, int p, const uint8_t *act, const T *lam, const void *lb, T *D, T *Q, T *X,
            T *R, T *alpha, T *beta, double *rz) {
    CHK(ensure_part(c, (size_t)c->grid * p));
    if (OFKS_PCG_HISTORY && pcg_history<T>(c, m, n, p)) {
        PcgDirs dirs{};
        T *dh = (T *)c->pcg_dh;
        for (int j = 0; j < m; ++j) dirs.d[j] = j == 0 ? (const void *)D : (const void *)(dh + (size_t)(j - 1) * n * p);
        T *ah = (T *)c->pcg_ah;
        for (int it = 0; it < m; ++it) {
            T *Dj = (T *)dirs.d[it];
            T *al = ah + (size_t)it * p;
            int used = 0;
            CHK(spmm_shift<T>(c, p, lb, lam, act, Dj, Q, &used));
            HIPCHK(launch_colsum(c->stream, used, p, c->part, c->red));
            HIPCHK(launch_pcg_scalars<T>(c->stream, p, 0, c->red, rz, al));
            if (it + 1 < m) {
                {
                    Scope sc(c, "pcg_r");
                    HIPCHK(launch_pcg_r<T>(c->stream, c->grid, n, p, al, act, c->lhd, c->bd, lam, Q, R, c->part));
                }
                HIPCHK(launch_colsum(c->stream, c->grid, p, c->part, c->red));
                HIPCHK(launch_pcg_scalars<T>(c->stream, p, 1, c->red, rz, beta));
                Scope sc(c, "pcg_dx");
                HIPCHK(launch_pcg_dnext<T>(c->stream, n, p, beta, act, c->lhd, c->bd, lam, R, Dj,
                                           (T *)dirs.d[it + 1]));
            }
        }
        Scope sc(c, "pcg_sum");
        HIPCHK(launch_pcg_sum<T>(c->stream, n, p, m, ah, act, dirs, X));
        return OFKS_OK;
    }
    for (int it = 0; it < m; ++it) {
        int used = 0;
        CHK(spmm_shift<T>(c, p, lb, lam, act, D, Q, &used));
        HIPCHK(launch_colsum(c->stream, used, p, c->part, c->red));
        HIPCHK(launch_pcg_scalars<T>(c->stream, p, 0, c->red, rz, alpha));
        const bool more = it + 1 < m;   // the last iteration needs no new residual or direction
        if (more) {
            {
                Scope sc(c, "pcg_r");
                HIPCHK(launch_pcg_r<T>(c->stream, c->grid, n, p, alpha, act, c->lhd, c->bd, lam, Q, R, c->part));
            }
            HIPCHK(launch_colsum(c->stream, c->grid, p, c->part, c->red));
            HIPCHK(launch_pcg_scalars<T>(c->stream, p, 1, c->red, rz, beta));
        }
        Scope sc(c, "pcg_dx");
        HIPCHK(launch_pcg_dx<T>(c->stream, n, p, it == 0, more, alpha, beta, act, c->lhd, c->bd, lam, R, D, X));
    }
    return OFKS_OK;
}

// the graph form's smoothing weights ft (FP32, n x p), grown when needed
int ensure_gl_ft(ofks_ctx *c, size_t count) {
    if (c->gl_ft_cap >= count) return OFKS_OK;
    if (c->gl_ft) CHK(sync(c));   // queued work may still read the old buffer
    dfree(c, c->gl_ft);
    c->gl_ft_cap = 0;
    CHK(walloc(c, &c->gl_ft, count));
    c->gl_ft_cap = count;
    return OFKS_OK;
}

template <typename T> int iterate(ofks_ctx *c, ofks_iter_stats *st, bool *stop) {
    Blocks<T> &B = blk<T>(c);
    const int p = c->p;
    const int64_t n = c->n;
    const auto t0 = std::chrono::steady_clock::now();
    const bool scf = c->prm.scf != 0;
    const bool plam = c->prm.algorithm == 1;   // Algorithm PLAM: no column normalization, Lambda = X^T H X

    // [SCF] normalize and rebuild H(X^k)
    if (scf) {
        std::vector<double> dn(p, 1.0);
        if (c->k > 0 && !plam) {
            {
                Scope sc(c, "spmm_dual");
                CHK(spmm_pair<T>(c, p, hbT<T>(c), B.Xt, B.BX, nullptr, 1));
            }
            std::vector<double> d2;
            CHK(coldot<T>(c, B.Xt, B.BX, d2));
            for (int i = 0; i < p; ++i) {
                if (!(d2[i] > 0.0)) return fail(c, OFKS_EZERONORM, "column %d has zero B-norm", i);
                dn[i] = 1.0 / std::sqrt(d2[i]);
            }
        }
        c->dinv_h = dn;
        CHK(upload<T>(c, B.dinv, dn));
        // inexact Hartree solves while the iteration is far from converged
        const double relp = (c->k > 0 && std::isfinite(c->last_rel)) ? c->last_rel : 1.0;
        c->poisson_tol_now = c->prm.poisson_adapt > 0.0
                                 ? std::max(c->prm.poisson_rtol, c->prm.poisson_adapt * relp)
                                 : 0.0;
        const int rc = build_h<T>(c, B.Xt, B.dinv);
        c->poisson_tol_now = 0.0;
        CHK(rc);
    }

    // HX~, BX~
    {
        Scope sc(c, "spmm_dual");
        CHK(spmm_pair<T>(c, p, hbT<T>(c), B.Xt, B.HX, B.BX, 0));
    }
    std::vector<double> St, Lt;
    CHK(gram<T>(c, B.Xt, B.BX, B.HX, St, Lt));
    const auto th0 = std::chrono::steady_clock::now();   // host p x p algebra from here to the uploads

    // deferred normalization
    std::vector<double> &dn = c->dinv_h;
    if (!scf) {
        dn.assign(p, 1.0);
        if (c->k > 0 && !plam)
            for (int i = 0; i < p; ++i) {
                if (!(St[i * p + i] > 0.0)) return fail(c, OFKS_EZERONORM, "column %d has zero B-norm", i);
                dn[i] = 1.0 / std::sqrt(St[i * p + i]);
            }
    }
    std::vector<double> S(p * p), L0(p * p);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            S[a * p + b] = 0.5 * (St[a * p + b] + St[b * p + a]) * dn[a] * dn[b];
            L0[a * p + b] = 0.5 * (Lt[a * p + b] + Lt[b * p + a]) * dn[a] * dn[b];
        }
    for (double v : S)
        if (!std::isfinite(v)) return fail(c, OFKS_ENONFINITE, "non-finite X^T B X");
    for (double v : L0)
        if (!std::isfinite(v)) return fail(c, OFKS_ENONFINITE, "non-finite X^T H X");
    double fea = 0.0;
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            const double e = S[a * p + b] - (a == b ? 1.0 : 0.0);
            fea += e * e;
        }
    fea = std::sqrt(fea);
    const double beta = c->prm.beta;
    // eq. lambda2: only the diagonal of Lambda0 - S Lambda0 + beta S (S - I) is needed
    std::vector<double> lam_diag(p);
    std::vector<double> CC((size_t)p * 2 * p);
    for (int i = 0; i < p; ++i) {
        double sl = 0.0, ss = 0.0;
        for (int k2 = 0; k2 < p; ++k2) {
            sl += S[i * p + k2] * L0[k2 * p + i];
            ss += S[i * p + k2] * (S[k2 * p + i] - (k2 == i ? 1.0 : 0.0));
        }
        lam_diag[i] = plam ? L0[i * p + i] : L0[i * p + i] + (L0[i * p + i] - sl + beta * ss);
    }
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            const double lam_ab = (a == b) ? lam_diag[a] : L0[a * p + b];
            CC[(size_t)a * 2 * p + b] = beta * (S[a * p + b] - (a == b ? 1.0 : 0.0)) - lam_ab;
            CC[(size_t)a * 2 * p + p + b] = -L0[a * p + b];
        }
    c->S = S;
    c->L0 = L0;

    // energy of X^k (needed before the preconditioner choice in the learned form)
    const bool learned_form = c->prm.precond == OFKS_PRECOND_LEARNED || c->prm.precond == OFKS_PRECOND_GRAPH;
    double energy = NAN;
    const int ee = learned_form ? 1 : std::max(1, c->prm.energy_every);
    if (scf) {
        double trl = 0.0;
        for (int i = 0; i < p; ++i) trl += L0[i * p + i];
        energy = c->prm.occupation * trl - c->scf_parts[3] - c->scf_parts[2] + c->scf_parts[1] + c->Enuc;
    } else if (c->k % ee == 0) {
        double tr;
        if (dense::trace_sinv_a(S, L0, p, tr)) energy = tr;
    }
    // learned form: fall back to the paper preconditioner for fallback_hold
    // iterations when the energy rises above the minimum (rule 0) or the
    // maximum (rule 1) of the last fallback_window iterates (no fallback when
    // fallback_window <= 0)
    bool use_learned = learned_form && c->lp_hold == 0;
    int fell_back = 0;
    if (learned_form && c->prm.fallback_window > 0 && std::isfinite(energy)) {
        if (use_learned && !c->ehist.empty()) {
            const double ref = c->prm.fallback_rule == 1 ? *std::max_element(c->ehist.begin(), c->ehist.end())
                                                         : *std::min_element(c->ehist.begin(), c->ehist.end());
            if (energy > ref + 1e-12 * std::fabs(energy)) {
                c->lp_hold = std::max(1, c->prm.fallback_hold);
                use_learned = false;
                fell_back = 1;
            }
        }
        c->ehist.push_back(energy);
        const size_t W = (size_t)c->prm.fallback_window;
        while (c->ehist.size() > W) c->ehist.erase(c->ehist.begin());
    }
    // ... or when the fallback_stall iterates before this one did not halve
    // the lowest residual (a stall while the energy still falls)
    const int S_stall = c->prm.fallback_stall;
    const int nr = (int)c->relmin.size();   // iterates evaluated before this one
    if (learned_form && use_learned && S_stall > 0 && nr > S_stall &&
        c->relmin[nr - 1] > 0.5 * c->relmin[nr - 1 - S_stall]) {
        c->lp_hold = std::max(1, c->prm.fallback_hold);
        use_learned = false;
        fell_back = 1;
    }
    const bool use_paper = c->prm.precond == OFKS_PRECOND_PAPER || (learned_form && !use_learned);
    const int kind = use_learned ? c->prm.precond : (use_paper ? OFKS_PRECOND_PAPER : OFKS_PRECOND_NONE);

    std::vector<double> shift(p, 0.0);
    std::vector<uint8_t> neg(p, 0);
    bool any_active = false;
    for (int i = 0; i < p; ++i) {
        const double li = c->prm.precond_lambda == 0 ? lam_diag[i] : L0[i * p + i];
        shift[i] = li;
        neg[i] = li < 0.0 ? 1 : 0;
        any_active |= use_paper && neg[i];
    }
    std::vector<uint8_t> act(p, 0);
    for (int i = 0; i < p; ++i) act[i] = (use_paper && neg[i]) ? 1 : 0;
    if (c->timing) {   // the serial host share: symmetrization, multiplier, energy, fallback rules
        Timer &th = c->timers["host"];
        th.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
        th.launches += 1;
    }
    if (!scf) CHK(upload<T>(c, B.dinv, dn));
    CHK(upload<T>(c, B.CC, CC));
    CHK(upload<T>(c, B.lam, shift));
    CHK(upload_bytes(c, c->active, use_learned ? neg.data() : act.data(), p));

    // G, R (kkt) and the start of the CG (paper) or the column norms of G (learned)
    int gx = 0;
    const int epi = (use_paper && any_active) ? EPI_GRAD_PCG : (use_learned ? EPI_GRAD_NORM : EPI_GRAD);
    const int gy = rowgemm_grid_y(2 * p);
    CHK(ensure_part(c, (size_t)c->gemm_rows * gy * (1 + p)));
    {
        // built after the partial buffer is final: it carries that pointer
        GradArgs ga{B.HX, B.P, B.R, B.D, c->lhd, c->bd, B.lam, c->active, c->part};
        {
            Scope sc(c, "update_a");
            HIPCHK(launch_rowgemm<T>(c->stream, epi, n, p, 2 * p, c->gemm_rows, B.BX, B.dinv, B.CC, nullptr, ga,
                                     &gx));
        }
        HIPCHK(launch_colsum(c->stream, (int64_t)gx * gy, 1 + p, c->part, c->red));
    }
    std::vector<double> r2;
    CHK(download(c, r2, c->red, 1 + p));
    const double kkt = std::sqrt(std::max(0.0, r2[0]));
    if (c->kkt0 < 0) c->kkt0 = kkt;
    // relative to kkt_0; a start that is already stationary (kkt_0 = 0) is
    // judged by the absolute value
    const double rel = c->kkt0 > 0.0 ? (kkt + fea) / c->kkt0 : kkt + fea;
    c->last_kkt = kkt;
    c->last_fea = fea;
    c->last_rel = rel;
    c->relmin.push_back(c->relmin.empty() ? rel : std::min(rel, c->relmin.back()));
    c->last_energy = energy;
    if (st) {
        st->k = c->k;
        st->kkt = kkt;
        st->fea = fea;
        st->rel = rel;
        st->energy = energy;
        st->eta = c->eta;
        st->precision = std::is_same<T, double>::value ? OFKS_F64 : OFKS_F32;
        st->precond_used = kind;
        st->fell_back = fell_back;
    }
    if (!std::isfinite(rel))
        return fail(c, OFKS_ENONFINITE, "non-finite residual at k=%d: kkt=%g fea=%g kkt0=%g", c->k, kkt, fea,
                    c->kkt0);
    if (rel < c->prm.tol || c->k >= c->prm.max_iter) {
        *stop = true;
        if (st) st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return OFKS_OK;
    }
    if (c->lp_hold > 0 && !use_learned) c->lp_hold -= 1;
    if (kind != c->last_kind) c->have_prev = false;   // BB restarts, eta carries over
    c->last_kind = kind;

    // graph-form training snapshots: G of this iterate and its shifts (FP64 plain method)
    if (c->gl_cap && std::is_same<T, double>::value && use_paper && any_active && c->gl_cap_count < c->gl_cap_max &&
        c->k % c->gl_cap_every == 0) {
        double *slot = c->gl_cap + (size_t)c->gl_cap_count * n * p;
        GradArgs gn{B.HX, slot, B.R, B.D, c->lhd, c->bd, B.lam, c->active, c->part};
        HIPCHK(launch_rowgemm<T>(c->stream, EPI_GRAD_NORM, n, p, 2 * p, c->gemm_rows, B.BX, B.dinv, B.CC, nullptr, gn,
                                 &gx));
        c->gl_cap_lam.insert(c->gl_cap_lam.end(), shift.begin(), shift.end());
        c->gl_cap_count += 1;
    }
    // training samples: keep G (and its column norms) before the CG overwrites it
    const bool collect = c->lp_buf && use_paper && any_active && c->lp_count < c->lp_cap;
    if (collect) {
        GradArgs gn{B.HX, B.P, B.R, B.D, c->lhd, c->bd, B.lam, c->active, c->part};
        HIPCHK(launch_rowgemm<T>(c->stream, EPI_GRAD_NORM, n, p, 2 * p, c->gemm_rows, B.BX, B.dinv, B.CC, nullptr, gn,
                                 &gx));
        HIPCHK(launch_colsum(c->stream, (int64_t)gx * gy, 1 + p, c->part, c->red));
        HIPCHK(hipMemcpyAsync(c->g2, c->red + 1, p * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(B.BX, B.P, (size_t)n * p * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        if (c->lp_objective == 1) {
            // u = T (J G): D holds J G on the active columns here
            const size_t bytes = (size_t)n * p * sizeof(T);
            if (c->lp_u_bytes < bytes) {
                char *u = (char *)c->lp_u;
                if (u) CHK(sync(c));   // the previous buffer may still be read by queued work
                dfree(c, u);
                c->lp_u = nullptr;
                c->lp_u_bytes = 0;
                CHK(dalloc(c, &u, bytes));
                c->lp_u = u;
                c->lp_u_bytes = bytes;
            }
            int used = 0;
            CHK(spmm_shift<T>(c, p, lbT<T>(c), B.lam, c->active, B.D, (T *)c->lp_u, &used));
        }
    }

    // preconditioner: columnwise Jacobi-PCG from zero, fixed iteration count
    if (use_paper && any_active) {
        CHK(upload_bytes(c, c->rz, r2.data() + 1, p * sizeof(double)));
        CHK(pcg_run<T>(c, c->prm.pcg_iters, n, p, c->active, B.lam, lbT<T>(c), B.D, B.HX, B.P, B.R, B.alpha, B.beta,
                       c->rz));
    }
    if (collect) {
        // t = T^-1 g (this step's P), every lp_stride-th row; per-column weights
        // n / <t, t> (objective 0) or n / <g, t> (objective 1)
        std::vector<double> pp;
        CHK(coldot<T>(c, c->lp_objective == 1 ? B.BX : B.P, B.P, pp));
        std::vector<double> w(p);
        for (int i = 0; i < p; ++i) w[i] = pp[i] > 0 ? (double)n / pp[i] : 0.0;
        CHK(upload<double>(c, c->tw, w));
        const int64_t stride = std::max<int64_t>(1, c->lp_stride);
        const int64_t offset = (c->k * 7919) % stride;
        int64_t rows = (n - offset + stride - 1) / stride;
        rows = std::min<int64_t>(rows, (c->lp_cap - c->lp_count) / p);
        if (rows > 0) {
            HIPCHK(launch_lp_sample<T>(c->stream, n, p, offset, stride, rows, c->lp_objective, B.BX, B.P,
                                       (const T *)c->lp_u, c->lhd, c->bd, c->hd, B.lam, c->active, c->g2, c->tw,
                                       c->lp_buf + c->lp_count * LP_SAMPLE));
            c->lp_count += rows * p;
        }
    }
    if (use_learned && c->prm.precond == OFKS_PRECOND_GRAPH) {
        // P = Z + ft J (G - T Z), Z = exp(fs) J G: heads, one shifted SpMM (Z in D, T Z in HX), sweep
        if (!c->gl_ready) return fail(c, OFKS_ESTATE, "graph preconditioner: no weights (ofks_gl_set_weights)");
        CHK(ensure_gl_ft(c, (size_t)n * p));
        HIPCHK(hipMemcpyAsync(c->g2, c->red + 1, p * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        {
            Scope sc(c, "graph");
            HIPCHK(launch_gl_heads<T>(c->stream, n, p, B.P, c->lhd, c->bd, c->hd, B.lam, c->active, c->g2, c->gl_W,
                                      c->gl_norm, B.D, c->gl_ft));
        }
        // sweep s: P_s = P_{s-1} + ft J (G - T P_{s-1}), P_0 = Z; G stays in P
        // until the last sweep writes there; the others alternate R and D
        const int m = std::max(1, c->prm.graph_sweeps);
        T *src = B.D;
        for (int sw = 1; sw <= m; ++sw) {
            int used = 0;
            CHK(spmm_shift<T>(c, p, lbT<T>(c), B.lam, c->active, src, B.HX, &used));
            T *dst = sw == m ? B.P : (src == B.R ? B.D : B.R);
            Scope sc(c, "graph");
            HIPCHK(launch_gl_out<T>(c->stream, n, p, B.P, src, c->gl_ft, B.HX, c->lhd, c->bd, B.lam, c->active, dst,
                                    (T *)nullptr));
            src = dst;
        }
    } else if (use_learned) {
        if (!c->lp_ready) return fail(c, OFKS_ESTATE, "learned preconditioner: no weights (ofks_lp_set_weights)");
        HIPCHK(hipMemcpyAsync(c->g2, c->red + 1, p * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        Scope sc(c, "mlp");
        HIPCHK(launch_lp_apply<T>(c->stream, n, p, B.P, c->lhd, c->bd, c->hd, B.lam, c->active, c->g2, c->lp_W,
                                  c->lp_norm));
    }

    // BB step
    CHK(ensure_part(c, (size_t)c->grid * 5));
    {
        Scope sc(c, "bbdot");
        HIPCHK(launch_bbdot<T>(c->stream, c->grid, n, p, B.Xt, B.dinv, B.P, c->have_prev ? B.Xp : nullptr,
                               c->have_prev ? B.Pp : nullptr, c->part));
    }
    HIPCHK(launch_colsum(c->stream, c->grid, 5, c->part, c->red));
    std::vector<double> s5;
    CHK(download(c, s5, c->red, 5));
    if (s5[3] == 0.0) {
        // P = 0: X is a fixed point of the update (a stationary start, e.g. a
        // single DOF); nothing further to do
        *stop = true;
        if (st) st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return OFKS_OK;
    }
    if (!c->have_prev) {
        if (c->eta0 <= 0.0) c->eta0 = c->prm.eta0 > 0 ? c->prm.eta0 : std::sqrt(s5[3]) / std::sqrt(s5[4]);
        if (c->eta <= 0.0) c->eta = c->eta0;
    } else {
        c->eta = bb_eta(c->prm.step_rule, c->k, s5[0], s5[1], s5[2], c->eta, c->eta0);
    }
    if (!(c->eta > 0.0) || !std::isfinite(c->eta)) return fail(c, OFKS_ENONFINITE, "bad step parameter");

    {
        Scope sc(c, "update_b");
        HIPCHK(launch_update_b<T>(c->stream, n, p, B.dinv, (T)c->eta, B.P, B.Xt, B.Xp));
    }
    std::swap(B.P, B.Pp);
    c->have_prev = true;
    c->k += 1;
    CHK(sync(c));
    if (st) {
        st->eta = c->eta;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return OFKS_OK;
}

// switch the iteration from FP32 to FP64 blocks (refinement sweeps)
// The three blocks that carry the iteration's state (X~, X^{k-1}, P^{k-1})
// are converted one at a time, after the FP32 scratch blocks are freed, so the
// peak is the FP64 set plus at most three FP32 blocks (at n = 8e6, p = 512:
// 262 GB + 49 GB falling to 262 GB, where both full sets would need 393 GB).
int promote_to_f64_impl(ofks_ctx *c) {
    Blocks<float> &F = c->b32;
    Blocks<double> &D = c->b64;
    const size_t np = (size_t)c->n * c->p;
    if (c->ws_base && c->ws_carve && ws_block_set(c->n, c->p, sizeof(double), 8) > c->ws_f64_cap)
        return fail(c, OFKS_ECAPACITY, "workspace: no room kept for the FP64 blocks (sized with refine_tol = 0)");
    CHK(sync(c));
    free_pcg_history(c);   // FP32 directions; the FP64 set comes first
    dfree(c, F.P);
    dfree(c, F.HX);
    dfree(c, F.BX);
    dfree(c, F.R);
    dfree(c, F.D);
    // with a workspace the FP64 set goes to the region set_x0 / state_set
    // kept for it (the start block's setup blocks there are dead)
    const size_t ws_hi = c->ws_off;
    if (c->ws_base && c->ws_carve) c->ws_off = c->ws_f64_base;
    float *src[3] = {F.Xt, F.Xp, F.Pp};
    double **dst[3] = {&D.Xt, &D.Xp, &D.Pp};
    for (int i = 0; i < 3; ++i) {
        CHK(walloc(c, dst[i], np));
        HIPCHK(launch_convert<float, double>(c->stream, (int64_t)np, src[i], *dst[i]));
        CHK(sync(c));
        dfree(c, src[i]);
    }
    F.Xt = F.Xp = F.Pp = nullptr;
    free_blocks<float>(c);
    dfree(c, c->hb32);   // the FP32 matrix copies are rebuilt if an FP32 run starts again
    dfree(c, c->lb32);
    CHK(walloc(c, &D.P, np));
    CHK(walloc(c, &D.HX, np));
    CHK(walloc(c, &D.BX, np));
    CHK(walloc(c, &D.R, np));
    CHK(walloc(c, &D.D, np));
    CHK(walloc(c, &D.dinv, c->p));
    CHK(walloc(c, &D.CC, (size_t)c->p * 2 * c->p));
    CHK(walloc(c, &D.lam, c->p));
    CHK(walloc(c, &D.alpha, c->p));
    CHK(walloc(c, &D.beta, c->p));
    if (c->ws_base && c->ws_carve) c->ws_off = std::max(ws_hi, c->ws_off);
    c->prec = OFKS_F64;
    return OFKS_OK;
}

// a switch that fails part-way leaves no usable iterate
int promote_to_f64(ofks_ctx *c) {
    const int rc = promote_to_f64_impl(c);
    if (rc < 0) c->has_x = false;
    return rc;
}

// turns workspace carving on for the duration of an entry point
struct WsScope {
    ofks_ctx *c;
    bool prev;
    explicit WsScope(ofks_ctx *c_) : c(c_), prev(c_->ws_carve) { c->ws_carve = true; }
    ~WsScope() { c->ws_carve = prev; }
};

// An FP64 run's set_x0 allocates only the three blocks the start block's
// orthonormalization uses; the other five come with the first call that
// needs them, so a caller can release its start block in between (at
// n = 8e6, p = 512 the eight FP64 blocks take 262 GB of the 288).
int complete_blocks(ofks_ctx *c) {
    if (c->prec != OFKS_F64 || c->b64.Xp) return OFKS_OK;
    WsScope wss(c);
    Blocks<double> &B = c->b64;
    const size_t np = (size_t)c->n * c->p;
    int rc = walloc(c, &B.Xp, np);
    if (rc == OFKS_OK) rc = walloc(c, &B.P, np);
    if (rc == OFKS_OK) rc = walloc(c, &B.Pp, np);
    if (rc == OFKS_OK) rc = walloc(c, &B.R, np);
    if (rc == OFKS_OK) rc = walloc(c, &B.D, np);
    if (rc != OFKS_OK) {
        dfree(c, B.Xp);
        dfree(c, B.P);
        dfree(c, B.Pp);
        dfree(c, B.R);
        dfree(c, B.D);
    }
    return rc;
}

// Releases every piece of device state a workspace may hold (those inside
// the workspace are only forgotten); the iterate is gone afterwards.
void release_state(ofks_ctx *c) {
    free_pcg_history(c);
    free_blocks<double>(c);
    free_blocks<float>(c);
    dfree(c, c->active);
    dfree(c, c->rz);
    dfree(c, c->g2);
    dfree(c, c->tw);
    dfree(c, c->part);
    c->part_cap = 0;
    dfree(c, c->gl_ft);
    c->gl_ft_cap = 0;
    dfree(c, c->hb32);
    dfree(c, c->lb32);
    free_scf_work(c);
    c->has_x = false;
}

// set_x0 and state_set rebuild the whole iteration state: with a workspace,
// release every carved piece and start again from its beginning
void ws_restart(ofks_ctx *c) {
    if (!c->ws_base) return;
    release_state(c);
    c->ws_off = 0;
}

int check_ready(ofks_ctx *c) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "no system: call ofks_assemble or ofks_csr_load");
    if (!c->has_params) return fail(c, OFKS_ESTATE, "call ofks_set_params first");
    if (!c->has_x) return fail(c, OFKS_ESTATE, "call ofks_set_x0 first");
    return OFKS_OK;
}

int ensure_f32_matrices(ofks_ctx *c) {
    if (!(c->hb32 && c->lb32)) {
        dfree(c, c->hb32);   // both or neither
        dfree(c, c->lb32);
        int rc = walloc(c, &c->hb32, c->nnz);
        if (rc == OFKS_OK) rc = walloc(c, &c->lb32, c->nnz);
        if (rc != OFKS_OK) {
            dfree(c, c->hb32);
            dfree(c, c->lb32);
            return rc;
        }
    }
    HIPCHK(launch_pairs_to_f32(c->stream, c->nnz, c->hb, c->hb32));
    HIPCHK(launch_pairs_to_f32(c->stream, c->nnz, c->lb, c->lb32));
    return OFKS_OK;
}

void free_halo(ofks_ctx *c) {
    dfree(c, c->halo_row0);
    dfree(c, c->halo_off);
    dfree(c, c->halo_idx);
    dfree(c, c->halo_rbase);
    dfree(c, c->halo_brp);
    dfree(c, c->halo_lcol);
    c->halo_nb = 0;
}

// LDS-halo plan from the CSR pattern on the device (halo_plan.hpp), checked
// independently on the host before upload.  A row with more entries than a
// wave has lanes, or alone more columns than the halo holds, leaves no plan:
// the row-gather kernel serves every p then.
int build_halo_plan(ofks_ctx *c) {
    free_halo(c);
    const int64_t n = c->n, nnz = c->nnz;
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> col(nnz);
    HIPCHK(hipMemcpyAsync(rp.data(), c->rp, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(col.data(), c->col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (rp[n] != nnz) return fail(c, OFKS_EINVAL, "csr: row_ptr[n] != nnz");
    const int HM = halo_max_rows(), RM = halo_max_block_rows(), EM = halo_max_row_entries();
    HaloPlan P;
    int64_t where = 0;
    int rc = halo_plan_build(n, rp.data(), col.data(), HM, RM, EM, P, &where);
    if (rc == HALO_TOO_WIDE) return OFKS_OK;
    if (rc == HALO_BAD_ROWPTR) return fail(c, OFKS_EINVAL, "csr: row_ptr malformed at row %lld", (long long)where);
    if (rc == HALO_BAD_COLUMN) return fail(c, OFKS_EINVAL, "csr: column index out of range at entry %lld",
                                           (long long)where);
    if (rc != HALO_OK || halo_plan_check(n, rp.data(), col.data(), HM, RM, EM, P, &where) != HALO_OK)
        return fail(c, OFKS_EINTERNAL, "halo plan: consistency check failed at %lld", (long long)where);
    const int64_t nb = P.nb();
    CHK(dalloc(c, &c->halo_row0, nb + 1));
    CHK(dalloc(c, &c->halo_off, nb + 1));
    // the kernel reads each block's halo rows at a fixed stride, padded with its last row
    const int HS = halo_pad_stride();
    std::vector<int32_t> hpad((size_t)nb * HS);
    for (int64_t k = 0; k < nb; ++k) {
        const int64_t h0 = P.hoff[k], hn = P.hoff[k + 1] - h0;   // 1 <= hn <= HS (the plan check)
        for (int s = 0; s < HS; ++s) hpad[(size_t)k * HS + s] = P.halo[h0 + std::min<int64_t>(s, hn - 1)];
    }
    // and each block's row pointers at a fixed stride, padded with the next block's first
    const int BS = halo_row_ptr_stride();
    std::vector<int64_t> bpad((size_t)nb * BS);
    for (int64_t k = 0; k < nb; ++k)
        for (int j = 0; j < BS; ++j) bpad[(size_t)k * BS + j] = rp[std::min(P.row0[k] + j, P.row0[k + 1])];
    CHK(dalloc(c, &c->halo_idx, hpad.size()));
    CHK(dalloc(c, &c->halo_brp, bpad.size()));
    CHK(dalloc(c, &c->halo_rbase, nb));
    CHK(dalloc(c, &c->halo_lcol, nnz));
    HIPCHK(hipMemcpyAsync(c->halo_row0, P.row0.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->halo_off, P.hoff.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->halo_idx, hpad.data(), hpad.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->halo_lcol, P.lcol.data(), nnz * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->halo_rbase, P.rbase.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->halo_brp, bpad.data(), bpad.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->halo_nb = nb;
    return OFKS_OK;
}

int alloc_system_common(ofks_ctx *c) {
    CHK(dalloc(c, &c->lhd, c->n));
    CHK(dalloc(c, &c->bd, c->n));
    CHK(dalloc(c, &c->hd, c->n));
    CHK(dalloc(c, &c->red, 2 * 1024 * 1024 + 64));   // p x 2p partial sums for p <= 1024
    return OFKS_OK;
}

void free_system(ofks_ctx *c) {
    drop_cg_graph(c);
    dfree(c, c->rp);
    dfree(c, c->col);
    dfree(c, c->Lv);
    dfree(c, c->Bv);
    dfree(c, c->Mv);
    dfree(c, c->hb);
    dfree(c, c->lb);
    dfree(c, c->hb32);
    dfree(c, c->lb32);
    dfree(c, c->lhd);
    dfree(c, c->bd);
    dfree(c, c->hd);
    dfree(c, c->Ldiag);
    dfree(c, c->red);
    free_halo(c);
    c->has_system = false;
    c->assembled = false;
    c->has_lhalf = false;
}

template <typename T>
int spmm_ex_typed(ofks_ctx *c, int p, int op, const double *lam, const T *X, T *Y1, T *Y2) {
    if (op == 0) return spmm_pair<T>(c, p, hbT<T>(c), X, Y1, Y2, 0);
    T *lamd = nullptr;
    uint8_t *act = nullptr;
    CHK(dalloc(c, &lamd, p));
    CHK(dalloc(c, &act, p));
    std::vector<double> lv(lam, lam + p);
    std::vector<uint8_t> ah(p);
    for (int i = 0; i < p; ++i) ah[i] = lam[i] < 0.0 ? 1 : 0;
    int rc = upload<T>(c, lamd, lv);
    if (rc >= 0) rc = upload_bytes(c, act, ah.data(), p);
    int used = 0;
    if (rc >= 0) rc = spmm_shift<T>(c, p, lbT<T>(c), lamd, act, X, Y1, &used);
    const int rs = sync(c);
    dfree(c, lamd);
    dfree(c, act);
    return rc < 0 ? rc : rs;
}
// Device address of `scratch` on the current device, resolved once per
// device (each device holds its own copy at its own address).
int noalloc_scratch(int device, double **out) {
    static std::mutex mu;
    static std::map<int, double *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return OFKS_EHIP;
        it = addr.emplace(device, (double *)ptr).first;
    }
    *out = it->second;
    return OFKS_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void ofks_default_params(ofks_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->beta = 1.0;
    p->eta0 = 0.0;
    p->tol = 1e-8;
    p->step_rule = OFKS_STEP_BB2;
    p->precond = OFKS_PRECOND_PAPER;
    p->pcg_iters = 10;
    p->precision = OFKS_F64;
    p->precond_lambda = 0;
    p->max_iter = 1000;
    p->occupation = 2.0;
    p->scf = 0;
    p->energy_every = 1;
    p->refine_tol = 0.0;
    p->poisson_rtol = 1e-12;
    p->poisson_max_iter = 20000;
    p->fallback_window = 5;
    p->fallback_hold = 20;
    p->fallback_rule = 0;
    p->use_graphs = 1;
    p->algorithm = 0;
    p->fallback_stall = 30;
    p->poisson_adapt = 0.0;
    p->graph_sweeps = 1;
}

int ofks_create(ofks_ctx **out, void *hip_stream) {
    if (!out) return OFKS_EINVAL;
    ofks_ctx *c = new ofks_ctx();
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess || noalloc_scratch(c->device, &c->scratch_dev) != OFKS_OK) {
        delete c;
        return OFKS_EHIP;
    }
    ofks_default_params(&c->prm);
    *out = c;
    return OFKS_OK;
}

int ofks_destroy(ofks_ctx *c) {
    if (!c) return OFKS_OK;
    (void)hipStreamSynchronize(c->stream);
    drop_cg_graph(c);
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    if (c->hup) (void)hipHostFree(c->hup);
    for (auto &pd : c->pending) {
        (void)hipEventDestroy(pd.a);
        (void)hipEventDestroy(pd.b);
    }
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    delete c;
    return OFKS_OK;
}

const char *ofks_last_error(const ofks_ctx *c) { return c ? c->err.c_str() : "null context"; }

int ofks_mesh_load(ofks_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets,
                   const uint8_t *dirichlet) {
    if (!c) return OFKS_EINVAL;
    if (n_nodes <= 0 || n_tets <= 0 || !xyz || !tets || !dirichlet)
        return fail(c, OFKS_EINVAL, "mesh_load: empty mesh or null pointer");
    if (n_nodes >= (int64_t(1) << 31) || n_tets >= (int64_t(1) << 29))
        return fail(c, OFKS_ECAPACITY, "mesh_load: mesh too large for 32-bit indices");
    for (int64_t i = 0; i < 4 * n_tets; ++i)
        if (tets[i] < 0 || tets[i] >= n_nodes) return fail(c, OFKS_EINVAL, "mesh_load: node index out of range");
    dfree(c, c->xyz);
    dfree(c, c->tets);
    dfree(c, c->dir);
    CHK(dalloc(c, &c->xyz, 3 * n_nodes));
    CHK(dalloc(c, &c->tets, 4 * n_tets));
    CHK(dalloc(c, &c->dir, n_nodes));
    HIPCHK(hipMemcpyAsync(c->xyz, xyz, 3 * n_nodes * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->tets, tets, 4 * n_tets * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->dir, dirichlet, n_nodes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->n_nodes = n_nodes;
    c->n_tets = n_tets;
    c->has_mesh = true;
    c->has_x = false;
    return OFKS_OK;
}

int ofks_nuclei_set(ofks_ctx *c, int32_t M, const double *Z, const double *R) {
    if (!c) return OFKS_EINVAL;
    if (M < 0 || (M > 0 && (!Z || !R))) return fail(c, OFKS_EINVAL, "nuclei_set: bad arguments");
    c->M = M;
    c->Zh.assign(Z, Z + M);
    c->Rh.assign(R, R + 3 * M);
    dfree(c, c->Zd);
    dfree(c, c->Rd);
    CHK(dalloc(c, &c->Zd, std::max(M, 1)));
    CHK(dalloc(c, &c->Rd, 3 * std::max(M, 1)));
    if (M > 0) {
        HIPCHK(hipMemcpy(c->Zd, Z, M * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->Rd, R, 3 * M * sizeof(double), hipMemcpyHostToDevice));
    }
    double e = 0.0;
    for (int j = 0; j < M; ++j)
        for (int k = j + 1; k < M; ++k) {
            const double dx = R[3 * j] - R[3 * k], dy = R[3 * j + 1] - R[3 * k + 1], dz = R[3 * j + 2] - R[3 * k + 2];
            e += Z[j] * Z[k] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
    c->Enuc = e;
    c->has_nuclei = true;
    return OFKS_OK;
}

int ofks_assemble(ofks_ctx *c) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_mesh) return fail(c, OFKS_ESTATE, "assemble: no mesh");
    if (!c->has_nuclei) return fail(c, OFKS_ESTATE, "assemble: no nuclei (call ofks_nuclei_set, M may be 0)");
    hipStream_t s = c->stream;
    const int64_t nn = c->n_nodes, nt = c->n_tets;
    free_system(c);
    dfree(c, c->dof);
    dfree(c, c->iptr);
    dfree(c, c->inc);
    dfree(c, c->geom);
    dfree(c, c->vext_q);
    int32_t *flags = nullptr, *errd = nullptr, *cursor = nullptr;
    int64_t *scan = nullptr, *bsum = nullptr;
    CHK(dalloc(c, &flags, nn + 1));
    CHK(dalloc(c, &scan, nn + 1));
    CHK(dalloc(c, &bsum, nn / 1024 + 2));
    CHK(dalloc(c, &errd, 1));
    CHK(dalloc(c, &cursor, nn));
    CHK(dalloc(c, &c->dof, nn));
    HIPCHK(hipMemsetAsync(errd, 0, sizeof(int32_t), s));
    {
        Scope sc(c, "assemble");
        // interior DOF numbering in node order
        HIPCHK(launch_interior_flags(s, nn, c->dir, flags));
        HIPCHK(scan_exclusive(s, nn, flags, scan, bsum));
        HIPCHK(launch_dof(s, nn, c->dir, scan, c->dof));
    }
    int64_t n = 0;
    HIPCHK(hipMemcpyAsync(&n, scan + nn, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (n <= 0) return fail(c, OFKS_EINVAL, "assemble: no interior nodes");
    // node -> tetrahedra incidence
    CHK(dalloc(c, &c->iptr, nn + 1));
    CHK(dalloc(c, &c->inc, 4 * nt));
    HIPCHK(hipMemsetAsync(flags, 0, (nn + 1) * sizeof(int32_t), s));
    HIPCHK(hipMemsetAsync(cursor, 0, nn * sizeof(int32_t), s));
    {
        Scope sc(c, "assemble");
        HIPCHK(launch_inc_count(s, nt, c->tets, flags));
        HIPCHK(scan_exclusive(s, nn, flags, c->iptr, bsum));
        HIPCHK(launch_inc_fill(s, nt, c->tets, c->iptr, cursor, c->inc));
        HIPCHK(launch_inc_sort(s, nn, c->iptr, c->inc, errd));
    }
    // CSR pattern
    CHK(dalloc(c, &c->rp, n + 1));
    int32_t *rowcnt = nullptr;
    CHK(dalloc(c, &rowcnt, n + 1));
    {
        Scope sc(c, "assemble");
        HIPCHK(launch_row_pattern(s, nn, 0, c->dof, c->iptr, c->inc, c->tets, rowcnt, nullptr, nullptr, errd));
        HIPCHK(scan_exclusive(s, n, rowcnt, c->rp, bsum));
    }
    int64_t nnz = 0;
    int32_t errh = 0;
    HIPCHK(hipMemcpyAsync(&nnz, c->rp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&errh, errd, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (errh & 1) return fail(c, OFKS_ECAPACITY, "assemble: a node touches more than 128 tetrahedra");
    if (errh & 2) return fail(c, OFKS_ECAPACITY, "assemble: a matrix row has more than 64 entries");
    if (nnz >= (int64_t(1) << 31)) return fail(c, OFKS_ECAPACITY, "assemble: nnz exceeds 2^31");
    CHK(dalloc(c, &c->col, nnz));
    CHK(dalloc(c, &c->Lv, nnz));
    CHK(dalloc(c, &c->Bv, nnz));
    CHK(dalloc(c, &c->Mv, nnz));
    CHK(dalloc(c, &c->hb, nnz));
    CHK(dalloc(c, &c->lb, nnz));
    CHK(dalloc(c, &c->geom, 13 * nt));
    CHK(dalloc(c, &c->vext_q, 4 * nt));
    c->n = n;
    c->nnz = nnz;
    CHK(alloc_system_common(c));
    {
        Scope sc(c, "assemble");
        HIPCHK(launch_row_pattern(s, nn, 1, c->dof, c->iptr, c->inc, c->tets, nullptr, c->rp, c->col, errd));
        HIPCHK(launch_tet_geom(s, nt, c->xyz, c->tets, c->geom, errd));
        HIPCHK(launch_vext(s, nt, c->xyz, c->tets, c->M, c->Zd, c->Rd, c->vext_q));
        HIPCHK(launch_assemble(s, nn, 0, c->dof, c->iptr, c->inc, c->tets, c->geom, c->vext_q, c->rp, c->col, c->Lv,
                               c->Bv, c->Mv, c->hb, c->lb, c->lhd, c->bd, c->hd));
    }
    HIPCHK(hipMemcpyAsync(&errh, errd, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (errh & 4) return fail(c, OFKS_EINVAL, "assemble: degenerate tetrahedron");
    dfree(c, flags);
    dfree(c, scan);
    dfree(c, bsum);
    dfree(c, errd);
    dfree(c, cursor);
    dfree(c, rowcnt);
    // SCF work arrays (the CG graph holds pointers to some of them)
    drop_cg_graph(c);
    dfree(c, c->rho_q);
    dfree(c, c->eps_q);
    dfree(c, c->vxc_q);
    dfree(c, c->veff_q);
    dfree(c, c->bvec);
    dfree(c, c->U);
    dfree(c, c->cg_r);
    dfree(c, c->cg_d);
    dfree(c, c->cg_q);
    dfree(c, c->cg_sc);
    dfree(c, c->cg_part);
    // the quadrature-point arrays of the density (4 per tetrahedron, four
    // of them: 6.2 GB at n = 8e6) are allocated on first use (ensure_scf_work)
    CHK(dalloc(c, &c->bvec, n));
    CHK(dalloc(c, &c->U, n));
    CHK(dalloc(c, &c->cg_r, n));
    CHK(dalloc(c, &c->cg_d, n));
    CHK(dalloc(c, &c->cg_q, n));
    CHK(dalloc(c, &c->cg_sc, 8));
    CHK(dalloc(c, &c->cg_part, 4 * CG_BLOCKS));
    HIPCHK(hipMemsetAsync(c->U, 0, n * sizeof(double), s));
    CHK(build_halo_plan(c));
    c->has_system = true;
    c->assembled = true;
    c->has_lhalf = true;
    c->has_x = false;
    return sync(c);
}

int ofks_csr_info(ofks_ctx *c, int64_t *n, int64_t *nnz) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "no system");
    if (n) *n = c->n;
    if (nnz) *nnz = c->nnz;
    return OFKS_OK;
}

int ofks_csr_get(ofks_ctx *c, int64_t *row_ptr, int32_t *col, double *L, double *B, double *H) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "no system");
    hipStream_t s = c->stream;
    if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, c->rp, (c->n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (col) HIPCHK(hipMemcpyAsync(col, c->col, c->nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    double *tx = nullptr, *ty = nullptr;
    if (L || B || H) {
        CHK(dalloc(c, &tx, c->nnz));
        CHK(dalloc(c, &ty, c->nnz));
    }
    if (L) {
        if (!c->Lv) return fail(c, OFKS_ESTATE, "csr_get: no stiffness matrix for a loaded system");
        HIPCHK(hipMemcpyAsync(L, c->Lv, c->nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (B || H) {
        HIPCHK(launch_split_pairs(s, c->nnz, c->hb, tx, ty));
        if (H) HIPCHK(hipMemcpyAsync(H, tx, c->nnz * sizeof(double), hipMemcpyDeviceToHost, s));
        if (B) HIPCHK(hipMemcpyAsync(B, ty, c->nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    dfree(c, tx);
    dfree(c, ty);
    return OFKS_OK;
}

int ofks_csr_load(ofks_ctx *c, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                  const double *H, const double *B, const double *Lhalf) {
    if (!c) return OFKS_EINVAL;
    if (n <= 0 || nnz <= 0 || !row_ptr || !col || !H || !B) return fail(c, OFKS_EINVAL, "csr_load: bad arguments");
    free_system(c);
    hipStream_t s = c->stream;
    c->n = n;
    c->nnz = nnz;
    CHK(dalloc(c, &c->rp, n + 1));
    CHK(dalloc(c, &c->col, nnz));
    CHK(dalloc(c, &c->hb, nnz));
    CHK(dalloc(c, &c->lb, nnz));
    CHK(alloc_system_common(c));
    HIPCHK(hipMemcpyAsync(c->rp, row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(c->col, col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_make_pairs(s, nnz, H, B, c->hb));
    int32_t *errd = nullptr;
    CHK(dalloc(c, &errd, 1));
    HIPCHK(hipMemsetAsync(errd, 0, sizeof(int32_t), s));
    if (Lhalf) {
        HIPCHK(launch_make_pairs(s, nnz, Lhalf, B, c->lb));
        HIPCHK(launch_diag(s, n, c->rp, c->col, c->lb, c->lhd, c->bd, errd));
        c->has_lhalf = true;
    } else {
        HIPCHK(launch_make_pairs(s, nnz, B, B, c->lb));
        HIPCHK(launch_diag(s, n, c->rp, c->col, c->lb, nullptr, c->bd, errd));
        c->has_lhalf = false;
    }
    HIPCHK(launch_diag(s, n, c->rp, c->col, c->hb, c->hd, nullptr, errd));
    int32_t errh = 0;
    HIPCHK(hipMemcpyAsync(&errh, errd, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dfree(c, errd);
    if (errh) return fail(c, OFKS_EINVAL, "csr_load: a row has no diagonal entry");
    CHK(build_halo_plan(c));
    c->has_system = true;
    c->assembled = false;
    c->has_x = false;
    return OFKS_OK;
}

int ofks_set_params(ofks_ctx *c, const ofks_params *prm) {
    if (!c || !prm) return OFKS_EINVAL;
    if (!(prm->beta >= 0.0) || !(prm->tol > 0.0) || prm->max_iter < 0 || prm->pcg_iters < 0 ||
        prm->precond < 0 || prm->precond > 3 || prm->step_rule < 0 || prm->step_rule > 4 ||
        (prm->precision != OFKS_F64 && prm->precision != OFKS_F32) || prm->fallback_rule < 0 ||
        prm->fallback_rule > 1 || prm->algorithm < 0 || prm->algorithm > 1 || prm->spmm_mode < 0 ||
        prm->spmm_mode > 2 || !(prm->poisson_adapt >= 0.0) || !std::isfinite(prm->poisson_adapt) ||
        prm->graph_sweeps < 1 || prm->graph_sweeps > 64)
        return fail(c, OFKS_EINVAL, "set_params: invalid parameter");
    if (prm->precond == OFKS_PRECOND_PAPER && prm->pcg_iters < 1)
        return fail(c, OFKS_EINVAL, "set_params: the paper preconditioner needs pcg_iters >= 1");
    if (prm->scf && !c->assembled) return fail(c, OFKS_ESTATE, "set_params: SCF needs an assembled mesh");
    if (prm->precond == OFKS_PRECOND_PAPER && c->has_system && !c->has_lhalf)
        return fail(c, OFKS_EINVAL, "set_params: the paper preconditioner needs L/2 (csr_load without Lhalf)");
    if ((prm->precond == OFKS_PRECOND_LEARNED || prm->precond == OFKS_PRECOND_GRAPH) && c->has_system &&
        !c->has_lhalf)
        return fail(c, OFKS_EINVAL, "set_params: the learned preconditioner needs L/2 (its fallback is the paper's)");
    c->prm = *prm;
    if (c->prm.energy_every < 1) c->prm.energy_every = 1;
    c->has_params = true;
    return OFKS_OK;
}

// ---- caller-owned workspace -------------------------------------------------

int ofks_workspace_size(ofks_ctx *c, int32_t p, const ofks_params *prm, size_t *bytes) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "workspace_size: no system");
    if (!prm || !bytes || p <= 0 || p > 1024) return fail(c, OFKS_EINVAL, "workspace_size: bad arguments");
    // the pieces in the order set_x0 / state_set / step carve them
    size_t total = 4 * ws_piece((size_t)p * sizeof(double));                  // active, rz, g2, tw
    total += ws_piece(partials_needed(c, p) * sizeof(double));                 // per-block partial sums
    if (prm->precision == OFKS_F64) {
        total += ws_block_set(c->n, p, sizeof(double), 8);
    } else {
        total += ws_block_set(c->n, p, sizeof(double), prm->refine_tol > 0.0 ? 8 : 3);
        total += 2 * ws_piece((size_t)c->nnz * sizeof(float2));               // FP32 copies of H and L/2
        total += ws_block_set(c->n, p, sizeof(float), 8);
    }
    if (prm->precond == OFKS_PRECOND_GRAPH) total += ws_piece((size_t)c->n * p * sizeof(float));
    if (prm->scf) total += 4 * ws_piece((size_t)4 * c->n_tets * sizeof(double));
    *bytes = total;
    return OFKS_OK;
}

int ofks_set_workspace(ofks_ctx *c, void *dev_ws, size_t bytes) {
    if (!c) return OFKS_EINVAL;
    if (dev_ws && (reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0 || bytes == 0))
        return fail(c, OFKS_EINVAL, "set_workspace: need a 256-byte aligned, non-empty device buffer");
    CHK(sync(c));
    // the iteration state moves: whatever exists (pieces of an earlier
    // workspace included) is released, and set_x0 or state_set must follow
    release_state(c);
    c->ws_base = (char *)dev_ws;
    c->ws_size = dev_ws ? bytes : 0;
    c->ws_off = 0;
    return OFKS_OK;
}

int ofks_set_x0(ofks_ctx *c, int32_t p, const double *X0, int32_t orth) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "set_x0: no system");
    if (!c->has_params) return fail(c, OFKS_ESTATE, "set_x0: call ofks_set_params first");
    if (p <= 0 || p > 1024 || !X0) return fail(c, OFKS_EINVAL, "set_x0: need 1 <= p <= 1024 and a block");
    if (p > c->n) return fail(c, OFKS_EINVAL, "set_x0: p exceeds n");
    WsScope wss(c);
    c->has_x = false;   // until the new state is complete
    free_blocks<double>(c);
    free_blocks<float>(c);
    dfree(c, c->active);
    dfree(c, c->rz);
    dfree(c, c->g2);
    dfree(c, c->tw);
    ws_restart(c);
    c->p = p;
    c->prec = c->prm.precision;
    dfree(c, c->g2);
    dfree(c, c->tw);
    CHK(walloc(c, &c->active, p));
    CHK(walloc(c, &c->rz, p));
    CHK(walloc(c, &c->g2, p));
    CHK(walloc(c, &c->tw, p));
    CHK(ensure_part(c, partials_needed(c, p)));
    c->ws_f64_base = c->ws_off;
    CHK(alloc_blocks<double>(c, true));   // the start block's setup; complete_blocks adds the rest
    if (c->ws_base && c->prec == OFKS_F32) {
        c->ws_f64_cap = ws_f64_region(c, p);
        c->ws_off = c->ws_f64_base + c->ws_f64_cap;
    }
    Blocks<double> &B = c->b64;
    HIPCHK(hipMemcpyAsync(B.Xt, X0, (size_t)c->n * p * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (orth) {
        // Cholesky-based Gram-Schmidt: V^T B V = R^T R, X0 = V R^-1
        CHK(spmm_pair<double>(c, p, c->hb, B.Xt, B.BX, nullptr, 1));
        std::vector<double> St, Lt;
        CHK(gram<double>(c, B.Xt, B.BX, B.BX, St, Lt));
        for (int a = 0; a < p; ++a)
            for (int b = a + 1; b < p; ++b) St[a * p + b] = St[b * p + a] = 0.5 * (St[a * p + b] + St[b * p + a]);
        if (!dense::cholesky(St, p)) return fail(c, OFKS_ENOTSPD, "set_x0: V^T B V is not positive definite");
        std::vector<double> Li = dense::lower_inverse(St, p);
        std::vector<double> Rinv((size_t)p * p);  // R^-1 = (L^-1)^T, upper triangular
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) Rinv[a * p + b] = Li[b * p + a];
        std::vector<double> ones(p, 1.0);
        CHK(upload<double>(c, B.dinv, ones));
        CHK(upload<double>(c, B.CC, Rinv));
        GradArgs ga{};
        HIPCHK(launch_rowgemm<double>(c->stream, EPI_PLAIN, c->n, p, p, c->gemm_rows, B.Xt, B.dinv, B.CC, B.HX, ga,
                                      nullptr));
        std::swap(B.Xt, B.HX);
    } else {
        // a block taken as given must have no column of zero B-norm
        CHK(spmm_pair<double>(c, p, c->hb, B.Xt, B.BX, nullptr, 1));
        std::vector<double> bn;
        CHK(coldot<double>(c, B.Xt, B.BX, bn));
        for (int i = 0; i < p; ++i)
            if (!(bn[i] > 0.0)) return fail(c, OFKS_EZERONORM, "set_x0: column %d has zero B-norm", i);
    }
    if (c->prec == OFKS_F32) {
        if (!c->hb32) CHK(ensure_f32_matrices(c));
        else CHK(ensure_f32_matrices(c));
        // free the FP64 products before the FP32 blocks exist (peak: X0, X and the FP32 blocks)
        CHK(sync(c));
        dfree(c, B.HX);
        dfree(c, B.BX);
        CHK(alloc_blocks<float>(c));
        HIPCHK(launch_convert<double, float>(c->stream, c->n * (int64_t)p, B.Xt, c->b32.Xt));
        CHK(sync(c));
        free_blocks<double>(c);
    }
    // a run from a start block depends on nothing an earlier run left: the
    // Hartree solve's warm start goes back to zero
    if (c->U) HIPCHK(hipMemsetAsync(c->U, 0, (size_t)c->n * sizeof(double), c->stream));
    c->dinv_h.assign(p, 1.0);
    c->k = 0;
    c->kkt0 = -1.0;
    c->eta = 0.0;
    c->eta0 = 0.0;
    c->have_prev = false;
    c->done = false;
    c->has_x = true;
    c->ehist.clear();
    c->lp_hold = 0;
    c->last_kind = -1;
    c->f32_best = INFINITY;
    c->f32_best_k = 0;
    c->relmin.clear();
    return sync(c);
}

int ofks_step(ofks_ctx *c, int32_t max_steps, ofks_iter_stats *stats, int32_t *n_stats, int32_t *done) {
    CHK(check_ready(c));
    WsScope wss(c);
    CHK(complete_blocks(c));
    int ns = 0;
    int rc = OFKS_OK;
    for (int s = 0; s < max_steps && !c->done; ++s) {
        bool stop = false;
        ofks_iter_stats st{};
        if (c->prec == OFKS_F64) rc = iterate<double>(c, &st, &stop);
        else rc = iterate<float>(c, &st, &stop);
        if (rc < 0) {
            // report what the failing iteration evaluated before the error
            if (stats && st.k == c->k && std::isfinite(st.kkt + st.fea)) stats[ns++] = st;
            break;
        }
        if (stats) stats[ns] = st;
        ++ns;
        if (stop) {
            c->done = true;
            break;
        }
        if (c->prec == OFKS_F32 && c->prm.refine_tol > 0.0) {
            // switch to FP64 below refine_tol, or when the FP32 phase has not
            // lowered its best residual for 50 iterations (its rounding floor),
            // or has not halved it over the last 100 (a crawl near the floor)
            if (st.rel < c->f32_best) {
                c->f32_best = st.rel;
                c->f32_best_k = st.k;
            }
            const int64_t nr = (int64_t)c->relmin.size();
            const bool crawl = nr > 100 && c->relmin[nr - 1] > 0.5 * c->relmin[nr - 101];
            if (st.rel < c->prm.refine_tol || st.k - c->f32_best_k > 50 || crawl) {
                rc = promote_to_f64(c);
                if (rc < 0) break;
            }
        }
    }
    if (n_stats) *n_stats = ns;
    if (done) *done = c->done ? 1 : 0;
    if (rc < 0) return rc;
    if (c->done && !(c->last_rel < c->prm.tol)) return OFKS_NOT_CONVERGED;
    return OFKS_OK;
}

int ofks_residual(ofks_ctx *c, double *kkt, double *fea, double *rel) {
    CHK(check_ready(c));
    if (std::isnan(c->last_rel)) {
        return fail(c, OFKS_ESTATE, "residual: no iteration evaluated yet (call ofks_step)");
    }
    if (kkt) *kkt = c->last_kkt;
    if (fea) *fea = c->last_fea;
    if (rel) *rel = c->last_rel;
    return OFKS_OK;
}

int ofks_energy(ofks_ctx *c, double *parts) {
    CHK(check_ready(c));
    if (!parts) return fail(c, OFKS_EINVAL, "energy: null output");
    for (int i = 0; i < 8; ++i) parts[i] = NAN;
    if (c->S.empty()) return fail(c, OFKS_ESTATE, "energy: no iteration evaluated yet");
    const int p = c->p;
    double trl = 0.0;
    for (int i = 0; i < p; ++i) trl += c->L0[i * p + i];
    if (c->prm.scf) {
        const double f = c->prm.occupation;
        const double har = c->scf_parts[3], xc = c->scf_parts[1], vrho = c->scf_parts[2];
        // f tr(X^T H X) = one-electron + int (V_H + v_xc) rho, int V_H rho = 2 E_H
        parts[0] = f * trl - 2.0 * har - vrho;
        parts[1] = har;
        parts[2] = xc;
        parts[3] = c->Enuc;
        parts[4] = parts[0] + har + xc + c->Enuc;
        parts[5] = c->scf_parts[0];
        parts[6] = f * trl;
        parts[7] = vrho;
    } else {
        double tr;
        if (!dense::trace_sinv_a(c->S, c->L0, p, tr)) return fail(c, OFKS_ENOTSPD, "energy: S not SPD");
        parts[4] = tr;
        parts[6] = trl;
    }
    return OFKS_OK;
}

int ofks_iterate_info(ofks_ctx *c, int32_t *p, int32_t *precision, int32_t *k) {
    CHK(check_ready(c));
    if (p) *p = c->p;
    if (precision) *precision = c->prec;
    if (k) *k = (int32_t)c->k;
    return OFKS_OK;
}

int ofks_get_x(ofks_ctx *c, double *dev_X) {
    CHK(check_ready(c));
    if (!dev_X) return fail(c, OFKS_EINVAL, "get_x: null output");
    if (c->prec == OFKS_F64) {
        CHK(upload<double>(c, c->b64.dinv, c->dinv_h));
        HIPCHK(launch_scale_copy<double, double>(c->stream, c->n, c->p, c->b64.Xt, c->b64.dinv, dev_X));
    } else {
        CHK(upload<float>(c, c->b32.dinv, c->dinv_h));
        HIPCHK(launch_scale_copy<float, double>(c->stream, c->n, c->p, c->b32.Xt, c->b32.dinv, dev_X));
    }
    return sync(c);
}

int ofks_postprocess(ofks_ctx *c, double *eigs) {
    CHK(check_ready(c));
    if (c->prec != OFKS_F64) {
        WsScope wss(c);
        CHK(promote_to_f64(c));
    }
    CHK(complete_blocks(c));
    Blocks<double> &B = c->b64;
    const int p = c->p;
    // normalized current iterate into Xt
    CHK(upload<double>(c, B.dinv, c->dinv_h));
    HIPCHK(launch_scale_copy<double, double>(c->stream, c->n, p, B.Xt, B.dinv, B.R));
    std::swap(B.Xt, B.R);
    std::vector<double> ones(p, 1.0);
    c->dinv_h = ones;
    CHK(upload<double>(c, B.dinv, ones));
    if (c->prm.scf) CHK(build_h<double>(c, B.Xt, B.dinv));
    CHK(spmm_pair<double>(c, p, c->hb, B.Xt, B.HX, B.BX, 0));
    std::vector<double> St, Lt;
    CHK(gram<double>(c, B.Xt, B.BX, B.HX, St, Lt));
    std::vector<double> S(p * p), L0(p * p);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            S[a * p + b] = 0.5 * (St[a * p + b] + St[b * p + a]);
            L0[a * p + b] = 0.5 * (Lt[a * p + b] + Lt[b * p + a]);
        }
    std::vector<double> w, Y;
    if (!dense::sym_gen_eig(L0, S, p, w, Y)) return fail(c, OFKS_ENOTSPD, "postprocess: X^T B X not SPD");
    CHK(upload<double>(c, B.CC, Y));
    GradArgs ga{};
    HIPCHK(launch_rowgemm<double>(c->stream, EPI_PLAIN, c->n, p, p, c->gemm_rows, B.Xt, B.dinv, B.CC, B.R, ga,
                                  nullptr));
    std::swap(B.Xt, B.R);
    // the rotated block starts a fresh BB history
    c->have_prev = false;
    c->eta = 0.0;
    if (eigs)
        for (int i = 0; i < p; ++i) eigs[i] = w[i];
    return sync(c);
}

int ofks_get_density(ofks_ctx *c, double *dev_rho) {
    CHK(check_ready(c));
    if (!c->assembled) return fail(c, OFKS_ESTATE, "get_density: needs an assembled mesh");
    if (!dev_rho) return fail(c, OFKS_EINVAL, "get_density: null output");
    if (!c->rho_q) return fail(c, OFKS_ESTATE, "get_density: no density evaluated yet (SCF steps or ofks_update_density)");
    HIPCHK(hipMemcpyAsync(dev_rho, c->rho_q, 4 * c->n_tets * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return sync(c);
}

// ---- single kernels ----------------------------------------------------------

int ofks_spmm(ofks_ctx *c, int32_t p, const double *X, double *HX, double *BX) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "spmm: no system");
    if (p <= 0 || p > 1024 || !X || !HX || !BX) return fail(c, OFKS_EINVAL, "spmm: bad arguments");
    CHK(spmm_pair<double>(c, p, c->hb, X, HX, BX, 0));
    return sync(c);
}


int ofks_spmm_ex(ofks_ctx *c, int32_t p, int32_t precision, int32_t op, const double *lam, const void *X, void *Y1,
                 void *Y2) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "spmm_ex: no system");
    if (p <= 0 || p > 1024 || !X || !Y1) return fail(c, OFKS_EINVAL, "spmm_ex: bad arguments");
    if (op != 0 && op != 1) return fail(c, OFKS_EINVAL, "spmm_ex: op must be 0 (dual) or 1 (shifted)");
    if (op == 0 && !Y2) return fail(c, OFKS_EINVAL, "spmm_ex: the dual product needs Y2");
    if (op == 1 && (!lam || !c->has_lhalf)) return fail(c, OFKS_ESTATE, "spmm_ex: the shifted product needs L/2 and lam");
    if (precision != OFKS_F64 && precision != OFKS_F32) return fail(c, OFKS_EINVAL, "spmm_ex: bad precision");
    if (op == 1) CHK(ensure_part(c, std::max((size_t)c->shift_grid * p,
                                             c->halo_nb ? spmm_halo_part_doubles(c->halo_nb, p) : (size_t)0)));
    if (precision == OFKS_F64) {
        CHK(spmm_ex_typed<double>(c, p, op, lam, (const double *)X, (double *)Y1, (double *)Y2));
    } else {
        if (!c->hb32) CHK(ensure_f32_matrices(c));
        CHK(spmm_ex_typed<float>(c, p, op, lam, (const float *)X, (float *)Y1, (float *)Y2));
    }
    return sync(c);
}

int ofks_gram(ofks_ctx *c, int32_t p, const double *X, const double *HX, const double *BX, double *S, double *L0) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "gram: no system");
    if (p <= 0 || p > 1024 || !X || !HX || !BX || !S || !L0) return fail(c, OFKS_EINVAL, "gram: bad arguments");
    const int keep = c->p;
    c->p = p;
    std::vector<double> St, Lt;
    int rc = gram<double>(c, X, BX, HX, St, Lt);
    c->p = keep;
    CHK(rc);
    std::memcpy(S, St.data(), sizeof(double) * p * p);
    std::memcpy(L0, Lt.data(), sizeof(double) * p * p);
    return OFKS_OK;
}

int ofks_gram_noalloc(ofks_ctx *c, int32_t p, const double *X, const double *HX, const double *BX, double *S,
                      double *L0) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "gram_noalloc: no system");
    if (!X || !HX || !BX || !S || !L0) return fail(c, OFKS_EINVAL, "gram_noalloc: null pointer");
    if (p <= 0 || p > OFKS_GRAM_NOALLOC_MAX_P)
        return fail(c, OFKS_ECAPACITY, "gram_noalloc: p = %d outside 1..%d (the fixed scratch of %zu bytes)", p,
                    OFKS_GRAM_NOALLOC_MAX_P, NOALLOC_SCRATCH_DOUBLES * sizeof(double));
    if (!c->scratch_dev) return fail(c, OFKS_ESTATE, "gram_noalloc: no scratch address for this device");
    // the split-K plan of ofks_gram, with fewer row splits where its partial
    // tiles would not fit beside their column sum
    const size_t pp2 = (size_t)p * 2 * p;
    const int64_t max_splits = (int64_t)(NOALLOC_SCRATCH_DOUBLES / pp2) - 1;
    GramPlan plan = gram_plan(c->n, p, 2048);
    if (plan.splits > max_splits) plan = gram_plan(c->n, p, (int)(max_splits * plan.gx * plan.gy));
    if (plan.splits < 1 || plan.splits > max_splits)
        return fail(c, OFKS_EINTERNAL, "gram_noalloc: no split plan fits the scratch");
    double *part = c->scratch_dev;
    double *red = c->scratch_dev + (size_t)plan.splits * pp2;
    HIPCHK(launch_gram<double>(c->stream, c->n, p, plan, X, BX, HX, part, (size_t)plan.splits * pp2));
    HIPCHK(launch_colsum(c->stream, plan.splits, (int64_t)pp2, part, red));
    // rows of the sums hold [S row | L0 row]; split them straight into the caller's arrays
    const size_t rowb = (size_t)p * sizeof(double);
    HIPCHK(hipMemcpy2DAsync(S, rowb, red, 2 * rowb, rowb, p, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpy2DAsync(L0, rowb, red + p, 2 * rowb, rowb, p, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return OFKS_OK;
}

int ofks_precondition(ofks_ctx *c, int32_t p, const double *lam, const double *G, double *P) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "precondition: needs L/2 and B");
    if (p <= 0 || p > 1024 || !lam || !G || !P) return fail(c, OFKS_EINVAL, "precondition: bad arguments");
    const int m = c->prm.pcg_iters;
    if (m < 1) return fail(c, OFKS_EINVAL, "precondition: pcg_iters must be >= 1");
    const int64_t n = c->n;
    const size_t np = (size_t)n * p;
    double *R = nullptr, *D = nullptr, *Q = nullptr, *lamd = nullptr, *alpha = nullptr, *betad = nullptr,
           *rzd = nullptr;
    uint8_t *act = nullptr;
    CHK(dalloc(c, &R, np));
    CHK(dalloc(c, &D, np));
    CHK(dalloc(c, &Q, np));
    CHK(dalloc(c, &lamd, p));
    CHK(dalloc(c, &alpha, p));
    CHK(dalloc(c, &betad, p));
    CHK(dalloc(c, &rzd, p));
    CHK(dalloc(c, &act, p));
    std::vector<double> lv(lam, lam + p);
    std::vector<uint8_t> ah(p);
    for (int i = 0; i < p; ++i) ah[i] = lam[i] < 0.0 ? 1 : 0;
    CHK(upload<double>(c, lamd, lv));
    CHK(upload_bytes(c, act, ah.data(), p));
    CHK(ensure_part(c, (size_t)c->grid * p));
    HIPCHK(launch_pcg_init<double>(c->stream, c->grid, n, p, act, c->lhd, c->bd, lamd, G, R, D, P, c->part));
    HIPCHK(launch_colsum(c->stream, c->grid, p, c->part, rzd));
    CHK(pcg_run<double>(c, m, n, p, act, lamd, c->lb, D, Q, P, R, alpha, betad, rzd));
    CHK(sync(c));
    dfree(c, R);
    dfree(c, D);
    dfree(c, Q);
    dfree(c, lamd);
    dfree(c, alpha);
    dfree(c, betad);
    dfree(c, rzd);
    dfree(c, act);
    return OFKS_OK;
}

int ofks_build_hamiltonian(ofks_ctx *c, int32_t p, const double *X, double *rho_q, double *eps_q, double *vxc_q,
                           double *U, double *parts) {
    if (!c) return OFKS_EINVAL;
    if (!c->assembled) return fail(c, OFKS_ESTATE, "build_hamiltonian: needs an assembled mesh");
    if (p <= 0 || p > 1024 || !X) return fail(c, OFKS_EINVAL, "build_hamiltonian: bad arguments");
    if (!c->has_params) ofks_default_params(&c->prm);
    double *ones = nullptr;
    CHK(dalloc(c, &ones, p));
    std::vector<double> o(p, 1.0);
    CHK(upload<double>(c, ones, o));
    const int keep = c->p;
    c->p = p;
    int rc = build_h<double>(c, X, ones);
    c->p = keep;
    dfree(c, ones);
    CHK(rc);
    hipStream_t s = c->stream;
    const size_t bq = 4 * c->n_tets * sizeof(double);
    if (rho_q) HIPCHK(hipMemcpyAsync(rho_q, c->rho_q, bq, hipMemcpyDeviceToDevice, s));
    if (eps_q) HIPCHK(hipMemcpyAsync(eps_q, c->eps_q, bq, hipMemcpyDeviceToDevice, s));
    if (vxc_q) HIPCHK(hipMemcpyAsync(vxc_q, c->vxc_q, bq, hipMemcpyDeviceToDevice, s));
    if (U) HIPCHK(hipMemcpyAsync(U, c->U, c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (parts)
        for (int i = 0; i < 4; ++i) parts[i] = c->scf_parts[i];
    return sync(c);
}

// ---- learned preconditioner ------------------------------------------------

int ofks_lp_set_weights(ofks_ctx *c, const float *w, const float *norm) {
    if (!c) return OFKS_EINVAL;
    if (!w || !norm) return fail(c, OFKS_EINVAL, "lp_set_weights: null pointer");
    for (int i = 0; i < 4; ++i)
        if (!(norm[4 + i] > 0.0f)) return fail(c, OFKS_EINVAL, "lp_set_weights: feature scales must be > 0");
    if (!c->lp_W) {
        CHK(dalloc(c, &c->lp_W, LP_NPAR));
        CHK(dalloc(c, &c->lp_norm, 8));
    }
    HIPCHK(hipMemcpyAsync(c->lp_W, w, LP_NPAR * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->lp_norm, norm, 8 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->lp_ready = true;
    return OFKS_OK;
}

int ofks_lp_collect(ofks_ctx *c, int64_t row_stride, int32_t objective, float *dev_buf, int64_t cap) {
    if (!c) return OFKS_EINVAL;
    if (dev_buf && (cap <= 0 || row_stride <= 0)) return fail(c, OFKS_EINVAL, "lp_collect: bad capacity or stride");
    if (objective != 0 && objective != 1) return fail(c, OFKS_EINVAL, "lp_collect: objective must be 0 or 1");
    c->lp_objective = objective;
    c->lp_buf = dev_buf;
    c->lp_cap = dev_buf ? cap : 0;
    c->lp_stride = row_stride;
    if (dev_buf) c->lp_count = 0;   // stopping keeps the count readable
    return OFKS_OK;
}

int ofks_lp_collected(ofks_ctx *c, int64_t *count) {
    if (!c || !count) return OFKS_EINVAL;
    *count = c->lp_count;
    return OFKS_OK;
}

namespace {
// sums of per-block partials of the loss and its gradient for the current weights
int lp_loss_grad_dev(ofks_ctx *c, const float *S, int64_t m, int grid) {
    HIPCHK(launch_lp_grad(c->stream, grid, m, S, c->lp_W, c->lp_norm, c->part));
    HIPCHK(launch_colsum(c->stream, grid, LP_NPAR + 1, c->part, c->red));
    return OFKS_OK;
}
}  // namespace

int ofks_lp_loss_grad(ofks_ctx *c, const float *dev_samples, int64_t m, const float *w, const float *norm,
                      double *loss, double *grad) {
    if (!c) return OFKS_EINVAL;
    if (!dev_samples || m <= 0 || !w || !norm || !loss || !grad) return fail(c, OFKS_EINVAL, "lp_loss_grad: bad arguments");
    CHK(ofks_lp_set_weights(c, w, norm));
    if (!c->red) CHK(dalloc(c, &c->red, 2 * 1024 * 1024 + 64));
    const int grid = 512;
    CHK(ensure_part(c, (size_t)grid * (LP_NPAR + 1)));
    CHK(lp_loss_grad_dev(c, dev_samples, m, grid));
    std::vector<double> out;
    CHK(download(c, out, c->red, LP_NPAR + 1));
    for (int k = 0; k < LP_NPAR; ++k) grad[k] = out[k];
    *loss = out[LP_NPAR];
    return OFKS_OK;
}

int ofks_lp_train(ofks_ctx *c, const float *dev_samples, int64_t m, int32_t epochs, float lr, float *w_inout,
                  float *norm_out, double *loss_out) {
    if (!c) return OFKS_EINVAL;
    if (!dev_samples || m <= 0 || epochs < 0 || !(lr > 0.0f) || !w_inout || !norm_out)
        return fail(c, OFKS_EINVAL, "lp_train: bad arguments");
    if (!c->red) CHK(dalloc(c, &c->red, 2 * 1024 * 1024 + 64));
    const int grid = 512;
    CHK(ensure_part(c, (size_t)grid * (LP_NPAR + 1)));
    // feature standardization from the samples
    HIPCHK(launch_lp_stats(c->stream, grid, m, dev_samples, c->part));
    HIPCHK(launch_colsum(c->stream, grid, 8, c->part, c->red));
    std::vector<double> st;
    CHK(download(c, st, c->red, 8));
    float norm[8];
    for (int j = 0; j < 4; ++j) {
        const double mu = st[j] / (double)m;
        const double var = std::max(0.0, st[4 + j] / (double)m - mu * mu);
        norm[j] = (float)mu;
        norm[4 + j] = (float)std::max(1e-6, std::sqrt(var));
    }
    CHK(ofks_lp_set_weights(c, w_inout, norm));
    float *m1 = nullptr, *m2 = nullptr;
    double *losses = nullptr;
    CHK(dalloc(c, &m1, LP_NPAR));
    CHK(dalloc(c, &m2, LP_NPAR));
    CHK(dalloc(c, &losses, std::max(epochs, 1)));
    HIPCHK(hipMemsetAsync(m1, 0, LP_NPAR * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(m2, 0, LP_NPAR * sizeof(float), c->stream));
    for (int t = 1; t <= epochs; ++t) {
        {
            Scope sc(c, "mlp_train");
            CHK(lp_loss_grad_dev(c, dev_samples, m, grid));
            HIPCHK(launch_lp_adam(c->stream, c->red, 1.0 / (double)m, c->lp_W, m1, m2, lr, 0.9f, 0.999f, 1e-8f, t));
        }
        HIPCHK(hipMemcpyAsync(losses + (t - 1), c->red + LP_NPAR, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(hipMemcpyAsync(w_inout, c->lp_W, LP_NPAR * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (loss_out && epochs > 0)
        HIPCHK(hipMemcpyAsync(loss_out, losses, epochs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CHK(sync(c));
    for (int j = 0; j < 8; ++j) norm_out[j] = norm[j];
    if (loss_out)
        for (int t = 0; t < epochs; ++t) loss_out[t] /= (double)m;
    dfree(c, m1);
    dfree(c, m2);
    dfree(c, losses);
    return OFKS_OK;
}

int ofks_lp_apply(ofks_ctx *c, int32_t p, const double *lam, const double *G, double *P) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "lp_apply: needs an assembled system");
    if (!c->lp_ready) return fail(c, OFKS_ESTATE, "lp_apply: no weights");
    if (p <= 0 || p > 1024 || !lam || !G || !P) return fail(c, OFKS_EINVAL, "lp_apply: bad arguments");
    const int keep = c->p;
    c->p = p;
    double *lamd = nullptr, *g2 = nullptr;
    uint8_t *neg = nullptr;
    CHK(dalloc(c, &lamd, p));
    CHK(dalloc(c, &g2, p));
    CHK(dalloc(c, &neg, p));
    std::vector<double> lv(lam, lam + p);
    std::vector<uint8_t> nh(p);
    for (int i = 0; i < p; ++i) nh[i] = lam[i] < 0.0 ? 1 : 0;
    CHK(upload<double>(c, lamd, lv));
    CHK(upload_bytes(c, neg, nh.data(), p));
    std::vector<double> gg;
    int rc = coldot<double>(c, G, G, gg);
    if (rc >= 0) rc = upload<double>(c, g2, gg);
    c->p = keep;
    CHK(rc);
    HIPCHK(hipMemcpyAsync(P, G, (size_t)c->n * p * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(launch_lp_apply<double>(c->stream, c->n, p, P, c->lhd, c->bd, c->hd, lamd, neg, g2, c->lp_W, c->lp_norm));
    CHK(sync(c));
    dfree(c, lamd);
    dfree(c, g2);
    dfree(c, neg);
    return OFKS_OK;
}

// ---- graph learned preconditioner ---------------------------------------------

namespace {
// column sums of G^2 into dev g2 (p doubles) for a caller's block of width p
int col_sq(ofks_ctx *c, int p, const double *G, double *g2) {
    CHK(ensure_part(c, (size_t)c->grid * p));
    HIPCHK(launch_coldot<double>(c->stream, c->grid, c->n, p, G, G, c->part));
    HIPCHK(launch_colsum(c->stream, c->grid, p, c->part, g2));
    return OFKS_OK;
}

// device shifts and identity-branch flags for host shifts lam[p]
int gl_shifts(ofks_ctx *c, int p, const double *lam, double **lamd, uint8_t **neg) {
    CHK(dalloc(c, lamd, p));
    CHK(dalloc(c, neg, p));
    std::vector<double> lv(lam, lam + p);
    std::vector<uint8_t> nh(p);
    for (int i = 0; i < p; ++i) nh[i] = lam[i] < 0.0 ? 1 : 0;
    CHK(upload<double>(c, *lamd, lv));
    CHK(upload_bytes(c, *neg, nh.data(), p));
    return OFKS_OK;
}

// training blocks: Z, QTP, PT, R, dR (FP64) and ft (FP32), each n x p
int gl_work(ofks_ctx *c, size_t np, double **Z, double **QTP, double **PT, double **Rb, double **dRb, float **FT) {
    if (c->gl_work_np < np) {
        if (c->gl_work) CHK(sync(c));
        dfree(c, c->gl_work);
        CHK(dalloc(c, &c->gl_work, 5 * np + (np + 1) / 2));
        c->gl_work_np = np;
    }
    *Z = c->gl_work;
    *QTP = c->gl_work + np;
    *PT = c->gl_work + 2 * np;
    *Rb = c->gl_work + 3 * np;
    *dRb = c->gl_work + 4 * np;
    *FT = (float *)(c->gl_work + 5 * np);
    return OFKS_OK;
}

constexpr int GL_GRID = 256;      // row chunks of the per-column training kernels
constexpr int GL_BWD_GRID = 512;  // blocks of the parameter-gradient kernel

// Loss and parameter gradient of the graph form's quadratic model for one
// block G (FP64, n x p) with device shifts lamd / flags neg, at the
// context's weights.  On return c->red[0..GL_NPAR) holds the gradient sums;
// *loss the loss.  One host sync for the column weights, one for the loss.
int gl_loss_grad_dev(ofks_ctx *c, int p, const double *G, const double *lamd, const uint8_t *neg, double *loss,
                     double *g2w) {
    const int64_t n = c->n;
    const size_t np = (size_t)n * p;
    double *Z, *QTP, *PT, *Rb, *dRb;
    float *FT;
    CHK(gl_work(c, np, &Z, &QTP, &PT, &Rb, &dRb, &FT));
    CHK(ensure_part(c, std::max({(size_t)GL_GRID * 2 * p, (size_t)GL_BWD_GRID * GL_NPAR_HOST,
                                 (size_t)c->shift_grid * p,
                                 c->halo_nb ? spmm_halo_part_doubles(c->halo_nb, p) : (size_t)0})));
    // column sums: g2 for the residual feature, w = 1 / <G, J G>
    HIPCHK(launch_gl_colsums(c->stream, GL_GRID, n, p, G, c->lhd, c->bd, lamd, neg, c->part));
    HIPCHK(launch_colsum(c->stream, GL_GRID, 2 * p, c->part, c->red));
    std::vector<double> cs;
    CHK(download(c, cs, c->red, 2 * p));
    std::vector<double> hw(2 * p);
    for (int l = 0; l < p; ++l) {
        hw[l] = cs[l];
        hw[p + l] = cs[p + l] > 0.0 ? 1.0 / cs[p + l] : 0.0;
    }
    CHK(upload<double>(c, g2w, hw));   // g2w[0..p) = g2, g2w[p..2p) = w
    const double *g2 = g2w, *w = g2w + p;
    int used = 0;
    // forward: Z, ft; Q = T Z; R = G - Q, P = Z + ft J R
    HIPCHK(launch_gl_heads<double>(c->stream, n, p, G, c->lhd, c->bd, c->hd, lamd, neg, g2, c->gl_W, c->gl_norm, Z,
                                   FT));
    CHK(spmm_shift<double>(c, p, c->lb, lamd, neg, Z, QTP, &used));
    HIPCHK(launch_gl_out<double>(c->stream, n, p, G, Z, FT, QTP, c->lhd, c->bd, lamd, neg, PT, Rb));
    // T P, then dP = w (T P - G) (in place) and dR = ft J dP; loss partials
    CHK(spmm_shift<double>(c, p, c->lb, lamd, neg, PT, QTP, &used));
    HIPCHK(launch_gl_bwd1(c->stream, GL_GRID, n, p, G, PT, QTP, FT, c->lhd, c->bd, lamd, neg, w, dRb, c->part));
    HIPCHK(launch_colsum(c->stream, GL_GRID, p, c->part, c->red));
    std::vector<double> lc;
    CHK(download(c, lc, c->red, p));
    double L = 0.0;
    for (int l = 0; l < p; ++l) L += hw[p + l] * lc[l];
    *loss = L;
    // T dR (into PT), then the parameter gradient
    CHK(spmm_shift<double>(c, p, c->lb, lamd, neg, dRb, PT, &used));
    HIPCHK(launch_gl_bwd2(c->stream, GL_BWD_GRID, n, p, G, QTP, Rb, Z, dRb, PT, c->lhd, c->bd, c->hd, lamd, neg, g2,
                          c->gl_W, c->gl_norm, c->part));
    HIPCHK(launch_colsum(c->stream, GL_BWD_GRID, GL_NPAR_HOST, c->part, c->red));
    return OFKS_OK;
}
}  // namespace

int ofks_gl_set_weights(ofks_ctx *c, const float *w, const float *norm) {
    if (!c) return OFKS_EINVAL;
    if (!w || !norm) return fail(c, OFKS_EINVAL, "gl_set_weights: null pointer");
    for (int i = 0; i < 4; ++i)
        if (!(norm[4 + i] > 0.0f)) return fail(c, OFKS_EINVAL, "gl_set_weights: feature scales must be > 0");
    if (!c->gl_W) {
        CHK(dalloc(c, &c->gl_W, GL_NPAR_HOST));
        CHK(dalloc(c, &c->gl_norm, 8));
    }
    HIPCHK(hipMemcpyAsync(c->gl_W, w, GL_NPAR_HOST * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->gl_norm, norm, 8 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->gl_ready = true;
    return OFKS_OK;
}

int ofks_gl_apply(ofks_ctx *c, int32_t p, const double *lam, const double *G, double *P) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "gl_apply: needs L/2 and B");
    if (!c->gl_ready) return fail(c, OFKS_ESTATE, "gl_apply: no weights");
    if (p <= 0 || p > 1024 || !lam || !G || !P) return fail(c, OFKS_EINVAL, "gl_apply: bad arguments");
    if (P == G) return fail(c, OFKS_EINVAL, "gl_apply: P must not alias G");
    const size_t np = (size_t)c->n * p;
    double *lamd = nullptr, *g2 = nullptr, *Z = nullptr, *Q = nullptr;
    uint8_t *neg = nullptr;
    float *FT = nullptr;
    CHK(gl_shifts(c, p, lam, &lamd, &neg));
    CHK(dalloc(c, &g2, p));
    CHK(dalloc(c, &Z, np));
    CHK(dalloc(c, &Q, np));
    CHK(dalloc(c, &FT, np));
    CHK(ensure_part(c, std::max({(size_t)c->grid * p, (size_t)c->shift_grid * p,
                                 c->halo_nb ? spmm_halo_part_doubles(c->halo_nb, p) : (size_t)0})));
    CHK(col_sq(c, p, G, g2));
    HIPCHK(launch_gl_heads<double>(c->stream, c->n, p, G, c->lhd, c->bd, c->hd, lamd, neg, g2, c->gl_W, c->gl_norm,
                                   Z, FT));
    int used = 0;
    CHK(spmm_shift<double>(c, p, c->lb, lamd, neg, Z, Q, &used));
    HIPCHK(launch_gl_out<double>(c->stream, c->n, p, G, Z, FT, Q, c->lhd, c->bd, lamd, neg, P, (double *)nullptr));
    CHK(sync(c));
    dfree(c, lamd);
    dfree(c, neg);
    dfree(c, g2);
    dfree(c, Z);
    dfree(c, Q);
    dfree(c, FT);
    return OFKS_OK;
}

int ofks_gl_loss_grad(ofks_ctx *c, int32_t p, const double *lam, const double *G, double *loss, double *grad) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "gl_loss_grad: needs L/2 and B");
    if (!c->gl_ready) return fail(c, OFKS_ESTATE, "gl_loss_grad: no weights");
    if (p <= 0 || p > 1024 || !lam || !G || !loss || !grad) return fail(c, OFKS_EINVAL, "gl_loss_grad: bad arguments");
    double *lamd = nullptr, *g2w = nullptr;
    uint8_t *neg = nullptr;
    CHK(gl_shifts(c, p, lam, &lamd, &neg));
    CHK(dalloc(c, &g2w, 2 * p));
    CHK(gl_loss_grad_dev(c, p, G, lamd, neg, loss, g2w));
    std::vector<double> gr;
    CHK(download(c, gr, c->red, GL_NPAR_HOST));
    for (int k = 0; k < GL_NPAR_HOST; ++k) grad[k] = gr[k];
    dfree(c, lamd);
    dfree(c, neg);
    dfree(c, g2w);
    return OFKS_OK;
}

int ofks_gl_capture(ofks_ctx *c, double *dev_buf, int32_t max_blocks, int64_t every) {
    if (!c) return OFKS_EINVAL;
    if (dev_buf && (max_blocks <= 0 || every <= 0)) return fail(c, OFKS_EINVAL, "gl_capture: bad capacity or stride");
    c->gl_cap = dev_buf;
    c->gl_cap_max = dev_buf ? max_blocks : 0;
    c->gl_cap_every = every > 0 ? every : 1;
    if (dev_buf) {
        c->gl_cap_count = 0;
        c->gl_cap_lam.clear();
    }
    return OFKS_OK;
}

int ofks_gl_captured(ofks_ctx *c, int32_t *count, double *host_lam) {
    if (!c || !count) return OFKS_EINVAL;
    *count = c->gl_cap_count;
    if (host_lam) std::memcpy(host_lam, c->gl_cap_lam.data(), c->gl_cap_lam.size() * sizeof(double));
    return OFKS_OK;
}

int ofks_gl_train(ofks_ctx *c, int32_t p, const double *dev_G, const double *host_lam, int32_t count,
                  int32_t epochs, float lr, float *w_inout, float *adam_inout, double *loss_out) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "gl_train: needs L/2 and B");
    if (!c->gl_ready) return fail(c, OFKS_ESTATE, "gl_train: set the weights and standardization first");
    if (p <= 0 || p > 1024 || !dev_G || !host_lam || count <= 0 || epochs < 0 || !(lr > 0.0f) || !w_inout ||
        !adam_inout)
        return fail(c, OFKS_EINVAL, "gl_train: bad arguments");
    const int np = GL_NPAR_HOST;
    HIPCHK(hipMemcpyAsync(c->gl_W, w_inout, np * sizeof(float), hipMemcpyHostToDevice, c->stream));
    float *m12 = nullptr;
    double *lamd = nullptr, *g2w = nullptr;
    uint8_t *neg = nullptr;
    CHK(dalloc(c, &m12, 2 * np));
    CHK(dalloc(c, &lamd, p));
    CHK(dalloc(c, &neg, p));
    CHK(dalloc(c, &g2w, 2 * p));
    HIPCHK(hipMemcpyAsync(m12, adam_inout, 2 * np * sizeof(float), hipMemcpyHostToDevice, c->stream));
    int t = (int)adam_inout[2 * np];
    const size_t nps = (size_t)c->n * p;
    for (int e = 0; e < epochs; ++e)
        for (int j = 0; j < count; ++j) {
            std::vector<double> lv(host_lam + (size_t)j * p, host_lam + (size_t)(j + 1) * p);
            std::vector<uint8_t> nh(p);
            for (int i = 0; i < p; ++i) nh[i] = lv[i] < 0.0 ? 1 : 0;
            CHK(upload<double>(c, lamd, lv));
            CHK(upload_bytes(c, neg, nh.data(), p));
            double L = 0.0;
            {
                Scope sc(c, "graph_train");
                CHK(gl_loss_grad_dev(c, p, dev_G + (size_t)j * nps, lamd, neg, &L, g2w));
                ++t;
                HIPCHK(launch_gl_adam(c->stream, np, c->red, 1.0, c->gl_W, m12, m12 + np, lr, 0.9f, 0.999f, 1e-8f,
                                      t));
            }
            if (loss_out) loss_out[(size_t)e * count + j] = L;
        }
    HIPCHK(hipMemcpyAsync(w_inout, c->gl_W, np * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(adam_inout, m12, 2 * np * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    CHK(sync(c));
    adam_inout[2 * np] = (float)t;
    dfree(c, m12);
    dfree(c, lamd);
    dfree(c, neg);
    dfree(c, g2w);
    return OFKS_OK;
}

int ofks_gl_feature_norm(ofks_ctx *c, float *norm_out) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "gl_feature_norm: needs an assembled system");
    if (!norm_out) return fail(c, OFKS_EINVAL, "gl_feature_norm: null output");
    const int grid = 256;
    CHK(ensure_part(c, (size_t)grid * 6));
    HIPCHK(launch_gl_node_stats(c->stream, grid, c->n, c->lhd, c->bd, c->hd, c->part));
    HIPCHK(launch_colsum(c->stream, grid, 6, c->part, c->red));
    std::vector<double> st;
    CHK(download(c, st, c->red, 6));
    for (int j = 0; j < 3; ++j) {
        const double mu = st[j] / (double)c->n;
        const double var = std::max(0.0, st[3 + j] / (double)c->n - mu * mu);
        norm_out[j] = (float)mu;
        norm_out[4 + j] = (float)std::max(1e-3, std::sqrt(var));   // a floor: uniform meshes give var = 0
    }
    norm_out[3] = 0.0f;   // g / rms(g) has mean ~0 and unit mean square by construction
    norm_out[7] = 1.0f;
    return OFKS_OK;
}

int ofks_lp_features(ofks_ctx *c, int32_t p, const double *G, float *dev_feat) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system || !c->has_lhalf) return fail(c, OFKS_ESTATE, "lp_features: needs an assembled system");
    if (p <= 0 || p > 1024 || !G || !dev_feat) return fail(c, OFKS_EINVAL, "lp_features: bad arguments");
    double *g2 = nullptr;
    CHK(dalloc(c, &g2, p));
    CHK(col_sq(c, p, G, g2));
    HIPCHK(launch_features(c->stream, c->n, p, G, c->lhd, c->bd, c->hd, g2, dev_feat));
    CHK(sync(c));
    dfree(c, g2);
    return OFKS_OK;
}

// ---- checkpoint / resume -------------------------------------------------------

extern "C++" {
namespace {
constexpr uint64_t STATE_MAGIC = 0x5441545346534b4fULL;   // "OKSFSTAT"
constexpr int32_t STATE_VERSION = 1;

struct StateHeader {
    uint64_t magic;
    int32_t version, prec, p, scf;
    int64_t n;
    int32_t k, have_prev, lp_hold, last_kind, f32_best_k, done, n_ehist, n_relmin, n_sl, pad;
    double kkt0, eta, eta0, f32_best, last_kkt, last_fea, last_rel, last_energy;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// bytes of the host part (header and vectors) and of one block
size_t state_host_bytes(ofks_ctx *c) {
    return align256(sizeof(StateHeader) +
                    8 * ((size_t)c->p + c->ehist.size() + c->relmin.size() + c->S.size() + c->L0.size()));
}
size_t state_block_bytes(ofks_ctx *c) {
    return (size_t)c->n * c->p * (c->prec == OFKS_F64 ? sizeof(double) : sizeof(float));
}

template <typename T> int state_blocks(ofks_ctx *c, char *buf, size_t off, bool get) {
    Blocks<T> &B = blk<T>(c);
    const size_t bb = (size_t)c->n * c->p * sizeof(T);
    T *blocks[3] = {B.Xt, B.Xp, B.Pp};
    for (int i = 0; i < 3; ++i) {
        char *d = buf + off + i * align256(bb);
        if (get) HIPCHK(hipMemcpyAsync(d, blocks[i], bb, hipMemcpyDeviceToDevice, c->stream));
        else HIPCHK(hipMemcpyAsync(blocks[i], d, bb, hipMemcpyDeviceToDevice, c->stream));
    }
    return OFKS_OK;
}

// (re)allocates the iteration blocks for width p in precision prec (the
// allocation part of ofks_set_x0, without a start block)
int setup_blocks(ofks_ctx *c, int p, int prec) {
    WsScope wss(c);
    c->has_x = false;   // until the new state is complete
    free_blocks<double>(c);
    free_blocks<float>(c);
    dfree(c, c->active);
    dfree(c, c->rz);
    dfree(c, c->g2);
    dfree(c, c->tw);
    ws_restart(c);
    c->p = p;
    c->prec = prec;
    CHK(walloc(c, &c->active, p));
    CHK(walloc(c, &c->rz, p));
    CHK(walloc(c, &c->g2, p));
    CHK(walloc(c, &c->tw, p));
    CHK(ensure_part(c, partials_needed(c, p)));
    if (prec == OFKS_F64) {
        CHK(alloc_blocks<double>(c));
    } else {
        c->ws_f64_base = c->ws_off;
        c->ws_f64_cap = c->ws_base ? ws_f64_region(c, p) : 0;
        c->ws_off += c->ws_f64_cap;
        CHK(ensure_f32_matrices(c));
        CHK(alloc_blocks<float>(c));
    }
    return OFKS_OK;
}

// H(X) for the stored iterate: column B-norms of X~ (the deferred
// normalization), then density, xc, Hartree and re-assembly
template <typename T> int update_density_t(ofks_ctx *c) {
    Blocks<T> &B = blk<T>(c);
    const int p = c->p;
    std::vector<double> dn(p, 1.0);
    if (c->prm.algorithm != 1) {
        CHK(spmm_pair<T>(c, p, hbT<T>(c), B.Xt, B.BX, nullptr, 1));
        std::vector<double> d2;
        CHK(coldot<T>(c, B.Xt, B.BX, d2));
        for (int i = 0; i < p; ++i) {
            if (!(d2[i] > 0.0)) return fail(c, OFKS_EZERONORM, "update_density: column %d has zero B-norm", i);
            dn[i] = 1.0 / std::sqrt(d2[i]);
        }
    }
    CHK(upload<T>(c, B.dinv, dn));
    return build_h<T>(c, B.Xt, B.dinv);
}
}  // namespace
}  // extern "C++"

int ofks_state_size(ofks_ctx *c, size_t *bytes) {
    CHK(check_ready(c));
    if (!bytes) return fail(c, OFKS_EINVAL, "state_size: null output");
    *bytes = state_host_bytes(c) + 3 * align256(state_block_bytes(c)) + (c->prm.scf ? 8 * (size_t)c->n : 0);
    return OFKS_OK;
}

int ofks_state_get(ofks_ctx *c, void *dev_buf, size_t bytes) {
    CHK(check_ready(c));
    CHK(complete_blocks(c));
    size_t need = 0;
    CHK(ofks_state_size(c, &need));
    if (!dev_buf || bytes < need) return fail(c, OFKS_EINVAL, "state_get: need a device buffer of %zu bytes", need);
    StateHeader h{};
    h.magic = STATE_MAGIC;
    h.version = STATE_VERSION;
    h.prec = c->prec;
    h.p = c->p;
    h.scf = c->prm.scf ? 1 : 0;
    h.n = c->n;
    h.k = c->k;
    h.have_prev = c->have_prev ? 1 : 0;
    h.lp_hold = c->lp_hold;
    h.last_kind = c->last_kind;
    h.f32_best_k = c->f32_best_k;
    h.done = c->done ? 1 : 0;
    h.n_ehist = (int32_t)c->ehist.size();
    h.n_relmin = (int32_t)c->relmin.size();
    h.n_sl = (int32_t)c->S.size();
    h.kkt0 = c->kkt0;
    h.eta = c->eta;
    h.eta0 = c->eta0;
    h.f32_best = c->f32_best;
    h.last_kkt = c->last_kkt;
    h.last_fea = c->last_fea;
    h.last_rel = c->last_rel;
    h.last_energy = c->last_energy;
    const size_t hb = state_host_bytes(c);
    std::vector<char> host(hb, 0);
    std::memcpy(host.data(), &h, sizeof h);
    double *v = (double *)(host.data() + sizeof h);
    for (double x : c->dinv_h) *v++ = x;
    for (double x : c->ehist) *v++ = x;
    for (double x : c->relmin) *v++ = x;
    for (double x : c->S) *v++ = x;
    for (double x : c->L0) *v++ = x;
    char *buf = (char *)dev_buf;
    CHK(upload_bytes(c, buf, host.data(), hb));
    if (c->prec == OFKS_F64) CHK(state_blocks<double>(c, buf, hb, true));
    else CHK(state_blocks<float>(c, buf, hb, true));
    if (c->prm.scf)
        HIPCHK(hipMemcpyAsync(buf + hb + 3 * align256(state_block_bytes(c)), c->U, 8 * (size_t)c->n,
                              hipMemcpyDeviceToDevice, c->stream));
    return sync(c);
}

int ofks_state_set(ofks_ctx *c, const void *dev_buf, size_t bytes) {
    if (!c) return OFKS_EINVAL;
    if (!c->has_system) return fail(c, OFKS_ESTATE, "state_set: no system");
    if (!c->has_params) return fail(c, OFKS_ESTATE, "state_set: call ofks_set_params first");
    if (!dev_buf || bytes < sizeof(StateHeader)) return fail(c, OFKS_EINVAL, "state_set: buffer too small");
    StateHeader h{};
    HIPCHK(hipMemcpyAsync(&h, dev_buf, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (h.magic != STATE_MAGIC || h.version != STATE_VERSION)
        return fail(c, OFKS_EINVAL, "state_set: not a state written by ofks_state_get");
    if (h.n != c->n) return fail(c, OFKS_EINVAL, "state_set: state is for n = %lld, system has n = %lld",
                                 (long long)h.n, (long long)c->n);
    if (h.p <= 0 || h.p > 1024 || (h.prec != OFKS_F64 && h.prec != OFKS_F32) || h.n_ehist < 0 || h.n_relmin < 0 ||
        h.n_sl < 0 || h.n_sl > 1024 * 1024)
        return fail(c, OFKS_EINVAL, "state_set: corrupt header");
    if ((h.scf != 0) != (c->prm.scf != 0))
        return fail(c, OFKS_EINVAL, "state_set: the state's SCF mode differs from the parameters'");
    if (h.scf && !c->assembled) return fail(c, OFKS_ESTATE, "state_set: an SCF state needs an assembled mesh");
    const size_t hb = align256(sizeof h + 8 * ((size_t)h.p + h.n_ehist + h.n_relmin + 2 * (size_t)h.n_sl));
    const size_t bb = (size_t)h.n * h.p * (h.prec == OFKS_F64 ? sizeof(double) : sizeof(float));
    const size_t need = hb + 3 * align256(bb) + (h.scf ? 8 * (size_t)h.n : 0);
    if (bytes < need) return fail(c, OFKS_EINVAL, "state_set: buffer holds %zu bytes, the state %zu", bytes, need);
    std::vector<char> host(hb);
    HIPCHK(hipMemcpyAsync(host.data(), dev_buf, hb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(setup_blocks(c, h.p, h.prec));
    const double *v = (const double *)(host.data() + sizeof h);
    c->dinv_h.assign(v, v + h.p);
    v += h.p;
    c->ehist.assign(v, v + h.n_ehist);
    v += h.n_ehist;
    c->relmin.assign(v, v + h.n_relmin);
    v += h.n_relmin;
    c->S.assign(v, v + h.n_sl);
    v += h.n_sl;
    c->L0.assign(v, v + h.n_sl);
    char *buf = (char *)dev_buf;
    if (h.prec == OFKS_F64) CHK(state_blocks<double>(c, buf, hb, false));
    else CHK(state_blocks<float>(c, buf, hb, false));
    if (h.scf)
        HIPCHK(hipMemcpyAsync(c->U, buf + hb + 3 * align256(bb), 8 * (size_t)h.n, hipMemcpyDeviceToDevice,
                              c->stream));
    c->k = h.k;
    c->have_prev = h.have_prev != 0;
    c->lp_hold = h.lp_hold;
    c->last_kind = h.last_kind;
    c->f32_best_k = h.f32_best_k;
    c->done = h.done != 0;
    c->kkt0 = h.kkt0;
    c->eta = h.eta;
    c->eta0 = h.eta0;
    c->f32_best = h.f32_best;
    c->last_kkt = h.last_kkt;
    c->last_fea = h.last_fea;
    c->last_rel = h.last_rel;
    c->last_energy = h.last_energy;
    c->has_x = true;
    return sync(c);
}

int ofks_update_density(ofks_ctx *c) {
    CHK(check_ready(c));
    if (!c->assembled) return fail(c, OFKS_ESTATE, "update_density: needs an assembled mesh");
    if (c->prec == OFKS_F64) CHK(update_density_t<double>(c));
    else CHK(update_density_t<float>(c));
    return sync(c);
}

int ofks_timing(ofks_ctx *c, int32_t enable) {
    if (!c) return OFKS_EINVAL;
    CHK(sync(c));
    c->timing = enable != 0;
    c->timers.clear();
    return OFKS_OK;
}

int ofks_timer_get(ofks_ctx *c, const char *name, double *ms, int64_t *launches) {
    if (!c || !name) return OFKS_EINVAL;
    CHK(sync(c));
    auto it = c->timers.find(name);
    if (ms) *ms = it == c->timers.end() ? 0.0 : it->second.ms;
    if (launches) *launches = it == c->timers.end() ? 0 : it->second.launches;
    return OFKS_OK;
}

}  // extern "C"
