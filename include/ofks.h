/*
 * ofks -- orthogonalization-free Kohn-Sham block solver for MI355X (gfx950).
 *
 * C ABI of the library libofks.so.  It implements the parallelizable
 * column-wise augmented-Lagrangian iteration (PCAL, Section 3.3 of Gao, Hu,
 * Kuang & Liu, "An orthogonalization-free parallelizable framework for
 * all-electron calculations in density functional theory") on a P1
 * tetrahedral finite-element discretization (Section 2.2).
 *
 * Conventions (apply to every entry point):
 *  - Every call returns an int status: OFKS_OK (0), a positive warning, or a
 *    negative error.  After a non-OK return ofks_last_error() gives a message.
 *    No C++ exception crosses the ABI.
 *  - All device work is enqueued on the HIP stream given to ofks_create.  Calls
 *    that return host values synchronize that stream only.
 *  - "host" pointers are read or written during the call only; "device"
 *    pointers are caller-owned device memory that must stay valid during the
 *    call.  The library owns the device memory it allocates for its state:
 *    the system in the setup calls (mesh load, assemble, csr load), the
 *    iteration's state in set_x0 and, lazily, in the first steps (the rest
 *    of the FP64 blocks, the precision switch, SCF and graph-form arrays),
 *    all freed in ofks_destroy.  With a caller workspace (ofks_set_workspace)
 *    the iteration's state is carved from it instead.  Without one, the
 *    paper preconditioner also takes m - 1 scratch blocks for its inner
 *    directions when free device memory stays above a quarter of the device
 *    after the allocation (same results; skipped otherwise, never an
 *    error); they are released with the iterate.
 *  - Blocks X (n x p) are row-major: the p values of one DOF are contiguous.
 *    n counts interior (non-Dirichlet) nodes, numbered in node order.
 *  - CSR matrices: row_ptr int64[n+1], col int32[nnz], columns sorted
 *    ascending within a row, the diagonal present in every row.
 *  - Call order: create -> (mesh_load, nuclei_set, assemble | csr_load)
 *    -> set_params -> set_x0 -> step ...  Out-of-order calls return
 *    OFKS_ESTATE.  A context is not thread-safe.
 */
#ifndef OFKS_H
#define OFKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ofks_ctx ofks_ctx;

enum {
    OFKS_OK = 0,
    OFKS_NOT_CONVERGED = 1,   /* warning: max_iter reached */
    OFKS_EINVAL = -1,         /* bad argument */
    OFKS_ESTATE = -2,         /* call out of order */
    OFKS_EHIP = -3,           /* HIP runtime error */
    OFKS_ECAPACITY = -4,      /* a compiled-in bound (mesh, no-allocation scratch) or the caller's workspace is exceeded */
    OFKS_ENONFINITE = -5,     /* NaN/Inf in a p x p quantity */
    OFKS_ENOTSPD = -6,        /* Gram matrix not positive definite */
    OFKS_EZERONORM = -7,      /* a column with zero B-norm */
    OFKS_EINTERNAL = -8       /* a host-side consistency check of the library's own data failed */
};

/* Preconditioner choice (eq. precondition-T, the learned pointwise form and the learned graph form). */
enum { OFKS_PRECOND_NONE = 0, OFKS_PRECOND_PAPER = 1, OFKS_PRECOND_LEARNED = 2, OFKS_PRECOND_GRAPH = 3 };
/* Step-size rule, Section 4.4 (Barzilai-Borwein variants). */
enum { OFKS_STEP_BB2 = 0, OFKS_STEP_BB1 = 1, OFKS_STEP_ABB1 = 2, OFKS_STEP_ABB2 = 3,
       OFKS_STEP_FIXED = 4 };
/* Arithmetic of the n x p blocks.  p x p algebra is always FP64. */
enum { OFKS_F64 = 0, OFKS_F32 = 1 };

typedef struct {
    double beta;            /* penalty parameter of L_beta (Section 4.4; default 1) */
    double eta0;            /* > 0: first proximal parameter; 0: ||P0||_F/||X0||_F */
    double tol;             /* stop when (kkt + fea)/kkt_0 < tol (Section 4.1) */
    int32_t step_rule;      /* OFKS_STEP_* */
    int32_t precond;        /* OFKS_PRECOND_* */
    int32_t pcg_iters;      /* Jacobi-PCG iterations for T_i^{-1} G_i */
    int32_t precision;      /* OFKS_F64 or OFKS_F32 */
    int32_t precond_lambda; /* 0: diagonal of the eq. lambda2 multiplier, 1: of X^T H X */
    int32_t max_iter;       /* iteration cap (paper: 1000) */
    double occupation;      /* electrons per orbital f (2) */
    int32_t scf;            /* 1: rebuild H(X) every iteration (Kohn-Sham); 0: fixed H */
    int32_t energy_every;   /* evaluate the energy every k-th iteration (>= 1) */
    double refine_tol;      /* F32 only: switch to FP64 when rel < refine_tol, or when the FP32
                               iterates have not lowered rel for 50 iterations or not halved their
                               lowest rel over the last 100 (0: never switch) */
    double poisson_rtol;    /* Hartree CG relative residual */
    int32_t poisson_max_iter;
    int32_t fallback_window;/* learned form: W iterations of energy history (<= 0: no fallback) */
    int32_t fallback_hold;  /* learned form: iterations on the paper preconditioner after a fallback */
    int32_t fallback_rule;  /* learned form: a fallback when E^k exceeds 0: the minimum, 1: the maximum
                               of the previous fallback_window energies */
    int32_t use_graphs;     /* 1: replay launch-bound inner loops (Hartree CG) as HIP graphs; 0: launch eagerly */
    int32_t algorithm;      /* 0: PCAL (Algorithm PCAL: eq. lambda2 multiplier, column B-normalization);
                               1: PLAM (Algorithm PLAM: Lambda = X^T H X (eq. multi), no normalization) */
    int32_t spmm_mode;      /* sparse products: 0 auto (LDS-halo kernel for FP64 blocks with p >= 64 and
                               FP32 blocks with p >= 96; row-gather otherwise);
                               1 row-gather kernel; 2 LDS-halo kernel (products then fail with OFKS_ESTATE
                               if the matrix has a row with more than 64 entries or more distinct columns
                               than the halo holds).  The kernels agree to rounding. */
    int32_t fallback_stall; /* learned forms: also fall back when the fallback_stall iterates before the
                               current one did not halve the lowest rel (<= 0: never; default 30) */
    double poisson_adapt;   /* SCF: inside the iteration the Hartree CG stops at relative residual
                               max(poisson_rtol, poisson_adapt x rel of the previous iterate), the
                               first at max(poisson_rtol, poisson_adapt) (0, default: always poisson_rtol);
                               the single-call density paths keep poisson_rtol.  1e-3 is safe on the
                               meshes measured; 1e-2 can stall the last decade */
    int32_t graph_sweeps;   /* graph form: damped sweeps through T_l per application (1..64, default 1):
                               the first after the heads, each further one P <- P + ft J (G - T P) with
                               the same weights (one shifted SpMM each); training covers one sweep */
} ofks_params;

typedef struct {
    int32_t k;              /* iteration index of the iterate X^k these values describe */
    int32_t precond_used;   /* OFKS_PRECOND_* applied in the step that produced X^{k+1} */
    int32_t precision;      /* OFKS_F64 / OFKS_F32 of this iteration */
    int32_t fell_back;      /* 1 if the learned form fell back in this iteration */
    double energy;          /* SCF: E_KS; fixed H: tr(S^{-1} Lambda0) (NaN when skipped) */
    double kkt;             /* ||H X - B X Lambda0||_F */
    double fea;             /* ||X^T B X - I||_F */
    double rel;             /* (kkt + fea) / kkt_0 */
    double eta;             /* proximal parameter used for the step from X^k */
    double ms;              /* wall time of this iteration (ms, stream-synchronous) */
} ofks_iter_stats;

/* Fills *p with the defaults documented above. */
void ofks_default_params(ofks_params *p);

/* Creates a context bound to a HIP stream (hipStream_t passed as void*; NULL =
 * the null stream).  The current HIP device at this call is the context's device. */
int ofks_create(ofks_ctx **out, void *hip_stream);
int ofks_destroy(ofks_ctx *ctx);
const char *ofks_last_error(const ofks_ctx *ctx);

/* ---- discretization (Section 2.2) -------------------------------------- */

/* Tetrahedral mesh: xyz host f64[n_nodes*3]; tets host i32[n_tets*4] node
 * indices; dirichlet host u8[n_nodes] (1 = boundary node, value fixed to 0).
 * Copies to the device.  EINVAL on out-of-range node indices. */
int ofks_mesh_load(ofks_ctx *ctx, int64_t n_nodes, const double *xyz, int64_t n_tets,
                   const int32_t *tets, const uint8_t *dirichlet);

/* Nuclei for V_ext(r) = -sum_j Z_j/|r - R_j| (eq. ext): Z host f64[M], R host f64[M*3]. */
int ofks_nuclei_set(ofks_ctx *ctx, int32_t M, const double *Z, const double *R);

/* On the device: interior-DOF numbering, sorted CSR pattern, stiffness L,
 * mass B and M_ext by the 4-point degree-2 rule, and H = L/2 + M_ext
 * (eq. hamiltonian without the density terms).  ECAPACITY if a node touches
 * more than 128 tetrahedra or a row has more than 64 entries. */
int ofks_assemble(ofks_ctx *ctx);

/* Sizes of the assembled (or loaded) system. */
int ofks_csr_info(ofks_ctx *ctx, int64_t *n, int64_t *nnz);

/* Copies the pattern and values to host arrays (any pointer may be NULL):
 * row_ptr[n+1], col[nnz], L[nnz], B[nnz], H[nnz] (current H). */
int ofks_csr_get(ofks_ctx *ctx, int64_t *row_ptr, int32_t *col, double *L, double *B, double *H);

/* Fixed problem given directly as CSR (all device pointers): H and B values;
 * Lhalf (= L/2, for the preconditioner) may be NULL, then only
 * OFKS_PRECOND_NONE is accepted.  Replaces any assembled system. */
int ofks_csr_load(ofks_ctx *ctx, int64_t n, int64_t nnz, const int64_t *row_ptr,
                  const int32_t *col, const double *H, const double *B, const double *Lhalf);

/* ---- problem setup ------------------------------------------------------ */

int ofks_set_params(ofks_ctx *ctx, const ofks_params *params);

/* Caller-owned workspace for the iteration's device state: the blocks of
 * width p and their per-column arrays, the per-block partial sums, the graph
 * form's smoothing weights, an FP32 run's FP32 copies of H and L/2 and the
 * FP64 set its refinement switches to, and the SCF density's quadrature
 * arrays.  ofks_workspace_size gives the bytes that width p and the given
 * parameters need on the current system.  After ofks_set_workspace(dev_ws,
 * bytes) (device memory, 256-byte aligned, owned by the caller and valid
 * until the context is destroyed or another workspace is set),
 * ofks_set_x0, ofks_state_set and ofks_step take that state from it and call
 * no hipMalloc.  The assembled system (CSR, values, halo plan, mesh arrays)
 * stays library-owned; the single-kernel, training, data-collection and
 * post-processing calls may still allocate.  Setting a workspace releases
 * the current iterate (ofks_set_x0 or ofks_state_set must follow);
 * dev_ws = NULL returns to library allocation.  ECAPACITY when the state
 * outgrows the workspace (other parameters than those it was sized for). */
int ofks_workspace_size(ofks_ctx *ctx, int32_t p, const ofks_params *params, size_t *bytes);
int ofks_set_workspace(ofks_ctx *ctx, void *dev_ws, size_t bytes);

/* Starting block X0 (device f64[n*p]).  b_orthonormalize = 1 applies the
 * Cholesky-based Gram-Schmidt of Section 4.2 (X0 = V R^{-1}, R^T R = V^T B V);
 * 0 takes X0 as given.  Allocates the iteration blocks for this p (for an
 * FP64 run the three the orthonormalization uses; the other five come with
 * the first ofks_step, ofks_state_get or ofks_postprocess, so the caller may
 * free X0 in between: the eight FP64 blocks of n = 8e6, p = 512 take 262 GB
 * of the 288, X0 another 33).  Resets
 * the iteration counter, the fallback history and the Hartree solve's warm
 * start, so the run depends only on X0 and the parameters.  ENOTSPD if V^T B V is not positive definite;
 * EZERONORM if a column taken as given has zero B-norm. */
int ofks_set_x0(ofks_ctx *ctx, int32_t p, const double *dev_X0, int32_t b_orthonormalize);

/* ---- main iteration (Algorithm PCAL) -------------------------------------- */

/* Runs up to max_steps iterations.  stats (host, may be NULL) receives one
 * entry per iteration evaluated; *n_stats their count; *done = 1 once the
 * stopping rule holds or max_iter is reached.  Returns OFKS_OK, or
 * OFKS_NOT_CONVERGED when max_iter was reached, or an error. */
int ofks_step(ofks_ctx *ctx, int32_t max_steps, ofks_iter_stats *stats, int32_t *n_stats,
              int32_t *done);

/* kkt, fea and rel of the current iterate (evaluates them if needed). */
int ofks_residual(ofks_ctx *ctx, double *kkt, double *fea, double *rel);

/* Energy of the current iterate.  parts (host f64[8]): SCF: kinetic+external
 * one-electron sum f tr(X^T (L/2 + M_ext) X), Hartree, xc, nuclear, total,
 * electron count, f tr(Lambda0), int v_xc rho; fixed H: parts[4] = tr(S^{-1} Lambda0). */
int ofks_energy(ofks_ctx *ctx, double *parts);

/* Post-processing (Section 4.3): Rayleigh-Ritz on (Lambda0, S), X <- X Y.
 * eigs host f64[p] ascending. */
int ofks_postprocess(ofks_ctx *ctx, double *eigs);

/* Current normalized iterate X^k into dev_X (device f64[n*p]). */
/* The current iterate's block width p, the precision of its blocks
 * (OFKS_F64 / OFKS_F32) and its iteration index k (any pointer may be NULL).
 * ESTATE before ofks_set_x0 or ofks_state_set. */
int ofks_iterate_info(ofks_ctx *ctx, int32_t *p, int32_t *precision, int32_t *k);
int ofks_get_x(ofks_ctx *ctx, double *dev_X);

/* SCF: density rho at the 4 quadrature points of every tetrahedron of the
 * current iterate, dev_rho device f64[n_tets*4]. */
int ofks_get_density(ofks_ctx *ctx, double *dev_rho);

/* Density/potential update (Sections 2.1-2.2): for the current iterate X^k,
 * the density rho = f sum_l psi_l^2 at the quadrature points, the LDA
 * exchange-correlation, the Hartree potential (L U = 4 pi b, warm-started
 * CG) and H(X) = L/2 + M(V_ext + V_H + v_xc), re-assembled in place.  The SCF
 * iteration does this at the start of every step; this call lets a caller
 * refresh H between steps of a fixed-H run.  ESTATE without an assembled
 * mesh or before ofks_set_x0; EZERONORM for a zero column. */
int ofks_update_density(ofks_ctx *ctx);

/* ---- checkpoint / resume ---------------------------------------------------
 * The iteration state after any number of steps: the current, previous and
 * previous-preconditioned blocks (the BB pair), the deferred column
 * normalization, k, eta, eta_0, kkt_0, the fallback and precision-switch
 * state, and (SCF) the Hartree potential that warm-starts the next solve.
 * ofks_state_get writes it into a caller-owned device buffer of at least
 * ofks_state_size bytes (the size grows by 8 bytes per iteration);
 * ofks_state_set restores it on a context with the same system and
 * parameters (and, for the learned forms, the same weights), allocating the
 * blocks for its width and precision; the following steps are bit-identical
 * to those of the uninterrupted run.  EINVAL for a buffer too small, a state
 * of another size or SCF mode, or one not written by ofks_state_get. */
int ofks_state_size(ofks_ctx *ctx, size_t *bytes);
int ofks_state_get(ofks_ctx *ctx, void *dev_buf, size_t bytes);
int ofks_state_set(ofks_ctx *ctx, const void *dev_buf, size_t bytes);

/* ---- single kernels, for parity checks ----------------------------------- */

/* HX = H X and BX = B X (dual SpMM) on the current system; device f64 blocks n x p. */
int ofks_spmm(ofks_ctx *ctx, int32_t p, const double *X, double *HX, double *BX);

/* One sparse product in either block precision, through the kernel the
 * iteration would use (params.spmm_mode):
 *   op 0: Y1 = H X, Y2 = B X (the dual product of eq. PCAL-main's gradient);
 *   op 1: Y1_l = (L/2 - lam_l B) X_l for columns with lam_l < 0 and 0 for the
 *         others (the operator T_l of eq. precondition-T); Y2 unused (may be
 *         NULL); lam host f64[p].
 * precision OFKS_F64: X, Y1, Y2 device f64[n*p]; OFKS_F32: device f32[n*p],
 * with the FP32 copies of the matrix values (made on first use).  Blocks are
 * row-major and caller-owned; Y1 and Y2 must not overlap X.  EINVAL on bad
 * arguments; ESTATE without a system (op 1: without L/2). */
int ofks_spmm_ex(ofks_ctx *ctx, int32_t p, int32_t precision, int32_t op, const double *lam, const void *X,
                 void *Y1, void *Y2);

/* S = X^T BX and L0 = X^T HX (tall-skinny Gram), host f64[p*p] each, not symmetrized. */
int ofks_gram(ofks_ctx *ctx, int32_t p, const double *X, const double *HX, const double *BX,
              double *S, double *L0);

/* ofks_gram for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same S = X^T BX and L0 = X^T HX (host f64[p*p] each, not symmetrized,
 * equal to ofks_gram's up to the summation order), with the split-K partial
 * tiles and their sums in a fixed 64 MiB device array that the library holds
 * per device until the process ends.  It calls no hipMalloc, hipFree or
 * hipHostMalloc; with large p it uses fewer row splits than ofks_gram.
 * 1 <= p <= OFKS_GRAM_NOALLOC_MAX_P, else OFKS_ECAPACITY.  Every call on one
 * device shares that array: calls that overlap on one device (two contexts
 * on different streams, or two threads) race and must be serialized by the
 * caller.  Synchronizes the context's stream. */
#define OFKS_GRAM_NOALLOC_MAX_P 1024
int ofks_gram_noalloc(ofks_ctx *ctx, int32_t p, const double *X, const double *HX, const double *BX,
                      double *S, double *L0);

/* P = T^{-1} G columnwise by the fixed-iteration Jacobi-PCG of the paper
 * preconditioner; lam host f64[p]; columns with lam >= 0 are copied. */
int ofks_precondition(ofks_ctx *ctx, int32_t p, const double *lam, const double *G, double *P);

/* SCF pieces for the iterate X (device f64 n x p, used as given):
 * rho_q, eps_q, vxc_q device f64[n_tets*4] (any may be NULL), U device f64[n]
 * (Hartree potential, may be NULL), parts host f64[4] = {int rho, int eps rho,
 * int vxc rho, U.b/2} (may be NULL).  Also rebuilds H = H(X). */
int ofks_build_hamiltonian(ofks_ctx *ctx, int32_t p, const double *X, double *rho_q,
                           double *eps_q, double *vxc_q, double *U, double *parts);

/* ---- learned pointwise preconditioner (not in the paper) --------------------
 *
 * With params.precond = OFKS_PRECOND_LEARNED the step uses
 *   P_il = exp(f(x_il)) J_il G_il,  f = MLP 4 -> 32 (tanh) -> 1 (FP32),
 *   x_il = standardized [log(L_ii/2), log B_ii, (H_ii - L_ii/2)/B_ii, g_il/rms(g_l)],
 *   J_il = 1/(L_ii/2 - Lambda_ll B_ii) if Lambda_ll < 0, else 1
 * and falls back to the paper preconditioner (eq. precondition-T) for
 * fallback_hold iterations whenever the energy of an iterate exceeds the
 * minimum (fallback_rule 1: maximum) of the previous fallback_window
 * iterates, or the fallback_stall iterates before it did not halve the
 * lowest residual (a stall while the energy falls).  Weight vector (193
 * floats): [W1 (32 x 4 row-major), b1 (32), W2 (32), b2 (1)]; norm (8 floats):
 * feature means then standard deviations (all > 0). */
int ofks_lp_set_weights(ofks_ctx *ctx, const float *host_w, const float *host_norm);

/* Training-sample collection: while dev_buf != NULL, every iteration that
 * applies the paper preconditioner appends, for every row_stride-th row and
 * all columns, one sample of 8 floats [4 raw features, a, t, w, 0] of the
 * weighted least-squares fit of exp(f) a to t (dev_buf: device, capacity cap
 * samples).  objective 0 imitates T^-1 g in the Euclidean norm: a = J g,
 * t = T^-1 g (the paper preconditioner's output), w = 1/mean_i t_il^2.
 * objective 1 imitates it in the energy norm of T with the scale taken as
 * locally constant, i.e. minimizes the quadratic model d^T T d / 2 - g^T d
 * over d = s J g node by node: a = 1, t = g/u, w = max(J g u, 0) n/<g, T^-1 g>
 * with u = T J g (u = g on identity-branch columns).
 * A new dev_buf restarts the count at zero; dev_buf = NULL stops collection
 * and leaves the count of the last buffer readable through
 * ofks_lp_collected.  The buffer is caller-owned. */
int ofks_lp_collect(ofks_ctx *ctx, int64_t row_stride, int32_t objective, float *dev_buf, int64_t cap);
int ofks_lp_collected(ofks_ctx *ctx, int64_t *count);

/* Trains on m device samples: standardization from the samples (norm_out,
 * host f32[8]), then `epochs` full-batch Adam steps (lr, betas 0.9/0.999) on
 * sum_s w_s (exp(f_s) a_s - t_s)^2 / m from the initial weights in w_inout
 * (host f32[193], overwritten with the result).  loss_out (host f64[epochs] or
 * NULL) receives the loss before each step.  The trained weights are also set
 * on the context. */
int ofks_lp_train(ofks_ctx *ctx, const float *dev_samples, int64_t m, int32_t epochs, float lr,
                  float *w_inout, float *norm_out, double *loss_out);

/* Loss and gradient sums (host f64 scalar and f64[193]) of the training
 * objective over m device samples for the given weights (parity checks). */
int ofks_lp_loss_grad(ofks_ctx *ctx, const float *dev_samples, int64_t m, const float *host_w,
                      const float *host_norm, double *loss, double *grad);

/* P = exp(f) J G for a device block G (f64 n x p) with shifts lam (host
 * f64[p]), using the context's weights (parity checks). */
int ofks_lp_apply(ofks_ctx *ctx, int32_t p, const double *lam, const double *G, double *P);

/* Raw features [n, p, 4] (device f32, row-major) of the learned forms for a
 * device block G (f64 n x p): log(L_ii/2), log B_ii, (H_ii - L_ii/2)/B_ii,
 * g_il / rms(g_l) (0 where the column is zero). */
int ofks_lp_features(ofks_ctx *ctx, int32_t p, const double *G, float *dev_feat);

/* ---- learned graph preconditioner (not in the paper) -------------------------
 *
 * With params.precond = OFKS_PRECOND_GRAPH the step uses one damped Jacobi
 * sweep through the paper's operator T_l (eq. precondition-T) over the CSR
 * pattern, with a per-(row, column) scale and smoothing weight from a
 * pointwise network on the learned forms' features:
 *   (fs, ft) = W2 tanh(W1 x + b1) + b2,  Z = exp(fs) J G,
 *   P = Z + ft J (G - T Z)       (T = I and J = 1 on columns with Lambda_ll >= 0),
 * and falls back to the paper preconditioner like the pointwise form.
 * Weights (226 floats): [W1 (32 x 4 row-major), b1 (32), W2 (2 x 32 row-major,
 * row 0 for fs), b2 (2)]; norm (8 floats): feature means, then standard
 * deviations (> 0).  Network arithmetic is FP32. */
int ofks_gl_set_weights(ofks_ctx *ctx, const float *host_w, const float *host_norm);

/* P for a device block G (f64 n x p, P must not alias G) and host shifts
 * lam[p], with the context's weights (parity checks). */
int ofks_gl_apply(ofks_ctx *ctx, int32_t p, const double *lam, const double *G, double *P);

/* The training objective for one block and its gradient (host f64 scalar and
 * f64[226]) at the context's weights:
 *   loss = sum_l w_l (P_l^T T_l P_l / 2 - G_l^T P_l),  w_l = 1 / (G_l^T J_l G_l),
 * the quadratic model of each column's system, smallest where P_l = T_l^-1 G_l. */
int ofks_gl_loss_grad(ofks_ctx *ctx, int32_t p, const double *lam, const double *G, double *loss, double *grad);

/* Training snapshots: while dev_buf != NULL, every `every`-th FP64 iterate that
 * applies the paper preconditioner writes its gradient block G (n x p) into
 * the next slot of dev_buf (caller-owned, max_blocks * n * p doubles) and
 * keeps its shifts; a new buffer restarts the count, NULL stops capturing. */
int ofks_gl_capture(ofks_ctx *ctx, double *dev_buf, int32_t max_blocks, int64_t every);
/* Count of captured blocks and their shifts (host f64[count * p] or NULL). */
int ofks_gl_captured(ofks_ctx *ctx, int32_t *count, double *host_lam);

/* Adam on the training objective over `count` device blocks G (f64, count
 * x n x p, on the context's system) with host shifts lam (count x p), for
 * `epochs` passes, one step per block.  w_inout (host f32[226]) holds the
 * starting weights and receives the result (also set on the context);
 * adam_inout (host f32[453]: first moments, second moments, step count)
 * carries the optimizer state across calls and systems; loss_out (host
 * f64[epochs * count] or NULL) receives each block's loss before its step.
 * The standardization must have been set with ofks_gl_set_weights. */
int ofks_gl_train(ofks_ctx *ctx, int32_t p, const double *dev_G, const double *host_lam, int32_t count,
                  int32_t epochs, float lr, float *w_inout, float *adam_inout, double *loss_out);

/* Standardization of the node features over the current system's rows (host
 * f32[8]: means, then standard deviations; the residual feature gets 0 and 1). */
int ofks_gl_feature_norm(ofks_ctx *ctx, float *host_norm);

/* ---- timing ------------------------------------------------------------ */

/* Kernel timers (HIP events on the context stream).  enable = 1 starts
 * recording and clears the totals. */
int ofks_timing(ofks_ctx *ctx, int32_t enable);
/* Totals for a kernel class: name is one of "spmm_dual", "spmm_shift",
 * "gram", "update_a", "update_b", "pcg_r", "pcg_dx", "density", "poisson",
 * "assemble_h", "bbdot", "mlp", "mlp_train", "graph", "graph_train", and "host" (the host's
 * p x p algebra of each iteration, wall time).  ms = summed duration, launches = count. */
int ofks_timer_get(ofks_ctx *ctx, const char *name, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* OFKS_H */
