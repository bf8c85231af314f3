// Kohn-Sham density and potential on the device (Sections 2.1-2.2).
//
//  k_density_xc : per tetrahedron, psi_l at the 4 quadrature points from the
//                 4 vertex rows of X (column scale dinv applied on the fly),
//                 rho = f sum_l psi_l^2, then the LDA energy density eps_xc
//                 and potential v_xc = d(rho eps)/d rho (Slater exchange and
//                 the Perdew-Wang 1992 correlation fit, unpolarized), plus
//                 per-block partial integrals.
//  k_load_vec   : b_i = int rho phi_i (row gather over incident tetrahedra).
//  k_veff       : V_eff(q) = V_ext(q) + sum_a U_a lambda_a(q) + v_xc(q).
//  Hartree CG   : L U = 4 pi b by Jacobi-preconditioned CG with the step
//                 scalars kept on the device (k_cg_*).
#include "common.hpp"

namespace ofks {

#define OFKS_QA 0.58541019662496845446
#define OFKS_QB 0.13819660112501051518

// LDA (Hartree atomic units).  rs = (3 / (4 pi rho))^(1/3).
__device__ void lda_eval(double rho, double &eps, double &v) {
    if (!(rho > 1e-30)) { eps = 0.0; v = 0.0; return; }
    const double pi = 3.14159265358979323846;
    // Slater exchange: eps_x = -3/4 (3 rho / pi)^(1/3), v_x = 4/3 eps_x
    const double kx = cbrt(3.0 * rho / pi);
    const double ex = -0.75 * kx, vx = -kx;
    // PW92 correlation
    const double A = 0.031091, a1 = 0.21370;
    const double b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
    const double rs = cbrt(3.0 / (4.0 * pi * rho));
    const double sr = sqrt(rs);
    const double den = 2.0 * A * (b1 * sr + b2 * rs + b3 * rs * sr + b4 * rs * rs);
    const double dden = A * (b1 / sr + 2.0 * b2 + 3.0 * b3 * sr + 4.0 * b4 * rs);
    const double lg = log1p(1.0 / den);
    const double pre = -2.0 * A * (1.0 + a1 * rs);
    const double ec = pre * lg;
    const double dec = -2.0 * A * a1 * lg - pre * dden / (den * den + den);
    eps = ex + ec;
    v = vx + ec - rs / 3.0 * dec;
}

// part[block][3] = {sum w rho, sum w eps rho, sum w v rho}, w = |K| / 4
template <typename T>
__global__ __launch_bounds__(256) void k_density_xc(int64_t nt, int p, const int32_t *__restrict__ tets,
                                                   const int32_t *__restrict__ dof,
                                                   const double *__restrict__ geom,
                                                   const T *__restrict__ X, const T *__restrict__ dinv,
                                                   double f, double *__restrict__ rho_q,
                                                   double *__restrict__ eps_q, double *__restrict__ vxc_q,
                                                   double *__restrict__ part) {
    __shared__ double red[3][256];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t row[4];
        for (int a = 0; a < 4; ++a) row[a] = dof[tets[4 * t + a]];
        double rq[4] = {0.0, 0.0, 0.0, 0.0};
        for (int l = 0; l < p; ++l) {
            double x[4];
            const double sc = (double)dinv[l];
            for (int a = 0; a < 4; ++a) x[a] = row[a] >= 0 ? (double)X[row[a] * p + l] * sc : 0.0;
            const double sum = x[0] + x[1] + x[2] + x[3];
            for (int q = 0; q < 4; ++q) {
                // psi(q) = QB * sum_a x_a + (QA - QB) x_q
                const double psi = OFKS_QB * sum + (OFKS_QA - OFKS_QB) * x[q];
                rq[q] = fma(psi, psi, rq[q]);
            }
        }
        const double w = 0.25 * geom[13 * t];
        for (int q = 0; q < 4; ++q) {
            const double rho = f * rq[q];
            double e, v;
            lda_eval(rho, e, v);
            if (rho_q) rho_q[4 * t + q] = rho;
            if (eps_q) eps_q[4 * t + q] = e;
            vxc_q[4 * t + q] = v;
            s0 += w * rho;
            s1 += w * e * rho;
            s2 += w * v * rho;
        }
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int wd = 128; wd > 0; wd >>= 1) {
        if (threadIdx.x < wd)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// b_i = sum_{K ni i} sum_q |K|/4 rho(q) lambda_a(q)
__global__ void k_load_vec(int64_t nn, const int32_t *__restrict__ dof, const int64_t *__restrict__ iptr,
                           const int32_t *__restrict__ inc, const double *__restrict__ geom,
                           const double *__restrict__ rho_q, double *__restrict__ b) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
    const int32_t i = dof[v];
    if (i < 0) return;
    double s = 0.0;
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k) {
        const int64_t t = inc[k] >> 2;
        const int a = inc[k] & 3;
        const double w = 0.25 * geom[13 * t];
        double acc = 0.0;
        for (int q = 0; q < 4; ++q) acc += rho_q[4 * t + q] * (q == a ? OFKS_QA : OFKS_QB);
        s += w * acc;
    }
    b[i] = s;
}

__global__ void k_veff(int64_t nt, const int32_t *__restrict__ tets, const int32_t *__restrict__ dof,
                       const double *__restrict__ U, const double *__restrict__ vext_q,
                       const double *__restrict__ vxc_q, double *__restrict__ veff_q) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double u[4];
    for (int a = 0; a < 4; ++a) {
        const int32_t j = dof[tets[4 * t + a]];
        u[a] = j >= 0 ? U[j] : 0.0;
    }
    const double sum = u[0] + u[1] + u[2] + u[3];
    for (int q = 0; q < 4; ++q) {
        const double vh = OFKS_QB * sum + (OFKS_QA - OFKS_QB) * u[q];
        veff_q[4 * t + q] = vext_q[4 * t + q] + vh + vxc_q[4 * t + q];
    }
}

// ---------------------------------------------------------------------------
// Hartree CG (one vector, FP64).  Scalars in sc[]: 0 rz, 1 rr, 2 bb, 3 alpha,
// 4 beta, 5 dq.  part holds per-block partials.
// ---------------------------------------------------------------------------
__device__ void block_sum2(double a, double b, double *out_a, double *out_b) {
    __shared__ double ra[256], rb[256];
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) { ra[threadIdx.x] += ra[threadIdx.x + w]; rb[threadIdx.x] += rb[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { *out_a = ra[0]; *out_b = rb[0]; }
}

// r = rhs_scale * b - q ; d = r / diag ; partials rz, rr, and bb = |rhs|^2
__global__ __launch_bounds__(256) void k_cg_start(int64_t n, double scale, const double *__restrict__ b,
                                                 const double *__restrict__ q, const double *__restrict__ dg,
                                                 double *__restrict__ r, double *__restrict__ d,
                                                 double *__restrict__ part) {
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double rhs = scale * b[i];
        const double ri = rhs - q[i];
        const double z = ri / dg[i];
        r[i] = ri;
        d[i] = z;
        rz += ri * z;
        rr += ri * ri;
        bb += rhs * rhs;
    }
    __shared__ double r3[3][256];
    r3[0][threadIdx.x] = rz;
    r3[1][threadIdx.x] = rr;
    r3[2][threadIdx.x] = bb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int j = 0; j < 3; ++j) r3[j][threadIdx.x] += r3[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = r3[threadIdx.x][0];
}

// sums the 3-wide partials of nb blocks in a fixed order into sc[0..2]
__global__ __launch_bounds__(256) void k_cg_reduce3(int nb, const double *__restrict__ part, double *__restrict__ sc) {
    __shared__ double r[3][256];
    double a = 0, b = 0, c = 0;
    for (int k = threadIdx.x; k < nb; k += 256) { a += part[3 * k]; b += part[3 * k + 1]; c += part[3 * k + 2]; }
    r[0][threadIdx.x] = a; r[1][threadIdx.x] = b; r[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) for (int j = 0; j < 3; ++j) r[j][threadIdx.x] += r[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) { sc[0] = r[0][0]; sc[1] = r[1][0]; sc[2] = r[2][0]; }
}

// Fixed-order sum of part[k * stride + off], k < nb, computed identically by
// every block that calls it (all 256 threads; the result is returned to all).
__device__ __forceinline__ double block_fixed_sum(int nb, int stride, int off, const double *__restrict__ part) {
    __shared__ double r[256];
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) a += part[(int64_t)k * stride + off];
    r[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    const double v = r[0];
    __syncthreads();
    return v;
}

// One CG iteration after q = L d (partials dq[nb]): every block forms
// alpha = rz / <d, q> from the partials itself (same fixed order in every
// block), then x += alpha d, r -= alpha q, partials of <r, z> and <r, r>.
// rz is read from sc[0] or sc[6] by iteration parity (k_cg_dir writes the
// other slot, so no block overwrites a value another block still reads).
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int parity, double *__restrict__ sc, int nb,
                                              const double *__restrict__ dq, const double *__restrict__ d,
                                              const double *__restrict__ q, const double *__restrict__ dg,
                                              double *__restrict__ x, double *__restrict__ r,
                                              double *__restrict__ part) {
    const double dqs = block_fixed_sum(nb, 1, 0, dq);
    const double rz_old = sc[parity ? 6 : 0];
    const double alpha = dqs > 0.0 ? rz_old / dqs : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[3] = alpha;
        sc[5] = dqs;
    }
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = fma(alpha, d[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        rz += ri * ri / dg[i];
        rr += ri * ri;
    }
    block_sum2(rz, rr, &part[3 * blockIdx.x], &part[3 * blockIdx.x + 1]);
}

// beta = <r, z>_new / <r, z>_old from the k_cg_xr partials (formed in every
// block), d = z + beta d; block 0 stores <r, z>_new in the other parity slot
// and <r, r> in sc[1] (the host's convergence check).
__global__ __launch_bounds__(256) void k_cg_dir(int64_t n, int parity, double *__restrict__ sc, int nb,
                                               const double *__restrict__ part, const double *__restrict__ r,
                                               const double *__restrict__ dg, double *__restrict__ d) {
    const double rz_new = block_fixed_sum(nb, 3, 0, part);
    const double rr = block_fixed_sum(nb, 3, 1, part);
    const double rz_old = sc[parity ? 6 : 0];
    const double beta = rz_old > 0.0 ? rz_new / rz_old : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[parity ? 0 : 6] = rz_new;
        sc[1] = rr;
        sc[4] = beta;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = fma(beta, d[i], r[i] / dg[i]);
}

// dot products for energies: part[block] = sum a .* b
__global__ __launch_bounds__(256) void k_dot(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                            double *__restrict__ part) {
    __shared__ double r[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s = fma(a[i], b[i], s);
    r[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = r[0];
}

// ---------------------------------------------------------------------------
static inline unsigned nb_of(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
hipError_t launch_density_xc(hipStream_t s, int grid, int64_t nt, int p, const int32_t *tets, const int32_t *dof,
                             const double *geom, const T *X, const T *dinv, double f, double *rho_q,
                             double *eps_q, double *vxc_q, double *part) {
    hipLaunchKernelGGL((k_density_xc<T>), dim3(grid), dim3(256), 0, s, nt, p, tets, dof, geom, X, dinv, f, rho_q,
                       eps_q, vxc_q, part);
    return hipGetLastError();
}
template hipError_t launch_density_xc<double>(hipStream_t, int, int64_t, int, const int32_t *, const int32_t *,
                                              const double *, const double *, const double *, double, double *,
                                              double *, double *, double *);
template hipError_t launch_density_xc<float>(hipStream_t, int, int64_t, int, const int32_t *, const int32_t *,
                                             const double *, const float *, const float *, double, double *,
                                             double *, double *, double *);

hipError_t launch_load_vec(hipStream_t s, int64_t nn, const int32_t *dof, const int64_t *iptr, const int32_t *inc,
                           const double *geom, const double *rho_q, double *b) {
    hipLaunchKernelGGL(k_load_vec, dim3(nb_of(nn, 256)), dim3(256), 0, s, nn, dof, iptr, inc, geom, rho_q, b);
    return hipGetLastError();
}
hipError_t launch_veff(hipStream_t s, int64_t nt, const int32_t *tets, const int32_t *dof, const double *U,
                       const double *vext_q, const double *vxc_q, double *veff_q) {
    hipLaunchKernelGGL(k_veff, dim3(nb_of(nt, 256)), dim3(256), 0, s, nt, tets, dof, U, vext_q, vxc_q, veff_q);
    return hipGetLastError();
}
hipError_t launch_cg_start(hipStream_t s, int grid, int64_t n, double scale, const double *b, const double *q,
                           const double *dg, double *r, double *d, double *part, double *sc) {
    hipLaunchKernelGGL(k_cg_start, dim3(grid), dim3(256), 0, s, n, scale, b, q, dg, r, d, part);
    hipLaunchKernelGGL(k_cg_reduce3, dim3(1), dim3(256), 0, s, grid, part, sc);
    return hipGetLastError();
}
// nb_dq: the number of <d, q> partials (the product's grid)
hipError_t launch_cg_xr(hipStream_t s, int grid, int64_t n, int parity, double *sc, int nb_dq, const double *dq,
                        const double *d, const double *q, const double *dg, double *x, double *r, double *part) {
    hipLaunchKernelGGL(k_cg_xr, dim3(grid), dim3(256), 0, s, n, parity, sc, nb_dq, dq, d, q, dg, x, r, part);
    return hipGetLastError();
}

hipError_t launch_cg_dir(hipStream_t s, int grid, int64_t n, int parity, double *sc, const double *part,
                         const double *r, const double *dg, double *d) {
    hipLaunchKernelGGL(k_cg_dir, dim3(grid), dim3(256), 0, s, n, parity, sc, grid, part, r, dg, d);
    return hipGetLastError();
}
hipError_t launch_dot(hipStream_t s, int grid, int64_t n, const double *a, const double *b, double *part) {
    hipLaunchKernelGGL(k_dot, dim3(grid), dim3(256), 0, s, n, a, b, part);
    return hipGetLastError();
}

}  // namespace ofks
