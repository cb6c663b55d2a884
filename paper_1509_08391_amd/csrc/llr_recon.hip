// llr_recon.hip -- FP64 reconstruction kernels (arXiv:1509.08391):
//   ln rho at the interval centres by the trapezium recursion (eq. (kk3a)),
//   in the convention a_k = -d ln rho/dE:  L_{k+1} = L_k - (s/2)(a_k + a_{k+1});
//   canonical moments by the midpoint sums (eqs. (l19)-(l20)):
//   p_k ~ exp(L_k + beta c_k), <E> = sum p_k c_k, Var(E) = sum p_k (c_k - <E>)^2,
//   <u> = <E>/(6V), C_V = Var(E)/(6V) (Sec. 3.4).
#include <hip/hip_runtime.h>

#include "llr_internal.hpp"

namespace llr {

constexpr int kRB = 256;

// the recursion is sequential by definition: one thread
__global__ void k_lnrho(const double* __restrict__ a, int n, double s, double* __restrict__ L) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double v = 0.0;
    L[0] = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        v = v - 0.5 * s * (a[k] + a[k + 1]);
        L[k + 1] = v;
    }
}

__device__ double block_max(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < kRB / 64; ++i) r = fmax(r, sh[i]);
    __syncthreads();
    return r;
}
__device__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < kRB / 64; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// block-wide (mean, variance) of E at coupling beta
__device__ void moments(const double* __restrict__ c, const double* __restrict__ L, int n, double beta, double* sh,
                        double* mean, double* var) {
    double m = -INFINITY;
    for (int k = threadIdx.x; k < n; k += kRB) m = fmax(m, L[k] + beta * c[k]);
    m = block_max(m, sh);
    double z = 0.0, s1 = 0.0;
    for (int k = threadIdx.x; k < n; k += kRB) {
        const double wk = exp(L[k] + beta * c[k] - m);
        z += wk;
        s1 += wk * c[k];
    }
    z = block_sum(z, sh);
    s1 = block_sum(s1, sh);
    const double mu = s1 / z;
    double s2 = 0.0;
    for (int k = threadIdx.x; k < n; k += kRB) {
        const double wk = exp(L[k] + beta * c[k] - m);
        s2 += wk * (c[k] - mu) * (c[k] - mu);
    }
    s2 = block_sum(s2, sh);
    *mean = mu;
    *var = s2 / z;
}

// one block per beta
__global__ __launch_bounds__(kRB) void k_moments(const double* __restrict__ c, const double* __restrict__ L, int n,
                                                  const double* __restrict__ beta, double six_v, double* __restrict__ u,
                                                  double* __restrict__ cv) {
    __shared__ double sh[kRB / 64];
    double mu, var;
    moments(c, L, n, beta[blockIdx.x], sh, &mu, &var);
    if (threadIdx.x == 0) {
        u[blockIdx.x] = mu / six_v;
        cv[blockIdx.x] = var / six_v;
    }
}

// Var(E) on the grid blo + i h, i = 0..ng (one block per point)
__global__ __launch_bounds__(kRB) void k_var_grid(const double* __restrict__ c, const double* __restrict__ L, int n,
                                                   double blo, double h, double* __restrict__ var) {
    __shared__ double sh[kRB / 64];
    double mu, v;
    moments(c, L, n, blo + (double)blockIdx.x * h, sh, &mu, &v);
    if (threadIdx.x == 0) var[blockIdx.x] = v;
}

// argmax of the grid, then golden section on [b* - h, b* + h] to tol (one block)
__global__ __launch_bounds__(kRB) void k_golden(const double* __restrict__ c, const double* __restrict__ L, int n,
                                                 const double* __restrict__ var, long ng, double blo, double bhi,
                                                 double h, double tol, double six_v, double* __restrict__ out) {
    __shared__ double sh[kRB / 64];
    __shared__ double sbest;
    __shared__ long sidx;
    if (threadIdx.x == 0) {
        double best = -INFINITY;
        long bi = 0;
        for (long i = 0; i <= ng; ++i)
            if (var[i] > best) { best = var[i]; bi = i; }
        sbest = best;
        sidx = bi;
    }
    __syncthreads();
    const double best = sbest, bb = blo + (double)sidx * h;
    double x0 = fmax(blo, bb - h), x3 = fmin(bhi, bb + h);
    const double gr = 0.61803398874989484820;
    double x1 = x3 - gr * (x3 - x0), x2 = x0 + gr * (x3 - x0), mu, f1, f2;
    moments(c, L, n, x1, sh, &mu, &f1);
    moments(c, L, n, x2, sh, &mu, &f2);
    while (x3 - x0 > tol) {
        if (f1 > f2) {
            x3 = x2; x2 = x1; f2 = f1;
            x1 = x3 - gr * (x3 - x0);
            moments(c, L, n, x1, sh, &mu, &f1);
        } else {
            x0 = x1; x1 = x2; f1 = f2;
            x2 = x0 + gr * (x3 - x0);
            moments(c, L, n, x2, sh, &mu, &f2);
        }
    }
    double bc = 0.5 * (x0 + x3), v;
    moments(c, L, n, bc, sh, &mu, &v);
    if (best > v) { bc = bb; v = best; }
    if (threadIdx.x == 0) {
        out[0] = bc;
        out[1] = v / six_v;
    }
}

void launch_recon(const double* c, const double* a, int n, double s, double six_v, const double* beta, int nb,
                  double* lnrho, double* u, double* cv, hipStream_t st) {
    hipLaunchKernelGGL(k_lnrho, dim3(1), dim3(64), 0, st, a, n, s, lnrho);
    if (nb > 0) hipLaunchKernelGGL(k_moments, dim3(nb), dim3(kRB), 0, st, c, lnrho, n, beta, six_v, u, cv);
}

// lnrho_scratch holds n + ng + 1 doubles
void launch_beta_c(const double* c, const double* a, int n, double s, double six_v, double blo, double bhi, double h,
                   double tol, double* lnrho_scratch, double* out2, hipStream_t st) {
    const long ng = (long)floor((bhi - blo) / h + 0.5);
    double* var = lnrho_scratch + n;
    hipLaunchKernelGGL(k_lnrho, dim3(1), dim3(64), 0, st, a, n, s, lnrho_scratch);
    hipLaunchKernelGGL(k_var_grid, dim3((unsigned)(ng + 1)), dim3(kRB), 0, st, c, lnrho_scratch, n, blo, h, var);
    hipLaunchKernelGGL(k_golden, dim3(1), dim3(kRB), 0, st, c, lnrho_scratch, n, var, ng, blo, bhi, h, tol, six_v, out2);
}

}  // namespace llr
