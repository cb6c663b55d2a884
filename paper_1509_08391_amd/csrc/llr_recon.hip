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

// The recursion is sequential by definition: one thread per set of a_k
// (row r of a and of L at offset r n).
__global__ void k_lnrho(const double* __restrict__ a, int n, int rows, double s, double* __restrict__ L) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= rows) return;
    const double* ar = a + (size_t)r * n;
    double* Lr = L + (size_t)r * n;
    double v = 0.0;
    Lr[0] = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        v = v - 0.5 * s * (ar[k] + ar[k + 1]);
        Lr[k + 1] = v;
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

// Var(E) on the grid blo + i h, i = 0..ng (one block per point; blockIdx.y
// selects the set of a_k: L row y, var row y of ng + 1)
__global__ __launch_bounds__(kRB) void k_var_grid(const double* __restrict__ c, const double* __restrict__ L, int n,
                                                   double blo, double h, long ng, double* __restrict__ var) {
    __shared__ double sh[kRB / 64];
    double mu, v;
    moments(c, L + (size_t)blockIdx.y * n, n, blo + (double)blockIdx.x * h, sh, &mu, &v);
    if (threadIdx.x == 0) var[(size_t)blockIdx.y * (size_t)(ng + 1) + blockIdx.x] = v;
}

// argmax of the grid, then golden section on [b* - h, b* + h] to tol (one
// block per set of a_k: L row, var row and out pair selected by blockIdx.x)
__global__ __launch_bounds__(kRB) void k_golden(const double* __restrict__ c, const double* __restrict__ Lrows, int n,
                                                 const double* __restrict__ var_rows, long ng, double blo, double bhi,
                                                 double h, double tol, double six_v, double* __restrict__ out_rows) {
    const double* L = Lrows + (size_t)blockIdx.x * n;
    const double* var = var_rows + (size_t)blockIdx.x * (size_t)(ng + 1);
    double* out = out_rows + 2 * (size_t)blockIdx.x;
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
    hipLaunchKernelGGL(k_lnrho, dim3(1), dim3(64), 0, st, a, n, 1, s, lnrho);
    if (nb > 0) hipLaunchKernelGGL(k_moments, dim3(nb), dim3(kRB), 0, st, c, lnrho, n, beta, six_v, u, cv);
}

// beta_c and the C_V peak for `rows` sets of a_k (a row r at a + r n);
// scratch holds rows (n + ng + 1) doubles, out2 rows pairs
void launch_beta_c_rows(const double* c, const double* a, int n, int rows, double s, double six_v, double blo,
                        double bhi, double h, double tol, double* scratch, double* out2, hipStream_t st) {
    const long ng = (long)floor((bhi - blo) / h + 0.5);
    double* L = scratch;
    double* var = scratch + (size_t)rows * n;
    hipLaunchKernelGGL(k_lnrho, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0, st, a, n, rows, s, L);
    hipLaunchKernelGGL(k_var_grid, dim3((unsigned)(ng + 1), (unsigned)rows), dim3(kRB), 0, st, c, L, n, blo, h, ng,
                       var);
    hipLaunchKernelGGL(k_golden, dim3((unsigned)rows), dim3(kRB), 0, st, c, L, n, var, ng, blo, bhi, h, tol, six_v,
                       out2);
}

void launch_beta_c(const double* c, const double* a, int n, double s, double six_v, double blo, double bhi, double h,
                   double tol, double* lnrho_scratch, double* out2, hipStream_t st) {
    launch_beta_c_rows(c, a, n, 1, s, six_v, blo, bhi, h, tol, lnrho_scratch, out2, st);
}

// ---------------------------------------------------------------------------
// Bootstrap over N_B independent runs (Algorithm 1 repeated N_B times, Sec. 2.4
// and Sec. 3.2): sample b draws n_runs runs with replacement, run j of sample
// b being floor(n_runs w / 2^32) for the first word w of Philox counter
// (j, kind 5, b, 0), and averages their a_k (runs summed in draw order).
// ---------------------------------------------------------------------------
constexpr int kMaxRuns = 1024;

__global__ __launch_bounds__(kRB) void k_boot_mean(const double* __restrict__ a_runs, int n_runs, int n, uint32_t k0,
                                                    uint32_t k1, double* __restrict__ abar) {
    __shared__ int idx[kMaxRuns];
    const uint32_t b = blockIdx.x;
    for (int j = threadIdx.x; j < n_runs; j += kRB) {
        const uint4 w = philox10(make_uint4((uint32_t)j, ctr1_word(0, 0, kBoot, 0), b, 0u), k0, k1);
        idx[j] = (int)(((uint64_t)w.x * (uint64_t)n_runs) >> 32);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += kRB) {
        double sum = 0.0;
        for (int j = 0; j < n_runs; ++j) sum += a_runs[(size_t)idx[j] * n + k];
        abar[(size_t)b * n + k] = sum / (double)n_runs;
    }
}

void launch_boot_mean(const double* a_runs, int n_runs, int n, int n_boot, uint64_t seed, double* abar,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_boot_mean, dim3((unsigned)n_boot), dim3(kRB), 0, st, a_runs, n_runs, n, (uint32_t)seed,
                       (uint32_t)(seed >> 32), abar);
}

// ---------------------------------------------------------------------------
// Probability density P_beta(E) = rho~(E) e^{beta E} / Z (Sec. 3.4) of the
// piecewise-exponential rho~ of eq. (rhoguess): in interval k (centre c_k,
// width s) ln rho~(E) = L_k - a_k (E - c_k), continuous at the edges by the
// trapezium recursion.  Z is the exact integral over the covered range:
// Z = sum_k s e^{L_k + beta c_k} sinh(x_k)/x_k, x_k = (beta - a_k) s / 2.
// ---------------------------------------------------------------------------
__device__ double log_sinhc(double x) {
    const double ax = fabs(x);
    if (ax < 1e-3) return ax * ax * (1.0 / 6.0) - ax * ax * ax * ax * (1.0 / 180.0);
    if (ax < 20.0) return log(sinh(ax) / ax);
    return ax - log(2.0 * ax) + log1p(-exp(-2.0 * ax));
}

// one block: ln Z, with the row maximum subtracted before the sum
__global__ __launch_bounds__(kRB) void k_logz(const double* __restrict__ c, const double* __restrict__ L,
                                               const double* __restrict__ a, int n, double s, double beta,
                                               double* __restrict__ lnz) {
    __shared__ double sh[kRB / 64];
    double m = -INFINITY;
    for (int k = threadIdx.x; k < n; k += kRB)
        m = fmax(m, L[k] + beta * c[k] + log_sinhc((beta - a[k]) * 0.5 * s));
    m = block_max(m, sh);
    double z = 0.0;
    for (int k = threadIdx.x; k < n; k += kRB)
        z += exp(L[k] + beta * c[k] + log_sinhc((beta - a[k]) * 0.5 * s) - m);
    z = block_sum(z, sh);
    if (threadIdx.x == 0) lnz[0] = m + log(s * z);
}

// ln P at m points E (one thread each; -inf outside the covered range)
__global__ void k_logp(const double* __restrict__ c, const double* __restrict__ L, const double* __restrict__ a,
                       int n, double s, double beta, const double* __restrict__ E, int m,
                       const double* __restrict__ lnz, double* __restrict__ logp) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= m) return;
    const double lo = c[0] - 0.5 * s, hi = c[n - 1] + 0.5 * s, e = E[i];
    if (!(e >= lo && e <= hi)) {
        logp[i] = -INFINITY;
        return;
    }
    int k = (int)floor((e - lo) / s);
    k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
    logp[i] = (L[k] + beta * c[k] - lnz[0]) + (beta - a[k]) * (e - c[k]);
}

// Interior local maxima of ln P: ln P is linear with slope beta - a_k in
// interval k, so the edge between k and k+1 is a maximum iff beta - a_k > 0
// and beta - a_{k+1} <= 0 (one thread; every maximum counted, at most
// max_peaks stored in order of E).
__global__ void k_peaks(const double* __restrict__ c, const double* __restrict__ L, const double* __restrict__ a,
                        int n, double s, double beta, const double* __restrict__ lnz, int max_peaks,
                        double* __restrict__ E_out, double* __restrict__ lp_out, int* __restrict__ n_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int np = 0;
    for (int k = 0; k + 1 < n; ++k) {
        if (beta - a[k] > 0.0 && beta - a[k + 1] <= 0.0) {
            if (np < max_peaks) {
                E_out[np] = c[k] + 0.5 * s;
                lp_out[np] = (L[k] + beta * c[k] - lnz[0]) + (beta - a[k]) * (0.5 * s);
            }
            ++np;
        }
    }
    *n_out = np;
}

// scratch: n (ln rho) + 1 (ln Z) doubles
void launch_prob(const double* c, const double* a, int n, double s, double beta, const double* E, int m,
                 double* logp, int max_peaks, double* E_pk, double* lp_pk, int* n_pk, double* scratch,
                 hipStream_t st) {
    double* L = scratch;
    double* lnz = scratch + n;
    hipLaunchKernelGGL(k_lnrho, dim3(1), dim3(64), 0, st, a, n, 1, s, L);
    hipLaunchKernelGGL(k_logz, dim3(1), dim3(kRB), 0, st, c, L, a, n, s, beta, lnz);
    if (m > 0) hipLaunchKernelGGL(k_logp, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, c, L, a, n, s, beta,
                                  E, m, lnz, logp);
    if (n_pk) hipLaunchKernelGGL(k_peaks, dim3(1), dim3(64), 0, st, c, L, a, n, s, beta, lnz, max_peaks, E_pk, lp_pk,
                                 n_pk);
}

// ---------------------------------------------------------------------------
// Reweighting of multicanonical samples (Sec. 2.6, eq. (4.7)): with the
// sampling weight W(E) = 1/rho~(E) (first and last pieces continued outside
// the intervals), <O>_beta = <O e^{beta E} / W(E)>_W / <e^{beta E} / W(E)>_W.
// One block per beta: <E>, Var(E) -> <u> = <E>/(6V), C_V = Var(E)/(6V).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rw_lnw(const double* c, const double* L, const double* a, int n, double s,
                                         double e) {
    int k = (int)floor((e - (c[0] - 0.5 * s)) / s);
    k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
    return -L[k] + a[k] * (e - c[k]);
}

__global__ __launch_bounds__(kRB) void k_rw_moments(const double* __restrict__ E, long m,
                                                     const double* __restrict__ c, const double* __restrict__ L,
                                                     const double* __restrict__ a, int n, double s,
                                                     const double* __restrict__ beta, double six_v,
                                                     double* __restrict__ u, double* __restrict__ cv) {
    __shared__ double sh[kRB / 64];
    const double b = beta[blockIdx.x];
    double mx = -INFINITY;
    for (long i = threadIdx.x; i < m; i += kRB) mx = fmax(mx, b * E[i] - rw_lnw(c, L, a, n, s, E[i]));
    mx = block_max(mx, sh);
    double z = 0.0, s1 = 0.0;
    for (long i = threadIdx.x; i < m; i += kRB) {
        const double w = exp(b * E[i] - rw_lnw(c, L, a, n, s, E[i]) - mx);
        z += w;
        s1 += w * E[i];
    }
    z = block_sum(z, sh);
    s1 = block_sum(s1, sh);
    const double mu = s1 / z;
    double s2 = 0.0;
    for (long i = threadIdx.x; i < m; i += kRB) {
        const double w = exp(b * E[i] - rw_lnw(c, L, a, n, s, E[i]) - mx);
        s2 += w * (E[i] - mu) * (E[i] - mu);
    }
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        u[blockIdx.x] = mu / six_v;
        cv[blockIdx.x] = s2 / z / six_v;
    }
}

// scratch: n doubles (ln rho)
void launch_reweight(const double* E, long m, const double* c, const double* a, int n, double s, const double* beta,
                     int nb, double six_v, double* u, double* cv, double* scratch, hipStream_t st) {
    hipLaunchKernelGGL(k_lnrho, dim3(1), dim3(64), 0, st, a, n, 1, s, scratch);
    hipLaunchKernelGGL(k_rw_moments, dim3((unsigned)nb), dim3(kRB), 0, st, E, m, c, scratch, a, n, s, beta, six_v, u,
                       cv);
}

// ---------------------------------------------------------------------------
// Observables from restricted double brackets (Sec. 2.3, eqs. (l9)-(l10)):
//   <B>_beta = sum_k rho~(c_k) e^{beta c_k} <<B e^{(beta - a_k)(E - c_k)}>>_k
//            / sum_k rho~(c_k) e^{beta c_k} <<e^{(beta - a_k)(E - c_k)}>>_k,
// with <<.>>_k the mean over the m samples (E, B) of interval k (row-major
// m x n, interval fastest).  One block per beta; the interval terms are
// combined in log space.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRB) void k_obs_bracket(const double* __restrict__ E, const double* __restrict__ B,
                                                      int m, const double* __restrict__ c,
                                                      const double* __restrict__ L, const double* __restrict__ a,
                                                      int n, const double* __restrict__ beta,
                                                      double* __restrict__ out) {
    __shared__ double sh[kRB / 64];
    const double b = beta[blockIdx.x];
    // per interval: ln D_k and N_k / D_k, D_k = <<e^{x}>>, x = (b - a_k)(E - c_k), shifted by the interval's max
    double wmax = -INFINITY;
    for (int k = threadIdx.x; k < n; k += kRB) {
        double xm = -INFINITY;
        for (int j = 0; j < m; ++j) xm = fmax(xm, (b - a[k]) * (E[(size_t)j * n + k] - c[k]));
        double d = 0.0;
        for (int j = 0; j < m; ++j) d += exp((b - a[k]) * (E[(size_t)j * n + k] - c[k]) - xm);
        wmax = fmax(wmax, L[k] + b * c[k] + xm + log(d / m));
    }
    wmax = block_max(wmax, sh);
    double num = 0.0, den = 0.0;
    for (int k = threadIdx.x; k < n; k += kRB) {
        double xm = -INFINITY;
        for (int j = 0; j < m; ++j) xm = fmax(xm, (b - a[k]) * (E[(size_t)j * n + k] - c[k]));
        double d = 0.0, nb = 0.0;
        for (int j = 0; j < m; ++j) {
            const double w = exp((b - a[k]) * (E[(size_t)j * n + k] - c[k]) - xm);
            d += w;
            nb += w * B[(size_t)j * n + k];
        }
        const double wk = exp(L[k] + b * c[k] + xm + log(d / m) - wmax);
        den += wk;
        num += wk * (nb / d);
    }
    den = block_sum(den, sh);
    num = block_sum(num, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = num / den;
}

// scratch: n doubles (ln rho)
void launch_obs_bracket(const double* E, const double* B, int m, const double* c, const double* a, int n, double s,
                        const double* beta, int nb, double* out, double* scratch, hipStream_t st) {
    hipLaunchKernelGGL(k_lnrho, dim3(1), dim3(64), 0, st, a, n, 1, s, scratch);
    hipLaunchKernelGGL(k_obs_bracket, dim3((unsigned)nb), dim3(kRB), 0, st, E, B, m, c, scratch, a, n, beta, out);
}

}  // namespace llr
