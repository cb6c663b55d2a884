/* Test driver for the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitizers.py): exercises the sweeps in every mode and
 * order (the staggered one through per-chain orders), the per-link pass, replica exchange, the reconstruction and the
 * network, on small lattices; any out-of-bounds access, leak or undefined
 * operation aborts with a non-zero status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_hot_start(int d, int L, int n_chains, uint64_t seed, int lattice_id, int f32, double *theta);
double or_energy(int d, int L, const double *theta);
void or_sweeps(int d, int L, int n_chains, double *theta, const double *a, const double *lo, const double *hi,
               const int *interval, double *E, int n_sweeps, uint32_t sweep0, int mode, int kind, int do_or,
               uint64_t seed, int lattice_id, int f32, int *bits, const int *do_or_ch);
int or_class_pass(int d, int L, double *theta, int hb, int colour, int mode, double a, double lo, double hi,
                  double *E, uint64_t seed, int kind, int lattice_id, uint32_t sweep, uint32_t interval, int f32,
                  double *margin, double *dE_out);
void or_link_pass(int d, int L, double *theta, int colour, double a, double lo, double hi, double *E,
                  uint64_t seed, int kind, int lattice_id, uint32_t sweep, uint32_t interval, int f32,
                  double *margin, int *how);
void or_replica_run(int d, int L, int n, double *theta, const double *a, const double *lo, const double *hi,
                    double *E, int *conf, int *itv, int n_sweeps, uint32_t sweep0, uint64_t seed,
                    int lattice_id, int order, double *E_vis, long long *re_acc);
void or_reconstruct(const double *centres, const double *a, int n, double s, double six_v, const double *beta,
                    int nb, double *lnrho, double *u_mean, double *cv);
void or_beta_c(const double *centres, const double *a, int n, double s, double six_v, double blo, double bhi,
               double h, double tol, double *beta_c, double *cv_peak);
int or_mlp_nparams(void);
void or_mlp_init(uint64_t seed, double *w);
void or_mlp_train(double *w, const double *u, const double *invL, const double *a, int n, int epochs, double lr,
                  double *loss_hist);

int main(void)
{
    const uint64_t seed = 1509083910ull;
    for (int d = 2; d <= 4; d += 2) {
        const int L = d == 2 ? 6 : 4;
        long V = 1;
        for (int m = 0; m < d; ++m) V *= L;
        const int n = 4;
        double *th = malloc(sizeof(double) * (size_t)(n * d * V));
        double E[4], a[4], lo[4], hi[4];
        int itv[4], conf[4], bits[4 * 3];
        or_hot_start(d, L, n, seed, 0, 0, th);
        for (int c = 0; c < n; ++c) {
            E[c] = or_energy(d, L, th + c * d * V);
            a[c] = 0.9 + 0.1 * c;
            lo[c] = -1e9;
            hi[c] = 1e9;
            itv[c] = c;
            conf[c] = c;
        }
        /* free, approach-like and restricted sweeps in both orders, and heatbath-only */
        for (int order = 1; order <= 2; ++order)
            or_sweeps(d, L, n, th, a, lo, hi, itv, E, 3, 5, 2, 0, order, seed, 0, 0, bits, NULL);
        or_sweeps(d, L, n, th, a, lo, hi, itv, E, 2, 9, 2, 0, 0, seed, 0, 1, bits, NULL);
        /* the staggered order: per-chain pass orders */
        const int stag[4] = {1, 1, 3, 3};
        or_sweeps(d, L, n, th, a, lo, hi, itv, E, 2, 7, 2, 0, 1, seed, 0, 0, bits, stag);
        for (int c = 0; c < n; ++c) {
            lo[c] = E[c] - 2.0;
            hi[c] = E[c] + 2.0;
        }
        or_sweeps(d, L, n, th, a, lo, hi, itv, E, 3, 11, 0, 0, 1, seed, 0, 0, bits, stag);
        double *mg = malloc(sizeof(double) * (size_t)(V / 2 + 1));
        int *how = malloc(sizeof(int) * (size_t)(V / 2 + 1));
        double dE = 0.0;
        for (int col = 0; col < 2 * d; ++col) {
            or_class_pass(d, L, th, 1, col, 0, a[0], lo[0], hi[0], &E[0], seed, 0, 0, 20, 0, 1, mg, &dE);
            or_link_pass(d, L, th + d * V, col, a[1], lo[1], hi[1], &E[1], seed, 0, 0, 21, 1, 0, mg, how);
        }
        /* overlapping intervals with replica exchange */
        double cen[4];
        for (int k = 0; k < n; ++k) {
            cen[k] = E[0] + 1.0 * (k - 1.5);
            lo[k] = cen[k] - 1.0;
            hi[k] = cen[k] + 1.0;
        }
        long long re[2] = {0, 0};
        double *vis = malloc(sizeof(double) * (size_t)(5 * n));
        or_replica_run(d, L, n, th, a, lo, hi, E, conf, itv, 5, 30, seed, 0, 1, vis, re);
        free(vis);
        free(how);
        free(mg);
        free(th);
    }
    /* reconstruction and beta_c on a smooth a_k */
    enum { NI = 24, NB = 11 };
    double cen[NI], ak[NI], beta[NB], lnrho[NI], u[NB], cv[NB], bc = 0.0, pk = 0.0;
    for (int k = 0; k < NI; ++k) {
        cen[k] = 900.0 + 10.0 * k;
        ak[k] = 1.05 - 0.004 * k;
    }
    for (int j = 0; j < NB; ++j) beta[j] = 0.98 + 0.01 * j;
    or_reconstruct(cen, ak, NI, 10.0, 1536.0, beta, NB, lnrho, u, cv);
    or_beta_c(cen, ak, NI, 10.0, 1536.0, 0.98, 1.08, 1e-5, 1e-9, &bc, &pk);
    /* the network: a few epochs on synthetic targets */
    const int np = or_mlp_nparams();
    double *w = malloc(sizeof(double) * (size_t)np);
    double uu[8], il[8], aa[8], loss[5];
    for (int i = 0; i < 8; ++i) {
        uu[i] = 0.58 + 0.01 * i;
        il[i] = i < 4 ? 0.125 : 0.0625;
        aa[i] = 1.0 + 0.01 * i;
    }
    or_mlp_init(seed, w);
    or_mlp_train(w, uu, il, aa, 8, 5, 1e-3, loss);
    free(w);
    printf("oracle sanitizer run: beta_c %.6f, loss %.3e -> %.3e\n", bc, loss[0], loss[4]);
    return 0;
}
