/*
 * llr_oracle.c -- plain, slow CPU reference of the LLR energy-restricted sweep
 * for compact U(1) lattice gauge theory (Langfeld, Lucini, Pellegrini, Rago,
 * "An efficient algorithm for numerical computations of continuous densities
 * of states", arXiv:1509.08391).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library; the only thing the two sides have in common
 * is the published definition of the counter-based generator (Philox4x32-10,
 * Salmon, Moraes, Dror, Shaw, SC'11), which each side implements on its own.
 *
 * Everything is FP64 and written in the order the paper states it:
 *   - model and action: Sec. 3.1 (plaquette angle, Wilson action, Haar measure)
 *   - restricted expectation values and the interval indicator: Sec. 2.2,
 *     eqs. (kk7)-(kk9)
 *   - the observable Delta E and its root: eqs. (kk10)-(kk15)
 *   - the under-relaxed Newton-Raphson / Robbins-Monro update: eq. (kk21) and
 *     Algorithm 1 (update with the minus sign, beta-convention a ~ beta)
 *   - the restriction imposed per link when each angle is drawn: Sec. 2.4
 *   - replica exchange between overlapping intervals: Sec. 2.5
 *   - reconstruction: trapezium recursion eq. (kk3a), midpoint sums
 *     eqs. (l19)-(l20), specific heat of Sec. 3.4
 *
 * Sign convention (beta-convention): the restricted weight in interval k is
 * exp(+a E) 1[E in I_k], so that a_k = -d ln rho/dE ~ beta > 0 for E > 0.
 * With this reading Algorithm 1's update a <- a - 12 dE/((n+1) w^2) is the
 * correct sign (the paper's general LLR section and its U(1) application
 * attach opposite signs to a; in this convention a_k approaches beta where
 * <E>(beta) is the interval centre, which the 4D oracle pin checks).
 *
 * Parity pins (tests/test_oracle_*.py) check this file against brute-force
 * enumeration, closed forms (2D U(1) character expansion, von Mises moments,
 * the Robbins-Monro root of a known density), invariants (gauge invariance,
 * overrelaxation preserves the local action) and library routines.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_TWO_PI 6.28318530717958647692

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11: multipliers, Weyl key increments and */
/* round structure as published).                                            */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* batch helper for tests: ctr is n x 4, out is n x 4 */
void or_philox_batch(long n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out)
{
    for (long i = 0; i < n; ++i) or_philox(ctr + 4 * i, key, out + 4 * i);
}

/* Counter word 1 layout (shared convention, documented in include/llr.h):
 * bits 0-7 attempt pair, 8-11 colour/pass, 12-15 kind, 16-23 lattice id,
 * 24-31 replica id (reserved). */
enum { KIND_SWEEP = 0, KIND_INIT = 1, KIND_APPROACH = 2, KIND_REPLICA = 3, KIND_MLP = 4, KIND_MUCA = 6 };

static uint32_t ctr1_word(int attempt_pair, int colour, int kind, int lattice_id)
{
    return (uint32_t)(attempt_pair & 0xff) | ((uint32_t)(colour & 0xf) << 8) |
           ((uint32_t)(kind & 0xf) << 12) | ((uint32_t)(lattice_id & 0xff) << 16);
}

/* Uniforms.  u24 selects the 23-bit conversion used by single-precision
 * state (exact in single precision); the default uses all 32 bits.  Both are
 * exact in double precision and lie strictly inside (0,1) resp. (-1,1). */
static double uni01(uint32_t w, int u24)
{
    if (u24) return ((double)(w >> 9) + 0.5) * 0x1p-23;
    return ((double)w + 0.5) * 0x1p-32;
}
static double uni_signed(uint32_t w, int u24)
{
    int32_t s = (int32_t)w;
    if (u24) return ((double)(s >> 9) + 0.5) * 0x1p-22;
    return ((double)s + 0.5) * 0x1p-31;
}

void or_uniforms(long n, const uint32_t *w, int u24, double *u, double *v)
{
    for (long i = 0; i < n; ++i) { u[i] = uni01(w[i], u24); v[i] = uni_signed(w[i], u24); }
}

/* ------------------------------------------------------------------------ */
/* Geometry: periodic L^d lattice, lexicographic site index                  */
/* s = x0 + L x1 + L^2 x2 + ...; link (mu, s) stored at theta[mu*V + s].      */
/* Neighbour tables are built by brute force from the coordinates.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d, L;
    long V;
    long *up;   /* up[s*d + mu]   = site s + mu^ */
    long *dn;   /* dn[s*d + mu]   = site s - mu^ */
    int *par;   /* parity of s */
} geo_t;

static void coords_of(int d, int L, long s, int x[4])
{
    for (int m = 0; m < d; ++m) { x[m] = (int)(s % L); s /= L; }
}
static long site_of(int d, int L, const int x[4])
{
    long s = 0;
    for (int m = d - 1; m >= 0; --m) s = s * L + x[m];
    return s;
}

static int geo_init(geo_t *g, int d, int L)
{
    g->d = d; g->L = L;
    long V = 1;
    for (int m = 0; m < d; ++m) V *= L;
    g->V = V;
    g->up = (long *)malloc(sizeof(long) * V * d);
    g->dn = (long *)malloc(sizeof(long) * V * d);
    g->par = (int *)malloc(sizeof(int) * V);
    if (!g->up || !g->dn || !g->par) return -1;
    for (long s = 0; s < V; ++s) {
        int x[4] = {0, 0, 0, 0}, y[4];
        coords_of(d, L, s, x);
        int p = 0;
        for (int m = 0; m < d; ++m) p += x[m];
        g->par[s] = p & 1;
        for (int m = 0; m < d; ++m) {
            memcpy(y, x, sizeof(y));
            y[m] = (x[m] + 1) % L;
            g->up[s * d + m] = site_of(d, L, y);
            y[m] = (x[m] + L - 1) % L;
            g->dn[s * d + m] = site_of(d, L, y);
        }
    }
    return 0;
}
static void geo_free(geo_t *g)
{
    free(g->up); free(g->dn); free(g->par);
}

/* Exported neighbour query (used by the brute-force colouring pins). */
long or_neighbour(int d, int L, long s, int mu, int step)
{
    int x[4] = {0, 0, 0, 0};
    coords_of(d, L, s, x);
    x[mu] = ((x[mu] + step) % L + L) % L;
    return site_of(d, L, x);
}

/* Plaquette angle theta_{mu nu}(x), Sec. 3.1 */
static double plaq_angle(const geo_t *g, const double *th, long s, int mu, int nu)
{
    long V = g->V;
    int d = g->d;
    return th[mu * V + s] + th[nu * V + g->up[s * d + mu]] - th[mu * V + g->up[s * d + nu]] - th[nu * V + s];
}

/* E = sum_{x, mu<nu} cos theta_{mu nu}(x)  (the action without beta) */
static double energy(const geo_t *g, const double *th)
{
    double E = 0.0;
    for (long s = 0; s < g->V; ++s)
        for (int mu = 0; mu < g->d; ++mu)
            for (int nu = mu + 1; nu < g->d; ++nu) E += cos(plaq_angle(g, th, s, mu, nu));
    return E;
}

double or_energy(int d, int L, const double *theta)
{
    geo_t g;
    if (geo_init(&g, d, L)) return NAN;
    double E = energy(&g, theta);
    geo_free(&g);
    return E;
}

/* Adjoint plaquette sum B = sum_P cos(2 theta_P): the non-action observable
 * measured through the restricted double brackets of Sec. 2.3. */
double or_adjoint(int d, int L, const double *theta)
{
    geo_t g;
    if (geo_init(&g, d, L)) return NAN;
    double B = 0.0;
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < g.d; ++mu)
            for (int nu = mu + 1; nu < g.d; ++nu) B += cos(2.0 * plaq_angle(&g, theta, s, mu, nu));
    geo_free(&g);
    return B;
}

/* Local field of link (mu, s): the 2(d-1) plaquettes that contain the link,
 * each oriented so that theta_mu(s) enters with a plus sign:
 *   forward  (plane mu,nu at s):      theta + [th_nu(s+mu) - th_mu(s+nu) - th_nu(s)]
 *   backward (plane mu,nu at s-nu):  -(theta + [-th_nu(s+mu-nu) - th_mu(s-nu) + th_nu(s-nu)])
 * Since cos is even, sum_P cos theta_P = C cos(theta) - S sin(theta) with
 * C = sum cos(staple), S = sum sin(staple). */
static void local_field(const geo_t *g, const double *th, int mu, long s, double *C, double *S)
{
    long V = g->V;
    int d = g->d;
    double c = 0.0, sn = 0.0;
    for (int nu = 0; nu < d; ++nu) {
        if (nu == mu) continue;
        long s_pmu = g->up[s * d + mu];
        long s_pnu = g->up[s * d + nu];
        long s_mnu = g->dn[s * d + nu];
        long s_pmu_mnu = g->dn[s_pmu * d + nu];
        double sf = th[nu * V + s_pmu] - th[mu * V + s_pnu] - th[nu * V + s];
        double sb = -th[nu * V + s_pmu_mnu] - th[mu * V + s_mnu] + th[nu * V + s_mnu];
        c += cos(sf) + cos(sb);
        sn += sin(sf) + sin(sb);
    }
    *C = c; *S = sn;
}

void or_local_field(int d, int L, const double *theta, int mu, long s, double *C, double *S)
{
    geo_t g;
    if (geo_init(&g, d, L)) return;
    local_field(&g, theta, mu, s, C, S);
    geo_free(&g);
}

static double eps_local(double C, double S, double t) { return C * cos(t) - S * sin(t); }

/* wrap into [-pi, pi) */
static double wrap(double x)
{
    double y = x - OR_TWO_PI * floor((x + OR_PI) / OR_TWO_PI);
    if (y >= OR_PI) y -= OR_TWO_PI;
    if (y < -OR_PI) y += OR_TWO_PI;
    return y;
}

/* ------------------------------------------------------------------------ */
/* von Mises sampler: Best & Fisher, Appl. Statist. 28 (1979) 152-157, in    */
/* the algebraically identical half-angle form                               */
/*   rho = 2k/(tau + sqrt(2 tau)),  tau = 1 + sqrt(1 + 4k^2)                 */
/*   r = (1 + rho^2)/(2 rho),  c = k (r^2 - 1)/(r + z),  z = cos(pi V1)      */
/*   X = 2 atan(q tan(pi V1 / 2)),  q = (1 - rho)/(1 + rho)                  */
/* with V1 uniform on (-1, 1) (its sign gives the sign of X) and U2 on       */
/* (0, 1).  Attempt j uses Philox call j/2 (counter word 1 attempt field),   */
/* words (0,1) for even j and (2,3) for odd j.  64 attempts at most; if none */
/* is accepted the link keeps its value (returns 0).                          */
/* ------------------------------------------------------------------------ */
#define VM_CAP 64

typedef struct {
    double k, r, gg, q; /* kappa; r, sqrt(r^2 - 1) and q of the wrapped-Cauchy envelope */
} bf_t;

static void bf_setup(double k, bf_t *b)
{
    double tau = 1.0 + sqrt(1.0 + 4.0 * k * k);
    double rho = 2.0 * k / (tau + sqrt(2.0 * tau));
    b->k = k;
    b->r = (1.0 + rho * rho) / (2.0 * rho);
    b->gg = (1.0 - rho * rho) / (2.0 * rho); /* r^2 - 1 = gg^2 */
    b->q = (1.0 - rho) / (1.0 + rho);
}

/* One attempt from the words (wv, wu); on acceptance X is set and 1 returned.
 * *mg is lowered to the smallest |test statistic| seen (decision margin). */
static int bf_attempt(const bf_t *b, uint32_t wv, uint32_t wu, int u24, double *X, double *mg)
{
    double V1 = uni_signed(wv, u24);
    double U2 = uni01(wu, u24);
    double z = cos(OR_PI * V1);
    double c = b->k * b->gg * b->gg / (b->r + z);
    double t1 = c * (2.0 - c) - U2;
    int acc = 0;
    if (fabs(t1) < *mg) *mg = fabs(t1);
    if (t1 > 0.0) acc = 1;
    else {
        double t2 = log(c / U2) + 1.0 - c;
        if (fabs(t2) < *mg) *mg = fabs(t2);
        if (t2 >= 0.0) acc = 1;
    }
    if (acc) *X = 2.0 * atan(b->q * tan(0.5 * OR_PI * V1));
    return acc;
}

static int vm_draw(double kappa, const uint32_t key[2], uint32_t c0, uint32_t c1base,
                   uint32_t c2, uint32_t c3, int u24, double *X, double *margin)
{
    uint32_t w[4] = {0, 0, 0, 0};
    double mg = INFINITY;
    if (kappa == 0.0) {
        uint32_t ctr[4] = {c0, c1base, c2, c3};
        or_philox(ctr, key, w);
        *X = OR_PI * uni_signed(w[0], u24);
        if (margin) *margin = mg;
        return 1;
    }
    bf_t b;
    bf_setup(kappa, &b);
    for (int j = 0; j < VM_CAP; ++j) {
        if ((j & 1) == 0) {
            uint32_t ctr[4] = {c0, c1base | (uint32_t)(j >> 1), c2, c3};
            or_philox(ctr, key, w);
        }
        if (bf_attempt(&b, w[2 * (j & 1)], w[2 * (j & 1) + 1], u24, X, &mg)) {
            if (margin) *margin = mg;
            return j + 1;
        }
    }
    if (margin) *margin = mg;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Heatbath draw under the per-link analytic constraint (Sec. 2.4: the       */
/* restriction imposed when the new variable is generated).  Target:         */
/*   p(X) ~ exp(k cos X) on the candidates that ok() accepts, k >= 0,        */
/* where ok() keeps the running energy inside the interval; [u_lo, u_hi] is  */
/* the same window written on cos X (used for the envelope only).            */
/* Stage 1, rejection from the unrestricted conditional: the class           */
/* heatbath's own attempts 0..63 (same counters); the first one that passes  */
/* Best-Fisher and ok() is taken.  Stage 2, if none does: with x = |X| in    */
/* [x_a, x_b] = [acos u_hi, acos u_lo], exp(k cos x) <= exp(k u_hi -         */
/* lam (x - x_a)) for lam = k min(sin x_a, (u_hi - u_lo)/(x_b - x_a)): the   */
/* secant slope (cos x_a - cos x)/(x - x_a) is the mean of sin over          */
/* [x_a, x], which has no interior minimum because sin is unimodal on        */
/* [0, pi], so its smallest value is at an end.  x is drawn from that        */
/* truncated exponential and kept with probability                           */
/* exp(k (cos x - u_hi) + lam (x - x_a)); X = +-x with a fair sign bit.      */
/* Attempt i of stage 2 uses counter word 1 attempt field 64 + i, words 0    */
/* (envelope), 1 (acceptance), top bit of 2 (sign); 64 attempts at most.     */
/* Both stages sample the target exactly, so their mixture does.  Returns 1  */
/* or 2 (stage that produced X) or 0 (nothing within the caps: the caller    */
/* keeps the link).                                                          */
/* ------------------------------------------------------------------------ */
#define LINK_B_BASE 64
#define LINK_B_CAP 64
#define LINK_TINY 1e-12

typedef int (*window_fn)(double X, void *ctx, double *mg);

static int link_draw(double k, double u_lo, double u_hi, window_fn ok, void *okc, const uint32_t key[2],
                     uint32_t c0, int colour, int kind, int lattice_id, uint32_t c2, uint32_t c3, int u24,
                     double *X, double *margin)
{
    uint32_t w[4] = {0, 0, 0, 0};
    double mg = INFINITY, x;
    int got = 0;
    if (k == 0.0) {
        uint32_t ctr[4] = {c0, ctr1_word(0, colour, kind, lattice_id), c2, c3};
        or_philox(ctr, key, w);
        x = OR_PI * uni_signed(w[0], u24);
        got = ok(x, okc, &mg);
    } else {
        bf_t b;
        bf_setup(k, &b);
        for (int j = 0; j < VM_CAP && !got; ++j) {
            if ((j & 1) == 0) {
                uint32_t ctr[4] = {c0, ctr1_word(j >> 1, colour, kind, lattice_id), c2, c3};
                or_philox(ctr, key, w);
            }
            if (bf_attempt(&b, w[2 * (j & 1)], w[2 * (j & 1) + 1], u24, &x, &mg)) got = ok(x, okc, &mg);
        }
    }
    if (got) {
        *X = x;
        *margin = mg;
        return 1;
    }
    double xa = acos(u_hi), xb = acos(u_lo), W = xb - xa;
    if (W > 0.0) {
        double lam = k * fmin(sin(xa), (u_hi - u_lo) / W);
        for (int i = 0; i < LINK_B_CAP; ++i) {
            uint32_t ctr[4] = {c0, ctr1_word(LINK_B_BASE + i, colour, kind, lattice_id), c2, c3};
            or_philox(ctr, key, w);
            double V = uni01(w[0], u24), U = uni01(w[1], u24);
            double T = lam * W < LINK_TINY ? V * W : -log1p(V * expm1(-lam * W)) / lam;
            double xx = fmin(xa + T, xb);
            double lhs = log(U), rhs = k * (cos(xx) - u_hi) + lam * T;
            if (fabs(lhs - rhs) < mg) mg = fabs(lhs - rhs);
            if (lhs <= rhs) {
                x = (w[2] >> 31) ? -xx : xx;
                if (ok(x, okc, &mg)) {
                    *X = x;
                    *margin = mg;
                    return 2;
                }
            }
        }
    }
    *margin = mg;
    return 0;
}

/* window test on cos X itself (the sampler's own test entry) */
static int cos_window(double X, void *ctx, double *mg)
{
    const double *u = (const double *)ctx;
    double c = cos(X);
    double m = fmin(fabs(c - u[0]), fabs(u[1] - c));
    if (m < *mg) *mg = m;
    return c >= u[0] && c <= u[1];
}

/* Test entry: n draws of the restricted sampler with counters (i, colour 0,
 * kind 0, lattice 0, c2, c3); how[i] = stage (1, 2) or 0. */
void or_link_draw_batch(long n, double kappa, double u_lo, double u_hi, uint64_t seed, uint32_t c2,
                        uint32_t c3, int u24, double *X, int *how)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double u[2] = {u_lo, u_hi};
    for (long i = 0; i < n; ++i) {
        double x = NAN, m;
        int h = link_draw(kappa, u_lo, u_hi, cos_window, u, key, (uint32_t)i, 0, 0, 0, c2, c3, u24, &x, &m);
        X[i] = h ? x : NAN;
        how[i] = h;
    }
}

/* Test entry: n draws with counters (ctr0 = i, ctr1 = c1base, ctr2, ctr3). */
void or_vonmises_batch(long n, double kappa, uint64_t seed, uint32_t c1base, uint32_t c2,
                       uint32_t c3, int u24, double *X, int *attempts, double *margin)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (long i = 0; i < n; ++i) {
        double x = 0.0, m = 0.0;
        int a = vm_draw(kappa, key, (uint32_t)i, c1base, c2, c3, u24, &x, &m);
        X[i] = a ? x : NAN;
        if (attempts) attempts[i] = a;
        if (margin) margin[i] = m;
    }
}

/* ------------------------------------------------------------------------ */
/* Hot start: theta = -pi + 2 pi U, Philox kind INIT, ctr0 = mu*V + s,       */
/* ctr3 = chain index.  f32 != 0 stores the single-precision rounding.       */
/* ------------------------------------------------------------------------ */
void or_hot_start(int d, int L, int n_chains, uint64_t seed, int lattice_id, int f32, double *theta)
{
    long V = 1;
    for (int m = 0; m < d; ++m) V *= L;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int ch = 0; ch < n_chains; ++ch)
        for (long l = 0; l < d * V; ++l) {
            uint32_t ctr[4] = {(uint32_t)l, ctr1_word(0, 0, KIND_INIT, lattice_id), 0u, (uint32_t)ch};
            uint32_t w[4];
            or_philox(ctr, key, w);
            double t = fma(OR_TWO_PI, uni01(w[0], f32), -OR_PI);
            if (f32) t = (double)(float)t;
            theta[(long)ch * d * V + l] = t;
        }
}

/* ------------------------------------------------------------------------ */
/* One class pass on one chain.                                              */
/*   colour c = 2 mu + p: all links (mu, s) with parity(s) == p; no two of   */
/*   them share a plaquette, so their conditionals factorise.                */
/*   hb != 0: heatbath; each link drawn from its exact conditional at        */
/*            coupling a (weight exp(a * local action)).                      */
/*   hb == 0: overrelaxation theta -> -2 phi - theta, which leaves every      */
/*            local action R cos(theta + phi) unchanged; the class move is    */
/*            taken with Delta E = 0 (always accepted).                       */
/*   mode 0: restricted: accept the whole class iff lo <= E + dE <= hi        */
/*           (closed interval, Sec. 2.2 indicator).                          */
/*   mode 1: approach: accept iff dist(E + dE) <= dist(E), dist = distance    */
/*           to [lo, hi].                                                    */
/*   mode 2: unrestricted (canonical heatbath, used by physics pins).         */
/*   mode 3: multicanonical (Sec. 2.6): target weight W(E) = 1/rho~(E) set by */
/*           or_set_muca; the heatbath proposal at coupling a has a           */
/*           normalisation that depends only on the other classes, so the     */
/*           class is accepted with probability min(1, W(E+dE)/W(E) e^{-a dE}) */
/*           against the uniform of Philox counter (interval, kind 6, sweep). */
/*   mode 4: restricted with the constraint imposed per link when the new    */
/*           angle is drawn (Sec. 2.4): see link_pass; the class is always   */
/*           accepted.                                                       */
/* Links are visited in ascending half index h = s >> 1 and Delta E is       */
/* summed sequentially in that order.                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t key[2];
    int kind;          /* KIND_SWEEP or KIND_APPROACH */
    int lattice_id;
    uint32_t sweep;    /* counter word 2 */
    uint32_t interval; /* counter word 3 */
    int f32;           /* single-precision state: 24-bit uniforms, stored angles rounded */
} pass_ctx_t;

/* Multicanonical weight: ln W(E) = -ln rho~(E), ln rho~ continuous with slope
 * -a_k on [c_k - s/2, c_k + s/2] (ln rho~(c_0) = 0, eq. (kk3a) recursion);
 * below the first and above the last interval the first and last pieces
 * continue (eq. (4.1) with beta_1 = a_0, beta_2 = a_{n-1}). */
static struct {
    int n;
    double s;
    double *c, *a, *lr;
} g_muca = {0, 0.0, NULL, NULL, NULL};

void or_set_muca(const double *centres, const double *a, int n, double s)
{
    free(g_muca.c);
    free(g_muca.a);
    free(g_muca.lr);
    g_muca.n = n;
    g_muca.s = s;
    g_muca.c = (double *)malloc(sizeof(double) * n);
    g_muca.a = (double *)malloc(sizeof(double) * n);
    g_muca.lr = (double *)malloc(sizeof(double) * n);
    memcpy(g_muca.c, centres, sizeof(double) * n);
    memcpy(g_muca.a, a, sizeof(double) * n);
    g_muca.lr[0] = 0.0;
    for (int k = 0; k + 1 < n; ++k) g_muca.lr[k + 1] = g_muca.lr[k] - 0.5 * s * (a[k] + a[k + 1]);
}

double or_muca_lnw(double E)
{
    int n = g_muca.n;
    double lo = g_muca.c[0] - 0.5 * g_muca.s;
    int k = (int)floor((E - lo) / g_muca.s);
    if (k < 0) k = 0;
    if (k > n - 1) k = n - 1;
    return -(g_muca.lr[k] - g_muca.a[k] * (E - g_muca.c[k]));
}

/* Window test of a class link under the per-link constraint: the candidate
 * angle is stored (rounded to single precision for an FP32 state) and the
 * energy change is taken from the stored angle, so the running energy stays
 * inside [lo, hi] in the arithmetic that carries it. */
typedef struct {
    double C, S, phi, eps_old, E, lo, hi;
    int flip, f32;
    double t, dE; /* out: the last candidate tested */
} link_win_t;

static int link_window(double X, void *ctx, double *mg)
{
    link_win_t *w = (link_win_t *)ctx;
    double t = wrap(X - w->phi + (w->flip ? OR_PI : 0.0));
    if (w->f32) t = (double)(float)t;
    double dE = eps_local(w->C, w->S, t) - w->eps_old;
    double En = w->E + dE;
    double m = fmin(fabs(En - w->lo), fabs(w->hi - En));
    if (m < *mg) *mg = m;
    w->t = t;
    w->dE = dE;
    return En >= w->lo && En <= w->hi;
}

/* Heatbath pass of one colour under the per-link constraint (mode 4): the
 * class links are updated one after another in site order, each from its
 * conditional restricted to the values that keep the running energy E in
 * [lo, hi], and E is carried from link to link.  Links of one class share no
 * plaquette, so the staples do not depend on the order; only E does.  The
 * pass is always accepted.  how_out (optional) receives the stage per link. */
static void link_pass(const geo_t *g, double *th, int colour, double a, double lo, double hi, double *E,
                      const pass_ctx_t *pc, double *margin_out, int *how_out)
{
    long V = g->V;
    int mu = colour >> 1, p = colour & 1;
    long nl = 0;
    for (long s = 0; s < V; ++s) {
        if (g->par[s] != p) continue;
        double t_old = th[mu * V + s];
        double C, S;
        local_field(g, th, mu, s, &C, &S);
        double R = hypot(C, S);
        double kappa = a * R;
        link_win_t w = {C, S, atan2(S, C), eps_local(C, S, t_old), *E, lo, hi, kappa < 0.0, pc->f32, 0.0, 0.0};
        /* window on the link's new local action sg R cos X, sg = sign(kappa) */
        double A = lo - (*E - w.eps_old), B = hi - (*E - w.eps_old);
        double u_lo = -1.0, u_hi = 1.0;
        if (R > 0.0) {
            u_lo = kappa < 0.0 ? -B / R : A / R;
            u_hi = kappa < 0.0 ? -A / R : B / R;
            u_lo = fmin(1.0, fmax(-1.0, u_lo));
            u_hi = fmin(1.0, fmax(-1.0, u_hi));
        }
        double X, mg;
        int how = link_draw(fabs(kappa), u_lo, u_hi, link_window, &w, pc->key, (uint32_t)(s >> 1), colour,
                            pc->kind, pc->lattice_id, pc->sweep, pc->interval, pc->f32, &X, &mg);
        if (R < 1e-4) mg = 0.0; /* ill-conditioned phase: flagged */
        if (how) {
            th[mu * V + s] = w.t;
            *E += w.dE;
        }
        if (margin_out) margin_out[nl] = mg;
        if (how_out) how_out[nl] = how;
        ++nl;
    }
}

static int class_pass(const geo_t *g, double *th, double *scratch, int hb, int colour,
                      int mode, double a, double lo, double hi, double *E,
                      const pass_ctx_t *pc, double *margin_out, double *dE_out)
{
    if (hb && mode == 4) {
        double E0 = *E;
        link_pass(g, th, colour, a, lo, hi, E, pc, margin_out, NULL);
        if (dE_out) *dE_out = *E - E0;
        return 1;
    }
    long V = g->V;
    int d = g->d;
    int mu = colour >> 1, p = colour & 1;
    double dE = 0.0;
    long nl = 0;
    for (long s = 0; s < V; ++s) {
        if (g->par[s] != p) continue;
        double t_old = th[mu * V + s];
        double C, S;
        local_field(g, th, mu, s, &C, &S);
        double phi = atan2(S, C);
        double t_new;
        double mg = INFINITY;
        if (hb) {
            double R = hypot(C, S);
            double kappa = a * R;
            double X;
            uint32_t c1 = ctr1_word(0, colour, pc->kind, pc->lattice_id);
            int n = vm_draw(fabs(kappa), pc->key, (uint32_t)(s >> 1), c1, pc->sweep, pc->interval,
                            pc->f32, &X, &mg);
            if (R < 1e-4) mg = 0.0; /* ill-conditioned phase: flagged */
            if (n == 0) t_new = t_old;
            else t_new = wrap(X - phi + (kappa < 0.0 ? OR_PI : 0.0));
        } else {
            t_new = wrap(-2.0 * phi - t_old);
        }
        if (pc->f32) t_new = (double)(float)t_new;
        if (hb) dE += eps_local(C, S, t_new) - eps_local(C, S, t_old);
        scratch[nl] = t_new;
        if (margin_out) margin_out[nl] = mg;
        ++nl;
    }
    int accept;
    double En = *E + dE;
    if (!hb) accept = 1;
    else if (mode == 0) accept = (En >= lo && En <= hi);
    else if (mode == 1) {
        double d0 = fmax(0.0, fmax(lo - *E, *E - hi));
        double d1 = fmax(0.0, fmax(lo - En, En - hi));
        accept = (d1 <= d0);
    } else if (mode == 3) {
        double lr = or_muca_lnw(En) - or_muca_lnw(*E) - a * dE;
        uint32_t ctr[4] = {pc->interval, ctr1_word(0, colour, KIND_MUCA, pc->lattice_id), pc->sweep, 0u};
        uint32_t w[4];
        or_philox(ctr, pc->key, w);
        accept = lr >= 0.0 || ((double)w[0] + 0.5) * 0x1p-32 < exp(lr);
    } else accept = 1;
    if (dE_out) *dE_out = dE;
    if (accept) {
        nl = 0;
        for (long s = 0; s < V; ++s) {
            if (g->par[s] != p) continue;
            th[mu * V + s] = scratch[nl++];
        }
        if (hb) *E = En;
    }
    return accept;
}

/* Exported single pass for the one-sweep parity tests.  theta is one chain in
 * canonical layout; E is in/out; margin (optional, V/2 entries) receives the
 * smallest sampler-test margin per class link (0 if R < 1e-4). */
int or_class_pass(int d, int L, double *theta, int hb, int colour, int mode, double a,
                  double lo, double hi, double *E, uint64_t seed, int kind, int lattice_id,
                  uint32_t sweep, uint32_t interval, int f32, double *margin, double *dE_out)
{
    geo_t g;
    if (geo_init(&g, d, L)) return -1;
    double *scr = (double *)malloc(sizeof(double) * (g.V / 2 + 1));
    pass_ctx_t pc = {{(uint32_t)seed, (uint32_t)(seed >> 32)}, kind, lattice_id, sweep, interval, f32};
    int acc = class_pass(&g, theta, scr, hb, colour, mode, a, lo, hi, E, &pc, margin, dE_out);
    free(scr);
    geo_free(&g);
    return acc;
}

/* Exported single pass under the per-link constraint (mode 4), with the
 * decision margin and the sampler stage of every class link. */
void or_link_pass(int d, int L, double *theta, int colour, double a, double lo, double hi, double *E,
                  uint64_t seed, int kind, int lattice_id, uint32_t sweep, uint32_t interval, int f32,
                  double *margin, int *how)
{
    geo_t g;
    if (geo_init(&g, d, L)) return;
    pass_ctx_t pc = {{(uint32_t)seed, (uint32_t)(seed >> 32)}, kind, lattice_id, sweep, interval, f32};
    link_pass(&g, theta, colour, a, lo, hi, E, &pc, margin, how);
    geo_free(&g);
}

/* One restricted sweep of one chain.  do_or 0: heatbath over all 2d colours;
 * 1: then overrelaxation over all 2d colours (grouped order); 2: heatbath and
 * overrelaxation of colour 0, then of colour 1, ... (interleaved order);
 * 3: overrelaxation over all 2d colours, then heatbath over all 2d colours
 * (the staggered order's second chain set: the grouped order's passes
 * continued half a sweep later, so that the sweep ends right after the
 * heatbath half, as the grouped sweep's overrelaxation leaves E unchanged).
 * Algorithm 1 asks only for one sweep of the whole system.  In the
 * interleaved order the overrelaxation of colour c reflects, on unchanged
 * staples, the heatbath draw just made: -2 phi - (X - phi) = -X - phi, again
 * a von Mises draw, so an accepted heatbath class followed by its
 * overrelaxation is one update of those links, not two.  bits receives the
 * accept bit of each pass (bit c: heatbath colour c, bit 2d + c:
 * overrelaxation colour c). */
static int sweep_chain(const geo_t *g, double *th, double *scr, int mode, double a, double lo,
                       double hi, double *E, const pass_ctx_t *pc, int do_or)
{
    int bits = 0;
    int nc = 2 * g->d;
    if ((do_or == 2 || do_or == 3) && (mode == 1 || mode == 4)) do_or = 1;   /* approach and per-link sweeps stay grouped */
    if (do_or == 3)
        for (int c = 0; c < nc; ++c)
            if (class_pass(g, th, scr, 0, c, mode, a, lo, hi, E, pc, NULL, NULL)) bits |= 1 << (nc + c);
    for (int c = 0; c < nc; ++c) {
        if (class_pass(g, th, scr, 1, c, mode, a, lo, hi, E, pc, NULL, NULL)) bits |= 1 << c;
        if (do_or == 2 && class_pass(g, th, scr, 0, c, mode, a, lo, hi, E, pc, NULL, NULL))
            bits |= 1 << (nc + c);
    }
    if (do_or == 1)
        for (int c = 0; c < nc; ++c)
            if (class_pass(g, th, scr, 0, c, mode, a, lo, hi, E, pc, NULL, NULL)) bits |= 1 << (nc + c);
    return bits;
}

/* Exported: n_sweeps sweeps on n_chains independent chains (chain ch uses
 * coupling a[ch], interval [lo[ch], hi[ch]], counter word 3 = interval[ch]).
 * mode as in class_pass.  Sweep indices run sweep0, sweep0+1, ...  E is
 * in/out per chain.  bits (optional) is n_sweeps x n_chains.  do_or_ch
 * (optional): per chain, the do_or of sweep_chain, in place of do_or. */
void or_sweeps(int d, int L, int n_chains, double *theta, const double *a, const double *lo,
               const double *hi, const int *interval, double *E, int n_sweeps, uint32_t sweep0,
               int mode, int kind, int do_or, uint64_t seed, int lattice_id, int f32, int *bits,
               const int *do_or_ch)
{
    geo_t g;
    if (geo_init(&g, d, L)) return;
    long nl = (long)d * g.V;
#pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < n_chains; ++ch) {
        double *scr = (double *)malloc(sizeof(double) * (g.V / 2 + 1));
        for (int t = 0; t < n_sweeps; ++t) {
            pass_ctx_t pc = {{(uint32_t)seed, (uint32_t)(seed >> 32)}, kind, lattice_id,
                             sweep0 + (uint32_t)t, (uint32_t)interval[ch], f32};
            int b = sweep_chain(&g, theta + ch * nl, scr, mode, a[ch], lo[ch], hi[ch], &E[ch], &pc,
                                do_or_ch ? do_or_ch[ch] : do_or);
            if (bits) bits[(long)t * n_chains + ch] = b;
        }
        free(scr);
    }
    geo_free(&g);
}

/* ------------------------------------------------------------------------ */
/* The LLR driver, Algorithm 1, with every interval of one lattice as an     */
/* independent chain.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d, L, n;          /* dimension, lattice size, number of intervals */
    int n_th, n_a, n_rm;  /* thermalisation / measured sweeps per RM iteration / RM iterations */
    int recompute_every;  /* K: full recompute of E after every K-th sweep of an iteration */
    int approach_cap;     /* maximum approach sweeps */
    int replica_exchange; /* 0/1 */
    int f32;              /* single-precision state */
    int lattice_id;
    int hot_start;        /* 1: hot start from seed; 0: theta is given */
    uint64_t seed;
    double dE;            /* centre spacing */
    double w;             /* restriction width */
    double eps;           /* convergence threshold on |a^(n+1) - a^(n)| */
    int link;             /* 1: restriction imposed per link (Sec. 2.4), 0: class-wise rejection */
    int interleave;       /* sweep order: 0 grouped, 1 interleaved, 2 staggered (chains from
                             ceil(n/2) on take their overrelaxation passes first) */
} or_run_params;

typedef struct {
    double *a;              /* in: a^(0) per interval; out: final a */
    double *a_hist;         /* (n_rm + 1) x n, optional */
    double *theta;          /* n x d V, in/out */
    double *E;              /* per chain, out */
    int *conf;              /* conf[k] = chain in interval k, out */
    int *conv_iter;         /* first n with |da| < eps, or -1 */
    long long *conv_sweeps; /* approach + (n+1)(n_th+n_a), or -1 */
    long long *approach_sweeps; /* out, scalar */
    uint16_t *bits;         /* optional: (approach + n_rm (n_th + n_a)) x n accept bits */
    double *sumE_hist;      /* optional: n_rm x n measured means */
    long long *re_acc;      /* optional: replica exchange [proposed, accepted] */
} or_run_out;

/* Replica exchange after sweep t (Sec. 2.5): the pairs of neighbouring
 * intervals (k, k+1) with k = t (mod 2).  A pair is eligible when each
 * configuration lies inside the other's interval, so that the swapped state
 * has non-zero restricted weight.  In the beta-convention the joint weight of
 * the chains is prod_k rho(E_k) exp(a_k E_k) 1[E_k in I_k]; exchanging the
 * configurations of intervals k and k+1 multiplies it by
 * exp[(a_k - a_{k+1}) (E_{k+1} - E_k)] (the paper prints the exponent for its
 * exp(-aS) weights), which is the Metropolis ratio of the swap.  The
 * configurations stay where they are: conf (interval -> chain) and itv
 * (chain -> interval) are exchanged.  Uniform: first word of Philox at
 * counter (k, kind 3 << 12 | lattice << 16, t, 0).
 *
 * OR_PLANT_RE_SIGN (test builds only) plants the mistake of taking the
 * printed exponent literally in this convention, exp[(a_k - a_{k+1})(E_k -
 * E_{k+1})]; the replica-exchange pin must detect it. */
static void replica_step(int n, int *conf, int *itv, const double *E, const double *a, const double *lo,
                         const double *hi, const uint32_t key[2], int lattice_id, uint32_t t,
                         long long *re_acc)
{
    for (int k = (int)(t & 1u); k + 1 < n; k += 2) {
        int A = conf[k], B = conf[k + 1];
        double EA = E[A], EB = E[B];
        if (!(EA >= lo[k + 1] && EA <= hi[k + 1] && EB >= lo[k] && EB <= hi[k])) continue;
        uint32_t ctr[4] = {(uint32_t)k, ctr1_word(0, 0, KIND_REPLICA, lattice_id), t, 0u};
        uint32_t w[4];
        or_philox(ctr, key, w);
        double u = uni01(w[0], 0);
#ifdef OR_PLANT_RE_SIGN
        double x = (a[k] - a[k + 1]) * (EA - EB);
#else
        double x = (a[k] - a[k + 1]) * (EB - EA);
#endif
        if (re_acc) re_acc[0]++;
        if (x >= 0.0 || u < exp(x)) {
            conf[k] = B; conf[k + 1] = A;
            itv[A] = k + 1; itv[B] = k;
            if (re_acc) re_acc[1]++;
        }
    }
}

/* Exported replica-exchange step for the pins: n intervals with coupling
 * a[k] and restriction [lo[k], hi[k]]; conf/itv/E per interval and chain as
 * in the driver; re_acc (optional) accumulates [proposed, accepted]. */
void or_replica_step(int n, int *conf, int *itv, const double *E, const double *a, const double *lo,
                     const double *hi, uint64_t seed, int lattice_id, uint32_t t, long long *re_acc)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    replica_step(n, conf, itv, E, a, lo, hi, key, lattice_id, t, re_acc);
}

/* Exported for the replica-exchange pins: n chains at fixed couplings, one
 * per interval, n_sweeps times a restricted sweep of every chain (at the
 * coupling, restriction and counter word 3 of the interval it serves; sweep
 * index sweep0 + t) followed by replica_step.  E, conf, itv in/out; E_vis
 * (optional, n_sweeps x n) receives the energy of the chain serving each
 * interval after the exchange.  Chains run one after another (tiny lattices). */
void or_replica_run(int d, int L, int n, double *theta, const double *a, const double *lo, const double *hi,
                    double *E, int *conf, int *itv, int n_sweeps, uint32_t sweep0, uint64_t seed,
                    int lattice_id, int order, double *E_vis, long long *re_acc)
{
    geo_t g;
    if (geo_init(&g, d, L)) return;
    long nl = (long)d * g.V;
    double *scr = (double *)malloc(sizeof(double) * (g.V / 2 + 1));
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int t = 0; t < n_sweeps; ++t) {
        uint32_t sw = sweep0 + (uint32_t)t;
        for (int c = 0; c < n; ++c) {
            int k = itv[c];
            pass_ctx_t pc = {{key[0], key[1]}, KIND_SWEEP, lattice_id, sw, (uint32_t)k, 0};
            sweep_chain(&g, theta + c * nl, scr, 0, a[k], lo[k], hi[k], &E[c], &pc, order == 1 ? 2 : 1);
        }
        replica_step(n, conf, itv, E, a, lo, hi, key, lattice_id, sw, re_acc);
        if (E_vis)
            for (int k = 0; k < n; ++k) E_vis[(long)t * n + k] = E[conf[k]];
    }
    free(scr);
    geo_free(&g);
}

/* Robbins-Monro step, eq. (kk21) with Algorithm 1's sign (beta-convention):
 * a^(n+1) = a^(n) - 12 (mean - centre) / ((n + 1) w^2), n = 0, 1, ... */
double or_rm_step(double a, double mean, double centre, int n, double w)
{
    return a - 12.0 * (mean - centre) / ((double)(n + 1) * w * w);
}

static int all_inside(int n, const double *E, const int *itv, const double *lo, const double *hi)
{
    for (int c = 0; c < n; ++c)
        if (!(E[c] >= lo[itv[c]] && E[c] <= hi[itv[c]])) return 0;
    return 1;
}

int or_llr_run(const or_run_params *p, const double *E_low, or_run_out *o)
{
    geo_t g;
    if (geo_init(&g, p->d, p->L)) return -2;
    int n = p->n;
    long nl = (long)p->d * g.V;
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    double *cen = (double *)malloc(sizeof(double) * n);
    double *lo = (double *)malloc(sizeof(double) * n);
    double *hi = (double *)malloc(sizeof(double) * n);
    double *b = (double *)malloc(sizeof(double) * n);
    double *sumE = (double *)malloc(sizeof(double) * n);
    int *itv = (int *)malloc(sizeof(int) * n);
    int *conf = o->conf;
    int nc = 2 * p->d;
    for (int k = 0; k < n; ++k) {
        cen[k] = E_low[k] + 0.5 * p->dE;
        lo[k] = cen[k] - 0.5 * p->w;
        hi[k] = cen[k] + 0.5 * p->w;
        itv[k] = k;
        conf[k] = k;
        b[k] = o->a[k];
    }
    if (p->hot_start) or_hot_start(p->d, p->L, n, p->seed, p->lattice_id, p->f32, o->theta);
    for (int c = 0; c < n; ++c) o->E[c] = energy(&g, o->theta + c * nl);
    if (o->a_hist) for (int k = 0; k < n; ++k) o->a_hist[k] = o->a[k];

    /* Approach (the paper is silent on how a hot start enters its interval):
     * heatbath passes only, each colour class c at its own coupling b_c
     * (initially a^(0)).  A class move is accepted iff it does not increase
     * the distance of E to the interval.  After every pass of colour c, b_c
     * moves by eta_c * sign(c_k - E_new), where E_new is the proposal's energy
     * (accepted or not); eta_c halves when that sign flips and grows by 1.2
     * while it repeats (within [1e-6, 0.05]): a sign-based root search for the
     * coupling whose proposals of that class land at the centre.  One coupling
     * per class is needed because far from equilibrium the classes' own
     * energies differ by more than a proposal's spread.  Sweeps run in blocks
     * of K followed by a full recompute of E; the phase ends once every chain
     * is inside. */
    long long t_ap = 0;
    long long bitrow = 0;
    int inside = all_inside(n, o->E, itv, lo, hi);
    int K = p->recompute_every > 0 ? p->recompute_every : 1;
    double *bc = (double *)malloc(sizeof(double) * n * 8);
    double *eta = (double *)malloc(sizeof(double) * n * 8);
    int *sprev = (int *)malloc(sizeof(int) * n * 8);
    for (int c = 0; c < n; ++c)
        for (int col = 0; col < 8; ++col) { bc[c * 8 + col] = b[c]; eta[c * 8 + col] = 0.05; sprev[c * 8 + col] = 0; }
    while (!inside) {
        if (t_ap >= p->approach_cap) {
            free(cen); free(lo); free(hi); free(b); free(sumE); free(itv); free(eta); free(sprev); free(bc);
            geo_free(&g);
            *o->approach_sweeps = t_ap;
            return -5;
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int c = 0; c < n; ++c) {
            double *scr = (double *)malloc(sizeof(double) * (g.V / 2 + 1));
            int k = itv[c];
            for (int t = 0; t < K; ++t) {
                pass_ctx_t pc = {{key[0], key[1]}, KIND_APPROACH, p->lattice_id,
                                 (uint32_t)(t_ap + t), (uint32_t)k, p->f32};
                int bits = 0;
                for (int col = 0; col < nc; ++col) {
                    const int q = c * 8 + col;
                    double dE = 0.0;
                    double E0 = o->E[c];
                    if (class_pass(&g, o->theta + c * nl, scr, 1, col, 1, bc[q], lo[k], hi[k],
                                   &o->E[c], &pc, NULL, &dE))
                        bits |= 1 << col;
                    double En = E0 + dE;
                    int sg = (cen[k] > En) ? 1 : (cen[k] < En ? -1 : 0);
                    if (sprev[q] != 0 && sg != 0)
                        eta[q] = (sg == sprev[q]) ? fmin(0.05, 1.2 * eta[q]) : fmax(1e-6, 0.5 * eta[q]);
                    bc[q] = fmin(4.0, fmax(0.0, bc[q] + eta[q] * (double)sg));
                    sprev[q] = sg;
                }
                if (o->bits) o->bits[(bitrow + t) * n + c] = (uint16_t)bits;
            }
            o->E[c] = energy(&g, o->theta + c * nl);
            free(scr);
        }
        t_ap += K;
        bitrow += K;
        inside = all_inside(n, o->E, itv, lo, hi);
    }
    free(bc);
    free(eta); free(sprev);
    *o->approach_sweeps = t_ap;

    for (int k = 0; k < n; ++k) { o->conv_iter[k] = -1; o->conv_sweeps[k] = -1; }
    int nsw = p->n_th + p->n_a;
    uint32_t t_glob = 0;
    if (o->re_acc) { o->re_acc[0] = 0; o->re_acc[1] = 0; }
    for (int it = 0; it < p->n_rm; ++it) {
        for (int k = 0; k < n; ++k) sumE[k] = 0.0;
        for (int j = 0; j < nsw; ++j, ++t_glob) {
            int recompute = ((j + 1) % K == 0) || (j == nsw - 1);
#pragma omp parallel for schedule(dynamic, 1)
            for (int c = 0; c < n; ++c) {
                double *scr = (double *)malloc(sizeof(double) * (g.V / 2 + 1));
                int k = itv[c];
                pass_ctx_t pc = {{key[0], key[1]}, KIND_SWEEP, p->lattice_id, t_glob, (uint32_t)k, p->f32};
                int dor = 1;
                if (!p->link && p->interleave == 1) dor = 2;
                if (!p->link && p->interleave == 2 && c >= (n + 1) / 2) dor = 3;
                int bits = sweep_chain(&g, o->theta + c * nl, scr, p->link ? 4 : 0, o->a[k], lo[k], hi[k],
                                       &o->E[c], &pc, dor);
                if (o->bits) o->bits[(bitrow + (long long)it * nsw + j) * n + c] = (uint16_t)bits;
                if (recompute) o->E[c] = energy(&g, o->theta + c * nl);
                free(scr);
            }
            if (p->replica_exchange)
                replica_step(n, conf, itv, o->E, o->a, lo, hi, key, p->lattice_id, t_glob, o->re_acc);
            if (j >= p->n_th)
                for (int k = 0; k < n; ++k) sumE[k] += o->E[conf[k]];
        }
        for (int k = 0; k < n; ++k) {
            double mean = sumE[k] / (double)p->n_a;
            if (o->sumE_hist) o->sumE_hist[(long)it * n + k] = mean;
            double an = or_rm_step(o->a[k], mean, cen[k], it, p->w);
            double da = an - o->a[k];
            o->a[k] = an;
            if (o->conv_iter[k] < 0 && fabs(da) < p->eps) {
                o->conv_iter[k] = it;
                o->conv_sweeps[k] = t_ap + (long long)(it + 1) * nsw;
            }
            if (o->a_hist) o->a_hist[(long)(it + 1) * n + k] = o->a[k];
        }
    }
    free(cen); free(lo); free(hi); free(b); free(sumE); free(itv);
    geo_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction (FP64).  ln rho at the centres by the trapezium recursion  */
/* eq. (kk3a) in the beta-convention: L_{k+1} = L_k - (s/2)(a_k + a_{k+1}).   */
/* Canonical averages by the midpoint sums eqs. (l19)-(l20):                 */
/*   p_k(beta) ~ exp(L_k + beta c_k),  <E> = sum p_k c_k,                     */
/*   Var(E) = sum p_k (c_k - <E>)^2;  <u> = <E>/(6V), C_V = Var(E)/(6V).      */
/* ------------------------------------------------------------------------ */
void or_ln_rho(const double *a, int n, double s, double *lnrho)
{
    lnrho[0] = 0.0;
    for (int k = 0; k + 1 < n; ++k) lnrho[k + 1] = lnrho[k] - 0.5 * s * (a[k] + a[k + 1]);
}

static void moments_at(const double *c, const double *L, int n, double beta, double *mean, double *var)
{
    double m = -INFINITY;
    for (int k = 0; k < n; ++k) m = fmax(m, L[k] + beta * c[k]);
    double Z = 0.0, s1 = 0.0;
    for (int k = 0; k < n; ++k) {
        double wk = exp(L[k] + beta * c[k] - m);
        Z += wk;
        s1 += wk * c[k];
    }
    double mu = s1 / Z;
    double s2 = 0.0;
    for (int k = 0; k < n; ++k) {
        double wk = exp(L[k] + beta * c[k] - m);
        s2 += wk * (c[k] - mu) * (c[k] - mu);
    }
    *mean = mu;
    *var = s2 / Z;
}

void or_reconstruct(const double *centres, const double *a, int n, double s, double six_v,
                    const double *beta, int nb, double *lnrho, double *u_mean, double *cv)
{
    or_ln_rho(a, n, s, lnrho);
    for (int i = 0; i < nb; ++i) {
        double mu, var;
        moments_at(centres, lnrho, n, beta[i], &mu, &var);
        u_mean[i] = mu / six_v;
        cv[i] = var / six_v;
    }
}

/* beta_c = argmax C_V on [blo, bhi]: grid of step h, then golden section on
 * [b* - h, b* + h] until the bracket is shorter than tol. */
void or_beta_c(const double *centres, const double *a, int n, double s, double six_v,
               double blo, double bhi, double h, double tol, double *beta_c, double *cv_peak)
{
    double *L = (double *)malloc(sizeof(double) * n);
    or_ln_rho(a, n, s, L);
    long ng = (long)floor((bhi - blo) / h + 0.5);
    double best = -INFINITY, bb = blo;
    for (long i = 0; i <= ng; ++i) {
        double b = blo + (double)i * h, mu, var;
        moments_at(centres, L, n, b, &mu, &var);
        if (var > best) { best = var; bb = b; }
    }
    double x0 = fmax(blo, bb - h), x3 = fmin(bhi, bb + h);
    const double gr = 0.61803398874989484820;
    double x1 = x3 - gr * (x3 - x0), x2 = x0 + gr * (x3 - x0), mu, f1, f2;
    moments_at(centres, L, n, x1, &mu, &f1);
    moments_at(centres, L, n, x2, &mu, &f2);
    while (x3 - x0 > tol) {
        if (f1 > f2) {
            x3 = x2; x2 = x1; f2 = f1;
            x1 = x3 - gr * (x3 - x0);
            moments_at(centres, L, n, x1, &mu, &f1);
        } else {
            x0 = x1; x1 = x2; f1 = f2;
            x2 = x0 + gr * (x3 - x0);
            moments_at(centres, L, n, x2, &mu, &f2);
        }
    }
    double bc = 0.5 * (x0 + x3), var;
    moments_at(centres, L, n, bc, &mu, &var);
    if (best > var) { bc = bb; var = best; }
    *beta_c = bc;
    *cv_peak = var / six_v;
    free(L);
}

/* ------------------------------------------------------------------------ */
/* Warm-start network a(u, 1/L): 2 -> 64 (tanh) -> 64 (tanh) -> 1, FP64.      */
/* Parameter vector (4417): W1[64][2], b1[64], W2[64][64], b2[64], W3[64],    */
/* b3.  Inputs normalised: uh = (u - 0.6)/0.1, lh = (1/L - 0.0875)/0.0375;    */
/* output a = 1 + 0.1 y.  Loss: mean squared error on a.  Adam.               */
/* ------------------------------------------------------------------------ */
#define MLP_H 64
#define MLP_NP (MLP_H * 2 + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * 2)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)

int or_mlp_nparams(void) { return MLP_NP; }

void or_mlp_init(uint64_t seed, double *w)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int i = 0; i < MLP_NP; ++i) {
        double lim = 0.0;
        if (i < OFF_B1) lim = sqrt(6.0 / (2 + MLP_H));
        else if (i >= OFF_W2 && i < OFF_B2) lim = sqrt(6.0 / (MLP_H + MLP_H));
        else if (i >= OFF_W3 && i < OFF_B3) lim = sqrt(6.0 / (MLP_H + 1));
        if (lim == 0.0) { w[i] = 0.0; continue; }
        uint32_t ctr[4] = {(uint32_t)i, ctr1_word(0, 0, KIND_MLP, 0), 0u, 0u};
        uint32_t o[4];
        or_philox(ctr, key, o);
        w[i] = fma(2.0 * lim, uni01(o[0], 0), -lim);
    }
}

/* forward; h1, h2 (n x 64, optional) receive the post-tanh activations */
void or_mlp_forward(const double *w, const double *u, const double *invL, int n, double *a_out,
                    double *h1o, double *h2o)
{
    for (int i = 0; i < n; ++i) {
        double x0 = (u[i] - 0.6) / 0.1, x1 = (invL[i] - 0.0875) / 0.0375;
        double h1[MLP_H], h2[MLP_H];
        for (int j = 0; j < MLP_H; ++j)
            h1[j] = tanh(w[OFF_W1 + 2 * j] * x0 + w[OFF_W1 + 2 * j + 1] * x1 + w[OFF_B1 + j]);
        for (int j = 0; j < MLP_H; ++j) {
            double z = w[OFF_B2 + j];
            for (int k = 0; k < MLP_H; ++k) z += w[OFF_W2 + MLP_H * j + k] * h1[k];
            h2[j] = tanh(z);
        }
        double y = w[OFF_B3];
        for (int k = 0; k < MLP_H; ++k) y += w[OFF_W3 + k] * h2[k];
        a_out[i] = 1.0 + 0.1 * y;
        if (h1o) memcpy(h1o + (long)i * MLP_H, h1, sizeof(h1));
        if (h2o) memcpy(h2o + (long)i * MLP_H, h2, sizeof(h2));
    }
}

/* loss = (1/n) sum (a_pred - a)^2 and its gradient by the chain rule */
double or_mlp_loss_grad(const double *w, const double *u, const double *invL, const double *a,
                        int n, double *grad)
{
    memset(grad, 0, sizeof(double) * MLP_NP);
    double loss = 0.0;
    for (int i = 0; i < n; ++i) {
        double x0 = (u[i] - 0.6) / 0.1, x1 = (invL[i] - 0.0875) / 0.0375;
        double h1[MLP_H], h2[MLP_H], d2[MLP_H], d1[MLP_H];
        for (int j = 0; j < MLP_H; ++j)
            h1[j] = tanh(w[OFF_W1 + 2 * j] * x0 + w[OFF_W1 + 2 * j + 1] * x1 + w[OFF_B1 + j]);
        for (int j = 0; j < MLP_H; ++j) {
            double z = w[OFF_B2 + j];
            for (int k = 0; k < MLP_H; ++k) z += w[OFF_W2 + MLP_H * j + k] * h1[k];
            h2[j] = tanh(z);
        }
        double y = w[OFF_B3];
        for (int k = 0; k < MLP_H; ++k) y += w[OFF_W3 + k] * h2[k];
        double r = 1.0 + 0.1 * y - a[i];
        loss += r * r / n;
        double dy = 2.0 * r / n * 0.1;
        grad[OFF_B3] += dy;
        for (int k = 0; k < MLP_H; ++k) {
            grad[OFF_W3 + k] += dy * h2[k];
            d2[k] = dy * w[OFF_W3 + k] * (1.0 - h2[k] * h2[k]);
        }
        for (int j = 0; j < MLP_H; ++j) {
            grad[OFF_B2 + j] += d2[j];
            for (int k = 0; k < MLP_H; ++k) grad[OFF_W2 + MLP_H * j + k] += d2[j] * h1[k];
        }
        for (int k = 0; k < MLP_H; ++k) {
            double s = 0.0;
            for (int j = 0; j < MLP_H; ++j) s += w[OFF_W2 + MLP_H * j + k] * d2[j];
            d1[k] = s * (1.0 - h1[k] * h1[k]);
        }
        for (int j = 0; j < MLP_H; ++j) {
            grad[OFF_B1 + j] += d1[j];
            grad[OFF_W1 + 2 * j] += d1[j] * x0;
            grad[OFF_W1 + 2 * j + 1] += d1[j] * x1;
        }
    }
    return loss;
}

/* Adam (Kingma & Ba 2015) step t (1-based) */
void or_mlp_adam(double *w, double *m, double *v, const double *g, int t, double lr, double b1,
                 double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < MLP_NP; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* full-batch training; loss_hist (optional, epochs entries) */
void or_mlp_train(double *w, const double *u, const double *invL, const double *a, int n,
                  int epochs, double lr, double *loss_hist)
{
    double *m = (double *)calloc(MLP_NP, sizeof(double));
    double *v = (double *)calloc(MLP_NP, sizeof(double));
    double *g = (double *)malloc(sizeof(double) * MLP_NP);
    for (int e = 0; e < epochs; ++e) {
        double loss = or_mlp_loss_grad(w, u, invL, a, n, g);
        if (loss_hist) loss_hist[e] = loss;
        or_mlp_adam(w, m, v, g, e + 1, lr, 0.9, 0.999, 1e-8);
    }
    free(m); free(v); free(g);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
