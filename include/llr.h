/*
 * llr.h -- C ABI of the MI355X (gfx950) LLR library: energy-restricted
 * Monte-Carlo for 4D compact U(1) lattice gauge theory and the Robbins-Monro
 * determination of the density-of-states slopes a_k (Langfeld, Lucini,
 * Pellegrini, Rago, arXiv:1509.08391).
 *
 * What the calls compute, with the passage that defines it:
 *   - the model: links theta_mu(x) in [-pi, pi), action without the coupling
 *     E = sum_{x, mu<nu} cos theta_{mu nu}(x) (Sec. 3.1);
 *   - the interval set E_k = E_min + k dE and the closed restriction
 *     E_k <= E <= E_k + dE (Sec. 2.2, interval indicator; Algorithm 1);
 *   - the restricted, reweighted measure exp(+a E) 1[E in I_k] sampled by
 *     colour-class heatbath and overrelaxation moves (eqs. (kk7)-(kk9)); the
 *     sign convention makes a_k = -d ln rho/dE ~ beta > 0;
 *   - the Robbins-Monro update a <- a - 12 (<E> - c_k)/((n+1) w^2)
 *     (eq. (kk21), Algorithm 1) and its stopping rule |a^(n+1)-a^(n)| < eps;
 *   - replica exchange between neighbouring overlapping intervals (Sec. 2.5);
 *   - ln rho at the interval centres by the trapezium rule (eq. (kk3a)) and
 *     <u>(beta), C_V(beta) by the midpoint sums (eqs. (l19)-(l20), Sec. 3.4);
 *   - a warm start a(u, 1/L) for the Robbins-Monro iteration from a small
 *     network (the paper's initial values a_i-bar "inverting <E(beta)>",
 *     Sec. 2.4, here learned from converged a_k).
 *
 * Conventions shared by every call:
 *   - Units: E in plaquette-sum units; u = E/(6V) with V = L^4.
 *   - Canonical link layout (import/export): [chain][mu][s], with
 *     s = x0 + L x1 + L^2 x2 + L^3 x3, in the precision of the context.
 *   - Colour c = 2 mu + p, p = parity of the site; a sweep is heatbath on
 *     colours 0..7, then overrelaxation on colours 0..7.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed lo,
 *     seed hi), counter = (w0, w1, w2, w3) with
 *       w0 = half index h = s >> 1 (sweeps), mu*V + s (hot start), k (pair),
 *       w1 = attempt pair | colour << 8 | kind << 12 | lattice id << 16,
 *            kind 0 sweep, 1 hot start, 2 approach, 3 replica exchange, 4 MLP init,
 *       w2 = sweep index, w3 = interval index within the lattice.
 *   - Pointers: "host" arrays are read or written synchronously by the call;
 *     "device" pointers are HIP device memory owned by the caller (e.g. torch
 *     tensors); the library never frees caller memory.  Work is enqueued on
 *     the stream given at creation and every call synchronises that stream
 *     before it returns unless stated otherwise.
 *   - Errors: every call returns an llr_status; < 0 is an error and
 *     llr_last_error() holds a message (thread-local).  No exception crosses
 *     the ABI.  A context is used by one host thread at a time.
 */
#ifndef LLR_H
#define LLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct llr_ctx llr_ctx;
typedef int llr_status;

enum {
    LLR_OK = 0,
    LLR_WARN_NOT_CONVERGED = 1, /* some interval never met |da| < eps */
    LLR_EINVAL = -1,            /* invalid argument */
    LLR_ENOMEM = -2,            /* device allocation failed */
    LLR_EDEVICE = -3,           /* HIP runtime error */
    LLR_ESTATE = -4,            /* call out of order (e.g. state not bound) */
    LLR_EAPPROACH = -5,         /* approach cap reached before every chain entered its interval */
    LLR_ENUMERIC = -6           /* non-finite value or failed health test (llr_health) */
};

enum { LLR_FP64 = 0, LLR_FP32 = 1 }; /* precision of link angles and local arithmetic;
                                        energies, interval tests, a_k, RM always FP64 */
enum { LLR_MODE_RESTRICTED = 0, LLR_MODE_APPROACH = 1, LLR_MODE_FREE = 2,
       LLR_MODE_MUCA = 3 /* multicanonical; only through llr_muca_sweeps */,
       LLR_MODE_LINK = 4 /* restricted, constraint imposed per link; llr_sweeps / llr_class_pass */ };

typedef struct {
    int n_th;             /* thermalisation sweeps per RM iteration (Algorithm 1 N_TH) */
    int n_a;              /* measured sweeps per RM iteration (N_A; N_SW = N_TH + N_A) */
    int n_rm;             /* Robbins-Monro iterations (N_RM) */
    uint64_t seed;        /* Philox key */
    int replica_exchange; /* 0/1: exchange between neighbouring intervals after every sweep */
    double overlap;       /* with replica exchange the restriction width is w = (1 + overlap) dE */
    int recompute_every;  /* K: full FP64 recompute of E after every K-th sweep and the last */
    double eps;           /* stopping threshold on |a^(n+1) - a^(n)| (1e-4) */
    int approach_cap;     /* maximum approach sweeps (multiple of K) */
} llr_params;

/* --- context ------------------------------------------------------------ */

/* Create a context on HIP device `hip_device`; `hip_stream` is a hipStream_t
 * (NULL = default stream), e.g. torch.cuda.current_stream().cuda_stream.
 * precision is LLR_FP64 or LLR_FP32.  Owns only small scratch buffers. */
llr_status llr_create(llr_ctx **out, int hip_device, void *hip_stream, int precision);
void llr_destroy(llr_ctx *ctx);
const char *llr_last_error(void);
llr_status llr_set_params(llr_ctx *ctx, const llr_params *p);

/* Add a lattice of size L (even, 2 <= L <= 32) with n_intervals chains, one
 * per interval; E_low (host, n_intervals) are the ascending lower edges E_k,
 * dE > 0 the spacing (Algorithm 1: E_k = E_min + k dE).  Interval k has centre
 * c_k = E_k + dE/2 and restriction [c_k - w/2, c_k + w/2] with w = dE, or
 * (1 + overlap) dE under replica exchange.  lattice_id receives 0, 1, ...
 * At most 8 lattices.  Must precede llr_bind_state.  Edges that are not
 * evenly spaced (|E_k - E_0 - k dE| > 1e-9 max(|E_0 + k dE|, dE)) are
 * accepted by the sweeps and the replica exchange, which test each chain
 * against its own interval (the test hooks centre one interval on each
 * chain), but the calls that rely on Algorithm 1's spacing refuse them with
 * LLR_EINVAL: llr_get_ln_rho (trapezium rule on spacing dE) and
 * llr_muca_begin (the weight's interval lookup floor((E - E_0)/dE)). */
llr_status llr_add_lattice(llr_ctx *ctx, int L, int n_intervals, const double *E_low, double dE,
                           int *lattice_id);

/* Bytes of device memory the caller must bind: 2 x 4V x n_intervals angles of
 * the context precision per lattice (two planes per colour: proposals are
 * written to the non-current plane). */
llr_status llr_state_bytes(llr_ctx *ctx, size_t *bytes);
/* Bind caller-owned device memory of exactly llr_state_bytes bytes, aligned
 * to 256 bytes.  The library reads and writes it until destroy/rebind.  It
 * sets every angle to 0 (a cold start); llr_hot_start or llr_import_state
 * then set the configuration. */
llr_status llr_bind_state(llr_ctx *ctx, void *dev_state, size_t bytes);

/* Initial a_k^(0) per interval (host, n_intervals); default 1.0. */
llr_status llr_set_a(llr_ctx *ctx, int lattice_id, const double *a);

/* Uniform hot start of every chain (kind 1 counters, w3 = chain index), then a
 * full FP64 energy computation. */
llr_status llr_hot_start(llr_ctx *ctx);
/* Import/export one lattice's angles in canonical layout (device pointer,
 * n_intervals x 4 x V values of the context precision), in radians and
 * expected in [-pi, pi) as every pass writes them (the energy and the FP64
 * staple arithmetic take plaquette and staple sums of such angles).  Import
 * resets the chain <-> interval assignment to the identity and recomputes E. */
llr_status llr_import_state(llr_ctx *ctx, int lattice_id, const void *dev_canonical);
llr_status llr_export_state(llr_ctx *ctx, int lattice_id, void *dev_canonical);

/* --- Algorithm 1 -------------------------------------------------------- */

/* Approach phase: heatbath-only sweeps that accept a class move iff it does
 * not move E away from the interval, coupling adapted per pass; in blocks of
 * K sweeps and a full recompute until every chain is inside.  *sweeps
 * (host, n_lattices) receives the approach sweeps per lattice.  LLR_EAPPROACH
 * if the cap is reached. */
llr_status llr_approach(llr_ctx *ctx, long long *sweeps);
/* The same in steps: llr_approach_begin initialises the approach couplings
 * from a_k^(0), recomputes E and marks lattices already inside;
 * llr_approach_continue performs up to max_sweeps further approach sweeps
 * (whole blocks of K) and reports in *all_done whether every chain is inside;
 * sweeps (host, n_lattices) receives the approach sweeps so far. */
llr_status llr_approach_begin(llr_ctx *ctx);
llr_status llr_approach_continue(llr_ctx *ctx, long long max_sweeps, long long *sweeps, int *all_done);
/* Robbins-Monro iterations of Algorithm 1 on every interval of every lattice
 * (chains batched in one launch per pass).  Requires state inside the
 * intervals (after llr_approach).  Returns LLR_WARN_NOT_CONVERGED if some
 * interval never met the stopping rule. */
llr_status llr_run(llr_ctx *ctx);
/* The same in steps: llr_rm_begin resets the iteration counter, the sweep
 * counter and the history; llr_rm_step performs the next `iterations`
 * Robbins-Monro iterations (at most n_rm in total since llr_rm_begin) and
 * returns LLR_WARN_NOT_CONVERGED after the last one if some interval never
 * met the stopping rule.  llr_run = llr_rm_begin + llr_rm_step(n_rm). */
llr_status llr_rm_begin(llr_ctx *ctx);
llr_status llr_rm_step(llr_ctx *ctx, int iterations);
/* Which restriction the restricted sweeps of llr_run / llr_rm_step and of the
 * measurements of llr_observables impose (Sec. 2.4: rejection of a
 * colour class whose energy leaves the interval, or the constraint applied per
 * link when each new angle is drawn).  per_link 0 (default): class-wise,
 * mode LLR_MODE_RESTRICTED; 1: per link, mode LLR_MODE_LINK (its buffers are
 * allocated by the next sweep).  The approach is unchanged.  LLR_EINVAL for a
 * null context or another value. */
llr_status llr_set_restriction(llr_ctx *ctx, int per_link);
/* Order of the class passes within one sweep (Algorithm 1 fixes only that a
 * sweep evolves the whole system once):
 *   LLR_SWEEP_GROUPED (default): heatbath of colours 0..7, then
 *     overrelaxation of colours 0..7; every pass updates every link of its
 *     class (2 x 4V link updates per sweep);
 *   LLR_SWEEP_INTERLEAVED: for c = 0..7, heatbath of colour c, then the
 *     overrelaxation of colour c.  The class's staples do not change between
 *     the two, so both run in one launch that writes the overrelaxed heatbath
 *     candidate and the overrelaxed old angle; the restricted decision of the
 *     heatbath picks one (overrelaxation leaves E unchanged).  The result is
 *     that of the two separate passes in this order up to rounding: the
 *     overrelaxed heatbath angle is computed as arg[e^{-iX}(C - iS)] rather
 *     than by reflecting the rounded heatbath angle.  Reflecting a fresh
 *     heatbath draw X on the same staples gives -X - phi, itself a von Mises
 *     draw: an accepted class gets one update per link, not two, and a
 *     rejected class one overrelaxation of its old angles (with the rejected
 *     proposal, (2 - acceptance) updates per class link).
 *   LLR_SWEEP_STAGGERED: the first ceil(n/2) chains of each lattice sweep in
 *     the grouped order; the others take the overrelaxation of colours 0..7
 *     first, then the heatbath of colours 0..7 (the grouped order's passes
 *     continued half a sweep later; overrelaxation leaves E unchanged, so
 *     every chain's sweep still ends with the E of its heatbath half).  The
 *     two chain sets share no link and run on two streams (the context's and
 *     a second one of default priority, joined at the end of each sweep), so
 *     the heatbath passes, bound by vector instructions, overlap the
 *     overrelaxation passes, bound by memory.  2 x 4V link updates per
 *     sweep, as grouped.
 * Applies to the restricted, free and multicanonical sweeps of llr_run /
 * llr_rm_step / llr_sweeps / llr_observables / the multicanonical run (whose
 * accepted classes then get heatbath-only dynamics in the interleaved order,
 * for the same reason); sweeps with the per-link restriction and
 * approach-mode sweeps stay grouped.  LLR_EINVAL for a null context or
 * another value; LLR_EDEVICE if the second stream cannot be created. */
enum { LLR_SWEEP_GROUPED = 0, LLR_SWEEP_INTERLEAVED = 1, LLR_SWEEP_STAGGERED = 2 };
llr_status llr_set_sweep_order(llr_ctx *ctx, int order);
/* Final a_k, first RM iteration n with |a^(n+1)-a^(n)| < eps (-1 if never)
 * and sweeps up to it (approach + (n+1)(N_TH+N_A)); host arrays, n_intervals. */
llr_status llr_get_a(llr_ctx *ctx, int lattice_id, double *a, int *conv_iter, long long *conv_sweeps);
/* a_k^(n) for n = 0..n_rm (host, (n_rm + 1) x n_intervals) of the last run. */
llr_status llr_get_history(llr_ctx *ctx, int lattice_id, double *a_hist);
/* Current energy per chain and chain in each interval (host, n_intervals each). */
llr_status llr_get_energy(llr_ctx *ctx, int lattice_id, double *E, int *conf);
/* ln rho at the centres (trapezium recursion, eq. (kk3a)), from the current a
 * (host, n_intervals each). */
llr_status llr_get_ln_rho(llr_ctx *ctx, int lattice_id, double *centres, double *ln_rho);

/* --- checkpoints -------------------------------------------------------- */

/* Save / resume the state of Algorithm 1 between calls (the iteration over
 * RM steps n, the sweeps within them and the approach are all resumable):
 *   - the lattice set (L, n_intervals, dE, E_k) and the parameters;
 *   - every angle of the bound state (both planes of each colour) and the
 *     current-plane bits;
 *   - per chain: E, the interval it serves, the approach couplings, the
 *     heatbath acceptance counts (plain and fused passes);
 *   - per interval: a_k, the chain serving it (replica exchange moves
 *     labels, not configurations), the running sum of measured energies of
 *     the open RM iteration, the convergence record and a^(n) so far;
 *   - the sweep and approach counter words, the RM iteration n, the
 *     replica-exchange counts, the sweep order, restriction and tiles, and
 *     the counts and time of llr_get_rates.
 * A multicanonical weight (llr_muca_begin) is saved with its flag; the bits
 * log, the per-kernel timing and the health flags (cleared) are not saved.
 * File layout (little endian): "LLRCKPT1", u32 version 2, u32 precision,
 * u32 number of lattices, per lattice i32 L, i32 n, f64 dE, f64 E_low[n];
 * the llr_params fields in declaration order (i32, i32, i32, u64, i32, f64,
 * i32, f64, i32); tagged sections (u32 tag, u64 bytes, data); the CRC-32
 * (IEEE 802.3, as zlib's crc32) of all preceding bytes.
 * llr_checkpoint writes `path` (through `path`.tmp and a rename); the
 * context must have a bound state.  LLR_EINVAL if the file cannot be
 * written.
 * llr_restore loads `path` into a context created with the same precision
 * and the same lattice set (llr_add_lattice calls with identical L, edges and
 * dE) whose state is bound; it replaces the parameters by the saved ones.
 * The next llr_rm_step / llr_approach_continue / llr_sweeps continues exactly
 * as the saved context would have (same random counters).  LLR_EINVAL, with
 * nothing written to the device, if the file is missing, truncated,
 * corrupted (CRC mismatch), of another version, or of another precision or
 * lattice set.
 * llr_checkpoint_info reads and validates a file on the host alone (no
 * device needed): precision, number of lattices, and per lattice L,
 * n_intervals and dE (host arrays of at least 8), E_low (host, the sum of
 * n_intervals, lattice after lattice; may be NULL) and the parameters (may be
 * NULL).  It checks the whole file as llr_restore does before touching the
 * device: magic, version, CRC, header values that llr_add_lattice and
 * llr_set_params would accept, and a section table that covers the rest of
 * the file with every section present once at the size the header implies
 * (a^(n) either empty or of n_rm + 1 entries per interval).  LLR_EINVAL
 * otherwise. */
llr_status llr_checkpoint(llr_ctx *ctx, const char *path);
llr_status llr_restore(llr_ctx *ctx, const char *path);
llr_status llr_checkpoint_info(const char *path, int *precision, int *n_lattices, int *L, int *n_intervals,
                               double *dE, double *E_low, llr_params *params);

/* --- test and measurement hooks ----------------------------------------- */

/* n_sweeps sweeps of every chain with the current a_k (mode LLR_MODE_*),
 * starting at sweep index sweep0 (kind 0 counters; no replica exchange, no
 * measurement, no recompute).  bits (host, n_sweeps x total chains, optional):
 * bit c = heatbath colour c accepted, bit 8 + c = overrelaxation colour c. */
llr_status llr_sweeps(llr_ctx *ctx, int n_sweeps, long long sweep0, int mode, uint16_t *bits);

/* Restriction imposed per link (mode LLR_MODE_LINK of llr_sweeps and
 * llr_class_pass; Sec. 2.4, the constraint applied when each new variable is
 * generated, against the class-wise rejection of mode LLR_MODE_RESTRICTED).
 * A heatbath pass of colour c takes the class links one after another in
 * half-index order; each is drawn from its conditional restricted to the
 * values that keep the running energy inside the chain's [lo, hi], and the
 * energy is carried from link to link, so every pass is accepted.  Per link:
 * the first of the class heatbath's 64 attempts (the same counters) that
 * passes the sampler test and keeps E inside; if none does, an exact sampler
 * of the restricted density on its arc (attempts 64..127 of the counter's
 * attempt field).  Overrelaxation passes are those of the restricted mode.
 * The first use allocates, per class link of all chains, 8 bytes plus three
 * angles (the Delta E, staples and old angle of the candidate pre-pass).
 * llr_link_stats: per chain (host, total chains each, optional), the links
 * whose free candidate left the interval and were re-drawn, and how many of
 * those the arc sampler produced, summed since the state was bound. */
llr_status llr_link_stats(llr_ctx *ctx, long long *redrawn, long long *arc);
/* Tiles of the class-pass kernels: class links per thread (1, 2 or 4) of the
 * heatbath and of the overrelaxation pass.  llr_autotune
 * times the choices on the bound, initialised state without changing it and
 * keeps the fastest per kernel (llr_rm_begin calls it if no choice was made);
 * in the interleaved sweep order the heatbath tile is timed on the fused
 * heatbath + overrelaxation pass.  llr_set_tiles fixes them.  Results are
 * bit-identical for every choice. */
llr_status llr_autotune(llr_ctx *ctx, int *hb_lpt, int *or_lpt);
llr_status llr_set_tiles(llr_ctx *ctx, int hb_lpt, int or_lpt);
/* Block order of the class passes: serpentine != 0 (default) walks the chains
 * in reverse order on odd-parity colours, so a pass starts on the data the
 * previous pass touched last (Infinity Cache reuse); 0 keeps one order.
 * Results do not depend on it. */
llr_status llr_set_order(llr_ctx *ctx, int serpentine);
/* on != 0 (default): the sweeps of llr_run / llr_rm_step are captured once per
 * variant into HIP graphs and replayed (not while per-kernel timing is on). */
llr_status llr_set_graphs(llr_ctx *ctx, int on);
/* One class pass of every chain: heatbath (heatbath != 0, acceptance by mode,
 * counters with sweep index sweep_index) or overrelaxation of colour c. */
llr_status llr_class_pass(llr_ctx *ctx, int heatbath, int colour, int mode, long long sweep_index);
/* Full FP64 recompute of every chain's E. */
llr_status llr_recompute_energy(llr_ctx *ctx);
/* Record per-sweep accept bits of approach and run (host readback). */
llr_status llr_enable_bits_log(llr_ctx *ctx, long long max_rows);
llr_status llr_get_bits_log(llr_ctx *ctx, uint16_t *bits, long long *rows);
/* Accumulated acceptance counts since creation (host, total chains each):
 * heatbath proposals/accepts; replica-exchange proposals/accepts (scalars). */
llr_status llr_stats(llr_ctx *ctx, long long *hb_prop, long long *hb_acc, long long *re_prop,
                     long long *re_acc);

/* Work done and rates since creation, summed over every chain.  A link update
 * is one heatbath or one overrelaxation of one link (Algorithm 1 counts
 * sweeps of the whole lattice; the local moves inside a sweep are this
 * library's, the paper names none).  A heatbath class pass (approach passes
 * included) updates the V/2 links of its class, accepted or not, since a
 * rejected class is a valid move that keeps its links; an overrelaxation
 * class pass updates V/2 links, except in the interleaved order after an
 * accepted heatbath of the same class, where it reflects the fresh heatbath
 * draw on unchanged staples: that is again a draw from the same conditional,
 * so those passes are counted as relabelled, not as updates.  The
 * overrelaxation keeps each link's local action, hence E, and is never
 * rejected: or_acceptance is 1.  seconds is host wall time inside the calls
 * that run sweeps (llr_run, llr_rm_step, llr_approach*, llr_sweeps,
 * llr_class_pass, llr_muca_sweeps, llr_observables), each of which returns
 * after the device has finished. */
typedef struct {
    long long sweeps;              /* full sweeps (llr_run, llr_rm_step, llr_sweeps, ...); approach not included */
    long long hb_class_passes;     /* per chain, summed over chains */
    long long hb_class_accepts;
    long long or_class_passes;     /* per chain, summed over chains (fused ones included) */
    long long or_class_relabelled; /* fused overrelaxation passes after an accepted heatbath class */
    long long re_proposals, re_accepts;
    double link_updates;
    double seconds;
    double link_updates_per_s;     /* link_updates / seconds */
    double hb_acceptance, or_acceptance, re_acceptance;
} llr_rates;
llr_status llr_get_rates(llr_ctx *ctx, llr_rates *out);

/* Runtime health of the chains, from the tests the FP64 energy recompute
 * applies before it replaces a chain's incremental E:
 * flags (host, one per chain, may be NULL) are sticky bits set since the last
 * clear: 1 a link angle is not finite, 2 |E incremental - E recomputed|
 * exceeded the drift bound (1e-5 x 6V with FP32 angles, 1e-9 x 6V in FP64),
 * 4 in restricted sweeps the recomputed E lay outside the chain's restriction
 * by more than that bound.  drift (host, per chain, may be NULL): the largest
 * drift seen.  clear != 0 resets both.  Every call that runs sweeps returns
 * LLR_ENUMERIC, after its work, while a flag is set. */
llr_status llr_health(llr_ctx *ctx, uint32_t *flags, double *drift, int clear);
/* Kernel timing with HIP events on the context stream: on/off, and the
 * summed duration (ms) and count of heatbath-pass, overrelaxation-pass and
 * energy launches since enabling.  The 8 heatbath (and the 8
 * overrelaxation) launches of a sweep share one event pair, so the average
 * per launch includes the short gaps between consecutive launches.  In the
 * staggered order one event pair spans a sweep's class passes on both
 * streams and counts as 16 heatbath launches (the two kinds overlap there). */
llr_status llr_set_timing(llr_ctx *ctx, int on);
llr_status llr_get_timing(llr_ctx *ctx, double *hb_ms, long long *hb_n, double *or_ms,
                          long long *or_n, double *en_ms, long long *en_n);
/* Philox4x32-10 of n counters (host n x 4) -> out (host n x 4). */
llr_status llr_test_philox(llr_ctx *ctx, long n, const uint32_t *ctr, uint64_t seed, uint32_t *out);
/* n von Mises draws (heatbath sampler of the context precision) with
 * counters (i, c1, c2, c3); X (host, n, FP64), attempts (host, n; 0 = cap). */
llr_status llr_test_vonmises(llr_ctx *ctx, long n, double kappa, uint64_t seed, uint32_t c1,
                             uint32_t c2, uint32_t c3, double *X, int *attempts);

/* --- reconstruction (FP64 kernels) -------------------------------------- */

/* ln rho at centres and, for nb couplings beta (host), <u> = <E>/(6V) and
 * C_V = Var(E)/(6V) from the midpoint sums (eqs. (l19)-(l20)); all host arrays. */
llr_status llr_reconstruct(llr_ctx *ctx, const double *centres, const double *a, int n, double s,
                           double six_v, const double *beta, int nb, double *ln_rho,
                           double *u_mean, double *cv);
/* beta_c = argmax C_V on [blo, bhi] (grid step h, then golden section to tol)
 * and the peak value C_V = Var(E)/(6V); the paper's tabulated C_V/(6V) is
 * this divided by 6V, i.e. Var(u). */
llr_status llr_beta_c(llr_ctx *ctx, const double *centres, const double *a, int n, double s,
                      double six_v, double blo, double bhi, double h, double tol,
                      double *beta_c, double *cv_peak);

/* llr_beta_c for callers that cannot allocate device memory (code running
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, with the device copies
 * of centres and a, ln rho, the grid of Var(E) and the result held in one
 * fixed library array of 1 MiB per GPU (created with the library, resolved by
 * llr_create for its device, never freed before the process ends) instead of
 * the context's growing staging buffer.  The call allocates nothing.
 * Requires 8 (3 n + ng + 8) <= 2^20 bytes, ng = round((bhi - blo)/h) (e.g.
 * n = 128 with ng up to 130 000), else LLR_EINVAL.  Every call on one GPU
 * uses that GPU's array: calls that overlap on one GPU (several host threads
 * or streams) race and must be serialised by the caller; the array keeps the
 * last call's contents, which nothing reads. */
llr_status llr_beta_c_noalloc(llr_ctx *ctx, const double *centres, const double *a, int n, double s,
                              double six_v, double blo, double bhi, double h, double tol,
                              double *beta_c, double *cv_peak);

/* --- analysis of repeated runs (Sec. 2.4 N_B repetitions, Sec. 3.4) ------ */

/* ln P_beta(E) at m energies E (host), P_beta(E) = rho~(E) e^{beta E} / Z with
 * the piecewise-exponential rho~ of eq. (rhoguess) built from a_k on intervals
 * of width s centred at centres (host, n, spaced by s; else LLR_EINVAL):
 * ln rho~ is continuous, with slope -a_k in interval k, and Z is its exact
 * integral over [c_0 - s/2, c_{n-1} + s/2].  log_p (host, m) is -inf outside
 * that range. */
llr_status llr_prob_density(llr_ctx *ctx, const double *centres, const double *a, int n,
                            double s, double beta, const double *E, int m, double *log_p);
/* Interior local maxima of P_beta(E) (the peaks of the two phases at a
 * first-order transition, Sec. 3.4): ln P is linear in each interval, so the
 * edge between intervals k and k+1 is a maximum iff a_k < beta <= a_{k+1}.
 * Up to max_peaks energies and ln P values (host) in ascending E; n_found
 * receives the total number, which may exceed max_peaks. */
llr_status llr_prob_peaks(llr_ctx *ctx, const double *centres, const double *a, int n, double s,
                          double beta, int max_peaks, double *E_peak, double *log_p_peak,
                          int *n_found);
/* Bootstrap of beta_c and the C_V peak over n_runs independent runs of
 * Algorithm 1 (repeated N_B times for the error analysis, Sec. 2.4 and 3.2).
 * a_runs (host, n_runs x n, row-major; 1 <= n_runs <= 1024).  Sample b
 * (0 <= b < n_boot) takes run floor(n_runs w / 2^32) as its j-th draw, w the
 * first word of Philox4x32-10 at counter (j, kind 5 << 12, b, 0) with key
 * (seed lo, seed hi), averages the drawn runs' a_k in draw order, and is
 * reconstructed as llr_beta_c does.  beta_c, cv_peak (host, n_boot): one
 * value per sample; their mean and standard deviation are the estimate and
 * its error.  (n_boot (ng + 1) <= 6.5e7 grid points, ng = (bhi - blo)/h.) */
llr_status llr_bootstrap(llr_ctx *ctx, const double *centres, const double *a_runs, int n_runs,
                         int n, double s, double six_v, double blo, double bhi, double h,
                         double tol, int n_boot, uint64_t seed, double *beta_c,
                         double *cv_peak);
/* Weighted least squares for the finite-size scaling forms of Sec. 3.4,
 * y(L) = sum_j p_j L^{powers_j} (e.g. beta_c(L) = beta_c + B_1 L^-4 + B_2 L^-8
 * with powers {0, -4, -8}; C_V/(6V) at the peak = G^2/4 + C_1 L^-4 + ...):
 * x (L > 0), y, sigma (> 0): host, m > n_par; powers: host, n_par <= 16.
 * params (host, n_par); errors (host, n_par, optional): sqrt of the diagonal
 * of the covariance (A^T A)^-1 of the weighted design matrix, not scaled by
 * chi2_red; chi2_red (optional): residual sum of squares / (m - n_par).
 * Host computation (Householder QR); needs no context. */
llr_status llr_fss_fit(const double *x, const double *y, const double *sigma, int m,
                       const double *powers, int n_par, double *params, double *errors,
                       double *chi2_red);

/* --- observables from restricted double brackets (Sec. 2.3) ------------- */

/* n_meas measurements with the current a_k: gap restricted sweeps (replica
 * exchange as set in llr_params) from sweep index sweep0 (choose it beyond
 * the sweeps of the Robbins-Monro run, whose counters it would reuse), then
 * a full FP64 evaluation of E and of the adjoint plaquette sum
 * B = sum_P cos 2 theta_P of every chain.  E, B (host, n_meas x total
 * intervals, row-major): the values of the chain serving each interval, so
 * column k holds the restricted samples of interval k. */
llr_status llr_observables(llr_ctx *ctx, int n_meas, int gap, long long sweep0, double *E, double *B);
/* <B>(beta) at nb couplings from m restricted samples (E, B) per interval
 * (host, m x n, interval fastest) on intervals of width s centred at centres
 * (spaced by s), eqs. (l9)-(l10):
 * <B> = sum_k rho~(c_k) e^{beta c_k} <<B e^{(beta - a_k)(E - c_k)}>>_k
 *     / sum_k rho~(c_k) e^{beta c_k} <<e^{(beta - a_k)(E - c_k)}>>_k. */
llr_status llr_obs_reconstruct(llr_ctx *ctx, const double *centres, const double *a, int n, double s,
                               const double *E, const double *B, int m, const double *beta, int nb,
                               double *B_mean);

/* --- multicanonical sampling with W = 1/rho~ and reweighting (Sec. 2.6) --- */

/* Builds each lattice's weight W(E) = 1/rho~(E) from its current a_k
 * (intervals of width dE: ln rho~ continuous, slope -a_k in interval k; below
 * the first and above the last interval the first and last pieces continue,
 * i.e. W = e^{a_0 E + c_1} and e^{a_{n-1} E + c_2}, eq. (4.1) with beta_1 =
 * a_0, beta_2 = a_{n-1} and c_1, c_2 from continuity), stores the heatbath
 * proposal couplings b (host, one per lattice, >= 0) and recomputes E in
 * FP64.  Any later change of a_k (llr_set_a, llr_run, llr_rm_*) requires a new
 * llr_muca_begin. */
llr_status llr_muca_begin(llr_ctx *ctx, const double *b);
/* n_sweeps multicanonical sweeps of every chain from sweep index sweep0: per
 * colour class a heatbath proposal at coupling b, accepted with probability
 * min(1, W(E') / W(E) e^{-b (E' - E)}) (the Metropolis-Hastings ratio of the
 * class heatbath, whose normalisation depends only on the other classes;
 * uniform from Philox counter (interval, colour << 8 | 6 << 12 | lattice <<
 * 16, sweep, 0), first word), then the overrelaxation classes (E unchanged,
 * always accepted); FP64 recompute after every K-th sweep of the call.
 * E_hist (host, n_sweeps x total chains, optional): each chain's E after each
 * sweep, chains in context order. */
llr_status llr_muca_sweeps(llr_ctx *ctx, int n_sweeps, long long sweep0, double *E_hist);
/* Canonical <u> = <E>/(6V) and C_V = Var(E)/(6V) at nb couplings beta (host)
 * from m multicanonical samples E (host) taken with the weight built from a_k
 * (host, n, on intervals of width s centred at centres, spaced by s):
 * <O>_beta = <O e^{beta E} / W(E)>_W / <e^{beta E} / W(E)>_W, eq. (4.7). */
llr_status llr_muca_reweight(llr_ctx *ctx, const double *E, long m, const double *centres,
                             const double *a, int n, double s, double six_v, const double *beta,
                             int nb, double *u_mean, double *cv);

/* --- warm-start network a(u, 1/L): 2 -> 64 (tanh) -> 64 (tanh) -> 1 ------ */
/* Parameter vector (host, 4417 FP32): W1[64][2], b1[64], W2[64][64], b2[64],
 * W3[64], b3.  Inputs uh = (u - 0.6)/0.1, lh = (1/L - 0.0875)/0.0375; output
 * a = 1 + 0.1 y.  bf16 != 0: the 64x64 layer runs on MFMA in bfloat16 with
 * FP32 accumulation; otherwise FP32 on the vector units. */
llr_status llr_mlp_init(llr_ctx *ctx, uint64_t seed, float *weights);
llr_status llr_mlp_predict(llr_ctx *ctx, const float *weights, const float *u, const float *inv_L,
                           int n, int bf16, double *a_out);
/* Warm start of Algorithm 1 from the network (Sec. 2.4: initial a_i close to
 * the result shorten the Robbins-Monro iteration): predicts a_k at the
 * centres c_k of lattice lattice_id (u = c_k/(6V), 1/L) and sets them as
 * a_k^(0) (llr_set_a).  Plain Robbins-Monro stays the fallback: a prediction
 * that is not finite or lies outside [a_min, a_max] (the caller passes the
 * range of the a_k the network was trained on, with any margin) is replaced
 * by a^(0) = 1, the cold start.  a_out (host, n_intervals, optional)
 * receives the a_k^(0) set; n_fallback (optional) the number replaced. */
llr_status llr_mlp_warm_start(llr_ctx *ctx, int lattice_id, const float *weights, int bf16, double a_min,
                              double a_max, double *a_out, int *n_fallback);
/* Mean squared error on a and its gradient (host, 4417). */
llr_status llr_mlp_loss_grad(llr_ctx *ctx, const float *weights, const float *u,
                             const float *inv_L, const double *a, int n, int bf16, float *grad,
                             double *loss);
/* Full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8) for `epochs` steps;
 * weights in/out; loss_hist (host, epochs, optional). n <= 4096. */
llr_status llr_mlp_train(llr_ctx *ctx, float *weights, const float *u, const float *inv_L,
                         const double *a, int n, int epochs, float lr, int bf16,
                         double *loss_hist);

#ifdef __cplusplus
}
#endif
#endif /* LLR_H */
