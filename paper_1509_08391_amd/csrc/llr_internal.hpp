// llr_internal.hpp -- structures shared by the kernel launchers and the
// host runtime of the LLR library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "llr_device.hpp"

namespace llr {

// One lattice of the batch: n_chains chains of size L^4, one per interval.
// Chain g of the lattice owns 2 planes x 8 colours x V/2 angles at
// base + (g - chain0) * 8 V, plane b, colour c at offset (8 b + c) V/2.
struct LatDev {
    int L, hL;             // L, L/2
    uint32_t V2;           // V/2
    uint32_t mL, mhL;      // ceil(2^32 / L), ceil(2^32 / (L/2))
    int n_chains;          // chains of the table (all of the lattice's, or one half in the staggered order)
    int chain0;            // first global chain index of the table
    int n_itv, itv0;       // the lattice's intervals: count and first global index (= its first chain)
    int hb_bpc, hb_block0; // heatbath pass: blocks per chain (npt x ceil(L / LPT)), first block
    int or_bpc, or_block0; // overrelaxation pass: the same
    uint32_t P;            // positions in the (x0h, x1, x2) slab: hL L^2 = V/(2L); h = pos + P x3
    int npt;               // position tiles of kBlock per slab, ceil(P / kBlock)
    int ebpc;              // blocks per chain in the site kernels (2 x V/2 / 256, rounded up)
    int hstr[4];           // half-index stride of a step along nu = 1..3: (L/2) L^(nu-1); [0] unused
    int hwrap[4];          // (L - 1) hstr[nu]: the periodic jump across the boundary
    double ds;             // interval spacing delta E
    int eblock0;           // first block of this lattice in the site grid
    int lat_id;
    long long base;        // element offset of the lattice's first chain
    long long lbase;       // offset of its first chain in the per-class-link buffers (chain-major, V/2 each)
    int fxb;               // fraction bits of the per-chain energy sums
    double fx, fxinv;      // 2^fxb and 2^-fxb
};

struct LatTable {
    LatDev l[kMaxLat];
    int n;
    int hb_lpt, or_lpt;    // class links per thread (1, 2 or 4), chosen by the autotuner
    int serpentine;        // odd-parity colours walk the blocks in reverse order (cache reuse)
    int hb_blocks;         // total blocks of a heatbath / overrelaxation launch
    int or_blocks;
    int site_blocks;       // total blocks of a site launch
    int n_chains;          // total chains = total intervals
};

// Per-chain and per-interval device state (all indices global).
struct DevState {
    // per chain
    double* E;             // current energy (incremental, FP64)
    unsigned long long* acc;   // arrivals << 51 | fixed-point Delta E of the running pass
    unsigned long long* eacc;  // the same for the energy recompute
    unsigned long long* oacc;  // the same for the observable of the measurement recompute
    double* obs;           // adjoint plaquette sum, sum_P cos 2 theta_P (FP64, at the last measurement)
    uint8_t* cur;          // 8 per chain: current plane of each colour
    int* itv;              // global index of the interval the chain serves
    double* b;             // approach coupling, 8 per chain (one per colour)
    double* eta;           // approach step, 8 per chain
    int* sprev;            // approach: sign of the previous proposal offset, 8 per chain
    uint16_t* bits;        // accept bits of the running sweep
    uint16_t* bits_last;   // accept bits of the last finished sweep
    unsigned long long* hb_prop;
    unsigned long long* hb_acc;
    unsigned long long* fu_acc;   // fused heatbath + overrelaxation passes whose heatbath class was accepted
    uint32_t* health;      // kHealth* flags raised by the energy recompute (sticky until read and cleared)
    double* drift;         // largest |E incremental - E recomputed| seen at a recompute
    // per interval (global index = chain0 of the lattice + local index)
    double* a;             // Robbins-Monro coupling
    double* lo;            // restriction [lo, hi]
    double* hi;
    double* cen;           // centre c_k
    double* w;             // restriction width
    double* sumE;          // sum of measured energies in the running RM iteration
    int* conf;             // chain serving the interval
    int* conv_iter;
    long long* conv_sweeps;
    double* a_hist;        // (n_rm + 1) x n_chains
    double* mu_lnrho;      // ln rho~ at the centre, for the multicanonical weight W = 1/rho~
    // per-link constraint: one entry per class link of every chain (lbase layout)
    long long* link_d;     // Delta E of the free heatbath candidate, fixed point (kLinkNone: none)
    void* link_cst;        // staple sums C, S and the old angle, three T arrays of link_n each
    long long link_n;
    unsigned long long* link_fix;   // per chain: links re-drawn by the walk
    unsigned long long* link_arc;   // per chain: of those, drawn by the arc sampler
    // per lattice
    int* lat_done;         // approach finished
    int* lat_outside;      // chains outside their interval (approach check)
    long long* lat_approach;   // approach sweeps performed
    double* mu_b;          // multicanonical heatbath proposal coupling
    // scalars
    uint32_t* sweep_ctr;   // RM sweep index (counter word 2)
    uint32_t* approach_ctr;
    int* rm_iter;          // current RM iteration n
    unsigned long long* re_cnt;  // [proposed, accepted]
    uint16_t* bits_log;    // optional, rows x n_chains
    long long* bits_row;   // next log row
    long long bits_rows_max;
};

// Health tests of the FP64 energy recompute.  The incremental E of a chain
// and the recomputed one differ by the rounding of the per-link Delta E (and,
// in FP32, of the overrelaxed angles, whose energy change is not tracked);
// the drift bound is 1e-5 x 6V in FP32 and 1e-9 x 6V in FP64, far above that
// rounding.  An angle that is not finite makes its plaquettes not finite.
enum { kHealthNonFinite = 1, kHealthDrift = 2, kHealthOutside = 4 };
enum { kCheckDrift = 1, kCheckInterval = 2 };

struct RunCfg {
    uint32_t k0, k1;       // Philox key
    int n_a;
    int nsw;               // n_th + n_a
    double eps;
};

// launchers (llr_sweep.hip); T = float or double
template <typename T> void launch_hot_start(const LatTable& lt, T* th, DevState s, uint32_t k0, uint32_t k1, hipStream_t st);
template <typename T> void launch_hb_pass(const LatTable& lt, T* th, DevState s, int colour, int mode, int kind,
                                          uint32_t k0, uint32_t k1, hipStream_t st);
template <typename T> void launch_or_pass(const LatTable& lt, T* th, DevState s, int colour, int to_alt,
                                          hipStream_t st);
// heatbath pass of colour c (sweep counters) immediately followed by the
// overrelaxation of the same class, in one launch
template <typename T> void launch_hb_or_pass(const LatTable& lt, T* th, DevState s, int colour, int mode,
                                             uint32_t k0, uint32_t k1, hipStream_t st);
// check: kCheck* bits (which health tests the recompute applies)
template <typename T> void launch_energy(const LatTable& lt, const T* th, DevState s, hipStream_t st,
                                          bool with_obs = false, int check = 0);
template <typename T> void launch_export(const LatTable& lt, int li, const T* th, DevState s, T* out, hipStream_t st);
template <typename T> void launch_import(const LatTable& lt, int li, T* th, DevState s, const T* in, hipStream_t st);
void launch_end_sweep(const LatTable& lt, DevState s, int measure, int approach, int with_or, hipStream_t st);
void launch_replica(const LatTable& lt, DevState s, uint32_t k0, uint32_t k1, hipStream_t st);
void launch_rm_update(const LatTable& lt, DevState s, RunCfg cfg, hipStream_t st);
void launch_approach_init(const LatTable& lt, DevState s, hipStream_t st);
void launch_approach_check(const LatTable& lt, DevState s, hipStream_t st);
void launch_test_philox(long n, const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, hipStream_t st);
template <typename T> void launch_test_vonmises(long n, double kappa, uint32_t k0, uint32_t k1, uint32_t c1,
                                                uint32_t c2, uint32_t c3, double* X, int* att, hipStream_t st);

// reconstruction (llr_recon.hip)
void launch_recon(const double* c, const double* a, int n, double s, double six_v, const double* beta, int nb,
                  double* lnrho, double* u, double* cv, hipStream_t st);
void launch_beta_c(const double* c, const double* a, int n, double s, double six_v, double blo, double bhi,
                   double h, double tol, double* lnrho_scratch, double* out2, hipStream_t st);
void launch_beta_c_rows(const double* c, const double* a, int n, int rows, double s, double six_v, double blo,
                        double bhi, double h, double tol, double* scratch, double* out2, hipStream_t st);
void launch_boot_mean(const double* a_runs, int n_runs, int n, int n_boot, uint64_t seed, double* abar,
                      hipStream_t st);
void launch_prob(const double* c, const double* a, int n, double s, double beta, const double* E, int m,
                 double* logp, int max_peaks, double* E_pk, double* lp_pk, int* n_pk, double* scratch,
                 hipStream_t st);
void launch_reweight(const double* E, long m, const double* c, const double* a, int n, double s, const double* beta,
                     int nb, double six_v, double* u, double* cv, double* scratch, hipStream_t st);
void launch_obs_bracket(const double* E, const double* B, int m, const double* c, const double* a, int n, double s,
                        const double* beta, int nb, double* out, double* scratch, hipStream_t st);

// network (llr_mlp.hip)
constexpr int kMlpH = 64;
constexpr int kMlpNP = 4417;
void launch_mlp_init(uint64_t seed, float* w, hipStream_t st);
void launch_mlp_forward(const float* w, const float* u, const float* invL, int n, int bf16, double* a_out,
                        hipStream_t st);
void launch_mlp_loss_grad(const float* w, const float* u, const float* invL, const double* a, int n, int bf16,
                          float* grad, double* loss, hipStream_t st);
void launch_mlp_adam(float* w, float* m, float* v, const float* g, int t, float lr, hipStream_t st);

}  // namespace llr
