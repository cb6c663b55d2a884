// llr_capi.hip -- host runtime and C ABI of the LLR library (include/llr.h).
// Drives Algorithm 1 of arXiv:1509.08391 on the GPU: approach, then per
// Robbins-Monro iteration N_TH + N_A sweeps of all chains (8 heatbath + 8
// overrelaxation class passes each, periodic FP64 recompute, optional replica
// exchange, measurement) and the update of every a_k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/llr.h"
#include "llr_internal.hpp"

using namespace llr;

static thread_local std::string g_err;

static llr_status fail(llr_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(LLR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

// Device memory for llr_beta_c_noalloc, for callers that cannot allocate:
// one fixed array per GPU, held until the process ends.  Host code never
// uses the array's name as an address: llr_create resolves each device's
// copy with hipGetSymbolAddress (that device current) and keeps the pointer.
constexpr size_t kNoAllocBytes = (size_t)1 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Resolve this device's copy of scratch once (the device must be current).
static llr_status scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(LLR_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return LLR_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LLR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return LLR_OK;
}

struct HostLat {
    int L;
    int n;
    double dE;
    bool even;             // E_low[k] = E_low[0] + k dE (Algorithm 1's interval set)
    std::vector<double> E_low;
    std::vector<double> a0;
};

// The calls that rely on Algorithm 1's evenly spaced interval set (ln rho by
// the trapezium rule on spacing dE, the multicanonical weight's interval
// lookup floor((E - E_0)/dE)) refuse a lattice whose edges deviate from it.
static bool evenly_spaced(const double* E_low, int n, double dE) {
    for (int k = 1; k < n; ++k) {
        const double want = E_low[0] + (double)k * dE;
        if (!(std::fabs(E_low[k] - want) <= 1e-9 * std::max(std::fabs(want), dE))) return false;
    }
    return true;
}

struct TimingPair {
    hipEvent_t a, b;
    int kind;   // 0 hb, 1 or, 2 energy
    int count;  // launches between the two events
};

struct llr_ctx {
    bool muca_ready = false;   // multicanonical weights built (llr_muca_begin)
    bool per_link = false;     // Algorithm 1's restricted sweeps impose the restriction per link
    bool interleave = false;   // sweep = (heatbath, overrelaxation) per colour, fused in one launch
    bool stagger = false;      // staggered order: the second half of each lattice's chains overrelaxes first
    int device = 0;
    hipStream_t stream = nullptr;
    int precision = LLR_FP64;
    llr_params prm{};
    std::vector<HostLat> lats;
    LatTable lt{};
    DevState ds{};
    bool laid_out = false;
    void* state = nullptr;
    size_t state_bytes = 0;
    bool have_energy = false;
    std::vector<void*> allocs;
    std::vector<long long> approach_sweeps;
    std::vector<int> ap_done;  // approach finished per lattice
    bool ap_open = false;
    int rm_done = 0;       // RM iterations performed since llr_rm_begin
    bool tuned = false;    // class-pass tiles chosen (autotuner or llr_set_tiles)
    // captured sweeps (kernel nodes only), keyed by recompute | replica << 1 | measure << 2
    bool use_graphs = true;
    hipGraphExec_t sweep_graph[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipStream_t cap_stream = nullptr;  // default priority
    hipStream_t side = nullptr;        // staggered order: the second chain set's stream (default priority)
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    bool rm_open = false;
    // timing
    bool timing = false;
    std::vector<TimingPair> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[3] = {0, 0, 0};
    long long t_n[3] = {0, 0, 0};
    // device staging of small host arrays (grown on demand)
    void* stage = nullptr;
    size_t stage_bytes = 0;
    // link-update accounting (llr_get_rates): class passes applied to every
    // chain, counted as they are enqueued or replayed
    bool capturing = false;        // a sweep is being captured into a graph, not run
    long long sweeps_run = 0;      // full sweeps (any mode) since creation
    long long or_passes = 0;       // plain overrelaxation class passes
    long long fused_passes = 0;    // fused heatbath + overrelaxation class passes
    double run_seconds = 0.0;      // host wall time inside the calls that run sweeps
};

// Wall time of one sweep-running call (each ends with a stream synchronisation).
struct RunClock {
    llr_ctx* c;
    std::chrono::steady_clock::time_point t0;
    explicit RunClock(llr_ctx* cc) : c(cc), t0(std::chrono::steady_clock::now()) {}
    ~RunClock() {
        if (c) c->run_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static size_t elem_size(const llr_ctx* c) { return c->precision == LLR_FP32 ? 4 : 8; }

static llr_status ensure_stage(llr_ctx* c, size_t bytes) {
    if (c->stage_bytes >= bytes) return LLR_OK;
    if (c->stage) HIPCHK(hipFree(c->stage));
    c->stage = nullptr;
    c->stage_bytes = 0;
    HIPCHK(hipMalloc(&c->stage, bytes));
    c->stage_bytes = bytes;
    return LLR_OK;
}

template <typename P>
static llr_status dalloc(llr_ctx* c, P** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count * sizeof(P), 8)) != hipSuccess)
        return fail(LLR_ENOMEM, "device allocation failed");
    HIPCHK(hipMemsetAsync(q, 0, std::max<size_t>(count * sizeof(P), 8), c->stream));
    c->allocs.push_back(q);
    *p = (P*)q;
    return LLR_OK;
}

// ceil(2^32 / d) for d >= 2 (divisor 1 is handled by the kernels directly)
static uint32_t magic(uint32_t d) { return d < 2 ? 0u : (uint32_t)(((1ull << 32) + d - 1) / d); }

static double restriction_width(const llr_ctx* c, double dE) {
    return c->prm.replica_exchange ? (1.0 + c->prm.overlap) * dE : dE;
}

// Upload per-interval tables (lo, hi, cen, w) from the host lattice set.
static llr_status upload_intervals(llr_ctx* c) {
    const int n = c->lt.n_chains;
    std::vector<double> lo(n), hi(n), cen(n), w(n), a(n);
    int k = 0;
    for (auto& hl : c->lats)
        for (int i = 0; i < hl.n; ++i, ++k) {
            const double ww = restriction_width(c, hl.dE);
            cen[k] = hl.E_low[i] + 0.5 * hl.dE;
            lo[k] = cen[k] - 0.5 * ww;
            hi[k] = cen[k] + 0.5 * ww;
            w[k] = ww;
            a[k] = hl.a0[i];
        }
    HIPCHK(hipMemcpyAsync(c->ds.lo, lo.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ds.hi, hi.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ds.cen, cen.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ds.w, w.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ds.a, a.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LLR_OK;
}

static void drop_graphs(llr_ctx* c) {
    for (auto& g : c->sweep_graph)
        if (g) { hipGraphExecDestroy(g); g = nullptr; }
}

// Block tables of the class-pass launches for hb_lpt / or_lpt class links per thread.
static void set_tiles(LatTable& lt, int hb_lpt, int or_lpt) {
    lt.hb_lpt = hb_lpt;
    lt.or_lpt = or_lpt;
    int hb0 = 0, or0 = 0;
    for (int i = 0; i < lt.n; ++i) {
        LatDev& d = lt.l[i];
        // column tiles: npt position tiles of the (x0h, x1, x2) slab times
        // ceil(L / LPT) groups of consecutive x3
        d.hb_bpc = d.npt * ((d.L + hb_lpt - 1) / hb_lpt);
        d.or_bpc = d.npt * ((d.L + or_lpt - 1) / or_lpt);
        d.hb_block0 = hb0;
        d.or_block0 = or0;
        hb0 += d.n_chains * d.hb_bpc;
        or0 += d.n_chains * d.or_bpc;
    }
    lt.hb_blocks = hb0;
    lt.or_blocks = or0;
}

// The staggered order's two chain sets: per lattice, the first ceil(n/2)
// chains (A) and the others (B), as tables of their own (a lattice may hold
// no chain in B; its block ranges are then empty).
static void half_tables(const LatTable& lt, LatTable& a, LatTable& b) {
    a = lt;
    b = lt;
    a.n_chains = b.n_chains = 0;
    for (int i = 0; i < lt.n; ++i) {
        const LatDev& d = lt.l[i];
        const int na = (d.n_chains + 1) / 2;
        a.l[i].n_chains = na;
        b.l[i].n_chains = d.n_chains - na;
        b.l[i].chain0 = d.chain0 + na;
        b.l[i].base = d.base + (long long)na * 16ll * (long long)d.V2;
        b.l[i].lbase = d.lbase + (long long)na * (long long)d.V2;
        a.n_chains += na;
        b.n_chains += d.n_chains - na;
    }
    set_tiles(a, lt.hb_lpt, lt.or_lpt);
    set_tiles(b, lt.hb_lpt, lt.or_lpt);
}

static llr_status layout(llr_ctx* c) {
    if (c->laid_out) return LLR_OK;
    if (c->lats.empty()) return fail(LLR_ESTATE, "no lattice added");
    LatTable& lt = c->lt;
    memset(&lt, 0, sizeof(lt));
    lt.n = (int)c->lats.size();
    int chain0 = 0, eblock0 = 0;
    long long base = 0, lbase = 0;
    for (int i = 0; i < lt.n; ++i) {
        const HostLat& h = c->lats[i];
        LatDev& d = lt.l[i];
        d.L = h.L;
        d.hL = h.L / 2;
        const long long V = (long long)h.L * h.L * h.L * h.L;
        d.V2 = (uint32_t)(V / 2);
        d.P = d.V2 / (uint32_t)h.L;
        d.npt = (int)((d.P + kBlock - 1) / kBlock);
        d.mL = magic((uint32_t)h.L);
        d.mhL = magic((uint32_t)(h.L / 2));
        d.n_chains = h.n;
        d.chain0 = chain0;
        d.n_itv = h.n;
        d.itv0 = chain0;
        // site kernels: the even and the odd sites of a chain in blocks of their own
        d.ebpc = 2 * (int)((V / 2 + kBlock - 1) / kBlock);
        d.eblock0 = eblock0;
        d.hstr[0] = 0;
        d.hwrap[0] = 0;
        for (int nu = 1; nu < 4; ++nu) {
            d.hstr[nu] = nu == 1 ? d.hL : d.hstr[nu - 1] * h.L;
            d.hwrap[nu] = (h.L - 1) * d.hstr[nu];
        }
        d.lat_id = i;
        d.ds = h.dE;
        d.base = base;
        d.lbase = lbase;
        lbase += (long long)h.n * (V / 2);
        // largest fxb with 6V 2^fxb <= 2^49
        const int fxb = (int)std::floor(49.0 - std::log2(6.0 * (double)V));
        d.fxb = fxb;
        d.fx = std::ldexp(1.0, fxb);
        d.fxinv = std::ldexp(1.0, -fxb);
        chain0 += h.n;
        eblock0 += h.n * d.ebpc;
        base += (long long)h.n * 8 * V;
    }
    lt.site_blocks = eblock0;
    lt.serpentine = 1;
    set_tiles(lt, 1, 1);
    lt.n_chains = chain0;
    c->state_bytes = (size_t)base * elem_size(c);
    const int n = chain0;
    DevState& s = c->ds;
    llr_status st;
#define AL(field, cnt) \
    if ((st = dalloc(c, &s.field, (cnt))) != LLR_OK) return st;
    AL(E, n) AL(acc, n) AL(eacc, n) AL(oacc, n) AL(obs, n) AL(cur, 8 * n) AL(itv, n) AL(b, 8 * n) AL(eta, 8 * n)
    AL(sprev, 8 * n) AL(bits, n + 2) AL(bits_last, n + 2) AL(hb_prop, n) AL(hb_acc, n) AL(fu_acc, n) AL(health, n)
    AL(drift, n) AL(a, n) AL(lo, n) AL(hi, n)
    AL(cen, n) AL(w, n) AL(sumE, n) AL(conf, n) AL(conv_iter, n) AL(conv_sweeps, n) AL(mu_lnrho, n)
    AL(mu_b, kMaxLat) AL(link_fix, n) AL(link_arc, n)
    AL(lat_done, kMaxLat) AL(lat_outside, kMaxLat) AL(lat_approach, kMaxLat) AL(sweep_ctr, 1)
    AL(approach_ctr, 1) AL(rm_iter, 1) AL(re_cnt, 2) AL(bits_row, 1)
#undef AL
    s.a_hist = nullptr;
    s.bits_log = nullptr;
    s.link_d = nullptr;
    s.link_cst = nullptr;
    s.link_n = lbase;
    s.bits_rows_max = 0;
    std::vector<int> ident(n);
    for (int i = 0; i < n; ++i) ident[i] = i;
    HIPCHK(hipMemcpyAsync(s.itv, ident.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(s.conf, ident.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    c->approach_sweeps.assign(lt.n, 0);
    c->laid_out = true;
    return upload_intervals(c);
}

// ---------------------------------------------------------------- timing
static hipEvent_t ev_get(llr_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
}
static void harvest(llr_ctx* c) {
    for (auto& p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->t_ms[p.kind] += ms;
            c->t_n[p.kind] += p.count;
        }
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
}
// Event pair around `count` consecutive launches of one kernel kind.
struct TimeScope {
    llr_ctx* c;
    int kind;
    int count;
    hipEvent_t a{}, b{};
    TimeScope(llr_ctx* cc, int k, int n = 1) : c(cc), kind(k), count(n) {
        if (c->timing) {
            a = ev_get(c);
            b = ev_get(c);
            hipEventRecord(a, c->stream);
        }
    }
    ~TimeScope() {
        if (c->timing) {
            hipEventRecord(b, c->stream);
            c->pending.push_back({a, b, kind, count});
            if (c->pending.size() >= 2048) {
                hipEventSynchronize(b);
                harvest(c);
            }
        }
    }
};

// ---------------------------------------------------------------- health
// The energy recompute's sticky per-chain flags (kHealth*): LLR_ENUMERIC with
// the first flagged chain named, the flags left set until llr_health clears
// them.  Called at the end of the calls that run sweeps.
static llr_status health_check(llr_ctx* c) {
    const int n = c->lt.n_chains;
    std::vector<uint32_t> f(n);
    std::vector<double> d(n);
    HIPCHK(hipMemcpy(f.data(), c->ds.health, 4 * (size_t)n, hipMemcpyDeviceToHost));
    for (int g = 0; g < n; ++g) {
        if (!f[g]) continue;
        HIPCHK(hipMemcpy(d.data(), c->ds.drift, 8 * (size_t)n, hipMemcpyDeviceToHost));
        char msg[256];
        snprintf(msg, sizeof msg, "chain %d failed a health test at an energy recompute:%s%s%s (largest drift %.3e)", g,
                 (f[g] & kHealthNonFinite) ? " non-finite angle" : "",
                 (f[g] & kHealthDrift) ? " incremental E drifted beyond the bound" : "",
                 (f[g] & kHealthOutside) ? " E outside its restriction" : "", d[g]);
        return fail(LLR_ENUMERIC, msg);
    }
    return LLR_OK;
}

// ---------------------------------------------------------------- sweep drivers
template <typename T>
static void enqueue_hb_pass(llr_ctx* c, int colour, int mode, int kind) {
    launch_hb_pass<T>(c->lt, (T*)c->state, c->ds, colour, mode, kind, (uint32_t)c->prm.seed,
                      (uint32_t)(c->prm.seed >> 32), c->stream);
}
template <typename T>
static void enqueue_or_pass(llr_ctx* c, int colour) {
    launch_or_pass<T>(c->lt, (T*)c->state, c->ds, colour, 0, c->stream);
}
template <typename T>
static void enqueue_energy(llr_ctx* c, int check = kCheckDrift) {
    TimeScope ts(c, 2);
    launch_energy<T>(c->lt, (const T*)c->state, c->ds, c->stream, false, check);
}

// the overrelaxation class passes one sweep applies to every chain: 8
// plain ones, or 8 fused into the heatbath passes
static void note_sweep(llr_ctx* c, bool fused) {
    if (c->capturing) return;
    c->sweeps_run += 1;
    if (fused) c->fused_passes += 8;
    else c->or_passes += 8;
}

// one restricted sweep of all chains, then recompute / replica exchange / measurement
template <typename T>
static void enqueue_sweep(llr_ctx* c, int mode, bool recompute, bool replica, bool measure) {
    const bool plain = mode == LLR_MODE_RESTRICTED || mode == LLR_MODE_FREE || mode == LLR_MODE_MUCA;
    const bool fused = c->interleave && plain;
    note_sweep(c, fused);
    if (fused) {
        TimeScope ts(c, 0, 8);
        for (int col = 0; col < 8; ++col)
            launch_hb_or_pass<T>(c->lt, (T*)c->state, c->ds, col, mode, (uint32_t)c->prm.seed,
                                 (uint32_t)(c->prm.seed >> 32), c->stream);
    } else if (c->stagger && plain) {   // c->stagger implies the side stream exists
        // chains of A on the context's stream: heatbath of colours 0..7, then
        // overrelaxation of 0..7; chains of B on the side stream:
        // overrelaxation first.  The two sets share no link, so the streams
        // join only at the end of the sweep.
        LatTable ha, hb;
        half_tables(c->lt, ha, hb);
        const uint32_t k0 = (uint32_t)c->prm.seed, k1 = (uint32_t)(c->prm.seed >> 32);
        TimeScope ts(c, 0, 16);
        hipEventRecord(c->fork_ev, c->stream);
        hipStreamWaitEvent(c->side, c->fork_ev, 0);
        for (int j = 0; j < 16; ++j) {
            const int col = j & 7;
            if (j < 8) launch_hb_pass<T>(ha, (T*)c->state, c->ds, col, mode, kSweep, k0, k1, c->stream);
            else launch_or_pass<T>(ha, (T*)c->state, c->ds, col, 0, c->stream);
            if (hb.n_chains == 0) continue;
            if (j < 8) launch_or_pass<T>(hb, (T*)c->state, c->ds, col, 0, c->side);
            else launch_hb_pass<T>(hb, (T*)c->state, c->ds, col, mode, kSweep, k0, k1, c->side);
        }
        hipEventRecord(c->join_ev, c->side);
        hipStreamWaitEvent(c->stream, c->join_ev, 0);
    } else {
        {
            TimeScope ts(c, 0, 8);
            for (int col = 0; col < 8; ++col) enqueue_hb_pass<T>(c, col, mode, kSweep);
        }
        {
            TimeScope ts(c, 1, 8);
            for (int col = 0; col < 8; ++col) enqueue_or_pass<T>(c, col);
        }
    }
    if (recompute)
        enqueue_energy<T>(c, kCheckDrift | (mode == LLR_MODE_RESTRICTED || mode == LLR_MODE_LINK ? kCheckInterval : 0));
    if (replica) launch_replica(c->lt, c->ds, (uint32_t)c->prm.seed, (uint32_t)(c->prm.seed >> 32), c->stream);
    launch_end_sweep(c->lt, c->ds, measure ? 1 : 0, 0, 1, c->stream);
}

static llr_status ensure_link_buffers(llr_ctx* c);

// the heatbath mode of Algorithm 1's restricted sweeps
static int restricted_mode(const llr_ctx* c) { return c->per_link ? LLR_MODE_LINK : LLR_MODE_RESTRICTED; }

// One restricted sweep of the Robbins-Monro loop.  Without per-kernel timing
// the 18-20 launches of a sweep (10-12 in the interleaved order) are captured
// once per variant into a HIP graph
// (kernel nodes only) and replayed; the sweep index lives in device memory, so
// every replay advances it.
template <typename T>
static llr_status launch_sweep(llr_ctx* c, bool recompute, bool replica, bool measure) {
    if (c->per_link) {   // before any capture: the first use allocates
        const llr_status st = ensure_link_buffers(c);
        if (st != LLR_OK) return st;
    }
    if (!c->use_graphs || c->timing) {
        enqueue_sweep<T>(c, restricted_mode(c), recompute, replica, measure);
        return LLR_OK;
    }
    const int key = (recompute ? 1 : 0) | (replica ? 2 : 0) | (measure ? 4 : 0);
    if (!c->sweep_graph[key]) {
        // capture on a library-owned stream (the caller's may be the null
        // stream, which cannot be captured); the graph runs on the caller's
        if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e0 = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e0 == hipSuccess) {
            c->capturing = true;
            enqueue_sweep<T>(c, restricted_mode(c), recompute, replica, measure);
            c->capturing = false;
            e0 = hipStreamEndCapture(c->stream, &g);
        }
        c->stream = user;
        if (e0 != hipSuccess) return fail(LLR_EDEVICE, std::string("stream capture: ") + hipGetErrorString(e0));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return fail(LLR_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        c->sweep_graph[key] = ex;
    }
    HIPCHK(hipGraphLaunch(c->sweep_graph[key], c->stream));
    note_sweep(c, c->interleave && restricted_mode(c) == LLR_MODE_RESTRICTED);
    return LLR_OK;
}

template <typename T>
static void enqueue_approach_sweep(llr_ctx* c) {
    for (int col = 0; col < 8; ++col) enqueue_hb_pass<T>(c, col, LLR_MODE_APPROACH, kApproach);
    launch_end_sweep(c->lt, c->ds, 0, 1, 0, c->stream);
}

// Autotuner: class links per thread (1, 2, 4) of the heatbath and the
// overrelaxation pass, timed with HIP events on the bound state without
// changing it (heatbath in a never-accepting mode, overrelaxation writing to
// the non-current planes); the fastest per kernel is kept for the context.
template <typename T>
static llr_status autotune_impl(llr_ctx* c) {
    const int cand[3] = {1, 2, 4};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_hb = 1e30f, best_or = 1e30f;
    int bh = 1, bo = 1;
    const bool was_timing = c->timing;
    c->timing = false;
    for (int ci = 0; ci < 3; ++ci) {
        set_tiles(c->lt, cand[ci], cand[ci]);
        for (int rep = 0; rep < 4; ++rep) {   // first repetition warms up; minimum of the others
            HIPCHK(hipEventRecord(e0, c->stream));
            // the heatbath pass the sweeps run: fused with the overrelaxation
            // in the interleaved order
            for (int col = 0; col < 8; ++col) {
                if (c->interleave)
                    launch_hb_or_pass<T>(c->lt, (T*)c->state, c->ds, col, kHbModeTune, (uint32_t)c->prm.seed,
                                         (uint32_t)(c->prm.seed >> 32), c->stream);
                else
                    launch_hb_pass<T>(c->lt, (T*)c->state, c->ds, col, kHbModeTune, kSweep, (uint32_t)c->prm.seed,
                                      (uint32_t)(c->prm.seed >> 32), c->stream);
            }
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms < best_hb) { best_hb = ms; bh = cand[ci]; }
            HIPCHK(hipEventRecord(e0, c->stream));
            for (int col = 0; col < 8; ++col) launch_or_pass<T>(c->lt, (T*)c->state, c->ds, col, 1, c->stream);
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms < best_or) { best_or = ms; bo = cand[ci]; }
        }
    }
    set_tiles(c->lt, bh, bo);
    drop_graphs(c);
    c->timing = was_timing;
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    HIPCHK(hipGetLastError());
    c->tuned = true;
    return LLR_OK;
}

static llr_status need_state(llr_ctx* c) {
    if (!c) return fail(LLR_EINVAL, "null context");
    if (!c->laid_out || !c->state) return fail(LLR_ESTATE, "state not bound");
    return LLR_OK;
}

template <typename T>
static llr_status approach_check(llr_ctx* c, bool* all) {
    std::vector<int> outside(c->lt.n, 0);
    launch_approach_check(c->lt, c->ds, c->stream);
    HIPCHK(hipMemcpyAsync(outside.data(), c->ds.lat_outside, 4 * c->lt.n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *all = true;
    for (int i = 0; i < c->lt.n; ++i) {
        if (!c->ap_done[i] && outside[i] == 0) c->ap_done[i] = 1;
        *all = *all && c->ap_done[i];
    }
    HIPCHK(hipMemcpyAsync(c->ds.lat_done, c->ap_done.data(), 4 * c->lt.n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LLR_OK;
}

template <typename T>
static llr_status approach_begin_impl(llr_ctx* c) {
    launch_approach_init(c->lt, c->ds, c->stream);
    HIPCHK(hipMemsetAsync(c->ds.approach_ctr, 0, 4, c->stream));
    c->ap_done.assign(c->lt.n, 0);
    c->approach_sweeps.assign(c->lt.n, 0);
    enqueue_energy<T>(c);
    bool all = false;
    llr_status st = approach_check<T>(c, &all);
    if (st != LLR_OK) return st;
    c->ap_open = true;
    return LLR_OK;
}

// up to max_sweeps approach sweeps, in blocks of K followed by a recompute
template <typename T>
static llr_status approach_continue_impl(llr_ctx* c, long long max_sweeps, int* all_done) {
    if (!c->ap_open) return fail(LLR_ESTATE, "call llr_approach_begin first");
    const int K = std::max(1, c->prm.recompute_every);
    bool all = true;
    for (int i = 0; i < c->lt.n; ++i) all = all && c->ap_done[i];
    long long t = 0;
    while (!all && t < max_sweeps) {
        for (int j = 0; j < K; ++j) enqueue_approach_sweep<T>(c);
        enqueue_energy<T>(c);
        for (int i = 0; i < c->lt.n; ++i)
            if (!c->ap_done[i]) c->approach_sweeps[i] += K;
        t += K;
        llr_status st = approach_check<T>(c, &all);
        if (st != LLR_OK) return st;
    }
    HIPCHK(hipGetLastError());
    if (all_done) *all_done = all ? 1 : 0;
    return health_check(c);
}

template <typename T>
static llr_status approach_impl(llr_ctx* c, long long* sweeps) {
    llr_status st = approach_begin_impl<T>(c);
    if (st != LLR_OK) return st;
    int all = 0;
    st = approach_continue_impl<T>(c, c->prm.approach_cap, &all);
    if (sweeps) for (int i = 0; i < c->lt.n; ++i) sweeps[i] = c->approach_sweeps[i];
    if (st != LLR_OK) return st;
    if (!all) return fail(LLR_EAPPROACH, "approach cap reached before every chain entered its interval");
    return LLR_OK;
}

template <typename T> static llr_status autotune_impl(llr_ctx* c);

static llr_status need_even(const llr_ctx* c, const char* what) {
    for (size_t i = 0; i < c->lats.size(); ++i)
        if (!c->lats[i].even)
            return fail(LLR_EINVAL, std::string(what) + " needs evenly spaced interval edges E_k = E_0 + k dE (lattice " +
                                        std::to_string(i) + ")");
    return LLR_OK;
}

static llr_status rm_begin(llr_ctx* c) {
    if (!c->tuned) {
        llr_status st0 = c->precision == LLR_FP32 ? autotune_impl<float>(c) : autotune_impl<double>(c);
        if (st0 != LLR_OK) return st0;
    }
    const llr_params& p = c->prm;
    const int n = c->lt.n_chains;
    if (p.n_a < 1 || p.n_th < 0 || p.n_rm < 1) return fail(LLR_EINVAL, "need n_a >= 1, n_th >= 0, n_rm >= 1");
    if (c->ds.a_hist) {
        HIPCHK(hipFree(c->ds.a_hist));
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void*)c->ds.a_hist), c->allocs.end());
        c->ds.a_hist = nullptr;
    }
    llr_status st = dalloc(c, &c->ds.a_hist, (size_t)(p.n_rm + 1) * n);
    if (st != LLR_OK) return st;
    HIPCHK(hipMemcpyAsync(c->ds.a_hist, c->ds.a, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemsetAsync(c->ds.sumE, 0, 8 * n, c->stream));
    HIPCHK(hipMemsetAsync(c->ds.sweep_ctr, 0, 4, c->stream));
    HIPCHK(hipMemsetAsync(c->ds.rm_iter, 0, 4, c->stream));
    HIPCHK(hipMemsetAsync(c->ds.conv_iter, 0xff, 4 * n, c->stream));
    HIPCHK(hipMemsetAsync(c->ds.conv_sweeps, 0xff, 8 * n, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->rm_done = 0;
    c->rm_open = true;
    return LLR_OK;
}

template <typename T>
static llr_status rm_step_impl(llr_ctx* c, int iters) {
    const llr_params& p = c->prm;
    if (!c->rm_open) return fail(LLR_ESTATE, "call llr_rm_begin first");
    if (iters < 0 || c->rm_done + iters > p.n_rm) return fail(LLR_EINVAL, "more RM iterations than n_rm");
    const int K = std::max(1, p.recompute_every);
    const int nsw = p.n_th + p.n_a;
    RunCfg cfg{(uint32_t)p.seed, (uint32_t)(p.seed >> 32), p.n_a, nsw, p.eps};
    llr_status st = LLR_OK;
    for (int it = 0; it < iters; ++it) {
        for (int j = 0; j < nsw; ++j) {
            const bool rec = ((j + 1) % K == 0) || (j == nsw - 1);
            st = launch_sweep<T>(c, rec, p.replica_exchange != 0, j >= p.n_th);
            if (st != LLR_OK) return st;
            if ((j & 255) == 255) HIPCHK(hipStreamSynchronize(c->stream));   // bound the queue depth
        }
        launch_rm_update(c->lt, c->ds, cfg, c->stream);
        c->rm_done += 1;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    if (c->timing) harvest(c);
    return health_check(c);
}

static llr_status rm_converged(llr_ctx* c) {
    const int n = c->lt.n_chains;
    std::vector<int> conv(n);
    HIPCHK(hipMemcpy(conv.data(), c->ds.conv_iter, 4 * n, hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k)
        if (conv[k] < 0) return LLR_WARN_NOT_CONVERGED;
    return LLR_OK;
}

template <typename T>
static llr_status run_impl(llr_ctx* c) {
    llr_status st = rm_begin(c);
    if (st != LLR_OK) return st;
    st = rm_step_impl<T>(c, c->prm.n_rm);
    if (st != LLR_OK) return st;
    return rm_converged(c);
}

template <typename T>
static llr_status sweeps_impl(llr_ctx* c, int n_sweeps, long long sweep0, int mode, uint16_t* bits) {
    const uint32_t s0 = (uint32_t)sweep0;
    HIPCHK(hipMemcpyAsync(c->ds.sweep_ctr, &s0, 4, hipMemcpyHostToDevice, c->stream));
    const int n = c->lt.n_chains;
    for (int t = 0; t < n_sweeps; ++t) {
        enqueue_sweep<T>(c, mode, false, false, false);
        if (bits) {
            HIPCHK(hipMemcpyAsync(bits + (size_t)t * n, c->ds.bits_last, 2 * n, hipMemcpyDeviceToHost, c->stream));
        }
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    if (c->timing) harvest(c);
    return health_check(c);
}

template <typename T>
static llr_status muca_sweeps_impl(llr_ctx* c, int n_sweeps, long long sweep0, double* E_hist) {
    const uint32_t s0 = (uint32_t)sweep0;
    HIPCHK(hipMemcpyAsync(c->ds.sweep_ctr, &s0, 4, hipMemcpyHostToDevice, c->stream));
    const int n = c->lt.n_chains;
    const int K = c->prm.recompute_every;
    for (int t = 0; t < n_sweeps; ++t) {
        enqueue_sweep<T>(c, LLR_MODE_MUCA, K > 0 && (t + 1) % K == 0, false, false);
        if (E_hist) HIPCHK(hipMemcpyAsync(E_hist + (size_t)t * n, c->ds.E, 8 * (size_t)n, hipMemcpyDeviceToHost,
                                          c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    if (c->timing) harvest(c);
    return health_check(c);
}

template <typename T>
static llr_status observables_impl(llr_ctx* c, int n_meas, int gap, long long sweep0, double* E_out, double* B_out) {
    if (c->per_link) {
        const llr_status st = ensure_link_buffers(c);
        if (st != LLR_OK) return st;
    }
    const uint32_t s0 = (uint32_t)sweep0;
    HIPCHK(hipMemcpyAsync(c->ds.sweep_ctr, &s0, 4, hipMemcpyHostToDevice, c->stream));
    const int n = c->lt.n_chains;
    std::vector<double> E(n), B(n);
    std::vector<int> conf(n);
    for (int m = 0; m < n_meas; ++m) {
        for (int t = 0; t < gap; ++t)
            enqueue_sweep<T>(c, restricted_mode(c), false, c->prm.replica_exchange != 0, false);
        {
            TimeScope ts(c, 2);
            launch_energy<T>(c->lt, (const T*)c->state, c->ds, c->stream, true, kCheckDrift | kCheckInterval);
        }
        HIPCHK(hipMemcpyAsync(E.data(), c->ds.E, 8 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(B.data(), c->ds.obs, 8 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(conf.data(), c->ds.conf, 4 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int k = 0; k < n; ++k) {
            E_out[(size_t)m * n + k] = E[conf[k]];
            B_out[(size_t)m * n + k] = B[conf[k]];
        }
    }
    HIPCHK(hipGetLastError());
    if (c->timing) harvest(c);
    return health_check(c);
}

// ================================================================= C ABI
// Checks shared by llr_set_params, llr_add_lattice and the checkpoint reader.
static llr_status check_params(const llr_params& p) {
    if (p.n_a < 1 || p.n_th < 0 || p.n_rm < 0 || p.recompute_every < 1 || p.approach_cap < 0 || !(p.eps >= 0) ||
        !(p.overlap >= 0))
        return fail(LLR_EINVAL, "invalid parameters");
    return LLR_OK;
}

static llr_status check_lattice(int L, int n_intervals, const double* E_low, double dE) {
    if (L < 2 || L > 32 || (L & 1)) return fail(LLR_EINVAL, "L must be even and in [2, 32]");
    if (n_intervals < 1 || n_intervals > 4096) return fail(LLR_EINVAL, "n_intervals must be in [1, 4096]");
    if (!(dE > 0)) return fail(LLR_EINVAL, "dE must be > 0");
    const double six_v = 6.0 * (double)L * L * L * L;
    for (int k = 0; k < n_intervals; ++k) {
        if (!std::isfinite(E_low[k])) return fail(LLR_EINVAL, "non-finite interval edge");
        if (k && !(E_low[k] > E_low[k - 1])) return fail(LLR_EINVAL, "interval edges must ascend");
        if (E_low[k] < -six_v || E_low[k] + dE > six_v) return fail(LLR_EINVAL, "interval outside [-6V, 6V]");
    }
    return LLR_OK;
}

extern "C" {

const char* llr_last_error(void) { return g_err.c_str(); }

llr_status llr_create(llr_ctx** out, int hip_device, void* hip_stream, int precision) {
    if (!out) return fail(LLR_EINVAL, "out is null");
    if (precision != LLR_FP64 && precision != LLR_FP32) return fail(LLR_EINVAL, "precision must be LLR_FP64 or LLR_FP32");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
        return fail(LLR_EDEVICE, "no such HIP device");
    HIPCHK(hipSetDevice(hip_device));
    const llr_status sst = scratch_setup(hip_device);
    if (sst != LLR_OK) return sst;
    llr_ctx* c = new llr_ctx();
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    c->precision = precision;
    c->prm.n_th = 100;
    c->prm.n_a = 100;
    c->prm.n_rm = 20;
    c->prm.seed = 1509083910ull;
    c->prm.replica_exchange = 0;
    c->prm.overlap = 1.0;
    c->prm.recompute_every = 10;
    c->prm.eps = 1e-4;
    c->prm.approach_cap = 100000;
    *out = c;
    return LLR_OK;
}

void llr_destroy(llr_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    if (c->side) {
        hipStreamSynchronize(c->side);
        hipStreamDestroy(c->side);
    }
    if (c->fork_ev) hipEventDestroy(c->fork_ev);
    if (c->join_ev) hipEventDestroy(c->join_ev);
    for (auto& p : c->pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
    for (auto e : c->pool) hipEventDestroy(e);
    for (void* p : c->allocs) hipFree(p);
    if (c->stage) hipFree(c->stage);
    delete c;
}

llr_status llr_set_params(llr_ctx* c, const llr_params* p) {
    if (!c || !p) return fail(LLR_EINVAL, "null argument");
    if (check_params(*p) != LLR_OK) return LLR_EINVAL;
    const bool width_changed = c->laid_out && (p->replica_exchange != c->prm.replica_exchange || p->overlap != c->prm.overlap);
    c->prm = *p;
    drop_graphs(c);
    if (width_changed) return upload_intervals(c);
    return LLR_OK;
}

llr_status llr_add_lattice(llr_ctx* c, int L, int n_intervals, const double* E_low, double dE, int* lattice_id) {
    if (!c || !E_low) return fail(LLR_EINVAL, "null argument");
    if (c->laid_out) return fail(LLR_ESTATE, "lattices must be added before llr_state_bytes/llr_bind_state");
    if (check_lattice(L, n_intervals, E_low, dE) != LLR_OK) return LLR_EINVAL;
    if ((int)c->lats.size() >= kMaxLat) return fail(LLR_EINVAL, "at most 8 lattices");
    HostLat h;
    h.L = L;
    h.n = n_intervals;
    h.dE = dE;
    h.even = evenly_spaced(E_low, n_intervals, dE);
    h.E_low.assign(E_low, E_low + n_intervals);
    h.a0.assign(n_intervals, 1.0);
    c->lats.push_back(h);
    if (lattice_id) *lattice_id = (int)c->lats.size() - 1;
    return LLR_OK;
}

llr_status llr_state_bytes(llr_ctx* c, size_t* bytes) {
    if (!c || !bytes) return fail(LLR_EINVAL, "null argument");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = layout(c);
    if (st != LLR_OK) return st;
    *bytes = c->state_bytes;
    return LLR_OK;
}

llr_status llr_bind_state(llr_ctx* c, void* dev_state, size_t bytes) {
    if (!c || !dev_state) return fail(LLR_EINVAL, "null argument");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = layout(c);
    if (st != LLR_OK) return st;
    if (bytes != c->state_bytes) return fail(LLR_EINVAL, "state buffer size differs from llr_state_bytes");
    if (((uintptr_t)dev_state) & 255) return fail(LLR_EINVAL, "state buffer must be 256-byte aligned");
    drop_graphs(c);
    c->state = dev_state;
    c->have_energy = false;
    // every angle 0 (a cold start): the energy pass that follows the import of
    // one lattice covers all lattices, and an uninitialised one would feed it
    // values outside [-pi, pi) whose fixed-point sums overflow into the
    // per-chain arrival counters
    HIPCHK(hipMemsetAsync(dev_state, 0, bytes, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LLR_OK;
}

llr_status llr_set_a(llr_ctx* c, int lat, const double* a) {
    if (c) c->muca_ready = false;   // the multicanonical weights follow a_k
    if (!c || !a) return fail(LLR_EINVAL, "null argument");
    if (lat < 0 || lat >= (int)c->lats.size()) return fail(LLR_EINVAL, "no such lattice");
    for (int k = 0; k < c->lats[lat].n; ++k)
        if (!std::isfinite(a[k])) return fail(LLR_EINVAL, "non-finite a");
    c->lats[lat].a0.assign(a, a + c->lats[lat].n);
    if (c->laid_out) {
        HIPCHK(hipSetDevice(c->device));
        HIPCHK(hipMemcpyAsync(c->ds.a + c->lt.l[lat].chain0, a, 8 * c->lats[lat].n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return LLR_OK;
}

llr_status llr_hot_start(llr_ctx* c) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    const uint32_t k0 = (uint32_t)c->prm.seed, k1 = (uint32_t)(c->prm.seed >> 32);
    if (c->precision == LLR_FP32) {
        launch_hot_start<float>(c->lt, (float*)c->state, c->ds, k0, k1, c->stream);
        enqueue_energy<float>(c, 0);
    } else {
        launch_hot_start<double>(c->lt, (double*)c->state, c->ds, k0, k1, c->stream);
        enqueue_energy<double>(c, 0);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    c->have_energy = true;
    return LLR_OK;
}

llr_status llr_import_state(llr_ctx* c, int lat, const void* dev) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (lat < 0 || lat >= c->lt.n || !dev) return fail(LLR_EINVAL, "bad lattice or pointer");
    HIPCHK(hipSetDevice(c->device));
    if (c->precision == LLR_FP32) {
        launch_import<float>(c->lt, lat, (float*)c->state, c->ds, (const float*)dev, c->stream);
        enqueue_energy<float>(c, 0);
    } else {
        launch_import<double>(c->lt, lat, (double*)c->state, c->ds, (const double*)dev, c->stream);
        enqueue_energy<double>(c, 0);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    c->have_energy = true;
    return LLR_OK;
}

llr_status llr_export_state(llr_ctx* c, int lat, void* dev) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (lat < 0 || lat >= c->lt.n || !dev) return fail(LLR_EINVAL, "bad lattice or pointer");
    HIPCHK(hipSetDevice(c->device));
    if (c->precision == LLR_FP32)
        launch_export<float>(c->lt, lat, (const float*)c->state, c->ds, (float*)dev, c->stream);
    else
        launch_export<double>(c->lt, lat, (const double*)c->state, c->ds, (double*)dev, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_approach(llr_ctx* c, long long* sweeps) {
    RunClock clk(c);
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    return c->precision == LLR_FP32 ? approach_impl<float>(c, sweeps) : approach_impl<double>(c, sweeps);
}

llr_status llr_approach_begin(llr_ctx* c) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    return c->precision == LLR_FP32 ? approach_begin_impl<float>(c) : approach_begin_impl<double>(c);
}

llr_status llr_approach_continue(llr_ctx* c, long long max_sweeps, long long* sweeps, int* all_done) {
    RunClock clk(c);
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (max_sweeps < 0) return fail(LLR_EINVAL, "max_sweeps < 0");
    HIPCHK(hipSetDevice(c->device));
    st = c->precision == LLR_FP32 ? approach_continue_impl<float>(c, max_sweeps, all_done)
                                  : approach_continue_impl<double>(c, max_sweeps, all_done);
    if (sweeps) for (int i = 0; i < c->lt.n; ++i) sweeps[i] = c->approach_sweeps[i];
    return st;
}

llr_status llr_run(llr_ctx* c) {
    RunClock clk(c);
    if (c) c->muca_ready = false;   // the multicanonical weights follow a_k
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    return c->precision == LLR_FP32 ? run_impl<float>(c) : run_impl<double>(c);
}

llr_status llr_rm_begin(llr_ctx* c) {
    if (c) c->muca_ready = false;   // the multicanonical weights follow a_k
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    return rm_begin(c);
}

llr_status llr_rm_step(llr_ctx* c, int iterations) {
    RunClock clk(c);
    if (c) c->muca_ready = false;   // the multicanonical weights follow a_k
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    st = c->precision == LLR_FP32 ? rm_step_impl<float>(c, iterations) : rm_step_impl<double>(c, iterations);
    if (st != LLR_OK) return st;
    return c->rm_done == c->prm.n_rm ? rm_converged(c) : LLR_OK;
}

llr_status llr_autotune(llr_ctx* c, int* hb_lpt, int* or_lpt) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (!c->have_energy) return fail(LLR_ESTATE, "initialise the state (hot start or import) before tuning");
    HIPCHK(hipSetDevice(c->device));
    st = c->precision == LLR_FP32 ? autotune_impl<float>(c) : autotune_impl<double>(c);
    if (st != LLR_OK) return st;
    if (hb_lpt) *hb_lpt = c->lt.hb_lpt;
    if (or_lpt) *or_lpt = c->lt.or_lpt;
    return LLR_OK;
}

llr_status llr_set_graphs(llr_ctx* c, int on) {
    if (!c) return fail(LLR_EINVAL, "null context");
    c->use_graphs = on != 0;
    drop_graphs(c);
    return LLR_OK;
}

llr_status llr_set_order(llr_ctx* c, int serpentine) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "lay out the lattices first");
    c->lt.serpentine = serpentine ? 1 : 0;
    drop_graphs(c);
    return LLR_OK;
}

}  // extern "C"

// The staggered order's second stream and its fork / join events.
// All three are created or none is kept, so c->side set means all exist.
static llr_status ensure_side_stream(llr_ctx* c) {
    if (c->side) return LLR_OK;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = nullptr;
    hipEvent_t fe = nullptr, je = nullptr;
    hipError_t e = hipEventCreateWithFlags(&fe, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&je, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (fe) hipEventDestroy(fe);
        if (je) hipEventDestroy(je);
        return fail(LLR_EDEVICE, std::string("second stream: ") + hipGetErrorString(e));
    }
    c->fork_ev = fe;
    c->join_ev = je;
    c->side = st;
    return LLR_OK;
}

extern "C" {

llr_status llr_set_sweep_order(llr_ctx* c, int order) {
    if (!c) return fail(LLR_EINVAL, "null context");
    if (order != LLR_SWEEP_GROUPED && order != LLR_SWEEP_INTERLEAVED && order != LLR_SWEEP_STAGGERED)
        return fail(LLR_EINVAL, "order must be LLR_SWEEP_GROUPED, LLR_SWEEP_INTERLEAVED or LLR_SWEEP_STAGGERED");
    if (order == LLR_SWEEP_STAGGERED) {
        const llr_status st = ensure_side_stream(c);
        if (st != LLR_OK) return st;
    }
    if (c->interleave != (order == LLR_SWEEP_INTERLEAVED) || c->stagger != (order == LLR_SWEEP_STAGGERED)) {
        c->interleave = order == LLR_SWEEP_INTERLEAVED;
        c->stagger = order == LLR_SWEEP_STAGGERED;
        drop_graphs(c);   // the captured sweeps hold the pass sequence
    }
    return LLR_OK;
}

llr_status llr_set_tiles(llr_ctx* c, int hb_lpt, int or_lpt) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "lay out the lattices first");
    auto ok = [](int v) { return v == 1 || v == 2 || v == 4; };
    if (!ok(hb_lpt) || !ok(or_lpt)) return fail(LLR_EINVAL, "links per thread must be 1, 2 or 4");
    set_tiles(c->lt, hb_lpt, or_lpt);
    drop_graphs(c);
    c->tuned = true;
    return LLR_OK;
}

// Per-class-link buffers of the per-link constraint, allocated on first use:
// the candidates' fixed-point Delta E and the staples and old angle of every
// class link of one colour, for all chains.
static llr_status ensure_link_buffers(llr_ctx* c) {
    if (c->ds.link_d && c->ds.link_cst) return LLR_OK;
    llr_status st;
    if (!c->ds.link_d && (st = dalloc(c, &c->ds.link_d, (size_t)c->ds.link_n)) != LLR_OK) return st;
    unsigned char* p = nullptr;
    if ((st = dalloc(c, &p, 3 * (size_t)c->ds.link_n * elem_size(c))) != LLR_OK) return st;
    c->ds.link_cst = p;
    drop_graphs(c);   // captured sweeps hold the device-state table by value
    return LLR_OK;
}

static bool sweep_mode_ok(int mode) { return mode == LLR_MODE_RESTRICTED || mode == LLR_MODE_FREE || mode == LLR_MODE_LINK; }

llr_status llr_sweeps(llr_ctx* c, int n_sweeps, long long sweep0, int mode, uint16_t* bits) {
    RunClock clk(c);
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (n_sweeps < 0 || !(sweep_mode_ok(mode) || mode == LLR_MODE_APPROACH))
        return fail(LLR_EINVAL, "bad n_sweeps or mode");
    HIPCHK(hipSetDevice(c->device));
    if (mode == LLR_MODE_LINK && (st = ensure_link_buffers(c)) != LLR_OK) return st;
    return c->precision == LLR_FP32 ? sweeps_impl<float>(c, n_sweeps, sweep0, mode, bits)
                                    : sweeps_impl<double>(c, n_sweeps, sweep0, mode, bits);
}

llr_status llr_class_pass(llr_ctx* c, int heatbath, int colour, int mode, long long sweep_index) {
    RunClock clk(c);
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (colour < 0 || colour > 7 || !(sweep_mode_ok(mode) || mode == LLR_MODE_APPROACH))
        return fail(LLR_EINVAL, "bad colour or mode");
    HIPCHK(hipSetDevice(c->device));
    if (heatbath && mode == LLR_MODE_LINK && (st = ensure_link_buffers(c)) != LLR_OK) return st;
    const uint32_t s0 = (uint32_t)sweep_index;
    HIPCHK(hipMemcpyAsync(c->ds.sweep_ctr, &s0, 4, hipMemcpyHostToDevice, c->stream));
    if (c->precision == LLR_FP32) {
        if (heatbath) enqueue_hb_pass<float>(c, colour, mode, kSweep);
        else enqueue_or_pass<float>(c, colour);
    } else {
        if (heatbath) enqueue_hb_pass<double>(c, colour, mode, kSweep);
        else enqueue_or_pass<double>(c, colour);
    }
    if (!heatbath) c->or_passes += 1;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_recompute_energy(llr_ctx* c) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    if (c->precision == LLR_FP32) enqueue_energy<float>(c);
    else enqueue_energy<double>(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return health_check(c);
}

llr_status llr_get_a(llr_ctx* c, int lat, double* a, int* conv_iter, long long* conv_sweeps) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "no state");
    if (lat < 0 || lat >= c->lt.n) return fail(LLR_EINVAL, "no such lattice");
    HIPCHK(hipSetDevice(c->device));
    const LatDev& L = c->lt.l[lat];
    HIPCHK(hipStreamSynchronize(c->stream));
    if (a) HIPCHK(hipMemcpy(a, c->ds.a + L.chain0, 8 * L.n_chains, hipMemcpyDeviceToHost));
    if (conv_iter) HIPCHK(hipMemcpy(conv_iter, c->ds.conv_iter + L.chain0, 4 * L.n_chains, hipMemcpyDeviceToHost));
    if (conv_sweeps) {
        HIPCHK(hipMemcpy(conv_sweeps, c->ds.conv_sweeps + L.chain0, 8 * L.n_chains, hipMemcpyDeviceToHost));
        for (int k = 0; k < L.n_chains; ++k)
            if (conv_sweeps[k] >= 0) conv_sweeps[k] += c->approach_sweeps[lat];
    }
    return LLR_OK;
}

llr_status llr_get_history(llr_ctx* c, int lat, double* a_hist) {
    if (!c || !c->laid_out || !c->ds.a_hist) return fail(LLR_ESTATE, "no run");
    if (lat < 0 || lat >= c->lt.n || !a_hist) return fail(LLR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(c->device));
    const LatDev& L = c->lt.l[lat];
    const int n = c->lt.n_chains;
    std::vector<double> all((size_t)(c->prm.n_rm + 1) * n);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(all.data(), c->ds.a_hist, 8 * all.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r <= c->prm.n_rm; ++r)
        for (int k = 0; k < L.n_chains; ++k) a_hist[(size_t)r * L.n_chains + k] = all[(size_t)r * n + L.chain0 + k];
    return LLR_OK;
}

llr_status llr_get_energy(llr_ctx* c, int lat, double* E, int* conf) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "no state");
    if (lat < 0 || lat >= c->lt.n) return fail(LLR_EINVAL, "no such lattice");
    HIPCHK(hipSetDevice(c->device));
    const LatDev& L = c->lt.l[lat];
    HIPCHK(hipStreamSynchronize(c->stream));
    if (E) HIPCHK(hipMemcpy(E, c->ds.E + L.chain0, 8 * L.n_chains, hipMemcpyDeviceToHost));
    if (conf) {
        HIPCHK(hipMemcpy(conf, c->ds.conf + L.chain0, 4 * L.n_chains, hipMemcpyDeviceToHost));
        for (int k = 0; k < L.n_chains; ++k) conf[k] -= L.chain0;
    }
    return LLR_OK;
}

llr_status llr_get_ln_rho(llr_ctx* c, int lat, double* centres, double* ln_rho) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "no state");
    if (lat < 0 || lat >= c->lt.n || !ln_rho) return fail(LLR_EINVAL, "bad argument");
    if (!c->lats[lat].even) return fail(LLR_EINVAL, "ln rho needs evenly spaced interval edges E_k = E_0 + k dE");
    HIPCHK(hipSetDevice(c->device));
    const HostLat& h = c->lats[lat];
    const int n = h.n;
    llr_status st = ensure_stage(c, 16 * (size_t)n + 64);
    if (st != LLR_OK) return st;
    double* d = (double*)c->stage;
    launch_recon(nullptr, c->ds.a + c->lt.l[lat].chain0, n, h.dE, 1.0, nullptr, 0, d, nullptr, nullptr, c->stream);
    HIPCHK(hipMemcpyAsync(ln_rho, d, 8 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (centres)
        for (int k = 0; k < n; ++k) centres[k] = h.E_low[k] + 0.5 * h.dE;
    return LLR_OK;
}

llr_status llr_enable_bits_log(llr_ctx* c, long long max_rows) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "lay out the lattices first");
    if (max_rows < 0) return fail(LLR_EINVAL, "max_rows < 0");
    HIPCHK(hipSetDevice(c->device));
    if (c->ds.bits_log) {
        HIPCHK(hipFree(c->ds.bits_log));
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void*)c->ds.bits_log), c->allocs.end());
        c->ds.bits_log = nullptr;
    }
    drop_graphs(c);
    c->ds.bits_rows_max = max_rows;
    if (max_rows > 0) {
        llr_status st = dalloc(c, &c->ds.bits_log, (size_t)max_rows * c->lt.n_chains);
        if (st != LLR_OK) return st;
    }
    HIPCHK(hipMemsetAsync(c->ds.bits_row, 0, 8, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LLR_OK;
}

llr_status llr_get_bits_log(llr_ctx* c, uint16_t* bits, long long* rows) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "no state");
    HIPCHK(hipSetDevice(c->device));
    long long r = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&r, c->ds.bits_row, 8, hipMemcpyDeviceToHost));
    r = std::min(r, c->ds.bits_rows_max);
    if (rows) *rows = r;
    if (bits && r > 0) HIPCHK(hipMemcpy(bits, c->ds.bits_log, 2 * (size_t)r * c->lt.n_chains, hipMemcpyDeviceToHost));
    return LLR_OK;
}

llr_status llr_stats(llr_ctx* c, long long* hb_prop, long long* hb_acc, long long* re_prop, long long* re_acc) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "no state");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int n = c->lt.n_chains;
    if (hb_prop) HIPCHK(hipMemcpy(hb_prop, c->ds.hb_prop, 8 * n, hipMemcpyDeviceToHost));
    if (hb_acc) HIPCHK(hipMemcpy(hb_acc, c->ds.hb_acc, 8 * n, hipMemcpyDeviceToHost));
    unsigned long long re[2] = {0, 0};
    HIPCHK(hipMemcpy(re, c->ds.re_cnt, 16, hipMemcpyDeviceToHost));
    if (re_prop) *re_prop = (long long)re[0];
    if (re_acc) *re_acc = (long long)re[1];
    return LLR_OK;
}

llr_status llr_get_rates(llr_ctx* c, llr_rates* out) {
    if (!c || !out) return fail(LLR_EINVAL, "null argument");
    if (!c->laid_out) return fail(LLR_ESTATE, "no state");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int n = c->lt.n_chains;
    std::vector<unsigned long long> hp(n), ha(n), fa(n), re(2);
    HIPCHK(hipMemcpy(hp.data(), c->ds.hb_prop, 8 * (size_t)n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ha.data(), c->ds.hb_acc, 8 * (size_t)n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(fa.data(), c->ds.fu_acc, 8 * (size_t)n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(re.data(), c->ds.re_cnt, 16, hipMemcpyDeviceToHost));
    llr_rates r{};
    r.sweeps = c->sweeps_run;
    double links = 0.0;   // link updates
    long long fused_acc = 0;
    for (int i = 0; i < c->lt.n; ++i) {
        const LatDev& L = c->lt.l[i];
        const double half = (double)L.V2;   // class links of one chain in one class pass
        for (int k = 0; k < L.n_chains; ++k) {
            const int g = L.chain0 + k;
            r.hb_class_passes += (long long)hp[g];
            r.hb_class_accepts += (long long)ha[g];
            fused_acc += (long long)fa[g];
            // every heatbath class pass updates its V/2 links; every
            // overrelaxation class pass too, except the one fused after an
            // accepted heatbath of its class (a relabelled draw)
            links += half * ((double)hp[g] + (double)(c->or_passes + c->fused_passes) - (double)fa[g]);
        }
    }
    r.or_class_passes = (c->or_passes + c->fused_passes) * (long long)n;
    r.or_class_relabelled = fused_acc;
    r.re_proposals = (long long)re[0];
    r.re_accepts = (long long)re[1];
    r.link_updates = links;
    r.seconds = c->run_seconds;
    r.link_updates_per_s = c->run_seconds > 0 ? links / c->run_seconds : 0.0;
    r.hb_acceptance = r.hb_class_passes ? (double)r.hb_class_accepts / (double)r.hb_class_passes : 0.0;
    r.or_acceptance = 1.0;
    r.re_acceptance = r.re_proposals ? (double)r.re_accepts / (double)r.re_proposals : 0.0;
    *out = r;
    return LLR_OK;
}

llr_status llr_health(llr_ctx* c, uint32_t* flags, double* drift, int clear) {
    if (!c) return fail(LLR_EINVAL, "null context");
    if (!c->laid_out) return fail(LLR_ESTATE, "no state");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int n = c->lt.n_chains;
    if (flags) HIPCHK(hipMemcpy(flags, c->ds.health, 4 * (size_t)n, hipMemcpyDeviceToHost));
    if (drift) HIPCHK(hipMemcpy(drift, c->ds.drift, 8 * (size_t)n, hipMemcpyDeviceToHost));
    if (clear) {
        HIPCHK(hipMemsetAsync(c->ds.health, 0, 4 * (size_t)n, c->stream));
        HIPCHK(hipMemsetAsync(c->ds.drift, 0, 8 * (size_t)n, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return LLR_OK;
}

llr_status llr_set_restriction(llr_ctx* c, int per_link) {
    if (!c) return fail(LLR_EINVAL, "null context");
    if (per_link != 0 && per_link != 1) return fail(LLR_EINVAL, "per_link must be 0 or 1");
    if (c->per_link != (per_link != 0)) {
        c->per_link = per_link != 0;
        drop_graphs(c);   // the captured sweeps hold the heatbath mode
    }
    return LLR_OK;
}

llr_status llr_link_stats(llr_ctx* c, long long* redrawn, long long* arc) {
    if (!c || !c->laid_out) return fail(LLR_ESTATE, "no state");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int n = c->lt.n_chains;
    if (redrawn) HIPCHK(hipMemcpy(redrawn, c->ds.link_fix, 8 * n, hipMemcpyDeviceToHost));
    if (arc) HIPCHK(hipMemcpy(arc, c->ds.link_arc, 8 * n, hipMemcpyDeviceToHost));
    return LLR_OK;
}

llr_status llr_set_timing(llr_ctx* c, int on) {
    if (!c) return fail(LLR_EINVAL, "null context");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    harvest(c);
    c->timing = on != 0;
    for (int i = 0; i < 3; ++i) { c->t_ms[i] = 0; c->t_n[i] = 0; }
    return LLR_OK;
}

llr_status llr_get_timing(llr_ctx* c, double* hb_ms, long long* hb_n, double* or_ms, long long* or_n, double* en_ms,
                          long long* en_n) {
    if (!c) return fail(LLR_EINVAL, "null context");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    harvest(c);
    if (hb_ms) *hb_ms = c->t_ms[0];
    if (hb_n) *hb_n = c->t_n[0];
    if (or_ms) *or_ms = c->t_ms[1];
    if (or_n) *or_n = c->t_n[1];
    if (en_ms) *en_ms = c->t_ms[2];
    if (en_n) *en_n = c->t_n[2];
    return LLR_OK;
}

llr_status llr_test_philox(llr_ctx* c, long n, const uint32_t* ctr, uint64_t seed, uint32_t* out) {
    if (!c || !ctr || !out || n < 0) return fail(LLR_EINVAL, "bad argument");
    if (n == 0) return LLR_OK;
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 32 * (size_t)n);
    if (st != LLR_OK) return st;
    uint4* d = (uint4*)c->stage;
    HIPCHK(hipMemcpyAsync(d, ctr, 16 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    launch_test_philox(n, d, (uint32_t)seed, (uint32_t)(seed >> 32), d + n, c->stream);
    HIPCHK(hipMemcpyAsync(out, d + n, 16 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_test_vonmises(llr_ctx* c, long n, double kappa, uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                             double* X, int* attempts) {
    if (!c || !X || !attempts || n < 0 || !(kappa >= 0)) return fail(LLR_EINVAL, "bad argument");
    if (n == 0) return LLR_OK;
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 12 * (size_t)n + 64);
    if (st != LLR_OK) return st;
    double* dX = (double*)c->stage;
    int* dA = (int*)(dX + n);
    if (c->precision == LLR_FP32)
        launch_test_vonmises<float>(n, kappa, (uint32_t)seed, (uint32_t)(seed >> 32), c1, c2, c3, dX, dA, c->stream);
    else
        launch_test_vonmises<double>(n, kappa, (uint32_t)seed, (uint32_t)(seed >> 32), c1, c2, c3, dX, dA, c->stream);
    HIPCHK(hipMemcpyAsync(X, dX, 8 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(attempts, dA, 4 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_reconstruct(llr_ctx* c, const double* centres, const double* a, int n, double s, double six_v,
                           const double* beta, int nb, double* ln_rho, double* u_mean, double* cv) {
    if (!c || !centres || !a || n < 1 || nb < 0 || !(s > 0) || !(six_v > 0)) return fail(LLR_EINVAL, "bad argument");
    if (nb > 0 && (!beta || !u_mean || !cv)) return fail(LLR_EINVAL, "bad beta arrays");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 8 * (size_t)(3 * n + 3 * nb) + 64);
    if (st != LLR_OK) return st;
    double* dc = (double*)c->stage;
    double* da = dc + n;
    double* dl = da + n;
    double* db = dl + n;
    double* du = db + nb;
    double* dv = du + nb;
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * n, hipMemcpyHostToDevice, c->stream));
    if (nb) HIPCHK(hipMemcpyAsync(db, beta, 8 * nb, hipMemcpyHostToDevice, c->stream));
    launch_recon(dc, da, n, s, six_v, db, nb, dl, du, dv, c->stream);
    if (ln_rho) HIPCHK(hipMemcpyAsync(ln_rho, dl, 8 * n, hipMemcpyDeviceToHost, c->stream));
    if (nb) {
        HIPCHK(hipMemcpyAsync(u_mean, du, 8 * nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(cv, dv, 8 * nb, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_beta_c(llr_ctx* c, const double* centres, const double* a, int n, double s, double six_v, double blo,
                      double bhi, double h, double tol, double* beta_c, double* cv_peak) {
    if (!c || !centres || !a || n < 1 || !(s > 0) || !(six_v > 0) || !(bhi > blo) || !(h > 0) || !(tol > 0) ||
        !beta_c || !cv_peak)
        return fail(LLR_EINVAL, "bad argument");
    const long ng = (long)std::floor((bhi - blo) / h + 0.5);
    if (ng > 10000000) return fail(LLR_EINVAL, "beta grid too fine");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 8 * (size_t)(3 * n + ng + 8) + 64);
    if (st != LLR_OK) return st;
    double* dc = (double*)c->stage;
    double* da = dc + n;
    double* out = da + n;
    double* scr = out + 4;
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * n, hipMemcpyHostToDevice, c->stream));
    launch_beta_c(dc, da, n, s, six_v, blo, bhi, h, tol, scr, out, c->stream);
    double r[2];
    HIPCHK(hipMemcpyAsync(r, out, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    *beta_c = r[0];
    *cv_peak = r[1];
    return LLR_OK;
}

llr_status llr_beta_c_noalloc(llr_ctx* c, const double* centres, const double* a, int n, double s, double six_v,
                              double blo, double bhi, double h, double tol, double* beta_c, double* cv_peak) {
    if (!c || !centres || !a || n < 1 || !(s > 0) || !(six_v > 0) || !(bhi > blo) || !(h > 0) || !(tol > 0) ||
        !beta_c || !cv_peak)
        return fail(LLR_EINVAL, "bad argument");
    const double ngd = std::floor((bhi - blo) / h + 0.5);
    // centres, a, the (beta_c, peak) pair, ln rho and the grid of ng + 1 variances
    const double need = 8.0 * (3.0 * (double)n + ngd + 8.0);
    if (!(need <= (double)kNoAllocBytes))
        return fail(LLR_EINVAL, "llr_beta_c_noalloc: 8 (3 n + ng + 8) = " + std::to_string((long long)need) +
                                    " bytes exceed its fixed 1 MiB device buffer");
    void* base = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
    if (!base) return fail(LLR_ESTATE, "no fixed device buffer for this context's device");
    HIPCHK(hipSetDevice(c->device));
    double* dc = (double*)base;
    double* da = dc + n;
    double* out = da + n;
    double* scr = out + 4;
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    launch_beta_c(dc, da, n, s, six_v, blo, bhi, h, tol, scr, out, c->stream);
    double r[2];
    HIPCHK(hipMemcpyAsync(r, out, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    *beta_c = r[0];
    *cv_peak = r[1];
    return LLR_OK;
}

static bool uniform_centres(const double* c, int n, double s) {
    for (int k = 0; k + 1 < n; ++k)
        if (!(std::fabs(c[k + 1] - c[k] - s) <= 1e-9 * std::max(1.0, std::fabs(s)))) return false;
    return true;
}

llr_status llr_observables(llr_ctx* c, int n_meas, int gap, long long sweep0, double* E, double* B) {
    RunClock clk(c);
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (n_meas < 1 || gap < 1 || !E || !B) return fail(LLR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(c->device));
    return c->precision == LLR_FP32 ? observables_impl<float>(c, n_meas, gap, sweep0, E, B)
                                    : observables_impl<double>(c, n_meas, gap, sweep0, E, B);
}

llr_status llr_obs_reconstruct(llr_ctx* c, const double* centres, const double* a, int n, double s, const double* E,
                               const double* B, int m, const double* beta, int nb, double* B_mean) {
    if (!c || !centres || !a || n < 1 || !(s > 0) || !E || !B || m < 1 || !beta || nb < 1 || !B_mean)
        return fail(LLR_EINVAL, "bad argument");
    if (!uniform_centres(centres, n, s)) return fail(LLR_EINVAL, "centres must be spaced by s");
    HIPCHK(hipSetDevice(c->device));
    const size_t mn = (size_t)m * n;
    llr_status st = ensure_stage(c, 8 * (2 * mn + 3 * (size_t)n + 2 * (size_t)nb) + 64);
    if (st != LLR_OK) return st;
    double* dE = (double*)c->stage;
    double* dB = dE + mn;
    double* dc = dB + mn;
    double* da = dc + n;
    double* dL = da + n;
    double* db = dL + n;
    double* dout = db + nb;
    HIPCHK(hipMemcpyAsync(dE, E, 8 * mn, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dB, B, 8 * mn, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(db, beta, 8 * (size_t)nb, hipMemcpyHostToDevice, c->stream));
    launch_obs_bracket(dE, dB, m, dc, da, n, s, db, nb, dout, dL, c->stream);
    HIPCHK(hipMemcpyAsync(B_mean, dout, 8 * (size_t)nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_muca_begin(llr_ctx* c, const double* b) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (!b) return fail(LLR_EINVAL, "null coupling array");
    if ((st = need_even(c, "the multicanonical weight")) != LLR_OK) return st;
    for (int i = 0; i < c->lt.n; ++i)
        if (!std::isfinite(b[i]) || b[i] < 0) return fail(LLR_EINVAL, "proposal couplings must be finite and >= 0");
    HIPCHK(hipSetDevice(c->device));
    for (int i = 0; i < c->lt.n; ++i) {
        const LatDev& L = c->lt.l[i];
        launch_recon(nullptr, c->ds.a + L.chain0, L.n_chains, L.ds, 1.0, nullptr, 0, c->ds.mu_lnrho + L.chain0,
                     nullptr, nullptr, c->stream);
    }
    HIPCHK(hipMemcpyAsync(c->ds.mu_b, b, 8 * (size_t)c->lt.n, hipMemcpyHostToDevice, c->stream));
    if (c->precision == LLR_FP32) enqueue_energy<float>(c);
    else enqueue_energy<double>(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    c->muca_ready = true;
    return LLR_OK;
}

llr_status llr_muca_sweeps(llr_ctx* c, int n_sweeps, long long sweep0, double* E_hist) {
    RunClock clk(c);
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (!c->muca_ready) return fail(LLR_ESTATE, "call llr_muca_begin first");
    if (n_sweeps < 0) return fail(LLR_EINVAL, "bad n_sweeps");
    HIPCHK(hipSetDevice(c->device));
    return c->precision == LLR_FP32 ? muca_sweeps_impl<float>(c, n_sweeps, sweep0, E_hist)
                                    : muca_sweeps_impl<double>(c, n_sweeps, sweep0, E_hist);
}

llr_status llr_muca_reweight(llr_ctx* c, const double* E, long m, const double* centres, const double* a, int n,
                             double s, double six_v, const double* beta, int nb, double* u_mean, double* cv) {
    if (!c || !E || m < 1 || !centres || !a || n < 1 || !(s > 0) || !(six_v > 0) || nb < 1 || !beta || !u_mean ||
        !cv)
        return fail(LLR_EINVAL, "bad argument");
    if (!uniform_centres(centres, n, s)) return fail(LLR_EINVAL, "centres must be spaced by s");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 8 * ((size_t)m + 3 * (size_t)n + 3 * (size_t)nb) + 64);
    if (st != LLR_OK) return st;
    double* dE = (double*)c->stage;
    double* dc = dE + m;
    double* da = dc + n;
    double* dL = da + n;
    double* db = dL + n;
    double* du = db + nb;
    double* dv = du + nb;
    HIPCHK(hipMemcpyAsync(dE, E, 8 * (size_t)m, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(db, beta, 8 * (size_t)nb, hipMemcpyHostToDevice, c->stream));
    launch_reweight(dE, m, dc, da, n, s, db, nb, six_v, du, dv, dL, c->stream);
    HIPCHK(hipMemcpyAsync(u_mean, du, 8 * (size_t)nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(cv, dv, 8 * (size_t)nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}


llr_status llr_prob_density(llr_ctx* c, const double* centres, const double* a, int n, double s, double beta,
                            const double* E, int m, double* log_p) {
    if (!c || !centres || !a || n < 1 || !(s > 0) || !std::isfinite(beta) || m < 0 || (m > 0 && (!E || !log_p)))
        return fail(LLR_EINVAL, "bad argument");
    if (!uniform_centres(centres, n, s)) return fail(LLR_EINVAL, "centres must be spaced by s");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 8 * (size_t)(3 * n + 2 * m + 4) + 64);
    if (st != LLR_OK) return st;
    double* dc = (double*)c->stage;
    double* da = dc + n;
    double* dE = da + n;
    double* dp = dE + m;
    double* scr = dp + m;
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    if (m) HIPCHK(hipMemcpyAsync(dE, E, 8 * (size_t)m, hipMemcpyHostToDevice, c->stream));
    launch_prob(dc, da, n, s, beta, dE, m, dp, 0, nullptr, nullptr, nullptr, scr, c->stream);
    if (m) HIPCHK(hipMemcpyAsync(log_p, dp, 8 * (size_t)m, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_prob_peaks(llr_ctx* c, const double* centres, const double* a, int n, double s, double beta,
                          int max_peaks, double* E_peak, double* log_p_peak, int* n_found) {
    if (!c || !centres || !a || n < 1 || !(s > 0) || !std::isfinite(beta) || max_peaks < 0 || !n_found ||
        (max_peaks > 0 && (!E_peak || !log_p_peak)))
        return fail(LLR_EINVAL, "bad argument");
    if (!uniform_centres(centres, n, s)) return fail(LLR_EINVAL, "centres must be spaced by s");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 8 * (size_t)(3 * n + 2 * max_peaks + 8) + 64);
    if (st != LLR_OK) return st;
    double* dc = (double*)c->stage;
    double* da = dc + n;
    double* dEp = da + n;
    double* dlp = dEp + max_peaks;
    int* dn = (int*)(dlp + max_peaks);
    double* scr = dlp + max_peaks + 2;
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(da, a, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    launch_prob(dc, da, n, s, beta, nullptr, 0, nullptr, max_peaks, dEp, dlp, dn, scr, c->stream);
    int nf = 0;
    HIPCHK(hipMemcpyAsync(&nf, dn, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int keep = std::min(nf, max_peaks);
    if (keep > 0) {
        HIPCHK(hipMemcpy(E_peak, dEp, 8 * (size_t)keep, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(log_p_peak, dlp, 8 * (size_t)keep, hipMemcpyDeviceToHost));
    }
    HIPCHK(hipGetLastError());
    *n_found = nf;
    return LLR_OK;
}

llr_status llr_bootstrap(llr_ctx* c, const double* centres, const double* a_runs, int n_runs, int n, double s,
                         double six_v, double blo, double bhi, double h, double tol, int n_boot, uint64_t seed,
                         double* beta_c, double* cv_peak) {
    if (!c || !centres || !a_runs || n < 1 || n_runs < 1 || n_runs > 1024 || n_boot < 1 || !(s > 0) ||
        !(six_v > 0) || !(bhi > blo) || !(h > 0) || !(tol > 0) || !beta_c || !cv_peak)
        return fail(LLR_EINVAL, "bad argument");
    const long ng = (long)std::floor((bhi - blo) / h + 0.5);
    if (ng > 1000000 || (double)n_boot * (double)(ng + 1) > 6.5e7) return fail(LLR_EINVAL, "beta grid too fine");
    HIPCHK(hipSetDevice(c->device));
    const size_t nd = (size_t)n * (1 + (size_t)n_runs + 2 * (size_t)n_boot) + (size_t)n_boot * (ng + 1 + 2) + 8;
    llr_status st = ensure_stage(c, 8 * nd + 64);
    if (st != LLR_OK) return st;
    double* dc = (double*)c->stage;
    double* druns = dc + n;
    double* dbar = druns + (size_t)n_runs * n;
    double* dout = dbar + (size_t)n_boot * n;
    double* scr = dout + 2 * (size_t)n_boot;
    HIPCHK(hipMemcpyAsync(dc, centres, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(druns, a_runs, 8 * (size_t)n * n_runs, hipMemcpyHostToDevice, c->stream));
    launch_boot_mean(druns, n_runs, n, n_boot, seed, dbar, c->stream);
    launch_beta_c_rows(dc, dbar, n, n_boot, s, six_v, blo, bhi, h, tol, scr, dout, c->stream);
    std::vector<double> r(2 * (size_t)n_boot);
    HIPCHK(hipMemcpyAsync(r.data(), dout, 16 * (size_t)n_boot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    for (int b = 0; b < n_boot; ++b) {
        beta_c[b] = r[2 * b];
        cv_peak[b] = r[2 * b + 1];
    }
    return LLR_OK;
}

// Weighted linear least squares y ~ sum_j p_j x^{e_j} by Householder QR of the
// column-equilibrated design matrix (the columns x^0, x^-4, x^-8 of a
// finite-size fit differ by many orders of magnitude, which the normal
// equations would square).
llr_status llr_fss_fit(const double* x, const double* y, const double* sigma, int m, const double* powers, int n_par,
                       double* params, double* errors, double* chi2_red) {
    if (!x || !y || !sigma || !powers || !params || m < 1 || n_par < 1 || n_par > 16 || m <= n_par)
        return fail(LLR_EINVAL, "bad argument (need m > n_par, n_par <= 16)");
    for (int i = 0; i < m; ++i)
        if (!(sigma[i] > 0) || !(x[i] > 0) || !std::isfinite(y[i])) return fail(LLR_EINVAL, "bad data point");
    std::vector<double> A((size_t)m * n_par), b(m), scale(n_par);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n_par; ++j) A[(size_t)i * n_par + j] = std::pow(x[i], powers[j]) / sigma[i];
        b[i] = y[i] / sigma[i];
    }
    for (int j = 0; j < n_par; ++j) {
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += A[(size_t)i * n_par + j] * A[(size_t)i * n_par + j];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0)) return fail(LLR_ENUMERIC, "zero column in the design matrix");
        scale[j] = nrm;
        for (int i = 0; i < m; ++i) A[(size_t)i * n_par + j] /= nrm;
    }
    // Householder: A = Q R, b <- Q^T b
    for (int j = 0; j < n_par; ++j) {
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += A[(size_t)i * n_par + j] * A[(size_t)i * n_par + j];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0)) return fail(LLR_ENUMERIC, "rank-deficient design matrix");
        const double ajj = A[(size_t)j * n_par + j];
        const double alpha = ajj > 0 ? -nrm : nrm;
        std::vector<double> v(m, 0.0);
        v[j] = ajj - alpha;
        for (int i = j + 1; i < m; ++i) v[i] = A[(size_t)i * n_par + j];
        double vv = 0.0;
        for (int i = j; i < m; ++i) vv += v[i] * v[i];
        if (vv > 0) {
            for (int k = j; k < n_par; ++k) {
                double d = 0.0;
                for (int i = j; i < m; ++i) d += v[i] * A[(size_t)i * n_par + k];
                d = 2.0 * d / vv;
                for (int i = j; i < m; ++i) A[(size_t)i * n_par + k] -= d * v[i];
            }
            double d = 0.0;
            for (int i = j; i < m; ++i) d += v[i] * b[i];
            d = 2.0 * d / vv;
            for (int i = j; i < m; ++i) b[i] -= d * v[i];
        }
    }
    // back substitution R z = (Q^T b)[0:n]; residual norm from the rest
    std::vector<double> z(n_par);
    for (int j = n_par - 1; j >= 0; --j) {
        double t = b[j];
        for (int k = j + 1; k < n_par; ++k) t -= A[(size_t)j * n_par + k] * z[k];
        z[j] = t / A[(size_t)j * n_par + j];
    }
    double rss = 0.0;
    for (int i = n_par; i < m; ++i) rss += b[i] * b[i];
    // covariance (R^T R)^{-1} = R^{-1} R^{-T}: invert the upper triangle
    std::vector<double> Ri((size_t)n_par * n_par, 0.0);
    for (int j = 0; j < n_par; ++j) {
        Ri[(size_t)j * n_par + j] = 1.0 / A[(size_t)j * n_par + j];
        for (int i = j - 1; i >= 0; --i) {
            double t = 0.0;
            for (int k = i + 1; k <= j; ++k) t += A[(size_t)i * n_par + k] * Ri[(size_t)k * n_par + j];
            Ri[(size_t)i * n_par + j] = -t / A[(size_t)i * n_par + i];
        }
    }
    for (int j = 0; j < n_par; ++j) {
        params[j] = z[j] / scale[j];
        if (errors) {
            double v = 0.0;
            for (int k = j; k < n_par; ++k) v += Ri[(size_t)j * n_par + k] * Ri[(size_t)j * n_par + k];
            errors[j] = std::sqrt(v) / scale[j];
        }
    }
    if (chi2_red) *chi2_red = rss / (double)(m - n_par);
    return LLR_OK;
}

llr_status llr_mlp_init(llr_ctx* c, uint64_t seed, float* weights) {
    if (!c || !weights) return fail(LLR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(c->device));
    llr_status st = ensure_stage(c, 4 * kMlpNP);
    if (st != LLR_OK) return st;
    launch_mlp_init(seed, (float*)c->stage, c->stream);
    HIPCHK(hipMemcpyAsync(weights, c->stage, 4 * kMlpNP, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

static llr_status stage_inputs(llr_ctx* c, const float* w, const float* u, const float* invL, const double* a, int n,
                               float** dw, float** du, float** dl, double** dA, size_t extra) {
    const size_t need = 4 * (size_t)kMlpNP + 8 * (size_t)n + 8 * (size_t)n + extra + 256;
    llr_status st = ensure_stage(c, need);
    if (st != LLR_OK) return st;
    char* p = (char*)c->stage;
    *dw = (float*)p; p += 4 * (size_t)kMlpNP; p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    *du = (float*)p; p += 4 * (size_t)n;
    *dl = (float*)p; p += 4 * (size_t)n; p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    *dA = (double*)p;
    HIPCHK(hipMemcpyAsync(*dw, w, 4 * kMlpNP, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(*du, u, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(*dl, invL, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    if (a) HIPCHK(hipMemcpyAsync(*dA, a, 8 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    return LLR_OK;
}

llr_status llr_mlp_predict(llr_ctx* c, const float* w, const float* u, const float* invL, int n, int bf16,
                           double* a_out) {
    if (!c || !w || !u || !invL || !a_out || n < 0) return fail(LLR_EINVAL, "bad argument");
    if (n == 0) return LLR_OK;
    HIPCHK(hipSetDevice(c->device));
    float *dw, *du, *dl;
    double* dA;
    llr_status st = stage_inputs(c, w, u, invL, nullptr, n, &dw, &du, &dl, &dA, 0);
    if (st != LLR_OK) return st;
    launch_mlp_forward(dw, du, dl, n, bf16, dA, c->stream);
    HIPCHK(hipMemcpyAsync(a_out, dA, 8 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_mlp_warm_start(llr_ctx* c, int lat, const float* w, int bf16, double a_min, double a_max,
                              double* a_out, int* n_fallback) {
    if (!c || !w) return fail(LLR_EINVAL, "bad argument");
    if (lat < 0 || lat >= (int)c->lats.size()) return fail(LLR_EINVAL, "no such lattice");
    if (!(a_max >= a_min) || !std::isfinite(a_min) || !std::isfinite(a_max))
        return fail(LLR_EINVAL, "need finite a_min <= a_max");
    const HostLat& hl = c->lats[lat];
    const double six_v = 6.0 * (double)hl.L * hl.L * hl.L * hl.L;
    std::vector<float> u(hl.n), il(hl.n, (float)(1.0 / hl.L));
    for (int k = 0; k < hl.n; ++k) u[k] = (float)((hl.E_low[k] + 0.5 * hl.dE) / six_v);
    std::vector<double> a(hl.n);
    llr_status st = llr_mlp_predict(c, w, u.data(), il.data(), hl.n, bf16, a.data());
    if (st != LLR_OK) return st;
    int nf = 0;
    for (int k = 0; k < hl.n; ++k)
        if (!std::isfinite(a[k]) || a[k] < a_min || a[k] > a_max) {
            a[k] = 1.0;
            ++nf;
        }
    if ((st = llr_set_a(c, lat, a.data())) != LLR_OK) return st;
    if (a_out) memcpy(a_out, a.data(), 8 * (size_t)hl.n);
    if (n_fallback) *n_fallback = nf;
    return LLR_OK;
}

llr_status llr_mlp_loss_grad(llr_ctx* c, const float* w, const float* u, const float* invL, const double* a, int n,
                             int bf16, float* grad, double* loss) {
    if (!c || !w || !u || !invL || !a || !grad || !loss || n < 1 || n > 4096) return fail(LLR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(c->device));
    float *dw, *du, *dl;
    double* dA;
    llr_status st = stage_inputs(c, w, u, invL, a, n, &dw, &du, &dl, &dA, 4 * (size_t)kMlpNP + 64);
    if (st != LLR_OK) return st;
    float* dg = (float*)(dA + n);
    double* dloss = (double*)(dg + kMlpNP + 2);
    dloss = (double*)(((uintptr_t)dloss + 7) & ~(uintptr_t)7);
    launch_mlp_loss_grad(dw, du, dl, dA, n, bf16, dg, dloss, c->stream);
    HIPCHK(hipMemcpyAsync(grad, dg, 4 * kMlpNP, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(loss, dloss, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

llr_status llr_mlp_train(llr_ctx* c, float* w, const float* u, const float* invL, const double* a, int n, int epochs,
                         float lr, int bf16, double* loss_hist) {
    if (!c || !w || !u || !invL || !a || n < 1 || n > 4096 || epochs < 0 || !(lr > 0))
        return fail(LLR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(c->device));
    float *dw, *du, *dl;
    double* dA;
    const size_t extra = 4 * 3 * (size_t)kMlpNP + 8 * (size_t)std::max(epochs, 1) + 256;
    llr_status st = stage_inputs(c, w, u, invL, a, n, &dw, &du, &dl, &dA, extra);
    if (st != LLR_OK) return st;
    float* dg = (float*)(dA + n);
    float* dm = dg + kMlpNP;
    float* dv = dm + kMlpNP;
    double* dloss = (double*)(((uintptr_t)(dv + kMlpNP) + 7) & ~(uintptr_t)7);
    HIPCHK(hipMemsetAsync(dm, 0, 4 * 2 * (size_t)kMlpNP, c->stream));
    for (int e = 0; e < epochs; ++e) {
        launch_mlp_loss_grad(dw, du, dl, dA, n, bf16, dg, dloss + e, c->stream);
        launch_mlp_adam(dw, dm, dv, dg, e + 1, lr, c->stream);
    }
    HIPCHK(hipMemcpyAsync(w, dw, 4 * kMlpNP, hipMemcpyDeviceToHost, c->stream));
    if (loss_hist && epochs > 0) HIPCHK(hipMemcpyAsync(loss_hist, dloss, 8 * (size_t)epochs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return LLR_OK;
}

}  // extern "C"

// ================================================================= checkpoints
// A checkpoint holds the whole state of Algorithm 1 between two calls: the
// lattice set (L, n, dE, E_k), the parameters, every angle (both planes of
// every colour, as bound), the current-plane bits, per chain E, the interval
// it serves, the approach couplings and the acceptance counters, per interval
// a_k, the chain serving it, the running sum of measured energies, the
// convergence record and the history a^(n), and the counters (sweep and
// approach indices, Robbins-Monro iteration, replica-exchange counts).
//
// File layout (little endian): the 8 bytes "LLRCKPT1"; u32 version (2); u32
// precision; u32 number of lattices; per lattice i32 L, i32 n, f64 dE,
// f64 E_low[n]; the parameters as listed in llr_params (i32 n_th, n_a, n_rm,
// u64 seed, i32 replica_exchange, f64 overlap, i32 recompute_every, f64 eps,
// i32 approach_cap); then named sections, each u32 tag, u64 byte count,
// bytes; last the u32 CRC-32 (IEEE 802.3 polynomial, reflected 0xEDB88320,
// initial and final xor 0xFFFFFFFF) of everything before it.
namespace {

const char kCkMagic[8] = {'L', 'L', 'R', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkVersion = 2;

struct Crc32Table {
    uint32_t t[256];
    Crc32Table() {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            t[i] = c;
        }
    }
};

uint32_t crc32_update(uint32_t crc, const unsigned char* p, size_t n) {
    static const Crc32Table tab;   // initialised once, thread-safe
    const uint32_t* table = tab.t;
    crc = ~crc;
    for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xffu] ^ (crc >> 8);
    return ~crc;
}

// Sections of the file, in the order they are written.
enum CkTag : uint32_t {
    kTagState = 1, kTagCur, kTagE, kTagItv, kTagB, kTagEta, kTagSprev, kTagHbProp, kTagHbAcc, kTagA, kTagConf,
    kTagSumE, kTagConvIter, kTagConvSweeps, kTagAHist, kTagLinkFix, kTagLinkArc, kTagLatDone, kTagMuLnRho, kTagMuB,
    kTagScalars, kTagHost, kTagFuAcc, kTagRates
};

struct CkWriter {
    std::vector<unsigned char> buf;
    void put(const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        buf.insert(buf.end(), c, c + n);
    }
    template <typename V> void val(V v) { put(&v, sizeof(V)); }
};

struct CkReader {
    const unsigned char* p;
    size_t n, off = 0;
    bool get(void* dst, size_t k) {
        if (k > n - off) return false;
        memcpy(dst, p + off, k);
        off += k;
        return true;
    }
    template <typename V> bool val(V* v) { return get(v, sizeof(V)); }
};

struct CkLattice {
    int L, n;
    double dE;
    std::vector<double> E_low;
};

struct CkSection {
    uint32_t tag;
    uint64_t bytes;
    const unsigned char* at;   // into the loaded file
};

struct CkHeader {
    uint32_t precision = 0;
    std::vector<CkLattice> lats;
    llr_params prm{};
    std::vector<CkSection> secs;
    const CkSection* find(uint32_t tag) const {
        for (const auto& x : secs)
            if (x.tag == tag) return &x;
        return nullptr;
    }
};

// Bytes of the driver's host section: 11 i32 flags and tiles, then per
// lattice the approach sweep count (i64), its done flag (i32) and a0[n].
size_t ck_host_bytes(const std::vector<CkLattice>& lats) {
    size_t b = 4 * 11;
    for (const auto& l : lats) b += 8 + 4 + 8 * (size_t)l.n;
    return b;
}

// Reads the whole file, checks magic, version, size and CRC, and parses the
// header.  Host only.
llr_status ck_load(const char* path, std::vector<unsigned char>& data, CkHeader& h) {
    if (!path) return fail(LLR_EINVAL, "null path");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(LLR_EINVAL, std::string("cannot open checkpoint ") + path);
    data.clear();
    unsigned char tmp[1 << 16];
    size_t got;
    while ((got = fread(tmp, 1, sizeof(tmp), f)) > 0) data.insert(data.end(), tmp, tmp + got);
    fclose(f);
    if (data.size() < sizeof(kCkMagic) + 4 + 4 || memcmp(data.data(), kCkMagic, sizeof(kCkMagic)) != 0)
        return fail(LLR_EINVAL, "not an LLR checkpoint (magic)");
    uint32_t crc_file;
    memcpy(&crc_file, data.data() + data.size() - 4, 4);
    if (crc32_update(0, data.data(), data.size() - 4) != crc_file)
        return fail(LLR_EINVAL, "checkpoint corrupted or truncated (CRC-32 mismatch)");
    CkReader r{data.data(), data.size() - 4};
    r.off = sizeof(kCkMagic);
    uint32_t ver = 0, nl = 0;
    if (!r.val(&ver) || ver != kCkVersion) return fail(LLR_EINVAL, "unsupported checkpoint version");
    if (!r.val(&h.precision) || (h.precision != LLR_FP64 && h.precision != LLR_FP32))
        return fail(LLR_EINVAL, "bad precision in checkpoint");
    if (!r.val(&nl) || nl < 1 || nl > (uint32_t)kMaxLat) return fail(LLR_EINVAL, "bad lattice count in checkpoint");
    h.lats.assign(nl, CkLattice{});
    for (auto& l : h.lats) {
        if (!r.val(&l.L) || !r.val(&l.n) || !r.val(&l.dE)) return fail(LLR_EINVAL, "checkpoint header truncated");
        if (l.L < 2 || l.L > 32 || (l.L & 1) || l.n < 1 || l.n > 4096 || !(l.dE > 0))
            return fail(LLR_EINVAL, "bad lattice in checkpoint");
        l.E_low.resize(l.n);
        if (!r.get(l.E_low.data(), 8 * (size_t)l.n)) return fail(LLR_EINVAL, "checkpoint header truncated");
        if (check_lattice(l.L, l.n, l.E_low.data(), l.dE) != LLR_OK) return fail(LLR_EINVAL, "bad lattice in checkpoint");
    }
    llr_params& p = h.prm;
    if (!r.val(&p.n_th) || !r.val(&p.n_a) || !r.val(&p.n_rm) || !r.val(&p.seed) || !r.val(&p.replica_exchange) ||
        !r.val(&p.overlap) || !r.val(&p.recompute_every) || !r.val(&p.eps) || !r.val(&p.approach_cap))
        return fail(LLR_EINVAL, "checkpoint header truncated");
    if (check_params(p) != LLR_OK) return fail(LLR_EINVAL, "bad parameters in checkpoint");
    // the section table: every section inside the file, each tag known and
    // present once, with the size the header implies
    h.secs.clear();
    while (r.off < r.n) {
        CkSection x{};
        if (!r.val(&x.tag) || !r.val(&x.bytes) || x.bytes > r.n - r.off) return fail(LLR_EINVAL, "checkpoint section truncated");
        if (x.tag < kTagState || x.tag > kTagRates) return fail(LLR_EINVAL, "unknown checkpoint section");
        if (h.find(x.tag)) return fail(LLR_EINVAL, "duplicate checkpoint section");
        x.at = r.p + r.off;
        r.off += (size_t)x.bytes;
        h.secs.push_back(x);
    }
    size_t n = 0, sites = 0;
    for (const auto& l : h.lats) {
        n += (size_t)l.n;
        sites += (size_t)l.n * 8 * ((size_t)l.L * l.L * l.L * l.L);   // both planes of every colour
    }
    const size_t state_bytes = sites * (h.precision == LLR_FP32 ? 4 : 8);
    struct Want { uint32_t tag; size_t bytes; };
    const Want want[] = {
        {kTagState, state_bytes}, {kTagCur, 8 * n}, {kTagE, 8 * n}, {kTagItv, 4 * n}, {kTagB, 64 * n},
        {kTagEta, 64 * n}, {kTagSprev, 32 * n}, {kTagHbProp, 8 * n}, {kTagHbAcc, 8 * n}, {kTagA, 8 * n},
        {kTagConf, 4 * n}, {kTagSumE, 8 * n}, {kTagConvIter, 4 * n}, {kTagConvSweeps, 8 * n},
        {kTagLinkFix, 8 * n}, {kTagLinkArc, 8 * n}, {kTagLatDone, 4 * (size_t)kMaxLat}, {kTagMuLnRho, 8 * n},
        {kTagMuB, 8 * (size_t)kMaxLat}, {kTagScalars, 28}, {kTagFuAcc, 8 * n}, {kTagRates, 32},
        {kTagHost, ck_host_bytes(h.lats)}};
    for (const auto& x : want) {
        const CkSection* q = h.find(x.tag);
        if (!q || q->bytes != x.bytes) return fail(LLR_EINVAL, "checkpoint section missing or of the wrong size");
    }
    const CkSection* ah = h.find(kTagAHist);   // empty, or a^(0..n_rm) of every interval
    if (!ah || (ah->bytes != 0 && ah->bytes != 8 * ((size_t)p.n_rm + 1) * n))
        return fail(LLR_EINVAL, "checkpoint history of the wrong size");
    return LLR_OK;
}

}  // namespace

extern "C" {

llr_status llr_checkpoint_info(const char* path, int* precision, int* n_lattices, int* L, int* n_intervals,
                               double* dE, double* E_low, llr_params* params) {
    std::vector<unsigned char> data;
    CkHeader h;
    llr_status st = ck_load(path, data, h);
    if (st != LLR_OK) return st;
    if (precision) *precision = (int)h.precision;
    if (n_lattices) *n_lattices = (int)h.lats.size();
    size_t off = 0;
    for (size_t i = 0; i < h.lats.size(); ++i) {
        if (L) L[i] = h.lats[i].L;
        if (n_intervals) n_intervals[i] = h.lats[i].n;
        if (dE) dE[i] = h.lats[i].dE;
        if (E_low) memcpy(E_low + off, h.lats[i].E_low.data(), 8 * (size_t)h.lats[i].n);
        off += (size_t)h.lats[i].n;
    }
    if (params) *params = h.prm;
    return LLR_OK;
}

llr_status llr_checkpoint(llr_ctx* c, const char* path) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    if (!path) return fail(LLR_EINVAL, "null path");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int n = c->lt.n_chains;
    const DevState& s = c->ds;
    CkWriter w;
    w.put(kCkMagic, sizeof(kCkMagic));
    w.val(kCkVersion);
    w.val((uint32_t)c->precision);
    w.val((uint32_t)c->lats.size());
    for (const auto& hl : c->lats) {
        w.val(hl.L);
        w.val(hl.n);
        w.val(hl.dE);
        w.put(hl.E_low.data(), 8 * (size_t)hl.n);
    }
    const llr_params& p = c->prm;
    w.val(p.n_th); w.val(p.n_a); w.val(p.n_rm); w.val(p.seed); w.val(p.replica_exchange); w.val(p.overlap);
    w.val(p.recompute_every); w.val(p.eps); w.val(p.approach_cap);
    auto dev = [&](uint32_t tag, const void* d, size_t bytes) -> llr_status {
        w.val(tag);
        w.val((uint64_t)bytes);
        const size_t at = w.buf.size();
        w.buf.resize(at + bytes);
        if (bytes) HIPCHK(hipMemcpy(w.buf.data() + at, d, bytes, hipMemcpyDeviceToHost));
        return LLR_OK;
    };
#define CKD(tag, ptr, bytes) \
    if ((st = dev(tag, ptr, bytes)) != LLR_OK) return st;
    CKD(kTagState, c->state, c->state_bytes)
    CKD(kTagCur, s.cur, 8 * (size_t)n)
    CKD(kTagE, s.E, 8 * (size_t)n)
    CKD(kTagItv, s.itv, 4 * (size_t)n)
    CKD(kTagB, s.b, 8 * 8 * (size_t)n)
    CKD(kTagEta, s.eta, 8 * 8 * (size_t)n)
    CKD(kTagSprev, s.sprev, 4 * 8 * (size_t)n)
    CKD(kTagHbProp, s.hb_prop, 8 * (size_t)n)
    CKD(kTagHbAcc, s.hb_acc, 8 * (size_t)n)
    CKD(kTagA, s.a, 8 * (size_t)n)
    CKD(kTagConf, s.conf, 4 * (size_t)n)
    CKD(kTagSumE, s.sumE, 8 * (size_t)n)
    CKD(kTagConvIter, s.conv_iter, 4 * (size_t)n)
    CKD(kTagConvSweeps, s.conv_sweeps, 8 * (size_t)n)
    CKD(kTagAHist, s.a_hist, s.a_hist ? 8 * ((size_t)p.n_rm + 1) * n : 0)
    CKD(kTagLinkFix, s.link_fix, 8 * (size_t)n)
    CKD(kTagLinkArc, s.link_arc, 8 * (size_t)n)
    CKD(kTagLatDone, s.lat_done, 4 * (size_t)kMaxLat)
    CKD(kTagMuLnRho, s.mu_lnrho, 8 * (size_t)n)
    CKD(kTagMuB, s.mu_b, 8 * (size_t)kMaxLat)
    CKD(kTagFuAcc, s.fu_acc, 8 * (size_t)n)
#undef CKD
    // device scalars: sweep index, approach index, RM iteration, replica counts
    uint32_t sc[2];
    int rmi = 0;
    unsigned long long re[2];
    HIPCHK(hipMemcpy(&sc[0], s.sweep_ctr, 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&sc[1], s.approach_ctr, 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&rmi, s.rm_iter, 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(re, s.re_cnt, 16, hipMemcpyDeviceToHost));
    w.val((uint32_t)kTagScalars);
    w.val((uint64_t)(8 + 4 + 16));
    w.put(sc, 8); w.val(rmi); w.put(re, 16);
    // host state of the driver
    CkWriter hw;
    hw.val(c->rm_done); hw.val((int)c->rm_open); hw.val((int)c->ap_open); hw.val((int)c->have_energy);
    hw.val(c->interleave ? (int)LLR_SWEEP_INTERLEAVED : c->stagger ? (int)LLR_SWEEP_STAGGERED : (int)LLR_SWEEP_GROUPED); hw.val((int)c->per_link); hw.val((int)c->muca_ready); hw.val((int)c->tuned);
    hw.val(c->lt.hb_lpt); hw.val(c->lt.or_lpt); hw.val(c->lt.serpentine);
    for (size_t i = 0; i < c->lats.size(); ++i) {
        hw.val(i < c->approach_sweeps.size() ? c->approach_sweeps[i] : 0ll);
        hw.val(i < c->ap_done.size() ? c->ap_done[i] : 0);
        hw.put(c->lats[i].a0.data(), 8 * (size_t)c->lats[i].n);
    }
    w.val((uint32_t)kTagHost);
    w.val((uint64_t)hw.buf.size());
    w.put(hw.buf.data(), hw.buf.size());
    // link-update accounting of llr_get_rates
    w.val((uint32_t)kTagRates);
    w.val((uint64_t)32);
    w.val(c->sweeps_run); w.val(c->or_passes); w.val(c->fused_passes); w.val(c->run_seconds);
    const uint32_t crc = crc32_update(0, w.buf.data(), w.buf.size());
    w.val(crc);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return fail(LLR_EINVAL, std::string("cannot write ") + tmp);
    const size_t put = fwrite(w.buf.data(), 1, w.buf.size(), f);
    const int cl = fclose(f);
    if (put != w.buf.size() || cl != 0 || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(LLR_EINVAL, std::string("cannot write ") + path);
    }
    return LLR_OK;
}

llr_status llr_restore(llr_ctx* c, const char* path) {
    llr_status st = need_state(c);
    if (st != LLR_OK) return st;
    std::vector<unsigned char> data;
    CkHeader h;
    if ((st = ck_load(path, data, h)) != LLR_OK) return st;
    if ((int)h.precision != c->precision) return fail(LLR_EINVAL, "checkpoint precision differs from the context's");
    if (h.lats.size() != c->lats.size()) return fail(LLR_EINVAL, "checkpoint lattice set differs from the context's");
    for (size_t i = 0; i < h.lats.size(); ++i) {
        const auto& a = h.lats[i];
        const auto& b = c->lats[i];
        if (a.L != b.L || a.n != b.n || a.dE != b.dE || memcmp(a.E_low.data(), b.E_low.data(), 8 * (size_t)a.n) != 0)
            return fail(LLR_EINVAL, "checkpoint lattice set differs from the context's");
    }
    const int n = c->lt.n_chains;
    const llr_params& p = h.prm;
    // the reader has size-checked every section against the header, and the
    // header equals the context's lattice set, so every section fits the
    // context's buffers; nothing is written to the device before this point
    auto find = [&](uint32_t tag) { return h.find(tag); };
    if (find(kTagState)->bytes != c->state_bytes) return fail(LLR_EINVAL, "checkpoint state of the wrong size");
    const CkSection* ah = find(kTagAHist);
    const CkSection* hs = find(kTagHost);
    CkReader hr{hs->at, (size_t)hs->bytes};
    int rm_done, rm_open, ap_open, have_e, inter, per_link, muca, tuned, hbl, orl, serp;
    hr.val(&rm_done); hr.val(&rm_open); hr.val(&ap_open); hr.val(&have_e); hr.val(&inter); hr.val(&per_link);
    hr.val(&muca); hr.val(&tuned); hr.val(&hbl); hr.val(&orl); hr.val(&serp);
    auto ok_lpt = [](int v) { return v == 1 || v == 2 || v == 4; };
    if (!ok_lpt(hbl) || !ok_lpt(orl) || rm_done < 0 || rm_done > p.n_rm || inter < LLR_SWEEP_GROUPED ||
        inter > LLR_SWEEP_STAGGERED)
        return fail(LLR_EINVAL, "bad driver state in checkpoint");
    // parameters (and with them the restriction widths), then the device state
    if ((st = llr_set_params(c, &p)) != LLR_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    if ((st = upload_intervals(c)) != LLR_OK) return st;
    const DevState& s = c->ds;
    auto up = [&](uint32_t tag, void* d) -> llr_status {
        const CkSection* q = find(tag);
        if (q->bytes) HIPCHK(hipMemcpy(d, q->at, (size_t)q->bytes, hipMemcpyHostToDevice));
        return LLR_OK;
    };
#define CKU(tag, ptr) \
    if ((st = up(tag, ptr)) != LLR_OK) return st;
    CKU(kTagState, c->state) CKU(kTagCur, s.cur) CKU(kTagE, s.E) CKU(kTagItv, s.itv) CKU(kTagB, s.b)
    CKU(kTagEta, s.eta) CKU(kTagSprev, s.sprev) CKU(kTagHbProp, s.hb_prop) CKU(kTagHbAcc, s.hb_acc) CKU(kTagA, s.a)
    CKU(kTagConf, s.conf) CKU(kTagSumE, s.sumE) CKU(kTagConvIter, s.conv_iter) CKU(kTagConvSweeps, s.conv_sweeps)
    CKU(kTagLinkFix, s.link_fix) CKU(kTagLinkArc, s.link_arc) CKU(kTagLatDone, s.lat_done) CKU(kTagMuLnRho, s.mu_lnrho)
    CKU(kTagMuB, s.mu_b) CKU(kTagFuAcc, s.fu_acc)
#undef CKU
    if (c->ds.a_hist) {
        HIPCHK(hipFree(c->ds.a_hist));
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void*)c->ds.a_hist), c->allocs.end());
        c->ds.a_hist = nullptr;
    }
    if (ah->bytes) {
        if ((st = dalloc(c, &c->ds.a_hist, ((size_t)p.n_rm + 1) * n)) != LLR_OK) return st;
        HIPCHK(hipMemcpy(c->ds.a_hist, ah->at, (size_t)ah->bytes, hipMemcpyHostToDevice));
    }
    const CkSection* sc = find(kTagScalars);
    HIPCHK(hipMemcpy(s.sweep_ctr, sc->at, 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s.approach_ctr, sc->at + 4, 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s.rm_iter, sc->at + 8, 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s.re_cnt, sc->at + 12, 16, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(s.bits, 0, 2 * (size_t)(n + 2)));
    HIPCHK(hipMemset(s.health, 0, 4 * (size_t)n));
    HIPCHK(hipMemset(s.drift, 0, 8 * (size_t)n));
    HIPCHK(hipDeviceSynchronize());
    {
        CkReader rr{find(kTagRates)->at, 32};
        rr.val(&c->sweeps_run); rr.val(&c->or_passes); rr.val(&c->fused_passes); rr.val(&c->run_seconds);
    }
    c->rm_done = rm_done;
    c->rm_open = rm_open != 0;
    c->ap_open = ap_open != 0;
    c->have_energy = have_e != 0;
    if (inter == LLR_SWEEP_STAGGERED && (st = ensure_side_stream(c)) != LLR_OK) return st;
    c->interleave = inter == LLR_SWEEP_INTERLEAVED;
    c->stagger = inter == LLR_SWEEP_STAGGERED;
    c->per_link = per_link != 0;
    c->muca_ready = muca != 0;
    set_tiles(c->lt, hbl, orl);
    c->tuned = tuned != 0;
    c->lt.serpentine = serp;
    c->approach_sweeps.assign(c->lats.size(), 0);
    c->ap_done.assign(c->lats.size(), 0);
    for (size_t i = 0; i < c->lats.size(); ++i) {
        hr.val(&c->approach_sweeps[i]);
        hr.val(&c->ap_done[i]);
        hr.get(c->lats[i].a0.data(), 8 * (size_t)c->lats[i].n);
    }
    drop_graphs(c);
    return LLR_OK;
}

}  // extern "C"
