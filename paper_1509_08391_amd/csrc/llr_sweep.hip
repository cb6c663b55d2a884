// llr_sweep.hip -- gfx950 kernels of the energy-restricted LLR sweep for 4D
// compact U(1) (arXiv:1509.08391, Sec. 2.2 restricted measure, Sec. 3.1 model).
//
// Layout: per chain, 2 planes x 8 colours x V/2 angles; colour c = 2 mu + p
// holds theta_mu at the sites of parity p, indexed by the half index
// h = s >> 1 of the lexicographic site s.  Links of one colour share no
// plaquette, so a colour class is updated in one data-parallel pass.
//
// A heatbath pass writes every proposal to the non-current plane of its
// colour, reduces the class Delta E per chain in int64 fixed point
// (order-independent, deterministic; one fence-free 64-bit atomic per block)
// and the last block of each chain takes the FP64 interval decision: on accept it flips the chain's current-plane
// bit, on reject nothing is written back.  An overrelaxation pass maps
// theta -> -2 phi - theta in place; it leaves every local action unchanged,
// so it needs neither a reduction nor a decision.
#include <hip/hip_runtime.h>

#include "llr_internal.hpp"

namespace llr {

// heatbath pass modes: the public LLR_MODE_* values 0-4, the tuner's timing
// mode, and the candidate pre-pass of the per-link constraint (every link's
// free heatbath candidate written with its Delta E and staples, nothing
// accepted, no counters touched; the walk kernel then decides)
enum { kModeRestricted = 0, kModeApproach = 1, kModeFree = 2, kModeMuca = 3, kModeLink = 4,
       kModeTune = kHbModeTune, kModeLinkPre = 6 };
// instantiations of the heatbath class pass
enum { kHbPlain = 0, kHbPre = 1, kHbFuseOr = 2 };

constexpr long long kLinkNone = (long long)0x8000000000000000ull;   // no free candidate within the cap

__device__ __forceinline__ int find_lat_site(const LatTable& lt, int b) {
    int li = 0;
#pragma unroll 1
    while (li + 1 < lt.n && b >= lt.l[li + 1].eblock0) ++li;
    return li;
}

// coordinates of the site with half index h and parity p
__device__ __forceinline__ void decode_half(const LatDev& L, uint32_t h, int p, int x[4]) {
    const uint32_t r1 = L.hL == 1 ? h : fdiv(h, L.mhL);   // ceil(2^32 / 1) does not fit 32 bits
    const int x0h = (int)(h - r1 * (uint32_t)L.hL);
    const uint32_t r2 = fdiv(r1, L.mL);
    x[1] = (int)(r1 - r2 * (uint32_t)L.L);
    const uint32_t r3 = fdiv(r2, L.mL);
    x[2] = (int)(r2 - r3 * (uint32_t)L.L);
    x[3] = (int)r3;
    x[0] = 2 * x0h + ((p + x[1] + x[2] + x[3]) & 1);
}
// Column tiles of the class passes.  The half index is h = pos + P x3 with
// pos = x0h + hL (x1 + L x2) the position in the (x0h, x1, x2) slab and
// P = hL L^2 its size, and the class's sites at one position and
// consecutive x3 alternate between x0 = 2 x0h and 2 x0h + 1 (the parity of
// x1 + x2 + x3 flips).  A tile is kBlock positions by LPT consecutive x3:
// thread tid owns position pos = pt kBlock + tid and x3 = xg LPT + r,
// r = 0..LPT-1, so its links share x0h, x1, x2 and the offsets along
// x1, x2, while x3 and its offsets are uniform over the wavefront.
struct ColTile {
    uint32_t pos;   // position in the slab; a lane past the slab's end gets 0
    uint32_t pos0;  // the tile's first position, pt kBlock
    bool in_slab;   // the lane's position lies in the slab (pt kBlock + tid < P)
    int x0h, x1, x2;
    int x3_0;       // x3 of the thread's first link
};
template <int LPT>
__device__ __forceinline__ ColTile col_tile(const LatDev& L, int tile, int tid) {
    ColTile t;
    const int xg = tile / L.npt;
    const int pt = tile - xg * L.npt;
    t.pos0 = (uint32_t)pt * kBlock;
    const uint32_t pos = t.pos0 + (uint32_t)tid;
    t.in_slab = pos < L.P;
    // a lane past the slab computes (and discards) the links of position 0,
    // so that its coordinates, neighbour offsets and addresses stay in range
    t.pos = t.in_slab ? pos : 0u;
    t.x3_0 = xg * LPT;
    const uint32_t r1 = L.hL == 1 ? t.pos : fdiv(t.pos, L.mhL);
    t.x0h = (int)(t.pos - r1 * (uint32_t)L.hL);
    const uint32_t r2 = fdiv(r1, L.mL);
    t.x1 = (int)(r1 - r2 * (uint32_t)L.L);
    t.x2 = (int)r2;
    return t;
}
__device__ __forceinline__ uint32_t half_of(const LatDev& L, int y0, int y1, int y2, int y3) {
    return (uint32_t)((y0 >> 1) + L.hL * (y1 + L.L * (y2 + L.L * y3)));
}
__device__ __forceinline__ int up(int v, int L) { return v + 1 == L ? 0 : v + 1; }
__device__ __forceinline__ int dn(int v, int L) { return v == 0 ? L - 1 : v - 1; }

template <typename T>
__device__ __forceinline__ T* chain_base(const LatDev& L, T* th, int cl) {
    return th + L.base + (long long)cl * 16ll * (long long)L.V2;
}
template <typename T>
__device__ __forceinline__ T* plane_ptr(T* chain, uint64_t curw, int c, uint32_t V2) {
    return chain + (size_t)((((curw >> (8 * c)) & 1ull) * 8ull) + (uint64_t)c) * V2;
}

// Element i of a plane through a 32-bit byte offset: the plane base is uniform
// (scalar registers) and every plane is < 4 GiB, so the access compiles to a
// global load/store with a scalar base and one 32-bit vector offset instead
// of a 64-bit vector address per access.
template <typename T>
__device__ __forceinline__ T ld_plane(const T* plane, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_plane(T* plane, uint32_t i, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + i * (uint32_t)sizeof(T)) = v;
}

// Half-index offsets of the neighbours of site x along each direction:
// up[nu] = h(x + nu) - h(x), dn[nu] = h(x - nu) - h(x), periodic.  Sites
// (2j, 2j+1) along x0 share a half index, so the x0 offsets depend on x0's
// parity; along nu >= 1 a step is L^nu / 2 half indices.
__device__ __forceinline__ void neighbour_offsets(const LatDev& L, const int x[4], int up[4], int dn[4]) {
    const int odd = x[0] & 1;
    up[0] = odd ? (x[0] == L.L - 1 ? 1 - L.hL : 1) : 0;
    dn[0] = odd ? 0 : (x[0] == 0 ? L.hL - 1 : -1);
#pragma unroll
    for (int nu = 1; nu < 4; ++nu) {
        // selects between per-lattice constants (no per-link multiply)
        up[nu] = x[nu] == L.L - 1 ? -L.hwrap[nu] : L.hstr[nu];
        dn[nu] = x[nu] == 0 ? L.hwrap[nu] : -L.hstr[nu];
    }
}

// Neighbour offsets of a thread's column (see col_tile), split into a
// per-lane part along x0, x1, x2 and a wavefront-uniform part along x3:
//   v_up[d], v_dn[d] (d < 3): half-index offsets of x +- d within the slab,
//   for the thread's links with x0 = 2 x0h + b[k], k = r & 1 (the parity of
//   x0 alternates along the column); v_up[3] = v_dn[3] = 0;
//   the offsets along x3 and the link's own shift P x3 are uniform and are
//   added to the plane's base address.
struct ColNbr {
    int up0[2], dn0[2];   // along x0 for the column's even / odd links
    int up1, dn1, up2, dn2;
};
__device__ __forceinline__ ColNbr col_nbr(const LatDev& L, const ColTile& t, int p) {
    ColNbr n;
    const int b0 = (p + t.x1 + t.x2 + t.x3_0) & 1;   // x0 = 2 x0h + b0 for the even links
    const int uo = t.x0h == L.hL - 1 ? 1 - L.hL : 1;  // x0 odd: the partner site 2 x0h + 2 (periodic)
    const int de = t.x0h == 0 ? L.hL - 1 : -1;        // x0 even: the partner site 2 x0h - 1 (periodic)
    n.up0[0] = b0 ? uo : 0;
    n.dn0[0] = b0 ? 0 : de;
    n.up0[1] = b0 ? 0 : uo;
    n.dn0[1] = b0 ? de : 0;
    n.up1 = t.x1 == L.L - 1 ? -L.hwrap[1] : L.hstr[1];
    n.dn1 = t.x1 == 0 ? L.hwrap[1] : -L.hstr[1];
    n.up2 = t.x2 == L.L - 1 ? -L.hwrap[2] : L.hstr[2];
    n.dn2 = t.x2 == 0 ? L.hwrap[2] : -L.hstr[2];
    return n;
}

// Local field of link (MU, x): staples of the 2 x 3 plaquettes containing it,
// each oriented so that theta_MU(x) enters with a plus sign:
//   forward  s_f = th_nu(x+mu) - th_mu(x+nu) - th_nu(x)
//   backward s_b = th_nu(x-nu) - th_nu(x+mu-nu) - th_mu(x-nu)
// C + i S = sum of e^{i s}.  The link sits at slab position pos (per lane) and
// x3 = x3 (uniform); K = x3 parity relative to the column's first link selects
// the x0 offsets.  Every neighbour's half index is pos + (per-lane offset
// along x0..x2) + (uniform: P x3 and the offset along x3).
// UB: the uniform part of every index goes into the plane's base address (a
// scalar 64-bit add per plane and link: the cheaper form when scalar
// registers are free); otherwise it is added to the per-lane 32-bit index.
template <bool UB, typename T>
__device__ __forceinline__ T ld_col(const T* plane, int uni, uint32_t lane) {
    if constexpr (UB) return ld_plane(plane + uni, lane);
    else return ld_plane(plane, lane + (uint32_t)uni);
}

template <typename T, int MU, int K, bool UB>
__device__ __forceinline__ void staples(const LatDev& L, const T* chain, uint64_t curw, int p, uint32_t pos,
                                        const ColNbr& nb, int x3, T& C, T& S) {
    using M = Math<T>;
    const int vu[4] = {nb.up0[K], nb.up1, nb.up2, 0};
    const int vd[4] = {nb.dn0[K], nb.dn1, nb.dn2, 0};
    const int sh = (int)L.P * x3;   // the link's own x3, uniform
    const int su[4] = {sh, sh, sh, sh + (x3 == L.L - 1 ? -L.hwrap[3] : L.hstr[3])};
    const int sd[4] = {0, 0, 0, x3 == 0 ? L.hwrap[3] : -L.hstr[3]};
    const int q = p ^ 1;
    const T* pmu_q = plane_ptr(chain, curw, 2 * MU + q, L.V2);
#pragma unroll
    for (int NU = 0; NU < 4; ++NU) {
        if (NU == MU) continue;
        const T* pnu_p = plane_ptr(chain, curw, 2 * NU + p, L.V2);
        const T* pnu_q = plane_ptr(chain, curw, 2 * NU + q, L.V2);
        const T t_nu_pmu = ld_col<UB>(pnu_q, su[MU], pos + vu[MU]);
        const T t_mu_pnu = ld_col<UB>(pmu_q, su[NU], pos + vu[NU]);
        const T t_nu_x = ld_col<UB>(pnu_p, sh, pos);
        const T t_nu_pmu_mnu = ld_col<UB>(pnu_p, su[MU] + sd[NU], pos + (vu[MU] + vd[NU]));
        const T t_mu_mnu = ld_col<UB>(pmu_q, sh + sd[NU], pos + vd[NU]);
        const T t_nu_mnu = ld_col<UB>(pnu_q, sh + sd[NU], pos + vd[NU]);
        const T sf = t_nu_pmu - t_mu_pnu - t_nu_x;
        const T sb = t_nu_mnu - t_nu_pmu_mnu - t_mu_mnu;
        T s1, c1, s2, c2;
        M::sincos_rad(sf, &s1, &c1);
        M::sincos_rad(sb, &s2, &c2);
        if (NU == (MU == 0 ? 1 : 0)) {   // the first direction seeds the sums
            C = c1 + c2;
            S = s1 + s2;
        } else {
            C += c1 + c2;
            S += s1 + s2;
        }
    }
}

// Staples and old angle of the LPT links of the thread's column; hl, in: the
// links' half indices and whether they lie in the lattice (pos < P, and
// x3 < L, uniform over the wavefront).
template <typename T, int MU, int LPT, bool UB>
__device__ __forceinline__ void col_staples(const LatDev& L, const T* chain, uint64_t curw, int p, const ColTile& ct,
                                            const ColNbr& nb, uint32_t pos, const T* pown, T* C, T* S, T* t_old,
                                            uint32_t* hl, bool* in) {
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
        const int x3 = ct.x3_0 + r;
        C[r] = T(0); S[r] = T(0); t_old[r] = T(0);
        hl[r] = pos + L.P * (uint32_t)x3;
        in[r] = ct.in_slab && x3 < L.L;
        if (x3 < L.L) {
            if (r & 1) staples<T, MU, 1, UB>(L, chain, curw, p, pos, nb, x3, C[r], S[r]);
            else staples<T, MU, 0, UB>(L, chain, curw, p, pos, nb, x3, C[r], S[r]);
            t_old[r] = ld_col<UB>(pown, (int)L.P * x3, pos);
        }
    }
}

// Reduce the per-thread fixed-point values of a block; returns the block sum
// in thread 0.
__device__ __forceinline__ long long block_sum_i64(long long v) {
    __shared__ long long part[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    long long tot = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) tot += part[i];
    }
    return tot;
}

// Per-chain reduction without fences: each block adds, in ONE 64-bit atomic,
// 2^51 (its arrival) plus its partial sum in the lattice's fixed point 2^-fxb
// (two's complement in the low 51 bits; fxb is chosen so that 6V 2^fxb <=
// 2^49 bounds every partial sum).  The block whose addition brings the count
// to nblocks (< 2^13) holds the exact total, independent of arrival order.
__device__ __forceinline__ bool chain_arrive(unsigned long long* acc, long long part, int nblocks, long long* total) {
    const unsigned long long add = (1ull << 51) + (unsigned long long)part;
    const unsigned long long nw = atomicAdd(acc, add) + add;
    const long long S = ((long long)(nw << 13)) >> 13;
    const unsigned long long nb = (nw - (unsigned long long)S) >> 51;
    *total = S;
    return nb == (unsigned long long)nblocks;
}

// Best-Fisher constants in the cancellation-free form: q = (1-rho)/(1+rho),
// r - 1 = (1-rho)^2/(2 rho), kappa (r^2 - 1) with sqrt(r^2-1) = (1-rho^2)/(2 rho).
template <typename T>
__device__ __forceinline__ void vm_constants(T ak, T& q, T& rm1, T& kg2) {
    using M = Math<T>;
    q = T(1); rm1 = T(1); kg2 = T(0);
    if (ak > T(0)) {
        // rho = 2 ak / D with D = tau + sqrt(2 tau); in terms of D:
        // q = (D - 2ak)/(D + 2ak), (1-rho)^2/(2 rho) = (D - 2ak)^2/(4 ak D),
        // (1-rho^2)/(2 rho) = (D - 2ak)(D + 2ak)/(4 ak D)
        const T tau = T(1) + M::sqrt_(T(1) + T(4) * ak * ak);
        const T D = tau + M::sqrt_(T(2) * tau);
        const T dm = D - T(2) * ak, dp = D + T(2) * ak;
        if constexpr (M::f32) {
            // 1/(4 ak D) and 1/dp from one reciprocal of their product
            const T fd = T(4) * ak * D;
            const T t = M::div_(T(1), fd * dp);
            const T r1 = dp * t;
            rm1 = dm * dm * r1;
            const T gg = dm * dp * r1;
            kg2 = ak * gg * gg;
            q = dm * (fd * t);
        } else {
            const T r1 = M::div_(T(1), T(4) * ak * D);
            rm1 = dm * dm * r1;
            const T gg = dm * dp * r1;
            kg2 = ak * gg * gg;
            q = M::div_(dm, dp);
        }
    }
}

// One sampler attempt from the word pair (wa, wb): accept test of Best &
// Fisher with z = cos(pi V1); on accept (ch, sh) = (cos, q sin)(pi V1 / 2).
template <typename T>
__device__ __forceinline__ bool vm_attempt(uint32_t wa, uint32_t wb, T q, T rm1, T kg2, T& ch, T& sh) {
    using M = Math<T>;
    T s_, c_;
    M::sincos_halfpi_w(wa, &s_, &c_);
    const T U2 = M::unif(wb);
    const T cc = M::div_(kg2, M::fma_(T(2) * c_, c_, rm1));   // kappa (r^2 - 1)/(r + z)
    bool acc = M::fma_(cc, T(2) - cc, -U2) > T(0);
    if constexpr (M::f32) {
        // ln(c/U2) + 1 - c >= 0 as c >= U2 e^(c - 1): one transcendental
        if (!acc) acc = cc >= U2 * __builtin_amdgcn_exp2f(M::fma_(cc, 1.44269504088896341f, -1.44269504088896341f));
    } else {
        if (!acc) acc = M::log_(M::div_(cc, U2)) + T(1) - cc >= T(0);
    }
    if (acc) { ch = c_; sh = q * s_; }
    return acc;
}

// A link's Delta E in the lattice's fixed point 2^-fxb (FP64 path).  The FP32
// path sums a thread's links at 2^-25 in 32 bits (|Delta E| <= 2 R <= 12 per
// link, at most 4 links per thread) and shifts once: fxb >= 26 for L <= 32.
__device__ __forceinline__ long long to_fixed(double v, const LatDev& L) { return __double2ll_rn(v * L.fx); }

// The per-link walk carries the energy kWalkBits finer than the class sums:
// it adds links into a plain 64-bit sum, so the 13 bits the class sums keep
// for their arrival count are free (|sum| <= 6V 2^(fxb + 12) <= 2^61).  An
// FP32 link's Delta E is the class sums' 2^-25 value shifted, so FP32 energies
// are those of the class-wise passes exactly.
constexpr int kWalkBits = 12;

template <typename T>
__device__ __forceinline__ long long link_fixed(T dE, const LatDev& L) {
    if constexpr (Math<T>::f32) return (long long)__float2int_rn(dE * 33554432.0f) << (L.fxb + kWalkBits - 25);
    else return __double2ll_rn((double)dE * (L.fx * (double)(1 << kWalkBits)));
}

// New angle and local-action change of a heatbath link from the accepted
// half-angle pair (c_, s_) = (cos, q sin)(pi V1 / 2): e^{iX} is
// (c_ + i s_)^2 / nrm, negated for a negative coupling, and
// theta' = arg[e^{iX} (C - i S)].
template <typename T>
__device__ __forceinline__ void hb_new_angle(T c_, T s_, T C, T S, T R, T kap, T eps_old, T& t_new, T& dE) {
    using M = Math<T>;
    T er = fms2(c_, c_, s_, s_), ei = T(2) * c_ * s_;
    const T nrm = fma2(c_, c_, s_, s_);
    if (kap < T(0)) { er = -er; ei = -ei; }
    T pr = C, pi = -S;
    if (R == T(0)) { pr = T(1); pi = T(0); }
    const T zr = fms2(er, pr, ei, pi), zi = fma2(er, pi, ei, pr);
    t_new = M::atan2_(zi, zr);
    if (!M::f32 && t_new >= M::pi()) t_new -= T(2) * M::pi();
    dE = M::div_(R * er, nrm) - eps_old;
}

// The fused pass's version of hb_new_angle: the heatbath angle is not
// stored, only its overrelaxation -2 phi - theta' = -phi - X (mod 2 pi), i.e.
// arg[e^{-iX} (C - i S)] (for vanishing staples, -X), so neither the heatbath
// angle's arctangent nor its sine and cosine are needed; dE as there.
template <typename T>
__device__ __forceinline__ void hb_or_new_angle(T c_, T s_, T C, T S, T R, T kap, T eps_old, T& t_or, T& dE) {
    using M = Math<T>;
    T er = fms2(c_, c_, s_, s_), ei = T(2) * c_ * s_;
    const T nrm = fma2(c_, c_, s_, s_);
    if (kap < T(0)) { er = -er; ei = -ei; }
    T pr = C, pi = -S;
    if (R == T(0)) { pr = T(1); pi = T(0); }
    const T zr = fma2(er, pr, ei, pi), zi = fms2(er, pi, ei, pr);   // (er - i ei)(pr + i pi)
    t_or = M::atan2_(zi, zr);
    if (!M::f32 && t_or >= M::pi()) t_or -= T(2) * M::pi();
    dE = M::div_(R * er, nrm) - eps_old;
}

// Overrelaxation of one link with staple sums (C, S): theta' = -2 phi - theta
// = arg[(C - i S)^2 e^{-i theta}]; a link with vanishing staples is reflected.
// (so, co) = (sin, cos) theta, as sincos_rad gives them.
template <typename T>
__device__ __forceinline__ T or_angle_sc(T t, T so, T co, T C, T S) {
    using M = Math<T>;
    T t_new;
    if (C == T(0) && S == T(0)) {
        t_new = -t;
    } else {
        const T ar = fms2(C, C, S, S), ai = T(-2) * C * S;   // (C - iS)^2
        const T zr = fma2(ar, co, ai, so);                   // times (cos - i sin)
        const T zi = fms2(ai, co, ar, so);
        t_new = M::atan2_(zi, zr);
    }
    if (!M::f32 && t_new >= M::pi()) t_new -= T(2) * M::pi();
    return t_new;
}

template <typename T>
__device__ __forceinline__ T or_angle(T t, T C, T S) {
    T so, co;
    Math<T>::sincos_rad(t, &so, &co);
    return or_angle_sc(t, so, co, C, S);
}

// ln W(E) = -ln rho~(E) of the multicanonical weight (Sec. 2.6): in interval
// k, -ln rho~(c_k) + a_k (E - c_k); below the first and above the last
// interval the first and last pieces continue, i.e. W = e^{a_0 E + c_1} and
// e^{a_{n-1} E + c_2} with the constants fixed by continuity.
__device__ __forceinline__ double muca_lnw(const LatDev& L, const DevState& s, double E) {
    const double* c = s.cen + L.itv0;
    const double lo = c[0] - 0.5 * L.ds;
    int k = (int)floor((E - lo) / L.ds);
    k = k < 0 ? 0 : (k > L.n_itv - 1 ? L.n_itv - 1 : k);
    return -s.mu_lnrho[L.itv0 + k] + s.a[L.itv0 + k] * (E - c[k]);
}

// ---------------------------------------------------------------------------
// Heatbath class pass.  Link conditional ~ exp(a R cos(theta + phi)) with
// (C, S) the staple sums, R = |C + iS|, phi = arg(C + iS); theta' = X - phi
// with X ~ von Mises(a R) by Best & Fisher's wrapped-Cauchy envelope in its
// half-angle form: tan(X/2) = q tan(pi V1 / 2), q = (1 - rho)/(1 + rho).
// theta' is formed as arg[(cos(pi V1/2) + i q sin(pi V1/2))^2 (C - i S)], and
// the new local action is R cos X.
//
// Each thread owns the LPT class links of its column in a tile (all their
// loads are issued before the arithmetic).  Sampler schedule: every link
// tries attempts 0 and 1 (one Philox call); the few links that reject both
// are queued in LDS and later rounds give each queued link its next two
// attempts with full lanes, so the lockstep cost of the acceptance tail is
// paid per block, not per wavefront.  Each link still takes its first
// accepted attempt in order.
// ---------------------------------------------------------------------------
template <typename T, int MU, int LPT, int VAR>
__device__ __forceinline__ void hb_block(const LatTable& lt, T* __restrict__ th, const DevState& s, int parity,
                                         int mode, int kind, uint32_t k0, uint32_t k1, int b) {
    using M = Math<T>;
    constexpr int NT = kBlock * LPT;
    // queued links keep only their |kappa|: the queue recomputes the sampler
    // constants (the same operations, so the same values), which keeps the
    // block's LDS small enough for one more resident block per CU
    __shared__ T s_ak[NT], s_ch[NT], s_sh[NT];
    __shared__ unsigned char s_res[NT];
    __shared__ short s_queue[2][NT];
    __shared__ int s_qn[2];
    int li = 0;
#pragma unroll 1
    while (li + 1 < lt.n && b >= lt.l[li + 1].hb_block0) ++li;
    const LatDev& L = lt.l[li];
    if (mode == kModeApproach && s.lat_done[li]) return;
    const int rel = b - L.hb_block0;
    const int cl = rel / L.hb_bpc;
    const int tile = rel - cl * L.hb_bpc;
    const int g = L.chain0 + cl;
    const int colour = 2 * MU + parity;
    const int tid = threadIdx.x;
    const uint64_t curw = *reinterpret_cast<const uint64_t*>(s.cur + 8 * g);
    T* chain = chain_base(L, th, cl);
    const int gi = s.itv[g];
    const double acoup = mode == kModeApproach ? s.b[8 * g + colour] : (mode == kModeMuca ? s.mu_b[li] : s.a[gi]);
    const uint32_t sweep = kind == kApproach ? *s.approach_ctr : *s.sweep_ctr;
    const uint32_t c1base = ctr1_word(0, (uint32_t)colour, (uint32_t)kind, (uint32_t)L.lat_id);
    const uint32_t c3 = (uint32_t)(gi - L.itv0);
    const int own = (int)((curw >> (8 * colour)) & 1ull);
    T* pcur = chain + (size_t)(own * 8 + colour) * L.V2;
    const T* pown = pcur;
    // the fused pass's in-place store; a tuner's timing launch leaves the
    // state as it is and writes both angles into the non-current plane
    T* pinpl = mode == kModeTune ? chain + (size_t)((own ^ 1) * 8 + colour) * L.V2 : pcur;
    T* palt = chain + (size_t)((own ^ 1) * 8 + colour) * L.V2;
    const ColTile ct = col_tile<LPT>(L, tile, tid);
    const ColNbr nb = col_nbr(L, ct, parity);
    const uint32_t pos = ct.pos;

    T C[LPT], S[LPT], t_old[LPT];
    uint32_t hl[LPT];
    bool in[LPT];
    col_staples<T, MU, LPT, false>(L, chain, curw, parity, ct, nb, pos, pown, C, S, t_old, hl, in);
    if (tid == 0) s_qn[0] = 0;
    T eps_old[LPT], R[LPT], kap[LPT], ch[LPT], sh[LPT];
    T t_or_old[LPT];   // fused pass: the old angle's overrelaxation, from the sine and cosine at hand
    bool got[LPT];
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
        const uint32_t h = hl[r];
        const int e = r * kBlock + tid;
        got[r] = true;
        ch[r] = T(1); sh[r] = T(0); eps_old[r] = T(0); R[r] = T(0); kap[r] = T(0);
        t_or_old[r] = T(0);
        if (in[r]) {
            T so, co;
            M::sincos_rad(t_old[r], &so, &co);
            eps_old[r] = fms2(C[r], co, S[r], so);
            if constexpr (VAR == kHbFuseOr) t_or_old[r] = or_angle_sc(t_old[r], so, co, C[r], S[r]);
            R[r] = M::sqrt_(fma2(C[r], C[r], S[r], S[r]));
            kap[r] = (T)acoup * R[r];
            const T ak = kap[r] < T(0) ? -kap[r] : kap[r];
            T q, rm1, kg2;
            vm_constants(ak, q, rm1, kg2);
            const uint4 w = philox10(make_uint4(h, c1base, sweep, c3), k0, k1);
            if (ak == T(0)) {
                M::sincos_halfpi_w(w.x, &sh[r], &ch[r]);
            } else {
                got[r] = vm_attempt(w.x, w.y, q, rm1, kg2, ch[r], sh[r]);
                if (!got[r]) got[r] = vm_attempt(w.z, w.w, q, rm1, kg2, ch[r], sh[r]);
            }
            if (!got[r]) {
                s_ak[e] = ak;
                s_res[e] = 0;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < LPT; ++r)
        if (!got[r]) s_queue[0][atomicAdd(&s_qn[0], 1)] = (short)(r * kBlock + tid);
    __syncthreads();
    int cq = 0;
    for (int m = 1; m < kVmCap / 2; ++m) {
        const int n = s_qn[cq];
        if (n == 0) break;
        if (tid == 0) s_qn[cq ^ 1] = 0;
        __syncthreads();
        for (int i = tid; i < n; i += kBlock) {
            const int e = s_queue[cq][i];
            // queue entry e = r kBlock + tid: link r of thread tid
            const uint32_t he = ct.pos0 + (uint32_t)(e & (kBlock - 1)) + L.P * (uint32_t)(ct.x3_0 + e / kBlock);
            const uint4 w = philox10(make_uint4(he, c1base | (uint32_t)m, sweep, c3), k0, k1);
            T qe, rme, kge;
            vm_constants(s_ak[e], qe, rme, kge);
            T che = T(1), she = T(0);
            bool acc = vm_attempt(w.x, w.y, qe, rme, kge, che, she);
            if (!acc) acc = vm_attempt(w.z, w.w, qe, rme, kge, che, she);
            if (acc) {
                s_ch[e] = che;
                s_sh[e] = she;
                s_res[e] = 1;
            } else {
                s_queue[cq ^ 1][atomicAdd(&s_qn[cq ^ 1], 1)] = (short)e;
            }
        }
        __syncthreads();
        cq ^= 1;
    }
    long long fx = 0;
    int fx32 = 0;   // FP32: the thread's class links at 2^-25 (|dE| <= 12 per link, LPT <= 4)
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
        const uint32_t h = hl[r];
        if (!in[r]) continue;
        const int e = r * kBlock + tid;
        bool ok = got[r];
        T c_ = ch[r], s_ = sh[r];
        if (!ok && s_res[e]) {
            c_ = s_ch[e];
            s_ = s_sh[e];
            ok = true;
        }
        T t_new = t_old[r];
        T dE = T(0);
        if constexpr (VAR == kHbFuseOr) {
            // the class's overrelaxation follows at once, on the same staples:
            // of the heatbath candidate into the alternate plane, of the old
            // angle in place; the pass's decision picks the plane
            T t_or_new = t_or_old[r];
            if (ok) hb_or_new_angle(c_, s_, C[r], S[r], R[r], kap[r], eps_old[r], t_or_new, dE);
            st_plane(palt, h, t_or_new);
            st_plane(pinpl, h, t_or_old[r]);
        } else {
            if (ok) hb_new_angle(c_, s_, C[r], S[r], R[r], kap[r], eps_old[r], t_new, dE);
            st_plane(palt, h, t_new);
        }
        if constexpr (VAR == kHbPre) {
            const size_t j = (size_t)L.lbase + (size_t)cl * L.V2 + h;
            T* lc = static_cast<T*>(s.link_cst);
            s.link_d[j] = ok ? link_fixed(dE, L) : kLinkNone;
            lc[j] = C[r];
            lc[s.link_n + j] = S[r];
            lc[2 * s.link_n + j] = t_old[r];
        }
        if constexpr (M::f32) fx32 += __float2int_rn(dE * 33554432.0f);
        else fx += to_fixed((double)dE, L);
    }
    if constexpr (VAR == kHbPre) return;
    if constexpr (M::f32) fx = (long long)fx32 << (L.fxb - 25);
    const long long tot = block_sum_i64(fx);
    long long total = 0;
    if (threadIdx.x == 0 && chain_arrive(s.acc + g, tot, L.hb_bpc, &total)) {
        const double E0 = s.E[g];
        const double En = E0 + (double)total * L.fxinv;
        const double lo = s.lo[gi], hi = s.hi[gi];
        bool acc;
        if (mode == kModeRestricted) {
            acc = En >= lo && En <= hi;
        } else if (mode == kModeApproach) {
            const double d0 = fmax(0.0, fmax(lo - E0, E0 - hi));
            const double d1 = fmax(0.0, fmax(lo - En, En - hi));
            acc = d1 <= d0;
            const double cen = s.cen[gi];
            const int sg = cen > En ? 1 : (cen < En ? -1 : 0);
            const int qq = 8 * g + colour;   // one coupling per colour class
            double eta = s.eta[qq];
            const int sp = s.sprev[qq];
            if (sp != 0 && sg != 0) eta = sg == sp ? fmin(0.05, 1.2 * eta) : fmax(1e-6, 0.5 * eta);
            s.eta[qq] = eta;
            s.b[qq] = fmin(4.0, fmax(0.0, s.b[qq] + eta * (double)sg));
            s.sprev[qq] = sg;
        } else if (mode == kModeMuca) {
            // target W(E) = 1/rho~(E), proposal the class heatbath at coupling
            // b: the proposal's normalisation depends only on the other
            // classes, so the Metropolis-Hastings ratio is
            // W(E')/W(E) e^{-b (E' - E)}
            const double lr = muca_lnw(L, s, En) - muca_lnw(L, s, E0) - acoup * (En - E0);
            const uint4 w = philox10(make_uint4(c3, ctr1_word(0, (uint32_t)colour, kMuca, (uint32_t)L.lat_id), sweep, 0u),
                                     k0, k1);
            acc = lr >= 0.0 || ((double)w.x + 0.5) * 0x1p-32 < exp(lr);
        } else {
            acc = mode == kModeFree;
        }
        if (mode != kModeTune) s.hb_prop[g] += 1ull;
        if (acc) {
            s.cur[8 * g + colour] ^= (uint8_t)1;
            s.E[g] = En;
            s.bits[g] |= (uint16_t)(1u << colour);
            s.hb_acc[g] += 1ull;
            if constexpr (VAR == kHbFuseOr) {
                if (mode != kModeTune) s.fu_acc[g] += 1ull;
            }
        }
        atomicExch(s.acc + g, 0ull);
    }
}

// The plain FP32 pass with 4 class links per thread: registers kept to 72
// so that seven wavefronts per SIMD fit (the LDS of the queue allows more).
// Measured: heatbath 98.1 -> 97.0 us at L=20 x 128; the fused pass, capped
// the same way, slowed from 108 to 132 us, so it keeps its registers.
template <typename T, int LPT, int VAR>
struct HbWaves { static constexpr int value = (sizeof(T) == 4 && LPT == 4 && VAR == kHbPlain) ? 7 : 1; };

template <typename T, int MU, int LPT, int VAR>
__global__ __launch_bounds__(kBlock, (HbWaves<T, LPT, VAR>::value)) void k_hb(LatTable lt, T* __restrict__ th, DevState s, int parity, int mode,
                                               int kind, uint32_t k0, uint32_t k1, int reverse) {
    const int b0 = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    hb_block<T, MU, LPT, VAR>(lt, th, s, parity, mode, kind, k0, k1, reverse ? (int)gridDim.x - 1 - b0 : b0);
}

// ---------------------------------------------------------------------------
// Heatbath class pass under the per-link constraint (Sec. 2.4: the energy
// restriction imposed when each new angle is generated).  The links of the
// class are taken one after another in half-index order, each from its
// conditional restricted to the values that keep the running energy in
// [lo, hi], and the energy is carried from link to link.  Links of one class
// share no plaquette, so only that energy couples them.  Per link: the first
// of the class heatbath's own attempts (same counters) that passes the
// sampler test AND keeps E inside; if none of the 64 does, the exact arc
// sampler (attempts 64..127 of the counter's attempt field): on
// x = |X| in [acos u_hi, acos u_lo], where the window on cos X is [u_lo, u_hi],
// exp(k cos x) lies under exp(k u_hi - lam (x - x_a)) with
// lam = k min(sin x_a, (u_hi - u_lo)/(x_b - x_a)), since the secant slope of
// cos from x_a is the mean of sin over [x_a, x], smallest at an end of the
// arc; x comes from that truncated exponential, is kept with probability
// exp(k (cos x - u_hi) + lam (x - x_a)), and its sign is a fair bit.
//
// The candidate pre-pass (k_hb<..., kHbPre>, mode kModeLinkPre) has
// written, per class link, the free heatbath candidate into the alternate
// plane, its Delta E in the walk's fixed point, and the link's staples and
// old angle.  That candidate is the first attempt passing the sampler test;
// it is the constrained draw whenever it keeps E inside.  The walk (one
// wavefront per chain, the block's other wavefronts staging the next tile of
// candidates in LDS) scans the candidates in order, 1024 at a time:
// wavefront prefix sums of Delta E give the running E before every link, the
// first link whose candidate leaves [lo, hi] is re-drawn (attempt j on lane
// j, then arc attempt i on lane i; the lowest successful lane wins, which is
// the first success in attempt order), and the rest of the step is checked
// again with its running sums shifted by that link's change of Delta E.  E
// is carried exactly in fixed point (12 bits finer than the class sums), so
// the result does not depend on the scan's blocking.
// ---------------------------------------------------------------------------
constexpr int kWalkTile = 2048;          // class links staged in LDS per tile
constexpr int kWalkPer = 16;             // links per lane per scan step (1024 per step)

__device__ __forceinline__ long long fx_bound(double v) {
    return v > 4.0e18 ? 4000000000000000000ll : (v < -4.0e18 ? -4000000000000000000ll : (long long)v);
}

// Re-draw class link h with the running sum Ssum before it (whole wavefront;
// staples and old angle from LDS).  Returns the link's fixed-point Delta E
// on every lane and writes its new angle into the alternate plane.
template <typename T>
__device__ __forceinline__ long long link_redraw(const LatDev& L, T* palt, uint32_t h, T C, T S, T t_old, int colour,
                                                 int kind, uint32_t sweep, uint32_t c3, uint32_t k0, uint32_t k1,
                                                 double a, double fxw, double Erun, double lo, double hi,
                                                 long long Ssum, long long lo_fx, long long hi_fx, unsigned& arcs) {
    using M = Math<T>;
    const int lane = threadIdx.x & 63;
    T so, co;
    M::sincos_rad(t_old, &so, &co);
    const T eps_old = fms2(C, co, S, so);
    const T R = M::sqrt_(fma2(C, C, S, S));
    const T kap = (T)a * R;
    const T ak = kap < T(0) ? -kap : kap;
    T q, rm1, kg2;
    vm_constants(ak, q, rm1, kg2);
    // the sampler's attempts, attempt j = lane on this lane
    const uint32_t c1base = ctr1_word(0, (uint32_t)colour, (uint32_t)kind, (uint32_t)L.lat_id);
    const uint4 w = philox10(make_uint4(h, c1base | (uint32_t)(lane >> 1), sweep, c3), k0, k1);
    T ch = T(1), sh = T(0);
    bool acc;
    if (ak == T(0)) {
        acc = lane == 0;
        M::sincos_halfpi_w(w.x, &sh, &ch);
    } else {
        acc = (lane & 1) ? vm_attempt(w.z, w.w, q, rm1, kg2, ch, sh) : vm_attempt(w.x, w.y, q, rm1, kg2, ch, sh);
    }
    T t_c = t_old, dE_c = T(0);
    long long d_c = 0;
    bool ok = false;
    if (acc) {
        hb_new_angle(ch, sh, C, S, R, kap, eps_old, t_c, dE_c);
        d_c = link_fixed(dE_c, L);
        ok = Ssum + d_c >= lo_fx && Ssum + d_c <= hi_fx;
    }
    const unsigned long long m1 = __ballot(ok);
    if (m1) {
        const int f = __ffsll((long long)m1) - 1;
        if (lane == f) st_plane(palt, h, t_c);
        return __shfl(d_c, f, 64);
    }
    // exact arc sampler, in FP64 for either state precision
    const double Rd = (double)R, kd = (double)kap, akd = (double)ak, ed = (double)eps_old;
    const double Aw = lo - (Erun - ed), Bw = hi - (Erun - ed);
    double ulo = -1.0, uhi = 1.0;
    if (Rd > 0.0) {
        ulo = fmin(1.0, fmax(-1.0, kd < 0.0 ? -Bw / Rd : Aw / Rd));
        uhi = fmin(1.0, fmax(-1.0, kd < 0.0 ? -Aw / Rd : Bw / Rd));
    }
    const double xa = acos(uhi), xb = acos(ulo), W = xb - xa;
    bool ok2 = false;
    double t2 = 0.0;
    long long d2 = 0;
    if (W > 0.0) {
        const double lam = akd * fmin(sin(xa), (uhi - ulo) / W);
        const uint4 v = philox10(
            make_uint4(h, ctr1_word((uint32_t)(64 + lane), (uint32_t)colour, (uint32_t)kind, (uint32_t)L.lat_id),
                       sweep, c3), k0, k1);
        const double V = (double)M::unif(v.x), U = (double)M::unif(v.y);
        const double Tt = lam * W < 1e-12 ? V * W : -log1p(V * expm1(-lam * W)) / lam;
        const double xx = fmin(xa + Tt, xb);
        if (log(U) <= akd * (cos(xx) - uhi) + lam * Tt) {
            const double X = (v.z >> 31) ? -xx : xx;
            const double sg = kd < 0.0 ? -1.0 : 1.0;
            double sx, cx;
            sincos(X, &sx, &cx);
            const double Cd = (double)C, Sd = (double)S;
            t2 = atan2(sg * (sx * Cd - cx * Sd), sg * (cx * Cd + sx * Sd));
            if (t2 >= 3.14159265358979323846) t2 -= 6.28318530717958647692;
            d2 = __double2ll_rn((sg * Rd * cx - ed) * fxw);
            ok2 = Ssum + d2 >= lo_fx && Ssum + d2 <= hi_fx;
        }
    }
    const unsigned long long m2 = __ballot(ok2);
    if (m2) {
        const int f = __ffsll((long long)m2) - 1;
        if (lane == f) st_plane(palt, h, (T)t2);
        ++arcs;
        return __shfl(d2, f, 64);
    }
    if (lane == 0) st_plane(palt, h, t_old);
    return 0;
}

// Stage tile k of a chain's candidates (Delta E, staples, old angle) into LDS
// buffer `buf`, by threads [first, first + count) of the block; every thread
// issues its loads for several entries before its LDS stores, so a tile costs
// a few memory round trips, not one per entry.
template <typename T>
__device__ __forceinline__ void walk_stage(const DevState& s, size_t jb, uint32_t V2, int k, long long* sd, T* sc,
                                           T* ss, T* st, int first, int count) {
    constexpr int U = 8;
    const uint32_t t0 = (uint32_t)k * kWalkTile;
    const int nt = (int)min((uint32_t)kWalkTile, V2 - t0);
    const T* lc = static_cast<const T*>(s.link_cst);
    for (int base = (int)threadIdx.x - first; base < nt; base += U * count) {
        long long dd[U];
        T cc[U], sn[U], tt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * count;
            if (i < nt) {
                const size_t j = jb + t0 + i;
                dd[u] = s.link_d[j];
                cc[u] = lc[j];
                sn[u] = lc[s.link_n + j];
                tt[u] = lc[2 * s.link_n + j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * count;
            if (i < nt) {
                sd[i] = dd[u];
                sc[i] = cc[u];
                ss[i] = sn[u];
                st[i] = tt[u];
            }
        }
    }
}

// One block per chain.  The walk is a chain of dependent steps and runs on
// wavefront 0 alone (no barriers inside a tile; the first link whose
// candidate leaves the window is found with one ballot, since lane l owns
// links 16 l .. 16 l + 15 of the step; after a re-draw only the entries
// after it are checked again, with their running sums shifted by the change
// of that link's Delta E), while wavefronts 1-3 stage the next tile into the
// other LDS buffer.
template <typename T, int MU>
__global__ __launch_bounds__(kBlock) void k_link_walk(LatTable lt, T* __restrict__ th, DevState s, int parity, int kind,
                                                      uint32_t k0, uint32_t k1) {
    __shared__ long long s_d[2][kWalkTile];
    __shared__ T s_c[2][kWalkTile], s_s[2][kWalkTile], s_t[2][kWalkTile];
    const int g = (int)blockIdx.x;
    int li = 0;
#pragma unroll 1
    while (li + 1 < lt.n && g >= lt.l[li + 1].chain0) ++li;
    const LatDev& L = lt.l[li];
    const int cl = g - L.chain0;
    const int colour = 2 * MU + parity;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const size_t jb = (size_t)L.lbase + (size_t)cl * L.V2;
    const int ntiles = (int)((L.V2 + kWalkTile - 1) / kWalkTile);
    walk_stage<T>(s, jb, L.V2, 0, s_d[0], s_c[0], s_s[0], s_t[0], 0, kBlock);
    __syncthreads();
    if (wid == 0) {
        const uint64_t curw = *reinterpret_cast<const uint64_t*>(s.cur + 8 * g);
        T* chain = chain_base(L, th, cl);
        const int own = (int)((curw >> (8 * colour)) & 1ull);
        T* palt = chain + (size_t)((own ^ 1) * 8 + colour) * L.V2;
        const int gi = s.itv[g];
        const double a = s.a[gi];
        const double E0 = s.E[g];
        const double lo = s.lo[gi], hi = s.hi[gi];
        const double fxw = L.fx * (double)(1 << kWalkBits), fxwinv = L.fxinv / (double)(1 << kWalkBits);
        const long long lo_fx = fx_bound(ceil((lo - E0) * fxw)), hi_fx = fx_bound(floor((hi - E0) * fxw));
        const uint32_t sweep = *s.sweep_ctr;
        const uint32_t c3 = (uint32_t)(gi - L.itv0);
        long long Ssum = 0;
        unsigned fixes = 0, arcs = 0;
        for (int k = 0; k < ntiles; ++k) {
            const int buf = k & 1;
            const uint32_t t0 = (uint32_t)k * kWalkTile;
            const int nt = (int)min((uint32_t)kWalkTile, L.V2 - t0);
            const long long* sd = s_d[buf];
            int j0 = 0;
            while (j0 < nt) {
                // one step: candidates j0 .. j0 + 1023, lane l owning 16 l .. 16 l + 15
                const int e0 = j0 + kWalkPer * lane;
                long long dv[kWalkPer], loc = 0;
                unsigned none = 0;   // entries without a free candidate
#pragma unroll
                for (int q = 0; q < kWalkPer; ++q) {
                    dv[q] = e0 + q < nt ? sd[e0 + q] : 0;
                    if (dv[q] == kLinkNone) {
                        dv[q] = 0;
                        none |= 1u << q;
                    }
                    loc += dv[q];
                }
                long long incl = loc;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const long long v = __shfl_up(incl, off, 64);
                    if (lane >= off) incl += v;
                }
                // running sum before this lane's first entry; a re-draw shifts
                // it by the same delta for every later entry of the step
                long long base = Ssum + incl - loc;
                const long long tot = __shfl(incl, 63, 64);
                long long shift = 0;
                int pos = j0;
                for (;;) {
                    long long run = base, before = 0;
                    int bad = -1;
#pragma unroll
                    for (int q = 0; q < kWalkPer; ++q) {
                        const int e = e0 + q;
                        if (bad >= 0 || e >= nt) continue;
                        const long long r1 = run + dv[q];
                        if (e >= pos && (((none >> q) & 1u) || r1 < lo_fx || r1 > hi_fx)) {
                            bad = e;
                            before = run;
                        }
                        run = r1;
                    }
                    const unsigned long long mb = __ballot(bad >= 0);
                    if (mb == 0) break;
                    const int f = __ffsll((long long)mb) - 1;
                    const int b = __shfl(bad, f, 64);
                    const long long S_b = __shfl(before, f, 64);
                    const long long d_old = sd[b] == kLinkNone ? 0 : sd[b];
                    const long long d_new =
                        link_redraw<T>(L, palt, t0 + (uint32_t)b, s_c[buf][b], s_s[buf][b], s_t[buf][b], colour, kind,
                                       sweep, c3, k0, k1, a, fxw, E0 + (double)S_b * fxwinv, lo, hi, S_b, lo_fx,
                                       hi_fx, arcs);
                    ++fixes;
                    const long long delta = d_new - d_old;
                    shift += delta;
                    if (lane >= f) base += delta;
                    pos = b + 1;
                }
                Ssum += tot + shift;
                j0 = min(j0 + kWalkPer * 64, nt);
            }
            __syncthreads();   // pairs with the stagers' barrier of this tile
        }
        if (lane == 0) {
            s.E[g] = E0 + (double)Ssum * fxwinv;
            s.cur[8 * g + colour] ^= (uint8_t)1;
            s.bits[g] |= (uint16_t)(1u << colour);
            s.hb_prop[g] += 1ull;
            s.hb_acc[g] += 1ull;
            s.link_fix[g] += fixes;
            s.link_arc[g] += arcs;
        }
    } else {
        for (int k = 0; k < ntiles; ++k) {
            if (k + 1 < ntiles) {
                const int nb = (k + 1) & 1;
                walk_stage<T>(s, jb, L.V2, k + 1, s_d[nb], s_c[nb], s_s[nb], s_t[nb], 64, kBlock - 64);
            }
            __syncthreads();   // tile k walked, tile k + 1 staged
        }
    }
}

// ---------------------------------------------------------------------------
// Overrelaxation class pass: theta' = arg[(C - i S)^2 e^{-i theta}] = -2 phi - theta,
// LPT class links per thread.
// ---------------------------------------------------------------------------
template <typename T, int MU, int LPT>
__device__ __forceinline__ void or_block(const LatTable& lt, T* __restrict__ th, const DevState& s, int parity,
                                         int to_alt, int b) {
    using M = Math<T>;
    constexpr int NT = kBlock * LPT;
    int li = 0;
#pragma unroll 1
    while (li + 1 < lt.n && b >= lt.l[li + 1].or_block0) ++li;
    const LatDev& L = lt.l[li];
    const int rel = b - L.or_block0;
    const int cl = rel / L.or_bpc;
    const int tile = rel - cl * L.or_bpc;
    const int g = L.chain0 + cl;
    const int colour = 2 * MU + parity;
    const uint64_t curw = *reinterpret_cast<const uint64_t*>(s.cur + 8 * g);
    T* chain = chain_base(L, th, cl);
    T* pown = plane_ptr(chain, curw, colour, L.V2);
    // timing runs of the tuner write to the non-current plane (state unchanged)
    T* pout = to_alt ? chain + (size_t)(((((curw >> (8 * colour)) & 1ull) ^ 1ull) * 8ull) + colour) * L.V2 : pown;
    const ColTile ct = col_tile<LPT>(L, tile, (int)threadIdx.x);
    const ColNbr nb = col_nbr(L, ct, parity);
    const uint32_t pos = ct.pos;
    T C[LPT], S[LPT], t_old[LPT];
    uint32_t hl[LPT];
    bool in[LPT];
    col_staples<T, MU, LPT, true>(L, chain, curw, parity, ct, nb, pos, pown, C, S, t_old, hl, in);
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
        if (!in[r]) continue;
        st_plane(pout, hl[r], or_angle(t_old[r], C[r], S[r]));
    }
}

template <typename T, int MU, int LPT>
__global__ __launch_bounds__(kBlock) void k_or(LatTable lt, T* __restrict__ th, DevState s, int parity, int to_alt,
                                               int reverse) {
    const int b0 = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    or_block<T, MU, LPT>(lt, th, s, parity, to_alt, reverse ? (int)gridDim.x - 1 - b0 : b0);
}

// ---------------------------------------------------------------------------
// cos of a plaquette angle in FP64 (four link angles in [-pi, pi], so
// |x| <= 4 pi): x = k pi + r with |r| <= pi/2 by Cody and Waite's two-part
// reduction (pi_hi keeps 48 significant bits, so k pi_hi is exact for
// |k| <= 8), cos x = (-1)^k cos r, and cos r by its Taylor series through r^22
// (truncation < 2e-17 on |r| <= pi/2; measured error < 2.5e-16 absolute over
// |x| <= 4 pi).  Fifteen FP64 operations, no branches.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cos_plaq(double x) {
    const double k = rint(x * 0.31830988618379067);          // 1/pi
    double r = __fma_rn(-k, 0x1.921fb54442d00p+1, x);         // pi_hi
    r = __fma_rn(-k, 0x1.8469898cc5170p-47, r);               // pi - pi_hi
    const double u = r * r;
    double c = -0x1.0ce396db7f853p-70;                        // -1/22!
    c = __fma_rn(c, u, 0x1.e542ba4020225p-62);                //  1/20!
    c = __fma_rn(c, u, -0x1.6827863b97d97p-53);               // -1/18!
    c = __fma_rn(c, u, 0x1.ae7f3e733b81fp-45);                //  1/16!
    c = __fma_rn(c, u, -0x1.93974a8c07c9dp-37);               // -1/14!
    c = __fma_rn(c, u, 0x1.1eed8eff8d898p-29);                //  1/12!
    c = __fma_rn(c, u, -0x1.27e4fb7789f5cp-22);               // -1/10!
    c = __fma_rn(c, u, 0x1.a01a01a01a01ap-16);                //  1/8!
    c = __fma_rn(c, u, -0x1.6c16c16c16c17p-10);               // -1/6!
    c = __fma_rn(c, u, 0x1.5555555555555p-5);                 //  1/4!
    c = __fma_rn(c, u, -0.5);
    c = __fma_rn(c, u, 1.0);
    return ((int)k & 1) ? -c : c;
}

// ---------------------------------------------------------------------------
// Full FP64 energy: E = sum_{x, mu<nu} cos theta_{mu nu}(x), one thread per
// site.  The first half of a chain's blocks takes the even sites, the second
// half the odd ones, so the parity and with it every plane base is uniform
// over a block.  check (kCheck* bits) adds the health tests of the chain's
// incremental E before it is replaced: any non-finite plaquette angle, the
// drift against the recomputed E, and the recomputed E against the chain's
// restriction; failures set sticky kHealth* flags that the host reads.
// ---------------------------------------------------------------------------
template <typename T, bool OBS>
__global__ __launch_bounds__(kBlock) void k_energy(LatTable lt, const T* __restrict__ th, DevState s, int check) {
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int li = find_lat_site(lt, b);
    const LatDev& L = lt.l[li];
    const int rel = b - L.eblock0;
    const int cl = rel / L.ebpc;
    const int tile = rel - cl * L.ebpc;
    const int g = L.chain0 + cl;
    const uint64_t curw = *reinterpret_cast<const uint64_t*>(s.cur + 8 * g);
    const T* chain = chain_base(L, const_cast<T*>(th), cl);
    const int half = L.ebpc >> 1;
    const int p = tile >= half ? 1 : 0;
    const uint32_t h = (uint32_t)(tile - p * half) * kBlock + threadIdx.x;
    long long fx = 0, fa = 0;
    int bad = 0;   // a plaquette angle that is not finite
    if (h < L.V2) {
        int x[4];
        decode_half(L, h, p, x);
        double own[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) own[m] = (double)ld_plane(plane_ptr(chain, curw, 2 * m + p, L.V2), h);
        int upo[4], dno[4];
        neighbour_offsets(L, x, upo, dno);
        uint32_t hup[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) hup[m] = h + upo[m];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                const double t_nu_pmu = (double)ld_plane(plane_ptr(chain, curw, 2 * nu + (p ^ 1), L.V2), hup[mu]);
                const double t_mu_pnu = (double)ld_plane(plane_ptr(chain, curw, 2 * mu + (p ^ 1), L.V2), hup[nu]);
                const double ang = own[mu] + t_nu_pmu - t_mu_pnu - own[nu];
                bad |= !(fabs(ang) < INFINITY);
                const double cp = cos_plaq(ang);
                fx += __double2ll_rn(cp * L.fx);
                if (OBS) fa += __double2ll_rn(__fma_rn(2.0 * cp, cp, -1.0) * L.fx);   // cos 2 theta_P
            }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(s.health + g, (uint32_t)kHealthNonFinite);
    const long long tot = block_sum_i64(fx);
    long long total = 0;
    if (threadIdx.x == 0 && chain_arrive(s.eacc + g, tot, L.ebpc, &total)) {
        const double En = (double)total * L.fxinv;
        if (check) {
            // health of the chain's incremental E: its drift from the
            // recomputed value, and (restricted sweeps) that the recomputed E
            // lies in the chain's restriction up to that drift bound
            const double bound = (sizeof(T) == 4 ? 1e-5 : 1e-9) * 12.0 * (double)L.V2;
            const double d = fabs(En - s.E[g]);
            uint32_t f = 0;
            if (check & kCheckDrift) {
                s.drift[g] = fmax(s.drift[g], d);
                if (!(d <= bound)) f |= kHealthDrift;
            }
            if (check & kCheckInterval) {
                const int gi = s.itv[g];
                if (!(En >= s.lo[gi] - bound && En <= s.hi[gi] + bound)) f |= kHealthOutside;
            }
            if (f) atomicOr(s.health + g, f);
        }
        s.E[g] = En;
        atomicExch(s.eacc + g, 0ull);
    }
    if (OBS) {
        __syncthreads();   // block_sum_i64's shared partials are reused
        const long long ta = block_sum_i64(fa);
        long long tb = 0;
        if (threadIdx.x == 0 && chain_arrive(s.oacc + g, ta, L.ebpc, &tb)) {
            s.obs[g] = (double)tb * L.fxinv;
            atomicExch(s.oacc + g, 0ull);
        }
    }
}

// ---------------------------------------------------------------------------
// Hot start: theta = -pi + 2 pi U (kind 1, w0 = mu V + s, w3 = chain index),
// computed in FP64 with one fused multiply-add and rounded to the precision.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_hot_start(LatTable lt, T* __restrict__ th, DevState s, uint32_t k0,
                                                      uint32_t k1) {
    const int b = (int)blockIdx.x;
    const int li = find_lat_site(lt, b);
    const LatDev& L = lt.l[li];
    const int rel = b - L.eblock0;
    const int cl = rel / L.ebpc;
    const int tile = rel - cl * L.ebpc;
    const int g = L.chain0 + cl;
    T* chain = chain_base(L, th, cl);
    const uint32_t V = 2u * L.V2;
    const uint32_t sidx = (uint32_t)tile * kBlock + threadIdx.x;   // lexicographic site
    if (sidx < V) {
        const uint32_t r1 = fdiv(sidx, L.mL);
        const int x0 = (int)(sidx - r1 * (uint32_t)L.L);
        const uint32_t r2 = fdiv(r1, L.mL);
        const int x1 = (int)(r1 - r2 * (uint32_t)L.L);
        const uint32_t r3 = fdiv(r2, L.mL);
        const int x2 = (int)(r2 - r3 * (uint32_t)L.L);
        const int x3 = (int)r3;
        const int p = (x0 + x1 + x2 + x3) & 1;
        const uint32_t h = sidx >> 1;
        for (int mu = 0; mu < 4; ++mu) {
            const uint4 w = philox10(make_uint4((uint32_t)mu * V + sidx, ctr1_word(0, 0, kInit, (uint32_t)L.lat_id), 0u,
                                                (uint32_t)cl),
                                     k0, k1);
            const double u = Math<T>::f32 ? ((double)(w.x >> 9) + 0.5) * 0x1p-23 : ((double)w.x + 0.5) * 0x1p-32;
            const double t = __fma_rn(6.28318530717958647692, u, -3.14159265358979323846);
            chain[(size_t)(2 * mu + p) * L.V2 + h] = (T)t;
        }
    }
    if (threadIdx.x == 0 && tile == 0) {
        *reinterpret_cast<uint64_t*>(s.cur + 8 * g) = 0ull;
        s.itv[g] = g;
        s.conf[g] = g;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_export(LatDev L, const T* __restrict__ th, DevState s, T* __restrict__ out) {
    const long long V = 2ll * L.V2;
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;   // over chains x 4 x V
    if (i >= (long long)L.n_chains * 4 * V) return;
    const int cl = (int)(i / (4 * V));
    const long long r = i - (long long)cl * 4 * V;
    const int mu = (int)(r / V);
    const uint32_t sidx = (uint32_t)(r - (long long)mu * V);
    const uint32_t r1 = fdiv(sidx, L.mL);
    const int x0 = (int)(sidx - r1 * (uint32_t)L.L);
    const uint32_t r2 = fdiv(r1, L.mL);
    const int x1 = (int)(r1 - r2 * (uint32_t)L.L);
    const uint32_t r3 = fdiv(r2, L.mL);
    const int x2 = (int)(r2 - r3 * (uint32_t)L.L);
    const int p = (x0 + x1 + x2 + (int)r3) & 1;
    const uint64_t curw = *reinterpret_cast<const uint64_t*>(s.cur + 8 * (L.chain0 + cl));
    const T* chain = chain_base(L, const_cast<T*>(th), cl);
    out[i] = plane_ptr(chain, curw, 2 * mu + p, L.V2)[sidx >> 1];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_import(LatDev L, T* __restrict__ th, DevState s, const T* __restrict__ in) {
    const long long V = 2ll * L.V2;
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (long long)L.n_chains * 4 * V) return;
    const int cl = (int)(i / (4 * V));
    const long long r = i - (long long)cl * 4 * V;
    const int mu = (int)(r / V);
    const uint32_t sidx = (uint32_t)(r - (long long)mu * V);
    const uint32_t r1 = fdiv(sidx, L.mL);
    const int x0 = (int)(sidx - r1 * (uint32_t)L.L);
    const uint32_t r2 = fdiv(r1, L.mL);
    const int x1 = (int)(r1 - r2 * (uint32_t)L.L);
    const uint32_t r3 = fdiv(r2, L.mL);
    const int x2 = (int)(r2 - r3 * (uint32_t)L.L);
    const int p = (x0 + x1 + x2 + (int)r3) & 1;
    T* chain = chain_base(L, th, cl);
    chain[(size_t)(2 * mu + p) * L.V2 + (sidx >> 1)] = in[i];
    if (r == 0) {
        const int g = L.chain0 + cl;
        *reinterpret_cast<uint64_t*>(s.cur + 8 * g) = 0ull;
        s.itv[g] = g;
        s.conf[g] = g;
    }
}

// ---------------------------------------------------------------------------
// Per-sweep bookkeeping (one block): accumulate the measured energy of every
// interval, move the accept bits to the log, advance the sweep counter.
// ---------------------------------------------------------------------------
// Overrelaxation passes are always accepted (E unchanged): their bits 8..15
// are set here for sweeps that ran them.
__global__ __launch_bounds__(1024) void k_end_sweep(int n, DevState s, int measure, int approach, int with_or) {
    const long long row = s.bits_row ? *s.bits_row : 0;
    for (int g = threadIdx.x; g < n; g += blockDim.x) {
        if (measure) s.sumE[s.itv[g]] += s.E[g];
        const uint16_t bits = (uint16_t)(s.bits[g] | (with_or ? 0xff00u : 0u));
        if (s.bits_log && row < s.bits_rows_max) s.bits_log[row * n + g] = bits;
        s.bits_last[g] = bits;
        s.bits[g] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (approach) *s.approach_ctr += 1u;
        else *s.sweep_ctr += 1u;
        if (s.bits_row) *s.bits_row = row + 1;
    }
}

// Replica exchange (Sec. 2.5) between intervals k and k+1 of one lattice, for
// k = t (mod 2) at sweep t; eligible iff each configuration lies in the other
// interval; accepted with min(1, exp[(a_k - a_{k+1})(E_{k+1} - E_k)]).  Only
// the chain <-> interval labels move.
__global__ __launch_bounds__(1024) void k_replica(LatTable lt, DevState s, uint32_t k0, uint32_t k1) {
    const uint32_t t = *s.sweep_ctr;
    unsigned long long prop = 0, accd = 0;
    for (int li = 0; li < lt.n; ++li) {
        const LatDev& L = lt.l[li];
        const int npair = (L.n_chains - (int)(t & 1u)) / 2;
        for (int i = threadIdx.x; i < npair; i += blockDim.x) {
            const int k = 2 * i + (int)(t & 1u);
            if (k + 1 >= L.n_chains) continue;
            const int kg = L.chain0 + k;
            const int A = s.conf[kg], B = s.conf[kg + 1];
            const double EA = s.E[A], EB = s.E[B];
            if (!(EA >= s.lo[kg + 1] && EA <= s.hi[kg + 1] && EB >= s.lo[kg] && EB <= s.hi[kg])) continue;
            const uint4 w = philox10(make_uint4((uint32_t)k, ctr1_word(0, 0, kReplica, (uint32_t)L.lat_id), t, 0u), k0, k1);
            const double u = ((double)w.x + 0.5) * 0x1p-32;
            const double xx = (s.a[kg] - s.a[kg + 1]) * (EB - EA);
            ++prop;
            if (xx >= 0.0 || u < exp(xx)) {
                s.conf[kg] = B;
                s.conf[kg + 1] = A;
                s.itv[A] = kg + 1;
                s.itv[B] = kg;
                ++accd;
            }
        }
    }
    if (prop) atomicAdd(s.re_cnt, prop);
    if (accd) atomicAdd(s.re_cnt + 1, accd);
}

// Robbins-Monro step of every interval (eq. (kk21), Algorithm 1 sign):
// a^(n+1) = a^(n) - 12 (mean - c_k) / ((n + 1) w^2).
__global__ __launch_bounds__(1024) void k_rm_update(int n, DevState s, RunCfg cfg) {
    const int it = *s.rm_iter;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double mean = s.sumE[k] / (double)cfg.n_a;
        const double a0 = s.a[k];
        const double wk = s.w[k];
        const double an = a0 - 12.0 * (mean - s.cen[k]) / ((double)(it + 1) * wk * wk);
        const double da = an - a0;
        s.a[k] = an;
        s.a_hist[(long long)(it + 1) * n + k] = an;
        if (s.conv_iter[k] < 0 && fabs(da) < cfg.eps) {
            s.conv_iter[k] = it;
            s.conv_sweeps[k] = (long long)(it + 1) * cfg.nsw;   // approach sweeps added on the host
        }
        s.sumE[k] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) *s.rm_iter = it + 1;
}

__global__ __launch_bounds__(1024) void k_approach_init(int n, DevState s) {
    for (int q = threadIdx.x; q < 8 * n; q += blockDim.x) {
        s.b[q] = s.a[s.itv[q >> 3]];
        s.eta[q] = 0.05;
        s.sprev[q] = 0;
    }
}

__global__ __launch_bounds__(1024) void k_approach_check(LatTable lt, DevState s) {
    __shared__ int outside[kMaxLat];
    if (threadIdx.x < kMaxLat) outside[threadIdx.x] = 0;
    __syncthreads();
    for (int li = 0; li < lt.n; ++li) {
        const LatDev& L = lt.l[li];
        for (int c = threadIdx.x; c < L.n_chains; c += blockDim.x) {
            const int g = L.chain0 + c;
            const int k = s.itv[g];
            const double E = s.E[g];
            if (!(E >= s.lo[k] && E <= s.hi[k])) atomicAdd(&outside[li], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)lt.n) s.lat_outside[threadIdx.x] = outside[threadIdx.x];
}

__global__ void k_test_philox(long n, const uint4* __restrict__ ctr, uint32_t k0, uint32_t k1, uint4* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox10(ctr[i], k0, k1);
}

// Stand-alone draws of the heatbath sampler (same arithmetic as k_hb, attempts
// taken sequentially).
template <typename T>
__global__ void k_test_vonmises(long n, double kappa, uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3,
                                double* X, int* att) {
    using M = Math<T>;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T ak = (T)kappa;
    T q, rm1, kg2;
    vm_constants(ak, q, rm1, kg2);
    int a = 0;
    T ch = T(1), sh = T(0);
    for (int m = 0; m < kVmCap / 2 && !a; ++m) {
        const uint4 w = philox10(make_uint4((uint32_t)i, c1 | (uint32_t)m, c2, c3), k0, k1);
        if (ak == T(0)) { M::sincos_halfpi_w(w.x, &sh, &ch); a = 1; break; }
        if (vm_attempt(w.x, w.y, q, rm1, kg2, ch, sh)) a = 2 * m + 1;
        else if (vm_attempt(w.z, w.w, q, rm1, kg2, ch, sh)) a = 2 * m + 2;
    }
    att[i] = a;
    X[i] = a ? 2.0 * (double)M::atan2_(sh, ch) : 0.0;
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_hot_start(const LatTable& lt, T* th, DevState s, uint32_t k0, uint32_t k1, hipStream_t st) {
    hipLaunchKernelGGL(k_hot_start<T>, dim3(lt.site_blocks), dim3(kBlock), 0, st, lt, th, s, k0, k1);
}

// VAR: kHbPlain, the candidate pre-pass of the per-link constraint (kHbPre),
// or the pass followed by the class's overrelaxation (kHbFuseOr); separate
// instantiations, so that the plain pass carries none of the others' code
template <typename T, int LPT, int VAR>
static void hb_dispatch(const LatTable& lt, T* th, DevState s, int colour, int mode, int kind, uint32_t k0,
                        uint32_t k1, hipStream_t st) {
    const int p = colour & 1;
    const int rv = lt.serpentine ? p : 0;
    dim3 gr(lt.hb_blocks), bl(kBlock);
    switch (colour >> 1) {
        case 0: hipLaunchKernelGGL((k_hb<T, 0, LPT, VAR>), gr, bl, 0, st, lt, th, s, p, mode, kind, k0, k1, rv); break;
        case 1: hipLaunchKernelGGL((k_hb<T, 1, LPT, VAR>), gr, bl, 0, st, lt, th, s, p, mode, kind, k0, k1, rv); break;
        case 2: hipLaunchKernelGGL((k_hb<T, 2, LPT, VAR>), gr, bl, 0, st, lt, th, s, p, mode, kind, k0, k1, rv); break;
        default: hipLaunchKernelGGL((k_hb<T, 3, LPT, VAR>), gr, bl, 0, st, lt, th, s, p, mode, kind, k0, k1, rv); break;
    }
}

template <typename T, int VAR>
static void hb_tiles(const LatTable& lt, T* th, DevState s, int colour, int mode, int kind, uint32_t k0, uint32_t k1,
                     hipStream_t st) {
    switch (lt.hb_lpt) {
        case 1: hb_dispatch<T, 1, VAR>(lt, th, s, colour, mode, kind, k0, k1, st); break;
        case 2: hb_dispatch<T, 2, VAR>(lt, th, s, colour, mode, kind, k0, k1, st); break;
        default: hb_dispatch<T, 4, VAR>(lt, th, s, colour, mode, kind, k0, k1, st); break;
    }
}

template <typename T>
void launch_hb_pass(const LatTable& lt, T* th, DevState s, int colour, int mode, int kind, uint32_t k0, uint32_t k1,
                    hipStream_t st) {
    if (mode != kModeLink) {
        hb_tiles<T, kHbPlain>(lt, th, s, colour, mode, kind, k0, k1, st);
        return;
    }
    hb_tiles<T, kHbPre>(lt, th, s, colour, kModeLinkPre, kind, k0, k1, st);
    const int p = colour & 1;
    dim3 gr(lt.n_chains), bl(kBlock);
    switch (colour >> 1) {
        case 0: hipLaunchKernelGGL((k_link_walk<T, 0>), gr, bl, 0, st, lt, th, s, p, kind, k0, k1); break;
        case 1: hipLaunchKernelGGL((k_link_walk<T, 1>), gr, bl, 0, st, lt, th, s, p, kind, k0, k1); break;
        case 2: hipLaunchKernelGGL((k_link_walk<T, 2>), gr, bl, 0, st, lt, th, s, p, kind, k0, k1); break;
        default: hipLaunchKernelGGL((k_link_walk<T, 3>), gr, bl, 0, st, lt, th, s, p, kind, k0, k1); break;
    }
}

template <typename T>
void launch_hb_or_pass(const LatTable& lt, T* th, DevState s, int colour, int mode, uint32_t k0, uint32_t k1,
                       hipStream_t st) {
    hb_tiles<T, kHbFuseOr>(lt, th, s, colour, mode, kSweep, k0, k1, st);
}

template <typename T, int LPT>
static void or_dispatch(const LatTable& lt, T* th, DevState s, int colour, int to_alt, hipStream_t st) {
    const int p = colour & 1;
    const int rv = lt.serpentine ? p : 0;
    dim3 gr(lt.or_blocks), bl(kBlock);
    switch (colour >> 1) {
        case 0: hipLaunchKernelGGL((k_or<T, 0, LPT>), gr, bl, 0, st, lt, th, s, p, to_alt, rv); break;
        case 1: hipLaunchKernelGGL((k_or<T, 1, LPT>), gr, bl, 0, st, lt, th, s, p, to_alt, rv); break;
        case 2: hipLaunchKernelGGL((k_or<T, 2, LPT>), gr, bl, 0, st, lt, th, s, p, to_alt, rv); break;
        default: hipLaunchKernelGGL((k_or<T, 3, LPT>), gr, bl, 0, st, lt, th, s, p, to_alt, rv); break;
    }
}

template <typename T>
void launch_or_pass(const LatTable& lt, T* th, DevState s, int colour, int to_alt, hipStream_t st) {
    switch (lt.or_lpt) {
        case 1: or_dispatch<T, 1>(lt, th, s, colour, to_alt, st); break;
        case 2: or_dispatch<T, 2>(lt, th, s, colour, to_alt, st); break;
        default: or_dispatch<T, 4>(lt, th, s, colour, to_alt, st); break;
    }
}

template <typename T>
void launch_energy(const LatTable& lt, const T* th, DevState s, hipStream_t st, bool with_obs, int check) {
    if (with_obs) hipLaunchKernelGGL((k_energy<T, true>), dim3(lt.site_blocks), dim3(kBlock), 0, st, lt, th, s, check);
    else hipLaunchKernelGGL((k_energy<T, false>), dim3(lt.site_blocks), dim3(kBlock), 0, st, lt, th, s, check);
}

template <typename T>
void launch_export(const LatTable& lt, int li, const T* th, DevState s, T* out, hipStream_t st) {
    const LatDev& L = lt.l[li];
    const long long n = (long long)L.n_chains * 8ll * L.V2;
    hipLaunchKernelGGL(k_export<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, L, th, s, out);
}

template <typename T>
void launch_import(const LatTable& lt, int li, T* th, DevState s, const T* in, hipStream_t st) {
    const LatDev& L = lt.l[li];
    const long long n = (long long)L.n_chains * 8ll * L.V2;
    hipLaunchKernelGGL(k_import<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, L, th, s, in);
}

void launch_end_sweep(const LatTable& lt, DevState s, int measure, int approach, int with_or, hipStream_t st) {
    hipLaunchKernelGGL(k_end_sweep, dim3(1), dim3(1024), 0, st, lt.n_chains, s, measure, approach, with_or);
}
void launch_replica(const LatTable& lt, DevState s, uint32_t k0, uint32_t k1, hipStream_t st) {
    hipLaunchKernelGGL(k_replica, dim3(1), dim3(1024), 0, st, lt, s, k0, k1);
}
void launch_rm_update(const LatTable& lt, DevState s, RunCfg cfg, hipStream_t st) {
    hipLaunchKernelGGL(k_rm_update, dim3(1), dim3(1024), 0, st, lt.n_chains, s, cfg);
}
void launch_approach_init(const LatTable& lt, DevState s, hipStream_t st) {
    hipLaunchKernelGGL(k_approach_init, dim3(1), dim3(1024), 0, st, lt.n_chains, s);
}
void launch_approach_check(const LatTable& lt, DevState s, hipStream_t st) {
    hipLaunchKernelGGL(k_approach_check, dim3(1), dim3(1024), 0, st, lt, s);
}
void launch_test_philox(long n, const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, hipStream_t st) {
    hipLaunchKernelGGL(k_test_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ctr, k0, k1, out);
}
template <typename T>
void launch_test_vonmises(long n, double kappa, uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3,
                          double* X, int* att, hipStream_t st) {
    hipLaunchKernelGGL(k_test_vonmises<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, kappa, k0, k1, c1,
                       c2, c3, X, att);
}

#define LLR_INST(T)                                                                                              \
    template void launch_hot_start<T>(const LatTable&, T*, DevState, uint32_t, uint32_t, hipStream_t);          \
    template void launch_hb_pass<T>(const LatTable&, T*, DevState, int, int, int, uint32_t, uint32_t, hipStream_t); \
    template void launch_or_pass<T>(const LatTable&, T*, DevState, int, int, hipStream_t);                           \
    template void launch_hb_or_pass<T>(const LatTable&, T*, DevState, int, int, uint32_t, uint32_t, hipStream_t);     \
    template void launch_energy<T>(const LatTable&, const T*, DevState, hipStream_t, bool, int);                    \
    template void launch_export<T>(const LatTable&, int, const T*, DevState, T*, hipStream_t);                 \
    template void launch_import<T>(const LatTable&, int, T*, DevState, const T*, hipStream_t);                 \
    template void launch_test_vonmises<T>(long, double, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, double*, \
                                          int*, hipStream_t);
LLR_INST(float)
LLR_INST(double)
#undef LLR_INST

}  // namespace llr
