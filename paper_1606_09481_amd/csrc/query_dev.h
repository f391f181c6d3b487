// query_dev.h -- device code of the band query shared by the multi-launch
// path (query.hip) and the one-launch small-request path (small.hip): window
// half-widths and searches, the per-batch window plan, the distance test,
// and the per-wavefront count and emit walks over one work unit.
#pragma once
#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    return ((uint64_t)uniform_u32((uint32_t)(x >> 32)) << 32) | uniform_u32((uint32_t)x);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int l) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
}

// Half-width of the window of query v in slab j >= 1.  The bound is
//   s = (Kw - cosh(r_v - c_j)) / (2 sinh r_v sinh c_j),  half-width 2 asin(sqrt s),
// with cosh(r_v - c_j) = (e^{r_v} e^{-c_j} + e^{-r_v} e^{c_j}) / 2 from the
// point's table and per-slab constants, and the division by per-point and
// per-slab reciprocals: every rounding here is a few u relative, far inside
// the 2^-30 K slack of Kw.  asin and sqrt run in FP32 on the rounded s (s in
// (0, 1/2)): at most a few ulp_32 relative, covered by the 2^-16 relative
// widening; values of s below FP32 range give half-widths far below the
// 2^-44 rad absolute widening.  Returns 1 for a whole slab (half-width >= pi/2).
struct QPlan {
    double hep, hem, inv2sh;  // 0.5 e^{r_v}, 0.5 e^{-r_v}, 1 / (2 sinh r_v) (0: whole slabs)
};

__device__ __forceinline__ int half_width(const Geo &g, const QPlan &q, int j, double *delta) {
    if (!(q.inv2sh > 0.0)) return 1;
    const double C = q.hep * g.emc[j] + q.hem * g.epc[j];
    double s = ((g.Kw - C) * q.inv2sh) * g.ishc[j];
    if (!(s < 0.5)) return 1;  // sin^2(D/2) >= 1/2  <=>  D >= pi/2
    if (s < 0.0) s = 0.0;
    const float d32 = 2.0f * asinf(sqrtf((float)s));
    const double d = (double)d32 * (1.0 + 0x1p-16) + 0x1p-44;
    if (!(d < HALF_PI)) return 1;
    *delta = d;
    return 0;
}

// First position of slab j with quantised angle >= t, for t <= 2^QBITS (t =
// 2^QBITS falls in the last bucket and gives the slab end).
__device__ __forceinline__ uint32_t first_at_least(const Geo &g, int j, uint32_t t) {
    const uint32_t *T = g.btab + g.bto[j];
    const int sh = g.bshift[j];
    const uint32_t bmax = QMASK >> sh;
    const uint32_t b = min(t >> sh, bmax);
    uint32_t lo = T[b], hi = T[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((g.keys[mid] & QMASK) < t) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// Both ends of an angular range at once (independent loads in flight together).
__device__ __forceinline__ uint2 range_pos(const Geo &g, int j, uint32_t xlo, uint32_t xhi) {
    const uint32_t *T = g.btab + g.bto[j];
    const int sh = g.bshift[j];
    const uint32_t bl = xlo >> sh, bh = xhi >> sh;
    uint32_t l0 = T[bl], l1 = T[bl + 1], h0 = T[bh], h1 = T[bh + 1];
    while (l0 < l1 || h0 < h1) {
        const uint32_t ml = (l0 + l1) >> 1, mh = (h0 + h1) >> 1;
        const uint32_t kl = (l0 < l1) ? (g.keys[ml] & QMASK) : 0u;
        const uint32_t kh = (h0 < h1) ? (g.keys[mh] & QMASK) : 0u;
        if (l0 < l1) {
            if (kl < xlo) l0 = ml + 1; else l1 = ml;
        }
        if (h0 < h1) {
            if (kh <= xhi) h0 = mh + 1; else h1 = mh;
        }
    }
    return make_uint2(l0, h0);
}

// Circular window (start, count) of sorted query s (slab i) in slab j: the
// forward range of the own-slab rule when fwd (j == i), else the two-sided
// range.  The bound with c_j holds for a slab j below the query's too: the
// largest sin^2 of the half-angle allowed at distance R,
// (K - cosh(r_v - x)) / (2 sinh r_v sinh x), decreases in the candidate's
// radius x for every x when r_v <= R (its derivative has the sign of
// cosh r_v - K cosh x), so over slab j it is largest at x = c_j.
__device__ uint2 window(const Geo &g, const QPlan &qp, uint32_t s, int i, int j, double thv, uint32_t qv, bool fwd) {
    const uint32_t bs = g.bs[j], be = g.bs[j + 1], nj = be - bs;
    if (nj == 0) return make_uint2(bs, 0u);
    double delta = 0.0;
    const int whole = (j == 0) ? 1 : half_width(g, qp, j, &delta);
    if (fwd) {
        // forward range from s + 1 to the first position with key >= t (a key
        // "> x" is one ">= x + 1"), past the slab end when it wraps; one
        // search for all four cases (whole slab or not, wrapping or not)
        const double hi = thv + delta;
        const bool wrap = whole ? qv >= QHALF : hi >= TWO_PI;
        const uint32_t t = whole ? (wrap ? qv - QHALF : qv + QHALF + 1u) : qang(wrap ? hi - TWO_PI : hi) + 1u;
        const uint32_t P = first_at_least(g, j, t);
        return make_uint2(s + 1, wrap ? (be - s - 1) + (P - bs) : P - s - 1);
    }
    if (whole) return make_uint2(bs, nj);
    // [lo, hi] wraps past 0 or past 2 pi (not both: the half-width is below
    // pi / 2); one search of both ends either way, so that lanes of one
    // wavefront on different sides of the wrap take the same path
    const double lo = thv - delta, hi = thv + delta;
    const bool wlo = lo < 0.0, whi = hi >= TWO_PI;
    const uint2 r = range_pos(g, j, qang(wlo ? lo + TWO_PI : lo), qang(whi ? hi - TWO_PI : hi));
    return (wlo || whi) ? make_uint2(r.x, (be - r.x) + (r.y - bs)) : make_uint2(r.x, r.y - r.x);
}

// Windows are stored slab-major: window (v, j) of sorted query v (slab(v) <= j)
// at win[winbase[j] + v], so the 64 queries of a batch read one slab's
// windows with one coalesced load.
// One wavefront plans one batch b of 64 sorted queries (lane = query b*64+lane).
// FULL: update mode (Geo::moved): windows of the moved queries only, in every
// slab, two-sided in their own slab as in the others.
template <bool FULL = false>
__device__ __forceinline__ void plan_batch(const Geo &g, uint2 *win, uint64_t *batch_cand, uint64_t *batch_slab_off,
                                           uint32_t b, int lane) {
    // b and the slab index are wave-uniform: kept in scalar registers, the
    // per-slab geometry (offsets, constants, bucket layout) is read with
    // scalar loads instead of one dependent vector load chain per slab
    b = uniform_u32(b);
    const uint32_t s = b * BATCH + (uint32_t)lane;
    const bool valid = s < g.n;
    constexpr bool full = FULL;  // update mode: moved queries, every slab
    const int jmin = full ? 0 : (int)uniform_u32(g.keys[b * BATCH] >> QBITS);
    int i = g.B;
    uint32_t qv = 0;
    double thv = 0.0;
    QPlan qp{0.0, 0.0, 0.0};
    if (valid) {
        const uint32_t key = g.keys[s];
        i = (int)(key >> QBITS);
        qv = key & QMASK;
        thv = g.th[s];
        const double2 e = g.epm[s];
        const double shv = 0.5 * (e.x - e.y);  // sinh r as the distance test takes it
        qp.hep = 0.5 * e.x;
        qp.hem = 0.5 * e.y;
        qp.inv2sh = (shv > 0.0) ? 1.0 / (2.0 * shv) : 0.0;
    }
    const bool asks = valid && (!full || bit_of(g.moved, s));
    const int ifirst = full ? 0 : i;  // first slab with a window
    uint64_t *row = batch_slab_off + (uint64_t)b * (g.B + 1);
    for (int j = lane; j <= jmin && j <= g.B; j += 64) row[j] = 0;
    uint64_t acc = 0;
    const bool small = 64ull * g.n < (1ull << 32);
    for (int j = jmin; j < g.B; ++j) {
        uint32_t cnt = 0;
        if (asks && j >= ifirst) {
            // (an unmoved query of update mode has no window entries: its
            // first slab is past the last, and its entries are never read)
            const uint2 x = window(g, qp, s, i, j, thv, qv, !full && j == i);
            win[g.winbase[j] + s] = x;
            cnt = x.y;
        }
        // 64 window counts of at most n each: a 32-bit DPP sum (no LDS
        // round trips) whenever 64 n < 2^32, else the 64-bit shuffle sum
        acc += small ? (uint64_t)wave_bcast_u32(wave_incl_scan_u32(cnt), 63) : wave_sum_u64(cnt);
        if (lane == 0) row[j + 1] = acc;
    }
    if (lane == 0) batch_cand[b] = acc;
}

// ---------------------------------------------------------------------------
// Distance test (Eq. 3).  The canonical FP64 value is
//   V = 0.5 (ep_u em_w + em_u ep_w) + 2 (sh_u sh_w) d^2,  d = hs_u hc_w - hc_u hs_w,
// one rounding per operation, with sh = 0.5 (ep - em) (sinh r from the
// table's two exponentials).  The query-side halves (0.5 ep_u, 0.5 em_u) are
// exact power-of-two scalings, and (ep_w - em_w) rounds to exactly 2 sh_w, so
// (sh_u (ep_w - em_w)) is exactly 2 (sh_u sh_w) (a doubling is exact) and
//   V = (hep_u em_w + hem_u ep_w) + (sh_u (ep_w - em_w)) d^2
// rounds to the same bits, reading no sinh column for the candidate.
// FP32 filter, from the FP64 d rounded once and 8-byte shadows (e^r, e^-r in
// FP32) per candidate:
//   V32 = (0.5 ep32_u) em32_w + (0.5 em32_u) ep32_w + (sh32_u d32)(t32_w d32),
//   t32_w = ep32_w - em32_w  (2 sinh r_w, from the shadows).
// Against the exact W of the FP64 table values (a + sh_u t_w d^2, t_w =
// ep_w - em_w), every FP32 operand and product adds at most a relative
// u32 = 2^-24 to sums of positive terms (gamma_8 in all), and the
// subtraction adds an absolute error of at most u32 (ep_w + em_w)(1 + u32),
// which through sh_u d^2 is at most u32 (1 + u32)(b + 2 ep_u em_w / 2) <=
// 2 u32 (1 + u32) W.  So |V32 - W| <= (gamma_8 + 2.1 u32) W < 6e-7 W, and
// |V64 - W| <= gamma_6(2^-53) W; with mu = 2^-20 (9.5e-7) above their sum,
// V32 <= RD(K(1-mu)) implies V64 < K and V32 >= RU(K(1+mu)) implies V64 >= K.
// Pairs between the two thresholds are decided by V64.
// ---------------------------------------------------------------------------
struct Qv {
    double hep, hem, sh, hs, hc;
    float hep32, hem32, sh32;
};

// Candidate operands, loaded for several candidates before any is decided so
// that their memory latencies overlap.
struct Cand {
    double2 hw;  // (sin, cos) of theta_w / 2
    double2 ew;  // (exp r_w, exp -r_w)        FP64 form
    float2 f;    // FP32 (exp r_w, exp -r_w)   FP32 form
    uint32_t wi; // original index             general model (T > 0)
};

// Element i of a table column.  Unless WIDE, the byte offset is formed in 32
// bits (tables under 4 GiB, n < 2^28), which lets the load take the column
// base from scalar registers with a 32-bit per-lane offset.
template <bool WIDE, typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t i) {
    if (WIDE) return base[i];
    return *(const T *)((const char *)base + (uint32_t)(i * (uint32_t)sizeof(T)));
}

template <int FP32, bool WIDE, bool SOFT = false>
__device__ __forceinline__ void load_cand(const Geo &g, uint32_t p, Cand &c) {
    c.hw = ld<WIDE>(g.hsc, p);
    if (SOFT) c.wi = ld<WIDE>(g.idx, p);
    if (!FP32) {
        c.ew = ld<WIDE>(g.epm, p);
    } else {
        c.f = ld<WIDE>(g.f32, p);
    }
}

// Returns bit 0 = edge, bit 1 = re-decided in FP64, bit 2 = FP32 decision
// differed from FP64 (exhaustive self-check only).
// ABL (FP32 form, an ablation measurement): every candidate is also decided
// by Eq. 3 as printed, cosh r_u cosh r_w - sinh r_u sinh r_w cos(theta_u -
// theta_w), in FP32 from the FP32 shadows (cos and sin of the angles from the
// half-angle table, rounded once): bit 3 = within the sound FP32 margin
// 8 u32 (A + S) of cosh R (A, S the two products: such a pair would need an
// FP64 recheck), bit 4 = its plain FP32 decision differs from the FP64 one.
template <int FP32, bool ABL = false>
__device__ __forceinline__ uint32_t edge_test(const Geo &g, const Qv &q, const Cand &c, uint32_t p, int exhaustive) {
    const double d = q.hs * c.hw.y - q.hc * c.hw.x;
    if (!FP32) {
        const double a = q.hep * c.ew.y + q.hem * c.ew.x;
        const double b = (q.sh * (c.ew.x - c.ew.y)) * (d * d);
        return (a + b) < g.K ? 1u : 0u;
    } else {
        const float d32 = (float)d;
        const float a32 = q.hep32 * c.f.y + q.hem32 * c.f.x;
        const float t32 = c.f.x - c.f.y;
        const float b32 = (q.sh32 * d32) * (t32 * d32);
        const float v32 = a32 + b32;
        const bool sure_in = v32 <= g.klo32, sure_out = v32 >= g.khi32;
        if (sure_in || sure_out) {
            if (!exhaustive && !ABL) return sure_in ? 1u : 0u;
        }
        const double2 e = g.epm[p];
        const double a = q.hep * e.y + q.hem * e.x;
        const double b = (q.sh * (e.x - e.y)) * (d * d);
        const uint32_t e64 = (a + b) < g.K ? 1u : 0u;
        uint32_t abl = 0u;
        if (ABL) {
            const float chu = q.hep32 + q.hem32, shu = q.sh32;
            const float chw = 0.5f * (c.f.x + c.f.y), shw = (float)(0.5 * (e.x - e.y));
            const float cu = (float)(q.hc * q.hc - q.hs * q.hs), su = (float)(2.0 * (q.hs * q.hc));
            const float cw = (float)(c.hw.y * c.hw.y - c.hw.x * c.hw.x), sw = (float)(2.0 * (c.hw.x * c.hw.y));
            const float A = chu * chw, S = shu * shw;
            const float C = cu * cw + su * sw;
            const float V = A - S * C;
            const float K32 = (float)g.K;
            abl |= (fabsf(V - K32) <= 8.0f * 0x1p-24f * (A + S)) ? 8u : 0u;
            abl |= ((V < K32 ? 1u : 0u) != e64) ? 16u : 0u;
        }
        if (!(sure_in || sure_out)) return e64 | 2u | abl;
        const uint32_t f32dec = sure_in ? 1u : 0u;
        return f32dec | (f32dec != e64 ? 4u : 0u) | abl;
    }
}

// General model at temperature T > 0 (Sec. II, Eq. 2): the pair is an edge
// iff its uniform U = k 2^-53 is below f = 1 / (1 + exp((x - R) / (2T))),
// x = acosh(V) (0 for V <= 1, where rounding can put coincident points),
// with V the canonical FP64 cosh distance above, in this order of FP64
// operations.  The windows and the first test belong to the enlarged radius
// Rc (K = cosh Rc): at or beyond it f < 2^-53 <= U.  Before any
// transcendental, U in [2^-(j+1), 2^-j) (j from the leading zeros of k)
// needs f > 2^-(j+1), which needs V < lev[j+1] (with a margin far above the
// rounding of f); most candidates stop there, so exp and acosh run for few.
// For j < SOFT_FINE_J the part of [2^-(j+1), 2^-j) that U falls in (the
// three bits after its leading one) is looked up next: below its acceptance
// threshold the pair is an edge whatever U is in that part, at or above its
// rejection threshold it is not; only the pairs in between, about a tenth
// of those past the level test, take the exact test.
// soft_pre is that first part: 0 = no edge, 1 = edge, 2 = the exact test
// must decide (with U).
__device__ __forceinline__ uint32_t soft_pre(const Geo &g, double V, uint32_t qi, uint32_t wi, double &U) {
    if (!(V < g.K)) return 0u;
    const uint32_t lo = qi < wi ? qi : wi, hi = qi < wi ? wi : qi;
    const uint64_t k = pair_k(g.pseed, lo, hi);
    const int j = __clzll((long long)k) - 11;  // U in [2^-(j+1), 2^-j); j = -1 for U = 1
    if (j < 0 || !(V < g.lev[j + 1])) return 0u;
    U = (double)k * 0x1p-53;
    if (j < SOFT_FINE_J) {
        const int m = (int)((k >> (52 - 3 - j)) & (uint64_t)(SOFT_SUB - 1));
        const int t = SOFT_SUB * j + (SOFT_SUB - 1 - m);
        if (!(V < g.stab[t])) return 0u;
        if (V < g.stab[SOFT_TICKS + t]) return 1u;
    }
    return 2u;
}
__device__ __forceinline__ uint32_t soft_exact(const Geo &g, double V, double U) {
    const double x = V > 1.0 ? acosh(V) : 0.0;
    const double y = (x - g.R) / g.t2;
    const double f = 1.0 / (1.0 + exp(y));
    return U < f ? 1u : 0u;
}

// Per-unit setup shared by the count and emit passes: the unit's batch and
// flattened range [r0, r1), the lane's query, the first slab whose segment
// reaches past r0, and the slab segments the unit meets: bit k of segmask is
// slab jmin + k, whose segment of the batch's flattened candidate list is
// [rlo, rhi) of lane k (the batch's per-slab offsets).
struct UnitSetup {
    uint32_t b;
    uint64_t r0, r1;
    uint32_t v;
    bool valid;
    int iv, jstart;
    uint64_t pos;  // flattened offset of slab jstart's segment
    int jmin;
    uint32_t segmask;
    uint64_t rlo, rhi;
};

// FULL: update mode; a moved query's windows start in slab 0, an unmoved one has none.
template <bool FULL = false>
__device__ __forceinline__ UnitSetup unit_setup_chain(const QueryArgs &A, uint64_t unit, int lane) {
    const Geo &g = A.geo;
    UnitSetup u;
    // unit, batch and range are wave-uniform: scalar registers, so the walk
    // over slabs indexes the geometry with scalar loads
    unit = uniform_u64(unit);
    u.b = uniform_u32(A.unit_batch[unit]);
    const uint64_t chunk = unit - uniform_u64(A.unit_off[u.b]);
    u.r0 = chunk * UNIT;
    const uint64_t bc = uniform_u64(A.batch_cand[u.b]);
    u.r1 = (u.r0 + UNIT < bc) ? u.r0 + UNIT : bc;
    u.v = u.b * BATCH + lane;
    u.valid = u.v < g.n;
    // first slab with windows: the query's own (update mode: slab 0 if it moved)
    if (FULL) u.iv = (u.valid && bit_of(g.moved, u.v)) ? 0 : g.B;
    else u.iv = u.valid ? (int)(g.keys[u.v] >> QBITS) : g.B;
    const int jmin = FULL ? 0 : (int)uniform_u32(g.keys[u.b * BATCH] >> QBITS);
    // segments of slabs jmin..B-1 end at row[j+1] (row[jmin] = 0)
    const uint64_t *row = A.batch_slab_off + (uint64_t)u.b * (g.B + 1);
    const int k = jmin + lane;
    u.rhi = (k < g.B) ? row[k + 1] : bc;
    u.rlo = __shfl_up(u.rhi, 1, 64);
    if (lane == 0) u.rlo = 0;
    const bool done = k < g.B && u.rhi <= u.r0;
    u.jstart = jmin + __popcll(__ballot(done));
    u.pos = (u.jstart < g.B) ? row[u.jstart] : bc;
    u.jmin = jmin;
    u.segmask = (uint32_t)__ballot(k < g.B && u.rhi > u.rlo && u.rhi > u.r0 && u.rlo < u.r1);
    return u;
}

// The same from the unit's descriptor: one scalar load, after which the
// lane's loads (its query's key, the batch's segment offsets, the windows)
// are all independent of each other, instead of a chain of dependent loads.
template <bool FULL = false>
__device__ __forceinline__ UnitSetup unit_setup(const QueryArgs &A, uint64_t unit, int lane) {
    if (!A.udesc) return unit_setup_chain<FULL>(A, unit, lane);
    const Geo &g = A.geo;
    UnitSetup u;
    unit = uniform_u64(unit);
    const UnitDesc d = A.udesc[unit - A.unit_base];
    u.b = d.b;
    u.jmin = (int)d.jmin;
    u.segmask = d.segmask;
    u.r0 = d.r0;
    u.r1 = d.r1;
    u.v = u.b * BATCH + lane;
    u.valid = u.v < g.n;
    if (FULL) u.iv = (u.valid && bit_of(g.moved, u.v)) ? 0 : g.B;
    else u.iv = u.valid ? (int)(g.keys[u.v] >> QBITS) : g.B;
    // segment starts: rlo of lane k = row[jmin + k] (row[jmin] = 0)
    const uint64_t *row = A.batch_slab_off + (uint64_t)u.b * (g.B + 1);
    const int k = u.jmin + lane;
    u.rlo = (k <= g.B) ? row[k] : 0ull;
    u.rhi = 0;
    u.jstart = u.jmin;
    u.pos = 0;
    return u;
}

// Exclusive wavefront scan of the 64 window counts of a slab segment, and
// their total.  A window holds at most n points: while 64 n < 2^32 one 32-bit
// scan is exact; beyond, the 16-bit halves are scanned apart (each sum < 2^22).
__device__ __forceinline__ void window_scan(uint32_t cnt, uint32_t n, uint64_t &excl, uint64_t &tot) {
    if (64ull * n < (1ull << 32)) {
        const uint32_t incl = wave_incl_scan_u32(cnt);
        tot = wave_bcast_u32(incl, 63);
        excl = incl - cnt;
    } else {
        const uint32_t il = wave_incl_scan_u32(cnt & 0xffffu), ih = wave_incl_scan_u32(cnt >> 16);
        tot = (uint64_t)wave_bcast_u32(il, 63) + ((uint64_t)wave_bcast_u32(ih, 63) << 16);
        excl = (uint64_t)il + ((uint64_t)ih << 16) - cnt;
    }
}

// Lane's window in slab j (0 count if none), scanned over the wavefront.
__device__ __forceinline__ void slab_windows(const Geo &g, const QueryArgs &A, const UnitSetup &u, int j,
                                             uint32_t &st, uint32_t &cnt, uint64_t &excl, uint64_t &tot) {
    st = 0;
    cnt = 0;
    if (u.valid && j >= u.iv) {
        const uint2 x = A.win[g.winbase[j] + u.v];
        st = x.x;
        cnt = x.y;
    }
    window_scan(cnt, g.n, excl, tot);
}

// Windows of the first SEG_PRE segments of a unit, loaded together at the
// unit's start (one memory round trip, before the pass issues any store) and
// kept in LDS; later segments load their windows when reached.
constexpr int SEG_PRE = 2;

__device__ __forceinline__ void prefetch_windows(const QueryArgs &A, const UnitSetup &u, int lane,
                                                 uint2 (*wpre)[64]) {
    const Geo &g = A.geo;
    uint32_t mk = u.segmask;
    uint2 x[SEG_PRE];
#pragma unroll
    for (int s = 0; s < SEG_PRE; ++s) {
        const bool any = mk != 0u;
        const int j = u.jmin + (any ? __builtin_ctz(mk) : 0);
        mk &= mk - 1u;
        // the address does not wait for the lane's slab: winbase[j] + v stays
        // below winbase[B] (slab j's block plus the later ones hold >= n
        // entries), and a window of a slab below the lane's is masked after
        const uint64_t at = (any && u.valid) ? g.winbase[j] + u.v : 0ull;
        const uint2 y = A.win[at];
        x[s] = (any && u.valid && j >= u.iv) ? y : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int s = 0; s < SEG_PRE; ++s) wpre[s][lane] = x[s];
}

// Lane's window in the seg-th segment of the unit (slab j, flattened start
// pos within the batch), scanned and rebased to the unit: offsets below count
// from the unit's first candidate in the segment, which keeps them in 32 bits
// for any n (the unit spans at most UNIT candidates).  Returns the window's
// count, pb with position = pb + offset (mod 2^32), its start relu (all ones:
// before the unit; clamped to 2^30 far after it), and the segment's end e.
constexpr uint32_t BEFORE_UNIT = 0xffffffffu;

__device__ __forceinline__ void segment_windows(const QueryArgs &A, const UnitSetup &u, int seg, int j, int lane,
                                                uint2 (*wpre)[64], uint64_t pos, uint32_t &cnt, uint32_t &pb,
                                                uint32_t &relu, uint32_t &e) {
    const Geo &g = A.geo;
    uint2 x;
    if (seg < SEG_PRE) {
        x = wpre[seg][lane];
    } else {
        x = make_uint2(0u, 0u);
        if (u.valid && j >= u.iv) x = A.win[g.winbase[j] + u.v];
    }
    cnt = x.y;
    uint64_t excl, tot;
    window_scan(cnt, g.n, excl, tot);
    const uint64_t a = (u.r0 > pos) ? u.r0 - pos : 0ull;
    const uint64_t e64 = (u.r1 - pos < tot) ? u.r1 - pos : tot;
    e = (uint32_t)(e64 > a ? e64 - a : 0ull);
    const int64_t rel = (int64_t)(excl - a);
    relu = rel < 0 ? BEFORE_UNIT : (rel > (1 << 30) ? (1u << 30) : (uint32_t)rel);
    pb = x.x - (uint32_t)rel;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Window lookup for one step of VT x 64 candidates of a slab segment.  The
// non-empty windows of the slab are numbered in lane order (their rank);
// window r covers flattened candidates [excl_r, excl_r + cnt_r).  Each window
// that starts inside [t0, t0 + VT*64) flags its start slot; the ballot M_i of
// the flags of sub-round i gives, for candidate t0 + 64 i + k,
// rank = (windows starting before t0 + 64 i) - 1 + popcount(M_i & bits 0..k).
// No per-candidate search.  Count and emit use different VT (register
// pressure vs. loads in flight); the flattened order is the same.
#ifndef RHG_VT_COUNT
#define RHG_VT_COUNT 2
#endif
#ifndef RHG_VT_EMIT
#define RHG_VT_EMIT 4
#endif
constexpr int VT_COUNT = RHG_VT_COUNT;
constexpr int VT_EMIT = RHG_VT_EMIT;

// Also returns, per sub-round, the number of windows starting at or before
// the lane's slot: the set bits of M below the lane (mbcnt) plus the lane's
// own flag, i.e. popcount(M & bits 0..lane) in two instructions fewer.
template <int VT>
__device__ __forceinline__ void step_starts(uint8_t *flags, int lane, bool nonempty, uint32_t excl, uint32_t t0,
                                            uint64_t (&M)[VT], uint32_t (&upto)[VT]) {
    if (nonempty && excl >= t0 && excl - t0 < 64u * VT) flags[excl - t0] = 1u;
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        const uint32_t f = flags[i * 64 + lane];
        flags[i * 64 + lane] = 0u;
        M[i] = __ballot(f != 0u);
        upto[i] = __builtin_amdgcn_mbcnt_hi((uint32_t)(M[i] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)M[i], 0u)) +
                  (f != 0u ? 1u : 0u);
    }
    wave_lds_sync();
}

// Decision bitmap of a unit: each slab segment the unit covers starts on a
// fresh 64-bit word, so the decisions of one 64-candidate round are exactly
// one word (its ballot).  A unit of <= UNIT candidates over <= 32 segments
// needs at most UNIT/64 + 31 words.
constexpr int BITW = (int)(UNIT / 64) + 32;

__device__ __forceinline__ uint32_t position_of(uint2 we, uint32_t t, uint32_t be, uint32_t nj) {
    uint32_t p = we.x + (t - we.y);
    if (p >= be) p -= nj;
    if (p >= be) p = be - 1;  // unreachable for consistent windows; keeps reads in bounds
    return p;
}

// Same with the window's (start - offset) precomputed: p = pb + t, wrapped once
// at the slab end, clamped into the slab (unreachable for consistent windows).
__device__ __forceinline__ uint32_t position_pb(uint32_t pb, uint32_t t, uint32_t be, uint32_t nj) {
    uint32_t p = pb + t;
    p = (p >= be) ? p - nj : p;
    return min(p, be - 1u);
}

// Count pass: decide every candidate of the unit, record the decisions as
// one bitmap word per 64-candidate round, count edges.
// Per-wavefront LDS of the count pass.
// (FP32 operands only in the filter form, to keep the FP64 form's LDS, and
// with it the workgroups per CU, down.)
constexpr uint32_t SOFT_Q = 128;
template <int FP32, bool FULL = false, bool SOFT = false>
struct CountSmem {
    uint32_t pb[64];    // per rank: start position - flattened offset
    uint8_t flag[64 * VT_COUNT];
    double qd[5][64];   // per rank: query operands
    float qf[FP32 ? 3 : 1][64];
    unsigned long long bits[BITW];
    uint2 wpre[SEG_PRE][64];
    uint32_t qpos[FULL ? 64 : 1];  // per rank: the query's sorted position (update mode)
    uint32_t qi[SOFT ? 64 : 1];    // per rank: the query's original index (general model)
    // general model: candidates waiting for the exact test (a ring of
    // SOFT_Q): V, U and the candidate's bit in the unit's bitmap
    double sv[SOFT ? SOFT_Q : 1], su[SOFT ? SOFT_Q : 1];
    uint32_t sp[SOFT ? SOFT_Q : 1];
};

// General model: the exact test of the first n (<= 64) queued candidates,
// lane l taking entry head + l; an edge sets its bit in the unit's bitmap
// (after that round's word was written).  Returns the edges found.
template <int FP32, bool FULL>
__device__ __forceinline__ uint32_t soft_drain(const Geo &g, CountSmem<FP32, FULL, true> &S, uint32_t head,
                                               uint32_t n, int lane) {
    wave_lds_sync();
    const uint32_t k = (head + (uint32_t)lane) & (SOFT_Q - 1);
    const bool mine = (uint32_t)lane < n;
    const uint32_t e = mine ? soft_exact(g, S.sv[k], S.su[k]) : 0u;
    const uint32_t pos = S.sp[k];
    if (e) atomicOr(&S.bits[pos >> 6], 1ull << (pos & 63u));
    const uint32_t got = (uint32_t)__popcll(__ballot(e != 0u));
    wave_lds_sync();
    return got;
}

// Ranks and positions of one count step (VT x 64 candidates from t0): the
// rank of each candidate's window and its position in the slab; lanes at or
// past the segment end e take the dummy position bs.  Advances base.
template <int VT>
__device__ __forceinline__ void count_positions(uint8_t *flags, const uint32_t *pbs, int lane, bool ne, uint32_t relu,
                                                uint32_t t0, uint32_t e, uint32_t bs, uint32_t be, uint32_t nj,
                                                uint32_t &base, uint32_t (&p)[VT], uint32_t (&rk)[VT]) {
    uint64_t M[VT];
    uint32_t upto[VT];
    step_starts<VT>(flags, lane, ne, relu, t0, M, upto);
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        const uint32_t t = t0 + 64u * i + lane;
        rk[i] = (base - 1u + upto[i]) & 63u;
        base += (uint32_t)__popcll(M[i]);
        const uint32_t pp = position_pb(pbs[rk[i]], t, be, nj);
        p[i] = t < e ? pp : bs;
    }
}

// FULL: update mode (Geo::moved): a candidate that passes the distance test
// is an edge unless it is the query itself, or a moved point that comes
// before the query in sorted order (that pair is the other query's).
// SOFT: the general model (FP64 only), each candidate decided by soft_pre and,
// queued, soft_exact.
// ABL: the FP32 form with the literal-Eq. 3 ablation counters (edge_test).
template <int FP32, bool WIDE, bool FULL = false, bool SOFT = false, bool ABL = false>
__device__ __forceinline__ void count_unit(const QueryArgs &A, uint64_t unit, uint64_t slot, int lane,
                                           CountSmem<FP32, FULL, SOFT> &S) {
    constexpr int VT = VT_COUNT;
    const Geo &g = A.geo;
    const UnitSetup u = unit_setup<FULL>(A, unit, lane);
    Qv mine{};
    uint32_t myqi = 0;
    if (u.valid) {
        const double2 e = g.epm[u.v];
        const double2 h = g.hsc[u.v];
        mine.hep = 0.5 * e.x;
        mine.hem = 0.5 * e.y;
        mine.sh = 0.5 * (e.x - e.y);
        mine.hs = h.x;
        mine.hc = h.y;
        if (SOFT) myqi = g.idx[u.v];
        if (FP32) {
            const float2 f = g.f32[u.v];
            mine.hep32 = 0.5f * f.x;
            mine.hem32 = 0.5f * f.y;
            mine.sh32 = (float)mine.sh;
        }
    }
#pragma unroll
    for (int i = 0; i < VT; ++i) S.flag[i * 64 + lane] = 0u;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    prefetch_windows(A, u, lane, S.wpre);
    uint32_t word = 0;     // next free bitmap word
    uint32_t found = 0, rechecks = 0, disagree = 0, lit_und = 0, lit_wrong = 0;
    uint32_t sq_head = 0, sq_n = 0;  // general model: the queue of exact tests (uniform)
    uint32_t segs = u.segmask;
    for (int seg = 0; segs != 0u; ++seg) {
        const int bit = __builtin_ctz(segs);
        segs &= segs - 1u;
        const int j = u.jmin + bit;
        const uint64_t pos = lane_u64(u.rlo, bit);  // flattened offset of slab j's segment within the batch
        uint32_t cnt, pb, relu, e;
        wave_lds_sync();
        segment_windows(A, u, seg, j, lane, S.wpre, pos, cnt, pb, relu, e);
        const bool ne = cnt != 0u;
        const uint64_t nem = __ballot(ne);
        wave_lds_sync();
        if (ne) {
            const uint32_t rk = (uint32_t)__popcll(nem & lt);
            S.pb[rk] = pb;
            S.qd[0][rk] = mine.hep;
            S.qd[1][rk] = mine.hem;
            S.qd[2][rk] = mine.sh;
            S.qd[3][rk] = mine.hs;
            S.qd[4][rk] = mine.hc;
            if (FULL) S.qpos[rk] = u.v;
            if (SOFT) S.qi[rk] = myqi;
            if (FP32) {
                S.qf[0][rk] = mine.hep32;
                S.qf[1][rk] = mine.hem32;
                S.qf[2][rk] = mine.sh32;
            }
        }
        uint32_t base = (uint32_t)__popcll(__ballot(ne && relu == BEFORE_UNIT));
        const uint32_t bs = g.bs[j], be = g.bs[j + 1], nj = be - bs;
        // The ranks and positions of step k+1 (LDS only) are worked out while
        // the gathers of step k are in flight, off the step's chain of waits.
        uint32_t p[VT], rk[VT];
        count_positions<VT>(S.flag, S.pb, lane, ne, relu, 0u, e, bs, be, nj, base, p, rk);
        for (uint32_t t0 = 0; t0 < e; t0 += 64u * VT) {
            Cand c[VT];
#pragma unroll
            for (int i = 0; i < VT; ++i) load_cand<FP32, WIDE, SOFT>(g, p[i], c[i]);
            uint32_t pn[VT] = {}, rkn[VT] = {};
            if (t0 + 64u * VT < e) count_positions<VT>(S.flag, S.pb, lane, ne, relu, t0 + 64u * VT, e, bs, be, nj, base, pn, rkn);
#pragma unroll
            for (int i = 0; i < VT; ++i) {
                const bool act = t0 + 64u * i + lane < e;
                Qv q;
                q.hep = S.qd[0][rk[i]];
                q.hem = S.qd[1][rk[i]];
                q.sh = S.qd[2][rk[i]];
                q.hs = S.qd[3][rk[i]];
                q.hc = S.qd[4][rk[i]];
                if (FP32) {
                    q.hep32 = S.qf[0][rk[i]];
                    q.hem32 = S.qf[1][rk[i]];
                    q.sh32 = S.qf[2][rk[i]];
                }
                // FP32 filter: test every lane and mask (the loads issue together);
                // FP64: lanes past the end skip the test (measured faster there)
                uint32_t r;
                if (SOFT) {
                    // the candidates the level and table tests leave open queue
                    // for the exact test, which sets their bits later
                    r = 0u;
                    double V = 0.0, U = 0.0;
                    bool need = false;
                    if (act) {
                        const double d = q.hs * c[i].hw.y - q.hc * c[i].hw.x;
                        const double a = q.hep * c[i].ew.y + q.hem * c[i].ew.x;
                        const double b = (q.sh * (c[i].ew.x - c[i].ew.y)) * (d * d);
                        V = a + b;
                        const uint32_t pre = soft_pre(g, V, S.qi[rk[i]], c[i].wi, U);
                        r = pre & 1u;
                        need = pre == 2u;
                    }
                    const uint64_t nm = __ballot(need);
                    if (need) {
                        const uint32_t k = (sq_head + sq_n + (uint32_t)__popcll(nm & lt)) & (SOFT_Q - 1);
                        S.sv[k] = V;
                        S.su[k] = U;
                        S.sp[k] = (word + i) * 64u + (uint32_t)lane;
                    }
                    sq_n += (uint32_t)__popcll(nm);
                } else {
                    r = FP32 ? (edge_test<FP32, ABL>(g, q, c[i], p[i], A.exhaustive) & (act ? 31u : 0u))
                             : (act ? edge_test<FP32>(g, q, c[i], p[i], A.exhaustive) : 0u);
                }
                int flag = (int)(r & 1u);
                if (FULL) {
                    const uint32_t qp = S.qpos[rk[i]];
                    flag &= (p[i] != qp && (!bit_of(g.moved, p[i]) || p[i] > qp)) ? 1 : 0;
                }
                if (FP32) {
                    rechecks += (r >> 1) & 1u;
                    disagree += (r >> 2) & 1u;
                    if (ABL) {
                        lit_und += (r >> 3) & 1u;
                        lit_wrong += (r >> 4) & 1u;
                    }
                }
                const uint64_t m = __ballot(flag);
                found += (uint32_t)__popcll(m);
                if (t0 + 64u * i < e && lane == 0) S.bits[word + i] = m;
                if constexpr (SOFT) {
                    if (sq_n >= 64u) {  // a whole wavefront of exact tests
                        found += soft_drain(g, S, sq_head, 64u, lane);
                        sq_head = (sq_head + 64u) & (SOFT_Q - 1);
                        sq_n -= 64u;
                    }
                }
            }
            word += (e - t0 < 64u * VT) ? (e - t0 + 63u) / 64u : (uint32_t)VT;
#pragma unroll
            for (int i = 0; i < VT; ++i) {
                p[i] = pn[i];
                rk[i] = rkn[i];
            }
        }
    }
    if constexpr (SOFT) {
        if (sq_n) found += soft_drain(g, S, sq_head, sq_n, lane);
    }
    wave_lds_sync();
    for (uint32_t k = lane; k < word; k += 64) A.bits[unit * BITW + k] = S.bits[k];
    if (lane == 0) A.unit_edges[slot] = found;
    if (FP32) {
        const uint64_t rc = wave_sum_u64(rechecks), dg = wave_sum_u64(disagree);
        if (lane == 0 && rc) atomicAdd(&A.stats[0], (unsigned long long)rc);
        if (lane == 0 && dg) atomicAdd(&A.stats[1], (unsigned long long)dg);
        if (ABL) {
            const uint64_t lu = wave_sum_u64(lit_und), lw = wave_sum_u64(lit_wrong);
            if (lane == 0 && lu) atomicAdd(&A.stats[2], (unsigned long long)lu);
            if (lane == 0 && lw) atomicAdd(&A.stats[3], (unsigned long long)lw);
        }
    }
}

// Emit pass: walk the unit exactly as the count pass did, take the decisions
// from its bitmap, and write (min, max) original-index pairs, compacted per
// 64-candidate round, at the unit's offset in the edge list.
//
// The walk is software-pipelined by one step: the index gathers of step k+1
// are issued before the stores of step k.  Loads and stores share one
// completion counter on this architecture and complete in order, so waiting
// for a step's gathers never waits for the previous step's write acks.  For
// the compiler to count the stores statically they must not sit behind
// exec-skipping branches: every lane stores, through a buffer resource that
// spans exactly this unit's output slice, and lanes without an edge give an
// offset outside it, which the hardware range check drops.  The same check
// keeps every store inside the unit's slice and the caller's capacity.
// Per-wavefront LDS of the emit pass.
struct EmitSmem {
    uint32_t pb[64];
    uint8_t flag[64 * VT_EMIT];
    uint32_t qi[64];
    unsigned long long bits[BITW + VT_EMIT];
    uint2 wpre[SEG_PRE][64];
};

typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int BUFFER_WORD3 = 0x00020000;   // raw buffer, 32-bit data format (gfx9 family)
constexpr uint32_t NO_STORE = 0x80000000u; // offset outside every unit's slice
constexpr int STORE_NT = 2;                 // non-temporal: edges are not read again by this pass

struct EmitStep {
    uint32_t wi[VT_EMIT];   // gathered original index of the candidate (in flight until stored)
    uint32_t qi[VT_EMIT];   // original index of the query
    uint32_t off[VT_EMIT];  // byte offset in the unit's slice, or NO_STORE
    bool valid;
};

// Walk state of one unit: the segments left, the current one and the position in it.
struct EmitWalk {
    uint32_t segs;
    int seg;
    uint32_t t0, e, base, word, be, nj, relu, out_rel;
    bool ne, in_seg;
};

// Decision words of a unit read with scalar loads through the constant
// address space: only where the bitmap was written by an earlier kernel (the
// scalar cache is invalidated at each dispatch); within one kernel the words
// go through LDS instead.
typedef const __attribute__((address_space(4))) unsigned long long *const_words_t;

template <bool WIDE, bool SBITS>
__device__ __forceinline__ void emit_prepare(const QueryArgs &A, const UnitSetup &u, uint32_t myqi, uint32_t todo,
                                             int lane, uint64_t lt, EmitSmem &S, const_words_t cw,
                                             EmitWalk &w, EmitStep &s) {
    constexpr int VT = VT_EMIT;
    const Geo &g = A.geo;
    s.valid = false;
    while (!w.in_seg) {
        if (w.segs == 0u || w.out_rel >= todo) return;
        const int bit = __builtin_ctz(w.segs);
        w.segs &= w.segs - 1u;
        const int j = u.jmin + bit;
        const uint64_t pos = lane_u64(u.rlo, bit);
        uint32_t cnt, pb;
        wave_lds_sync();
        segment_windows(A, u, w.seg, j, lane, S.wpre, pos, cnt, pb, w.relu, w.e);
        ++w.seg;
        w.ne = cnt != 0u;
        const uint64_t nem = __ballot(w.ne);
        wave_lds_sync();
        if (w.ne) {
            const uint32_t rk = (uint32_t)__popcll(nem & lt);
            S.pb[rk] = pb;
            S.qi[rk] = myqi;
        }
        w.base = (uint32_t)__popcll(__ballot(w.ne && w.relu == BEFORE_UNIT));
        w.be = g.bs[j + 1];
        w.nj = w.be - g.bs[j];
        w.t0 = 0;
        w.in_seg = 0u < w.e;
    }
    // The step's VT decision words (uniform: scalar registers), read
    // unconditionally as one run (the bitmap carries VT words of padding past
    // its last unit; words past the segment end are masked), so that one wait
    // covers them all instead of one per sub-round.
    uint64_t mw[VT];
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        if (SBITS) {
            mw[i] = cw[w.word + i];
        } else {
            const uint64_t x = S.bits[w.word + i];
            mw[i] = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
        }
    }
    uint64_t M[VT];
    uint32_t upto[VT];
    step_starts<VT>(S.flag, lane, w.ne, w.relu, w.t0, M, upto);
    // ranks first, then every LDS read of the step, then positions and gathers:
    // no read sits behind a branch, so the reads of all sub-rounds share one wait
    uint32_t rk[VT], pb[VT];
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        rk[i] = (w.base - 1u + upto[i]) & 63u;
        w.base += (uint32_t)__popcll(M[i]);
    }
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        pb[i] = S.pb[rk[i]];
        s.qi[i] = S.qi[rk[i]];
    }
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        const uint64_t m = (w.t0 + 64u * i < w.e) ? mw[i] : 0ull;
        const bool mine = (m >> lane) & 1ull;
        const uint32_t pp = position_pb(pb[i], w.t0 + 64u * i + lane, w.be, w.nj);
        const uint32_t p = mine ? pp : w.be - 1u;
        s.wi[i] = ld<WIDE>(g.idx, p);
        s.off[i] = mine ? (w.out_rel + (uint32_t)__popcll(m & lt)) * 8u : NO_STORE;
        w.out_rel += (uint32_t)__popcll(m);
    }
    w.word += (w.e - w.t0 < 64u * VT) ? (w.e - w.t0 + 63u) / 64u : (uint32_t)VT;
    w.t0 += 64u * VT;
    w.in_seg = w.t0 < w.e;
    s.valid = true;
}

__device__ __forceinline__ void emit_store(const EmitStep &s, __amdgpu_buffer_rsrc_t out) {
#pragma unroll
    for (int i = 0; i < VT_EMIT; ++i) {
        const uint32_t lo = s.qi[i] < s.wi[i] ? s.qi[i] : s.wi[i];
        const uint32_t hi = s.qi[i] < s.wi[i] ? s.wi[i] : s.qi[i];
        const u32x2_t v = {lo, hi};
        __builtin_amdgcn_raw_buffer_store_b64(v, out, (int)s.off[i], 0, STORE_NT);
    }
}

template <bool WIDE, bool SBITS = false, bool FULL = false>
__device__ __forceinline__ void emit_unit(const QueryArgs &A, uint64_t unit, uint64_t slot, int lane, EmitSmem &S) {
    const Geo &g = A.geo;
    const uint32_t todo = uniform_u32(A.unit_edges[slot]);
    if (todo == 0) return;
    const UnitSetup u = unit_setup<FULL>(A, unit, lane);
    const uint32_t myqi = u.valid ? g.idx[u.v] : 0u;
    const_words_t cw = (const_words_t)(A.bits + uniform_u64(unit) * BITW);
    if (!SBITS)
        for (int k = lane; k < BITW + VT_EMIT; k += 64) S.bits[k] = k < BITW ? A.bits[unit * BITW + k] : 0ull;
#pragma unroll
    for (int i = 0; i < VT_EMIT; ++i) S.flag[i * 64 + lane] = 0u;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t at = uniform_u64(A.unit_edge_off[slot]);  // the resource must sit in scalar registers
    uint64_t cap = A.out_capacity > at ? A.out_capacity - at : 0ull;
    cap = cap < todo ? cap : todo;
    const __amdgpu_buffer_rsrc_t out =
        __builtin_amdgcn_make_buffer_rsrc((void *)(A.out + at), 0, (int)(cap * 8u), BUFFER_WORD3);

    prefetch_windows(A, u, lane, S.wpre);
    EmitWalk w;
    w.segs = u.segmask;
    w.seg = 0;
    w.t0 = w.e = w.base = w.word = w.be = w.nj = w.relu = w.out_rel = 0u;
    w.ne = w.in_seg = false;
    EmitStep s0, s1;
    emit_prepare<WIDE, SBITS>(A, u, myqi, todo, lane, lt, S, cw, w, s0);
    while (s0.valid) {
        emit_prepare<WIDE, SBITS>(A, u, myqi, todo, lane, lt, S, cw, w, s1);  // gathers of the next step ...
        emit_store(s0, out);                                            // ... in flight over these stores
        if (!s1.valid) break;
        emit_prepare<WIDE, SBITS>(A, u, myqi, todo, lane, lt, S, cw, w, s0);
        emit_store(s1, out);
    }
}

}  // namespace rhgk
