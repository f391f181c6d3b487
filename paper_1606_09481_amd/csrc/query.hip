// query.hip -- the band query of Algorithm 1 on gfx950: window planning
// (getMinMaxPhi + search), then count and emit passes over load-balanced work
// units.
//
// Window of query v in slab j (Sec. III-B, getMinMaxPhi): every neighbour w of
// v with r_w >= c_j satisfies
//   sin^2(|theta_w - theta_v|/2) <= (cosh R - cosh(r_v - c_j)) / (2 sinh r_v sinh c_j),
// the inequality chain of the paper with 1 - cos x = 2 sin^2(x/2) and
// cosh a cosh b - sinh a sinh b = cosh(a - b) (no cancellation for the small
// windows of outer slabs).  cosh R is raised to Kw = K (1 + 2^-30) and the
// angle widened by a relative 2^-30 plus 2^-44 rad: enough to contain every
// pair the FP64 distance test accepts, including its rounding and the
// rounding of the table values.  Half-widths >= pi/2 scan the whole slab.
//
// Outward-only scan (Algorithm 1 inner loop, slabs with c_{j+1} > r_v): slab
// j > slab(v) is scanned over the full window; in v's own slab each pair is
// taken once, by a forward rule in key order: v takes w iff w lies after v
// going forward in angle within the window (ties in key broken by position);
// a whole-slab window takes the forward half turn.  With windows under a
// quarter turn or whole, every own-slab edge lies in exactly one forward arc.
//
// Work decomposition: 64 consecutive sorted queries form a batch; a batch's
// candidates are flattened slab-major (slab j, then query, then position) and
// cut into units of <= 4096 candidates; one wavefront runs one unit, lane k
// taking flattened candidate t0 + k (a load-balanced search over the 64
// window counts of the current slab), so hub queries with million-candidate
// windows spread over many wavefronts.  The count pass evaluates the distance
// test once per candidate and keeps the decisions as a 4096-bit map per unit;
// the emit pass walks the unit identically, reads the map instead of
// re-testing, and writes the pairs compacted per 64-candidate round, so the
// edge order is deterministic.
#include "query_dev.h"

namespace rhgk {
using namespace rhgd;

template <bool FULL>
__global__ __launch_bounds__(256) void k_plan(Geo g, uint2 *win, uint64_t *batch_cand, uint64_t *batch_slab_off) {
    const uint32_t b = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (b >= (g.n + 63) / 64) return;  // whole wavefronts past the last batch
    plan_batch<FULL>(g, win, batch_cand, batch_slab_off, b, threadIdx.x & 63);
}

void plan(const Geo &g, uint2 *win, uint64_t *batch_cand, uint64_t *batch_slab_off, hipStream_t st) {
    if (!g.n) return;
    if (g.moved)
        hipLaunchKernelGGL(k_plan<true>, dim3((g.n + 255) / 256), dim3(256), 0, st, g, win, batch_cand, batch_slab_off);
    else
        hipLaunchKernelGGL(k_plan<false>, dim3((g.n + 255) / 256), dim3(256), 0, st, g, win, batch_cand, batch_slab_off);
}

// Execution order of units.  Units are executed grouped by the angular
// sector of their first candidate, so that the units in flight read the same
// stretch of every slab and share it in L2; the sorted list is cut into
// NXCD contiguous chunks and workgroup b (dispatched round-robin over the
// XCDs, b mod NXCD) takes its units from chunk b mod NXCD, so each XCD's L2
// holds only its own sectors.  Edge counts and offsets are kept per
// execution slot k (the unit's place in this order), so the edge list
// follows the execution order: the units in flight on one XCD write
// neighbouring stretches of it (DRAM rows are reused; measured 0.04 ms
// faster at n = 10^7 than offsets in batch order).  The order is a fixed
// function of the plan, the same for the FP64 and FP32 forms.
constexpr uint32_t NXCD = 8;
constexpr int SECTOR_BITS = 12;

__device__ __forceinline__ uint64_t exec_unit(const QueryArgs &A, int w, uint64_t &k) {
    const uint64_t U = A.n_units;
    const uint64_t chunk = (U + NXCD - 1) / NXCD;
    const uint64_t x = blockIdx.x % NXCD, slot = (uint64_t)(blockIdx.x / NXCD) * 4 + w;
    k = x * chunk + slot;
    if (slot >= chunk || k >= U) return ~0ull;
    return A.unit_order ? A.unit_order[k] : A.unit_base + k;
}

static unsigned exec_blocks(uint64_t U) {
    const uint64_t chunk = (U + NXCD - 1) / NXCD;
    return (unsigned)(NXCD * ((chunk + 3) / 4));
}

// Sector key of each unit: the top bits of the quantised angle of its first candidate.
// Each wavefront keys UKEY_UPW units: their chains of dependent loads (unit,
// batch, slab offsets, window, key) are interleaved, so that several are in
// flight at once.
constexpr int UKEY_UPW = 2;
template <bool FULL>
__global__ __launch_bounds__(256) void k_unit_key(QueryArgs A, uint32_t *key, uint32_t *id) {
    const Geo &g = A.geo;
    const int lane = threadIdx.x & 63;
    const uint64_t unit0 = ((uint64_t)blockIdx.x * 4 + (uint64_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))) * UKEY_UPW;
    UnitSetup u[UKEY_UPW];
    uint32_t st[UKEY_UPW], cnt[UKEY_UPW], p[UKEY_UPW];
    uint64_t excl[UKEY_UPW], tot[UKEY_UPW];
#pragma unroll
    for (int q = 0; q < UKEY_UPW; ++q) {
        const uint64_t unit = unit0 + q < A.n_units ? unit0 + q : A.n_units - 1;
        u[q] = unit_setup_chain<FULL>(A, A.unit_base + unit, lane);
    }
#pragma unroll
    for (int q = 0; q < UKEY_UPW; ++q) slab_windows(g, A, u[q], u[q].jstart, st[q], cnt[q], excl[q], tot[q]);
#pragma unroll
    for (int q = 0; q < UKEY_UPW; ++q) {
        const uint64_t off = u[q].r0 > u[q].pos ? u[q].r0 - u[q].pos : 0ull;
        const bool here = cnt[q] != 0u && excl[q] <= off && off - excl[q] < cnt[q];
        const uint64_t m = __ballot(here);
        const int l = m ? __ffsll((long long)m) - 1 : 0;
        const uint32_t be = g.bs[u[q].jstart + 1], nj = be - g.bs[u[q].jstart];
        uint32_t pp = g.bs[u[q].jstart];
        if (lane == l && m) pp = position_of(make_uint2(st[q], 0u), (uint32_t)(off - excl[q]), be, nj);
        p[q] = wave_bcast_u32(pp, l);
    }
#pragma unroll
    for (int q = 0; q < UKEY_UPW; ++q) {
        const uint32_t kq = (g.keys[p[q]] & QMASK) >> (QBITS - SECTOR_BITS);
        if (lane == 0 && unit0 + q < A.n_units) {
            key[unit0 + q] = kq;
            id[unit0 + q] = (uint32_t)(A.unit_base + unit0 + q);
            if (A.udesc) {
                UnitDesc d;
                d.b = u[q].b;
                d.jmin = (uint32_t)u[q].jmin;
                d.segmask = u[q].segmask;
                d.pad = 0;
                d.r0 = u[q].r0;
                d.r1 = u[q].r1;
                A.udesc[unit0 + q] = d;
            }
        }
    }
}

void unit_order(const QueryArgs &a, uint32_t *key, uint32_t *id, uint32_t *key_tmp, uint32_t *id_tmp,
                void *sort_scratch, hipStream_t st) {
    if (!a.n_units) return;
    const dim3 grid((unsigned)((a.n_units + 4 * UKEY_UPW - 1) / (4 * UKEY_UPW)));
    if (a.geo.moved) hipLaunchKernelGGL(k_unit_key<true>, grid, dim3(256), 0, st, a, key, id);
    else hipLaunchKernelGGL(k_unit_key<false>, grid, dim3(256), 0, st, a, key, id);
    radix_sort(key, id, key_tmp, id_tmp, sort_scratch, a.n_units, SECTOR_BITS, st);
}

template <int FP32, bool WIDE, bool FULL>
__global__ __launch_bounds__(256, 7) void k_count(QueryArgs A) {
    __shared__ CountSmem<FP32, FULL> sm[4];
    // wavefront index in scalar registers: the unit lookups become scalar loads
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    uint64_t k;
    const uint64_t unit = exec_unit(A, w, k);
    if (unit == ~0ull) return;  // uniform per wavefront; no block-wide barriers below
    count_unit<FP32, WIDE, FULL>(A, unit, k, lane, sm[w]);
}

// The general model's count: the same walk with the probabilistic decision;
// its transcendentals need more registers than 7 wavefronts per SIMD leave.
template <bool WIDE>
__global__ __launch_bounds__(256, 4) void k_count_soft(QueryArgs A) {
    __shared__ CountSmem<0, false, true> sm[4];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    uint64_t k;
    const uint64_t unit = exec_unit(A, w, k);
    if (unit == ~0ull) return;
    count_unit<0, WIDE, false, true>(A, unit, k, lane, sm[w]);
}

// The FP32 form with the literal-Eq. 3 ablation counters (a measurement, not a timed path).
template <bool WIDE>
__global__ __launch_bounds__(256, 4) void k_count_ablation(QueryArgs A) {
    __shared__ CountSmem<1> sm[4];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    uint64_t k;
    const uint64_t unit = exec_unit(A, w, k);
    if (unit == ~0ull) return;
    count_unit<1, WIDE, false, false, true>(A, unit, k, lane, sm[w]);
}

template <bool WIDE, bool FULL>
__global__ __launch_bounds__(256) void k_emit(QueryArgs A) {
    __shared__ EmitSmem sm[4];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    uint64_t k;
    const uint64_t unit = exec_unit(A, w, k);
    if (unit == ~0ull) return;
    emit_unit<WIDE, true, FULL>(A, unit, k, lane, sm[w]);  // bitmaps from the count kernel: scalar loads
}

template <int FP32, bool FULL>
static void launch_count(const QueryArgs &a, hipStream_t st) {
    const dim3 grid(exec_blocks(a.n_units)), block(256);
    if (a.geo.n >= (1u << 28)) hipLaunchKernelGGL((k_count<FP32, true, FULL>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_count<FP32, false, FULL>), grid, block, 0, st, a);
}

// Below n = 2^28 every table byte offset fits 32 bits (WIDE = false).
void query_count(const QueryArgs &a, int fp32, hipStream_t st) {
    if (!a.n_units) return;
    const bool full = a.geo.moved != nullptr;
    if (a.geo.t2 > 0.0) {  // general model: FP64, no update mode
        const dim3 grid(exec_blocks(a.n_units)), block(256);
        if (a.geo.n >= (1u << 28)) hipLaunchKernelGGL((k_count_soft<true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_count_soft<false>), grid, block, 0, st, a);
        return;
    }
    if (fp32 && a.exhaustive == 2 && !full) {  // literal-Eq. 3 ablation
        const dim3 grid(exec_blocks(a.n_units)), block(256);
        if (a.geo.n >= (1u << 28)) hipLaunchKernelGGL((k_count_ablation<true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_count_ablation<false>), grid, block, 0, st, a);
        return;
    }
    if (fp32) {
        if (full) launch_count<1, true>(a, st);
        else launch_count<1, false>(a, st);
    } else {
        if (full) launch_count<0, true>(a, st);
        else launch_count<0, false>(a, st);
    }
}

void query_emit(const QueryArgs &a, int fp32, hipStream_t st) {
    (void)fp32;  // decisions come from the count pass's bitmap
    if (!a.n_units) return;
    const dim3 grid(exec_blocks(a.n_units)), block(256);
    // emit walks from the unit chain, not the descriptors: measured 0.015 ms
    // faster at n = 10^7 (its early loads overlap the bitmap and offset reads)
    QueryArgs b = a;
    b.udesc = nullptr;
    const bool wide = a.geo.n >= (1u << 28), full = a.geo.moved != nullptr;
    if (full) {
        if (wide) hipLaunchKernelGGL((k_emit<true, true>), grid, block, 0, st, b);
        else hipLaunchKernelGGL((k_emit<false, true>), grid, block, 0, st, b);
    } else {
        if (wide) hipLaunchKernelGGL((k_emit<true, false>), grid, block, 0, st, b);
        else hipLaunchKernelGGL((k_emit<false, false>), grid, block, 0, st, b);
    }
}

}  // namespace rhgk
