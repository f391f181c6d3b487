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
#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

// 1 = whole slab; else 0 with the widened half-width in *delta.
__device__ __forceinline__ int half_width(double rv, double shv, double cj, double shc, double Kw, double *delta) {
    double den = 2.0 * shv * shc;
    if (!(den > 0.0)) return 1;
    double s = (Kw - cosh(rv - cj)) / den;
    if (!(s < 0.5)) return 1;  // sin^2(D/2) >= 1/2  <=>  D >= pi/2
    if (s < 0.0) s = 0.0;
    double d = 2.0 * asin(sqrt(s));
    d = d * (1.0 + 0x1p-30) + 0x1p-44;
    if (!(d < HALF_PI)) return 1;
    *delta = d;
    return 0;
}

// First position of slab j with quantised angle >= x / > x.
__device__ __forceinline__ uint32_t lower_pos(const Geo &g, int j, uint32_t x) {
    const uint32_t *T = g.btab + g.bto[j];
    uint32_t b = x >> g.bshift[j];
    uint32_t lo = T[b], hi = T[b + 1];
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((g.keys[mid] & QMASK) < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ uint32_t upper_pos(const Geo &g, int j, uint32_t x) {
    const uint32_t *T = g.btab + g.bto[j];
    uint32_t b = x >> g.bshift[j];
    uint32_t lo = T[b], hi = T[b + 1];
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((g.keys[mid] & QMASK) <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Circular window (start, count) of sorted query s (slab i) in slab j >= i.
__device__ uint2 window(const Geo &g, uint32_t s, int i, int j, double thv, double rv, double shv, uint32_t qv) {
    const uint32_t bs = g.bs[j], be = g.bs[j + 1], nj = be - bs;
    if (nj == 0) return make_uint2(bs, 0u);
    double delta = 0.0;
    const int whole = (j == 0) ? 1 : half_width(rv, shv, g.c[j], g.shc[j], g.Kw, &delta);
    if (j == i) {
        uint32_t cnt;
        if (whole) {
            if (qv < QHALF) {
                cnt = upper_pos(g, j, qv + QHALF) - s - 1;
            } else {
                cnt = (be - s - 1) + (lower_pos(g, j, qv - QHALF) - bs);
            }
        } else {
            double hi = thv + delta;
            if (hi < TWO_PI) {
                cnt = upper_pos(g, j, qang(hi)) - s - 1;
            } else {
                cnt = (be - s - 1) + (upper_pos(g, j, qang(hi - TWO_PI)) - bs);
            }
        }
        return make_uint2(s + 1, cnt);
    }
    if (whole) return make_uint2(bs, nj);
    double lo = thv - delta, hi = thv + delta;
    if (lo < 0.0) {
        uint32_t a = lower_pos(g, j, qang(lo + TWO_PI));
        uint32_t e = upper_pos(g, j, qang(hi));
        return make_uint2(a, (be - a) + (e - bs));
    }
    if (hi >= TWO_PI) {
        uint32_t a = lower_pos(g, j, qang(lo));
        uint32_t e = upper_pos(g, j, qang(hi - TWO_PI));
        return make_uint2(a, (be - a) + (e - bs));
    }
    uint32_t a = lower_pos(g, j, qang(lo));
    uint32_t e = upper_pos(g, j, qang(hi));
    return make_uint2(a, e - a);
}

__device__ __forceinline__ uint64_t win_offset(const Geo &g, uint32_t s, int i) {
    return g.winbase[i] + (uint64_t)(s - g.bs[i]) * (uint64_t)(g.B - i);
}

__global__ __launch_bounds__(256) void k_plan(Geo g, uint2 *win, uint64_t *batch_cand) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t total = 0;
    if (s < g.n) {
        const uint32_t key = g.keys[s];
        const int i = (int)(key >> QBITS);
        const uint32_t qv = key & QMASK;
        const double thv = g.th[s], rv = g.rr[s], shv = g.sh[s];
        uint2 *w = win + win_offset(g, s, i);
        for (int j = i; j < g.B; ++j) {
            uint2 x = window(g, s, i, j, thv, rv, shv, qv);
            w[j - i] = x;
            total += x.y;
        }
    }
    uint64_t sum = wave_sum_u64(total);
    if ((threadIdx.x & 63) == 0 && (s >> 6) < (g.n + 63) / 64) batch_cand[s >> 6] = sum;
}

void plan(const Geo &g, uint2 *win, uint64_t *batch_cand, hipStream_t st) {
    if (!g.n) return;
    hipLaunchKernelGGL(k_plan, dim3((g.n + 255) / 256), dim3(256), 0, st, g, win, batch_cand);
}

// ---------------------------------------------------------------------------
// Distance test (Eq. 3).  The canonical FP64 value is
//   V = 0.5 (ep_u em_w + em_u ep_w) + 2 (sh_u sh_w) d^2,  d = hs_u hc_w - hc_u hs_w,
// one rounding per operation.  The query-side halves/doubles (0.5 ep_u,
// 0.5 em_u, 2 sh_u) are exact power-of-two scalings, so
//   V = (hep_u em_w + hem_u ep_w) + (sh2_u sh_w) d^2
// rounds to the same bits with two multiplications fewer.
// FP32 filter: with d computed in FP64 and rounded once, every FP32 operand
// and operation adds at most a relative u32 = 2^-24 to a sum of positive
// terms, so |V32 - W| <= gamma_8 W and |V64 - W| <= gamma_6(2^-53) W for the
// exact W of the table values; with mu = 2^-20 > gamma_8 + gamma_6,
// V32 <= RD(K(1-mu)) implies V64 < K and V32 >= RU(K(1+mu)) implies V64 >= K.
// Pairs between the two thresholds are decided by V64.
// ---------------------------------------------------------------------------
struct Qv {
    double hep, hem, sh2, hs, hc;
    float hep32, hem32, sh2_32;
};

template <int FP32>
__device__ __forceinline__ int edge_test(const Geo &g, const Qv &q, uint32_t p, uint32_t &rechecks,
                                         uint32_t &disagree, int exhaustive) {
    const double hsw = g.hs[p], hcw = g.hc[p];
    const double d = q.hs * hcw - q.hc * hsw;
    if (!FP32) {
        const double a = q.hep * g.em[p] + q.hem * g.ep[p];
        const double b = (q.sh2 * g.sh[p]) * (d * d);
        return (a + b) < g.K;
    } else {
        const float d32 = (float)d;
        const float a32 = q.hep32 * g.em32[p] + q.hem32 * g.ep32[p];
        const float b32 = (q.sh2_32 * d32) * (g.sh32[p] * d32);
        const float v32 = a32 + b32;
        int dec = (v32 <= g.klo32) ? 1 : ((v32 >= g.khi32) ? 0 : -1);
        if (dec < 0 || exhaustive) {
            const double a = q.hep * g.em[p] + q.hem * g.ep[p];
            const double b = (q.sh2 * g.sh[p]) * (d * d);
            const int e64 = (a + b) < g.K;
            if (dec < 0) {
                ++rechecks;
                dec = e64;
            } else if (dec != e64) {
                ++disagree;
            }
        }
        return dec;
    }
}

// Per-unit setup shared by the count and emit passes.
struct UnitSetup {
    uint32_t b;
    uint64_t r0, r1;
    uint32_t v;
    bool valid;
    int iv, jmin;
    const uint2 *mywin;
};

__device__ __forceinline__ UnitSetup unit_setup(const QueryArgs &A, uint64_t unit, int lane) {
    const Geo &g = A.geo;
    UnitSetup u;
    u.b = A.unit_batch[unit];
    const uint64_t chunk = unit - A.unit_off[u.b];
    u.r0 = chunk * UNIT;
    const uint64_t bc = A.batch_cand[u.b];
    u.r1 = (u.r0 + UNIT < bc) ? u.r0 + UNIT : bc;
    u.v = u.b * BATCH + lane;
    u.valid = u.v < g.n;
    u.iv = u.valid ? (int)(g.keys[u.v] >> QBITS) : g.B;
    u.jmin = (int)(g.keys[u.b * BATCH] >> QBITS);
    u.mywin = u.valid ? A.win + win_offset(g, u.v, u.iv) : nullptr;
    return u;
}

// Lane's window in slab j (0 count if none), scanned over the wavefront.
__device__ __forceinline__ void slab_windows(const UnitSetup &u, int j, uint32_t &st, uint32_t &cnt,
                                             uint32_t &excl, uint32_t &tot) {
    st = 0;
    cnt = 0;
    if (u.valid && j >= u.iv) {
        const uint2 x = u.mywin[j - u.iv];
        st = x.x;
        cnt = x.y;
    }
    const uint32_t incl = wave_incl_scan_u32(cnt);
    tot = wave_bcast_u32(incl, 63);
    excl = incl - cnt;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Window index of flattened candidate t: the last lane whose exclusive offset is <= t.
__device__ __forceinline__ int find_window(const uint32_t *excl, uint32_t t) {
    int l = 0;
#pragma unroll
    for (int stp = 32; stp; stp >>= 1)
        if (excl[l + stp] <= t) l += stp;
    return l;
}

// Count pass: decide every candidate of the unit, record the decisions as a
// bitmap over the unit's flattened positions (64 x 64 bits), count edges.
template <int FP32>
__global__ __launch_bounds__(256) void k_count(QueryArgs A) {
    __shared__ uint32_t s_excl[4][64];
    __shared__ uint32_t s_start[4][64];
    __shared__ double s_qd[4][5][64];
    __shared__ float s_qf[4][3][64];
    __shared__ unsigned long long s_bits[4][65];

    const Geo &g = A.geo;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t unit = (uint64_t)blockIdx.x * 4 + w;
    if (unit >= A.n_units) return;  // uniform per wavefront; no block-wide barriers below
    const UnitSetup u = unit_setup(A, unit, lane);
    if (u.valid) {
        s_qd[w][0][lane] = 0.5 * g.ep[u.v];
        s_qd[w][1][lane] = 0.5 * g.em[u.v];
        s_qd[w][2][lane] = 2.0 * g.sh[u.v];
        s_qd[w][3][lane] = g.hs[u.v];
        s_qd[w][4][lane] = g.hc[u.v];
        if (FP32) {
            s_qf[w][0][lane] = 0.5f * g.ep32[u.v];
            s_qf[w][1][lane] = 0.5f * g.em32[u.v];
            s_qf[w][2][lane] = 2.0f * g.sh32[u.v];
        }
    }
    s_bits[w][lane] = 0ull;
    if (lane == 0) s_bits[w][64] = 0ull;

    uint64_t pos = 0;  // flattened offset of slab j's segment within the batch
    uint32_t found = 0, rechecks = 0, disagree = 0;
    for (int j = u.jmin; j < g.B; ++j) {
        uint32_t st, cnt, excl, tot;
        slab_windows(u, j, st, cnt, excl, tot);
        if (pos + tot <= u.r0) {
            pos += tot;
            continue;
        }
        if (pos >= u.r1) break;
        wave_lds_sync();
        s_excl[w][lane] = excl;
        s_start[w][lane] = st;
        wave_lds_sync();
        const uint32_t a = (u.r0 > pos) ? (uint32_t)(u.r0 - pos) : 0u;
        const uint32_t e = (u.r1 - pos < tot) ? (uint32_t)(u.r1 - pos) : tot;
        const uint32_t be = g.bs[j + 1], nj = be - g.bs[j];
        for (uint32_t t0 = a; t0 < e; t0 += 64) {
            const uint32_t t = t0 + lane;
            int flag = 0;
            if (t < e) {
                const int l = find_window(s_excl[w], t);
                uint32_t p = s_start[w][l] + (t - s_excl[w][l]);
                if (p >= be) p -= nj;
                if (p >= be) p = be - 1;  // unreachable for consistent windows; keeps reads in bounds
                Qv q;
                q.hep = s_qd[w][0][l];
                q.hem = s_qd[w][1][l];
                q.sh2 = s_qd[w][2][l];
                q.hs = s_qd[w][3][l];
                q.hc = s_qd[w][4][l];
                if (FP32) {
                    q.hep32 = s_qf[w][0][l];
                    q.hem32 = s_qf[w][1][l];
                    q.sh2_32 = s_qf[w][2][l];
                }
                flag = edge_test<FP32>(g, q, p, rechecks, disagree, A.exhaustive);
            }
            const uint64_t m = __ballot(flag);
            if (m) {
                found += (uint32_t)__popcll(m);
                if (lane == 0) {
                    const uint32_t o = (uint32_t)(pos + t0 - u.r0);
                    const uint32_t wd = o >> 6, sh = o & 63u;
                    s_bits[w][wd] |= m << sh;
                    if (sh) s_bits[w][wd + 1] |= m >> (64u - sh);
                }
            }
        }
        pos += tot;
    }
    wave_lds_sync();
    A.bits[unit * 64 + lane] = s_bits[w][lane];
    if (lane == 0) A.unit_edges[unit] = found;
    if (FP32) {
        const uint64_t rc = wave_sum_u64(rechecks), dg = wave_sum_u64(disagree);
        if (lane == 0 && rc) atomicAdd(&A.stats[0], (unsigned long long)rc);
        if (lane == 0 && dg) atomicAdd(&A.stats[1], (unsigned long long)dg);
    }
}

// Emit pass: walk the unit exactly as the count pass did, take the decisions
// from its bitmap, and write (min, max) original-index pairs, compacted per
// 64-candidate round, at the unit's offset in the edge list.
__global__ __launch_bounds__(256) void k_emit(QueryArgs A) {
    __shared__ uint32_t s_excl[4][64];
    __shared__ uint32_t s_start[4][64];
    __shared__ uint32_t s_qi[4][64];
    __shared__ unsigned long long s_bits[4][65];

    const Geo &g = A.geo;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t unit = (uint64_t)blockIdx.x * 4 + w;
    if (unit >= A.n_units) return;
    const uint32_t todo = A.unit_edges[unit];
    if (todo == 0) return;
    const UnitSetup u = unit_setup(A, unit, lane);
    if (u.valid) s_qi[w][lane] = g.idx[u.v];
    s_bits[w][lane] = A.bits[unit * 64 + lane];
    if (lane == 0) s_bits[w][64] = 0ull;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t out_at = A.unit_edge_off[unit];
    const uint64_t out_end = out_at + todo;

    uint64_t pos = 0;
    for (int j = u.jmin; j < g.B && out_at < out_end; ++j) {
        uint32_t st, cnt, excl, tot;
        slab_windows(u, j, st, cnt, excl, tot);
        if (pos + tot <= u.r0) {
            pos += tot;
            continue;
        }
        if (pos >= u.r1) break;
        wave_lds_sync();
        s_excl[w][lane] = excl;
        s_start[w][lane] = st;
        wave_lds_sync();
        const uint32_t a = (u.r0 > pos) ? (uint32_t)(u.r0 - pos) : 0u;
        const uint32_t e = (u.r1 - pos < tot) ? (uint32_t)(u.r1 - pos) : tot;
        const uint32_t be = g.bs[j + 1], nj = be - g.bs[j];
        for (uint32_t t0 = a; t0 < e && out_at < out_end; t0 += 64) {
            const uint32_t o = (uint32_t)(pos + t0 - u.r0);
            const uint32_t wd = o >> 6, sh = o & 63u;
            uint64_t m = s_bits[w][wd] >> sh;
            if (sh) m |= s_bits[w][wd + 1] << (64u - sh);
            if (e - t0 < 64) m &= (~0ull >> (64u - (e - t0)));
            if (!m) continue;
            if ((m >> lane) & 1ull) {
                const uint32_t t = t0 + lane;
                const int l = find_window(s_excl[w], t);
                uint32_t p = s_start[w][l] + (t - s_excl[w][l]);
                if (p >= be) p -= nj;
                if (p >= be) p = be - 1;
                const uint32_t qi = s_qi[w][l], wi = g.idx[p];
                const uint32_t lo = qi < wi ? qi : wi, hi = qi < wi ? wi : qi;
                const uint64_t at = out_at + (uint64_t)__popcll(m & lt);
                if (at < A.out_capacity) A.out[at] = make_int2((int)lo, (int)hi);
            }
            out_at += (uint64_t)__popcll(m);
        }
        pos += tot;
    }
}

static unsigned query_blocks(uint64_t units) { return (unsigned)((units + 3) / 4); }

void query_count(const QueryArgs &a, int fp32, hipStream_t st) {
    if (!a.n_units) return;
    if (fp32)
        hipLaunchKernelGGL((k_count<1>), dim3(query_blocks(a.n_units)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_count<0>), dim3(query_blocks(a.n_units)), dim3(256), 0, st, a);
}

void query_emit(const QueryArgs &a, int fp32, hipStream_t st) {
    (void)fp32;  // decisions come from the count pass's bitmap
    if (!a.n_units) return;
    hipLaunchKernelGGL(k_emit, dim3(query_blocks(a.n_units)), dim3(256), 0, st, a);
}

}  // namespace rhgk
