// small.hip -- generation of many small graphs together (serving path, and
// the allocation-free entry point).
//
// k_small: each workgroup generates one request completely:
// sample + slab keys, a workgroup-wide stable bucket sort, table gather,
// slab starts and bucket index, the window plan (plan_batch), batch and unit
// scans, the count pass (count_unit), the edge scan, an atomic reservation
// of its slice of the shared output pool, and the emit pass (emit_unit).
// Phases are separated by workgroup barriers; nothing returns to the host
// between them.  The arithmetic (slab keys, windows, distance test, unit
// walk) is the same code as the multi-launch path, so a request's edge list
// is byte-identical to rhg_generate's for the same parameters.
//
// small_group_spread (the server's groups): the same phases in seven
// launches, the per-request ones (sort, slab starts and bucket index; batch
// and unit scans; edge scan and pool reservation) one workgroup per request,
// the keys, the table rows with the window plan, the count and the emit of
// the whole group one wavefront per 64 points or per unit over the chip.  A
// group then takes about as long as its largest request's sort, not its
// whole generation on one CU.
#include <cmath>
#include <cstring>
#include <mutex>

#include "query_dev.h"
#include "rhg_internal.h"

namespace rhgk {
using namespace rhgd;

constexpr int SM_THREADS = 1024;
constexpr int SM_WAVES = SM_THREADS / 64;
struct SortSmem {
    uint32_t h[SM_WAVES];  // wavefront totals of the bucket scan
    uint32_t top[256];     // counts of the keys' top byte (slab << 3 | 3 angle bits)
};
// interpolation buckets of the bucket sort: the one-launch kernel's
// requests (at most 8192 points) and the spread sort's (up to the server's
// group cutoff, 4 points per bucket at 65536)
constexpr uint32_t SM_BUCKETS_ONE = 8192, SM_BUCKETS_SPREAD = 16384;
struct SortBucketSmem {
    SortSmem s;
    uint32_t bcnt[SM_BUCKETS_ONE];
};
struct ScanSmem {
    uint64_t wsum[SM_WAVES];
};
union PhaseSmem {
    SortBucketSmem sort;
    CountSmem<0> count0[SM_WAVES];
    CountSmem<1> count1[SM_WAVES];
    EmitSmem emit[SM_WAVES];
};

__device__ __forceinline__ uint64_t blk_excl_scan(uint64_t x, uint64_t *total, ScanSmem &S) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint64_t incl = wave_incl_scan_u64(x);
    if (l == 63) S.wsum[w] = incl;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int k = 0; k < SM_WAVES; ++k) {
        if (k < w) before += S.wsum[k];
        tot += S.wsum[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

// out[0..len] = exclusive prefix of in[0..len) (out[len] = total), one workgroup.
template <typename T>
__device__ __forceinline__ void blk_scan_array(const T *in, uint64_t *out, uint32_t len, ScanSmem &S) {
    uint64_t carry = 0;
    for (uint32_t base = 0; base < len; base += SM_THREADS) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t x = i < len ? (uint64_t)in[i] : 0;
        uint64_t tot;
        const uint64_t ex = blk_excl_scan(x, &tot, S);
        if (i < len) out[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) out[len] = carry;
    __syncthreads();
}

// Global-memory views of the sort's buffers: their loads and stores then
// compile to global instructions, counted apart from the LDS ones, so that
// waiting for an LDS result does not also wait for every store in flight
// (generic pointers give flat instructions, counted with both).
typedef __attribute__((address_space(1))) uint32_t g_u32;
__device__ __forceinline__ const g_u32 *as_global(const uint32_t *p) { return (const g_u32 *)p; }
__device__ __forceinline__ g_u32 *as_global(uint32_t *p) { return (g_u32 *)p; }

// The counts of the keys' top byte into S.top, SM_UNROLL keys per thread in flight.
constexpr int SM_UNROLL = 8;
__device__ __forceinline__ void blk_top_counts(const uint32_t *keys_, uint32_t n, SortSmem &S) {
    const g_u32 *keys = as_global(keys_);
    const int t = threadIdx.x;
    for (int x = t; x < 256; x += SM_THREADS) S.top[x] = 0;
    __syncthreads();
    for (uint32_t base = t; base < n; base += SM_UNROLL * SM_THREADS) {
        uint32_t k[SM_UNROLL];
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {  // unconditional loads (index clamped): all in flight at once
            const uint32_t i = base + (uint32_t)u * SM_THREADS;
            k[u] = keys[i < n ? i : 0u];
        }
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u)
            if (base + (uint32_t)u * SM_THREADS < n) atomicAdd(&S.top[k[u] >> 24], 1u);
    }
    __syncthreads();
}

// Bucket of a slab key for the bucket sort: its rank estimated from its
// slab's start and size and its angle (uniform within the slab for sampled
// points), scaled to nbk buckets.  Non-decreasing in the key, so every key
// of bucket b is below every key of bucket b + 1 and equal keys share one.
// (scale = nbk / n in FP32: a rounded product is still non-decreasing in
// the estimate, and the clamp keeps the last bucket; no integer division)
__device__ __forceinline__ uint32_t sort_bucket(uint32_t key, const uint32_t *bs, float scale, uint32_t nbk) {
    const uint32_t j = key >> QBITS, start = bs[j], nj = bs[j + 1] - start;
    const uint32_t est = start + (uint32_t)(((uint64_t)(key & QMASK) * nj) >> QBITS);  // in [start, start + nj)
    const uint32_t b = (uint32_t)((float)est * scale);
    return b < nbk ? b : nbk - 1u;
}

// Stable sort of the keys with their payload by interpolation buckets, by
// one workgroup, given the slab starts bs[0..B]: bucket counts and offsets,
// the pairs scattered into their buckets (keys2, vals2, any order inside a
// bucket), and each pair written to keys, vals at its bucket's start plus
// the number of pairs of its bucket below it in (key, payload) order.  With
// the payload the original position, that is the order a stable sort of the
// keys gives.  The order holds for any bucket sizes; the cost assumes small
// buckets, which sampled points give (their angles are uniform within a
// slab, about Poisson(n / nbk) points per bucket).
template <uint32_t NBK>
__device__ __forceinline__ void blk_bucket_sort(const SmallDesc &D, uint32_t n, const uint32_t *bs, SortSmem &S,
                                                uint32_t *bcnt) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t nbk = n < NBK ? n : NBK;
    const float scale = (float)nbk / (float)n;
    const g_u32 *keys = as_global(D.keys), *vals = as_global(D.vals);
    g_u32 *k2 = as_global(D.keys2), *v2 = as_global(D.vals2);
    for (uint32_t b = t; b < nbk; b += SM_THREADS) bcnt[b] = 0;
    __syncthreads();
    for (uint32_t base = t; base < n; base += SM_UNROLL * SM_THREADS) {
        uint32_t k[SM_UNROLL];
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            const uint32_t i = base + (uint32_t)u * SM_THREADS;
            k[u] = keys[i < n ? i : 0u];
        }
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            if (base + (uint32_t)u * SM_THREADS < n) atomicAdd(&bcnt[sort_bucket(k[u], bs, scale, nbk)], 1u);
        }
    }
    __syncthreads();
    // exclusive offsets: NBK / SM_THREADS consecutive buckets per thread
    constexpr uint32_t PER = NBK / SM_THREADS;
    static_assert(NBK % SM_THREADS == 0, "buckets per thread");
    uint32_t c[PER], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t b = (uint32_t)t * PER + q;
        c[q] = b < nbk ? bcnt[b] : 0u;
        sum += c[q];
    }
    const uint32_t incl = wave_incl_scan_u32(sum);
    if (l == 63) S.h[w] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int q = 0; q < w; ++q) run += S.h[q];
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t b = (uint32_t)t * PER + q;
        if (b < nbk) bcnt[b] = run;
        run += c[q];
    }
    __syncthreads();
    // scatter: bcnt[b] advances from the bucket's start to its end
    for (uint32_t base = t; base < n; base += SM_UNROLL * SM_THREADS) {
        uint32_t k[SM_UNROLL], v[SM_UNROLL];
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            const uint32_t i = base + (uint32_t)u * SM_THREADS, ic = i < n ? i : 0u;
            k[u] = keys[ic];
            v[u] = vals[ic];
        }
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            if (base + (uint32_t)u * SM_THREADS < n) {
                const uint32_t pos = atomicAdd(&bcnt[sort_bucket(k[u], bs, scale, nbk)], 1u);
                k2[pos] = k[u];
                v2[pos] = v[u];
            }
        }
    }
    __syncthreads();
    // each pair to its place: its bucket's start plus its rank inside the
    // bucket; SM_UNROLL pairs per thread, the m-th members of their buckets
    // loaded together
    for (uint32_t base = t; base < n; base += SM_UNROLL * SM_THREADS) {
        uint32_t key[SM_UNROLL], val[SM_UNROLL], st[SM_UNROLL], en[SM_UNROLL], rank[SM_UNROLL];
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            const uint32_t p = base + (uint32_t)u * SM_THREADS, pc = p < n ? p : 0u;
            key[u] = k2[pc];
            val[u] = v2[pc];
        }
        uint32_t most = 0;
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            const uint32_t b = sort_bucket(key[u], bs, scale, nbk);
            st[u] = b ? bcnt[b - 1] : 0u;
            en[u] = base + (uint32_t)u * SM_THREADS < n ? bcnt[b] : st[u];
            rank[u] = 0;
            most = max(most, en[u] - st[u]);
        }
        for (uint32_t m = 0; m < most; ++m) {
            uint32_t kq[SM_UNROLL], vq[SM_UNROLL];
#pragma unroll
            for (int u = 0; u < SM_UNROLL; ++u) {
                const uint32_t q = st[u] + m < en[u] ? st[u] + m : 0u;
                kq[u] = k2[q];
                vq[u] = v2[q];
            }
#pragma unroll
            for (int u = 0; u < SM_UNROLL; ++u)
                if (st[u] + m < en[u]) rank[u] += (kq[u] < key[u] || (kq[u] == key[u] && vq[u] < val[u])) ? 1u : 0u;
        }
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            if (base + (uint32_t)u * SM_THREADS < n) {
                as_global(D.keys)[st[u] + rank[u]] = key[u];
                as_global(D.vals)[st[u] + rank[u]] = val[u];
            }
        }
    }
    __syncthreads();
}

// The static geometry of a request (n, B, R, K, Kw, FP32 thresholds, c,
// sinh/exp/reciprocal constants) into the LDS copy, a word per thread.
__device__ __forceinline__ void geo_to_lds(const Geo &src, Geo &dst) {
    static_assert(sizeof(Geo) % 4 == 0, "Geo words");
    const uint32_t *a = (const uint32_t *)&src;
    uint32_t *b = (uint32_t *)&dst;
    for (uint32_t k = threadIdx.x; k < sizeof(Geo) / 4; k += SM_THREADS) b[k] = a[k];
}

// a0 + a2 of point i: its sample, slab (thresholds of the static geometry
// g) and key, with the payload i.
__device__ __forceinline__ void small_key_of(const SmallDesc &D, const Geo &g, uint32_t i) {
    double th, r;
    load_point(D.src, i, th, r);
    int b = 0;
    while (b + 1 < g.B && g.c[b + 1] <= r) ++b;
    D.keys[i] = ((uint32_t)b << QBITS) | qang(th);
    D.vals[i] = i;
}

// a1 of sorted position s: the table row of the point there.
__device__ __forceinline__ void small_row_of(const SmallDesc &D, uint32_t s) {
    const uint32_t v = D.vals[s];
    double th, r, a, b, c, d, e;
    load_point(D.src, v, th, r);
    point_table(D.src, v, th, r, a, b, c, d, e);
    D.th[s] = th;
    D.epm[s] = make_double2(a, b);
    D.hsc[s] = make_double2(d, e);
    if (D.f32) D.f32[s] = make_float2((float)a, (float)b);
}

// a3 and the layout, by one workgroup, after the keys: stable bucket sort
// (result back in keys/vals), slab starts, bucket bits and window bases in
// sA.geo (whose static part is set).  False (with Z.status = 1) when the
// request outgrows its scratch.
template <uint32_t NBK>
__device__ __forceinline__ bool small_sort_layout(const SmallDesc &D, SmallResult &Z, QueryArgs &sA, SortSmem &SO,
                                                  uint32_t *bcnt, uint32_t *s_bs, int &s_flag) {
    const int t = threadIdx.x;
    const uint32_t n = (uint32_t)D.src.n;
    const int B = D.geo.B;
    blk_top_counts(D.keys, n, SO);

    // slab starts from the top-byte counts: the keys have QBITS + 1..5 bits,
    // so the top byte is (slab << (QBITS - 24)) | the top angle bits, and
    // slab j holds the keys whose top byte lies in [j, j + 1) << (QBITS - 24)
    static_assert(QBITS > 24 && QBITS + 5 <= 32 && (MAX_BANDS << (QBITS - 24)) <= 256, "slab starts from the top byte");
    if (t <= B) {
        const uint32_t dend = min((uint32_t)t << (QBITS - 24), 256u);
        uint32_t lo = 0;
        for (uint32_t d = 0; d < dend; ++d) lo += SO.top[d];
        s_bs[t] = t == B ? n : lo;
    }
    __syncthreads();

    blk_bucket_sort<NBK>(D, n, s_bs, SO, bcnt);

    if (t == 0) {
        uint64_t wins = 0, btl = 0;
        for (int j = 0; j < B; ++j) {
            sA.geo.bs[j] = s_bs[j];
            sA.geo.winbase[j] = wins;
            const uint32_t nj = s_bs[j + 1] - s_bs[j];
            wins += s_bs[j + 1];
            int cl = 0;
            while ((1u << cl) < nj) ++cl;
            const int bits = max(0, min(24, cl - 1));
            sA.geo.bshift[j] = QBITS - bits;
            sA.geo.bto[j] = (uint32_t)btl;
            btl += (1ull << bits) + 1;
        }
        sA.geo.bs[B] = n;
        sA.geo.winbase[B] = wins;
        sA.geo.keys = D.keys;
        sA.geo.idx = D.vals;
        sA.geo.th = D.th;
        sA.geo.epm = D.epm;
        sA.geo.hsc = D.hsc;
        sA.geo.f32 = D.f32;
        sA.geo.btab = D.btab;
        Z.windows = wins;
        if (wins > D.win_cap || btl > D.btab_cap) s_flag = 1;
    }
    __syncthreads();
    if (s_flag) {
        if (t == 0) Z.status = 1;
        return false;
    }
    return true;
}

// The slab bucket index of the sorted keys, by one workgroup.
__device__ __forceinline__ void small_bucket(const SmallDesc &D, const Geo &g) {
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint32_t n = (uint32_t)D.src.n;
    for (uint32_t base = t; base < n; base += SM_UNROLL * SM_THREADS) {
        uint32_t kc[SM_UNROLL], kp[SM_UNROLL];
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {  // unconditional loads (index clamped): all in flight at once
            const uint32_t s = base + (uint32_t)u * SM_THREADS, sc = s < n ? s : 0u;
            kc[u] = D.keys[sc];
            kp[u] = D.keys[sc > 0u ? sc - 1u : 0u];
        }
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
            const uint32_t s = base + (uint32_t)u * SM_THREADS;
            if (s < n) {
                const int j = (int)(kc[u] >> QBITS);
                const int sh = g.bshift[j];
                const int64_t b = (int64_t)((kc[u] & QMASK) >> sh);
                const int64_t bp = (s == g.bs[j]) ? -1 : (int64_t)((kp[u] & QMASK) >> sh);
                uint32_t *T = D.btab + g.bto[j];
                for (int64_t k = bp + 1; k <= b; ++k) T[k] = s;
            }
        }
    }
    for (int j = w; j < g.B; j += SM_WAVES) {
        const uint32_t nbk = 1u << (QBITS - g.bshift[j]);
        uint32_t *T = D.btab + g.bto[j];
        const uint32_t bs = g.bs[j], be = g.bs[j + 1];
        int64_t first = 0;
        if (be > bs) first = (int64_t)((D.keys[be - 1] & QMASK) >> g.bshift[j]) + 1;
        for (int64_t k = first + lane; k <= (int64_t)nbk; k += 64) T[k] = be;
    }
}

// Phases a0-a3 of one request by one workgroup (sample, slab keys, sort,
// slab starts, table, bucket index), leaving its geometry in sA.geo.  False
// (with Z.status = 1) when the request outgrows its scratch.
__device__ __forceinline__ bool small_tables(const SmallDesc &D, SmallResult &Z, QueryArgs &sA, PhaseSmem &P, uint32_t *s_bs,
                             int &s_flag) {
    const int t = threadIdx.x;
    const uint32_t n = (uint32_t)D.src.n;
    geo_to_lds(D.geo, sA.geo);
    if (t == 0) s_flag = 0;
    __syncthreads();
    for (uint32_t i = t; i < n; i += SM_THREADS) small_key_of(D, sA.geo, i);
    __syncthreads();
    if (!small_sort_layout<SM_BUCKETS_ONE>(D, Z, sA, P.sort.s, P.sort.bcnt, s_bs, s_flag)) return false;
    for (uint32_t s = t; s < n; s += SM_THREADS) small_row_of(D, s);
    small_bucket(D, sA.geo);
    __syncthreads();
    return true;
}

// Phase a4 after the window plan, by one workgroup: batch and unit scans and
// the units' batches; the query arguments completed in A (LDS or device
// memory) and the unit count in U.  False (with Z.status = 1) when the
// units outgrow the request's scratch.
__device__ __forceinline__ bool small_units(const SmallDesc &D, SmallResult &Z, QueryArgs &A, ScanSmem &SS, uint64_t &U_out) {
    const int t = threadIdx.x;
    const uint32_t n = (uint32_t)D.src.n;
    const uint32_t nb = (n + 63) / 64;
    blk_scan_array(D.bcand, D.boff, nb, SS);
    for (uint32_t b = t; b < nb; b += SM_THREADS) D.nunits[b] = (D.bcand[b] + UNIT - 1) / UNIT;
    __syncthreads();
    blk_scan_array(D.nunits, D.uoff, nb, SS);
    const uint64_t U = D.uoff[nb];
    if (U > D.unit_cap) {
        if (t == 0) Z.status = 1;
        return false;
    }
    for (uint32_t u = t; u < U; u += SM_THREADS) {
        uint32_t lo = 0, hi = nb;
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (D.uoff[mid] <= u) lo = mid; else hi = mid;
        }
        D.ubatch[u] = lo;
    }
    if (t == 0) {
        A.win = D.win;
        A.batch_cand = D.bcand;
        A.batch_slab_off = D.bsoff;
        A.unit_off = D.uoff;
        A.unit_batch = D.ubatch;
        A.unit_order = nullptr;
        A.n_units = U;
        A.unit_base = 0;
        A.udesc = nullptr;
        A.unit_edges = D.uedges;
        A.bits = D.bits;
        A.unit_edge_off = D.ueoff;
        A.out = nullptr;
        A.out_capacity = 0;
        A.stats = D.stats;
        A.exhaustive = 0;
        Z.candidates = D.boff[nb];
    }
    __syncthreads();

    U_out = U;
    return true;
}

__global__ __launch_bounds__(SM_THREADS) void k_small(const SmallDesc *descs, SmallResult *results, int2 *pool,
                                                      unsigned long long *pool_used, uint64_t pool_cap) {
    __shared__ QueryArgs sA;
    __shared__ PhaseSmem P;
    __shared__ ScanSmem SS;
    __shared__ uint32_t s_bs[MAX_BANDS + 1];
    __shared__ int s_flag;

    const SmallDesc &D = descs[blockIdx.x];
    SmallResult &Z = results[blockIdx.x];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint32_t n = (uint32_t)D.src.n;
    uint64_t U = 0;
    if (!small_tables(D, Z, sA, P, s_bs, s_flag)) return;
    // ---- a4: window plan per batch
    {
        const uint32_t nb = (n + 63) / 64;
        for (uint32_t b = w; b < nb; b += SM_WAVES) plan_batch(sA.geo, D.win, D.bcand, D.bsoff, b, lane);
        __syncthreads();
    }
    if (!small_units(D, Z, sA, SS, U)) return;

    // ---- a5: count
    for (uint64_t u = w; u < U; u += SM_WAVES) {
        if (D.fp32) count_unit<1, false>(sA, u, u, lane, P.count1[w]);
        else count_unit<0, false>(sA, u, u, lane, P.count0[w]);
    }
    __syncthreads();

    // ---- a6: edge offsets per unit, m, and this request's slice of the pool
    blk_scan_array(D.uedges, D.ueoff, (uint32_t)U, SS);
    if (t == 0) {
        // reserve [off, off + m) of the pool only if it fits, so that one
        // overflowing request leaves the pool to the others
        const uint64_t m = D.ueoff[U];
        unsigned long long cur = atomicAdd(pool_used, 0ull), off = 0;
        int fits = 0;
        for (;;) {
            if (cur + m > pool_cap) break;
            const unsigned long long prev = atomicCAS(pool_used, cur, cur + m);
            if (prev == cur) {
                off = cur;
                fits = 1;
                break;
            }
            cur = prev;
        }
        Z.m = m;
        Z.out_off = off;
        Z.rechecks = atomicAdd(&D.stats[0], 0ull);
        s_flag = fits ? 0 : 1;
        sA.out = pool + off;
        sA.out_capacity = m;
    }
    __syncthreads();
    if (s_flag) {
        if (t == 0) Z.status = 2;
        return;
    }

    // ---- a7: emit
    for (uint64_t u = w; u < U; u += SM_WAVES) emit_unit<false>(sA, u, u, lane, P.emit[w]);
    if (t == 0) Z.status = 0;
}

void small_group(const SmallDesc *descs, SmallResult *results, int count, int2 *pool,
                 unsigned long long *pool_used, uint64_t pool_cap, hipStream_t st) {
    if (count > 0)
        hipLaunchKernelGGL(k_small, dim3(count), dim3(SM_THREADS), 0, st, descs, results, pool, pool_used, pool_cap);
}

// ---- the spread launch: the per-point work (keys; table rows with the
// window plan) and the count and emit over the whole chip (grid-stride,
// wavefront per 64 points or per unit), the sort and scans per request

// Request of global item k: the last r with pre[r] <= k (pre: prefix of the
// items of the requests taking part, in LDS).
__device__ __forceinline__ int small_request_of(const uint64_t *pre, int count, uint64_t k) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (pre[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

// pre[r] = work items of the requests before r, pre[count] = their total.
// Items: units, or 64-point batches, of the requests whose status is 0 so
// far; or (ITEM_BATCHES_ALL, the group's first launch, before any status is
// written) the 64-point batches of every request.
// (count <= 128: the first wavefront scans two entries per lane)
constexpr int ITEM_UNITS = 0, ITEM_BATCHES = 1, ITEM_BATCHES_ALL = 2;
template <int ITEMS = ITEM_UNITS>
__device__ __forceinline__ void small_unit_prefix(const SmallDesc *descs, const SmallResult *results, int count,
                                                  uint64_t *pre) {
    static_assert(SMALL_GROUP_MAX <= 128, "two entries per lane");
    if (threadIdx.x < 64) {
        const int l = (int)threadIdx.x;
        auto items = [&](int r) -> uint64_t {
            if (r >= count) return 0;
            if (ITEMS != ITEM_BATCHES_ALL && results[r].status != 0) return 0;
            return ITEMS == ITEM_UNITS ? results[r].units : (descs[r].src.n + 63) / 64;
        };
        const uint64_t v0 = items(l), v1 = items(l + 64);
        const uint64_t i0 = wave_incl_scan_u64(v0);
        const uint64_t t0 = __shfl(i0, 63, 64);
        const uint64_t i1 = t0 + wave_incl_scan_u64(v1);
        if (l < count) pre[l] = i0 - v0;
        if (l + 64 < count) pre[l + 64] = i1 - v1;
        const uint64_t total = __shfl(i1, 63, 64);
        if (l == 0) pre[count] = total;
    }
    __syncthreads();
}

constexpr int SP_THREADS = 256, SP_WAVES = SP_THREADS / 64;

// a0 + a2 of every point of the group: sample, slab and key, a wavefront per 64 points
__global__ __launch_bounds__(SP_THREADS) void k_small_keys(const SmallDesc *descs, int count) {
    __shared__ uint64_t pre[SMALL_GROUP_MAX + 1];
    small_unit_prefix<ITEM_BATCHES_ALL>(descs, nullptr, count, pre);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const uint64_t total = pre[count];
    for (uint64_t k = (uint64_t)blockIdx.x * SP_WAVES + w; k < total; k += (uint64_t)gridDim.x * SP_WAVES) {
        const int r = small_request_of(pre, count, k);
        const SmallDesc &D = descs[r];
        const uint32_t i = (uint32_t)(k - pre[r]) * 64u + (uint32_t)lane;
        if (i < (uint32_t)D.src.n) small_key_of(D, D.geo, i);
    }
}

// a3 per request, one workgroup each: sort, slab starts, layout and bucket
// index; the query arguments (the geometry so far) then go to device memory
// for the next launches, and the status is set
__global__ __launch_bounds__(SM_THREADS) void k_small_sort(const SmallDesc *descs, SmallResult *results) {
    // the sort's LDS only (not the one-launch kernel's union of every
    // phase), so that the workgroup fits on a CU beside other work sooner
    __shared__ QueryArgs sA;
    __shared__ SortSmem P;
    __shared__ uint32_t bcnt[SM_BUCKETS_SPREAD];
    __shared__ uint32_t s_bs[MAX_BANDS + 1];
    __shared__ int s_flag;
    const SmallDesc &D = descs[blockIdx.x];
    SmallResult &Z = results[blockIdx.x];
    geo_to_lds(D.geo, sA.geo);
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    if (!small_sort_layout<SM_BUCKETS_SPREAD>(D, Z, sA, P, bcnt, s_bs, s_flag)) return;
    small_bucket(D, sA.geo);
    static_assert(sizeof(QueryArgs) % 4 == 0, "QueryArgs words");
    const uint32_t *src = (const uint32_t *)&sA;
    uint32_t *dst = (uint32_t *)D.qa;
    for (uint32_t k = threadIdx.x; k < sizeof(QueryArgs) / 4; k += SM_THREADS) dst[k] = src[k];
    if (threadIdx.x == 0) {
        Z.units = 0;
        Z.status = 0;
    }
}

// a1 and a4 of every batch of the group, a wavefront per batch: the table
// rows of its 64 points, then their windows (the plan reads back only the
// rows this lane has just written)
__global__ __launch_bounds__(SP_THREADS) void k_small_plan(const SmallDesc *descs, const SmallResult *results,
                                                           int count) {
    __shared__ uint64_t pre[SMALL_GROUP_MAX + 1];
    small_unit_prefix<ITEM_BATCHES>(descs, results, count, pre);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const uint64_t total = pre[count];
    for (uint64_t k = (uint64_t)blockIdx.x * SP_WAVES + w; k < total; k += (uint64_t)gridDim.x * SP_WAVES) {
        const int r = small_request_of(pre, count, k);
        const SmallDesc &D = descs[r];
        const uint32_t b = (uint32_t)(k - pre[r]);
        const uint32_t s = b * 64u + (uint32_t)lane;
        if (s < (uint32_t)D.src.n) small_row_of(D, s);
        plan_batch(D.qa->geo, D.win, D.bcand, D.bsoff, b, lane);
    }
}

__global__ __launch_bounds__(SM_THREADS) void k_small_units(const SmallDesc *descs, SmallResult *results) {
    __shared__ ScanSmem SS;
    const SmallDesc &D = descs[blockIdx.x];
    SmallResult &Z = results[blockIdx.x];
    if (Z.status != 0) return;  // uniform: set by the sort launch
    uint64_t U = 0;
    if (!small_units(D, Z, *D.qa, SS, U)) return;
    if (threadIdx.x == 0) Z.units = U;
}

__global__ __launch_bounds__(SP_THREADS) void k_small_count(const SmallDesc *descs, const SmallResult *results,
                                                            int count) {
    // one LDS area per wavefront, for either precision: the wavefronts of
    // a workgroup take units of different requests
    union WaveCount {
        CountSmem<0> c0;
        CountSmem<1> c1;
    };
    __shared__ uint64_t pre[SMALL_GROUP_MAX + 1];
    __shared__ WaveCount S[SP_WAVES];
    small_unit_prefix(descs, results, count, pre);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t total = pre[count];
    for (uint64_t k = (uint64_t)blockIdx.x * SP_WAVES + w; k < total; k += (uint64_t)gridDim.x * SP_WAVES) {
        const int r = small_request_of(pre, count, k);
        const uint64_t u = k - pre[r];
        const QueryArgs &A = *descs[r].qa;
        if (descs[r].fp32) count_unit<1, false>(A, u, u, lane, S[w].c1);
        else count_unit<0, false>(A, u, u, lane, S[w].c0);
    }
}

__global__ __launch_bounds__(SM_THREADS) void k_small_scan(const SmallDesc *descs, SmallResult *results, int2 *pool,
                                                           unsigned long long *pool_used, uint64_t pool_cap) {
    __shared__ ScanSmem SS;
    const SmallDesc &D = descs[blockIdx.x];
    SmallResult &Z = results[blockIdx.x];
    if (Z.status != 0) return;  // uniform: set by the setup launch
    const uint32_t U = (uint32_t)Z.units;
    blk_scan_array(D.uedges, D.ueoff, U, SS);
    if (threadIdx.x == 0) {
        // the pool reservation of the one-launch path
        const uint64_t m = D.ueoff[U];
        unsigned long long cur = atomicAdd(pool_used, 0ull), off = 0;
        int fits = 0;
        for (;;) {
            if (cur + m > pool_cap) break;
            const unsigned long long prev = atomicCAS(pool_used, cur, cur + m);
            if (prev == cur) {
                off = cur;
                fits = 1;
                break;
            }
            cur = prev;
        }
        Z.m = m;
        Z.out_off = off;
        Z.rechecks = atomicAdd(&D.stats[0], 0ull);
        D.qa->out = pool + off;
        D.qa->out_capacity = m;
        if (!fits) Z.status = 2;
    }
}

__global__ __launch_bounds__(SP_THREADS) void k_small_emit(const SmallDesc *descs, const SmallResult *results,
                                                           int count) {
    __shared__ uint64_t pre[SMALL_GROUP_MAX + 1];
    __shared__ EmitSmem S[SP_WAVES];
    small_unit_prefix(descs, results, count, pre);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t total = pre[count];
    for (uint64_t k = (uint64_t)blockIdx.x * SP_WAVES + w; k < total; k += (uint64_t)gridDim.x * SP_WAVES) {
        const int r = small_request_of(pre, count, k);
        const uint64_t u = k - pre[r];
        // decision words from the count launch: scalar loads
        emit_unit<false, true>(*descs[r].qa, u, u, lane, S[w]);
    }
}

void small_group_spread(const SmallDesc *descs, SmallResult *results, int count, int2 *pool,
                        unsigned long long *pool_used, uint64_t pool_cap, hipStream_t st) {
    if (count <= 0 || count > SMALL_GROUP_MAX) return;
    const unsigned spread = 1024;  // workgroups of 4 wavefronts: 4 per CU
    hipLaunchKernelGGL(k_small_keys, dim3(spread), dim3(SP_THREADS), 0, st, descs, count);
    hipLaunchKernelGGL(k_small_sort, dim3(count), dim3(SM_THREADS), 0, st, descs, results);
    hipLaunchKernelGGL(k_small_plan, dim3(spread), dim3(SP_THREADS), 0, st, descs, results, count);
    hipLaunchKernelGGL(k_small_units, dim3(count), dim3(SM_THREADS), 0, st, descs, results);
    hipLaunchKernelGGL(k_small_count, dim3(spread), dim3(SP_THREADS), 0, st, descs, results, count);
    hipLaunchKernelGGL(k_small_scan, dim3(count), dim3(SM_THREADS), 0, st, descs, results, pool, pool_used, pool_cap);
    hipLaunchKernelGGL(k_small_emit, dim3(spread), dim3(SP_THREADS), 0, st, descs, results, count);
}

}  // namespace rhgk

// ---------------------------------------------------------------------------
// Scratch layout of one request on this path (shared by the server's groups
// and the allocation-free entry point below).
// ---------------------------------------------------------------------------
namespace rhgi {

using rhgd::BITMAP_WORDS;

SmallLayout small_layout_units(uint64_t n, int B, uint64_t unit_cap, bool fp32) {
    SmallLayout L;
    const uint64_t nb = (n + 63) / 64;
    L.unit_cap = unit_cap;
    L.win_cap = n * (uint64_t)B;
    // slab j's bucket table has 2^bits_j + 1 <= n_j + 2 entries
    L.btab_cap = n + 2ull * B + 8;
    uint64_t b = 0;
    b += 4 * align256(4 * n);                          // keys, vals, keys2, vals2
    b += align256(8 * n) + 2 * align256(16 * n);       // th, epm, hsc
    if (fp32) b += align256(8 * n);                    // f32
    b += align256(4 * L.btab_cap) + align256(8 * L.win_cap);
    b += 2 * align256(8 * nb) + 2 * align256(8 * (nb + 1)) + align256(8 * nb * (uint64_t)(B + 1));
    // (the bitmap with 64 bytes past its last unit: the spread emit reads a
    // step's words as one run, up to 4 words past a unit's last)
    b += 2 * align256(4 * L.unit_cap) + align256(8 * (L.unit_cap + 1)) + align256(8 * L.unit_cap * BITMAP_WORDS + 64);
    L.bytes = b;
    return L;
}

void small_fill_desc(rhgk::SmallDesc &D, const Plan &pl, const Request &rq, const SmallLayout &lay, char *base,
                     unsigned long long *stats) {
    std::memset(&D, 0, sizeof(D));
    D.src.mode = rhgd::SRC_SEED;
    D.src.n = pl.n;
    D.src.seed = rq.seed;
    D.src.alpha = rq.alpha;
    D.src.R = rq.R;
    D.src.sinh_half_aR = std::sinh(rq.alpha * rq.R / 2.0);
    geo_static(pl, D.geo);
    D.fp32 = pl.fp32 ? 1 : 0;
    D.key_bits = key_bits_for(pl.B);
    const uint64_t n = pl.n, nb = (n + 63) / 64;
    char *p = base;
    auto take = [&](uint64_t bytes) {
        char *x = p;
        p += align256(bytes);
        return (void *)x;
    };
    D.keys = (uint32_t *)take(4 * n);
    D.vals = (uint32_t *)take(4 * n);
    D.keys2 = (uint32_t *)take(4 * n);
    D.vals2 = (uint32_t *)take(4 * n);
    D.th = (double *)take(8 * n);
    D.epm = (double2 *)take(16 * n);
    D.hsc = (double2 *)take(16 * n);
    D.f32 = pl.fp32 ? (float2 *)take(8 * n) : nullptr;
    D.btab_cap = lay.btab_cap;
    D.btab = (uint32_t *)take(4 * D.btab_cap);
    D.win_cap = lay.win_cap;
    D.win = (uint2 *)take(8 * D.win_cap);
    D.bcand = (uint64_t *)take(8 * nb);
    D.nunits = (uint64_t *)take(8 * nb);
    D.boff = (uint64_t *)take(8 * (nb + 1));
    D.uoff = (uint64_t *)take(8 * (nb + 1));
    D.bsoff = (uint64_t *)take(8 * nb * (uint64_t)(pl.B + 1));
    D.unit_cap = lay.unit_cap;
    D.ubatch = (uint32_t *)take(4 * D.unit_cap);
    D.uedges = (uint32_t *)take(4 * D.unit_cap);
    D.ueoff = (uint64_t *)take(8 * (D.unit_cap + 1));
    D.bits = (unsigned long long *)take(8 * D.unit_cap * BITMAP_WORDS + 64);
    D.stats = stats;
}

// ---------------------------------------------------------------------------
// Allocation-free generation (rhg_generate_noalloc): one request of at most
// NOALLOC_N points on the one-launch path, with every work array in `scratch`,
// a fixed device array of NOALLOC_BYTES that each device holds from the
// library's load until the process ends.
//
// Layout of the scratch (offsets in bytes):
//   0                  the request's descriptor (uploaded from pinned host memory)
//   HDR_ZERO           pool_used, rechecks, disagreements: three words that
//                      must start at zero, cleared by the same upload
//   HDR_RESULT         the request's SmallResult
//   HDR_BYTES ..       the request's arrays (small_layout_units with the
//                      worst-case unit count of n points)
//
// In host code `scratch` names a host-side stand-in: the device address of
// each device's copy is taken once per device with hipGetSymbolAddress
// (noalloc_setup, from rhg_ctx_create with that device current) and only
// that address is used.  Calls on one device share its array: calls that
// overlap in time on one device race and must be serialised by the caller.
// ---------------------------------------------------------------------------
constexpr uint64_t NOALLOC_N = 8192;
constexpr uint64_t NOALLOC_BYTES = 16ull << 20;
constexpr uint64_t HDR_ZERO = align256(sizeof(rhgk::SmallDesc));
constexpr uint64_t HDR_RESULT = HDR_ZERO + 256;
constexpr uint64_t HDR_BYTES = 4096;
constexpr uint64_t PIN_RESULT = 3072;  // the result's read-back place in the context's 4 KB pinned area
static_assert(HDR_RESULT + sizeof(rhgk::SmallResult) <= HDR_BYTES, "scratch header");
static_assert(HDR_ZERO + 3 * sizeof(unsigned long long) <= PIN_RESULT, "descriptor upload must not reach the result");
static_assert(PIN_RESULT + sizeof(rhgk::SmallResult) <= 4096, "pinned area");

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES];

// Most work units a request of n points can have: a query's windows hold at
// most n - 1 candidates in all (disjoint slabs; its own slab without
// itself), so a 64-query batch has at most 64 (n - 1), in ceil(64 (n-1) / UNIT)
// units.
static uint64_t max_units(uint64_t n) {
    const uint64_t nb = (n + 63) / 64;
    return nb * ((64 * (n - 1) + rhgd::UNIT - 1) / rhgd::UNIT);
}

rhg_status noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return RHG_EDEVICE;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return RHG_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return RHG_EDEVICE;
    }
    g_noalloc_ptr[device] = p;
    return RHG_OK;
}

}  // namespace rhgi

#define NOALLOC_HIP(expr)                                  \
    do {                                                   \
        const rhg_status _s = rhgi::hip_status(expr);      \
        if (_s != RHG_OK) return _s;                       \
    } while (0)

extern "C" rhg_status rhg_generate_noalloc(rhg_ctx *ctx, const rhg_params *params, int32_t *dev_pairs,
                                           uint64_t capacity_pairs, uint64_t *m) {
    using namespace rhgi;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !m) return RHG_EINVAL;
    if (c->shard_count != 1) return RHG_EINVAL;  // one whole graph per call
    Request rq;
    rhg_status s = request_from_params(params, rq);
    if (s != RHG_OK) return s;
    Plan pl;
    s = describe(rq, pl);
    if (s != RHG_OK) return s;
    if (pl.n > NOALLOC_N) return RHG_ERANGE;
    const SmallLayout lay = small_layout_units(pl.n, pl.B, max_units(pl.n), pl.fp32);
    if (HDR_BYTES + lay.bytes > NOALLOC_BYTES) return RHG_ERANGE;  // (not reached for n <= NOALLOC_N, B <= 32)
    if (!dev_pairs && capacity_pairs) return RHG_EINVAL;
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (c->device >= 0 && c->device < NOALLOC_MAX_DEVICES) base = (char *)g_noalloc_ptr[c->device];
    }
    if (!base || !c->pinned) return RHG_EDEVICE;
    NOALLOC_HIP(hipSetDevice(c->device));
    (void)hipGetLastError();
    const hipStream_t st = c->stream;
    // descriptor and the three zeroed words, staged in the context's pinned
    // area and uploaded with one copy
    char *pin = (char *)c->pinned;
    unsigned long long *zero_dev = (unsigned long long *)(base + HDR_ZERO);
    rhgk::SmallDesc &D = *(rhgk::SmallDesc *)pin;
    small_fill_desc(D, pl, rq, lay, base + HDR_BYTES, zero_dev + 1);
    std::memset(pin + HDR_ZERO, 0, 3 * sizeof(unsigned long long));
    NOALLOC_HIP(hipMemcpyAsync(base, pin, HDR_ZERO + 3 * sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    rhgk::SmallResult *res_dev = (rhgk::SmallResult *)(base + HDR_RESULT);
    rhgk::small_group((const rhgk::SmallDesc *)base, res_dev, 1, (int2 *)dev_pairs, zero_dev, capacity_pairs, st);
    NOALLOC_HIP(hipGetLastError());
    rhgk::SmallResult *res = (rhgk::SmallResult *)(pin + PIN_RESULT);
    NOALLOC_HIP(hipMemcpyAsync(res, res_dev, sizeof(rhgk::SmallResult), hipMemcpyDeviceToHost, st));
    NOALLOC_HIP(hipStreamSynchronize(st));
    *m = res->m;
    if (res->status == 2) return RHG_ETRUNC;  // m pairs do not fit: nothing written
    if (res->status != 0) return RHG_EDEVICE;  // scratch sized for the worst case: not expected
    return RHG_OK;
}
