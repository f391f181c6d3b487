// small.hip -- one-launch generation of many small graphs (serving path).
//
// Each workgroup generates one request of n <= SMALL_N points completely:
// sample + slab keys, a workgroup-wide stable LSD radix sort, table gather,
// slab starts and bucket index, the window plan (plan_batch), batch and unit
// scans, the count pass (count_unit), the edge scan, an atomic reservation
// of its slice of the shared output pool, and the emit pass (emit_unit).
// Phases are separated by workgroup barriers; nothing returns to the host
// between them.  The arithmetic (slab keys, windows, distance test, unit
// walk) is the same code as the multi-launch path, so a request's edge list
// is byte-identical to rhg_generate's for the same parameters.
#include "query_dev.h"

namespace rhgk {
using namespace rhgd;

constexpr int SM_THREADS = 1024;
constexpr int SM_WAVES = SM_THREADS / 64;
constexpr int SM_ITEMS = 16;
constexpr int SM_TILE = SM_THREADS * SM_ITEMS;  // keys ranked per sort step

struct SortSmem {
    uint32_t h[256];
    uint32_t off[256];
    uint32_t wcnt[SM_WAVES][256];
};
struct ScanSmem {
    uint64_t wsum[SM_WAVES];
};
union PhaseSmem {
    SortSmem sort;
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
__device__ void blk_scan_array(const T *in, uint64_t *out, uint32_t len, ScanSmem &S) {
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

// One stable LSD pass (8-bit digit at `shift`) of n keys with payload.
__device__ void blk_sort_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, uint32_t n,
                              int shift, SortSmem &S) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    if (t < 256) S.h[t] = 0;
    __syncthreads();
    for (uint32_t i = t; i < n; i += SM_THREADS) atomicAdd(&S.h[(kin[i] >> shift) & 255u], 1u);
    __syncthreads();
    if (t < 64) {  // exclusive scan of 256 counts by one wavefront, 4 per lane
        uint32_t c[4], s = 0;
        for (int k = 0; k < 4; ++k) {
            c[k] = S.h[4 * t + k];
            s += c[k];
        }
        const uint32_t ex = wave_incl_scan_u32(s) - s;
        uint32_t run = ex;
        for (int k = 0; k < 4; ++k) {
            S.off[4 * t + k] = run;
            run += c[k];
        }
    }
    __syncthreads();
    const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
    for (uint32_t base = 0; base < n; base += SM_TILE) {
        for (int d = l; d < 256; d += 64) S.wcnt[w][d] = 0;
        __syncthreads();
        const uint32_t wb = base + (uint32_t)w * (SM_ITEMS * 64);
        uint32_t k[SM_ITEMS], v[SM_ITEMS], rk[SM_ITEMS];
#pragma unroll
        for (int i = 0; i < SM_ITEMS; ++i) {
            const uint32_t p = wb + i * 64 + l;
            const bool ok = p < n;
            k[i] = ok ? kin[p] : 0u;
            v[i] = ok ? vin[p] : 0u;
            const uint32_t d = (k[i] >> shift) & 255u;
            uint64_t m = __ballot(ok);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            const uint32_t below = (uint32_t)__popcll(m & lt);
            const uint32_t prev = S.wcnt[w][d];
            rk[i] = prev + below;
            __builtin_amdgcn_wave_barrier();
            if (ok && below == 0) S.wcnt[w][d] = prev + (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        if (t < 256) {  // per digit: exclusive prefix over the wavefronts, tile total
            uint32_t run = 0;
            for (int q = 0; q < SM_WAVES; ++q) {
                const uint32_t c = S.wcnt[q][t];
                S.wcnt[q][t] = run;
                run += c;
            }
            S.h[t] = run;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SM_ITEMS; ++i) {
            const uint32_t p = wb + i * 64 + l;
            if (p < n) {
                const uint32_t d = (k[i] >> shift) & 255u;
                const uint32_t dst = S.off[d] + S.wcnt[w][d] + rk[i];
                kout[dst] = k[i];
                vout[dst] = v[i];
            }
        }
        __syncthreads();
        if (t < 256) S.off[t] += S.h[t];
        __syncthreads();
    }
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
    const int B = D.geo.B;
    if (t == 0) {
        sA.geo = D.geo;  // static part: n, B, R, K, Kw, FP32 thresholds, c, sinh/exp/reciprocal constants
        s_flag = 0;
    }
    __syncthreads();

    // ---- a0 + a2: sample, slab, key
    for (uint32_t i = t; i < n; i += SM_THREADS) {
        double th, r;
        load_point(D.src, i, th, r);
        int b = 0;
        while (b + 1 < B && sA.geo.c[b + 1] <= r) ++b;
        D.keys[i] = ((uint32_t)b << QBITS) | qang(th);
        D.vals[i] = i;
    }
    __syncthreads();

    // ---- a3: stable LSD radix sort (result back in keys/vals after an even number of passes)
    {
        const int passes = (D.key_bits + 7) / 8;
        uint32_t *ka = D.keys, *va = D.vals, *kb = D.keys2, *vb = D.vals2;
        for (int p = 0; p < passes; ++p) {
            blk_sort_pass(ka, va, kb, vb, n, 8 * p, P.sort);
            uint32_t *x = ka; ka = kb; kb = x;
            x = va; va = vb; vb = x;
        }
        if (ka != D.keys) {
            for (uint32_t i = t; i < n; i += SM_THREADS) {
                D.keys[i] = ka[i];
                D.vals[i] = va[i];
            }
        }
    }
    __syncthreads();

    // ---- slab starts, then layout (bucket bits, window bases) in the LDS copy of the geometry
    if (t <= B) {
        uint32_t lo = 0, hi = n;
        if (t == B) {
            lo = n;
        } else {
            const uint32_t x = (uint32_t)t << QBITS;
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (D.keys[mid] < x) lo = mid + 1; else hi = mid;
            }
        }
        s_bs[t] = lo;
    }
    __syncthreads();
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
        sA.geo.sh = D.sh;
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
        return;
    }
    const Geo &g = sA.geo;

    // ---- a1: table in sorted order
    for (uint32_t s = t; s < n; s += SM_THREADS) {
        const uint32_t v = D.vals[s];
        double th, r, a, b, c, d, e;
        load_point(D.src, v, th, r);
        point_table(D.src, v, th, r, a, b, c, d, e);
        D.th[s] = th;
        D.epm[s] = make_double2(a, b);
        D.sh[s] = c;
        D.hsc[s] = make_double2(d, e);
        if (D.f32) D.f32[s] = make_float4((float)a, (float)b, (float)c, 0.0f);
    }
    __syncthreads();

    // ---- slab bucket index
    for (uint32_t s = t; s < n; s += SM_THREADS) {
        const uint32_t key = D.keys[s];
        const int j = (int)(key >> QBITS);
        const int sh = g.bshift[j];
        const int64_t b = (int64_t)((key & QMASK) >> sh);
        const int64_t bp = (s == g.bs[j]) ? -1 : (int64_t)((D.keys[s - 1] & QMASK) >> sh);
        uint32_t *T = D.btab + g.bto[j];
        for (int64_t k = bp + 1; k <= b; ++k) T[k] = s;
    }
    for (int j = w; j < B; j += SM_WAVES) {
        const uint32_t nbk = 1u << (QBITS - g.bshift[j]);
        uint32_t *T = D.btab + g.bto[j];
        const uint32_t bs = g.bs[j], be = g.bs[j + 1];
        int64_t first = 0;
        if (be > bs) first = (int64_t)((D.keys[be - 1] & QMASK) >> g.bshift[j]) + 1;
        for (int64_t k = first + lane; k <= (int64_t)nbk; k += 64) T[k] = be;
    }
    __syncthreads();

    // ---- a4: window plan per batch, batch scans, units
    const uint32_t nb = (n + 63) / 64;
    for (uint32_t b = w; b < nb; b += SM_WAVES) plan_batch(g, D.win, D.bcand, D.bsoff, b, lane);
    __syncthreads();
    blk_scan_array(D.bcand, D.boff, nb, SS);
    for (uint32_t b = t; b < nb; b += SM_THREADS) D.nunits[b] = (D.bcand[b] + UNIT - 1) / UNIT;
    __syncthreads();
    blk_scan_array(D.nunits, D.uoff, nb, SS);
    const uint64_t U = D.uoff[nb];
    if (U > D.unit_cap) {
        if (t == 0) Z.status = 1;
        return;
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
        sA.win = D.win;
        sA.batch_cand = D.bcand;
        sA.batch_slab_off = D.bsoff;
        sA.unit_off = D.uoff;
        sA.unit_batch = D.ubatch;
        sA.unit_order = nullptr;
        sA.n_units = U;
        sA.unit_base = 0;
        sA.udesc = nullptr;
        sA.unit_edges = D.uedges;
        sA.bits = D.bits;
        sA.unit_edge_off = D.ueoff;
        sA.out = nullptr;
        sA.out_capacity = 0;
        sA.stats = D.stats;
        sA.exhaustive = 0;
        Z.candidates = D.boff[nb];
    }
    __syncthreads();

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

}  // namespace rhgk
