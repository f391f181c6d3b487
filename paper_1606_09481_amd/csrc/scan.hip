// scan.hip -- device-wide exclusive prefix sums built on wavefront scans, and
// the work-unit bookkeeping of the band query.
//
// Exclusive scan of len values into len+1 u64 outputs (out[len] = total):
// tiles of 4096 values (256 threads x 16); pass 1 reduces each tile, pass 2
// scans the tile sums in one workgroup, pass 3 rescans each tile and adds its
// prefix.  Inside a tile: per-thread serial sums, a 64-lane wavefront scan
// (DPP row shifts + row broadcasts for 32-bit partial sums, shuffles for
// 64-bit), then the 4 wavefront totals.
#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

template <typename T>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t *total) {
    __shared__ uint64_t wsum[SC_THREADS / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    uint64_t incl = wave_incl_scan_u64(x);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SC_THREADS / 64; ++k) {
        if (k < w) before += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

template <typename T>
__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const T *in, uint64_t len, uint64_t *tile_sum) {
    uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i)
        if (base + i < len) s += (uint64_t)in[base + i];
    uint64_t tot;
    block_excl_scan<T>(s, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// One workgroup scans the tile sums in place (exclusive) over chunks of 256.
__global__ __launch_bounds__(SC_THREADS) void k_scan_tiles(uint64_t *tile_sum, uint64_t ntiles) {
    uint64_t carry = 0;
    for (uint64_t base = 0; base < ntiles; base += SC_THREADS) {
        uint64_t i = base + threadIdx.x;
        uint64_t x = i < ntiles ? tile_sum[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan<uint64_t>(x, &tot);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(SC_THREADS) void k_scan_down(const T *in, uint64_t len, const uint64_t *tile_prefix,
                                                          uint64_t *out) {
    uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    uint64_t v[SC_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = (base + i < len) ? (uint64_t)in[base + i] : 0;
        s += v[i];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<T>(s, &tot) + tile_prefix[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        if (base + i < len) out[base + i] = run;
        run += v[i];
    }
    if (base < len && base + SC_ITEMS >= len) out[len] = run;  // the thread holding the last value
}

// Short arrays (len <= SCAN_ONE_MAX, one chunk of 16384): one workgroup of
// 1024 threads scans them in one launch (the three-launch form costs more
// than the work at this size; longer arrays keep it, since one workgroup
// walking many chunks is slower than three launches).
constexpr int S1_THREADS = 1024;
constexpr int S1_ITEMS = 16;
constexpr uint64_t SCAN_ONE_MAX = 1ull << 14;

template <typename T>
__global__ __launch_bounds__(S1_THREADS) void k_scan_one(const T *in, uint64_t len, uint64_t *out) {
    __shared__ uint64_t wsum[S1_THREADS / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    uint64_t carry = 0;
    for (uint64_t chunk = 0; chunk < len; chunk += (uint64_t)S1_THREADS * S1_ITEMS) {
        const uint64_t base = chunk + (uint64_t)threadIdx.x * S1_ITEMS;
        uint64_t v[S1_ITEMS];
        uint64_t s = 0;
#pragma unroll
        for (int i = 0; i < S1_ITEMS; ++i) {
            v[i] = (base + i < len) ? (uint64_t)in[base + i] : 0;
            s += v[i];
        }
        const uint64_t incl = wave_incl_scan_u64(s);
        if (l == 63) wsum[w] = incl;
        __syncthreads();
        uint64_t before = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < S1_THREADS / 64; ++k) {
            if (k < w) before += wsum[k];
            tot += wsum[k];
        }
        __syncthreads();
        uint64_t run = carry + before + incl - s;
#pragma unroll
        for (int i = 0; i < S1_ITEMS; ++i) {
            if (base + i < len) out[base + i] = run;
            run += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[len] = carry;
}

size_t scan_scratch_bytes(uint64_t len) {
    uint64_t ntiles = (len + SC_TILE - 1) / SC_TILE;
    return (ntiles + 1) * sizeof(uint64_t);
}

template <typename T>
static void scan_impl(const T *in, uint64_t *out, uint64_t len, void *scratch, hipStream_t st) {
    if (len == 0) {
        (void)hipMemsetAsync(out, 0, sizeof(uint64_t), st);
        return;
    }
    if (len <= SCAN_ONE_MAX) {
        hipLaunchKernelGGL(k_scan_one<T>, dim3(1), dim3(S1_THREADS), 0, st, in, len, out);
        return;
    }
    uint64_t ntiles = (len + SC_TILE - 1) / SC_TILE;
    uint64_t *ts = (uint64_t *)scratch;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)ntiles), dim3(SC_THREADS), 0, st, in, len, ts);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(SC_THREADS), 0, st, ts, ntiles);
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)ntiles), dim3(SC_THREADS), 0, st, in, len, ts, out);
}

void scan_u64(const uint64_t *in, uint64_t *out, uint64_t len, void *scratch, hipStream_t st) {
    scan_impl<uint64_t>(in, out, len, scratch, st);
}
void scan_u32(const uint32_t *in, uint64_t *out, uint64_t len, void *scratch, hipStream_t st) {
    scan_impl<uint32_t>(in, out, len, scratch, st);
}

__global__ __launch_bounds__(256) void k_units(const uint64_t *cand, uint64_t nb, uint64_t *nunits) {
    uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) nunits[b] = (cand[b] + UNIT - 1) / UNIT;
}

void units_per_batch(const uint64_t *cand, uint64_t nb, uint64_t *nunits, hipStream_t st) {
    if (nb) hipLaunchKernelGGL(k_units, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, cand, nb, nunits);
}

// Both scans of the plan's batch totals in one workgroup (short plans):
// boff = exclusive scan of the candidates per batch, uoff = exclusive scan of
// the units per batch (ceil(candidates / UNIT)).
__global__ __launch_bounds__(S1_THREADS) void k_scan_plan(const uint64_t *cand, uint64_t nb, uint64_t *boff,
                                                          uint64_t *uoff) {
    __shared__ uint64_t wsum[2][S1_THREADS / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    uint64_t carry_c = 0, carry_u = 0;
    for (uint64_t chunk = 0; chunk < nb; chunk += (uint64_t)S1_THREADS * S1_ITEMS) {
        const uint64_t base = chunk + (uint64_t)threadIdx.x * S1_ITEMS;
        uint64_t c[S1_ITEMS];
        uint64_t sc = 0, su = 0;
#pragma unroll
        for (int i = 0; i < S1_ITEMS; ++i) {
            c[i] = (base + i < nb) ? cand[base + i] : 0;
            sc += c[i];
            su += (c[i] + UNIT - 1) / UNIT;
        }
        const uint64_t ic = wave_incl_scan_u64(sc), iu = wave_incl_scan_u64(su);
        if (l == 63) {
            wsum[0][w] = ic;
            wsum[1][w] = iu;
        }
        __syncthreads();
        uint64_t bc = 0, bu = 0, tc = 0, tu = 0;
#pragma unroll
        for (int k = 0; k < S1_THREADS / 64; ++k) {
            if (k < w) {
                bc += wsum[0][k];
                bu += wsum[1][k];
            }
            tc += wsum[0][k];
            tu += wsum[1][k];
        }
        __syncthreads();
        uint64_t rc = carry_c + bc + ic - sc, ru = carry_u + bu + iu - su;
#pragma unroll
        for (int i = 0; i < S1_ITEMS; ++i) {
            if (base + i < nb) {
                boff[base + i] = rc;
                uoff[base + i] = ru;
            }
            rc += c[i];
            ru += (c[i] + UNIT - 1) / UNIT;
        }
        carry_c += tc;
        carry_u += tu;
    }
    if (threadIdx.x == 0) {
        boff[nb] = carry_c;
        uoff[nb] = carry_u;
    }
}

void plan_scans(const uint64_t *cand, uint64_t nb, uint64_t *boff, uint64_t *nunits, uint64_t *uoff, void *scratch,
                hipStream_t st) {
    if (nb && nb <= SCAN_ONE_MAX) {
        hipLaunchKernelGGL(k_scan_plan, dim3(1), dim3(S1_THREADS), 0, st, cand, nb, boff, uoff);
        return;
    }
    scan_u64(cand, boff, nb, scratch, st);
    units_per_batch(cand, nb, nunits, st);
    scan_u64(nunits, uoff, nb, scratch, st);
}

// unit_off[b] .. unit_off[b+1]-1 are the units of batch b: unit u belongs to
// the last batch b with unit_off[b] <= u.
__global__ void k_shard_cut(const uint64_t *boff, const uint64_t *uoff, uint64_t nb, uint32_t S, uint32_t k,
                            uint64_t *out) {
    if (threadIdx.x != 0) return;
    const uint64_t total = boff[nb];
    uint64_t b[2];
    for (int e = 0; e < 2; ++e) {
        const uint64_t q = (uint64_t)k + (uint64_t)e;  // cut number 0..S
        if (q == 0) { b[e] = 0; continue; }
        if (q >= S) { b[e] = nb; continue; }
        // first batch whose candidate prefix reaches ceil(total q / S), without overflow
        const uint64_t t = (total / S) * q + ((total % S) * q + S - 1) / S;
        uint64_t lo = 0, hi = nb;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (boff[mid] < t) lo = mid + 1; else hi = mid;
        }
        b[e] = lo;
    }
    out[0] = b[0];
    out[1] = b[1];
    out[2] = uoff[b[0]];
    out[3] = uoff[b[1]];
    out[4] = boff[b[0]];
    out[5] = boff[b[1]];
}

void shard_cut(const uint64_t *boff, const uint64_t *uoff, uint64_t nb, uint32_t S, uint32_t k, uint64_t *out,
               hipStream_t st) {
    hipLaunchKernelGGL(k_shard_cut, dim3(1), dim3(64), 0, st, boff, uoff, nb, S, k, out);
}

__global__ __launch_bounds__(256) void k_unit_fill(const uint64_t *unit_off, uint64_t nb, uint64_t n_units,
                                                   uint32_t *unit_batch) {
    uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    uint64_t lo = 0, hi = nb;  // search in unit_off[0..nb)
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (unit_off[mid] <= u) lo = mid; else hi = mid;
    }
    unit_batch[u] = (uint32_t)lo;
}

void unit_batch_fill(const uint64_t *unit_off, uint64_t nb, uint64_t n_units, uint32_t *unit_batch,
                     hipStream_t st) {
    if (nb && n_units)
        hipLaunchKernelGGL(k_unit_fill, dim3((unsigned)((n_units + 255) / 256)), dim3(256), 0, st, unit_off, nb,
                           n_units, unit_batch);
}

}  // namespace rhgk
