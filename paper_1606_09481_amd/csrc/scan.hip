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

// unit_off[b] .. unit_off[b+1]-1 are the units of batch b: unit u belongs to
// the last batch b with unit_off[b] <= u.
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
