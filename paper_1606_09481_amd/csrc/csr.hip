// csr.hip -- symmetric CSR adjacency of an edge list: row v holds every w
// with (v, w) or (w, v) in the list.  Each pair (x, y) stands for two
// directed entries (row, neighbour), (x, y) then (y, x); a stable LSD radix
// sort by row (the sort of the slab keys, whose first pass reads the pairs
// and expands them) orders them, so within a row the neighbours keep the
// order of the pairs in the list; the row pointers are the first entry of
// each row in the sorted rows.
#include <algorithm>

#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

// The rows of the entries of pair e are its two ends.  An end outside 0..n-1
// raises *err (the caller stops before sorting).  The row digits of every
// sort pass are counted here, one read of the pairs: LDS histograms in 8
// copies, lane l counting into copy l mod 8, since a query's row repeats over
// runs of pairs and would otherwise put the lanes of an LDS atomic on one
// bin; one global add per bin and workgroup.
constexpr int DIR_COPIES = 8;
constexpr int DIR_UNROLL = 4;
__global__ __launch_bounds__(256) void k_directed_counts(const int2 *pairs, uint64_t m, uint32_t n, uint32_t *err,
                                                         int passes, uint32_t *counts) {
    __shared__ uint32_t h[DIR_COPIES][4][256];
    const int c = threadIdx.x & (DIR_COPIES - 1);
    for (int q = 0; q < 4; ++q)
        for (int x = 0; x < DIR_COPIES; ++x) h[x][q][threadIdx.x] = 0;
    __syncthreads();
    bool bad = false;
    // DIR_UNROLL pairs per thread in flight at once (one dependent load per
    // step would leave the read latency-bound)
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < m; e0 += DIR_UNROLL * stride) {
        int2 p[DIR_UNROLL];
#pragma unroll
        for (int u = 0; u < DIR_UNROLL; ++u) {
            const uint64_t e = e0 + (uint64_t)u * stride;
            p[u] = pairs[e < m ? e : 0];
        }
#pragma unroll
        for (int u = 0; u < DIR_UNROLL; ++u) {
            if (e0 + (uint64_t)u * stride >= m) continue;
            uint32_t a = (uint32_t)p[u].x, b = (uint32_t)p[u].y;
            if (a >= n || b >= n) {
                bad = true;
                a = b = 0u;
            }
            for (int q = 0; q < passes; ++q) {
                atomicAdd(&h[c][q][(a >> (8 * q)) & 255u], 1u);
                atomicAdd(&h[c][q][(b >> (8 * q)) & 255u], 1u);
            }
        }
    }
    if (bad) atomicOr(err, 1u);
    __syncthreads();
    for (int q = 0; q < passes; ++q) {
        uint32_t t = 0;
        for (int x = 0; x < DIR_COPIES; ++x) t += h[x][q][threadIdx.x];
        if (t) atomicAdd(&counts[q * 256 + threadIdx.x], t);
    }
}

void directed_counts(const int2 *pairs, uint64_t m, uint64_t n, uint32_t *err, int passes, uint32_t *counts,
                     hipStream_t st) {
    if (!m) return;
    const unsigned blocks = (unsigned)std::min<uint64_t>(2048, (m + 255) / 256);
    hipLaunchKernelGGL(k_directed_counts, dim3(blocks), dim3(256), 0, st, pairs, m, (uint32_t)n, err, passes, counts);
}

// row_ptr[v] = first sorted entry with row >= v, v = 0..n: entry i writes the
// rows in (row[i-1], row[i]] (with row[-1] = -1 and row[len] = n), so every
// row pointer is written once, the empty rows by the entry after them.  A
// thread takes entries 4q .. 4q+3 (one 16-byte load where all four exist and
// rows is 16-byte aligned).
__global__ __launch_bounds__(256) void k_row_ptr(const uint32_t *rows, uint64_t len, uint32_t n, uint64_t *row_ptr) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i0 = 4 * q;
    if (i0 > len) return;
    uint32_t k[4];
    if (i0 + 4 <= len && ((uintptr_t)rows & 15u) == 0) {
        const uint4 x = ((const uint4 *)rows)[q];
        k[0] = x.x;
        k[1] = x.y;
        k[2] = x.z;
        k[3] = x.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[j] = i0 + j < len ? rows[i0 + j] : n;
    }
    int64_t prev = i0 ? (int64_t)rows[i0 - 1] : -1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint64_t i = i0 + j;
        if (i > len) break;
        const int64_t cur = i < len ? (int64_t)k[j] : (int64_t)n;
        for (int64_t v = prev + 1; v <= cur; ++v) row_ptr[v] = i;
        prev = cur;
    }
}

void row_pointers(const uint32_t *rows, uint64_t len, uint64_t n, uint64_t *row_ptr, hipStream_t st) {
    const uint64_t threads = len / 4 + 1;
    hipLaunchKernelGGL(k_row_ptr, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, rows, len, (uint32_t)n,
                       row_ptr);
}

}  // namespace rhgk
