// dynamic.hip -- the dynamic model's movement step (Sec. III-C): every node
// rotates by its angular step and takes the radial step of Algorithm 2,
// reflected at the centre and at the rim.
//
// The radial step is taken on s = sinh^2(alpha r / 2) = (cosh(alpha r) - 1) / 2,
// the coordinate in which Eq. 1's radius density is uniform (on
// [0, sinh^2(alpha R / 2)]), so that a shift folded back by mirror reflection
// keeps the density (Theorem 1).  The step tau_r is given in units of
// cosh(alpha r), i.e. s moves by tau_r / 2; the sinh^2 form keeps full relative
// precision near the centre, where cosh(alpha r) - 1 would cancel.
// One thread per node; the arrays are read and written once.  The step is
// bound by its FP64 sinh and asinh, not by the 48 bytes it moves per node.
#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

__global__ __launch_bounds__(256) void k_move(uint64_t n, double alpha, double R, double S, double *theta, double *r,
                                              const double *tau_phi, double *tau_r) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // rotation, into [0, fl(2 pi)); inside it the quotient's floor is 0 (the
    // rounded quotient of t < fl(2 pi) stays below 1), so the division is skipped
    double t = theta[i] + tau_phi[i];
    if (!(t >= 0.0 && t < TWO_PI)) {
        t = t - TWO_PI * floor(t / TWO_PI);
        if (t >= TWO_PI || t < 0.0) t = 0.0;
    }
    theta[i] = t;
    // radial step: y = s + tau_r / 2 folded into [0, S]; k = floor(y / S)
    // boundary crossings, each a mirror reflection that negates the step
    const double tr = tau_r[i];
    if (tr == 0.0) return;  // a zero step leaves the radius exactly as it is
    const double h = sinh(alpha * r[i] / 2.0);
    const double y = h * h + tr / 2.0;
    double k = 0.0;  // y in [0, S): no crossing (floor of the quotient is 0, as above)
    if (!(y >= 0.0 && y < S)) k = floor(y / S);
    // parity of the integer k: |k| >= 2^53 is even (as fmod(|k|, 2) says)
    const double ak = fabs(k);
    const bool odd = ak < 9007199254740992.0 && (((unsigned long long)ak) & 1ull) != 0ull;
    double s2 = odd ? (k + 1.0) * S - y : y - k * S;
    if (s2 < 0.0) s2 = 0.0;
    if (s2 > S) s2 = S;
    if (odd) tau_r[i] = -tr;
    const double r2 = 2.0 * asinh(sqrt(s2)) / alpha;
    r[i] = r2 > R ? R : r2;
}

void move(uint64_t n, double alpha, double R, double S, double *theta, double *r, const double *tau_phi,
          double *tau_r, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_move, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, alpha, R, S, theta, r,
                       tau_phi, tau_r);
}

}  // namespace rhgk

// ---------------------------------------------------------------------------
// Graph update after a move.  The edges between two points that did not move
// are still edges; every edge at a moved point is found again by the band
// query of the moved points (Geo::moved).  The old list is compacted in its
// own order: tiles of KEEP_TILE pairs, a per-tile count, an exclusive scan of
// the counts, then each tile writes its kept pairs in order.
// ---------------------------------------------------------------------------
namespace rhgk {
using namespace rhgd;

// Moved flags as bits (1.25 MB at n = 10^7, held in L2 by the random lookups
// of the keep passes): bit s of out is moved[idx[s]] (moved[s] without idx).
// One ballot per wavefront; out holds moved_bit_words(n) words.
__global__ __launch_bounds__(256) void k_moved_bits(const uint32_t *idx, const uint8_t *moved, uint32_t n,
                                                    uint32_t *out) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = s < n && moved[idx ? idx[s] : s] != 0;
    const uint64_t b = __ballot(f);
    if ((threadIdx.x & 63) == 0) {
        out[s >> 5] = (uint32_t)b;
        out[(s >> 5) + 1] = (uint32_t)(b >> 32);
    }
}

uint64_t moved_bit_words(uint64_t n) { return (n + 255) / 256 * 8; }

void moved_bits(const uint32_t *idx, const uint8_t *moved, uint64_t n, uint32_t *out, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_moved_bits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, idx, moved, (uint32_t)n,
                       out);
}

constexpr int KEEP_ITEMS = 16;
constexpr uint64_t KEEP_TILE = 256 * KEEP_ITEMS;

// Pair k is kept iff both ends are points 0..n-1 that did not move; an end
// outside 0..n-1 sets bad (the caller raises the error flag once) and drops
// the pair, its lookups clamped into moved[].  No branch: the loads of a
// thread's pairs, then of their flags, are all in flight together.
__device__ __forceinline__ bool keep_pair(const int2 *pairs, uint64_t m, uint64_t k, const uint32_t *moved,
                                          uint32_t n, bool &bad, int2 &e) {
    const bool in = k < m;
    e = pairs[in ? k : 0];
    const uint32_t a = (uint32_t)e.x, b = (uint32_t)e.y;
    const bool ok = a < n && b < n;
    bad |= in && !ok;
    return in && ok && !bit_of(moved, min(a, n - 1u)) && !bit_of(moved, min(b, n - 1u));
}

__global__ __launch_bounds__(256) void k_keep_count(const int2 *pairs, uint64_t m, const uint32_t *moved, uint32_t n,
                                                    uint32_t *counts, uint32_t *err) {
    __shared__ uint32_t wsum[4];
    const uint64_t base = (uint64_t)blockIdx.x * KEEP_TILE;
    uint32_t c = 0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < KEEP_ITEMS; ++i) {
        int2 e;
        c += keep_pair(pairs, m, base + i * 256 + threadIdx.x, moved, n, bad, e) ? 1u : 0u;
    }
    if (bad) atomicOr(err, 1u);
    c = (uint32_t)wave_sum_u64(c);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Tile order: item i of thread t is pair base + 256 i + t; a pair's place
// among the tile's kept pairs counts those of earlier items, then of lower
// threads of the same item (per-wave ballots, then the waves before).
__global__ __launch_bounds__(256) void k_keep_write(const int2 *pairs, uint64_t m, const uint32_t *moved, uint32_t n,
                                                    const uint64_t *offs, int2 *out, uint32_t *err) {
    __shared__ uint32_t wcnt[KEEP_ITEMS][4];
    const uint64_t base = (uint64_t)blockIdx.x * KEEP_TILE;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool kp[KEEP_ITEMS];
    uint32_t below[KEEP_ITEMS];
    int2 e[KEEP_ITEMS];
    bool bad = false;
#pragma unroll
    for (int i = 0; i < KEEP_ITEMS; ++i) {
        kp[i] = keep_pair(pairs, m, base + i * 256 + threadIdx.x, moved, n, bad, e[i]);
        const uint64_t bal = __ballot(kp[i]);
        below[i] = (uint32_t)__popcll(bal & lt);
        if (lane == 0) wcnt[i][w] = (uint32_t)__popcll(bal);
    }
    if (bad) atomicOr(err, 1u);
    __syncthreads();
    uint64_t at = offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < KEEP_ITEMS; ++i) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            before += q < w ? wcnt[i][q] : 0u;
            all += wcnt[i][q];
        }
        if (kp[i]) out[at + before + below[i]] = e[i];
        at += all;
    }
}

void keep_count(const int2 *pairs, uint64_t m, const uint32_t *moved, uint64_t n, uint32_t *counts, uint32_t *err,
                hipStream_t st) {
    if (!m) return;
    hipLaunchKernelGGL(k_keep_count, dim3((unsigned)((m + KEEP_TILE - 1) / KEEP_TILE)), dim3(256), 0, st, pairs, m,
                       moved, (uint32_t)n, counts, err);
}

void keep_write(const int2 *pairs, uint64_t m, const uint32_t *moved, uint64_t n, const uint64_t *offs, int2 *out,
                uint32_t *err, hipStream_t st) {
    if (!m) return;
    hipLaunchKernelGGL(k_keep_write, dim3((unsigned)((m + KEEP_TILE - 1) / KEEP_TILE)), dim3(256), 0, st, pairs, m,
                       moved, (uint32_t)n, offs, out, err);
}

uint64_t keep_tiles(uint64_t m) { return (m + KEEP_TILE - 1) / KEEP_TILE; }

}  // namespace rhgk
