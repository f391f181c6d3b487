// rhg_device.h -- device-side definitions of the gfx950 threshold RHG generator.
//
// Layout of one generation in HBM (n points, B slabs, all arrays in the
// slab-major, angle-sorted order produced by the sort):
//   keys[n]   u32  (slab << 27) | q(theta): q is a monotone 27-bit
//                  quantisation of the angle; the sort key and the search key
//   idx[n]    u32  original point index of each sorted position
//   th[n]            f64 angle
//   epm[n]           f64x2 (exp(r), exp(-r)); the distance test takes sinh r
//                    as (exp(r) - exp(-r)) / 2 from these two (no column of its own)
//   hsc[n]           f64x2 (sin(theta/2), cos(theta/2))
//   f32[n]           f32x2 (exp(r), exp(-r)) rounded once to FP32
//   btab[]    u32  per slab j, 2^bits_j + 1 bucket starts over the top bits
//                  of q (a direct-mapped index into the sorted slab)
//   win[]     uint2 per (query, slab j >= slab(query)): circular position
//                  window (start, count) in slab j, slab-major
//                  (win[winbase[j] + v], winbase[j] = sum_{j'<j} bs[j'+1])
//   per 64-query batch: candidate totals and work units; per unit: edges.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rhgd {

constexpr int MAX_BANDS = 32;
constexpr int QBITS = 27;
constexpr uint32_t QMASK = (1u << QBITS) - 1u;
constexpr uint32_t QHALF = 1u << (QBITS - 1);     // half a turn in key units
constexpr double TWO_PI = 6.283185307179586;     // fl(2 pi), the angle period of the sampler
constexpr double HALF_PI = 1.5707963267948966;
constexpr double QSCALE = 134217728.0 / TWO_PI;  // 2^27 / fl(2 pi)
constexpr int WAVE = 64;
constexpr int BATCH = 64;        // queries per batch (one wavefront)
#ifndef RHG_UNIT
#define RHG_UNIT 4096
#endif
constexpr uint32_t UNIT = RHG_UNIT;  // candidates per work unit (upper bound)
constexpr uint32_t BITMAP_WORDS = UNIT / 64 + 32;  // decision bitmap words per unit
constexpr int SOFT_LEVELS = 54;  // probability levels 2^-i, i = 0..53, of the general model
// Finer levels: U in [2^-(j+1), 2^-j), j < SOFT_FINE_J, cut into SOFT_SUB
// equal parts by the bits after its leading one (tick t = SOFT_SUB j +
// SOFT_SUB - 1 - m for part m, so the ticks' lower ends u_t fall with t).
constexpr int SOFT_SUB = 8, SOFT_FINE_J = 50, SOFT_TICKS = SOFT_SUB * SOFT_FINE_J;

enum SrcMode { SRC_SEED = 0, SRC_COORDS = 1, SRC_TABLE = 2 };

// Where the points come from.
struct Source {
    int mode;
    uint64_t n;
    uint64_t seed;
    double alpha, R;
    double sinh_half_aR;    // sinh(alpha R / 2), host libm
    const double *theta, *r;  // SRC_COORDS / SRC_TABLE (device)
    const double *table;      // SRC_TABLE: 5 x n (device)
};

// Everything the window plan and the query kernels read.
struct Geo {
    uint32_t n;
    int B;
    double R, K, Kw;          // cosh R and the widened threshold used for windows
    float klo32, khi32;       // FP32 filter thresholds (round-down / round-up of K(1 -+ mu))
    double c[MAX_BANDS + 1];  // slab boundaries
    double shc[MAX_BANDS + 1];  // sinh c_j
    double epc[MAX_BANDS + 1];  // e^{c_j}
    double emc[MAX_BANDS + 1];  // e^{-c_j}
    double ishc[MAX_BANDS + 1]; // 1 / sinh c_j (j >= 1)
    uint32_t bs[MAX_BANDS + 1]; // slab start positions, bs[B] = n
    uint64_t winbase[MAX_BANDS + 1];  // window (v, j) at winbase[j] + v
    uint32_t bto[MAX_BANDS + 1];  // bucket table offset of slab j
    int bshift[MAX_BANDS + 1];    // q >> bshift -> bucket
    const uint32_t *keys, *idx;
    const double *th;
    const double2 *epm;  // (exp(r), exp(-r)); sinh r = (exp(r) - exp(-r)) / 2
    const double2 *hsc;  // (sin(theta/2), cos(theta/2))
    const float2 *f32;   // (exp(r), exp(-r)) rounded to FP32 (FP32 filter only)
    const uint32_t *btab;
    // Update mode (re-query after a move), else null: bit s % 32 of word
    // s / 32 is set for the points that moved, in sorted order.  Only moved
    // points query, in every slab and in both directions, and a pair of two
    // moved points is taken by the one that comes first in sorted order.
    const uint32_t *moved;
    // General model at temperature T > 0 (Sec. II, Eq. 2), else t2 = 0.  K
    // and Kw then belong to the enlarged radius Rc beyond which no pair can
    // be an edge; R stays the model's radius.  t2 = 2T; pseed seeds the
    // pairs' uniforms; lev[i] (i = 1..53) bounds the cosh distance of a pair
    // whose uniform is at least 2^-i: at or above lev[i] its probability is
    // below 2^-i, so it cannot be an edge.
    double t2;
    uint64_t pseed;
    double lev[SOFT_LEVELS];
    // stab[t] (t < SOFT_TICKS): a pair at or above it has f < u_t, so no
    // edge for U >= u_t; stab[SOFT_TICKS + t]: a pair below it has f > the
    // upper end of tick t's part of U, so an edge (device memory)
    const double *stab;
};

__device__ __forceinline__ bool bit_of(const uint32_t *bits, uint32_t s) { return (bits[s >> 5] >> (s & 31u)) & 1u; }

__device__ __forceinline__ uint32_t qang(double x) {
    // min(floor(x 2^27 / fl(2 pi)), 2^27 - 1), 0 below 0 (and for NaN); clamped
    // as doubles so that it compiles without branches
    const double y = fmin(fmax(x * QSCALE, 0.0), 134217727.0);
    return (uint32_t)y;
}

// SplitMix64 (Steele, Lea, Flood 2014): k-th output of the generator seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The uniform deciding pair {lo, hi} of the general model (lo < hi, original
// indices), as its 53-bit integer k in [1, 2^53] (the uniform is k 2^-53 in
// (0, 1]): output 2^62 + lo 2^31 + hi of the points' generator, far from the
// outputs 0 .. 2n - 1 the points take.
__device__ __forceinline__ uint64_t pair_k(uint64_t seed, uint32_t lo, uint32_t hi) {
    return (splitmix64(seed, (1ull << 62) + ((uint64_t)lo << 31) + (uint64_t)hi) >> 11) + 1ull;
}

// Point i of the seeded model (Eq. 1): angle uniform on [0, 2pi), radius by
// inverting F(r) = sinh^2(alpha r/2)/sinh^2(alpha R/2).
__device__ __forceinline__ void sample_point(const Source &s, uint64_t i, double &theta, double &r) {
    uint64_t x1 = splitmix64(s.seed, 2ull * i);
    uint64_t x2 = splitmix64(s.seed, 2ull * i + 1ull);
    double u1 = (double)(x1 >> 11) * 0x1p-53;
    double u2 = (double)(x2 >> 11) * 0x1p-53;
    theta = u1 * TWO_PI;
    double rv = 2.0 * asinh(sqrt(u2) * s.sinh_half_aR) / s.alpha;
    r = rv > s.R ? s.R : rv;
}

__device__ __forceinline__ void load_point(const Source &s, uint64_t i, double &theta, double &r) {
    if (s.mode == SRC_SEED) {
        sample_point(s, i, theta, r);
    } else {
        theta = s.theta[i];
        r = s.r[i];
    }
}

// Per-point values the distance test reads: exp(r), exp(-r), sin(theta/2),
// cos(theta/2), and sinh r taken as (exp(r) - exp(-r)) / 2 from the first two
// (one rounded subtraction and an exact halving; a caller table's sinh column
// is not read).
__device__ __forceinline__ void point_table(const Source &s, uint64_t i, double theta, double r, double &ep,
                                            double &em, double &sh, double &hs, double &hc) {
    if (s.mode == SRC_TABLE) {
        ep = s.table[i];
        em = s.table[s.n + i];
        hs = s.table[3 * s.n + i];
        hc = s.table[4 * s.n + i];
    } else {
        ep = exp(r);
        em = exp(-r);
        sincos(theta * 0.5, &hs, &hc);  // one argument reduction for both
    }
    sh = 0.5 * (ep - em);
}

// ---- wavefront primitives ------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); // row_bcast:31
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
    const int l = (int)lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_bcast_u32(uint32_t x, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

}  // namespace rhgd
