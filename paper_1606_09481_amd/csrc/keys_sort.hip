// keys_sort.hip -- slab assignment, sort keys, LSD radix sort, gather of the
// per-point table into slab-major angle order, and the slab bucket index.
//
// Slabs (Sec. III-A, Eq. 4): point v is in slab i iff c_i <= r_v < c_{i+1},
// r_v = R in the last slab.  Each slab is sorted by angle (Algorithm 1, the
// per-slab sort), here as one stable radix sort of the 32-bit key
// (slab << 27 | q(theta)), q a monotone 27-bit quantisation of the angle.
// Searching windows on the same quantised keys keeps every window a superset
// of the exact angular interval, so the key resolution only affects how many
// candidates are tested, never the edge set.
#include <algorithm>
#include <cmath>

#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

struct BandsArg {
    int B;
    double c[MAX_BANDS + 1];
    // Seeded points: the sampled radius r(u) = 2 asinh(sqrt(u) sinh(alpha R/2)) / alpha
    // is increasing in the radius uniform u, so r >= c_i exactly when
    // u >= ut[i] = (sinh(alpha c_i / 2) / sinh(alpha R / 2))^2.  The slab is read
    // off ut without the transcendental; a u within UT_TOL (relative) of a
    // threshold, where rounding could disagree, takes the radius itself.
    double ut[MAX_BANDS + 1];
};
constexpr double UT_TOL = 1e-9;

__global__ __launch_bounds__(256) void k_keys(Source src, BandsArg bands, uint32_t *keys, uint32_t *vals, int *err) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= src.n) return;
    double th, r;
    int b = 0;
    if (src.mode == SRC_SEED) {
        const uint64_t x1 = splitmix64(src.seed, 2ull * i);
        const uint64_t x2 = splitmix64(src.seed, 2ull * i + 1ull);
        th = (double)(x1 >> 11) * 0x1p-53 * TWO_PI;
        const double u = (double)(x2 >> 11) * 0x1p-53;
        // the boundaries are increasing: the slab is the number at or below u;
        // the loop index is uniform, so each boundary is one scalar load
        bool near = false;
        for (int j = 1; j < bands.B; ++j) {
            b += bands.ut[j] <= u ? 1 : 0;
            near |= fabs(u - bands.ut[j]) <= UT_TOL * bands.ut[j];
        }
        if (near) {
            sample_point(src, i, th, r);
            b = 0;
            for (int j = 1; j < bands.B; ++j) b += bands.c[j] <= r ? 1 : 0;
        }
    } else {
        load_point(src, i, th, r);
        if (!(th >= 0.0 && th <= TWO_PI && r >= 0.0 && r <= src.R)) atomicOr(err, 1);
        for (int j = 1; j < bands.B; ++j) b += bands.c[j] <= r ? 1 : 0;
    }
    keys[i] = ((uint32_t)b << QBITS) | qang(th);
    vals[i] = (uint32_t)i;
}

void keys(const Source &src, int B, const double *c_host, uint32_t *k, uint32_t *v, int *err, hipStream_t st) {
    BandsArg ba;
    ba.B = B;
    for (int j = 0; j <= B; ++j) {
        ba.c[j] = c_host[j];
        const double q = std::sinh(src.alpha * c_host[j] / 2.0) / src.sinh_half_aR;
        ba.ut[j] = (src.mode == SRC_SEED && src.sinh_half_aR > 0.0) ? q * q : 0.0;
    }
    (void)hipMemsetAsync(err, 0, sizeof(int), st);
    uint64_t blocks = (src.n + 255) / 256;
    if (blocks) hipLaunchKernelGGL(k_keys, dim3((unsigned)blocks), dim3(256), 0, st, src, ba, k, v, err);
}

// Slab starts in the sorted keys: bs[j] = first position with slab >= j.
__global__ void k_band_starts(const uint32_t *keys, uint32_t n, int B, uint32_t *bs) {
    int j = threadIdx.x;
    if (j > B) return;
    uint32_t lo = 0, hi = n, x = (uint32_t)j << QBITS;
    if (j == B) {
        bs[j] = n;
        return;
    }
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < x) lo = mid + 1; else hi = mid;
    }
    bs[j] = lo;
}

void band_starts(const uint32_t *keys, uint64_t n, int B, uint32_t *bs, hipStream_t st) {
    hipLaunchKernelGGL(k_band_starts, dim3(1), dim3(64), 0, st, keys, (uint32_t)n, B, bs);
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits, one kernel per digit pass.
//
// The digit counts of every pass do not depend on the order of the keys, so
// one read of the keys gives them all (k_digit_counts).  A pass then takes
// its 6144-key tiles in ticket order (an atomic counter: a workgroup only
// ever waits for tiles whose tickets were drawn before its own, by
// workgroups already running), ranks its keys stably per digit (per-wave
// ballots), and finds, per digit, how many keys of that digit the earlier
// tiles hold by a decoupled look-back over their published per-digit
// counts: each tile publishes its own count at once (LOCAL) and its running
// total once known (TOTAL), so a look-back stops at the first TOTAL and adds
// the LOCAL counts it passes.  The keys are then staged in LDS in digit order
// and written out in runs of consecutive addresses per digit.
//
// Status words are 64-bit (2-bit flag, 62-bit count) and go through
// device-coherent atomic loads and stores.  A look-back that sees no progress
// for SORT_SPIN_LIMIT polls (never expected) raises the error flag and goes
// on, so no workgroup waits forever.
// ---------------------------------------------------------------------------
constexpr int S_THREADS = 256;
constexpr int S_ITEMS = 24;  // 6144-key tiles: fewer tiles to look back over
constexpr int S_TILE = S_THREADS * S_ITEMS;
constexpr int S_MAX_PASSES = 4;
constexpr uint64_t ST_LOCAL = 1ull << 62, ST_TOTAL = 2ull << 62, ST_VALUE = (1ull << 62) - 1;
constexpr uint32_t SORT_SPIN_LIMIT = 1u << 22;
constexpr int S_LOOK = 4;  // look-back: status words read per round trip

// Scratch layout: [tickets (S_MAX_PASSES u32) | error u32 | pad] [digit counts S_MAX_PASSES x 256 u32]
//                 [status S_MAX_PASSES x ntiles x 256 u64]
struct SortScratch {
    uint32_t *tickets;
    uint32_t *error;
    uint32_t *counts;
    uint64_t *status;
};
static SortScratch sort_scratch(void *scratch, uint32_t ntiles) {
    SortScratch x;
    char *p = (char *)scratch;
    x.tickets = (uint32_t *)p;
    x.error = x.tickets + S_MAX_PASSES;
    x.counts = (uint32_t *)(p + 256);
    x.status = (uint64_t *)(p + 256 + S_MAX_PASSES * 256 * sizeof(uint32_t));
    (void)ntiles;
    return x;
}

__global__ __launch_bounds__(S_THREADS) void k_digit_counts(const uint32_t *keys, uint32_t n, int passes,
                                                            uint32_t *counts) {
    // 16 copies of the histograms, lane l counting into copy l mod 16: keys
    // that repeat over long runs (the rows of a CSR's directed entries) then
    // put at most 4 lanes of an LDS atomic on one address, not 64
    __shared__ uint32_t h[16][S_MAX_PASSES][256];
    const int w = threadIdx.x & 15;
    for (int q = 0; q < S_MAX_PASSES; ++q)
        for (int x = 0; x < 16; ++x) h[x][q][threadIdx.x] = 0;
    __syncthreads();
    // 16-byte loads where the keys are 16-byte aligned (every buffer here is);
    // otherwise the scalar tail below takes all of them
    const uint32_t n4 = ((uintptr_t)keys & 15u) == 0 ? n / 4 : 0u;
    const uint4 *k4 = (const uint4 *)keys;
    for (uint32_t i = blockIdx.x * S_THREADS + threadIdx.x; i < n4; i += gridDim.x * S_THREADS) {
        const uint4 k = k4[i];
        for (int q = 0; q < passes; ++q) {
            atomicAdd(&h[w][q][(k.x >> (8 * q)) & 255u], 1u);
            atomicAdd(&h[w][q][(k.y >> (8 * q)) & 255u], 1u);
            atomicAdd(&h[w][q][(k.z >> (8 * q)) & 255u], 1u);
            atomicAdd(&h[w][q][(k.w >> (8 * q)) & 255u], 1u);
        }
    }
    for (uint32_t i = 4 * n4 + blockIdx.x * S_THREADS + threadIdx.x; i < n; i += gridDim.x * S_THREADS) {
        const uint32_t k = keys[i];
        for (int q = 0; q < passes; ++q) atomicAdd(&h[w][q][(k >> (8 * q)) & 255u], 1u);
    }
    __syncthreads();
    for (int q = 0; q < passes; ++q) {
        uint32_t t = 0;
        for (int x = 0; x < 16; ++x) t += h[x][q][threadIdx.x];
        if (t) atomicAdd(&counts[q * 256 + threadIdx.x], t);
    }
}

// Exclusive scan of 256 values, one per thread of the workgroup (4 wavefronts).
__device__ __forceinline__ uint32_t block_excl_256(uint32_t x, uint32_t *wtot) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint32_t incl = wave_incl_scan_u32(x);
    if (l == 63) wtot[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += wtot[k];
    __syncthreads();
    return before + incl - x;
}

// PAIRS: the input is a list of n/2 pairs (x, y) read as the n entries
// (x, y), (y, x) of each pair in turn (key, value): the directed entries of
// a CSR, expanded on the way in.
template <bool PAIRS>
__global__ __launch_bounds__(S_THREADS) void k_sort_pass(const uint32_t *keys, const uint32_t *vals,
                                                         uint32_t *keys_out, uint32_t *vals_out, uint32_t n,
                                                         int shift, const uint32_t *counts, uint64_t *status,
                                                         uint32_t *ticket, uint32_t *error) {
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t lstart[256], gbase[256], wtot[4];
    __shared__ uint32_t sk[S_TILE], sv[S_TILE];
    __shared__ uint32_t sh_tile;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (threadIdx.x == 0) sh_tile = atomicAdd(ticket, 1u);
    for (int d = l; d < 256; d += 64) wcnt[w][d] = 0;
    __syncthreads();
    const uint32_t tile = sh_tile;
    const uint32_t base = tile * S_TILE + w * (S_ITEMS * 64);
    const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
    uint32_t k[S_ITEMS], v[S_ITEMS], rk[S_ITEMS];
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        const uint32_t p = base + i * 64 + l;
        const bool ok = p < n;
        if (PAIRS) {
            // lanes 2k and 2k + 1 read the same pair: one coalesced 8-byte load each
            const uint2 q = ok ? ((const uint2 *)keys)[p >> 1] : make_uint2(0u, 0u);
            k[i] = (p & 1u) ? q.y : q.x;
            v[i] = (p & 1u) ? q.x : q.y;
        } else {
            k[i] = ok ? keys[p] : 0u;
            v[i] = ok ? vals[p] : 0u;
        }
    }
    // stable rank per wavefront and digit
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        const uint32_t p = base + i * 64 + l;
        const bool ok = p < n;
        const uint32_t d = (k[i] >> shift) & 255u;
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(m & lt);
        const uint32_t prev = wcnt[w][d];
        rk[i] = prev + below;
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) wcnt[w][d] = prev + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit (thread d): tile count, wavefront prefixes, publish, look back
    const int d = threadIdx.x;
    const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
    const uint32_t h = c0 + c1 + c2 + c3;
    uint64_t *my = status + (uint64_t)tile * 256 + d;
    __hip_atomic_store(my, (tile == 0 ? ST_TOTAL : ST_LOCAL) | (uint64_t)h, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t ls = block_excl_256(h, wtot);
    const uint32_t gd = block_excl_256(counts[d], wtot);
    uint64_t before = 0;
    if (tile > 0) {
        // S_LOOK predecessors per round trip (tile k2 and the ones below it),
        // taken in order: LOCAL counts are added, the first TOTAL ends the
        // walk, an unpublished word is read again on the next round
        int k2 = (int)tile - 1;
        uint32_t spins = 0;
        for (;;) {
            uint64_t sw[S_LOOK];
#pragma unroll
            for (int q = 0; q < S_LOOK; ++q) {
                const int t = k2 - q > 0 ? k2 - q : 0;  // tile 0 is TOTAL: the walk never passes it
                sw[q] = __hip_atomic_load(status + (uint64_t)t * 256 + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            int q = 0;
            bool done = false;
            for (; q < S_LOOK; ++q) {
                const uint64_t flag = sw[q] & ~ST_VALUE;
                if (flag == 0) break;
                before += sw[q] & ST_VALUE;
                if (flag == ST_TOTAL || k2 - q == 0) {
                    done = true;
                    break;
                }
            }
            if (done) break;
            k2 -= q;
            if (q == 0) {
                if (++spins > SORT_SPIN_LIMIT) {
                    atomicOr(error, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(my, ST_TOTAL | (before + h), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    wcnt[0][d] = 0;
    wcnt[1][d] = c0;
    wcnt[2][d] = c0 + c1;
    wcnt[3][d] = c0 + c1 + c2;
    lstart[d] = ls;
    gbase[d] = gd + (uint32_t)before;
    __syncthreads();
    // stage in digit order, then write runs of consecutive addresses
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        const uint32_t p = base + i * 64 + l;
        if (p < n) {
            const uint32_t dd = (k[i] >> shift) & 255u;
            const uint32_t lp = lstart[dd] + wcnt[w][dd] + rk[i];
            sk[lp] = k[i];
            sv[lp] = v[i];
        }
    }
    __syncthreads();
    const uint32_t valid = (n - tile * S_TILE < (uint32_t)S_TILE) ? n - tile * S_TILE : (uint32_t)S_TILE;
    for (uint32_t j = threadIdx.x; j < valid; j += S_THREADS) {
        const uint32_t key = sk[j];
        const uint32_t dd = (key >> shift) & 255u;
        const uint32_t dst = gbase[dd] + (j - lstart[dd]);
        keys_out[dst] = key;
        vals_out[dst] = sv[j];
    }
}

uint32_t *sort_error_flag(void *scratch) { return sort_scratch(scratch, 0).error; }

size_t sort_scratch_bytes(uint64_t n) {
    const uint64_t ntiles = (n + S_TILE - 1) / S_TILE;
    return 256 + S_MAX_PASSES * 256 * sizeof(uint32_t) +
           (uint64_t)S_MAX_PASSES * (ntiles ? ntiles : 1) * 256 * sizeof(uint64_t);
}

int sort_passes(int bits) { return std::min((bits + 7) / 8, S_MAX_PASSES); }

uint64_t sort_max_keys() { return (1ull << 32) - (uint64_t)S_TILE; }

void sort_prepare(void *scratch, uint64_t n, int bits, hipStream_t st) {
    const uint64_t ntiles = (n + S_TILE - 1) / S_TILE;
    const size_t status_bytes = (size_t)sort_passes(bits) * ntiles * 256 * sizeof(uint64_t);
    // tickets, error flag, digit counts and the status words of every pass start at zero
    (void)hipMemsetAsync(scratch, 0, 256 + S_MAX_PASSES * 256 * sizeof(uint32_t) + status_bytes, st);
}

uint32_t *sort_counts(void *scratch) { return sort_scratch(scratch, 0).counts; }

void radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, void *scratch, uint64_t n,
                int bits, hipStream_t st, bool copy_back) {
    if (n < 2) return;
    sort_prepare(scratch, n, bits, st);
    // few workgroups: each adds its 4 x 256 counts to the same global words
    const unsigned cblocks = (unsigned)std::min<uint64_t>(256, (n + S_THREADS * 16 - 1) / (S_THREADS * 16));
    hipLaunchKernelGGL(k_digit_counts, dim3(cblocks), dim3(S_THREADS), 0, st, keys, (uint32_t)n, sort_passes(bits),
                       sort_counts(scratch));
    sort_by_counts(keys, vals, keys_tmp, vals_tmp, scratch, n, bits, st, copy_back);
}

void sort_by_counts(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, void *scratch, uint64_t n,
                    int bits, hipStream_t st, bool copy_back) {
    if (n < 2) return;
    const uint32_t ntiles = (uint32_t)((n + S_TILE - 1) / S_TILE);
    const int passes = sort_passes(bits);
    const SortScratch x = sort_scratch(scratch, ntiles);
    uint32_t *ka = keys, *va = vals, *kb = keys_tmp, *vb = vals_tmp;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_pass<false>, dim3(ntiles), dim3(S_THREADS), 0, st, ka, va, kb, vb, (uint32_t)n, 8 * p,
                           x.counts + p * 256, x.status + (size_t)p * ntiles * 256, x.tickets + p, x.error);
        uint32_t *t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    if (ka != keys && copy_back) {
        (void)hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    }
}

void sort_pairs_by_counts(const int2 *pairs, uint64_t n, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp,
                          uint32_t *vals_tmp, void *scratch, int bits, hipStream_t st) {
    if (n == 0) return;
    const uint32_t ntiles = (uint32_t)((n + S_TILE - 1) / S_TILE);
    const int passes = sort_passes(bits);
    const SortScratch x = sort_scratch(scratch, ntiles);
    // the last pass must write (keys, vals): passes alternate from there back
    uint32_t *ka = passes % 2 ? keys : keys_tmp, *va = passes % 2 ? vals : vals_tmp;
    uint32_t *kb = passes % 2 ? keys_tmp : keys, *vb = passes % 2 ? vals_tmp : vals;
    hipLaunchKernelGGL(k_sort_pass<true>, dim3(ntiles), dim3(S_THREADS), 0, st, (const uint32_t *)pairs, nullptr, ka,
                       va, (uint32_t)n, 0, x.counts, x.status, x.tickets, x.error);
    for (int p = 1; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_pass<false>, dim3(ntiles), dim3(S_THREADS), 0, st, ka, va, kb, vb, (uint32_t)n, 8 * p,
                           x.counts + p * 256, x.status + (size_t)p * ntiles * 256, x.tickets + p, x.error);
        uint32_t *t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
}

// ---------------------------------------------------------------------------
// Gather: sorted position s takes point idx[s]; its angle and radius are
// re-sampled (seeded mode) or read, its table computed or copied.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather(Source src, const uint32_t *idx, uint32_t n, double *th,
                                                double2 *epm, double2 *hsc, float2 *f32) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t v = idx[s];
    double t, r, a, b, c, d, e;
    load_point(src, v, t, r);
    point_table(src, v, t, r, a, b, c, d, e);
    th[s] = t;
    epm[s] = make_double2(a, b);
    hsc[s] = make_double2(d, e);
    if (f32) f32[s] = make_float2((float)a, (float)b);
}

void gather(const Source &src, const uint32_t *idx, uint64_t n, double *th, double2 *epm, double2 *hsc,
            float2 *f32, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, idx, (uint32_t)n, th,
                       epm, hsc, f32);
}

__global__ __launch_bounds__(256) void k_point_values(Source src, uint32_t n, double *th, double *rr,
                                                      double *tab) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double t, r, a, b, c, d, e;
    load_point(src, v, t, r);
    point_table(src, v, t, r, a, b, c, d, e);
    if (th) th[v] = t;
    if (rr) rr[v] = r;
    if (tab) {
        tab[v] = a;
        tab[(uint64_t)n + v] = b;
        tab[2ull * n + v] = c;
        tab[3ull * n + v] = d;
        tab[4ull * n + v] = e;
    }
}

void point_values(const Source &src, uint64_t n, double *th, double *rr, double *tab, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_point_values, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, (uint32_t)n, th,
                       rr, tab);
}

// ---------------------------------------------------------------------------
// Slab bucket index: T_j[b] = first position of slab j whose bucket
// (q >> bshift_j) is >= b, for b = 0 .. 2^bits_j; T_j[2^bits_j] = end of slab.
// Every entry is written exactly once: position s writes the buckets in
// (bucket(s-1), bucket(s)]; the tail kernel writes (bucket(last), 2^bits_j].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bucket(Geo g, uint32_t *btab) {
    // per-slab layout in LDS (a point's slab is per lane: indexing the kernel
    // arguments with it would be a vector load per field)
    __shared__ uint32_t lbs[MAX_BANDS + 1], lbto[MAX_BANDS + 1];
    __shared__ int lsh[MAX_BANDS + 1];
    if (threadIdx.x <= (unsigned)g.B) {
        lbs[threadIdx.x] = g.bs[threadIdx.x];
        lbto[threadIdx.x] = g.bto[threadIdx.x];
        lsh[threadIdx.x] = g.bshift[threadIdx.x];
    }
    __syncthreads();
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    uint32_t key = g.keys[s];
    int j = (int)(key >> QBITS);
    int sh = lsh[j];
    int64_t b = (int64_t)((key & QMASK) >> sh);
    int64_t bp = (s == lbs[j]) ? -1 : (int64_t)((g.keys[s - 1] & QMASK) >> sh);
    uint32_t *T = btab + lbto[j];
    for (int64_t k = bp + 1; k <= b; ++k) T[k] = s;
}

__global__ __launch_bounds__(256) void k_bucket_tail(Geo g, uint32_t *btab) {
    int j = blockIdx.x;
    uint32_t nb = 1u << (QBITS - g.bshift[j]);
    uint32_t *T = btab + g.bto[j];
    uint32_t bs = g.bs[j], be = g.bs[j + 1];
    int64_t first = 0;
    if (be > bs) first = (int64_t)((g.keys[be - 1] & QMASK) >> g.bshift[j]) + 1;
    for (int64_t k = first + threadIdx.x; k <= (int64_t)nb; k += blockDim.x) T[k] = be;
}

void bucket_index(const Geo &g, uint32_t *btab, hipStream_t st) {
    if (g.n) hipLaunchKernelGGL(k_bucket, dim3((g.n + 255) / 256), dim3(256), 0, st, g, btab);
    hipLaunchKernelGGL(k_bucket_tail, dim3(g.B), dim3(256), 0, st, g, btab);
}

}  // namespace rhgk
