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
#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

struct BandsArg {
    int B;
    double c[MAX_BANDS + 1];
};

__global__ __launch_bounds__(256) void k_keys(Source src, BandsArg bands, uint32_t *keys, uint32_t *vals, int *err) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= src.n) return;
    double th, r;
    load_point(src, i, th, r);
    if (src.mode != SRC_SEED) {
        if (!(th >= 0.0 && th <= TWO_PI && r >= 0.0 && r <= src.R)) atomicOr(err, 1);
    }
    int b = 0;
    while (b + 1 < bands.B && bands.c[b + 1] <= r) ++b;
    keys[i] = ((uint32_t)b << QBITS) | qang(th);
    vals[i] = (uint32_t)i;
}

void keys(const Source &src, int B, const double *c_host, uint32_t *k, uint32_t *v, int *err, hipStream_t st) {
    BandsArg ba;
    ba.B = B;
    for (int j = 0; j <= B; ++j) ba.c[j] = c_host[j];
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
// LSD radix sort, 8-bit digits.  Per pass: tile histograms (digit-major),
// exclusive scan, stable scatter.  A tile is 4096 keys: 4 wavefronts x 16
// items x 64 lanes, position = tile + wave*1024 + item*64 + lane.
// ---------------------------------------------------------------------------
constexpr int S_THREADS = 256;
constexpr int S_ITEMS = 16;
constexpr int S_TILE = S_THREADS * S_ITEMS;

__global__ __launch_bounds__(S_THREADS) void k_sort_hist(const uint32_t *keys, uint32_t n, int shift,
                                                         uint64_t *hist, uint32_t ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t base = blockIdx.x * S_TILE;
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        uint32_t p = base + i * S_THREADS + threadIdx.x;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(S_THREADS) void k_sort_scatter(const uint32_t *keys, const uint32_t *vals,
                                                            uint32_t *keys_out, uint32_t *vals_out, uint32_t n,
                                                            int shift, const uint64_t *offs, uint32_t ntiles) {
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t toff[256];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int d = l; d < 256; d += 64) wcnt[w][d] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * S_TILE + w * (S_ITEMS * 64);
    const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
    uint32_t k[S_ITEMS], v[S_ITEMS], rk[S_ITEMS];
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        uint32_t p = base + i * 64 + l;
        bool ok = p < n;
        k[i] = ok ? keys[p] : 0u;
        v[i] = ok ? vals[p] : 0u;
    }
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        uint32_t p = base + i * 64 + l;
        bool ok = p < n;
        uint32_t d = (k[i] >> shift) & 255u;
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t below = (uint32_t)__popcll(m & lt);
        uint32_t prev = wcnt[w][d];
        rk[i] = prev + below;
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) wcnt[w][d] = prev + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d];
        wcnt[0][d] = 0;
        wcnt[1][d] = c0;
        wcnt[2][d] = c0 + c1;
        wcnt[3][d] = c0 + c1 + c2;
        toff[d] = (uint32_t)offs[(uint64_t)d * ntiles + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < S_ITEMS; ++i) {
        uint32_t p = base + i * 64 + l;
        if (p < n) {
            uint32_t d = (k[i] >> shift) & 255u;
            uint32_t dst = toff[d] + wcnt[w][d] + rk[i];
            keys_out[dst] = k[i];
            vals_out[dst] = v[i];
        }
    }
}

size_t sort_scratch_bytes(uint64_t n) {
    uint64_t ntiles = (n + S_TILE - 1) / S_TILE;
    uint64_t len = 256 * (ntiles ? ntiles : 1);
    return 2 * (len + 1) * sizeof(uint64_t) + scan_scratch_bytes(len) + 256;
}

void radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, void *scratch, uint64_t n,
                int bits, hipStream_t st) {
    if (n < 2) return;
    uint32_t ntiles = (uint32_t)((n + S_TILE - 1) / S_TILE);
    uint64_t len = 256ull * ntiles;
    uint64_t *hist = (uint64_t *)scratch;
    uint64_t *offs = hist + (len + 1);
    void *sscr = (void *)(offs + (len + 1));
    int passes = (bits + 7) / 8;
    uint32_t *ka = keys, *va = vals, *kb = keys_tmp, *vb = vals_tmp;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(S_THREADS), 0, st, ka, (uint32_t)n, shift, hist, ntiles);
        scan_u64(hist, offs, len, sscr, st);
        hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(S_THREADS), 0, st, ka, va, kb, vb, (uint32_t)n, shift,
                           offs, ntiles);
        uint32_t *t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    if (ka != keys) {
        (void)hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    }
}

// ---------------------------------------------------------------------------
// Gather: sorted position s takes point idx[s]; its angle and radius are
// re-sampled (seeded mode) or read, its table computed or copied.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather(Source src, const uint32_t *idx, uint32_t n, double *th,
                                                double *rr, double2 *epm, double *shv, double2 *hsc, float4 *f32) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t v = idx[s];
    double t, r, a, b, c, d, e;
    load_point(src, v, t, r);
    point_table(src, v, t, r, a, b, c, d, e);
    th[s] = t;
    rr[s] = r;
    epm[s] = make_double2(a, b);
    shv[s] = c;
    hsc[s] = make_double2(d, e);
    if (f32) f32[s] = make_float4((float)a, (float)b, (float)c, 0.0f);
}

void gather(const Source &src, const uint32_t *idx, uint64_t n, double *th, double *rr, double2 *epm, double *sh,
            double2 *hsc, float4 *f32, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, idx, (uint32_t)n, th, rr,
                       epm, sh, hsc, f32);
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
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    uint32_t key = g.keys[s];
    int j = (int)(key >> QBITS);
    int sh = g.bshift[j];
    int64_t b = (int64_t)((key & QMASK) >> sh);
    int64_t bp = (s == g.bs[j]) ? -1 : (int64_t)((g.keys[s - 1] & QMASK) >> sh);
    uint32_t *T = btab + g.bto[j];
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
