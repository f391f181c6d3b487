// runtime.cpp -- C ABI of the threshold RHG generator: parameters, contexts,
// device buffers, phase orchestration and graph handles.
//
// One generation (Algorithm 1) on the context stream:
//   keys (sample/read points, slab, sort key) -> [sync: slab sizes]
//   -> radix sort -> gather table -> slab bucket index -> window plan
//   -> batch scan -> units -> [sync: unit count] -> count -> unit scan
//   -> [sync: m] -> emit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rhg.h"
#include "rhg_internal.h"
#include "rhg_kernels.h"

using namespace rhgd;

// ---------------------------------------------------------------------------
// Parameters (host only)
// ---------------------------------------------------------------------------
namespace {

// Average-degree approximation (Sec. III-B) with zeta = 1:
//   kbar(R) = (2/pi) xi^2 n [ e^{-R/2} + e^{-alpha R} (alpha R/2 (pi/4 a^-2 - (pi-1) a^-1 + (pi-2)) - 1) ],
// xi = alpha / (alpha - 1/2), a = alpha.
double kbar_of_R(double n, double alpha, double R) {
    const double pi = M_PI;
    const double xi = alpha / (alpha - 0.5);
    const double inv = 1.0 / alpha;
    const double poly = (pi / 4.0) * inv * inv - (pi - 1.0) * inv + (pi - 2.0);
    return (2.0 / pi) * xi * xi * n * (std::exp(-R / 2.0) + std::exp(-alpha * R) * (alpha * R / 2.0 * poly - 1.0));
}

}  // namespace

extern "C" rhg_status rhg_target_radius(uint64_t n, double alpha, double kbar, double *R_out) {
    if (!R_out || n < 2 || !std::isfinite(alpha) || !std::isfinite(kbar) || !(alpha > 0.5) || !(kbar > 0.0))
        return RHG_EINVAL;
    const double nd = (double)n;
    // Walk left from a radius where the approximation is below kbar; the
    // function rises towards its single maximum, so the first point at or
    // above kbar brackets the root of the decreasing branch.
    const double xi = alpha / (alpha - 0.5);
    double hi = std::max(1.0, 2.0 * std::log((2.0 / M_PI) * xi * xi * nd / kbar) + 4.0);
    for (int k = 0; k < 4096 && kbar_of_R(nd, alpha, hi) >= kbar; ++k) hi += 1.0;
    if (kbar_of_R(nd, alpha, hi) >= kbar) return RHG_EINVAL;
    double lo = hi, prev = kbar_of_R(nd, alpha, hi);
    for (;;) {
        double x = lo - 0.125;
        if (x <= 0.0) return RHG_EINVAL;
        double f = kbar_of_R(nd, alpha, x);
        if (f >= kbar) { lo = x; break; }
        if (f < prev) return RHG_EINVAL;  // past the maximum without reaching kbar
        prev = f;
        hi = x;
        lo = x;
    }
    // bisection to adjacent doubles: f(lo) >= kbar > f(hi)
    for (int it = 0; it < 2000; ++it) {
        double mid = lo + (hi - lo) / 2.0;
        if (mid <= lo || mid >= hi) break;
        if (kbar_of_R(nd, alpha, mid) >= kbar) lo = mid; else hi = mid;
    }
    *R_out = 0.5 * (lo + hi);
    return RHG_OK;
}

static bool make_boundaries(double R, int B, double p, double *c) {
    if (!(R > 0.0) || !std::isfinite(R) || B < 1 || B > MAX_BANDS || !(p > 0.0) || !(p <= 1.0)) return false;
    c[0] = 0.0;
    if (p == 1.0) {
        for (int i = 1; i < B; ++i) c[i] = R * i / B;
    } else {
        // c_i = c_1 (1 - p^i) / (1 - p) with c_1 = (1 - p) R / (1 - p^B): c_i = R (1 - p^i)/(1 - p^B)
        const double denom = 1.0 - std::pow(p, (double)B);
        for (int i = 1; i < B; ++i) c[i] = R * (1.0 - std::pow(p, (double)i)) / denom;
    }
    c[B] = R;
    for (int i = 0; i < B; ++i)
        if (!(c[i + 1] > c[i])) return false;
    return true;
}

// Default slab count: ceil(log2 n) - 8.  The edge set does not depend on the
// slabs; their number trades windows (plan work, slab segments per work
// unit) against candidates (count and emit work).  The paper's ceil(log2 n)
// is tuned for one thread per query on a CPU; on this GPU the step is
// fastest about 8 slabs lower (measured at n = 10^6 .. 10^7, alpha 0.55 ..
// 1.5: 4-10% faster than ceil(log2 n)).
static int default_bands(uint64_t n) {
    int b = 0;
    while (b < 63 && (1ull << b) < n) ++b;
    return std::max(1, std::min(b - 8, MAX_BANDS));
}

extern "C" rhg_status rhg_band_boundaries(double R, uint32_t num_bands, double band_ratio, double *c_out) {
    if (!c_out) return RHG_EINVAL;
    int B = num_bands ? (int)num_bands : 0;
    double p = band_ratio > 0.0 ? band_ratio : 0.9;
    if (B < 1 || B > MAX_BANDS) return RHG_EINVAL;
    return make_boundaries(R, B, p, c_out) ? RHG_OK : RHG_EINVAL;
}

extern "C" const char *rhg_status_str(rhg_status s) {
    switch (s) {
        case RHG_OK: return "ok";
        case RHG_EINVAL: return "invalid argument";
        case RHG_ENOMEM: return "out of memory";
        case RHG_EDEVICE: return "HIP device error";
        case RHG_ERANGE: return "size out of range";
        case RHG_ETRUNC: return "buffer too small";
        case RHG_EBUSY: return "not ready";
    }
    return "unknown status";
}

extern "C" const char *rhg_version(void) { return "rhg-gfx950 0.1.0"; }

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
using namespace rhgi;

void *Ctx::dev_alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (alloc_fn) return alloc_fn(bytes, alloc_user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Ctx::dev_free(void *p) {
    if (!p) return;
    if (free_fn) free_fn(p, alloc_user);
    else (void)hipFree(p);
}

void *Ctx::buf(int slot, size_t bytes) {
    SlotBuf &s = slots[slot];
    if (s.cap >= bytes && s.ptr) return s.ptr;
    if (s.ptr) dev_free(s.ptr);
    s.ptr = nullptr;
    s.cap = 0;
    size_t want = std::max<size_t>(bytes + bytes / 8, 4096);
    s.ptr = dev_alloc(want);
    if (!s.ptr) return nullptr;
    s.cap = want;
    return s.ptr;
}

Ctx::~Ctx() {
    for (auto &s : slots) dev_free(s.ptr);
    for (auto &e : ev) if (e) (void)hipEventDestroy(e);
    if (pinned) (void)hipHostFree(pinned);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

extern "C" rhg_status rhg_ctx_create(int device, void *hip_stream, rhg_ctx **out) {
    if (!out) return RHG_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return count == 0 ? RHG_EDEVICE : RHG_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) return RHG_EDEVICE;
    // the device address of this device's fixed scratch (rhg_generate_noalloc)
    if (noalloc_setup(device) != RHG_OK) return RHG_EDEVICE;
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return RHG_ENOMEM;
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        // a blocking stream: ordered with work on the device's null stream (e.g.
        // PyTorch's default stream), so caller arrays written there are ready
        if (hipStreamCreateWithFlags(&c->stream, hipStreamDefault) != hipSuccess) {
            delete c;
            return RHG_EDEVICE;
        }
        c->own_stream = true;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return RHG_EDEVICE;
        }
    if (hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        delete c;
        return RHG_ENOMEM;
    }
    *out = reinterpret_cast<rhg_ctx *>(c);
    return RHG_OK;
}

extern "C" rhg_status rhg_ctx_set_allocator(rhg_ctx *ctx, void *(*alloc)(size_t, void *),
                                            void (*free_fn)(void *, void *), void *user) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || (alloc && !free_fn)) return RHG_EINVAL;
    for (auto &s : c->slots) {
        c->dev_free(s.ptr);
        s.ptr = nullptr;
        s.cap = 0;
    }
    c->alloc_fn = alloc;
    c->free_fn = alloc ? free_fn : nullptr;
    c->alloc_user = alloc ? user : nullptr;
    return RHG_OK;
}

extern "C" rhg_status rhg_ctx_set_option(rhg_ctx *ctx, int option, int64_t value) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return RHG_EINVAL;
    if (option == RHG_OPT_FP32_EXHAUSTIVE) {
        c->exhaustive = value ? 1 : 0;
        return RHG_OK;
    }
    if (option == RHG_OPT_LITERAL_ABLATION) {
        c->ablation = value ? 1 : 0;
        return RHG_OK;
    }
    if (option == RHG_OPT_SHARD_COUNT) {
        if (value < 1 || value > 65536) return RHG_EINVAL;
        c->shard_count = (uint32_t)value;
        return RHG_OK;
    }
    if (option == RHG_OPT_SHARD_INDEX) {
        if (value < 0 || value >= 65536) return RHG_EINVAL;
        c->shard_index = (uint32_t)value;
        return RHG_OK;
    }
    return RHG_EINVAL;
}

extern "C" void rhg_ctx_destroy(rhg_ctx *ctx) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

// ---------------------------------------------------------------------------
// Generation
// ---------------------------------------------------------------------------
namespace rhgi {

rhg_status hip_status(hipError_t e) {
    if (e == hipSuccess) return RHG_OK;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? RHG_ENOMEM : RHG_EDEVICE;
}

#define RHG_TRY(expr)                      \
    do {                                   \
        rhg_status _s = (expr);            \
        if (_s != RHG_OK) return _s;       \
    } while (0)
#define RHG_HIP(expr) RHG_TRY(hip_status(expr))
#define RHG_BUF(var, type, slot, count)                                  \
    type *var = (type *)c->buf((slot), sizeof(type) * (size_t)(count));  \
    if (!var) return RHG_ENOMEM

// Largest disk radius accepted.  The distance test forms (2 sinh r_u) sinh r_w,
// about e^{r_u + r_w} / 2, which must stay finite for every pair of points
// in the disk: at r_u = r_w = R that needs e^{2R} < 2 DBL_MAX, R < 355.23.
// Past it a pair of coincident points on the rim would give inf * 0 = NaN
// and be declared non-adjacent.  354 leaves a factor e^{2.4} of headroom for
// the rounding of sinh; every table entry (e^{+-r}, sinh r) and cosh R are
// then finite as well.
bool radius_in_domain(double R) { return R > 0.0 && R <= R_MAX; }

int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

// Validates and fills the generation description.
// n < 2^31: positions and original indices are 32-bit (int32 output).
constexpr uint64_t N_MAX = 1ull << 31;

rhg_status describe(const Request &rq, Plan &pl) {
    if (rq.n < 2 || rq.n >= N_MAX) return rq.n < 2 ? RHG_EINVAL : RHG_ERANGE;
    if (!radius_in_domain(rq.R)) return RHG_EINVAL;
    if (rq.precision != RHG_FP64 && rq.precision != RHG_FP32_RECHECK) return RHG_EINVAL;
    if (rq.precision == RHG_FP32_RECHECK && rq.R > 43.0) return RHG_EINVAL;
    if (rq.mode == SRC_SEED && !(rq.alpha > 0.0 && std::isfinite(rq.alpha))) return RHG_EINVAL;
    // the sampler inverts Eq. 1's radius law through sinh(alpha R / 2)
    if (rq.mode == SRC_SEED && !std::isfinite(std::sinh(rq.alpha * rq.R / 2.0))) return RHG_EINVAL;
    // the general model: 0 < T < 1, FP64, the enlarged radius in the domain
    if (std::isnan(rq.T) || rq.T < 0.0 || rq.T >= 1.0) return RHG_EINVAL;
    if (rq.T > 0.0 && (rq.precision != RHG_FP64 || rq.moved || !radius_in_domain(rq.R + 2.0 * SOFT_CUT * rq.T)))
        return RHG_EINVAL;
    int B = rq.num_bands ? (int)rq.num_bands : default_bands(rq.n);
    double p = rq.band_ratio > 0.0 ? rq.band_ratio : 0.9;
    if (B < 1 || B > MAX_BANDS) return RHG_EINVAL;
    pl.B = B;
    pl.p = p;
    if (!make_boundaries(rq.R, B, p, pl.c)) return RHG_EINVAL;
    pl.n = rq.n;
    pl.R = rq.R;
    pl.K = std::cosh(rq.R);
    pl.fp32 = rq.precision == RHG_FP32_RECHECK;
    pl.T = rq.T;
    pl.pseed = rq.seed;
    pl.Kc = rq.T > 0.0 ? std::cosh(rq.R + 2.0 * SOFT_CUT * rq.T) : 0.0;
    return RHG_OK;
}

static float round_down_f32(double x) {
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, 0.0f);
    return f;
}
static float round_up_f32(double x) {
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

// Geometry that does not depend on the points: slab boundaries and their
// sinh / exp / reciprocal constants, cosh R, the widened window threshold and
// the FP32 filter thresholds.
void geo_static(const Plan &pl, Geo &g) {
    std::memset(&g, 0, sizeof(Geo));
    g.n = (uint32_t)pl.n;
    g.B = pl.B;
    g.R = pl.R;
    g.K = pl.K;
    g.Kw = pl.K * (1.0 + 0x1p-30);
    g.klo32 = round_down_f32(pl.K * (1.0 - 0x1p-20));
    g.khi32 = round_up_f32(pl.K * (1.0 + 0x1p-20));
    if (pl.T > 0.0) {
        // general model: windows and the first test for the enlarged radius;
        // lev[i] = cosh(R + 2T ln(2^i - 1)) raised by 2^-30, where f = 2^-i:
        // a pair at or beyond it has f < 2^-i (the margin moves f by a
        // relative 2^-31 / T at least, far above the rounding of f)
        g.K = pl.Kc;
        g.Kw = pl.Kc * (1.0 + 0x1p-30);
        g.t2 = 2.0 * pl.T;
        g.pseed = pl.pseed;
        g.lev[0] = INFINITY;
        for (int i = 1; i < SOFT_LEVELS; ++i)
            g.lev[i] = std::cosh(pl.R + 2.0 * pl.T * std::log(std::ldexp(1.0, i) - 1.0)) * (1.0 + 0x1p-30);
    }
    for (int j = 0; j <= pl.B; ++j) {
        g.c[j] = pl.c[j];
        g.shc[j] = std::sinh(pl.c[j]);
        g.epc[j] = std::exp(pl.c[j]);
        g.emc[j] = std::exp(-pl.c[j]);
        g.ishc[j] = j > 0 ? 1.0 / g.shc[j] : 0.0;
    }
}

// The general model's finer sure-decision thresholds (Geo::stab), in the
// levels' terms: f(V) <= u iff acosh V >= x(u) = R + 2T ln(1/u - 1).  The
// same 2^-30 margin, on the side that makes each shortcut safe: a rejection
// threshold raised, an acceptance threshold lowered.  Where x(u) is within
// 1e-6 of 0 neither shortcut is taken (the exact test decides); below it
// every pair has f < u (always reject); an acceptance needs x(u) > 0.
static void soft_table(const Plan &pl, std::vector<double> &tab) {
    tab.assign(2 * SOFT_TICKS, 0.0);
    auto x_of = [&](double u) { return pl.R + 2.0 * pl.T * std::log(1.0 / u - 1.0); };
    auto u_of = [](int t) {
        const int j = t / SOFT_SUB, m = SOFT_SUB - 1 - t % SOFT_SUB;
        return std::ldexp(1.0 + (double)m / SOFT_SUB, -(j + 1));
    };
    for (int t = 0; t < SOFT_TICKS; ++t) {
        const double xr = x_of(u_of(t));
        tab[t] = xr < -1e-6 ? -INFINITY : (xr <= 1e-6 ? INFINITY : std::cosh(xr) * (1.0 + 0x1p-30));
        const double uh = t == 0 ? 1.0 : u_of(t - 1);  // upper end of tick t's part
        const double xa = uh < 1.0 ? x_of(uh) : -1.0;
        tab[SOFT_TICKS + t] = xa <= 1e-6 ? -INFINITY : std::cosh(xa) * (1.0 - 0x1p-30);
    }
}

int key_bits_for(int B) { return QBITS + std::max(1, ceil_log2((uint64_t)B)); }

constexpr uint64_t UNIT_ORDER_MIN = 8192;

rhg_status run_count(Ctx *c, const Request &rq, Plan &pl) {
    RHG_HIP(hipSetDevice(c->device));
    (void)hipGetLastError();  // launch errors checked below are this call's own
    const hipStream_t st = c->stream;
    const uint64_t n = pl.n;
    const int B = pl.B;
    const uint32_t S = c->shard_count, K = c->shard_index;
    if (K >= S) return RHG_EINVAL;  // query share out of range
    c->generation++;
    pl.generation = c->generation;

    Source src{};
    src.mode = rq.mode;
    src.n = n;
    src.seed = rq.seed;
    src.alpha = rq.alpha;
    src.R = rq.R;
    src.sinh_half_aR = std::sinh(rq.alpha * rq.R / 2.0);
    src.theta = rq.theta;
    src.r = rq.r;
    src.table = rq.table;

    RHG_BUF(keys, uint32_t, S_KEYS, n);
    RHG_BUF(vals, uint32_t, S_VALS, n);
    RHG_BUF(keys2, uint32_t, S_KEYS2, n);
    RHG_BUF(vals2, uint32_t, S_VALS2, n);
    RHG_BUF(hist, uint32_t, S_HIST, MAX_BANDS + 8);
    uint32_t *bstart = hist;
    int *err = (int *)(hist + MAX_BANDS + 4);

    RHG_HIP(hipEventRecord(c->ev[EV_KEYS0], st));
    rhgk::keys(src, B, pl.c, keys, vals, err, st);
    RHG_HIP(hipEventRecord(c->ev[EV_KEYS1], st));

    // sort, then the slab starts from the sorted keys
    const int key_bits = key_bits_for(B);
    void *sort_scr = c->buf(S_SORTSCR, rhgk::sort_scratch_bytes(n));
    if (!sort_scr) return RHG_ENOMEM;
    RHG_HIP(hipEventRecord(c->ev[EV_SORT0], st));
    rhgk::radix_sort(keys, vals, keys2, vals2, sort_scr, n, key_bits, st);
    rhgk::band_starts(keys, n, B, bstart, st);
    RHG_HIP(hipEventRecord(c->ev[EV_SORT1], st));

    // table in sorted order (needs no layout)
    RHG_BUF(th, double, S_TH, n);
    RHG_BUF(epm, double2, S_EP, n);
    RHG_BUF(hsc, double2, S_HS, n);
    float2 *f32 = nullptr;
    if (pl.fp32) {
        f32 = (float2 *)c->buf(S_EP32, sizeof(float2) * n);
        if (!f32) return RHG_ENOMEM;
    }
    rhgk::gather(src, vals, n, th, epm, hsc, f32, st);
    const bool update = rq.moved != nullptr;
    uint32_t *msorted = nullptr, *morig = nullptr;
    if (update) {
        if (S > 1) return RHG_EINVAL;  // an update is one whole graph
        msorted = (uint32_t *)c->buf(S_MOVED, sizeof(uint32_t) * rhgk::moved_bit_words(n));
        morig = (uint32_t *)c->buf(S_MOVEDO, sizeof(uint32_t) * rhgk::moved_bit_words(n));
        if (!msorted || !morig) return RHG_ENOMEM;
        rhgk::moved_bits(vals, rq.moved, n, msorted, st);
        rhgk::moved_bits(nullptr, rq.moved, n, morig, st);
    }
    RHG_HIP(hipEventRecord(c->ev[EV_TABLE1], st));

    // slab sizes -> layout of windows and bucket index
    RHG_HIP(hipMemcpyAsync(c->pinned, hist, sizeof(uint32_t) * (MAX_BANDS + 8), hipMemcpyDeviceToHost, st));
    uint32_t *sort_err = (uint32_t *)((char *)c->pinned + 1024);
    RHG_HIP(hipMemcpyAsync(sort_err, rhgk::sort_error_flag(sort_scr), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    RHG_HIP(hipStreamSynchronize(st));
    const uint32_t *hh = (const uint32_t *)c->pinned;
    if (hh[MAX_BANDS + 4] != 0) return RHG_EINVAL;  // coordinates out of range
    if (*sort_err != 0) return RHG_EDEVICE;         // a sort pass gave up waiting (never expected)

    Geo &g = pl.geo;
    geo_static(pl, g);
    uint64_t wins = 0, btab_len = 0;
    if (hh[0] != 0 || hh[B] != n) return RHG_EDEVICE;
    for (int j = 0; j < B; ++j) {
        if (hh[j + 1] < hh[j]) return RHG_EDEVICE;
        g.bs[j] = hh[j];
        g.winbase[j] = wins;
        const uint32_t nj = hh[j + 1] - hh[j];
        // queries of slabs <= j each have a window in slab j (in an update
        // every query has one in every slab)
        wins += update ? n : hh[j + 1];
        int bits = std::max(0, std::min(24, ceil_log2(nj) - 1));
        g.bshift[j] = QBITS - bits;
        g.bto[j] = (uint32_t)btab_len;
        btab_len += (1ull << bits) + 1;
    }
    g.bs[B] = (uint32_t)n;
    g.winbase[B] = wins;
    pl.windows = wins;

    RHG_BUF(btab, uint32_t, S_BTAB, btab_len);
    g.keys = keys;
    g.idx = vals;
    g.th = th;
    g.epm = epm;
    g.hsc = hsc;
    g.f32 = f32;
    g.btab = btab;
    g.moved = msorted;
    if (pl.T > 0.0) {  // the general model's finer thresholds (kept on the host until the copy is done)
        soft_table(pl, c->stab_host);
        RHG_BUF(stab, double, S_SOFTTAB, 2 * SOFT_TICKS);
        RHG_HIP(hipMemcpyAsync(stab, c->stab_host.data(), sizeof(double) * 2 * SOFT_TICKS, hipMemcpyHostToDevice, st));
        g.stab = stab;
    }
    RHG_HIP(hipEventRecord(c->ev[EV_PLAN0], st));
    rhgk::bucket_index(g, btab, st);

    // window plan and work units
    const uint64_t nb = (n + BATCH - 1) / BATCH;
    RHG_BUF(win, uint2, S_WIN, std::max<uint64_t>(wins, 1));
    RHG_BUF(bcand, uint64_t, S_BCAND, nb);
    RHG_BUF(bsoff, uint64_t, S_BANDSTART, nb * (uint64_t)(B + 1));
    RHG_BUF(boff, uint64_t, S_BOFF, nb + 1);
    RHG_BUF(nunits, uint64_t, S_NUNITS, nb);
    RHG_BUF(uoff, uint64_t, S_UOFF, nb + 1);
    void *scan_scr = c->buf(S_SCANSCR, rhgk::scan_scratch_bytes(std::max<uint64_t>(nb, 1ull << 22)));
    if (!scan_scr) return RHG_ENOMEM;
    rhgk::plan(g, win, bcand, bsoff, st);
    rhgk::plan_scans(bcand, nb, boff, nunits, uoff, scan_scr, st);
    // a query share: its batch range, cut on the candidate prefix (whole table planned)
    uint64_t *shard = nullptr;
    if (S > 1) {
        shard = (uint64_t *)c->buf(S_SHARD, 8 * sizeof(uint64_t));
        if (!shard) return RHG_ENOMEM;
        rhgk::shard_cut(boff, uoff, nb, S, K, shard, st);
    }
    RHG_HIP(hipEventRecord(c->ev[EV_PLAN1], st));
    uint64_t *pin = (uint64_t *)c->pinned;
    RHG_HIP(hipMemcpyAsync(pin + 0, boff + nb, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    RHG_HIP(hipMemcpyAsync(pin + 1, uoff + nb, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    if (shard) RHG_HIP(hipMemcpyAsync(pin + 16, shard, 6 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    RHG_HIP(hipStreamSynchronize(st));
    const uint64_t Uall = pin[1];
    if (Uall >= (1ull << 31)) return RHG_ERANGE;
    uint64_t u0 = 0, U = Uall;  // units of this share: global ids u0 .. u0 + U - 1
    pl.candidates = pin[0];
    if (shard) {
        if (pin[18] > pin[19] || pin[19] > Uall || pin[20] > pin[21]) return RHG_EDEVICE;
        u0 = pin[18];
        U = pin[19] - pin[18];
        pl.candidates = pin[21] - pin[20];
    }
    pl.n_units = U;

    // ubatch is indexed by global unit id (a share touches its range only);
    // uedges and ueoff by the share's execution slot 0 .. U-1
    RHG_BUF(ubatch, uint32_t, S_UBATCH, std::max<uint64_t>(Uall, 1));
    RHG_BUF(uedges, uint32_t, S_UEDGES, std::max<uint64_t>(Uall, 1));
    RHG_BUF(ueoff, uint64_t, S_UEOFF, Uall + 1);
    RHG_BUF(stats, unsigned long long, S_STATS, 4);
    RHG_BUF(bits, unsigned long long, S_BITS, std::max<uint64_t>(Uall, 1) * BITMAP_WORDS + 8);  // + the emit's read-ahead
    void *scan2 = c->buf(S_SCANSCR2, rhgk::scan_scratch_bytes(std::max<uint64_t>(U, 1)));
    if (!scan2) return RHG_ENOMEM;
    RHG_HIP(hipEventRecord(c->ev[EV_COUNT0], st));  // count phase: unit bookkeeping + order + count
    rhgk::unit_batch_fill(uoff, nb, Uall, ubatch, st);
    RHG_HIP(hipMemsetAsync(stats, 0, sizeof(unsigned long long) * 4, st));

    rhgk::QueryArgs &qa = pl.qa;
    std::memset(&qa, 0, sizeof(qa));
    qa.geo = g;
    qa.win = win;
    qa.batch_cand = bcand;
    qa.batch_slab_off = bsoff;
    qa.unit_off = uoff;
    qa.unit_batch = ubatch;
    qa.n_units = U;
    qa.unit_base = u0;
    qa.unit_edges = uedges;
    qa.bits = bits;
    qa.unit_edge_off = ueoff;
    qa.stats = stats;
    qa.exhaustive = (c->ablation && pl.fp32 && !update) ? 2 : c->exhaustive;
    RHG_BUF(ukey, uint32_t, S_UKEY, std::max<uint64_t>(U, 1));
    RHG_BUF(uorder, uint32_t, S_UORDER, std::max<uint64_t>(U, 1));
    RHG_BUF(ukey2, uint32_t, S_UKEY2, std::max<uint64_t>(U, 1));
    RHG_BUF(uorder2, uint32_t, S_UORDER2, std::max<uint64_t>(U, 1));
    void *usort = c->buf(S_SORTSCR2, rhgk::sort_scratch_bytes(std::max<uint64_t>(U, 1)));
    if (!usort) return RHG_ENOMEM;
    // sector order of the units (for L2 reuse across a large plan; below
    // UNIT_ORDER_MIN units the tables fit in cache and the launches cost more)
    qa.unit_order = nullptr;
    qa.udesc = nullptr;
    if (U >= UNIT_ORDER_MIN) {
        // the unit-key pass also leaves each unit's walk descriptor for the count pass
        qa.udesc = (rhgk::UnitDesc *)c->buf(S_UDESC, sizeof(rhgk::UnitDesc) * U);
        if (!qa.udesc) return RHG_ENOMEM;
        rhgk::unit_order(qa, ukey, uorder, ukey2, uorder2, usort, st);
        qa.unit_order = uorder;
    }
    RHG_HIP(hipEventRecord(c->ev[EV_QCOUNT0], st));
    rhgk::query_count(qa, pl.fp32, st);
    RHG_HIP(hipEventRecord(c->ev[EV_COUNT1], st));
    // edge offsets of the share's units, from 0 at its first unit
    rhgk::scan_u32(uedges, ueoff, U, scan2, st);
    // an update keeps the old pairs whose ends both stayed: per-tile counts and offsets
    pl.old_pairs = nullptr;
    pl.keep_off = nullptr;
    pl.m_old = pl.m_keep = 0;
    pin[6] = 0;
    uint32_t *keep_err_host = (uint32_t *)((char *)c->pinned + 1032);
    *keep_err_host = 0;
    if (update && rq.m_old) {
        const uint64_t tiles = rhgk::keep_tiles(rq.m_old);
        RHG_BUF(kcnt, uint32_t, S_KEEPC, tiles);
        RHG_BUF(koff, uint64_t, S_KEEPO, tiles + 1);
        RHG_BUF(kerr, uint32_t, S_KEEPERR, 1);
        void *scan3 = c->buf(S_SCANSCR3, rhgk::scan_scratch_bytes(tiles));
        if (!scan3) return RHG_ENOMEM;
        RHG_HIP(hipMemsetAsync(kerr, 0, sizeof(uint32_t), st));
        rhgk::keep_count((const int2 *)rq.old_pairs, rq.m_old, morig, n, kcnt, kerr, st);
        rhgk::scan_u32(kcnt, koff, tiles, scan3, st);
        RHG_HIP(hipMemcpyAsync(pin + 6, koff + tiles, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        RHG_HIP(hipMemcpyAsync(keep_err_host, kerr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        pl.old_pairs = (const int2 *)rq.old_pairs;
        pl.moved_orig = morig;
        pl.m_old = rq.m_old;
        pl.keep_off = koff;
        pl.keep_err = kerr;
    }
    RHG_HIP(hipEventRecord(c->ev[EV_SCAN1], st));
    RHG_HIP(hipMemcpyAsync(pin + 2, ueoff + U, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    // (pinned words: 0-2 totals, 6 kept pairs, 16-21 the share's cut, 24-27 the counters)
    RHG_HIP(hipMemcpyAsync(pin + 24, stats, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    uint32_t *usort_err = (uint32_t *)((char *)c->pinned + 1028);
    *usort_err = 0;
    if (qa.unit_order)
        RHG_HIP(hipMemcpyAsync(usort_err, rhgk::sort_error_flag(usort), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    RHG_HIP(hipStreamSynchronize(st));
    RHG_HIP(hipGetLastError());
    if (*usort_err != 0) return RHG_EDEVICE;
    if (*keep_err_host != 0) return RHG_EINVAL;  // an old pair names a point outside 0..n-1
    pl.m_keep = pin[6];
    pl.m = pin[2] + pl.m_keep;
    pl.rechecks = pin[24];
    pl.disagreements = pin[25];
    pl.lit_undecided = qa.exhaustive == 2 ? pin[26] : 0;
    pl.lit_wrong = qa.exhaustive == 2 ? pin[27] : 0;
    return RHG_OK;
}

rhg_status run_emit(Ctx *c, Plan &pl, int2 *out) {
    if (pl.generation != c->generation) return RHG_EINVAL;  // context reused since the count
    RHG_HIP(hipSetDevice(c->device));
    (void)hipGetLastError();
    const hipStream_t st = c->stream;
    // an update writes the kept old pairs first, the pairs at moved points after them
    pl.qa.out = out + pl.m_keep;
    pl.qa.out_capacity = pl.m - pl.m_keep;
    RHG_HIP(hipEventRecord(c->ev[EV_EMIT0], st));
    if (pl.keep_off)
        rhgk::keep_write(pl.old_pairs, pl.m_old, pl.moved_orig, pl.n, pl.keep_off, out, pl.keep_err, st);
    rhgk::query_emit(pl.qa, pl.fp32, st);
    RHG_HIP(hipEventRecord(c->ev[EV_EMIT1], st));
    RHG_HIP(hipStreamSynchronize(st));
    RHG_HIP(hipGetLastError());
    // phase device times: each pair of events brackets only that phase's launches
    const int pairs[7][2] = {{EV_KEYS0, EV_KEYS1}, {EV_SORT0, EV_SORT1}, {EV_SORT1, EV_TABLE1},
                             {EV_PLAN0, EV_PLAN1}, {EV_COUNT0, EV_COUNT1}, {EV_COUNT1, EV_SCAN1},
                             {EV_EMIT0, EV_EMIT1}};
    double tot = 0;
    for (int k = 0; k < 7; ++k) {
        float t = 0;
        (void)hipEventElapsedTime(&t, c->ev[pairs[k][0]], c->ev[pairs[k][1]]);
        pl.ms[k] = t;
        tot += t;
    }
    pl.ms[7] = tot;
    float tq = 0;
    (void)hipEventElapsedTime(&tq, c->ev[EV_QCOUNT0], c->ev[EV_COUNT1]);
    pl.count_kernel_ms = tq;
    pl.emitted = true;
    return RHG_OK;
}

}  // namespace rhgi

// ---------------------------------------------------------------------------
// Graph handles and ABI entry points
// ---------------------------------------------------------------------------
double rhgi::expected_degree(uint64_t n, double alpha, double R) {
    return alpha > 0.5 ? kbar_of_R((double)n, alpha, R) : (double)n;
}

rhg_status rhgi::request_from_params(const rhg_params *p, Request &rq) {
    if (!p) return RHG_EINVAL;
    rq = Request{};
    rq.mode = SRC_SEED;
    rq.n = p->n;
    rq.alpha = p->alpha;
    rq.seed = p->seed;
    rq.precision = p->precision;
    rq.num_bands = p->num_bands;
    rq.band_ratio = p->band_ratio;
    if (std::isnan(p->R) || std::isnan(p->kbar) || std::isnan(p->band_ratio)) return RHG_EINVAL;
    if (p->R > 0.0) {
        rq.R = p->R;
    } else {
        rhg_status s = rhg_target_radius(p->n, p->alpha, p->kbar, &rq.R);
        if (s != RHG_OK) return s;
    }
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return RHG_EINVAL;
    return RHG_OK;
}

namespace rhgi {

void graph_release(Graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    auto fr = [&](void *p) {
        if (!p) return;
        if (g->free_fn) g->free_fn(p, g->alloc_user);
        else (void)hipFree(p);
    };
    if (g->edge_owner) g->edge_owner.reset();  // slice of a shared output pool
    else fr(g->edges);
    fr(g->d_theta);
    fr(g->d_r);
    fr(g->d_table);
    delete g;
}

static void *graph_alloc(Ctx *c, size_t bytes) { return c->dev_alloc(bytes); }

// Full generation into a graph; emit=false leaves a count-only plan.
rhg_status generate(Ctx *c, const Request &rq, bool emit, Graph **out, uint64_t *m_out) {
    if (!c || !out) return RHG_EINVAL;
    Graph *g = new (std::nothrow) Graph();
    if (!g) return RHG_ENOMEM;
    g->device = c->device;
    g->ctx = c;
    g->free_fn = c->free_fn;
    g->alloc_user = c->alloc_user;
    g->rq = rq;
    rhg_status s = describe(rq, g->pl);
    if (s != RHG_OK) {
        delete g;
        return s;
    }
    (void)hipSetDevice(c->device);
    // keep caller coordinates for the coordinate forms (copy_points / emit)
    if (rq.mode != SRC_SEED) {
        const size_t nb = sizeof(double) * rq.n;
        g->d_theta = (double *)graph_alloc(c, nb);
        g->d_r = (double *)graph_alloc(c, nb);
        if (rq.mode == SRC_TABLE) g->d_table = (double *)graph_alloc(c, 5 * nb);
        if (!g->d_theta || !g->d_r || (rq.mode == SRC_TABLE && !g->d_table)) {
            graph_release(g);
            return RHG_ENOMEM;
        }
        hipMemcpyKind k = rq.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        s = hip_status(hipMemcpyAsync(g->d_theta, rq.theta, nb, k, c->stream));
        if (s == RHG_OK) s = hip_status(hipMemcpyAsync(g->d_r, rq.r, nb, k, c->stream));
        if (s == RHG_OK && rq.mode == SRC_TABLE)
            s = hip_status(hipMemcpyAsync(g->d_table, rq.table, 5 * nb, k, c->stream));
        if (s != RHG_OK) {
            graph_release(g);
            return s;
        }
        g->rq.theta = g->d_theta;
        g->rq.r = g->d_r;
        g->rq.table = g->d_table;
        g->rq.on_device = 1;
    }
    s = run_count(c, g->rq, g->pl);
    if (s == RHG_OK && emit) {
        const uint64_t m = g->pl.m;
        g->edges = (int32_t *)graph_alloc(c, std::max<uint64_t>(m, 1) * 2 * sizeof(int32_t));
        if (!g->edges) s = RHG_ENOMEM;
        if (s == RHG_OK) s = run_emit(c, g->pl, (int2 *)g->edges);
    }
    if (s != RHG_OK) {
        graph_release(g);
        return s;
    }
    if (m_out) *m_out = g->pl.m;
    *out = g;
    return RHG_OK;
}

}  // namespace rhgi

extern "C" rhg_status rhg_generate(rhg_ctx *ctx, const rhg_params *params, rhg_graph **out) {
    Request rq;
    rhg_status s = request_from_params(params, rq);
    if (s != RHG_OK) return s;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, true, &g, nullptr);
    if (s == RHG_OK) *out = reinterpret_cast<rhg_graph *>(g);
    return s;
}

static rhg_status coords_request(uint64_t n, const double *theta, const double *r, const double *table, double R,
                                 rhg_precision precision, int on_device, Request &rq) {
    if (!theta || !r) return RHG_EINVAL;
    rq = Request{};
    rq.mode = table ? SRC_TABLE : SRC_COORDS;
    rq.n = n;
    rq.alpha = 1.0;
    rq.R = R;
    rq.precision = precision;
    rq.theta = theta;
    rq.r = r;
    rq.table = table;
    rq.on_device = on_device ? 1 : 0;
    return RHG_OK;
}

extern "C" rhg_status rhg_generate_from_coords(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r,
                                               double R, rhg_precision precision, int coords_on_device,
                                               rhg_graph **out) {
    Request rq;
    rhg_status s = coords_request(n, theta, r, nullptr, R, precision, coords_on_device, rq);
    if (s != RHG_OK || !out) return s != RHG_OK ? s : RHG_EINVAL;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, true, &g, nullptr);
    if (s == RHG_OK) *out = reinterpret_cast<rhg_graph *>(g);
    return s;
}

extern "C" rhg_status rhg_generate_from_table(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r,
                                              const double *table5xn, double R, rhg_precision precision,
                                              int on_device, rhg_graph **out) {
    if (!table5xn) return RHG_EINVAL;
    Request rq;
    rhg_status s = coords_request(n, theta, r, table5xn, R, precision, on_device, rq);
    if (s != RHG_OK || !out) return s != RHG_OK ? s : RHG_EINVAL;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, true, &g, nullptr);
    if (s == RHG_OK) *out = reinterpret_cast<rhg_graph *>(g);
    return s;
}

extern "C" rhg_status rhg_update_after_move(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r, double R,
                                            rhg_precision precision, const uint8_t *moved, const int32_t *old_pairs,
                                            uint64_t m_old, rhg_graph **out) {
    if (!out || !moved || (m_old && !old_pairs)) return RHG_EINVAL;
    Request rq;
    rhg_status s = coords_request(n, theta, r, nullptr, R, precision, 1, rq);
    if (s != RHG_OK) return s;
    rq.moved = moved;
    rq.old_pairs = old_pairs;
    rq.m_old = m_old;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, true, &g, nullptr);
    if (s == RHG_OK) *out = reinterpret_cast<rhg_graph *>(g);
    return s;
}

extern "C" rhg_status rhg_csr_from_pairs(rhg_ctx *ctx, uint64_t n, const int32_t *pairs, uint64_t m,
                                         uint64_t *row_ptr, int32_t *col) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || n < 1 || !row_ptr || (m && (!pairs || !col))) return RHG_EINVAL;
    if (n >= N_MAX || m >= (1ull << 31)) return RHG_ERANGE;  // rows and entries indexed in 32 bits
    if (2 * m > rhgk::sort_max_keys()) return RHG_ERANGE;     // the sort's tile positions are 32-bit
    RHG_HIP(hipSetDevice(c->device));
    (void)hipGetLastError();
    const hipStream_t st = c->stream;
    const uint64_t len = 2 * m;
    uint32_t *rows = nullptr;
    if (len) {
        rows = (uint32_t *)c->buf(S_CSRROWS, sizeof(uint32_t) * len);
        uint32_t *rows2 = (uint32_t *)c->buf(S_CSRROWS2, sizeof(uint32_t) * len);
        uint32_t *nbrs2 = (uint32_t *)c->buf(S_CSRNBRS2, sizeof(uint32_t) * len);
        uint32_t *err = (uint32_t *)c->buf(S_CSRERR, sizeof(uint32_t));
        void *scr = c->buf(S_CSRSCR, rhgk::sort_scratch_bytes(len));
        if (!rows || !rows2 || !nbrs2 || !err || !scr) return RHG_ENOMEM;
        // the ends are checked (and the sort's digits counted) before any
        // sort pass writes: col is untouched when they are rejected
        const int bits = std::max(1, ceil_log2(n));
        RHG_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), st));
        rhgk::sort_prepare(scr, len, bits, st);
        rhgk::directed_counts((const int2 *)pairs, m, n, err, rhgk::sort_passes(bits), rhgk::sort_counts(scr), st);
        uint32_t *err_host = (uint32_t *)((char *)c->pinned + 1036);
        RHG_HIP(hipMemcpyAsync(err_host, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        RHG_HIP(hipStreamSynchronize(st));
        if (*err_host != 0) return RHG_EINVAL;  // an end outside 0..n-1: nothing sorted or written
        // stable by row: a row's neighbours keep the order of their pairs
        rhgk::sort_pairs_by_counts((const int2 *)pairs, len, rows, (uint32_t *)col, rows2, nbrs2, scr, bits, st);
        RHG_HIP(hipMemcpyAsync(err_host, rhgk::sort_error_flag(scr), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    }
    rhgk::row_pointers(rows, len, n, row_ptr, st);
    RHG_HIP(hipStreamSynchronize(st));
    RHG_HIP(hipGetLastError());
    if (len && *(uint32_t *)((char *)c->pinned + 1036) != 0) return RHG_EDEVICE;  // a sort pass gave up waiting
    return RHG_OK;
}

extern "C" rhg_status rhg_move(rhg_ctx *ctx, uint64_t n, double alpha, double R, double *theta, double *r,
                               const double *tau_phi, double *tau_r) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return RHG_EINVAL;
    if (!(std::isfinite(alpha) && alpha > 0.0 && radius_in_domain(R))) return RHG_EINVAL;
    if (n == 0) return RHG_OK;
    if (!theta || !r || !tau_phi || !tau_r) return RHG_EINVAL;
    if (n >= (1ull << 31)) return RHG_ERANGE;  // one thread per node in one launch
    const double h = std::sinh(alpha * R / 2.0);
    const double S = h * h;  // sinh^2(alpha R / 2): the top of the uniform radius coordinate
    if (!(std::isfinite(S) && S > 0.0)) return RHG_EINVAL;
    RHG_HIP(hipSetDevice(c->device));
    (void)hipGetLastError();
    rhgk::move(n, alpha, R, S, theta, r, tau_phi, tau_r, c->stream);
    return hip_status(hipGetLastError());
}

extern "C" rhg_status rhg_count(rhg_ctx *ctx, const rhg_params *params, rhg_graph **plan, uint64_t *m) {
    if (!plan || !m) return RHG_EINVAL;
    Request rq;
    rhg_status s = request_from_params(params, rq);
    if (s != RHG_OK) return s;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, false, &g, m);
    if (s == RHG_OK) *plan = reinterpret_cast<rhg_graph *>(g);
    return s;
}

// General model (Sec. II, Eq. 2) from rhg_params: a kbar request takes R
// from getTargetRadius at kbar sin(pi T) / (pi T): at temperature T the
// expected degree of a disk of radius R grows by pi T / sin(pi T) to leading
// order (the integral of e^{x/2} against Eq. 2's probability over the
// distance, against the step of T = 0).
static rhg_status soft_request(const rhg_params *p, double T, Request &rq) {
    if (!p || !(T > 0.0 && T < 1.0)) return RHG_EINVAL;
    rhg_params q = *p;
    if (!(q.R > 0.0)) {
        if (std::isnan(q.kbar)) return RHG_EINVAL;
        const double pi = 3.14159265358979323846;
        q.kbar = p->kbar * std::sin(pi * T) / (pi * T);
    }
    rhg_status s = request_from_params(&q, rq);
    if (s != RHG_OK) return s;
    rq.T = T;
    return RHG_OK;
}

extern "C" rhg_status rhg_generate_soft(rhg_ctx *ctx, const rhg_params *params, double T, rhg_graph **out) {
    if (!out) return RHG_EINVAL;
    Request rq;
    rhg_status s = soft_request(params, T, rq);
    if (s != RHG_OK) return s;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, true, &g, nullptr);
    if (s == RHG_OK) *out = reinterpret_cast<rhg_graph *>(g);
    return s;
}

extern "C" rhg_status rhg_count_soft(rhg_ctx *ctx, const rhg_params *params, double T, rhg_graph **plan,
                                     uint64_t *m) {
    if (!plan || !m) return RHG_EINVAL;
    Request rq;
    rhg_status s = soft_request(params, T, rq);
    if (s != RHG_OK) return s;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, false, &g, m);
    if (s == RHG_OK) *plan = reinterpret_cast<rhg_graph *>(g);
    return s;
}

extern "C" rhg_status rhg_generate_soft_from_table(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r,
                                                   const double *table5xn, double R, double T, uint64_t seed,
                                                   int on_device, rhg_graph **out) {
    if (!table5xn || !out || !(T > 0.0 && T < 1.0)) return RHG_EINVAL;
    Request rq;
    rhg_status s = coords_request(n, theta, r, table5xn, R, RHG_FP64, on_device, rq);
    if (s != RHG_OK) return s;
    rq.T = T;
    rq.seed = seed;
    Graph *g = nullptr;
    s = generate(reinterpret_cast<Ctx *>(ctx), rq, true, &g, nullptr);
    if (s == RHG_OK) *out = reinterpret_cast<rhg_graph *>(g);
    return s;
}

extern "C" rhg_status rhg_emit(rhg_ctx *ctx, rhg_graph *plan, int32_t *dev_pairs, uint64_t capacity_pairs) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    Graph *g = reinterpret_cast<Graph *>(plan);
    if (!c || !g || g->ctx != c || g->pl.emitted) return RHG_EINVAL;
    if (capacity_pairs < g->pl.m) return RHG_ETRUNC;
    if (!dev_pairs && g->pl.m) return RHG_EINVAL;
    return run_emit(c, g->pl, (int2 *)dev_pairs);
}

extern "C" rhg_status rhg_graph_num_edges(const rhg_graph *gr, uint64_t *m) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g || !m) return RHG_EINVAL;
    *m = g->pl.m;
    return RHG_OK;
}

extern "C" rhg_status rhg_graph_num_points(const rhg_graph *gr, uint64_t *n) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g || !n) return RHG_EINVAL;
    *n = g->pl.n;
    return RHG_OK;
}

extern "C" rhg_status rhg_graph_radius(const rhg_graph *gr, double *R) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g || !R) return RHG_EINVAL;
    *R = g->pl.R;
    return RHG_OK;
}

extern "C" rhg_status rhg_graph_edges_device(const rhg_graph *gr, const int32_t **pairs) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g || !pairs || !g->edges) return RHG_EINVAL;
    *pairs = g->edges;
    return RHG_OK;
}

extern "C" rhg_status rhg_graph_copy_edges(const rhg_graph *gr, int32_t *host_pairs, uint64_t capacity_pairs) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g || !g->edges) return RHG_EINVAL;
    if (capacity_pairs < g->pl.m) return RHG_ETRUNC;
    if (!g->pl.m) return RHG_OK;
    if (!host_pairs) return RHG_EINVAL;
    (void)hipSetDevice(g->device);
    return hip_status(hipMemcpy(host_pairs, g->edges, g->pl.m * 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
}

extern "C" rhg_status rhg_graph_copy_points(const rhg_graph *gr, double *theta, double *r, double *table5xn,
                                           double *K) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g) return RHG_EINVAL;
    if (K) *K = g->pl.K;
    if (!theta && !r && !table5xn) return RHG_OK;
    (void)hipSetDevice(g->device);
    const uint64_t n = g->pl.n;
    Source src{};
    src.mode = g->rq.mode;
    src.n = n;
    src.seed = g->rq.seed;
    src.alpha = g->rq.alpha;
    src.R = g->rq.R;
    src.sinh_half_aR = std::sinh(g->rq.alpha * g->rq.R / 2.0);
    src.theta = g->d_theta;
    src.r = g->d_r;
    src.table = g->d_table;
    double *d = nullptr;
    if (hipMalloc(&d, sizeof(double) * 7 * n) != hipSuccess) {
        (void)hipGetLastError();
        return RHG_ENOMEM;
    }
    rhgk::point_values(src, n, d, d + n, d + 2 * n, nullptr);
    rhg_status s = hip_status(hipDeviceSynchronize());
    if (s == RHG_OK && theta) s = hip_status(hipMemcpy(theta, d, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (s == RHG_OK && r) s = hip_status(hipMemcpy(r, d + n, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (s == RHG_OK && table5xn)
        s = hip_status(hipMemcpy(table5xn, d + 2 * n, sizeof(double) * 5 * n, hipMemcpyDeviceToHost));
    (void)hipFree(d);
    return s;
}

extern "C" rhg_status rhg_graph_stats(const rhg_graph *gr, rhg_stats *st) {
    const Graph *g = reinterpret_cast<const Graph *>(gr);
    if (!g || !st) return RHG_EINVAL;
    std::memset(st, 0, sizeof(*st));
    st->edges = g->pl.m;
    st->candidates = g->pl.candidates;
    st->rechecks = g->pl.rechecks;
    st->windows = g->pl.windows;
    st->disagreements = g->pl.disagreements;
    st->literal_undecided = g->pl.lit_undecided;
    st->literal_wrong = g->pl.lit_wrong;
    for (int k = 0; k < 8; ++k) st->ms[k] = g->pl.ms[k];
    st->bytes_moved = algorithmic_bytes(g->pl);
    st->count_kernel_ms = g->pl.count_kernel_ms;
    return RHG_OK;
}

extern "C" void rhg_graph_free(rhg_graph *gr) { graph_release(reinterpret_cast<Graph *>(gr)); }
