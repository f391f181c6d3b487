// rhg_internal.h -- host-side structures behind the C ABI (library internal).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include <stdint.h>

#include <memory>

#include "../../include/rhg.h"
#include "rhg_device.h"
#include "rhg_kernels.h"

namespace rhgi {

enum Slot {
    S_KEYS, S_VALS, S_KEYS2, S_VALS2, S_HIST, S_SORTSCR,
    S_TH, S_EP, S_EM, S_SH, S_HS, S_HC, S_EP32, S_EM32, S_SH32,
    S_BTAB, S_WIN, S_BCAND, S_BOFF, S_NUNITS, S_UOFF, S_SCANSCR,
    S_UBATCH, S_UEDGES, S_UEOFF, S_STATS, S_SCANSCR2, S_BITS, S_BANDSTART, S_UKEY, S_UORDER, S_UKEY2, S_UORDER2, S_SORTSCR2,
    S_SHARD, S_UDESC, S_MOVED, S_MOVEDO, S_KEEPC, S_KEEPO, S_KEEPERR, S_SCANSCR3,
    S_CSRROWS, S_CSRROWS2, S_CSRNBRS2, S_CSRSCR, S_CSRERR, S_SOFTTAB,
    S_COUNT
};

enum Ev { EV_KEYS0, EV_KEYS1, EV_SORT0, EV_SORT1, EV_TABLE1, EV_PLAN0, EV_PLAN1, EV_COUNT0, EV_COUNT1, EV_SCAN1,
          EV_EMIT0, EV_EMIT1, EV_QCOUNT0, EV_COUNT_ };

struct SlotBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_user = nullptr;
    SlotBuf slots[S_COUNT];
    hipEvent_t ev[EV_COUNT_] = {};
    std::vector<double> stab_host;  // the general model's threshold table, as last uploaded
    void *pinned = nullptr;  // 4 KB host readback area
    int exhaustive = 0;
    int ablation = 0;  // RHG_OPT_LITERAL_ABLATION
    uint32_t shard_count = 1, shard_index = 0;  // query share of this context (RHG_OPT_SHARD_*)
    uint64_t generation = 0;  // bumped by every count; a plan may emit only while current

    void *dev_alloc(size_t bytes);
    void dev_free(void *p);
    void *buf(int slot, size_t bytes);  // grow-only work buffer
    ~Ctx();
};

// What to generate.
struct Request {
    int mode = rhgd::SRC_SEED;
    uint64_t n = 0;
    double alpha = 1.0, R = 0.0;
    uint64_t seed = 0;
    int precision = RHG_FP64;
    uint32_t num_bands = 0;
    double band_ratio = 0.0;
    const double *theta = nullptr, *r = nullptr, *table = nullptr;
    int on_device = 0;
    // graph update after a move (device): per-point moved flags in original
    // order, and the edge list before the move
    const uint8_t *moved = nullptr;
    const int32_t *old_pairs = nullptr;
    uint64_t m_old = 0;
    // general model (Sec. II, Eq. 2): temperature, 0 = the threshold model
    double T = 0.0;
};

// One planned generation.
struct Plan {
    uint64_t n = 0;
    int B = 1;
    double p = 0.9;
    double R = 0, K = 0;
    // general model: T > 0, the pairs' seed, and cosh of the enlarged radius
    // Rc = R + 74 T that bounds its candidates (K stays cosh R)
    double T = 0, Kc = 0;
    uint64_t pseed = 0;
    double c[rhgd::MAX_BANDS + 1] = {};
    bool fp32 = false;
    rhgd::Geo geo;
    rhgk::QueryArgs qa;
    uint64_t n_units = 0, windows = 0, candidates = 0, m = 0, rechecks = 0, disagreements = 0;
    uint64_t lit_undecided = 0, lit_wrong = 0;  // literal-Eq. 3 ablation counters
    uint64_t generation = 0;
    bool emitted = false;
    double ms[8] = {};
    double count_kernel_ms = 0;  // the count kernel alone (ms[4] also holds unit bookkeeping and order)
    // graph update: the old pairs kept (m_keep, written first, by the tile
    // offsets keep_off), then the m - m_keep pairs at moved points
    const int2 *old_pairs = nullptr;
    const uint32_t *moved_orig = nullptr;  // moved flags as bits, original order
    uint64_t m_old = 0, m_keep = 0;
    const uint64_t *keep_off = nullptr;
    uint32_t *keep_err = nullptr;
};

struct Graph {
    int device = 0;
    Ctx *ctx = nullptr;  // context that planned it (count-only plans emit through it)
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_user = nullptr;
    Request rq;
    Plan pl;
    int32_t *edges = nullptr;
    std::shared_ptr<void> edge_owner;  // set when edges are a slice of a shared buffer
    double *d_theta = nullptr, *d_r = nullptr, *d_table = nullptr;
};

// Algorithmic HBM bytes of the timed path (sort through emit), the traffic
// the method itself needs: per point the key and index written and read
// once per sort digit pass, the angle and table (6 x 8 B) written once and read by the
// plan and by both query passes, per window 8 B written and read twice, per
// edge one 8-byte pair written.
inline uint64_t algorithmic_bytes(const Plan &p) {
    const uint64_t n = p.n;
    const uint64_t per_point = 8ull * 2 * 4 + 48 + 5 * 8 * 3;
    return n * per_point + p.windows * 8 * 3 + p.m * 8;
}

rhg_status describe(const Request &rq, Plan &pl);
// Largest disk radius R accepted by every entry point (the FP64 distance test
// stays finite for all pairs of points up to it).
constexpr double R_MAX = 354.0;
// General model: candidates lie within Rc = R + SOFT_CUT * 2T; beyond it
// y = (x - R) / (2T) > 37, f < e^-37 < 2^-53, and the smallest uniform is
// 2^-53, so no pair there can be an edge.
constexpr double SOFT_CUT = 37.0;
bool radius_in_domain(double R);
rhg_status request_from_params(const rhg_params *p, Request &rq);
// Average degree the model approximation gives for (n, alpha, R) (n when alpha <= 1/2).
double expected_degree(uint64_t n, double alpha, double R);
void geo_static(const Plan &pl, rhgd::Geo &g);
int key_bits_for(int B);
int ceil_log2(uint64_t x);
rhg_status hip_status(hipError_t e);
void graph_release(Graph *g);
rhg_status run_count(Ctx *c, const Request &rq, Plan &pl);
rhg_status run_emit(Ctx *c, Plan &pl, int2 *out);
rhg_status generate(Ctx *c, const Request &rq, bool emit, Graph **out, uint64_t *m_out);

// Scratch of one request on the one-launch path (small.hip): capacities of
// the arrays whose size depends on the plan, and the bytes of all arrays.
struct SmallLayout {
    uint64_t bytes = 0;
    uint64_t unit_cap = 0, win_cap = 0, btab_cap = 0;
};
constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }
// Layout for n points in B slabs with room for unit_cap work units.
SmallLayout small_layout_units(uint64_t n, int B, uint64_t unit_cap, bool fp32);
// Fills the descriptor of one seeded request: geometry, source, and the
// arrays of `lay` carved from `base` (device memory of lay.bytes);
// stats: two zeroed device words for its counters.
void small_fill_desc(rhgk::SmallDesc &D, const Plan &pl, const Request &rq, const SmallLayout &lay, char *base,
                     unsigned long long *stats);
// Per-device set-up of the fixed scratch of rhg_generate_noalloc (once per
// device, with that device current); called by rhg_ctx_create.
rhg_status noalloc_setup(int device);

}  // namespace rhgi
