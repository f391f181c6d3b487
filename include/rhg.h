/*
 * rhg.h -- C ABI of the MI355X (gfx950) threshold random hyperbolic graph
 * generator.
 *
 * The method is the band-based neighbour query of von Looz, Oezdayi, Laue,
 * Meyerhenke, "Generating massive complex networks with hyperbolic geometry
 * faster in practice" (HPEC 2016), Sec. III, Algorithm 1:
 *   - n points in a hyperbolic disk of radius R, angle uniform, radius with
 *     density alpha sinh(alpha r)/(cosh(alpha R) - 1)  (Sec. II, Eq. 1);
 *   - edge {u, v} iff dist_H(u, v) < R, dist_H by the hyperbolic law of
 *     cosines (Sec. II, Eq. 3);
 *   - R from the average degree by getTargetRadius (Sec. III-B), or given;
 *   - the disk is cut in ring slabs with geometric widths (Sec. III-A,
 *     Eq. 4), each slab angle-sorted, and every point scans the angular
 *     window of each slab outward of it (getMinMaxPhi, Sec. III-B).
 *
 * Conventions shared by every call:
 *   - Every call returns rhg_status (0 = RHG_OK, negative = error) unless it
 *     returns void.  No call aborts the process; invalid arguments give
 *     RHG_EINVAL and leave outputs untouched.
 *   - Device pointers are HIP device addresses on the context's device; host
 *     pointers are ordinary process memory.  Each argument says which.
 *   - Output edges are int32 pairs (lo, hi), lo < hi, in the original point
 *     indices (the sampler's index i, or the position in the caller's
 *     coordinate arrays).  Each undirected edge appears exactly once, no
 *     self loops.  The order is deterministic for given inputs and library
 *     build but otherwise unspecified: compare edge lists as sets.
 *   - The distance test is evaluated in IEEE binary64 in a fixed order
 *     (cosh(r_u - r_v) + 2 sinh r_u sinh r_v sin^2(dtheta/2), from per-point
 *     exp(r), exp(-r), sin(theta/2), cos(theta/2), with sinh r taken as
 *     (exp(r) - exp(-r)) / 2 of the first two), strict "< cosh R".
 *     RHG_FP32_RECHECK decides the same predicate with an FP32 filter and a
 *     proven margin and re-decides the undecided pairs in FP64: its edge set
 *     is identical to RHG_FP64's.
 *   - One context = one HIP stream; a context is not thread safe.  A server
 *     (rhg_server_*) is thread safe.
 */
#ifndef RHG_H
#define RHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RHG_OK = 0,
    RHG_EINVAL = -1,  /* invalid argument (range, NaN, NULL, unreachable average degree) */
    RHG_ENOMEM = -2,  /* device or host allocation failed */
    RHG_EDEVICE = -3, /* HIP runtime error (no device, launch failure) */
    RHG_ERANGE = -4,  /* size beyond what the int32 output or internal counters can hold */
    RHG_ETRUNC = -5,  /* caller buffer smaller than the result */
    RHG_EBUSY = -6    /* server: result not ready (non-blocking wait) */
} rhg_status;

typedef enum {
    RHG_FP64 = 0,         /* distance test in FP64 */
    RHG_FP32_RECHECK = 1  /* FP32 filter with margin, undecided pairs in FP64; same edges */
} rhg_precision;

/* Generation parameters (Algorithm 1 input: n, average degree, alpha = (gamma-1)/2).
 *   n          number of points, 2 <= n < 2^31 (RHG_ERANGE above: int32 indices).
 *   alpha      dispersion, > 0; with kbar (R <= 0) it must be > 1/2.
 *   kbar       target average degree, used when R <= 0: R = getTargetRadius(n, alpha, kbar).
 *   R          disk radius; R > 0 overrides kbar.  0 < R <= 354 (RHG_EINVAL
 *              beyond: the FP64 distance test forms 2 sinh r_u sinh r_w, which
 *              must be finite for every pair of points, up to e^{2R}/2 <
 *              DBL_MAX); the sampler also needs sinh(alpha R / 2) finite.
 *              FP32_RECHECK needs R <= 43.
 *   seed       SplitMix64 seed; point i uses outputs 2i (angle) and 2i+1 (radius).
 *   precision  RHG_FP64 or RHG_FP32_RECHECK.
 *   num_bands  number of slabs B, 0 = max(1, ceil(log2 n) - 8); 1 <= B <= 32.
 *              The edge set does not depend on B or band_ratio; they set
 *              the balance of window planning against distance tests.
 *   band_ratio width ratio p of consecutive slabs, 0 = 0.9; 0 < p <= 1 (p = 1: equal widths). */
typedef struct {
    uint64_t n;
    double alpha;
    double kbar;
    double R;
    uint64_t seed;
    rhg_precision precision;
    uint32_t num_bands;
    double band_ratio;
} rhg_params;

typedef struct rhg_ctx rhg_ctx;
typedef struct rhg_graph rhg_graph;
typedef struct rhg_server rhg_server;

/* Per-graph counters and phase times.
 *   edges       m
 *   candidates  distance tests performed (window sizes summed)
 *   rechecks    pairs the FP32 filter left undecided (FP32_RECHECK only)
 *   windows     (query, slab) windows planned
 *   ms[8]       device time per phase from HIP events on the context stream,
 *               each pair of events bracketing only that phase's launches:
 *               0 sample + slab keys, 1 sort + slab starts, 2 table gather,
 *               3 slab index + window plan + unit scans, 4 count, 5 edge scan,
 *               6 emit, 7 sum of 0-6 (host synchronisation gaps excluded)
 *   bytes_moved algorithmic HBM bytes of phases 1-6 (reads + writes the
 *               method needs), for roofline reporting
 *   count_kernel_ms  device time of the count kernel alone (ms[4] without the
 *               unit bookkeeping and ordering launches) */
typedef struct {
    uint64_t edges;
    uint64_t candidates;
    uint64_t rechecks;
    uint64_t windows;
    uint64_t disagreements; /* FP32 decisions differing from FP64 (exhaustive option only; must be 0) */
    double ms[8];
    uint64_t bytes_moved;
    double count_kernel_ms;
    uint64_t literal_undecided; /* RHG_OPT_LITERAL_ABLATION: candidates Eq. 3 as printed, in FP32, leaves undecided */
    uint64_t literal_wrong;     /* RHG_OPT_LITERAL_ABLATION: its plain FP32 decisions that differ from FP64 */
} rhg_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run
 * on (e.g. the caller's PyTorch stream), or NULL for a library-owned blocking
 * stream, which is ordered with work on the device's null stream (PyTorch's
 * default stream has handle 0 and lands here).  The context keeps device work
 * buffers between calls (grown as needed). */
rhg_status rhg_ctx_create(int device, void *hip_stream, rhg_ctx **out);

/* Route the context's device allocations through the caller (e.g. a caching
 * allocator).  alloc(bytes, user) returns a device pointer or NULL; free(ptr,
 * user).  Pass alloc = NULL to restore hipMalloc/hipFree.  Must be called
 * before the first generation on the context. */
rhg_status rhg_ctx_set_allocator(rhg_ctx *ctx, void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *),
                                 void *user);

/* Context options.
 *   RHG_OPT_FP32_EXHAUSTIVE (value 0/1): in RHG_FP32_RECHECK count passes also
 *   evaluate the FP64 test on every candidate the filter decided and count
 *   disagreements into rhg_stats.disagreements (a self-check of the margin;
 *   slower).
 *   RHG_OPT_SHARD_COUNT (S, 1..65536, default 1) and RHG_OPT_SHARD_INDEX
 *   (k, 0..S-1, default 0): one share of the query side of Alg. 1, as one of
 *   S devices would run it.  Every point is still sampled, sorted and planned
 *   (the whole table), but only the queries of shard k are counted and
 *   emitted: a contiguous range of 64-query batches of the sorted order, cut
 *   where the running candidate total crosses k/S and (k+1)/S of the whole.
 *   Each edge is found by exactly one query, so the S shards' edge lists are
 *   disjoint and together are the whole graph.  rhg_stats.edges and
 *   .candidates then count the shard only.  A generation with k >= S returns
 *   RHG_EINVAL.  The serving path ignores these options.
 *   RHG_OPT_LITERAL_ABLATION (value 0/1): in RHG_FP32_RECHECK count passes
 *   also decide every candidate by Eq. 3 as printed (cosh r_u cosh r_v -
 *   sinh r_u sinh r_v cos(theta_u - theta_v)) in FP32 and count into
 *   rhg_stats.literal_undecided the candidates within its sound rounding
 *   margin 8 u32 (A + S) of cosh R (A, S the two products) and into
 *   .literal_wrong its plain FP32 decisions that differ from the FP64 test
 *   (the edges themselves stay those of the FP64 test; slower). */
typedef enum {
    RHG_OPT_FP32_EXHAUSTIVE = 1,
    RHG_OPT_SHARD_COUNT = 2,
    RHG_OPT_SHARD_INDEX = 3,
    RHG_OPT_LITERAL_ABLATION = 4
} rhg_option;
rhg_status rhg_ctx_set_option(rhg_ctx *ctx, int option, int64_t value);

/* Release the context and its work buffers (graphs stay valid). */
void rhg_ctx_destroy(rhg_ctx *ctx);

/* ---- parameters (host only, no device use) ------------------------------ */

/* getTargetRadius (Sec. III-B): the R on the decreasing branch of the
 * average-degree approximation with zeta = 1 that equals kbar.
 * RHG_EINVAL if alpha <= 1/2, kbar <= 0, n < 2, non-finite input, or kbar
 * above the approximation's maximum. */
rhg_status rhg_target_radius(uint64_t n, double alpha, double kbar, double *R_out);

/* Slab boundaries c_0 = 0 < ... < c_B = R (Sec. III-A, Eq. 4) as used by the
 * library; c_out holds B+1 doubles (host). */
rhg_status rhg_band_boundaries(double R, uint32_t num_bands, double band_ratio, double *c_out);

/* ---- generation ----------------------------------------------------------- */

/* Sample n points (Eq. 1) from params->seed on the device and return the
 * threshold RHG (Algorithm 1).  *out receives a library-owned graph whose
 * edges stay in device memory until rhg_graph_free. */
rhg_status rhg_generate(rhg_ctx *ctx, const rhg_params *params, rhg_graph **out);

/* Same for caller coordinates (the polar coordinates of Sec. II; Algorithm 1
 * from its slab step on): theta[n] in [0, 2pi] (2pi meaning fl(2*pi)),
 * r[n] in [0, R], 0 < R <= 354, FP64, host or device memory (coords_on_device
 * = 0/1; device arrays are only read).  Edges use the positions in these
 * arrays: {u, v} iff dist_H(u, v) < R by Eq. 3. */
rhg_status rhg_generate_from_coords(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r, double R,
                                    rhg_precision precision, int coords_on_device, rhg_graph **out);

/* Same, with the per-point table supplied instead of computed on the device:
 * table5xn = [exp(r) | exp(-r) | sinh r | sin(theta/2) | cos(theta/2)], each
 * n doubles, row-major (5 x n), same memory kind as theta/r.  The distance
 * test reads exactly the bits of columns 0, 1, 3 and 4, so any caller-side
 * evaluation of the same table gives a bit-identical edge set; it takes
 * sinh r as (exp(r) - exp(-r)) / 2 of columns 0 and 1 (column 2 is not read;
 * rhg_graph_copy_points fills it with that value).  theta and r still place
 * points in slabs and windows. */
rhg_status rhg_generate_from_table(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r,
                                   const double *table5xn, double R, rhg_precision precision, int on_device,
                                   rhg_graph **out);

/* Dynamic model (Sec. III-C): one movement step of n nodes, in place, on
 * the context stream (asynchronous; no host synchronisation).
 *   theta[n], r[n]  device FP64 angles in [0, 2pi) and radii in [0, R]; updated.
 *   tau_phi[n]      device FP64 angular steps (radians); read only.
 *   tau_r[n]        device FP64 radial steps in units of cosh(alpha r) (the
 *                   transform of Algorithm 2 under which Eq. 1's radius law is
 *                   uniform); negated where the step is reflected an odd
 *                   number of times (the node bounces off the centre or rim).
 * theta' = (theta + tau_phi) mod 2pi; cosh(alpha r') = cosh(alpha r) + tau_r,
 * mirrored at 1 and cosh(alpha R) as often as it crosses them (computed on
 * sinh^2(alpha r / 2), which keeps relative precision near the centre).  With
 * both signs of each step size equally likely the point density is preserved
 * exactly (Theorem 1).  A zero step leaves the coordinate bit for bit as it
 * is, so nodes with tau_phi = tau_r = 0 stay put.
 * The arrays are owned by the caller and must not
 * overlap.  RHG_EINVAL: null context, null arrays with n > 0, alpha not
 * finite and positive, R outside (0, 354]; RHG_ERANGE: n >= 2^31.  Regenerate the graph of the moved points with
 * rhg_generate_from_coords (coords_on_device = 1), or update it with
 * rhg_update_after_move. */
rhg_status rhg_move(rhg_ctx *ctx, uint64_t n, double alpha, double R, double *theta, double *r,
                    const double *tau_phi, double *tau_r);

/* Dynamic model (Sec. III-C): the graph after a move, updated from the graph
 * before it instead of generated anew.  An edge between two points that did
 * not move is still an edge; every edge at a moved point is found by the band
 * query of the moved points alone, in every slab and both directions (the
 * window bound of Sec. III-B holds for slabs below the query's too), a pair
 * of two moved points being taken once.
 *   theta[n], r[n]   device FP64 coordinates after the move; read only.
 *   moved[n]         device bytes, original order: nonzero for every point
 *                    whose coordinates changed (points may be flagged that
 *                    did not move; they are queried again); read only.
 *   old_pairs        device int32 pairs (2 * m_old), the edge list of the
 *                    same n points before the move, each edge once, any
 *                    order; read only.
 * *out is a graph as rhg_generate_from_coords returns, with library-owned
 * edges: the old pairs whose ends both stayed, in their old order, then the
 * pairs at moved points.  If old_pairs is the threshold graph of the
 * coordinates before the move and moved covers every point that moved, its
 * edge set is that of rhg_generate_from_coords(theta, r), the same bits of
 * the same distance test deciding every pair.  The arrays must stay valid
 * until the call returns.  RHG_EINVAL: null arrays, a pair naming a point
 * outside 0..n-1, or a query share set on the context; other errors as for
 * rhg_generate_from_coords. */
rhg_status rhg_update_after_move(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r, double R,
                                 rhg_precision precision, const uint8_t *moved, const int32_t *old_pairs,
                                 uint64_t m_old, rhg_graph **out);

/* Symmetric CSR adjacency of an edge list (the graph-construction step after
 * generation): row v of the n rows holds every w with (v, w) or (w, v) among
 * the pairs.
 *   pairs    device int32 (lo, hi) pairs, m of them, ends in 0..n-1 (e.g.
 *            rhg_graph_edges_device or an rhg_emit tensor); read only.
 *   row_ptr  device uint64[n + 1]: row v is col[row_ptr[v] .. row_ptr[v+1]).
 *   col      device int32[2m].
 * Each pair becomes two directed entries, ordered by a stable sort by row, so
 * within a row the neighbours keep the order of their pairs in the list and
 * the result is deterministic.  Work buffers of about 14 bytes per entry
 * belong to the context.  Synchronous on the context stream.  RHG_EINVAL:
 * null context, n < 1, null arrays, an end outside 0..n-1 (nothing written);
 * RHG_ERANGE: n >= 2^31 or m >= 2^31. */
rhg_status rhg_csr_from_pairs(rhg_ctx *ctx, uint64_t n, const int32_t *pairs, uint64_t m, uint64_t *row_ptr,
                              int32_t *col);

/* Two-phase form for caller-owned output (e.g. a PyTorch tensor) of
 * rhg_generate (Algorithm 1, Sec. III-B): rhg_count samples the points,
 * sorts the slabs, plans the getMinMaxPhi windows and decides every
 * candidate pair by Eq. 3 (m = the number of edges); rhg_emit adds the edges
 * (the decisions replayed, not re-tested), writing the m pairs into
 * dev_pairs (device, >= 2*m int32, capacity_pairs in pairs; RHG_ETRUNC if
 * smaller, nothing written).  *plan is a graph handle without edges; free it
 * with rhg_graph_free.  rhg_emit may be called once per plan. */
rhg_status rhg_count(rhg_ctx *ctx, const rhg_params *params, rhg_graph **plan, uint64_t *m);
rhg_status rhg_emit(rhg_ctx *ctx, rhg_graph *plan, int32_t *dev_pairs, uint64_t capacity_pairs);

/* ---- general model, temperature T > 0 (Sec. II, Eq. 2) -------------------
 * Each pair {u, v} at hyperbolic distance x (Eq. 3) is an edge with
 * probability f(x) = 1 / (exp((x - R) / (2T)) + 1).  The paper gives no
 * algorithm for T > 0; this library decides every unordered pair {lo, hi}
 * (lo < hi, original indices) once with its own uniform
 *   U = ((z >> 11) + 1) 2^-53 in (0, 1],  z = SplitMix64 output number
 *   2^62 + lo 2^31 + hi of the generator seeded with `seed`
 * (the points' outputs are 0 .. 2n - 1), edge iff U < f(x), evaluated in FP64
 * in this order: V the cosh distance as for the threshold model,
 * x = acosh(V) (0 for V <= 1), y = (x - R) / (2T), f = 1 / (1 + exp(y)).  The
 * band query of Algorithm 1 runs for the enlarged radius Rc = R + 74 T:
 * beyond it f < 2^-53 <= U, so no pair there can be an edge, and the edge set
 * is that of the all-pairs rule.  The work grows about like e^{37 T} times
 * the threshold model's: meant for small T (the limit T -> 0 is the
 * threshold graph).  Same output, ownership and error conventions as the
 * threshold calls; only RHG_FP64.  RHG_EINVAL besides: T outside (0, 1),
 * RHG_FP32_RECHECK, or R + 74 T > 354. */

/* Seeded points (Eq. 1) from params->seed, which also seeds the pairs'
 * uniforms.  With R <= 0, R = getTargetRadius(n, alpha, kbar sin(pi T) /
 * (pi T)): the expected degree at temperature T is about pi T / sin(pi T)
 * times that of the threshold model with the same R. */
rhg_status rhg_generate_soft(rhg_ctx *ctx, const rhg_params *params, double T, rhg_graph **out);
/* The same as a count-only plan, emitted with rhg_emit into caller memory. */
rhg_status rhg_count_soft(rhg_ctx *ctx, const rhg_params *params, double T, rhg_graph **plan, uint64_t *m);
/* Caller points and table (layout and memory kinds as rhg_generate_from_table),
 * disk radius R, temperature T, and the seed of the pairs' uniforms. */
rhg_status rhg_generate_soft_from_table(rhg_ctx *ctx, uint64_t n, const double *theta, const double *r,
                                        const double *table5xn, double R, double T, uint64_t seed, int on_device,
                                        rhg_graph **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rhg_count
 * + rhg_emit of one seeded request in one call that allocates nothing.  All
 * work arrays live in a fixed device array of 16 MiB that each device holds
 * from the library's load until the process ends; its address is taken at
 * rhg_ctx_create.  The whole generation is one launch of the one-launch
 * small-request kernel (the serving path's), so the edge list is
 * byte-identical to rhg_generate's / rhg_emit's for the same params.
 *   params     as for rhg_generate; n <= 8192 (RHG_ERANGE above), any slab
 *              count and precision.
 *   dev_pairs  device int32 output, capacity_pairs pairs (NULL only with 0).
 *   m          (host) receives the number of edges, also on RHG_ETRUNC.
 * Synchronous on the context stream.  RHG_ETRUNC: m > capacity_pairs,
 * nothing written.  RHG_EINVAL: as rhg_generate, or a query share set on the
 * context.  Calls on one device share the fixed array: calls that overlap in
 * time on one device (other contexts or threads) race, and the caller must
 * serialise them; each call clears what it needs, so sequential calls are
 * independent. */
rhg_status rhg_generate_noalloc(rhg_ctx *ctx, const rhg_params *params, int32_t *dev_pairs,
                                uint64_t capacity_pairs, uint64_t *m);

/* ---- graph handle --------------------------------------------------------- */

rhg_status rhg_graph_num_edges(const rhg_graph *g, uint64_t *m);
rhg_status rhg_graph_num_points(const rhg_graph *g, uint64_t *n);
rhg_status rhg_graph_radius(const rhg_graph *g, double *R);

/* Borrowed device pointer to the 2*m int32 edge array; valid until
 * rhg_graph_free.  RHG_EINVAL for a count-only plan before rhg_emit. */
rhg_status rhg_graph_edges_device(const rhg_graph *g, const int32_t **pairs);

/* Copy the edges to host memory host_pairs (capacity_pairs pairs);
 * RHG_ETRUNC (nothing copied) if capacity_pairs < m. */
rhg_status rhg_graph_copy_edges(const rhg_graph *g, int32_t *host_pairs, uint64_t capacity_pairs);

/* Copy the points and the exact table bits the distance test used, in
 * original point order, to host memory: theta[n], r[n], table5xn[5*n]
 * (layout as in rhg_generate_from_table); any pointer may be NULL to skip it.
 * K receives cosh R as used.  Only graphs from rhg_generate/rhg_count keep
 * the points; for the coordinate forms this returns what was passed. */
rhg_status rhg_graph_copy_points(const rhg_graph *g, double *theta, double *r, double *table5xn, double *K);

rhg_status rhg_graph_stats(const rhg_graph *g, rhg_stats *stats);

/* Release a graph or plan and its device memory.  NULL is ignored. */
void rhg_graph_free(rhg_graph *g);

/* ---- serving --------------------------------------------------------------- */

/* A request server on one device: submitted generation requests are admitted
 * while their estimated edge memory (n * kbar / 2 pairs, 8 bytes each, plus
 * per-point work memory) fits in mem_budget_bytes; admitted requests run
 * concurrently on several streams, small ones packed together into shared
 * launches; results are identical to rhg_generate's for the same params. */
rhg_status rhg_server_create(int device, uint64_t mem_budget_bytes, rhg_server **out);
/* Device memory a request is charged at admission (host only, no device use):
 * its edge list, n * kbar / 2 pairs of 8 bytes with 25% headroom (kbar: the
 * requested average degree, or for R-given requests the model's expected
 * degree for that R, clamped to [1, n]), plus 256 bytes per point of work
 * buffers and 1 MiB.  RHG_EINVAL for parameters rhg_generate would refuse. */
rhg_status rhg_server_estimate_bytes(const rhg_params *params, uint64_t *bytes);
/* Queue a request (params copied).  Returns at once with a ticket. */
rhg_status rhg_server_submit(rhg_server *s, const rhg_params *params, uint64_t *ticket);
/* Wait for a ticket: blocks until done (timeout_ms < 0), or waits at most
 * timeout_ms and returns RHG_EBUSY if not done.  *out receives the graph
 * (caller frees it); latency_ms the time from submit to device completion.
 * A request that failed returns its error here. */
rhg_status rhg_server_wait(rhg_server *s, uint64_t ticket, int timeout_ms, rhg_graph **out, double *latency_ms);
/* Server counters:
 *   completed    requests finished (success or error)
 *   batched      requests run inside a shared group of small requests (one
 *                host synchronisation per group)
 *   groups       such groups
 *   fallbacks    grouped requests that outgrew their preallocated scratch or
 *                output slice and were rerun on the multi-launch path
 *   peak_bytes   highest admitted estimated memory in flight
 *   budget_bytes the admission budget */
typedef struct {
    uint64_t completed;
    uint64_t batched;
    uint64_t groups;
    uint64_t fallbacks;
    uint64_t peak_bytes;
    uint64_t budget_bytes;
} rhg_server_stats;
rhg_status rhg_server_counters(rhg_server *s, rhg_server_stats *out);
/* Stop accepting, finish pending requests, release everything (results never
 * waited for are freed). */
void rhg_server_destroy(rhg_server *s);

/* Static string for a status code. */
const char *rhg_status_str(rhg_status s);

/* Library version string (for determinism claims: same inputs + same version -> same bytes). */
const char *rhg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RHG_H */
