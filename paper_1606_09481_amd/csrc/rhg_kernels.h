// rhg_kernels.h -- host-side launchers of the gfx950 kernels (library internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rhg_device.h"

namespace rhgk {

// a0 + a2: sample or read each point, find its slab (c_i <= r < c_{i+1},
// r = R in the last), build the sort key (slab << 27 | q(theta)) and the
// identity payload; err |= 1 on a coordinate outside [0, 2pi] x [0, R] or
// non-finite (err zeroed here).
void keys(const rhgd::Source &src, int B, const double *c_host, uint32_t *keys, uint32_t *vals, int *err,
          hipStream_t st);

// Slab starts bs[0..B] in the sorted keys (bs[B] = n).
void band_starts(const uint32_t *keys, uint64_t n, int B, uint32_t *bs, hipStream_t st);

// a3: stable LSD radix sort of (keys, vals), `bits` low key bits, 8 per pass;
// the result ends in (keys, vals) (copied back after an odd number of
// passes); tmp buffers of n each; scratch from sort_scratch_bytes.
// sort_passes(bits) passes: with an odd count a caller that wants no copy
// back passes its buffers the other way round.
// Device flag (u32) a sort raises if a look-back made no progress for its
// whole spin budget (never expected; the sorted output is then invalid).
uint32_t *sort_error_flag(void *scratch);
size_t sort_scratch_bytes(uint64_t n);
// Most keys one sort takes: tile positions are formed in 32 bits, and the
// last tile must end at or below 2^32.
uint64_t sort_max_keys();
void radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, void *scratch, uint64_t n,
                int bits, hipStream_t st, bool copy_back = true);
int sort_passes(int bits);
// The same in parts, for a caller that counts the digits itself: sort_prepare
// zeroes the scratch, the caller adds the digit counts of every pass to
// sort_counts(scratch) (pass p at [256 p, 256 p + 256)), sort_by_counts sorts.
void sort_prepare(void *scratch, uint64_t n, int bits, hipStream_t st);
uint32_t *sort_counts(void *scratch);
void sort_by_counts(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, void *scratch, uint64_t n,
                    int bits, hipStream_t st, bool copy_back = true);
// The same for the n entries (x, y), (y, x) of n/2 pairs (n even), read from
// the pairs by the first pass: sorted entries end in (keys, vals); the
// *_tmp buffers, and keys and vals themselves, serve the passes in between.
void sort_pairs_by_counts(const int2 *pairs, uint64_t n, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp,
                          uint32_t *vals_tmp, void *scratch, int bits, hipStream_t st);

// a1 + a3 gather: per sorted position, the point's angle and table
// (computed, or copied from the caller's table) in sorted order.
void gather(const rhgd::Source &src, const uint32_t *idx, uint64_t n, double *th, double2 *epm,
            double2 *hsc, float2 *f32, hipStream_t st);

// Same values in original order (for exporting the exact bits used).
void point_values(const rhgd::Source &src, uint64_t n, double *th, double *rr, double *table5xn, hipStream_t st);

// Slab bucket index: btab (geo.bto / geo.bshift layout).
void bucket_index(const rhgd::Geo &geo, uint32_t *btab, hipStream_t st);

// a4: windows of every (query, slab >= slab(query)), stored slab-major;
// per-batch candidate totals and per-batch slab segment offsets (B+1 each).
void plan(const rhgd::Geo &geo, uint2 *win, uint64_t *batch_cand, uint64_t *batch_slab_off, hipStream_t st);

// a6 scans: out[0..len] = exclusive prefix of in[0..len) (out[len] = total).
size_t scan_scratch_bytes(uint64_t len);
void scan_u64(const uint64_t *in, uint64_t *out, uint64_t len, void *scratch, hipStream_t st);
void scan_u32(const uint32_t *in, uint64_t *out, uint64_t len, void *scratch, hipStream_t st);

// Work units: units per batch = ceil(cand / UNIT).
void units_per_batch(const uint64_t *batch_cand, uint64_t nb, uint64_t *nunits, hipStream_t st);
// boff / uoff (nb + 1 each): exclusive scans of the candidates and of the
// units per batch (nunits: nb scratch, used above one workgroup's size).
void plan_scans(const uint64_t *cand, uint64_t nb, uint64_t *boff, uint64_t *nunits, uint64_t *uoff, void *scratch,
                hipStream_t st);
// Dynamic model: one movement step of n nodes in place (S = sinh^2(alpha R / 2)).
void move(uint64_t n, double alpha, double R, double S, double *theta, double *r, const double *tau_phi,
          double *tau_r, hipStream_t st);
// Graph update after a move: bit s of out = moved[idx[s]] != 0 (sorted
// order; idx null: moved[s], original order), moved_bit_words(n) words; the
// old pairs whose ends both stayed (bits in original order), counted per tile
// of the list (keep_tiles(m) tiles; *err set for an end outside 0..n-1) and
// written in their order at out[offs[tile] ..].
uint64_t moved_bit_words(uint64_t n);
// CSR: the row digits of the 2m directed entries of m pairs (both ends of
// every pair) added to the sort's counts (`passes` passes), *err set for an
// end outside 0..n-1; and the row pointers row_ptr[0..n] of rows sorted by
// row (len entries, rows < n).
void directed_counts(const int2 *pairs, uint64_t m, uint64_t n, uint32_t *err, int passes, uint32_t *counts,
                     hipStream_t st);
void row_pointers(const uint32_t *rows, uint64_t len, uint64_t n, uint64_t *row_ptr, hipStream_t st);
void moved_bits(const uint32_t *idx, const uint8_t *moved, uint64_t n, uint32_t *out, hipStream_t st);
uint64_t keep_tiles(uint64_t m);
void keep_count(const int2 *pairs, uint64_t m, const uint32_t *moved, uint64_t n, uint32_t *counts, uint32_t *err,
                hipStream_t st);
void keep_write(const int2 *pairs, uint64_t m, const uint32_t *moved, uint64_t n, const uint64_t *offs, int2 *out,
                uint32_t *err, hipStream_t st);
// Query share k of S: out = {b0, b1, u0, u1, c0, c1}, the batch range [b0, b1)
// cut where the candidate prefix boff crosses k/S and (k+1)/S of the total,
// its unit range (uoff) and candidate range (boff).  One thread.
void shard_cut(const uint64_t *boff, const uint64_t *uoff, uint64_t nb, uint32_t S, uint32_t k, uint64_t *out,
               hipStream_t st);
void unit_batch_fill(const uint64_t *unit_off, uint64_t nb, uint64_t n_units, uint32_t *unit_batch,
                     hipStream_t st);

// a5 / a7 / a8: the band query.  count: edges per unit into unit_edges,
// stats[0] += rechecks, stats[1] += filter/FP64 disagreements (exhaustive).
// emit: pairs at unit_off_edges[u].
// Per-unit walk descriptor (written with the unit keys, read by the count
// pass): the unit's batch, first slab of the batch, slab segments met, and
// flattened candidate range [r0, r1) within the batch.
struct UnitDesc {
    uint32_t b, jmin, segmask, pad;
    uint64_t r0, r1;
};

struct QueryArgs {
    rhgd::Geo geo;
    const uint2 *win;
    const uint64_t *batch_cand;
    const uint64_t *batch_slab_off;  // per batch, B+1 flattened slab segment offsets
    const uint64_t *unit_off;   // per batch, first unit (exclusive scan of units)
    const uint32_t *unit_batch;
    const uint32_t *unit_order;    // execution order of units (sector-sorted), or null
    uint64_t n_units;              // units executed: global ids unit_base .. unit_base + n_units - 1
    uint64_t unit_base;            // (a query share runs a contiguous range of the units)
    UnitDesc *udesc;               // per unit from unit_base (with the unit order), or null
    uint32_t *unit_edges;          // count: edges per unit
    unsigned long long *bits;      // count -> emit: BITMAP_WORDS words of decisions per unit
    const uint64_t *unit_edge_off; // emit
    int2 *out;                     // emit
    uint64_t out_capacity;         // emit: pairs available at out
    unsigned long long *stats;     // count: [rechecks, disagreements]
    int exhaustive;
};
void query_count(const QueryArgs &a, int fp32, hipStream_t st);
// Sector-sorted execution order of the units into id (key/key_tmp/id_tmp: n_units each).
void unit_order(const QueryArgs &a, uint32_t *key, uint32_t *id, uint32_t *key_tmp, uint32_t *id_tmp,
                void *sort_scratch, hipStream_t st);
void query_emit(const QueryArgs &a, int fp32, hipStream_t st);

// One-launch generation of small requests: one workgroup per descriptor.
// The host fills src, the static geometry (n, B, R, K, Kw, FP32 thresholds,
// slab constants), fp32, key_bits and the scratch pointers with their
// capacities (stats zeroed); the device writes one SmallResult per request.
// status: 0 done, 1 scratch too small (rerun on the multi-launch path),
// 2 output pool full (same).
struct SmallDesc {
    rhgd::Source src;
    rhgd::Geo geo;
    int fp32, key_bits;
    uint32_t *keys, *vals, *keys2, *vals2;
    double *th;
    double2 *epm, *hsc;
    float2 *f32;
    uint32_t *btab;
    uint64_t btab_cap;
    uint2 *win;
    uint64_t win_cap;
    uint64_t *bcand, *boff, *nunits, *uoff, *bsoff;
    uint32_t *ubatch, *uedges;
    uint64_t *ueoff;
    unsigned long long *bits;
    uint64_t unit_cap;
    unsigned long long *stats;  // [rechecks, disagreements], zero at launch
    QueryArgs *qa;              // spread launch only: the request's query arguments (device, written there)
};
struct SmallResult {
    uint64_t m, candidates, windows, out_off, rechecks;
    uint64_t units;  // spread launch: the request's work units (valid with status 0 after its first kernel)
    int status;
};
void small_group(const SmallDesc *descs, SmallResult *results, int count, int2 *pool,
                 unsigned long long *pool_used, uint64_t pool_cap, hipStream_t st);
// The same group in seven launches with no host step in between: the keys
// of all the group's points spread across the chip (a0, a2), one workgroup
// per request for the sort, slab starts and bucket index (a3), the table
// rows and window plan of all the group's batches spread across the chip
// (a1, a4), one workgroup per request for the batch and unit scans, the
// count pass over the group's units spread across the chip, one workgroup
// per request for the edge scan and pool reservation, and the emit pass
// spread across the chip.  count <= SMALL_GROUP_MAX; every descriptor's qa
// set.
constexpr int SMALL_GROUP_MAX = 128;
void small_group_spread(const SmallDesc *descs, SmallResult *results, int count, int2 *pool,
                        unsigned long long *pool_used, uint64_t pool_cap, hipStream_t st);

}  // namespace rhgk
