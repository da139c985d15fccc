// Internal declarations shared by the HIP translation units of libnbreg.
// Not part of the public ABI (that is include/nbreg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nb {

// Work-group shape of every force kernel: 256 lanes = 4 wave64s.
constexpr int kBlock = 256;
constexpr int kWave = 64;
// j bodies staged per LDS tile by the row-per-lane kernel.
constexpr int kTile = 256;
// Mixed precision: FP32 partial sums run over this many j before they are
// folded into the FP64 running sums.
constexpr int kFold = 32;
// Capacity of one split's neighbour segment in scratch.  A segment that
// overflows is rebuilt by the merge kernel from its j-range.
constexpr int kSegCap = 96;

// Position used for padding bodies in a partial LDS tile / past the end of a
// j-range: far away (finite in FP32 after the FP64 difference), mass 0, so the
// pair adds exactly zero and never passes the neighbour test.
constexpr double kFar = 1.0e18;

// Status bits (mirrors include/nbreg.h).
constexpr uint32_t kStOverflow = 1u, kStBadIndex = 2u, kStNonFinite = 4u;

// A contiguous range of j-set bodies [j_begin, j_end) and the rows that see it.
struct ForceArgs {
    int64_t n;            // bodies in the whole concatenated arrays (plane stride)
    const double *xp;     // [3][n]
    const double *vp;     // [3][n]
    const double *m;      // [n]
    int32_t n_i;          // rows (plane stride of per-row arrays)
    const int32_t *i_block;
    const double *rs2;
    int32_t cap;          // caller's nb_cap
    // final outputs (used directly when splits == 1)
    double *acc, *jerk;   // [3][n_i]
    int32_t *nb_count, *nb_list;
    int32_t *overflow;
    uint32_t *status;
    // words the force kernel zeroes as it starts (null: none).  Set only for
    // split launches, whose force kernel writes neither the overflow word nor
    // the refinement counter (the merge does), so no separate clearing launch
    // is needed.
    int32_t *clear0, *clear1;
    // split layout: split s covers j in [s * split_len, min(n, (s+1) * split_len))
    int32_t splits;
    int64_t split_len;
    // scratch (splits > 1): one slot per (row, split), slot = b * splits + split;
    // part [total_slots][kSlotComp], seg_cnt [total_slots],
    // seg_list [total_slots][kSegCap]
    int64_t total_slots;
    double *part;
    int32_t *seg_cnt;
    int32_t *seg_list;
    // mixed precision: rows whose estimated error is too large are appended
    // (row, j-range) to the redo list and recomputed in FP64 afterwards
    double redo_k;        // 2^-24 * safety / tolerance; 0 disables
    int32_t *redo_count;  // device counter, zeroed before the force kernel
    int32_t *redo_arrive; // work-groups done with the first refinement pass;
                          // zero between calls (the last arrival resets it)
    int32_t *redo_rows;   // [n_i]
    int32_t *redo_j0, *redo_j1;
    float near_factor;    // mixed: FP64 near field below near_factor * rs2
    int32_t redo_groups;  // work-groups of the refinement kernel
    int32_t redo_chunks;  // chunks per refined row (j-range / kRedoChunk, rounded up)
    int32_t redo_rcap;    // rows refined through the chunk-partials buffer
    double *redo_part;    // [redo_rcap][redo_chunks][6] chunk partials
};

// Refinement works on fixed chunks of kRedoChunk bodies so that a refined
// row's FP64 sum does not depend on how many rows were refined in the call.
constexpr int64_t kRedoChunk = 8192;
constexpr int64_t kRedoPartItems = int64_t(1) << 20;   // chunk partials held at most

// Components per slot: acc x,y,z, jerk x,y,z, and the two error-scale sums.
constexpr int kSlotComp = 8;
// Extra scratch for the redo list of n_i rows (row / j-range arrays and the
// chunk partials); the counter is a separate word owned by the caller, so
// that it outlives later reuse of the scratch.
int32_t redo_groups_for(int cu_count);
// max_len: longest j-range of any row of the launch.  rcap_limit > 0 bounds
// the rows summed through chunk partials (the others are summed one
// work-group per row, to the same bits), and with it the partials' bytes.
size_t redo_scratch_bytes(int32_t n_i, int64_t max_len, int32_t rcap_limit = 0);
void bind_redo_scratch(ForceArgs &a, void *base, int32_t *counter, int32_t groups,
                       int64_t max_len, int32_t rcap_limit = 0);
hipError_t launch_redo(const ForceArgs &a, hipStream_t s);

struct Plan {
    int mapping;        // 1 = row per lane (LDS j-tiles), 2 = row group per wave
    int rows_per_lane;  // mapping 1: 1, 2, 4;  mapping 2: rows per wave 1, 2, 4
    int splits;         // j-ranges (mapping 1: per work-group; mapping 2: per wave)
    int f64;            // 1: a mixed-precision request runs the FP64 kernels
};

// Scratch bytes needed for a plan (0 when splits == 1).
size_t force_scratch_bytes(const Plan &p, int32_t n_i);
// Scratch bytes for 'slots' split slots, and binding of the slot arrays.
size_t slot_scratch_bytes(int64_t slots);
void bind_slot_scratch(ForceArgs &a, int64_t slots, void *base);
// Carves the scratch pointers of 'a' out of 'base'.
void force_bind_scratch(ForceArgs &a, void *base);

// Launchers (return hipError_t of the launch).
hipError_t launch_force(const Plan &p, bool mixed, const ForceArgs &a, hipStream_t s);
hipError_t launch_merge(bool mixed, const ForceArgs &a, hipStream_t s);
hipError_t launch_predict(int64_t n, double t, const double *x, const double *v,
                          const double *a, const double *jrk, const double *t0,
                          const double *m, double *xp, double *vp, float *m32,
                          hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s);
// Zeroes *a and, if b is not null, *b in one launch.
hipError_t launch_clear_words(int32_t *a, int32_t *b, hipStream_t s);

// Adjoint: two recompute passes.
struct AdjointArgs {
    int64_t n;
    const double *xp, *vp, *m;
    int32_t n_i;
    const int32_t *i_block;
    const double *rs2;
    const double *w_a, *w_j;  // [3][n_i]
    double *gx, *gv, *gm;     // [3][n], [n]
    uint32_t *status;
    double *row_part;         // scratch [6][n_i]: per-row "-" terms (set by the launcher)
};
size_t adjoint_scratch_bytes(int64_t n, int32_t n_i, int row_splits, int body_splits);
hipError_t launch_adjoint_plan(const AdjointArgs &a, int row_splits, int body_splits,
                               void *scratch, hipStream_t s);

// Batched ensemble: clusters of the concatenated arrays.
struct BCluster {
    int64_t j_begin, j_end;   // bodies of the cluster
    int64_t split_len;        // j per split
    int64_t slot_base;        // first slot of the cluster (splits > 1 only)
    int32_t row_begin;        // rows of the cluster
    int32_t n_rows;
    int32_t splits;
    float near;               // mixed: near-field factor of this cluster
};
struct BItem {
    int32_t cluster;
    int32_t row0;             // first row of the item's row tile
    int32_t split;
    int32_t pad;
};
struct BatchArgs {
    ForceArgs f;              // n, arrays, outputs, total_slots/part/seg_*
    const BCluster *clusters;
    const BItem *items;
    int32_t n_items;
    int32_t *queue;           // work counter, zeroed before each launch
    const int32_t *merge_rows;   // rows of clusters with splits > 1
    const int32_t *row_cluster;  // cluster of each merge row
    int32_t n_merge_rows;
    int32_t max_splits;          // largest split count of any cluster
};
// Shapes the batched kernel is built for: LDS tile length (j bodies per
// tile), work-group lanes, and rows per lane (a row tile is lanes x rows).
struct BShape {
    int tile;
    int lanes;
    int rows_per_lane;
};
constexpr int kBatchedShapes = 6;
constexpr BShape kBatchedShape[kBatchedShapes] = {
    {256, 256, 1}, {256, 256, 2}, {128, 128, 1}, {64, 64, 1}, {512, 512, 1}, {256, 512, 1}};
// j-splits of the batched ensemble are multiples of this many bodies, for
// every shape, so a cluster's split boundaries (and so its sums) depend only
// on its split count.
constexpr int kSplitUnit = 256;
// Index of a shape in kBatchedShape, or -1.
int batched_shape_index(int tile, int lanes, int rows_per_lane);
hipError_t launch_batched(bool mixed, int shape, int grid, const BatchArgs &a, hipStream_t s);
hipError_t launch_batched_merge(const BatchArgs &a, hipStream_t s);
int batched_max_blocks_per_cu(bool mixed, int shape);

}  // namespace nb
