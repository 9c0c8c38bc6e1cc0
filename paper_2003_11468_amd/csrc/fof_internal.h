// Internal types shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fof.h"

namespace fof {

// The edge list is split into slices with a counter each, so that no single
// address takes every append.
constexpr int kEdgeSlices = 256;

// Per-box parameters as the kernels see them (one entry per box).
struct BoxDev {
    int64_t p0, p1;       // particle range [p0, p1): input and sorted order use the same range
    int64_t cell_base;    // first global cell index of the box
    int32_t nc;           // cells per axis (>= 3)
    int32_t use_fp64;     // 1: this box is decided in double for every candidate pair
    double L;             // box side
    double half;          // L / 2
    double inv_h;         // nc / L
    double l2;            // l_x * l_x, rounded once
    float L32;            // L as FP32 (equal to L whenever the FP32 filter is used)
    float lo32;           // FP32 r2 below this: linked (proven)
    float hi32;           // FP32 r2 above this: not linked (proven)
    int32_t sub_k;        // sub-cells per cell axis whose diagonal is below l_x (0: none used)
    int32_t sub_adj;      // 1: any two points of two touching sub-cells are linked too
};

// Device counters (one block of the workspace, cleared by every build).
struct Counters {
    unsigned long long pair_tests;
    unsigned long long links;
    unsigned long long band_hits;
    unsigned long long cas_retries;
    unsigned long long sparse_tests;   // pair tests of the per-lane (sparse) search
    unsigned int error;         // bit 0: coordinate outside [0, L) or not finite; bit 1: sort inconsistency
    unsigned int n_items;       // work items of the dense link kernel
    unsigned int n_edges;       // linked pairs queued for the union kernel (summed after the search)
    unsigned int n_boundary;    // domain mode: linked pairs across domains (may exceed the list's capacity)
    unsigned int n_bgroups;     // domain mode: distinct local groups met by those pairs
    unsigned int depth_max;     // stats: longest path to a root before the flatten
    int giant;                  // giant-component skip: a node of the largest group in the sample
    unsigned long long depth_sum;   // stats: sum of those path lengths
};

// Everything a launch needs: raw pointers into the caller's workspace.
struct Plan {
    int64_t n;              // particles over all boxes
    int64_t n_cells;        // cells over all boxes
    int32_t n_boxes;
    int32_t predicate;      // 0 fp64, 1 fp32 filter
    int32_t strict;         // 1: r2 < l2
    int32_t stats;          // 1: count pair tests etc.
    int64_t scan_tiles;     // scratch ints for the tile sums of the scans
    int64_t n_tiles;        // input tiles of the bucket pass (2048 particles each)
    int32_t bucket_shift;   // bucket of a cell = cell >> bucket_shift
    int32_t n_buckets;      // at most 256
    int32_t seg_shift;      // segment of a cell = cell >> seg_shift (6..16; a segment's counts fit in LDS)
    int32_t sub_log2;       // segments per bucket = 1 << sub_log2 (bucket_shift - seg_shift, at most 10)
    int64_t n_segments;     // ceil(n_cells / 2^seg_shift)
    int32_t dense_min;      // cells with at least this many particles use the wave kernel
    int32_t dense_blocks;   // grid of the persistent dense link kernel
    int32_t sparse_blocks;  // grid of the persistent sparse link kernel
    int32_t domains;        // > 1: slabs along x, local union-find per slab, then a global merge
    int32_t link_random;    // 1: roots hook by a pseudo-random priority of the index, not the index
    int32_t premerge;       // 1: dense cells are pre-merged by sub-cells before the wavefront search
    int32_t find_mode;      // 0: finds halve paths; 1: a path of length >= 2 is compressed onto its root
    int32_t giant_skip;     // 1: Afforest-style linking (sampled axis links, then the rest skipping the
                            // largest group found)
    int32_t sample;         // set for the first pass of giant_skip: axis-neighbour cells only
    int32_t tile_join;      // 1: the per-particle search joins the links inside its 64-particle tiles
    int64_t max_items;      // capacity of `items`
    int64_t max_edges;      // capacity of `edges`: kEdgeSlices slices of max_edges / kEdgeSlices

    BoxDev box0;            // the box itself when n_boxes == 1 (no table read)
    const float *pos;       // [n][3] input
    const BoxDev *boxes;    // [n_boxes] (read only when n_boxes > 1)
    const int64_t *box_p0;  // [n_boxes + 1] particle offsets

    int32_t *cstart;        // [n + 4] first sorted slot of each occupied cell, by rank (see occ);
                            // entries n .. n + 3 hold n
    int32_t *seg_end;       // [n_segments] counts, exclusive prefix, then (after the segment pass) end slots
    int32_t *scan_part;     // [scan_tiles] tile sums of every scan level
    int32_t *bucket_hist;   // [n_buckets * n_tiles + 1] counts, then output offsets (bucket-major);
                            // the group catalogue reuses it for its tile counts
    float4 *staging;        // [n] bucket order: x, y, z, original index (bits); after resolve: {label, size}
    int32_t *stpos;         // [n] staging slot of input particle i
    float4 *staging2;       // [n] segment order (cells of a segment together, unordered inside)
    int32_t *stage2_k;      // [n] staging slot of each segment-order slot
    uint2 *occ;             // [n_segments << (seg_shift - 5) + 2] per 32 cells: .x bit k: cell 32w + k
                            // holds a particle; .y the cstart index of the first occupied cell at or
                            // after cell 32w. Cell c starts at sorted slot
                            // cstart[occ[c/32].y + (occupied cells of that word below c)]
    int32_t *wave_roots;    // [n_waves] roots among the 64 sorted slots of each wave (resolve)
    unsigned long long *tile_dense;   // [n_waves] bit l: sorted slot 64 w + l lies in a dense cell
    int64_t n_waves;
    int32_t *kmap;          // [n] staging slot of each sorted slot
    float4 *sorted;         // [n] cell-sorted x, y, z
    int32_t *orig;          // [n] original index of sorted particle s
    int32_t *gmin;          // [n] smallest original index of the group, at its root
    int32_t *parent;        // [n] union-find forest over sorted indices
    int32_t *gsize;         // [n] group member count at roots (sorted indices)
    int4 *items;            // [max_items] dense work: {cx | cy << 16, first home particle, box, cz}
    int2 *edges;            // [max_edges] linked pairs found by the sparse search
    int2 *bnd;              // domain mode: [max_edges] linked pairs across domains, then their root pairs
    unsigned int *edge_fill;   // [kEdgeSlices] pairs appended to each slice (may exceed its capacity)
    unsigned long long *n_groups;  // [n_boxes]
    Counters *counters;

    int32_t *label;         // [n] output, input order
    int32_t *size;          // [n] output, input order
};

// Scratch ints the scans of `len` values need, and input tiles of the bucket
// pass (fof_kernels.hip).
int64_t scan_scratch_for(int64_t len);
int64_t sort_tiles_for(int64_t n);

// Cells per segment of the in-LDS cell sort: 2^kSegLog2Min .. 2^kSegLog2Max;
// segments per bucket at most 2^kMaxSubLog2.
constexpr int kSegLog2Min = 6;
constexpr int kSegLog2Max = 16;
constexpr int kSegLog2Auto = 16;      // largest segment the automatic choice takes
constexpr int kSegTarget = 1365;      // default: about this many particles per segment
constexpr int kMaxSubLog2 = 10;

// Capacity of the dense work-item list (fof_link.hip).
int64_t max_dense_items(int64_t n, int dense_min);

// Kernels in launch order; the ids index per-kernel timings.
enum KernelId {
    K_CLEAR, K_BUCKET_HIST, K_BUCKET_SCAN, K_BUCKET_SCATTER, K_SEG_HIST, K_SEG_SCAN, K_SEG_SCATTER, K_CELL_SORT,
    K_LINK_SPARSE, K_UNION_EDGES, K_PREMERGE, K_LINK_DENSE, K_FLATTEN, K_RESOLVE, K_GATHER, K_COUNT_KERNELS
};
const char *kernel_name(int k);

// Optional hook around every launch (records HIP events on the launch stream).
struct KernelTimer {
    virtual void mark(int kernel, bool end, hipStream_t stream) = 0;
    virtual ~KernelTimer() = default;
};

// Kernel launchers (fof_kernels.hip, fof_link.hip). All enqueue on `stream`;
// `t` may be null.
hipError_t launch_clear(const Plan &p, hipStream_t stream, KernelTimer *t);
hipError_t launch_build(const Plan &p, hipStream_t stream, KernelTimer *t);
// A second stream onto which the link phase may fork a kernel that is
// independent of the others, with the events of the fork and of the join
// (all null: every kernel on `stream`).
struct Fork {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t launch_link(const Plan &p, hipStream_t stream, KernelTimer *t, const Fork *fk = nullptr);
// A fresh forest over the built cells (fof_kernels.hip): parent, sizes, group
// minima and the per-run counters reset, cells and dense work items kept.
hipError_t launch_relink_reset(const Plan &p, hipStream_t stream);
// Exclusive prefix sum of data[0, len) in place (fof_kernels.hip); scratch
// holds scan_scratch_for(len) ints.
void scan_exclusive(int *data, int64_t len, int *scratch, hipStream_t stream);
hipError_t launch_finalize(const Plan &p, hipStream_t stream, KernelTimer *t);
// Groups of at least min_size members (fof_kernels.hip); the total is left in
// p.bucket_hist[p.n_tiles].
hipError_t launch_catalogue(const Plan &p, const int32_t *label, const int32_t *size, int min_size,
                            int32_t *g_first, int32_t *g_size, int32_t *g_box, int64_t capacity, hipStream_t stream);

// One box of n particles on a workspace chosen by the caller (fof_api.cpp):
// validates the options and the box like fof_workspace_bytes, returns in
// *need the bytes the run needs and, when they fit in `bytes`, fills *out
// with the launch parameters (positions and outputs left unset).
fof_status plan_one_box(const fof_options &o, int64_t n, double box, double lx, void *ws, size_t bytes, Plan *out,
                        size_t *need);

}  // namespace fof
