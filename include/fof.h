/*
 * fof.h - periodic Friends-of-Friends group labelling on one AMD Instinct
 * MI355X (gfx950).
 *
 * Operation (paper, Section 1 footnote): the groups are the connected
 * components of the graph whose edges join every pair of particles at most
 * l_x apart. Distances are periodic minimum-image distances in a cubic box of
 * side L. Each group is labelled with its smallest particle index, the label a
 * union-by-root forest produces when the larger root always points to the
 * smaller one and roots start at the particle's own offset (Section 2,
 * Section 3.1). Group sizes are counted at the root (Section 3.4.1).
 *
 * Link predicate (fixed here because the paper does not print it): for FP32
 * coordinates promoted exactly to double, per axis t = a - b, then t -= L if
 * t > L/2 and t += L if t < -L/2; r2 = (tx*tx + ty*ty) + tz*tz, every
 * operation rounded to nearest in double with no fused multiply-add; the pair
 * is linked iff r2 <= l_x*l_x (or r2 < l_x*l_x with fof_options.strict_less).
 * FOF_PRED_FP32_FILTER decides almost every pair in FP32 and re-decides in
 * double only the pairs inside a proven rounding band around l_x^2, so both
 * predicates give exactly the same groups.
 *
 * Pipeline: fof_build_cells (bin particles into cells of side >= l_x with a
 * counting sort), fof_link (cell-pair link search plus lock-free union-find:
 * find with path halving, a compare-and-swap that hooks the larger root under
 * the smaller, Section 3.2), fof_finalize (flatten the forest, relabel to the
 * smallest original index, count group sizes).
 *
 * Conventions
 *  - All device pointers are HIP device memory on the context's device. The
 *    caller owns the positions, the outputs and the workspace; the library
 *    owns only the context and two small pinned staging buffers.
 *  - build/link/finalize enqueue work on the context's stream and return
 *    without waiting, except where a host output pointer is given. A
 *    multi-box build (or relink) copies its box table to the workspace through
 *    one of two pinned host staging buffers used in turn: refilling one waits
 *    only for that buffer's previous copy (two uploads back), and a buffer is
 *    (re)allocated -- pinned host memory, never device memory -- only when a
 *    larger table than any before comes along.
 *  - build/link/finalize allocate no device memory.
 *  - Host-detectable errors return before any device work is enqueued. A
 *    coordinate that is not finite or lies outside [0, L) is detected on the
 *    device, latched, and returned by the next synchronising call
 *    (fof_finalize with a non-NULL h_n_groups, fof_read_n_groups,
 *    fof_get_stats); the outputs of that run are then undefined.
 *  - No C++ exception crosses this interface.
 *  - Boxes: n_boxes >= 1 independent periodic boxes are processed together.
 *    Box k holds particles h_box_offsets[k] .. h_box_offsets[k+1]-1 of the
 *    position array, with side h_box[k] and linking length h_lx[k]. Labels
 *    are box-local indices. n_boxes = 1 is the plain single-box problem.
 */
#ifndef FOF_H
#define FOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fof_ctx fof_ctx;

typedef enum {
    FOF_OK = 0,
    FOF_ERR_INVALID_ARG = 1,   /* null pointer, bad count, bad box or linking length */
    FOF_ERR_OUT_OF_BOX = 2,    /* a coordinate not finite or outside [0, L) (latched on the device) */
    FOF_ERR_BAD_STATE = 3,     /* calls out of order (link before build, finalize before link) */
    FOF_ERR_WORKSPACE = 4,     /* workspace missing, too small or misaligned */
    FOF_ERR_DEVICE = 5,        /* a HIP runtime call failed, or a device-side consistency check */
    FOF_ERR_UNSUPPORTED = 6    /* valid request the library cannot serve (e.g. too many cells) */
} fof_status;

typedef enum {
    FOF_PRED_FP64 = 0,         /* every candidate pair decided with the double predicate */
    FOF_PRED_FP32_FILTER = 1   /* FP32 decision, double re-decision inside the rounding band */
} fof_predicate;

typedef struct {
    int32_t predicate;       /* fof_predicate */
    int32_t strict_less;     /* 0: link iff r2 <= l2 (default); 1: r2 < l2 */
    double cell_factor;      /* cell side in units of l_x (>= 1); 0 picks cells of about one
                                particle each, never narrower than l_x */
    int32_t collect_stats;   /* 1: count pair tests, links, band hits, CAS retries (slower) */
    int32_t dense_min;       /* cells holding at least this many particles are searched by whole
                                wavefronts (64 particles against broadcast candidates); the others
                                per particle. 0 = default (32) */
    int32_t collect_timings; /* 1: record HIP events around every kernel launch on the context's
                                stream (read with fof_get_kernel_times) */
    int32_t sort_segment_log2; /* the cell sort takes 2^k consecutive cells per work-group (their
                                occupancy bits and the counts of the occupied cells in on-chip
                                memory): k in 6..16; 0 = automatic (about 1.4k particles per
                                work-group on average). Changes speed only */
    int32_t domains;         /* > 1: domain-decomposed merge on one GPU (paper, Section 3.3): every box
                                is cut into this many slabs along x; union-find runs on the links
                                inside each slab, links across slabs are collected, their groups are
                                numbered densely and merged by a second union-find, and the roots are
                                updated. Same labels as without; at most 4096. 0 or 1 = off */
    int32_t link_order;      /* which root a merge hooks under the other (paper, Section 3.2):
                                0 = by index, the larger under the smaller (default);
                                1 = randomised linking: by a fixed pseudo-random priority of the index
                                (a bijection), a contention variant. Same labels either way: the label
                                is the smallest original index of the group, whatever its root */
    int32_t schedule;        /* work schedule of the link pass, bit fields (0 = defaults; changes speed only):
                                bits 0-1: work-groups of the per-particle search (1024, 512, 2048, 4096);
                                bits 2-3: work-groups of the wavefront search (2048, 1024, 4096, 8192);
                                bit 4: no sub-cell pre-merge of dense cells (see fof_box_info);
                                bit 5: giant-component skip (a contention variant in the manner of
                                Afforest, Sutton et al. 2018): the per-particle search first links each
                                particle to its three axis-neighbour cells only, the largest group is
                                found from a sample of 4096 roots, then the full periodic shell is
                                searched, both ways, from the particles outside that group alone (pairs
                                inside it are never visited). Pays off when one group spans most of the
                                box; not with domains > 1;
                                bit 6: the per-particle search does not join the links inside its tiles
                                of 64 consecutive particles (by default it does, in a bit matrix, and
                                only the links between tiles go to the union pass) */
    int32_t compression;     /* path compression of the finds (paper, Section 3.4.3): 0 = path halving
                                (each visited node re-pointed to its grandparent; default); 1 = a path is
                                compressed onto its root only when it is at least 2 long. Same labels */
    int32_t reserved[2];     /* must be zero */
} fof_options;

typedef struct {
    int64_t n_particles;     /* particles in the last build */
    int64_t n_cells;         /* cells over all boxes */
    int64_t n_groups;        /* groups over all boxes (after finalize) */
    int64_t pair_tests;      /* candidate pairs tested        (collect_stats only) */
    int64_t links;           /* pairs found linked            (collect_stats only) */
    int64_t band_hits;       /* FP32 results inside the band  (collect_stats only) */
    int64_t cas_retries;     /* failed compare-and-swaps      (collect_stats only) */
    int64_t fp64_boxes;      /* boxes the FP32 filter could not serve (decided in double) */
    int64_t sparse_pair_tests; /* of pair_tests, those made by the per-particle search (collect_stats only) */
    int64_t queued_links;    /* linked pairs queued for the deferred union pass */
    int64_t dense_items;     /* wavefront work items (64 particles of a dense cell each) */
    int64_t boundary_links;  /* domain mode: linked pairs across slabs (the exchanged link list) */
    int64_t boundary_groups; /* domain mode: distinct slab-local groups in that list */
    int64_t find_depth_max;  /* longest path to a root when linking ends (collect_stats only) */
    int64_t find_depth_sum;  /* sum over particles of their path length to the root (collect_stats
                                only; mean depth = find_depth_sum / n_particles) */
    int64_t reserved[1];
} fof_stats;

/* Geometry and FP32 decision thresholds the library uses for one box. */
typedef struct {
    int64_t cells_per_axis;  /* n_c: cells of side L / n_c per axis */
    double l2;               /* l_x * l_x, rounded once (the double predicate's threshold) */
    float lo32;              /* FP32 squared distance below this: linked, proven */
    float hi32;              /* FP32 squared distance above this: not linked, proven */
    int32_t fp64_only;       /* 1: the FP32 filter cannot be proven for this box; every pair is
                                decided in double */
    int32_t sub_cells_per_axis; /* k: dense cells are pre-merged by k^3 sub-cells whose diagonal is
                                at most l_x (1 - 1e-6); 0 = no pre-merge */
    int32_t sub_cells_adjacent; /* 1: the sub-cells are small enough (2 sqrt(3) s <= l_x (1 - 1e-6),
                                s their side) that any two points of two touching sub-cells are
                                linked, and touching occupied sub-cells are merged too */
    int32_t reserved[1];
} fof_box_info;

/* Re-links the particles of the last successful fof_build_cells with new
 * linking lengths h_lx[0 .. n_boxes-1] (one per box, as many boxes as that
 * build) without rebuilding the cells, as an on-the-fly group finder inside
 * a simulation would reuse its cell structure (paper, Section 1). Each new
 * l_x must be at most the l_x the cells were built for (the cells stay at
 * least l_x (1 + 2^-20) wide); the FP32 thresholds are recomputed. Allowed
 * after fof_build_cells, fof_link or fof_finalize; resets the forest, after
 * which fof_link and fof_finalize run as usual. Enqueues on the context's
 * stream. Errors: FOF_ERR_INVALID_ARG (null, count differs from the build, an
 * l_x not positive or larger than the build's), FOF_ERR_BAD_STATE (no
 * successful build on this context), FOF_ERR_DEVICE. */
fof_status fof_relink(fof_ctx *ctx, const double *h_lx, int32_t n_boxes);

/* Group catalogue (the step after labelling; the paper's group-size pass,
 * Section 3.4.1-3.4.2, and its catalogue of groups above a size cut): the
 * groups of at least `min_size` members of the outputs of the last
 * fof_finalize on this context (`d_group_index`, `d_group_size`, same
 * particles and boxes), in order of box and label. For group g:
 * d_first[g] = its label (smallest box-local member index), d_size[g] = its
 * member count, d_box[g] = its box (d_box may be NULL). At most `capacity`
 * entries are written (capacity 0 counts only); *h_count receives the number
 * of groups selected, which may exceed capacity. Device arrays are int32 and
 * caller-owned. Enqueues on the context's stream and waits for it.
 * Errors: FOF_ERR_INVALID_ARG (null pointer, min_size < 1, capacity < 0),
 * FOF_ERR_BAD_STATE (no build on this context), FOF_ERR_DEVICE. */
fof_status fof_catalogue(fof_ctx *ctx, const int32_t *d_group_index, const int32_t *d_group_size, int32_t min_size,
                         int32_t *d_first, int32_t *d_size, int32_t *d_box, int64_t capacity, int64_t *h_count);

/* Host only: the cell count per axis and FP32 thresholds for a box of
 * `n_particles` particles, side `box` and linking length `lx` under options
 * `opt` (NULL = defaults). Same validation as fof_workspace_bytes. */
fof_status fof_describe_box(const fof_options *opt, int64_t n_particles, double box, double lx, fof_box_info *out);

/* Fills *opt with the defaults: FP32 filter, r2 <= l2, automatic cells, no stats. */
void fof_default_options(fof_options *opt);

/* Creates a context bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the null stream). `opt` may be NULL for defaults.
 * Errors: FOF_ERR_INVALID_ARG (null out, bad option), FOF_ERR_DEVICE. */
fof_status fof_create(fof_ctx **out, const fof_options *opt, void *hip_stream);

/* Re-binds the context to another stream of the same device. */
fof_status fof_set_stream(fof_ctx *ctx, void *hip_stream);

/* Host only, touches no device memory: validates the box description and
 * returns in *bytes the workspace the following fof_build_cells needs.
 * h_box_offsets has n_boxes + 1 non-decreasing entries starting at 0; the
 * total count must be below 2^31. Each box needs L > 0 finite, 0 < l_x and at
 * least 3 cells of side >= l_x (1 + 2^-20) per axis (so l_x < L / 3).
 * Errors: FOF_ERR_INVALID_ARG, FOF_ERR_UNSUPPORTED (a box of more than 2048
 * cells per axis, or more than 2^34 cells over all boxes). */
fof_status fof_workspace_bytes(fof_ctx *ctx, const int64_t *h_box_offsets, const double *h_box,
                               const double *h_lx, int32_t n_boxes, size_t *bytes);

/* Hands the library a device workspace of `bytes` bytes (256-byte aligned),
 * owned by the caller and kept alive until the context is destroyed or another
 * workspace is set. Setting a different (or smaller) workspace discards the
 * captured graph, whose kernels point into the old one. */
fof_status fof_set_workspace(fof_ctx *ctx, void *d_ws, size_t bytes);

/* Bins the particles into cells (Section 3.1: only cells within l_x of each
 * other are searched; cells as wide as the linking length work best).
 * d_pos: [n_total][3] FP32, x y z interleaved, on the device, read only; it
 * must stay unchanged until fof_link has run. Validates like
 * fof_workspace_bytes, then checks the workspace (FOF_ERR_WORKSPACE). */
fof_status fof_build_cells(fof_ctx *ctx, const float *d_pos, const int64_t *h_box_offsets,
                           const double *h_box, const double *h_lx, int32_t n_boxes);

/* Finds every linked pair among each cell and its 13 half-shell neighbour
 * cells and merges their groups with lock-free union-find (Section 3.2,
 * Listing 2, with the compare-and-swap expecting the root value found by the
 * find). Errors: FOF_ERR_BAD_STATE if no build preceded it. */
fof_status fof_link(fof_ctx *ctx);

/* Writes, for every particle i (input order), d_group_index[i] = the smallest
 * box-local index in its group, and d_group_size[i] = the group size if i is
 * that smallest index (the root), else 0 (Section 3.4). Both are [n_total]
 * int32 device arrays. If h_n_groups is not NULL it receives the number of
 * groups of each box ([n_boxes] int64, host) and the call waits for the stream;
 * a latched coordinate error is returned then. */
fof_status fof_finalize(fof_ctx *ctx, int32_t *d_group_index, int32_t *d_group_size, int64_t *h_n_groups);

/* Waits for the stream and copies the per-box group counts of the last
 * finalize (or graph launch) to h_n_groups[n_boxes]; returns a latched error. */
fof_status fof_read_n_groups(fof_ctx *ctx, int64_t *h_n_groups);

/* Waits for the stream and returns counters of the last run. */
fof_status fof_get_stats(fof_ctx *ctx, fof_stats *out);

/* Captures build + link + finalize for these exact arguments into a HIP graph
 * owned by the context (replacing any previous one). The box description is
 * planned and uploaded before capture (this call waits for the stream), so
 * the graph holds kernel launches only. d_pos, d_group_index, d_group_size
 * and the workspace must stay allocated while the graph may be replayed.
 * fof_graph_launch replays it on the context's stream; the per-box group
 * counts stay on the device (fof_read_n_groups). Inside the graph the
 * sub-cell pre-merge of dense cells runs beside the union pass of the
 * per-particle search's links (the two touch disjoint sets of particles); a
 * replay as a whole is still ordered on the context's stream.
 * A graph of several boxes reads the box table held in the workspace. Eager
 * calls on the same context may replace that table: a build of one box or of
 * another geometry, or fof_relink. fof_graph_launch then returns
 * FOF_ERR_BAD_STATE and enqueues nothing (capture again, or first build the
 * captured geometry eagerly, which puts its table back). A one-box graph
 * carries its box in the kernel arguments and stays valid. Errors of
 * fof_graph_launch: FOF_ERR_BAD_STATE (no graph, or its table replaced),
 * FOF_ERR_DEVICE. */
fof_status fof_graph_capture(fof_ctx *ctx, const float *d_pos, const int64_t *h_box_offsets,
                             const double *h_box, const double *h_lx, int32_t n_boxes,
                             int32_t *d_group_index, int32_t *d_group_size);
fof_status fof_graph_launch(fof_ctx *ctx);

/* Device scratch of fof_label_noalloc on each GPU (bytes). */
#define FOF_NOALLOC_SCRATCH_BYTES (128u << 20)

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): fof_build_cells +
 * fof_link + fof_finalize of ONE box (n particles, side `box`, linking length
 * `lx`) in one call, on a scratch array the library holds in device memory,
 * FOF_NOALLOC_SCRATCH_BYTES on each GPU it runs on (taken when the library's
 * code is loaded onto that GPU and held until the process ends), instead of a
 * caller's workspace. No context is needed and nothing is allocated: no
 * device or host memory, no events. Same kernels, same results (labels,
 * sizes, group count) as the three calls with a workspace.
 * opt: options (NULL = defaults); collect_timings must be 0; collect_stats
 * counts on the device but the counters are not readable. hip_stream: the
 * stream to enqueue on (NULL = the null stream), on the current device.
 * d_pos [n][3] FP32, d_group_index and d_group_size [n] int32: device
 * memory owned by the caller, as for the workspace path. If h_n_groups is not
 * NULL it receives the group count and the call waits for the stream (a
 * latched coordinate error is returned then); otherwise it returns after
 * enqueueing. Every call on one GPU uses that GPU's single scratch array:
 * calls that overlap in time on one GPU (other host threads, or other
 * streams before the previous call's work has finished) race and give
 * undefined results; calls ordered on one stream are safe, and each call
 * clears what it needs, whatever the previous call left.
 * Errors, all before any device work: FOF_ERR_INVALID_ARG (bad options,
 * collect_timings set, n < 0 or > 2^31 - 1, a null pointer with n > 0, bad
 * box or linking length), FOF_ERR_UNSUPPORTED (the run needs more than
 * FOF_NOALLOC_SCRATCH_BYTES -- fof_workspace_bytes gives the need for the
 * same options and box -- or too many cells); FOF_ERR_DEVICE (no device, or
 * the scratch address could not be found). */
fof_status fof_label_noalloc(const fof_options *opt, void *hip_stream, const float *d_pos, int64_t n, double box,
                             double lx, int32_t *d_group_index, int32_t *d_group_size, int64_t *h_n_groups);

/* Waits for the stream and returns, per kernel of the pipeline, the summed
 * device time (ms, from HIP events recorded around each launch on the
 * context's stream) and the number of launches since the previous call; the
 * record is then cleared. Needs fof_options.collect_timings = 1 (graph
 * replays are not recorded). h_ms and h_launches (may be NULL) hold at least
 * `capacity` entries; *n_kernels receives the number of kernels (names via
 * fof_kernel_name). At most the latest 1024 launches are kept.
 * Errors: FOF_ERR_INVALID_ARG (capacity too small), FOF_ERR_BAD_STATE
 * (timings not enabled). */
fof_status fof_get_kernel_times(fof_ctx *ctx, double *h_ms, int32_t *h_launches, int32_t capacity,
                                int32_t *n_kernels);

/* Name of kernel k of fof_get_kernel_times ("?" when out of range). */
const char *fof_kernel_name(int32_t k);

/* Releases the context, its graph and its pinned staging buffer (not the
 * caller's workspace). Waits for the stream. NULL is accepted. */
fof_status fof_destroy(fof_ctx *ctx);

/* Static description of a status code. */
const char *fof_status_string(fof_status s);

#ifdef __cplusplus
}
#endif

#endif /* FOF_H */
