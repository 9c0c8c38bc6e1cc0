// C-ABI of the gfx950 Friends-of-Friends library: argument validation, cell
// geometry, FP32 guard-band thresholds, workspace carve-up, launch sequencing
// and HIP graph capture. Every compute step runs in fof_kernels.hip.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fof.h"
#include "fof_internal.h"

namespace {

using fof::BoxDev;
using fof::Counters;
using fof::Plan;

constexpr size_t kAlign = 256;
// Cells over all boxes: 256 buckets of at most 2^kMaxSubLog2 segments of at
// most 2^kSegLog2Max cells.
constexpr int64_t kMaxCells = (int64_t)1 << (8 + fof::kMaxSubLog2 + fof::kSegLog2Max);
constexpr double kMaxCellsPerAxis = 2048.0;   // a box of 2048^3 cells is 2^33
constexpr int kMaxDomains = 4096;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Round a double to FP32 toward -inf / +inf.
float round_down_f32(double v)
{
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -INFINITY);
    return f;
}

float round_up_f32(double v)
{
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, INFINITY);
    return f;
}

// Sort levels and workspace carve-up of one run. Plain data, so the
// no-allocation entry point can build it on the stack.
struct Layout {
    int32_t n_boxes = 0;
    int64_t n = 0;
    int64_t n_cells = 0;
    int64_t scan_tiles = 0;
    int64_t n_tiles = 0;
    int32_t bucket_shift = 0, n_buckets = 1;
    int32_t seg_shift = 0, sub_log2 = 0;
    int64_t n_segments = 0;
    int64_t max_items = 0;
    int64_t max_edges = 0;
    // workspace layout (byte offsets)
    size_t o_boxes = 0, o_p0 = 0, o_counters = 0, o_groups = 0, o_cell = 0, o_part = 0, o_kmap = 0, o_sorted = 0,
           o_orig = 0, o_gmin = 0, o_parent = 0, o_gsize = 0, o_items = 0, o_edges = 0, o_hist = 0, o_staging = 0,
           o_stpos = 0, o_wave_roots = 0, o_tile_dense = 0, o_occ = 0, o_edge_fill = 0, o_seg = 0, o_staging2 = 0,
           o_stage2_k = 0, o_bnd = 0, total = 0;
};

struct HostPlan : Layout {
    int64_t fp64_boxes = 0;
    std::vector<BoxDev> boxes;
    std::vector<int64_t> p0;
    std::vector<double> lx_cells;   // linking length each box's cells were sized for

    bool same_geometry(const HostPlan &o) const
    {
        if (n_boxes != o.n_boxes || n != o.n || n_cells != o.n_cells) return false;
        if (p0 != o.p0) return false;
        return std::memcmp(boxes.data(), o.boxes.data(), sizeof(BoxDev) * boxes.size()) == 0;
    }
};

}  // namespace

// Per-kernel HIP events: a ring of (start, stop) pairs, summed and reset by
// fof_get_kernel_times. When more launches are recorded than the ring holds,
// the oldest are overwritten and not counted.
struct EventTimer final : fof::KernelTimer {
    static constexpr int kSlots = 1024;
    hipEvent_t start[kSlots] = {}, stop[kSlots] = {};
    int kernel[kSlots] = {};
    int next = 0, used = 0;
    bool ok = false;
    int pending_kernel = -1;

    bool init()
    {
        for (int k = 0; k < kSlots; ++k) {
            if (hipEventCreate(&start[k]) != hipSuccess || hipEventCreate(&stop[k]) != hipSuccess) return false;
        }
        ok = true;
        return true;
    }
    ~EventTimer() override
    {
        for (int k = 0; k < kSlots; ++k) {
            if (start[k]) (void)hipEventDestroy(start[k]);
            if (stop[k]) (void)hipEventDestroy(stop[k]);
        }
    }
    void mark(int k, bool end, hipStream_t s) override
    {
        if (!ok) return;
        if (!end) {
            kernel[next] = k;
            (void)hipEventRecord(start[next], s);
        } else {
            (void)hipEventRecord(stop[next], s);
            next = (next + 1) % kSlots;
            if (used < kSlots) ++used;
        }
    }
};

struct fof_ctx {
    fof_options opt{};
    EventTimer *timer = nullptr;
    hipStream_t stream = nullptr;
    int device = -1;

    HostPlan plan;
    bool planned = false;

    void *ws = nullptr;
    size_t ws_bytes = 0;

    // The box table currently held by the workspace: its geometry and an
    // upload number (0: none, or overwritten by a single-box run).
    HostPlan table_plan;
    uint64_t table_id = 0;
    uint64_t upload_seq = 0;

    // Pinned host staging for the box table, two buffers used in turn; the
    // event after each buffer's last copy says when it may be refilled.
    void *stage[2] = {nullptr, nullptr};
    size_t stage_bytes[2] = {0, 0};
    hipEvent_t stage_done[2] = {nullptr, nullptr};
    bool stage_pending[2] = {false, false};
    int stage_next = 0;

    int state = 0;             // 0 idle, 1 cells built, 2 linked
    bool cells_valid = false;  // the last build's cells and sorted positions are in the workspace
    Plan dev{};                // pointers of the current run

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_boxes = 0;       // boxes of the captured run
    HostPlan graph_plan;           // its geometry (a multi-box graph reads that box table)
};

namespace {

fof_status dev_err(hipError_t e) { return e == hipSuccess ? FOF_OK : FOF_ERR_DEVICE; }

bool options_valid(const fof_options &o)
{
    if (o.predicate != FOF_PRED_FP64 && o.predicate != FOF_PRED_FP32_FILTER) return false;
    if (o.strict_less != 0 && o.strict_less != 1) return false;
    if (!(o.cell_factor == 0.0 || (o.cell_factor >= 1.0 && std::isfinite(o.cell_factor)))) return false;
    if (o.collect_stats != 0 && o.collect_stats != 1) return false;
    if (o.dense_min < 0) return false;
    if (o.collect_timings != 0 && o.collect_timings != 1) return false;
    if (o.sort_segment_log2 != 0 && (o.sort_segment_log2 < fof::kSegLog2Min || o.sort_segment_log2 > fof::kSegLog2Max))
        return false;
    if (o.domains < 0 || o.domains > kMaxDomains) return false;
    if (o.link_order != 0 && o.link_order != 1) return false;
    if (o.schedule < 0 || o.schedule >= 128) return false;
    if ((o.schedule & 32) && o.domains > 1) return false;   // the giant-component skip has no domain mode
    if (o.compression != 0 && o.compression != 1) return false;
    for (int k = 0; k < 2; ++k)
        if (o.reserved[k] != 0) return false;
    return true;
}

// Cells per axis for one box: as many as the option asks for (cells of about
// one particle by default), never narrower than l_x (1 + 2^-20), at least 3.
fof_status cells_per_axis(const fof_options &o, int64_t n_box, double L, double lx, int64_t *nc_out)
{
    const double fit = std::floor(L / (lx * (1.0 + 1.0 / 1048576.0)));
    if (!(fit >= 3.0)) return FOF_ERR_INVALID_ARG;
    double want;
    if (o.cell_factor > 0.0) want = std::floor(L / (o.cell_factor * lx));
    else want = std::floor(std::cbrt((double)(n_box > 1 ? n_box : 1)) + 1e-9);
    double nc = want < fit ? want : fit;
    if (nc < 3.0) nc = 3.0;
    if (nc > kMaxCellsPerAxis) return FOF_ERR_UNSUPPORTED;
    *nc_out = (int64_t)nc;
    return FOF_OK;
}

// FP32 decision thresholds. With u = 2^-24 the FP32 squared distance R32 of a
// pair satisfies (1-u)^5 R <= R32 <= (1+u)^5 R, R being the exact squared
// minimum-image distance (one rounding per axis difference, three in the
// sum). The double predicate's value lies within E64 of R. Hence
//   R32 < lo32 = RD((l2 - E64)(1 - 8u))  =>  r2_64 < l2   (linked), and
//   R32 > hi32 = RU((l2 + E64)(1 + 8u))  =>  r2_64 > l2   (not linked).
// The filter is used only where that argument holds: L exact in FP32, l2 and
// L far from FP32 underflow and overflow.
void fp32_thresholds(BoxDev &b, double lx)
{
    const double U = DBL_EPSILON / 2.0, u = 1.0 / 16777216.0;
    const double l2 = b.l2;
    const bool ok = (double)(float)b.L == b.L && l2 >= 0x1p-100 && l2 <= 0x1p100 && b.L <= 0x1p60;
    b.use_fp64 = ok ? 0 : 1;
    b.L32 = (float)b.L;
    if (!ok) {   // every pair falls in the band: decided in double
        b.lo32 = -INFINITY;
        b.hi32 = INFINITY;
        return;
    }
    const double e = U * b.L;                       // per-axis error of the double difference
    const double g3 = 3.0 * U / (1.0 - 3.0 * U);
    const double D = e * (4.0 * std::sqrt(3.0) * lx + 3.0 * e);
    const double E64 = 2.0 * (g3 * (4.0 * l2 + D) + D);
    b.lo32 = round_down_f32((l2 - E64) * (1.0 - 8.0 * u));
    b.hi32 = round_up_f32((l2 + E64) * (1.0 + 8.0 * u));
}

constexpr int kDefaultDenseMin = 32;
constexpr int kMaxSubK = 8;              // at most 512 sub-cells per dense cell
constexpr int kDenseBlocks = 2048;
constexpr int kSparseBlocks = 1024;

// Sub-cells per cell axis for the pre-merge of dense cells, and whether they
// are "adjacent-linked". Points in one sub-cell (side s = L / (nc k)) are at
// most s sqrt(3) apart, points in two touching sub-cells (across a face, an
// edge or a corner) less than 2 s sqrt(3). With the smallest k for which
// 2 s sqrt(3) <= l_x (1 - 1e-6), any two points of touching sub-cells are
// linked under both predicates (the margin dwarfs every rounding error of the
// double predicate and of the sub-cell assignment); if that k exceeds
// kMaxSubK, the smallest k with s sqrt(3) <= l_x (1 - 1e-6) (points of one
// sub-cell linked); if that exceeds kMaxSubK too, 0 (no pre-merge).
void sub_cells(double L, int64_t nc, double lx, int32_t *k_out, int32_t *adj_out)
{
    const double side = L / (double)nc, reach = lx * (1.0 - 1e-6);
    const double k_adj = std::ceil(side * 2.0 * std::sqrt(3.0) / reach);
    const double k_one = std::ceil(side * std::sqrt(3.0) / reach);
    *adj_out = 0;
    *k_out = 0;
    if (k_adj >= 1.0 && k_adj <= (double)kMaxSubK) {
        *k_out = (int32_t)k_adj;
        *adj_out = 1;
    } else if (k_one >= 1.0 && k_one <= (double)kMaxSubK) {
        *k_out = (int32_t)k_one;
    }
}

int dense_min_of(const fof_options &o) { return o.dense_min > 0 ? o.dense_min : kDefaultDenseMin; }

// Validates one box (nb particles, side L, linking length l) and fills its
// descriptor, cells starting at global cell `cell_base`.
fof_status box_geometry(const fof_options &o, int64_t nb, double L, double l, int64_t cell_base, BoxDev *out)
{
    if (!(L > 0.0) || !std::isfinite(L) || !(l > 0.0) || !std::isfinite(l)) return FOF_ERR_INVALID_ARG;
    int64_t nc = 0;
    fof_status st = cells_per_axis(o, nb, L, l, &nc);
    if (st != FOF_OK) return st;
    BoxDev &b = *out;
    std::memset(&b, 0, sizeof(b));
    b.cell_base = cell_base;
    b.nc = (int32_t)nc;
    b.L = L;
    b.half = 0.5 * L;
    b.inv_h = (double)nc / L;
    b.l2 = l * l;
    fp32_thresholds(b, l);
    sub_cells(L, nc, l, &b.sub_k, &b.sub_adj);
    return FOF_OK;
}

// Sort levels and the workspace carve-up for n particles in `cells` cells
// over n_boxes boxes.
fof_status make_layout(const fof_options &o, int64_t n_total, int64_t cells, int32_t n_boxes, Layout *out)
{
    Layout p;
    p.n_boxes = n_boxes;
    p.n = n_total;
    p.n_cells = cells;
    // Counting sort levels: at most 256 buckets of consecutive cells, each cut
    // into 2^sub_log2 segments of 2^seg_shift cells (the cells one work-group
    // counts in LDS). A segment never exceeds a bucket.
    const int64_t last = cells > 0 ? cells - 1 : 0;
    p.bucket_shift = 0;
    while ((last >> p.bucket_shift) >= 256) ++p.bucket_shift;
    // By default a segment holds about kSegTarget particles on average (its
    // particles are then placed through LDS), within 2^6 .. 2^16 cells.
    if (o.sort_segment_log2) {
        p.seg_shift = o.sort_segment_log2;
    } else {
        const double want = (double)fof::kSegTarget * (double)(cells > 0 ? cells : 1) /
                            (double)(n_total > 0 ? n_total : 1);
        p.seg_shift = fof::kSegLog2Min;
        while (p.seg_shift < fof::kSegLog2Auto && (double)(int64_t(1) << (p.seg_shift + 1)) <= want) ++p.seg_shift;
    }
    if (p.seg_shift < p.bucket_shift - fof::kMaxSubLog2) p.seg_shift = p.bucket_shift - fof::kMaxSubLog2;
    if (p.seg_shift > fof::kSegLog2Max) return FOF_ERR_UNSUPPORTED;   // more cells than the levels hold
    if (p.bucket_shift < p.seg_shift) p.bucket_shift = p.seg_shift;
    p.sub_log2 = p.bucket_shift - p.seg_shift;
    p.n_buckets = (int32_t)((last >> p.bucket_shift) + 1);
    p.n_segments = (last >> p.seg_shift) + 1;
    p.n_tiles = fof::sort_tiles_for(n_total);
    {
        const int64_t a = fof::scan_scratch_for(p.n_segments);
        const int64_t b = fof::scan_scratch_for((int64_t)p.n_buckets * p.n_tiles);
        const int64_t t = fof::scan_scratch_for(p.n_tiles + 1);   // the group catalogue
        p.scan_tiles = a > b ? a : b;
        if (t > p.scan_tiles) p.scan_tiles = t;
        if (o.domains > 1) {   // the global merge numbers the groups of the boundary links
            const int64_t g = fof::scan_scratch_for(n_total + 1);
            if (g > p.scan_tiles) p.scan_tiles = g;
        }
    }
    if ((int64_t)p.n_buckets * p.n_tiles > (int64_t)INT32_MAX) return FOF_ERR_UNSUPPORTED;

    const size_t n = (size_t)n_total;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t here = at;
        at = align_up(at + (bytes ? bytes : 1));
        return here;
    };
    // the box table comes first: a multi-box run never writes over its own table
    p.o_boxes = take(sizeof(BoxDev) * (size_t)n_boxes);
    p.o_p0 = take(sizeof(int64_t) * ((size_t)n_boxes + 1));
    p.o_counters = take(sizeof(Counters));
    p.o_groups = take(sizeof(unsigned long long) * (size_t)n_boxes);
    p.o_cell = take(sizeof(int32_t) * (n + 4));   // starts of the occupied cells (at most n) + sentinels
    p.o_part = take(sizeof(int32_t) * (size_t)p.scan_tiles);
    p.o_kmap = take(sizeof(int32_t) * n);
    p.o_sorted = take(sizeof(float) * 4 * n);
    p.o_orig = take(sizeof(int32_t) * n);
    p.o_gmin = take(sizeof(int32_t) * n);
    p.o_parent = take(sizeof(int32_t) * n);
    p.o_gsize = take(sizeof(int32_t) * n);
    p.max_items = fof::max_dense_items(n_total, dense_min_of(o));
    p.o_items = take(sizeof(int32_t) * 4 * (size_t)p.max_items);
    // linked pairs of sparse cells, merged after the search; a pair that finds
    // the list full is merged on the spot instead
    p.max_edges = n_total > (1 << 20) ? n_total : (1 << 20);
    p.max_edges = (p.max_edges + fof::kEdgeSlices - 1) / fof::kEdgeSlices * fof::kEdgeSlices;
    p.o_edges = take(sizeof(int32_t) * 2 * (size_t)p.max_edges);
    p.o_edge_fill = take(sizeof(uint32_t) * fof::kEdgeSlices);
    p.o_hist = take(sizeof(int32_t) * ((size_t)p.n_buckets * (size_t)p.n_tiles + 1));
    p.o_staging = take(sizeof(float) * 4 * n);
    p.o_stpos = take(sizeof(int32_t) * n);
    p.o_wave_roots = take(sizeof(int32_t) * ((n + 63) / 64));
    p.o_tile_dense = take(sizeof(unsigned long long) * ((n + 63) / 64));
    p.o_occ = take(sizeof(uint2) * (((size_t)p.n_segments << (p.seg_shift - 5)) + 2));
    p.o_seg = take(sizeof(int32_t) * (size_t)p.n_segments);
    p.o_staging2 = take(sizeof(float) * 4 * n);
    p.o_stage2_k = take(sizeof(int32_t) * n);
    p.o_bnd = o.domains > 1 ? take(sizeof(int32_t) * 2 * (size_t)p.max_edges) : 0;
    p.total = at;
    *out = p;
    return FOF_OK;
}

fof_status make_plan(const fof_ctx *c, const int64_t *offsets, const double *box, const double *lx, int32_t n_boxes,
                     HostPlan *out)
{
    if (!offsets || !box || !lx || n_boxes < 1) return FOF_ERR_INVALID_ARG;
    if (offsets[0] != 0) return FOF_ERR_INVALID_ARG;
    HostPlan p;
    p.boxes.resize((size_t)n_boxes);
    p.p0.assign(offsets, offsets + n_boxes + 1);
    int64_t cells = 0;
    for (int32_t k = 0; k < n_boxes; ++k) {
        const int64_t nb = offsets[k + 1] - offsets[k];
        if (nb < 0 || offsets[k + 1] > (int64_t)INT32_MAX) return FOF_ERR_INVALID_ARG;
        BoxDev &b = p.boxes[(size_t)k];
        fof_status st = box_geometry(c->opt, nb, box[k], lx[k], cells, &b);
        if (st != FOF_OK) return st;
        b.p0 = offsets[k];
        b.p1 = offsets[k + 1];
        p.lx_cells.push_back(lx[k]);
        if (c->opt.predicate == FOF_PRED_FP32_FILTER && b.use_fp64) ++p.fp64_boxes;
        cells += (int64_t)b.nc * b.nc * b.nc;
        if (cells > kMaxCells) return FOF_ERR_UNSUPPORTED;
    }
    fof_status st = make_layout(c->opt, offsets[n_boxes], cells, n_boxes, &p);
    if (st != FOF_OK) return st;
    *out = std::move(p);
    return FOF_OK;
}

template <typename T>
T *at(void *base, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

// The launch parameters of a run: options, sort levels and pointers into the
// workspace `ws` carved as `p`. `box0` is the first (or only) box.
void carve(const fof_options &o, const Layout &p, const BoxDev &box0, void *ws, Plan *out)
{
    Plan &d = *out;
    d.n = p.n;
    d.n_cells = p.n_cells;
    d.n_boxes = p.n_boxes;
    d.predicate = o.predicate;
    d.strict = o.strict_less;
    d.stats = o.collect_stats;
    d.scan_tiles = p.scan_tiles;
    d.n_tiles = p.n_tiles;
    d.bucket_shift = p.bucket_shift;
    d.n_buckets = p.n_buckets;
    d.seg_shift = p.seg_shift;
    d.sub_log2 = p.sub_log2;
    d.n_segments = p.n_segments;
    d.dense_min = dense_min_of(o);
    static const int32_t sparse_grid[4] = {kSparseBlocks, kSparseBlocks / 2, kSparseBlocks * 2, kSparseBlocks * 4};
    static const int32_t dense_grid[4] = {kDenseBlocks, kDenseBlocks / 2, kDenseBlocks * 2, kDenseBlocks * 4};
    d.sparse_blocks = sparse_grid[o.schedule & 3];
    d.dense_blocks = dense_grid[(o.schedule >> 2) & 3];
    d.premerge = (o.schedule & 16) ? 0 : 1;
    d.find_mode = o.compression;
    d.giant_skip = (o.schedule & 32) ? 1 : 0;
    d.tile_join = (o.schedule & 64) ? 0 : 1;
    d.sample = 0;
    d.domains = o.domains > 1 ? o.domains : 0;
    d.link_random = o.link_order == 1 ? 1 : 0;
    d.max_items = p.max_items;
    d.max_edges = p.max_edges;
    d.box0 = box0;
    d.boxes = at<BoxDev>(ws, p.o_boxes);
    d.box_p0 = at<int64_t>(ws, p.o_p0);
    d.counters = at<Counters>(ws, p.o_counters);
    d.n_groups = at<unsigned long long>(ws, p.o_groups);
    d.cstart = at<int32_t>(ws, p.o_cell);
    d.scan_part = at<int32_t>(ws, p.o_part);
    d.kmap = at<int32_t>(ws, p.o_kmap);
    d.sorted = at<float4>(ws, p.o_sorted);
    d.orig = at<int32_t>(ws, p.o_orig);
    d.gmin = at<int32_t>(ws, p.o_gmin);
    d.parent = at<int32_t>(ws, p.o_parent);
    d.gsize = at<int32_t>(ws, p.o_gsize);
    d.items = at<int4>(ws, p.o_items);
    d.edges = at<int2>(ws, p.o_edges);
    d.bnd = o.domains > 1 ? at<int2>(ws, p.o_bnd) : nullptr;
    d.bucket_hist = at<int32_t>(ws, p.o_hist);
    d.staging = at<float4>(ws, p.o_staging);
    d.stpos = at<int32_t>(ws, p.o_stpos);
    d.wave_roots = at<int32_t>(ws, p.o_wave_roots);
    d.tile_dense = at<unsigned long long>(ws, p.o_tile_dense);
    d.occ = at<uint2>(ws, p.o_occ);
    d.seg_end = at<int32_t>(ws, p.o_seg);
    d.staging2 = at<float4>(ws, p.o_staging2);
    d.stage2_k = at<int32_t>(ws, p.o_stage2_k);
    d.edge_fill = at<unsigned int>(ws, p.o_edge_fill);
    d.n_waves = (p.n + 63) / 64;
    d.label = nullptr;
    d.size = nullptr;
}

fof_status ensure_device(fof_ctx *c)
{
    if (c->device >= 0) return FOF_OK;
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d < 0) return FOF_ERR_DEVICE;
    c->device = d;
    return FOF_OK;
}

// Copies the box table and offsets of `np` to the start of the workspace,
// through one of two pinned staging buffers used in turn. Refilling a buffer
// waits only for that buffer's previous copy (two uploads back), not for the
// stream; a buffer grows (pinned host memory, not device memory) only when a
// larger table than before comes along.
fof_status upload_table(fof_ctx *c, const HostPlan &np)
{
    const size_t table = np.o_counters;   // boxes + p0 region
    const int k = c->stage_next;
    if (!c->stage_done[k] && hipEventCreateWithFlags(&c->stage_done[k], hipEventDisableTiming) != hipSuccess)
        return FOF_ERR_DEVICE;
    if (c->stage_pending[k]) {
        if (hipEventSynchronize(c->stage_done[k]) != hipSuccess) return FOF_ERR_DEVICE;
        c->stage_pending[k] = false;
    }
    if (c->stage_bytes[k] < table) {
        if (c->stage[k]) (void)hipHostFree(c->stage[k]);
        c->stage[k] = nullptr;
        c->stage_bytes[k] = 0;
        if (hipHostMalloc(&c->stage[k], table, hipHostMallocDefault) != hipSuccess) return FOF_ERR_DEVICE;
        c->stage_bytes[k] = table;
    }
    std::memset(c->stage[k], 0, table);
    std::memcpy(at<char>(c->stage[k], np.o_boxes), np.boxes.data(), sizeof(BoxDev) * np.boxes.size());
    std::memcpy(at<char>(c->stage[k], np.o_p0), np.p0.data(), sizeof(int64_t) * np.p0.size());
    if (hipMemcpyAsync(c->ws, c->stage[k], table, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return FOF_ERR_DEVICE;
    if (hipEventRecord(c->stage_done[k], c->stream) != hipSuccess) return FOF_ERR_DEVICE;
    c->stage_pending[k] = true;
    c->stage_next = k ^ 1;
    c->table_plan = np;
    c->table_id = ++c->upload_seq;
    return FOF_OK;
}

// Adopt `np` as the current plan; upload its box table unless the workspace
// already holds the same one. A single box travels in the kernel arguments,
// and its run writes over the table region of any earlier multi-box layout.
fof_status install_plan(fof_ctx *c, HostPlan &&np)
{
    if (!c->ws) return FOF_ERR_WORKSPACE;
    if (c->ws_bytes < np.total) return FOF_ERR_WORKSPACE;
    fof_status st = ensure_device(c);
    if (st != FOF_OK) return st;
    if (np.n_boxes == 1) {
        c->table_id = 0;
    } else if (!(c->table_id && c->table_plan.same_geometry(np))) {
        st = upload_table(c, np);
        if (st != FOF_OK) return st;
    }
    c->plan = std::move(np);
    c->planned = true;
    carve(c->opt, c->plan, c->plan.boxes[0], c->ws, &c->dev);
    return FOF_OK;
}

void drop_graph(fof_ctx *c)
{
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
    c->graph_boxes = 0;
}

fof_status do_build(fof_ctx *c, const float *d_pos, const int64_t *off, const double *box, const double *lx,
                    int32_t n_boxes)
{
    if (c->opt.collect_timings && !c->timer) {
        if (ensure_device(c) != FOF_OK) return FOF_ERR_DEVICE;
        c->timer = new (std::nothrow) EventTimer();
        if (!c->timer || !c->timer->init()) return FOF_ERR_DEVICE;
    }
    HostPlan np;
    fof_status st = make_plan(c, off, box, lx, n_boxes, &np);
    if (st != FOF_OK) return st;
    if (!d_pos && np.n > 0) return FOF_ERR_INVALID_ARG;
    st = install_plan(c, std::move(np));
    if (st != FOF_OK) return st;
    c->dev.pos = d_pos;
    return FOF_OK;
}

fof_status enqueue_build(fof_ctx *c, hipStream_t s)
{
    hipError_t e = fof::launch_clear(c->dev, s, c->timer);
    if (e == hipSuccess) e = fof::launch_build(c->dev, s, c->timer);
    return dev_err(e);
}

fof_status read_back(fof_ctx *c, int64_t *h_n_groups, Counters *h_counters)
{
    const HostPlan &p = c->plan;
    std::vector<unsigned long long> g((size_t)p.n_boxes);
    Counters cnt{};
    if (hipMemcpyAsync(g.data(), c->dev.n_groups, sizeof(unsigned long long) * g.size(), hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return FOF_ERR_DEVICE;
    if (hipMemcpyAsync(&cnt, c->dev.counters, sizeof(Counters), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return FOF_ERR_DEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return FOF_ERR_DEVICE;
    if (h_n_groups)
        for (size_t k = 0; k < g.size(); ++k) h_n_groups[k] = (int64_t)g[k];
    if (h_counters) *h_counters = cnt;
    if (cnt.error & 2u) return FOF_ERR_DEVICE;   // a device-side consistency check failed
    return (cnt.error & 1u) ? FOF_ERR_OUT_OF_BOX : FOF_OK;
}

}  // namespace

namespace fof {

fof_status plan_one_box(const fof_options &o, int64_t n, double box, double lx, void *ws, size_t bytes, Plan *out,
                        size_t *need)
{
    *need = 0;
    if (!options_valid(o)) return FOF_ERR_INVALID_ARG;
    if (n < 0 || n > (int64_t)INT32_MAX) return FOF_ERR_INVALID_ARG;
    BoxDev b;
    fof_status st = box_geometry(o, n, box, lx, 0, &b);
    if (st != FOF_OK) return st;
    b.p0 = 0;
    b.p1 = n;
    Layout lay;
    st = make_layout(o, n, (int64_t)b.nc * b.nc * b.nc, 1, &lay);
    if (st != FOF_OK) return st;
    *need = lay.total;
    if (lay.total > bytes) return FOF_OK;
    carve(o, lay, b, ws, out);
    return FOF_OK;
}

}  // namespace fof

extern "C" {

void fof_default_options(fof_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->predicate = FOF_PRED_FP32_FILTER;
}

fof_status fof_create(fof_ctx **out, const fof_options *opt, void *hip_stream)
{
    if (!out) return FOF_ERR_INVALID_ARG;
    *out = nullptr;
    fof_options o;
    fof_default_options(&o);
    if (opt) o = *opt;
    if (!options_valid(o)) return FOF_ERR_INVALID_ARG;
    fof_ctx *c = new (std::nothrow) fof_ctx();
    if (!c) return FOF_ERR_DEVICE;
    c->opt = o;
    c->stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    return FOF_OK;
}

fof_status fof_set_stream(fof_ctx *ctx, void *hip_stream)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return FOF_OK;
}

fof_status fof_workspace_bytes(fof_ctx *ctx, const int64_t *h_box_offsets, const double *h_box, const double *h_lx,
                               int32_t n_boxes, size_t *bytes)
{
    if (!ctx || !bytes) return FOF_ERR_INVALID_ARG;
    HostPlan p;
    fof_status st = make_plan(ctx, h_box_offsets, h_box, h_lx, n_boxes, &p);
    if (st != FOF_OK) return st;
    *bytes = p.total;
    return FOF_OK;
}

fof_status fof_set_workspace(fof_ctx *ctx, void *d_ws, size_t bytes)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    if (d_ws && (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0) return FOF_ERR_WORKSPACE;
    if (ctx->ws != d_ws || (d_ws && bytes < ctx->ws_bytes)) {
        ctx->table_id = 0;
        ctx->planned = false;   // the carved pointers refer to the old workspace
        ctx->cells_valid = false;
        drop_graph(ctx);        // its kernels hold pointers into the old workspace
    }
    ctx->ws = d_ws;
    ctx->ws_bytes = d_ws ? bytes : 0;
    ctx->state = 0;
    return FOF_OK;
}

fof_status fof_build_cells(fof_ctx *ctx, const float *d_pos, const int64_t *h_box_offsets, const double *h_box,
                           const double *h_lx, int32_t n_boxes)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    ctx->cells_valid = false;
    fof_status st = do_build(ctx, d_pos, h_box_offsets, h_box, h_lx, n_boxes);
    if (st != FOF_OK) return st;
    st = enqueue_build(ctx, ctx->stream);
    ctx->state = st == FOF_OK ? 1 : 0;
    ctx->cells_valid = st == FOF_OK;
    return st;
}

fof_status fof_relink(fof_ctx *ctx, const double *h_lx, int32_t n_boxes)
{
    if (!ctx || !h_lx) return FOF_ERR_INVALID_ARG;
    if (!ctx->cells_valid || !ctx->planned) return FOF_ERR_BAD_STATE;
    HostPlan &p = ctx->plan;
    if (n_boxes != p.n_boxes) return FOF_ERR_INVALID_ARG;
    for (int32_t k = 0; k < n_boxes; ++k)
        if (!(h_lx[k] > 0.0) || !std::isfinite(h_lx[k]) || h_lx[k] > p.lx_cells[(size_t)k]) return FOF_ERR_INVALID_ARG;
    p.fp64_boxes = 0;
    for (int32_t k = 0; k < n_boxes; ++k) {
        BoxDev &b = p.boxes[(size_t)k];
        const double l = h_lx[k];
        b.l2 = l * l;
        fp32_thresholds(b, l);
        sub_cells(b.L, b.nc, l, &b.sub_k, &b.sub_adj);
        if (ctx->opt.predicate == FOF_PRED_FP32_FILTER && b.use_fp64) ++p.fp64_boxes;
    }
    ctx->dev.box0 = p.boxes[0];
    if (p.n_boxes > 1) {
        fof_status st = upload_table(ctx, p);
        if (st != FOF_OK) return st;
    }
    fof_status st = dev_err(fof::launch_relink_reset(ctx->dev, ctx->stream));
    ctx->state = st == FOF_OK ? 1 : 0;
    return st;
}

fof_status fof_link(fof_ctx *ctx)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    if (ctx->state != 1) return FOF_ERR_BAD_STATE;
    fof_status st = dev_err(fof::launch_link(ctx->dev, ctx->stream, ctx->timer));
    ctx->state = st == FOF_OK ? 2 : 0;
    return st;
}

fof_status fof_finalize(fof_ctx *ctx, int32_t *d_group_index, int32_t *d_group_size, int64_t *h_n_groups)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    if (ctx->state != 2) return FOF_ERR_BAD_STATE;
    if ((!d_group_index || !d_group_size) && ctx->plan.n > 0) return FOF_ERR_INVALID_ARG;
    ctx->dev.label = d_group_index;
    ctx->dev.size = d_group_size;
    fof_status st = dev_err(fof::launch_finalize(ctx->dev, ctx->stream, ctx->timer));
    ctx->state = 0;   // the forest is consumed: a new build is needed
    if (st != FOF_OK) return st;
    if (h_n_groups) return read_back(ctx, h_n_groups, nullptr);
    return FOF_OK;
}

fof_status fof_catalogue(fof_ctx *ctx, const int32_t *d_group_index, const int32_t *d_group_size, int32_t min_size,
                         int32_t *d_first, int32_t *d_size, int32_t *d_box, int64_t capacity, int64_t *h_count)
{
    if (!ctx || !h_count || min_size < 1 || capacity < 0) return FOF_ERR_INVALID_ARG;
    *h_count = 0;
    if (!ctx->planned || !ctx->ws) return FOF_ERR_BAD_STATE;
    if (ctx->plan.n > 0 && (!d_group_index || !d_group_size)) return FOF_ERR_INVALID_ARG;
    if (capacity > 0 && (!d_first || !d_size)) return FOF_ERR_INVALID_ARG;
    const fof::Plan &p = ctx->dev;
    fof_status st = dev_err(fof::launch_catalogue(p, d_group_index, d_group_size, min_size, d_first, d_size, d_box,
                                                  capacity, ctx->stream));
    if (st != FOF_OK) return st;
    int total = 0;
    if (hipMemcpyAsync(&total, p.bucket_hist + p.n_tiles, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) !=
        hipSuccess)
        return FOF_ERR_DEVICE;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return FOF_ERR_DEVICE;
    *h_count = total;
    return FOF_OK;
}

fof_status fof_read_n_groups(fof_ctx *ctx, int64_t *h_n_groups)
{
    if (!ctx || !h_n_groups) return FOF_ERR_INVALID_ARG;
    if (!ctx->planned) return FOF_ERR_BAD_STATE;
    return read_back(ctx, h_n_groups, nullptr);
}

fof_status fof_get_stats(fof_ctx *ctx, fof_stats *out)
{
    if (!ctx || !out) return FOF_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    if (!ctx->planned) return FOF_ERR_BAD_STATE;
    std::vector<int64_t> g((size_t)ctx->plan.n_boxes);
    Counters cnt{};
    fof_status st = read_back(ctx, g.data(), &cnt);
    out->n_particles = ctx->plan.n;
    out->n_cells = ctx->plan.n_cells;
    for (int64_t v : g) out->n_groups += v;
    out->pair_tests = (int64_t)cnt.pair_tests;
    out->links = (int64_t)cnt.links;
    out->band_hits = (int64_t)cnt.band_hits;
    out->cas_retries = (int64_t)cnt.cas_retries;
    out->fp64_boxes = ctx->plan.fp64_boxes;
    out->sparse_pair_tests = (int64_t)cnt.sparse_tests;
    out->queued_links = (int64_t)cnt.n_edges;
    out->dense_items = (int64_t)cnt.n_items;
    out->boundary_links = (int64_t)cnt.n_boundary;
    out->boundary_groups = (int64_t)cnt.n_bgroups;
    out->find_depth_max = (int64_t)cnt.depth_max;
    out->find_depth_sum = (int64_t)cnt.depth_sum;
    return st;
}

fof_status fof_graph_capture(fof_ctx *ctx, const float *d_pos, const int64_t *h_box_offsets, const double *h_box,
                             const double *h_lx, int32_t n_boxes, int32_t *d_group_index, int32_t *d_group_size)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    ctx->cells_valid = false;
    fof_status st = do_build(ctx, d_pos, h_box_offsets, h_box, h_lx, n_boxes);
    if (st != FOF_OK) return st;
    if ((!d_group_index || !d_group_size) && ctx->plan.n > 0) return FOF_ERR_INVALID_ARG;
    ctx->dev.label = d_group_index;
    ctx->dev.size = d_group_size;
    drop_graph(ctx);
    // the descriptor upload above is ordered on ctx->stream; capture on a
    // private stream that first waits for it
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return FOF_ERR_DEVICE;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return FOF_ERR_DEVICE;
    // a second captured stream, onto which the link phase forks the pre-merge
    fof::Fork fk;
    hipError_t e = hipStreamCreateWithFlags(&fk.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fk.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fk.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // no per-kernel events inside a graph
        e = fof::launch_clear(ctx->dev, cs, nullptr);
        if (e == hipSuccess) e = fof::launch_build(ctx->dev, cs, nullptr);
        if (e == hipSuccess) e = fof::launch_link(ctx->dev, cs, nullptr, &fk);
        if (e == hipSuccess) e = fof::launch_finalize(ctx->dev, cs, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) {
            ctx->graph = g;
            e = hipGraphInstantiate(&ctx->exec, g, nullptr, nullptr, 0);
            if (e == hipSuccess) {
                ctx->graph_boxes = ctx->plan.n_boxes;
                ctx->graph_plan = ctx->plan;
            } else {
                drop_graph(ctx);
            }
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (fk.side) (void)hipStreamDestroy(fk.side);
    if (fk.fork) (void)hipEventDestroy(fk.fork);
    if (fk.join) (void)hipEventDestroy(fk.join);
    ctx->state = 0;
    return dev_err(e);
}

fof_status fof_graph_launch(fof_ctx *ctx)
{
    if (!ctx) return FOF_ERR_INVALID_ARG;
    if (!ctx->exec) return FOF_ERR_BAD_STATE;
    // a multi-box graph reads the box table in the workspace: refuse when a
    // later build or relink of another geometry has replaced it
    if (ctx->graph_boxes > 1 && !(ctx->table_id && ctx->table_plan.same_geometry(ctx->graph_plan)))
        return FOF_ERR_BAD_STATE;
    return dev_err(hipGraphLaunch(ctx->exec, ctx->stream));
}

fof_status fof_destroy(fof_ctx *ctx)
{
    if (!ctx) return FOF_OK;
    if (ctx->device >= 0) (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    for (int k = 0; k < 2; ++k) {
        if (ctx->stage[k]) (void)hipHostFree(ctx->stage[k]);
        if (ctx->stage_done[k]) (void)hipEventDestroy(ctx->stage_done[k]);
    }
    delete ctx->timer;
    delete ctx;
    return FOF_OK;
}

fof_status fof_describe_box(const fof_options *opt, int64_t n_particles, double box, double lx, fof_box_info *out)
{
    if (!out) return FOF_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    fof_options o;
    fof_default_options(&o);
    if (opt) o = *opt;
    if (!options_valid(o)) return FOF_ERR_INVALID_ARG;
    if (n_particles < 0 || n_particles > (int64_t)INT32_MAX) return FOF_ERR_INVALID_ARG;
    if (!(box > 0.0) || !std::isfinite(box) || !(lx > 0.0) || !std::isfinite(lx)) return FOF_ERR_INVALID_ARG;
    int64_t nc = 0;
    fof_status st = cells_per_axis(o, n_particles, box, lx, &nc);
    if (st != FOF_OK) return st;
    BoxDev b;
    std::memset(&b, 0, sizeof(b));
    b.L = box;
    b.l2 = lx * lx;
    fp32_thresholds(b, lx);
    out->cells_per_axis = nc;
    out->l2 = b.l2;
    out->lo32 = b.lo32;
    out->hi32 = b.hi32;
    out->fp64_only = b.use_fp64;
    sub_cells(box, nc, lx, &out->sub_cells_per_axis, &out->sub_cells_adjacent);
    return FOF_OK;
}

fof_status fof_get_kernel_times(fof_ctx *ctx, double *h_ms, int32_t *h_launches, int32_t capacity,
                                int32_t *n_kernels)
{
    if (!ctx || !n_kernels) return FOF_ERR_INVALID_ARG;
    *n_kernels = fof::K_COUNT_KERNELS;
    if (!h_ms || capacity < fof::K_COUNT_KERNELS) return FOF_ERR_INVALID_ARG;
    for (int k = 0; k < fof::K_COUNT_KERNELS; ++k) {
        h_ms[k] = 0.0;
        if (h_launches) h_launches[k] = 0;
    }
    EventTimer *t = ctx->timer;
    if (!t) return ctx->opt.collect_timings ? FOF_OK : FOF_ERR_BAD_STATE;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return FOF_ERR_DEVICE;
    const int first = (t->next - t->used + EventTimer::kSlots) % EventTimer::kSlots;
    for (int u = 0; u < t->used; ++u) {
        const int slot = (first + u) % EventTimer::kSlots;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t->start[slot], t->stop[slot]) != hipSuccess) return FOF_ERR_DEVICE;
        h_ms[t->kernel[slot]] += ms;
        if (h_launches) h_launches[t->kernel[slot]] += 1;
    }
    t->used = 0;
    return FOF_OK;
}

const char *fof_kernel_name(int32_t k) { return fof::kernel_name(k); }

const char *fof_status_string(fof_status s)
{
    switch (s) {
    case FOF_OK: return "ok";
    case FOF_ERR_INVALID_ARG: return "invalid argument";
    case FOF_ERR_OUT_OF_BOX: return "coordinate not finite or outside [0, L)";
    case FOF_ERR_BAD_STATE: return "calls out of order";
    case FOF_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case FOF_ERR_DEVICE: return "HIP runtime error";
    case FOF_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

}  // extern "C"
