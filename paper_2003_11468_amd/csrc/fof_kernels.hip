// Friends-of-Friends kernels for gfx950 (CDNA4, wave64).
//
// Pipeline over all boxes at once (every kernel is a flat launch over particles
// or cells; per-box parameters come from a small descriptor table):
//   clear    zero the cell counts, group counters and error word
//   count    validate coordinates, cell key, slot inside the cell (atomic add);
//            also seeds the union-find forest parent[s] = s and member counts
//   scan     exclusive prefix over the cell counts -> cell start offsets
//   scatter  counting-sort scatter into cell order (x, y, z as float4) + the
//            sorted -> original index map
//   link     (fof_link.hip) cell-pair link search + lock-free union-find
//   flatten  pointer jumping to the root; group minimum original index
//            (atomic min) and member count (atomic add) at the root
//   resolve  label and size per sorted slot, per-box group counts
//   gather   labels and sizes into input order
//
// The whole translation unit is compiled with -ffp-contract=off: the double
// predicate below must round every product and sum separately. The FP32
// filter requests its fused multiply-adds explicitly (fmaf), which its error
// bound allows.
#include "fof_device.h"

namespace fof {
namespace {

using namespace dev;

constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = kBlock * kScanItems;      // 2048 counts per tile
constexpr int kPartBlock = 1024;

// ---------------------------------------------------------------- kernels --

__global__ void __launch_bounds__(kBlock) k_clear(Plan p)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= p.n_cells; i += stride) p.cell[i] = 0;
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < p.n_boxes) p.n_groups[t] = 0;
    if (t == 0) {
        p.counters->pair_tests = 0;
        p.counters->links = 0;
        p.counters->band_hits = 0;
        p.counters->cas_retries = 0;
        p.counters->sparse_tests = 0;
        p.counters->error = 0;
        p.counters->n_items = 0;
        p.counters->n_edges = 0;
    }
}

__global__ void __launch_bounds__(kBlock) k_count(Plan p)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const BoxDev bd = p.n_boxes == 1 ? p.box0 : p.boxes[b];
    const float x = p.pos[3 * i + 0], y = p.pos[3 * i + 1], z = p.pos[3 * i + 2];
    if (!(in_box(x, bd.L) && in_box(y, bd.L) && in_box(z, bd.L))) atomicOr(&p.counters->error, 1u);
    const int key = particle_cell(bd, x, y, z);
    p.rank[i] = atomicAdd(p.cell + key, 1);
    p.parent[i] = (int)i;
    p.gsize[i] = 1;
}

// The 8 counts of a thread; whole groups of 8 are read as two 16-byte loads.
__device__ __forceinline__ void load8(const int *a, int64_t base, int64_t m, int v[kScanItems])
{
    if (base + kScanItems <= m) {
        const int4 u = *reinterpret_cast<const int4 *>(a + base);
        const int4 w = *reinterpret_cast<const int4 *>(a + base + 4);
        v[0] = u.x; v[1] = u.y; v[2] = u.z; v[3] = u.w;
        v[4] = w.x; v[5] = w.y; v[6] = w.z; v[7] = w.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < m) ? a[base + k] : 0;
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(Plan p)
{
    __shared__ int lds[kBlock / 64];
    const int64_t m = p.n_cells + 1;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    load8(p.cell, base, m, v);
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    int total;
    block_excl_scan<kBlock>(s, lds, &total);
    if (threadIdx.x == 0) p.scan_part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kPartBlock) k_scan_partials(Plan p)
{
    __shared__ int lds[kPartBlock / 64];
    const int64_t t = p.scan_tiles;
    const int64_t chunk = (t + kPartBlock - 1) / kPartBlock;
    const int64_t b0 = (int64_t)threadIdx.x * chunk;
    int s = 0;
    for (int64_t k = b0; k < b0 + chunk && k < t; ++k) s += p.scan_part[k];
    int total;
    int run = block_excl_scan<kPartBlock>(s, lds, &total);
    for (int64_t k = b0; k < b0 + chunk && k < t; ++k) {
        int v = p.scan_part[k];
        p.scan_part[k] = run;
        run += v;
    }
}

// Writes the cell start offsets and, for every cell holding at least
// dense_min particles, one dense link work item per 64 of its particles:
// {cell, first home particle, box, 0}.
__global__ void __launch_bounds__(kBlock) k_scan_apply(Plan p)
{
    __shared__ int lds[kBlock / 64];
    const int64_t m = p.n_cells + 1;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    load8(p.cell, base, m, v);
    int s = 0, chunks = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        s += v[k];
        const bool dense = base + k < p.n_cells && v[k] >= p.dense_min && v[k] > 0;
        chunks += dense ? (v[k] + 63) >> 6 : 0;
    }
    int total;
    const int start = block_excl_scan<kBlock>(s, lds, &total) + p.scan_part[blockIdx.x];
    int o[kScanItems];
    int run = start;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (base + kScanItems <= m) {
        *reinterpret_cast<int4 *>(p.cell + base) = make_int4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<int4 *>(p.cell + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < m) p.cell[base + k] = o[k];
    }
    // dense work items: one atomic per wave reserves the slots
    const int incl = wave_incl_scan(chunks);
    const int wave_total = __shfl(incl, 63, 64);
    int slot = 0;
    if (lane_id() == 63 && wave_total > 0) slot = (int)atomicAdd(&p.counters->n_items, (unsigned)wave_total);
    slot = __shfl(slot, 63, 64) + incl - chunks;
    if (chunks) {
#pragma unroll 1
        for (int k = 0; k < kScanItems; ++k) {
            const bool dense = base + k < p.n_cells && v[k] >= p.dense_min && v[k] > 0;
            if (!dense) continue;
            const int first = o[k];
            const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, first);
            for (int q = 0; q < v[k]; q += 64) p.items[slot++] = make_int4((int)(base + k), first + q, b, 0);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter(Plan p)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const BoxDev bd = p.n_boxes == 1 ? p.box0 : p.boxes[b];
    const float x = p.pos[3 * i + 0], y = p.pos[3 * i + 1], z = p.pos[3 * i + 2];
    const int key = particle_cell(bd, x, y, z);
    const int dst = p.cell[key] + p.rank[i];
    p.sorted[dst] = make_float4(x, y, z, 0.0f);
    p.perm[dst] = make_int2((int)i, (int)i);
    p.rank[i] = dst;   // from here on: sorted slot of input particle i
}

// Consecutive sorted particles mostly share their root, so the root updates
// are combined per wave before the atomics.
__global__ void __launch_bounds__(kBlock) k_flatten(Plan p)
{
    const int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int root_key = -1, orig = 0;
    if (s64 < p.n) {
        const int s = (int)s64;
        int r = s, q = p.parent[s];
        while (q != r) {
            r = q;
            q = p.parent[r];
        }
        if (r != s) {
            p.parent[s] = r;
            root_key = r;
            orig = p.perm[s].x;
        }
    }
    wave_min_by_key(p.perm, root_key, orig);
    wave_add_by_key(p.gsize, root_key, 1);
}

// Resolve, in sorted order: out[s] = {group label (box-local), size at the
// root's smallest member, else 0}. Reads are local (the root of s sits near
// s in cell order) and the write is coalesced. Each thread handles kOutItems
// particles spaced one block apart; roots are counted per box in registers and
// flushed once per box change and at the end.
constexpr int kOutItems = 8;

__global__ void __launch_bounds__(kBlock) k_resolve(Plan p)
{
    const int64_t base = (int64_t)blockIdx.x * kBlock * kOutItems + threadIdx.x;
    int2 *out = reinterpret_cast<int2 *>(p.sorted);   // positions are no longer needed
    int cur_box = -1, cur_count = 0;
    for (int k = 0; k < kOutItems; ++k) {
        const int64_t s64 = base + (int64_t)k * kBlock;
        if (s64 >= p.n) break;
        const int s = (int)s64;
        const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, s64);
        const int r = p.parent[s];
        const int o = p.perm[s].x;
        const int m = p.perm[r].y;
        const int p0 = p.n_boxes == 1 ? 0 : (int)p.box_p0[b];
        out[s] = make_int2(m - p0, (o == m) ? p.gsize[r] : 0);
        if (r == s) {
            if (b != cur_box) {
                if (cur_count) atomicAdd(p.n_groups + cur_box, (unsigned long long)cur_count);
                cur_box = b;
                cur_count = 0;
            }
            ++cur_count;
        }
    }
    wave_add_by_key(p.n_groups, cur_count ? cur_box : -1, (unsigned long long)cur_count);
}

// Gather into input order: one random 8-byte read per particle, coalesced
// reads of the slot map and coalesced writes of both outputs.
__global__ void __launch_bounds__(kBlock) k_gather(Plan p)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int2 *out = reinterpret_cast<const int2 *>(p.sorted);
    const int2 v = out[p.rank[i]];
    p.label[i] = v.x;
    p.size[i] = v.y;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// Launch `k` bracketed by the timer marks.
#define FOF_TIMED(id, ...)                 \
    do {                                   \
        if (t) t->mark(id, false, stream); \
        __VA_ARGS__;                       \
        if (t) t->mark(id, true, stream);  \
    } while (0)

const char *kernel_name(int k)
{
    static const char *names[K_COUNT_KERNELS] = {"k_clear", "k_count", "k_scan_reduce", "k_scan_partials",
                                                 "k_scan_apply", "k_scatter", "k_link_sparse", "k_union_edges",
                                                 "k_link_dense", "k_flatten", "k_resolve", "k_gather"};
    return (k >= 0 && k < K_COUNT_KERNELS) ? names[k] : "?";
}

hipError_t launch_clear(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    int64_t work = p.n_cells + 1 > p.n_boxes ? p.n_cells + 1 : p.n_boxes;
    unsigned g = grid_for(work);
    if (g > 65536u) g = 65536u;
    FOF_TIMED(K_CLEAR, hipLaunchKernelGGL(k_clear, dim3(g), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

hipError_t launch_build(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    if (p.n > 0) FOF_TIMED(K_COUNT, hipLaunchKernelGGL(k_count, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_SCAN_REDUCE,
              hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)p.scan_tiles), dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_SCAN_PARTIALS, hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kPartBlock), 0, stream, p));
    FOF_TIMED(K_SCAN_APPLY,
              hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)p.scan_tiles), dim3(kBlock), 0, stream, p));
    if (p.n > 0)
        FOF_TIMED(K_SCATTER, hipLaunchKernelGGL(k_scatter, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

hipError_t launch_finalize(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    if (p.n == 0) return hipSuccess;
    FOF_TIMED(K_FLATTEN, hipLaunchKernelGGL(k_flatten, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_RESOLVE,
              hipLaunchKernelGGL(k_resolve, dim3((unsigned)((p.n + kBlock * kOutItems - 1) / (kBlock * kOutItems))),
                                 dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_GATHER, hipLaunchKernelGGL(k_gather, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

int64_t scan_tiles_for(int64_t n_cells) { return (n_cells + 1 + kScanTile - 1) / kScanTile; }

}  // namespace fof
