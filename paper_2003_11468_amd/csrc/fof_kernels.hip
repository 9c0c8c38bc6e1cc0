// Friends-of-Friends kernels for gfx950 (CDNA4, wave64).
//
// Pipeline over all boxes at once (every kernel is a flat launch over particles
// or cells; per-box parameters come from a small descriptor table).
//
// The counting sort into cells runs in two levels so that no pass scatters
// over the whole array. Cells are grouped into at most 256 buckets of
// consecutive cell indices.
//   clear          zero the cell counts, group counters and error word
//   bucket_hist    per tile of 2048 input particles: validate coordinates,
//                  bucket histogram in LDS
//   bucket_scan    exclusive prefix over (bucket, tile) -> where each tile's
//                  share of each bucket goes
//   bucket_scatter sort each tile by bucket in LDS and write it out as runs:
//                  the "staging" order, bucket by bucket
//   count          in staging order: slot inside the cell (atomic add); the
//                  atomics of a bucket stay inside its window of cells. Also
//                  seeds the union-find forest and member counts
//   cell_scan      exclusive prefix over the cell counts -> cell starts, and
//                  the dense link work items
//   scatter        in staging order into cell order (x, y, z as float4) + the
//                  sorted -> original index map; writes stay in the bucket's
//                  window of slots
//   link           (fof_link.hip) cell-pair link search + lock-free union-find
//   flatten  pointer jumping to the root; group minimum original index
//            (atomic min) and member count (atomic add) at the root
//   resolve  label and size per sorted slot, per-box group counts
//   unsort   back into staging order (reads stay in the bucket's window)
//   gather   back into input order (reads are runs of each tile's buckets)
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
constexpr int kSortItems = 8;                       // input particles per thread
constexpr int kSortTile = kBlock * kSortItems;      // 2048 input particles per tile
constexpr int kMaxBuckets = 256;

// ---------------------------------------------------------------- kernels --

__global__ void __launch_bounds__(kBlock) k_clear(Plan p)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= p.n_cells; i += stride) p.cell[i] = 0;
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < p.n_boxes) p.n_groups[t] = 0;
    if (t < kEdgeSlices) p.edge_fill[t] = 0;
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

// Cell key of input particle i; `ok` tells whether its coordinates are finite
// and inside [0, L).
__device__ __forceinline__ int input_key(const Plan &p, int64_t i, float &x, float &y, float &z, bool &ok)
{
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const BoxDev &bd = box_of(p, b);
    x = p.pos[3 * i + 0];
    y = p.pos[3 * i + 1];
    z = p.pos[3 * i + 2];
    ok = in_box(x, bd.L) && in_box(y, bd.L) && in_box(z, bd.L);
    return particle_cell(bd, x, y, z);
}

// Bucket histogram of one tile, written bucket-major: hist[b * n_tiles + tile].
__global__ void __launch_bounds__(kBlock) k_bucket_hist(Plan p)
{
    __shared__ int cnt[kMaxBuckets];
    const int64_t tile = blockIdx.x;
    for (int b = threadIdx.x; b < kMaxBuckets; b += kBlock) cnt[b] = 0;
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = tile * kSortTile + k * kBlock + threadIdx.x;
        if (i < p.n) {
            float x, y, z;
            bool ok;
            const int key = input_key(p, i, x, y, z, ok);
            bad |= !ok;
            atomicAdd(&cnt[key >> p.bucket_shift], 1);
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&p.counters->error, 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < p.n_buckets; b += kBlock) p.bucket_hist[(int64_t)b * p.n_tiles + tile] = cnt[b];
}

// Sorts one tile by bucket in LDS and writes each bucket's run to its place in
// the staging order (x, y, z, original index as bits); stpos[i] = staging slot.
__global__ void __launch_bounds__(kBlock) k_bucket_scatter(Plan p)
{
    __shared__ float4 stage[kSortTile];
    __shared__ unsigned char stage_b[kSortTile];
    __shared__ int cnt[kMaxBuckets], first[kMaxBuckets], dst0[kMaxBuckets];
    __shared__ int lds[kBlock / 64];
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kSortTile;
    for (int b = threadIdx.x; b < kMaxBuckets; b += kBlock) cnt[b] = 0;
    __syncthreads();
    float4 v[kSortItems];
    int bk[kSortItems], rk[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + k * kBlock + threadIdx.x;
        bk[k] = -1;
        if (i < p.n) {
            float x, y, z;
            bool ok;
            const int key = input_key(p, i, x, y, z, ok);
            bk[k] = key >> p.bucket_shift;
            rk[k] = atomicAdd(&cnt[bk[k]], 1);
            v[k] = make_float4(x, y, z, __int_as_float((int)i));
        }
    }
    __syncthreads();
    {
        const int b = threadIdx.x;   // kBlock == kMaxBuckets: one bucket per thread
        int total;
        const int c = cnt[b];
        first[b] = block_excl_scan<kBlock>(c, lds, &total);
        dst0[b] = b < p.n_buckets ? p.bucket_hist[(int64_t)b * p.n_tiles + tile] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k)
        if (bk[k] >= 0) {
            const int at = first[bk[k]] + rk[k];
            stage[at] = v[k];
            stage_b[at] = (unsigned char)bk[k];
        }
    __syncthreads();
    const int count = (int)min((int64_t)kSortTile, p.n - base);
    for (int j = threadIdx.x; j < count; j += kBlock) {
        const float4 e = stage[j];
        const int b = stage_b[j];
        const int dst = dst0[b] + (j - first[b]);
        p.staging[dst] = e;
        p.stpos[__float_as_int(e.w)] = dst;
    }
}

// In staging order: slot of the particle inside its cell. Consecutive staging
// slots belong to the same bucket, so the atomics stay in a window of cells.
__global__ void __launch_bounds__(kBlock) k_count(Plan p)
{
    const int64_t k = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (k >= p.n) return;
    const float4 e = p.staging[k];
    const int i = __float_as_int(e.w);
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const int key = particle_cell(box_of(p, b), e.x, e.y, e.z);
    p.rank[k] = atomicAdd(p.cell + key, 1);
    p.parent[k] = (int)k;
    p.gsize[k] = 1;
}

// ------------------------------------------------------------------ scans --
// Exclusive prefix sums in place, in tiles of 2048 (8 per thread, 16-byte
// loads); tile sums are scanned recursively, so no level is a long serial loop.

struct ScanArgs {
    int *data;
    int64_t len;
    const int *part;   // exclusive prefix of the tile sums (null for a single tile)
};

// The 8 values of a thread; whole groups of 8 are read as two 16-byte loads.
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

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int *data, int64_t len, int *sums)
{
    __shared__ int lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    load8(data, base, len, v);
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    int total;
    block_excl_scan<kBlock>(s, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// kCells: the scan over the cell counts, which also emits one dense link work
// item {cell, first home particle, box, 0} per 64 particles of every cell with
// at least dense_min particles.
template <bool kCells>
__global__ void __launch_bounds__(kBlock) k_scan_apply(ScanArgs a, Plan p)
{
    __shared__ int lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    load8(a.data, base, a.len, v);
    int s = 0, chunks = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        s += v[k];
        if (kCells) {
            const bool dense = base + k < p.n_cells && v[k] >= p.dense_min && v[k] > 0;
            chunks += dense ? (v[k] + 63) >> 6 : 0;
        }
    }
    int total;
    const int start = block_excl_scan<kBlock>(s, lds, &total) + (a.part ? a.part[blockIdx.x] : 0);
    int o[kScanItems];
    int run = start;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (base + kScanItems <= a.len) {
        *reinterpret_cast<int4 *>(a.data + base) = make_int4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<int4 *>(a.data + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < a.len) a.data[base + k] = o[k];
    }
    if (kCells) {
        // occupancy bits: the 8 cells of 4 consecutive threads form one word
        unsigned bits = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) bits |= (v[k] > 0 ? 1u : 0u) << k;
        const int lane = lane_id();
        const unsigned b1 = __shfl_down(bits, 1, 64), b2 = __shfl_down(bits, 2, 64), b3 = __shfl_down(bits, 3, 64);
        if ((lane & 3) == 0 && base < a.len) p.occ[base >> 5] = bits | (b1 << 8) | (b2 << 16) | (b3 << 24);
        // one atomic per wave reserves the item slots
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
                const int first_p = o[k];
                const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, first_p);
                for (int q = 0; q < v[k]; q += 64) p.items[slot++] = make_int4((int)(base + k), first_p + q, b, 0);
            }
        }
    }
}

// In staging order into cell order; rank[k] becomes the sorted slot of staging slot k.
__global__ void __launch_bounds__(kBlock) k_scatter(Plan p)
{
    const int64_t k = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (k >= p.n) return;
    const float4 e = p.staging[k];
    const int i = __float_as_int(e.w);
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const int key = particle_cell(box_of(p, b), e.x, e.y, e.z);
    const int dst = p.cell[key] + p.rank[k];
    p.sorted[dst] = make_float4(e.x, e.y, e.z, 0.0f);
    p.perm[dst] = make_int2(i, i);
    p.rank[k] = dst;
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
// s in cell order) and the write is coalesced. Roots are counted per wave:
// a wave inside one box stores its count in wave_roots[], one that straddles
// boxes adds per lane; k_group_count sums wave_roots per box.
__global__ void __launch_bounds__(kBlock) k_resolve(Plan p)
{
    const int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int2 *out = reinterpret_cast<int2 *>(p.sorted);   // positions are no longer needed
    bool root = false;
    int b = 0;
    if (s64 < p.n) {
        const int s = (int)s64;
        b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, s64);
        const int r = p.parent[s];
        const int o = p.perm[s].x;
        const int2 pr = p.perm[r];
        const int m = pr.y;
        const int p0 = p.n_boxes == 1 ? 0 : (int)p.box_p0[b];
        out[s] = make_int2(m - p0, (o == m) ? p.gsize[r] : 0);
        root = r == s;
    }
    const int64_t wave = s64 >> 6;
    const int b0 = __shfl(b, 0, 64);
    const bool one_box = __ballot(s64 < p.n && b != b0) == 0;
    const int roots = __popcll(__ballot(root));
    if (one_box) {
        if (lane_id() == 0 && wave < p.n_waves) p.wave_roots[wave] = roots;
    } else {
        if (lane_id() == 0 && wave < p.n_waves) p.wave_roots[wave] = 0;
        if (root) atomicAdd(p.n_groups + b, 1ull);
    }
}

// n_groups[box] += sum of wave_roots over the waves of the box (a wave belongs
// to the box of its first particle). One block per box, strided.
__global__ void __launch_bounds__(kBlock) k_group_count(Plan p)
{
    __shared__ unsigned long long part[kBlock / 64];
    for (int b = blockIdx.x; b < p.n_boxes; b += gridDim.x) {
        const int64_t p0 = p.n_boxes == 1 ? 0 : p.box_p0[b];
        const int64_t p1 = p.n_boxes == 1 ? p.n : p.box_p0[b + 1];
        // waves whose first particle lies in [p0, p1)
        const int64_t w0 = (p0 + 63) >> 6, w1 = (p1 + 63) >> 6;
        unsigned long long sum = 0;
        for (int64_t w = w0 + threadIdx.x; w < w1; w += kBlock) sum += (unsigned)p.wave_roots[w];
        sum = wave_sum_u64(sum);
        if (lane_id() == 0) part[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int k = 0; k < kBlock / 64; ++k) t += part[k];
            if (t) atomicAdd(p.n_groups + b, t);
        }
        __syncthreads();
    }
}

// Back into staging order: the sorted slots of a bucket's staging slots lie in
// that bucket's window, so the reads stay local.
__global__ void __launch_bounds__(kBlock) k_unsort(Plan p)
{
    const int64_t k = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (k >= p.n) return;
    const int2 *out = reinterpret_cast<const int2 *>(p.sorted);
    int2 *staged = reinterpret_cast<int2 *>(p.staging);   // staging positions are no longer needed
    staged[k] = out[p.rank[k]];
}

// Back into input order: a tile's particles were written as one run per
// bucket, so these reads are runs too; the writes are coalesced.
__global__ void __launch_bounds__(kBlock) k_gather(Plan p)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int2 *staged = reinterpret_cast<const int2 *>(p.staging);
    const int2 v = staged[p.stpos[i]];
    p.label[i] = v.x;
    p.size[i] = v.y;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline int64_t grid_tiles(int64_t n) { return (n + kBlock - 1) / kBlock; }

// Exclusive scan of data[0, len) in place; `scratch` holds the tile sums of
// every level (scan_scratch_for(len) ints).
void scan_exclusive(int *data, int64_t len, int *scratch, const Plan &p, bool cells, hipStream_t stream)
{
    const int64_t tiles = (len + kScanTile - 1) / kScanTile;
    ScanArgs a{data, len, nullptr};
    if (tiles > 1) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kBlock), 0, stream, data, len, scratch);
        scan_exclusive(scratch, tiles, scratch + tiles, p, false, stream);
        a.part = scratch;
    }
    if (cells) hipLaunchKernelGGL((k_scan_apply<true>), dim3((unsigned)tiles), dim3(kBlock), 0, stream, a, p);
    else hipLaunchKernelGGL((k_scan_apply<false>), dim3((unsigned)tiles), dim3(kBlock), 0, stream, a, p);
}

}  // namespace

// Launch bracketed by the timer marks.
#define FOF_TIMED(id, ...)                 \
    do {                                   \
        if (t) t->mark(id, false, stream); \
        __VA_ARGS__;                       \
        if (t) t->mark(id, true, stream);  \
    } while (0)

const char *kernel_name(int k)
{
    static const char *names[K_COUNT_KERNELS] = {
        "k_clear", "k_bucket_hist", "k_bucket_scan", "k_bucket_scatter", "k_count", "k_cell_scan", "k_scatter",
        "k_link_sparse", "k_union_edges", "k_link_dense", "k_flatten", "k_resolve", "k_unsort", "k_gather"};
    return (k >= 0 && k < K_COUNT_KERNELS) ? names[k] : "?";
}

int64_t scan_scratch_for(int64_t len)
{
    int64_t total = 0;
    while (len > kScanTile) {
        len = (len + kScanTile - 1) / kScanTile;
        total += len;
    }
    return total + 1;
}

int64_t sort_tiles_for(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

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
    if (p.n > 0) {
        const unsigned tiles = (unsigned)p.n_tiles;
        FOF_TIMED(K_BUCKET_HIST, hipLaunchKernelGGL(k_bucket_hist, dim3(tiles), dim3(kBlock), 0, stream, p));
        FOF_TIMED(K_BUCKET_SCAN,
                  scan_exclusive(p.bucket_hist, (int64_t)p.n_buckets * p.n_tiles, p.scan_part, p, false, stream));
        FOF_TIMED(K_BUCKET_SCATTER,
                  hipLaunchKernelGGL(k_bucket_scatter, dim3(tiles), dim3(kBlock), 0, stream, p));
        FOF_TIMED(K_COUNT,
                  hipLaunchKernelGGL(k_count, dim3(xcd_grid(grid_tiles(p.n))), dim3(kBlock), 0, stream, p));
    }
    FOF_TIMED(K_CELL_SCAN, scan_exclusive(p.cell, p.n_cells + 1, p.scan_part, p, true, stream));
    if (p.n > 0)
        FOF_TIMED(K_SCATTER,
                  hipLaunchKernelGGL(k_scatter, dim3(xcd_grid(grid_tiles(p.n))), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

hipError_t launch_finalize(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    if (p.n == 0) return hipSuccess;
    FOF_TIMED(K_FLATTEN, hipLaunchKernelGGL(k_flatten, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_RESOLVE, {
        hipLaunchKernelGGL(k_resolve, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k_group_count, dim3((unsigned)min(p.n_boxes, 4096)), dim3(kBlock), 0, stream, p);
    });
    FOF_TIMED(K_UNSORT, hipLaunchKernelGGL(k_unsort, dim3(xcd_grid(grid_tiles(p.n))), dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_GATHER, hipLaunchKernelGGL(k_gather, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

}  // namespace fof
