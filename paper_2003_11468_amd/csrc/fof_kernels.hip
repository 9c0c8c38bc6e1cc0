// Friends-of-Friends kernels for gfx950 (CDNA4, wave64).
//
// Pipeline over all boxes at once (every kernel is a flat launch over particles
// or cells; per-box parameters come from a small descriptor table).
//
// The counting sort into cells runs in three levels so that no pass scatters
// over the whole array and no pass counts cells in global memory. Cells are
// grouped into at most 256 buckets of consecutive cell indices, and buckets
// into segments of at most 2^16 cells (a segment's occupancy bits fit in LDS).
// Cells are indexed by rank: per 32 cells an occupancy word {bits, rank base},
// and the first slot of each occupied cell only (no array per cell).
//   clear          zero the segment counts, group counters and error word
//   bucket_hist    per tile of 2048 input particles: validate coordinates,
//                  bucket histogram in LDS
//   bucket_scan    exclusive prefix over (bucket, tile) -> where each tile's
//                  share of each bucket goes
//   bucket_scatter sort each tile by bucket in LDS and write it out as runs:
//                  the "staging" order, bucket by bucket
//   seg_hist       per tile of 2048 staging slots inside one bucket: segment
//                  histogram in LDS, added to the global segment counts
//   seg_scan       exclusive prefix over the segment counts
//   seg_scatter    sort each such tile by segment in LDS and write it out as
//                  runs: the segment order
//   cell_sort      one work-group per segment: occupancy bits and rank bases,
//                  counts of the occupied cells in LDS, scan, write the
//                  occupancy words, the starts of the occupied cells and the
//                  dense link work items, then place every particle in cell
//                  order (x, y, z as float4) with its original index, and seed
//                  the union-find forest
//   link           (fof_link.hip) cell-pair link search + lock-free union-find
//   flatten  pointer jumping to the root; group minimum original index
//            (atomic min) and member count (atomic add) at the root, combined
//            over runs of equal roots (a wave's last run carries over)
//   resolve  label and size per sorted slot, stored at its staging slot
//            (writes stay in bucket windows); per-box group counts
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
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < p.n_segments; i += stride) p.seg_end[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < p.n_waves; i += stride) p.tile_dense[i] = 0ull;
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
        p.counters->n_boundary = 0;
        p.counters->n_bgroups = 0;
        p.counters->depth_max = 0;
        p.counters->depth_sum = 0;
        p.counters->giant = 0;
    }
}

// Cell key of input particle i; `ok` tells whether its coordinates are finite
// and inside [0, L).
__device__ __forceinline__ int64_t input_key(const Plan &p, int64_t i, float &x, float &y, float &z, bool &ok,
                                             BoxHint &hint)
{
    const int b = p.n_boxes == 1 ? 0 : find_box_hint(p.box_p0, p.n_boxes, i, hint);
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
    BoxHint hint;
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
            const int64_t key = input_key(p, i, x, y, z, ok, hint);
            bad |= !ok;
            atomicAdd(&cnt[(int)(key >> p.bucket_shift)], 1);
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
    BoxHint hint;
    __shared__ float4 stage[kSortTile];
    __shared__ unsigned char stage_b[kSortTile];
    __shared__ int cnt[kMaxBuckets], first[kMaxBuckets], dst0[kMaxBuckets];
    __shared__ int lds[kBlock / 64];
    // tiles go to XCDs in contiguous ranges: neighbouring tiles' runs share
    // cache lines of the staging buffer
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= p.n_tiles) return;
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
            const int64_t key = input_key(p, i, x, y, z, ok, hint);
            bk[k] = (int)(key >> p.bucket_shift);
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

__global__ void __launch_bounds__(kBlock) k_scan_apply(ScanArgs a)
{
    __shared__ int lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    load8(a.data, base, a.len, v);
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
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
}

// ---------------------------------------------------------- segment pass --

// Cell of a staged particle (x, y, z, original index as bits).
__device__ __forceinline__ int64_t staged_cell(const Plan &p, const float4 &v, BoxHint &hint)
{
    const int b = p.n_boxes == 1 ? 0 : find_box_hint(p.box_p0, p.n_boxes, __float_as_int(v.w), hint);
    return particle_cell(box_of(p, b), v.x, v.y, v.z);
}

// Tiles of the segment pass: each bucket's window of staging slots is cut
// into tiles of kSortTile, so no tile straddles buckets. Work-group g takes
// tile g of that list (the list has at most n_tiles + n_buckets entries).
// Returns the bucket, or -1 for a work-group past the last tile.
__device__ __forceinline__ int seg_tile(const Plan &p, int *info, int *lds, int &lo, int &hi)
{
    const int t = threadIdx.x;   // one bucket per thread (kBlock == kMaxBuckets)
    int start = 0, end = 0, tiles = 0;
    if (t < p.n_buckets) {
        start = p.bucket_hist[(int64_t)t * p.n_tiles];
        end = t + 1 < p.n_buckets ? p.bucket_hist[(int64_t)(t + 1) * p.n_tiles] : (int)p.n;
        tiles = (end - start + kSortTile - 1) / kSortTile;
    }
    if (t == 0) info[0] = -1;
    int total;
    const int first = block_excl_scan<kBlock>(tiles, lds, &total);   // synchronises after info[0] = -1
    const int g = (int)xcd_tile(blockIdx.x, gridDim.x);   // contiguous tile ranges per XCD
    if (g >= first && g < first + tiles) {
        info[0] = t;
        info[1] = start + (g - first) * kSortTile;
        info[2] = min(end, start + (g - first + 1) * kSortTile);
    }
    __syncthreads();
    lo = info[1];
    hi = info[2];
    return info[0];
}

constexpr int kMaxSubs = 1 << kMaxSubLog2;

// Segment histogram of one tile (LDS), added to the global segment counts.
__global__ void __launch_bounds__(kBlock) k_seg_hist(Plan p)
{
    BoxHint hint;
    __shared__ int cnt[kMaxSubs];
    __shared__ int info[3], lds[kBlock / 64];
    int lo, hi;
    const int b = seg_tile(p, info, lds, lo, hi);
    if (b < 0) return;
    const int subs = 1 << p.sub_log2;
    const int seg0 = b << p.sub_log2;
    for (int s = threadIdx.x; s < subs; s += kBlock) cnt[s] = 0;
    __syncthreads();
    for (int k = lo + (int)threadIdx.x; k < hi; k += kBlock)
        atomicAdd(&cnt[(int)(staged_cell(p, p.staging[k], hint) >> p.seg_shift) - seg0], 1);
    __syncthreads();
    for (int s = threadIdx.x; s < subs; s += kBlock)
        if (cnt[s]) atomicAdd(p.seg_end + seg0 + s, cnt[s]);
}

// Sorts one tile by segment in LDS and appends each segment's run at that
// segment's cursor (seg_end: start before, end after this pass).
__global__ void __launch_bounds__(kBlock) k_seg_scatter(Plan p)
{
    BoxHint hint;
    __shared__ float4 stage[kSortTile];
    __shared__ int stage_k[kSortTile];
    __shared__ unsigned short stage_s[kSortTile];
    __shared__ int cnt[kMaxSubs], first[kMaxSubs], dst0[kMaxSubs];
    __shared__ int info[3], lds[kBlock / 64];
    int lo, hi;
    const int b = seg_tile(p, info, lds, lo, hi);
    if (b < 0) return;
    const int subs = 1 << p.sub_log2;
    const int seg0 = b << p.sub_log2;
    for (int s = threadIdx.x; s < subs; s += kBlock) cnt[s] = 0;
    __syncthreads();
    float4 v[kSortItems];
    int sb[kSortItems], rk[kSortItems];
#pragma unroll
    for (int q = 0; q < kSortItems; ++q) {
        const int k = lo + q * kBlock + (int)threadIdx.x;
        sb[q] = -1;
        if (k < hi) {
            v[q] = p.staging[k];
            sb[q] = (int)(staged_cell(p, v[q], hint) >> p.seg_shift) - seg0;
            rk[q] = atomicAdd(&cnt[sb[q]], 1);
        }
    }
    __syncthreads();
    {
        // exclusive prefix over the segments: thread t owns `per` consecutive ones
        const int per = subs >= kBlock ? subs / kBlock : 1;
        const int s0 = (int)threadIdx.x * per;
        int c[kMaxSubs / kBlock];
        int sum = 0;
#pragma unroll
        for (int q = 0; q < kMaxSubs / kBlock; ++q) {
            c[q] = (q < per && s0 + q < subs) ? cnt[s0 + q] : 0;
            sum += c[q];
        }
        int total;
        int run = block_excl_scan<kBlock>(sum, lds, &total);
#pragma unroll
        for (int q = 0; q < kMaxSubs / kBlock; ++q)
            if (q < per && s0 + q < subs) {
                first[s0 + q] = run;
                dst0[s0 + q] = c[q] ? atomicAdd(p.seg_end + seg0 + s0 + q, c[q]) : 0;
                run += c[q];
            }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortItems; ++q)
        if (sb[q] >= 0) {
            const int at = first[sb[q]] + rk[q];
            stage[at] = v[q];
            stage_k[at] = lo + q * kBlock + (int)threadIdx.x;
            stage_s[at] = (unsigned short)sb[q];
        }
    __syncthreads();
    const int count = hi - lo;
    for (int j = threadIdx.x; j < count; j += kBlock) {
        const int s = stage_s[j];
        const int dst = dst0[s] + (j - first[s]);
        p.staging2[dst] = stage[j];
        p.stage2_k[dst] = stage_k[j];
    }
}

// ------------------------------------------------------------- cell sort --

constexpr int kSegBlock = 512;
constexpr int kSegWaves = kSegBlock / 64;
constexpr int kSegUnroll = 4;            // particles in flight per thread
constexpr int kOrderCap = 4080;          // segments up to this many particles are placed through LDS
constexpr int kCntCap = 4080;            // occupied cells counted at once (a window of ranks)
static_assert(kCntCap >= kOrderCap, "a segment placed through LDS is one window");

// One work-group per segment of 2^seg_shift consecutive cells, whose P
// particles own sorted slots [a, a + P) (seg_end). Its work grows with P and
// with the segment's occupancy words (one per 32 cells), not with its cells:
//  1. occupancy bits in LDS (an atomic OR per particle);
//  2. rank base of every word (an exclusive prefix of the popcounts); the
//     occupancy words {bits, a + base} go out. The k-th occupied cell of the
//     segment (in cell order) has rank k and stores its first slot at
//     cstart[a + k]: a segment has at most P occupied cells, so segments
//     never overlap. The entry after the last occupied cell holds e: written
//     here when the segment has fewer occupied cells than particles, else it
//     is the next segment's first entry (or the final sentinel), which is e
//     too;
// Steps 3-6 run per window of kCntCap ranks, so the LDS does not grow with
// the segment's cells (one window unless a segment placed directly has more
// occupied cells than that):
//  3. particle count per occupied cell, indexed by rank;
//  4. exclusive prefix over the occupied cells (thread t owns a run);
//  5. cell starts out, and dense link work items {cx | cy << 16, first home
//     particle, box, cz}, one per 64 particles of every cell with at least dense_min
//     particles (the cell of a rank is found from the rank bases);
//  6. place the particles: the LDS cursors give each its slot; up to
//     kOrderCap particles the slot order is kept in LDS and the outputs are
//     written in slot order (coalesced), otherwise written directly.
// A slot outside [0, P) cannot happen with consistent counts; it is latched
// as error bit 1 instead of being written.
// kWordsMax: the occupancy words of the largest segment this instance takes
// (segments of up to 2^14 cells: one word per thread, the smaller LDS
// footprint; above: several per thread).
// Position of the t-th lowest set bit of m (t < popcount(m)), by halving the
// window with population counts.
__device__ __forceinline__ int nth_bit(unsigned m, int t)
{
    int pos = 0;
#pragma unroll
    for (int w = 16; w > 0; w >>= 1) {
        const unsigned low = m & ((1u << w) - 1u);
        const int c = __popc(low);
        if (t >= c) {
            t -= c;
            m >>= w;
            pos += w;
        } else {
            m = low;
        }
    }
    return pos;
}

template <int kWordsMax>
__global__ void __launch_bounds__(kSegBlock) __attribute__((amdgpu_waves_per_eu(kWordsMax <= 1024 ? 8 : 6))) k_cell_sort(Plan p)
{
    BoxHint hint;
    constexpr int kWordsPerThread = (kWordsMax + kSegBlock - 1) / kSegBlock;
    static_assert(kWordsMax % kSegBlock == 0 || kWordsMax < kSegBlock, "whole words per thread");
    __shared__ int cnt[kCntCap];                     // per occupied cell of a window: count, start, cursor
    __shared__ unsigned bits[kWordsMax];             // occupancy of the segment's cells
    __shared__ int wbase[kWordsMax];                 // occupied cells before each word
    __shared__ unsigned short order[kOrderCap];
    __shared__ unsigned short lrank[kOrderCap];      // per particle (P <= kOrderCap): its cell, then the cell's rank
    __shared__ int lds[kSegWaves];
    __shared__ int occ_total;
    const int j = (int)blockIdx.x;
    const int words = 1 << (p.seg_shift - 5);
    const int64_t cell0 = (int64_t)j << p.seg_shift;
    const int a = j ? p.seg_end[j - 1] : 0;
    const int e = p.seg_end[j];
    const int P = e - a;
    const int tid = (int)threadIdx.x;
    const bool through_lds = P <= kOrderCap;
    const int seg_cells = words << 5;
    bool bad = false;
    // the segment's cell of a staged particle; a cell outside the segment
    // cannot happen with a consistent partition and is latched, not used
    auto local_cell = [&](const float4 &v) {
        const int64_t c = staged_cell(p, v, hint) - cell0;
        if ((uint64_t)c >= (uint64_t)seg_cells) {
            bad = true;
            return 0;
        }
        return (int)c;
    };
    for (int w = tid; w < words; w += kSegBlock) bits[w] = 0u;
    __syncthreads();

    // 1. occupancy bits (and, for a segment placed through LDS, each particle's cell)
    for (int k0 = a + tid; k0 < e; k0 += kSegUnroll * kSegBlock) {
        float4 v[kSegUnroll];
#pragma unroll
        for (int q = 0; q < kSegUnroll; ++q)
            if (k0 + q * kSegBlock < e) v[q] = p.staging2[k0 + q * kSegBlock];
#pragma unroll
        for (int q = 0; q < kSegUnroll; ++q)
            if (k0 + q * kSegBlock < e) {
                const int c = local_cell(v[q]);
                atomicOr(&bits[c >> 5], 1u << (c & 31));
                if (through_lds) lrank[k0 + q * kSegBlock - a] = (unsigned short)c;
            }
    }
    __syncthreads();

    // 2. rank bases, occupancy words out: thread t owns the wpt consecutive
    //    words t wpt .. t wpt + wpt - 1 (one word up to 2^14 cells)
    {
        const int wpt = words > kSegBlock ? words / kSegBlock : 1;
        const int w0 = tid * wpt;
        unsigned b[kWordsPerThread];
        int sum = 0;
#pragma unroll
        for (int q = 0; q < kWordsPerThread; ++q) {
            b[q] = (q < wpt && w0 + q < words) ? bits[w0 + q] : 0u;
            sum += __popc(b[q]);
        }
        int n_occ;
        int run = block_excl_scan<kSegBlock>(sum, lds, &n_occ);
#pragma unroll
        for (int q = 0; q < kWordsPerThread; ++q)
            if (q < wpt && w0 + q < words) {
                wbase[w0 + q] = run;
                p.occ[(cell0 >> 5) + w0 + q] = make_uint2(b[q], (unsigned)(a + run));
                run += __popc(b[q]);
            }
        if (tid == 0) {
            occ_total = n_occ;
            if (n_occ < P) p.cstart[a + n_occ] = e;
        }
    }
    __syncthreads();
    const int n_occ = occ_total;
    auto rank_of = [&](int c) { return wbase[c >> 5] + __popc(bits[c >> 5] & ((1u << (c & 31)) - 1u)); };

    // 3.-6. per window of kCntCap ranks: one window, unless the segment is
    // placed directly and has more occupied cells than that (then every
    // window reads the segment's particles again)
    int slot0 = 0;   // local slot of the window's first particle
    for (int r0 = 0; r0 < n_occ; r0 += kCntCap) {
        const int nw = min(kCntCap, n_occ - r0);
        for (int k = tid; k < nw; k += kSegBlock) cnt[k] = 0;
        __syncthreads();

        // 3. particles per occupied cell of the window
        if (through_lds) {   // a single window: n_occ <= P <= kOrderCap <= kCntCap
            for (int idx = tid; idx < P; idx += kSegBlock) {
                const int r = rank_of(lrank[idx]);
                lrank[idx] = (unsigned short)r;
                atomicAdd(&cnt[r], 1);
            }
        } else {
            constexpr int kCountUnroll = 2;
            for (int k0 = a + tid; k0 < e; k0 += kCountUnroll * kSegBlock) {
                float4 v[kCountUnroll];
#pragma unroll
                for (int q = 0; q < kCountUnroll; ++q)
                    if (k0 + q * kSegBlock < e) v[q] = p.staging2[k0 + q * kSegBlock];
#pragma unroll
                for (int q = 0; q < kCountUnroll; ++q)
                    if (k0 + q * kSegBlock < e) {
                        const int r = rank_of(local_cell(v[q])) - r0;
                        if ((unsigned)r < (unsigned)nw) atomicAdd(&cnt[r], 1);
                    }
            }
        }
        __syncthreads();

        // 4. exclusive prefix over the window's occupied cells (local slots)
        int total;
        {
            const int per = (nw + kSegBlock - 1) / kSegBlock;
            const int k0 = tid * per;
            const int k1 = min(k0 + per, nw);
            int sum = 0;
            for (int k = k0; k < k1; ++k) sum += cnt[k];
            int run = slot0 + block_excl_scan<kSegBlock>(sum, lds, &total);
            for (int k = k0; k < k1; ++k) {
                const int v = cnt[k];
                cnt[k] = run;
                run += v;
            }
        }
        __syncthreads();

        // 5. cell starts, dense work items
        {
            const int lane = lane_id();
            for (int kb = 0; kb < nw; kb += kSegBlock) {
                const int k = kb + tid;
                int v = 0, start = 0;
                if (k < nw) {
                    const int st = cnt[k];
                    v = (k + 1 < nw ? cnt[k + 1] : slot0 + total) - st;
                    start = a + st;
                    p.cstart[a + r0 + k] = start;
                }
                const int chunks = (k < nw && v >= p.dense_min) ? (v + 63) >> 6 : 0;
                if (__ballot(chunks > 0)) {
                    const int cincl = wave_incl_scan(chunks);
                    const int wave_items = __shfl(cincl, 63, 64);
                    int slot = 0;
                    if (lane == 63) slot = (int)atomicAdd(&p.counters->n_items, (unsigned)wave_items);
                    slot = __shfl(slot, 63, 64) + cincl - chunks;
                    if (chunks) {
                        // the word holding rank r0 + k: the last one whose base is at most that
                        const int rk = r0 + k;
                        int lo = 0, hi = words - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (wbase[mid] <= rk) lo = mid;
                            else hi = mid - 1;
                        }
                        const int64_t gc = cell0 + (lo << 5) + nth_bit(bits[lo], rk - wbase[lo]);
                        // the segment's box, kept from step 1, unless the cell lies in another
                        const int bx = p.n_boxes == 1 ? 0 : find_box_hint(p.box_p0, p.n_boxes, start, hint);
                        // the cell's coordinates in its box: local < nc^3 <= 2^33 and the
                        // divisors are below 2^22, so the double quotients truncate exactly
                        const BoxDev &bd = box_of(p, bx);
                        const int nc = bd.nc;
                        const int64_t local = gc - bd.cell_base, nc2 = (int64_t)nc * nc;
                        const int cz = (int)((double)local / (double)nc2);
                        const int rem = (int)(local - cz * nc2);
                        const int cy = (int)((double)rem / (double)nc);
                        const int cx = rem - cy * nc;
                        for (int q = 0; q < v; q += 64, ++slot)
                            if (slot < p.max_items) p.items[slot] = make_int4(cx | (cy << 16), start + q, bx, cz);
                        // the cell's slots, in the masks by which the per-particle search skips dense tiles
                        for (int s0 = start; s0 < start + v;) {
                            const int lo = s0 & 63, hi = min(64, lo + (start + v - s0));
                            const unsigned long long m = (hi == 64 ? ~0ull : (1ull << hi) - 1ull) & ~((1ull << lo) - 1ull);
                            atomicOr(&p.tile_dense[s0 >> 6], m);
                            s0 += hi - lo;
                        }
                    }
                }
            }
        }
        __syncthreads();

        // 6. placement: the slot order in LDS (ranks known from step 3), or direct writes
        if (through_lds) {
            for (int idx = tid; idx < P; idx += kSegBlock) {
                const int local = atomicAdd(&cnt[lrank[idx]], 1);
                if ((unsigned)local >= (unsigned)P) bad = true;
                else order[local] = (unsigned short)idx;
            }
        } else {
            constexpr int kPlaceUnroll = 2;
            for (int k0 = a + tid; k0 < e; k0 += kPlaceUnroll * kSegBlock) {
                float4 v[kPlaceUnroll];
                int kk[kPlaceUnroll];
#pragma unroll
                for (int q = 0; q < kPlaceUnroll; ++q)
                    if (k0 + q * kSegBlock < e) {
                        v[q] = p.staging2[k0 + q * kSegBlock];
                        kk[q] = p.stage2_k[k0 + q * kSegBlock];
                    }
#pragma unroll
                for (int q = 0; q < kPlaceUnroll; ++q) {
                    if (k0 + q * kSegBlock >= e) continue;
                    const int r = rank_of(local_cell(v[q])) - r0;
                    if ((unsigned)r >= (unsigned)nw) continue;   // another window's particle
                    const int local = atomicAdd(&cnt[r], 1);
                    if ((unsigned)local >= (unsigned)P) {
                        bad = true;
                        continue;
                    }
                    const int dst = a + local;
                    const int i = __float_as_int(v[q].w);
                    p.sorted[dst] = make_float4(v[q].x, v[q].y, v[q].z, 0.0f);
                    p.orig[dst] = i;
                    p.gmin[dst] = i;
                    p.parent[dst] = dst;
                    p.gsize[dst] = 1;
                    p.kmap[dst] = kk[q];
                }
            }
        }
        slot0 += total;
        __syncthreads();   // the next window clears cnt
    }
    // the final sentinel (the end of the last occupied cell, and the padding
    // of 16-byte reads) and the two occupancy words after the last segment
    // (the end of the last cell when the cells fill it exactly)
    if (j + 1 == (int)gridDim.x && tid < 4) {
        p.cstart[p.n + tid] = (int)p.n;
        if (tid < 2) p.occ[((int64_t)gridDim.x << (p.seg_shift - 5)) + tid] = make_uint2(0u, (unsigned)p.n);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&p.counters->error, 2u);
    if (!through_lds) return;
    __syncthreads();
    for (int d0 = tid; d0 < P; d0 += kSegUnroll * kSegBlock) {
        float4 v[kSegUnroll];
        int from[kSegUnroll], k_of[kSegUnroll];
#pragma unroll
        for (int q = 0; q < kSegUnroll; ++q)
            if (d0 + q * kSegBlock < P) {
                from[q] = a + order[d0 + q * kSegBlock];
                v[q] = p.staging2[from[q]];
                k_of[q] = p.stage2_k[from[q]];
            }
#pragma unroll
        for (int q = 0; q < kSegUnroll; ++q)
            if (d0 + q * kSegBlock < P) {
                const int dst = a + d0 + q * kSegBlock;
                const int i = __float_as_int(v[q].w);
                p.sorted[dst] = make_float4(v[q].x, v[q].y, v[q].z, 0.0f);
                p.orig[dst] = i;
                p.gmin[dst] = i;
                p.parent[dst] = dst;
                p.gsize[dst] = 1;
                p.kmap[dst] = k_of[q];
            }
    }
}

// Statistics only, before the flatten: the length of every particle's path
// to its root (the find depth that the cost of linking depends on, paper,
// Section 4), as a maximum and a sum.
__global__ void __launch_bounds__(kBlock) k_find_depth(Plan p)
{
    unsigned dmax = 0;
    unsigned long long dsum = 0;
    for (int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x; s64 < p.n; s64 += (int64_t)gridDim.x * kBlock) {
        unsigned d = 0;
        int r = (int)s64;
        for (int q = p.parent[r]; q != r; q = p.parent[r]) {
            r = q;
            ++d;
        }
        dmax = max(dmax, d);
        dsum += d;
    }
    // one pair of atomics per wave, after its whole share of the particles
    for (int k = 32; k >= 1; k >>= 1) dmax = max(dmax, (unsigned)__shfl_xor((int)dmax, k, 64));
    dsum = wave_sum_u64(dsum);
    if (lane_id() == 0) {
        atomicMax(&p.counters->depth_max, dmax);
        atomicAdd(&p.counters->depth_sum, dsum);
    }
}

// Consecutive sorted particles often share their root, so the root updates of
// runs of equal roots in a wave are combined before the atomics. The run that
// ends at the wave's last lane stays pending into the wave's next stretch of
// particles and is merged with its first run when the root is the same: the
// atomics on the root of one giant group (every particle of the box, in the
// worst case) then come to one pair per wave instead of one per 64 particles.
__global__ void __launch_bounds__(kBlock) k_flatten(Plan p)
{
    constexpr int kFlatIlp = 4;   // stretches whose chases advance together
    const int lane = lane_id();
    int pend_key = -1, pend_m = INT_MAX, pend_c = 0;   // the same in every lane
    const int64_t stretch = (int64_t)gridDim.x * kBlock;
    for (int64_t base0 = (int64_t)blockIdx.x * kBlock; base0 < p.n; base0 += kFlatIlp * stretch) {
        // the roots of this thread's particle in each of kFlatIlp stretches
        int r[kFlatIlp], q[kFlatIlp];
        bool live[kFlatIlp];
#pragma unroll
        for (int u = 0; u < kFlatIlp; ++u) {
            const int64_t s64 = base0 + u * stretch + threadIdx.x;
            live[u] = s64 < p.n;
            r[u] = live[u] ? (int)s64 : 0;
        }
#pragma unroll
        for (int u = 0; u < kFlatIlp; ++u) q[u] = p.parent[r[u]];
        while (true) {
            bool more = false;
#pragma unroll
            for (int u = 0; u < kFlatIlp; ++u) more = more || q[u] != r[u];
            if (!more) break;
#pragma unroll
            for (int u = 0; u < kFlatIlp; ++u)
                if (q[u] != r[u]) r[u] = q[u];
#pragma unroll
            for (int u = 0; u < kFlatIlp; ++u) q[u] = p.parent[r[u]];
        }
#pragma unroll
        for (int u = 0; u < kFlatIlp; ++u) {
            const int64_t base = base0 + u * stretch;
            if (base >= p.n) break;   // uniform: later stretches are past the end too
            const int64_t s64 = base + threadIdx.x;
            int root_key = -1, m = INT_MAX, c = 0;
            if (live[u]) {
                const int s = (int)s64;
                if (r[u] != s) {
                    p.parent[s] = r[u];
                    root_key = r[u];
                    m = p.orig[s];
                    c = 1;
                }
            }
            const int prev = __shfl_up(root_key, 1, 64);
            const unsigned long long heads = __ballot(lane == 0 || prev != root_key);
            const int last_head = 63 - __clzll((long long)heads);   // first lane of the run holding lane 63
            const int key_first = __shfl(root_key, 0, 64), key_last = __shfl(root_key, 63, 64);
            const bool head = wave_runs_min_add(root_key, m, c);
            if (pend_key >= 0) {
                if (pend_key == key_first) {
                    if (lane == 0) {   // lane 0 heads the first run
                        m = min(m, pend_m);
                        c += pend_c;
                    }
                } else if (lane == 0) {
                    atomicMin(&p.gmin[pend_key], pend_m);
                    atomicAdd(&p.gsize[pend_key], pend_c);
                }
            }
            const int lm = __shfl(m, last_head, 64), lc = __shfl(c, last_head, 64);
            if (head && lane != last_head) {
                atomicMin(&p.gmin[root_key], m);
                atomicAdd(&p.gsize[root_key], c);
            }
            pend_key = key_last;
            pend_m = lm;
            pend_c = lc;
        }
    }
    if (pend_key >= 0 && lane == 0) {
        atomicMin(&p.gmin[pend_key], pend_m);
        atomicAdd(&p.gsize[pend_key], pend_c);
    }
}

// Resolve, in sorted order: {group label (box-local), size at the member whose
// index is the label, else 0}, stored at the particle's staging slot (kmap).
// Reads are local (the root of s sits near s in cell order); the staging
// slots of a stretch of sorted slots lie in a few bucket windows, and tiles go
// to XCDs in contiguous ranges, so the scattered writes combine in each XCD's
// L2. Roots are counted per wave: a wave inside one box stores its count in
// wave_roots[], one that straddles boxes adds per lane; k_group_count sums
// wave_roots per box.
__device__ __forceinline__ void resolve_tile(const Plan &p, int64_t s64)
{
    int2 *staged = reinterpret_cast<int2 *>(p.staging);   // staged positions are no longer needed
    bool root = false;
    int b = 0;
    if (s64 < p.n) {
        const int s = (int)s64;
        b = p.n_boxes == 1 ? 0 : find_box_wave(p.box_p0, p.n_boxes, s64);
        const int r = p.parent[s];
        const int o = p.orig[s];
        const int m = p.gmin[r];
        const int p0 = p.n_boxes == 1 ? 0 : (int)p.box_p0[b];
        staged[p.kmap[s]] = make_int2(m - p0, (o == m) ? p.gsize[r] : 0);
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

__global__ void __launch_bounds__(kBlock) k_resolve(Plan p)
{
    resolve_tile(p, xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x);
}

// n_groups[box] += sum of wave_roots over the waves of the box (a wave belongs
// to the box of its first particle). Each work-group sums a contiguous run of
// kGroupRun entries; boxes are contiguous in the wave index, so a single box
// takes one atomic per work-group and several boxes one per box per wave.
constexpr int kGroupItems = 4;
constexpr int kGroupRun = kBlock * kGroupItems;

__global__ void __launch_bounds__(kBlock) k_group_count(Plan p)
{
    __shared__ unsigned long long part[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kGroupRun;
    if (p.n_boxes == 1) {
        unsigned long long sum = 0;
#pragma unroll
        for (int k = 0; k < kGroupItems; ++k) {
            const int64_t w = base + k * kBlock + threadIdx.x;
            if (w < p.n_waves) sum += (unsigned)p.wave_roots[w];
        }
        sum = wave_sum_u64(sum);
        if (lane_id() == 0) part[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int k = 0; k < kBlock / 64; ++k) t += part[k];
            if (t) atomicAdd(p.n_groups, t);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kGroupItems; ++k) {
        const int64_t w = base + k * kBlock + threadIdx.x;
        int key = -1;
        unsigned long long v = 0;
        if (w < p.n_waves) {
            v = (unsigned)p.wave_roots[w];
            if (v) key = find_box(p.box_p0, p.n_boxes, w << 6);
        }
        wave_add_by_key(p.n_groups, key, v);
    }
}

// Back into input order: a tile's particles were written as one run per
// bucket, so these reads are runs too; the writes are coalesced.
__global__ void __launch_bounds__(kBlock) k_gather(Plan p)
{
    const int64_t i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int2 *staged = reinterpret_cast<const int2 *>(p.staging);
    const int2 v = staged[p.stpos[i]];
    p.label[i] = v.x;
    p.size[i] = v.y;
}

// Relink: every particle its own group again; counters of the link and
// finalize passes cleared (the dense item count of the build is kept).
__global__ void __launch_bounds__(kBlock) k_relink_reset(Plan p)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < p.n; s += stride) {
        p.parent[s] = (int)s;
        p.gsize[s] = 1;
        p.gmin[s] = p.orig[s];
    }
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < p.n_boxes) p.n_groups[t] = 0;
    if (t < kEdgeSlices) p.edge_fill[t] = 0;
    if (t == 0) {
        p.counters->pair_tests = 0;
        p.counters->links = 0;
        p.counters->band_hits = 0;
        p.counters->cas_retries = 0;
        p.counters->sparse_tests = 0;
        p.counters->n_edges = 0;
        p.counters->n_boundary = 0;
        p.counters->n_bgroups = 0;
        p.counters->depth_max = 0;
        p.counters->depth_sum = 0;
    }
}

__global__ void k_clear_ints(int *a, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = 0;
}

// ------------------------------------------------------------- catalogue --
// Groups of at least min_size members, in input order (box by box, label
// ascending): a group appears once, at the particle whose index is its label,
// the only one with a non-zero size. Per tile of kSortTile particles: count,
// then an exclusive prefix over the tiles, then each tile writes its groups
// in order (thread t owns kSortItems consecutive particles).

__global__ void __launch_bounds__(kBlock) k_cat_count(const Plan p, const int32_t *size, int min_size, int *tile_count)
{
    __shared__ int lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    int c = 0;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) c += (base + k < p.n && size[base + k] >= min_size) ? 1 : 0;
    int total;
    block_excl_scan<kBlock>(c, lds, &total);
    if (threadIdx.x == 0) tile_count[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) k_cat_write(const Plan p, const int32_t *label, const int32_t *size,
                                                      int min_size, const int *tile_off, int32_t *g_first,
                                                      int32_t *g_size, int32_t *g_box, int64_t capacity)
{
    __shared__ int lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    bool take[kSortItems];
    int c = 0;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        take[k] = base + k < p.n && size[base + k] >= min_size;
        c += take[k] ? 1 : 0;
    }
    int total;
    int64_t at = (int64_t)tile_off[blockIdx.x] + block_excl_scan<kBlock>(c, lds, &total);
#pragma unroll
    for (int k = 0; k < kSortItems; ++k)
        if (take[k]) {
            if (at < capacity) {
                const int64_t i = base + k;
                g_first[at] = label[i];
                g_size[at] = size[i];
                if (g_box) g_box[at] = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
            }
            ++at;
        }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Grid of the persistent flatten: a few work-groups per compute unit, each
// looping over tiles (measured faster than one work-group per tile).
constexpr int64_t kStreamBlocks = 2048;
inline int64_t grid_tiles(int64_t n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

// Exclusive scan of data[0, len) in place; `scratch` holds the tile sums of
// every level (scan_scratch_for(len) ints).
void scan_exclusive(int *data, int64_t len, int *scratch, hipStream_t stream)
{
    const int64_t tiles = (len + kScanTile - 1) / kScanTile;
    ScanArgs a{data, len, nullptr};
    if (tiles > 1) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kBlock), 0, stream, data, len, scratch);
        scan_exclusive(scratch, tiles, scratch + tiles, stream);
        a.part = scratch;
    }
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kBlock), 0, stream, a);
}


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
        "k_clear", "k_bucket_hist", "k_bucket_scan", "k_bucket_scatter", "k_seg_hist", "k_seg_scan", "k_seg_scatter",
        "k_cell_sort",
        "k_link_sparse", "k_union_edges", "k_dense_premerge", "k_link_dense", "k_flatten", "k_resolve", "k_gather"};
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
    int64_t work = p.n_segments > p.n_boxes ? p.n_segments : p.n_boxes;
    if (work < p.n_waves) work = p.n_waves;
    if (work < kEdgeSlices) work = kEdgeSlices;
    unsigned g = grid_for(work);
    if (g > 65536u) g = 65536u;
    FOF_TIMED(K_CLEAR, hipLaunchKernelGGL(k_clear, dim3(g), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

hipError_t launch_build(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    const unsigned seg_tiles = xcd_grid(p.n_tiles + p.n_buckets);
    if (p.n > 0) {
        const unsigned tiles = (unsigned)p.n_tiles;
        FOF_TIMED(K_BUCKET_HIST, hipLaunchKernelGGL(k_bucket_hist, dim3(tiles), dim3(kBlock), 0, stream, p));
        FOF_TIMED(K_BUCKET_SCAN, scan_exclusive(p.bucket_hist, (int64_t)p.n_buckets * p.n_tiles, p.scan_part, stream));
        FOF_TIMED(K_BUCKET_SCATTER,
                  hipLaunchKernelGGL(k_bucket_scatter, dim3(xcd_grid(tiles)), dim3(kBlock), 0, stream, p));
        FOF_TIMED(K_SEG_HIST, hipLaunchKernelGGL(k_seg_hist, dim3(seg_tiles), dim3(kBlock), 0, stream, p));
    }
    FOF_TIMED(K_SEG_SCAN, scan_exclusive(p.seg_end, p.n_segments, p.scan_part, stream));
    if (p.n > 0)
        FOF_TIMED(K_SEG_SCATTER, hipLaunchKernelGGL(k_seg_scatter, dim3(seg_tiles), dim3(kBlock), 0, stream, p));
    const dim3 grid((unsigned)p.n_segments), block(kSegBlock);
    if (p.seg_shift <= 14)
        FOF_TIMED(K_CELL_SORT, hipLaunchKernelGGL(k_cell_sort<(1 << 14) / 32>, grid, block, 0, stream, p));
    else if (p.seg_shift == 15)
        FOF_TIMED(K_CELL_SORT, hipLaunchKernelGGL(k_cell_sort<(1 << 15) / 32>, grid, block, 0, stream, p));
    else
        FOF_TIMED(K_CELL_SORT, hipLaunchKernelGGL(k_cell_sort<(1 << kSegLog2Max) / 32>, grid, block, 0, stream, p));
    return hipGetLastError();
}

hipError_t launch_catalogue(const Plan &p, const int32_t *label, const int32_t *size, int min_size,
                            int32_t *g_first, int32_t *g_size, int32_t *g_box, int64_t capacity, hipStream_t stream)
{
    // tile counts go to the bucket histogram (free after the build), then an
    // exclusive prefix over n_tiles + 1 entries leaves the total in the last
    int *count = p.bucket_hist;
    const unsigned tiles = (unsigned)p.n_tiles;
    hipLaunchKernelGGL(k_clear_ints, dim3(1), dim3(kBlock), 0, stream, count + p.n_tiles, 1);
    if (tiles) hipLaunchKernelGGL(k_cat_count, dim3(tiles), dim3(kBlock), 0, stream, p, size, min_size, count);
    scan_exclusive(count, p.n_tiles + 1, p.scan_part, stream);
    if (tiles)
        hipLaunchKernelGGL(k_cat_write, dim3(tiles), dim3(kBlock), 0, stream, p, label, size, min_size, count,
                           g_first, g_size, g_box, capacity);
    return hipGetLastError();
}

hipError_t launch_relink_reset(const Plan &p, hipStream_t stream)
{
    int64_t work = p.n > p.n_boxes ? p.n : p.n_boxes;
    if (work < kEdgeSlices) work = kEdgeSlices;
    unsigned g = grid_for(work);
    if (g > 65536u) g = 65536u;
    hipLaunchKernelGGL(k_relink_reset, dim3(g), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_finalize(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    if (p.n == 0) return hipSuccess;
    const unsigned flatten_grid = (unsigned)min(kStreamBlocks, grid_tiles(p.n));
    if (p.stats) hipLaunchKernelGGL(k_find_depth, dim3(flatten_grid), dim3(kBlock), 0, stream, p);
    FOF_TIMED(K_FLATTEN, hipLaunchKernelGGL(k_flatten, dim3(flatten_grid), dim3(kBlock), 0, stream, p));
    FOF_TIMED(K_RESOLVE, {
        hipLaunchKernelGGL(k_resolve, dim3(xcd_grid(grid_tiles(p.n))), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k_group_count, dim3((unsigned)((p.n_waves + kGroupRun - 1) / kGroupRun)), dim3(kBlock), 0,
                           stream, p);
    });
    FOF_TIMED(K_GATHER, hipLaunchKernelGGL(k_gather, dim3(xcd_grid(grid_tiles(p.n))), dim3(kBlock), 0, stream, p));
    return hipGetLastError();
}

}  // namespace fof
