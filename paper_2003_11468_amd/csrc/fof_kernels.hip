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
//   link     each particle tests its own cell and the 13 half-shell neighbour
//            cells; linked pairs are merged with lock-free union-find
//   flatten  pointer jumping to the root; group minimum original index
//            (atomic min) and member count (atomic add) at the root
//   output   labels and sizes in input order, per-box group counts
//
// The whole translation unit is compiled with -ffp-contract=off: the double
// predicate below must round every product and sum separately. The FP32
// filter requests its fused multiply-adds explicitly (fmaf), which its error
// bound allows.
#include "fof_internal.h"

namespace fof {
namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = kBlock * kScanItems;      // 2048 counts per tile
constexpr int kPartBlock = 1024;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int find_box(const int64_t *p0, int n_boxes, int64_t i)
{
    int lo = 0, hi = n_boxes - 1;   // last box whose first particle is <= i
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (p0[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Cell coordinate along one axis: floor(x * nc / L) clamped to [0, nc - 1].
// The product is formed in double, so for L = 1 it is exact; a NaN lands in
// cell 0 (the coordinate error is latched separately).
__device__ __forceinline__ int cell_coord(float x, double inv_h, int nc)
{
    double t = (double)x * inv_h;
    t = fmin(fmax(t, 0.0), (double)(nc - 1));
    return (int)t;
}

__device__ __forceinline__ bool in_box(float x, double L)
{
    double d = (double)x;
    return d >= 0.0 && d < L;  // false for NaN and infinities
}

// The link predicate, in double, exactly as the oracle states it: subtract,
// wrap to the minimum image, square and sum left to right, no FMA.
__device__ __forceinline__ bool link_fp64(float ax, float ay, float az, float bx, float by, float bz,
                                          double L, double half, double l2, bool strict)
{
    double tx = (double)ax - (double)bx;
    if (tx > half) tx = tx - L;
    else if (tx < -half) tx = tx + L;
    double ty = (double)ay - (double)by;
    if (ty > half) ty = ty - L;
    else if (ty < -half) ty = ty + L;
    double tz = (double)az - (double)bz;
    if (tz > half) tz = tz - L;
    else if (tz < -half) tz = tz + L;
    double sxy = tx * tx + ty * ty;
    double r2 = sxy + tz * tz;
    return strict ? (r2 < l2) : (r2 <= l2);
}

// ------------------------------------------------------------ union-find --
// parent[] is read and written with device-scope relaxed atomics: the eight
// XCDs have private L2 caches, and plain loads could keep returning a stale
// line while other XCDs hook roots.

__device__ __forceinline__ int ld_rel(const int *a)
{
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_rel(int *a, int v)
{
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving: each visited node is re-pointed to its
// grandparent. The store may race with other finds; every value written is an
// ancestor of the node with a smaller index, so the forest stays valid.
__device__ __forceinline__ int find_halve(int *parent, int x)
{
    while (true) {
        int px = ld_rel(parent + x);
        if (px == x) return x;
        int gx = ld_rel(parent + px);
        if (gx == px) return px;
        st_rel(parent + x, gx);
        x = gx;
    }
}

// Merge the groups of a and b: hook the larger root under the smaller with a
// compare-and-swap that expects the larger root to still be a root. On failure
// the CAS returns the node's new parent, and the search continues from there.
__device__ __forceinline__ unsigned unite(int *parent, int a, int b)
{
    unsigned retries = 0;
    while (true) {
        a = find_halve(parent, a);
        b = find_halve(parent, b);
        if (a == b) return retries;
        int lo = a < b ? a : b;
        int hi = a < b ? b : a;
        int expected = hi;
        if (__hip_atomic_compare_exchange_strong(parent + hi, &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return retries;
        ++retries;
        a = expected;
        b = lo;
    }
}

// ------------------------------------------------------------ wave utils --

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = lane_id();
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over the block; `lds` holds one int per wave. Returns the
// exclusive prefix of v and the block total in *total.
template <int kThreads>
__device__ __forceinline__ int block_excl_scan(int v, int *lds, int *total)
{
    constexpr int kWaves = kThreads / 64;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        int s = lds[w];
        off += (w < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// One atomic add per distinct key among the lanes of a wave (key < 0: none).
__device__ __forceinline__ void wave_count_by_key(unsigned long long *arr, int key)
{
    unsigned long long todo = __ballot(key >= 0);
    while (todo) {
        int leader = __ffsll((long long)todo) - 1;
        int k = __shfl(key, leader, 64);
        unsigned long long same = __ballot(key == k) & todo;
        if (lane_id() == leader) atomicAdd(arr + k, (unsigned long long)__popcll(same));
        todo &= ~same;
    }
}

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
        p.counters->error = 0;
    }
}

__device__ __forceinline__ int particle_cell(const BoxDev &bd, float x, float y, float z)
{
    const int nc = bd.nc;
    int cx = cell_coord(x, bd.inv_h, nc);
    int cy = cell_coord(y, bd.inv_h, nc);
    int cz = cell_coord(z, bd.inv_h, nc);
    return (int)(bd.cell_base + ((int64_t)cz * nc + cy) * nc + cx);
}

__global__ void __launch_bounds__(kBlock) k_count(Plan p)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const BoxDev bd = p.boxes[b];
    const float x = p.pos[3 * i + 0], y = p.pos[3 * i + 1], z = p.pos[3 * i + 2];
    if (!(in_box(x, bd.L) && in_box(y, bd.L) && in_box(z, bd.L))) atomicOr(&p.counters->error, 1u);
    const int key = particle_cell(bd, x, y, z);
    p.rank[i] = atomicAdd(p.cell + key, 1);
    p.parent[i] = (int)i;
    p.gsize[i] = 1;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(Plan p)
{
    __shared__ int lds[kBlock / 64];
    const int64_t m = p.n_cells + 1;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += p.cell[base + k];
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

__global__ void __launch_bounds__(kBlock) k_scan_apply(Plan p)
{
    __shared__ int lds[kBlock / 64];
    const int64_t m = p.n_cells + 1;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? p.cell[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_excl_scan<kBlock>(s, lds, &total) + p.scan_part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) p.cell[base + k] = run;
        run += v[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter(Plan p)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, i);
    const BoxDev bd = p.boxes[b];
    const float x = p.pos[3 * i + 0], y = p.pos[3 * i + 1], z = p.pos[3 * i + 2];
    const int key = particle_cell(bd, x, y, z);
    const int dst = p.cell[key] + p.rank[i];
    p.sorted[dst] = make_float4(x, y, z, 0.0f);
    p.perm[dst] = make_int2((int)i, (int)i);
}

// Tests particle s against the sorted particles [j0, j1). The FP32 distance
// uses the home coordinate hx (x or x - L) and the neighbour shift cx (0 or L)
// so that every subtraction of a periodic image is exact: with the home in the
// top cell, x - L is exact (Sterbenz); with the neighbour in the top cell,
// xj - L is. Each axis difference then carries one rounding only.
template <bool kStats>
__device__ __forceinline__ void scan_range(const Plan &p, const BoxDev &bd, bool fp64, int s, float4 pi, int j0,
                                           int j1, float hx, float hy, float hz, float sx, float sy, float sz,
                                           unsigned long long &tests, unsigned long long &links,
                                           unsigned long long &band, unsigned long long &retries)
{
    const bool strict = p.strict != 0;
    for (int j = j0; j < j1; ++j) {
        const float4 pj = p.sorted[j];
        bool link;
        if (fp64) {
            link = link_fp64(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, bd.L, bd.half, bd.l2, strict);
        } else {
            const float dx = hx - (pj.x - sx);
            const float dy = hy - (pj.y - sy);
            const float dz = hz - (pj.z - sz);
            const float r = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            if (r < bd.lo32) link = true;
            else if (r > bd.hi32) link = false;
            else {
                if (kStats) ++band;
                link = link_fp64(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, bd.L, bd.half, bd.l2, strict);
            }
        }
        if (kStats) ++tests;
        if (link) {
            if (kStats) ++links;
            unsigned r = unite(p.parent, s, j);
            if (kStats) retries += r;
        }
    }
}

template <bool kStats>
__global__ void __launch_bounds__(kBlock) k_link(Plan p)
{
    const int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long tests = 0, links = 0, band = 0, retries = 0;
    if (s64 < p.n) {
        const int s = (int)s64;
        const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, s64);
        const BoxDev bd = p.boxes[b];
        const bool fp64 = p.predicate == 0 || bd.use_fp64;
        const float4 pi = p.sorted[s];
        const int nc = bd.nc;
        const int cx = cell_coord(pi.x, bd.inv_h, nc);
        const int cy = cell_coord(pi.y, bd.inv_h, nc);
        const int cz = cell_coord(pi.z, bd.inv_h, nc);
        const int cb = (int)bd.cell_base;
        const float L32 = bd.L32;
        const int *cell = p.cell;

        // Own row: the rest of the own cell (sorted index above s) and cell cx + 1.
        int rb = cb + (cz * nc + cy) * nc;
        if (cx + 1 < nc) {
            scan_range<kStats>(p, bd, fp64, s, pi, s + 1, cell[rb + cx + 2], pi.x, pi.y, pi.z, 0.f, 0.f, 0.f,
                               tests, links, band, retries);
        } else {
            scan_range<kStats>(p, bd, fp64, s, pi, s + 1, cell[rb + nc], pi.x, pi.y, pi.z, 0.f, 0.f, 0.f, tests,
                               links, band, retries);
            scan_range<kStats>(p, bd, fp64, s, pi, cell[rb], cell[rb + 1], pi.x - L32, pi.y, pi.z, 0.f, 0.f, 0.f,
                               tests, links, band, retries);
        }
        // Rows (dy, dz) = (1, 0), (-1, 1), (0, 1), (1, 1): with the own row these
        // hold the 13 half-shell neighbour cells.
        const int dys[4] = {1, -1, 0, 1};
        const int dzs[4] = {0, 1, 1, 1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int ny = cy + dys[k], nz = cz + dzs[k];
            float hy = pi.y, sy = 0.f, hz = pi.z;
            if (ny >= nc) { ny -= nc; hy = pi.y - L32; }
            else if (ny < 0) { ny += nc; sy = L32; }
            if (nz >= nc) { nz -= nc; hz = pi.z - L32; }
            rb = cb + (nz * nc + ny) * nc;
            if (cx >= 1 && cx + 1 < nc) {
                scan_range<kStats>(p, bd, fp64, s, pi, cell[rb + cx - 1], cell[rb + cx + 2], pi.x, hy, hz, 0.f, sy,
                                   0.f, tests, links, band, retries);
            } else if (cx == 0) {
                scan_range<kStats>(p, bd, fp64, s, pi, cell[rb], cell[rb + 2], pi.x, hy, hz, 0.f, sy, 0.f, tests,
                                   links, band, retries);
                scan_range<kStats>(p, bd, fp64, s, pi, cell[rb + nc - 1], cell[rb + nc], pi.x, hy, hz, L32, sy,
                                   0.f, tests, links, band, retries);
            } else {
                scan_range<kStats>(p, bd, fp64, s, pi, cell[rb + nc - 2], cell[rb + nc], pi.x, hy, hz, 0.f, sy,
                                   0.f, tests, links, band, retries);
                scan_range<kStats>(p, bd, fp64, s, pi, cell[rb], cell[rb + 1], pi.x - L32, hy, hz, 0.f, sy, 0.f,
                                   tests, links, band, retries);
            }
        }
    }
    if (kStats) {
        tests = wave_sum_u64(tests);
        links = wave_sum_u64(links);
        band = wave_sum_u64(band);
        retries = wave_sum_u64(retries);
        if (lane_id() == 0) {
            atomicAdd(&p.counters->pair_tests, tests);
            atomicAdd(&p.counters->links, links);
            atomicAdd(&p.counters->band_hits, band);
            atomicAdd(&p.counters->cas_retries, retries);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_flatten(Plan p)
{
    const int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s64 >= p.n) return;
    const int s = (int)s64;
    int r = s, q = p.parent[s];
    while (q != r) {
        r = q;
        q = p.parent[r];
    }
    if (r != s) {
        p.parent[s] = r;
        atomicMin(&p.perm[r].y, p.perm[s].x);
        atomicAdd(p.gsize + r, 1);
    }
}

__global__ void __launch_bounds__(kBlock) k_output(Plan p)
{
    const int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int key = -1;
    if (s64 < p.n) {
        const int s = (int)s64;
        const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, s64);
        const int r = p.parent[s];
        const int o = p.perm[s].x;
        const int m = p.perm[r].y;
        const int p0 = (int)p.box_p0[b];
        p.label[o] = m - p0;
        p.size[o] = (o == m) ? p.gsize[r] : 0;
        if (r == s) key = b;
    }
    wave_count_by_key(p.n_groups, key);
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_clear(const Plan &p, hipStream_t stream)
{
    int64_t work = p.n_cells + 1 > p.n_boxes ? p.n_cells + 1 : p.n_boxes;
    unsigned g = grid_for(work);
    if (g > 65536u) g = 65536u;
    hipLaunchKernelGGL(k_clear, dim3(g), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_build(const Plan &p, hipStream_t stream)
{
    if (p.n > 0) hipLaunchKernelGGL(k_count, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)p.scan_tiles), dim3(kBlock), 0, stream, p);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kPartBlock), 0, stream, p);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)p.scan_tiles), dim3(kBlock), 0, stream, p);
    if (p.n > 0) hipLaunchKernelGGL(k_scatter, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_link(const Plan &p, hipStream_t stream)
{
    if (p.n == 0) return hipSuccess;
    if (p.stats) hipLaunchKernelGGL(k_link<true>, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    else hipLaunchKernelGGL(k_link<false>, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_finalize(const Plan &p, hipStream_t stream)
{
    if (p.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_flatten, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    hipLaunchKernelGGL(k_output, dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

int64_t scan_tiles_for(int64_t n_cells) { return (n_cells + 1 + kScanTile - 1) / kScanTile; }

}  // namespace fof
