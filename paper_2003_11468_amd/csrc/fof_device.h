// Device helpers shared by the gfx950 kernels (build, link, finalize).
#pragma once

#include <climits>

#include "fof_internal.h"

namespace fof {
namespace dev {

constexpr int kBlock = 256;

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

// find_box for one index per lane: the box of the first active lane is found
// once (uniform, scalar loads); only lanes outside it search on their own.
// Consecutive particles, in input or cell order, nearly always share a box.
__device__ __forceinline__ int find_box_wave(const int64_t *p0, int n_boxes, int64_t i)
{
    const unsigned lo32 = __builtin_amdgcn_readfirstlane((unsigned)(uint64_t)i);
    const unsigned hi32 = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)i >> 32));
    const int64_t i0 = (int64_t)(((uint64_t)hi32 << 32) | lo32);
    const int b0 = find_box(p0, n_boxes, i0);
    if (i >= p0[b0] && i < p0[b0 + 1]) return b0;
    return find_box(p0, n_boxes, i);
}

// The box a wave looked up last, with its slot range (uniform across the
// wave): lookups that stay inside it skip the binary search.
struct BoxHint {
    int b = 0;
    int64_t lo = 0, hi = 0;
};

// find_box_wave with a hint: the first active lane's box is searched for only
// when it lies outside the hinted box, which it then replaces.
__device__ __forceinline__ int find_box_hint(const int64_t *p0, int n_boxes, int64_t i, BoxHint &h)
{
    const unsigned lo32 = __builtin_amdgcn_readfirstlane((unsigned)(uint64_t)i);
    const unsigned hi32 = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)i >> 32));
    const int64_t i0 = (int64_t)(((uint64_t)hi32 << 32) | lo32);
    if (!(i0 >= h.lo && i0 < h.hi)) {
        h.b = find_box(p0, n_boxes, i0);
        h.lo = p0[h.b];
        h.hi = p0[h.b + 1];
    }
    if (i >= h.lo && i < h.hi) return h.b;
    return find_box(p0, n_boxes, i);
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
// The forest's reads and path-halving writes go through the XCD's own L2
// (relaxed atomics of work-group scope: they skip the compute unit's L1 but
// not the L2); only the hooking compare-and-swap is device-wide. A read may
// then return an older value, which is still safe:
//  - parent pointers only move to nodes of smaller hooking key (a hook puts a
//    root under a root of smaller key; halving puts a node under an
//    ancestor), so every chain of values read, current or older, has
//    strictly decreasing keys: a find ends, and never runs in a cycle;
//  - sets only merge, so every node reached from x is in x's set: a find
//    returns a node of x's set, and two finds that meet prove one set;
//  - a node seen as a non-root stays one, so halving never writes a root, and
//    the compare-and-swap (device scope, expecting the root itself) alone
//    decides whether a root is still a root. A stale root makes it fail and
//    return the current parent, whose key is smaller: each failure lowers the
//    largest key the next attempt can target, so merging ends too.
// Reading through the L2 keeps the neighbouring nodes of a find (nearby in
// cell order) in cache, instead of a trip past the L2 per step.

__device__ __forceinline__ int ld_rel(const int *a)
{
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void st_rel(int *a, int v)
{
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving: each visited node is re-pointed to its
// grandparent. The store may race with other finds; every value written is an
// ancestor of the node, so the forest stays valid.
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

// Hooking priority of node x (paper, Section 3.2): the index itself, or, for
// randomised linking, a fixed pseudo-random bijection of it (the 32-bit
// finaliser of MurmurHash3: xor-shifts and odd multipliers, each invertible
// modulo 2^32). A strict total order either way, so two roots never tie.
__device__ __forceinline__ unsigned link_key(int x, bool random)
{
    unsigned h = (unsigned)x;
    if (random) {
        h ^= h >> 16;
        h *= 0x85ebca6bu;
        h ^= h >> 13;
        h *= 0xc2b2ae35u;
        h ^= h >> 16;
    }
    return h;
}

// Root of x, compressing the path only when it is at least 2 long (paper,
// Section 3.4.3): a first walk to the root, then, for a long path, a second
// walk that points its nodes at the root. A node is re-pointed only while it
// is not a root and only to a node of smaller key (the root found lies in its
// set), so the forest stays valid whatever other finds and hooks do.
__device__ __forceinline__ int find_depth2(int *parent, int x, bool random)
{
    int r = x, depth = 0;
    for (int q = ld_rel(parent + r); q != r; q = ld_rel(parent + r)) {
        r = q;
        ++depth;
    }
    if (depth >= 2) {
        const unsigned kr = link_key(r, random);
        for (int y = x;;) {
            const int ny = ld_rel(parent + y);
            if (ny == y || ny == r) break;
            if (kr < link_key(y, random)) st_rel(parent + y, r);
            y = ny;
        }
    }
    return r;
}

// The find of the run's compression mode (0: halving, 1: depth >= 2).
__device__ __forceinline__ int find_root(int *parent, int x, int mode, bool random)
{
    return mode == 1 ? find_depth2(parent, x, random) : find_halve(parent, x);
}

// Roots of the kN nodes x[] by path halving, advanced in lockstep: every
// round issues the loads of all nodes still searching together, so their
// latencies overlap instead of adding up. Every x[v] is a valid node, so the
// loads need no guard; nodes already at their root just repeat a load.
template <int kN>
__device__ __forceinline__ void find_many(int *parent, int (&x)[kN], bool (&done)[kN])
{
    while (true) {
        int px[kN], gx[kN];
#pragma unroll
        for (int v = 0; v < kN; ++v) px[v] = ld_rel(parent + x[v]);
#pragma unroll
        for (int v = 0; v < kN; ++v) done[v] = done[v] | (px[v] == x[v]);
#pragma unroll
        for (int v = 0; v < kN; ++v) gx[v] = ld_rel(parent + px[v]);
        // a node still searching moves to its grandparent (its parent when
        // that is the root, which is then equal) and, below the root, halves
        // the path; only the store is conditional, the rest has no branch
        bool any = false;
#pragma unroll
        for (int v = 0; v < kN; ++v) {
            const bool halve = !done[v] & (gx[v] != px[v]);
            if (halve) st_rel(parent + x[v], gx[v]);
            x[v] = done[v] ? x[v] : gx[v];
            done[v] = done[v] | (gx[v] == px[v]);
            any = any | halve;
        }
        if (!any) return;
    }
}

// Merge the groups of a and b: hook the root of lower priority under the other
// with a compare-and-swap that expects it to still be a root. On failure the
// CAS returns the node's new parent, and the search continues from there.
__device__ __forceinline__ unsigned unite(int *parent, int a, int b, bool random, int mode = 0)
{
    unsigned retries = 0;
    while (true) {
        a = find_root(parent, a, mode, random);
        b = find_root(parent, b, mode, random);
        if (a == b) return retries;
        const bool a_first = link_key(a, random) < link_key(b, random);
        int lo = a_first ? a : b;
        int hi = a_first ? b : a;
        int expected = hi;
        if (__hip_atomic_compare_exchange_strong(parent + hi, &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return retries;
        ++retries;
        a = expected;
        b = lo;
    }
}

// ------------------------------------------------------------ cell index --
// Sorted slots [x, y) of cell c: its occupancy word gives the rank of the cell
// among the occupied cells, and cstart the slot of that rank (an empty cell
// gives an empty range).
__device__ __forceinline__ int2 cell_span(const Plan &p, int64_t c)
{
    const uint2 w = p.occ[c >> 5];
    const unsigned bit = (unsigned)c & 31u;
    const int r = (int)w.y + __popc(w.x & ((1u << bit) - 1u));
    const int s = p.cstart[r];
    return make_int2(s, ((w.x >> bit) & 1u) ? p.cstart[r + 1] : s);
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

// Adds `v` into arr[key] with one atomic per distinct key among the active
// lanes of the wave (key < 0: nothing to add). Every lane must call it.
__device__ __forceinline__ void wave_add_by_key(int *arr, int key, int v)
{
    unsigned long long todo = __ballot(key >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, leader, 64);
        const bool mine = key == k;
        int sum = mine ? v : 0;
        for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
        if (lane_id() == leader) atomicAdd(arr + k, sum);
        todo &= ~__ballot(mine);
    }
}

__device__ __forceinline__ void wave_add_by_key(unsigned long long *arr, int key, unsigned long long v)
{
    unsigned long long todo = __ballot(key >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, leader, 64);
        const bool mine = key == k;
        unsigned long long sum = mine ? v : 0ull;
        for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
        if (lane_id() == leader) atomicAdd(arr + k, sum);
        todo &= ~__ballot(mine);
    }
}

// Runs of equal keys in consecutive lanes: on return the first lane of each
// run holds the minimum of the run's `m` and the sum of its `c`, and the
// function returns true there (for key >= 0 only). Six shuffle steps whatever
// the number of distinct keys; every lane must call it.
__device__ __forceinline__ bool wave_runs_min_add(int key, int &m, int &c)
{
    const int lane = lane_id();
    const int prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || prev != key;
    const unsigned long long heads = __ballot(head);
    const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
    const int end = above ? __ffsll((long long)above) - 2 : 63;   // last lane of this run
    for (int d = 1; d < 64; d <<= 1) {
        const int om = __shfl_down(m, d, 64);
        const int oc = __shfl_down(c, d, 64);
        if (lane + d <= end) {
            m = min(m, om);
            c += oc;
        }
    }
    return head && key >= 0;
}

// Atomic min of `v` into arr[key].y, one atomic per distinct key in the wave.
__device__ __forceinline__ void wave_min_by_key(int2 *arr, int key, int v)
{
    unsigned long long todo = __ballot(key >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, leader, 64);
        const bool mine = key == k;
        int m = mine ? v : INT_MAX;
        for (int d = 32; d >= 1; d >>= 1) m = min(m, __shfl_xor(m, d, 64));
        if (lane_id() == leader) atomicMin(&arr[k].y, m);
        todo &= ~__ballot(mine);
    }
}

__device__ __forceinline__ int64_t particle_cell(const BoxDev &bd, float x, float y, float z)
{
    const int nc = bd.nc;
    int cx = cell_coord(x, bd.inv_h, nc);
    int cy = cell_coord(y, bd.inv_h, nc);
    int cz = cell_coord(z, bd.inv_h, nc);
    return bd.cell_base + ((int64_t)cz * nc + cy) * nc + cx;
}

// Work-groups are dispatched round-robin over the 8 XCDs, each with its own
// L2. For kernels whose accesses are local in the tile index, tile t goes to
// XCD t / per, so each XCD works through one contiguous range of tiles and
// keeps that range's window in its own L2. Launch with 8 * per groups
// (per = ceil(tiles / 8)); groups mapped past the last tile return.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_tile(int64_t group, int64_t groups)
{
    const int64_t per = groups / kXcds;
    return (group % kXcds) * per + group / kXcds;
}

inline unsigned xcd_grid(int64_t tiles) { return (unsigned)(((tiles + kXcds - 1) / kXcds) * kXcds); }

// Persistent kernels: the waves of XCD x (groups g with g % 8 == x) share the
// contiguous work range [x * span, (x + 1) * span), span = ceil(total / 8).
// Call with a grid that is a multiple of 8.
struct XcdRange {
    int64_t first, end, stride;
};

__device__ __forceinline__ XcdRange xcd_range(int64_t total, int waves_per_group, int wave_in_group)
{
    const int64_t xcd = blockIdx.x % kXcds, g = blockIdx.x / kXcds, groups = gridDim.x / kXcds;
    const int64_t span = (total + kXcds - 1) / kXcds;
    const int64_t lo = xcd * span;
    const int64_t hi = lo + span < total ? lo + span : total;
    return {lo + g * waves_per_group + wave_in_group, hi, groups * waves_per_group};
}

__device__ __forceinline__ const BoxDev &box_of(const Plan &p, int b)
{
    return p.n_boxes == 1 ? p.box0 : p.boxes[b];
}

}  // namespace dev
}  // namespace fof
