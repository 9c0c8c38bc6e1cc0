// Link search + lock-free union-find for gfx950 (wave64).
//
// Cells are split by occupancy. A cell holding at least `dense_min`
// particles is "dense" and is processed by k_link_dense: one wavefront takes
// up to 64 of its particles (one per lane), stages the candidates of each
// neighbour cell in LDS, 64 at a time, and tests every staged candidate
// against all 64 lanes at once (the candidate address is uniform, so the LDS
// read is a broadcast). All other ("sparse") cells are processed per lane by
// k_link_sparse: each lane walks its own neighbour cells.
//
// Every unordered pair of adjacent cells is searched exactly once:
//   both sparse  -> k_link_sparse, from the cell whose half shell holds the other;
//   one dense    -> k_link_dense of the dense cell (it searches all 26 neighbours,
//                   its lower half only where the neighbour is sparse);
//   both dense   -> k_link_dense, from the cell whose half shell holds the other.
// The half shell of (cx, cy, cz) is the 13 offsets with dz > 0, or dz == 0 and
// dy > 0, or dz == dy == 0 and dx > 0. With at least 3 cells per axis the 27
// periodic neighbours are distinct cells.
//
// Periodic images: the neighbour offset fixes the image, so no distance is
// wrapped per pair. In FP32 the image shift is applied where it is exact: the
// home coordinate minus L when the home cell is the top one (Sterbenz), the
// neighbour coordinate minus L when the neighbour is the top one. Each axis
// difference is then one correctly rounded subtraction of two exact values.
// In double, the difference is rounded first and the shift of +-L added after
// it, which is the very operation sequence of the link predicate.
//
// Union-find: each lane keeps the root it last saw for its particle, and each
// staged candidate carries the root found when it was staged. A linked pair
// whose two cached roots agree is already in one group and is skipped: both
// roots were observed as members of the respective groups, and groups only
// grow. Otherwise the lane hooks the root of lower priority under the other
// (CAS): by index, the larger under the smaller, or by a fixed pseudo-random
// priority (randomised linking).
#include "fof_device.h"

namespace fof {
namespace {

using namespace dev;

constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ float qnan() { return __builtin_nanf(""); }

// Merge the groups that contain roots-or-members a and b; returns a node of the
// merged group (the root that stayed a root at the time of the merge).
__device__ __forceinline__ int unite_root(int *parent, int a, int b, bool random, int mode, unsigned &retries)
{
    while (true) {
        a = find_root(parent, a, mode, random);
        b = find_root(parent, b, mode, random);
        if (a == b) return a;
        const bool a_first = link_key(a, random) < link_key(b, random);
        const int lo = a_first ? a : b;
        const int hi = a_first ? b : a;
        int expected = hi;
        if (__hip_atomic_compare_exchange_strong(parent + hi, &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return lo;
        ++retries;
        a = expected;
        b = lo;
    }
}

constexpr unsigned kGlobalMergeBlocks = 2048;

// ------------------------------------------------------ domain decomposition --
// Domain mode (paper, Section 3.3, on one GPU): a box is cut into `domains`
// slabs along x. Union-find merges only links inside a slab; a link across
// slabs goes to the boundary list (the list the paper's ranks exchange), and
// the global merge after the search joins the groups it names.

// Slab of a particle at x in a box of side L.
__device__ __forceinline__ int slab_of(float x, int domains, double L)
{
    const int d = (int)((double)x * (double)domains / L);
    return d < domains ? d : domains - 1;
}

// Slab of sorted particle s.
__device__ __forceinline__ int domain_of(const Plan &p, int s)
{
    const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, s);
    return slab_of(p.sorted[s].x, p.domains, box_of(p, b).L);
}

// Appends the pair to the boundary list; a pair that finds the list full is
// merged at once (the groups come out the same).
__device__ __forceinline__ void defer_boundary(const Plan &p, int a, int b, unsigned &retries)
{
    const unsigned at = atomicAdd(&p.counters->n_boundary, 1u);
    if ((int64_t)at < p.max_edges) p.bnd[at] = make_int2(a, b);
    else retries += unite(p.parent, a, b, p.link_random, p.find_mode);
}

// Merge of a linked pair found by the search: at once, or in domain mode
// through the boundary list when the pair crosses slabs.
__device__ __forceinline__ void merge_pair(const Plan &p, int a, int b, unsigned &retries)
{
    if (p.domains > 1 && domain_of(p, a) != domain_of(p, b)) defer_boundary(p, a, b, retries);
    else retries += unite(p.parent, a, b, p.link_random, p.find_mode);
}

__device__ __forceinline__ int lds_ld(int *a) { return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void lds_st(int *a, int v)
{
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of sub-cell x in the LDS forest f (path halving; parents only point to
// smaller indices).
__device__ __forceinline__ int lds_find(int *f, int x)
{
    while (true) {
        const int px = lds_ld(f + x);
        if (px == x) return x;
        const int gx = lds_ld(f + px);
        if (gx == px) return px;
        lds_st(f + x, gx);
        x = gx;
    }
}

// Warshall's closure of 64 boolean rows, one per lane (bit v of lane u's row:
// u is joined to v; every row holds its own bit): for each k in `todo` (the
// lanes whose rows hold other bits), every row holding bit k takes in row k,
// read with readlane. Afterwards a row is its lane's component, so its lowest
// bit is the component's smallest member. No branch and no memory access.
__device__ __forceinline__ unsigned long long close_rows(unsigned long long row, unsigned long long todo)
{
    // the two words of each row apart, so that the test of bit k reads one
    // word (k below 32: the low one) and its sign-extended bit masks row k in
    unsigned lo = (unsigned)row, hi = (unsigned)(row >> 32);
    for (unsigned t = (unsigned)todo; t; t &= t - 1u) {
        const int k = __ffs(t) - 1;
        const unsigned klo = (unsigned)__builtin_amdgcn_readlane((int)lo, k);
        const unsigned khi = (unsigned)__builtin_amdgcn_readlane((int)hi, k);
        const unsigned m = (unsigned)__builtin_amdgcn_sbfe((int)lo, (unsigned)k, 1u);
        lo |= klo & m;
        hi |= khi & m;
    }
    for (unsigned t = (unsigned)(todo >> 32); t; t &= t - 1u) {
        const int k = __ffs(t) - 1;
        const unsigned klo = (unsigned)__builtin_amdgcn_readlane((int)lo, k + 32);
        const unsigned khi = (unsigned)__builtin_amdgcn_readlane((int)hi, k + 32);
        const unsigned m = (unsigned)__builtin_amdgcn_sbfe((int)hi, (unsigned)k, 1u);
        lo |= klo & m;
        hi |= khi & m;
    }
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ void lds_unite(int *f, int a, int b)
{
    while (true) {
        a = lds_find(f, a);
        b = lds_find(f, b);
        if (a == b) return;
        const int lo = min(a, b), hi = max(a, b);
        int expected = hi;
        if (__hip_atomic_compare_exchange_strong(f + hi, &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
        a = expected;
        b = lo;
    }
}

// --------------------------------------------------------- sparse (lane) --

// Periodic shift code of one axis for a candidate range: 0 none; 1 the
// neighbour cell is the top one reached across the low face (candidate - L is
// exact); 2 the home cell is the top one and the neighbour lies across the
// high face (home - L is exact). Codes of x, y, z sit in bits 0-1, 2-3, 4-5.
__device__ __forceinline__ float axis_diff(float h, float q, int code, float L32)
{
    const float hh = code == 2 ? h - L32 : h;
    const float qq = code == 1 ? q - L32 : q;
    return hh - qq;
}

__device__ __forceinline__ double axis_shift(int code, double L) { return code == 1 ? L : (code == 2 ? -L : 0.0); }

constexpr int kMaxRanges = 10;

// One candidate range of a home particle: slots [j0, j1) (empty when
// j1 <= j0) and their periodic shift code.
struct Span {
    int j0 = 0, j1 = 0, code = 0;
};

// The three cells (x = cx-1, cx, cx+1) of one neighbour row, given their
// boundaries (st[e], en[e]) and whether the row wraps at either end. Runs of
// sparse, memory-contiguous cells are merged into one range: at most two per
// row (the cells of a row follow each other in memory except across the
// wrap, which is at one end, and around a dense middle cell).
__device__ __forceinline__ void row_spans(const int st[3], const int en[3], const int xcode[3], int yz_code,
                                          int dense_min, Span &A, Span &B)
{
    int a = -1, b = -1, code = 0;
    bool first = true;
    auto emit = [&](int j0, int j1, int c) {
        if (first) A = Span{j0, j1, c};
        else B = Span{j0, j1, c};
        first = false;
    };
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const bool sparse = en[e] - st[e] < dense_min;
        const int c = xcode[e] | yz_code;
        if (sparse && en[e] > st[e]) {
            if (a >= 0 && st[e] == b && c == code) {
                b = en[e];
            } else {
                if (a >= 0) emit(a, b, code);
                a = st[e];
                b = en[e];
                code = c;
            }
        }
    }
    if (a >= 0) emit(a, b, code);
}

// Linked pairs of the sparse search are not merged where they are found: a
// union is a chain of dependent memory accesses, and inside the search it
// would stall the whole wavefront round after round. Each wave collects its
// pairs in LDS and appends them to a global edge list 64 at a time; the
// union kernel then merges all of them with one thread per pair.
constexpr int kEdgeBuf = 128;

struct EdgeSink {
    int2 *buf;      // this wave's LDS buffer [kEdgeBuf]
    int count;      // wave-uniform fill level

    // Appends (s, j) for every lane with `has`; flushes once 64 are waiting.
    __device__ __forceinline__ void push(const Plan &p, bool has, int s, int j, unsigned &retries)
    {
        const unsigned long long m = __ballot(has);
        if (!m) return;
        if (has) {
            const int at = count + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            buf[at] = make_int2(s, j);
        }
        count += __popcll(m);
        __builtin_amdgcn_wave_barrier();
        if (count >= 64) flush(p, retries);
    }

    // Appends the buffer to this work-group's slice of the edge list (one
    // atomic on the slice counter); pairs that find the slice full are merged here.
    __device__ __forceinline__ void flush(const Plan &p, unsigned &retries)
    {
        if (count == 0) return;
        const int lane = lane_id();
        const int slice = blockIdx.x % kEdgeSlices;
        const int64_t cap = p.max_edges / kEdgeSlices;
        unsigned base = 0;
        if (lane == 0) base = atomicAdd(&p.edge_fill[slice], (unsigned)count);
        base = (unsigned)__shfl((int)base, 0, 64);
        for (int k = lane; k < count; k += 64) {
            const int2 e = buf[k];
            const int64_t at = (int64_t)base + k;
            if (at < cap) p.edges[slice * cap + at] = e;
            else merge_pair(p, e.x, e.y, retries);
        }
        __builtin_amdgcn_wave_barrier();
        count = 0;
    }
};

// Per-wave LDS for the sparse search: the candidate ranges ("units") of the
// wave's 64 home particles, flattened into one list of pairs by a prefix sum,
// so that every lane tests a pair in every step whatever the range lengths.
constexpr int kMaxUnits = 64 * kMaxRanges;

struct SparseLds {
    int start[kMaxUnits + 1];   // first pair of each unit (exclusive prefix)
    int j0[kMaxUnits];          // first candidate of each unit
    unsigned short tag[kMaxUnits];   // shift code (bits 0-5) | home lane << 8
    float4 home[64];                 // the home particles
    int2 ebuf[kEdgeBuf];             // edge sink buffer
    unsigned long long adj[64];      // links inside the tile: bit v of adj[u] for home u, slot s0 + v
};

// Box parameters of the pair test, in registers.
struct BoxPair {
    double L, half, l2;
    float L32, lo32, hi32;
    __device__ __forceinline__ static BoxPair of(const BoxDev &bd)
    {
        return BoxPair{bd.L, bd.half, bd.l2, bd.L32, bd.lo32, bd.hi32};
    }
};

// The pair loop of the per-particle search over the wave's flattened units.
// Merge-path split: lane l takes the pairs [T l / 64, T (l + 1) / 64) of the
// wave's T pairs, finds the unit of its first pair by one binary search, then
// walks forward; every lane runs the same number of steps. kOneBox: every
// home particle of the tile lies in one box, whose parameters are `bp`.
template <bool kFP64, bool kStats, bool kOneBox>
__device__ __forceinline__ void sparse_pairs(const Plan &p, SparseLds &L, EdgeSink &sink, int s0, int n_units,
                                             int n_pairs, int b, BoxPair bp, bool in_tile, unsigned long long &tests,
                                             unsigned long long &links, unsigned long long &band, unsigned &retries)
{
    const int lane = lane_id();
    const bool strict = p.strict != 0;
    const int q0 = (int)(((int64_t)n_pairs * lane) >> 6);
    const int q1 = (int)(((int64_t)n_pairs * (lane + 1)) >> 6);
    int u = 0;
#pragma unroll
    for (int step = 512; step > 0; step >>= 1) {
        const int nxt = u + step;
        if (nxt < n_units && L.start[nxt] <= q0) u = nxt;
    }
    int next_start = L.start[u + 1];
    int jq = L.j0[u] + (q0 - L.start[u]);   // candidate of pair q
    int tag = L.tag[u];
    float4 h = L.home[tag >> 8];
    // four steps at a time: their candidate loads are in flight together
    constexpr int kAhead = 4;
    const int steps = (n_pairs + 63) >> 6;
    int q = q0;
    for (int k = 0; k < steps; k += kAhead) {
        int jj[kAhead], tg[kAhead];
        float4 hh[kAhead], cc[kAhead];
        bool lv[kAhead];
#pragma unroll
        for (int a = 0; a < kAhead; ++a) {
            lv[a] = q < q1 && k + a < steps;
            if (lv[a] && q == next_start) {   // the next unit starts here
                ++u;
                next_start = L.start[u + 1];
                jq = L.j0[u];
                tag = L.tag[u];
                h = L.home[tag >> 8];
            }
            jj[a] = jq;
            tg[a] = tag;
            hh[a] = h;
            if (lv[a]) {
                ++jq;
                ++q;
            }
        }
#pragma unroll
        for (int a = 0; a < kAhead; ++a)
            if (lv[a]) cc[a] = p.sorted[jj[a]];
        // no lane's pairs of these steps need a periodic shift (the common
        // case away from the box faces): plain differences, the same values
        bool plain = false;
        if constexpr (!kFP64) {
            int codes = 0;
#pragma unroll
            for (int a = 0; a < kAhead; ++a) codes |= tg[a];
            plain = __ballot((codes & 63) != 0) == 0;
        }
#pragma unroll
        for (int a = 0; a < kAhead; ++a) {
            const int hl = tg[a] >> 8, code = tg[a] & 63;
            BoxPair bx = bp;
            if constexpr (!kOneBox) {
                const int bq = __shfl(b, hl, 64);   // all lanes take part in the shuffle
                if (lv[a]) bx = BoxPair::of(p.boxes[bq]);
            }
            bool link = false;
            if (lv[a]) {
                const float4 c = cc[a];
                const float4 hp = hh[a];
                if constexpr (kFP64) {
                    const double tx = ((double)hp.x - (double)c.x) + axis_shift(code & 3, bx.L);
                    const double ty = ((double)hp.y - (double)c.y) + axis_shift((code >> 2) & 3, bx.L);
                    const double tz = ((double)hp.z - (double)c.z) + axis_shift((code >> 4) & 3, bx.L);
                    const double sxy = tx * tx + ty * ty;
                    const double r2 = sxy + tz * tz;
                    link = strict ? (r2 < bx.l2) : (r2 <= bx.l2);
                } else {
                    float dx, dy, dz;
                    if (plain) {
                        dx = hp.x - c.x;
                        dy = hp.y - c.y;
                        dz = hp.z - c.z;
                    } else {
                        dx = axis_diff(hp.x, c.x, code & 3, bx.L32);
                        dy = axis_diff(hp.y, c.y, (code >> 2) & 3, bx.L32);
                        dz = axis_diff(hp.z, c.z, (code >> 4) & 3, bx.L32);
                    }
                    const float rr = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    link = rr < bx.lo32;
                    // the guard band (rare), decided in double; one branch, the
                    // compares flat (a NaN lands in the band and fails there)
                    if (!(rr < bx.lo32) & !(rr > bx.hi32)) {
                        if (kStats) ++band;
                        link = link_fp64(hp.x, hp.y, hp.z, c.x, c.y, c.z, bx.L, bx.half, bx.l2, strict);
                    }
                }
                if (kStats) ++tests;
                if (kStats && link) ++links;
            }
            // a link inside the tile goes to the tile's bit matrix, the others to the edge list
            const unsigned v = (unsigned)(jj[a] - s0);
            const bool local = in_tile && v < 64u;
            if (link && local) {   // both directions: the rows are then the tile's undirected links
                atomicOr(&L.adj[hl], 1ull << v);
                atomicOr(&L.adj[v & 63u], 1ull << hl);
            }
            sink.push(p, link && !local, s0 + hl, jj[a], retries);
        }
    }
}

template <bool kFP64, bool kStats>
__global__ void __launch_bounds__(kBlock) k_link_sparse(Plan p)
{
    __shared__ SparseLds lds[kWaves];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    SparseLds &L = lds[wid];
    EdgeSink sink{L.ebuf, 0};
    unsigned long long tests = 0, links = 0, band = 0;
    unsigned retries = 0;
    // links inside a tile are joined by the search itself (index order only:
    // the hook goes under the smallest slot; not in domain mode, whose links
    // across slabs must go through the boundary list)
    const bool tile_union = p.tile_join != 0 && p.link_random == 0 && p.domains <= 1;
    BoxHint hint;   // consecutive tiles of a wave nearly always lie in one box
    const bool any_dense = p.counters->n_items != 0;
    int hook_x = -1, hook_r = 0, hook_old = 0;   // this lane's last tile hook
    auto check_hook = [&]() {
        if (hook_x >= 0 && hook_old != hook_x) retries += 1 + unite(p.parent, hook_x, hook_r, false, p.find_mode);
        hook_x = -1;
    };
    const int64_t n_tiles = (p.n + 63) / 64;
    // each XCD sweeps one contiguous range of tiles, so the neighbour rows of
    // consecutive tiles are reused from its own L2
    const XcdRange xr = xcd_range(n_tiles, kWaves, wid);
    for (int64_t tile = xr.first; tile < xr.end; tile += xr.stride) {
        // a tile whose slots all lie in dense cells has nothing to search here
        // (slots past the end count as dense)
        if (any_dense) {
            const int64_t left = p.n - tile * 64;
            const unsigned long long dm = p.tile_dense[tile] | (left < 64 ? ~0ull << left : 0ull);
            if (dm == ~0ull) continue;
        }
        const int64_t s64 = tile * 64 + lane;
        Span R[kMaxRanges];   // own cell, next cell, then two per neighbour row
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
        int b = 0;
        if (s64 < p.n) {
            const int s = (int)s64;
            b = p.n_boxes == 1 ? 0 : find_box_hint(p.box_p0, p.n_boxes, s64, hint);
            const BoxDev &bd = box_of(p, b);
            pi = p.sorted[s];
            const int nc = bd.nc;
            const int cx = cell_coord(pi.x, bd.inv_h, nc);
            const int cy = cell_coord(pi.y, bd.inv_h, nc);
            const int cz = cell_coord(pi.z, bd.inv_h, nc);
            const int64_t c = bd.cell_base + ((int64_t)cz * nc + cy) * nc + cx;
            const int *cst = p.cstart;
            const int dense_min = p.dense_min;
            const int seg_shift = p.seg_shift;
            const int64_t rb0 = c - cx;
            // Boundaries of the own row and the four neighbour rows (dy, dz) =
            // (1, 0), (-1, 1), (0, 1), (1, 1): with the own cell these hold the
            // 13 half-shell cells. Occupancy words (bits and rank base per 32
            // cells, a small array that stays in cache) give the rank of each
            // cell among the occupied ones, and cstart the boundaries.
            const uint2 *occ = p.occ;
            typedef unsigned uint4a8 __attribute__((ext_vector_type(4), aligned(8)));
            typedef int int4a4 __attribute__((ext_vector_type(4), aligned(4)));
            auto rank_in = [](unsigned bits, unsigned base, int64_t cell_index) {
                return (int)base + __popc(bits & ((1u << ((unsigned)cell_index & 31u)) - 1u));
            };
            auto span = [&](int64_t cell_index, int &s0, int &s1) {   // left at 0, 0 for an empty cell
                const uint2 w = occ[cell_index >> 5];
                if ((w.x >> ((unsigned)cell_index & 31u)) & 1u) {
                    const int r = rank_in(w.x, w.y, cell_index);
                    s0 = cst[r];
                    s1 = cst[r + 1];
                }
            };
            const int nxp = cx + 1 < nc ? cx + 1 : 0;
            const bool inner = cx >= 1 && cx + 1 < nc;
            const int rdy[4] = {1, -1, 0, 1}, rdz[4] = {0, 1, 1, 1};
            int64_t rb[4], c0[4];
            int yz[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int ny = cy + rdy[r], nz = cz + rdz[r], code = 0;
                if (ny >= nc) { ny -= nc; code |= 2 << 2; }
                else if (ny < 0) { ny += nc; code |= 1 << 2; }
                if (nz >= nc) { nz -= nc; code |= 2 << 4; }
                yz[r] = code;
                rb[r] = bd.cell_base + ((int64_t)nz * nc + ny) * nc;
                c0[r] = rb[r] + (inner ? cx - 1 : 0);
            }
            // Two rounds of loads, each issued whole before any of its results
            // is used, with no branch among them: first the occupancy words of
            // the own cell and of each row (two words each, so cells across a
            // word boundary are covered), then, from the ranks, one 16-byte
            // read of cell starts for the own cell and for each row. Every
            // address is in range whatever the bits: a rank is at most n and
            // cstart has n + 4 entries; a word index is at most the last one
            // plus one, inside the two words of padding.
            const uint4a8 wo = *reinterpret_cast<const uint4a8 *>(occ + (c >> 5));
            uint4a8 wr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) wr[r] = *reinterpret_cast<const uint4a8 *>(occ + (c0[r] >> 5));
            const int4a4 qo = *reinterpret_cast<const int4a4 *>(cst + rank_in(wo.x, wo.y, c));   // the own cell holds s
            int4a4 qr[4];
            unsigned mr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                mr[r] = (unsigned)((((uint64_t)wr[r].x | ((uint64_t)wr[r].z << 32)) >> ((unsigned)c0[r] & 31u)) & 7u);
                qr[r] = *reinterpret_cast<const int4a4 *>(cst + rank_in(wr[r].x, wr[r].y, c0[r]));
            }
            const int own_start = qo.x, own_end = qo.y;
            int nxt_start = 0, nxt_end = 0;
            if (nxp && ((c ^ (c + 1)) >> seg_shift) == 0) {
                // the next cell in the same segment: its entries follow the own cell's
                const unsigned b1 = (unsigned)(c + 1) & 31u;
                const unsigned nbits = b1 ? wo.x : wo.z;
                if ((nbits >> b1) & 1u) {
                    nxt_start = qo.y;
                    nxt_end = qo.z;
                }
            } else {
                span(rb0 + nxp, nxt_start, nxt_end);
            }
            int st[4][3], en[4][3];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int e = 0; e < 3; ++e) st[r][e] = en[r][e] = 0;
                const unsigned m = mr[r];
                if (inner && ((c0[r] ^ (c0[r] + 2)) >> seg_shift) == 0) {
                    // the three cells in one segment: their occupied cells have
                    // consecutive entries, so the 16-byte read holds every boundary
                    const int4a4 q = qr[r];
                    auto pick = [&](unsigned k) { return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w)); };
                    const unsigned o1 = m & 1u, o2 = o1 + ((m >> 1) & 1u), o3 = o2 + (m >> 2);
                    const int b1 = pick(o1), b2 = pick(o2);
                    st[r][0] = q.x; en[r][0] = b1;
                    st[r][1] = b1; en[r][1] = b2;
                    st[r][2] = b2; en[r][2] = pick(o3);
                } else if (inner) {
                    if (m) {
#pragma unroll
                        for (int e = 0; e < 3; ++e) span(c0[r] + e, st[r][e], en[r][e]);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        int nx = cx - 1 + e;
                        nx += nx < 0 ? nc : (nx >= nc ? -nc : 0);
                        span(rb[r] + nx, st[r][e], en[r][e]);
                    }
                }
            }
            if (own_end - own_start < dense_min) {
                // own cell above s, then cell cx + 1 (across the high x face when cx is the top cell)
                const int xcode_next = cx + 1 < nc ? 0 : 2;
                if (nxt_end - nxt_start < dense_min && xcode_next == 0 && nxt_start == own_end) {
                    R[0] = Span{s + 1, nxt_end, 0};
                } else {
                    R[0] = Span{s + 1, own_end, 0};
                    if (nxt_end - nxt_start < dense_min) R[1] = Span{nxt_start, nxt_end, xcode_next};
                }
                const int xcode[3] = {cx == 0 ? 1 : 0, 0, cx + 1 == nc ? 2 : 0};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (p.sample) {
                        // the first pass of the giant-component skip: the axis
                        // neighbours (dy, dz) = (1, 0) and (0, 1), centre cells only
#pragma unroll
                        for (int e = 0; e < 3; ++e)
                            if (!((r == 0 || r == 2) && e == 1)) en[r][e] = st[r][e];
                    }
                    row_spans(st[r], en[r], xcode, yz[r], dense_min, R[2 + 2 * r], R[3 + 2 * r]);
                }
            }
        }
        // flatten the units of the wave: unit and pair offsets by prefix sums
        int my_pairs = 0, my_units = 0;
#pragma unroll
        for (int r = 0; r < kMaxRanges; ++r)
            if (R[r].j1 > R[r].j0) {
                my_pairs += R[r].j1 - R[r].j0;
                ++my_units;
            }
        const int unit_incl = wave_incl_scan(my_units);
        const int pair_incl = wave_incl_scan(my_pairs);
        const int n_units = __shfl(unit_incl, 63, 64);
        const int n_pairs = __shfl(pair_incl, 63, 64);
        if (n_pairs == 0) continue;
        {
            int u = unit_incl - my_units, pr = pair_incl - my_pairs;
#pragma unroll
            for (int r = 0; r < kMaxRanges; ++r)
                if (R[r].j1 > R[r].j0) {
                    L.start[u] = pr;
                    L.j0[u] = R[r].j0;
                    L.tag[u] = R[r].code | (lane << 8);
                    pr += R[r].j1 - R[r].j0;
                    ++u;
                }
            if (lane == 63) L.start[n_units] = n_pairs;
            L.home[lane] = pi;
        }
        __builtin_amdgcn_wave_barrier();
        check_hook();
        L.adj[lane] = 0ull;
        __builtin_amdgcn_wave_barrier();
        // a tile inside one box keeps that box's parameters in registers for
        // every pair; otherwise each pair reads the box of its home particle
        const int s0 = (int)(tile * 64);
        const int b0 = __builtin_amdgcn_readfirstlane(b);
        if (__ballot(b != b0) == 0)
            sparse_pairs<kFP64, kStats, true>(p, L, sink, s0, n_units, n_pairs, b, BoxPair::of(box_of(p, b0)),
                                              tile_union, tests, links, band, retries);
        else
            sparse_pairs<kFP64, kStats, false>(p, L, sink, s0, n_units, n_pairs, b, BoxPair{}, tile_union, tests,
                                               links, band, retries);
        __builtin_amdgcn_wave_barrier();
        if (tile_union) {
            // The components of the links inside the tile, by Warshall's
            // closure over the rows of the bit matrix (one per lane): row u
            // starts as u's links and u itself; for each slot k with links,
            // every row that holds k takes in row k. Afterwards row u is u's
            // component, and its lowest bit the component's smallest slot,
            // the node of smallest hooking key, under which u is hooked.
            // Every particle is still its own root while the search runs,
            // unless a full edge-list slice made a search merge its surplus
            // at once: so the hook is a compare-and-swap, and one that finds
            // its slot hooked already becomes an ordinary union.
            const unsigned long long tile_links = L.adj[lane];
            const unsigned long long todo = __ballot(tile_links != 0ull);
            if (todo) {
                const unsigned long long row = close_rows(tile_links | (1ull << lane), todo);
                const int r = __ffsll((long long)row) - 1;
                if (r != lane) {   // read back with the next tile, so the wave does not wait for it
                    hook_x = s0 + lane;
                    hook_r = s0 + r;
                    hook_old = atomicCAS(p.parent + hook_x, hook_x, hook_r);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    check_hook();
    sink.flush(p, retries);
    if (kStats) {
        tests = wave_sum_u64(tests);
        links = wave_sum_u64(links);
        band = wave_sum_u64(band);
        unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane == 0) {
            atomicAdd(&p.counters->sparse_tests, tests);
            atomicAdd(&p.counters->pair_tests, tests);
            atomicAdd(&p.counters->links, links);
            atomicAdd(&p.counters->band_hits, band);
            atomicAdd(&p.counters->cas_retries, r);
        }
    }
}

constexpr int kUnionIlp = 8;   // queued pairs a lane merges at once

// Merges the queued pairs, no ordering needed. Each lane carries kUnionIlp
// pairs at once: the finds of their 2 kUnionIlp end points advance together,
// then each pair whose roots differ hooks the root of lower priority under
// the other; a compare-and-swap that finds the root moved continues as an
// ordinary union from the value it returned. Slice s holds the pairs found on
// XCD s % 8 (the search's work-group b appends to slice b % 256, and
// work-groups go to XCDs round-robin), whose home particles are that XCD's
// contiguous range of cells; its kUnionParts work-groups run on the same XCD,
// so the finds of a slice stay in one L2. Domain mode and the depth-2
// compression take the plain path, one pair at a time.
constexpr int kUnionParts = 16;
static_assert(kEdgeSlices % kXcds == 0, "slices split evenly over the XCDs");

template <bool kStats>
__global__ void __launch_bounds__(kBlock) k_union_edges(Plan p)
{
    const int xcd = blockIdx.x % kXcds, g = blockIdx.x / kXcds;
    const int slice = (g % (kEdgeSlices / kXcds)) * kXcds + xcd;
    const int part = g / (kEdgeSlices / kXcds);
    const int64_t cap = p.max_edges / kEdgeSlices;
    const unsigned fill = p.edge_fill[slice];
    const int64_t ne = (int64_t)fill < cap ? (int64_t)fill : cap;
    const int2 *edges = p.edges + slice * cap;
    const int64_t stride = (int64_t)kUnionParts * kBlock;
    unsigned retries = 0;
    if (p.domains > 1 || p.find_mode != 0) {
        for (int64_t k = (int64_t)part * kBlock + threadIdx.x; k < ne; k += stride) {
            const int2 e = edges[k];
            merge_pair(p, e.x, e.y, retries);
        }
    } else {
        const bool rnd = p.link_random != 0;
        for (int64_t k0 = (int64_t)part * kBlock + threadIdx.x; k0 < ne; k0 += kUnionIlp * stride) {
            int x[2 * kUnionIlp];
            bool done[2 * kUnionIlp];
#pragma unroll
            for (int u = 0; u < kUnionIlp; ++u) {
                const int64_t k = k0 + u * stride;
                const bool in = k < ne;
                const int2 e = in ? edges[k] : make_int2(0, 0);
                x[2 * u] = e.x;
                x[2 * u + 1] = e.y;
                done[2 * u] = done[2 * u + 1] = !in;
            }
            find_many<2 * kUnionIlp>(p.parent, x, done);
#pragma unroll
            for (int u = 0; u < kUnionIlp; ++u) {
                const int a = x[2 * u], b = x[2 * u + 1];
                if (a == b || k0 + u * stride >= ne) continue;
                const bool a_first = link_key(a, rnd) < link_key(b, rnd);
                const int lo = a_first ? a : b;
                const int hi = a_first ? b : a;
                int expected = hi;
                if (!__hip_atomic_compare_exchange_strong(p.parent + hi, &expected, lo, __ATOMIC_RELAXED,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    retries += 1 + unite(p.parent, expected, lo, rnd);
            }
        }
    }
    if (kStats) {
        unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane_id() == 0 && r) atomicAdd(&p.counters->cas_retries, r);
        // queued pairs, for the statistics
        if (part == 0 && threadIdx.x == 0) atomicAdd(&p.counters->n_edges, fill);
    }
}

// ---------------------------------------------------------- dense (wave) --
//
// One work item = up to 64 particles of a dense cell, one per lane ("home"
// particles). Candidates are staged in LDS, 64 at a time, and every staged
// candidate is tested against all home lanes at once (its LDS address is
// uniform, so the read is a broadcast). A stage is filled from a list of
// candidate ranges (the cell itself, or several neighbour cells at once), so
// that small neighbour cells do not each cost a round of loads:
//  - the cell itself (only candidates above the home particle count);
//  - every neighbour cell the item searches (the upper half shell, and the
//    lower half where the neighbour is sparse) whose periodic image needs no
//    shift of the home coordinate, together in one list;
//  - FP32 only: each neighbour reached across a high face of the box, where
//    the home coordinate is shifted by -L (exact there), on its own.
// When every home lane knows the same root, candidates of that root are
// already in their group and are dropped while the stage is filled.

struct StageF {
    float4 v[64];            // x, y, z (candidate-side periodic shift applied), cached root (bits)
    int slot[64];            // sorted slot of the candidate
};

struct StageD {
    double x[64], y[64], z[64];
    double sx[64], sy[64], sz[64];   // periodic shift, added after the rounded difference
    int root[64];
    int slot[64];
};

template <bool kFP64>
struct Stage;
template <>
struct Stage<false> {
    using T = StageF;
};
template <>
struct Stage<true> {
    using T = StageD;
};

// Candidate ranges of one stage fill: range r covers slots
// [j0[r], j0[r] + pre[r + 1] - pre[r]) with periodic shift code code[r]
// (bits 0-1, 2-3, 4-5 for x, y, z: 1 = the neighbour is the top cell across
// the low face, its FP32 coordinate minus L is exact; 2 = the neighbour lies
// across the high face, handled on the home side in FP32). In double the
// shift (+L for 1, -L for 2) is added after the rounded difference.
struct RangeList {
    int pre[28];
    int j0[27];
    int code[27];
};

// Box parameters the inner loops need, held in registers.
struct BoxRegs {
    double L, half, l2;
    float lo32, hi32, L32;
    bool strict;
};

// The slow path of one staged candidate kk for the lanes in `cand`: an FP32
// result below lo32 links; one inside the band is re-decided in double from
// the original coordinates; a link merges the groups unless they are already
// known to be one. kGeneral: domain mode (a link across slabs goes to the
// boundary list) and randomised linking, decided at run time; the plain
// instance has neither, which keeps its registers and code size down.
//
// Known roots: root_i is the root last seen for the home particle; known0
// and known1 are two more nodes of its group (the two roots of its last
// merge). A candidate whose cached root is any of them is in the group
// already (groups only grow), so the pair needs no union whatever its
// distance. Without statistics the caller drops such candidates before the
// distance decides anything.
template <bool kFP64, bool kStats, bool kGeneral>
__device__ __forceinline__ void dense_hit(const Plan &p, const BoxRegs &br, const typename Stage<kFP64>::T &st,
                                          int kk, bool cand, float r, float4 pi, int &root_i, int &known0,
                                          int &known1, unsigned long long &links, unsigned long long &band,
                                          unsigned &retries)
{
    if (!cand) return;
    const int j = st.slot[kk];
    bool link = true;
    if constexpr (!kFP64) {
        if (!(r < br.lo32)) {
            if (kStats) ++band;
            const float4 oj = p.sorted[j];
            link = link_fp64(pi.x, pi.y, pi.z, oj.x, oj.y, oj.z, br.L, br.half, br.l2, br.strict);
        }
    }
    if (link) {
        if (kStats) ++links;
        int rj;
        if constexpr (kFP64) rj = st.root[kk];
        else rj = __float_as_int(st.v[kk].w);
        if (rj != root_i && rj != known0 && rj != known1) {
            if (kGeneral && p.domains > 1 && domain_of(p, j) != slab_of(pi.x, p.domains, br.L)) {
                defer_boundary(p, root_i, rj, retries);
            } else {
                const int old = root_i;
                root_i = unite_root(p.parent, root_i, rj, kGeneral && p.link_random, p.find_mode, retries);
                known0 = rj;
                known1 = old;
            }
        }
    }
}

// FP32 squared distance of the home lane to a staged candidate.
__device__ __forceinline__ float dist2_f32(const float4 cj, float hx, float hy, float hz)
{
    const float dx = hx - cj.x, dy = hy - cj.y, dz = hz - cj.z;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// The double predicate of the home lane and staged candidate kk, with the
// candidate's periodic shift added after the rounded difference.
__device__ __forceinline__ bool link_f64_staged(const StageD &st, int kk, double dxi, double dyi, double dzi,
                                                const BoxRegs &br)
{
    const double tx = (dxi - st.x[kk]) + st.sx[kk];
    const double ty = (dyi - st.y[kk]) + st.sy[kk];
    const double tz = (dzi - st.z[kk]) + st.sz[kk];
    const double sxy = tx * tx + ty * ty;
    const double r2 = sxy + tz * tz;
    return br.strict ? (r2 < br.l2) : (r2 <= br.l2);
}

// Tests the staged candidates [0, cnt) against the wave's home particles.
// An item of at most 32 (or 16) home particles holds copies of them in both
// halves (all four quarters) of the wave: lane l is home particle l % H and
// tests candidate kk + l / H, so one step tests G = 64 / H candidates.
// kSelf: the candidates come from the home cell; only slots above the home
// particle's count. Without statistics a candidate whose cached root is
// known to be in the home particle's group is dropped together with the
// distance test's verdict.
template <bool kFP64, bool kStats, bool kGeneral, bool kSelf>
__device__ __forceinline__ void dense_batch(const Plan &p, const BoxRegs &br, const typename Stage<kFP64>::T &st,
                                            int cnt, int G, int q, int i, bool vi, float4 pi, float hx, float hy,
                                            float hz, double dxi, double dyi, double dzi, int &root_i, int &known0,
                                            int &known1, unsigned long long &links, unsigned long long &band,
                                            unsigned &retries)
{
    // non-short-circuit forms: the compares run flat, with no branch around them
    auto fresh = [&](int rj) { return kStats || ((rj != root_i) & (rj != known0)); };
    int kk = 0;
    if constexpr (!kFP64) {
        const int G4 = 4 * G;
        for (; kk + G4 <= cnt; kk += G4) {
            const int k0 = kk + q, k1 = k0 + G, k2 = k1 + G, k3 = k2 + G;
            const float4 q0 = st.v[k0], q1 = st.v[k1], q2 = st.v[k2], q3 = st.v[k3];
            const float r0 = dist2_f32(q0, hx, hy, hz);
            const float r1 = dist2_f32(q1, hx, hy, hz);
            const float r2 = dist2_f32(q2, hx, hy, hz);
            const float r3 = dist2_f32(q3, hx, hy, hz);
            bool c0 = (r0 <= br.hi32) & fresh(__float_as_int(q0.w));
            bool c1 = (r1 <= br.hi32) & fresh(__float_as_int(q1.w));
            bool c2 = (r2 <= br.hi32) & fresh(__float_as_int(q2.w));
            bool c3 = (r3 <= br.hi32) & fresh(__float_as_int(q3.w));
            if constexpr (kSelf) {
                c0 = c0 & (st.slot[k0] > i);
                c1 = c1 & (st.slot[k1] > i);
                c2 = c2 & (st.slot[k2] > i);
                c3 = c3 & (st.slot[k3] > i);
            }
            if (__ballot(c0 || c1 || c2 || c3)) {
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, k0, c0, r0, pi, root_i, known0, known1, links, band,
                                                   retries);
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, k1, c1, r1, pi, root_i, known0, known1, links, band,
                                                   retries);
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, k2, c2, r2, pi, root_i, known0, known1, links, band,
                                                   retries);
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, k3, c3, r3, pi, root_i, known0, known1, links, band,
                                                   retries);
            }
        }
    }
    for (; kk < cnt; kk += G) {
        const int k = kk + q;
        const bool in = k < cnt;
        const int kr = in ? k : 0;   // a valid stage entry for lanes past the end
        bool c;
        float r = 0.f;
        if constexpr (kFP64) {
            c = in && vi && fresh(st.root[kr]) && link_f64_staged(st, kr, dxi, dyi, dzi, br);
        } else {
            const float4 cq = st.v[kr];
            r = dist2_f32(cq, hx, hy, hz);
            c = in && r <= br.hi32 && fresh(__float_as_int(cq.w));   // false for invalid (NaN) lanes
        }
        if constexpr (kSelf) c = c && st.slot[kr] > i;
        if (__ballot(c))
            dense_hit<kFP64, kStats, kGeneral>(p, br, st, kr, c, r, pi, root_i, known0, known1, links, band, retries);
    }
}

// Fills stages from the ranges in `rl` (lane l < 27 holds range l's length
// in `len`, its first slot in `j0`, its shift code in `code`) and tests them
// against the home lanes (home coordinates hx, hy, hz, already shifted where
// the group needs it).
template <bool kFP64, bool kStats, bool kGeneral, bool kSelf>
__device__ __forceinline__ void dense_ranges(const Plan &p, const BoxRegs &br, typename Stage<kFP64>::T &st,
                                             RangeList &rl, int len, int j0, int code, int G, int q, int i, bool vi,
                                             float4 pi, float hx, float hy, float hz, int n_home, int &root_i,
                                             int &known0,
                                             int &known1, unsigned long long &tests, unsigned long long &links,
                                             unsigned long long &band, unsigned &retries)
{
    const int lane = lane_id();
    const int incl = wave_incl_scan(lane < 27 ? len : 0);
    const int total = __shfl(incl, 63, 64);
    if (total == 0) return;
    if (lane < 27) {
        rl.pre[lane + 1] = incl;
        rl.j0[lane] = j0;
        rl.code[lane] = code;
    }
    if (lane == 0) rl.pre[0] = 0;
    __builtin_amdgcn_wave_barrier();
    const bool rnd = kGeneral && p.link_random;
    const double dxi = (double)pi.x, dyi = (double)pi.y, dzi = (double)pi.z;
#pragma unroll 1
    for (int t0 = 0; t0 < total; t0 += 64) {
        const int t = t0 + lane;
        const bool vj = t < total;
        int r = 0;
        if (vj) {
#pragma unroll
            for (int step = 16; step > 0; step >>= 1)
                if (r + step < 27 && rl.pre[r + step] <= t) r += step;
        }
        const int j = vj ? rl.j0[r] + (t - rl.pre[r]) : 0;
        const int cj = vj ? rl.code[r] : 0;
        const float4 cq = vj ? p.sorted[j] : make_float4(qnan(), qnan(), qnan(), 0.f);
        // the home particle's cached root, checked once per stage fill
        // (other waves may have merged its group meanwhile)
        const int pr = (!kStats && t0 == 0 && vi) ? ld_rel(p.parent + root_i) : root_i;
        const int rj = vj ? find_root(p.parent, j, p.find_mode, rnd) : -2;
        bool keep = vj;
        if constexpr (!kStats) {
            if (pr != root_i) root_i = find_root(p.parent, pr, p.find_mode, rnd);
            // one root for every home lane: candidates of that root are in its group
            const int rh = __builtin_amdgcn_readfirstlane(root_i);   // lane 0 is a home particle
            if (__ballot(vi && root_i != rh) == 0) keep = keep && rj != rh;
        }
        const unsigned long long km = __ballot(keep);
        const int cnt = __popcll(km);
        if (kStats) tests += (unsigned long long)min(64, total - t0) * (unsigned long long)n_home;
        if (cnt == 0) continue;
        __builtin_amdgcn_wave_barrier();   // the previous stage has been read
        if (keep) {
            const int at = __builtin_amdgcn_mbcnt_hi((unsigned)(km >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)km, 0u));
            st.slot[at] = j;
            if constexpr (kFP64) {
                st.x[at] = (double)cq.x;
                st.y[at] = (double)cq.y;
                st.z[at] = (double)cq.z;
                st.sx[at] = axis_shift(cj & 3, br.L);
                st.sy[at] = axis_shift((cj >> 2) & 3, br.L);
                st.sz[at] = axis_shift((cj >> 4) & 3, br.L);
                st.root[at] = rj;
            } else {
                st.v[at] = make_float4((cj & 3) == 1 ? cq.x - br.L32 : cq.x,
                                       ((cj >> 2) & 3) == 1 ? cq.y - br.L32 : cq.y,
                                       ((cj >> 4) & 3) == 1 ? cq.z - br.L32 : cq.z, __int_as_float(rj));
            }
        }
        __builtin_amdgcn_wave_barrier();
        dense_batch<kFP64, kStats, kGeneral, kSelf>(p, br, st, cnt, G, q, i, vi, pi, hx, hy, hz, dxi, dyi, dzi,
                                                    root_i, known0, known1, links, band, retries);
    }
    __builtin_amdgcn_wave_barrier();   // rl and the stage are reused by the next call
}

template <bool kFP64, bool kStats, bool kGeneral>
__global__ void __launch_bounds__(kBlock) k_link_dense(Plan p)
{
    using StageT = typename Stage<kFP64>::T;
    __shared__ StageT stage[kWaves];
    __shared__ RangeList ranges[kWaves];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    StageT &st = stage[wid];
    RangeList &rl = ranges[wid];
    unsigned long long tests = 0, links = 0, band = 0;
    unsigned retries = 0;
    const int n_items = (int)p.counters->n_items;
    const XcdRange xr = xcd_range(n_items, kWaves, wid);   // items come in cell order
    for (int64_t it = xr.first; it < xr.end; it += xr.stride) {
        const int4 item = p.items[it];
        const int cxy = __builtin_amdgcn_readfirstlane(item.x);
        const int first = __builtin_amdgcn_readfirstlane(item.y);
        const int b = __builtin_amdgcn_readfirstlane(item.z);
        const int cx = cxy & 0xffff, cy = cxy >> 16, cz = __builtin_amdgcn_readfirstlane(item.w);
        const BoxDev &bd = box_of(p, b);
        const int nc = bd.nc;
        const int64_t cb = bd.cell_base;
        BoxRegs br;
        br.L = bd.L;
        br.half = bd.half;
        br.l2 = bd.l2;
        br.lo32 = bd.lo32;
        br.hi32 = bd.hi32;
        br.L32 = bd.L32;
        br.strict = p.strict != 0;
        // the 27 neighbour cells, one per lane (lanes 0-26, neighbour
        // nb = 9 (dz + 1) + 3 (dy + 1) + dx + 1), looked up at once; code:
        // per axis 1 = the neighbour is the top cell across the low face,
        // 2 = the home cell is the top one and the neighbour across the high face
        int nb_j0 = 0, nb_j1 = 0, code = 0;
        if (lane < 27) {
            int nx = cx + lane % 3 - 1, ny = cy + (lane / 3) % 3 - 1, nz = cz + lane / 9 - 1;
            if (nx < 0) { nx += nc; code |= 1; } else if (nx >= nc) { nx -= nc; code |= 2; }
            if (ny < 0) { ny += nc; code |= 1 << 2; } else if (ny >= nc) { ny -= nc; code |= 2 << 2; }
            if (nz < 0) { nz += nc; code |= 1 << 4; } else if (nz >= nc) { nz -= nc; code |= 2 << 4; }
            const int2 sp = cell_span(p, cb + ((int64_t)nz * nc + ny) * nc + nx);
            nb_j0 = sp.x;
            nb_j1 = sp.y;
        }
        const int ce = __shfl(nb_j1, 13, 64);   // the cell itself
        const int n_home = min(64, ce - first);
        // home particles per copy (H) and copies (G = 64 / H)
        const int H = n_home > 32 ? 64 : (n_home > 16 ? 32 : 16);
        const int G = 64 / H, q = lane / H;
        const int i = first + (lane & (H - 1));
        const bool vi = i < ce;
        const float4 pi = vi ? p.sorted[i] : make_float4(qnan(), qnan(), qnan(), 0.f);
        int root_i = vi ? find_root(p.parent, i, p.find_mode, kGeneral && p.link_random) : -1;
        int known0 = -3, known1 = -3;   // never a node
        // neighbours searched from here: the upper half shell, and the lower
        // half where the neighbour is sparse (a dense one searches the pair)
        const int nlen = nb_j1 - nb_j0;
        const bool searched = lane < 27 && lane != 13 && nlen > 0 && (lane > 13 || nlen < p.dense_min);
        const bool home_shift = (code & 0x2a) != 0;   // some axis has code 2
        const bool together = searched && (kFP64 || !home_shift);

        // the cell itself
        dense_ranges<kFP64, kStats, kGeneral, true>(p, br, st, rl, lane == 13 ? ce - first : 0, first, 0, G, q, i, vi,
                                                    pi, pi.x, pi.y, pi.z, n_home, root_i, known0, known1, tests, links,
                                                    band, retries);
        // every neighbour that needs no shift of the home coordinate, at once
        dense_ranges<kFP64, kStats, kGeneral, false>(p, br, st, rl, together ? nlen : 0, nb_j0, code, G, q, i, vi,
                                                     pi, pi.x, pi.y, pi.z, n_home, root_i, known0, known1, tests,
                                                     links, band, retries);
        if constexpr (!kFP64) {
            // neighbours across a high face, one at a time
            unsigned long long rest = __ballot(searched && !together);
            while (rest) {
                const int nb = __ffsll((long long)rest) - 1;
                rest &= rest - 1;
                const int cd = __shfl(code, nb, 64);
                const float hx = (cd & 3) == 2 ? pi.x - br.L32 : pi.x;
                const float hy = ((cd >> 2) & 3) == 2 ? pi.y - br.L32 : pi.y;
                const float hz = ((cd >> 4) & 3) == 2 ? pi.z - br.L32 : pi.z;
                dense_ranges<kFP64, kStats, kGeneral, false>(p, br, st, rl, lane == nb ? nlen : 0, nb_j0, code, G, q,
                                                             i, vi, pi, hx, hy, hz, n_home, root_i, known0, known1,
                                                             tests, links, band, retries);
            }
        }
    }
    if (kStats) {
        links = wave_sum_u64(links);
        band = wave_sum_u64(band);
        unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane == 0) {
            atomicAdd(&p.counters->pair_tests, tests);
            atomicAdd(&p.counters->links, links);
            atomicAdd(&p.counters->band_hits, band);
            atomicAdd(&p.counters->cas_retries, r);
        }
    }
}

// Pre-merge of dense cells (before the pair search): one wavefront per dense
// cell splits it into k^3 sub-cells small enough that any two particles of
// one sub-cell are linked. When the sub-cells are smaller still (sub_adj:
// any two particles of two sub-cells that touch, across a face, an edge or a
// corner, are linked), a union-find over the occupied sub-cells in LDS joins
// every two touching occupied sub-cells. Every particle is then hooked
// straight under the particle of highest hooking priority (smallest key) of
// its sub-cell or joined set: only particles joined by chains of linked pairs
// are merged, so the groups are unchanged, and the pair search meets few
// groups per dense cell (its staging drops the candidates of the home
// particles' own group). The particles of dense cells are still their own
// roots when this runs (the per-particle search and its union pass never
// link them) and each dense cell has one wavefront, so the hooks are plain
// stores.
constexpr int kMaxSub = 512;

// Coordinates of sub-cell t on a k^3 grid (t < k^3 <= kMaxSub): the float
// quotients of t + 1/2 lie at least 1/(2 k^2) from an integer, far above
// their rounding error, so truncation gives the integer quotients.
__device__ __forceinline__ void sub_xyz(int t, int k, float inv_k, float inv_k2, int &sx, int &sy, int &sz)
{
    sz = (int)(((float)t + 0.5f) * inv_k2);
    const int r = t - sz * k * k;
    sy = (int)(((float)r + 0.5f) * inv_k);
    sx = r - sy * k;
}

__global__ void __launch_bounds__(kBlock) k_dense_premerge(Plan p)
{
    // per sub-cell: (hooking key << 32 | particle) of its first particle, ~0 when empty
    __shared__ unsigned long long rep[kWaves][kMaxSub];
    __shared__ int join[kWaves][kMaxSub];   // forest over the sub-cells (sub_adj)
    __shared__ int used[kWaves][kMaxSub];   // the occupied sub-cells (sub_adj)
    const int wid = threadIdx.x >> 6, lane = lane_id();
    unsigned long long *rp = rep[wid];
    int *jf = join[wid];
    int *ul = used[wid];
    const bool rnd = p.link_random != 0;
    constexpr unsigned long long kEmpty = ~0ull;
    const int n_items = (int)p.counters->n_items;
    const XcdRange xr = xcd_range(n_items, kWaves, wid);
    for (int64_t it = xr.first; it < xr.end; it += xr.stride) {
        const int4 item = p.items[it];
        const int cxy = __builtin_amdgcn_readfirstlane(item.x);
        const int first = __builtin_amdgcn_readfirstlane(item.y);
        const int b = __builtin_amdgcn_readfirstlane(item.z);
        const int cx = cxy & 0xffff, cy = cxy >> 16, cz = __builtin_amdgcn_readfirstlane(item.w);
        const BoxDev &bd = box_of(p, b);
        const int nc = bd.nc;
        const int2 sp = cell_span(p, bd.cell_base + ((int64_t)cz * nc + cy) * nc + cx);
        const int cs = __builtin_amdgcn_readfirstlane(sp.x);
        if (first != cs) continue;   // the cell's first item does the whole cell
        const int k = bd.sub_k;
        if (k == 0) continue;
        const bool adj = bd.sub_adj != 0;
        const float inv_k = 1.0f / (float)k, inv_k2 = 1.0f / (float)(k * k);
        const int ce = __builtin_amdgcn_readfirstlane(sp.y);
        const int nsub = k * k * k;
        for (int t = lane; t < nsub; t += 64) {
            rp[t] = kEmpty;
            jf[t] = t;
        }
        __builtin_amdgcn_wave_barrier();
        auto sub_of = [&](int j) {
            const float4 q = p.sorted[j];
            const double fx = (double)q.x * bd.inv_h - cx, fy = (double)q.y * bd.inv_h - cy,
                         fz = (double)q.z * bd.inv_h - cz;
            const int sx = min(max((int)floor(fx * k), 0), k - 1);
            const int sy = min(max((int)floor(fy * k), 0), k - 1);
            const int sz = min(max((int)floor(fz * k), 0), k - 1);
            return (sz * k + sy) * k + sx;
        };
        int sj0 = 0;   // the sub-cell of this lane's first particle, kept for the hooks below
        for (int j = cs + lane; j < ce; j += 64) {
            const int sj = sub_of(j);
            if (j < cs + 64) sj0 = sj;
            atomicMin(&rp[sj], ((unsigned long long)link_key(j, rnd) << 32) | (unsigned)j);
        }
        __builtin_amdgcn_wave_barrier();
        if (adj) {
            // the occupied sub-cells, listed (there are at most as many as
            // particles), then each joined with the touching occupied ones
            // among the 13 of its 26 neighbours that come after it
            int n_used = 0;
            for (int t0 = 0; t0 < nsub; t0 += 64) {
                const int t = t0 + lane;
                const bool occ = t < nsub && rp[t] != kEmpty;
                const unsigned long long m = __ballot(occ);
                if (occ) ul[n_used + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = t;
                n_used += __popcll(m);
            }
            __builtin_amdgcn_wave_barrier();
            if (n_used <= 64) {
                // at most 64 occupied sub-cells: lane q holds a row of bits, the
                // listed sub-cells touching sub-cell ul[q], and the components
                // come from the closure of the rows; jf maps a listed sub-cell
                // to its place in the list, then to its component's first one
                if (lane < n_used) jf[ul[lane]] = lane;
                __builtin_amdgcn_wave_barrier();
                unsigned long long row = 0ull;
                int t = 0;
                if (lane < n_used) {
                    t = ul[lane];
                    int sx, sy, sz;
                    sub_xyz(t, k, inv_k, inv_k2, sx, sy, sz);
                    row = 1ull << lane;
#pragma unroll
                    for (int o = 0; o < 27; ++o) {   // no branch: an outside neighbour reads sub-cell t
                        const int ux = sx + o % 3 - 1, uy = sy + (o / 3) % 3 - 1, uz = sz + o / 9 - 1;
                        const bool in = (unsigned)ux < (unsigned)k && (unsigned)uy < (unsigned)k &&
                                        (unsigned)uz < (unsigned)k;
                        const int u = in ? (uz * k + uy) * k + ux : t;
                        row |= (rp[u] != kEmpty ? 1ull : 0ull) << jf[u];
                    }
                }
                row = close_rows(row, __ballot(lane < n_used && row != (1ull << lane)));
                __builtin_amdgcn_wave_barrier();   // every map entry read
                if (lane < n_used) {
                    const int rt = ul[__ffsll((long long)row) - 1];
                    jf[t] = rt;
                    if (rt != t) atomicMin(&rp[rt], rp[t]);
                }
            } else {
                for (int q = lane; q < n_used; q += 64) {
                    const int t = ul[q];
                    int sx, sy, sz;
                    sub_xyz(t, k, inv_k, inv_k2, sx, sy, sz);
                    for (int o = 14; o < 27; ++o) {
                        const int ux = sx + o % 3 - 1, uy = sy + (o / 3) % 3 - 1, uz = sz + o / 9 - 1;
                        if (ux < 0 || ux >= k || uy < 0 || uy >= k || uz >= k) continue;
                        const int u = (uz * k + uy) * k + ux;
                        if (rp[u] != kEmpty) lds_unite(jf, t, u);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                // the particle of smallest key of each joined set, at its root sub-cell
                for (int q = lane; q < n_used; q += 64) {
                    const int t = ul[q];
                    const int r = lds_find(jf, t);
                    if (r != t) atomicMin(&rp[r], rp[t]);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int j = cs + lane; j < ce; j += 64) {
            const int sj = j < cs + 64 ? sj0 : sub_of(j);
            const int r = (int)(unsigned)(rp[adj ? lds_find(jf, sj) : sj] & 0xffffffffull);
            if (r != j) p.parent[j] = r;   // a key smaller than j's: a valid hook of a root
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Global merge of domain mode, after the search. Workspace: the segment-order
// staging buffer (free after the build) holds flag/number [n + 1], the
// merge forest [n] and the group of each number [n].
//   roots: replace each boundary pair by the roots of its two groups and flag them
//   (an exclusive prefix over the flags numbers the flagged groups densely:
//    the paper's global-ID map, order-preserving so the smallest root of a
//    merged set also has the smallest number)
//   init:  a one-node tree per numbered group
//   union: union-find over the numbered pairs
//   apply: hook each merged group's root under its set's smallest root
__device__ __forceinline__ int *gm_flag(const Plan &p) { return reinterpret_cast<int *>(p.staging2); }
__device__ __forceinline__ int *gm_parent(const Plan &p) { return gm_flag(p) + p.n + 1; }
__device__ __forceinline__ int *gm_group(const Plan &p) { return gm_flag(p) + 2 * p.n + 1; }
__device__ __forceinline__ int64_t gm_pairs(const Plan &p)
{
    const int64_t nb = p.counters->n_boundary;
    return nb < p.max_edges ? nb : p.max_edges;
}

__global__ void __launch_bounds__(kBlock) k_gm_clear(Plan p)
{
    int *flag = gm_flag(p);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= p.n; i += (int64_t)gridDim.x * kBlock) flag[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_gm_roots(Plan p)
{
    int *flag = gm_flag(p);
    const int64_t nb = gm_pairs(p);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nb; k += (int64_t)gridDim.x * kBlock) {
        const int2 e = p.bnd[k];
        const int ra = find_halve(p.parent, e.x), rb = find_halve(p.parent, e.y);
        p.bnd[k] = make_int2(ra, rb);
        flag[ra] = 1;
        flag[rb] = 1;
    }
}

__global__ void __launch_bounds__(kBlock) k_gm_init(Plan p)
{
    const int *num = gm_flag(p);   // exclusive prefix of the flags
    int *gp = gm_parent(p), *grp = gm_group(p);
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < p.n; r += (int64_t)gridDim.x * kBlock) {
        const int k = num[r];
        if (num[r + 1] != k) {
            gp[k] = k;
            grp[k] = (int)r;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.counters->n_bgroups = (unsigned)num[p.n];
}

__global__ void __launch_bounds__(kBlock) k_gm_union(Plan p)
{
    const int *num = gm_flag(p);
    int *gp = gm_parent(p);
    const int64_t nb = gm_pairs(p);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nb; k += (int64_t)gridDim.x * kBlock) {
        const int2 e = p.bnd[k];
        (void)unite(gp, num[e.x], num[e.y], false);
    }
}

__global__ void __launch_bounds__(kBlock) k_gm_apply(Plan p)
{
    const int *num = gm_flag(p);
    int *gp = gm_parent(p);
    const int *grp = gm_group(p);
    const int m = num[p.n];
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < m; k += gridDim.x * kBlock) {
        const int r = find_halve(gp, k);
        if (r != k) p.parent[grp[k]] = grp[r];   // grp[r] < grp[k]: numbers keep the order of the roots
    }
}

// ------------------------------------------------- giant-component skip --
// In the manner of Afforest (Sutton et al., IPDPS 2018): after a first pass
// that links every particle to its axis-neighbour cells only (the per-particle
// search with Plan::sample set) and the dense-cell search, the largest group
// of a sample of roots is taken as "giant". The rest of the links is then
// searched over the whole periodic shell, both ways, but only from particles
// outside the giant group: a pair with one end inside is found from the other
// end, and a pair with both ends inside needs no union. Every linked pair of
// sparse cells is thereby merged; dense cells keep their own search.

__global__ void __launch_bounds__(kBlock) k_edge_reset(Plan p)
{
    if (threadIdx.x < kEdgeSlices) p.edge_fill[threadIdx.x] = 0;
}

constexpr int kGiantSamples = 4096;
constexpr int kGiantBlock = 1024;

// One work-group: the roots of kGiantSamples evenly spaced particles, sorted
// in LDS (bitonic), and the value of the longest run of equal roots.
__global__ void __launch_bounds__(kGiantBlock) k_giant(Plan p)
{
    __shared__ int r[kGiantSamples];
    __shared__ unsigned long long best;
    const int tid = (int)threadIdx.x;
    const bool rnd = p.link_random != 0;
    for (int k = tid; k < kGiantSamples; k += kGiantBlock)
        r[k] = find_root(p.parent, (int)((int64_t)k * p.n / kGiantSamples), p.find_mode, rnd);
    if (tid == 0) best = 0;
    __syncthreads();
    for (int k = 2; k <= kGiantSamples; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int idx = tid; idx < kGiantSamples; idx += kGiantBlock) {
                const int ixj = idx ^ j;
                if (ixj > idx) {
                    const int a = r[idx], b = r[ixj];
                    if ((a > b) == ((idx & k) == 0)) {
                        r[idx] = b;
                        r[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int idx = tid; idx < kGiantSamples; idx += kGiantBlock) {
        if (idx > 0 && r[idx - 1] == r[idx]) continue;   // not the start of a run
        int lo = idx, hi = kGiantSamples;                 // first entry above r[idx]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (r[mid] <= r[idx]) lo = mid + 1;
            else hi = mid;
        }
        atomicMax(&best, ((unsigned long long)(lo - idx) << 32) | (unsigned)r[idx]);
    }
    __syncthreads();
    if (tid == 0) p.counters->giant = (int)(unsigned)(best & 0xffffffffull);
}

// The pair test of the per-particle search: FP32 with the image shift applied
// where it is exact (shift codes as for candidate ranges), re-decided in
// double inside the band; or the double predicate with the shift added after
// the rounded difference.
template <bool kFP64, bool kStats>
__device__ __forceinline__ bool pair_link(const float4 h, const float4 c, int code, const BoxPair &bx, bool strict,
                                          unsigned long long &band)
{
    if constexpr (kFP64) {
        const double tx = ((double)h.x - (double)c.x) + axis_shift(code & 3, bx.L);
        const double ty = ((double)h.y - (double)c.y) + axis_shift((code >> 2) & 3, bx.L);
        const double tz = ((double)h.z - (double)c.z) + axis_shift((code >> 4) & 3, bx.L);
        const double sxy = tx * tx + ty * ty;
        const double r2 = sxy + tz * tz;
        return strict ? (r2 < bx.l2) : (r2 <= bx.l2);
    } else {
        const float dx = axis_diff(h.x, c.x, code & 3, bx.L32);
        const float dy = axis_diff(h.y, c.y, (code >> 2) & 3, bx.L32);
        const float dz = axis_diff(h.z, c.z, (code >> 4) & 3, bx.L32);
        const float rr = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (rr < bx.lo32) return true;
        if (rr > bx.hi32) return false;
        if (kStats) ++band;
        return link_fp64(h.x, h.y, h.z, c.x, c.y, c.z, bx.L, bx.half, bx.l2, strict);
    }
}

// The second pass: one home particle per lane, skipped when it lies in the
// giant group or in a dense cell; otherwise every sparse cell of its periodic
// shell (all 27, both ways, the home particle itself excluded), each cell's
// candidates in lockstep over the wave so that the edge sink is reached by
// every lane together.
template <bool kFP64, bool kStats>
__global__ void __launch_bounds__(kBlock) k_link_rest(Plan p)
{
    __shared__ int2 ebuf[kWaves][kEdgeBuf];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    EdgeSink sink{ebuf[wid], 0};
    unsigned long long tests = 0, links = 0, band = 0;
    unsigned retries = 0;
    const bool rnd = p.link_random != 0;
    const bool strict = p.strict != 0;
    BoxHint hint;
    const int64_t n_tiles = (p.n + 63) / 64;
    const XcdRange xr = xcd_range(n_tiles, kWaves, wid);
    for (int64_t tile = xr.first; tile < xr.end; tile += xr.stride) {
        const int64_t s64 = tile * 64 + lane;
        bool active = s64 < p.n;
        const int s = active ? (int)s64 : 0;
        const int g = find_root(p.parent, p.counters->giant, p.find_mode, rnd);
        if (active) active = find_root(p.parent, s, p.find_mode, rnd) != g;
        int cx = 0, cy = 0, cz = 0, nc = 3;
        int64_t cb = 0;
        float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
        BoxPair bx{};
        const int b = p.n_boxes == 1 ? 0 : find_box_hint(p.box_p0, p.n_boxes, s, hint);
        if (active) {
            const BoxDev &bd = box_of(p, b);
            bx = BoxPair::of(bd);
            h = p.sorted[s];
            nc = bd.nc;
            cb = bd.cell_base;
            cx = cell_coord(h.x, bd.inv_h, nc);
            cy = cell_coord(h.y, bd.inv_h, nc);
            cz = cell_coord(h.z, bd.inv_h, nc);
            const int2 own = cell_span(p, cb + ((int64_t)cz * nc + cy) * nc + cx);
            if (own.y - own.x >= p.dense_min) active = false;   // the dense search covers its pairs
        }
        if (__ballot(active) == 0) continue;
#pragma unroll 1
        for (int nb = 0; nb < 27; ++nb) {
            int j0 = 0, len = 0, code = 0;
            if (active) {
                int nx = cx + nb % 3 - 1, ny = cy + (nb / 3) % 3 - 1, nz = cz + nb / 9 - 1;
                if (nx < 0) { nx += nc; code |= 1; } else if (nx >= nc) { nx -= nc; code |= 2; }
                if (ny < 0) { ny += nc; code |= 1 << 2; } else if (ny >= nc) { ny -= nc; code |= 2 << 2; }
                if (nz < 0) { nz += nc; code |= 1 << 4; } else if (nz >= nc) { nz -= nc; code |= 2 << 4; }
                const int2 sp = cell_span(p, cb + ((int64_t)nz * nc + ny) * nc + nx);
                if (sp.y - sp.x < p.dense_min) {
                    j0 = sp.x;
                    len = sp.y - sp.x;
                }
            }
            int most = len;
            for (int d = 32; d >= 1; d >>= 1) most = max(most, __shfl_xor(most, d, 64));
            for (int t = 0; t < most; ++t) {
                const int j = j0 + t;
                const bool valid = t < len && j != s;
                bool link = false;
                if (valid) {
                    const float4 c = p.sorted[j];
                    link = pair_link<kFP64, kStats>(h, c, code, bx, strict, band);
                    if (kStats) {
                        ++tests;
                        if (link) ++links;
                    }
                }
                sink.push(p, link, s, j, retries);
            }
        }
    }
    sink.flush(p, retries);
    if (kStats) {
        tests = wave_sum_u64(tests);
        links = wave_sum_u64(links);
        band = wave_sum_u64(band);
        unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane == 0) {
            atomicAdd(&p.counters->sparse_tests, tests);
            atomicAdd(&p.counters->pair_tests, tests);
            atomicAdd(&p.counters->links, links);
            atomicAdd(&p.counters->band_hits, band);
            atomicAdd(&p.counters->cas_retries, r);
        }
    }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <bool kFP64, bool kStats>
hipError_t launch_link_t(const Plan &p, hipStream_t stream, KernelTimer *t, const Fork *fk)
{
    Plan first = p;
    first.sample = p.giant_skip;   // the giant-component skip starts from the axis links
    if (t) t->mark(K_LINK_SPARSE, false, stream);
    hipLaunchKernelGGL((k_link_sparse<kFP64, kStats>), dim3((unsigned)p.sparse_blocks), dim3(kBlock), 0, stream,
                       first);
    if (t) t->mark(K_LINK_SPARSE, true, stream);
    // the sub-cell pre-merge would merge across slab faces: not in domain mode
    const bool premerge = p.domains <= 1 && p.premerge;
    // The pre-merge reads and writes the parents of particles in dense cells
    // only, the union pass those of particles in sparse cells only (the
    // per-particle search pairs sparse cells with sparse cells): given a
    // second stream the two run side by side, the pre-merge waiting for the
    // cell sort alone, and the wavefront search waits for both. Not with
    // per-kernel timers, whose events time each kernel alone.
    const bool beside = premerge && fk && fk->side && !t;
    if (beside) {
        hipError_t e = hipEventRecord(fk->fork, stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(fk->side, fk->fork, 0);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_dense_premerge, dim3((unsigned)p.dense_blocks), dim3(kBlock), 0, fk->side, p);
        e = hipEventRecord(fk->join, fk->side);
        if (e != hipSuccess) return e;
    }
    if (t) t->mark(K_UNION_EDGES, false, stream);
    hipLaunchKernelGGL((k_union_edges<kStats>), dim3(kUnionParts * kEdgeSlices), dim3(kBlock), 0, stream, p);
    if (t) t->mark(K_UNION_EDGES, true, stream);
    if (beside) {
        const hipError_t e = hipStreamWaitEvent(stream, fk->join, 0);
        if (e != hipSuccess) return e;
    } else if (premerge) {
        if (t) t->mark(K_PREMERGE, false, stream);
        hipLaunchKernelGGL(k_dense_premerge, dim3((unsigned)p.dense_blocks), dim3(kBlock), 0, stream, p);
        if (t) t->mark(K_PREMERGE, true, stream);
    }
    if (t) t->mark(K_LINK_DENSE, false, stream);
    if (p.domains > 1 || p.link_random)
        hipLaunchKernelGGL((k_link_dense<kFP64, kStats, true>), dim3((unsigned)p.dense_blocks), dim3(kBlock), 0,
                           stream, p);
    else
        hipLaunchKernelGGL((k_link_dense<kFP64, kStats, false>), dim3((unsigned)p.dense_blocks), dim3(kBlock), 0,
                           stream, p);
    if (t) t->mark(K_LINK_DENSE, true, stream);
    if (p.giant_skip) {
        // the rest of the sparse pairs, from the particles outside the giant
        // group (timed with the per-particle search and the union pass)
        hipLaunchKernelGGL(k_edge_reset, dim3(1), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k_giant, dim3(1), dim3(kGiantBlock), 0, stream, p);
        if (t) t->mark(K_LINK_SPARSE, false, stream);
        hipLaunchKernelGGL((k_link_rest<kFP64, kStats>), dim3((unsigned)p.sparse_blocks), dim3(kBlock), 0, stream,
                           p);
        if (t) t->mark(K_LINK_SPARSE, true, stream);
        if (t) t->mark(K_UNION_EDGES, false, stream);
        hipLaunchKernelGGL((k_union_edges<kStats>), dim3(kUnionParts * kEdgeSlices), dim3(kBlock), 0, stream, p);
        if (t) t->mark(K_UNION_EDGES, true, stream);
    }
    if (p.domains > 1) {
        // global merge, timed with the union pass
        if (t) t->mark(K_UNION_EDGES, false, stream);
        const unsigned g = kGlobalMergeBlocks;
        hipLaunchKernelGGL(k_gm_clear, dim3(g), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k_gm_roots, dim3(g), dim3(kBlock), 0, stream, p);
        scan_exclusive(reinterpret_cast<int *>(p.staging2), p.n + 1, p.scan_part, stream);
        hipLaunchKernelGGL(k_gm_init, dim3(g), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k_gm_union, dim3(g), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k_gm_apply, dim3(g), dim3(kBlock), 0, stream, p);
        if (t) t->mark(K_UNION_EDGES, true, stream);
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_link(const Plan &p, hipStream_t stream, KernelTimer *t, const Fork *fk)
{
    if (p.n == 0) return hipSuccess;
    const bool fp64 = p.predicate == 0;
    hipError_t e;
    if (fp64) e = p.stats ? launch_link_t<true, true>(p, stream, t, fk) : launch_link_t<true, false>(p, stream, t, fk);
    else e = p.stats ? launch_link_t<false, true>(p, stream, t, fk) : launch_link_t<false, false>(p, stream, t, fk);
    return e != hipSuccess ? e : hipGetLastError();
}

int64_t max_dense_items(int64_t n, int dense_min)
{
    const int64_t t = dense_min > 0 ? dense_min : 1;
    return n / 64 + n / t + 64;
}

}  // namespace fof
