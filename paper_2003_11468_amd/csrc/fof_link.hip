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

struct Ranges {
    int j0[kMaxRanges], j1[kMaxRanges], code[kMaxRanges];
    int n = 0;
    __device__ __forceinline__ void add(int a, int b, int c)
    {
        if (b <= a) return;
#pragma unroll
        for (int r = 0; r < kMaxRanges; ++r)
            if (r == n) {
                j0[r] = a;
                j1[r] = b;
                code[r] = c;
            }
        ++n;
    }
};

// The three cells (x = cx-1, cx, cx+1) of one neighbour row, given their
// boundaries b0..b3 (b_e = start of cell e, b_{e+1} its end when the cells
// are contiguous) and whether the row wraps at either end. Runs of sparse,
// memory-contiguous cells are merged into one range: at most two per row.
__device__ __forceinline__ void add_row(Ranges &R, const int st[3], const int en[3], const int xcode[3],
                                        int yz_code, int dense_min)
{
    int a = -1, b = -1, code = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const bool sparse = en[e] - st[e] < dense_min;
        const int c = xcode[e] | yz_code;
        if (sparse && en[e] > st[e]) {
            if (a >= 0 && st[e] == b && c == code) {
                b = en[e];
            } else {
                if (a >= 0) R.add(a, b, code);
                a = st[e];
                b = en[e];
                code = c;
            }
        }
    }
    if (a >= 0) R.add(a, b, code);
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
    int tag[kMaxUnits];         // shift code (bits 0-5) | home lane << 8
    float4 home[64];            // the home particles
    int2 ebuf[kEdgeBuf];        // edge sink buffer
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
                                             int n_pairs, int b, BoxPair bp, unsigned long long &tests,
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
                    const float dx = axis_diff(hp.x, c.x, code & 3, bx.L32);
                    const float dy = axis_diff(hp.y, c.y, (code >> 2) & 3, bx.L32);
                    const float dz = axis_diff(hp.z, c.z, (code >> 4) & 3, bx.L32);
                    const float rr = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    if (rr < bx.lo32) link = true;
                    else if (rr > bx.hi32) link = false;
                    else {
                        if (kStats) ++band;
                        link = link_fp64(hp.x, hp.y, hp.z, c.x, c.y, c.z, bx.L, bx.half, bx.l2, strict);
                    }
                }
                if (kStats) ++tests;
                if (kStats && link) ++links;
            }
            sink.push(p, link, s0 + hl, jj[a], retries);
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
    const int64_t n_tiles = (p.n + 63) / 64;
    // each XCD sweeps one contiguous range of tiles, so the neighbour rows of
    // consecutive tiles are reused from its own L2
    const XcdRange xr = xcd_range(n_tiles, kWaves, wid);
    for (int64_t tile = xr.first; tile < xr.end; tile += xr.stride) {
        const int64_t s64 = tile * 64 + lane;
        Ranges R;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
        int b = 0;
        if (s64 < p.n) {
            const int s = (int)s64;
            b = p.n_boxes == 1 ? 0 : find_box_wave(p.box_p0, p.n_boxes, s64);
            const BoxDev &bd = box_of(p, b);
            pi = p.sorted[s];
            const int nc = bd.nc;
            const int cx = cell_coord(pi.x, bd.inv_h, nc);
            const int cy = cell_coord(pi.y, bd.inv_h, nc);
            const int cz = cell_coord(pi.z, bd.inv_h, nc);
            const int cb = (int)bd.cell_base;
            const int c = cb + (cz * nc + cy) * nc + cx;
            const int *cst = p.cstart;
            const int dense_min = p.dense_min;
            const int seg_shift = p.seg_shift;
            const int rb0 = c - cx;
            // Boundaries of the own row and the four neighbour rows (dy, dz) =
            // (1, 0), (-1, 1), (0, 1), (1, 1): with the own cell these hold the
            // 13 half-shell cells. Occupancy words (bits and rank base per 32
            // cells, a small array that stays in cache) give the rank of each
            // cell among the occupied ones, and cstart the boundaries.
            const uint2 *occ = p.occ;
            typedef unsigned uint4a8 __attribute__((ext_vector_type(4), aligned(8)));
            typedef int int4a4 __attribute__((ext_vector_type(4), aligned(4)));
            auto rank_in = [](unsigned bits, unsigned base, int cell_index) {
                return (int)base + __popc(bits & ((1u << (cell_index & 31)) - 1u));
            };
            auto span = [&](int cell_index, int &s0, int &s1) {   // left at 0, 0 for an empty cell
                const uint2 w = occ[cell_index >> 5];
                if ((w.x >> (cell_index & 31)) & 1u) {
                    const int r = rank_in(w.x, w.y, cell_index);
                    s0 = cst[r];
                    s1 = cst[r + 1];
                }
            };
            const int nxp = cx + 1 < nc ? cx + 1 : 0;
            const bool inner = cx >= 1 && cx + 1 < nc;
            const int rdy[4] = {1, -1, 0, 1}, rdz[4] = {0, 1, 1, 1};
            int rb[4], yz[4], c0[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int ny = cy + rdy[r], nz = cz + rdz[r], code = 0;
                if (ny >= nc) { ny -= nc; code |= 2 << 2; }
                else if (ny < 0) { ny += nc; code |= 1 << 2; }
                if (nz >= nc) { nz -= nc; code |= 2 << 4; }
                yz[r] = code;
                rb[r] = cb + (nz * nc + ny) * nc;
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
                mr[r] = (unsigned)((((uint64_t)wr[r].x | ((uint64_t)wr[r].z << 32)) >> (c0[r] & 31)) & 7u);
                qr[r] = *reinterpret_cast<const int4a4 *>(cst + rank_in(wr[r].x, wr[r].y, c0[r]));
            }
            const int own_start = qo.x, own_end = qo.y;
            int nxt_start = 0, nxt_end = 0;
            if (nxp && ((c ^ (c + 1)) >> seg_shift) == 0) {
                // the next cell in the same segment: its entries follow the own cell's
                const unsigned nbits = ((c + 1) & 31) ? wo.x : wo.z;
                if ((nbits >> ((c + 1) & 31)) & 1u) {
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
                    R.add(s + 1, nxt_end, 0);
                } else {
                    R.add(s + 1, own_end, 0);
                    if (nxt_end - nxt_start < dense_min) R.add(nxt_start, nxt_end, xcode_next);
                }
                const int xcode[3] = {cx == 0 ? 1 : 0, 0, cx + 1 == nc ? 2 : 0};
#pragma unroll
                for (int r = 0; r < 4; ++r) add_row(R, st[r], en[r], xcode, yz[r], dense_min);
            }
        }
        // flatten the units of the wave: unit and pair offsets by prefix sums
        int my_pairs = 0;
#pragma unroll
        for (int r = 0; r < kMaxRanges; ++r)
            if (r < R.n) my_pairs += R.j1[r] - R.j0[r];
        const int unit_incl = wave_incl_scan(R.n);
        const int pair_incl = wave_incl_scan(my_pairs);
        const int n_units = __shfl(unit_incl, 63, 64);
        const int n_pairs = __shfl(pair_incl, 63, 64);
        if (n_pairs == 0) continue;
        {
            int u = unit_incl - R.n, pr = pair_incl - my_pairs;
#pragma unroll
            for (int r = 0; r < kMaxRanges; ++r)
                if (r < R.n) {
                    L.start[u] = pr;
                    L.j0[u] = R.j0[r];
                    L.tag[u] = R.code[r] | (lane << 8);
                    pr += R.j1[r] - R.j0[r];
                    ++u;
                }
            if (lane == 63) L.start[n_units] = n_pairs;
            L.home[lane] = pi;
        }
        __builtin_amdgcn_wave_barrier();
        // a tile inside one box keeps that box's parameters in registers for
        // every pair; otherwise each pair reads the box of its home particle
        const int b0 = __builtin_amdgcn_readfirstlane(b);
        if (__ballot(b != b0) == 0)
            sparse_pairs<kFP64, kStats, true>(p, L, sink, (int)(tile * 64), n_units, n_pairs, b, BoxPair::of(box_of(p, b0)),
                                              tests, links, band, retries);
        else
            sparse_pairs<kFP64, kStats, false>(p, L, sink, (int)(tile * 64), n_units, n_pairs, b, BoxPair{},
                                               tests, links, band, retries);
        __builtin_amdgcn_wave_barrier();
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

// Merges the queued pairs: one thread per pair, no ordering needed. Slice s
// holds the pairs found on XCD s % 8 (the search's work-group b appends to
// slice b % 256, and work-groups go to XCDs round-robin), whose home
// particles are that XCD's contiguous range of cells; its kUnionParts
// work-groups run on the same XCD, so the finds of a slice stay in one L2.
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
    unsigned retries = 0;
    for (int64_t k = (int64_t)part * kBlock + threadIdx.x; k < ne; k += (int64_t)kUnionParts * kBlock) {
        const int2 e = edges[k];
        merge_pair(p, e.x, e.y, retries);
    }
    if (kStats) {
        unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane_id() == 0 && r) atomicAdd(&p.counters->cas_retries, r);
        // queued pairs, for the statistics
        if (part == 0 && threadIdx.x == 0) atomicAdd(&p.counters->n_edges, fill);
    }
}

// ---------------------------------------------------------- dense (wave) --

struct StageF {
    float4 v[64];            // x, y, z (neighbour shift applied), cached root (bits)
};

struct StageD {
    double x[64], y[64], z[64];
    int root[64];
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

// Box parameters the inner loops need, held in registers.
struct BoxRegs {
    double L, half, l2;
    float lo32, hi32;
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
                                          int kk, int jb, bool cand, float r, float4 pi, int &root_i, int &known0,
                                          int &known1, unsigned long long &links, unsigned long long &band,
                                          unsigned &retries)
{
    if (!cand) return;
    const int j = jb + kk;
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
// neighbour's periodic shift added after the rounded difference.
__device__ __forceinline__ bool link_f64_staged(const StageD &st, int kk, double dxi, double dyi, double dzi,
                                                double Lx, double Ly, double Lz, const BoxRegs &br)
{
    const double tx = (dxi - st.x[kk]) + Lx;
    const double ty = (dyi - st.y[kk]) + Ly;
    const double tz = (dzi - st.z[kk]) + Lz;
    const double sxy = tx * tx + ty * ty;
    const double r2 = sxy + tz * tz;
    return br.strict ? (r2 < br.l2) : (r2 <= br.l2);
}

// Tests the staged candidates [0, cnt) against the wave's home particles.
// kSelf: the candidates come from the home cell; only j > i counts. Without
// statistics a candidate whose cached root is known to be in the home
// particle's group is dropped together with the distance test's verdict, so
// once a halo's groups have merged the batch runs without branching.
template <bool kFP64, bool kStats, bool kGeneral, bool kSelf>
__device__ __forceinline__ void dense_batch(const Plan &p, const BoxRegs &br, const typename Stage<kFP64>::T &st,
                                            int cnt, int jb, int i, bool vi, float4 pi, float hx, float hy,
                                            float hz, double dxi, double dyi, double dzi, double Lx, double Ly,
                                            double Lz, int &root_i, int &known0, int &known1,
                                            unsigned long long &links, unsigned long long &band, unsigned &retries)
{
    const int rel = i - jb;   // candidate kk is above the home particle iff kk > rel
    auto fresh = [&](int rj) { return kStats || (rj != root_i && rj != known0); };
    int kk = 0;
    if constexpr (!kFP64) {
        for (; kk + 4 <= cnt; kk += 4) {
            const float4 q0 = st.v[kk + 0], q1 = st.v[kk + 1], q2 = st.v[kk + 2], q3 = st.v[kk + 3];
            const float r0 = dist2_f32(q0, hx, hy, hz);
            const float r1 = dist2_f32(q1, hx, hy, hz);
            const float r2 = dist2_f32(q2, hx, hy, hz);
            const float r3 = dist2_f32(q3, hx, hy, hz);
            bool c0 = r0 <= br.hi32 && fresh(__float_as_int(q0.w));
            bool c1 = r1 <= br.hi32 && fresh(__float_as_int(q1.w));
            bool c2 = r2 <= br.hi32 && fresh(__float_as_int(q2.w));
            bool c3 = r3 <= br.hi32 && fresh(__float_as_int(q3.w));
            if constexpr (kSelf) {
                c0 = c0 && kk + 0 > rel;
                c1 = c1 && kk + 1 > rel;
                c2 = c2 && kk + 2 > rel;
                c3 = c3 && kk + 3 > rel;
            }
            if (__ballot(c0 || c1 || c2 || c3)) {
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, kk + 0, jb, c0, r0, pi, root_i, known0, known1, links,
                                                   band, retries);
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, kk + 1, jb, c1, r1, pi, root_i, known0, known1, links,
                                                   band, retries);
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, kk + 2, jb, c2, r2, pi, root_i, known0, known1, links,
                                                   band, retries);
                dense_hit<kFP64, kStats, kGeneral>(p, br, st, kk + 3, jb, c3, r3, pi, root_i, known0, known1, links,
                                                   band, retries);
            }
        }
    }
    for (; kk < cnt; ++kk) {
        bool c;
        float r = 0.f;
        if constexpr (kFP64) {
            c = vi && fresh(st.root[kk]) && link_f64_staged(st, kk, dxi, dyi, dzi, Lx, Ly, Lz, br);
        } else {
            const float4 q = st.v[kk];
            r = dist2_f32(q, hx, hy, hz);
            c = r <= br.hi32 && fresh(__float_as_int(q.w));   // false for invalid (NaN) lanes and candidates
        }
        if constexpr (kSelf) c = c && kk > rel;
        if (__ballot(c))
            dense_hit<kFP64, kStats, kGeneral>(p, br, st, kk, jb, c, r, pi, root_i, known0, known1, links, band,
                                               retries);
    }
}

template <bool kFP64, bool kStats, bool kGeneral>
__global__ void __launch_bounds__(kBlock) k_link_dense(Plan p)
{
    using StageT = typename Stage<kFP64>::T;
    __shared__ StageT stage[kWaves];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    StageT &st = stage[wid];
    unsigned long long tests = 0, links = 0, band = 0;
    unsigned retries = 0;
    const int n_items = (int)p.counters->n_items;
    const XcdRange xr = xcd_range(n_items, kWaves, wid);   // items come in cell order
    for (int64_t it = xr.first; it < xr.end; it += xr.stride) {
        const int4 item = p.items[it];
        const int c = __builtin_amdgcn_readfirstlane(item.x);
        const int first = __builtin_amdgcn_readfirstlane(item.y);
        const int b = __builtin_amdgcn_readfirstlane(item.z);
        const BoxDev &bd = box_of(p, b);
        const int nc = bd.nc, cb = (int)bd.cell_base;
        BoxRegs br;
        br.L = bd.L;
        br.half = bd.half;
        br.l2 = bd.l2;
        br.lo32 = bd.lo32;
        br.hi32 = bd.hi32;
        br.strict = p.strict != 0;
        const float L32 = bd.L32;
        const int local = c - cb;
        const int cx = local % nc, cy = (local / nc) % nc, cz = local / (nc * nc);
        // the slots of the 27 neighbour cells, one cell per lane (lanes 0-26,
        // neighbour nb = 9 (dz + 1) + 3 (dy + 1) + dx + 1), all looked up at once
        int nb_j0 = 0, nb_j1 = 0;
        if (lane < 27) {
            int nx = cx + lane % 3 - 1, ny = cy + (lane / 3) % 3 - 1, nz = cz + lane / 9 - 1;
            nx += nx < 0 ? nc : (nx >= nc ? -nc : 0);
            ny += ny < 0 ? nc : (ny >= nc ? -nc : 0);
            nz += nz < 0 ? nc : (nz >= nc ? -nc : 0);
            const int2 sp = cell_span(p, cb + (nz * nc + ny) * nc + nx);
            nb_j0 = sp.x;
            nb_j1 = sp.y;
        }
        const int ce = __shfl(nb_j1, 13, 64);   // the cell itself
        const int i = first + lane;
        const bool vi = i < ce;
        const float4 pi = vi ? p.sorted[i] : make_float4(qnan(), qnan(), qnan(), 0.f);
        const bool rnd = kGeneral && p.link_random;
        const int mode = p.find_mode;
        int root_i = vi ? find_root(p.parent, i, mode, rnd) : -1;
        int known0 = -3, known1 = -3;   // never a node
        const double dxi = (double)pi.x, dyi = (double)pi.y, dzi = (double)pi.z;
        const int n_home = min(64, ce - first);

#pragma unroll 1
        for (int nb = 0; nb < 27; ++nb) {
            const int dz = nb / 9 - 1, dy = (nb / 3) % 3 - 1, dx = nb % 3 - 1;
            const bool self = nb == 13;
            const bool upper = nb > 13;
            int nx = cx + dx, ny = cy + dy, nz = cz + dz;
            float hx = pi.x, hy = pi.y, hz = pi.z, sx = 0.f, sy = 0.f, sz = 0.f;
            double Lx = 0.0, Ly = 0.0, Lz = 0.0;
            if (nx < 0) { nx += nc; sx = L32; Lx = br.L; }
            else if (nx >= nc) { nx -= nc; hx = pi.x - L32; Lx = -br.L; }
            if (ny < 0) { ny += nc; sy = L32; Ly = br.L; }
            else if (ny >= nc) { ny -= nc; hy = pi.y - L32; Ly = -br.L; }
            if (nz < 0) { nz += nc; sz = L32; Lz = br.L; }
            else if (nz >= nc) { nz -= nc; hz = pi.z - L32; Lz = -br.L; }
            int j0 = __builtin_amdgcn_readfirstlane(__shfl(nb_j0, nb, 64));
            const int j1 = __builtin_amdgcn_readfirstlane(__shfl(nb_j1, nb, 64));
            if (self) j0 = first;
            else if (!upper && j1 - j0 >= p.dense_min) continue;   // that dense cell searches this pair
#pragma unroll 1
            for (int jb = j0; jb < j1; jb += 64) {
                const int j = jb + lane;
                const bool vj = j < j1;
                const float4 q = vj ? p.sorted[j] : make_float4(qnan(), qnan(), qnan(), 0.f);
                // the home particle's cached root, checked once per neighbour
                // cell (other waves may have merged its group meanwhile)
                const int pr = (!kStats && jb == j0 && vi) ? ld_rel(p.parent + root_i) : root_i;
                const int rj = vj ? find_root(p.parent, j, mode, rnd) : -2;
                if constexpr (!kStats) {
                    if (pr != root_i) root_i = find_root(p.parent, pr, mode, rnd);
                    // a batch whose candidates all have one root that every
                    // home particle knows as its own group needs no test
                    const int r0 = __builtin_amdgcn_readfirstlane(rj);   // lane 0 holds a candidate
                    if (__ballot(vj && rj != r0) == 0 &&
                        __ballot(vi && root_i != r0 && known0 != r0 && known1 != r0) == 0)
                        continue;
                }
                if constexpr (kFP64) {
                    st.x[lane] = (double)q.x;
                    st.y[lane] = (double)q.y;
                    st.z[lane] = (double)q.z;
                    st.root[lane] = rj;
                } else {
                    st.v[lane] = make_float4(q.x - sx, q.y - sy, q.z - sz, __int_as_float(rj));
                }
                __builtin_amdgcn_wave_barrier();
                const int cnt = min(64, j1 - jb);
                if (kStats) tests += (unsigned long long)cnt * (unsigned long long)n_home;
                if (self)
                    dense_batch<kFP64, kStats, kGeneral, true>(p, br, st, cnt, jb, i, vi, pi, hx, hy, hz, dxi, dyi,
                                                               dzi, Lx, Ly, Lz, root_i, known0, known1, links, band,
                                                               retries);
                else
                    dense_batch<kFP64, kStats, kGeneral, false>(p, br, st, cnt, jb, i, vi, pi, hx, hy, hz, dxi, dyi,
                                                                dzi, Lx, Ly, Lz, root_i, known0, known1, links, band,
                                                                retries);
                __builtin_amdgcn_wave_barrier();
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
// cell splits it into k^3 sub-cells whose diagonal is below l_x, so any two
// particles of a sub-cell are linked, and hooks every particle under the
// lowest particle of its sub-cell. The pair search then meets at most k^3
// groups per dense cell instead of one per particle, and its cached roots
// agree far more often. The groups found are unchanged (only linked pairs
// are merged).
constexpr int kMaxSub = 1000;

__global__ void __launch_bounds__(kBlock) k_dense_premerge(Plan p)
{
    __shared__ int rep[kWaves][kMaxSub];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    int *rp = rep[wid];
    unsigned retries = 0;
    const int n_items = (int)p.counters->n_items;
    const XcdRange xr = xcd_range(n_items, kWaves, wid);
    for (int64_t it = xr.first; it < xr.end; it += xr.stride) {
        const int4 item = p.items[it];
        const int c = __builtin_amdgcn_readfirstlane(item.x);
        const int first = __builtin_amdgcn_readfirstlane(item.y);
        const int b = __builtin_amdgcn_readfirstlane(item.z);
        const int2 sp = cell_span(p, c);
        const int cs = __builtin_amdgcn_readfirstlane(sp.x);
        if (first != cs) continue;   // the cell's first item does the whole cell
        const BoxDev &bd = box_of(p, b);
        const int k = bd.sub_k;
        if (k == 0) continue;
        const int ce = __builtin_amdgcn_readfirstlane(sp.y);
        const int nc = bd.nc, local = c - (int)bd.cell_base;
        const int cx = local % nc, cy = (local / nc) % nc, cz = local / (nc * nc);
        const int nsub = k * k * k;
        for (int t = lane; t < nsub; t += 64) rp[t] = INT_MAX;
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
        for (int j = cs + lane; j < ce; j += 64) atomicMin(&rp[sub_of(j)], j);
        __builtin_amdgcn_wave_barrier();
        for (int j = cs + lane; j < ce; j += 64) {
            const int r = rp[sub_of(j)];
            if (r != j) retries += unite(p.parent, j, r, p.link_random, p.find_mode);
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (p.stats) {
        const unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane == 0 && r) atomicAdd(&p.counters->cas_retries, r);
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

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <bool kFP64, bool kStats>
void launch_link_t(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    if (t) t->mark(K_LINK_SPARSE, false, stream);
    hipLaunchKernelGGL((k_link_sparse<kFP64, kStats>), dim3((unsigned)p.sparse_blocks), dim3(kBlock), 0, stream, p);
    if (t) t->mark(K_LINK_SPARSE, true, stream);
    if (t) t->mark(K_UNION_EDGES, false, stream);
    hipLaunchKernelGGL((k_union_edges<kStats>), dim3(kUnionParts * kEdgeSlices), dim3(kBlock), 0, stream, p);
    if (t) t->mark(K_UNION_EDGES, true, stream);
    if (t) t->mark(K_LINK_DENSE, false, stream);
    // the sub-cell pre-merge would merge across slab faces: not in domain mode
    if (p.domains <= 1 && p.premerge)
        hipLaunchKernelGGL(k_dense_premerge, dim3((unsigned)p.dense_blocks), dim3(kBlock), 0, stream, p);
    if (p.domains > 1 || p.link_random)
        hipLaunchKernelGGL((k_link_dense<kFP64, kStats, true>), dim3((unsigned)p.dense_blocks), dim3(kBlock), 0,
                           stream, p);
    else
        hipLaunchKernelGGL((k_link_dense<kFP64, kStats, false>), dim3((unsigned)p.dense_blocks), dim3(kBlock), 0,
                           stream, p);
    if (t) t->mark(K_LINK_DENSE, true, stream);
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
}

}  // namespace

hipError_t launch_link(const Plan &p, hipStream_t stream, KernelTimer *t)
{
    if (p.n == 0) return hipSuccess;
    const bool fp64 = p.predicate == 0;
    if (fp64) {
        if (p.stats) launch_link_t<true, true>(p, stream, t);
        else launch_link_t<true, false>(p, stream, t);
    } else {
        if (p.stats) launch_link_t<false, true>(p, stream, t);
        else launch_link_t<false, false>(p, stream, t);
    }
    return hipGetLastError();
}

int64_t max_dense_items(int64_t n, int dense_min)
{
    const int64_t t = dense_min > 0 ? dense_min : 1;
    return n / 64 + n / t + 64;
}

}  // namespace fof
