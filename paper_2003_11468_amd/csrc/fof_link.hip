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
// grow. Otherwise the lane hooks the larger root under the smaller (CAS).
#include "fof_device.h"

namespace fof {
namespace {

using namespace dev;

constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ float qnan() { return __builtin_nanf(""); }

// Merge the groups that contain roots-or-members a and b; returns a node of the
// merged group (the smaller root at the time of the merge).
__device__ __forceinline__ int unite_root(int *parent, int a, int b, unsigned &retries)
{
    while (true) {
        a = find_halve(parent, a);
        b = find_halve(parent, b);
        if (a == b) return a;
        const int lo = a < b ? a : b;
        const int hi = a < b ? b : a;
        int expected = hi;
        if (__hip_atomic_compare_exchange_strong(parent + hi, &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return lo;
        ++retries;
        a = expected;
        b = lo;
    }
}

// --------------------------------------------------------- sparse (lane) --

// Particle s against the sorted particles [j0, j1). hx/hy/hz: home coordinates
// (minus L on axes where the home cell is the top one); sx/sy/sz: L on axes
// where the neighbour cell is the top one reached through the boundary.
template <bool kFP64, bool kStats>
__device__ __forceinline__ void lane_range(const Plan &p, const BoxDev &bd, int s, float4 pi, int j0, int j1,
                                           float hx, float hy, float hz, float sx, float sy, float sz, double Lx,
                                           double Ly, double Lz, int &root, unsigned long long &tests,
                                           unsigned long long &links, unsigned long long &band, unsigned &retries)
{
    const bool strict = p.strict != 0;
    for (int j = j0; j < j1; ++j) {
        const float4 pj = p.sorted[j];
        bool link;
        if constexpr (kFP64) {
            double tx = ((double)pi.x - (double)pj.x) + Lx;
            double ty = ((double)pi.y - (double)pj.y) + Ly;
            double tz = ((double)pi.z - (double)pj.z) + Lz;
            double sxy = tx * tx + ty * ty;
            double r2 = sxy + tz * tz;
            link = strict ? (r2 < bd.l2) : (r2 <= bd.l2);
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
            root = unite_root(p.parent, root, j, retries);
        }
    }
}

template <bool kFP64, bool kStats>
__global__ void __launch_bounds__(kBlock) k_link_sparse(Plan p)
{
    const int64_t s64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long tests = 0, links = 0, band = 0;
    unsigned retries = 0;
    if (s64 < p.n) {
        const int s = (int)s64;
        const int b = p.n_boxes == 1 ? 0 : find_box(p.box_p0, p.n_boxes, s64);
        const BoxDev &bd = box_of(p, b);
        const float4 pi = p.sorted[s];
        const int nc = bd.nc;
        const int cx = cell_coord(pi.x, bd.inv_h, nc);
        const int cy = cell_coord(pi.y, bd.inv_h, nc);
        const int cz = cell_coord(pi.z, bd.inv_h, nc);
        const int cb = (int)bd.cell_base;
        const int c = cb + (cz * nc + cy) * nc + cx;
        const int *cell = p.cell;
        const int dense_min = p.dense_min;
        // The 13 half-shell cells lie in 5 rows of x-consecutive cells: the own
        // row (cell cx + 1) and the rows (dy, dz) = (1, 0), (-1, 1), (0, 1),
        // (1, 1) (cells cx - 1, cx, cx + 1). Away from the x faces one 16-byte
        // load per row returns the four boundaries of its three cells; all
        // rows are requested before any candidate is read.
        int j0[13], j1[13];
        const int own_start = cell[c];
        const int own_end = cell[c + 1];
        const bool inner = cx >= 1 && cx + 1 < nc;   // boundaries cx-1 .. cx+2 lie in the row (cx+2 may be the next row's start = end of this row)
        {
            const int nxp = cx + 1 < nc ? cx + 1 : 0;
            const int rb0 = c - cx;
            j0[0] = cell[rb0 + nxp];
            j1[0] = cell[rb0 + nxp + 1];
        }
        const int rdy[4] = {1, -1, 0, 1}, rdz[4] = {0, 1, 1, 1};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int ny = cy + rdy[r], nz = cz + rdz[r];
            ny += ny < 0 ? nc : (ny >= nc ? -nc : 0);
            nz += nz >= nc ? -nc : 0;
            const int rb = cb + (nz * nc + ny) * nc;
            if (inner) {
                typedef int int4a4 __attribute__((ext_vector_type(4), aligned(4)));
                const int4a4 q = *reinterpret_cast<const int4a4 *>(cell + rb + cx - 1);
                j0[1 + 3 * r] = q.x; j1[1 + 3 * r] = q.y;
                j0[2 + 3 * r] = q.y; j1[2 + 3 * r] = q.z;
                j0[3 + 3 * r] = q.z; j1[3 + 3 * r] = q.w;
            } else {
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    int nx = cx - 1 + e;
                    nx += nx < 0 ? nc : (nx >= nc ? -nc : 0);
                    j0[1 + 3 * r + e] = cell[rb + nx];
                    j1[1 + 3 * r + e] = cell[rb + nx + 1];
                }
            }
        }
        // neighbour k: offset (dx, dy, dz) of slot k in the table above
        const int kdx[13] = {1, -1, 0, 1, -1, 0, 1, -1, 0, 1, -1, 0, 1};
        const int kdy[13] = {0, 1, 1, 1, -1, -1, -1, 0, 0, 0, 1, 1, 1};
        const int kdz[13] = {0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1};
        if (own_end - own_start < dense_min) {
            const float L32 = bd.L32;
            const double L = bd.L;
            int root = s;
            lane_range<kFP64, kStats>(p, bd, s, pi, s + 1, own_end, pi.x, pi.y, pi.z, 0.f, 0.f, 0.f, 0.0, 0.0, 0.0,
                                      root, tests, links, band, retries);
#pragma unroll 1
            for (int k = 0; k < 13; ++k) {
                if (j1[k] - j0[k] >= dense_min || j1[k] == j0[k]) continue;   // dense: that cell searches the pair
                const int dx = kdx[k], dy = kdy[k], dz = kdz[k];
                float hx = pi.x, hy = pi.y, hz = pi.z, sx = 0.f, sy = 0.f, sz = 0.f;
                double Lx = 0.0, Ly = 0.0, Lz = 0.0;
                if (cx + dx < 0) { sx = L32; Lx = L; }
                else if (cx + dx >= nc) { hx = pi.x - L32; Lx = -L; }
                if (cy + dy < 0) { sy = L32; Ly = L; }
                else if (cy + dy >= nc) { hy = pi.y - L32; Ly = -L; }
                if (cz + dz >= nc) { hz = pi.z - L32; Lz = -L; }
                lane_range<kFP64, kStats>(p, bd, s, pi, j0[k], j1[k], hx, hy, hz, sx, sy, sz, Lx, Ly, Lz, root,
                                          tests, links, band, retries);
            }
        }
    }
    if (kStats) {
        tests = wave_sum_u64(tests);
        links = wave_sum_u64(links);
        band = wave_sum_u64(band);
        unsigned long long r = wave_sum_u64((unsigned long long)retries);
        if (lane_id() == 0) {
            atomicAdd(&p.counters->pair_tests, tests);
            atomicAdd(&p.counters->links, links);
            atomicAdd(&p.counters->band_hits, band);
            atomicAdd(&p.counters->cas_retries, r);
        }
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
// the original coordinates; a link merges the groups unless the cached roots
// already agree.
template <bool kFP64, bool kStats>
__device__ __forceinline__ void dense_hit(const Plan &p, const BoxRegs &br, const typename Stage<kFP64>::T &st,
                                          int kk, int jb, bool cand, float r, float4 pi, int &root_i,
                                          unsigned long long &links, unsigned long long &band, unsigned &retries)
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
        if (rj != root_i) root_i = unite_root(p.parent, root_i, rj, retries);
    }
}

// FP32 squared distance of the home lane to staged candidate kk.
__device__ __forceinline__ float dist2_f32(const StageF &st, int kk, float hx, float hy, float hz)
{
    const float4 cj = st.v[kk];
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
// kSelf: the candidates come from the home cell; only j > i counts.
template <bool kFP64, bool kStats, bool kSelf>
__device__ __forceinline__ void dense_batch(const Plan &p, const BoxRegs &br, const typename Stage<kFP64>::T &st,
                                            int cnt, int jb, int i, bool vi, float4 pi, float hx, float hy,
                                            float hz, double dxi, double dyi, double dzi, double Lx, double Ly,
                                            double Lz, int &root_i, unsigned long long &links,
                                            unsigned long long &band, unsigned &retries)
{
    const int rel = i - jb;   // candidate kk is above the home particle iff kk > rel
    int kk = 0;
    if constexpr (!kFP64) {
        for (; kk + 4 <= cnt; kk += 4) {
            const float r0 = dist2_f32(st, kk + 0, hx, hy, hz);
            const float r1 = dist2_f32(st, kk + 1, hx, hy, hz);
            const float r2 = dist2_f32(st, kk + 2, hx, hy, hz);
            const float r3 = dist2_f32(st, kk + 3, hx, hy, hz);
            bool c0 = r0 <= br.hi32, c1 = r1 <= br.hi32, c2 = r2 <= br.hi32, c3 = r3 <= br.hi32;
            if constexpr (kSelf) {
                c0 = c0 && kk + 0 > rel;
                c1 = c1 && kk + 1 > rel;
                c2 = c2 && kk + 2 > rel;
                c3 = c3 && kk + 3 > rel;
            }
            if (__ballot(c0 || c1 || c2 || c3)) {
                dense_hit<kFP64, kStats>(p, br, st, kk + 0, jb, c0, r0, pi, root_i, links, band, retries);
                dense_hit<kFP64, kStats>(p, br, st, kk + 1, jb, c1, r1, pi, root_i, links, band, retries);
                dense_hit<kFP64, kStats>(p, br, st, kk + 2, jb, c2, r2, pi, root_i, links, band, retries);
                dense_hit<kFP64, kStats>(p, br, st, kk + 3, jb, c3, r3, pi, root_i, links, band, retries);
            }
        }
    }
    for (; kk < cnt; ++kk) {
        bool c;
        float r = 0.f;
        if constexpr (kFP64) {
            c = vi && link_f64_staged(st, kk, dxi, dyi, dzi, Lx, Ly, Lz, br);
        } else {
            r = dist2_f32(st, kk, hx, hy, hz);
            c = r <= br.hi32;   // false for invalid (NaN) lanes and candidates
        }
        if constexpr (kSelf) c = c && kk > rel;
        if (__ballot(c)) dense_hit<kFP64, kStats>(p, br, st, kk, jb, c, r, pi, root_i, links, band, retries);
    }
}

template <bool kFP64, bool kStats>
__global__ void __launch_bounds__(kBlock) k_link_dense(Plan p)
{
    using StageT = typename Stage<kFP64>::T;
    __shared__ StageT stage[kWaves];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    StageT &st = stage[wid];
    unsigned long long tests = 0, links = 0, band = 0;
    unsigned retries = 0;
    const int n_items = (int)p.counters->n_items;
    const int stride = (int)gridDim.x * kWaves;

    for (int it = (int)blockIdx.x * kWaves + wid; it < n_items; it += stride) {
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
        const int ce = __builtin_amdgcn_readfirstlane(p.cell[c + 1]);
        const int i = first + lane;
        const bool vi = i < ce;
        const float4 pi = vi ? p.sorted[i] : make_float4(qnan(), qnan(), qnan(), 0.f);
        int root_i = vi ? find_halve(p.parent, i) : -1;
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
            const int c2 = cb + (nz * nc + ny) * nc + nx;
            int j0 = __builtin_amdgcn_readfirstlane(p.cell[c2]);
            const int j1 = __builtin_amdgcn_readfirstlane(p.cell[c2 + 1]);
            if (self) j0 = first;
            else if (!upper && j1 - j0 >= p.dense_min) continue;   // that dense cell searches this pair
#pragma unroll 1
            for (int jb = j0; jb < j1; jb += 64) {
                const int j = jb + lane;
                const bool vj = j < j1;
                const float4 q = vj ? p.sorted[j] : make_float4(qnan(), qnan(), qnan(), 0.f);
                const int rj = vj ? find_halve(p.parent, j) : -2;
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
                    dense_batch<kFP64, kStats, true>(p, br, st, cnt, jb, i, vi, pi, hx, hy, hz, dxi, dyi, dzi, Lx,
                                                     Ly, Lz, root_i, links, band, retries);
                else
                    dense_batch<kFP64, kStats, false>(p, br, st, cnt, jb, i, vi, pi, hx, hy, hz, dxi, dyi, dzi,
                                                      Lx, Ly, Lz, root_i, links, band, retries);
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

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <bool kFP64, bool kStats>
void launch_link_t(const Plan &p, hipStream_t stream)
{
    hipLaunchKernelGGL((k_link_sparse<kFP64, kStats>), dim3(grid_for(p.n)), dim3(kBlock), 0, stream, p);
    hipLaunchKernelGGL((k_link_dense<kFP64, kStats>), dim3((unsigned)p.dense_blocks), dim3(kBlock), 0, stream, p);
}

}  // namespace

hipError_t launch_link(const Plan &p, hipStream_t stream)
{
    if (p.n == 0) return hipSuccess;
    const bool fp64 = p.predicate == 0;
    if (fp64) {
        if (p.stats) launch_link_t<true, true>(p, stream);
        else launch_link_t<true, false>(p, stream);
    } else {
        if (p.stats) launch_link_t<false, true>(p, stream);
        else launch_link_t<false, false>(p, stream);
    }
    return hipGetLastError();
}

int64_t max_dense_items(int64_t n, int dense_min)
{
    const int64_t t = dense_min > 0 ? dense_min : 1;
    return n / 64 + n / t + 64;
}

}  // namespace fof
