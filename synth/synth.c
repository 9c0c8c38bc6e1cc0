/*
 * Seeded synthetic particle sets shaped like N-body snapshots.
 *
 * This module only produces inputs. It holds none of the Friends-of-Friends
 * arithmetic (no distances, no cells, no union-find), so both the GPU path and
 * the CPU oracle can be fed from it without sharing any of the method's code.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), a counter-based generator. Every draw
 * is addressed by (key = {seed, stream}, counter = {index lo, index hi, tag, 0}),
 * so any particle can be generated independently of every other one and the
 * output does not depend on the number of threads.
 *
 * Shuffle: particles are generated in a natural order (halo by halo, then the
 * uniform background) and written to out[pi(k)], where pi is a keyed bijection
 * of [0, n): a 4-round Feistel network on the smallest even bit width that
 * covers n, with cycle walking back into [0, n). The shuffle makes the
 * minimum-index group labels non-trivial.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { TAG_HALO_MASS = 1, TAG_HALO_CENTRE = 2, TAG_HALO_PART = 3, TAG_BACKGROUND = 4,
       TAG_PERMUTE = 5, TAG_BOX_SIZE = 6, TAG_LATTICE = 7 };

/* Philox4x32-10: ten rounds of the S-box below, with the Weyl key schedule. */
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(uint32_t seed, uint32_t stream, uint64_t index, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), tag, 0u};
    uint32_t key[2] = {seed, stream};
    philox4x32_10(ctr, key, out);
}

/* 24-bit uniform on [0, 1): exact in FP32. */
static double u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }
/* 24-bit uniform on (0, 1]. */
static double u24_open0(uint32_t w) { return (double)((w >> 8) + 1u) * (1.0 / 16777216.0); }
/* 53-bit uniform on [0, 1) from two words. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t v = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return (double)v * (1.0 / 9007199254740992.0);
}

/* Wrap a double coordinate into [0, L) and round it to FP32; a value that
 * rounds up to L becomes 0. */
static float wrap_to_f32(double x, double L)
{
    x = x - L * floor(x / L);
    float f = (float)x;
    if (!(f < (float)L) || f < 0.0f) f = 0.0f;
    return f;
}

/* ---------------------------------------------------------------- shuffle -- */

typedef struct {
    uint64_t n;
    uint32_t half_bits;
    uint64_t half_mask;
    uint32_t seed, stream;
} perm_t;

static void perm_init(perm_t *p, uint64_t n, uint32_t seed, uint32_t stream)
{
    uint32_t bits = 2;
    while (bits < 62 && (1ull << bits) < n) bits += 2;
    p->n = n;
    p->half_bits = bits / 2;
    p->half_mask = (1ull << p->half_bits) - 1ull;
    p->seed = seed;
    p->stream = stream;
}

static uint64_t feistel(const perm_t *p, uint64_t x)
{
    uint64_t l = x >> p->half_bits, r = x & p->half_mask;
    for (uint32_t round = 0; round < 4; ++round) {
        uint32_t w[4];
        uint32_t ctr[4] = {(uint32_t)r, (uint32_t)(r >> 32), TAG_PERMUTE, round};
        uint32_t key[2] = {p->seed, p->stream};
        philox4x32_10(ctr, key, w);
        uint64_t f = (((uint64_t)w[1] << 32) | w[0]) & p->half_mask;
        uint64_t nl = r, nr = l ^ f;
        l = nl;
        r = nr;
    }
    return (l << p->half_bits) | r;
}

static uint64_t perm_apply(const perm_t *p, uint64_t k)
{
    uint64_t y = feistel(p, k);
    while (y >= p->n) y = feistel(p, y);
    return y;
}

/* ------------------------------------------------------------ public API -- */

void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    philox4x32_10(ctr, key, out);
}

uint64_t synth_permute(uint64_t n, uint32_t seed, uint32_t stream, uint64_t k)
{
    perm_t p;
    perm_init(&p, n, seed, stream);
    return perm_apply(&p, k);
}

/* n i.i.d. uniform points in [0, L)^3 (in generation order: already random). */
void synth_uniform(int64_t n, double L, uint32_t seed, uint32_t stream, float *pos)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        uint32_t w[4];
        draw4(seed, stream, (uint64_t)k, TAG_BACKGROUND, w);
        pos[3 * k + 0] = wrap_to_f32(u24(w[0]) * L, L);
        pos[3 * k + 1] = wrap_to_f32(u24(w[1]) * L, L);
        pos[3 * k + 2] = wrap_to_f32(u24(w[2]) * L, L);
    }
}

/* Halo particle counts: power law dN/dM ~ M^-slope on [m_min, m_max] by
 * inverse CDF, rounded to the nearest integer, the last one clipped so the
 * counts sum to exactly `budget`. Returns the number of halos written, or -1
 * if max_halos is too small. */
int64_t synth_halo_counts(int64_t budget, double m_min, double m_max, double slope,
                          uint32_t seed, uint32_t stream, int64_t *counts, int64_t max_halos)
{
    const double e = 1.0 - slope;
    const double a = pow(m_min, e), b = pow(m_max, e);
    int64_t used = 0, h = 0;
    while (used < budget) {
        if (h >= max_halos) return -1;
        uint32_t w[4];
        draw4(seed, stream, (uint64_t)h, TAG_HALO_MASS, w);
        double u = u53(w[0], w[1]);
        double m = pow(a + u * (b - a), 1.0 / e);
        int64_t c = (int64_t)floor(m + 0.5);
        if (c < 1) c = 1;
        if (c > budget - used) c = budget - used;
        counts[h++] = c;
        used += c;
    }
    return h;
}

/* Clustered snapshot: a fraction `halo_frac` of the n particles sit in
 * spherical Plummer halos (counts from synth_halo_counts, scale radius
 * a = 0.005 L (M/1000)^(1/3), radius r = a (u^(-2/3) - 1)^(-1/2) with the
 * enclosed-mass fraction u uniform on (0, 0.999], isotropic directions,
 * centres uniform in the box); the rest is uniform background. The result is
 * shuffled. `counts` / `n_halos` come from synth_halo_counts. */
void synth_clustered(int64_t n, double L, const int64_t *counts, int64_t n_halos,
                     uint32_t seed, uint32_t stream, float *pos)
{
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_halos + 1));
    double *centre = (double *)malloc(sizeof(double) * 3 * (size_t)(n_halos > 0 ? n_halos : 1));
    double *scale = (double *)malloc(sizeof(double) * (size_t)(n_halos > 0 ? n_halos : 1));
    start[0] = 0;
    for (int64_t h = 0; h < n_halos; ++h) {
        start[h + 1] = start[h] + counts[h];
        uint32_t w[4];
        draw4(seed, stream, (uint64_t)h, TAG_HALO_CENTRE, w);
        centre[3 * h + 0] = u24(w[0]) * L;
        centre[3 * h + 1] = u24(w[1]) * L;
        centre[3 * h + 2] = u24(w[2]) * L;
        scale[h] = 0.005 * L * cbrt((double)counts[h] / 1000.0);
    }
    const int64_t n_halo_parts = start[n_halos];
    perm_t perm;
    perm_init(&perm, (uint64_t)n, seed, stream);
    const double two_pi = 6.283185307179586476925286766559;

#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        uint32_t w[4];
        double x, y, z;
        if (k < n_halo_parts) {
            int64_t lo = 0, hi = n_halos - 1; /* halo h with start[h] <= k < start[h+1] */
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (start[mid] <= k) lo = mid; else hi = mid - 1;
            }
            draw4(seed, stream, (uint64_t)k, TAG_HALO_PART, w);
            double u = 0.999 * u24_open0(w[0]);
            double r = scale[lo] / sqrt(pow(u, -2.0 / 3.0) - 1.0);
            double ct = 2.0 * ((double)(w[1] >> 8) + 0.5) * (1.0 / 16777216.0) - 1.0;
            double st = sqrt(1.0 - ct * ct);
            double ph = two_pi * u24(w[2]);
            x = centre[3 * lo + 0] + r * st * cos(ph);
            y = centre[3 * lo + 1] + r * st * sin(ph);
            z = centre[3 * lo + 2] + r * ct;
        } else {
            draw4(seed, stream, (uint64_t)k, TAG_BACKGROUND, w);
            x = u24(w[0]) * L;
            y = u24(w[1]) * L;
            z = u24(w[2]) * L;
        }
        uint64_t dst = perm_apply(&perm, (uint64_t)k);
        pos[3 * dst + 0] = wrap_to_f32(x, L);
        pos[3 * dst + 1] = wrap_to_f32(y, L);
        pos[3 * dst + 2] = wrap_to_f32(z, L);
    }
    free(start);
    free(centre);
    free(scale);
}

/* A jittered cubic lattice: side^3 sites of spacing s = L / side, site
 * (i, j, k) at ((i + 1/2 + d_x) s, (j + 1/2 + d_y) s, (k + 1/2 + d_z) s) with
 * each d uniform on [-jitter, jitter), stored in shuffled order. */
void synth_lattice(int64_t side, double L, double jitter, uint32_t seed, uint32_t stream, float *pos)
{
    const int64_t n = side * side * side;
    const double s = L / (double)side;
    perm_t perm;
    perm_init(&perm, (uint64_t)n, seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        uint32_t w[4];
        draw4(seed, stream, (uint64_t)k, TAG_LATTICE, w);
        const double i = (double)(k % side), j = (double)((k / side) % side), l = (double)(k / (side * side));
        const double x = (i + 0.5 + jitter * (2.0 * u24(w[0]) - 1.0)) * s;
        const double y = (j + 0.5 + jitter * (2.0 * u24(w[1]) - 1.0)) * s;
        const double z = (l + 0.5 + jitter * (2.0 * u24(w[2]) - 1.0)) * s;
        uint64_t dst = perm_apply(&perm, (uint64_t)k);
        pos[3 * dst + 0] = wrap_to_f32(x, L);
        pos[3 * dst + 1] = wrap_to_f32(y, L);
        pos[3 * dst + 2] = wrap_to_f32(z, L);
    }
}

/* Box particle counts for the batched workload: round(exp(U[ln lo, ln hi])). */
void synth_box_sizes(int32_t n_boxes, double lo, double hi, uint32_t seed, int64_t *sizes)
{
    for (int32_t b = 0; b < n_boxes; ++b) {
        uint32_t w[4];
        draw4(seed, 0xB0B0u, (uint64_t)b, TAG_BOX_SIZE, w);
        double u = u53(w[0], w[1]);
        sizes[b] = (int64_t)floor(exp(log(lo) + u * (log(hi) - log(lo))) + 0.5);
    }
}
