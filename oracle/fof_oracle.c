/*
 * CPU oracle for periodic Friends-of-Friends labelling.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct
 * reference that the GPU library is checked against. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction, IEEE
 * double arithmetic with round-to-nearest, no x87 on x86-64).
 *
 * What is computed (paper, Section 1 footnote): the connected components of
 * the graph G = (P, E) whose edges join two particles at distance at most l_x.
 * Representation (paper, Section 2 and Section 3.1): a union-find forest in an
 * array whose entries start as the particle's own offset; a union makes the
 * larger root point to the smaller, so every root is the minimum index of its
 * set and the labels depend only on the partition. Group sizes (Section 3.4.1)
 * are counted at the root.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - distance: periodic minimum image, per axis t = a - b then t -= L if
 *    t > L/2, t += L if t < -L/2; r2 = (tx*tx + ty*ty) + tz*tz in that order,
 *    each operation rounded to nearest in double, no FMA; FP32 inputs are
 *    promoted exactly to double.
 *  - link iff r2 <= l2 with l2 = l_x * l_x rounded once (the footnote's
 *    "at most"); `strict` selects r2 < l2 (Listing 1's comparison).
 *  - r2 is compared with l2 (no square root).
 *  - labels: minimum 0-based input index of the component; size[r] is the
 *    component size at roots (label[r] == r) and 0 elsewhere.
 *  - inputs must be finite and inside [0, L); anything else is an error.
 *
 * Neighbour search (paper, Section 3.1: only nearby cells are searched, and
 * cells matching the linking length work best): a Hockney-Eastwood
 * head/next linked cell list with n_c cells per axis, side L/n_c at least
 * l_x (1 + 2^-20), all 27 cells of the periodic shell, each unordered pair
 * visited from its lower index. If fewer than 3 cells fit per axis the
 * brute-force all-pairs loop (Listing 1) is used instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORACLE_OK = 0,
    ORACLE_ERR_N = -1,
    ORACLE_ERR_BOX = -2,
    ORACLE_ERR_LX = -3,
    ORACLE_ERR_COORD = -4,
    ORACLE_ERR_MEM = -5
};

/* ------------------------------------------------------------ predicate -- */

static double wrap_axis(double t, double L, double half)
{
    if (t > half) return t - L;
    if (t < -half) return t + L;
    return t;
}

/* Squared minimum-image distance of two FP32 points, in double. */
double oracle_r2(const float *a, const float *b, double L)
{
    const double half = 0.5 * L;
    double tx = wrap_axis((double)a[0] - (double)b[0], L, half);
    double ty = wrap_axis((double)a[1] - (double)b[1], L, half);
    double tz = wrap_axis((double)a[2] - (double)b[2], L, half);
    double sxy = tx * tx + ty * ty;
    return sxy + tz * tz;
}

static int linked(const float *a, const float *b, double L, double l2, int strict)
{
    double r2 = oracle_r2(a, b, L);
    return strict ? (r2 < l2) : (r2 <= l2);
}

/* ----------------------------------------------------------- union-find -- */

static int32_t find_root(int32_t *parent, int32_t x)
{
    int32_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) { /* full path compression */
        int32_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

static void unite(int32_t *parent, int32_t a, int32_t b)
{
    int32_t ra = find_root(parent, a), rb = find_root(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra; /* the larger root points to the smaller */
    else parent[ra] = rb;
}

/* Labels and sizes from a finished forest. Returns the number of groups. */
static int64_t emit(int32_t *parent, int64_t n, int32_t *label, int32_t *size)
{
    int64_t groups = 0;
    for (int64_t i = 0; i < n; ++i) size[i] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t r = find_root(parent, (int32_t)i);
        label[i] = r;
        size[r] += 1;
        if (r == i) ++groups;
    }
    return groups;
}

static int validate(int64_t n, const float *pos, double L, double lx)
{
    if (n < 0 || n > INT32_MAX) return ORACLE_ERR_N;
    if (!(L > 0.0) || !isfinite(L)) return ORACLE_ERR_BOX;
    if (!(lx > 0.0) || !isfinite(lx)) return ORACLE_ERR_LX;
    for (int64_t i = 0; i < 3 * n; ++i) {
        double x = (double)pos[i];
        if (!isfinite(x) || x < 0.0 || x >= L) return ORACLE_ERR_COORD;
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------- brute force -- */

/* Listing 1 of the paper, every unordered pair once. O(n^2). */
int oracle_fof_brute(int64_t n, const float *pos, double L, double lx, int strict,
                     int32_t *label, int32_t *size, int64_t *n_groups)
{
    int st = validate(n, pos, L, lx);
    if (st) return st;
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!parent) return ORACLE_ERR_MEM;
    const double l2 = lx * lx;
    for (int64_t i = 0; i < n; ++i) parent[i] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            if (linked(pos + 3 * i, pos + 3 * j, L, l2, strict)) unite(parent, (int32_t)i, (int32_t)j);
    *n_groups = emit(parent, n, label, size);
    free(parent);
    return ORACLE_OK;
}

/* ------------------------------------------------------------ cell list -- */

/* Cells per axis: as many as fit with side >= l_x (1 + 2^-20), but no more
 * than about one per particle. Returns 0 when fewer than 3 fit. */
int64_t oracle_cells_per_axis(int64_t n, double L, double lx)
{
    double fit = floor(L / (lx * (1.0 + 1.0 / 1048576.0)));
    if (!(fit >= 3.0)) return 0;
    double cap = floor(cbrt((double)(n > 27 ? n : 27)) + 1e-9);
    if (cap < 3.0) cap = 3.0;
    if (cap > 1290.0) cap = 1290.0; /* head array below 2^31 cells */
    return (int64_t)(fit < cap ? fit : cap);
}

static int64_t cell_of(double x, int64_t nc, double L)
{
    int64_t c = (int64_t)floor(x * (double)nc / L);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

int oracle_fof(int64_t n, const float *pos, double L, double lx, int strict,
               int32_t *label, int32_t *size, int64_t *n_groups)
{
    int st = validate(n, pos, L, lx);
    if (st) return st;
    const int64_t nc = oracle_cells_per_axis(n, L, lx);
    if (nc == 0) return oracle_fof_brute(n, pos, L, lx, strict, label, size, n_groups);

    const int64_t ncell = nc * nc * nc;
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!head || !next || !parent) {
        free(head); free(next); free(parent);
        return ORACLE_ERR_MEM;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_of(pos[3 * i + 0], nc, L);
        int64_t cy = cell_of(pos[3 * i + 1], nc, L);
        int64_t cz = cell_of(pos[3 * i + 2], nc, L);
        int64_t c = (cz * nc + cy) * nc + cx;
        next[i] = head[c];
        head[c] = (int32_t)i;
        parent[i] = (int32_t)i;
    }

    const double l2 = lx * lx;
    for (int64_t cz = 0; cz < nc; ++cz)
        for (int64_t cy = 0; cy < nc; ++cy)
            for (int64_t cx = 0; cx < nc; ++cx)
                for (int32_t i = head[(cz * nc + cy) * nc + cx]; i >= 0; i = next[i])
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                int64_t ox = (cx + dx + nc) % nc, oy = (cy + dy + nc) % nc,
                                        oz = (cz + dz + nc) % nc;
                                for (int32_t j = head[(oz * nc + oy) * nc + ox]; j >= 0; j = next[j])
                                    if (j > i && linked(pos + 3 * (int64_t)i, pos + 3 * (int64_t)j, L, l2, strict))
                                        unite(parent, i, j);
                            }
    *n_groups = emit(parent, n, label, size);
    free(head); free(next); free(parent);
    return ORACLE_OK;
}

/* Many independent boxes: box k is particles offsets[k]..offsets[k+1]-1 with
 * its own side and linking length; labels are box-local indices. Boxes are
 * independent, so `threads` > 1 runs one box per thread (each box is still the
 * sequential algorithm above). */
int oracle_fof_boxes(int32_t n_boxes, const int64_t *offsets, const float *pos, const double *L,
                     const double *lx, int strict, int32_t *label, int32_t *size, int64_t *n_groups,
                     int threads)
{
    int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
    for (int32_t k = 0; k < n_boxes; ++k) {
        int64_t o = offsets[k];
        int st = oracle_fof(offsets[k + 1] - o, pos + 3 * o, L[k], lx[k], strict, label + o, size + o,
                            n_groups + k);
        if (st) {
#pragma omp critical
            status = st;
        }
    }
    return status;
}

/* ----------------------------------------------- one component, by BFS -- */

/* Breadth-first search of the component that contains `start`, over the same
 * link predicate, using a cell list built here. Writes the members (sorted
 * ascending) to `members` (capacity `cap`) and returns their count, or a
 * negative status. Used to check single groups of inputs too large for the
 * full oracle. */
int64_t oracle_component(int64_t n, const float *pos, double L, double lx, int strict, int64_t start,
                         int32_t *members, int64_t cap)
{
    int st = validate(n, pos, L, lx);
    if (st) return st;
    if (start < 0 || start >= n) return ORACLE_ERR_N;
    const double l2 = lx * lx;
    const int64_t nc = oracle_cells_per_axis(n, L, lx);
    int64_t count = 0;
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!seen || !queue) { free(seen); free(queue); return ORACLE_ERR_MEM; }
    int64_t qh = 0, qt = 0;
    queue[qt++] = (int32_t)start;
    seen[start] = 1;
    if (nc == 0) {
        while (qh < qt) {
            int32_t i = queue[qh++];
            for (int64_t j = 0; j < n; ++j)
                if (!seen[j] && linked(pos + 3 * (int64_t)i, pos + 3 * j, L, l2, strict)) {
                    seen[j] = 1;
                    queue[qt++] = (int32_t)j;
                }
        }
    } else {
        const int64_t ncell = nc * nc * nc;
        int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
        int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!head || !next) { free(head); free(next); free(seen); free(queue); return ORACLE_ERR_MEM; }
        for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = (cell_of(pos[3 * i + 2], nc, L) * nc + cell_of(pos[3 * i + 1], nc, L)) * nc +
                        cell_of(pos[3 * i + 0], nc, L);
            next[i] = head[c];
            head[c] = (int32_t)i;
        }
        while (qh < qt) {
            int64_t i = queue[qh++];
            int64_t cx = cell_of(pos[3 * i + 0], nc, L), cy = cell_of(pos[3 * i + 1], nc, L),
                    cz = cell_of(pos[3 * i + 2], nc, L);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t ox = (cx + dx + nc) % nc, oy = (cy + dy + nc) % nc, oz = (cz + dz + nc) % nc;
                        for (int64_t j = head[(oz * nc + oy) * nc + ox]; j >= 0; j = next[j])
                            if (!seen[j] && linked(pos + 3 * i, pos + 3 * j, L, l2, strict)) {
                                seen[j] = 1;
                                queue[qt++] = (int32_t)j;
                            }
                    }
        }
        free(head);
        free(next);
    }
    for (int64_t i = 0; i < n; ++i)
        if (seen[i]) {
            if (count < cap) members[count] = (int32_t)i;
            ++count;
        }
    free(seen);
    free(queue);
    return count;
}

/* Breadth-first search from several start particles over one cell list. For
 * start k: sizes[k] = size of its group, mins[k] = smallest index in it;
 * mark[i] = k for the members found from start k (-1 elsewhere). A start that
 * lies in a group already searched from an earlier start k' gets the sizes
 * and minimum of k' and leaves mark untouched. Returns 0 or a negative status. */
int oracle_components_of(int64_t n, const float *pos, double L, double lx, int strict, const int64_t *starts,
                         int32_t k, int32_t *mark, int64_t *sizes, int32_t *mins)
{
    int st = validate(n, pos, L, lx);
    if (st) return st;
    const double l2 = lx * lx;
    const int64_t nc = oracle_cells_per_axis(n, L, lx);
    int32_t *head = NULL, *next = NULL;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return ORACLE_ERR_MEM;
    for (int64_t i = 0; i < n; ++i) mark[i] = -1;
    if (nc > 0) {
        const int64_t ncell = nc * nc * nc;
        head = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
        next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!head || !next) { free(head); free(next); free(queue); return ORACLE_ERR_MEM; }
        for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = (cell_of(pos[3 * i + 2], nc, L) * nc + cell_of(pos[3 * i + 1], nc, L)) * nc +
                        cell_of(pos[3 * i + 0], nc, L);
            next[i] = head[c];
            head[c] = (int32_t)i;
        }
    }
    for (int32_t s = 0; s < k; ++s) {
        const int64_t start = starts[s];
        if (start < 0 || start >= n) { free(head); free(next); free(queue); return ORACLE_ERR_N; }
        if (mark[start] >= 0) {
            sizes[s] = sizes[mark[start]];
            mins[s] = mins[mark[start]];
            continue;
        }
        int64_t qh = 0, qt = 0;
        int32_t lo = (int32_t)start;
        queue[qt++] = (int32_t)start;
        mark[start] = s;
        while (qh < qt) {
            const int64_t i = queue[qh++];
            if (i < lo) lo = (int32_t)i;
            if (nc == 0) {
                for (int64_t j = 0; j < n; ++j)
                    if (mark[j] < 0 && linked(pos + 3 * i, pos + 3 * j, L, l2, strict)) {
                        mark[j] = s;
                        queue[qt++] = (int32_t)j;
                    }
                continue;
            }
            const int64_t cx = cell_of(pos[3 * i + 0], nc, L), cy = cell_of(pos[3 * i + 1], nc, L),
                          cz = cell_of(pos[3 * i + 2], nc, L);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t ox = (cx + dx + nc) % nc, oy = (cy + dy + nc) % nc, oz = (cz + dz + nc) % nc;
                        for (int64_t j = head[(oz * nc + oy) * nc + ox]; j >= 0; j = next[j])
                            if (mark[j] < 0 && linked(pos + 3 * i, pos + 3 * j, L, l2, strict)) {
                                mark[j] = s;
                                queue[qt++] = (int32_t)j;
                            }
                    }
        }
        sizes[s] = qt;
        mins[s] = lo;
    }
    free(head);
    free(next);
    free(queue);
    return ORACLE_OK;
}

/* ------------------------------------- the same result over host threads -- */

/* A growing list of linked pairs (slot pairs, see below). */
typedef struct {
    int32_t *pair;
    int64_t count, cap;
} link_list;

static int link_push(link_list *l, int32_t a, int32_t b)
{
    if (l->count == l->cap) {
        int64_t cap = l->cap ? 2 * l->cap : 4096;
        int32_t *p = (int32_t *)realloc(l->pair, sizeof(int32_t) * 2 * (size_t)cap);
        if (!p) return ORACLE_ERR_MEM;
        l->pair = p;
        l->cap = cap;
    }
    l->pair[2 * l->count] = a;
    l->pair[2 * l->count + 1] = b;
    l->count += 1;
    return ORACLE_OK;
}

/* oracle_fof for inputs of up to ~10^9 particles, where one thread would take
 * hours: the same graph, the same components and the same outputs, with the
 * distance tests spread over `threads` host threads. The steps:
 *  1. cells of side L/n_c >= l_x (1 + 2^-20), as many per axis as fit but
 *     at most 1290 (n_c^3 < 2^31): finer than oracle_fof's, which are capped
 *     at about one particle per cell, since here the slots make empty cells
 *     cheap; brute force (through oracle_fof) when fewer than 3 fit;
 *  2. the particles grouped by cell into "slots": the particle count of every
 *     cell, a prefix sum over the cells, and each particle takes the next
 *     free slot of its cell (their order inside a cell is arbitrary). Only
 *     memory locality differs from the head/next list: the slots of a cell
 *     are contiguous;
 *  3. for every particle i, every particle j of the 27 cells of its periodic
 *     shell with input index j > i is tested with the canonical predicate
 *     (each unordered pair once); the cells of each z-plane are searched by
 *     one thread, which keeps that plane's linked pairs, as slot pairs, in a
 *     list of its own;
 *  4. union-find over the slot pairs, one thread, plane by plane (union by the
 *     smaller root, full path compression, as in oracle_fof);
 *  5. outputs: label = the smallest input index of the component, size at the
 *     particle with that index, the number of components.
 * The link set is the graph's edge set whatever the order inside cells and
 * the thread count, and the outputs depend only on its components. */
int oracle_fof_parallel(int64_t n, const float *pos, double L, double lx, int strict,
                        int32_t *label, int32_t *size, int64_t *n_groups, int threads)
{
    int st = validate(n, pos, L, lx);
    if (st) return st;
    const double fit = floor(L / (lx * (1.0 + 1.0 / 1048576.0)));
    if (!(fit >= 3.0) || n == 0) return oracle_fof(n, pos, L, lx, strict, label, size, n_groups);
    const int64_t nc = fit < 1290.0 ? (int64_t)fit : 1290;
    const int nt = threads > 0 ? threads : 1;
    const int64_t ncell = nc * nc * nc;
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t *first = (uint32_t *)calloc((size_t)ncell + 1, sizeof(uint32_t));
    float *spos = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    int32_t *orig = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *parent = NULL;
    link_list *lists = (link_list *)calloc((size_t)nc, sizeof(link_list));
    if (!cell || !first || !spos || !orig || !lists) {
        free(cell); free(first); free(spos); free(orig); free(lists);
        return ORACLE_ERR_MEM;
    }

    /* 2. cells, counts, prefix sum, slots */
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = (cell_of(pos[3 * i + 2], nc, L) * nc + cell_of(pos[3 * i + 1], nc, L)) * nc +
                    cell_of(pos[3 * i + 0], nc, L);
        cell[i] = (int32_t)c;
        __atomic_fetch_add(&first[c + 1], 1u, __ATOMIC_RELAXED);
    }
    for (int64_t c = 0; c < ncell; ++c) first[c + 1] += first[c];
    /* first[c] is the next free slot of cell c; afterwards it is the end of c */
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t s = __atomic_fetch_add(&first[cell[i]], 1u, __ATOMIC_RELAXED);
        spos[3 * (int64_t)s + 0] = pos[3 * i + 0];
        spos[3 * (int64_t)s + 1] = pos[3 * i + 1];
        spos[3 * (int64_t)s + 2] = pos[3 * i + 2];
        orig[s] = (int32_t)i;
    }
    memmove(first + 1, first, sizeof(uint32_t) * (size_t)ncell);
    first[0] = 0; /* cell c: slots first[c] .. first[c+1]-1 */

    /* 3. link search, one z-plane of cells per task */
    const double l2 = lx * lx;
    int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t cz = 0; cz < nc; ++cz) {
        link_list *out = &lists[cz];
        int bad = 0;
        for (int64_t cy = 0; cy < nc && !bad; ++cy)
            for (int64_t cx = 0; cx < nc && !bad; ++cx) {
                const int64_t c = (cz * nc + cy) * nc + cx;
                if (first[c] == first[c + 1]) continue;
                /* the slots of the 27 cells of the periodic shell */
                uint32_t lo[27], hi[27];
                int k = 0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx, ++k) {
                            int64_t ox = cx + dx, oy = cy + dy, oz = cz + dz;
                            ox += ox < 0 ? nc : (ox >= nc ? -nc : 0);
                            oy += oy < 0 ? nc : (oy >= nc ? -nc : 0);
                            oz += oz < 0 ? nc : (oz >= nc ? -nc : 0);
                            const int64_t o = (oz * nc + oy) * nc + ox;
                            lo[k] = first[o];
                            hi[k] = first[o + 1];
                        }
                for (uint32_t s = first[c]; s < first[c + 1] && !bad; ++s)
                    for (k = 0; k < 27; ++k)
                        for (uint32_t t = lo[k]; t < hi[k]; ++t)
                            if (orig[t] > orig[s] &&
                                linked(spos + 3 * (int64_t)s, spos + 3 * (int64_t)t, L, l2, strict))
                                if (link_push(out, (int32_t)s, (int32_t)t)) bad = 1;
            }
        if (bad) {
#pragma omp critical
            status = ORACLE_ERR_MEM;
        }
    }

    free(spos);
    free(first);

    /* 4. union-find over slots */
    if (status == ORACLE_OK) {
        parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!parent) status = ORACLE_ERR_MEM;
    }
    if (status == ORACLE_OK) {
        for (int64_t s = 0; s < n; ++s) parent[s] = (int32_t)s;
        for (int64_t cz = 0; cz < nc; ++cz)
            for (int64_t k = 0; k < lists[cz].count; ++k)
                unite(parent, lists[cz].pair[2 * k], lists[cz].pair[2 * k + 1]);
    }
    for (int64_t cz = 0; cz < nc; ++cz) free(lists[cz].pair);
    free(lists);

    /* 5. outputs: root of every slot (paths fully compressed by the first
     * pass), smallest input index and member count per root */
    int32_t *count = status == ORACLE_OK ? (int32_t *)calloc((size_t)n, sizeof(int32_t)) : NULL;
    if (status == ORACLE_OK && !count) status = ORACLE_ERR_MEM;
    if (status == ORACLE_OK) {
        int32_t *low = cell; /* reused: smallest input index at each root */
        int64_t groups = 0;
        for (int64_t s = 0; s < n; ++s) low[s] = INT32_MAX;
        for (int64_t s = 0; s < n; ++s) {
            int32_t r = find_root(parent, (int32_t)s);
            if (orig[s] < low[r]) low[r] = orig[s];
            count[r] += 1;
        }
#pragma omp parallel for schedule(static) num_threads(nt) reduction(+ : groups)
        for (int64_t s = 0; s < n; ++s) {
            const int32_t r = parent[s];
            label[orig[s]] = low[r];
            size[orig[s]] = orig[s] == low[r] ? count[r] : 0;
            if (r == s) groups += 1;
        }
        *n_groups = groups;
    }
    free(count);
    free(cell);
    free(orig);
    free(parent);
    return status;
}
