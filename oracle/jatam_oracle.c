/*
 * jatam_oracle.c - plain, slow, obviously correct CPU oracle for JaTAM
 * stochastic assembly and classification.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.  Every step follows the paper's definitions
 * directly (citations per function); no blocking, fusion or bit tricks:
 * cells are plain arrays, the frontier is a sorted list, options are found
 * by scanning every oriented tile, the interaction rule is the matrix M.
 */
#include "jatam_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of the  */
/* S-P network with the two published multipliers, the key bumped by the    */
/* two Weyl constants between rounds.  The paper's own generator (cuRAND    */
/* XORWOW, §3) is replaced by this counter-based one so that every run of   */
/* every genotype is reproducible from (seed, step, run, rng_id).           */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void jref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Jenkins one-at-a-time hash (App. F.4), over unsigned bytes.               */
/* ------------------------------------------------------------------------ */
uint32_t jref_oaat(const uint8_t* bytes, int64_t n)
{
    uint32_t h = 0;
    for (int64_t i = 0; i < n; ++i) {
        h += bytes[i];
        h += h << 10;
        h ^= h >> 6;
    }
    h += h << 3;
    h ^= h >> 11;
    h += h << 15;
    return h;
}

uint64_t jref_default_rng_id(uint64_t genome, int t)
{
    return genome | ((uint64_t)(unsigned)t << 56);
}

/* ------------------------------------------------------------------------ */
/* Shape hash made invariant under the dihedral group (§3.3 describes it   */
/* for the four rotations; mirrors are added here): hash the cropped shape  */
/* in each of the 8 orientations, each re-normalised to start at (0,0),    */
/* listing occupied cells in (y, x) order as the bytes x, y; sort the 8     */
/* hashes ascending and hash their 32 little-endian bytes again.            */
/* ------------------------------------------------------------------------ */
#define MAXG 64
#define MAXW (MAXG + 1)

/* (x', y') = (a*x + b*y, c*x + d*y), the 8 signed permutation matrices. */
static const int D4_MAPS[8][4] = {
    { 1, 0, 0, 1 }, { 0, -1, 1, 0 }, { -1, 0, 0, -1 }, { 0, 1, -1, 0 },
    { -1, 0, 0, 1 }, { 1, 0, 0, -1 }, { 0, 1, 1, 0 }, { 0, -1, -1, 0 },
};

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* The first nmaps maps of D4_MAPS: 8 for the dihedral group, 4 (the
 * rotations, determinant +1) for the rotation group C4 that §3.3 names. */
static uint32_t shape_hash_group(const uint8_t* mask, int w, int h, int nmaps)
{
    if (w <= 0 || h <= 0 || w > MAXW || h > MAXW)
        return 0;
    int n = 0;
    for (int i = 0; i < w * h; ++i)
        n += mask[i] != 0;
    if (n == 0)
        return 0;

    uint32_t hashes[8];
    static const int side = MAXW;
    uint8_t* img = (uint8_t*)malloc((size_t)side * side);
    uint8_t* bytes = (uint8_t*)malloc((size_t)2 * n);
    for (int k = 0; k < nmaps; ++k) {
        const int* T = D4_MAPS[k];
        /* transformed coordinates, then shift so the minimum is 0 */
        int minx = 1 << 30, miny = 1 << 30;
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x)
                if (mask[y * w + x]) {
                    int tx = T[0] * x + T[1] * y, ty = T[2] * x + T[3] * y;
                    if (tx < minx) minx = tx;
                    if (ty < miny) miny = ty;
                }
        memset(img, 0, (size_t)side * side);
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x)
                if (mask[y * w + x]) {
                    int tx = T[0] * x + T[1] * y - minx, ty = T[2] * x + T[3] * y - miny;
                    img[ty * side + tx] = 1;
                }
        int m = 0;
        for (int y = 0; y < side; ++y)
            for (int x = 0; x < side; ++x)
                if (img[y * side + x]) {
                    bytes[m++] = (uint8_t)x;
                    bytes[m++] = (uint8_t)y;
                }
        hashes[k] = jref_oaat(bytes, m);
    }
    free(img);
    free(bytes);
    qsort(hashes, (size_t)nmaps, sizeof(uint32_t), cmp_u32);
    uint8_t le[32];
    for (int k = 0; k < nmaps; ++k)
        for (int b = 0; b < 4; ++b)
            le[4 * k + b] = (uint8_t)(hashes[k] >> (8 * b));
    return jref_oaat(le, 4 * nmaps);
}

uint32_t jref_shape_hash_d4(const uint8_t* mask, int w, int h)
{
    return shape_hash_group(mask, w, h, 8);
}

/* Rotations only (§3.3: hash the four orthogonal rotations, sort the hashes
 * and hash them again): 16 little-endian bytes. */
uint32_t jref_shape_hash_c4(const uint8_t* mask, int w, int h)
{
    return shape_hash_group(mask, w, h, 4);
}

/* ------------------------------------------------------------------------ */
/* The tile model (§1.2, App. B.2, App. B.3).                                */
/* ------------------------------------------------------------------------ */

/* Interaction matrix of App. B.2: M_ij = (1 - i mod 2) d(i, j+1)
 * + (i mod 2) d(i, j-1); colours bond in adjacent pairs 1-2, 3-4, ...    */
static int interacts(int i, int j)
{
    return (1 - i % 2) * (i == j + 1) + (i % 2) * (i == j - 1);
}

/* y grows downwards ("looking down on the configuration grid", App. B.3) */
static const int DX[4] = { 0, 1, 0, -1 };
static const int DY[4] = { -1, 0, 1, 0 };

static int opposite(int d) { return (d + 2) % 4; }

typedef struct {
    int t, c, n;          /* n = 4t oriented tiles                          */
    int tup[16][4];       /* colour oriented tile 4i+r shows on side d      */
    int canon[16];        /* smallest oriented tile with the same tuple     */
} model_t;

static int log2_colours(int c)
{
    int b = 0;
    while ((1 << b) < c)
        ++b;
    return b;
}

/* Colour of tile i on side d: tiles in order, seed first, each as its N, E,
 * S, W colours, log2(c) bits each, most significant first (App. B.3). */
static int colour_of(uint64_t genome, int t, int c, int i, int d)
{
    int b = log2_colours(c);
    int shift = b * (4 * t - 1 - (4 * i + d));
    return (int)((genome >> shift) & (uint64_t)(c - 1));
}

/* Oriented tiles: tile i turned clockwise by r quarter turns shows on side d
 * the colour its side (d - r) mod 4 had; tiles rotate but never flip. */
static void build_model(uint64_t genome, int t, int c, model_t* m)
{
    m->t = t;
    m->c = c;
    m->n = 4 * t;
    for (int i = 0; i < t; ++i)
        for (int r = 0; r < 4; ++r)
            for (int d = 0; d < 4; ++d)
                m->tup[4 * i + r][d] = colour_of(genome, t, c, i, (d - r + 4) % 4);
    /* duplicate tile types and symmetric orientations are one tile (§3.2) */
    for (int k = 0; k < m->n; ++k) {
        m->canon[k] = k;
        for (int k2 = 0; k2 < k; ++k2)
            if (memcmp(m->tup[k2], m->tup[k], sizeof(m->tup[k])) == 0) {
                m->canon[k] = m->canon[k2];
                break;
            }
    }
}

/* The distinct tiles that can be placed next to a tile showing colour x,
 * on the side of the new tile facing back (side `facing`).  Returns how
 * many distinct tiles there are; *id receives one of them.            */
static int options(const model_t* m, int x, int facing, int* id)
{
    int seen[16];
    int count = 0;
    for (int k = 0; k < m->n; ++k) {
        if (!interacts(x, m->tup[k][facing]))
            continue;
        int ck = m->canon[k], dup = 0;
        for (int s = 0; s < count; ++s)
            dup |= seen[s] == ck;
        if (!dup)
            seen[count++] = ck;
    }
    if (count > 0)
        *id = seen[0];
    return count;
}

/* ------------------------------------------------------------------------ */
/* One assembly run (§1.2, §3.2).                                            */
/* ------------------------------------------------------------------------ */
enum { EV_NONE = 0, EV_UNBOUND = 1, EV_AMBIG = 2 };

typedef struct {
    int G, W;                      /* W = G + 1: cells (x, y) in [0, G]^2  */
    int16_t cell[MAXW * MAXW];     /* -1 empty, else the placed tile       */
    int16_t pend[MAXW * MAXW];     /* -1 not on the frontier, else its tile */
    int front[MAXW * MAXW];        /* frontier positions, ascending y*W+x  */
    int nf;
    int size;
} grid_t;

static int on_ring(const grid_t* g, int x, int y)
{
    return x == 0 || y == 0 || x == g->G || y == g->G;
}

static void frontier_insert(grid_t* g, int p)
{
    int i = g->nf;
    while (i > 0 && g->front[i - 1] > p) {
        g->front[i] = g->front[i - 1];
        --i;
    }
    g->front[i] = p;
    g->nf++;
}

static void frontier_remove_at(grid_t* g, int j)
{
    for (int i = j; i + 1 < g->nf; ++i)
        g->front[i] = g->front[i + 1];
    g->nf--;
}

/* Checks the empty neighbours of the tile just placed at p.  Any bondable
 * site on the ring means the structure is not bounded by the box (App.
 * B.2); a site whose occupied neighbours admit two distinct tiles is
 * ambiguous (§3.2).  Otherwise a site with one admissible tile joins the
 * frontier with that tile pending. */
static int update(const model_t* m, grid_t* g, int p)
{
    int px = p % g->W, py = p / g->W;
    int placed = g->cell[p];
    int unbound = 0, ambiguous = 0;
    for (int d = 0; d < 4; ++d) {
        int qx = px + DX[d], qy = py + DY[d];
        int q = qy * g->W + qx;
        if (g->cell[q] >= 0)
            continue;
        int id = -1;
        int k = options(m, m->tup[placed][d], opposite(d), &id);
        if (k == 0)
            continue;
        if (on_ring(g, qx, qy))
            unbound = 1;
        else if (k >= 2 || (g->pend[q] >= 0 && g->pend[q] != id))
            ambiguous = 1;
        else if (g->pend[q] < 0) {
            g->pend[q] = (int16_t)id;
            frontier_insert(g, q);
        }
    }
    return unbound ? EV_UNBOUND : ambiguous ? EV_AMBIG : EV_NONE;
}

typedef struct {
    int event;
    int steps;
    int choice;     /* the frontier held >= 2 sites at some draw */
} run_out_t;

/* Grows one structure from the seed.  Each step draws one 32-bit word of
 * the Philox stream keyed by the seed at counter (step/4, run, rng_id) and
 * places the pending tile of the frontier site with rank floor(u*|F|/2^32)
 * in row-major order.  trace, if not NULL, receives placed positions. */
static run_out_t run_once(const model_t* m, grid_t* g, int run, uint64_t seed,
                          uint64_t rng_id, int32_t* trace, int cap, int* ntrace)
{
    run_out_t out = { EV_NONE, 0, 0 };
    int W = g->W;
    for (int i = 0; i < W * W; ++i) {
        g->cell[i] = -1;
        g->pend[i] = -1;
    }
    g->nf = 0;
    int centre = (g->G / 2) * W + g->G / 2;
    g->cell[centre] = (int16_t)m->canon[0];
    g->size = 1;
    if (trace && *ntrace < cap)
        trace[(*ntrace)++] = centre;
    int ev = update(m, g, centre);
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (;;) {
        if (ev != EV_NONE)
            break;
        if (g->nf == 0)
            break;
        if (g->nf >= 2)
            out.choice = 1;
        uint32_t ctr[4] = { (uint32_t)out.steps >> 2, (uint32_t)run,
                            (uint32_t)rng_id, (uint32_t)(rng_id >> 32) };
        uint32_t words[4];
        jref_philox4x32_10(ctr, key, words);
        uint32_t u = words[out.steps & 3];
        int j = (int)(((uint64_t)u * (uint64_t)g->nf) >> 32);
        int p = g->front[j];
        frontier_remove_at(g, j);
        g->cell[p] = g->pend[p];
        g->pend[p] = -1;
        g->size++;
        out.steps++;
        if (trace && *ntrace < cap)
            trace[(*ntrace)++] = p;
        ev = update(m, g, p);
    }
    out.event = ev;
    return out;
}

/* The movelist variant (§3.2): the frontier sites form a LIFO stack.  A
 * site that joins the frontier (in direction order N, E, S, W of each
 * update) is inserted at position floor(u * (len + 1) / 2^32) counted from
 * the bottom of the len sites on the stack, u the next word of the run's
 * stream (word d of the run for its d-th draw; no word is drawn while the
 * stack is empty); every step places the pending tile of the site on top. */
typedef struct {
    int sites[MAXW * MAXW];
    int len;
    int draws;
    int choice;
} movelist_t;

static void movelist_insert(movelist_t* ml, int q, const uint32_t key[2], int run,
                            uint64_t rng_id)
{
    int pos = 0;
    if (ml->len > 0) {
        uint32_t ctr[4] = { (uint32_t)ml->draws >> 2, (uint32_t)run, (uint32_t)rng_id,
                            (uint32_t)(rng_id >> 32) };
        uint32_t words[4];
        jref_philox4x32_10(ctr, key, words);
        uint32_t u = words[ml->draws & 3];
        ml->draws++;
        ml->choice = 1;
        pos = (int)(((uint64_t)u * (uint64_t)(ml->len + 1)) >> 32);
    }
    for (int i = ml->len; i > pos; --i)
        ml->sites[i] = ml->sites[i - 1];
    ml->sites[pos] = q;
    ml->len++;
}

/* update() that also pushes every site joining the frontier on the stack. */
static int update_lifo(const model_t* m, grid_t* g, int p, movelist_t* ml,
                       const uint32_t key[2], int run, uint64_t rng_id)
{
    int before[4], qs[4];
    int px = p % g->W, py = p / g->W;
    for (int d = 0; d < 4; ++d) {
        qs[d] = (py + DY[d]) * g->W + (px + DX[d]);
        before[d] = g->cell[qs[d]] < 0 && g->pend[qs[d]] < 0;
    }
    int ev = update(m, g, p);
    for (int d = 0; d < 4; ++d)
        if (before[d] && g->pend[qs[d]] >= 0)
            movelist_insert(ml, qs[d], key, run, rng_id);
    return ev;
}

static run_out_t run_once_lifo(const model_t* m, grid_t* g, int run, uint64_t seed,
                               uint64_t rng_id, int32_t* trace, int cap, int* ntrace)
{
    run_out_t out = { EV_NONE, 0, 0 };
    int W = g->W;
    static __thread movelist_t ml;
    for (int i = 0; i < W * W; ++i) {
        g->cell[i] = -1;
        g->pend[i] = -1;
    }
    g->nf = 0;
    ml.len = 0;
    ml.draws = 0;
    ml.choice = 0;
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    int centre = (g->G / 2) * W + g->G / 2;
    g->cell[centre] = (int16_t)m->canon[0];
    g->size = 1;
    if (trace && *ntrace < cap)
        trace[(*ntrace)++] = centre;
    int ev = update_lifo(m, g, centre, &ml, key, run, rng_id);
    while (ev == EV_NONE && ml.len > 0) {
        int p = ml.sites[--ml.len];
        /* the sorted frontier list mirrors the stack's sites */
        for (int j = 0; j < g->nf; ++j)
            if (g->front[j] == p) {
                frontier_remove_at(g, j);
                break;
            }
        g->cell[p] = g->pend[p];
        g->pend[p] = -1;
        g->size++;
        out.steps++;
        if (trace && *ntrace < cap)
            trace[(*ntrace)++] = p;
        ev = update_lifo(m, g, p, &ml, key, run, rng_id);
    }
    out.event = ev;
    out.choice = ml.choice;
    return out;
}

/* ------------------------------------------------------------------------ */
/* Classification of one genotype (§3.2, §3.3).                              */
/* ------------------------------------------------------------------------ */
int jref_check_args(int t, int c, int grid, int runs)
{
    if (t < 1 || t > 4)
        return JREF_E_INVALID_ARG;
    if (c != 2 && c != 4 && c != 8 && c != 16)
        return JREF_E_INVALID_ARG;
    if (4 * t * log2_colours(c) > 64)
        return JREF_E_INVALID_ARG;
    if (grid < 8 || grid > MAXG || grid % 2 != 0)
        return JREF_E_INVALID_ARG;
    if (runs < 1 || runs > 64)
        return JREF_E_INVALID_ARG;
    return JREF_OK;
}

static int genome_fits(uint64_t genome, int t, int c)
{
    int bits = 4 * t * log2_colours(c);
    return bits >= 64 || (genome >> bits) == 0;
}

/* Crop an occupancy mask of W*W cells to its bounding box (App. F.6) and
 * hash the cropped shape. */
static uint32_t hash_of_occupancy(const uint8_t* occ, int W, int variant)
{
    int minx = W, miny = W, maxx = -1, maxy = -1;
    for (int y = 0; y < W; ++y)
        for (int x = 0; x < W; ++x)
            if (occ[y * W + x]) {
                if (x < minx) minx = x;
                if (y < miny) miny = y;
                if (x > maxx) maxx = x;
                if (y > maxy) maxy = y;
            }
    if (maxx < 0)
        return 0;
    int w = maxx - minx + 1, h = maxy - miny + 1;
    uint8_t* mask = (uint8_t*)calloc((size_t)w * h, 1);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x)
            mask[y * w + x] = occ[(y + miny) * W + (x + minx)];
    uint32_t hv = (variant & JREF_VARIANT_C4) ? jref_shape_hash_c4(mask, w, h)
                                              : jref_shape_hash_d4(mask, w, h);
    free(mask);
    return hv;
}

static void occupancy_of(const grid_t* g, uint8_t* occ)
{
    for (int i = 0; i < g->W * g->W; ++i)
        occ[i] = g->cell[i] >= 0;
}

typedef struct {
    int steps;
    int event;
    int choice;
    int forced;     /* the first run's shape is forced (forced_shape)   */
    int guarded;    /* the first run's shape is guarded (guarded_shape) */
} run0_info_t;

/* Whether the shape the run left in g is forced: for every occupied cell
 * and every occupied neighbour, the tiles that bond to the neighbour's tile
 * on the side facing the cell are none, or exactly the cell's own tile.  A
 * cell's options in any growth order are the union of such sets over the
 * neighbours present at the time, so every order then places the same tile
 * in every cell of the shape, and never meets two options.  (Sites outside
 * the shape that a shape tile bonds to cannot exist after a run that ended
 * with an empty frontier and no event.) */
static int forced_shape(const model_t* m, const grid_t* g)
{
    for (int p = 0; p < g->W * g->W; ++p) {
        if (g->cell[p] < 0)
            continue;
        int px = p % g->W, py = p / g->W;
        for (int d = 0; d < 4; ++d) {
            int qx = px + DX[d], qy = py + DY[d];
            if (qx < 0 || qy < 0 || qx >= g->W || qy >= g->W)
                continue;
            int q = qy * g->W + qx;
            if (g->cell[q] < 0)
                continue;
            /* the neighbour shows this colour towards p; p's tile faces
             * back on side d */
            int id = -1;
            int k = options(m, m->tup[g->cell[q]][opposite(d)], d, &id);
            if (k >= 2 || (k == 1 && id != g->cell[p]))
                return 0;
        }
    }
    return 1;
}

/* The tiles that the tile at q admits at its neighbour p (direction d from
 * p to q), as (count, one id) from options(): q shows its side facing p,
 * the new tile at p faces back on side d. */
static int options_from(const model_t* m, const grid_t* g, int q, int d, int* id)
{
    return options(m, m->tup[g->cell[q]][opposite(d)], d, id);
}

/* Whether target can be reached from the seed, in the shape the run left in
 * g, by steps from an occupied cell a to an occupied neighbour b that a's
 * tile admits exactly b's tile at (and nothing else), never entering cell x.
 * Plain breadth-first search over the grid. */
static int reached_without(const model_t* m, const grid_t* g, int x, int target)
{
    int W = g->W, seed = (g->G / 2) * W + g->G / 2;
    static __thread int queue[MAXW * MAXW];
    static __thread uint8_t seen[MAXW * MAXW];
    if (seed == x)
        return 0;
    memset(seen, 0, sizeof(seen));
    int head = 0, tail = 0;
    queue[tail++] = seed;
    seen[seed] = 1;
    while (head < tail) {
        int a = queue[head++];
        if (a == target)
            return 1;
        int ax = a % W, ay = a / W;
        for (int d = 0; d < 4; ++d) {
            int bx = ax + DX[d], by = ay + DY[d];
            if (bx < 0 || by < 0 || bx >= W || by >= W)
                continue;
            int b = by * W + bx;
            if (b == x || seen[b] || g->cell[b] < 0)
                continue;
            int id = -1;
            int k = options_from(m, g, a, opposite(d), &id);   /* a seen from b */
            if (k != 1 || id != g->cell[b])
                continue;
            seen[b] = 1;
            queue[tail++] = b;
        }
    }
    return 0;
}

/* Whether the shape the run left in g (run ended with no event) is guarded:
 * for every occupied cell p other than the seed and every occupied
 * neighbour q whose tile admits at p anything but p's own tile, q cannot be
 * reached from the seed by exact bonds without passing through p.  Then in
 * every growth order q is placed after p, and every order places the same
 * tiles in the same cells without events.  Forced shapes are the guarded
 * shapes with no such pair.  (Not a step of the paper's method: an exact
 * shortcut that a pipelined implementation may take, pinned by tests
 * against the classification itself and against the brute-force
 * explorer.) */
static int guarded_shape(const model_t* m, const grid_t* g)
{
    int W = g->W, seed = (g->G / 2) * W + g->G / 2;
    for (int p = 0; p < W * W; ++p) {
        if (g->cell[p] < 0 || p == seed)
            continue;
        int px = p % W, py = p / W;
        for (int d = 0; d < 4; ++d) {
            int qx = px + DX[d], qy = py + DY[d];
            if (qx < 0 || qy < 0 || qx >= W || qy >= W)
                continue;
            int q = qy * W + qx;
            if (g->cell[q] < 0)
                continue;
            int id = -1;
            int k = options_from(m, g, q, d, &id);
            int conflict = k >= 2 || (k == 1 && id != g->cell[p]);
            if (conflict && reached_without(m, g, p, q))
                return 0;
        }
    }
    return 1;
}

static int classify_with(grid_t* g, uint8_t* occ0, uint8_t* occ, uint64_t genome,
                         uint64_t rng_id, int t, int c, int grid, int runs,
                         uint64_t seed, jref_result_t* out, uint8_t* occ_out,
                         run0_info_t* info0, int variant)
{
    if (jref_check_args(t, c, grid, runs) != JREF_OK || !genome_fits(genome, t, c))
        return JREF_E_INVALID_ARG;
    model_t m;
    build_model(genome, t, c, &m);
    g->G = grid;
    g->W = grid + 1;
    int cells = g->W * g->W;
    int work = 0, size0 = 0;
    for (int r = 0; r < runs; ++r) {
        run_out_t ro = (variant & JREF_VARIANT_LIFO)
                           ? run_once_lifo(&m, g, r, seed, rng_id, NULL, 0, NULL)
                           : run_once(&m, g, r, seed, rng_id, NULL, 0, NULL);
        work += ro.steps;
        if (r == 0 && info0) {
            info0->steps = ro.steps;
            info0->event = ro.event;
            info0->choice = ro.choice;
            info0->forced = ro.event == EV_NONE && forced_shape(&m, g);
            info0->guarded = ro.event == EV_NONE && guarded_shape(&m, g);
        }
        if (ro.event != EV_NONE) {
            out->cls = ro.event == EV_UNBOUND ? JREF_UNBOUND : JREF_ND_SITE;
            out->size = g->size;
            out->hash = 0;
            out->steps = work;
            if (occ_out)
                occupancy_of(g, occ_out);
            return JREF_OK;
        }
        if (r == 0) {
            occupancy_of(g, occ0);
            size0 = g->size;
            if (!ro.choice)  /* no draw ever chose: every run is this run */
                break;
        } else {
            occupancy_of(g, occ);
            if (memcmp(occ, occ0, (size_t)cells) != 0) {
                out->cls = JREF_ND_RUNS;
                out->size = g->size;
                out->hash = 0;
                out->steps = work;
                if (occ_out)
                    memcpy(occ_out, occ, (size_t)cells);
                return JREF_OK;
            }
        }
    }
    out->cls = JREF_DET;
    out->size = size0;
    out->hash = hash_of_occupancy(occ0, g->W, variant);
    out->steps = work;
    if (occ_out)
        memcpy(occ_out, occ0, (size_t)cells);
    return JREF_OK;
}

typedef struct {
    grid_t g;
    uint8_t occ0[MAXW * MAXW];
    uint8_t occ[MAXW * MAXW];
} workspace_t;

int jref_classify_one(uint64_t genome, uint64_t rng_id, int t, int c, int grid,
                      int runs, uint64_t seed, jref_result_t* out, uint8_t* occ_out)
{
    workspace_t* ws = (workspace_t*)malloc(sizeof(workspace_t));
    if (!ws)
        return JREF_E_INVALID_ARG;
    int rc = classify_with(&ws->g, ws->occ0, ws->occ, genome, rng_id, t, c, grid,
                           runs, seed, out, occ_out, NULL, 0);
    free(ws);
    return rc;
}

int jref_trace_run_variant(uint64_t genome, uint64_t rng_id, int t, int c, int grid,
                           int run, uint64_t seed, int variant, int32_t* cells_out, int cap,
                           int* event, int* choice)
{
    if (jref_check_args(t, c, grid, 1) != JREF_OK || !genome_fits(genome, t, c) || run < 0)
        return JREF_E_INVALID_ARG;
    workspace_t* ws = (workspace_t*)malloc(sizeof(workspace_t));
    if (!ws)
        return JREF_E_INVALID_ARG;
    model_t m;
    build_model(genome, t, c, &m);
    ws->g.G = grid;
    ws->g.W = grid + 1;
    int n = 0;
    run_out_t ro = (variant & JREF_VARIANT_LIFO)
                       ? run_once_lifo(&m, &ws->g, run, seed, rng_id, cells_out, cap, &n)
                       : run_once(&m, &ws->g, run, seed, rng_id, cells_out, cap, &n);
    if (event)
        *event = ro.event;
    if (choice)
        *choice = ro.choice;
    free(ws);
    return n;
}

int jref_trace_run(uint64_t genome, uint64_t rng_id, int t, int c, int grid,
                   int run, uint64_t seed, int32_t* cells_out, int cap,
                   int* event, int* choice)
{
    return jref_trace_run_variant(genome, rng_id, t, c, grid, run, seed, 0, cells_out, cap,
                                  event, choice);
}

/* ------------------------------------------------------------------------ */
/* Host thread pool: dynamic chunks of genotypes.                            */
/* ------------------------------------------------------------------------ */
enum { MODE_LIST = 0, MODE_RANGE = 1, MODE_ITEMS = 2 };

typedef struct {
    int mode;
    const uint64_t* genomes;
    const jref_item_t* items;
    uint64_t first;
    int64_t n;
    int t, c, grid, runs;
    uint64_t seed;
    jref_result_t* out;
    int32_t* run0_steps;   /* optional run-0 detail          */
    int8_t* run0_event;
    int8_t* run0_choice;
    int8_t* run0_forced;
    int64_t next;          /* next unclaimed index (atomic)  */
    int error;             /* first error seen (atomic)      */
    int variant;           /* JREF_VARIANT_* flags           */
} job_t;

#define CHUNK 4096

static void* worker(void* arg)
{
    job_t* job = (job_t*)arg;
    workspace_t* ws = (workspace_t*)malloc(sizeof(workspace_t));
    if (!ws) {
        __atomic_store_n(&job->error, JREF_E_INVALID_ARG, __ATOMIC_RELAXED);
        return NULL;
    }
    for (;;) {
        int64_t begin = __atomic_fetch_add(&job->next, CHUNK, __ATOMIC_RELAXED);
        if (begin >= job->n)
            break;
        int64_t end = begin + CHUNK < job->n ? begin + CHUNK : job->n;
        for (int64_t i = begin; i < end; ++i) {
            int rc;
            if (job->mode == MODE_ITEMS) {
                const jref_item_t* it = &job->items[i];
                rc = classify_with(&ws->g, ws->occ0, ws->occ, it->genome, it->rng_id,
                                   it->t, job->c, it->grid, job->runs, job->seed,
                                   &job->out[i], NULL, NULL, job->variant);
            } else {
                uint64_t g = job->mode == MODE_RANGE ? job->first + (uint64_t)i
                                                     : job->genomes[i];
                run0_info_t info = { 0, 0, 0, 0, 0 };
                rc = classify_with(&ws->g, ws->occ0, ws->occ, g,
                                   jref_default_rng_id(g, job->t), job->t, job->c,
                                   job->grid, job->runs, job->seed, &job->out[i], NULL,
                                   job->run0_steps ? &info : NULL, job->variant);
                if (job->run0_steps) {
                    job->run0_steps[i] = info.steps;
                    job->run0_event[i] = (int8_t)info.event;
                    job->run0_choice[i] = (int8_t)info.choice;
                    job->run0_forced[i] = (int8_t)(info.forced | (info.guarded << 1));
                }
            }
            if (rc != JREF_OK)
                __atomic_store_n(&job->error, rc, __ATOMIC_RELAXED);
        }
    }
    free(ws);
    return NULL;
}

static int run_job(job_t* job, int threads)
{
    if (job->n < 0)
        return JREF_E_INVALID_ARG;
    if (threads <= 0) {
        long online = sysconf(_SC_NPROCESSORS_ONLN);
        threads = online > 0 ? (int)online : 1;
    }
    if (threads > 256)
        threads = 256;
    job->next = 0;
    job->error = JREF_OK;
    pthread_t tid[256];
    int started = 0;
    for (int i = 1; i < threads; ++i)
        if (pthread_create(&tid[started], NULL, worker, job) == 0)
            ++started;
    worker(job);
    for (int i = 0; i < started; ++i)
        pthread_join(tid[i], NULL);
    return job->error;
}

int jref_classify(const uint64_t* genomes, int64_t n, int t, int c, int grid,
                  int runs, uint64_t seed, jref_result_t* out, int threads)
{
    if (jref_check_args(t, c, grid, runs) != JREF_OK)
        return JREF_E_INVALID_ARG;
    job_t job = { MODE_LIST, genomes, NULL, 0, n, t, c, grid, runs, seed, out,
                  NULL, NULL, NULL, NULL, 0, 0, 0 };
    return run_job(&job, threads);
}

int jref_classify_range(uint64_t first, int64_t n, int t, int c, int grid,
                        int runs, uint64_t seed, jref_result_t* out, int threads)
{
    if (jref_check_args(t, c, grid, runs) != JREF_OK)
        return JREF_E_INVALID_ARG;
    job_t job = { MODE_RANGE, NULL, NULL, first, n, t, c, grid, runs, seed, out,
                  NULL, NULL, NULL, NULL, 0, 0, 0 };
    return run_job(&job, threads);
}

int jref_classify_variant(const uint64_t* genomes, uint64_t first, int64_t n, int t, int c,
                          int grid, int runs, uint64_t seed, int variant, jref_result_t* out,
                          int threads)
{
    if (jref_check_args(t, c, grid, runs) != JREF_OK ||
        (variant & ~(JREF_VARIANT_C4 | JREF_VARIANT_LIFO)) != 0)
        return JREF_E_INVALID_ARG;
    job_t job = { genomes ? MODE_LIST : MODE_RANGE, genomes, NULL, first, n, t, c, grid, runs,
                  seed, out, NULL, NULL, NULL, NULL, 0, 0, variant };
    return run_job(&job, threads);
}

int jref_classify_range_run0(uint64_t first, int64_t n, int t, int c, int grid,
                             int runs, uint64_t seed, jref_result_t* out,
                             int32_t* run0_steps, int8_t* run0_event,
                             int8_t* run0_choice, int8_t* run0_forced, int threads)
{
    if (jref_check_args(t, c, grid, runs) != JREF_OK || !run0_steps || !run0_event ||
        !run0_choice || !run0_forced)
        return JREF_E_INVALID_ARG;
    job_t job = { MODE_RANGE, NULL, NULL, first, n, t, c, grid, runs, seed, out,
                  run0_steps, run0_event, run0_choice, run0_forced, 0, 0, 0 };
    return run_job(&job, threads);
}

int jref_classify_items(const jref_item_t* items, int64_t n, int c, int runs,
                        uint64_t seed, jref_result_t* out, int threads)
{
    if (jref_check_args(1, c, 16, runs) != JREF_OK)
        return JREF_E_INVALID_ARG;
    job_t job = { MODE_ITEMS, NULL, items, 0, n, 1, c, 16, runs, seed, out,
                  NULL, NULL, NULL, NULL, 0, 0, 0 };
    return run_job(&job, threads);
}

/* ------------------------------------------------------------------------ */
/* True class by exhaustive exploration of every growth order.               */
/*                                                                           */
/* The k runs of §3.2 sample growth orders; a genotype is deterministic when */
/* every order ends in one shape without an event, and k runs can miss an    */
/* order that shows otherwise (the misclassification that falls with k,      */
/* §4.1).  Here every order is followed: a state is the set of placed        */
/* (cell, tile) pairs, states are visited breadth first, each once, and a    */
/* state is analysed from scratch (every occupied cell's neighbours, the     */
/* isotropic check of §3.2).  The exploration stops at the first event (a    */
/* bondable ring site or an ambiguous site) or at a second terminal shape    */
/* (occupancy, compared without rotation): the genotype is then not         */
/* deterministic.  More than `cap` states: undecided.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t* arena;        /* each state: its (cell << 8 | tile) pairs, ascending */
    int64_t arena_used, arena_cap;
    int64_t* start;        /* state k's first pair in the arena                   */
    int32_t* len;          /* state k's pair count                                */
    int64_t n, cap;
    int64_t* slot;         /* open addressing: state index + 1, 0 = empty         */
    int64_t nslots;
    int64_t* slot_of;      /* state k's slot, to empty the table afterwards       */
} state_set_t;

static uint64_t pairs_hash(const int32_t* p, int len)
{
    uint64_t h = 1469598103934665603ull;   /* FNV-1a over the pairs */
    for (int i = 0; i < len; ++i) {
        h ^= (uint32_t)p[i];
        h *= 1099511628211ull;
    }
    return h;
}

/* Adds the state unless present.  Returns 1 if added, 0 if present, -1 if
 * the set is full. */
static int state_add(state_set_t* s, const int32_t* p, int len)
{
    uint64_t h = pairs_hash(p, len) & (uint64_t)(s->nslots - 1);
    for (;;) {
        int64_t k = s->slot[h];
        if (k == 0)
            break;
        k -= 1;
        if (s->len[k] == len && memcmp(s->arena + s->start[k], p, sizeof(int32_t) * len) == 0)
            return 0;
        h = (h + 1) & (uint64_t)(s->nslots - 1);
    }
    if (s->n == s->cap)
        return -1;
    if (s->arena_used + len > s->arena_cap) {
        int64_t nc = s->arena_cap * 2 + len;
        int32_t* na = (int32_t*)realloc(s->arena, sizeof(int32_t) * nc);
        if (!na)
            return -1;
        s->arena = na;
        s->arena_cap = nc;
    }
    memcpy(s->arena + s->arena_used, p, sizeof(int32_t) * len);
    s->start[s->n] = s->arena_used;
    s->len[s->n] = len;
    s->slot_of[s->n] = (int64_t)h;
    s->arena_used += len;
    s->slot[h] = ++s->n;
    return 1;
}

enum { TRUTH_DET = 0, TRUTH_ND = 1, TRUTH_CAPPED = 2 };

static int explore_all(const model_t* m, grid_t* g, int64_t cap, state_set_t* s,
                       uint8_t* term, uint8_t* occ, int* size_out, uint32_t* hash_out,
                       int64_t* states_out)
{
    int W = g->W, cells = W * W;
    int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (cells + 1));
    int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (cells + 1));
    int verdict = TRUTH_DET, have_term = 0, term_size = 0;
    s->n = 0;
    s->arena_used = 0;
    s->cap = cap;
    int centre = (g->G / 2) * W + g->G / 2;
    cur[0] = (centre << 8) | m->canon[0];
    state_add(s, cur, 1);
    for (int64_t k = 0; k < s->n; ++k) {
        int len = s->len[k];
        memcpy(cur, s->arena + s->start[k], sizeof(int32_t) * len);
        /* the state's grid, analysed from scratch */
        for (int i = 0; i < cells; ++i) {
            g->cell[i] = -1;
            g->pend[i] = -1;
        }
        g->nf = 0;
        for (int i = 0; i < len; ++i)
            g->cell[cur[i] >> 8] = (int16_t)(cur[i] & 0xFF);
        int ev = EV_NONE;
        for (int i = 0; i < len; ++i) {
            int e = update(m, g, cur[i] >> 8);
            if (e != EV_NONE)
                ev = e;
        }
        if (ev != EV_NONE) {
            verdict = TRUTH_ND;
            break;
        }
        if (g->nf == 0) {
            occupancy_of(g, occ);
            if (!have_term) {
                memcpy(term, occ, (size_t)cells);
                term_size = len;
                have_term = 1;
            } else if (memcmp(term, occ, (size_t)cells) != 0) {
                verdict = TRUTH_ND;
                break;
            }
            continue;
        }
        for (int j = 0; j < g->nf; ++j) {
            int q = g->front[j];
            /* the state plus (q, its pending tile), pairs kept ascending */
            int o = 0, placed = 0;
            for (int i = 0; i < len; ++i) {
                if (!placed && (cur[i] >> 8) > q) {
                    nxt[o++] = (q << 8) | g->pend[q];
                    placed = 1;
                }
                nxt[o++] = cur[i];
            }
            if (!placed)
                nxt[o++] = (q << 8) | g->pend[q];
            if (state_add(s, nxt, o) < 0) {
                verdict = TRUTH_CAPPED;
                break;
            }
        }
        if (verdict == TRUTH_CAPPED)
            break;
    }
    *states_out = s->n;
    for (int64_t k = 0; k < s->n; ++k)   /* empty the table for the next genotype */
        s->slot[s->slot_of[k]] = 0;
    *size_out = verdict == TRUTH_DET ? term_size : 0;
    *hash_out = verdict == TRUTH_DET ? hash_of_occupancy(term, W, 0) : 0;
    free(cur);
    free(nxt);
    return verdict;
}

int jref_true_class(const uint64_t* genomes, int64_t n, int t, int c, int grid, int64_t cap,
                    jref_result_t* out)
{
    if (jref_check_args(t, c, grid, 1) != JREF_OK || n < 0 || cap < 1 || cap > (1 << 24))
        return JREF_E_INVALID_ARG;
    state_set_t s;
    s.nslots = 1;
    while (s.nslots < 2 * cap)
        s.nslots *= 2;
    s.arena_cap = 1 << 16;
    s.arena = (int32_t*)malloc(sizeof(int32_t) * s.arena_cap);
    s.start = (int64_t*)malloc(sizeof(int64_t) * cap);
    s.len = (int32_t*)malloc(sizeof(int32_t) * cap);
    s.slot = (int64_t*)calloc((size_t)s.nslots, sizeof(int64_t));
    s.slot_of = (int64_t*)malloc(sizeof(int64_t) * cap);
    workspace_t* ws = (workspace_t*)malloc(sizeof(workspace_t));
    int rc = JREF_OK;
    if (!s.arena || !s.start || !s.len || !s.slot || !s.slot_of || !ws)
        rc = JREF_E_INVALID_ARG;
    for (int64_t i = 0; i < n && rc == JREF_OK; ++i) {
        if (!genome_fits(genomes[i], t, c)) {
            rc = JREF_E_INVALID_ARG;
            break;
        }
        model_t m;
        build_model(genomes[i], t, c, &m);
        ws->g.G = grid;
        ws->g.W = grid + 1;
        int size = 0;
        uint32_t hv = 0;
        int64_t states = 0;
        int v = explore_all(&m, &ws->g, cap, &s, ws->occ0, ws->occ, &size, &hv, &states);
        out[i].cls = v == TRUTH_DET ? JREF_DET : v == TRUTH_ND ? JREF_ND_SITE : -2;
        out[i].size = size;
        out[i].hash = hv;
        out[i].steps = (int32_t)states;
    }
    free(s.arena);
    free(s.start);
    free(s.len);
    free(s.slot);
    free(s.slot_of);
    free(ws);
    return rc;
}
