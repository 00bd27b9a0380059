/*
 * oracle/alg1.c -- the paper's own incremental method on the CPU (section
 * IV-B, Algorithm 1), in two schedules, for comparison only.
 *
 * TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU leg use it to
 * show what the paper's wave procedure computes on the same inputs (its
 * deviation from the exact field, the lowered / raised counts of Table II)
 * and what it costs on this CPU.  It is not the oracle (the exact field comes
 * from edt_oracle.c) and shares no code with the HIP path.
 *
 * What the method does (section IV-B):
 *   - every cell keeps the obstacle it points at, its squared distance to it
 *     (capped at D = d_max^2, reading R1) and a raise key; changed cells are
 *     the wave centres;
 *   - a removed obstacle starts a raising wave: cells that point at an
 *     obstacle that is gone forget it (back to D) and pass the raise on;
 *     cells that still point at a valid obstacle are where the raising wave
 *     stops, and they are queued to lower the cleared area again;
 *   - an added obstacle (and every boundary cell) starts a lowering wave: a
 *     cell offers its obstacle to its 26 neighbours, which take it when it
 *     is nearer than what they hold (or as near, when theirs is gone);
 *   - all fronts are popped in order of their key, the transform radius, so
 *     waves spread at the same speed (a bucket queue over 0..D, first in
 *     first out within a key: reading R22); stale duplicates are skipped.
 * Schedules:
 *   TRANSFORM_STATUS (the paper's "-Ex"): the raise key of a raising cell is
 *     its old transform radius, so a lowering wave that reaches a raising
 *     cell with a candidate no larger than that key takes the cell over at
 *     once and turns it into a lowering front;
 *   CONVENTIONAL (the scheme the paper improves on): the raise key is only a
 *     flag, raising cells are never touched by a lowering wave, and they are
 *     lowered again only after their raise has been processed.
 * Storage is dense arrays rather than a VDB tree: the procedure, not the
 * memory layout, is what is measured.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { SCHED_CONVENTIONAL = 0, SCHED_TRANSFORM_STATUS = 1 };
enum { SETTLED = -1 };          /* raise key of a cell that is not raising */

/* ---- bucket queue keyed by transform radius ---------------------------- */
typedef struct {
    int64_t* cell;
    int64_t len, cap, head;
} bucket;

typedef struct {
    bucket* b;
    int32_t kmax;     /* keys 0 .. kmax */
    int32_t low;      /* no bucket below this key holds an unread entry */
} wave_queue;

static int wq_init(wave_queue* q, int32_t kmax) {
    q->b = (bucket*)calloc((size_t)kmax + 1, sizeof(bucket));
    q->kmax = kmax;
    q->low = kmax + 1;
    return q->b ? 0 : -1;
}

static void wq_free(wave_queue* q) {
    if (!q->b) return;
    for (int32_t k = 0; k <= q->kmax; ++k) free(q->b[k].cell);
    free(q->b);
    q->b = NULL;
}

static int wq_push(wave_queue* q, int64_t c, int32_t key) {
    key = key < 0 ? 0 : (key > q->kmax ? q->kmax : key);
    bucket* b = &q->b[key];
    if (b->len == b->cap) {
        const int64_t cap = b->cap ? 2 * b->cap : 16;
        int64_t* p = (int64_t*)realloc(b->cell, (size_t)cap * sizeof(int64_t));
        if (!p) return -1;
        b->cell = p;
        b->cap = cap;
    }
    b->cell[b->len++] = c;
    if (key < q->low) q->low = key;
    return 0;
}

/* next entry of the smallest key (-1 when empty); drained buckets are reset */
static int64_t wq_pop(wave_queue* q) {
    for (; q->low <= q->kmax; ++q->low) {
        bucket* b = &q->b[q->low];
        if (b->head < b->len) return b->cell[b->head++];
        b->head = b->len = 0;
    }
    return -1;
}

/* ---- the distance field and its waves ----------------------------------- */
typedef struct alg1 {
    int nx, ny, nz, sched;
    int32_t D;
    int64_t n;
    uint8_t* occ;
    uint8_t* queued;    /* waiting in the queue */
    int64_t* obst;      /* obstacle the cell points at, -1 for none */
    int32_t* dist;      /* squared distance to it, capped at D */
    int32_t* rkey;      /* SETTLED, or the raise key of a raising cell */
    wave_queue q;
    int64_t lowered, raised;
} alg1;

void alg1_destroy(alg1* a) {
    if (!a) return;
    wq_free(&a->q);
    free(a->occ);
    free(a->queued);
    free(a->obst);
    free(a->dist);
    free(a->rkey);
    free(a);
}

/* Initialize: no obstacle anywhere, every cell at the cap and settled */
alg1* alg1_create(int nx, int ny, int nz, int dmax, int sched) {
    if (nx < 1 || ny < 1 || nz < 1 || dmax < 1 || dmax > 4095) return NULL;
    if (sched != SCHED_CONVENTIONAL && sched != SCHED_TRANSFORM_STATUS) return NULL;
    alg1* a = (alg1*)calloc(1, sizeof(alg1));
    if (!a) return NULL;
    a->nx = nx;
    a->ny = ny;
    a->nz = nz;
    a->sched = sched;
    a->D = dmax * dmax;
    a->n = (int64_t)nx * ny * nz;
    a->occ = (uint8_t*)calloc((size_t)a->n, 1);
    a->queued = (uint8_t*)calloc((size_t)a->n, 1);
    a->obst = (int64_t*)malloc((size_t)a->n * sizeof(int64_t));
    a->dist = (int32_t*)malloc((size_t)a->n * sizeof(int32_t));
    a->rkey = (int32_t*)malloc((size_t)a->n * sizeof(int32_t));
    if (!a->occ || !a->queued || !a->obst || !a->dist || !a->rkey || wq_init(&a->q, a->D)) {
        alg1_destroy(a);
        return NULL;
    }
    for (int64_t c = 0; c < a->n; ++c) {
        a->obst[c] = -1;
        a->dist[c] = a->D;
        a->rkey[c] = SETTLED;
    }
    return a;
}

static void enqueue(alg1* a, int64_t c, int32_t key) {
    a->queued[c] = 1;
    wq_push(&a->q, c, key);
}

static int32_t capped_sqdist(const alg1* a, int64_t p, int64_t c) {
    const int64_t nxy = (int64_t)a->nx * a->ny;
    const int64_t dx = p % a->nx - c % a->nx;
    const int64_t dy = (p / a->nx) % a->ny - (c / a->nx) % a->ny;
    const int64_t dz = p / nxy - c / nxy;
    const int64_t d = dx * dx + dy * dy + dz * dz;
    return d > a->D ? a->D : (int32_t)d;
}

/* a raising wave reaches cell c */
static void spread_raise(alg1* a, int64_t c) {
    const int64_t o = a->obst[c];
    if (o < 0) return;                     /* already cleared, nothing to pass on */
    if (a->occ[o]) {
        /* c still points at a valid obstacle: the raise stops here, and c
           will lower the cleared cells around it */
        if (!a->queued[c]) enqueue(a, c, a->dist[c]);
        return;
    }
    /* c pointed at a removed obstacle: it raises too, keyed by its old radius
       (transform status) or merely flagged (conventional), and forgets it */
    a->rkey[c] = a->sched == SCHED_TRANSFORM_STATUS ? a->dist[c] : 0;
    enqueue(a, c, a->dist[c]);
    a->obst[c] = -1;
    a->dist[c] = a->D;
}

/* a lowering wave offers obstacle o to cell c */
static void offer(alg1* a, int64_t c, int64_t o) {
    const int32_t d = capped_sqdist(a, o, c);
    if (a->rkey[c] != SETTLED) {
        /* a raising cell: only the transform-status schedule may take it over,
           when the offer is no farther than the radius it raises from */
        if (a->sched == SCHED_TRANSFORM_STATUS && a->rkey[c] >= d) {
            a->obst[c] = o;
            a->dist[c] = d;
            a->rkey[c] = SETTLED;
            enqueue(a, c, d);
        }
        return;
    }
    const int64_t held = a->obst[c];
    const int held_gone = held < 0 || !a->occ[held];
    if (d < a->dist[c] || (d == a->dist[c] && held_gone)) {
        a->obst[c] = o;
        a->dist[c] = d;
        if (d < a->D) enqueue(a, c, d);
    }
}

/* one popped front: pass its raise, or its obstacle, to the 26 neighbours,
   then the cell is settled and out of the queue */
static void relax(alg1* a, int64_t s) {
    const int raising = a->rkey[s] != SETTLED;
    const int64_t o = a->obst[s];
    if (raising) a->raised++;
    else a->lowered++;
    if (raising || o >= 0) {
        const int x = (int)(s % a->nx), y = (int)((s / a->nx) % a->ny),
                  z = (int)(s / ((int64_t)a->nx * a->ny));
        for (int dz = -1; dz <= 1; ++dz) {
            const int w = z + dz;
            if (w < 0 || w >= a->nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int v = y + dy;
                if (v < 0 || v >= a->ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int u = x + dx;
                    if (u < 0 || u >= a->nx || (!dx && !dy && !dz)) continue;
                    const int64_t c = u + (int64_t)a->nx * (v + (int64_t)a->ny * w);
                    if (raising) spread_raise(a, c);
                    else offer(a, c, o);
                }
            }
        }
    }
    a->rkey[s] = SETTLED;
    a->queued[s] = 0;
}

/* SetObstacle / RemoveObstacle: a cell already in the target state, or
   already waiting in the queue, is left alone (the guards of the paper's
   procedures); a new obstacle points at itself at distance 0 and starts a
   lowering wave, a removed one forgets its distance and starts a raising
   wave (raise key 0) */
static void change(alg1* a, int64_t c, int occupied) {
    if (!a->occ[c] == !occupied || a->queued[c]) return;
    a->occ[c] = occupied ? 1 : 0;
    a->obst[c] = occupied ? c : -1;
    a->dist[c] = occupied ? 0 : a->D;
    a->rkey[c] = occupied ? SETTLED : 0;
    enqueue(a, c, 0);
}

/* the changes of n entries (x, y, z) with target states, in order; entries
   outside the grid are ignored */
void alg1_apply(alg1* a, const int32_t* xyz, const uint8_t* state, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (x < 0 || y < 0 || z < 0 || x >= a->nx || y >= a->ny || z >= a->nz) continue;
        change(a, x + (int64_t)a->nx * (y + (int64_t)a->ny * z), state[i] != 0);
    }
}

/* DistanceTransform: pop fronts in key order until the queue is empty;
   counts[0] and counts[1] receive the fronts lowered and raised */
void alg1_transform(alg1* a, int64_t* counts) {
    a->lowered = a->raised = 0;
    for (int64_t s; (s = wq_pop(&a->q)) >= 0;)
        if (a->queued[s]) relax(a, s);
    if (counts) {
        counts[0] = a->lowered;
        counts[1] = a->raised;
    }
}

/* the distance field (squared, capped at D), x fastest */
void alg1_read(const alg1* a, int32_t* out) {
    memcpy(out, a->dist, (size_t)a->n * sizeof(int32_t));
}
