/*
 * oracle/alg1.c -- the paper's own method on the CPU: the incremental
 * Euclidean distance transform of Algorithm 1 (SetObstacle, RemoveObstacle,
 * DistanceTransform with Raise and Lower over the 26-neighbourhood, a priority
 * queue ordered by squared distance, one nearest-obstacle pointer per cell).
 * TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU leg use it to
 * show what the paper's procedure computes on the same inputs (its
 * deviation from the exact field, its lowered / raised cell counts as in
 * Table II) and how long it takes on this CPU.  It is not the oracle (the
 * exact field comes from edt_oracle.c) and shares no code with the HIP path.
 *
 * Readings: distances are squared and capped at D = d_max^2 (R1); the raise
 * field holds -1 when a cell is not raising and the old distance otherwise
 * (the key of the raise wave); the queue is a bucket queue over the integer
 * keys 0..D, first in first out within a key (the paper leaves the order of
 * equal keys open); a cell is processed when popped while still marked
 * queued, so stale duplicates are dropped.  Storage is dense arrays rather
 * than a VDB tree: the procedure, not the memory layout, is what is measured.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { NOT_QUEUED = 0, QUEUED = 1 };

typedef struct {
    int nx, ny, nz, dmax;
    int32_t D;
    int64_t n;
    uint8_t* occ;
    int64_t* obst;     /* index of the nearest obstacle, -1 for none */
    int32_t* dist;
    int32_t* raise;    /* -1: not raising; else the key of the raise */
    uint8_t* state;
    /* bucket queue: per key a growable array of cell indices */
    int64_t** bucket;
    int64_t* blen;     /* entries pushed into each key */
    int64_t* bcap;
    int64_t* qhead;    /* entries already popped from each key */
    int32_t cur;       /* smallest key that may be non-empty */
    int64_t size;
    int64_t lowered, raised;
} alg1;

static int qpush(alg1* a, int64_t cell, int32_t key) {
    if (key < 0) key = 0;
    if (key > a->D) key = a->D;
    if (a->blen[key] == a->bcap[key]) {
        int64_t c = a->bcap[key] ? 2 * a->bcap[key] : 16;
        int64_t* p = (int64_t*)realloc(a->bucket[key], (size_t)c * sizeof(int64_t));
        if (!p) return -1;
        a->bucket[key] = p;
        a->bcap[key] = c;
    }
    a->bucket[key][a->blen[key]++] = cell;
    if (key < a->cur) a->cur = key;
    a->size++;
    return 0;
}

/* next cell of the smallest key, first in first out within a key */
static int64_t qpop(alg1* a) {
    while (a->cur <= a->D) {
        const int32_t k = a->cur;
        if (a->qhead[k] < a->blen[k]) {
            a->size--;
            return a->bucket[k][a->qhead[k]++];
        }
        a->blen[k] = 0;
        a->qhead[k] = 0;
        a->cur++;
    }
    return -1;
}

void alg1_destroy(alg1* a);

alg1* alg1_create(int nx, int ny, int nz, int dmax) {
    if (nx < 1 || ny < 1 || nz < 1 || dmax < 1 || dmax > 4095) return NULL;
    alg1* a = (alg1*)calloc(1, sizeof(alg1));
    if (!a) return NULL;
    a->nx = nx; a->ny = ny; a->nz = nz; a->dmax = dmax;
    a->D = dmax * dmax;
    a->n = (int64_t)nx * ny * nz;
    a->occ = (uint8_t*)calloc((size_t)a->n, 1);
    a->obst = (int64_t*)malloc((size_t)a->n * sizeof(int64_t));
    a->dist = (int32_t*)malloc((size_t)a->n * sizeof(int32_t));
    a->raise = (int32_t*)malloc((size_t)a->n * sizeof(int32_t));
    a->state = (uint8_t*)calloc((size_t)a->n, 1);
    a->bucket = (int64_t**)calloc((size_t)a->D + 1, sizeof(int64_t*));
    a->blen = (int64_t*)calloc((size_t)a->D + 1, sizeof(int64_t));
    a->bcap = (int64_t*)calloc((size_t)a->D + 1, sizeof(int64_t));
    a->qhead = (int64_t*)calloc((size_t)a->D + 1, sizeof(int64_t));
    if (!a->occ || !a->obst || !a->dist || !a->raise || !a->state || !a->bucket || !a->blen ||
        !a->bcap || !a->qhead) {
        alg1_destroy(a);
        return NULL;
    }
    /* Initialize: no obstacle, distance at the cap, not raising, not queued */
    for (int64_t i = 0; i < a->n; ++i) {
        a->obst[i] = -1;
        a->dist[i] = a->D;
        a->raise[i] = -1;
    }
    a->cur = a->D + 1;
    return a;
}

void alg1_destroy(alg1* a) {
    if (!a) return;
    if (a->bucket)
        for (int64_t k = 0; k <= a->D; ++k) free(a->bucket[k]);
    free(a->bucket); free(a->blen); free(a->bcap); free(a->qhead);
    free(a->occ); free(a->obst); free(a->dist); free(a->raise); free(a->state);
    free(a);
}

static int64_t idx(const alg1* a, int x, int y, int z) {
    return x + (int64_t)a->nx * (y + (int64_t)a->ny * z);
}

/* SetObstacle: a free cell that is not waiting in the queue becomes its own
   nearest obstacle at distance 0 and starts a lower wave */
void alg1_set_obstacle(alg1* a, int x, int y, int z) {
    const int64_t s = idx(a, x, y, z);
    if (a->occ[s] || a->state[s] == QUEUED) return;
    a->occ[s] = 1;
    a->obst[s] = s;
    a->dist[s] = 0;
    a->raise[s] = -1;
    a->state[s] = QUEUED;
    qpush(a, s, 0);
}

/* RemoveObstacle: an obstacle that is not waiting in the queue loses its
   distance and starts a raise wave */
void alg1_remove_obstacle(alg1* a, int x, int y, int z) {
    const int64_t s = idx(a, x, y, z);
    if (!a->occ[s] || a->state[s] == QUEUED) return;
    a->occ[s] = 0;
    a->obst[s] = -1;
    a->dist[s] = a->D;
    a->raise[s] = 0;
    a->state[s] = QUEUED;
    qpush(a, s, 0);
}

static int32_t sqdist(const alg1* a, int64_t p, int64_t q) {
    const int64_t nxy = (int64_t)a->nx * a->ny;
    const int64_t dx = p % a->nx - q % a->nx;
    const int64_t dy = (p / a->nx) % a->ny - (q / a->nx) % a->ny;
    const int64_t dz = p / nxy - q / nxy;
    const int64_t d = dx * dx + dy * dy + dz * dz;
    return d > a->D ? a->D : (int32_t)d;
}

/* the 26 neighbours of cell s inside the grid */
static int neighbours(const alg1* a, int64_t s, int64_t* out) {
    const int x = (int)(s % a->nx), y = (int)((s / a->nx) % a->ny),
              z = (int)(s / ((int64_t)a->nx * a->ny));
    int k = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                const int u = x + dx, v = y + dy, w = z + dz;
                if (u < 0 || v < 0 || w < 0 || u >= a->nx || v >= a->ny || w >= a->nz) continue;
                out[k++] = idx(a, u, v, w);
            }
    return k;
}

/* Raise: neighbours whose nearest obstacle is gone start raising (their old
   distance is the key) and lose their distance; neighbours with a valid
   obstacle are queued so that they lower the raised area again */
static void raise_cell(alg1* a, int64_t s) {
    int64_t nb[26];
    const int m = neighbours(a, s, nb);
    a->raised++;
    for (int i = 0; i < m; ++i) {
        const int64_t n = nb[i];
        if (a->obst[n] < 0) continue;
        if (!a->occ[a->obst[n]]) {
            a->raise[n] = a->dist[n];
            a->state[n] = QUEUED;
            qpush(a, n, a->dist[n]);
            a->obst[n] = -1;
            a->dist[n] = a->D;
        } else if (a->state[n] != QUEUED) {
            a->state[n] = QUEUED;
            qpush(a, n, a->dist[n]);
        }
    }
    a->raise[s] = -1;
    a->state[s] = NOT_QUEUED;
}

/* Lower: offer the cell's obstacle to each neighbour; a raising neighbour
   whose raise key is no smaller takes it outright, a settled neighbour
   takes it when it is nearer (or equally near while its own obstacle is
   gone) */
static void lower_cell(alg1* a, int64_t s) {
    int64_t nb[26];
    const int m = neighbours(a, s, nb);
    a->lowered++;
    const int64_t ob = a->obst[s];
    if (ob >= 0) {
        for (int i = 0; i < m; ++i) {
            const int64_t n = nb[i];
            const int32_t dn = sqdist(a, ob, n);
            if (a->raise[n] >= dn) {
                a->obst[n] = ob;
                a->dist[n] = dn;
                a->raise[n] = -1;
                a->state[n] = QUEUED;
                qpush(a, n, dn);
            } else if (a->raise[n] < 0) {
                const int gone = a->obst[n] < 0 || !a->occ[a->obst[n]];
                if (dn < a->dist[n] || (dn == a->dist[n] && gone)) {
                    a->obst[n] = ob;
                    a->dist[n] = dn;
                    a->raise[n] = -1;
                    if (dn < a->D) {
                        a->state[n] = QUEUED;
                        qpush(a, n, dn);
                    }
                }
            }
        }
    }
    a->raise[s] = -1;
    a->state[s] = NOT_QUEUED;
}

/* DistanceTransform: process the queue in key order; counts[0] and
   counts[1] receive the cells lowered and raised by this call */
void alg1_transform(alg1* a, int64_t* counts) {
    a->lowered = a->raised = 0;
    for (;;) {
        const int64_t s = qpop(a);
        if (s < 0) break;
        if (a->state[s] != QUEUED) continue;
        if (a->raise[s] >= 0) raise_cell(a, s);
        else lower_cell(a, s);
    }
    if (counts) {
        counts[0] = a->lowered;
        counts[1] = a->raised;
    }
}

/* the distance field (squared, capped at D), x fastest */
void alg1_read(const alg1* a, int32_t* out) {
    memcpy(out, a->dist, (size_t)a->n * sizeof(int32_t));
}

/* SetObstacle / RemoveObstacle for n entries (x, y, z) with target states,
   in order; entries outside the grid are ignored */
void alg1_apply(alg1* a, const int32_t* xyz, const uint8_t* state, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (x < 0 || y < 0 || z < 0 || x >= a->nx || y >= a->ny || z >= a->nz) continue;
        if (state[i]) alg1_set_obstacle(a, x, y, z);
        else alg1_remove_obstacle(a, x, y, z);
    }
}
