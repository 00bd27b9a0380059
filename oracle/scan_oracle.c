/*
 * oracle/scan_oracle.c -- CPU oracle for the occupancy integration of a range
 * scan.  TEST INFRASTRUCTURE ONLY, like edt_oracle.c: it shares no code with
 * the HIP path.
 *
 * The mapping step in front of the transform in the paper's online pipeline
 * (section V-B integrates LIDAR range scans into an occupancy grid before
 * each distance-field update).  The paper fixes no traversal rule; the
 * reading used here: a ray from sensor voxel o to end voxel e visits o and
 * then, walking along the segment between the two voxel centres, every voxel
 * it enters through a face, one axis step at a time.  The next step is taken
 * on the axis whose next face crossing comes first along the segment; the
 * i-th crossing (i = 0, 1, ...) on axis a lies at parameter
 * (2i + 1) / (2 |e_a - o_a|), and equal parameters are taken in the order
 * x, y, z.  This is the voxel walk of Amanatides and Woo done in exact
 * integer arithmetic (parameters compared by cross-multiplication).
 *
 * One scan: every visited voxel of every ray becomes free, except the end
 * voxel of a ray with a return ("hit"), which becomes occupied; a hit wins
 * over any ray passing through the same voxel.  Rays with an endpoint
 * outside the grid are skipped.
 */
#include <stdint.h>
#include <stdlib.h>

typedef void (*visit_fn)(const int v[3], void* ctx);

/* The sequential walk: visits o, then each voxel entered, ending at e. */
static void ray_walk(const int o[3], const int e[3], visit_fn visit, void* ctx) {
    int v[3], step[3], ad[3], c[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        v[a] = o[a];
        const int d = e[a] - o[a];
        step[a] = d < 0 ? -1 : 1;
        ad[a] = d < 0 ? -d : d;
    }
    visit(v, ctx);
    for (;;) {
        int best = -1;
        for (int a = 0; a < 3; ++a) {
            if (c[a] >= ad[a]) continue;
            /* crossing parameter of axis a is (2 c_a + 1) / (2 ad_a); take a
               if it is strictly earlier than the best so far */
            if (best < 0 || (int64_t)(2 * c[a] + 1) * ad[best] <
                                (int64_t)(2 * c[best] + 1) * ad[a])
                best = a;
        }
        if (best < 0) break;
        c[best] += 1;
        v[best] += step[best];
        visit(v, ctx);
    }
}

struct collect { int32_t* out; int64_t n, cap; };

static void collect_visit(const int v[3], void* p) {
    struct collect* c = (struct collect*)p;
    if (c->n < c->cap) {
        c->out[3 * c->n] = v[0];
        c->out[3 * c->n + 1] = v[1];
        c->out[3 * c->n + 2] = v[2];
    }
    c->n += 1;
}

/* The voxels of one ray in walk order into out[cap][3]; returns their count
 * (|dx| + |dy| + |dz| + 1), which may exceed cap (then out holds the first
 * cap voxels). */
int64_t oracle_ray_voxels(const int32_t* o, const int32_t* e, int32_t* out, int64_t cap) {
    int oo[3] = {o[0], o[1], o[2]}, ee[3] = {e[0], e[1], e[2]};
    struct collect c = {out, 0, cap};
    ray_walk(oo, ee, collect_visit, &c);
    return c.n;
}

struct mark { uint8_t* m; int nx, ny; };

static void mark_free(const int v[3], void* p) {
    struct mark* k = (struct mark*)p;
    uint8_t* cell = k->m + v[0] + (int64_t)k->nx * (v[1] + (int64_t)k->ny * v[2]);
    if (*cell == 0) *cell = 1;
}

/* Integrates one scan into occ (uint8, x fastest, updated in place):
 * origin int32[3], ends int32[n][3], hits uint8[n].  Returns the number of
 * rays skipped for an endpoint outside the grid, or -1 on bad arguments. */
int64_t oracle_integrate_scan(uint8_t* occ, int nx, int ny, int nz, const int32_t* origin,
                              const int32_t* ends, const uint8_t* hits, int64_t n) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || n < 0) return -1;
    const int64_t nv = (int64_t)nx * ny * nz;
    uint8_t* m = (uint8_t*)calloc((size_t)nv, 1);   /* 0 untouched, 1 free, 2 hit */
    if (!m) return -1;
    const int o[3] = {origin[0], origin[1], origin[2]};
    const int ext[3] = {nx, ny, nz};
    int o_in = 1;
    for (int a = 0; a < 3; ++a) o_in = o_in && o[a] >= 0 && o[a] < ext[a];
    int64_t skipped = 0;
    struct mark k = {m, nx, ny};
    for (int64_t r = 0; r < n; ++r) {
        const int e[3] = {ends[3 * r], ends[3 * r + 1], ends[3 * r + 2]};
        int in = o_in;
        for (int a = 0; a < 3; ++a) in = in && e[a] >= 0 && e[a] < ext[a];
        if (!in) { ++skipped; continue; }
        ray_walk(o, e, mark_free, &k);
    }
    /* the end voxel of a hit is occupied, whatever other rays did there */
    for (int64_t r = 0; r < n; ++r) {
        if (!hits[r]) continue;
        const int e[3] = {ends[3 * r], ends[3 * r + 1], ends[3 * r + 2]};
        int in = o_in;
        for (int a = 0; a < 3; ++a) in = in && e[a] >= 0 && e[a] < ext[a];
        if (in) m[e[0] + (int64_t)nx * (e[1] + (int64_t)ny * e[2])] = 2;
    }
    /* the walk marks a hit ray's own end voxel free too; the hit pass above
       overrides it, so only voxels never hit end up free */
    for (int64_t i = 0; i < nv; ++i) {
        if (m[i] == 1) occ[i] = 0;
        else if (m[i] == 2) occ[i] = 1;
    }
    free(m);
    return skipped;
}
