// edt_api.hip -- host runtime and C ABI of libedt (see include/edt.h).
//
// The host side owns no device memory: edt_create carves the caller's
// workspace into the block pool, the block hash table, work lists and the
// update scratch; every entry point only enqueues kernels on the caller's
// stream.  Kernels whose amount of work is only known on the device (block
// counts, list lengths) run on fixed grids and read their counts from device
// counters, so no call waits on the GPU except edt_get_stats / edt_get_error.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include "edt.h"

// The kernels live in one translation unit with their launches.
#include "edt_kernels.hip"

using namespace edt;

constexpr int NPHASE = 6;   // ingest, region, items, pass_x, pass_y, pass_z

struct edt_ctx {
    edt_config cfg;
    Grid g;
    hipEvent_t* ev;     // timing events, (NPHASE + 1) per recorded call
    int ev_calls;       // calls to record
    int ev_used;        // calls recorded so far
    int ev_phase;       // phase bracketed by the events, or -1 for all of them
    int cap;            // envelope ring capacity (entries per lane)
    size_t env_lds;     // dynamic LDS bytes of the envelope passes
    int64_t tcap;       // tile hash capacity
    int64_t ucap;       // update hash capacity
    int64_t stats_host[C_N];
    bool interior_valid;   // edt_interior ran after the last global / update
    int32_t* scan_xyz;     // change list built by edt_integrate_scan
    uint8_t* scan_state;
    int32_t* scan_cnt;     // [0] free entries, [1] hit entries, [2] list length,
                           // [3] finished workgroups of the hit kernel, [4..5] int64
                           // number of visited-voxel slots
    int64_t* scan_off;     // per ray: first slot within its group of 1024 rays
    int64_t* scan_blk;     // per group of 1024 rays: slot total, then first slot
};

namespace {

int64_t next_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

struct Layout {
    int64_t max_blocks, max_changes, max_int, tcap, ucap;
    int64_t off[40];
    int64_t total;
};

enum {
    O_TKEYS, O_TSLOTS, O_BKEY, O_OCC, O_G1, O_G2, O_S, O_BMAX, O_FLAGS, O_CNT,
    O_YI, O_ZI, O_SEED, O_DIRTY, O_XS, O_YS, O_NEWDIL, O_CHGA, O_CHGR,
    O_UKEYS, O_UVALS, O_UPOS, O_DUMMY, O_DBLOCK, O_TOBST, O_TLIST, O_BMIN, O_TINFO, O_TFLAG, O_IIDX, O_ILIST, O_IC1, O_IC2, O_SCANXYZ, O_SCANST, O_SCANCNT, O_SCANOFF, O_SCANBLK, O_N
};

bool valid_cfg(const edt_config* c) {
    if (!c) return false;
    const int32_t lim = 1 << 20;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1 || c->nx > lim || c->ny > lim || c->nz > lim)
        return false;
    if (c->d_max < 1 || c->d_max > 255) return false;
    if (c->max_blocks < 0 || c->max_changes < 0 || c->max_interior_blocks < 0) return false;
    return true;
}

bool layout_of(const edt_config* c, Layout* L) {
    if (!valid_cfg(c)) return false;
    const int64_t nbx = (c->nx + 7) / 8, nby = (c->ny + 7) / 8, nbz = (c->nz + 7) / 8;
    int64_t mb = c->max_blocks ? c->max_blocks : nbx * nby * nbz;
    if (mb > nbx * nby * nbz) mb = nbx * nby * nbz;
    if (mb > (1 << 22)) return false;                   // slot*512 stays in int32
    const int64_t mc = c->max_changes ? c->max_changes : (1 << 20);
    if (mc > (1 << 28)) return false;
    const int64_t mi = c->max_interior_blocks < mb ? c->max_interior_blocks : mb;
    L->max_blocks = mb;
    L->max_changes = mc;
    L->max_int = mi;
    // tiles of 8x8x8 blocks: at most one per tile of the extent and one per block
    const int64_t ntx = (nbx + 7) / 8, nty = (nby + 7) / 8, ntz = (nbz + 7) / 8;
    int64_t tiles = ntx * nty * ntz;
    if (tiles > mb) tiles = mb;
    L->tcap = next_pow2(tiles * 2 < 64 ? 64 : tiles * 2);
    if (L->tcap > (1 << 24)) return false;
    L->ucap = next_pow2(mc * 2 < 64 ? 64 : mc * 2);
    const int64_t sz[O_N] = {
        L->tcap * 8, L->tcap * 2048, mb * 8, mb * 64, mb * 1024, mb * 1024, mb * 1024, mb * 4,
        mb * 4, 64 * 4,
        mb * 4, mb * 4, mb * 4, mb * 4, mb * 4, mb * 4, mb * 4, mb * 64, mb * 64,
        L->ucap * 8, L->ucap * 4, mc * 4, 256 * 256 * 4 + 1024, 1024,
        L->tcap * 64, L->tcap * 4, mb * 4, L->tcap * 32, L->tcap * 4,
        mi ? mb * 4 : 0, mi * 4, mi * 1024, mi * 1024, mc * 12, mc, 256, mc * 8, (mc / 1024 + 1) * 16};
    int64_t o = 0;
    for (int i = 0; i < O_N; ++i) {
        L->off[i] = o;
        o += (sz[i] + 255) & ~(int64_t)255;
    }
    L->total = o;
    return true;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// Workgroups of the dense readbacks: strips of RB_BLOCKS blocks along x per
// block row (at most the number of blocks, checked by the callers).
inline int64_t read_strips(const Grid& g) {
    return (int64_t)((g.nbx + RB_BLOCKS - 1) / RB_BLOCKS) * g.nby * g.nbz;
}

// Event k of the current timed call (no-op unless timing is armed).
inline void mark(edt_ctx* c, int k, hipStream_t st) {
    if (c->ev && c->ev_used < c->ev_calls &&
        (c->ev_phase < 0 || k == c->ev_phase || k == c->ev_phase + 1))
        (void)hipEventRecord(c->ev[c->ev_used * (NPHASE + 1) + k], st);
}

void free_events(edt_ctx* c) {
    if (!c->ev) return;
    for (int i = 0; i < c->ev_calls * (NPHASE + 1); ++i) (void)hipEventDestroy(c->ev[i]);
    free(c->ev);
    c->ev = nullptr;
    c->ev_calls = c->ev_used = 0;
}

inline int grid_for(int64_t work, int per, int cap) {
    int64_t g = (work + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

#define LAUNCH_CHECK()                                   \
    do {                                                 \
        if (hipGetLastError() != hipSuccess) return EDT_ERR_HIP; \
    } while (0)

// Pass along y (axis 1) or z (axis 2) over the item list of that axis.
// d_max <= 64: windowed minimum (one instantiation per block radius);
// larger radii: streaming lower envelope.
template <int AXIS>
void launch_win(const Grid& g, int grid, hipStream_t st, const int32_t* items, int counter,
                uint32_t runflag) {
    switch (g.R) {
#define EDT_WIN_CASE(m)                                                                     \
    case m:                                                                                \
        hipLaunchKernelGGL((k_pass_win<m, AXIS>), dim3(grid), dim3(64), 0, st, g, items, counter, \
                           runflag);                                                       \
        break;
        EDT_WIN_CASE(1) EDT_WIN_CASE(2) EDT_WIN_CASE(3) EDT_WIN_CASE(4)
        EDT_WIN_CASE(5) EDT_WIN_CASE(6) EDT_WIN_CASE(7) EDT_WIN_CASE(8)
#undef EDT_WIN_CASE
        default: break;
    }
}

void launch_pass(edt_ctx* c, const Grid& g, int axis, hipStream_t st, const int32_t* items,
                 int counter, uint32_t runflag) {
    const int grid = grid_for(g.max_blocks, 1, 8192);
    if (g.R <= 8) {
        if (axis == 1) launch_win<1>(g, grid, st, items, counter, runflag);
        else launch_win<2>(g, grid, st, items, counter, runflag);
    } else if (axis == 1) {
        hipLaunchKernelGGL(k_pass_y, dim3(grid), dim3(64), c->env_lds, st, g, items, counter,
                           runflag, c->cap);
    } else {
        hipLaunchKernelGGL(k_pass_z, dim3(grid), dim3(64), c->env_lds, st, g, items, counter,
                           runflag, c->cap);
    }
}

// Tile forms of the three passes for d_max <= 64 (block radius M = R <= 8).
template <int M>
void launch_tile_passes(edt_ctx* c, hipStream_t st) {
    const Grid& g = c->g;
    const int grid = grid_for(c->tcap * 64, 1, 16384);
    hipLaunchKernelGGL(k_pass_x_rows<M>, dim3(grid), dim3(64), 0, st, g);
    mark(c, 4, st);
    hipLaunchKernelGGL((k_pass_win_tiles<M, 1>), dim3(grid), dim3(64), 0, st, g);
    mark(c, 5, st);
    hipLaunchKernelGGL((k_pass_win_tiles<M, 2>), dim3(grid), dim3(64), 0, st, g);
    mark(c, 6, st);
}

// Passes of the global transform.  d_max <= 64 runs the tile forms (no
// work-item lists); larger radii build the y/z item lists per tile and run
// the list-driven passes.
edt_status run_passes_global(edt_ctx* c, hipStream_t st) {
    Grid& g = c->g;
    const int mb = g.max_blocks;
    if (g.R <= 8) {
        mark(c, 3, st);
        switch (g.R) {
#define EDT_TP_CASE(m) \
    case m: launch_tile_passes<m>(c, st); break;
            EDT_TP_CASE(1) EDT_TP_CASE(2) EDT_TP_CASE(3) EDT_TP_CASE(4)
            EDT_TP_CASE(5) EDT_TP_CASE(6) EDT_TP_CASE(7) EDT_TP_CASE(8)
#undef EDT_TP_CASE
            default: break;
        }
    } else {
        hipLaunchKernelGGL(k_items_tiles, dim3(grid_for(c->tcap, 1, 8192)), dim3(64), 0, st, g);
        mark(c, 3, st);
        hipLaunchKernelGGL(k_pass_x, dim3(grid_for(mb, 1, 16384)), dim3(64), 0, st, g,
                           (const int32_t*)nullptr, 0);
        mark(c, 4, st);
        launch_pass(c, g, 1, st, g.list_yi, (int)C_NYI, 0u);
        mark(c, 5, st);
        launch_pass(c, g, 2, st, g.list_zi, (int)C_NZI, 0u);
        mark(c, 6, st);
    }
    if (c->ev && c->ev_used < c->ev_calls) c->ev_used++;
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status dilate_region(edt_ctx* c, hipStream_t st) {
    Grid& g = c->g;
    const int TR = (g.R + 7) / 8, w = 2 * TR + 1;
    const int E = 8 + 2 * g.R;
    const size_t lds = (size_t)w * w * w * 64 + E * E + E * 8 + 64;
    const dim3 grid(grid_for(c->tcap, 1, 4096));
    switch (g.R) {
#define EDT_DIL_CASE(r) \
    case r: hipLaunchKernelGGL(k_tile_dilate<r>, grid, dim3(64), lds, st, g); break;
        EDT_DIL_CASE(1) EDT_DIL_CASE(2) EDT_DIL_CASE(3) EDT_DIL_CASE(4)
        EDT_DIL_CASE(5) EDT_DIL_CASE(6) EDT_DIL_CASE(7) EDT_DIL_CASE(8)
#undef EDT_DIL_CASE
        default: hipLaunchKernelGGL(k_tile_dilate<0>, grid, dim3(64), lds, st, g); break;
    }
    LAUNCH_CHECK();
    return EDT_OK;
}

}  // namespace

// Points the context's grid at the regions of workspace b for layout L.
static void bind_workspace(edt_ctx* c, const edt_config* cfg, const Layout& L, char* b) {
    c->cfg = *cfg;
    c->tcap = L.tcap;
    c->ucap = L.ucap;
    Grid& g = c->g;
    g.nx = cfg->nx; g.ny = cfg->ny; g.nz = cfg->nz;
    g.nbx = (cfg->nx + 7) / 8; g.nby = (cfg->ny + 7) / 8; g.nbz = (cfg->nz + 7) / 8;
    g.dmax = cfg->d_max;
    g.D = cfg->d_max * cfg->d_max;
    g.R = (cfg->d_max + 7) / 8;
    g.max_blocks = (int)L.max_blocks;
    g.lrun = LRUN;
    g.tmask = (uint32_t)(L.tcap - 1);
    g.umask = (uint32_t)(L.ucap - 1);
    g.max_changes = (int)L.max_changes;
    g.tkeys = (unsigned long long*)(b + L.off[O_TKEYS]);
    g.tslots = (int32_t*)(b + L.off[O_TSLOTS]);
    g.bkey = (unsigned long long*)(b + L.off[O_BKEY]);
    g.occ = (uint32_t*)(b + L.off[O_OCC]);
    g.g1 = (uint16_t*)(b + L.off[O_G1]);
    g.g2 = (uint16_t*)(b + L.off[O_G2]);
    g.s = (uint16_t*)(b + L.off[O_S]);
    g.bmax = (int32_t*)(b + L.off[O_BMAX]);
    g.flags = (uint32_t*)(b + L.off[O_FLAGS]);
    g.cnt = (int32_t*)(b + L.off[O_CNT]);
    g.list_yi = (int32_t*)(b + L.off[O_YI]);
    g.list_zi = (int32_t*)(b + L.off[O_ZI]);
    g.list_seed = (int32_t*)(b + L.off[O_SEED]);
    g.list_dirty = (int32_t*)(b + L.off[O_DIRTY]);
    g.list_xs = (int32_t*)(b + L.off[O_XS]);
    g.list_ys = (int32_t*)(b + L.off[O_YS]);
    g.list_newdil = (int32_t*)(b + L.off[O_NEWDIL]);
    g.chg_add = (uint32_t*)(b + L.off[O_CHGA]);
    g.chg_rem = (uint32_t*)(b + L.off[O_CHGR]);
    g.ukeys = (unsigned long long*)(b + L.off[O_UKEYS]);
    g.uvals = (int32_t*)(b + L.off[O_UVALS]);
    g.upos = (int32_t*)(b + L.off[O_UPOS]);
    g.dummy = (uint32_t*)(b + L.off[O_DUMMY]);
    g.dblock = (uint16_t*)(b + L.off[O_DBLOCK]);
    g.tobst = (uint32_t*)(b + L.off[O_TOBST]);
    g.tlist = (int32_t*)(b + L.off[O_TLIST]);
    g.tinfo = (int32_t*)(b + L.off[O_TINFO]);
    g.tflag = (int32_t*)(b + L.off[O_TFLAG]);
    g.bmin1 = (uint16_t*)(b + L.off[O_BMIN]);
    g.bmin2 = g.bmin1 + L.max_blocks;
    g.max_int = (int)L.max_int;
    g.iidx = (int32_t*)(b + L.off[O_IIDX]);
    g.ilist = (int32_t*)(b + L.off[O_ILIST]);
    g.ic1 = (uint16_t*)(b + L.off[O_IC1]);
    g.ic2 = (uint16_t*)(b + L.off[O_IC2]);
    c->scan_xyz = (int32_t*)(b + L.off[O_SCANXYZ]);
    c->scan_state = (uint8_t*)(b + L.off[O_SCANST]);
    c->scan_cnt = (int32_t*)(b + L.off[O_SCANCNT]);
    c->scan_off = (int64_t*)(b + L.off[O_SCANOFF]);
    c->scan_blk = (int64_t*)(b + L.off[O_SCANBLK]);
}

// Enqueues the initial state of a freshly bound workspace: empty tile and
// dedupe tables, zero counters, the block of D values.
static edt_status init_workspace(edt_ctx* c, const Layout& L, hipStream_t st) {
    const Grid& g = c->g;
    hipLaunchKernelGGL(k_begin_global, dim3(grid_for(L.tcap * 128, 256, 4096)), dim3(256), 0, st,
                       g, L.tcap);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(L.ucap, 256, 4096)), dim3(256), 0, st, g.ukeys,
                       L.ucap, KEY_EMPTY);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(L.ucap, 256, 4096)), dim3(256), 0, st, g.uvals,
                       L.ucap, -1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, g.cnt, (int64_t)64, 0);
    // the block of D values that the window passes read for absent blocks of
    // g1 / g2, in their representation (binary16 for small radii)
    const uint32_t dw = win_f16(g.R) ? f16_bits((uint32_t)g.D) : (uint32_t)g.D;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, (int32_t*)g.dblock, (int64_t)256,
                       (int32_t)(dw | (dw << 16)));
    return hipGetLastError() == hipSuccess ? EDT_OK : EDT_ERR_HIP;
}

// Rebuilds the pool of c from a device list of blocks holding an obstacle
// (int32 coordinates and 64 bytes of occupancy bits each; *count entries, at
// most nmax) and recomputes the field: the global transform of that map.
static edt_status rebuild_from_list(edt_ctx* c, const int32_t* count, const int32_t* lxyz,
                                    const uint8_t* lbits, int64_t nmax, hipStream_t st) {
    Grid& g = c->g;
    c->interior_valid = false;
    mark(c, 0, st);
    hipLaunchKernelGGL(k_begin_global, dim3(grid_for(c->tcap * 128, 256, 4096)), dim3(256), 0, st,
                       g, c->tcap);
    const int grid = grid_for((nmax + 7) / 8, 1, 16384);
    hipLaunchKernelGGL(k_ingest_blocks_mark<true>, dim3(grid), dim3(64), 0, st, g, lxyz, lbits,
                       (int64_t)0, count);
    mark(c, 1, st);
    edt_status r = dilate_region(c, st);
    if (r) return r;
    hipLaunchKernelGGL(k_ingest_blocks_write<true>, dim3(grid), dim3(64), 0, st, g, lxyz, lbits,
                       (int64_t)0, count);
    mark(c, 2, st);
    LAUNCH_CHECK();
    return run_passes_global(c, st);
}

extern "C" {

const char* edt_status_str(int s) {
    switch (s) {
        case EDT_OK: return "EDT_OK";
        case EDT_ERR_ARG: return "EDT_ERR_ARG";
        case EDT_ERR_RANGE: return "EDT_ERR_RANGE";
        case EDT_ERR_CAPACITY: return "EDT_ERR_CAPACITY";
        case EDT_ERR_HIP: return "EDT_ERR_HIP";
        case EDT_ERR_STATE: return "EDT_ERR_STATE";
        default: return "EDT_UNKNOWN";
    }
}

int64_t edt_workspace_bytes(const edt_config* cfg) {
    Layout L;
    if (!layout_of(cfg, &L)) return EDT_ERR_ARG;
    return L.total;
}

edt_status edt_create(const edt_config* cfg, void* d_ws, int64_t ws_bytes, void* stream,
                      edt_ctx** out) {
    if (!out) return EDT_ERR_ARG;
    *out = nullptr;
    Layout L;
    if (!layout_of(cfg, &L) || !d_ws) return EDT_ERR_ARG;
    if (((uintptr_t)d_ws & 255) != 0) return EDT_ERR_ARG;
    if (ws_bytes < L.total) return EDT_ERR_CAPACITY;
    edt_ctx* c = (edt_ctx*)calloc(1, sizeof(edt_ctx));
    if (!c) return EDT_ERR_CAPACITY;
    char* b = (char*)d_ws;
    bind_workspace(c, cfg, L, b);
    Grid& g = c->g;
    c->cap = 2 * g.dmax + 4;   // live envelope sites never exceed 2 * d_max + 2
    c->env_lds = (96 + 24) * 4 + (size_t)c->cap * 64 * 4;
    // the envelope ring must fit the device's LDS per workgroup
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess) {
        free(c);
        return EDT_ERR_HIP;
    }
    if ((int64_t)c->env_lds > lds_max) {
        free(c);
        return EDT_ERR_ARG;
    }
    if (c->env_lds > 65536) {
        if (hipFuncSetAttribute((const void*)k_pass_y, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)c->env_lds) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_pass_z, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)c->env_lds) != hipSuccess) {
            free(c);
            return EDT_ERR_HIP;
        }
    }

    const edt_status e = init_workspace(c, L, S(stream));
    if (e != EDT_OK) {
        free(c);
        return e;
    }
    *out = c;
    return EDT_OK;
}

edt_status edt_destroy(edt_ctx* ctx) {
    if (!ctx) return EDT_ERR_ARG;
    free_events(ctx);
    free(ctx);
    return EDT_OK;
}

edt_status edt_timing_begin(edt_ctx* c, int32_t n_calls) {
    return edt_timing_begin_phase(c, n_calls, -1);
}

edt_status edt_timing_begin_phase(edt_ctx* c, int32_t n_calls, int32_t phase) {
    if (!c || n_calls < 0 || n_calls > 100000 || phase < -1 || phase >= NPHASE)
        return EDT_ERR_ARG;
    free_events(c);
    c->ev_phase = phase;
    if (n_calls == 0) return EDT_OK;
    const int ne = n_calls * (NPHASE + 1);
    c->ev = (hipEvent_t*)calloc((size_t)ne, sizeof(hipEvent_t));
    if (!c->ev) return EDT_ERR_CAPACITY;
    for (int i = 0; i < ne; ++i) {
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->ev[j]);
            free(c->ev);
            c->ev = nullptr;
            return EDT_ERR_HIP;
        }
    }
    c->ev_calls = n_calls;
    c->ev_used = 0;
    return EDT_OK;
}

edt_status edt_timing_read(edt_ctx* c, float* ms, int32_t* n_recorded) {
    if (!c || !ms || !n_recorded) return EDT_ERR_ARG;
    for (int k = 0; k < NPHASE; ++k) ms[k] = 0.0f;
    *n_recorded = c->ev_used;
    for (int i = 0; i < c->ev_used; ++i) {
        hipEvent_t* e = c->ev + i * (NPHASE + 1);
        if (hipEventSynchronize(e[NPHASE]) != hipSuccess) return EDT_ERR_HIP;
        for (int k = 0; k < NPHASE; ++k) {
            if (c->ev_phase >= 0 && k != c->ev_phase) continue;
            float t = 0.0f;
            if (hipEventElapsedTime(&t, e[k], e[k + 1]) != hipSuccess) return EDT_ERR_HIP;
            ms[k] += t / (float)c->ev_used;
        }
    }
    return EDT_OK;
}

edt_status edt_global(edt_ctx* c, const edt_map* map, void* stream) {
    if (!c || !map) return EDT_ERR_ARG;
    Grid& g = c->g;
    hipStream_t st = S(stream);
    if (map->kind == EDT_MAP_DENSE) {
        if (!map->d_occ) return EDT_ERR_ARG;
        // one workgroup per strip of 8 blocks along x (a one-dimensional grid)
        if ((int64_t)((g.nbx + 7) / 8) * g.nby * g.nbz > 0x7fffffff) return EDT_ERR_ARG;
    } else if (map->kind == EDT_MAP_BLOCKS) {
        if (map->n_blocks < 0) return EDT_ERR_ARG;
        if (map->n_blocks > 0 && (!map->d_block_xyz || !map->d_block_occ)) return EDT_ERR_ARG;
    } else {
        return EDT_ERR_ARG;
    }
    c->interior_valid = false;
    mark(c, 0, st);
    hipLaunchKernelGGL(k_begin_global, dim3(grid_for(c->tcap * 128, 256, 4096)), dim3(256), 0, st,
                       g, c->tcap);
    if (map->kind == EDT_MAP_DENSE) {
        // obstacle blocks get their slots and occupancy here, the dilation
        // adds (and zeroes) the rest of the region
        const int64_t strips = (int64_t)((g.nbx + 7) / 8) * g.nby * g.nbz;
        hipLaunchKernelGGL(k_ingest_dense, dim3((unsigned)strips), dim3(64), 0, st, g,
                           map->d_occ);
        mark(c, 1, st);
        edt_status r = dilate_region(c, st);
        if (r) return r;
        mark(c, 2, st);
    } else {
        // obstacle blocks are only marked in their tiles; the dilation
        // creates (and zeroes) every slot of the region, then the bits are
        // ORed in
        const int64_t n = map->n_blocks;
        if (n > 0)
            hipLaunchKernelGGL(k_ingest_blocks_mark<false>, dim3(grid_for((n + 7) / 8, 1, 16384)),
                               dim3(64), 0, st, g, map->d_block_xyz, map->d_block_occ, n,
                               (const int32_t*)nullptr);
        mark(c, 1, st);
        edt_status r = dilate_region(c, st);
        if (r) return r;
        if (n > 0)
            hipLaunchKernelGGL(k_ingest_blocks_write<false>, dim3(grid_for((n + 7) / 8, 1, 16384)),
                               dim3(64), 0, st, g, map->d_block_xyz, map->d_block_occ, n,
                               (const int32_t*)nullptr);
        mark(c, 2, st);
    }
    LAUNCH_CHECK();
    return run_passes_global(c, st);
}

edt_status edt_compact(edt_ctx* c, void* stream) {
    if (!c) return EDT_ERR_ARG;
    Grid& g = c->g;
    hipStream_t st = S(stream);
    // the list lives in the g1 storage (rewritten by the passes that follow):
    // 12 bytes of coordinates and 64 bytes of occupancy per block; the count
    // in the first word of g2 (rewritten by the passes too)
    const int64_t mb = g.max_blocks;
    int32_t* count = (int32_t*)g.g2;
    int32_t* lxyz = (int32_t*)g.g1;
    uint8_t* lbits = (uint8_t*)g.g1 + ((12 * mb + 255) & ~(int64_t)255);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, count, (int64_t)1, 0);
    hipLaunchKernelGGL(k_compact_gather, dim3(grid_for(mb, 256, 16384)), dim3(64), 0, st, g, count,
                       lxyz, (uint32_t*)lbits);
    return rebuild_from_list(c, count, lxyz, lbits, mb, st);
}

edt_status edt_grow(edt_ctx* c, int64_t max_blocks, void* d_ws, int64_t ws_bytes, void* stream) {
    if (!c || !d_ws || ((uintptr_t)d_ws & 255) != 0) return EDT_ERR_ARG;
    edt_config cfg = c->cfg;
    cfg.max_blocks = max_blocks;
    Layout L;
    if (!layout_of(&cfg, &L)) return EDT_ERR_ARG;
    if (L.max_blocks < c->g.max_blocks) return EDT_ERR_ARG;   // the pool never shrinks here
    if (ws_bytes < L.total) return EDT_ERR_CAPACITY;
    hipStream_t st = S(stream);
    const Grid o = c->g;
    edt_ctx n = *c;              // timing events, call number, envelope sizes carry over
    bind_workspace(&n, &cfg, L, (char*)d_ws);
    edt_status e = init_workspace(&n, L, st);
    if (e != EDT_OK) return e;
    const Grid& g = n.g;
    // tile tables: rehashed into the new capacity; the position map lives in
    // the new g1 storage until g1 is copied below (stream order)
    int32_t* map = (int32_t*)g.g1;
    hipLaunchKernelGGL(k_tile_rehash, dim3(grid_for(c->tcap, 1, 8192)), dim3(64), 0, st, o, g, map);
    hipLaunchKernelGGL(k_tile_remap, dim3(grid_for(c->tcap, 256, 1024)), dim3(256), 0, st, o, g,
                       (const int32_t*)map);
    // per-slot state of the old pool's slots: the same slot numbers
    const int64_t mb = o.max_blocks;
    struct { void* dst; const void* src; int64_t bytes; } cp[] = {
        {g.bkey, o.bkey, mb * 8},       {g.occ, o.occ, mb * 64},
        {g.g1, o.g1, mb * 1024},        {g.g2, o.g2, mb * 1024},
        {g.s, o.s, mb * 1024},          {g.bmax, o.bmax, mb * 4},
        {g.flags, o.flags, mb * 4},     {g.chg_add, o.chg_add, mb * 64},
        {g.chg_rem, o.chg_rem, mb * 64}, {g.bmin1, o.bmin1, mb * 2},
        {g.bmin2, o.bmin2, mb * 2},     {g.cnt, o.cnt, (int64_t)C_N * 4},
    };
    for (const auto& x : cp)
        if (hipMemcpyAsync(x.dst, x.src, (size_t)x.bytes, hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
            return EDT_ERR_HIP;
    hipLaunchKernelGGL(k_grow_counts, dim3(1), dim3(1), 0, st, g, (int32_t)mb);
    LAUNCH_CHECK();
    n.interior_valid = false;
    *c = n;                      // from here on the context lives in the new workspace
    return EDT_OK;
}

// The incremental transform over n change entries; n_dev, when given, holds
// the entry count on the device and n is then only its upper bound (grids).
static edt_status run_update(edt_ctx* c, const int32_t* d_xyz, const uint8_t* d_state,
                             int64_t n, const int32_t* n_dev, hipStream_t st) {
    c->interior_valid = false;
    Grid& g = c->g;
    const int mb = g.max_blocks;
    // every update kernel loops grid-stride; a device-side count only bounds
    // n, so its grids stay moderate
    const int tn = grid_for(n_dev && n > 65536 ? 65536 : n, 256, 4096);
    const int w3 = (2 * g.R + 1) * (2 * g.R + 1) * (2 * g.R + 1);
    // dedupe, and every block the call needs exists before any occupancy
    // changes
    hipLaunchKernelGGL(k_upd_dedupe_alloc, dim3(tn), dim3(256), 0, st, g, d_xyz, d_state, n, n_dev);
    // occupancy changes and the dilation of the listed blocks in one launch
    const int td = grid_for((int64_t)n * w3, 256, 4096);
    hipLaunchKernelGGL(k_upd_apply_dilate, dim3(tn + td), dim3(256), 0, st, g, d_xyz, d_state, n,
                       n_dev, tn);
    // fronts: one workgroup per seed block (at most one per change entry),
    // wide enough for the seed's whole neighbourhood when it has at most 1024
    // blocks
    const int fwg = w3 <= 256 ? 256 : (w3 <= 512 ? 512 : 1024);
    hipLaunchKernelGGL(k_upd_fronts, dim3(grid_for(n, 1, 4096)), dim3(fwg), 0, st, g);
    // short work items: the recompute sets are small, and short runs give
    // more waves to hide each item's latency
    Grid gu = g;
    gu.lrun = 2;
    const int nxw = grid_for(mb, 1, 2048);
    hipLaunchKernelGGL(k_upd_x_items, dim3(nxw + grid_for(2 * (int64_t)mb + 64, 64, 2048)), dim3(64),
                       0, st, gu, nxw);
    launch_pass(c, gu, 1, st, g.list_yi, (int)C_NYI, (uint32_t)F_YS);
    launch_pass(c, gu, 2, st, g.list_zi, (int)C_NZI, (uint32_t)F_DIRTY);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_update(edt_ctx* c, const int32_t* d_xyz, const uint8_t* d_state, int64_t n,
                      void* stream) {
    if (!c || n < 0) return EDT_ERR_ARG;
    if (n == 0) return EDT_OK;
    if (!d_xyz || !d_state) return EDT_ERR_ARG;
    if (n > c->g.max_changes) return EDT_ERR_CAPACITY;
    return run_update(c, d_xyz, d_state, n, nullptr, S(stream));
}

edt_status edt_integrate_scan(edt_ctx* c, const int32_t* d_origin, const int32_t* d_ends,
                              const uint8_t* d_hits, int64_t n, void* stream) {
    if (!c || n < 0) return EDT_ERR_ARG;
    if (n == 0) return EDT_OK;
    if (!d_origin || !d_ends || !d_hits) return EDT_ERR_ARG;
    const Grid& g = c->g;
    const int64_t mc = g.max_changes;
    if (n > mc) return EDT_ERR_CAPACITY;
    hipStream_t st = S(stream);
    // list: free entries first (capacity mc - n), then one entry per hit
    const int64_t cap = mc - n;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, c->scan_cnt, (int64_t)4, 0);
    int64_t* total = (int64_t*)(c->scan_cnt + 4);
    const int64_t nb = (n + 1023) / 1024;
    int64_t* btot = c->scan_blk;
    int64_t* bpre = c->scan_blk + nb;
    hipLaunchKernelGGL(k_scan_offsets, dim3((unsigned)nb), dim3(1024), 0, st, g, d_origin, d_ends,
                       n, c->scan_off, btot);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, (const int64_t*)btot, nb, bpre,
                       total);
    hipLaunchKernelGGL(k_scan_clear, dim3(2048), dim3(1024), 0, st, g, d_origin, d_ends, d_hits, n,
                       (const int64_t*)c->scan_off, (const int64_t*)bpre, (const int64_t*)total,
                       c->scan_cnt, c->scan_xyz, c->scan_state, cap);
    hipLaunchKernelGGL(k_scan_hits, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, g, d_origin,
                       d_ends, d_hits, n, c->scan_cnt, c->scan_xyz, c->scan_state, cap);
    LAUNCH_CHECK();
    return run_update(c, c->scan_xyz, c->scan_state, mc, c->scan_cnt + 2, st);
}

edt_status edt_query(edt_ctx* c, const int32_t* d_xyz, int64_t n, int32_t* d_out, void* stream) {
    if (!c || n < 0) return EDT_ERR_ARG;
    if (n == 0) return EDT_OK;
    if (!d_xyz || !d_out) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_query, dim3(grid_for(n, 256, 8192)), dim3(256), 0, S(stream), c->g, d_xyz,
                       n, d_out);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_query_nearest(edt_ctx* c, const int32_t* d_xyz, int64_t n, int32_t* d_nearest,
                             void* stream) {
    if (!c || n < 0) return EDT_ERR_ARG;
    if (n == 0) return EDT_OK;
    if (!d_xyz || !d_nearest) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_query_nearest, dim3(grid_for(n, 256, 8192)), dim3(256), 0, S(stream),
                       c->g, d_xyz, n, d_nearest);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_interior(edt_ctx* c, void* stream) {
    if (!c) return EDT_ERR_ARG;
    const Grid& g = c->g;
    if (g.max_int <= 0) return EDT_ERR_STATE;
    hipStream_t st = S(stream);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, g.cnt + C_NINT, (int64_t)1, 0);
    hipLaunchKernelGGL(k_int_list, dim3(grid_for(g.max_blocks, 256, 16384)), dim3(64), 0, st, g);
    const int grid = grid_for(g.max_int, 1, 16384);
    hipLaunchKernelGGL(k_int_x, dim3(grid), dim3(64), 0, st, g);
    hipLaunchKernelGGL(k_int_yz<1>, dim3(grid), dim3(64), 0, st, g);
    hipLaunchKernelGGL(k_int_yz<2>, dim3(grid), dim3(64), 0, st, g);
    LAUNCH_CHECK();
    c->interior_valid = true;
    return EDT_OK;
}

edt_status edt_query_signed(edt_ctx* c, const int32_t* d_xyz, int64_t n, int32_t* d_out,
                            void* stream) {
    if (!c || n < 0) return EDT_ERR_ARG;
    if (!c->interior_valid) return EDT_ERR_STATE;
    if (n == 0) return EDT_OK;
    if (!d_xyz || !d_out) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_query_signed, dim3(grid_for(n, 256, 8192)), dim3(256), 0, S(stream),
                       c->g, d_xyz, n, d_out);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_read_signed_dense(edt_ctx* c, int32_t* d_out, void* stream) {
    if (!c || !d_out) return EDT_ERR_ARG;
    if (!c->interior_valid) return EDT_ERR_STATE;
    const Grid& g = c->g;
    const int64_t nblk = (int64_t)g.nbx * g.nby * g.nbz;
    if (nblk > 0x7fffffff) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_read_strip<RB_SIGNED>, dim3((unsigned)read_strips(g)), dim3(256), 0, S(stream), g,
                       (void*)d_out);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_read_dense(edt_ctx* c, int32_t* d_out, void* stream) {
    if (!c || !d_out) return EDT_ERR_ARG;
    const Grid& g = c->g;
    const int64_t nblk = (int64_t)g.nbx * g.nby * g.nbz;
    if (nblk > 0x7fffffff) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_read_strip<RB_FIELD>, dim3((unsigned)read_strips(g)), dim3(256), 0, S(stream), g,
                       (void*)d_out);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_read_occupancy(edt_ctx* c, uint8_t* d_occ, void* stream) {
    if (!c || !d_occ) return EDT_ERR_ARG;
    const Grid& g = c->g;
    const int64_t nblk = (int64_t)g.nbx * g.nby * g.nbz;
    if (nblk > 0x7fffffff) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_read_strip<RB_OCC>, dim3((unsigned)read_strips(g)), dim3(256), 0, S(stream), g,
                       (void*)d_occ);
    LAUNCH_CHECK();
    return EDT_OK;
}

edt_status edt_get_stats(edt_ctx* c, edt_stats* o, void* stream) {
    if (!c || !o) return EDT_ERR_ARG;
    int32_t h[C_N];
    hipStream_t st = S(stream);
    if (hipMemcpyAsync(h, c->g.cnt, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess)
        return EDT_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return EDT_ERR_HIP;
    memset(o, 0, sizeof(*o));
    o->blocks = h[C_NBLK] < c->g.max_blocks ? h[C_NBLK] : c->g.max_blocks;
    o->obstacle_blocks = h[C_NDIL];
    o->added = h[C_NADD];
    o->removed = h[C_NREM];
    o->changed = (int64_t)h[C_NADD] + h[C_NREM];
    o->seed_blocks = h[C_NSEED];
    o->raise_blocks = h[C_NRAISE];
    o->lower_blocks = h[C_NLOWER];
    o->dirty_blocks = h[C_NDIRTY];
    o->error = h[C_ERR];
    o->d_max = c->g.dmax;
    return EDT_OK;
}

edt_status edt_get_error(edt_ctx* c, void* stream) {
    if (!c) return EDT_ERR_ARG;
    int32_t e = 0;
    hipStream_t st = S(stream);
    if (hipMemcpyAsync(&e, c->g.cnt + C_ERR, sizeof(e), hipMemcpyDeviceToHost, st) != hipSuccess)
        return EDT_ERR_HIP;
    hipLaunchKernelGGL(k_clear_error, dim3(1), dim3(1), 0, st, c->g);
    if (hipStreamSynchronize(st) != hipSuccess) return EDT_ERR_HIP;
    return (edt_status)e;
}

}  // extern "C"
