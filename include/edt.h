/*
 * edt.h -- C ABI of libedt, an exact truncated squared Euclidean distance
 * transform (EDT) of voxel occupancy maps on one AMD Instinct MI355X (gfx950).
 *
 * The method is VDB-EDT (Zhu et al., "VDB-EDT: An Efficient Euclidean Distance
 * Transform Algorithm Based on VDB Data Structure").  What is computed is the
 * paper's distance field: Eq. 1 (section III) with the squared Euclidean
 * distance, limited to the transform radius d_max (section III, the LIDT
 * restriction); cells beyond the radius hold the background value, as the
 * Initialize procedure of Algorithm 1 sets it.  Distances are squared and in
 * voxel units, so for every voxel x of the map extent
 *
 *     s(x) = min( D, min over occupied y of |x - y|^2 ),   D = d_max^2,
 *
 * 0 on obstacles, D where no obstacle lies within d_max.  Results are exact
 * int32; a global transform and any sequence of incremental updates give the
 * same bits.  Inside the workspace s is held as 16-bit values (D <= 255^2 <
 * 2^16), widened on readback.
 *
 * Conventions
 *  - Every pointer named d_* is a device pointer (HIP global memory); the
 *    caller owns all of them.  The library never allocates device memory: the
 *    caller passes one workspace buffer at create time (edt_workspace_bytes).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    calls except edt_create, edt_destroy, edt_workspace_bytes and
 *    edt_status_str enqueue work on that stream and return without waiting,
 *    unless stated otherwise.
 *  - Grid layout of dense arrays: x fastest, index x + nx*(y + ny*z).
 *  - Occupancy bytes: nonzero = occupied.
 *  - Coordinates outside [0,nx)x[0,ny)x[0,nz) are never obstacles and read as
 *    D.
 *  - A context is not thread-safe; use it from one host thread and one
 *    stream at a time.
 *  - Every call returns an edt_status; nothing aborts, throws or prints.
 */
#ifndef EDT_H_
#define EDT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EDT_OK = 0,
    EDT_ERR_ARG = -1,       /* invalid argument (null pointer, bad size)      */
    EDT_ERR_RANGE = -2,     /* coordinates outside the map extent             */
    EDT_ERR_CAPACITY = -3,  /* workspace / block pool / change list too small */
    EDT_ERR_HIP = -4,       /* a HIP runtime call failed                      */
    EDT_ERR_STATE = -5      /* call not valid in the context's current state  */
} edt_status;

/* Human-readable name of a status code (static string). */
const char* edt_status_str(int status);

/* Map configuration, fixed for the life of a context.
 *   nx, ny, nz   extent in voxels, each 1 .. 2^20.
 *   d_max        transform radius in voxels, 1 .. 255 (so D <= 65025).
 *   max_blocks   capacity of the leaf-block pool (8x8x8 voxels per block);
 *                0 = one slot per block of the extent.  Blocks are created
 *                only where the field can differ from D: blocks holding an
 *                obstacle and the blocks within ceil(d_max/8) blocks of them
 *                (Chebyshev distance).
 *   max_changes  capacity for one edt_update call (entries), 0 = 2^20.
 *   max_interior_blocks  capacity for interior distances (edt_interior):
 *                the number of blocks holding an obstacle it can serve;
 *                0 = no interior storage.                                   */
typedef struct {
    int32_t nx, ny, nz;
    int32_t d_max;
    int64_t max_blocks;
    int64_t max_changes;
    int64_t max_interior_blocks;
} edt_config;

typedef struct edt_ctx edt_ctx;

/* Bytes of device workspace that edt_create needs for `cfg`, or a negative
 * edt_status if cfg is invalid. */
int64_t edt_workspace_bytes(const edt_config* cfg);

/* Creates a context over the caller's device workspace d_ws (at least
 * edt_workspace_bytes(cfg) bytes, 256-byte aligned, owned by the caller and
 * kept alive until edt_destroy).  The field starts empty: s = D everywhere
 * (Algorithm 1, Initialize).  Initialisation is enqueued on `stream`.
 * On success *out receives a host object owned by the library. */
edt_status edt_create(const edt_config* cfg, void* d_ws, int64_t ws_bytes,
                      void* stream, edt_ctx** out);

/* Frees the host object.  Does not touch the caller's workspace. */
edt_status edt_destroy(edt_ctx* ctx);

/* Input of a global transform: either a dense grid or a list of leaf blocks.
 *   EDT_MAP_DENSE   d_occ: nx*ny*nz bytes, grid layout.
 *   EDT_MAP_BLOCKS  d_block_xyz: int32[n_blocks][3] block coordinates
 *                   (bx, by, bz), voxel (8bx+i, 8by+j, 8bz+k) for in-block
 *                   offsets i, j, k in 0..7; d_block_occ: uint8[n_blocks][512]
 *                   in-block occupancy, index i + 8j + 64k.  Voxels of a block
 *                   that fall outside the extent are ignored.  Repeated block
 *                   coordinates are merged (union of occupancy).  Blocks with
 *                   coordinates outside the extent set the device error word
 *                   (EDT_ERR_RANGE, see edt_get_error) and are skipped.     */
typedef enum { EDT_MAP_DENSE = 0, EDT_MAP_BLOCKS = 1 } edt_map_kind;
typedef struct {
    int32_t kind;
    const uint8_t* d_occ;
    const int32_t* d_block_xyz;
    const uint8_t* d_block_occ;
    int64_t n_blocks;
} edt_map;

/* Global transform: replaces the context's occupancy with `map` and computes
 * s everywhere (paper section V-A, global transform; Eq. 1).  Exact. */
edt_status edt_global(edt_ctx* ctx, const edt_map* map, void* stream);

/* Incremental transform (Algorithm 1: SetObstacle / RemoveObstacle followed
 * by DistanceTransform).  d_xyz: int32[n][3] voxel coordinates (x, y, z);
 * d_state: uint8[n] target state, nonzero = occupied.  States are absolute:
 * an entry equal to the current occupancy is a no-op (as SetObstacle on an
 * obstacle, RemoveObstacle on a free cell); when a voxel appears several
 * times the last entry wins (the same result as applying the entries in
 * order).  Afterwards s equals edt_global of the new occupancy, bit for bit.
 * n == 0 is a no-op.  n > max_changes returns EDT_ERR_CAPACITY with nothing
 * enqueued.  Entries outside the extent make the whole call a no-op and set
 * the device error word to EDT_ERR_RANGE.  Every block the call needs is
 * created before any occupancy changes: if the block pool fills up, the call
 * is cancelled with the map unchanged (blocks it created hold the background
 * value, which is their correct field) and the error word becomes
 * EDT_ERR_CAPACITY; edt_grow then makes room and the call can be repeated. */
edt_status edt_update(edt_ctx* ctx, const int32_t* d_xyz, const uint8_t* d_state,
                      int64_t n, void* stream);

/* Occupancy integration of one range scan followed by the incremental
 * transform: the mapping step in front of the transform in the paper's
 * online pipeline (section V-B builds its dataset maps from LIDAR scans this
 * way).  d_origin: int32[3] sensor voxel; d_ends: int32[n][3] end voxels of
 * the rays; d_hits: uint8[n], nonzero = the ray ended on a return (its end
 * voxel is an obstacle).  A ray visits its origin voxel and then every voxel
 * that the segment between the two voxel centres enters through a face: the
 * i-th crossing on axis a lies at segment parameter (2i + 1) / (2|d_a|),
 * d = end - origin, and crossings at equal parameters are taken in the order
 * x, y, z (an exact integer form of the Amanatides-Woo voxel walk).  Every
 * visited voxel becomes free except a hit's end voxel, which becomes
 * occupied; a hit wins over any ray passing through the same voxel.  The
 * resulting changes then go through edt_update, so afterwards s equals
 * edt_global of the new occupancy.  n > max_changes: EDT_ERR_CAPACITY with
 * nothing enqueued.  Rays with the origin or end outside the extent are
 * skipped and set EDT_ERR_RANGE in the device error word.  If more than
 * max_changes - n voxels would be freed, the excess is dropped (the field
 * still matches the occupancy) and the error word becomes EDT_ERR_CAPACITY.
 * Shares the update's scratch: not to be overlapped with edt_update. */
edt_status edt_integrate_scan(edt_ctx* ctx, const int32_t* d_origin, const int32_t* d_ends,
                              const uint8_t* d_hits, int64_t n, void* stream);

/* Compaction: rebuilds the block pool from the current occupancy and
 * recomputes s (the global transform of the current map).  Updates only add
 * blocks; blocks whose obstacles have all been removed stay in the pool.
 * This drops every block that no longer holds an obstacle and lies beyond
 * ceil(d_max/8) blocks of all that do (the background-value pruning of a VDB
 * tree, section IV-A), so the pool follows the map again.  s is unchanged;
 * pool slots are renumbered. */
edt_status edt_compact(edt_ctx* ctx, void* stream);

/* Growth of the block pool (section IV-A: the tree grows as cells are
 * transformed, memory is allocated only where the field is computed).  Moves
 * the context onto the caller's new workspace d_ws (256-byte aligned, at
 * least edt_workspace_bytes of the context's configuration with max_blocks
 * replaced by the new max_blocks, which must not be smaller than the current
 * capacity).  The map is carried over without recomputation: every pool
 * block (occupancy, intermediates, field, per-block state) keeps its slot
 * number and is copied, and the tile index is rehashed into the new table,
 * so s, the occupancy and every later result are those the old context
 * would give (interior distances must be recomputed).  The old workspace is
 * read by work enqueued on `stream` and may be released once that work has
 * completed.  An update cancelled because the pool was full
 * (edt_get_error returns EDT_ERR_CAPACITY) leaves the map unchanged, so it
 * can be issued again after edt_grow. */
edt_status edt_grow(edt_ctx* ctx, int64_t max_blocks, void* d_ws, int64_t ws_bytes,
                    void* stream);

/* s at n voxel coordinates d_xyz (int32[n][3]) into d_out (int32[n]);
 * out-of-extent coordinates and voxels of blocks that hold no field read D
 * (the VDB background value). */
edt_status edt_query(edt_ctx* ctx, const int32_t* d_xyz, int64_t n,
                     int32_t* d_out, void* stream);

/* Nearest obstacle (the `obst` of a cell in Algorithm 1; the feature
 * transform of Eq. 1): for each of n voxel coordinates d_xyz (int32[n][3])
 * writes to d_nearest (int32[n][3]) the coordinates of one occupied voxel o
 * with |x - o|^2 = s(x).  Where several obstacles are that close, any one of
 * them is returned.  Voxels with s(x) = D (no obstacle within d_max) and
 * out-of-extent coordinates get (-1, -1, -1).  The answer is reconstructed
 * from the stored per-axis minima (z, then y, then x), so it is consistent
 * with edt_query after any sequence of updates. */
edt_status edt_query_nearest(edt_ctx* ctx, const int32_t* d_xyz, int64_t n,
                             int32_t* d_nearest, void* stream);

/* Interior distances, the inside half of a signed distance field (the
 * Euclidean signed distance fields of the voxel-hashing systems surveyed in
 * section II): the field's definition (Eq. 1, clamped to D) with occupied
 * and free voxels exchanged.  For every occupied voxel x,
 *
 *     s_in(x) = min( D, min over free voxels y of the extent of |x - y|^2 ),
 *
 * so s_in >= 1, and D where no free voxel lies within d_max (voxels outside
 * the extent are neither free nor occupied).  Computed exactly from the
 * current occupancy over the blocks holding an obstacle; valid until the next
 * edt_global or edt_update.  EDT_ERR_STATE if the context was created with
 * max_interior_blocks = 0.  More blocks holding an obstacle than
 * max_interior_blocks set the device error word to EDT_ERR_CAPACITY; the
 * interior values are then not valid. */
edt_status edt_interior(edt_ctx* ctx, void* stream);

/* Signed squared distance at n voxel coordinates d_xyz (int32[n][3]) into
 * d_out (int32[n]): s(x) (>= 1) for a free voxel, -s_in(x) (<= -1) for an
 * occupied one, D out of the extent; the signed Euclidean distance is
 * sign(v) * sqrt(|v|).  EDT_ERR_STATE unless edt_interior ran after the
 * last edt_global / edt_update. */
edt_status edt_query_signed(edt_ctx* ctx, const int32_t* d_xyz, int64_t n,
                            int32_t* d_out, void* stream);

/* Dense signed readback (int32[nx*ny*nz], grid layout, values as
 * edt_query_signed).  Same state requirement as edt_query_signed. */
edt_status edt_read_signed_dense(edt_ctx* ctx, int32_t* d_out, void* stream);

/* Dense readback: s for the whole extent into d_out (int32[nx*ny*nz]).
 * The dense forms (dense input, the three dense readbacks) need fewer than
 * 2^31 blocks of 8^3 in the extent, else EDT_ERR_ARG. */
edt_status edt_read_dense(edt_ctx* ctx, int32_t* d_out, void* stream);

/* Dense occupancy readback into d_occ (uint8[nx*ny*nz], 0/1). */
edt_status edt_read_occupancy(edt_ctx* ctx, uint8_t* d_occ, void* stream);

/* Counters of the context (host struct).  Synchronises `stream`.
 *   blocks         leaf blocks holding field values (the computed region)
 *   obstacle_blocks blocks whose neighbourhood has been added to the region
 *   changed        voxels whose occupancy changed in the last edt_update
 *   added, removed split of `changed`
 *   seed_blocks    blocks holding those voxels (the wave centres)
 *   raise_blocks   blocks marked by the raise front in the last update
 *   lower_blocks   blocks marked by the lower front in the last update
 *   dirty_blocks   union of the two: blocks whose values were recomputed
 *   error          device error word (EDT_OK or a negative edt_status)     */
typedef struct {
    int64_t blocks, obstacle_blocks;
    int64_t changed, added, removed;
    int64_t seed_blocks, raise_blocks, lower_blocks, dirty_blocks;
    int32_t error, d_max;
} edt_stats;
edt_status edt_get_stats(edt_ctx* ctx, edt_stats* host_out, void* stream);

/* Synchronises `stream`, returns the device error word and clears it. */
edt_status edt_get_error(edt_ctx* ctx, void* stream);

/* Profiling.  edt_timing_begin arms HIP events around the phases of the
 * next n_calls calls of edt_global on this context (0 disarms and frees
 * them).  edt_timing_read waits for the recorded events and writes into
 * ms[0..5] the mean duration in milliseconds of each phase over the recorded
 * calls: ingest, region growth, work lists, pass x, pass y, pass z;
 * *n_recorded receives the number of calls recorded.  The events are recorded
 * on the stream the calls were made on. */
edt_status edt_timing_begin(edt_ctx* ctx, int32_t n_calls);
edt_status edt_timing_read(edt_ctx* ctx, float* ms, int32_t* n_recorded);
/* As edt_timing_begin, but only phase `phase` (0 .. 5, in the order above; -1
 * = all) is bracketed, two events per call, so the other phases run without
 * event records between them; edt_timing_read then reports 0 for the other
 * phases. */
edt_status edt_timing_begin_phase(edt_ctx* ctx, int32_t n_calls, int32_t phase);

/* ------------------------------------------------------------------------ */
/* Batched global transform of many dense maps (same definition as edt_global
 * per map), with 1 <= d_max <= 64.  Map i occupies bytes
 * d_occ[occ_offset .. occ_offset + nx*ny*nz) (grid layout) and its field is
 * written to d_out[out_offset .. out_offset + nx*ny*nz) (int32, grid layout);
 * sides 1 .. 4096.  Callers own d_occ, d_out and the workspace. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;
    int64_t occ_offset;
    int64_t out_offset;
} edt_batch_map;

/* Schedule of a batched run (edt_batch_run; NULL = defaults {8, 8, 4, 0, 4}):
 *   lrun          blocks per work item along y and z (1 .. 64)
 *   waves_per_cu  waves resident per compute unit (0 = default, <= 64)
 *   chunk         work items taken per queue atomic (1 .. 1024)
 *   schedule      0 = dynamic queue, 1 = static stride
 *   wg_waves      waves per workgroup: 1, 2, 4 or 8 (0 = 4); each wave
 *                 takes its own work items, the workgroup size only changes
 *                 how the waves are dispatched and share a compute unit, and
 *                 how many workgroups meet at the fused launch's grid-wide
 *                 barriers (fewer is cheaper)                             */
typedef struct {
    int32_t lrun;
    int32_t waves_per_cu;
    int32_t chunk;
    int32_t schedule;
    int32_t wg_waves;
} edt_tune;

/* EDT_BATCH_FUSED: one persistent cooperative launch for all maps and
 * passes, a grid-wide barrier between the x, y and z passes.
 * EDT_BATCH_PER_MAP: three launches (x, y, z) per map.
 * EDT_BATCH_PHASED: three launches (x, y, z) for all maps, with the fused
 * launch's schedule; each launch holds the code of its pass only. */
typedef enum {
    EDT_BATCH_FUSED = 0,
    EDT_BATCH_PER_MAP = 1,
    EDT_BATCH_PHASED = 2
} edt_batch_mode;

typedef struct edt_batch edt_batch;

/* Device workspace bytes for the maps, or a negative edt_status. */
int64_t edt_batch_workspace_bytes(const edt_batch_map* maps, int32_t n_maps, int32_t d_max);

/* Prepares a batch over the caller's workspace (256-byte aligned, at least
 * edt_batch_workspace_bytes).  `maps` is a host array, copied; the call
 * synchronises `stream` once. */
edt_status edt_batch_create(const edt_batch_map* maps, int32_t n_maps, int32_t d_max,
                            void* d_ws, int64_t ws_bytes, void* stream, edt_batch** out);

/* Transforms every map of the batch (mode: edt_batch_mode). */
edt_status edt_batch_run(edt_batch* batch, const uint8_t* d_occ, int32_t* d_out,
                         int32_t mode, const edt_tune* tune, void* stream);

edt_status edt_batch_destroy(edt_batch* batch);

/* ------------------------------------------------------------------------ */
/* Full (uncapped) transform of a dense grid: the distance field with which
 * the paper runs its dataset benchmarks, d_max = infinity (section V-B), and
 * radii beyond the 255 of the sparse field.  Same definition as Eq. 1, with
 *     s(x) = min over occupied y of |x - y|^2      (d_max = 0: no limit)
 *     s(x) = min(d_max^2, that)                    (1 <= d_max <= 46340)
 * and EDT_DENSE_INF for every voxel of a grid without obstacles when
 * d_max = 0.  d_occ: uint8[nz][ny][nx] (nonzero = occupied); d_out:
 * int32[nz][ny][nx], written in place by the three passes.  The extent must
 * satisfy nx^2 + ny^2 + nz^2 < 2^31 (every squared distance fits in int32),
 * else EDT_ERR_ARG.  The caller's workspace (8-byte aligned,
 * edt_dense_workspace_bytes) holds the per-column parabola envelopes.
 * The incremental form is the dense context below. */
#define EDT_DENSE_INF 0x7fffffff
int64_t edt_dense_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);
edt_status edt_dense_global(int32_t nx, int32_t ny, int32_t nz, int32_t d_max,
                            const uint8_t* d_occ, int32_t* d_out, void* d_ws, int64_t ws_bytes,
                            void* stream);

/* Allocation-free form of edt_dense_global, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and result, without the
 * workspace: the column envelopes live in a static device buffer of the
 * library, EDT_DENSE_STATIC_BYTES (64 MiB) on each GPU it runs on, held
 * until the process ends.  Grids with edt_dense_workspace_bytes(nx, ny, nz)
 * above that (more than 8,388,608 voxels, e.g. beyond 256 x 256 x 128)
 * return EDT_ERR_CAPACITY with nothing enqueued.  Runs on the current
 * device; `stream` must belong to it.  The call allocates nothing (its first
 * call on a device looks up the buffer's device address).  Every call on one
 * GPU uses the same buffer: calls that overlap on one GPU (several streams
 * or host threads) race, and the caller must serialise them. */
#define EDT_DENSE_STATIC_BYTES (64ll << 20)
edt_status edt_dense_global_noalloc(int32_t nx, int32_t ny, int32_t nz, int32_t d_max,
                                    const uint8_t* d_occ, int32_t* d_out, void* stream);

/* Dense context: the uncapped (or large-radius) field of a dense grid kept
 * current under occupancy changes, the incremental counterpart of
 * edt_dense_global (paper section IV-B, Algorithm 1's SetObstacle /
 * RemoveObstacle followed by DistanceTransform, with d_max = infinity as in
 * its section V-B runs).  The context holds the occupancy (uint8 per voxel),
 * both int32 intermediates and the int32 field in the caller's workspace
 * (256-byte aligned, edt_dense_ctx_bytes bytes; about 21 bytes per voxel);
 * it is owned by the caller and must outlive the context.  d_max: 0 = no
 * limit (voxels of a map without obstacles read EDT_DENSE_INF), else
 * 1 ..  46340 (values clamped to d_max^2).  max_changes: the most entries
 * one update may carry.  Extent: as edt_dense_global.  Errors: EDT_ERR_ARG
 * for invalid sizes or pointers, EDT_ERR_CAPACITY for a short workspace.
 * create enqueues the field of the empty map on `stream`. */
typedef struct edt_dense_ctx edt_dense_ctx;
int64_t edt_dense_ctx_bytes(int32_t nx, int32_t ny, int32_t nz, int64_t max_changes);
edt_status edt_dense_ctx_create(int32_t nx, int32_t ny, int32_t nz, int32_t d_max,
                                int64_t max_changes, void* d_ws, int64_t ws_bytes, void* stream,
                                edt_dense_ctx** out);
edt_status edt_dense_ctx_destroy(edt_dense_ctx* ctx);

/* Replaces the context's occupancy with d_occ (uint8[nz][ny][nx], nonzero =
 * occupied; copied) and recomputes everything: edt_dense_global's result. */
edt_status edt_dense_ctx_global(edt_dense_ctx* ctx, const uint8_t* d_occ, void* stream);

/* Incremental transform: n entries (int32[n][3] voxel coordinates and
 * uint8[n] absolute target states), same rules as edt_update (an entry equal
 * to the current occupancy is a no-op; for a voxel listed several times the
 * last entry wins; entries outside the extent make the call a no-op and set
 * the device error word to EDT_ERR_RANGE; n > max_changes returns
 * EDT_ERR_CAPACITY with nothing enqueued).  Rows holding a changed voxel are
 * recomputed along x, then every column along y whose input changed, then
 * every column along z whose input changed, each over its whole length, so
 * afterwards the field equals edt_dense_global of the new occupancy bit for
 * bit. */
edt_status edt_dense_ctx_update(edt_dense_ctx* ctx, const int32_t* d_xyz,
                                const uint8_t* d_state, int64_t n, void* stream);

/* Device address of the field (int32[nz][ny][nx], inside the workspace):
 * read it after the work enqueued before has completed; valid until the
 * context is destroyed.  NULL for a NULL context. */
const int32_t* edt_dense_ctx_field(const edt_dense_ctx* ctx);

/* Device error word of the context (EDT_OK or the first error of the updates
 * since the last read); reading clears it.  Waits for `stream`. */
edt_status edt_dense_ctx_get_error(edt_dense_ctx* ctx, void* stream);

/* ------------------------------------------------------------------------ */
/* Clearance cost on a dense field (paper section III, Eq. 2, clearance
 * term, in the squared-hinge form  c(p) = max(0, margin - d(p))^2).
 *   d_s        int32[nz][ny][nx] squared voxel distances (e.g. from
 *              edt_read_dense); each side >= 2.
 *   h          voxel edge in metres; voxel center (i,j,k) sits at (i,j,k)*h.
 *   d(p)       trilinear interpolation of h*sqrt(s) at p (metres), with the
 *              cell index clamped to [0, n-2] and the cell coordinate to
 *              [0, 1] per axis; u = p/h, the cell and its coordinate are
 *              computed in double precision, everything else in float.
 *   d_wp       float[T][W][3] waypoints (x, y, z) in metres.
 *   d_cost     float[T]: sum over the W waypoints of c(p), accumulated in
 *              fp32 in a fixed order (deterministic).
 * edt_clearance_bwd writes d_gwp (float[T][W][3]) = d_gcost[t] * dc/dp,
 * zero on axes whose cell coordinate was clamped and where d >= margin.    */
edt_status edt_clearance_fwd(const int32_t* d_s, int32_t nx, int32_t ny, int32_t nz,
                             double h, float margin, const float* d_wp,
                             int64_t T, int32_t W, float* d_cost, void* stream);
edt_status edt_clearance_bwd(const int32_t* d_s, int32_t nx, int32_t ny, int32_t nz,
                             double h, float margin, const float* d_wp,
                             int64_t T, int32_t W, const float* d_gcost,
                             float* d_gwp, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EDT_H_ */
