// edt_dev.h -- device-side data structures of libedt (gfx950).
//
// Storage: a pool of 8x8x8 leaf blocks under a two-level index, the GPU
// counterpart of the paper's VDB tree (section IV-A): a device hash table
// keyed by tile coordinates (a tile = 8x8x8 blocks = 64^3 voxels) whose
// probe position is the tile's id, and per tile a dense table of 512 pool
// slots (-1 = absent).  Both give O(1) access to sparse leaves and treat every
// absent leaf as the background value D (Algorithm 1, Initialize); the tile
// tables are small enough to stay in L2, so neighbour lookups are cheap.
//
// Per pool slot (one leaf block):
//   occ    512 occupancy bits, 16 x uint32; byte (y + 8z) holds row (y,z),
//          bit x = voxel x of that row.
//   g1     uint16 per voxel, layout (x + 8z) * 8 + y: squared distance
//          along x to the nearest obstacle of the same row, clamped to D.
//          The 8 values of one y-column are contiguous (one 16-byte load per
//          block and lane in pass y).
//   g2     uint16 per voxel, layout (x + 8y) * 8 + z: min over dy of
//          g1(x, y+dy, z) + dy^2, clamped to D (contiguous z-columns).
//   s      uint16 per voxel, layout x + 8y + 64z: the field, min(D, |x-y|^2).
//          g1, g2 and s hold integers, or for radii whose windowed minimum
//          runs in binary16 (d_max <= 40) the binary16 bit patterns of the
//          same integers.
//   bmax   int32: max of s over the block (pruning bound for updates).
//   flags  uint32: state bits (F_*).
// Blocks exist exactly where s can differ from D: blocks that held an
// obstacle at some point and all blocks within R = ceil(d_max/8) blocks of
// them (Chebyshev).  A voxel outside that region has no obstacle within
// distance 8R >= d_max along at least one axis, so its value is D.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace edt {

constexpr unsigned long long KEY_EMPTY = ~0ull;
constexpr int LRUN = 16;        // longest y / z work item (blocks); Grid::lrun <= LRUN
constexpr int32_t FINF = 1 << 28;

enum : uint32_t {
    F_DILATED = 1u,  // block's R-neighbourhood is in the pool
    F_SEED = 2u,     // block holds a changed voxel in the current update
    F_DIRTY = 4u,    // block's values are recomputed in the current update
    F_XS = 8u,       // g1 recomputed in the current update
    F_YS = 16u,      // g2 recomputed in the current update
    F_RAISE = 32u,   // marked by the raise front
    F_LOWER = 64u,   // marked by the lower front
    F_NEWDIL = 128u, // gains its first obstacle in the current update (listed for dilation)
    F_DILNEW = 256u, // F_DILATED set by the current update (undone if the call is cancelled)
};

// device counters (int32 slots of the counter array).  C_ABORT: the global
// transform ran out of pool; C_UABORT: nonzero once the current update is
// cancelled (read by the first three kernels of the update, cleared by the
// fourth, so a captured update replays with the same arguments).
enum {
    C_NBLK = 0, C_NDIL, C_ERR, C_ABORT, C_NINT, C_UABORT,
    C_NYI, C_NZI, C_NADD, C_NREM, C_NSEED, C_NDIRTY, C_NRAISE, C_NLOWER,
    C_NXS, C_NYS, C_NNEWDIL, C_DONE, C_NTILE, C_N
};

struct Grid {
    int nx, ny, nz;          // extent (voxels)
    int nbx, nby, nbz;       // extent (blocks)
    int dmax, D, R;          // radius, D = dmax^2, R = ceil(dmax / 8)
    int max_blocks;
    int lrun;                // output blocks per y / z work item of the list-driven passes
    uint32_t tmask;          // tile hash capacity - 1
    uint32_t umask;          // update-dedupe hash capacity - 1
    int max_changes;
    unsigned long long* tkeys;   // tile hash keys
    int32_t* tslots;             // [tile position][512] pool slot of each block
    uint32_t* tobst;             // [tile position][16] blocks holding an obstacle (global)
    int32_t* tflag;              // [tile position] nonzero once the tile holds an obstacle
                                 // block (global transform)
    int32_t* tlist;              // tile positions in use (global transform)
    int32_t* tinfo;              // [tile list index][8] tile position, then its face
                                 // neighbours -x, +x, -y, +y, -z, +z (-1 absent;
                                 // written by the dilation when d_max <= 64)
    unsigned long long* bkey;
    uint32_t* occ;
    uint16_t* g1;
    uint16_t* g2;
    uint16_t* s;             // [slot][512] squared distance, layout x + 8y + 64z (D <= 255^2)
    int32_t* bmax;
    uint32_t* flags;
    int32_t* cnt;
    int32_t* list_yi;        // y work items (start slots)
    int32_t* list_zi;        // z work items
    int32_t* list_seed;      // update: seed blocks
    int32_t* list_dirty;     // update: dirty blocks
    int32_t* list_xs;        // update: blocks whose g1 is recomputed
    int32_t* list_ys;        // update: blocks whose g2 is recomputed
    int32_t* list_newdil;    // update: blocks that became obstacle blocks
    uint32_t* chg_add;       // [slot][16] voxels added in this update
    uint32_t* chg_rem;       // [slot][16] voxels removed in this update
    unsigned long long* ukeys;
    int32_t* uvals;
    int32_t* upos;
    uint16_t* bmin1;         // [slot] least g1 value of the block (global transform)
    uint16_t* bmin2;         // [slot] least g2 value of the block (global transform)
    int max_int;             // capacity of the interior-distance blocks
    int32_t* iidx;           // [slot] index among the blocks holding an obstacle, or -1
                             // (written by the interior transform)
    int32_t* ilist;          // [interior index] pool slot
    uint16_t* ic1;           // [interior index][512] interior pass x (layout y + 8x + 64z),
                             // then the interior field (layout x + 8y + 64z)
    uint16_t* ic2;           // [interior index][512] interior pass y (layout z + 8x + 64y)
    uint32_t* dummy;         // 256 x 256 words of write-only scratch rows
    uint16_t* dblock;        // one block of D values (stands for absent blocks)
};

__host__ __device__ inline unsigned long long pack_key(int bx, int by, int bz) {
    return (unsigned long long)(uint32_t)bx | ((unsigned long long)(uint32_t)by << 21) |
           ((unsigned long long)(uint32_t)bz << 42);
}
__device__ inline void unpack_key(unsigned long long k, int& bx, int& by, int& bz) {
    bx = (int)(k & 0x1fffff);
    by = (int)((k >> 21) & 0x1fffff);
    bz = (int)((k >> 42) & 0x1fffff);
}

__device__ inline uint32_t hash_of(unsigned long long k, uint32_t mask) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return (uint32_t)k & mask;
}

// Table position of key, or -1 (read-only probe).
__device__ inline int32_t hpos(const unsigned long long* keys, uint32_t mask,
                               unsigned long long key) {
    uint32_t h = hash_of(key, mask);
    for (uint32_t i = 0; i <= mask; ++i) {
        const unsigned long long k = keys[h];
        if (k == key) return (int32_t)h;
        if (k == KEY_EMPTY) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

__device__ inline int block_local(int bx, int by, int bz) {
    return (bx & 7) + 8 * (by & 7) + 64 * (bz & 7);
}

__device__ inline int32_t find_block(const Grid& g, int bx, int by, int bz) {
    if (bx < 0 || by < 0 || bz < 0 || bx >= g.nbx || by >= g.nby || bz >= g.nbz) return -1;
    const int32_t t = hpos(g.tkeys, g.tmask, pack_key(bx >> 3, by >> 3, bz >> 3));
    return t < 0 ? -1 : g.tslots[(int64_t)t * 512 + block_local(bx, by, bz)];
}

// Find-or-insert: returns the table position, or -1 when the table is full.
// *created is true for the one thread whose CAS placed the key.
__device__ inline int32_t hinsert(unsigned long long* keys, uint32_t mask,
                                  unsigned long long key, bool* created) {
    uint32_t h = hash_of(key, mask);
    for (uint32_t i = 0; i <= mask; ++i) {
        unsigned long long k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) { *created = false; return (int32_t)h; }
        if (k == KEY_EMPTY) {
            unsigned long long old = atomicCAS(&keys[h], KEY_EMPTY, key);
            if (old == KEY_EMPTY) { *created = true; return (int32_t)h; }
            if (old == key) { *created = false; return (int32_t)h; }
        }
        h = (h + 1) & mask;
    }
    *created = false;
    return -1;
}

__device__ inline void set_error(const Grid& g, int code) {
    atomicCAS(&g.cnt[C_ERR], 0, code);
}

constexpr int32_t SLOT_PENDING = -2;   // block claimed, pool slot not yet written

// Find-or-insert of block (bx, by, bz) (inside the extent): returns its entry
// in the tile tables, or -1 when the tile hash is full.  The one thread that
// turns the entry from -1 into SLOT_PENDING gets *created = true and must
// write the pool slot (claim_slots); others only learn that the block exists.
__device__ inline int64_t insert_block(const Grid& g, int bx, int by, int bz, bool* created,
                                      bool* tile_created = nullptr) {
    bool tnew;
    const int32_t t = hinsert(g.tkeys, g.tmask, pack_key(bx >> 3, by >> 3, bz >> 3), &tnew);
    *created = false;
    if (tile_created) *tile_created = t >= 0 && tnew;
    if (t < 0) return -1;
    const int64_t e = (int64_t)t * 512 + block_local(bx, by, bz);
    if (__hip_atomic_load(&g.tslots[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1) return e;
    *created = atomicCAS(&g.tslots[e], -1, SLOT_PENDING) == -1;
    return e;
}

// Wave-aggregated append of `pred` lanes to list[] (ballot + mbcnt + one
// atomicAdd per wave).  Returns the lane's index or -1.
__device__ inline int wave_append(bool pred, int32_t* counter) {
    unsigned long long m = __ballot(pred);
    if (m == 0) return -1;
    int lane = __lane_id();
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    unsigned int lo = __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0);
    unsigned int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), lo);
    return pred ? base + (int)rank : -1;
}

__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ inline int wave_sum(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

// Wave-wide max / min of two packed unsigned 16-bit halves (each half on its
// own), returned to every lane as a uniform value.  Every lane of the wave
// must be active.  Data moves between lanes with DPP: swaps inside quads, the
// half-row and row mirrors make each row of 16 lanes uniform, the row
// broadcasts of lanes 15 and 31 fold the four rows into lane 63.
template <bool MAX>
__device__ inline uint32_t wave_reduce_pk_u16(uint32_t v) {
    typedef unsigned short u2 __attribute__((ext_vector_type(2)));
    auto op = [](uint32_t a, uint32_t b) -> uint32_t {
        const u2 x = __builtin_bit_cast(u2, a), y = __builtin_bit_cast(u2, b);
        return __builtin_bit_cast(uint32_t, MAX ? __builtin_elementwise_max(x, y)
                                                : __builtin_elementwise_min(x, y));
    };
    v = op(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));  // lane ^ 1
    v = op(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));  // lane ^ 2
    v = op(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false)); // half-row mirror
    v = op(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false)); // row mirror
    // rows 1 and 3 take lane 15 / 47 of the row before; then rows 2 and 3 take lane 31
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

}  // namespace edt
