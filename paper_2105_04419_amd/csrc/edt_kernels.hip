// edt_kernels.hip -- HIP kernels of the exact truncated EDT for gfx950.
//
// Global transform (the field of Eq. 1, section III, limited to d_max):
//   ingest          dense grid or leaf-block list -> occupancy bits + hash
//   tile dilation   region = obstacle blocks grown by R blocks (per tile)
//   items (y,z)     runs of consecutive region blocks, at most LRUN long
//   pass_x          g1 = squared distance along x, from the occupancy bits
//   pass_y          g2(y) = min_j g1(y+j) + j^2
//   pass_z          s(z)  = min(D, min_k g2(z+k) + k^2)
// The squared Euclidean distance splits into per-axis terms, so the three
// passes give exactly Eq. 1; terms with an axis offset beyond d_max exceed D
// and never change the clamped result.  For d_max <= 64 the y and z passes
// take the windowed minimum directly, branch-free on packed 16-bit pairs;
// for larger radii they follow the lower envelope of parabolas (Felzenszwalb
// & Huttenlocher, cited by the paper as the global transform), streamed with
// one lane per row and a ring of the sites that can still reach the next
// outputs.
//
// Incremental transform (Algorithm 1's raise and lower waves, at block
// granularity): changed voxels are the wave centres; a block is on the lower
// front if some added voxel is closer to the block than its largest value,
// and on the raise front if some removed voxel is no farther than its largest
// value (only such blocks can change); the g1/g2 intermediates are kept
// current for every block and the marked blocks are recomputed exactly.
#include "edt_dev.h"
#include "edt_win.h"

namespace edt {

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Global transform start: empty block table, counters reset (the error word
// is kept until it is read).
__global__ void k_begin_global(Grid g, int64_t tcap) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < tcap; i += stride) g.tkeys[i] = KEY_EMPTY;
    int4* ts = (int4*)g.tslots;
    for (int64_t i = tid; i < tcap * 128; i += stride) ts[i] = make_int4(-1, -1, -1, -1);
    for (int64_t i = tid; i < tcap * 16; i += stride) g.tobst[i] = 0u;
    for (int64_t i = tid; i < tcap; i += stride) g.tflag[i] = 0;
    if (tid < C_N && tid != C_ERR) g.cnt[tid] = 0;
}

// Every tile within ceil(R / 8) tiles of an obstacle tile must exist before
// the dilation.  Called by a whole wave: for each lane whose block is the
// first obstacle block of its tile (tile coordinates tx, ty, tz), the wave
// inserts the tile's neighbours, one neighbour per lane.  The trigger is the
// tile's first obstacle, not the tile's creation: a tile may already exist
// as the neighbour of another obstacle tile.
__device__ inline void grow_tiles(const Grid& g, bool first, int tx, int ty, int tz) {
    unsigned long long m = __ballot(first);
    if (m == 0ull) return;
    const int TR = (g.R + 7) >> 3, w = 2 * TR + 1, w3 = w * w * w;
    const int ntx = (g.nbx + 7) >> 3, nty = (g.nby + 7) >> 3, ntz = (g.nbz + 7) >> 3;
    const int lane = __lane_id();
    while (m) {
        const int src = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const int cx = __shfl(tx, src), cy = __shfl(ty, src), cz = __shfl(tz, src);
        for (int o0 = 0; o0 < w3; o0 += 64) {
            const int o = o0 + lane;
            bool tnew = false;
            int32_t t = -1;
            if (o < w3 && o != w3 / 2) {
                const int ax = cx + o % w - TR, ay = cy + (o / w) % w - TR, az = cz + o / (w * w) - TR;
                if (ax >= 0 && ay >= 0 && az >= 0 && ax < ntx && ay < nty && az < ntz) {
                    t = hinsert(g.tkeys, g.tmask, pack_key(ax, ay, az), &tnew);
                    if (t < 0) set_error(g, -3 /* EDT_ERR_CAPACITY */);
                }
            }
            const int j = wave_append(tnew, &g.cnt[C_NTILE]);
            if (tnew) g.tlist[j] = t;
        }
    }
}

// Record a new tile (and its neighbourhood) and, for obstacle blocks, the
// block in its tile's obstacle mask.  Called by a whole wave.
__device__ inline void note_tile(const Grid& g, bool tile_created, int64_t e, bool obstacle,
                                 int bx, int by, int bz) {
    const int t = e >= 0 ? (int)(e >> 9) : -1;
    const int j = wave_append(tile_created, &g.cnt[C_NTILE]);
    if (tile_created) g.tlist[j] = t;
    bool first = false;
    if (obstacle && e >= 0) {
        const int local = (int)(e & 511);
        atomicOr(&g.tobst[(int64_t)t * 16 + (local >> 5)], 1u << (local & 31));
        first = atomicOr(&g.tflag[t], 1) == 0;
    }
    grow_tiles(g, first, bx >> 3, by >> 3, bz >> 3);
}

// Pool slots for the lanes that just created a block at tile entry e: one
// counter atomic per wave.  Returns the slot, or -1 (not created / pool full).
__device__ inline int32_t claim_slots(const Grid& g, bool created, int64_t e,
                                      unsigned long long key, uint32_t flags) {
    const int idx = wave_append(created, &g.cnt[C_NBLK]);
    if (!created) return -1;
    if (idx >= g.max_blocks) {
        g.tslots[e] = -1;
        set_error(g, -3 /* EDT_ERR_CAPACITY */);
        g.cnt[C_ABORT] = 1;
        return -1;
    }
    g.bkey[idx] = key;
    g.flags[idx] = flags;
    g.tslots[e] = idx;
    return idx;
}

// ---------------------------------------------------------------------------
// ingest
// ---------------------------------------------------------------------------
// Workgroup b of a one-dimensional grid over an (nxb, nyb, nzb) box of
// blocks (a 3-D grid would cap y and z at 65535 workgroups).
__device__ inline void block_of(int nxb, int nyb, int& bx, int& by, int& bz) {
    const int64_t b = blockIdx.x;
    bx = (int)(b % nxb);
    const int64_t r = b / nxb;
    by = (int)(r % nyb);
    bz = (int)(r / nyb);
}

// Dense grid.  One wave per strip of 8 blocks along x; lane = row (y + 8z).
// Each lane reads 64 contiguous bytes of its row, packs 8 bits per block and
// the wave ballot decides whether a block holds any obstacle.
__global__ void __launch_bounds__(64) k_ingest_dense(Grid g, const uint8_t* __restrict__ occ) {
    const int lane = threadIdx.x;
    int sx, by, bz;
    block_of((g.nbx + 7) / 8, g.nby, sx, by, bz);
    const int bx0 = sx * 8;
    const int y = 8 * by + (lane & 7), z = 8 * bz + (lane >> 3);
    const int x0 = 8 * bx0;
    uint32_t bytes[8];
    const bool row_ok = (y < g.ny) && (z < g.nz);
    const uint8_t* row = occ + ((int64_t)z * g.ny + y) * (int64_t)g.nx;
    if (row_ok && x0 + 64 <= g.nx && (((uintptr_t)(row + x0)) & 15) == 0) {
        const uint4* p = (const uint4*)(row + x0);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint4 v = p[w];
            uint32_t a[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t lo = a[2 * h], hi = a[2 * h + 1];
                uint32_t b = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    b |= (((lo >> (8 * k)) & 0xff) != 0) << k;
                    b |= (((hi >> (8 * k)) & 0xff) != 0) << (k + 4);
                }
                bytes[2 * w + h] = b;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            uint32_t b = 0;
            for (int k = 0; k < 8; ++k) {
                int x = x0 + 8 * j + k;
                if (row_ok && x < g.nx && row[x]) b |= 1u << k;
            }
            bytes[j] = b;
        }
    }
    // lane j (< 8) learns whether block bx0 + j holds an obstacle
    bool mine = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool any = __ballot(bytes[j] != 0) != 0;
        if (lane == j) mine = any && (bx0 + j < g.nbx);
    }
    int64_t e = -1;
    bool created = false, tnew = false;
    const unsigned long long key = pack_key(bx0 + lane, by, bz);
    if (mine) {
        e = insert_block(g, bx0 + lane, by, bz, &created, &tnew);
        if (e < 0) set_error(g, -3);
    }
    note_tile(g, tnew, e, mine, bx0 + lane, by, bz);
    const int32_t slot = claim_slots(g, created, e, key, F_DILATED);
    const int ndil = __popcll(__ballot(slot >= 0));
    if (lane == 0 && ndil) atomicAdd(&g.cnt[C_NDIL], ndil);
    uint8_t* occ8 = (uint8_t*)g.occ;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int32_t sj = __shfl(slot, j);
        if (sj >= 0) {
            occ8[(int64_t)sj * 64 + lane] = (uint8_t)bytes[j];
            uint32_t* chg = lane < 16 ? g.chg_add : g.chg_rem;
            if (lane < 32) chg[(int64_t)sj * 16 + (lane & 15)] = 0u;
        }
    }
}

// Block list: eight input blocks per wave, eight lanes per block.  Lane q of
// a block reads rows 8q .. 8q + 7 (64 bytes: z = q, y = 0..7) and returns
// their bit rows as one 64-bit word, which is word q of the block's
// occupancy; voxels beyond the extent are dropped.
__device__ inline unsigned long long block_rows8(const Grid& g, const int32_t* xyz,
                                                 const uint8_t* data, int64_t i, int q,
                                                 int& bx, int& by, int& bz, bool& in_range) {
    bx = xyz[3 * i];
    by = xyz[3 * i + 1];
    bz = xyz[3 * i + 2];
    in_range = bx >= 0 && by >= 0 && bz >= 0 && bx < g.nbx && by < g.nby && bz < g.nbz;
    const uint4* p = (const uint4*)(data + i * 512 + 64 * q);
    uint4 v[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) v[w] = p[w];
    const int xr = g.nx - 8 * bx;
    const uint32_t xm = xr >= 8 ? 0xffu : (xr <= 0 ? 0u : (1u << xr) - 1u);
    const bool zok = 8 * bz + q < g.nz;
    unsigned long long rows = 0ull;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t d[4] = {v[w].x, v[w].y, v[w].z, v[w].w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {              // row y = 2w + h
            uint32_t b = 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                b |= (((d[2 * h] >> (8 * k)) & 0xffu) != 0u) << k;
                b |= (((d[2 * h + 1] >> (8 * k)) & 0xffu) != 0u) << (k + 4);
            }
            const bool ok = zok && 8 * by + 2 * w + h < g.ny;
            rows |= (unsigned long long)(ok ? (b & xm) : 0u) << (8 * (2 * w + h));
        }
    }
    return rows;
}

// Word q of input block i's occupancy.  BITS: the input already holds the
// pool's bit layout (64 bytes per block, as the compaction gathers it);
// otherwise one byte per voxel (block_rows8).
template <bool BITS>
__device__ inline unsigned long long input_rows(const Grid& g, const int32_t* xyz,
                                                const uint8_t* data, int64_t i, int q, int& bx,
                                                int& by, int& bz, bool& in_range) {
    if (!BITS) return block_rows8(g, xyz, data, i, q, bx, by, bz, in_range);
    bx = xyz[3 * i];
    by = xyz[3 * i + 1];
    bz = xyz[3 * i + 2];
    in_range = bx >= 0 && by >= 0 && bz >= 0 && bx < g.nbx && by < g.nby && bz < g.nbz;
    return ((const unsigned long long*)data)[i * 8 + q];
}

// Block list, phase 1: record every block holding an obstacle in its tile's
// obstacle mask (creating the tile and its neighbourhood).  Pool slots are
// assigned by the dilation.  The block count is n, or *n_dev when given.
template <bool BITS>
__global__ void __launch_bounds__(64) k_ingest_blocks_mark(Grid g, const int32_t* xyz,
                                                          const uint8_t* data, int64_t n0,
                                                          const int32_t* n_dev) {
    const int lane = threadIdx.x, sub = lane >> 3, q = lane & 7;
    const int64_t n = n_dev ? (int64_t)*n_dev : n0;
    for (int64_t i0 = (int64_t)blockIdx.x * 8; i0 < n; i0 += (int64_t)gridDim.x * 8) {
        const int64_t i = i0 + sub;
        int bx = 0, by = 0, bz = 0;
        bool ok = false;
        unsigned long long rows = 0ull;
        if (i < n) rows = input_rows<BITS>(g, xyz, data, i, q, bx, by, bz, ok);
        const bool any = ((__ballot(rows != 0ull) >> (8 * sub)) & 0xffull) != 0ull;
        // lane q = 0 of each obstacle block finds or creates the block's tile
        bool act = false, tnew = false;
        int32_t t = -1;
        if (q == 0 && i < n) {
            if (!ok) {
                set_error(g, -2 /* EDT_ERR_RANGE */);
            } else if (any) {
                t = hinsert(g.tkeys, g.tmask, pack_key(bx >> 3, by >> 3, bz >> 3), &tnew);
                if (t < 0) set_error(g, -3 /* EDT_ERR_CAPACITY */);
                else act = true;
            }
        }
        const int j = wave_append(tnew, &g.cnt[C_NTILE]);
        if (tnew) g.tlist[j] = t;
        // the wave's blocks of one tile merge their mask bits into one atomic
        // per mask word, and only the first of them sets the tile's flag
        const int local = block_local(bx, by, bz);
        const int word = act ? local >> 5 : -1;
        const uint32_t bit = act ? 1u << (local & 31) : 0u;
        const int32_t tk = act ? t : -1;
        uint32_t bits = 0u;
        bool wlead = act, tlead = act;
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
            const int32_t ot = __shfl(tk, 8 * s2);
            const int ow = __shfl(word, 8 * s2);
            const uint32_t ob = __shfl(bit, 8 * s2);
            if (act && ot == t) {
                if (8 * s2 < lane) tlead = false;
                if (ow == word) {
                    bits |= ob;
                    if (8 * s2 < lane) wlead = false;
                }
            }
        }
        if (wlead) atomicOr(&g.tobst[(int64_t)t * 16 + word], bits);
        bool first = false;
        if (tlead) first = atomicOr(&g.tflag[t], 1) == 0;
        grow_tiles(g, first, bx >> 3, by >> 3, bz >> 3);
    }
}

// Block list, phase 2 (after the dilation created and zeroed every slot): OR
// the bits in (repeated listings merge), one 64-bit word per lane.
template <bool BITS>
__global__ void __launch_bounds__(64) k_ingest_blocks_write(Grid g, const int32_t* xyz,
                                                           const uint8_t* data, int64_t n0,
                                                           const int32_t* n_dev) {
    const int lane = threadIdx.x, sub = lane >> 3, q = lane & 7;
    const int64_t n = n_dev ? (int64_t)*n_dev : n0;
    for (int64_t i0 = (int64_t)blockIdx.x * 8; i0 < n; i0 += (int64_t)gridDim.x * 8) {
        const int64_t i = i0 + sub;
        if (i >= n) continue;
        int bx, by, bz;
        bool ok;
        const unsigned long long rows = input_rows<BITS>(g, xyz, data, i, q, bx, by, bz, ok);
        if (!ok || rows == 0ull) continue;
        const int32_t slot = find_block(g, bx, by, bz);
        if (slot < 0) continue;
        atomicOr((unsigned long long*)g.occ + (int64_t)slot * 8 + q, rows);
    }
}

// ---------------------------------------------------------------------------
// region growth on tiles: every block within R blocks (Chebyshev) of an
// obstacle block joins the pool.  TR = ceil(R / 8) tiles of neighbourhood.
// ---------------------------------------------------------------------------
// One workgroup per tile: OR the obstacle masks of the tile neighbourhood
// shifted by -R..R along x, then y, then z (separable Chebyshev dilation on
// bit rows in LDS) and create the missing blocks of the dilated mask.  RT:
// the block radius R as a constant (1 .. 8, one tile of neighbourhood, loops
// unrolled), or 0 for any R read from the grid.
template <int RT>
__global__ void __launch_bounds__(64) k_tile_dilate(Grid g) {
    extern __shared__ uint32_t sm[];
    const int R = RT > 0 ? RT : g.R, TR = RT > 0 ? 1 : (R + 7) >> 3, w = 2 * TR + 1,
              NN = w * w * w;
    const int E = 8 + 2 * R;                 // rows of the dilation window per axis
    uint32_t* nmask = sm;                    // [NN][16] neighbour obstacle masks
    uint8_t* s1 = (uint8_t*)(sm + NN * 16);  // [E][E]  x-dilated rows (y', z')
    uint8_t* s2 = s1 + E * E;                // [E][8]  y-dilated rows (z', y)
    uint8_t* dil = s2 + E * 8;               // [64]    result rows (y, z)
    const int lane = threadIdx.x;
    const int64_t ntiles = g.cnt[C_NTILE];
    for (int64_t it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const int t = g.tlist[it];
        int tx, ty, tz;
        unpack_key(g.tkeys[t], tx, ty, tz);
        // this lane's 8 table entries (row y + 8z), read now so the load
        // overlaps the dilation; only this workgroup writes them
        const int64_t e0 = (int64_t)t * 512 + 8 * lane;
        const int4 ta = *(const int4*)(g.tslots + e0), tb = *(const int4*)(g.tslots + e0 + 4);
        for (int n = lane; n < NN; n += 64) {
            const int dx = n % w - TR, dy = (n / w) % w - TR, dz = n / (w * w) - TR;
            const int nt = (tx + dx < 0 || ty + dy < 0 || tz + dz < 0)
                               ? -1
                               : hpos(g.tkeys, g.tmask, pack_key(tx + dx, ty + dy, tz + dz));
            for (int k = 0; k < 16; ++k) nmask[n * 16 + k] = nt >= 0 ? g.tobst[(int64_t)nt * 16 + k] : 0u;
            // the tile and its face neighbours for the tile passes
            // (n = dx + 1 + 3 (dy + 1) + 9 (dz + 1) when TR = 1)
            if (TR == 1) {
                const int k = n == 13 ? 0 : n == 12 ? 1 : n == 14 ? 2 : n == 10 ? 3
                            : n == 16 ? 4 : n == 4 ? 5 : n == 22 ? 6 : -1;
                if (k >= 0) g.tinfo[it * 8 + k] = nt;
            }
        }
        __syncthreads();
        for (int r = lane; r < E * E; r += 64) {            // x dilation
            const int Y = r % E - R, Z = r / E - R;
            // the row across the w tiles along x: one mask byte per tile, bit
            // position X + 8 TR for X = -8 TR .. 8 + 8 TR - 1 (<= 72 bits)
            const int ny = ((Y >> 3) + TR), nz = ((Z >> 3) + TR);
            const int byte = (Y & 7) + 8 * (Z & 7);
            if (RT > 0) {
                // the row over the three tiles in 24 bits (bit 8 + X for
                // X = -8 .. 15); bit x of the result ORs bits 8 + x - R ..
                // 8 + x + R
                uint32_t row = 0u;
#pragma unroll
                for (int tx2 = 0; tx2 < 3; ++tx2) {
                    const int n = tx2 + 3 * (ny + 3 * nz);
                    row |= ((nmask[n * 16 + (byte >> 2)] >> (8 * (byte & 3))) & 0xffu) << (8 * tx2);
                }
                uint32_t d = 0u;
#pragma unroll
                for (int sh = 8 - RT; sh <= 8 + RT; ++sh) d |= row >> sh;
                s1[r] = (uint8_t)d;
                continue;
            }
            unsigned long long lo = 0ull, hi = 0ull;
            for (int tx2 = 0; tx2 < w; ++tx2) {
                const int n = tx2 + w * (ny + w * nz);
                const unsigned long long b =
                    (nmask[n * 16 + (byte >> 2)] >> (8 * (byte & 3))) & 0xffu;
                const int pos = 8 * tx2;
                if (pos < 64) lo |= b << pos;
                else hi |= b << (pos - 64);
            }
            uint32_t d = 0u;
            for (int x = 0; x < 8; ++x) {       // any bit in [x - R, x + R] + 8 TR
                const int a0 = x - R + 8 * TR, end = x + R + 8 * TR;
                const unsigned long long mlo =
                    (end >= 63 ? ~0ull : ((1ull << (end + 1)) - 1ull)) & (~0ull << a0);
                bool any = a0 < 64 && (lo & mlo) != 0ull;
                if (end >= 64) {
                    const int hs = a0 > 64 ? a0 - 64 : 0, he = end - 64;
                    const unsigned long long mhi =
                        (he >= 63 ? ~0ull : ((1ull << (he + 1)) - 1ull)) & (~0ull << hs);
                    any = any || (hi & mhi) != 0ull;
                }
                d |= (any ? 1u : 0u) << x;
            }
            s1[r] = (uint8_t)d;
        }
        __syncthreads();
        for (int r = lane; r < E * 8; r += 64) {            // y dilation
            const int y = r & 7, zp = r >> 3;
            uint32_t d = 0u;
#pragma unroll
            for (int dy = 0; dy <= 2 * (RT > 0 ? RT : 8); ++dy)
                if (RT > 0 || dy <= 2 * R) d |= s1[(y + dy) + E * zp];
            if (RT == 0)
                for (int dy = 17; dy <= 2 * R; ++dy) d |= s1[(y + dy) + E * zp];
            s2[r] = (uint8_t)d;
        }
        __syncthreads();
        {                                                   // z dilation, lane = y + 8z
            const int y = lane & 7, z = lane >> 3;
            uint32_t d = 0u;
#pragma unroll
            for (int dz = 0; dz <= 2 * (RT > 0 ? RT : 8); ++dz)
                if (RT > 0 || dz <= 2 * R) d |= s2[y + 8 * (z + dz)];
            if (RT == 0)
                for (int dz = 17; dz <= 2 * R; ++dz) d |= s2[y + 8 * (z + dz)];
            dil[lane] = (uint8_t)d;
        }
        __syncthreads();
        // create the dilated blocks that are missing; lane = row (y, z), its
        // 8 table entries are 8 lane .. 8 lane + 7.  One counter atomic per
        // tile; the new slots are contiguous.
        const int y = lane & 7, z = lane >> 3;
        const int by = 8 * ty + y, bz = 8 * tz + z;
        const uint32_t d = dil[lane];
        const int32_t ex[8] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
        const int nc = TR + w * (TR + w * TR);            // centre tile in nmask
        const uint32_t ob = (nmask[nc * 16 + (lane >> 2)] >> (8 * (lane & 3))) & 0xffu;
        uint32_t want = 0u;
#pragma unroll
        for (int x = 0; x < 8; ++x)
            if (((d >> x) & 1u) && 8 * tx + x < g.nbx && by < g.nby && bz < g.nbz && ex[x] == -1)
                want |= 1u << x;
        const int c = __popc(want);
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        const int total = __shfl(incl, 63);
        // obstacle blocks created here (block-list input) are counted as
        // obstacle blocks; one 64-bit atomic advances both the block count
        // (low word) and that count (high word)
        const int nobst = wave_sum(__popc(want & ob));
        if (total > 0) {
            int base = 0;
            if (lane == 0) {
                static_assert(C_NDIL == C_NBLK + 1 && C_NBLK == 0, "adjacent counters");
                const unsigned long long old = atomicAdd(
                    (unsigned long long*)&g.cnt[C_NBLK],
                    (unsigned long long)total | ((unsigned long long)nobst << 32));
                base = (int)(uint32_t)old;
            }
            base = __shfl(base, 0);
            int slot = base + incl - c;
#pragma unroll
            for (int x = 0; x < 8; ++x) {
                if (!((want >> x) & 1u)) continue;
                const bool o = (ob >> x) & 1u;
                if (slot < g.max_blocks) {
                    g.tslots[e0 + x] = slot;
                    g.bkey[slot] = pack_key(8 * tx + x, by, bz);
                    g.flags[slot] = o ? F_DILATED : 0u;
                } else {
                    g.tslots[e0 + x] = -1;
                    set_error(g, -3 /* EDT_ERR_CAPACITY */);
                    g.cnt[C_ABORT] = 1;
                }
                ++slot;
            }
            // zero the occupancy and change masks of the new slots
            // [base, base + total), 16-byte stores (4 per mask of 64 bytes)
            const int64_t lo = base, hi = min((int64_t)base + total, (int64_t)g.max_blocks);
            const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
            for (int64_t k = lo * 4 + lane; k < hi * 4; k += 64) {
                ((uint4*)g.occ)[k] = zero;
                ((uint4*)g.chg_add)[k] = zero;
                ((uint4*)g.chg_rem)[k] = zero;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// work items: run starts along `axis` (1 = y, 2 = z)
// ---------------------------------------------------------------------------
__device__ inline bool run_member(const Grid& g, int32_t slot, uint32_t runflag) {
    return slot >= 0 && (runflag == 0u || (g.flags[slot] & runflag));
}

// A block starts a work item along `axis` when it is the first member of a
// run (the previous block is absent or not a member) or sits on an LRUN
// boundary.  axes: 1 = y only, 2 = z only, 3 = both (global transform).
__device__ inline bool run_start(const Grid& g, int bx, int by, int bz, int axis,
                                 uint32_t runflag) {
    const int c = axis == 1 ? by : bz;
    if (c % g.lrun == 0) return true;
    return !run_member(g, axis == 1 ? find_block(g, bx, by - 1, bz) : find_block(g, bx, by, bz - 1),
                       runflag);
}

// y items from the ys list and z items from the dirty list in one launch
// (incremental transform).
// Workgroups vb of vgrid (of blockDim.x threads) share the lists.
__device__ inline void items_update_body(const Grid& g, int64_t vb, int64_t vgrid) {
    const int64_t ny = min((int64_t)g.cnt[C_NYS], (int64_t)g.max_blocks);
    const int64_t nd = min((int64_t)g.cnt[C_NDIRTY], (int64_t)g.max_blocks);
    // a wave takes entries of one list only (the y part is padded to 64)
    const int64_t nyp = (ny + 63) & ~(int64_t)63;
    for (int64_t i = vb * blockDim.x + threadIdx.x; i - __lane_id() < nyp + nd;
         i += vgrid * blockDim.x) {
        const bool zpart = i - __lane_id() >= nyp;
        const int64_t k = zpart ? i - nyp : i;
        const bool ok = zpart ? k < nd : k < ny;
        bool st = false;
        int32_t slot = -1;
        if (ok) {
            slot = zpart ? g.list_dirty[k] : g.list_ys[k];
            int bx, by, bz;
            unpack_key(g.bkey[slot], bx, by, bz);
            st = run_start(g, bx, by, bz, zpart ? 2 : 1, zpart ? F_DIRTY : F_YS);
        }
        const int idx = wave_append(st, &g.cnt[zpart ? C_NZI : C_NYI]);
        if (st) (zpart ? g.list_zi : g.list_yi)[idx] = slot;
    }
}

// ---------------------------------------------------------------------------
// per-tile variants for the global transform
// ---------------------------------------------------------------------------
// Slot of the block at position a in [-8, 16) along one axis of a tile row
// or column (other coordinates inside the tile; `local` is the in-tile
// index with that axis' coordinate zero, `stride` its step): the tile below,
// the tile itself or the tile above, from the face neighbours recorded by
// the dilation.
__device__ inline int32_t axis_slot(const Grid& g, int lo, int self, int hi, int a, int local,
                                    int stride) {
    const int t = a < 0 ? lo : (a >= 8 ? hi : self);
    return t < 0 ? -1 : g.tslots[(int64_t)t * 512 + local + stride * (a & 7)];
}

// Slot of the block at tile-relative position (x, y, z) (each coordinate in
// [-8, 16)) of the tile at `tpos`, whose tile coordinates are (tx, ty, tz);
// neighbouring tiles are looked up in the tile hash.
__device__ inline int32_t tile_rel_slot(const Grid& g, int tpos, int tx, int ty, int tz, int x,
                                        int y, int z) {
    const int dx = x >> 3, dy = y >> 3, dz = z >> 3;
    int t = tpos;
    if (dx | dy | dz) {
        const int ax = tx + dx, ay = ty + dy, az = tz + dz;
        if (ax < 0 || ay < 0 || az < 0) return -1;
        t = hpos(g.tkeys, g.tmask, pack_key(ax, ay, az));
        if (t < 0) return -1;
    }
    return g.tslots[(int64_t)t * 512 + (x & 7) + 8 * (y & 7) + 64 * (z & 7)];
}

// Work items of the global transform, one workgroup per tile: a block starts
// a y (z) item when it sits on an LRUN boundary or the block before it along
// y (z) is absent.
__global__ void __launch_bounds__(64) k_items_tiles(Grid g) {
    __shared__ int32_t own[512];
    __shared__ int32_t below[64];     // (x, 7, z) of the tile at ty - 1
    __shared__ int32_t behind[64];    // (x, y, 7) of the tile at tz - 1
    const int lane = threadIdx.x;
    const int64_t ntiles = g.cnt[C_NTILE];
    for (int64_t it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const int t = g.tlist[it];
        int tx, ty, tz;
        unpack_key(g.tkeys[t], tx, ty, tz);
        for (int i = lane; i < 512; i += 64) own[i] = g.tslots[(int64_t)t * 512 + i];
        below[lane] = tile_rel_slot(g, t, tx, ty, tz, lane & 7, -1, lane >> 3);
        behind[lane] = tile_rel_slot(g, t, tx, ty, tz, lane & 7, lane >> 3, -1);
        __syncthreads();
        for (int i = lane; i < 512; i += 64) {
            const int x = i & 7, y = (i >> 3) & 7, z = i >> 6;
            const int32_t slot = own[i];
            const int by = 8 * ty + y, bz = 8 * tz + z;
            const bool ex = slot >= 0;
            const int32_t py = y > 0 ? own[i - 8] : below[x + 8 * z];
            const int32_t pz = z > 0 ? own[i - 64] : behind[x + 8 * y];
            const bool sy = ex && ((by % g.lrun) == 0 || py < 0);
            const bool sz = ex && ((bz % g.lrun) == 0 || pz < 0);
            const int jy = wave_append(sy, &g.cnt[C_NYI]);
            if (sy) g.list_yi[jy] = slot;
            const int jz = wave_append(sz, &g.cnt[C_NZI]);
            if (sz) g.list_zi[jz] = slot;
        }
        __syncthreads();
    }
}

// pass X for the global transform: one wave per row of 8 blocks along x
// inside a tile (64 per tile), lane = row (y + 8z) of the blocks.  Each lane
// sweeps its row twice with a carried distance (left to right, then right to
// left inside each block); a voxel's distance to the nearest obstacle along x
// is the smaller of the two, capped at d_max (M = R <= 8 blocks of context on
// each side cover d_max <= 64).  The squared values are transposed through
// LDS so that every lane stores 16 contiguous bytes of the y-major g1 block.
template <int M>
__global__ void __launch_bounds__(64) k_pass_x_rows(Grid g) {
    constexpr int NB = 8 + 2 * M;
    constexpr uint32_t FAR = 1u << 20;
    __shared__ int32_t sl[NB];
    __shared__ uint4 tr[2][72];       // row r at r + r / 8: conflict-free reads
    const int lane = threadIdx.x;
    const int64_t nrows = (int64_t)g.cnt[C_NTILE] * 64;
    const uint8_t* occ8 = (const uint8_t*)g.occ;
    const uint32_t dmax = (uint32_t)g.dmax;
    for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
        const int32_t* ti = g.tinfo + (it >> 6) * 8;
        const int jy = (int)(it & 7), jz = (int)((it >> 3) & 7);
        // raised priority for the chain of lookups and loads, as in the
        // window passes
        __builtin_amdgcn_s_setprio(2);
        if (lane < NB) sl[lane] = axis_slot(g, ti[1], ti[0], ti[2], lane - M, 8 * jy + 64 * jz, 1);
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int j = 0; j < 8; ++j) any = any || sl[M + j] >= 0;
        if (any) {
            uint32_t b[NB];
            uint32_t orb = 0u;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int32_t s2 = sl[k];
                b[k] = s2 >= 0 ? (uint32_t)occ8[(int64_t)s2 * 64 + lane] : 0u;
                orb |= b[k];
            }
            __builtin_amdgcn_s_setprio(0);
            if (!__any(orb != 0u)) {
                // no obstacle in the strip or its context: every g1 is D,
                // and a block that is D everywhere needs only its minimum
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int32_t slot = sl[M + j];
                    if (lane == 0 && slot >= 0) g.bmin1[slot] = (uint16_t)g.D;
                }
                __syncthreads();
                continue;
            }
            // distance from the last voxel before the central blocks back to
            // the nearest obstacle at or before it
            uint32_t L = FAR;
#pragma unroll
            for (int k = 0; k < M; ++k) L = b[k] ? (uint32_t)__clz(b[k]) - 24u : L + 8u;
            // rc[j]: distance from the first voxel after central block j to
            // the nearest obstacle at or after it
            uint32_t rc[8];
            uint32_t R = FAR;
#pragma unroll
            for (int k = NB - 1; k >= M + 8; --k) R = b[k] ? (uint32_t)(__ffs(b[k]) - 1) : R + 8u;
#pragma unroll
            for (int j = 7; j >= 0; --j) {
                rc[j] = R;
                const uint32_t bj = b[M + j];
                R = bj ? (uint32_t)(__ffs(bj) - 1) : R + 8u;
            }
            // least g1 of each block: 0 on a row holding an obstacle, else set
            // by the end voxels (voxel 0 is nearest the left obstacle, voxel 7
            // the right one).  lc: distance from the voxel before block j to
            // the nearest obstacle at or before it.  The squares (<= 64^2) are
            // reduced over the wave two blocks at a time, packed.
            uint32_t bmins[4];
            {
                uint32_t lc = L, nsq[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t bj = b[M + j];
                    const uint32_t near = bj ? 0u : min(min(lc + 1u, rc[j] + 1u), dmax);
                    nsq[j] = near * near;
                    lc = bj ? (uint32_t)__clz(bj) - 24u : lc + 8u;
                }
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    bmins[h] = wave_reduce_pk_u16<false>(nsq[2 * h] | (nsq[2 * h + 1] << 16));
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t bj = b[M + j];
                const int bmin = (int)((bmins[j >> 1] >> (16 * (j & 1))) & 0xffffu);
                uint32_t m[8], d[8];
#pragma unroll
                for (int x = 0; x < 8; ++x) m[x] = (uint32_t)((int32_t)(bj << (31 - x)) >> 31);
#pragma unroll
                for (int x = 0; x < 8; ++x) { L = (L + 1u) & ~m[x]; d[x] = L; }
                uint32_t r = rc[j];
#pragma unroll
                for (int x = 7; x >= 0; --x) {
                    r = (r + 1u) & ~m[x];
                    const uint32_t v = min(min(d[x], r), dmax);
                    d[x] = win_f16(M) ? (uint32_t)__builtin_bit_cast(unsigned short,
                                                                     (_Float16)(v * v))
                                      : v * v;
                }
                const int32_t slot = sl[M + j];
                if (lane == 0 && slot >= 0) g.bmin1[slot] = (uint16_t)bmin;
                // a block that is D everywhere is not stored: its readers see
                // the block minimum D and take the shared D block instead
                if (slot >= 0 && bmin < g.D) {
                    uint4* buf = tr[j & 1];
                    buf[lane + (lane >> 3)] = make_uint4(d[0] | (d[1] << 16), d[2] | (d[3] << 16),
                                                         d[4] | (d[5] << 16), d[6] | (d[7] << 16));
                    __syncthreads();
                    // lane = x + 8z gathers column x of rows y + 8z, y = 0..7
                    const uint16_t* t16 = (const uint16_t*)buf + 72 * (lane >> 3) + (lane & 7);
                    uint32_t w[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        w[q] = (uint32_t)t16[16 * q] | ((uint32_t)t16[16 * q + 8] << 16);
                    *reinterpret_cast<uint4*>(g.g1 + (int64_t)slot * 512 + 8 * lane) =
                        make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// pass X: squared 1-D distance along x from the bits, clamped to D.  One wave
// per block, lane = row (y + 8z).
// ---------------------------------------------------------------------------
__device__ inline void pass_x_body(const Grid& g, const int32_t* list, int list_counter,
                                   int64_t vb, int64_t vgrid, int32_t* nb) {
    const int lane = threadIdx.x;
    const int64_t n0 = list ? g.cnt[list_counter] : g.cnt[C_NBLK];
    const int64_t n = n0 < g.max_blocks ? n0 : g.max_blocks;
    const int R = g.R;
    const uint8_t* occ8 = (const uint8_t*)g.occ;
    for (int64_t w = vb; w < n; w += vgrid) {
        const int32_t slot = list ? list[w] : (int32_t)w;
        int bx, by, bz;
        unpack_key(g.bkey[slot], bx, by, bz);
        for (int i = lane; i < 2 * R + 1; i += 64)
            nb[i] = (i == R) ? slot : find_block(g, bx - R + i, by, bz);
        __syncthreads();
        const uint32_t c = occ8[(int64_t)slot * 64 + lane];
        int prev = -100000, next = 100000;
        if (R <= 8) {
            // issue all neighbour loads at once, then scan in registers
            uint32_t lb[8], rb[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t sl = k < R ? nb[R - 1 - k] : -1;
                const int32_t sr = k < R ? nb[R + 1 + k] : -1;
                lb[k] = sl >= 0 ? (uint32_t)occ8[(int64_t)sl * 64 + lane] : 0u;
                rb[k] = sr >= 0 ? (uint32_t)occ8[(int64_t)sr * 64 + lane] : 0u;
            }
#pragma unroll
            for (int k = 7; k >= 0; --k) {
                if (lb[k]) prev = -8 * (k + 1) + (31 - __clz(lb[k]));
                if (rb[k]) next = 8 * (k + 1) + (__ffs(rb[k]) - 1);
            }
        } else {
            for (int k = 1; k <= R; ++k) {
                const int32_t s2 = nb[R - k];
                if (s2 < 0) continue;
                const uint32_t b = occ8[(int64_t)s2 * 64 + lane];
                if (b) { prev = -8 * k + (31 - __clz(b)); break; }
            }
            for (int k = 1; k <= R; ++k) {
                const int32_t s2 = nb[R + k];
                if (s2 < 0) continue;
                const uint32_t b = occ8[(int64_t)s2 * 64 + lane];
                if (b) { next = 8 * k + (__ffs(b) - 1); break; }
            }
        }
        int dl[8];
        int p = prev;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            if ((c >> x) & 1u) p = x;
            dl[x] = x - p;
        }
        int q = next;
        const int y = lane & 7, z = lane >> 3;
        const int dmax = g.dmax;
        uint16_t* dst = g.g1 + (int64_t)slot * 512 + 64 * z + y;
        int mn = dmax;
        const bool f16 = win_f16(R);
#pragma unroll
        for (int x = 7; x >= 0; --x) {
            if ((c >> x) & 1u) q = x;
            const int d = min(min(dl[x], q - x), dmax);
            dst[8 * x] = f16 ? __builtin_bit_cast(uint16_t, (_Float16)(d * d)) : (uint16_t)(d * d);
            mn = min(mn, d);
        }
        mn = (int)(wave_reduce_pk_u16<false>((uint32_t)(mn * mn)) & 0xffffu);
        if (lane == 0) g.bmin1[slot] = (uint16_t)mn;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) k_pass_x(Grid g, const int32_t* list, int list_counter) {
    __shared__ int32_t nb[72];
    pass_x_body(g, list, list_counter, blockIdx.x, gridDim.x, nb);
}

// Incremental transform: pass x over the xs list and the y / z work items
// are independent, so they share one launch; the first nxw workgroups take
// pass x.
__global__ void __launch_bounds__(64) k_upd_x_items(Grid g, int nxw) {
    __shared__ int32_t nb[72];
    // no kernel from here on reads the cancel mark: clear it for the next call
    if (blockIdx.x == 0 && threadIdx.x == 0) g.cnt[C_UABORT] = 0;
    if ((int)blockIdx.x < nxw) pass_x_body(g, g.list_xs, C_NXS, blockIdx.x, nxw, nb);
    else items_update_body(g, (int64_t)blockIdx.x - nxw, (int64_t)gridDim.x - nxw);
}

// ---------------------------------------------------------------------------
// streaming lower envelope of parabolas, one row per lane
// ---------------------------------------------------------------------------
// Sites are pushed in increasing position q with value f < D; outputs are
// evaluated at i = q - dmax once every site that can reach i is in.  The
// envelope is kept only on [next output, inf): the bottom site is removed
// when the new site is no worse at the next output, and sites more than dmax
// left of the output (values > D) are dropped.  The live sites then lie in a
// window of 2*dmax + 2 positions, which bounds the ring.  The two sites at
// each end of the envelope are mirrored in registers, so LDS is read only
// when a site is popped from the top or passed at the bottom.
struct Envelope {
    uint32_t* ring;   // LDS, entry e of this lane at ring[e * 64 + lane]
    int cap;          // ring capacity (entries)
    int lane;
    int n;            // live entries
    int bp, tp;       // physical bottom / top index
    uint32_t t0, t1;  // top, below top      (entry = position << 16 | value)
    uint32_t b0, b1;  // bottom, above bottom

    __device__ void init(uint32_t* r, int c, int l) {
        ring = r; cap = c; lane = l; n = 0; bp = 0; tp = c - 1; t0 = t1 = b0 = b1 = 0u;
    }
    __device__ int inc(int p) const { return p + 1 == cap ? 0 : p + 1; }
    __device__ int dec(int p) const { return p == 0 ? cap - 1 : p - 1; }
    __device__ uint32_t at(int phys) const { return ring[phys * 64 + lane]; }
    static __device__ int pos(uint32_t e) { return (int)(e >> 16); }
    static __device__ int val(uint32_t e) { return (int)(e & 0xffffu); }

    __device__ void push(int q, int f, int inext) {
        const int kq = f + q * q;
        while (n > 0) {
            const int pt = pos(t0);
            const int kt = val(t0) + pt * pt;
            if (n == 1) {
                // the only site: drop it if the new one is no worse on [inext, inf)
                if (kq - kt <= 2 * inext * (q - pt)) {
                    n = 0;
                    tp = dec(bp);
                }
                break;
            }
            const int p0 = pos(t1);
            const int k0 = val(t1) + p0 * p0;
            // top is hidden when the new site meets t1 no later than top does
            if ((kq - k0) * (pt - p0) <= (kt - k0) * (q - p0)) {
                tp = dec(tp);
                --n;
                t0 = t1;
                if (n >= 2) t1 = at(dec(tp));
            } else {
                break;
            }
        }
        tp = inc(tp);
        const uint32_t e = ((uint32_t)q << 16) | (uint32_t)f;
        ring[tp * 64 + lane] = e;
        ++n;
        t1 = t0;
        t0 = e;
        if (n == 1) b0 = e;
        else if (n == 2) b1 = e;
    }

    __device__ void advance() {
        bp = inc(bp);
        --n;
        if (n >= 1) b0 = b1;
        if (n >= 2) b1 = at(inc(bp));
    }

    // min over live sites of f + (i - p)^2, clamped to D
    __device__ int eval(int i, int dmax, int D) {
        while (n > 0 && pos(b0) < i - dmax) advance();
        if (n == 0) return D;
        int d0 = i - pos(b0);
        int vb = val(b0) + d0 * d0;
        while (n >= 2) {
            const int d1 = i - pos(b1);
            const int v1 = val(b1) + d1 * d1;
            if (v1 > vb) break;
            advance();
            vb = v1;
        }
        return vb < D ? vb : D;
    }
};

// Resolve the run of a y/z work item into LDS: sl[0 .. LRUN + 2R) holds the
// slots of blocks start-R .. start+LRUN+R-1 along `axis` (-1 = absent).
// Returns (hb, len, ha): halo blocks before, run length, halo blocks after.
__device__ inline void resolve_run(const Grid& g, int32_t* sl, uint8_t* mem, int bx, int by,
                                   int bz, int axis, uint32_t runflag, int& hb, int& len,
                                   int& ha) {
    const int R = g.R;
    const int nl = g.lrun + 2 * R;
    const int lane = threadIdx.x;
    for (int i = lane; i < nl; i += 64) {
        const int o = i - R;
        const int32_t s = axis == 1 ? find_block(g, bx, by + o, bz) : find_block(g, bx, by, bz + o);
        sl[i] = s;
        mem[i] = run_member(g, s, runflag) ? 1 : 0;
    }
    __syncthreads();
    const int start = axis == 1 ? by : bz;
    hb = 0;
    while (hb < R && sl[R - 1 - hb] >= 0) ++hb;
    len = 1;
    while (len < g.lrun && ((start + len) % g.lrun) != 0 && mem[R + len]) ++len;
    ha = 0;
    while (ha < R && sl[R + len + ha] >= 0) ++ha;
}

// An incremental pass is done with the run's own blocks (sl[R .. R + len))
// once its outputs are stored: pass Y clears their g1 / g2 marks and the seed
// mark, pass Z the front marks, so the next update starts with clean flags.
// Runs of one pass never share a block, and a run only reads the membership
// of its own blocks, so clearing cannot change another run.
__device__ inline void finish_run(const Grid& g, const int32_t* sl, int len, int axis,
                                  uint32_t runflag) {
    if (runflag == 0u) return;                  // global transform: no marks
    const uint32_t clear =
        axis == 1 ? (F_YS | F_XS | F_SEED | F_DILNEW) : (F_DIRTY | F_RAISE | F_LOWER);
    const int lane = threadIdx.x;
    if (lane < len) atomicAnd(&g.flags[sl[g.R + lane]], ~clear);
}

// The envelope passes walk the blocks of a work item two at a time with two
// explicit input buffers (no register copies), and every step issues exactly
// one global store (halo steps store to a per-wave scratch row), so the
// memory operations form a fixed sequence and a step never waits for the
// stores of the steps before it.
//
// pass Y: lane = x + 8z.  Reads g1 (layout (x + 8z) * 8 + y: one 16-byte
// load per block and lane), writes g2 (layout (x + 8y) * 8 + z) and the
// least g2 value of each output block (bmin2, read by the nearest-obstacle
// query to tell blocks that are D everywhere).
struct PassYItem {
    const Grid& g;
    const int32_t* sl;
    Envelope& env;
    int base, nb, o0, o1, qa, qb, dmax, D, lane, out_lane;
    uint16_t* dummy;
    int bm;

    __device__ uint4 load(int j) const {
        const int jj = j < nb ? j : nb - 1;
        return ((const uint4*)g.g1)[(int64_t)sl[base + jj] * 64 + lane];
    }
    __device__ void block(uint4 cur, int j) {
        const int jo = (j * 8 - dmax) >> 3;
        const int32_t slo = (jo >= 0 && jo < nb) ? sl[base + jo] : -1;
        const int32_t shi = (jo + 1 >= 0 && jo + 1 < nb) ? sl[base + jo + 1] : -1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * j + k;
            if (q >= qa && q < qb) {
                const uint32_t wk = k < 2 ? cur.x : (k < 4 ? cur.y : (k < 6 ? cur.z : cur.w));
                const int f = (int)((wk >> (16 * (k & 1))) & 0xffffu);
                if (f < D) env.push(q, f, max(o0, q - dmax));
            }
            const int i = q - dmax;
            const bool out = i >= o0 && i < o1;
            int v = 0;
            if (out) v = env.eval(i, dmax, D);
            const int32_t slot = ((i >> 3) == jo) ? slo : shi;
            uint16_t* dst = out ? g.g2 + (int64_t)slot * 512 + out_lane + 64 * (i & 7)
                                : dummy + lane;
            *dst = (uint16_t)v;
            bm = min(bm, v);
            if (((k - dmax) & 7) == 7) {          // the step that ends an output block
                const int m = wave_min(bm);
                uint16_t* bd = out ? g.bmin2 + slot : dummy + 64 + lane;
                *bd = (uint16_t)m;
                bm = D;
            }
        }
    }
};

__global__ void __launch_bounds__(64) k_pass_y(Grid g, const int32_t* items, int item_counter,
                                               uint32_t runflag, int cap) {
    extern __shared__ uint32_t smem[];
    int32_t* sl = (int32_t*)smem;                 // 96 entries
    uint8_t* mem = (uint8_t*)(smem + 96);         // 96 bytes
    uint32_t* ring = smem + 96 + 24;
    const int lane = threadIdx.x;
    const int64_t nit = g.cnt[item_counter];
    const int R = g.R;
    uint16_t* dummy = (uint16_t*)(g.dummy + (blockIdx.x & 255) * 64);
    for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
        const int32_t s0 = items[it];
        int bx, by, bz;
        unpack_key(g.bkey[s0], bx, by, bz);
        int hb, len, ha;
        resolve_run(g, sl, mem, bx, by, bz, 1, runflag, hb, len, ha);
        Envelope env;
        env.init(ring, cap, lane);
        const int nb = hb + len + ha;
        const int o0 = 8 * hb, o1 = 8 * (hb + len);
        PassYItem P{g, sl, env, R - hb, nb, o0, o1, max(0, o0 - g.dmax), min(8 * nb, o1 + g.dmax),
                    g.dmax, g.D, lane, (lane & 7) * 8 + (lane >> 3), dummy, g.D};
        const int jlo = P.qa >> 3, jhi = (o1 + g.dmax - 1) >> 3;
        uint4 A = P.load(jlo), B = P.load(jlo + 1);
        for (int j = jlo; j <= jhi; j += 2) {
            P.block(A, j);
            A = P.load(j + 2);
            if (j + 1 > jhi) break;
            P.block(B, j + 1);
            B = P.load(j + 3);
        }
        finish_run(g, sl, len, 1, runflag);
        __syncthreads();
    }
}

// pass Z: lane = x + 8y.  Reads g2 (one 16-byte load per block and lane),
// writes s (uint16, layout x + 8y + 64z) and the per-block maximum.
struct PassZItem {
    const Grid& g;
    const int32_t* sl;
    Envelope& env;
    int base, nb, o0, o1, qa, qb, dmax, D, lane;
    int32_t* dummy;
    int bm;

    __device__ uint4 load(int j) const {
        const int jj = j < nb ? j : nb - 1;
        return ((const uint4*)g.g2)[(int64_t)sl[base + jj] * 64 + lane];
    }
    __device__ void block(uint4 cur, int j) {
        const int jo = (j * 8 - dmax) >> 3;
        const int32_t slo = (jo >= 0 && jo < nb) ? sl[base + jo] : -1;
        const int32_t shi = (jo + 1 >= 0 && jo + 1 < nb) ? sl[base + jo + 1] : -1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * j + k;
            if (q >= qa && q < qb) {
                const uint32_t wk = k < 2 ? cur.x : (k < 4 ? cur.y : (k < 6 ? cur.z : cur.w));
                const int f = (int)((wk >> (16 * (k & 1))) & 0xffffu);
                if (f < D) env.push(q, f, max(o0, q - dmax));
            }
            const int i = q - dmax;
            const bool out = i >= o0 && i < o1;
            int v = 0;
            if (out) v = env.eval(i, dmax, D);
            const int32_t slot = ((i >> 3) == jo) ? slo : shi;
            uint16_t* dst =
                out ? g.s + (int64_t)slot * 512 + lane + 64 * (i & 7) : (uint16_t*)dummy + lane;
            *dst = (uint16_t)v;
            bm = max(bm, v);
            if (((k - dmax) & 7) == 7) {          // the step that ends an output block
                const int m = wave_max(bm);
                int32_t* bd = out ? g.bmax + slot : dummy + 64 + lane;
                *bd = m;
                bm = 0;
            }
        }
    }
};

__global__ void __launch_bounds__(64) k_pass_z(Grid g, const int32_t* items, int item_counter,
                                               uint32_t runflag, int cap) {
    extern __shared__ uint32_t smem[];
    int32_t* sl = (int32_t*)smem;
    uint8_t* mem = (uint8_t*)(smem + 96);
    uint32_t* ring = smem + 96 + 24;
    const int lane = threadIdx.x;
    const int64_t nit = g.cnt[item_counter];
    const int R = g.R;
    int32_t* dummy = (int32_t*)(g.dummy + (blockIdx.x & 255) * 64);
    for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
        const int32_t s0 = items[it];
        int bx, by, bz;
        unpack_key(g.bkey[s0], bx, by, bz);
        int hb, len, ha;
        resolve_run(g, sl, mem, bx, by, bz, 2, runflag, hb, len, ha);
        Envelope env;
        env.init(ring, cap, lane);
        const int nb = hb + len + ha;
        const int o0 = 8 * hb, o1 = 8 * (hb + len);
        PassZItem P{g, sl, env, R - hb, nb, o0, o1, max(0, o0 - g.dmax), min(8 * nb, o1 + g.dmax),
                    g.dmax, g.D, lane, dummy, 0};
        const int jlo = P.qa >> 3, jhi = (o1 + g.dmax - 1) >> 3;
        uint4 A = P.load(jlo), B = P.load(jlo + 1);
        for (int j = jlo; j <= jhi; j += 2) {
            P.block(A, j);
            A = P.load(j + 2);
            if (j + 1 > jhi) break;
            P.block(B, j + 1);
            B = P.load(j + 3);
        }
        finish_run(g, sl, len, 2, runflag);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// windowed minimum along y or z for d_max <= 64 (core in edt_win.h)
// ---------------------------------------------------------------------------
// The stored field s holds integers (uint16), or for radii whose window runs
// in binary16 (win_f16) the binary16 bit patterns of those integers, as the
// window computes them; readers take the integer with s_int / s_pair_int.
__device__ inline int s_int(const Grid& g, uint32_t bits) {
    return win_f16(g.R) ? f16_int(bits) : (int)bits;
}
__device__ inline uint32_t s_pair_int(const Grid& g, uint32_t w) {
    return win_f16(g.R) ? ((uint32_t)f16_int(w & 0xffffu) | ((uint32_t)f16_int(w >> 16) << 16))
                        : w;
}

// Stores the results of one step of the windowed minimum: acc[o] holds output
// row o of two consecutive blocks (low half: slot0, high half: slot1; a
// negative slot has no storage and its half is dropped).  Pass Y writes g2
// (z-major rows) and the block minima; pass Z writes s and the block maxima.
// The slots are wave-uniform, so the branches are scalar and each store
// takes its block's base from scalar registers and the row from an
// immediate offset.  The block extrema are reduced on the packed values,
// both blocks at once (binary16 patterns of non-negative values order like
// the values).
template <int AXIS, bool F16>
__device__ inline void win_store(const Grid& g, int32_t slot0, int32_t slot1, const u16x2* acc,
                                 int lane) {
    if (AXIS == 1) {
        const int out_lane = (lane & 7) * 8 + (lane >> 3);
        if (slot0 >= 0) {
            uint16_t* d0 = g.g2 + (int64_t)slot0 * 512 + out_lane;
#pragma unroll
            for (int o = 0; o < 8; ++o) d0[64 * o] = acc[o].x;
        }
        if (slot1 >= 0) {
            uint16_t* d1 = g.g2 + (int64_t)slot1 * 512 + out_lane;
#pragma unroll
            for (int o = 0; o < 8; ++o) d1[64 * o] = acc[o].y;
        }
        // least output of each block, for the skip bounds of pass Z
        const uint32_t m = wave_reduce_pk_u16<false>(as_u32(min8<F16>(acc)));
        if (lane == 0) {
            if (slot0 >= 0) g.bmin2[slot0] = F16 ? (uint16_t)f16_int(m & 0xffffu) : (uint16_t)m;
            if (slot1 >= 0) g.bmin2[slot1] = F16 ? (uint16_t)f16_int(m >> 16) : (uint16_t)(m >> 16);
        }
    } else {
        // s is written once and not read again by the transform: the
        // stores are marked non-temporal (streamed past the caches)
        const uint32_t m = wave_reduce_pk_u16<true>(as_u32(max8<F16>(acc)));
        if (slot0 >= 0) {
            uint16_t* d0 = g.s + (int64_t)slot0 * 512 + lane;
#pragma unroll
            for (int o = 0; o < 8; ++o) __builtin_nontemporal_store(acc[o].x, &d0[64 * o]);
            if (lane == 0) g.bmax[slot0] = F16 ? f16_int(m & 0xffffu) : (int)(m & 0xffffu);
        }
        if (slot1 >= 0) {
            uint16_t* d1 = g.s + (int64_t)slot1 * 512 + lane;
#pragma unroll
            for (int o = 0; o < 8; ++o) __builtin_nontemporal_store(acc[o].y, &d1[64 * o]);
            if (lane == 0) g.bmax[slot1] = F16 ? f16_int(m >> 16) : (int)(m >> 16);
        }
    }
}

// List-driven form: one wave per work item (a run of up to LRUN blocks,
// extended by the halo of resolve_run).
template <int M, int AXIS>
__global__ void __launch_bounds__(64) k_pass_win(Grid g, const int32_t* items, int item_counter,
                                                 uint32_t runflag) {
    __shared__ int32_t sl[96];
    __shared__ uint8_t mem[96];
    const int lane = threadIdx.x;
    const int64_t nit = g.cnt[item_counter];
    const uint16_t* src = AXIS == 1 ? g.g1 : g.g2;
    constexpr bool F16 = win_f16(M);
    const uint32_t Dw = F16 ? f16_bits((uint32_t)g.D) : (uint32_t)g.D;
    const uint32_t Dp = Dw | (Dw << 16);      // D in the window's representation
    for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
        const int32_t s0 = items[it];
        int bx, by, bz;
        unpack_key(g.bkey[s0], bx, by, bz);
        int hb, len, ha;
        resolve_run(g, sl, mem, bx, by, bz, AXIS, runflag, hb, len, ha);
        const int base = M - hb;          // sl index of item block 0
        const int nb = hb + len + ha;
        // skip masks over window positions j (block hb - M + j of the run,
        // the window of output block hb): least input of the block, D for
        // absent blocks and past the run
        const uint16_t* bmin = AXIS == 1 ? g.bmin1 : g.bmin2;
        int bm = g.D;
        {
            const int b = hb - M + lane;
            if (b >= 0 && b < nb) {
                const int32_t s2 = sl[base + b];
                if (s2 >= 0) bm = bmin[s2];
            }
        }
        WinSkip sk;
        sk.d = __ballot(bm >= g.D);
#pragma unroll
        for (int G = 0; G < M; ++G) {
            const int kg = G == 0 ? 1 : 8 * G;
            sk.g[G] = __ballot(bm + kg * kg >= g.D);
        }
        auto blk = [&](int b) -> uint4 {
            const int j = b - hb + M;
            const bool own = b >= 0 && b < nb && !((sk.d >> j) & 1ull);
            const int32_t s2 = own ? sl[base + b] : -1;
            const uint4* p = s2 >= 0 ? (const uint4*)src + (int64_t)s2 * 64 + lane
                                     : (const uint4*)g.dblock + lane;
            return *p;
        };
        auto emit = [&](int ob, const u16x2* acc, bool has1) {
            const int32_t slot0 = __builtin_amdgcn_readfirstlane(sl[base + ob]);
            const int32_t slot1 = __builtin_amdgcn_readfirstlane(has1 ? sl[base + ob + 1] : -1);
            win_store<AXIS, F16>(g, slot0, slot1, acc, lane);
        };
        window_min<M, false, F16>(hb, len, Dp, blk, emit, [](int) { return true; }, sk);
        finish_run(g, sl, len, AXIS, runflag);
        __syncthreads();
    }
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Tile form for the global transform: one wave per column of 8 blocks along
// the pass axis inside a tile (64 columns per tile), with M blocks of context
// on each side taken from the neighbouring tiles.  Absent blocks hold no
// obstacle within d_max, so they read as the constant D block.
template <int M, int AXIS>
__global__ void __launch_bounds__(64) k_pass_win_tiles(Grid g) {
    constexpr int NB = 8 + 2 * M;
    __shared__ int32_t sl[NB];
    const int lane = threadIdx.x;
    const int64_t ncol = (int64_t)g.cnt[C_NTILE] * 64;
    const uint16_t* src = AXIS == 1 ? g.g1 : g.g2;
    constexpr bool F16 = win_f16(M);
    const uint32_t Dw = F16 ? f16_bits((uint32_t)g.D) : (uint32_t)g.D;
    const uint32_t Dpw = Dw | (Dw << 16);     // D in the window's representation
    for (int64_t it = blockIdx.x; it < ncol; it += gridDim.x) {
        const int32_t* ti = g.tinfo + (it >> 6) * 8;
        const int ca = (int)(it & 7), cb = (int)((it >> 3) & 7);
        // the lookups and the window's first loads form a chain of
        // dependent loads; a raised wave priority issues its links ahead of
        // the other waves' window arithmetic (back to normal once the first
        // window blocks are requested)
        __builtin_amdgcn_s_setprio(2);
        if (lane < NB)
            sl[lane] = AXIS == 1 ? axis_slot(g, ti[3], ti[0], ti[4], lane - M, ca + 64 * cb, 8)
                                 : axis_slot(g, ti[5], ti[0], ti[6], lane - M, ca + 8 * cb, 64);
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int j = 0; j < 8; ++j) any = any || sl[M + j] >= 0;
        if (any) {
            // skip masks over window positions j (block j - M): least input
            // of the block, D for absent blocks and past the context
            const uint16_t* bmin = AXIS == 1 ? g.bmin1 : g.bmin2;
            int bm = g.D;
            if (lane < NB) {
                const int32_t s2 = sl[lane];
                if (s2 >= 0) bm = bmin[s2];
            }
            WinSkip sk;
            sk.d = __ballot(bm >= g.D);
#pragma unroll
            for (int G = 0; G < M; ++G) {
                const int kg = G == 0 ? 1 : 8 * G;
                sk.g[G] = __ballot(bm + kg * kg >= g.D);
            }
            if (sk.d == ~0ull) {
                // every block of the window is D everywhere, so is every
                // output: pass Y records the block minimum D and stores no
                // g2 (its readers take the shared D block); pass Z stores s
                // as whole D blocks, 16 bytes per lane (non-temporal, as
                // every store of s), and the maximum D
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int32_t slot = __builtin_amdgcn_readfirstlane(sl[M + j]);
                    if (slot < 0) continue;
                    if (AXIS == 1) {
                        if (lane == 0) g.bmin2[slot] = (uint16_t)g.D;
                    } else {
                        __builtin_nontemporal_store((u32x4){Dpw, Dpw, Dpw, Dpw},
                                                    (u32x4*)(g.s + (int64_t)slot * 512) + lane);
                        if (lane == 0) g.bmax[slot] = g.D;
                    }
                }
                __syncthreads();
                continue;
            }
            // a block that is D everywhere reads the shared D block (cache
            // resident) instead of its own copy
            auto blk = [&](int b) -> uint4 {
                const int j = b + M;
                const int32_t s2 = (j < NB && !((sk.d >> j) & 1ull)) ? sl[j] : -1;
                const uint4* p = s2 >= 0 ? (const uint4*)src + (int64_t)s2 * 64 + lane
                                         : (const uint4*)g.dblock + lane;
                return *p;
            };
            auto emit = [&](int ob, const u16x2* acc, bool) {
                const int32_t slot0 = __builtin_amdgcn_readfirstlane(sl[M + ob]);
                const int32_t slot1 = __builtin_amdgcn_readfirstlane(sl[M + ob + 1]);
                win_store<AXIS, F16>(g, slot0, slot1, acc, lane);
            };
            auto need = [&](int ob) { return sl[M + ob] >= 0 || sl[M + ob + 1] >= 0; };
            window_min<M, false, F16>(0, 8, Dpw, blk, emit, need, sk);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// readback and query
// ---------------------------------------------------------------------------
// Dense readbacks: one workgroup of four waves per strip of RB_BLOCKS blocks
// along x (256 voxels) at one block row (by, bz).  The strip's blocks are
// first staged in LDS with coalesced loads (a block's 1 KiB of s as one
// 16-byte load per lane), then each wave writes whole rows of the strip, four
// consecutive voxels per lane: one store instruction covers 1 KiB of int32
// output (256 bytes of occupancy), so every row of the output is written
// contiguously, with non-temporal stores (the output is not read back by the
// library; streaming it past the caches took the int32 readback of the
// tunnel field from 4.6 to 6.7 TB/s).  Absent blocks read D (free for the
// occupancy).
constexpr int RB_BLOCKS = 32;
typedef int i32x4 __attribute__((ext_vector_type(4)));
enum { RB_FIELD = 0, RB_SIGNED = 1, RB_OCC = 2 };

template <int KIND>
__global__ void __launch_bounds__(256) k_read_strip(Grid g, void* __restrict__ out) {
    constexpr int NV = KIND == RB_OCC ? 1 : RB_BLOCKS * 65;
    __shared__ int32_t sl[RB_BLOCKS];
    __shared__ uint4 val[NV];                  // block b, row r at b * 65 + r (8 values of s)
    __shared__ uint8_t bits[RB_BLOCKS * 64];   // occupancy byte of block b, row r
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nsx = (g.nbx + RB_BLOCKS - 1) / RB_BLOCKS;
    const int64_t wg = blockIdx.x;
    const int bx0 = (int)(wg % nsx) * RB_BLOCKS;
    const int by = (int)((wg / nsx) % g.nby), bz = (int)((wg / nsx) / g.nby);
    const uint8_t* occ8 = (const uint8_t*)g.occ;
    if (t < RB_BLOCKS) sl[t] = bx0 + t < g.nbx ? find_block(g, bx0 + t, by, bz) : -1;
    __syncthreads();
    // stage: wave w takes blocks w, w + 4, ...; lane = row (y + 8z)
    for (int bb = w; bb < RB_BLOCKS; bb += 4) {
        const int32_t slot = sl[bb];
        if (slot < 0) continue;
        const uint8_t ob = occ8[(int64_t)slot * 64 + lane];
        if (KIND != RB_FIELD) bits[bb * 64 + lane] = ob;
        if (KIND == RB_OCC) continue;
        uint4 v = ((const uint4*)(g.s + (int64_t)slot * 512))[lane];
        v = make_uint4(s_pair_int(g, v.x), s_pair_int(g, v.y), s_pair_int(g, v.z),
                       s_pair_int(g, v.w));
        if (KIND == RB_SIGNED && __any(ob != 0u)) {
            // occupied voxels take their interior value (D without storage)
            const int32_t ii = g.iidx[slot];
            const uint32_t dd = (uint32_t)g.D | ((uint32_t)g.D << 16);
            const uint4 iv = ii >= 0 ? ((const uint4*)(g.ic1 + (int64_t)ii * 512))[lane]
                                     : make_uint4(dd, dd, dd, dd);
            uint32_t* vw = &v.x;
            const uint32_t* iw = &iv.x;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = (ob >> (2 * q)) & 1u ? 0x0000ffffu : 0u;
                const uint32_t hi = (ob >> (2 * q + 1)) & 1u ? 0xffff0000u : 0u;
                vw[q] = (vw[q] & ~(lo | hi)) | (iw[q] & (lo | hi));
            }
        }
        val[bb * 65 + lane] = v;
    }
    __syncthreads();
    // write: wave w takes rows w, w + 4, ...
    const int x = 8 * bx0 + 4 * lane;
    const int bb = lane >> 1;
    const int32_t slot = sl[bb];
    if (x >= g.nx) return;
    for (int r = w; r < 64; r += 4) {
        const int y = 8 * by + (r & 7), z = 8 * bz + (r >> 3);
        if (y >= g.ny || z >= g.nz) continue;
        const int64_t off = ((int64_t)z * g.ny + y) * (int64_t)g.nx + x;
        const uint32_t ob = slot >= 0 && KIND != RB_FIELD ? (bits[bb * 64 + r] >> (4 * (lane & 1))) & 15u
                                                          : 0u;
        if (KIND == RB_OCC) {
            const uint32_t v = (ob & 1u) | ((ob & 2u) << 7) | ((ob & 4u) << 14) | ((ob & 8u) << 21);
            uint8_t* o = (uint8_t*)out + off;
            if (x + 4 <= g.nx && ((uintptr_t)o & 3) == 0) {
                __builtin_nontemporal_store(v, (uint32_t*)o);
            } else {
                for (int k = 0; k < 4 && x + k < g.nx; ++k) o[k] = (uint8_t)(v >> (8 * k));
            }
        } else {
            int32_t v[4];
            if (slot < 0) {
                v[0] = v[1] = v[2] = v[3] = g.D;
            } else {
                const uint2 h = ((const uint2*)&val[bb * 65 + r])[lane & 1];
                v[0] = (int32_t)(h.x & 0xffffu);
                v[1] = (int32_t)(h.x >> 16);
                v[2] = (int32_t)(h.y & 0xffffu);
                v[3] = (int32_t)(h.y >> 16);
                if (KIND == RB_SIGNED) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if ((ob >> k) & 1u) v[k] = -v[k];
                }
            }
            int32_t* o = (int32_t*)out + off;
            if (x + 4 <= g.nx && ((uintptr_t)o & 15) == 0) {
                __builtin_nontemporal_store((i32x4){v[0], v[1], v[2], v[3]}, (i32x4*)o);
            } else {
                for (int k = 0; k < 4 && x + k < g.nx; ++k) o[k] = v[k];
            }
        }
    }
}

// g1, g2 and s of voxel (x, y, z) inside the extent (absent block: D).  The
// global passes X and Y do not always store a block that is D everywhere, so
// g1 and g2 are D wherever their block minimum is.
__device__ inline int field_g1(const Grid& g, int x, int y, int z) {
    const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
    if (slot < 0 || (int)g.bmin1[slot] >= g.D) return g.D;
    const uint16_t v = g.g1[(int64_t)slot * 512 + (y & 7) + 8 * (x & 7) + 64 * (z & 7)];
    return win_f16(g.R) ? f16_int(v) : (int)v;
}
__device__ inline int field_g2(const Grid& g, int x, int y, int z) {
    const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
    if (slot < 0 || (int)g.bmin2[slot] >= g.D) return g.D;
    const uint16_t v = g.g2[(int64_t)slot * 512 + (z & 7) + 8 * (x & 7) + 64 * (y & 7)];
    return win_f16(g.R) ? f16_int(v) : (int)v;
}
__device__ inline bool field_occ(const Grid& g, int x, int y, int z) {
    const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
    if (slot < 0) return false;
    const int v = (x & 7) + 8 * (y & 7) + 64 * (z & 7);
    return (g.occ[(int64_t)slot * 16 + (v >> 5)] >> (v & 31)) & 1u;
}

// One thread per query.  s = min over k of g2(z + k) + k^2 and
// g2 = min over j of g1(y + j) + j^2, g1 = (x - x')^2 for the nearest
// obstacle x' of the row: the offsets are found again by equality, nearest
// first (uncapped values: s < D), then the obstacle sits at x +- sqrt(g1).
__global__ void k_query_nearest(Grid g, const int32_t* __restrict__ xyz, int64_t n,
                                int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int ox = -1, oy = -1, oz = -1;
        if (x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz) {
            const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
            const int sv = slot < 0 ? g.D
                                    : s_int(g, g.s[(int64_t)slot * 512 + (x & 7) + 8 * (y & 7) + 64 * (z & 7)]);
            if (sv < g.D) {
                // z offset
                int kz = 0, t2 = -1;
                for (int a = 0; a * a <= sv && t2 < 0; ++a) {
                    for (int sg = 0; sg < 2 && t2 < 0; ++sg) {
                        const int zz = sg ? z + a : z - a;
                        if ((sg && a == 0) || zz < 0 || zz >= g.nz) continue;
                        const int v = field_g2(g, x, y, zz);
                        if (v + a * a == sv) { kz = zz; t2 = v; }
                    }
                }
                // y offset
                int ky = 0, t1 = -1;
                for (int a = 0; t2 >= 0 && a * a <= t2 && t1 < 0; ++a) {
                    for (int sg = 0; sg < 2 && t1 < 0; ++sg) {
                        const int yy = sg ? y + a : y - a;
                        if ((sg && a == 0) || yy < 0 || yy >= g.ny) continue;
                        const int v = field_g1(g, x, yy, kz);
                        if (v + a * a == t2) { ky = yy; t1 = v; }
                    }
                }
                // x offset: g1 is a perfect square d^2
                if (t1 >= 0) {
                    int d = (int)sqrtf((float)t1);
                    while (d * d > t1) --d;
                    while ((d + 1) * (d + 1) <= t1) ++d;
                    if (x - d >= 0 && field_occ(g, x - d, ky, kz)) ox = x - d;
                    else if (x + d < g.nx && field_occ(g, x + d, ky, kz)) ox = x + d;
                    if (ox >= 0) { oy = ky; oz = kz; }
                }
            }
        }
        out[3 * i] = ox;
        out[3 * i + 1] = oy;
        out[3 * i + 2] = oz;
    }
}

__global__ void k_query(Grid g, const int32_t* __restrict__ xyz, int64_t n, int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int32_t v = g.D;
        if (x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz) {
            const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
            if (slot >= 0) v = s_int(g, g.s[(int64_t)slot * 512 + (x & 7) + 8 * (y & 7) + 64 * (z & 7)]);
        }
        out[i] = v;
    }
}

// ---------------------------------------------------------------------------
// incremental update
// ---------------------------------------------------------------------------

__device__ inline bool upd_winner(const Grid& g, int64_t i) {
    const int32_t h = g.upos[i];
    return h >= 0 && g.uvals[h] == (int32_t)i;
}

// Fresh pool slots claimed by lanes of this wave: an empty block with
// background values.  Called by the whole wave (each slot's 1 KiB arrays are
// written as one 16-byte store per lane).
__device__ inline void init_slots(const Grid& g, int32_t slot) {
    unsigned long long m = __ballot(slot >= 0);
    const int lane = __lane_id();
    // g1, g2 and s hold D in their own representation (binary16 for small radii)
    const uint32_t dw = win_f16(g.R) ? f16_bits((uint32_t)g.D) : (uint32_t)g.D;
    const uint4 dg = make_uint4(dw | (dw << 16), dw | (dw << 16), dw | (dw << 16), dw | (dw << 16));
    while (m) {
        const int src = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const int64_t s = __shfl(slot, src);
        if (lane < 16) {
            g.occ[s * 16 + lane] = 0u;
            g.chg_add[s * 16 + lane] = 0u;
            g.chg_rem[s * 16 + lane] = 0u;
        }
        ((uint4*)(g.g1 + s * 512))[lane] = dg;
        ((uint4*)(g.g2 + s * 512))[lane] = dg;
        ((uint4*)(g.s + s * 512))[lane] = dg;    // s holds D like g1, g2
        if (lane == 0) {
            g.bmax[s] = g.D;
            g.bmin1[s] = (uint16_t)g.D;
            g.bmin2[s] = (uint16_t)g.D;
        }
    }
}

// First kernel of an update: range check (any entry outside the extent
// cancels the whole call), last-entry-wins dedupe through a voxel-keyed hash
// (value = max entry index), and the blocks the call needs.  Every entry that
// sets a voxel gets its block (fresh slots hold background values), not only
// the winning ones: a block made for an entry that loses to a later one is
// harmless (background values are its field, and the region may be larger
// than needed), and the allocation need not wait for the dedupe.  A block
// that holds no obstacle yet and is not listed is listed for dilation (its
// creator appends it; for an existing block the listing flag decides).  The
// update's counters are zeroed here by the first workgroup, except the
// dilation list's (zeroed by the previous call's fronts kernel), to which
// every workgroup of this kernel appends.  A cancelled update sets
// C_UABORT, which the x-items kernel clears after its last reader.
__global__ void k_upd_dedupe_alloc(Grid g, const int32_t* __restrict__ xyz,
                                   const uint8_t* __restrict__ state, int64_t n0,
                                   const int32_t* n_dev) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n0;
    if (blockIdx.x == 0 && threadIdx.x >= C_NYI && threadIdx.x < C_N &&
        threadIdx.x != C_NNEWDIL)
        g.cnt[threadIdx.x] = 0;
    const int lane = __lane_id();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i - lane < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool want = false;
        int bx = 0, by = 0, bz = 0;
        if (i < n) {
            const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
            g.upos[i] = -1;
            if (x < 0 || y < 0 || z < 0 || x >= g.nx || y >= g.ny || z >= g.nz) {
                set_error(g, -2);
                g.cnt[C_UABORT] = 1;
            } else {
                const unsigned long long key = (unsigned long long)x +
                    (unsigned long long)g.nx * ((unsigned long long)y + (unsigned long long)g.ny * z);
                bool created;
                const int32_t h = hinsert(g.ukeys, g.umask, key, &created);
                if (h < 0) {
                    set_error(g, -3);
                    g.cnt[C_UABORT] = 1;
                } else {
                    g.upos[i] = h;
                    atomicMax(&g.uvals[h], (int32_t)i);
                    want = state[i] != 0;
                    bx = x >> 3; by = y >> 3; bz = z >> 3;
                }
            }
        }
        bool created = false;
        int64_t e = -1;
        unsigned long long key = 0;
        if (want) {
            key = pack_key(bx, by, bz);
            e = insert_block(g, bx, by, bz, &created);
            if (e < 0) {
                set_error(g, -3);
                g.cnt[C_UABORT] = 1;
            }
        }
        const int32_t sl = claim_slots(g, created, e, key, 0u);
        if (created && sl < 0) g.cnt[C_UABORT] = 1;   // pool full
        init_slots(g, sl);
        bool newdil = created && sl >= 0;
        int32_t dslot = sl;
        if (!created && e >= 0) {
            const int32_t s2 = __hip_atomic_load(&g.tslots[e], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (s2 >= 0 && !(g.flags[s2] & (F_DILATED | F_NEWDIL))) {
                const uint32_t o = atomicOr(&g.flags[s2], F_NEWDIL);
                newdil = !(o & (F_DILATED | F_NEWDIL));
                dslot = s2;
            }
        }
        const int j = wave_append(newdil, &g.cnt[C_NNEWDIL]);
        if (newdil) g.list_newdil[j] = dslot;
    }
}

// Apply the winning entries: flip occupancy bits, record the changed voxels
// per block (the wave centres) and list the blocks that hold them.  The
// voxel-keyed dedupe table is emptied here for the next call: each winner
// clears its entry once it has read it (the entries that lose to it only
// ever compare the stored index with their own), and a call cancelled before
// this kernel clears the entry of every input.  Workgroups vb of vgrid.
__device__ inline void upd_apply_body(const Grid& g, const int32_t* __restrict__ xyz,
                                      const uint8_t* __restrict__ state, int64_t n,
                                      int64_t vb, int64_t vgrid) {
    const int64_t t0 = vb * blockDim.x + threadIdx.x, stride = vgrid * blockDim.x;
    {
        // the blocks listed for dilation are being dilated by the other
        // workgroups of this launch (or the call is cancelled): their
        // listing mark goes
        const int64_t nd = g.cnt[C_NNEWDIL];
        for (int64_t i = t0; i < nd; i += stride) atomicAnd(&g.flags[g.list_newdil[i]], ~F_NEWDIL);
    }
    if (g.cnt[C_UABORT] != 0) {
        for (int64_t i = t0; i < n; i += stride) {
            const int32_t h = g.upos[i];
            if (h >= 0) {
                g.ukeys[h] = KEY_EMPTY;
                g.uvals[h] = -1;
            }
        }
        return;
    }
    for (int64_t i = t0; i - __lane_id() < n; i += stride) {
        bool add = false, rem = false, first_seed = false, new_dil = false;
        int32_t slot = -1;
        if (i < n && upd_winner(g, i)) {
            const int32_t h = g.upos[i];
            g.ukeys[h] = KEY_EMPTY;
            g.uvals[h] = -1;
            const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
            slot = find_block(g, x >> 3, y >> 3, z >> 3);
            if (slot >= 0) {
                const int v = (x & 7) + 8 * (y & 7) + 64 * (z & 7);
                const uint32_t bit = 1u << (v & 31);
                const int64_t w = (int64_t)slot * 16 + (v >> 5);
                const bool cur = (g.occ[w] & bit) != 0;
                const bool tgt = state[i] != 0;
                if (tgt != cur) {
                    if (tgt) {
                        atomicOr(&g.occ[w], bit);
                        atomicOr(&g.chg_add[w], bit);
                        add = true;
                        const uint32_t o = atomicOr(&g.flags[slot], F_DILATED | F_SEED);
                        new_dil = !(o & F_DILATED);
                        first_seed = !(o & F_SEED);
                        if (new_dil) atomicOr(&g.flags[slot], F_DILNEW);
                    } else {
                        atomicAnd(&g.occ[w], ~bit);
                        atomicOr(&g.chg_rem[w], bit);
                        rem = true;
                        const uint32_t o = atomicOr(&g.flags[slot], F_SEED);
                        first_seed = !(o & F_SEED);
                    }
                }
            }
        }
        const unsigned long long ma = __ballot(add), mr = __ballot(rem);
        if (__lane_id() == (int)(__ffsll((long long)(ma | mr | 1ull)) - 1) && (ma | mr)) {
            atomicAdd(&g.cnt[C_NADD], __popcll(ma));
            atomicAdd(&g.cnt[C_NREM], __popcll(mr));
        }
        const int j = wave_append(first_seed, &g.cnt[C_NSEED]);
        if (first_seed) g.list_seed[j] = slot;
        if (new_dil) atomicAdd(&g.cnt[C_NDIL], 1);   // obstacle blocks (statistics)
    }
}

// Blocks that gain their first obstacle bring their R-neighbourhood in, one
// thread per neighbour.  Workgroups vb of vgrid.
__device__ inline void upd_dilate_body(const Grid& g, int64_t vb, int64_t vgrid) {
    if (g.cnt[C_UABORT] != 0) return;
    const int R = g.R, w = 2 * R + 1, w3 = w * w * w;
    const int64_t total = (int64_t)g.cnt[C_NNEWDIL] * w3;
    const int lane = __lane_id();
    for (int64_t i = vb * blockDim.x + threadIdx.x; i - lane < total; i += vgrid * blockDim.x) {
        bool created = false;
        int64_t e = -1;
        unsigned long long key = 0;
        if (i < total) {
            const int32_t slot = g.list_newdil[i / w3];
            const int o = (int)(i % w3);
            int bx, by, bz;
            unpack_key(g.bkey[slot], bx, by, bz);
            bx += o % w - R;
            by += (o / w) % w - R;
            bz += o / (w * w) - R;
            key = pack_key(bx, by, bz);
            if (bx >= 0 && by >= 0 && bz >= 0 && bx < g.nbx && by < g.nby && bz < g.nbz) {
                e = insert_block(g, bx, by, bz, &created);
                if (e < 0) {
                    set_error(g, -3);
                    g.cnt[C_UABORT] = 1;
                }
            }
        }
        const int32_t sl = claim_slots(g, created, e, key, 0u);
        if (created && sl < 0) g.cnt[C_UABORT] = 1;   // pool full
        init_slots(g, sl);
    }
}

// The occupancy changes and the dilation of the listed blocks share a
// launch: the first napply workgroups apply the entries, the others dilate.
// The two never touch the same block (dilation only creates absent blocks;
// every block an entry changes exists since the first kernel), so they need
// no order.  A full pool found by the dilation cancels the call after the
// bits may have changed: the fronts kernel then restores them from the
// change masks (and undoes the call's F_DILATED marks), so a cancelled call
// still leaves the map as it was.
__global__ void k_upd_apply_dilate(Grid g, const int32_t* __restrict__ xyz,
                                   const uint8_t* __restrict__ state, int64_t n0,
                                   const int32_t* n_dev, int napply) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n0;
    if ((int)blockIdx.x < napply) upd_apply_body(g, xyz, state, n, blockIdx.x, napply);
    else upd_dilate_body(g, (int64_t)blockIdx.x - napply, (int64_t)gridDim.x - napply);
}

// Bounding boxes (block-local) of the added and removed voxels of each seed.
// Packed as xmin | xmax<<4 | ymin<<8 | ymax<<12 | zmin<<16 | zmax<<20 | 1<<24.
// byte = the wave's row (y, z) = lane of the voxel set; x from one ballot per
// bit, y and z from the ballot of nonempty rows (bit y + 8z).
__device__ inline int32_t row_box(uint32_t byte) {
    const unsigned long long rows = __ballot(byte != 0u);
    if (rows == 0ull) return 0;
    uint32_t xo = 0u;
#pragma unroll
    for (int x = 0; x < 8; ++x) xo |= (__ballot((byte >> x) & 1u) != 0ull ? 1u : 0u) << x;
    unsigned long long f = rows | (rows >> 32);
    f |= f >> 16;
    f |= f >> 8;
    const uint32_t yo = (uint32_t)f & 0xffu;
    uint32_t zo = 0u;
#pragma unroll
    for (int z = 0; z < 8; ++z) zo |= (((rows >> (8 * z)) & 0xffull) != 0ull ? 1u : 0u) << z;
    const int xmn = __ffs(xo) - 1, xmx = 31 - __clz(xo);
    const int ymn = __ffs(yo) - 1, ymx = 31 - __clz(yo);
    const int zmn = __ffs(zo) - 1, zmx = 31 - __clz(zo);
    return xmn | (xmx << 4) | (ymn << 8) | (ymx << 12) | (zmn << 16) | (zmx << 20) | (1 << 24);
}

// squared distance between voxel boxes [a0,a1] and [b0,b1] per axis
__device__ inline int box_gap2(int a0, int a1, int b0, int b1) {
    const int d = max(0, max(b0 - a1, a0 - b1));
    return d * d;
}
__device__ inline int box_dist2(int32_t pk, int sx, int sy, int sz, int bx, int by, int bz) {
    const int xmn = 8 * sx + (pk & 15), xmx = 8 * sx + ((pk >> 4) & 15);
    const int ymn = 8 * sy + ((pk >> 8) & 15), ymx = 8 * sy + ((pk >> 12) & 15);
    const int zmn = 8 * sz + ((pk >> 16) & 15), zmx = 8 * sz + ((pk >> 20) & 15);
    return box_gap2(xmn, xmx, 8 * bx, 8 * bx + 7) + box_gap2(ymn, ymx, 8 * by, 8 * by + 7) +
           box_gap2(zmn, zmx, 8 * bz, 8 * bz + 7);
}

// Raise / lower fronts around every seed and the g1/g2 recompute sets.  One
// workgroup (up to 1024 threads: every block within R of the seed at once for
// d_max <= 32) per seed block: its first wave takes the bounding boxes of the
// seed's added and removed voxels (and, for d_max <= 64, the positions of the
// 27 tiles around its tile, since the fronts reach at most one tile beyond
// it), then every thread marks blocks within R of the seed:
//   lower: some added voxel a has |box(B) - a|^2 < bmax(B)   (a value can drop)
//   raise: some removed voxel r has |box(B) - r|^2 <= bmax(B) and < D
//   xs:    blocks within R along x of a seed (their g1 can change)
//   ys:    blocks within R in x and y of a seed (their g2 can change)
// The seed's change masks are emptied for the next call once read, and the
// dilation-list count is cleared (no later kernel of the update reads it;
// the next call's first kernel appends to that list).  In a call cancelled
// after the occupancy changed (the pool filled during the dilation) the
// workgroup instead restores the seed's bits from its change masks, drops
// its marks and the F_DILATED it gained, and builds no fronts.
__global__ void __launch_bounds__(1024) k_upd_fronts(Grid g) {
    __shared__ int32_t rec[32];     // boxes, block coordinates, 27 tile positions
    __shared__ int wcnt[16][5];     // per wave: dirty, ys, xs, raise, lower
    __shared__ int bbase[3];        // the workgroup's list positions
    const int R = g.R, w = 2 * R + 1, w3 = w * w * w;
    const int64_t ns = g.cnt[C_NSEED];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const bool cancel = g.cnt[C_UABORT] != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) g.cnt[C_NNEWDIL] = 0;
    for (int64_t si = blockIdx.x; si < ns; si += gridDim.x) {
        if (cancel) {
            if (wid == 0) {
                const int32_t seed = g.list_seed[si];
                if (lane < 16) {
                    const int64_t w = (int64_t)seed * 16 + lane;
                    const uint32_t a = g.chg_add[w], r = g.chg_rem[w];
                    g.occ[w] = (g.occ[w] & ~a) | r;
                    g.chg_add[w] = 0u;
                    g.chg_rem[w] = 0u;
                }
                if (lane == 0) {
                    const uint32_t f = atomicAnd(&g.flags[seed], ~(F_SEED | F_DILNEW));
                    if (f & F_DILNEW) {
                        atomicAnd(&g.flags[seed], ~F_DILATED);
                        atomicSub(&g.cnt[C_NDIL], 1);
                    }
                }
            }
            continue;
        }
        if (wid == 0) {
            const int32_t seed = g.list_seed[si];
            const uint32_t a = ((const uint8_t*)g.chg_add)[(int64_t)seed * 64 + lane];
            const uint32_t r = ((const uint8_t*)g.chg_rem)[(int64_t)seed * 64 + lane];
            int sx, sy, sz;
            unpack_key(g.bkey[seed], sx, sy, sz);
            const int32_t ba = row_box(a);
            const int32_t br = row_box(r);
            if (lane < 16) {
                g.chg_add[(int64_t)seed * 16 + lane] = 0u;
                g.chg_rem[(int64_t)seed * 16 + lane] = 0u;
            }
            if (lane == 0) {
                rec[0] = ba;
                rec[1] = br;
                rec[2] = sx;
                rec[3] = sy;
                rec[4] = sz;
            }
            if (R <= 8 && lane < 27) {
                const int tx = (sx >> 3) + lane % 3 - 1, ty = (sy >> 3) + (lane / 3) % 3 - 1,
                          tz = (sz >> 3) + lane / 9 - 1;
                rec[5 + lane] = (tx < 0 || ty < 0 || tz < 0)
                                    ? -1
                                    : hpos(g.tkeys, g.tmask, pack_key(tx, ty, tz));
            }
        }
        __syncthreads();
        const int32_t pa = rec[0], pr = rec[1], sx = rec[2], sy = rec[3], sz = rec[4];
        for (int o0 = 0; o0 < w3; o0 += blockDim.x) {
            const int o = o0 + (int)threadIdx.x;
            bool new_dirty = false, new_xs = false, new_ys = false, raise = false, lower = false;
            int32_t slot = -1;
            if (o < w3) {
                const int ox = o % w - R, oy = (o / w) % w - R, oz = o / (w * w) - R;
                const int bx = sx + ox, by = sy + oy, bz = sz + oz;
                // box distances need no loads: a block beyond D of both boxes
                // can only join the g1 / g2 sets (its own x row or xy plane of
                // the seed)
                const int da = pa != 0 ? box_dist2(pa, sx, sy, sz, bx, by, bz) : 0x7fffffff;
                const int dr = pr != 0 ? box_dist2(pr, sx, sy, sz, bx, by, bz) : 0x7fffffff;
                const bool maybe = da < g.D || dr < g.D || oz == 0;
                if (!maybe) {
                } else if (R <= 8) {
                    // the block's tile among the 27 recorded around the seed's tile
                    if (bx >= 0 && by >= 0 && bz >= 0) {
                        const int k = ((bx >> 3) - (sx >> 3) + 1) + 3 * ((by >> 3) - (sy >> 3) + 1) +
                                      9 * ((bz >> 3) - (sz >> 3) + 1);
                        const int32_t t = rec[5 + k];
                        if (t >= 0) slot = g.tslots[(int64_t)t * 512 + block_local(bx, by, bz)];
                    }
                } else {
                    slot = find_block(g, bx, by, bz);
                }
                if (slot >= 0) {
                    const int bm = g.bmax[slot];
                    const uint32_t seen = g.flags[slot];   // bits only get set in this kernel
                    lower = da < bm;
                    raise = dr <= bm && dr < g.D;
                    uint32_t want = 0;
                    if (lower) want |= F_LOWER | F_DIRTY;
                    if (raise) want |= F_RAISE | F_DIRTY;
                    if (oz == 0) want |= F_YS;
                    if (oz == 0 && oy == 0) want |= F_XS;
                    if (!(want & ~seen)) {
                        raise = lower = false;              // already marked by another seed
                    } else {
                        const uint32_t old = atomicOr(&g.flags[slot], want);
                        new_dirty = (want & F_DIRTY) && !(old & F_DIRTY);
                        new_ys = (want & F_YS) && !(old & F_YS);
                        new_xs = (want & F_XS) && !(old & F_XS);
                        raise = raise && !(old & F_RAISE);
                        lower = lower && !(old & F_LOWER);
                    }
                }
            }
            // list appends and statistics: one counter atomic per list and
            // workgroup, positions from the waves' ballots
            const unsigned long long md = __ballot(new_dirty), my = __ballot(new_ys),
                                     mx = __ballot(new_xs), mr = __ballot(raise),
                                     ml = __ballot(lower);
            if (lane == 0) {
                wcnt[wid][0] = __popcll(md);
                wcnt[wid][1] = __popcll(my);
                wcnt[wid][2] = __popcll(mx);
                wcnt[wid][3] = __popcll(mr);
                wcnt[wid][4] = __popcll(ml);
            }
            __syncthreads();
            const int nw = (int)(blockDim.x >> 6);
            if (threadIdx.x < 5) {
                const int c = threadIdx.x;
                int sum = 0;
                for (int v = 0; v < nw; ++v) sum += wcnt[v][c];
                const int ctr = c == 0 ? C_NDIRTY : c == 1 ? C_NYS : c == 2 ? C_NXS
                              : c == 3 ? C_NRAISE : C_NLOWER;
                const int base = sum ? atomicAdd(&g.cnt[ctr], sum) : 0;
                if (c < 3) bbase[c] = base;
            }
            __syncthreads();
            int bd = bbase[0], by_ = bbase[1], bx_ = bbase[2];
            for (int v = 0; v < wid; ++v) {
                bd += wcnt[v][0];
                by_ += wcnt[v][1];
                bx_ += wcnt[v][2];
            }
            const unsigned long long below = (1ull << lane) - 1ull;
            if (new_dirty) g.list_dirty[bd + __popcll(md & below)] = slot;
            if (new_ys) g.list_ys[by_ + __popcll(my & below)] = slot;
            if (new_xs) g.list_xs[bx_ + __popcll(mx & below)] = slot;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Occupancy integration of a range scan: rays from the sensor voxel o to end
// voxels e.  A ray visits o and every voxel the segment between the two voxel
// centres enters through a face; the i-th face crossing on axis a lies at
// segment parameter (2i + 1) / (2 |d_a|), d = e - o, and crossings at equal
// parameters are taken in the order x, y, z.  Visited voxels become free, the
// end voxel of a ray with a return becomes occupied, and hits win.
// ---------------------------------------------------------------------------

// Voxel entered at crossing j of the ray (crossings numbered per axis: the
// |dx| crossings on x first, then y, then z).  On every axis b the voxel has
// moved by the number of b-crossings up to it: all strictly earlier ones, and
// those at the same parameter when b comes before the crossing's axis (its
// own axis counts the crossing itself).
__device__ inline void ray_crossing_voxel(const int o[3], const int d[3], const int ad[3],
                                          int64_t j, int v[3]) {
    int a = 0;
    while (a < 2 && j >= ad[a]) { j -= ad[a]; ++a; }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        int64_t c;
        if (b == a) {
            c = j + 1;
        } else if (ad[b] == 0) {
            c = 0;
        } else {
            // crossing i' of axis b is earlier iff (2i' + 1) |d_a| < (2j + 1) |d_b|
            const int64_t P = (2 * j + 1) * (int64_t)ad[b], Q = ad[a];
            // floor(P / Q) and ceil(P / Q), in 32 bits when P fits
            int64_t fl, ce;
            if (P < (1ll << 31)) {
                const uint32_t p32 = (uint32_t)P, q32 = (uint32_t)Q;
                const uint32_t f = p32 / q32;
                fl = f;
                ce = f + (f * q32 != p32 ? 1 : 0);
            } else {
                fl = P / Q;
                ce = fl + (fl * Q != P ? 1 : 0);
            }
            c = b < a ? (fl + 1) / 2     // (2i' + 1) Q <= P
                      : ce / 2;          // (2i' + 1) Q <  P
            if (c > ad[b]) c = ad[b];
        }
        v[b] = o[b] + (int)(d[b] < 0 ? -c : c);
    }
}

__device__ inline bool in_extent(const Grid& g, const int v[3]) {
    return v[0] >= 0 && v[1] >= 0 && v[2] >= 0 && v[0] < g.nx && v[1] < g.ny && v[2] < g.nz;
}

// Occupancy bit of voxel v (inside the extent) for U voxels at once: the
// tile-hash probes, the slot-table reads and the occupancy reads of all U
// are issued together (the first probe position almost always decides; a
// collision falls back to the probing loop).
template <int U>
__device__ inline void occ_bits(const Grid& g, const int (*v)[3], const bool* want, bool* bit) {
    unsigned long long key[U], got[U];
    uint32_t h[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        key[u] = pack_key(v[u][0] >> 6, v[u][1] >> 6, v[u][2] >> 6);
        h[u] = hash_of(key[u], g.tmask);
        got[u] = want[u] ? g.tkeys[h[u]] : KEY_EMPTY;
    }
    int32_t slot[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int32_t t = -1;
        if (want[u]) {
            if (got[u] == key[u]) t = (int32_t)h[u];
            else if (got[u] != KEY_EMPTY) t = hpos(g.tkeys, g.tmask, key[u]);
        }
        const int local = ((v[u][0] >> 3) & 7) + 8 * ((v[u][1] >> 3) & 7) + 64 * ((v[u][2] >> 3) & 7);
        slot[u] = t >= 0 ? g.tslots[(int64_t)t * 512 + local] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = (v[u][0] & 7) + 8 * (v[u][1] & 7) + 64 * (v[u][2] & 7);
        bit[u] = slot[u] >= 0 && ((g.occ[(int64_t)slot[u] * 16 + (b >> 5)] >> (b & 31)) & 1u);
    }
}

// Slots of ray r in the flat enumeration of visited voxels: its origin and one
// per crossing, or none when an endpoint lies outside the extent.
__device__ inline int64_t ray_slots(const Grid& g, const int o[3], bool o_in,
                                    const int32_t* ends, int64_t r) {
    const int e[3] = {ends[3 * r], ends[3 * r + 1], ends[3 * r + 2]};
    if (!o_in || !in_extent(g, e)) return 0;
    return (int64_t)abs(e[0] - o[0]) + abs(e[1] - o[1]) + abs(e[2] - o[2]) + 1;
}

// Exclusive prefix sum of the rays' slot counts in two levels: every
// workgroup of 1024 threads scans its 1024 rays (one ray per thread, a
// shuffle scan per wave, then the 16 wave totals) into loff[] and its total
// into btot[]; k_scan_blocks then scans the totals into bpre[].  The first
// slot of ray r is bpre[r / 1024] + loff[r].  Rays with an endpoint outside
// the extent get no slots and set EDT_ERR_RANGE.
__global__ void __launch_bounds__(1024) k_scan_offsets(Grid g, const int32_t* __restrict__ origin,
                                                       const int32_t* __restrict__ ends, int64_t n,
                                                       int64_t* loff, int64_t* btot) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int o[3] = {origin[0], origin[1], origin[2]};
    const bool o_in = in_extent(g, o);
    const int64_t r = (int64_t)blockIdx.x * 1024 + t;
    const int64_t k = r < n ? ray_slots(g, o, o_in, ends, r) : 0;
    if (r < n && k == 0) set_error(g, -2 /* EDT_ERR_RANGE */);
    int64_t incl = k;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int64_t before = 0;
    for (int j = 0; j < w; ++j) before += wsum[j];
    if (r < n) loff[r] = before + incl - k;
    if (t == 1023) btot[blockIdx.x] = before + incl;
}

// Exclusive scan of the nb workgroup totals (one workgroup, chunks of 1024
// with a carried sum); the total slot count goes to *total.
__global__ void __launch_bounds__(1024) k_scan_blocks(const int64_t* __restrict__ btot, int64_t nb,
                                                      int64_t* bpre, int64_t* total) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t i = c0 + t;
        const int64_t k = i < nb ? btot[i] : 0;
        int64_t incl = k;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int64_t before = carry;
        for (int j = 0; j < w; ++j) before += wsum[j];
        if (i < nb) bpre[i] = before + incl - k;
        __syncthreads();
        if (t == 1023) carry = before + incl;
        __syncthreads();
    }
    if (t == 0) *total = carry;
}

__device__ inline int64_t ray_first_slot(const int64_t* loff, const int64_t* bpre, int64_t r) {
    return bpre[r >> 10] + loff[r];
}

// Change entries "free" for the visited voxels that are occupied now (the
// end voxel of a hit excepted).  Lanes take consecutive slots of the flat
// enumeration, so short rays share a wave; each lane finds its ray by binary
// search over the offsets.  Entries go to the list front through cnt[0]
// (capacity cap).
__global__ void __launch_bounds__(1024) k_scan_clear(Grid g, const int32_t* __restrict__ origin,
                                                   const int32_t* __restrict__ ends,
                                                   const uint8_t* __restrict__ hits, int64_t n,
                                                   const int64_t* __restrict__ loff,
                                                   const int64_t* __restrict__ bpre,
                                                   const int64_t* total_p, int32_t* cnt,
                                                   int32_t* lxyz, uint8_t* lst, int64_t cap) {
    __shared__ int wcnt[16];
    __shared__ int wgbase;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int o[3] = {origin[0], origin[1], origin[2]};
    const int64_t total = *total_p;
    // sixteen waves per workgroup, one chunk of 64 slots each; the list
    // positions take one counter atomic per workgroup
    for (int64_t b0 = 1024 * (int64_t)blockIdx.x; b0 < total; b0 += 1024 * (int64_t)gridDim.x) {
        const int64_t base = b0 + 64 * wid;
        const int64_t f = base + lane;
        // rb: the last ray whose first slot is at or before `base`, by a
        // 64-way search of the whole wave (rays without slots share the next
        // ray's offset and are passed over)
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t span = hi - lo + 1;
            const int64_t stp = (span + 63) / 64;
            const int64_t q = lo + (int64_t)lane * stp;
            const bool le = q <= hi && ray_first_slot(loff, bpre, q) <= base;
            const unsigned long long m = __ballot(le);   // lane 0 always qualifies
            const int top = 63 - __clzll((long long)m);
            lo = lo + (int64_t)top * stp;
            hi = lo + stp - 1 < hi ? lo + stp - 1 : hi;
            if (stp == 1) break;
        }
        const int64_t rb = lo;
        // each lane: the last ray in rb .. rb + 63 whose first slot is at or
        // before f, by binary search over the 64 offsets held across lanes
        const int64_t wj = rb + lane < n ? ray_first_slot(loff, bpre, rb + lane) : INT64_MAX;
        int j = 0;
#pragma unroll
        for (int stp = 32; stp > 0; stp >>= 1) {
            const int64_t x = __shfl(wj, j + stp);
            if (x <= f) j += stp;
        }
        int v[1][3] = {{o[0], o[1], o[2]}};
        bool want[1] = {false}, bit[1];
        if (f < total) {
            int64_t r = rb + j;
            // more than 63 rays without slots in between: continue linearly
            while (r + 1 < n && ray_first_slot(loff, bpre, r + 1) <= f) ++r;
            lo = r;
            const int64_t k = f - ray_first_slot(loff, bpre, lo);     // 0: the sensor voxel, k >= 1: crossing k - 1
            const int e[3] = {ends[3 * lo], ends[3 * lo + 1], ends[3 * lo + 2]};
            if (k > 0) {
                const int d[3] = {e[0] - o[0], e[1] - o[1], e[2] - o[2]};
                const int ad[3] = {abs(d[0]), abs(d[1]), abs(d[2])};
                ray_crossing_voxel(o, d, ad, k - 1, v[0]);
            }
            const bool at_end = v[0][0] == e[0] && v[0][1] == e[1] && v[0][2] == e[2];
            want[0] = !(hits[lo] && at_end);
        }
        occ_bits<1>(g, v, want, bit);
        const bool emit = want[0] && bit[0];
        const unsigned long long m = __ballot(emit);
        if (lane == 0) wcnt[wid] = __popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            int sum = 0;
            for (int j = 0; j < 16; ++j) sum += wcnt[j];
            wgbase = sum ? atomicAdd(cnt, sum) : 0;
        }
        __syncthreads();
        int idx = wgbase;
        for (int j = 0; j < wid; ++j) idx += wcnt[j];
        idx += __popcll(m & ((1ull << lane) - 1ull));
        __syncthreads();
        if (emit) {
            if (idx < cap) {
                lxyz[3 * (int64_t)idx] = v[0][0];
                lxyz[3 * (int64_t)idx + 1] = v[0][1];
                lxyz[3 * (int64_t)idx + 2] = v[0][2];
                lst[idx] = 0;
            } else {
                set_error(g, -3 /* EDT_ERR_CAPACITY */);
            }
        }
    }
}

// Change entries "occupied" for every hit end voxel, after all free entries
// (the update takes the last entry of a voxel, so hits win).  cnt[1] counts
// them, cnt[3] the finished workgroups; cnt[2] receives the list length.
__global__ void k_scan_hits(Grid g, const int32_t* __restrict__ origin,
                            const int32_t* __restrict__ ends, const uint8_t* __restrict__ hits,
                            int64_t n, int32_t* cnt, int32_t* lxyz, uint8_t* lst, int64_t cap) {
    const int o[3] = {origin[0], origin[1], origin[2]};
    const bool o_in = in_extent(g, o);
    const int64_t base = cnt[0] < cap ? cnt[0] : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r0 = blockIdx.x * (int64_t)blockDim.x; r0 < n; r0 += stride) {
        const int64_t r = r0 + threadIdx.x;
        int e[3] = {0, 0, 0};
        bool emit = false;
        if (r < n) {
            e[0] = ends[3 * r];
            e[1] = ends[3 * r + 1];
            e[2] = ends[3 * r + 2];
            emit = hits[r] != 0 && o_in && in_extent(g, e);
        }
        const int idx = wave_append(emit, cnt + 1);
        if (emit) {
            const int64_t p = base + idx;
            lxyz[3 * p] = e[0];
            lxyz[3 * p + 1] = e[1];
            lxyz[3 * p + 2] = e[2];
            lst[p] = 1;
        }
    }
    // the last workgroup to finish writes the list length into cnt[2]
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(cnt + 3, 1) == (int)gridDim.x - 1)
            cnt[2] = (int32_t)(base + atomicAdd(cnt + 1, 0));
    }
}

// Pool slots holding an obstacle, in chunks of 256 slots per wave: lane l
// reads slots 4l .. 4l + 3 of the chunk whole (four 16-byte loads each, all
// in flight together), the wave takes an exclusive prefix sum of the lanes'
// counts, and one counter atomic per chunk reserves the list positions.
// The occupancy words stay in w[t][0..3] for the caller.
struct SlotChunk {
    uint4 w[4][4];
    uint32_t has;     // bit t: slot 4 lane + t holds an obstacle
    int pos;          // first list position of this lane's slots
    int total;        // obstacle slots in the chunk
};

__device__ inline void scan_chunk(const Grid& g, int64_t c0, int64_t n, int32_t* counter,
                                  SlotChunk& c) {
    const int lane = __lane_id();
    c.has = 0u;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t slot = c0 + 4 * lane + t;
        const uint4* p = (const uint4*)(g.occ + (slot < n ? slot : 0) * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) c.w[t][q] = slot < n ? p[q] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint32_t a = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) a |= c.w[t][q].x | c.w[t][q].y | c.w[t][q].z | c.w[t][q].w;
        c.has |= (a != 0u ? 1u : 0u) << t;
    }
    const int mine = __popc(c.has);
    int incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    c.total = __shfl(incl, 63);
    int base = 0;
    if (lane == 63 && c.total > 0) base = atomicAdd(counter, c.total);
    base = __shfl(base, 63);
    c.pos = base + incl - mine;
}

// ---------------------------------------------------------------------------
// Compaction: the blocks holding an obstacle (coordinates and occupancy
// words) are copied into a list, from which a global transform rebuilds the
// pool; blocks that no longer hold an obstacle and lie beyond R blocks of
// every obstacle block drop out.
// ---------------------------------------------------------------------------
// Pool growth (the context moves onto a larger workspace; the blocks and
// their field are copied, nothing is recomputed).  Tile positions depend on
// the hash capacity, so the tile tables are rebuilt: k_tile_rehash, one wave
// per old table position, inserts the tile's key into the new hash, records
// the new position in map[old position] (-1 for an empty position) and
// copies the tile's slot table, obstacle mask and flag.
__global__ void __launch_bounds__(64) k_tile_rehash(Grid o, Grid n, int32_t* map) {
    const int lane = threadIdx.x;
    for (int64_t p = blockIdx.x; p <= (int64_t)o.tmask; p += gridDim.x) {
        const unsigned long long key = o.tkeys[p];
        int32_t q = -1;
        if (key != KEY_EMPTY && lane == 0) {
            bool created;
            q = hinsert(n.tkeys, n.tmask, key, &created);
            if (q < 0) set_error(n, -3 /* EDT_ERR_CAPACITY */);
        }
        q = __shfl(q, 0);
        if (lane == 0) map[p] = q;
        if (q < 0) continue;
        const int4* src = (const int4*)(o.tslots + p * 512);
        int4* dst = (int4*)(n.tslots + (int64_t)q * 512);
        dst[lane] = src[lane];
        dst[lane + 64] = src[lane + 64];
        if (lane < 16) n.tobst[(int64_t)q * 16 + lane] = o.tobst[p * 16 + lane];
        if (lane == 0) n.tflag[q] = o.tflag[p];
    }
}

// Second step of the growth: the tile list and the face-neighbour records
// hold table positions; translate them through map.  Entries that do not
// name a position of the old table (face records are only written for
// d_max <= 64) become -1.
__global__ void k_tile_remap(Grid o, Grid n, const int32_t* map) {
    const int64_t nt = o.cnt[C_NTILE];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nt;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t t = o.tlist[i];
        n.tlist[i] = (t >= 0 && t <= (int64_t)o.tmask) ? map[t] : -1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t v = o.tinfo[i * 8 + k];
            n.tinfo[i * 8 + k] = (v >= 0 && v <= (int64_t)o.tmask) ? map[v] : -1;
        }
    }
}

// Last step of the growth: a call that ran out of pool advanced the block
// counter past the old capacity without writing those slots; only the slots
// below it were claimed.  The pool abort flag no longer applies.
__global__ void k_grow_counts(Grid n, int32_t old_max_blocks) {
    if (n.cnt[C_NBLK] > old_max_blocks) n.cnt[C_NBLK] = old_max_blocks;
    n.cnt[C_ABORT] = 0;
}

__global__ void __launch_bounds__(64) k_compact_gather(Grid g, int32_t* count, int32_t* xyz,
                                                       uint32_t* bits) {
    const int lane = threadIdx.x;
    const int64_t n0 = g.cnt[C_NBLK];
    const int64_t n = n0 < g.max_blocks ? n0 : g.max_blocks;
    for (int64_t c0 = 256 * (int64_t)blockIdx.x; c0 < n; c0 += 256 * (int64_t)gridDim.x) {
        SlotChunk c;
        scan_chunk(g, c0, n, count, c);
        int idx = c.pos;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (!((c.has >> t) & 1u)) continue;
            uint4* dst = (uint4*)(bits + (int64_t)idx * 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = c.w[t][q];
            int bx, by, bz;
            unpack_key(g.bkey[c0 + 4 * lane + t], bx, by, bz);
            xyz[3 * (int64_t)idx] = bx;
            xyz[3 * (int64_t)idx + 1] = by;
            xyz[3 * (int64_t)idx + 2] = bz;
            ++idx;
        }
    }
}

// ---------------------------------------------------------------------------
// Interior distances: for an occupied voxel, the squared distance to the
// nearest free voxel of the extent, clamped to D (the definition of the field
// with occupied and free exchanged: the inside half of a signed distance
// field).  Only blocks holding an obstacle carry interior values.  Every other
// block of the extent, in the pool or not, is all free, so both intermediate
// passes are 0 on it; the passes below take such blocks as 0 without storage.
// ---------------------------------------------------------------------------

// Lists the pool blocks holding an obstacle and writes every slot's interior
// index (-1 for the others).
__global__ void __launch_bounds__(64) k_int_list(Grid g) {
    const int lane = threadIdx.x;
    const int64_t n0 = g.cnt[C_NBLK];
    const int64_t n = n0 < g.max_blocks ? n0 : g.max_blocks;
    for (int64_t c0 = 256 * (int64_t)blockIdx.x; c0 < n; c0 += 256 * (int64_t)gridDim.x) {
        SlotChunk c;
        scan_chunk(g, c0, n, &g.cnt[C_NINT], c);
        int idx = c.pos;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t slot = c0 + 4 * lane + t;
            if (slot >= n) continue;
            int32_t v = -1;
            if ((c.has >> t) & 1u) {
                if (idx < g.max_int) {
                    g.ilist[idx] = (int32_t)slot;
                    v = idx;
                } else {
                    set_error(g, -3 /* EDT_ERR_CAPACITY */);
                }
                ++idx;
            }
            g.iidx[slot] = v;
        }
    }
}

// Interior pass x: per row of a listed block, the distance along x to the
// nearest free voxel of the extent, squared and clamped to D.  One wave per
// block, lane = row y + 8z.  Neighbour blocks are read outwards until every
// lane has met a free voxel on both sides, at most R blocks each way (a voxel
// farther than that is beyond d_max).  Rows outside the extent get D.
__global__ void __launch_bounds__(64) k_int_x(Grid g) {
    __shared__ int32_t nb[72];
    const int lane = threadIdx.x;
    const int64_t n0 = g.cnt[C_NINT];
    const int64_t n = n0 < g.max_int ? n0 : g.max_int;
    const int R = g.R;
    const uint8_t* occ8 = (const uint8_t*)g.occ;
    const int y = lane & 7, z = lane >> 3;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int32_t slot = g.ilist[i];
        int bx, by, bz;
        unpack_key(g.bkey[slot], bx, by, bz);
        for (int k = lane; k < 2 * R + 1; k += 64)
            nb[k] = k == R ? slot : find_block(g, bx - R + k, by, bz);
        __syncthreads();
        const bool in = 8 * by + y < g.ny && 8 * bz + z < g.nz;
        // free voxels of row (y, z) in block bx + k (extent voxels only)
        auto freebits = [&](int k) -> uint32_t {
            const int w = g.nx - 8 * (bx + k);
            const uint32_t ext = w >= 8 ? 0xffu : (1u << w) - 1u;
            const int32_t s2 = nb[R + k];
            return s2 < 0 ? ext : ~(uint32_t)occ8[(int64_t)s2 * 64 + lane] & ext;
        };
        const uint32_t own = freebits(0);
        // nearest free voxel left of the block (offset from voxel 0 of the
        // block, negative) and right of it (offset, >= 8)
        int left = -(1 << 16), right = 1 << 16;
        bool dl = !in, dr = !in;
        for (int k = 1; k <= R; ++k) {
            if (!dl) {
                if (bx - k < 0) {
                    dl = true;
                } else {
                    const uint32_t f = freebits(-k);
                    if (f) { left = -8 * k + (31 - __clz(f)); dl = true; }
                }
            }
            if (!dr) {
                if (bx + k >= g.nbx) {
                    dr = true;
                } else {
                    const uint32_t f = freebits(k);
                    if (f) { right = 8 * k + (__ffs(f) - 1); dr = true; }
                }
            }
            if (__ballot(!(dl && dr)) == 0ull) break;
        }
        uint16_t* dst = g.ic1 + i * 512 + y + 64 * z;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int d = min(x - left, right - x);
#pragma unroll
            for (int xx = 0; xx < 8; ++xx)
                if ((own >> xx) & 1u) d = min(d, abs(x - xx));
            d = min(d, g.dmax);
            dst[8 * x] = (uint16_t)(in ? d * d : g.D);
        }
        __syncthreads();
    }
}

// Interior pass along y (AXIS 1: ic1 -> ic2) or z (AXIS 2: ic2 -> ic1, the
// interior field): out(t) = min(D, min over t' of in(t') + (t - t')^2) along
// the axis, where `in` is the previous interior pass on listed blocks and 0
// on every other voxel of the extent.  One wave per listed block, lane = one
// column of 8 outputs.  Neighbour blocks are visited outwards and the walk
// stops once no lane can improve: every voxel of block offset k is at least
// 8(k - 1) + 1 away.  Columns outside the extent get D.
template <int AXIS>
__global__ void __launch_bounds__(64) k_int_yz(Grid g) {
    __shared__ int32_t nb[72];   // interior index of block offset k - R; -1 all free; -2 outside
    const int lane = threadIdx.x;
    const int64_t n0 = g.cnt[C_NINT];
    const int64_t n = n0 < g.max_int ? n0 : g.max_int;
    const int R = g.R;
    const int D = g.D;
    const uint16_t* src = AXIS == 1 ? g.ic1 : g.ic2;
    uint16_t* dst = AXIS == 1 ? g.ic2 : g.ic1;
    const int ca = lane & 7, cb = lane >> 3;   // column (x, z) for y, (x, y) for z
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        int bx, by, bz;
        unpack_key(g.bkey[g.ilist[i]], bx, by, bz);
        const int bc = AXIS == 1 ? by : bz;
        const int nbc = AXIS == 1 ? g.nby : g.nbz;
        for (int k = lane; k < 2 * R + 1; k += 64) {
            const int b = bc - R + k;
            int32_t e = -2;
            if (k == R) {
                e = (int32_t)i;
            } else if (b >= 0 && b < nbc) {
                const int32_t s2 = AXIS == 1 ? find_block(g, bx, b, bz) : find_block(g, bx, by, b);
                e = s2 < 0 ? -1 : g.iidx[s2];
            }
            nb[k] = e;
        }
        __syncthreads();
        const bool in = 8 * bx + ca < g.nx &&
                        (AXIS == 1 ? 8 * bz + cb < g.nz : 8 * by + cb < g.ny);
        int best[8];
        {
            const uint4 q = *reinterpret_cast<const uint4*>(src + i * 512 + 8 * lane);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                int b = D;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int v = (int)((w[u >> 1] >> (16 * (u & 1))) & 0xffffu);
                    b = min(b, v + (t - u) * (t - u));
                }
                best[t] = b;
            }
        }
        for (int k = 1; k <= R; ++k) {
            int worst = 0;
#pragma unroll
            for (int t = 0; t < 8; ++t) worst = max(worst, best[t]);
            const int lb = 8 * (k - 1) + 1;
            if (__ballot(in && lb * lb < worst) == 0ull) break;
#pragma unroll
            for (int side = -1; side <= 1; side += 2) {
                const int32_t e = nb[R + side * k];
                if (e == -2) continue;
                if (e == -1) {
                    // all free: the block's voxel nearest to the column
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int d = side < 0 ? t + 8 * (k - 1) + 1 : 8 * k - t;
                        best[t] = min(best[t], d * d);
                    }
                } else {
                    const uint4 q = *reinterpret_cast<const uint4*>(src + (int64_t)e * 512 + 8 * lane);
                    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int v = (int)((w[u >> 1] >> (16 * (u & 1))) & 0xffffu);
                        const int tu = side * 8 * k + u;
#pragma unroll
                        for (int t = 0; t < 8; ++t) best[t] = min(best[t], v + (t - tu) * (t - tu));
                    }
                }
            }
        }
        uint16_t* o = dst + i * 512;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint16_t v = (uint16_t)(in ? min(best[t], D) : D);
            if (AXIS == 1) o[cb + 8 * ca + 64 * t] = v;     // layout z + 8x + 64y
            else o[lane + 64 * t] = v;                      // layout x + 8y + 64z
        }
        __syncthreads();
    }
}

// Signed squared distance of voxel (x, y, z) inside the extent: s for a free
// voxel, minus the interior value for an occupied one.
__device__ inline int32_t signed_at(const Grid& g, int x, int y, int z) {
    const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
    if (slot < 0) return g.D;
    const int v = (x & 7) + 8 * (y & 7) + 64 * (z & 7);
    if ((g.occ[(int64_t)slot * 16 + (v >> 5)] >> (v & 31)) & 1u) {
        const int32_t ii = g.iidx[slot];
        return -(ii >= 0 ? (int32_t)g.ic1[(int64_t)ii * 512 + v] : g.D);
    }
    return s_int(g, g.s[(int64_t)slot * 512 + v]);
}

__global__ void k_query_signed(Grid g, const int32_t* __restrict__ xyz, int64_t n,
                               int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        const bool in = x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz;
        out[i] = in ? signed_at(g, x, y, z) : g.D;
    }
}

__global__ void k_clear_error(Grid g) { g.cnt[C_ERR] = 0; }

}  // namespace edt
