// edt_batch.hip -- global transform of many dense maps in one launch.
//
// Every map goes through the same three separable passes as the single-map
// transform (x from the occupancy bytes, then the windowed minimum along y
// and z; d_max <= 64).  Maps are dense, so a block is addressed by its
// position in the map's block grid and no region growth is needed.
//
// Work items (per map, in map order; maps are ordered largest first):
//   phase 0 (x)  a strip of 8 blocks along x at (by, bz)
//   phase 1 (y)  a run of up to `lrun` blocks along y at (bx, bz)
//   phase 2 (z)  a run of up to `lrun` blocks along z at (bx, by)
// FUSED runs all three phases of all maps in one cooperative persistent
// launch: waves take items from a per-phase queue (chunks of `chunk` items
// through one atomic, or a static stride), and a grid-wide barrier separates
// the phases, so a map's y pass starts only after every x item is written.
// PHASED runs the same schedule as three plain launches, one per phase, each
// a kernel of its own phase only (its own register and LDS footprint; the
// kernel boundary replaces the grid barrier).  PER_MAP launches the phase
// kernels three times per map.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include "edt.h"
#include "edt_win.h"

namespace {

using namespace edt;

struct MapDev {
    int nx, ny, nz;
    int nbx, nby, nbz;
    int nxr;                 // strips of 8 blocks along x
    int pad;
    int64_t occ_off;         // bytes into the occupancy input
    int64_t out_off;         // int32 elements into the output
    int64_t blk_off;         // blocks into g1 / g2
    int64_t pad2;            // (64 bytes: read as four 16-byte words)
};

struct BArgs {
    const MapDev* maps;
    const int32_t* pref;     // [3][n_maps + 1] item prefix sums (phase-major)
    int32_t* queues;         // [3][n_maps + 1] grab counters
    const int32_t* itemmap;  // [3][icap] map of each work item
    int64_t icap;
    const uint8_t* occ;
    int32_t* out;
    uint8_t* g1;             // distance along x, min(d, d_max) (8 bits per voxel)
    uint16_t* g2;
    const uint16_t* dblock;
    const uint8_t* dblock8;  // g1 of blocks beyond a map: d_max everywhere
    uint32_t* dummy;
    int n_maps;
    int dmax, D;
    int lrun, chunk, schedule;
};


// g1 of block (bx, by, bz): this lane's 8 bytes (the 8 values along y of
// column x + 8z), or the d_max block beyond the map.
__device__ inline const uint2* blk_ptr8(const uint8_t* arr, const MapDev& m, int bx, int by,
                                        int bz, const uint8_t* dblock8, int lane) {
    if (bx < 0 || by < 0 || bz < 0 || bx >= m.nbx || by >= m.nby || bz >= m.nbz)
        return (const uint2*)dblock8 + lane;
    const int64_t b = m.blk_off + ((int64_t)bz * m.nby + by) * m.nbx + bx;
    return (const uint2*)arr + b * 64 + lane;
}

// Eight 8-bit distances (at most 64) to their squares in the window's
// representation, packed in 16-bit pairs in order.  v_perm builds each pair
// with the high bytes 0x64 (F16: 0x64nn is the binary16 of 1024 + n, exact,
// so subtracting 1024 leaves n, and n^2 <= 1600 is exact) or zero (integer
// squares <= 4096).
template <bool F16>
__device__ inline uint4 g1_squares(uint2 w) {
    const uint32_t hi = F16 ? 0x64646464u : 0u;
    auto pair = [&](uint32_t word, uint32_t k) -> uint32_t {
        const uint32_t sel = k | (4u << 8) | ((k + 1u) << 16) | (4u << 24);
        const uint32_t x = __builtin_amdgcn_perm(hi, word, sel);
        if (F16) {
            const h16x2 f = as_h16x2(as_u16x2(x)) - (h16x2){(_Float16)1024, (_Float16)1024};
            return as_u32(as_u16x2(f * f));
        }
        const u16x2 v = as_u16x2(x);
        return as_u32(v * v);
    };
    return make_uint4(pair(w.x, 0u), pair(w.x, 2u), pair(w.y, 0u), pair(w.y, 2u));
}

// phase 0: distance along x for a strip of 8 blocks.  The wave walks
// the strip's 64 rows (y, z); for each row the lanes read the window
// x = 8 (bx0 - M) .. 8 (bx0 + 8 + M) - 1 with coalesced byte loads (64 + 16M
// bytes, up to three per lane), ballots make it a bit string, which goes
// through LDS to lane r.  Then
// every lane holds its own row and sweeps it with carried distances, in
// packed 16-bit pairs: blocks j and j + 4 of the strip at once (the carry
// into block 4 comes from the bits of blocks 0..3, the carry out of block 3
// from those of blocks 4..7), about 6 operations per voxel; M = ceil(d_max /
// 8) blocks of context cover d_max.  Results, min(d, d_max) in one byte
// (phase 1 squares them as it loads them: half the bytes of a stored
// square), gather in LDS in the g1 block layout (y + 8x + 64z), two blocks
// at a time, and leave as 8-byte stores.
// LDS of item_x: the row words of the window (64 rows of up to three 64-bit
// words), which two result blocks (2 x 512 bytes) reuse once they are read;
// the workgroup's share is sized at launch, one slice per wave
constexpr size_t XBYTES_PER_WAVE = 2 * 512 * sizeof(uint16_t);
extern __shared__ __align__(16) uint16_t xlds[];

// each 16-bit half of t: all ones if its bit 15 is set, else zero.  Written
// as the instruction itself: as plain code the compiler turns the masks into
// per-half compares and selects, three times the work of this one operation.
__device__ inline uint32_t pk_sign_mask(uint32_t t) {
    uint32_t r;
    // op_sel_hi:[0,1]: the high half shifts by the constant's low half too
    asm("v_pk_ashrrev_i16 %0, 15, %1 op_sel_hi:[0,1]" : "=v"(r) : "v"(t));
    return r;
}

template <int M>
__device__ void item_x(const BArgs& a, const MapDev& m, int li) {
    constexpr int NBYTES = 64 + 16 * M;          // window bytes per row
    constexpr int NWIN = (NBYTES + 63) / 64;     // 64-bit words of the window
    // rows whose loads are in flight together (32 measured fastest: 16 keeps
    // fewer loads in flight, 64 needs 143 registers)
    constexpr int RB = 32;
    constexpr int NB = 8 + 2 * M;                // window blocks
    uint16_t* buf = xlds + (threadIdx.x >> 6) * (XBYTES_PER_WAVE / sizeof(uint16_t));
    const int lane = threadIdx.x & 63;
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const int bx0 = 8 * (li % m.nxr);
    const int rest = li / m.nxr;
    const int by = rest % m.nby, bz = rest / m.nby;
    const int xs = 8 * (bx0 - M);
    // loads always hit a voxel of the map (clamped); bytes outside it are
    // dropped afterwards
    uint32_t xo[NWIN];
    bool vx[NWIN];
#pragma unroll
    for (int w = 0; w < NWIN; ++w) {
        const int x = xs + 64 * w + lane;
        vx[w] = 64 * w + lane < NBYTES && x >= 0 && x < nx;
        xo[w] = (uint32_t)min(max(x, 0), nx - 1);
    }
    const uint8_t* base = a.occ + m.occ_off;
    const int64_t zst = (int64_t)ny * nx;
    // the rows' window words (row r, word w at rowbits[NWIN r + w]) share the
    // buffer: they are read back before any result is written
    static_assert(NWIN * 64 * sizeof(unsigned long long) <= XBYTES_PER_WAVE, "row words");
    unsigned long long* rowbits = (unsigned long long*)buf;
#pragma unroll
    for (int r0 = 0; r0 < 64; r0 += RB) {
        uint32_t bt[RB][NWIN];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int r = r0 + k;
            const int Y = min(8 * by + (r & 7), ny - 1), Z = min(8 * bz + (r >> 3), nz - 1);
            const uint8_t* row = base + Z * zst + (int64_t)Y * nx;
#pragma unroll
            for (int w = 0; w < NWIN; ++w) bt[k][w] = row[xo[w]];
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int r = r0 + k;
            const bool rok = 8 * by + (r & 7) < ny && 8 * bz + (r >> 3) < nz;
#pragma unroll
            for (int w = 0; w < NWIN; ++w) {
                // every lane stores the same word (no per-lane branch)
                rowbits[NWIN * r + w] =
                    __builtin_amdgcn_ballot_w64(rok && vx[w] && bt[k][w] != 0u);
            }
        }
    }
    // window words of row `lane` (lo and hi halves)
    uint32_t rlo[NWIN], rhi[NWIN];
#pragma unroll
    for (int w = 0; w < NWIN; ++w) {
        const unsigned long long W = rowbits[NWIN * lane + w];
        rlo[w] = (uint32_t)W;
        rhi[w] = (uint32_t)(W >> 32);
    }
    // bytes of the row: block k of the window (k = 0 .. NB - 1)
    uint32_t b[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int w = k >> 3, h = (k >> 2) & 1, sh = 8 * (k & 3);
        b[k] = ((h ? rhi[w] : rlo[w]) >> sh) & 0xffu;
    }
    // "no obstacle": beyond every radius, and small enough that the carried
    // distances (at most 16 (M + 8) more) stay within 16 bits
    constexpr uint32_t FAR = 0x3000u;
    const uint32_t dmax = (uint32_t)a.dmax;
    // distance from the last voxel before the strip back to the nearest obstacle
    uint32_t L = FAR;
#pragma unroll
    for (int k = 0; k < M; ++k) L = b[k] ? (uint32_t)__clz(b[k]) - 24u : L + 8u;
    // the same from the last voxel of strip block 3
    const uint32_t W0 = b[M] | (b[M + 1] << 8) | (b[M + 2] << 16) | (b[M + 3] << 24);
    const uint32_t L4 = W0 ? (uint32_t)__clz(W0) : L + 32u;
    // rc[j]: distance from the first voxel after strip block j to the nearest
    // obstacle at or after it
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
    const int rofs = (lane & 7) + 64 * (lane >> 3);      // this row in the g1 block layout
    uint8_t* buf8 = (uint8_t*)buf;
    const int64_t brow = m.blk_off + ((int64_t)bz * m.nby + by) * m.nbx;
    // the row words are in registers from here on: the buffer takes results
    __builtin_amdgcn_wave_barrier();
    const u16x2 one = {1, 1};
    const u16x2 dmp = {(unsigned short)dmax, (unsigned short)dmax};
    uint32_t Lp = L | (L4 << 16);       // blocks 0..3 | blocks 4..7
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t bp = b[M + j] | (b[M + j + 4] << 16);
        uint32_t mk[8];
        u16x2 dp[8];
#pragma unroll
        for (int x = 0; x < 8; ++x)      // all ones where voxel x of the block is occupied
            mk[x] = pk_sign_mask(bp << (15 - x));
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            Lp = as_u32(as_u16x2(Lp) + one) & ~mk[x];
            dp[x] = as_u16x2(Lp);
        }
        uint32_t rr = rc[j] | (rc[j + 4] << 16);
#pragma unroll
        for (int x = 7; x >= 0; --x) {
            rr = as_u32(as_u16x2(rr) + one) & ~mk[x];
            const u16x2 v =
                __builtin_elementwise_min(__builtin_elementwise_min(dp[x], as_u16x2(rr)), dmp);
            buf8[rofs + 8 * x] = (uint8_t)v.x;
            buf8[512 + rofs + 8 * x] = (uint8_t)v.y;
        }
        // blocks j and j + 4: lane writes g1 elements 8 lane .. 8 lane + 7 of
        // each (8 bytes); the wave's LDS operations complete in order, the
        // barriers keep the compiler from moving them across
        __builtin_amdgcn_wave_barrier();
        const uint2 v0 = ((const uint2*)buf8)[lane];
        const uint2 v1 = ((const uint2*)buf8)[64 + lane];
        __builtin_amdgcn_wave_barrier();
        if (bx0 + j < m.nbx) *(uint2*)(a.g1 + (brow + bx0 + j) * 512 + 8 * lane) = v0;
        if (bx0 + j + 4 < m.nbx) *(uint2*)(a.g1 + (brow + bx0 + j + 4) * 512 + 8 * lane) = v1;
    }
}

// phase 1: windowed minimum along y (lane = x + 8z), g1 -> g2
template <int M>
__device__ void item_y(const BArgs& a, const MapDev& m, int li, uint32_t Dp) {
    const int lane = threadIdx.x & 63;
    const int nseg = (m.nby + a.lrun - 1) / a.lrun;
    const int bx = li % m.nbx;
    const int rest = li / m.nbx;
    const int bz = rest % m.nbz, seg = rest / m.nbz;
    (void)nseg;
    const int by0 = seg * a.lrun;
    const int len = min(a.lrun, m.nby - by0);
    const int out_lane = (lane & 7) * 8 + (lane >> 3);
    auto blk = [&](int b) -> uint4 {
        return g1_squares<win_f16(M)>(*blk_ptr8(a.g1, m, bx, b, bz, a.dblock8, lane));
    };
    // the block bases are uniform (scalar branch, scalar base, immediate row
    // offsets)
    auto emit = [&](int ob, const u16x2* acc, bool has1) {
        const int64_t b0 = m.blk_off + ((int64_t)bz * m.nby + ob) * m.nbx + bx;
        uint16_t* d0 = a.g2 + b0 * 512 + out_lane;
#pragma unroll
        for (int o = 0; o < 8; ++o) d0[64 * o] = acc[o].x;
        if (has1) {
            uint16_t* d1 = a.g2 + (b0 + m.nbx) * 512 + out_lane;
#pragma unroll
            for (int o = 0; o < 8; ++o) d1[64 * o] = acc[o].y;
        }
    };
    window_min<M, true, win_f16(M)>(by0, len, Dp, blk, emit);
}

// phase 2: windowed minimum along z, g2 -> dense int32 field.  An item is a
// strip of 64 voxels along x (8 blocks) at one y and a run of lrun blocks
// along z; lane l owns the column x = 8 bx0 + l, so every output store is 256
// contiguous bytes of the x-fastest field.
template <int M>
__device__ void item_z(const BArgs& a, const MapDev& m, int li, uint32_t Dp) {
    const int lane = threadIdx.x & 63;
    const int bx0 = 8 * (li % m.nxr);
    const int rest = li / m.nxr;
    const int Y = rest % m.ny, seg = rest / m.ny;
    const int bz0 = seg * a.lrun;
    const int len = min(a.lrun, m.nbz - bz0);
    const int bx = bx0 + (lane >> 3), by = Y >> 3;
    const int X = 8 * bx0 + lane;
    const bool col_ok = X < m.nx;
    const int rofs = (lane & 7) + 8 * (Y & 7);        // z-row (x' + 8y') of a g2 block
    const int64_t bcol = m.blk_off + (int64_t)by * m.nbx + bx;
    const int64_t bzst = (int64_t)m.nby * m.nbx;
    auto blk = [&](int b) -> uint4 {
        const bool ok = bx < m.nbx && b >= 0 && b < m.nbz;
        const uint4* p = ok ? (const uint4*)a.g2 + (bcol + b * bzst) * 64 + rofs
                            : (const uint4*)a.dblock + lane;
        return *p;
    };
    // the strip's row at z = 0 (uniform base; lane l writes x = 8 bx0 + l)
    int32_t* row0 = a.out + m.out_off + (int64_t)Y * m.nx + 8 * bx0;
    const int64_t zstride = (int64_t)m.nx * m.ny;
    auto emit = [&](int ob, const u16x2* acc, bool has1) {
        if (!col_ok) return;
        const int nz0 = min(8, m.nz - 8 * ob);                       // rows of block ob
        const int nz1 = has1 ? min(8, m.nz - 8 * ob - 8) : 0;        // rows of block ob + 1
        int32_t* p0 = row0 + (int64_t)(8 * ob) * zstride;
#pragma unroll
        for (int o = 0; o < 8; ++o)
            if (o < nz0) p0[o * zstride + lane] = win_f16(M) ? f16_int(acc[o].x) : (int)acc[o].x;
        int32_t* p1 = p0 + 8 * zstride;
#pragma unroll
        for (int o = 0; o < 8; ++o)
            if (o < nz1) p1[o * zstride + lane] = win_f16(M) ? f16_int(acc[o].y) : (int)acc[o].y;
    };
    window_min<M, true, win_f16(M)>(bz0, len, Dp, blk, emit);
}

// The item -> map table, the map records and the item offsets are read-only
// while the batch runs, and an item's index is wave-uniform: read through
// the constant address space they become scalar loads, so the map record and
// everything derived from it stay in scalar registers.
template <typename T>
__device__ inline const __attribute__((address_space(4))) T* as_const(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ inline MapDev load_map(const MapDev* maps, int mi) {
    static_assert(sizeof(MapDev) == 4 * sizeof(i32x4), "map record size");
    const auto* p = as_const((const i32x4*)(maps + mi));
    struct { i32x4 w0, w1, w2, w3; } r = {p[0], p[1], p[2], p[3]};
    return __builtin_bit_cast(MapDev, r);
}

template <int M, int PHASE>
__device__ inline void run_item(const BArgs& a, int gi, uint32_t Dp) {
    const int mi = as_const(a.itemmap)[PHASE * a.icap + gi];
    const MapDev m = load_map(a.maps, mi);
    const int li = gi - as_const(a.pref)[PHASE * (a.n_maps + 1) + mi];
    if (PHASE == 0) item_x<M>(a, m, li);
    else if (PHASE == 1) item_y<M>(a, m, li, Dp);
    else item_z<M>(a, m, li, Dp);
}

// Items [lo, hi) of phase PHASE; one wave per item.  Dynamic schedule: a
// wave takes `chunk` items per atomic on the phase's counter (cidx); static:
// wave w takes items lo + w, lo + w + nwaves, ...
template <int M, int PHASE>
__device__ void run_phase(const BArgs& a, int lo, int hi, int cidx) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    // item indices are wave-uniform: kept in scalar registers, so the map
    // record, the item's block coordinates and the row addresses derived
    // from them are scalar too
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const int nwaves = gridDim.x * wpb;
    const uint32_t Dw = win_f16(M) ? f16_bits((uint32_t)a.D) : (uint32_t)a.D;
    const uint32_t Dp = Dw | (Dw << 16);        // D in the window's representation
    if (a.schedule == 0) {
        for (;;) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&a.queues[cidx], a.chunk);
            base = __builtin_amdgcn_readfirstlane(base) + lo;   // lane 0's grab
            if (base >= hi) break;
            const int end = min(base + a.chunk, hi);
            for (int i = base; i < end; ++i) run_item<M, PHASE>(a, i, Dp);
        }
    } else {
        for (int i = lo + wid; i < hi; i += nwaves) run_item<M, PHASE>(a, i, Dp);
    }
}

// FUSED: phases 0..2 of all maps, grid barrier between phases.
template <int M>
__global__ void __launch_bounds__(512) k_batch_fused(BArgs a) {
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    const int n = a.n_maps;
    run_phase<M, 0>(a, a.pref[0], a.pref[n], n);
    grid.sync();
    run_phase<M, 1>(a, a.pref[n + 1], a.pref[2 * n + 1], 2 * n + 1);
    grid.sync();
    run_phase<M, 2>(a, a.pref[2 * n + 2], a.pref[3 * n + 2], 3 * n + 2);
}

// PHASED: one phase of all maps (map = -1), PER_MAP: one phase of one map.
template <int M, int PHASE>
__global__ void __launch_bounds__(512) k_batch_phase(BArgs a, int map) {
    const int n = a.n_maps;
    const int* pref = a.pref + PHASE * (n + 1);
    if (map < 0) run_phase<M, PHASE>(a, pref[0], pref[n], PHASE * (n + 1) + n);
    else run_phase<M, PHASE>(a, pref[map], pref[map + 1], PHASE * (n + 1) + map);
}

// Item prefix sums of the three phases over the maps (processing order), one
// workgroup of 1024 threads: every thread counts one map's items, a scan
// across the workgroup gives the offsets, chunks of 1024 maps carry on.
__global__ void __launch_bounds__(1024) k_batch_prefix(const MapDev* maps, int n, int lrun,
                                                       int32_t* pref) {
    __shared__ int wsum[16][3];
    __shared__ int carry[3];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t < 3) carry[t] = 0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += 1024) {
        const int i = i0 + t;
        int c[3] = {0, 0, 0};
        if (i < n) {
            const MapDev m = maps[i];
            c[0] = m.nxr * m.nby * m.nbz;
            c[1] = m.nbx * m.nbz * ((m.nby + lrun - 1) / lrun);
            c[2] = m.nxr * m.ny * ((m.nbz + lrun - 1) / lrun);
        }
        int incl[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            incl[p] = c[p];
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(incl[p], o);
                if (lane >= o) incl[p] += v;
            }
            if (lane == 63) wsum[w][p] = incl[p];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            int before = carry[p];
            for (int v = 0; v < w; ++v) before += wsum[v][p];
            if (i < n) pref[p * (n + 1) + i] = before + incl[p] - c[p];
            if (i == n - 1) pref[p * (n + 1) + n] = before + incl[p];
        }
        __syncthreads();
        if (t < 3) {
            int tot = 0;
            for (int v = 0; v < 16; ++v) tot += wsum[v][t];
            carry[t] += tot;
        }
        __syncthreads();
    }
}

// The map of every work item of every phase (one workgroup per map), so an
// item finds its map with one load.
__global__ void k_batch_itemmap(const int32_t* pref, int n, int32_t* itemmap, int64_t icap) {
    const int i = blockIdx.x;
    for (int p = 0; p < 3; ++p) {
        const int lo = pref[p * (n + 1) + i], hi = pref[p * (n + 1) + i + 1];
        for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) itemmap[p * icap + k] = i;
    }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

struct BLayout {
    int64_t off_maps, off_pref, off_queues, off_itemmap, off_g1, off_g2, off_dblock,
        off_dblock8, off_dummy, total;
    int64_t nblocks;
    int64_t icap;            // item-map entries per phase
};

bool blayout(const edt_batch_map* maps, int n, int dmax, BLayout* L) {
    if (!maps || n < 1 || n > (1 << 16) || dmax < 1 || dmax > 64) return false;
    int64_t nb = 0, ic0 = 0, ic1 = 0, ic2 = 0;
    for (int i = 0; i < n; ++i) {
        const edt_batch_map& m = maps[i];
        if (m.nx < 1 || m.ny < 1 || m.nz < 1 || m.nx > 4096 || m.ny > 4096 || m.nz > 4096)
            return false;
        if (m.occ_offset < 0 || m.out_offset < 0) return false;
        nb += (int64_t)((m.nx + 7) / 8) * ((m.ny + 7) / 8) * ((m.nz + 7) / 8);
        // most items per phase (run length 1): x strips, y runs, z strips
        const int64_t nbx = (m.nx + 7) / 8, nby = (m.ny + 7) / 8, nbz = (m.nz + 7) / 8;
        const int64_t nxr = (nbx + 7) / 8;
        ic0 += nxr * nby * nbz;
        ic1 += nbx * nby * nbz;
        ic2 += nxr * m.ny * nbz;
    }
    const int64_t icap = ic0 > ic1 ? (ic0 > ic2 ? ic0 : ic2) : (ic1 > ic2 ? ic1 : ic2);
    if (nb > (1ll << 26)) return false;
    int64_t o = 0;
    L->off_maps = o; o += align256((int64_t)n * sizeof(MapDev));
    L->off_pref = o; o += align256((int64_t)3 * (n + 1) * 4);
    L->off_queues = o; o += align256((int64_t)3 * (n + 1) * 4);
    L->off_itemmap = o; o += align256(3 * icap * 4);
    L->icap = icap;
    L->off_g1 = o; o += align256(nb * 512);
    L->off_g2 = o; o += align256(nb * 1024);
    L->off_dblock = o; o += 1024;
    L->off_dblock8 = o; o += 512;
    L->off_dummy = o; o += align256(256 * 64 * 4 + 1024);
    L->total = o;
    L->nblocks = nb;
    return true;
}

int grid_cap(int64_t work, int cap) {
    int64_t g = work < 1 ? 1 : work;
    return (int)(g > cap ? cap : g);
}

}  // namespace

struct edt_batch {
    int n;
    int dmax;
    int M;
    BLayout L;
    char* ws;
    MapDev* host_maps;       // in processing order
    int64_t* map_items[3];   // per map item counts at the last lrun (host copy)
    int last_lrun;
    int cus;
};

namespace {

template <int M>
edt_status launch_batch(edt_batch* b, const BArgs& a, int mode, int waves_per_cu, int wg_waves,
                        hipStream_t st) {
    const int bs = 64 * wg_waves;
    const size_t lds = wg_waves * XBYTES_PER_WAVE;
    if (mode == EDT_BATCH_FUSED) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_fused<M>, bs, lds) !=
            hipSuccess)
            return EDT_ERR_HIP;
        int wgs_per_cu =
            waves_per_cu > 0 ? (waves_per_cu + wg_waves - 1) / wg_waves : 8 / wg_waves;
        if (wgs_per_cu < 1) wgs_per_cu = 1;
        const int g = b->cus * (wgs_per_cu < per_cu ? wgs_per_cu : per_cu);
        if (g < 1) return EDT_ERR_HIP;
        void* args[] = {(void*)&a};
        if (hipLaunchCooperativeKernel((const void*)k_batch_fused<M>, dim3(g), dim3(bs), args,
                                       (unsigned)lds, st) != hipSuccess)
            return EDT_ERR_HIP;
        return EDT_OK;
    }
    // only the x phase uses LDS
    const void* kern[3] = {(const void*)k_batch_phase<M, 0>, (const void*)k_batch_phase<M, 1>,
                           (const void*)k_batch_phase<M, 2>};
    const size_t klds[3] = {lds, 0, 0};
    const int wpc = waves_per_cu > 0 ? waves_per_cu : 8;
    if (mode == EDT_BATCH_PHASED) {
        // as many waves as the fused launch would have, per phase
        for (int phase = 0; phase < 3; ++phase) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern[phase], bs,
                                                             klds[phase]) != hipSuccess)
                return EDT_ERR_HIP;
            const int wgs_per_cu = (wpc + wg_waves - 1) / wg_waves;
            const int g = b->cus * (wgs_per_cu < per_cu ? wgs_per_cu : per_cu);
            if (g < 1) return EDT_ERR_HIP;
            int map = -1;
            void* args[] = {(void*)&a, (void*)&map};
            if (hipLaunchKernel(kern[phase], dim3(g), dim3(bs), args, klds[phase], st) !=
                hipSuccess)
                return EDT_ERR_HIP;
        }
        return EDT_OK;
    }
    // PER_MAP: three launches per map, each sized to the map's items
    for (int mi = 0; mi < b->n; ++mi) {
        const MapDev& m = b->host_maps[mi];
        const int64_t items[3] = {
            (int64_t)m.nxr * m.nby * m.nbz,
            (int64_t)m.nbx * m.nbz * ((m.nby + a.lrun - 1) / a.lrun),
            (int64_t)m.nxr * m.ny * ((m.nbz + a.lrun - 1) / a.lrun)};
        for (int phase = 0; phase < 3; ++phase) {
            const int waves = grid_cap(items[phase], b->cus * wpc);
            int map = mi;
            void* args[] = {(void*)&a, (void*)&map};
            if (hipLaunchKernel(kern[phase], dim3((waves + wg_waves - 1) / wg_waves), dim3(bs),
                                args, klds[phase], st) != hipSuccess)
                return EDT_ERR_HIP;
        }
    }
    return hipGetLastError() == hipSuccess ? EDT_OK : EDT_ERR_HIP;
}

}  // namespace

extern "C" {

int64_t edt_batch_workspace_bytes(const edt_batch_map* maps, int32_t n_maps, int32_t d_max) {
    BLayout L;
    if (!blayout(maps, n_maps, d_max, &L)) return EDT_ERR_ARG;
    return L.total;
}

edt_status edt_batch_create(const edt_batch_map* maps, int32_t n_maps, int32_t d_max, void* d_ws,
                            int64_t ws_bytes, void* stream, edt_batch** out) {
    if (!out) return EDT_ERR_ARG;
    *out = nullptr;
    BLayout L;
    if (!blayout(maps, n_maps, d_max, &L) || !d_ws || ((uintptr_t)d_ws & 255)) return EDT_ERR_ARG;
    if (ws_bytes < L.total) return EDT_ERR_CAPACITY;
    edt_batch* b = (edt_batch*)calloc(1, sizeof(edt_batch));
    if (!b) return EDT_ERR_CAPACITY;
    b->host_maps = (MapDev*)calloc((size_t)n_maps, sizeof(MapDev));
    if (!b->host_maps) {
        free(b);
        return EDT_ERR_CAPACITY;
    }
    b->n = n_maps;
    b->dmax = d_max;
    b->M = (d_max + 7) / 8;
    b->L = L;
    b->ws = (char*)d_ws;
    // processing order: largest map first (longest-processing-time first)
    int* order = (int*)malloc(sizeof(int) * (size_t)n_maps);
    if (!order) {
        free(b->host_maps);
        free(b);
        return EDT_ERR_CAPACITY;
    }
    for (int i = 0; i < n_maps; ++i) order[i] = i;
    for (int i = 1; i < n_maps; ++i) {   // insertion sort by volume, descending
        const int v = order[i];
        const int64_t vol = (int64_t)maps[v].nx * maps[v].ny * maps[v].nz;
        int j = i - 1;
        while (j >= 0 && (int64_t)maps[order[j]].nx * maps[order[j]].ny * maps[order[j]].nz < vol) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
    int64_t blk = 0;
    for (int k = 0; k < n_maps; ++k) {
        const edt_batch_map& s = maps[order[k]];
        MapDev& m = b->host_maps[k];
        m.nx = s.nx; m.ny = s.ny; m.nz = s.nz;
        m.nbx = (s.nx + 7) / 8; m.nby = (s.ny + 7) / 8; m.nbz = (s.nz + 7) / 8;
        m.nxr = (m.nbx + 7) / 8;
        m.occ_off = s.occ_offset;
        m.out_off = s.out_offset;
        m.blk_off = blk;
        blk += (int64_t)m.nbx * m.nby * m.nbz;
    }
    free(order);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        free(b->host_maps);
        free(b);
        return EDT_ERR_HIP;
    }
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(b->ws + L.off_maps, b->host_maps, sizeof(MapDev) * (size_t)n_maps,
                       hipMemcpyHostToDevice, st) != hipSuccess) {
        free(b->host_maps);
        free(b);
        return EDT_ERR_HIP;
    }
    // the block of D values read for blocks beyond a map, in the window's
    // representation (binary16 for small radii)
    const uint32_t D = win_f16(b->M) ? f16_bits((uint32_t)(d_max * d_max))
                                     : (uint32_t)(d_max * d_max);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, (uint32_t*)(b->ws + L.off_dblock),
                       (int64_t)256, D | (D << 16));
    // and the x distance d_max, one byte per voxel, for g1
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(128), 0, st, (uint32_t*)(b->ws + L.off_dblock8),
                       (int64_t)128, (uint32_t)d_max * 0x01010101u);
    if (hipStreamSynchronize(st) != hipSuccess) {   // the host map table may go away now
        free(b->host_maps);
        free(b);
        return EDT_ERR_HIP;
    }
    b->last_lrun = 0;
    *out = b;
    return EDT_OK;
}

edt_status edt_batch_destroy(edt_batch* b) {
    if (!b) return EDT_ERR_ARG;
    free(b->host_maps);
    free(b);
    return EDT_OK;
}

edt_status edt_batch_run(edt_batch* b, const uint8_t* d_occ, int32_t* d_out, int32_t mode,
                         const edt_tune* tune, void* stream) {
    if (!b || !d_occ || !d_out) return EDT_ERR_ARG;
    if (mode != EDT_BATCH_FUSED && mode != EDT_BATCH_PER_MAP && mode != EDT_BATCH_PHASED)
        return EDT_ERR_ARG;
    edt_tune t = {8, 8, 4, 0, 4};
    if (tune) t = *tune;
    if (t.wg_waves == 0) t.wg_waves = 4;
    if (t.lrun < 1 || t.lrun > 64 || t.chunk < 1 || t.chunk > 1024 || t.waves_per_cu < 0 ||
        t.waves_per_cu > 64 || (t.schedule != 0 && t.schedule != 1) ||
        (t.wg_waves != 1 && t.wg_waves != 2 && t.wg_waves != 4 && t.wg_waves != 8))
        return EDT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const BLayout& L = b->L;
    BArgs a;
    a.maps = (const MapDev*)(b->ws + L.off_maps);
    a.pref = (const int32_t*)(b->ws + L.off_pref);
    a.queues = (int32_t*)(b->ws + L.off_queues);
    a.occ = d_occ;
    a.out = d_out;
    a.g1 = (uint8_t*)(b->ws + L.off_g1);
    a.g2 = (uint16_t*)(b->ws + L.off_g2);
    a.dblock = (const uint16_t*)(b->ws + L.off_dblock);
    a.dblock8 = (const uint8_t*)(b->ws + L.off_dblock8);
    a.dummy = (uint32_t*)(b->ws + L.off_dummy);
    a.n_maps = b->n;
    a.dmax = b->dmax;
    a.D = b->dmax * b->dmax;
    a.lrun = t.lrun;
    a.chunk = t.chunk;
    a.schedule = t.schedule;
    a.itemmap = (const int32_t*)(b->ws + L.off_itemmap);
    a.icap = L.icap;
    // item offsets and the item -> map table depend on the run length only:
    // rebuilt when it changes; the dynamic schedule's grab counters start at
    // zero on every run
    if (t.lrun != b->last_lrun) {
        hipLaunchKernelGGL(k_batch_prefix, dim3(1), dim3(1024), 0, st, a.maps, b->n, t.lrun,
                           (int32_t*)a.pref);
        hipLaunchKernelGGL(k_batch_itemmap, dim3(b->n), dim3(256), 0, st, a.pref, b->n,
                           (int32_t*)a.itemmap, a.icap);
        b->last_lrun = t.lrun;
    }
    if (t.schedule == 0)
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, (uint32_t*)a.queues,
                           (int64_t)3 * (b->n + 1), 0u);
    if (hipGetLastError() != hipSuccess) return EDT_ERR_HIP;
    switch (b->M) {
        case 1: return launch_batch<1>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 2: return launch_batch<2>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 3: return launch_batch<3>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 4: return launch_batch<4>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 5: return launch_batch<5>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 6: return launch_batch<6>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 7: return launch_batch<7>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        case 8: return launch_batch<8>(b, a, mode, t.waves_per_cu, t.wg_waves, st);
        default: return EDT_ERR_ARG;
    }
}

}  // extern "C"
