// edt_kernels.hip -- HIP kernels of the exact truncated EDT for gfx950.
//
// Global transform (the field of Eq. 1, section III, limited to d_max):
//   ingest          dense grid or leaf-block list -> occupancy bits + hash
//   dilate (x,y,z)  region = obstacle blocks grown by R blocks (separable)
//   items (y,z)     runs of consecutive region blocks, at most LRUN long
//   pass_x          1-D distance along x from the occupancy bits
//   pass_y          g2(y) = min_j dist(y+j)^2 + j^2        (lower envelope)
//   pass_z          s(z)  = min(D, min_k g2(z+k) + k^2)    (lower envelope)
// The squared Euclidean distance splits into per-axis terms, so the three
// passes give exactly Eq. 1; terms with an axis offset beyond d_max exceed D
// and never change the clamped result.  The envelope passes follow the lower
// envelope of parabolas (Felzenszwalb & Huttenlocher, cited by the paper as
// the global transform), streamed with one lane per row and a ring of the
// envelope sites that can still reach the next outputs.
//
// Incremental transform (Algorithm 1's raise and lower waves, at block
// granularity): changed voxels are the wave centres; a block is on the lower
// front if some added voxel is closer to the block than its largest value,
// and on the raise front if some removed voxel is no farther than its largest
// value (only such blocks can change); the dist/g2 intermediates are kept
// current for every block and the marked blocks are recomputed exactly.
#include "edt_dev.h"

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

// counters: reset all but the error word (global transform start)
__global__ void k_reset_counters(Grid g) {
    int i = threadIdx.x;
    if (i < C_N && i != C_ERR) g.cnt[i] = 0;
}

__global__ void k_snapshot(Grid g, int dst) { g.cnt[dst] = g.cnt[C_NBLK]; }

// Allocate a pool slot for a key just placed at table position h.
__device__ inline int32_t claim_slot(const Grid& g, int32_t h, unsigned long long key,
                                     uint32_t flags) {
    int32_t slot = atomicAdd(&g.cnt[C_NBLK], 1);
    if (slot >= g.max_blocks) {
        g.hvals[h] = -1;
        set_error(g, -3 /* EDT_ERR_CAPACITY */);
        g.cnt[C_ABORT] = 1;
        return -1;
    }
    g.bkey[slot] = key;
    g.flags[slot] = flags;
    g.hvals[h] = slot;
    return slot;
}

// ---------------------------------------------------------------------------
// ingest
// ---------------------------------------------------------------------------
// Dense grid.  One wave per strip of 8 blocks along x; lane = row (y + 8z).
// Each lane reads 64 contiguous bytes of its row, packs 8 bits per block and
// the wave ballot decides whether a block holds any obstacle.
__global__ void __launch_bounds__(64) k_ingest_dense(Grid g, const uint8_t* __restrict__ occ) {
    const int lane = threadIdx.x;
    const int bx0 = blockIdx.x * 8, by = blockIdx.y, bz = blockIdx.z;
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
    uint8_t* occ8 = (uint8_t*)g.occ;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int bx = bx0 + j;
        if (bx >= g.nbx) break;
        unsigned long long m = __ballot(bytes[j] != 0);
        if (m == 0) continue;
        int32_t slot = -1;
        if (lane == 0) {
            unsigned long long key = pack_key(bx, by, bz);
            bool created;
            int32_t h = hinsert(g.hkeys, g.hmask, key, &created);
            if (h < 0) {
                set_error(g, -3);
            } else if (created) {
                slot = claim_slot(g, h, key, F_DILATED);
                if (slot >= 0) atomicAdd(&g.cnt[C_NDIL], 1);
            }
        }
        slot = __shfl(slot, 0);
        if (slot >= 0) occ8[(int64_t)slot * 64 + lane] = (uint8_t)bytes[j];
    }
}

// Block list, phase 1: insert every block holding an obstacle.
// One wave per input block; lane = row (y + 8z) reads its 8 bytes.
__device__ inline uint32_t block_row_bits(const Grid& g, const int32_t* xyz,
                                          const uint8_t* data, int64_t i, int lane,
                                          int& bx, int& by, int& bz, bool& in_range) {
    bx = xyz[3 * i];
    by = xyz[3 * i + 1];
    bz = xyz[3 * i + 2];
    in_range = bx >= 0 && by >= 0 && bz >= 0 && bx < g.nbx && by < g.nby && bz < g.nbz;
    const uint2 v = *(const uint2*)(data + i * 512 + 8 * lane);
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b |= (((v.x >> (8 * k)) & 0xff) != 0) << k;
        b |= (((v.y >> (8 * k)) & 0xff) != 0) << (k + 4);
    }
    // voxels beyond the extent are not part of the map
    const int y = 8 * by + (lane & 7), z = 8 * bz + (lane >> 3);
    if (y >= g.ny || z >= g.nz) b = 0;
    const int xr = g.nx - 8 * bx;
    if (xr < 8) b &= (xr <= 0) ? 0u : ((1u << xr) - 1u);
    return b;
}

__global__ void __launch_bounds__(64) k_ingest_blocks_insert(Grid g, const int32_t* xyz,
                                                             const uint8_t* data, int64_t n) {
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        int bx, by, bz;
        bool ok;
        uint32_t b = block_row_bits(g, xyz, data, i, lane, bx, by, bz, ok);
        if (!ok) {
            if (lane == 0) set_error(g, -2 /* EDT_ERR_RANGE */);
            continue;
        }
        if (__ballot(b != 0) == 0) continue;
        if (lane == 0) {
            unsigned long long key = pack_key(bx, by, bz);
            bool created;
            int32_t h = hinsert(g.hkeys, g.hmask, key, &created);
            if (h < 0) {
                set_error(g, -3);
            } else if (created) {
                if (claim_slot(g, h, key, F_DILATED) >= 0) atomicAdd(&g.cnt[C_NDIL], 1);
            }
        }
    }
}

// phase 2 (after zeroing the occupancy of the new slots): OR the bits in.
__global__ void __launch_bounds__(64) k_ingest_blocks_write(Grid g, const int32_t* xyz,
                                                            const uint8_t* data, int64_t n) {
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        int bx, by, bz;
        bool ok;
        uint32_t b = block_row_bits(g, xyz, data, i, lane, bx, by, bz, ok);
        if (!ok || b == 0) continue;
        int32_t slot = find_block(g, bx, by, bz);
        if (slot < 0) continue;
        atomicOr(&g.occ[(int64_t)slot * 16 + (lane >> 2)], b << (8 * (lane & 3)));
    }
}

// zero the occupancy words of slots [first, NBLK) and the update-change
// masks of all slots
__global__ void k_zero_occ(Grid g, int first_counter) {
    const int64_t first = first_counter < 0 ? 0 : g.cnt[first_counter];
    const int64_t n = g.cnt[C_NBLK];
    const int64_t lim = (n < g.max_blocks ? n : g.max_blocks);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < lim * 16;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i >= first * 16) g.occ[i] = 0u;
        g.chg_add[i] = 0u;
        g.chg_rem[i] = 0u;
    }
}

// ---------------------------------------------------------------------------
// region growth: every slot < snapshot inserts its +-R neighbours on `axis`
// ---------------------------------------------------------------------------
__global__ void k_dilate_axis(Grid g, int axis) {
    const int R = g.R;
    const int64_t n0 = g.cnt[C_SNAP];
    const int64_t n = n0 < g.max_blocks ? n0 : g.max_blocks;
    const int64_t total = n * 2 * R;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int slot = (int)(i / (2 * R));
        const int k = (int)(i % (2 * R));
        const int off = k < R ? -(k + 1) : (k - R + 1);
        int c[3];
        unpack_key(g.bkey[slot], c[0], c[1], c[2]);
        c[axis] += off;
        const int lim = axis == 0 ? g.nbx : (axis == 1 ? g.nby : g.nbz);
        if (c[axis] < 0 || c[axis] >= lim) continue;
        unsigned long long key = pack_key(c[0], c[1], c[2]);
        bool created;
        int32_t h = hinsert(g.hkeys, g.hmask, key, &created);
        if (h < 0) {
            set_error(g, -3);
            continue;
        }
        if (created) claim_slot(g, h, key, 0u);
    }
}

// ---------------------------------------------------------------------------
// work items: run starts along `axis` (1 = y, 2 = z)
// ---------------------------------------------------------------------------
__device__ inline bool run_member(const Grid& g, int32_t slot, uint32_t runflag) {
    return slot >= 0 && (runflag == 0u || (g.flags[slot] & runflag));
}

__global__ void k_items(Grid g, const int32_t* src, int src_counter, uint32_t runflag,
                        int axis, int32_t* out, int out_counter) {
    const int64_t n = src ? g.cnt[src_counter] : g.cnt[C_NBLK];
    const int64_t lim = n < g.max_blocks ? n : g.max_blocks;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < lim;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t slot = src ? src[i] : (int32_t)i;
        int c[3];
        unpack_key(g.bkey[slot], c[0], c[1], c[2]);
        bool start = (c[axis] % LRUN) == 0;
        if (!start) {
            c[axis] -= 1;
            start = !run_member(g, find_block(g, c[0], c[1], c[2]), runflag);
        }
        int idx = wave_append(start, &g.cnt[out_counter]);
        if (start) out[idx] = slot;
    }
}

// ---------------------------------------------------------------------------
// pass X: 1-D distance along x from the bits.  One wave per block,
// lane = row (y + 8z).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_pass_x(Grid g, const int32_t* list, int list_counter) {
    __shared__ int32_t nb[72];
    const int lane = threadIdx.x;
    const int64_t n0 = list ? g.cnt[list_counter] : g.cnt[C_NBLK];
    const int64_t n = n0 < g.max_blocks ? n0 : g.max_blocks;
    const int R = g.R;
    const uint8_t* occ8 = (const uint8_t*)g.occ;
    for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
        const int32_t slot = list ? list[w] : (int32_t)w;
        int bx, by, bz;
        unpack_key(g.bkey[slot], bx, by, bz);
        for (int i = lane; i < 2 * R + 1; i += 64)
            nb[i] = (i == R) ? slot : find_block(g, bx - R + i, by, bz);
        __syncthreads();
        const uint32_t c = occ8[(int64_t)slot * 64 + lane];
        int prev = -100000, next = 100000;
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
        int dl[8];
        int p = prev;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            if ((c >> x) & 1u) p = x;
            dl[x] = x - p;
        }
        unsigned long long packed = 0;
        int q = next;
#pragma unroll
        for (int x = 7; x >= 0; --x) {
            if ((c >> x) & 1u) q = x;
            int d = min(min(dl[x], q - x), 255);
            packed |= (unsigned long long)d << (8 * x);
        }
        const int y = lane & 7, z = lane >> 3;
        *(unsigned long long*)(g.dist + (int64_t)slot * 512 + 8 * z + 64 * y) = packed;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// streaming lower envelope of parabolas, one row per lane
// ---------------------------------------------------------------------------
// Sites are pushed in increasing position q with value f < D; outputs are
// evaluated at i = q - dmax once every site that can reach i is in.  The
// envelope is kept only on [next output, inf): the bottom site is removed
// when the new site is no worse at the next output; sites more than dmax left
// of the output give values > D and are dropped.  The live sites then lie in
// a window of 2*dmax + 2 positions, which bounds the ring.
struct Envelope {
    uint32_t* ring;   // LDS, element e of this lane at ring[e * 64 + lane]
    int cap;          // ring capacity (entries)
    int lane;
    int n;            // live entries
    int bp, tp;       // physical bottom / top index
    int pt, kt;       // top site position and key f + p^2

    __device__ void init(uint32_t* r, int c, int l) {
        ring = r; cap = c; lane = l; n = 0; bp = 0; tp = c - 1; pt = 0; kt = 0;
    }
    __device__ uint32_t at(int phys) const { return ring[phys * 64 + lane]; }

    __device__ void push(int q, int f, int inext) {
        const int kq = f + q * q;
        while (n > 0) {
            if (n == 1) {
                // bottom: the new site is no worse on [inext, inf)
                if (kq - kt <= 2 * inext * (q - pt)) {
                    n = 0;
                    tp = bp == 0 ? cap - 1 : bp - 1;
                }
                break;
            }
            const int below = tp == 0 ? cap - 1 : tp - 1;
            const uint32_t e = at(below);
            const int p0 = (int)(e >> 16), f0 = (int)(e & 0xffffu);
            const int k0 = f0 + p0 * p0;
            // top is hidden when the new site meets `below` no later than top does
            if ((kq - k0) * (pt - p0) <= (kt - k0) * (q - p0)) {
                --n;
                tp = below;
                pt = p0;
                kt = k0;
            } else {
                break;
            }
        }
        tp = tp + 1 == cap ? 0 : tp + 1;
        ring[tp * 64 + lane] = ((uint32_t)q << 16) | (uint32_t)f;
        ++n;
        pt = q;
        kt = kq;
    }

    // min over live sites of f + (i - p)^2, clamped to D
    __device__ int eval(int i, int dmax, int D) {
        while (n > 0) {
            const uint32_t e = at(bp);
            if ((int)(e >> 16) >= i - dmax) break;
            bp = bp + 1 == cap ? 0 : bp + 1;
            --n;
        }
        if (n == 0) return D;
        uint32_t e = at(bp);
        int pb = (int)(e >> 16);
        int vb = (int)(e & 0xffffu) + (i - pb) * (i - pb);
        while (n > 1) {
            const int nx = bp + 1 == cap ? 0 : bp + 1;
            const uint32_t e1 = at(nx);
            const int p1 = (int)(e1 >> 16);
            const int v1 = (int)(e1 & 0xffffu) + (i - p1) * (i - p1);
            if (v1 > vb) break;
            bp = nx;
            --n;
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
    const int nl = LRUN + 2 * R;
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
    while (len < LRUN && ((start + len) % LRUN) != 0 && mem[R + len]) ++len;
    ha = 0;
    while (ha < R && sl[R + len + ha] >= 0) ++ha;
}

// pass Y: lane = (x, z) with lane = x + 8z; reads dist (layout x+8z+64y),
// writes g2 (layout x+8y+64z).
__global__ void __launch_bounds__(64) k_pass_y(Grid g, const int32_t* items, int item_counter,
                                               uint32_t runflag, int cap) {
    extern __shared__ uint32_t smem[];
    int32_t* sl = (int32_t*)smem;                 // 96 entries
    uint8_t* mem = (uint8_t*)(smem + 96);         // 96 bytes
    uint32_t* ring = smem + 96 + 24;
    const int lane = threadIdx.x;
    const int64_t nit = g.cnt[item_counter];
    const int dmax = g.dmax, D = g.D, R = g.R;
    const int x = lane & 7, z = lane >> 3;
    for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
        const int32_t s0 = items[it];
        int bx, by, bz;
        unpack_key(g.bkey[s0], bx, by, bz);
        int hb, len, ha;
        resolve_run(g, sl, mem, bx, by, bz, 1, runflag, hb, len, ha);
        const int base = R - hb;
        const int o0 = 8 * hb, o1 = 8 * (hb + len), nq = 8 * (hb + len + ha);
        const int qa = max(0, o0 - dmax), qb = min(nq, o1 + dmax);
        Envelope env;
        env.init(ring, cap, lane);
        for (int q = qa; q < o1 + dmax; ++q) {
            if (q < qb) {
                const int32_t slot = sl[base + (q >> 3)];
                const int d = g.dist[(int64_t)slot * 512 + lane + 64 * (q & 7)];
                if (d < dmax) env.push(q, d * d, max(o0, q - dmax));
            }
            const int i = q - dmax;
            if (i >= o0) {
                const int v = env.eval(i, dmax, D);
                const int32_t slot = sl[base + (i >> 3)];
                g.g2[(int64_t)slot * 512 + x + 8 * (i & 7) + 64 * z] = (uint16_t)v;
            }
        }
        __syncthreads();
    }
}

// pass Z: lane = (x, y) with lane = x + 8y; reads g2, writes s and bmax.
__global__ void __launch_bounds__(64) k_pass_z(Grid g, const int32_t* items, int item_counter,
                                               uint32_t runflag, int cap) {
    extern __shared__ uint32_t smem[];
    int32_t* sl = (int32_t*)smem;
    uint8_t* mem = (uint8_t*)(smem + 96);
    uint32_t* ring = smem + 96 + 24;
    const int lane = threadIdx.x;
    const int64_t nit = g.cnt[item_counter];
    const int dmax = g.dmax, D = g.D, R = g.R;
    for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
        const int32_t s0 = items[it];
        int bx, by, bz;
        unpack_key(g.bkey[s0], bx, by, bz);
        int hb, len, ha;
        resolve_run(g, sl, mem, bx, by, bz, 2, runflag, hb, len, ha);
        const int base = R - hb;
        const int o0 = 8 * hb, o1 = 8 * (hb + len), nq = 8 * (hb + len + ha);
        const int qa = max(0, o0 - dmax), qb = min(nq, o1 + dmax);
        Envelope env;
        env.init(ring, cap, lane);
        int bm = 0;
        for (int q = qa; q < o1 + dmax; ++q) {
            if (q < qb) {
                const int32_t slot = sl[base + (q >> 3)];
                const int f = g.g2[(int64_t)slot * 512 + lane + 64 * (q & 7)];
                if (f < D) env.push(q, f, max(o0, q - dmax));
            }
            const int i = q - dmax;
            if (i >= o0) {
                const int v = env.eval(i, dmax, D);
                const int32_t slot = sl[base + (i >> 3)];
                g.s[(int64_t)slot * 512 + lane + 64 * (i & 7)] = v;
                bm = max(bm, v);
                if ((i & 7) == 7) {
                    const int m = wave_max(bm);
                    if (lane == 0) g.bmax[slot] = m;
                    bm = 0;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// readback and query
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_read_dense(Grid g, int32_t* __restrict__ out) {
    const int lane = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    const int32_t slot = find_block(g, bx, by, bz);
    const int y = 8 * by + (lane & 7), z = 8 * bz + (lane >> 3);
    if (y >= g.ny || z >= g.nz) return;
    int32_t* row = out + ((int64_t)z * g.ny + y) * (int64_t)g.nx + 8 * bx;
    const int nxr = min(8, g.nx - 8 * bx);
    if (slot < 0) {
        for (int k = 0; k < nxr; ++k) row[k] = g.D;
        return;
    }
    const int32_t* src = g.s + (int64_t)slot * 512 + 8 * lane;
    for (int k = 0; k < nxr; ++k) row[k] = src[k];
}

__global__ void __launch_bounds__(64) k_read_occ(Grid g, uint8_t* __restrict__ out) {
    const int lane = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    const int32_t slot = find_block(g, bx, by, bz);
    const int y = 8 * by + (lane & 7), z = 8 * bz + (lane >> 3);
    if (y >= g.ny || z >= g.nz) return;
    uint8_t* row = out + ((int64_t)z * g.ny + y) * (int64_t)g.nx + 8 * bx;
    const int nxr = min(8, g.nx - 8 * bx);
    const uint32_t b = slot < 0 ? 0u : ((const uint8_t*)g.occ)[(int64_t)slot * 64 + lane];
    for (int k = 0; k < nxr; ++k) row[k] = (b >> k) & 1u;
}

__global__ void k_query(Grid g, const int32_t* __restrict__ xyz, int64_t n, int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int32_t v = g.D;
        if (x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz) {
            const int32_t slot = find_block(g, x >> 3, y >> 3, z >> 3);
            if (slot >= 0) v = g.s[(int64_t)slot * 512 + (x & 7) + 8 * (y & 7) + 64 * (z & 7)];
        }
        out[i] = v;
    }
}

// ---------------------------------------------------------------------------
// incremental update
// ---------------------------------------------------------------------------
__global__ void k_upd_begin(Grid g) {
    const int i = threadIdx.x;
    if (i == 0) g.cnt[C_SNAP] = g.cnt[C_NBLK];
    if (i == C_ABORT || (i >= C_NYI && i < C_N)) g.cnt[i] = 0;
}

// Range check (any entry outside the extent cancels the whole call) and
// last-entry-wins dedupe through a voxel-keyed hash (value = max entry index).
__global__ void k_upd_dedupe(Grid g, const int32_t* __restrict__ xyz, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        g.upos[i] = -1;
        if (x < 0 || y < 0 || z < 0 || x >= g.nx || y >= g.ny || z >= g.nz) {
            set_error(g, -2);
            g.cnt[C_ABORT] = 1;
            continue;
        }
        const unsigned long long key = (unsigned long long)x +
            (unsigned long long)g.nx * ((unsigned long long)y + (unsigned long long)g.ny * z);
        bool created;
        const int32_t h = hinsert(g.ukeys, g.umask, key, &created);
        if (h < 0) {
            set_error(g, -3);
            g.cnt[C_ABORT] = 1;
            continue;
        }
        g.upos[i] = h;
        atomicMax(&g.uvals[h], (int32_t)i);
    }
}

__device__ inline bool upd_winner(const Grid& g, int64_t i) {
    const int32_t h = g.upos[i];
    return h >= 0 && g.uvals[h] == (int32_t)i;
}

// New blocks for voxels that become occupied.
__global__ void k_upd_alloc(Grid g, const int32_t* __restrict__ xyz,
                            const uint8_t* __restrict__ state, int64_t n) {
    if (g.cnt[C_ABORT]) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!state[i] || !upd_winner(g, i)) continue;
        const int bx = xyz[3 * i] >> 3, by = xyz[3 * i + 1] >> 3, bz = xyz[3 * i + 2] >> 3;
        const unsigned long long key = pack_key(bx, by, bz);
        bool created;
        const int32_t h = hinsert(g.hkeys, g.hmask, key, &created);
        if (h < 0) {
            set_error(g, -3);
            g.cnt[C_ABORT] = 1;
        } else if (created) {
            claim_slot(g, h, key, 0u);
        }
    }
}

// Fresh slots [cnt[first], NBLK): empty block with background values.
__global__ void __launch_bounds__(64) k_init_new(Grid g, int first_counter) {
    const int64_t first = g.cnt[first_counter];
    const int64_t n0 = g.cnt[C_NBLK];
    const int64_t n = n0 < g.max_blocks ? n0 : g.max_blocks;
    const int lane = threadIdx.x;
    for (int64_t s = first + blockIdx.x; s < n; s += gridDim.x) {
        if (lane < 16) {
            g.occ[s * 16 + lane] = 0u;
            g.chg_add[s * 16 + lane] = 0u;
            g.chg_rem[s * 16 + lane] = 0u;
        }
        ((unsigned long long*)(g.dist + s * 512))[lane] = ~0ull;
        const uint32_t d2 = (uint32_t)g.D | ((uint32_t)g.D << 16);
        for (int k = lane; k < 256; k += 64) ((uint32_t*)(g.g2 + s * 512))[k] = d2;
        for (int k = lane; k < 512; k += 64) g.s[s * 512 + k] = g.D;
        if (lane == 0) g.bmax[s] = g.D;
    }
}

// Apply the winning entries: flip occupancy bits, record the changed voxels
// per block (the wave centres) and list the blocks that hold them.
__global__ void k_upd_apply(Grid g, const int32_t* __restrict__ xyz,
                            const uint8_t* __restrict__ state, int64_t n) {
    if (g.cnt[C_ABORT]) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool add = false, rem = false, first_seed = false, new_dil = false;
        int32_t slot = -1;
        if (upd_winner(g, i)) {
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
        int j = wave_append(first_seed, &g.cnt[C_NSEED]);
        if (first_seed) g.list_seed[j] = slot;
        j = wave_append(new_dil, &g.cnt[C_NNEWDIL]);
        if (new_dil) {
            g.list_newdil[j] = slot;
            atomicAdd(&g.cnt[C_NDIL], 1);
        }
    }
}

// Blocks that just became obstacle blocks bring their R-neighbourhood in.
__global__ void k_upd_dilate(Grid g) {
    const int R = g.R, w = 2 * R + 1, w3 = w * w * w;
    const int64_t total = (int64_t)g.cnt[C_NNEWDIL] * w3;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t slot = g.list_newdil[i / w3];
        const int o = (int)(i % w3);
        int bx, by, bz;
        unpack_key(g.bkey[slot], bx, by, bz);
        bx += o % w - R;
        by += (o / w) % w - R;
        bz += o / (w * w) - R;
        if (bx < 0 || by < 0 || bz < 0 || bx >= g.nbx || by >= g.nby || bz >= g.nbz) continue;
        const unsigned long long key = pack_key(bx, by, bz);
        bool created;
        const int32_t h = hinsert(g.hkeys, g.hmask, key, &created);
        if (h < 0) {
            set_error(g, -3);
        } else if (created) {
            claim_slot(g, h, key, 0u);
        }
    }
}

// Bounding boxes (block-local) of the added and removed voxels of each seed.
// Packed as xmin | xmax<<4 | ymin<<8 | ymax<<12 | zmin<<16 | zmax<<20 | 1<<24.
__device__ inline int32_t row_box(uint32_t byte, int lane) {
    int xmn = 8, xmx = -1, ymn = 8, ymx = -1, zmn = 8, zmx = -1;
    if (byte) {
        xmn = __ffs(byte) - 1;
        xmx = 31 - __clz(byte);
        ymn = ymx = lane & 7;
        zmn = zmx = lane >> 3;
    }
    xmn = wave_min(xmn); ymn = wave_min(ymn); zmn = wave_min(zmn);
    xmx = wave_max(xmx); ymx = wave_max(ymx); zmx = wave_max(zmx);
    if (xmx < 0) return 0;
    return xmn | (xmx << 4) | (ymn << 8) | (ymx << 12) | (zmn << 16) | (zmx << 20) | (1 << 24);
}

__global__ void __launch_bounds__(64) k_seed_box(Grid g) {
    const int64_t n = g.cnt[C_NSEED];
    const int lane = threadIdx.x;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        const int32_t slot = g.list_seed[s];
        const uint32_t a = ((const uint8_t*)g.chg_add)[(int64_t)slot * 64 + lane];
        const uint32_t r = ((const uint8_t*)g.chg_rem)[(int64_t)slot * 64 + lane];
        const int32_t ba = row_box(a, lane);
        const int32_t br = row_box(r, lane);
        if (lane == 0) {
            g.seed_box[2 * s] = ba;
            g.seed_box[2 * s + 1] = br;
        }
    }
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

// Raise / lower fronts around every seed and the dist/g2 recompute sets.
//   lower: some added voxel a has |box(B) - a|^2 < bmax(B)   (a value can drop)
//   raise: some removed voxel r has |box(B) - r|^2 <= bmax(B) and < D
//   xs:    blocks within R along x of a seed (their dist can change)
//   ys:    blocks within R in x and y of a seed (their g2 can change)
__global__ void k_upd_mark(Grid g) {
    const int R = g.R, w = 2 * R + 1, w3 = w * w * w;
    const int64_t total = (int64_t)g.cnt[C_NSEED] * w3;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t si = i / w3;
        const int o = (int)(i % w3);
        const int32_t seed = g.list_seed[si];
        int sx, sy, sz;
        unpack_key(g.bkey[seed], sx, sy, sz);
        const int ox = o % w - R, oy = (o / w) % w - R, oz = o / (w * w) - R;
        const int bx = sx + ox, by = sy + oy, bz = sz + oz;
        int32_t slot = find_block(g, bx, by, bz);
        bool new_dirty = false, new_xs = false, new_ys = false, raise = false, lower = false;
        if (slot >= 0) {
            const int32_t pa = g.seed_box[2 * si], pr = g.seed_box[2 * si + 1];
            const int bm = g.bmax[slot];
            lower = pa != 0 && box_dist2(pa, sx, sy, sz, bx, by, bz) < bm;
            if (pr != 0) {
                const int d2 = box_dist2(pr, sx, sy, sz, bx, by, bz);
                raise = d2 <= bm && d2 < g.D;
            }
            uint32_t want = 0;
            if (lower) want |= F_LOWER | F_DIRTY;
            if (raise) want |= F_RAISE | F_DIRTY;
            if (oz == 0) want |= F_YS;
            if (oz == 0 && oy == 0) want |= F_XS;
            if (want) {
                const uint32_t old = atomicOr(&g.flags[slot], want);
                new_dirty = (want & F_DIRTY) && !(old & F_DIRTY);
                new_ys = (want & F_YS) && !(old & F_YS);
                new_xs = (want & F_XS) && !(old & F_XS);
                raise = raise && !(old & F_RAISE);
                lower = lower && !(old & F_LOWER);
            }
        }
        int j = wave_append(new_dirty, &g.cnt[C_NDIRTY]);
        if (new_dirty) g.list_dirty[j] = slot;
        j = wave_append(new_ys, &g.cnt[C_NYS]);
        if (new_ys) g.list_ys[j] = slot;
        j = wave_append(new_xs, &g.cnt[C_NXS]);
        if (new_xs) g.list_xs[j] = slot;
        const unsigned long long mr = __ballot(raise), ml = __ballot(lower);
        if (__lane_id() == (int)(__ffsll((long long)(mr | ml | 1ull)) - 1) && (mr | ml)) {
            atomicAdd(&g.cnt[C_NRAISE], __popcll(mr));
            atomicAdd(&g.cnt[C_NLOWER], __popcll(ml));
        }
    }
}

// Clear per-update state: dedupe table entries, change masks and flags.
__global__ void k_upd_cleanup(Grid g, int64_t n) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += stride) {
        const int32_t h = g.upos[i];
        if (h >= 0) {
            g.ukeys[h] = KEY_EMPTY;
            g.uvals[h] = -1;
        }
    }
    const int64_t ns = g.cnt[C_NSEED];
    for (int64_t i = tid; i < ns * 16; i += stride) {
        const int32_t slot = g.list_seed[i / 16];
        g.chg_add[(int64_t)slot * 16 + (i % 16)] = 0u;
        g.chg_rem[(int64_t)slot * 16 + (i % 16)] = 0u;
    }
    const uint32_t clear = ~(F_SEED | F_DIRTY | F_XS | F_YS | F_RAISE | F_LOWER);
    for (int64_t i = tid; i < ns; i += stride) atomicAnd(&g.flags[g.list_seed[i]], clear);
    const int64_t nd = g.cnt[C_NDIRTY];
    for (int64_t i = tid; i < nd; i += stride) atomicAnd(&g.flags[g.list_dirty[i]], clear);
    const int64_t ny = g.cnt[C_NYS];
    for (int64_t i = tid; i < ny; i += stride) atomicAnd(&g.flags[g.list_ys[i]], clear);
}

__global__ void k_clear_error(Grid g) { g.cnt[C_ERR] = 0; }

}  // namespace edt
