// edt_dense.hip -- uncapped (or arbitrarily capped) exact squared EDT of a
// dense grid: the full distance transform, d_max = infinity, with which the
// paper runs its dataset benchmarks (section V-B), and radii beyond the
// 16-bit storage of the sparse field.
//
// s(x) = min over occupied y of |x - y|^2 (Eq. 1 without the limit), then
// min(D, s) when a radius is given; voxels of a grid without any obstacle get
// EDT_DENSE_INF.  Values are int32: the extent must satisfy
// nx^2 + ny^2 + nz^2 < 2^31, so every squared distance fits.
//
// Three passes over the caller's int32 output array, in place:
//   x   one wave per row, 64 voxels per step: a ballot of the occupancy
//       bytes gives, per lane, the nearest obstacle at or left of it (and in
//       a second sweep at or right of it), carried across steps;
//   y,z one lane per column (64 consecutive x per wave, coalesced rows): the
//       lower envelope of the parabolas q -> f(v) + (q - v)^2 of the column's
//       finite values (Felzenszwalb and Huttenlocher's separable transform,
//       the one the paper cites in section I), built left to right with
//       parabola intersections compared exactly as int64 cross products,
//       then read off left to right.  The envelope of every column lives in
//       the workspace (one int2 (v, f) per voxel), entry k of column c at
//       k * ncols + c.
//
// The dense context (edt_dense_ctx_*) keeps the occupancy and both
// intermediates (g1 after x, g2 after y) beside the field, so a change list
// is applied incrementally and exactly: the rows holding a changed voxel are
// recomputed by pass x; a y column is recomputed when some g1 value in it
// changed, a z column when some g2 value in it changed.  Columns are handled
// in groups of 64 consecutive x (one wave), marked by the pass before
// (a flag per group and a list of the marked groups), so every recomputed
// column is an exact pass over its whole length and the field equals the
// global transform of the new occupancy.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "edt.h"
#include "edt_dev.h"

// Scratch of the allocation-free entry point (edt_dense_global_noalloc): the
// column envelopes of grids up to EDT_DENSE_STATIC_BYTES / 8 voxels.  Each
// device holds its own copy for the life of the process.  Host code never
// passes this name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returned on
// that device (scratch_address below).  Nothing in it has to start at zero:
// every envelope entry is written before it is read.
static __device__ __align__(256) unsigned char scratch[EDT_DENSE_STATIC_BYTES];

namespace edt {

constexpr int32_t DINF = 0x7fffffff;

// Pass x.  One wave per row; the row is taken 1024 voxels at a time, 16
// consecutive voxels per lane (one 16-byte load).  The nearest obstacle at
// or before each voxel comes from the lane's own bits and an exclusive max
// scan of the lanes' last obstacle positions (carried across chunks); the
// nearest at or after it from a min scan the other way.  Rows longer than
// 1024 keep the left distances in out between the two sweeps.
__device__ inline uint32_t byte_bits(const uint4& w) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
    uint32_t m = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) m |= (((v[i] >> (8 * k)) & 0xffu) != 0u ? 1u : 0u) << (4 * i + k);
    return m;
}

__device__ inline uint32_t chunk_bits(const uint8_t* row, int x0, int nx, int lane) {
    const int x = x0 + 16 * lane;
    if (x + 16 <= nx && ((uintptr_t)(row + x) & 15) == 0) return byte_bits(*(const uint4*)(row + x));
    uint32_t m = 0u;
    for (int k = 0; k < 16; ++k)
        if (x + k < nx && row[x + k]) m |= 1u << k;
    return m;
}

// Marks of an incremental update (dense context).  cnt: [0] error word,
// [1] the current call is cancelled (set by the dedupe, read by the apply
// kernel, cleared by the pass-x kernel), [2] rows listed, [3] y groups listed,
// [4] z groups listed.  A y group is (x / 64, z), a z group (x / 64, y); one
// wave recomputes the group's 64 columns.
struct DenseMarks {
    int32_t* cnt;
    int32_t* rowflag;        // [ny * nz] row listed for pass x
    int32_t* rows;           // listed rows
    int32_t* gy;             // [nxc * nz] y group listed
    int32_t* ly;             // listed y groups
    int32_t* gz;             // [nxc * ny] z group listed
    int32_t* lz;             // listed z groups
    int32_t* tmp;            // left distances of rows longer than 1024 (nx * ny * nz)
};
enum { DC_ERR = 0, DC_CANCEL, DC_NROW, DC_NY, DC_NZ, DC_N };

// Lists entry g of flag array f (list l, counter c) once per update.
__device__ inline void list_once(int32_t* f, int32_t* l, int32_t* c, int64_t g) {
    if (__hip_atomic_load(&f[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    if (atomicExch(&f[g], 1) == 0) l[atomicAdd(c, 1)] = (int32_t)g;
}

// INC: only the listed rows (each row's flag is cleared), the left distances
// of long rows go to the scratch rows instead of out, and every 64-voxel
// group whose g1 changed lists its y group (x / 64, z).
template <bool INC>
__global__ void __launch_bounds__(64) k_dense_x(int nx, int ny, int nz,
                                                const uint8_t* __restrict__ occ, int32_t* out,
                                                DenseMarks mk) {
    constexpr int64_t FAR = 1ll << 40;
    const int lane = threadIdx.x;
    const int nxc = (nx + 63) / 64;
    if (INC && blockIdx.x == 0 && lane == 0) mk.cnt[DC_CANCEL] = 0;   // its last reader is done
    const int64_t rows = INC ? (int64_t)mk.cnt[DC_NROW] : (int64_t)ny * nz;
    for (int64_t ri = blockIdx.x; ri < rows; ri += gridDim.x) {
        const int64_t r = INC ? (int64_t)mk.rows[ri] : ri;
        if (INC && lane == 0) mk.rowflag[r] = 0;
        const uint8_t* row = occ + r * nx;
        int32_t* o = out + r * nx;
        int32_t* lt = (INC ? mk.tmp : out) + r * nx;     // left distances of long rows
        const int z = (int)(r / ny);
        const bool one = nx <= 1024;
        // left sweep
        int64_t carry = -FAR;
        uint32_t keep = 0u;
        for (int x0 = 0; x0 < nx; x0 += 1024) {
            const uint32_t m = chunk_bits(row, x0, nx, lane);
            if (one) keep = m;
            const int64_t mylast = m ? (int64_t)x0 + 16 * lane + 31 - __clz(m) : -FAR;
            int64_t incl = mylast;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int64_t v = __shfl_up(incl, d);
                if (lane >= d && v > incl) incl = v;
            }
            int64_t prev = __shfl_up(incl, 1);
            if (lane == 0) prev = -FAR;
            if (carry > prev) prev = carry;
            if (!one) {
                int64_t near = prev;
                for (int k = 0; k < 16; ++k) {
                    const int x = x0 + 16 * lane + k;
                    if ((m >> k) & 1u) near = x;
                    if (x < nx) lt[x] = x - near > (1 << 30) ? DINF : (int32_t)(x - near);
                }
            }
            const int64_t tot = __shfl(incl, 63);
            if (tot > carry) carry = tot;
            if (one) carry = prev;     // the lane's own carry-in, used below
        }
        // right sweep (and the result)
        int64_t rcarry = FAR;
        const int top = (nx - 1) & ~1023;
        for (int x0 = top; x0 >= 0; x0 -= 1024) {
            const uint32_t m = one ? keep : chunk_bits(row, x0, nx, lane);
            const int64_t myfirst = m ? (int64_t)x0 + 16 * lane + __ffs(m) - 1 : FAR;
            int64_t incl = myfirst;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int64_t v = __shfl_down(incl, d);
                if (lane + d < 64 && v < incl) incl = v;
            }
            int64_t next = __shfl_down(incl, 1);
            if (lane == 63) next = FAR;
            if (rcarry < next) next = rcarry;
            int32_t res[16];
            int64_t nr = next;
#pragma unroll
            for (int k = 15; k >= 0; --k) {
                const int64_t x = x0 + 16 * lane + k;
                if ((m >> k) & 1u) nr = x;
                res[k] = (int32_t)((nr - x) > (1 << 30) ? (1 << 30) + 1 : nr - x);
            }
            int64_t nl = carry;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int64_t x = x0 + 16 * lane + k;
                int64_t dl;
                if (one) {
                    if ((m >> k) & 1u) nl = x;
                    dl = x - nl;
                } else {
                    dl = x < nx ? (int64_t)lt[x] : FAR;
                }
                const int64_t d = (int64_t)res[k] < dl ? (int64_t)res[k] : dl;
                res[k] = d > (1 << 30) ? DINF : (int32_t)(d * d);
            }
            const int xs = x0 + 16 * lane;
            bool changed = false;
            if (xs + 16 <= nx && ((uintptr_t)(o + xs) & 15) == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int4 v = make_int4(res[4 * q], res[4 * q + 1], res[4 * q + 2], res[4 * q + 3]);
                    if (INC) {
                        const int4 w = *(const int4*)(o + xs + 4 * q);
                        changed = changed || w.x != v.x || w.y != v.y || w.z != v.z || w.w != v.w;
                    }
                    *(int4*)(o + xs + 4 * q) = v;
                }
            } else {
                for (int k = 0; k < 16; ++k)
                    if (xs + k < nx) {
                        if (INC) changed = changed || o[xs + k] != res[k];
                        o[xs + k] = res[k];
                    }
            }
            if (INC) {
                // lanes 4g .. 4g + 3 hold the 64 voxels of group x0 / 64 + g
                const unsigned long long cm = __ballot(changed);
                if (lane < 16 && ((cm >> (4 * lane)) & 0xfull) && x0 / 64 + lane < nxc)
                    list_once(mk.gy, mk.ly, &mk.cnt[DC_NY], (int64_t)(x0 / 64 + lane) + (int64_t)nxc * z);
            }
            const int64_t tot = __shfl(incl, 0);
            if (tot < rcarry) rcarry = tot;
        }
    }
}

// Passes y (AXIS 1) and z (AXIS 2) from `in` to `out` (the same array for the
// in-place transform), with the envelope in env.  Column (x, w): x fastest
// within a wave; w = z for y, y for z.  The column is read and written CH
// values at a time.  INC: only the listed groups (each group's flag is
// cleared); pass y lists the z group (x / 64, y) of every y whose g2 changed.
template <int AXIS, int CH, bool INC>
__global__ void __launch_bounds__(64) k_dense_col(int nx, int ny, int nz, const int32_t* in,
                                                  int32_t* out, int2* env, int32_t cap,
                                                  DenseMarks mk) {
    const int lane = threadIdx.x;
    const int n = AXIS == 1 ? ny : nz;                 // column length
    const int nw = AXIS == 1 ? nz : ny;
    const int64_t stride = AXIS == 1 ? (int64_t)nx : (int64_t)nx * ny;
    const int nxc = (nx + 63) / 64;
    const int64_t ncols = (int64_t)nx * nw;
    const int64_t waves = INC ? (int64_t)mk.cnt[AXIS == 1 ? DC_NY : DC_NZ] : (int64_t)nxc * nw;
    for (int64_t wi = blockIdx.x; wi < waves; wi += gridDim.x) {
        const int64_t wv = INC ? (int64_t)(AXIS == 1 ? mk.ly : mk.lz)[wi] : wi;
        if (INC && lane == 0) (AXIS == 1 ? mk.gy : mk.gz)[wv] = 0;
        const int x = (int)(wv % nxc) * 64 + lane;
        const int w = (int)(wv / nxc);
        const bool live = x < nx;
        const int64_t base = AXIS == 1 ? (int64_t)x + (int64_t)nx * ny * w
                                       : (int64_t)x + (int64_t)nx * w;
        const int64_t col = (int64_t)x + (int64_t)nx * w;   // column index among ncols
        int2* E = env + col;                                 // entry k at E[k * ncols]
        // build the lower envelope; (v1, F1) is the top, (v0, F0) the entry
        // below it and (v2, F2) the one below that, held in registers so a
        // pop needs no load (the entry under v2 is fetched at each pop and
        // used only at the next)
        int k = -1;
        if (live) {
            int v0 = 0, v1 = 0, v2 = 0;
            int64_t F0 = 0, F1 = 0, F2 = 0;                  // f + v^2
            // the column is read CH values at a time, the next CH in flight
            // while the current ones are pushed (positions past the end read
            // as DINF)
            const int32_t* src = in + base;
            int32_t buf[CH], nbuf[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) buf[u] = u < n ? src[stride * u] : DINF;
            for (int q0 = 0; q0 < n; q0 += CH) {
#pragma unroll
                for (int u = 0; u < CH; ++u)
                    nbuf[u] = q0 + CH + u < n ? src[stride * (q0 + CH + u)] : DINF;
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int q = q0 + u;
                    const int32_t f = buf[u];
                    if (f == DINF) continue;
                    const int64_t Fq = (int64_t)f + (int64_t)q * q;
                    // pop while the top parabola's interval is empty: the new
                    // one overtakes it no later than the top overtook the one
                    // below
                    while (k >= 1 &&
                           (Fq - F1) * (int64_t)(v1 - v0) <= (F1 - F0) * (int64_t)(q - v1)) {
                        --k;
                        v1 = v0;
                        F1 = F0;
                        v0 = v2;
                        F0 = F2;
                        if (k >= 2) {
                            const int2 e = E[(int64_t)(k - 2) * ncols];
                            v2 = e.x;
                            F2 = (int64_t)e.y + (int64_t)e.x * e.x;
                        }
                    }
                    ++k;
                    E[(int64_t)k * ncols] = make_int2(q, f);
                    v2 = v0;
                    F2 = F0;
                    v0 = v1;
                    F0 = F1;
                    v1 = q;
                    F1 = Fq;
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) buf[u] = nbuf[u];
            }
        }
        // read off: parabola j covers q while the next one is not yet lower;
        // a column without finite values is `cap` everywhere
        int j = 0;
        int2 cur = make_int2(0, 0), nxt = cur, nx2 = cur;
        if (live && k >= 0) {
            cur = E[0];
            nxt = k >= 1 ? E[ncols] : cur;
            nx2 = k >= 2 ? E[2 * ncols] : nxt;               // fetched one entry ahead
        }
        // CH outputs are computed, then stored together
        int32_t* dst = out + base;
        for (int q0 = 0; q0 < n; q0 += CH) {
            int32_t res[CH], old[CH];
            if (INC && live) {
#pragma unroll
                for (int u = 0; u < CH; ++u) old[u] = q0 + u < n ? dst[stride * (q0 + u)] : 0;
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int q = q0 + u;
                // next parabola is at least as low at q:
                // (F_next - F_cur) <= 2 q (v_next - v_cur)
                while (j < k) {
                    const int64_t Fc = (int64_t)cur.y + (int64_t)cur.x * cur.x;
                    const int64_t Fn = (int64_t)nxt.y + (int64_t)nxt.x * nxt.x;
                    if (Fn - Fc > 2ll * q * (int64_t)(nxt.x - cur.x)) break;
                    ++j;
                    cur = nxt;
                    nxt = nx2;
                    if (j + 2 <= k) nx2 = E[(int64_t)(j + 2) * ncols];
                }
                const int64_t d = (int64_t)(q - cur.x) * (q - cur.x) + cur.y;
                res[u] = (k < 0 || d >= (int64_t)cap) ? cap : (int32_t)d;
            }
            if (live) {
                // the global transform's z pass writes the result, which it
                // does not read again: non-temporal (2% on the tunnel extent)
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (q0 + u >= n) continue;
                    if (AXIS == 2 && !INC) __builtin_nontemporal_store(res[u], &dst[stride * (q0 + u)]);
                    else dst[stride * (q0 + u)] = res[u];
                }
            }
            if (INC && AXIS == 1) {
                // y = q0 + u changed in some column of the group: list the z
                // group (x / 64, y)
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const bool ch = live && q0 + u < n && old[u] != res[u];
                    if (__ballot(ch) != 0ull && lane == 0)
                        list_once(mk.gz, mk.lz, &mk.cnt[DC_NZ],
                                  (int64_t)(wv % nxc) + (int64_t)nxc * (q0 + u));
                }
            }
        }
    }
}

// Lower envelope of the finite values in[q] (q = qb .. qe - 1, step `stride`
// from src) of one column, kept as entries (q, f) at E[k * ncols]; returns
// the index of the top entry (-1: none).  The top three entries are held in
// registers so a pop needs no load; the column is read CH values at a time,
// the next CH in flight while the current ones are pushed.
template <int CH>
__device__ inline int build_envelope(const int32_t* src, int64_t stride, int qb, int qe,
                                     int2* E, int64_t ncols) {
    int k = -1;
    int v0 = 0, v1 = 0, v2 = 0;
    int64_t F0 = 0, F1 = 0, F2 = 0;                  // f + v^2
    int32_t buf[CH], nbuf[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) buf[u] = qb + u < qe ? src[stride * (qb + u)] : DINF;
    for (int q0 = qb; q0 < qe; q0 += CH) {
#pragma unroll
        for (int u = 0; u < CH; ++u)
            nbuf[u] = q0 + CH + u < qe ? src[stride * (q0 + CH + u)] : DINF;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int q = q0 + u;
            const int32_t f = buf[u];
            if (f == DINF) continue;
            const int64_t Fq = (int64_t)f + (int64_t)q * q;
            while (k >= 1 && (Fq - F1) * (int64_t)(v1 - v0) <= (F1 - F0) * (int64_t)(q - v1)) {
                --k;
                v1 = v0;
                F1 = F0;
                v0 = v2;
                F0 = F2;
                if (k >= 2) {
                    const int2 e = E[(int64_t)(k - 2) * ncols];
                    v2 = e.x;
                    F2 = (int64_t)e.y + (int64_t)e.x * e.x;
                }
            }
            ++k;
            E[(int64_t)k * ncols] = make_int2(q, f);
            v2 = v0;
            F2 = F0;
            v0 = v1;
            F0 = F1;
            v1 = q;
            F1 = Fq;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) buf[u] = nbuf[u];
    }
    return k;
}

// Read-off state of one envelope: entry j covers q while the next one is not
// yet lower; the entry after next is fetched one step ahead.
struct EnvCursor {
    const int2* E;
    int64_t ncols;
    int k, j;
    int2 cur, nxt, nx2;
    __device__ void init(const int2* e, int64_t nc, int top) {
        E = e;
        ncols = nc;
        k = top;
        j = 0;
        cur = nxt = nx2 = make_int2(0, 0);
        if (k >= 0) {
            cur = E[0];
            nxt = k >= 1 ? E[ncols] : cur;
            nx2 = k >= 2 ? E[2 * ncols] : nxt;
        }
    }
    // the envelope's value at q (rows taken in increasing order); INT64_MAX
    // for an empty envelope
    __device__ int64_t at(int q) {
        if (k < 0) return INT64_MAX;
        while (j < k) {
            const int64_t Fc = (int64_t)cur.y + (int64_t)cur.x * cur.x;
            const int64_t Fn = (int64_t)nxt.y + (int64_t)nxt.x * nxt.x;
            if (Fn - Fc > 2ll * q * (int64_t)(nxt.x - cur.x)) break;
            ++j;
            cur = nxt;
            nxt = nx2;
            if (j + 2 <= k) nx2 = E[(int64_t)(j + 2) * ncols];
        }
        return (int64_t)(q - cur.x) * (q - cur.x) + cur.y;
    }
};

// Pass y of the global dense transform with two lanes per column: lanes
// 0..31 take rows [0, n0) of 32 columns, lanes 32..63 rows [n0, ny) of the
// same columns, and each builds the envelope of its own half.  The envelope
// of all of a column's sites is the pointwise minimum of the envelopes of
// the two halves, so each lane reads its own envelope and its partner's over
// its rows.  Long y columns give few column groups (2,048 at 1024 x 1024 x
// 128, two waves per SIMD); this form has twice as many waves, each with
// half the build and twice the read-off.  No cap (the z pass caps).  `in`
// and `out` may be the same array: every lane of the wave has read its rows
// before any lane writes.
template <int CH>
__global__ void __launch_bounds__(64) k_dense_col_y2(int nx, int ny, int nz,
                                                     const int32_t* in, int32_t* out,
                                                     int2* env) {
    const int lane = threadIdx.x, half = lane >> 5;
    const int n0 = (ny + 1) / 2;
    const int qb = half ? n0 : 0, qe = half ? ny : n0;
    const int64_t stride = nx;
    const int nxc = (nx + 31) / 32;
    const int64_t ncols = (int64_t)nx * nz;
    const int64_t waves = (int64_t)nxc * nz;
    for (int64_t wv = blockIdx.x; wv < waves; wv += gridDim.x) {
        const int x = (int)(wv % nxc) * 32 + (lane & 31);
        const int w = (int)(wv / nxc);
        const bool live = x < nx;
        const int64_t base = (int64_t)x + (int64_t)nx * ny * w;
        const int64_t col = (int64_t)x + (int64_t)nx * w;
        // half h keeps its entries from row h n0 of the column's envelope space
        int2* E = env + col + (int64_t)qb * ncols;
        const int k = live ? build_envelope<CH>(in + base, stride, qb, qe, E, ncols) : -1;
        // the partner's entries were written by this wave: complete them
        // before they are read
        __threadfence_block();
        const int ko = __shfl_xor(k, 32);
        EnvCursor own, oth;
        own.init(E, ncols, k);
        oth.init(env + col + (int64_t)(half ? 0 : n0) * ncols, ncols, ko);
        int32_t* dst = out + base;
        for (int q0 = qb; q0 < qe; q0 += CH) {
            int32_t res[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int q = q0 + u;
                res[u] = DINF;
                if (live && q < qe) {
                    const int64_t d = min(own.at(q), oth.at(q));
                    res[u] = d >= (int64_t)DINF ? DINF : (int32_t)d;
                }
            }
            if (live) {
#pragma unroll
                for (int u = 0; u < CH; ++u)
                    if (q0 + u < qe) dst[stride * (q0 + u)] = res[u];
            }
        }
    }
}

// Incremental update of the dense context, step 1: range check and
// voxel-keyed dedupe (the last entry of a voxel wins), as in the sparse
// update.  ukeys / uvals: open-addressing table of capacity umask + 1.
__global__ void k_dn_dedupe(int nx, int ny, int nz, const int32_t* __restrict__ xyz, int64_t n,
                            unsigned long long* ukeys, int32_t* uvals, uint32_t umask,
                            int32_t* upos, DenseMarks mk) {
    if (blockIdx.x == 0 && threadIdx.x >= DC_NROW && threadIdx.x < DC_N) mk.cnt[threadIdx.x] = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        upos[i] = -1;
        if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) {
            atomicCAS(&mk.cnt[DC_ERR], 0, -2 /* EDT_ERR_RANGE */);
            mk.cnt[DC_CANCEL] = 1;
            continue;
        }
        const unsigned long long key =
            (unsigned long long)x + (unsigned long long)nx * ((unsigned long long)y + (unsigned long long)ny * z);
        bool created;
        const int32_t h = hinsert(ukeys, umask, key, &created);
        if (h < 0) {                    // cannot happen: capacity >= 2 n
            atomicCAS(&mk.cnt[DC_ERR], 0, -3 /* EDT_ERR_CAPACITY */);
            mk.cnt[DC_CANCEL] = 1;
            continue;
        }
        upos[i] = h;
        atomicMax(&uvals[h], (int32_t)i);
    }
}

// Step 2: the winning entries change the occupancy and list their rows; the
// table entries are cleared for the next call (all of them when the call is
// cancelled, which then changes nothing).
__global__ void k_dn_apply(int nx, int ny, const int32_t* __restrict__ xyz,
                           const uint8_t* __restrict__ state, int64_t n, uint8_t* occ,
                           unsigned long long* ukeys, int32_t* uvals, const int32_t* upos,
                           DenseMarks mk) {
    const bool cancel = mk.cnt[DC_CANCEL] != 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t h = upos[i];
        if (h < 0) continue;
        if (cancel) {
            ukeys[h] = KEY_EMPTY;
            uvals[h] = -1;
            continue;
        }
        if (uvals[h] != (int32_t)i) continue;            // a later entry wins
        ukeys[h] = KEY_EMPTY;
        uvals[h] = -1;
        const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        const int64_t v = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
        const uint8_t want = state[i] ? 1 : 0;
        if ((occ[v] != 0) == (want != 0)) continue;
        occ[v] = want;
        list_once(mk.rowflag, mk.rows, &mk.cnt[DC_NROW], (int64_t)y + (int64_t)ny * z);
    }
}

__global__ void k_dn_fill(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace edt

namespace {

inline int grid_of(int64_t work, int cap) {
    return (int)(work < 1 ? 1 : (work > cap ? cap : work));
}

bool dense_ok(int32_t nx, int32_t ny, int32_t nz) {
    if (nx < 1 || ny < 1 || nz < 1) return false;
    const int64_t d2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
    return d2 < (int64_t)edt::DINF;
}

// The three passes of the dense transform on `st`: x into g1, y from g1 into
// g2, z from g2 into s (the same array for the in-place transform),
// envelopes in env.
edt_status launch_dense3(int32_t nx, int32_t ny, int32_t nz, int32_t d_max, const uint8_t* d_occ,
                         int32_t* g1, int32_t* g2, int32_t* s, int2* env, hipStream_t st) {
    using namespace edt;
    const int32_t cap = d_max > 0 ? d_max * d_max : DINF;
    const int nxc = (nx + 63) / 64;
    const DenseMarks none{};
    hipLaunchKernelGGL(k_dense_x<false>, dim3(grid_of((int64_t)ny * nz, 65536)), dim3(64), 0, st,
                       nx, ny, nz, d_occ, g1, none);
    // chunk lengths measured on a 1024x1024x128 extent: 16 for the long y
    // columns, 8 for z (fewer registers, more resident waves)
    const int nxc32 = (nx + 31) / 32;
    hipLaunchKernelGGL((k_dense_col_y2<8>), dim3(grid_of((int64_t)nxc32 * nz, 65536)), dim3(64),
                       0, st, nx, ny, nz, (const int32_t*)g1, g2, env);
    hipLaunchKernelGGL((k_dense_col<2, 8, false>), dim3(grid_of((int64_t)nxc * ny, 65536)),
                       dim3(64), 0, st, nx, ny, nz, (const int32_t*)g2, s, env, cap, none);
    if (hipGetLastError() != hipSuccess) return EDT_ERR_HIP;
    return EDT_OK;
}

// The three passes of the dense transform on `st`, in place on d_out,
// envelopes in env.
edt_status launch_dense(int32_t nx, int32_t ny, int32_t nz, int32_t d_max, const uint8_t* d_occ,
                        int32_t* d_out, int2* env, hipStream_t st) {
    using namespace edt;
    return launch_dense3(nx, ny, nz, d_max, d_occ, d_out, d_out, d_out, env, st);
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices];

edt_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EDT_ERR_HIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EDT_ERR_HIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return EDT_OK;
}

// Regions of a dense context's workspace (256-byte aligned).
struct DenseLayout {
    int64_t occ, g1, g2, s, env, rowflag, rows, gy, ly, gz, lz, cnt, ukeys, uvals, upos, total;
    int64_t ucap;
};

bool dense_layout(int32_t nx, int32_t ny, int32_t nz, int64_t max_changes, DenseLayout* L) {
    if (!dense_ok(nx, ny, nz) || max_changes < 1 || max_changes > (1ll << 28)) return false;
    const int64_t n = (int64_t)nx * ny * nz, nxc = (nx + 63) / 64;
    int64_t ucap = 64;
    while (ucap < 2 * max_changes) ucap <<= 1;
    L->ucap = ucap;
    int64_t o = 0;
    auto take = [&](int64_t bytes) { const int64_t at = o; o += (bytes + 255) & ~(int64_t)255; return at; };
    L->occ = take(n);
    L->g1 = take(4 * n);
    L->g2 = take(4 * n);
    L->s = take(4 * n);
    L->env = take(8 * n);
    L->rowflag = take(4ll * ny * nz);
    L->rows = take(4ll * ny * nz);
    L->gy = take(4 * nxc * nz);
    L->ly = take(4 * nxc * nz);
    L->gz = take(4 * nxc * ny);
    L->lz = take(4 * nxc * ny);
    L->cnt = take(4 * edt::DC_N);
    L->ukeys = take(8 * ucap);
    L->uvals = take(4 * ucap);
    L->upos = take(4 * max_changes);
    L->total = o;
    return true;
}

}  // namespace

using namespace edt;

struct edt_dense_ctx {
    int32_t nx, ny, nz, d_max;
    int64_t max_changes;
    DenseLayout L;
    char* ws;
    DenseMarks mk;
};

extern "C" {

int64_t edt_dense_ctx_bytes(int32_t nx, int32_t ny, int32_t nz, int64_t max_changes) {
    DenseLayout L;
    if (!dense_layout(nx, ny, nz, max_changes, &L)) return EDT_ERR_ARG;
    return L.total;
}

edt_status edt_dense_ctx_global(edt_dense_ctx* c, const uint8_t* d_occ, void* stream) {
    if (!c || !d_occ) return EDT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)c->nx * c->ny * c->nz;
    uint8_t* occ = (uint8_t*)(c->ws + c->L.occ);
    if (hipMemcpyAsync(occ, d_occ, (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return EDT_ERR_HIP;
    return launch_dense3(c->nx, c->ny, c->nz, c->d_max, occ, (int32_t*)(c->ws + c->L.g1),
                         (int32_t*)(c->ws + c->L.g2), (int32_t*)(c->ws + c->L.s),
                         (int2*)(c->ws + c->L.env), st);
}

edt_status edt_dense_ctx_create(int32_t nx, int32_t ny, int32_t nz, int32_t d_max,
                                int64_t max_changes, void* d_ws, int64_t ws_bytes, void* stream,
                                edt_dense_ctx** out) {
    if (!out) return EDT_ERR_ARG;
    *out = nullptr;
    DenseLayout L;
    if (!dense_layout(nx, ny, nz, max_changes, &L) || d_max < 0 || d_max > 46340 || !d_ws ||
        ((uintptr_t)d_ws & 255) != 0)
        return EDT_ERR_ARG;
    if (ws_bytes < L.total) return EDT_ERR_CAPACITY;
    edt_dense_ctx* c = (edt_dense_ctx*)calloc(1, sizeof(edt_dense_ctx));
    if (!c) return EDT_ERR_CAPACITY;
    c->nx = nx; c->ny = ny; c->nz = nz; c->d_max = d_max;
    c->max_changes = max_changes;
    c->L = L;
    c->ws = (char*)d_ws;
    char* b = c->ws;
    c->mk.cnt = (int32_t*)(b + L.cnt);
    c->mk.rowflag = (int32_t*)(b + L.rowflag);
    c->mk.rows = (int32_t*)(b + L.rows);
    c->mk.gy = (int32_t*)(b + L.gy);
    c->mk.ly = (int32_t*)(b + L.ly);
    c->mk.gz = (int32_t*)(b + L.gz);
    c->mk.lz = (int32_t*)(b + L.lz);
    c->mk.tmp = (int32_t*)(b + L.env);   // long-row scratch of pass x (env is free then)
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)nx * ny * nz, nxc = (nx + 63) / 64;
    // empty map, no marks, empty dedupe table; then the field of the empty map
    auto fill = [&](int64_t off, int64_t words, int32_t v) {
        hipLaunchKernelGGL(k_dn_fill, dim3(grid_of((words + 255) / 256, 4096)), dim3(256), 0, st,
                           (int32_t*)(b + off), words, v);
    };
    fill(L.occ, (n + 3) / 4, 0);
    fill(L.rowflag, (int64_t)ny * nz, 0);
    fill(L.gy, nxc * nz, 0);
    fill(L.gz, nxc * ny, 0);
    fill(L.cnt, DC_N, 0);
    fill(L.ukeys, 2 * L.ucap, -1);                        // KEY_EMPTY = all ones
    fill(L.uvals, L.ucap, -1);
    if (hipGetLastError() != hipSuccess) {
        free(c);
        return EDT_ERR_HIP;
    }
    const edt_status e = launch_dense3(nx, ny, nz, d_max, (const uint8_t*)(b + L.occ),
                                       (int32_t*)(b + L.g1), (int32_t*)(b + L.g2),
                                       (int32_t*)(b + L.s), (int2*)(b + L.env), st);
    if (e != EDT_OK) {
        free(c);
        return e;
    }
    *out = c;
    return EDT_OK;
}

edt_status edt_dense_ctx_destroy(edt_dense_ctx* c) {
    free(c);
    return EDT_OK;
}

edt_status edt_dense_ctx_update(edt_dense_ctx* c, const int32_t* d_xyz, const uint8_t* d_state,
                                int64_t n, void* stream) {
    if (!c || n < 0) return EDT_ERR_ARG;
    if (n == 0) return EDT_OK;
    if (!d_xyz || !d_state) return EDT_ERR_ARG;
    if (n > c->max_changes) return EDT_ERR_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    const DenseLayout& L = c->L;
    char* b = c->ws;
    const int nx = c->nx, ny = c->ny, nz = c->nz, nxc = (nx + 63) / 64;
    unsigned long long* ukeys = (unsigned long long*)(b + L.ukeys);
    int32_t* uvals = (int32_t*)(b + L.uvals);
    int32_t* upos = (int32_t*)(b + L.upos);
    uint8_t* occ = (uint8_t*)(b + L.occ);
    int32_t* g1 = (int32_t*)(b + L.g1);
    int32_t* g2 = (int32_t*)(b + L.g2);
    int32_t* sf = (int32_t*)(b + L.s);
    int2* env = (int2*)(b + L.env);
    const int tn = grid_of((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_dn_dedupe, dim3(tn), dim3(256), 0, st, nx, ny, nz, d_xyz, n, ukeys, uvals,
                       (uint32_t)(L.ucap - 1), upos, c->mk);
    hipLaunchKernelGGL(k_dn_apply, dim3(tn), dim3(256), 0, st, nx, ny, d_xyz, d_state, n, occ,
                       ukeys, uvals, (const int32_t*)upos, c->mk);
    // listed rows (at most n), then the listed y and z groups
    const int32_t cap = c->d_max > 0 ? c->d_max * c->d_max : DINF;
    hipLaunchKernelGGL(k_dense_x<true>, dim3(grid_of(n, 65536)), dim3(64), 0, st, nx, ny, nz,
                       (const uint8_t*)occ, g1, c->mk);
    hipLaunchKernelGGL((k_dense_col<1, 16, true>), dim3(grid_of((int64_t)nxc * nz, 16384)),
                       dim3(64), 0, st, nx, ny, nz, (const int32_t*)g1, g2, env, (int32_t)DINF,
                       c->mk);
    hipLaunchKernelGGL((k_dense_col<2, 8, true>), dim3(grid_of((int64_t)nxc * ny, 16384)),
                       dim3(64), 0, st, nx, ny, nz, (const int32_t*)g2, sf, env, cap, c->mk);
    return hipGetLastError() == hipSuccess ? EDT_OK : EDT_ERR_HIP;
}

const int32_t* edt_dense_ctx_field(const edt_dense_ctx* c) {
    return c ? (const int32_t*)(c->ws + c->L.s) : nullptr;
}

edt_status edt_dense_ctx_get_error(edt_dense_ctx* c, void* stream) {
    if (!c) return EDT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    int32_t e = 0;
    if (hipMemcpyAsync(&e, c->mk.cnt + DC_ERR, sizeof(e), hipMemcpyDeviceToHost, st) != hipSuccess)
        return EDT_ERR_HIP;
    hipLaunchKernelGGL(k_dn_fill, dim3(1), dim3(64), 0, st, c->mk.cnt + DC_ERR, (int64_t)1, 0);
    if (hipStreamSynchronize(st) != hipSuccess) return EDT_ERR_HIP;
    return (edt_status)e;
}

int64_t edt_dense_workspace_bytes(int32_t nx, int32_t ny, int32_t nz) {
    if (!dense_ok(nx, ny, nz)) return EDT_ERR_ARG;
    return (int64_t)nx * ny * nz * (int64_t)sizeof(int2);
}

edt_status edt_dense_global(int32_t nx, int32_t ny, int32_t nz, int32_t d_max,
                            const uint8_t* d_occ, int32_t* d_out, void* d_ws, int64_t ws_bytes,
                            void* stream) {
    if (!dense_ok(nx, ny, nz) || d_max < 0 || d_max > 46340 || !d_occ || !d_out || !d_ws)
        return EDT_ERR_ARG;
    if (((uintptr_t)d_ws & 7) != 0) return EDT_ERR_ARG;
    if (ws_bytes < edt_dense_workspace_bytes(nx, ny, nz)) return EDT_ERR_CAPACITY;
    return launch_dense(nx, ny, nz, d_max, d_occ, d_out, (int2*)d_ws, (hipStream_t)stream);
}

edt_status edt_dense_global_noalloc(int32_t nx, int32_t ny, int32_t nz, int32_t d_max,
                                    const uint8_t* d_occ, int32_t* d_out, void* stream) {
    if (!dense_ok(nx, ny, nz) || d_max < 0 || d_max > 46340 || !d_occ || !d_out)
        return EDT_ERR_ARG;
    if (edt_dense_workspace_bytes(nx, ny, nz) > EDT_DENSE_STATIC_BYTES) return EDT_ERR_CAPACITY;
    void* env = nullptr;
    const edt_status e = scratch_address(&env);
    if (e != EDT_OK) return e;
    return launch_dense(nx, ny, nz, d_max, d_occ, d_out, (int2*)env, (hipStream_t)stream);
}

}  // extern "C"
