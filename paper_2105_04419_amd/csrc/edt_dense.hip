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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "edt.h"

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

__global__ void __launch_bounds__(64) k_dense_x(int nx, int ny, int nz,
                                                const uint8_t* __restrict__ occ, int32_t* out) {
    constexpr int64_t FAR = 1ll << 40;
    const int lane = threadIdx.x;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const uint8_t* row = occ + r * nx;
        int32_t* o = out + r * nx;
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
                    if (x < nx) o[x] = x - near > (1 << 30) ? DINF : (int32_t)(x - near);
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
                    dl = x < nx ? (int64_t)o[x] : FAR;
                }
                const int64_t d = (int64_t)res[k] < dl ? (int64_t)res[k] : dl;
                res[k] = d > (1 << 30) ? DINF : (int32_t)(d * d);
            }
            const int xs = x0 + 16 * lane;
            if (xs + 16 <= nx && ((uintptr_t)(o + xs) & 15) == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    *(int4*)(o + xs + 4 * q) =
                        make_int4(res[4 * q], res[4 * q + 1], res[4 * q + 2], res[4 * q + 3]);
            } else {
                for (int k = 0; k < 16; ++k)
                    if (xs + k < nx) o[xs + k] = res[k];
            }
            const int64_t tot = __shfl(incl, 0);
            if (tot < rcarry) rcarry = tot;
        }
    }
}

// Passes y (AXIS 1) and z (AXIS 2), in place on out, with the envelope in
// env.  Column (x, w): x fastest within a wave; w = z for y, y for z.  The
// column is read and written CH values at a time.
template <int AXIS, int CH>
__global__ void __launch_bounds__(64) k_dense_col(int nx, int ny, int nz, int32_t* out, int2* env,
                                                  int32_t cap) {
    const int lane = threadIdx.x;
    const int n = AXIS == 1 ? ny : nz;                 // column length
    const int nw = AXIS == 1 ? nz : ny;
    const int64_t stride = AXIS == 1 ? (int64_t)nx : (int64_t)nx * ny;
    const int nxc = (nx + 63) / 64;
    const int64_t ncols = (int64_t)nx * nw;
    const int64_t waves = (int64_t)nxc * nw;
    for (int64_t wv = blockIdx.x; wv < waves; wv += gridDim.x) {
        const int x = (int)(wv % nxc) * 64 + lane;
        const int w = (int)(wv / nxc);
        if (x >= nx) continue;
        const int64_t base = AXIS == 1 ? (int64_t)x + (int64_t)nx * ny * w
                                       : (int64_t)x + (int64_t)nx * w;
        const int64_t col = (int64_t)x + (int64_t)nx * w;   // column index among ncols
        int2* E = env + col;                                 // entry k at E[k * ncols]
        // build the lower envelope; (v1, F1) is the top, (v0, F0) the entry
        // below it and (v2, F2) the one below that, held in registers so a
        // pop needs no load (the entry under v2 is fetched at each pop and
        // used only at the next)
        int k = -1;
        int v0 = 0, v1 = 0, v2 = 0;
        int64_t F0 = 0, F1 = 0, F2 = 0;                      // f + v^2
        // the column is read CH values at a time, the next CH in flight while
        // the current ones are pushed (positions past the end read as DINF)
        const int32_t* src = out + base;
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
                // pop while the top parabola's interval is empty: the new one
                // overtakes it no later than the top overtook the one below
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
        // read off: parabola j covers q while the next one is not yet lower
        if (k < 0) {
            for (int q = 0; q < n; ++q) out[base + stride * q] = cap;
            continue;
        }
        int j = 0;
        int2 cur = E[0];
        int2 nxt = k >= 1 ? E[ncols] : cur;
        int2 nx2 = k >= 2 ? E[2 * ncols] : nxt;              // fetched one entry ahead
        // CH outputs are computed, then stored together
        int32_t* dst = out + base;
        for (int q0 = 0; q0 < n; q0 += CH) {
            int32_t res[CH];
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
                res[u] = d < (int64_t)cap ? (int32_t)d : cap;
            }
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (q0 + u < n) dst[stride * (q0 + u)] = res[u];
        }
    }
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

// The three passes of the dense transform on `st`, envelopes in env.
edt_status launch_dense(int32_t nx, int32_t ny, int32_t nz, int32_t d_max, const uint8_t* d_occ,
                        int32_t* d_out, int2* env, hipStream_t st) {
    using namespace edt;
    const int32_t cap = d_max > 0 ? d_max * d_max : DINF;
    const int nxc = (nx + 63) / 64;
    hipLaunchKernelGGL(k_dense_x, dim3(grid_of((int64_t)ny * nz, 65536)), dim3(64), 0, st, nx, ny,
                       nz, d_occ, d_out);
    // chunk lengths measured on a 1024x1024x128 extent: 16 for the long y
    // columns, 8 for z (fewer registers, more resident waves)
    hipLaunchKernelGGL((k_dense_col<1, 16>), dim3(grid_of((int64_t)nxc * nz, 65536)), dim3(64),
                       0, st, nx, ny, nz, d_out, env, (int32_t)DINF);
    hipLaunchKernelGGL((k_dense_col<2, 8>), dim3(grid_of((int64_t)nxc * ny, 65536)), dim3(64), 0,
                       st, nx, ny, nz, d_out, env, cap);
    if (hipGetLastError() != hipSuccess) return EDT_ERR_HIP;
    return EDT_OK;
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

}  // namespace

using namespace edt;

extern "C" {

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
