// edt_win.h -- windowed minimum along one axis, the inner loop of the y and z
// passes for d_max <= 64 (M = ceil(d_max / 8) blocks).
//
// out(i) = min over |k| <= 8M - 1 of in(i + k) + k^2, taken directly: offsets
// beyond d_max - 1 give in + k^2 >= D and change nothing, so the window is
// rounded up to whole blocks.  One lane per row; a wave produces two output
// blocks at a time, with outputs i and i + 8 packed in one 32-bit register
// (16-bit halves; values stay below D + k^2 < 2^16 for d_max <= 64), so each
// candidate costs one packed add and one packed min for two outputs.  The
// 2M + 2 input blocks of the window stay in registers and slide by two
// blocks per step.  Callers make every load and store unconditional (absent
// blocks read a block of D values, halo outputs go to a scratch row) so the
// loop issues a fixed sequence of memory operations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace edt {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline uint32_t word_of(const uint4& v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// Output blocks first .. first + count - 1 (indices in the caller's run).
// blk(b): this lane's 8 values (uint16, along the pass axis) of block b,
// for any b (the caller supplies D for absent blocks).
// emit(ob, acc, has1): acc[o] holds out(8 ob + o) in the low half and
// out(8 ob + 8 + o) in the high half; has1 tells whether block ob + 1 is an
// output block.
template <int M, class Blk, class Emit>
__device__ inline void window_min(int first, int count, uint32_t Dp, Blk&& blk, Emit&& emit) {
    constexpr int NW = 2 * M + 2;        // window blocks
    constexpr int K = 8 * M - 1;         // largest offset
    uint4 W[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) W[w] = blk(first - M + w);
    for (int ob = first; ob < first + count; ob += 2) {
        const uint4 N0 = blk(ob + M + 2), N1 = blk(ob + M + 3);
        u16x2 acc[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[o] = as_u16x2(Dp);
#pragma unroll
        for (int b = 0; b + 1 < NW; ++b) {
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                // input pair (position p, position p + 8), p = 8 (b - M) + z
                const uint32_t lo = word_of(W[b], z >> 1), hi = word_of(W[b + 1], z >> 1);
                const u16x2 P = as_u16x2(
                    __builtin_amdgcn_perm(hi, lo, (z & 1) ? 0x07060302u : 0x05040100u));
                const int p = 8 * (b - M) + z;
                // all sums first, then all minima: independent instructions
                // back to back instead of each min waiting on its add
                u16x2 t[8];
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int k = p - o;
                    const unsigned short kk = (unsigned short)(k * k);
                    if (k >= -K && k <= K) t[o] = P + (u16x2){kk, kk};
                }
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int k = p - o;
                    if (k >= -K && k <= K) acc[o] = __builtin_elementwise_min(acc[o], t[o]);
                }
            }
        }
        emit(ob, acc, ob + 1 < first + count);
#pragma unroll
        for (int w = 0; w + 2 < NW; ++w) W[w] = W[w + 2];
        W[NW - 2] = N0;
        W[NW - 1] = N1;
    }
}

}  // namespace edt
