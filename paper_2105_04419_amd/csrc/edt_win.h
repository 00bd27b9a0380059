// edt_win.h -- windowed minimum along one axis, the inner loop of the y and z
// passes for d_max <= 64 (M = ceil(d_max / 8) blocks).
//
// out(i) = min over |k| <= 8M - 1 of in(i + k) + k^2, taken directly: offsets
// beyond d_max - 1 give in + k^2 >= D and change nothing, so the window is
// rounded up to whole blocks.  One lane per row; a wave produces two output
// blocks at a time, with outputs i and i + 8 packed in one 32-bit register
// (16-bit halves; values stay below D + k^2 < 2^16 for d_max <= 64).  The
// offsets +k and -k share k^2, so each pair of candidates costs one packed
// min, one packed add and one packed min for two outputs; offsets are taken
// outward from 0, and the wave stops early once every output is already no
// larger than the square of the next offset.  The 2M + 2 input blocks of the
// window stay in registers and slide by two blocks per step.  Callers make
// every load unconditional (absent blocks read a block of D values) and
// guard stores only by wave-uniform conditions, so the loop issues a fixed
// sequence of loads.
//
// Half-precision mode (F16, for d_max <= 40, so D <= 1600): the values are
// held as IEEE binary16 instead of integers.  Every integer up to 2048 is
// exact in binary16, so inputs (<= D), squares of offsets and every candidate
// sum below 2048 are exact; a candidate whose exact sum is 2048 or more
// rounds to a value >= 2048 > D, so it can never beat an output, which stays
// <= D.  The results are therefore the same integers.  Non-negative binary16
// values order like their bit patterns, so the mins of the two candidates of
// an offset stay integer mins on the bits; the additions are binary16, and
// the candidates of two offsets join an output with one three-way minimum
// (v_pk_minimum3_f16), 2.5 instructions per offset and output pair instead of
// 3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace edt {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

__device__ inline u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline h16x2 as_h16x2(u16x2 v) { return __builtin_bit_cast(h16x2, v); }
__device__ inline u16x2 as_u16x2(h16x2 v) { return __builtin_bit_cast(u16x2, v); }

// Block radii whose intermediates (g1, g2) are stored as binary16.
__host__ __device__ constexpr bool win_f16(int M) { return M <= 5; }

// binary16 bit pattern of an integer 0 <= n <= 2048 (exact).
__host__ __device__ constexpr uint32_t f16_bits(uint32_t n) {
    uint32_t e = 0;
    while ((2u << e) <= n) ++e;                // n in [2^e, 2^(e+1))
    return n == 0 ? 0u : ((e + 15u) << 10) | ((n << (10u - e)) & 0x3ffu);
}
// Integer value of a binary16 bit pattern holding an integer <= 2048.
__device__ inline int f16_int(uint32_t bits) {
    return (int)(unsigned short)__builtin_bit_cast(_Float16, (unsigned short)bits);
}
__device__ inline uint32_t word_of(const uint4& v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// Largest / least of the 8 packed output pairs, per half.  Binary16 values
// here are non-negative, so the float extrema (three-way packed
// instructions) equal the extrema of the bit patterns.
template <bool F16>
__device__ inline u16x2 max8(const u16x2* a) {
    if (F16) {
        const h16x2 x = __builtin_elementwise_maximum(
            __builtin_elementwise_maximum(as_h16x2(a[0]), as_h16x2(a[1])), as_h16x2(a[2]));
        const h16x2 y = __builtin_elementwise_maximum(
            __builtin_elementwise_maximum(as_h16x2(a[3]), as_h16x2(a[4])), as_h16x2(a[5]));
        const h16x2 z = __builtin_elementwise_maximum(as_h16x2(a[6]), as_h16x2(a[7]));
        return as_u16x2(__builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z));
    }
    u16x2 m = __builtin_elementwise_max(a[0], a[1]);
#pragma unroll
    for (int o = 2; o < 8; ++o) m = __builtin_elementwise_max(m, a[o]);
    return m;
}
template <bool F16>
__device__ inline u16x2 min8(const u16x2* a) {
    if (F16) {
        const h16x2 x = __builtin_elementwise_minimum(
            __builtin_elementwise_minimum(as_h16x2(a[0]), as_h16x2(a[1])), as_h16x2(a[2]));
        const h16x2 y = __builtin_elementwise_minimum(
            __builtin_elementwise_minimum(as_h16x2(a[3]), as_h16x2(a[4])), as_h16x2(a[5]));
        const h16x2 z = __builtin_elementwise_minimum(as_h16x2(a[6]), as_h16x2(a[7]));
        return as_u16x2(__builtin_elementwise_minimum(__builtin_elementwise_minimum(x, y), z));
    }
    u16x2 m = __builtin_elementwise_min(a[0], a[1]);
#pragma unroll
    for (int o = 2; o < 8; ++o) m = __builtin_elementwise_min(m, a[o]);
    return m;
}

// Output blocks first .. first + count - 1 (indices in the caller's run).
// blk(b): this lane's 8 values (uint16, along the pass axis) of block b,
// for any b (the caller supplies D for absent blocks).
// emit(ob, acc, has1): acc[o] holds out(8 ob + o) in the low half and
// out(8 ob + 8 + o) in the high half; has1 tells whether block ob + 1 is an
// output block.
// Uniform skip masks over window positions j (block first - M + j).
// Every output stays <= D, and group G of offsets (k = max(1, 8G) ..
// 8G + 7) offers from block b only candidates >= min(b) + k^2; so group G
// is skipped when every block it reads has bit j of g[G] set, meaning
// min(b) + max(1, 8G)^2 >= D.  Bit j of d: block b is D everywhere.  A pair
// whose two output blocks are D everywhere and whose groups are all skipped
// is D without any arithmetic.
struct WinSkip {
    uint64_t g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t d = 0;
};

// need(ob): false when neither output block ob nor ob + 1 is wanted (must be
// uniform across the wave); the window still slides over such a pair.
// LB: before each offset group G >= 1, also test a per-lane bound (the least
// input in the group's position ranges plus (8G)^2 against the lane's largest
// output) and skip the group when no lane can improve.  It pays on maps where
// most groups are decided that way (dense maps), not where the block bounds
// already skip them.
// F16: values are binary16 bit patterns (see above); Dp then holds D as two
// binary16 halves, and so do the outputs handed to emit.
template <int M, bool LB = false, bool F16 = false, class Blk, class Emit, class Need>
__device__ inline void window_min(int first, int count, uint32_t Dp, Blk&& blk, Emit&& emit,
                                  Need&& need, const WinSkip& sk) {
    constexpr int NW = 2 * M + 2;        // window blocks
    constexpr int K = 8 * M - 1;         // largest offset
    constexpr int NP = 8 * (NW - 1);     // input pairs: positions p = -8M .. 8M + 7
    // P[q]: (in(p), in(p + 8)) for p = q - 8M relative to the step's first
    // output, packed.  The window slides by 16 positions per step, so all but
    // the last 16 pairs of a step are the previous step's pairs moved down;
    // only the newest input block (Wl) is kept besides P.
    u16x2 P[NP];
    uint4 Wl;
    {
        uint4 W[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) W[w] = blk(first - M + w);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int b = q >> 3, z = q & 7;
            const uint32_t lo = word_of(W[b], z >> 1), hi = word_of(W[b + 1], z >> 1);
            P[q] = as_u16x2(__builtin_amdgcn_perm(hi, lo, (z & 1) ? 0x07060302u : 0x05040100u));
        }
        Wl = W[NW - 1];
    }
    // a caller may raise the wave's priority for its lookups and the loads
    // above; the window arithmetic runs at the normal priority
    __builtin_amdgcn_s_setprio(0);
    for (int ob = first; ob < first + count; ob += 2) {
        const uint4 N0 = blk(ob + M + 2), N1 = blk(ob + M + 3);
        u16x2 acc[8];
        if (need(ob)) {
            // bit j of the shifted masks: block ob - M + j
            const int sh = ob - first;
            bool flat = ((sk.d >> sh) & (3ull << M)) == (3ull << M);
#pragma unroll
            for (int G = 0; G < M; ++G) {
                const uint64_t CG = (7ull << (M - G - 1)) | (7ull << (M + G));
                flat = flat && ((sk.g[G] >> sh) & CG) == CG;
            }
            if (flat) {
#pragma unroll
                for (int o = 0; o < 8; ++o) acc[o] = as_u16x2(Dp);
            } else {
#pragma unroll
                for (int o = 0; o < 8; ++o) acc[o] = P[o + 8 * M];
                // offsets outward in groups of 8: group G (k = 8G .. 8G + 7,
                // k >= 1) reads blocks ob - G - 1 .. ob - G + 1 and
                // ob + G .. ob + G + 2; the two candidates at +-k share k^2,
                // so min(in(i - k), in(i + k)) + k^2 covers both
                // per-lane bound: group G offers candidates no smaller than the
                // least input in its two position ranges plus (8G)^2; mx is the
                // lane's largest output so far (both halves)
                u16x2 mx = LB ? max8<F16>(acc) : acc[0];
#pragma unroll
                for (int G = 0; G < M; ++G) {
                    const uint64_t CG = (7ull << (M - G - 1)) | (7ull << (M + G));
                    if (((sk.g[G] >> sh) & CG) == CG) continue;
                    if (LB && G > 0) {
                        // candidates of group G for output o lie at o + 8M -+ k,
                        // k = 8G .. 8G + 7: positions 8M - 8G - 7 .. 8M - 8G + 7
                        // and 8M + 8G .. 8M + 8G + 14 (packed: the high half
                        // covers the outputs o + 8)
                        u16x2 lb = P[8 * M - 8 * G - 7];
#pragma unroll
                        for (int q = 8 * M - 8 * G - 6; q <= 8 * M - 8 * G + 7; ++q)
                            lb = __builtin_elementwise_min(lb, P[q]);
#pragma unroll
                        for (int q = 8 * M + 8 * G; q <= 8 * M + 8 * G + 14 && q < NP; ++q)
                            lb = __builtin_elementwise_min(lb, P[q]);
                        if (F16) {
                            const _Float16 g2 = (_Float16)(64 * G * G);
                            lb = as_u16x2(as_h16x2(lb) + (h16x2){g2, g2});
                        } else {
                            const unsigned short g2 = (unsigned short)(64 * G * G);
                            lb = lb + (u16x2){g2, g2};
                        }
                        if (!__any(lb.x < mx.x || lb.y < mx.y)) continue;
                    }
                    const int k0 = G == 0 ? 1 : 8 * G, k1 = 8 * G + 7;
                    // one side of the group can be skipped on its own: the
                    // candidates of offsets -k then come from the blocks
                    // before the outputs only, those of +k from the blocks
                    // after them only (side 0 both, 1 minus, 2 plus)
                    const uint64_t CL = 7ull << (M - G - 1), CR = 7ull << (M + G);
                    const bool skipL = ((sk.g[G] >> sh) & CL) == CL;
                    const bool skipR = ((sk.g[G] >> sh) & CR) == CR;
                    auto cand = [&](int o, int k, int side) -> u16x2 {
                        return side == 1 ? P[o + 8 * M - k]
                             : side == 2 ? P[o + 8 * M + k]
                                         : __builtin_elementwise_min(P[o + 8 * M - k],
                                                                     P[o + 8 * M + k]);
                    };
                    auto run = [&](int side) {
                        if (F16) {
                            // offsets in pairs: two candidates and the output
                            // meet in one three-way minimum
#pragma unroll
                            for (int k = k0; k <= k1; k += 2) {
                                const _Float16 ka = (_Float16)(k * k);
                                const _Float16 kb = (_Float16)((k + 1) * (k + 1));
#pragma unroll
                                for (int o = 0; o < 8; ++o) {
                                    const h16x2 ca = as_h16x2(cand(o, k, side)) + (h16x2){ka, ka};
                                    h16x2 a = __builtin_elementwise_minimum(as_h16x2(acc[o]), ca);
                                    if (k + 1 <= k1) {
                                        const h16x2 cb =
                                            as_h16x2(cand(o, k + 1, side)) + (h16x2){kb, kb};
                                        a = __builtin_elementwise_minimum(a, cb);
                                    }
                                    acc[o] = as_u16x2(a);
                                }
                            }
                        } else {
#pragma unroll
                            for (int k = k0; k <= k1; ++k) {
                                const unsigned short kk = (unsigned short)(k * k);
#pragma unroll
                                for (int o = 0; o < 8; ++o)
                                    acc[o] = __builtin_elementwise_min(
                                        acc[o], cand(o, k, side) + (u16x2){kk, kk});
                            }
                        }
                    };
                    if (!skipL && !skipR) run(0);
                    else if (!skipL) run(1);
                    else run(2);
                    // stop once no output of the wave can still drop, i.e. all
                    // are <= (8G + 8)^2, the least any further candidate adds
                    // (binary16 patterns order like their values)
                    if (G + 1 < M) {
                        mx = max8<F16>(acc);
                        const uint32_t sq = (8 * G + 8) * (8 * G + 8);
                        const int lim = F16 ? (int)f16_bits(sq) : (int)sq;
                        const bool more = (int)mx.x > lim || (int)mx.y > lim;
                        if (!__any(more)) break;
                    }
                }
            }
        }
        // slide: pairs move down by 16 positions; the 16 new ones pair the
        // old last block with N0 and N0 with N1.  This waits for the loads of
        // N0 and N1 (and the stores before them), so it comes before this
        // step's stores, which then stay in flight during the next step.
#pragma unroll
        for (int q = 0; q + 16 < NP; ++q) P[q] = P[q + 16];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const uint32_t sel = (z & 1) ? 0x07060302u : 0x05040100u;
            P[NP - 16 + z] = as_u16x2(__builtin_amdgcn_perm(word_of(N0, z >> 1),
                                                            word_of(Wl, z >> 1), sel));
            P[NP - 8 + z] = as_u16x2(__builtin_amdgcn_perm(word_of(N1, z >> 1),
                                                           word_of(N0, z >> 1), sel));
        }
        Wl = N1;
        if (need(ob)) emit(ob, acc, ob + 1 < first + count);
    }
}

template <int M, bool LB = false, bool F16 = false, class Blk, class Emit>
__device__ inline void window_min(int first, int count, uint32_t Dp, Blk&& blk, Emit&& emit) {
    window_min<M, LB, F16>(first, count, Dp, blk, emit, [](int) { return true; }, WinSkip{});
}

}  // namespace edt
