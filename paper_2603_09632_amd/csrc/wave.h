// Cross-lane exchanges of a 64-lane wavefront that stay in registers.
//
// A butterfly step K (32, 16, 8, 4, 2, 1) pairs each lane whose bit K is 0
// ("lower") with a partner whose bit K is 1 and whose higher bits agree:
//   K = 32, 16: v_permlane32_swap / v_permlane16_swap, which swap the partner
//               halves of two registers (one add then finishes a pair);
//   K = 8 .. 1: DPP within rows of 16 lanes -- row_ror:8, row_half_mirror,
//               quad_perm [3,2,1,0], quad_perm [1,0,3,2].
// Each partner map is an involution; the six generators (32, 16, 8, 7, 3, 1)
// span all 64 lanes, so six steps combine every lane exactly once.
#pragma once
#include "common.h"

namespace xgs {

// Partner's value for step K <= 8 (DPP, within a row of 16 lanes).
template <int K>
__device__ __forceinline__ float xlane_dpp(float v) {
    static_assert(K == 8 || K == 4 || K == 2 || K == 1, "DPP steps");
    constexpr int ctrl = K == 8 ? 0x128 : K == 4 ? 0x141 : K == 2 ? 0x1B : 0xB1;
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, true));
}

// Swap step K = 32 or 16 on (x, y): returns the two registers after the swap;
// lower lanes hold (x, partner x), upper lanes (partner y, y).
template <int K>
__device__ __forceinline__ void xlane_swap(float x, float y, float& r0, float& r1) {
    static_assert(K == 32 || K == 16, "lane swaps are for the two upper steps");
    if constexpr (K == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        r0 = __uint_as_float(r[0]);
        r1 = __uint_as_float(r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        r0 = __uint_as_float(r[0]);
        r1 = __uint_as_float(r[1]);
    }
}

// Partner's value at step K (any of the six), for integer payloads.
template <int K>
__device__ __forceinline__ int xlane_partner(int v, int lane) {
    if constexpr (K >= 16) {
        const auto r = K == 32 ? __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false)
                               : __builtin_amdgcn_permlane16_swap((uint32_t)v, (uint32_t)v, false, false);
        return (lane & K) == 0 ? (int)r[1] : (int)r[0];
    } else {
        constexpr int ctrl = K == 8 ? 0x128 : K == 4 ? 0x141 : K == 2 ? 0x1B : 0xB1;
        return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xF, 0xF, true);
    }
}

// Sum (or max) over all 64 lanes, result in every lane.
__device__ __forceinline__ float wave_sum(float v) {
    float a, b;
    xlane_swap<32>(v, v, a, b);
    v = a + b;
    xlane_swap<16>(v, v, a, b);
    v = a + b;
    v += xlane_dpp<8>(v);
    v += xlane_dpp<4>(v);
    v += xlane_dpp<2>(v);
    v += xlane_dpp<1>(v);
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
    float a, b;
    xlane_swap<32>(v, v, a, b);
    v = fmaxf(a, b);
    xlane_swap<16>(v, v, a, b);
    v = fmaxf(a, b);
    v = fmaxf(v, xlane_dpp<8>(v));
    v = fmaxf(v, xlane_dpp<4>(v));
    v = fmaxf(v, xlane_dpp<2>(v));
    v = fmaxf(v, xlane_dpp<1>(v));
    return v;
}

// One halving step of the reduce-scatter of N values: the lower lane keeps
// the first half (summed with its partner's), the upper lane the second; an
// odd leftover value is summed on both and owned by the lower.
template <int N, int K>
__device__ __forceinline__ void rs_step(float* a, bool lower) {
    constexpr int H = N / 2;
    if constexpr (K >= 16) {
        float r0, r1;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            xlane_swap<K>(a[i], a[H + i], r0, r1);
            a[i] = r0 + r1;
        }
        if (N % 2) {
            xlane_swap<K>(a[2 * H], a[2 * H], r0, r1);
            a[H] = r0 + r1;
        }
    } else {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const float send = lower ? a[H + i] : a[i];
            const float keep = lower ? a[i] : a[H + i];
            a[i] = keep + xlane_dpp<K>(send);
        }
        if (N % 2) a[H] = a[2 * H] + xlane_dpp<K>(a[2 * H]);
    }
}

template <int N, int K>
__device__ __forceinline__ void rs_ids(int* id, bool* own, bool lower) {
    constexpr int H = N / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        id[i] = lower ? id[i] : id[H + i];
        own[i] = lower ? own[i] : own[H + i];
    }
    if (N % 2) {
        id[H] = id[2 * H];
        own[H] = own[2 * H] && lower;
    }
}

constexpr int ceil2(int n) { return (n + 1) / 2; }

// Reduces V values over the 64 lanes; afterwards a[0] holds the full sum of
// value `id` (computed once by rs_layout), written by the lane with own=true.
template <int V>
__device__ __forceinline__ void reduce_scatter(float* a, int lane) {
    constexpr int N1 = V, N2 = ceil2(N1), N3 = ceil2(N2), N4 = ceil2(N3), N5 = ceil2(N4), N6 = ceil2(N5);
    rs_step<N1, 32>(a, (lane & 32) == 0);
    rs_step<N2, 16>(a, (lane & 16) == 0);
    rs_step<N3, 8>(a, (lane & 8) == 0);
    rs_step<N4, 4>(a, (lane & 4) == 0);
    rs_step<N5, 2>(a, (lane & 2) == 0);
    rs_step<N6, 1>(a, (lane & 1) == 0);
}

template <int V>
__device__ __forceinline__ void rs_layout(int lane, int* out_id, bool* out_own) {
    static_assert(V <= 64, "one value per lane after the reduce-scatter");
    int id[V];
    bool own[V];
#pragma unroll
    for (int i = 0; i < V; ++i) { id[i] = i; own[i] = true; }
    constexpr int N1 = V, N2 = ceil2(N1), N3 = ceil2(N2), N4 = ceil2(N3), N5 = ceil2(N4), N6 = ceil2(N5);
    rs_ids<N1, 32>(id, own, (lane & 32) == 0);
    rs_ids<N2, 16>(id, own, (lane & 16) == 0);
    rs_ids<N3, 8>(id, own, (lane & 8) == 0);
    rs_ids<N4, 4>(id, own, (lane & 4) == 0);
    rs_ids<N5, 2>(id, own, (lane & 2) == 0);
    rs_ids<N6, 1>(id, own, (lane & 1) == 0);
    *out_id = id[0];
    *out_own = own[0];
}

}  // namespace xgs
