// f4: region-indexed grid targets (App. D, Eq. (target_discrete)) and the
// occluder pruning test of the mapping phase (Sec. 3.2.1, relative margin).
#include "common.h"

namespace xgs {

// channels per thread: the labels of a pixel are looked up once per chunk
constexpr int kRegChunk = 32;

// Same layout as the grid sample: each thread owns four consecutive grid
// pixels, looks their labels up once and streams a chunk of channels of
// Phi[label] out with 16-byte non-temporal stores (Phi stays in cache).
// PV: D % 4 == 0 and Phi 16-byte aligned, so four channels of a label row
// come in one load and are turned into four per-channel output vectors.
template <bool VEC, bool PV>
__global__ void __launch_bounds__(256) region_targets_kernel(const int32_t* __restrict__ S, int H, int W,
                                                            const float* __restrict__ Phi, int R, int D, int s,
                                                            int oy, int ox, int Hs, int Ws,
                                                            float* __restrict__ G, uint8_t* __restrict__ V) {
    const int64_t hw = (int64_t)Hs * Ws;
    const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (p0 >= hw) return;
    int lab[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t p = p0 + k < hw ? p0 + k : hw - 1;
        // hw < 2^31 (checked by the caller): 32-bit division
        const int m = (int)p / Ws, n = (int)p - m * Ws;
        const int64_t u = (int64_t)oy + (int64_t)m * s, v = (int64_t)ox + (int64_t)n * s;
        int l = -1;
        if (u < H && v < W) l = S[u * W + v];
        lab[k] = (l >= 0 && l < R) ? l : -1;  // labels outside [0, R): unannotated
    }
    const int d0 = blockIdx.y * kRegChunk;
    const int d1 = d0 + kRegChunk < D ? d0 + kRegChunk : D;
    auto put = [&](int d, f32x4_t val) {
        float* out = G + (int64_t)d * hw + p0;
        if (VEC) {
            __builtin_nontemporal_store(val, reinterpret_cast<f32x4_t*>(out));
        } else {
            for (int k = 0; k < 4 && p0 + k < hw; ++k) __builtin_nontemporal_store(val[k], out + k);
        }
    };
    if constexpr (PV) {
        for (int d = d0; d < d1; d += 4) {
            f32x4_t row[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                row[k] = lab[k] >= 0 ? *reinterpret_cast<const f32x4_t*>(Phi + (size_t)lab[k] * D + d)
                                     : f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < 4; ++j) put(d + j, f32x4_t{row[0][j], row[1][j], row[2][j], row[3][j]});
        }
    } else {
        for (int d = d0; d < d1; ++d) {
            f32x4_t val;
#pragma unroll
            for (int k = 0; k < 4; ++k) val[k] = lab[k] >= 0 ? Phi[(size_t)lab[k] * D + d] : 0.f;
            put(d, val);
        }
    }
    if (V && blockIdx.y == 0)
        for (int k = 0; k < 4 && p0 + k < hw; ++k) V[p0 + k] = lab[k] >= 0 ? 1 : 0;
}

// One thread per Gaussian: visible (radius > 0), projected mean inside the
// image, depth map positive at the pixel floor(mean2d), camera depth below
// (1 - margin) times that depth.  The count is an integer sum.
__global__ void __launch_bounds__(256) occluder_kernel(int64_t n, const float4* __restrict__ splat,
                                                      const int32_t* __restrict__ radius,
                                                      const float* __restrict__ depth_map, int H, int W,
                                                      float keep, uint8_t* __restrict__ prune,
                                                      unsigned long long* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int hit = 0;
    if (i < n) {
        if (radius[i] > 0) {
            const float4 s0 = splat[2 * i], s1 = splat[2 * i + 1];
            const float x = s0.x, y = s0.y, z = s1.z;
            if (x >= 0.f && y >= 0.f) {
                const float fx = floorf(x), fy = floorf(y);
                if (fx < (float)W && fy < (float)H) {
                    const float d = depth_map[(int64_t)fy * W + (int64_t)fx];
                    hit = d > 0.f && z < keep * d;
                }
            }
        }
        prune[i] = (uint8_t)hit;
    }
    unsigned long long c = (unsigned long long)hit;
    for (int k = 32; k >= 1; k >>= 1) c += __shfl_xor(c, k, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void occ_zero_kernel(unsigned long long* __restrict__ c) { *c = 0ull; }

}  // namespace xgs

using namespace xgs;

extern "C" xgs_status xgs_region_targets(const int32_t* S, int32_t H, int32_t W, const float* Phi, int32_t R,
                                         int32_t D, int32_t stride, int32_t off_y, int32_t off_x, float* G,
                                         uint8_t* V, xgs_stream_t stream) {
    clear_error();
    if (H < 1 || W < 1 || R < 0 || D < 0 || stride < 1)
        return fail(XGS_ERR_INVALID_ARG, "xgs_region_targets: sizes must be positive (R, D >= 0)");
    if (off_y < 0 || off_x < 0 || off_y >= stride || off_x >= stride)
        return fail(XGS_ERR_INVALID_ARG, "xgs_region_targets: offsets must lie in [0, stride)");
    if (!S || (D > 0 && (!G || (R > 0 && !Phi)))) return fail(XGS_ERR_INVALID_ARG, "xgs_region_targets: null pointer");
    const int Hs = (H + stride - 1) / stride, Ws = (W + stride - 1) / stride;
    const int64_t hw = (int64_t)Hs * Ws;
    if (D == 0 && !V) return XGS_OK;
    const bool vec = (hw % 4 == 0) && aligned(G, 16);
    const unsigned bx = (unsigned)((hw + 1023) / 1024);
    const unsigned by = (unsigned)(D > 0 ? (D + kRegChunk - 1) / kRegChunk : 1);
    if (by > 65535) return fail(XGS_ERR_UNSUPPORTED, "xgs_region_targets: too many channels");
    if (hw >= (int64_t(1) << 31) - 4)
        return fail(XGS_ERR_UNSUPPORTED, "xgs_region_targets: sampled grid above 2^31 pixels");
    const bool pv = D % 4 == 0 && (R == 0 || aligned(Phi, 16));
    hipStream_t st = (hipStream_t)stream;
#define XGS_RT_LAUNCH(V4, P4)                                                                               \
    hipLaunchKernelGGL((region_targets_kernel<V4, P4>), dim3(bx, by), dim3(256), 0, st, S, H, W, Phi, R, D, stride, \
                       off_y, off_x, Hs, Ws, G, V)
    if (vec && pv) XGS_RT_LAUNCH(true, true);
    else if (vec) XGS_RT_LAUNCH(true, false);
    else if (pv) XGS_RT_LAUNCH(false, true);
    else XGS_RT_LAUNCH(false, false);
#undef XGS_RT_LAUNCH
    return check_launch("xgs_region_targets");
}

extern "C" xgs_status xgs_occluder_mask(const xgs_projected* p, int64_t n, const float* depth_map, int32_t H,
                                        int32_t W, float margin, uint8_t* prune, uint64_t* count,
                                        xgs_stream_t stream) {
    clear_error();
    if (!p || n < 0 || H < 1 || W < 1) return fail(XGS_ERR_INVALID_ARG, "xgs_occluder_mask: bad arguments");
    if (!(margin >= 0.f && margin < 1.f)) return fail(XGS_ERR_INVALID_ARG, "xgs_occluder_mask: margin must be in [0, 1)");
    if (!count || (n > 0 && (!p->splat || !p->radius || !depth_map || !prune)))
        return fail(XGS_ERR_INVALID_ARG, "xgs_occluder_mask: null pointer");
    if (!aligned(p->splat, 16)) return fail(XGS_ERR_INVALID_ARG, "xgs_occluder_mask: splat must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    auto* c = reinterpret_cast<unsigned long long*>(count);
    hipLaunchKernelGGL(occ_zero_kernel, dim3(1), dim3(1), 0, st, c);
    if (n > 0)
        hipLaunchKernelGGL(occluder_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                           reinterpret_cast<const float4*>(p->splat), p->radius, depth_map, H, W, 1.f - margin,
                           prune, c);
    return check_launch("xgs_occluder_mask");
}
