// a5: grid-sampled distillation targets from a low-resolution feature map
// (App. D, Eq. (sampled_loc) and Eq. (target_continuous)).  The kernel is
// write-bound: P (a few MB) stays in cache while G (D x H_s x W_s floats) is
// streamed out with 16-byte non-temporal stores.  Each thread owns four
// consecutive grid pixels, computes their source coordinates once, and loops
// over a chunk of channels.
#include "common.h"

namespace xgs {

struct Src {
    int y0, y1, x0, x1;
    float wy, wx;
    bool valid;
};

// I: integer type of the exact source arithmetic.  int32_t when every
// product below fits (checked by the caller), else int64_t; both give the
// same integers and hence the same weights.
template <typename I>
__device__ __forceinline__ Src source_of(int64_t p, int Ws, int H, int W, int Hf, int Wf, int s,
                                         int oy, int ox, int mode) {
    Src r;
    const I m = (I)p / (I)Ws, n = (I)p - m * (I)Ws;
    const I u = (I)oy + m * (I)s, v = (I)ox + n * (I)s;
    r.valid = u < H && v < W;
    const I by = H > 1 ? H - 1 : 1, bx = W > 1 ? W - 1 : 1;
    const I ay = u * (I)(Hf - 1), ax = v * (I)(Wf - 1);
    const I qy = ay / by, ry = ay - qy * by;
    const I qx = ax / bx, rx = ax - qx * bx;
    if (mode == XGS_GRID_NEAREST) {
        // round half to even of ay/by and ax/bx, exactly
        I iy = qy + ((2 * ry > by) || (2 * ry == by && (qy & 1)));
        I ix = qx + ((2 * rx > bx) || (2 * rx == bx && (qx & 1)));
        r.y0 = r.y1 = (int)(iy < Hf - 1 ? iy : Hf - 1);
        r.x0 = r.x1 = (int)(ix < Wf - 1 ? ix : Wf - 1);
        r.wy = r.wx = 0.f;
    } else {
        r.y0 = (int)(qy < Hf - 1 ? qy : Hf - 1);
        r.x0 = (int)(qx < Wf - 1 ? qx : Wf - 1);
        r.y1 = r.y0 + 1 < Hf ? r.y0 + 1 : Hf - 1;
        r.x1 = r.x0 + 1 < Wf ? r.x0 + 1 : Wf - 1;
        r.wy = (float)ry / (float)by;
        r.wx = (float)rx / (float)bx;
    }
    if (!r.valid) { r.y0 = r.y1 = r.x0 = r.x1 = 0; }
    return r;
}

__device__ __forceinline__ float sample(const float* __restrict__ Pd, int Wf, const Src& s) {
    if (!s.valid) return 0.f;
    const float p00 = Pd[s.y0 * Wf + s.x0], p01 = Pd[s.y0 * Wf + s.x1];
    const float p10 = Pd[s.y1 * Wf + s.x0], p11 = Pd[s.y1 * Wf + s.x1];
    const float top = p00 + s.wx * (p01 - p00);
    const float bot = p10 + s.wx * (p11 - p10);
    return top + s.wy * (bot - top);
}

// channels per thread: the source coordinates of a pixel are computed once per chunk
constexpr int kChanChunk = 16;

// ALL: blockIdx.z is the grid offset o = oy s + ox, whose grid goes to
// G + o D Hs Ws and V + o Hs Ws (the oy, ox arguments are ignored).
template <bool VEC, typename I, bool ALL>
__global__ void __launch_bounds__(256) grid_sample_kernel(const float* __restrict__ P, int D, int Hf,
                                                         int Wf, int H, int W, int s, int oy, int ox,
                                                         int mode, int Hs, int Ws,
                                                         float* __restrict__ G, uint8_t* __restrict__ V) {
    const int64_t hw = (int64_t)Hs * Ws;
    if constexpr (ALL) {
        const int o = blockIdx.z;
        oy = o / s;
        ox = o - oy * s;
        G += (int64_t)o * D * hw;
        if (V) V += (int64_t)o * hw;
    }
    const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (p0 >= hw) return;
    Src src[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t p = p0 + k < hw ? p0 + k : hw - 1;
        src[k] = source_of<I>(p, Ws, H, W, Hf, Wf, s, oy, ox, mode);
    }
    const int d0 = blockIdx.y * kChanChunk;
    const int d1 = d0 + kChanChunk < D ? d0 + kChanChunk : D;
    const int64_t plane = (int64_t)Hf * Wf;
    // Shared sources: the four pixels read the same two source rows and at most
    // three consecutive source columns, so six loads per channel serve all four
    // samples (same operands, same arithmetic as sample()).
    const int xa = src[0].x0;
    bool shared = true;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        shared = shared && src[k].valid && src[k].y0 == src[0].y0 && src[k].y1 == src[0].y1 &&
                 src[k].x0 >= xa && src[k].x1 <= xa + 2;
    if (shared) {
        int o0[4], o1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { o0[k] = src[k].x0 - xa; o1[k] = src[k].x1 - xa; }
        const int c1 = xa + 1 < Wf ? xa + 1 : Wf - 1, c2 = xa + 2 < Wf ? xa + 2 : Wf - 1;
        const int ra = src[0].y0 * Wf, rb = src[0].y1 * Wf;
        auto pick3 = [](float a, float b, float c, int i) { return i == 0 ? a : (i == 1 ? b : c); };
        for (int d = d0; d < d1; ++d) {
            const float* Pd = P + d * plane;
            const float a0 = Pd[ra + xa], a1 = Pd[ra + c1], a2 = Pd[ra + c2];
            const float b0 = Pd[rb + xa], b1 = Pd[rb + c1], b2 = Pd[rb + c2];
            f32x4_t v;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float p00 = pick3(a0, a1, a2, o0[k]), p01 = pick3(a0, a1, a2, o1[k]);
                const float p10 = pick3(b0, b1, b2, o0[k]), p11 = pick3(b0, b1, b2, o1[k]);
                const float top = p00 + src[k].wx * (p01 - p00);
                const float bot = p10 + src[k].wx * (p11 - p10);
                v[k] = top + src[k].wy * (bot - top);
            }
            float* out = G + (int64_t)d * hw + p0;
            if (VEC) {
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4_t*>(out));
            } else {
                for (int k = 0; k < 4 && p0 + k < hw; ++k) __builtin_nontemporal_store(v[k], out + k);
            }
        }
    } else {
        for (int d = d0; d < d1; ++d) {
            const float* Pd = P + d * plane;
            f32x4_t v = {sample(Pd, Wf, src[0]), sample(Pd, Wf, src[1]), sample(Pd, Wf, src[2]),
                         sample(Pd, Wf, src[3])};
            float* out = G + (int64_t)d * hw + p0;
            if (VEC) {
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4_t*>(out));
            } else {
                for (int k = 0; k < 4 && p0 + k < hw; ++k) __builtin_nontemporal_store(v[k], out + k);
            }
        }
    }
    if (V && blockIdx.y == 0) {
        for (int k = 0; k < 4 && p0 + k < hw; ++k) V[p0 + k] = src[k].valid ? 1 : 0;
    }
}

}  // namespace xgs

using namespace xgs;

// Checks shared by both entry points; fills the grid shape and launch mode.
static xgs_status grid_setup(const char* who, const float* P, int32_t D, int32_t Hf, int32_t Wf, int32_t H,
                             int32_t W, int32_t stride, int32_t mode, const float* G, int64_t* hw_out, int* Hs_out,
                             int* Ws_out, bool* i32_out) {
    const std::string w = who;
    if (D < 0 || Hf < 1 || Wf < 1 || H < 1 || W < 1 || stride < 1)
        return fail(XGS_ERR_INVALID_ARG, w + ": sizes must be positive (D >= 0)");
    if (mode != XGS_GRID_BILINEAR && mode != XGS_GRID_NEAREST) return fail(XGS_ERR_INVALID_ARG, w + ": unknown mode");
    if ((int64_t)Hf * Wf * D >= (int64_t(1) << 31))
        return fail(XGS_ERR_UNSUPPORTED, w + ": feature map above 2^31 elements");
    const int Hs = (H + stride - 1) / stride, Ws = (W + stride - 1) / stride;
    if (D > 0 && (!P || !G)) return fail(XGS_ERR_INVALID_ARG, w + ": null P or G");
    if ((D + kChanChunk - 1) / kChanChunk > 65535) return fail(XGS_ERR_UNSUPPORTED, w + ": too many channels");
    // 32-bit source arithmetic when every intermediate fits: p < hw, u < H + stride,
    // u (Hf - 1) and v (Wf - 1), and the doubled remainders
    const int64_t hw = (int64_t)Hs * Ws;
    const int64_t lim = (int64_t(1) << 30);
    *i32_out = hw < lim && (int64_t)(H + stride) * Hf < lim && (int64_t)(W + stride) * Wf < lim;
    *hw_out = hw;
    *Hs_out = Hs;
    *Ws_out = Ws;
    return XGS_OK;
}

template <bool ALL>
static void grid_launch(const float* P, int32_t D, int32_t Hf, int32_t Wf, int32_t H, int32_t W, int32_t stride,
                        int32_t off_y, int32_t off_x, int32_t mode, int Hs, int Ws, int64_t hw, bool i32, float* G,
                        uint8_t* V, unsigned grids, hipStream_t st) {
    const bool vec = (hw % 4 == 0) && aligned(G, 16);
    const unsigned bx = (unsigned)((hw + 1023) / 1024);
    const unsigned by = (unsigned)(D > 0 ? (D + kChanChunk - 1) / kChanChunk : 1);
    const dim3 grid(bx, by, grids);
#define XGS_GS_LAUNCH(V4, I)                                                                               \
    hipLaunchKernelGGL((grid_sample_kernel<V4, I, ALL>), grid, dim3(256), 0, st, P, D, Hf, Wf, H, W, stride, \
                       off_y, off_x, mode, Hs, Ws, G, V)
    if (vec && i32) XGS_GS_LAUNCH(true, int32_t);
    else if (vec) XGS_GS_LAUNCH(true, int64_t);
    else if (i32) XGS_GS_LAUNCH(false, int32_t);
    else XGS_GS_LAUNCH(false, int64_t);
#undef XGS_GS_LAUNCH
}

extern "C" xgs_status xgs_grid_sample(const float* P, int32_t D, int32_t Hf, int32_t Wf, int32_t H,
                                      int32_t W, int32_t stride, int32_t off_y, int32_t off_x,
                                      int32_t mode, float* G, uint8_t* V, xgs_stream_t stream) {
    clear_error();
    int64_t hw;
    int Hs, Ws;
    bool i32;
    if (xgs_status s = grid_setup("xgs_grid_sample", P, D, Hf, Wf, H, W, stride, mode, G, &hw, &Hs, &Ws, &i32))
        return s;
    if (off_y < 0 || off_x < 0 || off_y >= stride || off_x >= stride)
        return fail(XGS_ERR_INVALID_ARG, "xgs_grid_sample: offsets must lie in [0, stride)");
    if (D == 0 && !V) return XGS_OK;
    grid_launch<false>(P, D, Hf, Wf, H, W, stride, off_y, off_x, mode, Hs, Ws, hw, i32, G, V, 1u,
                       (hipStream_t)stream);
    return check_launch("xgs_grid_sample");
}

extern "C" xgs_status xgs_grid_sample_offsets(const float* P, int32_t D, int32_t Hf, int32_t Wf, int32_t H,
                                              int32_t W, int32_t stride, int32_t mode, float* G, uint8_t* V,
                                              xgs_stream_t stream) {
    clear_error();
    if (stride > XGS_GRID_MAX_STRIDE)
        return fail(XGS_ERR_UNSUPPORTED, "xgs_grid_sample_offsets: stride above XGS_GRID_MAX_STRIDE");
    int64_t hw;
    int Hs, Ws;
    bool i32;
    if (xgs_status s = grid_setup("xgs_grid_sample_offsets", P, D, Hf, Wf, H, W, stride, mode, G, &hw, &Hs, &Ws,
                                  &i32))
        return s;
    if (D == 0 && !V) return XGS_OK;
    grid_launch<true>(P, D, Hf, Wf, H, W, stride, 0, 0, mode, Hs, Ws, hw, i32, G, V,
                      (unsigned)(stride * stride), (hipStream_t)stream);
    return check_launch("xgs_grid_sample_offsets");
}
