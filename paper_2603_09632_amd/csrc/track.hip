// Tracking loss (Eq. (tracking), Eq. (loss_track)): the pose is refined
// against the colour image and the depth map with the map frozen.
//   L = (1/(3 P)) sum_x sum_{c<3} |I^_c(x) - I_c(x)|
//     + lambda_d (1/P_D) sum_{x: D(x) > 0} |D^(x) - D(x)|,
// P grid pixels, P_D pixels with a depth value (no depth term when P_D = 0),
// d|t|/dt = sign(t) with sign(0) = 0.  The kernel writes dL/dout for every
// channel (zero on the semantic ones), the input of xgs_render_bwd.
#include <algorithm>

#include "common.h"

namespace xgs {

__global__ void __launch_bounds__(256) trk_count_kernel(const float* __restrict__ depth, int64_t P,
                                                       int* __restrict__ count) {
    int c = 0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256)
        c += depth[p] > 0.f;
    for (int k = 32; k >= 1; k >>= 1) c += __shfl_xor(c, k, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);  // integer sum: order-independent
}

__global__ void trk_zero_kernel(int* __restrict__ count) { *count = 0; }

__device__ __forceinline__ float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// One thread per grid pixel; each workgroup sums its pixels' losses in a
// fixed order into partial[block].
__global__ void __launch_bounds__(256) trk_loss_kernel(const float* __restrict__ out, int C, int64_t P,
                                                      const float* __restrict__ image,
                                                      const float* __restrict__ depth, float lambda_d,
                                                      const int* __restrict__ count, float* __restrict__ d_out,
                                                      float* __restrict__ partial) {
    __shared__ float red[4];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float v = 0.f;
    if (p < P) {
        const float inv3p = 1.f / (3.f * (float)P);
        float photo = 0.f;
        for (int c = 0; c < 3; ++c) {
            const float df = out[(size_t)c * P + p] - image[(size_t)c * P + p];
            photo += fabsf(df);
            d_out[(size_t)c * P + p] = sgn(df) * inv3p;
        }
        v = photo * inv3p;
        float gd = 0.f;
        const int nd = depth ? *count : 0;
        if (nd > 0 && lambda_d != 0.f && depth[p] > 0.f) {
            const float dd = out[(size_t)3 * P + p] - depth[p];
            const float s = lambda_d / (float)nd;
            v += s * fabsf(dd);
            gd = s * sgn(dd);
        }
        d_out[(size_t)3 * P + p] = gd;
        for (int c = 4; c < C; ++c) d_out[(size_t)c * P + p] = 0.f;
    }
    for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) trk_total_kernel(const float* __restrict__ partial, int nb,
                                                       float* __restrict__ loss) {
    __shared__ float r[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < nb; i += 256) s += partial[i];
    r[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) r[threadIdx.x] += r[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = r[0];
}

static size_t trk_blocks(int64_t P) { return (size_t)((P + 255) / 256); }

}  // namespace xgs

using namespace xgs;

extern "C" size_t xgs_tracking_loss_workspace(int32_t Hs, int32_t Ws) {
    if (Hs < 1 || Ws < 1) return 0;
    Carve c(nullptr);
    c.take<int>(1);
    c.take<float>(trk_blocks((int64_t)Hs * Ws));
    return c.total();
}

extern "C" xgs_status xgs_tracking_loss(const float* out, int32_t C, int32_t Hs, int32_t Ws, const float* image,
                                        const float* depth, float lambda_d, float* d_out, float* loss, void* ws,
                                        size_t ws_bytes, xgs_stream_t stream) {
    clear_error();
    if (C < 4 || Hs < 1 || Ws < 1) return fail(XGS_ERR_INVALID_ARG, "xgs_tracking_loss: need C >= 4, Hs, Ws >= 1");
    if (!out || !image || !d_out || !loss) return fail(XGS_ERR_INVALID_ARG, "xgs_tracking_loss: null pointer");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_tracking_loss: workspace must be 256-byte aligned");
    const int64_t P = (int64_t)Hs * Ws;
    Carve cv(ws);
    int* count = cv.take<int>(1);
    float* partial = cv.take<float>(trk_blocks(P));
    if (!ws || ws_bytes < cv.total()) return fail(XGS_ERR_CAPACITY, "xgs_tracking_loss: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(trk_zero_kernel, dim3(1), dim3(1), 0, st, count);
    if (depth) {
        const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 1024);
        hipLaunchKernelGGL(trk_count_kernel, dim3(g), dim3(256), 0, st, depth, P, count);
    }
    const unsigned nb = (unsigned)trk_blocks(P);
    hipLaunchKernelGGL(trk_loss_kernel, dim3(nb), dim3(256), 0, st, out, C, P, image, depth, lambda_d, count, d_out,
                       partial);
    hipLaunchKernelGGL(trk_total_kernel, dim3(1), dim3(256), 0, st, partial, (int)nb, loss);
    return check_launch("xgs_tracking_loss");
}
