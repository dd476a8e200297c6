// Semantic phase: mixture weights, per-pixel decode and the masked grid loss.
//
// Sec. 3.2.2 (online VQ module): every Gaussian carries logits z_i over the L
// codewords of the shared codebook E [L][D]; its mixture weights are
// w_i = softmax(z_i) and its decoded feature is E^T w_i.  The weights are
// rendered as the semantic channels (a3), and App. E decodes per pixel,
// G^(x) = E^T w(x).  App. D (masked loss evaluation) compares G^ with the grid
// targets G* under the validity mask V:
//   L = lambda [ (1/n) sum_{x valid} (1 - cos(G^(x), G*(x)))
//              + (1/(n D)) sum_{x valid} |G^(x) - G*(x)|_1 ],
// n = number of valid pixels, cos(a, b) = <a, b> / max(|a||b|, 1e-8).
// The geometry is frozen in this phase (Sec. 3.2.2, parallelized pipeline),
// so the backward is the feature-only pass of a4 followed by the softmax.
#include <algorithm>
#include <cstdint>

#include "common.h"

namespace xgs {

constexpr float kCosEps = 1e-8f;
constexpr int SEM_PIX = 64;  // grid pixels per workgroup (one per lane)

// ------------------------------------------------------------------ softmax
template <int L>
__global__ void __launch_bounds__(256) sem_softmax_kernel(const float* __restrict__ z, int64_t N,
                                                         float* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    float v[L];
    const float4* zr = reinterpret_cast<const float4*>(z + i * L);
#pragma unroll
    for (int k = 0; k < L / 4; ++k) {
        const float4 q = zr[k];
        v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
    }
    float m = v[0];
#pragma unroll
    for (int k = 1; k < L; ++k) m = fmaxf(m, v[k]);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        v[k] = expf(v[k] - m);
        s += v[k];
    }
    const float inv = 1.f / s;
    float4* wr = reinterpret_cast<float4*>(w + i * L);
#pragma unroll
    for (int k = 0; k < L / 4; ++k)
        wr[k] = make_float4(v[4 * k] * inv, v[4 * k + 1] * inv, v[4 * k + 2] * inv, v[4 * k + 3] * inv);
}

// dL/dz = w (dL/dw - <dL/dw, w>)
template <int L>
__global__ void __launch_bounds__(256) sem_softmax_bwd_kernel(const float* __restrict__ w,
                                                             const float* __restrict__ dw, int64_t N,
                                                             float* __restrict__ dz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    float wv[L], gv[L];
    const float4* wr = reinterpret_cast<const float4*>(w + i * L);
    const float4* gr = reinterpret_cast<const float4*>(dw + i * L);
#pragma unroll
    for (int k = 0; k < L / 4; ++k) {
        const float4 a = wr[k], b = gr[k];
        wv[4 * k] = a.x; wv[4 * k + 1] = a.y; wv[4 * k + 2] = a.z; wv[4 * k + 3] = a.w;
        gv[4 * k] = b.x; gv[4 * k + 1] = b.y; gv[4 * k + 2] = b.z; gv[4 * k + 3] = b.w;
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < L; ++k) s += gv[k] * wv[k];
    float4* out = reinterpret_cast<float4*>(dz + i * L);
#pragma unroll
    for (int k = 0; k < L / 4; ++k)
        out[k] = make_float4(wv[4 * k] * (gv[4 * k] - s), wv[4 * k + 1] * (gv[4 * k + 1] - s),
                             wv[4 * k + 2] * (gv[4 * k + 2] - s), wv[4 * k + 3] * (gv[4 * k + 3] - s));
}

// ------------------------------------------------------------- valid count
__global__ void __launch_bounds__(256) sem_count_kernel(const uint8_t* __restrict__ V, int64_t P,
                                                       int* __restrict__ count) {
    int c = 0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256)
        c += V[p] != 0;
    for (int k = 32; k >= 1; k >>= 1) c += __shfl_xor(c, k, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);  // integer sum: order-independent
}

__global__ void sem_zero_kernel(int* __restrict__ count) { *count = 0; }
__global__ void sem_fill_count_kernel(int* __restrict__ count, int v) { *count = v; }

// ----------------------------------------------------------- decode + loss
// One workgroup: 64 consecutive grid pixels (lane = pixel) x 4 wavefronts,
// wavefront q covering codeword columns [q D/4, (q+1) D/4).  E^T sits in LDS
// as [D][L] (column d of E contiguous), read as broadcasts.  Pass 1 sums, per
// pixel, <a, b>, |a|^2, |b|^2 and |a - b|_1 over the wavefront's columns
// (a = G^, b = G*); the four partials are added in wavefront order.  Pass 2
// recomputes a column by column, forms
//   g_d = lambda [ -(b_d / den - [den > eps] cos a_d / |a|^2) / n + sign(a_d - b_d) / (n D) ]
// and accumulates dL/dw_l = sum_d E[l][d] g_d, again added in wavefront
// order.  The loss of the workgroup's valid pixels goes to partial[block].
template <int L>
__global__ void __launch_bounds__(256) sem_loss_kernel(const float* __restrict__ wmap, int64_t P, int D,
                                                      const float* __restrict__ E,
                                                      const float* __restrict__ Gs,
                                                      const uint8_t* __restrict__ V, float lambda,
                                                      const int* __restrict__ count,
                                                      float* __restrict__ d_out, float* __restrict__ partial) {
    extern __shared__ __align__(16) float sh[];
    float* et = sh;                                   // [D][L]
    float* red = sh + (size_t)D * L;                  // [SEM_PIX][L] (pass 2), [4][SEM_PIX] x 4 (pass 1)
    const int t = threadIdx.x, lane = t & 63;
    const int q = __builtin_amdgcn_readfirstlane(t >> 6);
    for (int e = t; e < L * D; e += 256) {
        const int l = e / D, d = e - l * D;
        et[d * L + l] = E[e];
    }
    const int64_t pix = (int64_t)blockIdx.x * SEM_PIX + lane;
    const bool in = pix < P;
    const int64_t pc = in ? pix : P - 1;
    const bool valid = in && (V == nullptr || V[pc] != 0);
    float w[L];
#pragma unroll
    for (int l = 0; l < L; ++l) w[l] = wmap[(size_t)(4 + l) * P + pc];
    __syncthreads();

    const int dq = D / 4, d0 = q * dq;
    float dot = 0.f, na = 0.f, nb = 0.f, l1 = 0.f;
    for (int d = d0; d < d0 + dq; ++d) {
        const float4* col = reinterpret_cast<const float4*>(et + (size_t)d * L);
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < L / 4; ++k) {
            const float4 e4 = col[k];
            a += w[4 * k] * e4.x + w[4 * k + 1] * e4.y + w[4 * k + 2] * e4.z + w[4 * k + 3] * e4.w;
        }
        const float b = Gs[(size_t)d * P + pc];
        dot += a * b;
        na += a * a;
        nb += b * b;
        l1 += fabsf(a - b);
    }
    float* r1 = red;  // [4 sums][4 waves][SEM_PIX]
    r1[(0 * 4 + q) * SEM_PIX + lane] = dot;
    r1[(1 * 4 + q) * SEM_PIX + lane] = na;
    r1[(2 * 4 + q) * SEM_PIX + lane] = nb;
    r1[(3 * 4 + q) * SEM_PIX + lane] = l1;
    __syncthreads();
    float s4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        s4[k] = ((r1[(k * 4 + 0) * SEM_PIX + lane] + r1[(k * 4 + 1) * SEM_PIX + lane]) +
                 r1[(k * 4 + 2) * SEM_PIX + lane]) + r1[(k * 4 + 3) * SEM_PIX + lane];
    __syncthreads();
    const int n = *count;
    const float fn = (float)(n > 0 ? n : 1);
    const float nrm_a = sqrtf(s4[1]), nrm_b = sqrtf(s4[2]);
    const float prod = nrm_a * nrm_b;
    const float den = fmaxf(prod, kCosEps);
    const float cosv = s4[0] / den;
    // g_d = k1 b_d + k2 a_d + k3 sign(a_d - b_d)
    const bool live = valid && n > 0;
    const float k1 = live ? -lambda / (fn * den) : 0.f;
    const float k2 = (live && prod > kCosEps && s4[1] > 0.f) ? lambda * cosv / (fn * s4[1]) : 0.f;
    const float k3 = live ? lambda / (fn * (float)D) : 0.f;
    if (q == 0) {
        // this workgroup's share of the loss, summed over its pixels in lane order
        float v = live ? lambda * ((1.f - cosv) / fn + s4[3] / (fn * (float)D)) : 0.f;
        for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k, 64);
        if (lane == 0) partial[blockIdx.x] = v;
    }

    float acc[L];
#pragma unroll
    for (int l = 0; l < L; ++l) acc[l] = 0.f;
    if (live) {
        for (int d = d0; d < d0 + dq; ++d) {
            const float4* col = reinterpret_cast<const float4*>(et + (size_t)d * L);
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < L / 4; ++k) {
                const float4 e4 = col[k];
                a += w[4 * k] * e4.x + w[4 * k + 1] * e4.y + w[4 * k + 2] * e4.z + w[4 * k + 3] * e4.w;
            }
            const float b = Gs[(size_t)d * P + pc];
            const float df = a - b;
            const float sg = df > 0.f ? 1.f : (df < 0.f ? -1.f : 0.f);
            const float gd = k1 * b + k2 * a + k3 * sg;
#pragma unroll
            for (int k = 0; k < L / 4; ++k) {
                const float4 e4 = col[k];
                acc[4 * k] += gd * e4.x;
                acc[4 * k + 1] += gd * e4.y;
                acc[4 * k + 2] += gd * e4.z;
                acc[4 * k + 3] += gd * e4.w;
            }
        }
    }
    // add the four wavefronts' partial sums in wavefront order
    float* r2 = red;  // [SEM_PIX][L + 1]
    for (int k = 0; k < 4; ++k) {
        if (q == k)
#pragma unroll
            for (int l = 0; l < L; ++l) r2[lane * (L + 1) + l] = (k == 0 ? 0.f : r2[lane * (L + 1) + l]) + acc[l];
        __syncthreads();
    }
    // write dL/dw (channels 4..), zero the colour and depth channels
    for (int e = t; e < SEM_PIX * (4 + L); e += 256) {
        const int c = e / SEM_PIX, px = e - c * SEM_PIX;
        const int64_t p = (int64_t)blockIdx.x * SEM_PIX + px;
        if (p < P) d_out[(size_t)c * P + p] = c < 4 ? 0.f : r2[px * (L + 1) + (c - 4)];
    }
}

// Sums the per-workgroup losses in a fixed order.
__global__ void __launch_bounds__(256) sem_loss_total_kernel(const float* __restrict__ partial, int nb,
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

static bool sem_l_ok(int L) { return L == 4 || L == 8 || L == 16 || L == 32 || L == 64; }

}  // namespace xgs

using namespace xgs;

#define XGS_SEM_DISPATCH(L, call) \
    switch (L) {                  \
        case 4: call(4); break;   \
        case 8: call(8); break;   \
        case 16: call(16); break; \
        case 32: call(32); break; \
        default: call(64); break; \
    }

extern "C" xgs_status xgs_semantic_softmax(const float* z, int64_t N, int32_t L, float* w, xgs_stream_t stream) {
    clear_error();
    if (N < 0 || !sem_l_ok(L)) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_softmax: L must be 4, 8, 16, 32 or 64");
    if (N == 0) return XGS_OK;
    if (!z || !w) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_softmax: null pointer");
    if (!aligned(z, 16) || !aligned(w, 16)) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_softmax: 16-byte alignment");
    const dim3 grid((unsigned)((N + 255) / 256));
#define XGS_SM(LL) hipLaunchKernelGGL(sem_softmax_kernel<LL>, grid, dim3(256), 0, (hipStream_t)stream, z, N, w)
    XGS_SEM_DISPATCH(L, XGS_SM)
#undef XGS_SM
    return check_launch("xgs_semantic_softmax");
}

extern "C" xgs_status xgs_semantic_softmax_bwd(const float* w, const float* dw, int64_t N, int32_t L, float* dz,
                                               xgs_stream_t stream) {
    clear_error();
    if (N < 0 || !sem_l_ok(L)) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_softmax_bwd: L must be 4, 8, 16, 32 or 64");
    if (N == 0) return XGS_OK;
    if (!w || !dw || !dz) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_softmax_bwd: null pointer");
    if (!aligned(w, 16) || !aligned(dw, 16) || !aligned(dz, 16))
        return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_softmax_bwd: 16-byte alignment");
    const dim3 grid((unsigned)((N + 255) / 256));
#define XGS_SMB(LL) hipLaunchKernelGGL(sem_softmax_bwd_kernel<LL>, grid, dim3(256), 0, (hipStream_t)stream, w, dw, N, dz)
    XGS_SEM_DISPATCH(L, XGS_SMB)
#undef XGS_SMB
    return check_launch("xgs_semantic_softmax_bwd");
}

static size_t sem_blocks(int64_t P) { return (size_t)((P + SEM_PIX - 1) / SEM_PIX); }

extern "C" size_t xgs_semantic_loss_workspace(int32_t Hs, int32_t Ws) {
    if (Hs < 1 || Ws < 1) return 0;
    Carve c(nullptr);
    c.take<int>(1);
    c.take<float>(sem_blocks((int64_t)Hs * Ws));
    return c.total();
}

extern "C" xgs_status xgs_semantic_loss(const float* wmap, int32_t L, int32_t Hs, int32_t Ws, const float* E,
                                        int32_t D, const float* Gstar, const uint8_t* V, float lambda,
                                        float* d_out, float* loss, void* ws, size_t ws_bytes,
                                        xgs_stream_t stream) {
    clear_error();
    if (!sem_l_ok(L)) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_loss: L must be 4, 8, 16, 32 or 64");
    if (Hs < 1 || Ws < 1 || D < 4 || D % 4 != 0)
        return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_loss: need Hs, Ws >= 1 and D a positive multiple of 4");
    const size_t lds = ((size_t)D * L + (size_t)SEM_PIX * (L + 1) + 16 * SEM_PIX) * sizeof(float);
    if (lds > 160 * 1024) return fail(XGS_ERR_UNSUPPORTED, "xgs_semantic_loss: L x D too large for LDS");
    if (!wmap || !E || !Gstar || !d_out || !loss) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_loss: null pointer");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_loss: workspace must be 256-byte aligned");
    const int64_t P = (int64_t)Hs * Ws;
    Carve c(ws);
    int* count = c.take<int>(1);
    float* partial = c.take<float>(sem_blocks(P));
    if (!ws || ws_bytes < c.total()) return fail(XGS_ERR_CAPACITY, "xgs_semantic_loss: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(sem_zero_kernel, dim3(1), dim3(1), 0, st, count);
    if (V) {
        const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 1024);
        hipLaunchKernelGGL(sem_count_kernel, dim3(g), dim3(256), 0, st, V, P, count);
    } else {
        hipLaunchKernelGGL(sem_fill_count_kernel, dim3(1), dim3(1), 0, st, count, (int)std::min<int64_t>(P, INT32_MAX));
    }
    const unsigned nb = (unsigned)sem_blocks(P);
#define XGS_SL(LL)                                                                                              \
    {                                                                                                           \
        if (hipFuncSetAttribute((const void*)sem_loss_kernel<LL>, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                                (int)lds) != hipSuccess)                                                        \
            return fail(XGS_ERR_HIP, "xgs_semantic_loss: cannot reserve LDS");                                  \
        hipLaunchKernelGGL(sem_loss_kernel<LL>, dim3(nb), dim3(256), lds, st, wmap, P, D, E, Gstar, V, lambda,  \
                           count, d_out, partial);                                                              \
    }
    XGS_SEM_DISPATCH(L, XGS_SL)
#undef XGS_SL
    hipLaunchKernelGGL(sem_loss_total_kernel, dim3(1), dim3(256), 0, st, partial, (int)nb, loss);
    return check_launch("xgs_semantic_loss");
}
