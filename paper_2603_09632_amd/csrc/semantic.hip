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
#include "wave.h"

namespace xgs {

constexpr float kCosEps = 1e-8f;
constexpr int SEM_NPT = 2;              // 16-pixel tiles per wavefront (decode + loss)
constexpr int SEM_PIX = 64 * SEM_NPT;   // grid pixels per workgroup (decode + loss)

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
// One workgroup: 64 SEM_NPT consecutive grid pixels, wavefront q taking
// SEM_NPT tiles of 16 pixels and every codeword column (two tiles per wave:
// each G* plane is then read in 128-byte runs; measured 0.39 -> 0.35 ms at
// 640 x 480, D = 512, against one tile, and four tiles was slower).  The decode F = W E (W the
// pixels' mixture weights, E the L x D codebook) and the gradient product
// dL/dW = g E^T both run on v_mfma_f32_16x16x4_f32 (FP32 products, FP32
// sums), in transposed form so that no operand changes lanes:
//   F^T tile (16 columns d x 16 pixels p) = sum over codes of E^T W^T, with
//     A[d][code] = E[code][d] (from L2) and B[code][p] = W[p][code] (held in
//     registers for the whole kernel); the accumulator puts column
//     d = 16 mt + 4 (lane / 16) + r and pixel p = lane % 16 in lane `lane`,
//     element r;
//   dL/dW^T (16 codes x 16 pixels) += sum over d of E g^T, contracting over
//     d = 16 mt + 4 k + r in step (mt, r), k = lane / 16: then the B operand
//     g[p][d] is exactly the lane's own accumulator element r, and A is the
//     float4 E[code][16 mt + 4 (lane / 16) .. + 3].
// Pass 1 sums, per pixel, <a, b>, |a|^2, |b|^2 and |a - b|_1 (a = G^, b = G*)
// over the lane's columns, then over the four lanes holding the pixel (lane
// swaps at distance 32 and 16: every lane ends with the same bits).  Pass 2
// recomputes the tiles, forms
//   g_d = lambda [ -(b_d / den - [den > eps] cos a_d / |a|^2) / n + sign(a_d - b_d) / (n D) ]
// and accumulates dL/dw.  The loss of the workgroup's valid pixels goes to
// partial[block], summed in a fixed order.
template <int L>
__global__ void __launch_bounds__(256) sem_loss_kernel(const float* __restrict__ wmap, int64_t P, int D,
                                                      const float* __restrict__ E,
                                                      const float* __restrict__ Gs,
                                                      const uint8_t* __restrict__ V, float lambda,
                                                      const int* __restrict__ count,
                                                      float* __restrict__ d_out, float* __restrict__ partial) {
    constexpr int KS = L / 4;             // code steps of the decode
    constexpr int CT = (L + 15) / 16;     // code tiles of the gradient
    constexpr int NP = SEM_NPT;           // 16-pixel tiles per wavefront
    __shared__ float wsum[4];
    const int t = threadIdx.x, lane = t & 63, hi = lane >> 4, lo = lane & 15;
    const int q = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t p0 = (int64_t)blockIdx.x * SEM_PIX + 16 * NP * q;
    int64_t pix[NP], pc[NP];
    bool in[NP], valid[NP];
    float wb[NP][KS];  // B operand of the decode: W[p][code = 4 ks + hi]
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        pix[j] = p0 + 16 * j + lo;  // this lane's pixel in tile j (B and accumulator column)
        in[j] = pix[j] < P;
        pc[j] = in[j] ? pix[j] : P - 1;
        valid[j] = in[j] && (V == nullptr || V[pc[j]] != 0);
#pragma unroll
        for (int k = 0; k < KS; ++k) wb[j][k] = wmap[(size_t)(4 + 4 * k + hi) * P + pc[j]];
    }
    const int MT = (D + 15) / 16;

    // Operands of column tile mt, loaded one tile ahead of their use: the
    // decode's A values (E^T) and the targets b (G*).
    struct Tile {
        float ea[KS];
        float b[NP][4];
    };
    auto load_tile = [&](int mt, Tile& o) {
        const int d = 16 * mt + lo;
#pragma unroll
        for (int k = 0; k < KS; ++k) o.ea[k] = d < D ? E[(size_t)(4 * k + hi) * D + d] : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int dr = 16 * mt + 4 * hi + r;
#pragma unroll
            for (int j = 0; j < NP; ++j) o.b[j][r] = dr < D ? Gs[(size_t)dr * P + pc[j]] : 0.f;
        }
    };
    auto decode = [&](const Tile& o, int j) {
        f32x4_t f = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < KS; ++k) f = __builtin_amdgcn_mfma_f32_16x16x4f32(o.ea[k], wb[j][k], f, 0, 0, 0);
        return f;
    };

    float s4[NP][4];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) s4[j][k] = 0.f;
    {
        Tile cur, nxt;
        load_tile(0, cur);
        for (int mt = 0; mt < MT; ++mt) {
            if (mt + 1 < MT) load_tile(mt + 1, nxt);
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const f32x4_t f = decode(cur, j);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float bv = cur.b[j][r];
                    s4[j][0] += f[r] * bv;
                    s4[j][1] += f[r] * f[r];
                    s4[j][2] += bv * bv;
                    s4[j][3] += fabsf(f[r] - bv);
                }
            }
            if (mt + 1 < MT) cur = nxt;
        }
    }
    const int n = *count;
    const float fn = (float)(n > 0 ? n : 1);
    float k1[NP], k2[NP], k3[NP], lj[NP];
    bool live[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float x, y;
            xlane_swap<32>(s4[j][k], s4[j][k], x, y);
            s4[j][k] = x + y;
            xlane_swap<16>(s4[j][k], s4[j][k], x, y);
            s4[j][k] = x + y;
        }
        const float nrm_a = sqrtf(s4[j][1]), nrm_b = sqrtf(s4[j][2]);
        const float prod = nrm_a * nrm_b;
        const float den = fmaxf(prod, kCosEps);
        const float cosv = s4[j][0] / den;
        // g_d = k1 b_d + k2 a_d + k3 sign(a_d - b_d)
        live[j] = valid[j] && n > 0;
        k1[j] = live[j] ? -lambda / (fn * den) : 0.f;
        k2[j] = (live[j] && prod > kCosEps && s4[j][1] > 0.f) ? lambda * cosv / (fn * s4[j][1]) : 0.f;
        k3[j] = live[j] ? lambda / (fn * (float)D) : 0.f;
        lj[j] = live[j] ? lambda * ((1.f - cosv) / fn + s4[j][3] / (fn * (float)D)) : 0.f;
    }
    {
        // this workgroup's share of the loss: pixels in order within a tile
        // (lanes 0..15), tiles in order, then the waves in order
        float wtot = 0.f;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            float v = hi == 0 ? lj[j] : 0.f;
            v += xlane_dpp<8>(v);
            v += xlane_dpp<4>(v);
            v += xlane_dpp<2>(v);
            v += xlane_dpp<1>(v);
            wtot += v;
        }
        if (lane == 0) wsum[q] = wtot;
    }

    f32x4_t acc[NP][CT];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[j][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    bool any = false;
#pragma unroll
    for (int j = 0; j < NP; ++j) any = any || live[j];
    if (__ballot(any) != 0ull) {
        Tile cur, nxt;
        float4 ec[CT], en[CT];  // gradient A operands: E[16 c + lo][16 mt + 4 hi .. + 3]
        auto load_e4 = [&](int mt, float4 (&o)[CT]) {
            const int d4 = 16 * mt + 4 * hi;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int code = 16 * c + lo;
                o[c] = (code < L && d4 < D) ? *reinterpret_cast<const float4*>(E + (size_t)code * D + d4)
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        load_tile(0, cur);
        load_e4(0, ec);
        for (int mt = 0; mt < MT; ++mt) {
            if (mt + 1 < MT) {
                load_tile(mt + 1, nxt);
                load_e4(mt + 1, en);
            }
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const f32x4_t f = decode(cur, j);
                float gd[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float df = f[r] - cur.b[j][r];
                    const float sg = df > 0.f ? 1.f : (df < 0.f ? -1.f : 0.f);
                    gd[r] = k1[j] * cur.b[j][r] + k2[j] * f[r] + k3[j] * sg;
                }
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ec[c].x, gd[0], acc[j][c], 0, 0, 0);
                    acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ec[c].y, gd[1], acc[j][c], 0, 0, 0);
                    acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ec[c].z, gd[2], acc[j][c], 0, 0, 0);
                    acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ec[c].w, gd[3], acc[j][c], 0, 0, 0);
                }
            }
            if (mt + 1 < MT) {
                cur = nxt;
#pragma unroll
                for (int c = 0; c < CT; ++c) ec[c] = en[c];
            }
        }
    }
    // acc[j][c][r]: code 16 c + 4 hi + r, pixel tile j column lo
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        if (!in[j]) continue;
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int code = 16 * c + 4 * hi + r;
                if (code < L) d_out[(size_t)(4 + code) * P + pix[j]] = acc[j][c][r];
            }
        if (hi == 0)
#pragma unroll
            for (int c = 0; c < 4; ++c) d_out[(size_t)c * P + pix[j]] = 0.f;
    }
    __syncthreads();
    if (t == 0) partial[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
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
    if (!wmap || !E || !Gstar || !d_out || !loss) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_loss: null pointer");
    if (!aligned(E, 16)) return fail(XGS_ERR_INVALID_ARG, "xgs_semantic_loss: E must be 16-byte aligned");
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
#define XGS_SL(LL)                                                                                             \
    hipLaunchKernelGGL(sem_loss_kernel<LL>, dim3(nb), dim3(256), 0, st, wmap, P, D, E, Gstar, V, lambda, count, \
                       d_out, partial)
    XGS_SEM_DISPATCH(L, XGS_SL)
#undef XGS_SL
    hipLaunchKernelGGL(sem_loss_total_kernel, dim3(1), dim3(256), 0, st, partial, (int)nb, loss);
    return check_launch("xgs_semantic_loss");
}
