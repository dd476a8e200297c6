// a6/a7: nearest-codeword assignment and the EMA codebook update of the
// online VQ module (Sec. 3.2.2, Eq. (ema_update)).
//
// Assignment, BF16 form: the distance contraction is the only dense GEMM on
// the hot path, so it runs on MFMA.  A workgroup keeps 64 rows of X resident
// in LDS as bf16 and its four wavefronts sweep the codebook (bf16 shadow read
// straight from L2 into registers), each computing a 64-row x 128-codeword
// tile per step with v_mfma_f32_32x32x16_bf16.  The accumulators start at
// -||e^||^2/2, so each output is x^.e^ - ||e^||^2/2 and the nearest codeword
// is the largest.  Every lane keeps a running top-4 per row; the candidates
// are merged through LDS and rescored with the direct FP32 form sum (x - e)^2.
//
// Update: rows are grouped by codeword with the stable radix sort, each
// codeword's rows are summed in ascending row order (bitwise reproducible),
// and one pass applies the EMA and refreshes the bf16 shadow and its norms.
#include "sort.h"

namespace xgs {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------- prepare
__global__ void __launch_bounds__(256) vq_prepare_kernel(const float* __restrict__ E, int K, int D,
                                                        uint16_t* __restrict__ Eb, float* __restrict__ en) {
    __shared__ float red[4];
    const int l = blockIdx.x;
    float s = 0.f;
    for (int d = threadIdx.x; d < D; d += 256) {
        const uint16_t h = to_bf16(E[(size_t)l * D + d]);
        Eb[(size_t)l * D + d] = h;
        const float v = from_bf16(h);
        s += v * v;
    }
    for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) en[l] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------------------------- FP32 plain path
// 64 rows x 64 codewords per tile, D in chunks of 32 through LDS; each thread
// owns a 4x4 block of distances.  Direct form sum (x - e)^2.
constexpr int P_BM = 64, P_BN = 64, P_BD = 32;

__device__ __forceinline__ bool better(float d, int i, float bd, int bi) {
    return d < bd || (d == bd && i < bi);
}

__global__ void __launch_bounds__(256) vq_fp32_kernel(const float* __restrict__ X, int64_t N, int D,
                                                     const float* __restrict__ E, int K,
                                                     int32_t* __restrict__ idx, float* __restrict__ dist) {
    __shared__ float xs[P_BD][P_BM + 4];
    __shared__ float es[P_BD][P_BN + 4];
    const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
    const int64_t r0 = (int64_t)blockIdx.x * P_BM;
    float bd[4];
    int bi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { bd[i] = INFINITY; bi[i] = 0x7FFFFFFF; }
    for (int c0 = 0; c0 < K; c0 += P_BN) {
        float acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
        for (int d0 = 0; d0 < D; d0 += P_BD) {
            // 64 x 32 floats of X and of E: 8 per thread each
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = k * 256 + t, row = e >> 5, dd = e & 31;
                const int64_t gr = r0 + row;
                const int gc = c0 + row;
                xs[dd][row] = (gr < N && d0 + dd < D) ? X[gr * D + d0 + dd] : 0.f;
                es[dd][row] = (gc < K && d0 + dd < D) ? E[(size_t)gc * D + d0 + dd] : 0.f;
            }
            __syncthreads();
#pragma unroll 8
            for (int dd = 0; dd < P_BD; ++dd) {
                const float4 xv = *reinterpret_cast<const float4*>(&xs[dd][tr * 4]);
                const float4 ev = *reinterpret_cast<const float4*>(&es[dd][tc * 4]);
                const float xa[4] = {xv.x, xv.y, xv.z, xv.w}, ea[4] = {ev.x, ev.y, ev.z, ev.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float df = xa[i] - ea[j];
                        acc[i][j] += df * df;
                    }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + tc * 4 + j;
            if (c < K)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (better(acc[i][j], c, bd[i], bi[i])) { bd[i] = acc[i][j]; bi[i] = c; }
        }
    }
    // merge the 16 threads (consecutive lanes) that share a row group
#pragma unroll
    for (int k = 8; k >= 1; k >>= 1)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float od = __shfl_xor(bd[i], k, 64);
            const int oi = __shfl_xor(bi[i], k, 64);
            if (better(od, oi, bd[i], bi[i])) { bd[i] = od; bi[i] = oi; }
        }
    if (tc == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + tr * 4 + i;
            if (r < N) { idx[r] = bi[i]; dist[r] = bd[i]; }
        }
}

// -------------------------------------------------- BF16 MFMA + rescore
constexpr int B_BM = 64;     // rows per workgroup (resident in LDS)
constexpr int B_PAD = 8;     // bf16 padding per LDS row (bank spread)
constexpr int B_FRAGS = 4;   // 32-codeword fragments per wave step (128 codewords)

struct Top4 {
    float s[4];
    int i[4];
};

// higher score wins; equal scores go to the lower codeword index
__device__ __forceinline__ bool beats(float s, int i, float os, int oi) {
    return s > os || (s == os && i < oi);
}

__device__ __forceinline__ void top4_insert(Top4& t, float s, int i) {
    if (!beats(s, i, t.s[3], t.i[3])) return;
    t.s[3] = s; t.i[3] = i;
#pragma unroll
    for (int k = 3; k > 0; --k) {
        if (beats(t.s[k], t.i[k], t.s[k - 1], t.i[k - 1])) {
            float ts = t.s[k]; t.s[k] = t.s[k - 1]; t.s[k - 1] = ts;
            int ti = t.i[k]; t.i[k] = t.i[k - 1]; t.i[k - 1] = ti;
        }
    }
}

// NKC > 0: D = 16 * NKC is a compile-time constant and the K loop is fully
// unrolled (no loop back-edge, so the prefetches stay in flight);
// NKC == 0: runtime D, rolled loop.
template <int PF, int NKC>
__global__ void __launch_bounds__(256) vq_bf16_kernel(const float* __restrict__ X, int64_t N, int D_rt,
                                                     const float* __restrict__ E,
                                                     const uint16_t* __restrict__ Eb,
                                                     const float* __restrict__ en, int K,
                                                     int32_t* __restrict__ idx, float* __restrict__ dist) {
    extern __shared__ __align__(16) uint16_t xs[];  // [B_BM][D + B_PAD]
    const int D = NKC > 0 ? 16 * NKC : D_rt;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ld = D + B_PAD;
    const int64_t r0 = (int64_t)blockIdx.x * B_BM;
    // X rows -> bf16 in LDS (float4 reads along rows)
    const int q4 = D / 4;
    for (int e = t; e < B_BM * q4; e += 256) {
        const int row = e / q4, c4 = e - row * q4;
        const int64_t gr = r0 + row;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gr < N) {
            const f32x4_t q = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(X + gr * D) + c4);
            v = make_float4(q[0], q[1], q[2], q[3]);
        }
        uint2 p;
        p.x = (uint32_t)to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16);
        p.y = (uint32_t)to_bf16(v.z) | ((uint32_t)to_bf16(v.w) << 16);
        *reinterpret_cast<uint2*>(&xs[row * ld + c4 * 4]) = p;
    }
    __syncthreads();

    Top4 top[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 4; ++k) { top[h].s[k] = -INFINITY; top[h].i[k] = 0x7FFFFFFF; }

    const int col = lane & 31, half = lane >> 5;
    const uint16_t* xrow0 = xs + col * ld + 8 * half;
    const uint16_t* xrow1 = xs + (32 + col) * ld + 8 * half;
    const int per_wave = (K + 3) / 4;  // codewords swept by this wave: [w*per_wave, ...)
    const int cw0 = w * per_wave, cw1 = min(K, cw0 + per_wave);
    const int nk = D / 16;
    for (int c0 = cw0; c0 < cw1; c0 += 32 * B_FRAGS) {
        f32x16_t acc[B_FRAGS][2];
        const uint16_t* arow[B_FRAGS];
#pragma unroll
        for (int f = 0; f < B_FRAGS; ++f) {
            const int cbase = c0 + 32 * f;
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = cbase + 8 * g4 + 4 * half + r;
                    const float v = en[min(c, K - 1)];
                    const float init = c < cw1 ? -0.5f * v : -INFINITY;
                    acc[f][0][4 * g4 + r] = init;
                    acc[f][1][4 * g4 + r] = init;
                }
            }
            arow[f] = Eb + (size_t)min(cbase + col, K - 1) * D + 8 * half;
        }
        // A fragments are loaded PF k-steps ahead of their use, the X
        // fragments from LDS one step ahead.
        bf16x8_t abuf[PF][B_FRAGS];
#pragma unroll
        for (int s = 0; s < PF; ++s)
#pragma unroll
            for (int f = 0; f < B_FRAGS; ++f)
                abuf[s][f] = *reinterpret_cast<const bf16x8_t*>(arow[f] + 16 * min(s, nk - 1));
        bf16x8_t b0 = *reinterpret_cast<const bf16x8_t*>(xrow0);
        bf16x8_t b1 = *reinterpret_cast<const bf16x8_t*>(xrow1);
        // nk is a multiple of PF (the host picks PF accordingly)
#pragma unroll
        for (int k = 0; k < (NKC > 0 ? NKC : nk); k += PF) {
#pragma unroll
            for (int s = 0; s < PF; ++s) {
                const int kk = k + s;
                const int kb = min(kk + 1, nk - 1);
                const bf16x8_t nb0 = *reinterpret_cast<const bf16x8_t*>(xrow0 + 16 * kb);
                const bf16x8_t nb1 = *reinterpret_cast<const bf16x8_t*>(xrow1 + 16 * kb);
#pragma unroll
                for (int f = 0; f < B_FRAGS; ++f) {
                    acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(abuf[s][f], b0, acc[f][0], 0, 0, 0);
                    acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(abuf[s][f], b1, acc[f][1], 0, 0, 0);
                }
                const int kn = min(kk + PF, nk - 1);
#pragma unroll
                for (int f = 0; f < B_FRAGS; ++f)
                    abuf[s][f] = *reinterpret_cast<const bf16x8_t*>(arow[f] + 16 * kn);
                b0 = nb0;
                b1 = nb1;
                // keep the prefetches where they are: the scheduler would
                // otherwise sink them next to their use, PF steps later
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // top-4 per row: candidates i = c0 + 32 f + 8 (r/4) + 4 half + r%4
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float mx = -INFINITY;
#pragma unroll
            for (int f = 0; f < B_FRAGS; ++f)
#pragma unroll
                for (int r = 0; r < 16; ++r) mx = fmaxf(mx, acc[f][h][r]);
            if (mx >= top[h].s[3]) {
#pragma unroll
                for (int f = 0; f < B_FRAGS; ++f)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int c = c0 + 32 * f + 8 * (r >> 2) + 4 * half + (r & 3);
                        top4_insert(top[h], acc[f][h][r], c);
                    }
            }
        }
    }
    __syncthreads();  // X tile no longer needed: reuse LDS for candidates
    // candidate lists: row (0..63) x 8 lists (4 waves x 2 halves) x 4
    float* cs = reinterpret_cast<float*>(xs);
    int* ci = reinterpret_cast<int*>(cs + B_BM * 32);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int row = 32 * h + col;
        const int list = 2 * w + half;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cs[row * 32 + list * 4 + k] = top[h].s[k];
            ci[row * 32 + list * 4 + k] = top[h].i[k];
        }
    }
    __syncthreads();
    // each wave takes 16 rows; per row, lane k < 32 holds one candidate
    for (int rr = 0; rr < 16; ++rr) {
        const int row = 16 * w + rr;
        const int64_t gr = r0 + row;
        float s = lane < 32 ? cs[row * 32 + lane] : -INFINITY;
        int ii = lane < 32 ? ci[row * 32 + lane] : 0x7FFFFFFF;
        // pick the 4 best of the 32 by repeated arg-max
        int pick[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float bs = s;
            int bi = ii;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const float os = __shfl_xor(bs, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (beats(os, oi, bs, bi)) { bs = os; bi = oi; }
            }
            pick[k] = bi;
            if (ii == bi) { s = -INFINITY; ii = 0x7FFFFFFF; }
        }
        if (gr >= N) continue;  // uniform per wave
        // FP32 rescore of the 4 picks, lanes across D
        const float* xr = X + gr * D;
        float part[4] = {0.f, 0.f, 0.f, 0.f};
        for (int d = lane; d < D; d += 64) {
            const float xv = xr[d];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = pick[k] < K ? pick[k] : K - 1;
                const float df = xv - E[(size_t)c * D + d];
                part[k] += df * df;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) part[k] += __shfl_xor(part[k], o, 64);
        if (lane == 0) {
            float bd = INFINITY;
            int bi = 0x7FFFFFFF;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (pick[k] < K && better(part[k], pick[k], bd, bi)) { bd = part[k]; bi = pick[k]; }
            idx[gr] = bi;
            dist[gr] = bd;
        }
    }
}

// ------------------------------------------------------------------- EMA
__global__ void ema_keys_kernel(const int32_t* __restrict__ idx, int64_t N, int K,
                                uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                int64_t* __restrict__ count) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0) *count = N;
    if (n >= N) return;
    int a = idx[n];
    a = a < 0 ? 0 : (a >= K ? K - 1 : a);
    keys[n] = (uint64_t)(uint32_t)a;
    vals[n] = (uint32_t)n;
}

// One workgroup per codeword: counts, row sums in ascending row order, EMA of
// N and M.  Row ids are staged in LDS; each thread owns up to 4 columns and
// issues the loads of 8 rows before adding them in order, so the sum order
// (and hence the result) does not depend on timing.
constexpr int EMA_COLS = 4, EMA_ROWS = 8;

__global__ void __launch_bounds__(256) ema_accum_kernel(const float* __restrict__ X, int D,
                                                       const uint32_t* __restrict__ rows,
                                                       const uint32_t* __restrict__ ranges,
                                                       float decay, float* __restrict__ N_ema,
                                                       float* __restrict__ M_ema,
                                                       float* __restrict__ counts) {
    __shared__ uint32_t rid[256];
    const int l = blockIdx.x, t = threadIdx.x;
    const uint32_t b = ranges[2 * l], e = ranges[2 * l + 1];
    for (int d0 = 0; d0 < D; d0 += 256 * EMA_COLS) {
        float acc[EMA_COLS];
#pragma unroll
        for (int c = 0; c < EMA_COLS; ++c) acc[c] = 0.f;
        for (uint32_t k0 = b; k0 < e; k0 += 256) {
            __syncthreads();
            if (k0 + t < e) rid[t] = rows[k0 + t];
            __syncthreads();
            const int cnt = (int)min(256u, e - k0);
            for (int k = 0; k < cnt; k += EMA_ROWS) {
                float v[EMA_ROWS][EMA_COLS];
#pragma unroll
                for (int j = 0; j < EMA_ROWS; ++j) {
                    const bool rok = k + j < cnt;
                    const size_t base = rok ? (size_t)rid[k + j] * D : 0;
#pragma unroll
                    for (int c = 0; c < EMA_COLS; ++c) {
                        const int d = d0 + t + 256 * c;
                        v[j][c] = (rok && d < D) ? X[base + d] : 0.f;
                    }
                }
#pragma unroll
                for (int j = 0; j < EMA_ROWS; ++j)
#pragma unroll
                    for (int c = 0; c < EMA_COLS; ++c) acc[c] += v[j][c];
            }
        }
#pragma unroll
        for (int c = 0; c < EMA_COLS; ++c) {
            const int d = d0 + t + 256 * c;
            if (d < D) {
                float* m = M_ema + (size_t)l * D + d;
                *m = decay * *m + (1.f - decay) * acc[c];
            }
        }
    }
    if (t == 0) {
        const float c = (float)(e - b);
        N_ema[l] = decay * N_ema[l] + (1.f - decay) * c;
        if (counts) counts[l] = c;
    }
}

// One workgroup: n = sum_l N_l in a fixed tree order.
__global__ void __launch_bounds__(256) ema_total_kernel(const float* __restrict__ N_ema, int K,
                                                       float* __restrict__ total) {
    __shared__ float red[256];
    float s = 0.f;
    for (int l = threadIdx.x; l < K; l += 256) s += N_ema[l];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = red[0];
}

__global__ void __launch_bounds__(256) ema_finalize_kernel(const float* __restrict__ N_ema,
                                                          const float* __restrict__ M_ema, int K, int D,
                                                          float eps, int mode,
                                                          const float* __restrict__ total,
                                                          float* __restrict__ E, uint16_t* __restrict__ Eb,
                                                          float* __restrict__ en) {
    __shared__ float red[4];
    const int l = blockIdx.x;
    float denom;
    if (mode == XGS_EMA_PAPER) {
        denom = N_ema[l] + eps;
    } else {
        const float n = *total;
        denom = (N_ema[l] + eps) / (n + (float)K * eps) * n;
    }
    float s = 0.f;
    for (int d = threadIdx.x; d < D; d += 256) {
        const float v = M_ema[(size_t)l * D + d] / denom;
        E[(size_t)l * D + d] = v;
        if (Eb) {
            const uint16_t h = to_bf16(v);
            Eb[(size_t)l * D + d] = h;
            const float f = from_bf16(h);
            s += f * f;
        }
    }
    if (!en) return;
    for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) en[l] = (red[0] + red[1]) + (red[2] + red[3]);
}

struct EmaWs {
    uint64_t* keys;
    uint32_t* vals;
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* hist;
    uint32_t* ranges;
    int64_t* count;
    float* total;
};

static EmaWs carve_ema(void* base, int64_t N, int K, size_t* bytes) {
    Carve c(base);
    EmaWs w;
    const int64_t n1 = N > 0 ? N : 1;
    w.keys = c.take<uint64_t>(n1);
    w.vals = c.take<uint32_t>(n1);
    w.keys_alt = c.take<uint64_t>(n1);
    w.vals_alt = c.take<uint32_t>(n1);
    w.hist = c.take<uint32_t>(radix_hist_words(n1, 64));
    w.ranges = c.take<uint32_t>(2 * (size_t)(K > 0 ? K : 1));
    w.count = c.take<int64_t>(1);
    w.total = c.take<float>(1);
    *bytes = c.total();
    return w;
}

static int bits_for(int64_t k) {
    int b = 1;
    while ((int64_t(1) << b) < k) ++b;
    return b;
}

}  // namespace xgs

using namespace xgs;

extern "C" size_t xgs_vq_assign_workspace(int64_t N, int32_t D, int32_t K, int32_t precision) {
    (void)N; (void)D; (void)K; (void)precision;
    return 0;
}

extern "C" xgs_status xgs_vq_prepare(const float* E, int32_t K, int32_t D, uint16_t* E_bf16,
                                     float* e_norm2, xgs_stream_t stream) {
    clear_error();
    if (K < 1 || D < 1) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_prepare: K and D must be positive");
    if (!E || !E_bf16 || !e_norm2) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_prepare: null pointer");
    hipLaunchKernelGGL(vq_prepare_kernel, dim3((unsigned)K), dim3(256), 0, (hipStream_t)stream, E, K, D,
                       E_bf16, e_norm2);
    return check_launch("xgs_vq_prepare");
}

extern "C" xgs_status xgs_vq_assign(const float* X, int64_t N, int32_t D, const float* E,
                                    const uint16_t* E_bf16, const float* e_norm2, int32_t K,
                                    int32_t precision, int32_t* idx, float* dist, void* ws,
                                    size_t ws_bytes, xgs_stream_t stream) {
    (void)ws; (void)ws_bytes;
    clear_error();
    if (N < 0 || D < 1 || K < 1) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: bad sizes");
    if (N == 0) return XGS_OK;
    if (!X || !E || !idx || !dist) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: null pointer");
    if (N > (int64_t)1 << 40) return fail(XGS_ERR_UNSUPPORTED, "xgs_vq_assign: N too large");
    hipStream_t st = (hipStream_t)stream;
    if (precision == XGS_VQ_FP32) {
        const int64_t blocks = (N + P_BM - 1) / P_BM;
        hipLaunchKernelGGL(vq_fp32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, N, D, E, K, idx, dist);
        return check_launch("xgs_vq_assign fp32");
    }
    if (precision != XGS_VQ_BF16_RESCORE4) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: unknown precision");
    if (!E_bf16 || !e_norm2) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: bf16 shadow or norms missing");
    if (D % 16 != 0) return fail(XGS_ERR_UNSUPPORTED, "xgs_vq_assign: BF16 path needs D % 16 == 0");
    if (!aligned(X, 16) || !aligned(E_bf16, 16) || !aligned(e_norm2, 16))
        return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: X, E_bf16, e_norm2 must be 16-byte aligned");
    const size_t lds = (size_t)B_BM * (D + B_PAD) * sizeof(uint16_t);
    const size_t lds_cand = (size_t)B_BM * 32 * 8;
    const size_t lds_bytes = lds > lds_cand ? lds : lds_cand;
    if (lds_bytes > 160 * 1024) return fail(XGS_ERR_UNSUPPORTED, "xgs_vq_assign: D too large for the LDS-resident row tile");
    const int64_t blocks = (N + B_BM - 1) / B_BM;
    const int nk = D / 16;
    const void* fn;
    void (*launch)(dim3, size_t, hipStream_t, const float*, int64_t, int, const float*, const uint16_t*,
                   const float*, int, int32_t*, float*);
#define XGS_VQ_KERNEL(PF, NKC)                                                                          \
    fn = (const void*)vq_bf16_kernel<PF, NKC>;                                                          \
    launch = [](dim3 g, size_t l, hipStream_t s, const float* X_, int64_t N_, int D_, const float* E_,  \
                const uint16_t* Eb_, const float* en_, int K_, int32_t* i_, float* d_) {                \
        hipLaunchKernelGGL((vq_bf16_kernel<PF, NKC>), g, dim3(256), l, s, X_, N_, D_, E_, Eb_, en_, K_, \
                           i_, d_);                                                                      \
    };
    switch (nk) {
        case 48: XGS_VQ_KERNEL(4, 48) break;
        case 32: XGS_VQ_KERNEL(4, 32) break;
        case 16: XGS_VQ_KERNEL(4, 16) break;
        case 8: XGS_VQ_KERNEL(4, 8) break;
        case 4: XGS_VQ_KERNEL(4, 4) break;
        default:
            if (nk % 4 == 0) { XGS_VQ_KERNEL(4, 0) }
            else if (nk % 2 == 0) { XGS_VQ_KERNEL(2, 0) }
            else { XGS_VQ_KERNEL(1, 0) }
    }
#undef XGS_VQ_KERNEL
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess)
        return fail(XGS_ERR_HIP, "xgs_vq_assign: cannot reserve " + std::to_string(lds_bytes) + " bytes of LDS");
    launch(dim3((unsigned)blocks), lds_bytes, st, X, N, D, E, E_bf16, e_norm2, K, idx, dist);
    return check_launch("xgs_vq_assign bf16");
}

extern "C" size_t xgs_vq_ema_workspace(int64_t N, int32_t D, int32_t K) {
    (void)D;
    size_t bytes = 0;
    carve_ema(nullptr, N < 0 ? 0 : N, K, &bytes);
    return bytes;
}

extern "C" xgs_status xgs_vq_ema_update(const float* X, const int32_t* idx, int64_t N, int32_t D,
                                        int32_t K, float* N_ema, float* M_ema, float* E,
                                        uint16_t* E_bf16, float* e_norm2, float* counts, float decay,
                                        float eps, int32_t mode, void* ws, size_t ws_bytes,
                                        xgs_stream_t stream) {
    clear_error();
    if (N < 0 || D < 1 || K < 1) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_ema_update: bad sizes");
    if (N >= ((int64_t)1 << 32)) return fail(XGS_ERR_UNSUPPORTED, "xgs_vq_ema_update: N must be below 2^32");
    if (!(decay >= 0.f && decay < 1.f)) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_ema_update: decay must be in [0, 1)");
    if (mode != XGS_EMA_PAPER && mode != XGS_EMA_LAPLACE)
        return fail(XGS_ERR_INVALID_ARG, "xgs_vq_ema_update: unknown mode");
    if ((N > 0 && (!X || !idx)) || !N_ema || !M_ema || !E)
        return fail(XGS_ERR_INVALID_ARG, "xgs_vq_ema_update: null pointer");
    if ((E_bf16 == nullptr) != (e_norm2 == nullptr))
        return fail(XGS_ERR_INVALID_ARG, "xgs_vq_ema_update: E_bf16 and e_norm2 go together");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_ema_update: workspace must be 256-byte aligned");
    size_t need = 0;
    EmaWs w = carve_ema(ws, N, K, &need);
    if (!ws || ws_bytes < need) return fail(XGS_ERR_CAPACITY, "xgs_vq_ema_update: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    xgs_status s;
    if ((s = fill_u32(w.ranges, 2 * (int64_t)K, 0u, st))) return s;
    const int64_t n1 = N > 0 ? N : 1;
    hipLaunchKernelGGL(ema_keys_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, idx, N, K, w.keys,
                       w.vals, w.count);
    if ((s = check_launch("xgs_vq_ema_update keys"))) return s;
    const int bits = bits_for(K);
    if ((s = radix_sort(w.keys, w.vals, w.keys_alt, w.vals_alt, w.count, N, bits, w.hist, st))) return s;
    const bool even = radix_passes(bits) % 2 == 0;
    const uint64_t* sk = even ? w.keys : w.keys_alt;
    const uint32_t* sv = even ? w.vals : w.vals_alt;
    if ((s = segment_ranges(sk, w.count, N, 0, w.ranges, st))) return s;
    hipLaunchKernelGGL(ema_accum_kernel, dim3((unsigned)K), dim3(256), 0, st, X, D, sv, w.ranges, decay, N_ema,
                       M_ema, counts);
    hipLaunchKernelGGL(ema_total_kernel, dim3(1), dim3(256), 0, st, N_ema, K, w.total);
    hipLaunchKernelGGL(ema_finalize_kernel, dim3((unsigned)K), dim3(256), 0, st, N_ema, M_ema, K, D, eps, mode,
                       w.total, E, E_bf16, e_norm2);
    return check_launch("xgs_vq_ema_update");
}
