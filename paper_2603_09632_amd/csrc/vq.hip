// a6/a7: nearest-codeword assignment and the EMA codebook update of the
// online VQ module (Sec. 3.2.2, Eq. (ema_update)).
//
// Assignment, BF16 form (precision form): the distance contraction is the
// only dense GEMM on the hot path, so it runs on MFMA in three stages.
//  1. Staging: X and the codebook are rounded to bf16 and written
//     chunk-tiled (for a block of rows, the 32 columns of a chunk are
//     contiguous row after row) with one extra chunk per row that carries the
//     squared norm as three bf16 pieces against ones on the other operand,
//     so the plain dot product of two staged rows is half their squared
//     distance (the ranking key); padded codewords carry +inf.
//  2. Sweep: a workgroup owns 128 X rows and one codebook part (at least 4
//     parts; the parts of a row block go to one XCD so its X chunks are read
//     once into one L2), swept in 256-codeword tiles.  Four wavefronts each
//     accumulate all 128 rows x 64 codewords with v_mfma_f32_32x32x16_bf16 in
//     FP32: the X chunk goes through LDS (loaded into registers one chunk
//     ahead, stored into one of two buffers, read by all four), while each
//     wavefront loads its own codeword fragments straight into registers two
//     chunks ahead (vq_gemm_ereg_kernel).  Each lane keeps a running top-4
//     per row of 32-bit rank keys (distance with the candidate's position in
//     its low bits, so ties go to the lower index).  The confidence form
//     (an online log-sum-exp per row and part beside the top-4) needs more
//     registers than that layout leaves, so it runs vq_gemm_kernel, where both
//     operands arrive by direct global->LDS loads into three chunk buffers and
//     four wavefronts each accumulate 64 rows x 128 codewords; both sweeps
//     form the same products in the same order.
//  3. Rescore: the 4 x parts candidates of a row are reduced to the best 4
//     and rescored with the direct FP32 form sum (x - e)^2; the smallest wins
//     (lowest index on ties).
// The FP32 plain path (vq_fp32_kernel) tiles the direct form through LDS.
//
// Update: rows are grouped by codeword with the stable radix sort, each
// codeword's rows are summed as pieces of at most 128 rows whose sums are
// added in piece order (bitwise reproducible), and one pass applies the EMA
// and refreshes the bf16 shadow and its norms.
#include <algorithm>

#include "sort.h"
#include "wave.h"

namespace xgs {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

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
//
// Four kernels.  vq_xprep and vq_eprep lay out bf16 operands with one extra
// 32-column chunk per row that carries the squared norms:
//   X row n:     -x^_n, zero padding,  1,  1,  1, h0, h1, h2, 0 ...
//   codeword c:   e^_c, zero padding, g0, g1, g2,  1,  1,  1, 0 ...
// with h0 + h1 + h2 = |x^_n|^2 / 2 and g0 + g1 + g2 = |e^_c|^2 / 2 split into
// three bf16 pieces (exact to about 2^-24 relative), so the plain dot product
// of the two rows is half the squared distance of the bf16 operands.  The
// codebook is padded to whole tiles with rows whose g0 is +inf.
// vq_gemm gives a workgroup 128 rows and one part of the codebook, swept in
// tiles of 256 codewords.  Both operands go straight from memory into LDS in
// chunks of 32 columns (direct global->LDS loads, three buffers, issued two
// chunks ahead) and each of the four wavefronts accumulates a 64-row x
// 128-codeword block with v_mfma_f32_32x32x16_bf16.  Per row, every lane
// keeps its 4 smallest as 32-bit rank keys: the value's bits with the lowest
// seq_bits bits replaced by the candidate's position in the lane's stream
// (which increases with the codeword index), so ties go to the lower index
// and an insertion is four min/med3 operations with no branches.  The four
// lists of a row are merged in LDS.  vq_rescore takes the best 4 over the
// parts and picks the smallest direct FP32 distance.
constexpr int Q_BN = 256;                      // codewords per tile
constexpr int Q_BK = 32;                       // bf16 columns per chunk (64 bytes of a row)
constexpr int Q_MAX_TILES = 16;                // tiles per part: position fits in 10 bits
constexpr int Q_MAX_PARTS = 16;                // candidate lists per row in the rescore (x4 <= 64 lanes)
constexpr int Q_MIN_PARTS = 4;

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// Slot of (row, 16-byte segment) in a chunk buffer.  The XOR spreads the rows
// that one ds_read_b128 touches (32 rows, fixed segment) over distinct banks.
__device__ __forceinline__ int q_swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }
__device__ __forceinline__ int q_slot(int row, int seg) { return 4 * row + (seg ^ q_swz(row)); }

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const lds_void_t*)p;
}

// LDS fragment read issued as inline asm: the compiler would otherwise wait
// for every outstanding direct global->LDS load (vmcnt(0)) before it, which
// serialises the prefetch.  The caller waits on lgkmcnt itself (lds_wait).
typedef int i32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ i32x4_t lds_read16(uint32_t a) {
    i32x4_t v;
    asm volatile("ds_read_b128 %0, %1" : "=v"(v) : "v"(a));
    return v;
}

__device__ __forceinline__ int med3i(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

// v = h0 + h1 + h2 with bf16 pieces (each the rounding of what is left).
__device__ __forceinline__ void split3(float v, uint16_t& h0, uint16_t& h1, uint16_t& h2) {
    h0 = to_bf16(v);
    const float r1 = v - from_bf16(h0);
    h1 = to_bf16(r1);
    h2 = to_bf16(r1 - from_bf16(h1));
}

constexpr uint16_t kBf16One = 0x3F80;

// (key, codeword) order: smaller key first, then the lower codeword; empty
// entries (codeword -1) last.
__device__ __forceinline__ bool cand_before(int ka, int ca, int kb, int cb) {
    if (ca < 0) return false;
    if (cb < 0) return true;
    return ka < kb || (ka == kb && ca < cb);
}


// Both operands are stored chunk-tiled: the 32 columns of chunk kc of a block
// of rows (128 X rows, or one 256-codeword tile) are contiguous, row after
// row (64 bytes each), so one direct load of a wavefront reads 1 KB of
// consecutive memory.  Element (row, col) of a block of B rows sits at
// ((blk * nkc + col / 32) * B + row % B) * 32 + col % 32, blk = row / B.
__device__ __forceinline__ size_t tiled_at(int64_t row, int col, int B, int nkc) {
    return ((size_t)(row / B) * nkc + col / Q_BK) * ((size_t)B * Q_BK) + (size_t)(row % B) * Q_BK + col % Q_BK;
}

// One wavefront per row of the padded row count Np (rows >= N are zero);
// Dp = D rounded up to 32, Dx = Dp + 32 columns.
__global__ void __launch_bounds__(256) vq_xprep_kernel(const float* __restrict__ X, int64_t N, int64_t Np, int D,
                                                      int Dp, int Dx, int B, uint16_t* __restrict__ Xa) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= Np) return;
    const int nkc = Dx / Q_BK;
    const bool real = row < N;
    const f32x4_t* xr = reinterpret_cast<const f32x4_t*>(X + (real ? row : 0) * D);
    float s = 0.f;
    for (int q = lane; q < Dp / 4; q += 64) {
        uint2 p = make_uint2(0u, 0u);
        if (real && q < D / 4) {
            const f32x4_t v = __builtin_nontemporal_load(xr + q);
            uint16_t h[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                h[k] = to_bf16(v[k]);
                const float f = from_bf16(h[k]);
                s += f * f;
            }
            p.x = ((uint32_t)h[0] | ((uint32_t)h[1] << 16)) ^ 0x80008000u;  // -x^ (sign flip is exact)
            p.y = ((uint32_t)h[2] | ((uint32_t)h[3] << 16)) ^ 0x80008000u;
        }
        *reinterpret_cast<uint2*>(Xa + tiled_at(row, 4 * q, B, nkc)) = p;
    }
    for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
    if (lane < 8) {
        uint16_t h0, h1, h2;
        split3(0.5f * s, h0, h1, h2);
        uint16_t v[4] = {0, 0, 0, 0};
        if (real && lane == 0) { v[0] = kBf16One; v[1] = kBf16One; v[2] = kBf16One; v[3] = h0; }
        if (real && lane == 1) { v[0] = h1; v[1] = h2; }
        uint2 p;
        p.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        p.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
        *reinterpret_cast<uint2*>(Xa + tiled_at(row, Dp + 4 * lane, B, nkc)) = p;
    }
}

// One wavefront per (padded) codeword row.
__global__ void __launch_bounds__(256) vq_eprep_kernel(const uint16_t* __restrict__ Eb, const float* __restrict__ en,
                                                      int K, int D, int Kp, int Dp, int Dx,
                                                      uint16_t* __restrict__ Ea) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= Kp) return;
    const int nkc = Dx / Q_BK;
    const bool real = c < K;
    const uint4* in = reinterpret_cast<const uint4*>(Eb + (size_t)(real ? c : 0) * D);
    for (int q = lane; q < Dp / 8; q += 64)
        *reinterpret_cast<uint4*>(Ea + tiled_at(c, 8 * q, Q_BN, nkc)) =
            (real && q < D / 8) ? in[q] : make_uint4(0u, 0u, 0u, 0u);
    if (lane < 4) {
        uint16_t g0 = 0x7F80, g1 = 0, g2 = 0;  // +inf: a padded codeword is never chosen
        if (real) split3(0.5f * en[c], g0, g1, g2);
        uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (lane == 0) { v[0] = g0; v[1] = g1; v[2] = g2; v[3] = kBf16One; v[4] = kBf16One; v[5] = kBf16One; }
        uint4 p;
        p.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        p.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
        p.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
        p.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
        *reinterpret_cast<uint4*>(Ea + tiled_at(c, Dp + 8 * lane, Q_BN, nkc)) = p;
    }
}

// Tiling of the sweep: WMW x WNW wavefronts, each accumulating FX x FE
// fragments of 32 x 32 (rows x codewords), NBUF chunk buffers in LDS, OCC
// workgroups per CU.
template <int WMW_, int WNW_, int FX_, int FE_, int NBUF_, int OCC_>
struct GemmCfg {
    static constexpr int WMW = WMW_, WNW = WNW_, FX = FX_, FE = FE_, NBUF = NBUF_, OCC = OCC_;
    static constexpr int NW = WMW * WNW, THREADS = 64 * NW;
    static constexpr int ROWS = WMW * FX * 32, COLS = WNW * FE * 32;
    static constexpr int XSLOTS = ROWS * 4, SLOTS = (ROWS + COLS) * 4;
    static constexpr int NX = ROWS / (16 * NW), NE = COLS / (16 * NW), NI = NX + NE;
    static constexpr int NF = FX + FE;
    static_assert(COLS == Q_BN && FE <= 4 && ROWS % (16 * NW) == 0 && COLS % (16 * NW) == 0, "tiling");
};

// 128 rows x 256 codewords per workgroup, 4 wavefronts of 64 x 128 (128
// accumulators each), 3 chunk buffers (72 KB of LDS), two workgroups per CU.
// Measured alternatives: 256 x 256 with 4 wavefronts of 128 x 128 and 4
// buffers (one workgroup per CU) 14% slower; 256 x 256 with 8 wavefronts of
// 64 x 128 and 4 buffers equal.
using VqCfg = GemmCfg<2, 2, 2, 4, 3, 2>;

template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(N) : "memory");
}
template <int N>
__device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Waits until at most N LDS operations are outstanding (they complete in
// order, so reads issued N operations ago or earlier are done); the operands
// tie the fragments to the wait.  N < 0 only ties them.
template <int N, int NF>
__device__ __forceinline__ void lds_waitn(i32x4_t (&f)[NF]) {
    static_assert(NF == 6 || NF == 8, "fragment count");
    if constexpr (NF == 6) {
        if constexpr (N >= 0)
            asm volatile("s_waitcnt lgkmcnt(%6)" : "+v"(f[0]), "+v"(f[1]), "+v"(f[2]), "+v"(f[3]), "+v"(f[4]), "+v"(f[5]) : "n"(N));
        else
            asm volatile("" : "+v"(f[0]), "+v"(f[1]), "+v"(f[2]), "+v"(f[3]), "+v"(f[4]), "+v"(f[5]));
    } else {
        if constexpr (N >= 0)
            asm volatile("s_waitcnt lgkmcnt(%8)"
                         : "+v"(f[0]), "+v"(f[1]), "+v"(f[2]), "+v"(f[3]), "+v"(f[4]), "+v"(f[5]), "+v"(f[6]), "+v"(f[7])
                         : "n"(N));
        else
            asm volatile("" : "+v"(f[0]), "+v"(f[1]), "+v"(f[2]), "+v"(f[3]), "+v"(f[4]), "+v"(f[5]), "+v"(f[6]), "+v"(f[7]));
    }
}

// CONF: also the confidence of App. C, Eq. (confidence_score), from the same
// accumulators: per row a running log-sum-exp (m, s) of v_k = -d_k / tau over
// every codeword, d_k = sqrt(2 acc_k) the unsquared bf16 distance; merged over
// the lists of a row and written to lse[row][part].
template <class C, bool CONF>
__global__ void __launch_bounds__(C::THREADS, C::OCC) vq_gemm_kernel(const uint16_t* __restrict__ Xa, int64_t N, int Dx,
                                                                    const uint16_t* __restrict__ Ea, int K, int parts,
                                                                    int tiles_part, int seq_bits,
                                                                    int2* __restrict__ cand, float inv_tau,
                                                                    float2* __restrict__ lse) {
    constexpr int FX = C::FX, FE = C::FE, NF = C::NF, NBUF = C::NBUF, NI = C::NI;
    constexpr int ROWS = C::ROWS, COLS = C::COLS, NW = C::NW;
    constexpr int LISTS = 2 * C::WNW;
    __shared__ __align__(16) uint4 qbuf[NBUF * C::SLOTS];
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w % C::WMW, wn = w / C::WMW;
    // Workgroups go round-robin to the 8 XCDs.  The parts of one row block
    // take the same XCD (and neighbouring dispatch slots), so its X chunks
    // are fetched into one L2 and served to all of them.
    const int64_t blk = blockIdx.x;
    const int64_t grp = blk / (8 * parts);
    const int within = (int)(blk - grp * 8 * parts);
    const int p = within >> 3;
    const int64_t rb = grp * 8 + (within & 7);
    const int64_t r0 = rb * ROWS;
    if (r0 >= N) return;  // padding of the last group (whole workgroup)
    const int c_part = p * tiles_part * COLS;
    const int tiles = min(tiles_part, (K - c_part + COLS - 1) / COLS);
    const int nkc = Dx / Q_BK;
    const int total = tiles * nkc;
    const int rows_here = (int)min((int64_t)ROWS, N - r0);

    // This wave's direct loads: instruction m fills slots 64 j .. 64 j + 63
    // of a buffer, j = w + NW m: X rows 16 j + lane / 4 for m < NX, codeword
    // rows 16 (w + NW (m - NX)) + lane / 4 after; lane & 3 is the slot within
    // the row, holding segment (lane & 3) ^ q_swz(row).  In the chunk-tiled
    // operands those 16 rows are 1 KB of consecutive memory; the per-lane
    // byte offsets are fixed and the chunk moves the (scalar) bases.
    const int lr = lane >> 2;
    const char* xbase = reinterpret_cast<const char*>(Xa + (size_t)rb * nkc * ROWS * Q_BK);
    const char* ebase = reinterpret_cast<const char*>(Ea + (size_t)c_part * Dx);
    uint32_t off[NI];
#pragma unroll
    for (int m = 0; m < NI; ++m) {
        const int row = 16 * (w + NW * (m < C::NX ? m : m - C::NX)) + lr;
        off[m] = (uint32_t)row * 64u + 16u * (uint32_t)((lane & 3) ^ q_swz(row));
    }
    // next chunk to issue: tile, chunk within the tile, buffer
    int n_tl = 0, n_kc = 0, n_b = 0;
    auto issue = [&]() {
        const int tl = n_tl, kc = n_kc;
        uint4* dst = qbuf + n_b * C::SLOTS;
        if (++n_kc == nkc) { n_kc = 0; ++n_tl; }
        n_b = n_b == NBUF - 1 ? 0 : n_b + 1;
        const char* xb = xbase + (size_t)kc * (ROWS * Q_BK * 2);
        const char* eb = ebase + ((size_t)tl * nkc + kc) * (COLS * Q_BK * 2);
#pragma unroll
        for (int m = 0; m < C::NX; ++m)
            __builtin_amdgcn_global_load_lds((glb_void_t*)(xb + off[m]), (lds_void_t*)(dst + 64 * (w + NW * m)), 16,
                                             0, 0);
#pragma unroll
        for (int m = 0; m < C::NE; ++m)
            __builtin_amdgcn_global_load_lds((glb_void_t*)(eb + off[C::NX + m]),
                                             (lds_void_t*)(dst + C::XSLOTS + 64 * (w + NW * m)), 16, 0, 0);
    };

    // Fragment addresses: X fragment jx covers rows wm 32 FX + 32 jx + lane % 32,
    // codeword fragment i rows wn 32 FE + 32 i + lane % 32; step ks reads
    // segment 2 ks + lane / 32.  Rows 32 apart share the swizzle, so the
    // fragments of one step are 128 slots (2048 bytes) apart.
    const int fr = lane & 31, hf = lane >> 5;
    const uint32_t qb0 = lds_addr(qbuf);
    uint32_t xa[2], ea[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        xa[ks] = qb0 + 16u * (uint32_t)q_slot(wm * 32 * FX + fr, 2 * ks + hf);
        ea[ks] = qb0 + 16u * (uint32_t)(C::XSLOTS + q_slot(wn * 32 * FE + fr, 2 * ks + hf));
    }
    auto read_frags = [&](int b, int ks, i32x4_t (&f)[NF]) {
        const uint32_t o = (uint32_t)(b * C::SLOTS * 16);
#pragma unroll
        for (int jx = 0; jx < FX; ++jx) f[jx] = lds_read16(xa[ks] + o + 2048u * jx);
#pragma unroll
        for (int i = 0; i < FE; ++i) f[FX + i] = lds_read16(ea[ks] + o + 2048u * i);
    };

    // accumulator r of codeword fragment i holds codeword
    // tile base + wn 32 FE + 32 i + 8 (r / 4) + 4 hf + r % 4, row 32 jx + fr
    f32x16_t acc[FE][FX];
    int top[FX][4];
#pragma unroll
    for (int jx = 0; jx < FX; ++jx)
#pragma unroll
        for (int q = 0; q < 4; ++q) top[jx][q] = 0x7FFFFFFF;
    const uint32_t keep = ~((1u << seq_bits) - 1u);
    float lm[FX], ls[FX];
#pragma unroll
    for (int jx = 0; jx < FX; ++jx) { lm[jx] = -INFINITY; ls[jx] = 0.f; }
    auto tile_lse = [&]() {
#pragma unroll
        for (int jx = 0; jx < FX; ++jx) {
            float mt = -INFINITY;
#pragma unroll
            for (int i = 0; i < FE; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    mt = fmaxf(mt, -__builtin_sqrtf(fmaxf(2.f * acc[i][jx][r], 0.f)) * inv_tau);
            const float mn = fmaxf(lm[jx], mt);
            if (mn > -INFINITY) {  // a lane whose codewords are all padding adds nothing
                float sum = ls[jx] * __expf(lm[jx] - mn);
#pragma unroll
                for (int i = 0; i < FE; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        sum += __expf(-__builtin_sqrtf(fmaxf(2.f * acc[i][jx][r], 0.f)) * inv_tau - mn);
                ls[jx] = sum;
                lm[jx] = mn;
            }
        }
    };
    auto tile_top4 = [&](int tl) {
#pragma unroll
        for (int jx = 0; jx < FX; ++jx)
#pragma unroll
            for (int i = 0; i < FE; ++i) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int k = (int)((__float_as_uint(acc[i][jx][r]) & keep) |
                                        (uint32_t)((tl << 6) | (i << 4) | r));
                    top[jx][3] = med3i(top[jx][2], top[jx][3], k);
                    top[jx][2] = med3i(top[jx][1], top[jx][2], k);
                    top[jx][1] = med3i(top[jx][0], top[jx][1], k);
                    top[jx][0] = min(top[jx][0], k);
                }
                // one fragment at a time: the scheduler would otherwise read
                // every accumulator out at once
                __builtin_amdgcn_sched_barrier(0);
            }
    };
    auto mfma_step = [&](const i32x4_t (&f)[NF]) {
#pragma unroll
        for (int i = 0; i < FE; ++i)
#pragma unroll
            for (int jx = 0; jx < FX; ++jx)
                acc[i][jx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, f[FX + i]),
                                                                    __builtin_bit_cast(bf16x8_t, f[jx]),
                                                                    acc[i][jx], 0, 0, 0);
    };
    auto mfma_first = [&](const i32x4_t (&f)[NF]) {
        const f32x16_t z = {};
#pragma unroll
        for (int i = 0; i < FE; ++i)
#pragma unroll
            for (int jx = 0; jx < FX; ++jx)
                acc[i][jx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, f[FX + i]),
                                                                    __builtin_bit_cast(bf16x8_t, f[jx]), z, 0,
                                                                    0, 0);
    };

    // prologue: chunks 0 .. NBUF-2 in flight, wait for chunk 0
    const int pre = min(total, NBUF - 1);
    for (int c = 0; c < pre; ++c) issue();
    if (pre == NBUF - 1) wait_vm<NI * (NBUF - 2)>();
    else wait_vm<0>();
    __builtin_amdgcn_s_barrier();
    if (total > NBUF - 1) issue();
    i32x4_t f0[NF], f1[NF];
    read_frags(0, 0, f0);
    int g = 0, b = 0;
    for (int tl = 0; tl < tiles; ++tl) {
        for (int kc = 0; kc < nkc; ++kc, ++g) {
            const int bn = b == NBUF - 1 ? 0 : b + 1;
            read_frags(b, 1, f1);
            lds_waitn<NF, NF>(f0);  // f0 was read before f1's reads
            if (kc == 0) mfma_first(f0);
            else mfma_step(f0);
            // chunk g + 1 must have landed (own loads, then everyone's);
            // chunks g + 2 .. g + NBUF - 1 may still be in flight.  All reads
            // of buffer b are complete (lgkmcnt(0)), so after the barrier it
            // can be refilled with chunk g + NBUF.
            if (g + NBUF - 1 < total) wait_vm_lgkm0<NI * (NBUF - 2)>();
            else wait_vm_lgkm0<0>();
            __builtin_amdgcn_s_barrier();
            if (g + NBUF < total) issue();
            if (g + 1 < total) read_frags(bn, 0, f0);
            lds_waitn<-1, NF>(f1);  // complete since the lgkmcnt(0) above
            mfma_step(f1);
            b = bn;
        }
        if constexpr (CONF) tile_lse();
        tile_top4(tl);
    }
    __syncthreads();

    // merge: row x LISTS lists (wn, hf) x 4 candidates
    int2* mc = reinterpret_cast<int2*>(qbuf);
    const uint32_t pos_mask = (1u << seq_bits) - 1u;
#pragma unroll
    for (int jx = 0; jx < FX; ++jx) {
        const int row = wm * 32 * FX + 32 * jx + fr;
        const int list = 2 * wn + hf;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = top[jx][q];
            const uint32_t s = (uint32_t)k & pos_mask;
            const int c = c_part + (int)(s >> 6) * COLS + wn * 32 * FE + 32 * (int)((s >> 4) & 3) +
                          8 * (int)((s >> 2) & 3) + 4 * hf + (int)(s & 3);
            const bool ok = k != 0x7FFFFFFF && c < K;
            mc[(row * LISTS + list) * 4 + q] = make_int2(ok ? (int)((uint32_t)k & keep) : 0x7FFFFFFF, ok ? c : -1);
        }
    }
    __syncthreads();
    for (int row = t; row < rows_here; row += C::THREADS) {
        int bk[4] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
        int bc[4] = {-1, -1, -1, -1};
        for (int e = 0; e < LISTS * 4; ++e) {
            const int2 v = mc[row * LISTS * 4 + e];
            int k = v.x, c = v.y;
            // carry the entry up the sorted list (static indices: registers)
#pragma unroll
            for (int q = 3; q >= 0; --q)
                if (cand_before(k, c, bk[q], bc[q])) {
                    const int tk = bk[q], tc = bc[q];
                    bk[q] = k; bc[q] = c; k = tk; c = tc;
                }
        }
        int2* out = cand + ((r0 + row) * parts + p) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = make_int2(bk[q], bc[q]);
    }
    if constexpr (CONF) {
        // (m, s) of the lists of each row, merged in list order
        float2* ml = reinterpret_cast<float2*>(mc + ROWS * LISTS * 4);
#pragma unroll
        for (int jx = 0; jx < FX; ++jx)
            ml[(wm * 32 * FX + 32 * jx + fr) * LISTS + 2 * wn + hf] = make_float2(lm[jx], ls[jx]);
        __syncthreads();
        for (int row = t; row < rows_here; row += C::THREADS) {
            float m = -INFINITY;
            for (int e = 0; e < LISTS; ++e) m = fmaxf(m, ml[row * LISTS + e].x);
            float sum = 0.f;
            for (int e = 0; e < LISTS; ++e) {
                const float2 q = ml[row * LISTS + e];
                if (q.x > -INFINITY) sum += q.y * __expf(q.x - m);
            }
            lse[(r0 + row) * parts + p] = make_float2(m, sum);
        }
    }
}

// Sweep whose codeword operand bypasses LDS.  WNW wavefronts each own all
// ROWS = 32 FX rows of the block and 32 FE codewords of every tile.  Each
// wavefront loads its codeword fragments from global memory straight into
// registers two chunks ahead; the X chunk is loaded into registers one chunk
// ahead, written to one of two LDS buffers and read back by every wavefront.
// Per chunk and workgroup the LDS carries the X chunk once in and WNW times
// out, instead of both operands in and each operand twice out as in
// vq_gemm_kernel.  Every load is an ordinary load, so the compiler places
// all the waits.  Same products in the same order as vq_gemm_kernel, so the
// accumulators, and the candidates, are bitwise the same.
template <int FX_, int FE_, int WNW_, int OCC_>
struct RegCfg {
    static constexpr int FX = FX_, FE = FE_, WNW = WNW_, OCC = OCC_;
    static constexpr int NW = WNW, THREADS = 64 * NW;
    static constexpr int ROWS = FX * 32, COLS = WNW * FE * 32;
    static constexpr int SLOTS = ROWS * 4;           // 16-byte slots of one X chunk buffer
    static constexpr int NX = ROWS / (16 * NW);      // X loads per wavefront and chunk
    static constexpr int NEL = 2 * FE;               // codeword fragment loads per wavefront and chunk
    static constexpr int LISTS = 2 * WNW;
    static constexpr int MERGE_U4 = (ROWS * LISTS * 4 * 8 + ROWS * LISTS * 8 + 15) / 16;
    static constexpr int LDS_U4 = 2 * SLOTS > MERGE_U4 ? 2 * SLOTS : MERGE_U4;
    static_assert(COLS == Q_BN && FE <= 4 && ROWS % (16 * NW) == 0, "tiling");
};

// 128 rows x 256 codewords per workgroup, 4 wavefronts of 128 x 64.
using VqRegCfg = RegCfg<4, 2, 4, 2>;
static_assert(VqRegCfg::ROWS == VqCfg::ROWS, "both sweeps read X staged in blocks of the same rows");

template <class C, bool CONF>
__global__ void __launch_bounds__(C::THREADS, C::OCC) vq_gemm_ereg_kernel(const uint16_t* __restrict__ Xa, int64_t N,
                                                                         int Dx, const uint16_t* __restrict__ Ea, int K,
                                                                         int parts, int tiles_part, int seq_bits,
                                                                         int2* __restrict__ cand, float inv_tau,
                                                                         float2* __restrict__ lse) {
    constexpr int FX = C::FX, FE = C::FE, NX = C::NX, NEL = C::NEL;
    constexpr int ROWS = C::ROWS, COLS = C::COLS, NW = C::NW, LISTS = C::LISTS;
    __shared__ __align__(16) i32x4_t qbuf[C::LDS_U4];
    const int t = threadIdx.x, lane = t & 63;
    const int wn = __builtin_amdgcn_readfirstlane(t >> 6);
    // block -> (row block, part): the parts of one row block share an XCD
    const int64_t blk = blockIdx.x;
    const int64_t grp = blk / (8 * parts);
    const int within = (int)(blk - grp * 8 * parts);
    const int p = within >> 3;
    const int64_t rb = grp * 8 + (within & 7);
    const int64_t r0 = rb * ROWS;
    if (r0 >= N) return;
    const int c_part = p * tiles_part * COLS;
    const int tiles = min(tiles_part, (K - c_part + COLS - 1) / COLS);
    const int nkc = Dx / Q_BK;
    const int total = tiles * nkc;
    const int rows_here = (int)min((int64_t)ROWS, N - r0);

    // X: load m of this lane reads row 16 (wn + NW m) + lane / 4, segment
    // (lane & 3) ^ q_swz(row), and writes it to slot 64 (wn + NW m) + lane.
    const int lr = lane >> 2, fr = lane & 31, hf = lane >> 5;
    const char* xbase = reinterpret_cast<const char*>(Xa + (size_t)rb * nkc * ROWS * Q_BK);
    uint32_t off[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) {
        const int row = 16 * (wn + NW * m) + lr;
        off[m] = (uint32_t)row * 64u + 16u * (uint32_t)((lane & 3) ^ q_swz(row));
    }
    // Codeword fragment (i, ks) of this lane: row wn 32 FE + 32 i + fr of the
    // tile, segment 2 ks + hf.  Chunk c = tile * nkc + kc of the part is 256
    // rows x 64 bytes of consecutive memory at c * 16 KB.
    const char* ebase = reinterpret_cast<const char*>(Ea + (size_t)c_part * Dx) +
                        (uint32_t)(wn * 32 * FE + fr) * 64u + 16u * (uint32_t)hf;
    auto load_x = [&](int kc, i32x4_t (&x)[NX]) {
        const char* xb = xbase + (size_t)kc * (ROWS * Q_BK * 2);
#pragma unroll
        for (int m = 0; m < NX; ++m) x[m] = *reinterpret_cast<const i32x4_t*>(xb + off[m]);
    };
    auto store_x = [&](int buf, const i32x4_t (&x)[NX]) {
#pragma unroll
        for (int m = 0; m < NX; ++m) qbuf[buf * C::SLOTS + 64 * (wn + NW * m) + lane] = x[m];
    };
    auto load_e = [&](int c, i32x4_t (&e)[NEL]) {
        const char* eb = ebase + (size_t)c * (COLS * Q_BK * 2);
#pragma unroll
        for (int i = 0; i < FE; ++i)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                e[2 * i + ks] = *reinterpret_cast<const i32x4_t*>(eb + 2048 * i + 32 * ks);
    };
    int xs0[2], xs1[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        xs0[ks] = q_slot(fr, 2 * ks + hf);
        xs1[ks] = C::SLOTS + xs0[ks];
    }
    auto read_frags = [&](int buf, int ks, i32x4_t (&f)[FX]) {
        const int s = buf ? xs1[ks] : xs0[ks];
#pragma unroll
        for (int jx = 0; jx < FX; ++jx) f[jx] = qbuf[s + 128 * jx];
    };

    // accumulator r of codeword fragment i holds codeword
    // tile base + wn 32 FE + 32 i + 8 (r / 4) + 4 hf + r % 4, row 32 jx + fr
    f32x16_t acc[FE][FX];
    int top[FX][4];
#pragma unroll
    for (int jx = 0; jx < FX; ++jx)
#pragma unroll
        for (int q = 0; q < 4; ++q) top[jx][q] = 0x7FFFFFFF;
    const uint32_t keep = ~((1u << seq_bits) - 1u);
    float lm[FX], ls[FX];
#pragma unroll
    for (int jx = 0; jx < FX; ++jx) { lm[jx] = -INFINITY; ls[jx] = 0.f; }
    auto tile_lse = [&]() {
#pragma unroll
        for (int jx = 0; jx < FX; ++jx) {
            float mt = -INFINITY;
#pragma unroll
            for (int i = 0; i < FE; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    mt = fmaxf(mt, -__builtin_sqrtf(fmaxf(2.f * acc[i][jx][r], 0.f)) * inv_tau);
            const float mn = fmaxf(lm[jx], mt);
            if (mn > -INFINITY) {
                float sum = ls[jx] * __expf(lm[jx] - mn);
#pragma unroll
                for (int i = 0; i < FE; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        sum += __expf(-__builtin_sqrtf(fmaxf(2.f * acc[i][jx][r], 0.f)) * inv_tau - mn);
                ls[jx] = sum;
                lm[jx] = mn;
            }
        }
    };
    auto tile_top4 = [&](int tl) {
#pragma unroll
        for (int jx = 0; jx < FX; ++jx)
#pragma unroll
            for (int i = 0; i < FE; ++i) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int k = (int)((__float_as_uint(acc[i][jx][r]) & keep) |
                                        (uint32_t)((tl << 6) | (i << 4) | r));
                    top[jx][3] = med3i(top[jx][2], top[jx][3], k);
                    top[jx][2] = med3i(top[jx][1], top[jx][2], k);
                    top[jx][1] = med3i(top[jx][0], top[jx][1], k);
                    top[jx][0] = min(top[jx][0], k);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
    };
    auto mfma_half = [&](const i32x4_t (&f)[FX], const i32x4_t (&e)[NEL], int ks) {
#pragma unroll
        for (int i = 0; i < FE; ++i)
#pragma unroll
            for (int jx = 0; jx < FX; ++jx)
                acc[i][jx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, e[2 * i + ks]),
                                                                    __builtin_bit_cast(bf16x8_t, f[jx]), acc[i][jx],
                                                                    0, 0, 0);
    };
    auto mfma_first = [&](const i32x4_t (&f)[FX], const i32x4_t (&e)[NEL]) {
        const f32x16_t z = {};
#pragma unroll
        for (int i = 0; i < FE; ++i)
#pragma unroll
            for (int jx = 0; jx < FX; ++jx)
                acc[i][jx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, e[2 * i]),
                                                                    __builtin_bit_cast(bf16x8_t, f[jx]), z, 0, 0, 0);
    };

    // Chunk g: X(g) sits in LDS buffer g % 2, X(g + 1) in registers, E(g)
    // and E(g + 1) in registers.  The first half of g's products is followed
    // by the loads of E(g + 2), the store of X(g + 1) into the other buffer
    // and the load of X(g + 2); the barrier publishes X(g + 1), whose first
    // fragments are read before the second half.  Past the last chunk the
    // loads repeat in-bounds chunks that nobody uses, so every chunk issues
    // the same loads and the compiler's counts stay exact.
    if (total > 0) {  // a part past the last codeword has no tiles
        const int last = total - 1;
        i32x4_t e0[NEL], e1[NEL], e2[NEL], xr[NX];
        int x_kc = 0;  // chunk within the tile of the X chunk in xr
        load_x(0, xr);
        load_e(0, e0);
        load_e(min(1, last), e1);
        store_x(0, xr);
        x_kc = nkc > 1 ? 1 : 0;
        load_x(x_kc, xr);
        __syncthreads();
        i32x4_t f0[FX], f1[FX];
        read_frags(0, 0, f0);
        int tl = 0, kc = 0, b = 0;
        auto chunk = [&](int g, i32x4_t (&ec)[NEL], i32x4_t (&el)[NEL]) {
            read_frags(b, 1, f1);
            if (kc == 0) mfma_first(f0, ec);
            else mfma_half(f0, ec, 0);
            load_e(min(g + 2, last), el);
            store_x(b ^ 1, xr);
            x_kc = x_kc == nkc - 1 ? 0 : x_kc + 1;
            load_x(x_kc, xr);
            __syncthreads();
            b ^= 1;
            read_frags(b, 0, f0);
            mfma_half(f1, ec, 1);
            if (++kc == nkc) {
                if constexpr (CONF) tile_lse();
                tile_top4(tl);
                kc = 0;
                ++tl;
            }
        };
        int g = 0;
        for (; g + 3 <= total; g += 3) {
            chunk(g, e0, e2);
            chunk(g + 1, e1, e0);
            chunk(g + 2, e2, e1);
        }
        if (g < total) chunk(g, e0, e2);
        if (g + 1 < total) chunk(g + 1, e1, e0);
    }
    __syncthreads();

    // merge: row x LISTS lists (wn, hf) x 4 candidates
    int2* mc = reinterpret_cast<int2*>(qbuf);
    const uint32_t pos_mask = (1u << seq_bits) - 1u;
#pragma unroll
    for (int jx = 0; jx < FX; ++jx) {
        const int row = 32 * jx + fr;
        const int list = 2 * wn + hf;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = top[jx][q];
            const uint32_t s = (uint32_t)k & pos_mask;
            const int c = c_part + (int)(s >> 6) * COLS + wn * 32 * FE + 32 * (int)((s >> 4) & 3) +
                          8 * (int)((s >> 2) & 3) + 4 * hf + (int)(s & 3);
            const bool ok = k != 0x7FFFFFFF && c < K;
            mc[(row * LISTS + list) * 4 + q] = make_int2(ok ? (int)((uint32_t)k & keep) : 0x7FFFFFFF, ok ? c : -1);
        }
    }
    __syncthreads();
    for (int row = t; row < rows_here; row += C::THREADS) {
        int bk[4] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
        int bc[4] = {-1, -1, -1, -1};
        for (int e = 0; e < LISTS * 4; ++e) {
            const int2 v = mc[row * LISTS * 4 + e];
            int k = v.x, c = v.y;
#pragma unroll
            for (int q = 3; q >= 0; --q)
                if (cand_before(k, c, bk[q], bc[q])) {
                    const int tk = bk[q], tc = bc[q];
                    bk[q] = k; bc[q] = c; k = tk; c = tc;
                }
        }
        int2* out = cand + ((r0 + row) * parts + p) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = make_int2(bk[q], bc[q]);
    }
    if constexpr (CONF) {
        float2* ml = reinterpret_cast<float2*>(mc + ROWS * LISTS * 4);
#pragma unroll
        for (int jx = 0; jx < FX; ++jx) ml[(32 * jx + fr) * LISTS + 2 * wn + hf] = make_float2(lm[jx], ls[jx]);
        __syncthreads();
        for (int row = t; row < rows_here; row += C::THREADS) {
            float m = -INFINITY;
            for (int e = 0; e < LISTS; ++e) m = fmaxf(m, ml[row * LISTS + e].x);
            float sum = 0.f;
            for (int e = 0; e < LISTS; ++e) {
                const float2 q = ml[row * LISTS + e];
                if (q.x > -INFINITY) sum += q.y * __expf(q.x - m);
            }
            lse[(r0 + row) * parts + p] = make_float2(m, sum);
        }
    }
}

template <bool V4, bool CONF>
__global__ void __launch_bounds__(256) vq_rescore_kernel(const float* __restrict__ X, int64_t N, int D,
                                                        const float* __restrict__ E, int K,
                                                        const int2* __restrict__ cand, int parts,
                                                        int32_t* __restrict__ idx, float* __restrict__ dist,
                                                        const float2* __restrict__ lse,
                                                        float* __restrict__ conf) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= N) return;  // uniform per wave
    // The row's 4 * parts (<= 64) candidates, one per lane; four rounds of a
    // wavefront minimum in registers (lane swaps and DPP) pick them in order.
    const int nc = 4 * parts;
    const int2 v = lane < nc ? cand[row * nc + lane] : make_int2(0x7FFFFFFF, -1);
    int ck = v.x, cc = v.y;
    int pick[4];
    auto take = [&](int& bk, int& bc, int ok, int oc) {
        if (cand_before(ok, oc, bk, bc)) { bk = ok; bc = oc; }
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int bk = ck, bc = cc;
        take(bk, bc, xlane_partner<32>(bk, lane), xlane_partner<32>(bc, lane));
        take(bk, bc, xlane_partner<16>(bk, lane), xlane_partner<16>(bc, lane));
        take(bk, bc, xlane_partner<8>(bk, lane), xlane_partner<8>(bc, lane));
        take(bk, bc, xlane_partner<4>(bk, lane), xlane_partner<4>(bc, lane));
        take(bk, bc, xlane_partner<2>(bk, lane), xlane_partner<2>(bc, lane));
        take(bk, bc, xlane_partner<1>(bk, lane), xlane_partner<1>(bc, lane));
        pick[q] = __builtin_amdgcn_readfirstlane(bc);
        if (cc == pick[q]) cc = -1;  // codewords are distinct across lists
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
    const float* xr = X + row * D;
    const float* er[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) er[q] = E + (size_t)(pick[q] >= 0 ? pick[q] : 0) * D;
    if constexpr (V4) {
#pragma unroll 4
        for (int d4 = lane; d4 < D / 4; d4 += 64) {
            const f32x4_t xv = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(xr) + d4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4_t ev = reinterpret_cast<const f32x4_t*>(er[q])[d4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float df = xv[k] - ev[k];
                    part[q] += df * df;
                }
            }
        }
    } else {
        for (int d = lane; d < D; d += 64) {
            const float xv = xr[d];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float df = xv - er[q][d];
                part[q] += df * df;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q] = wave_sum(part[q]);
    if (lane == 0) {
        float bd = INFINITY;
        int bi = 0x7FFFFFFF;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (pick[q] >= 0 && better(part[q], pick[q], bd, bi)) { bd = part[q]; bi = pick[q]; }
        idx[row] = bi;
        dist[row] = bd;
    }
    if constexpr (CONF) {
        // merge the parts' (m, s): conf = max_k p_k = 1 / sum_k exp(v_k - max v)
        float2 q = lane < parts ? lse[row * parts + lane] : make_float2(-INFINITY, 0.f);
        const float m = wave_max(q.x);
        const float sum = wave_sum(q.x > -INFINITY ? q.y * __expf(q.x - m) : 0.f);
        if (lane == 0) conf[row] = 1.f / sum;
    }
}

// Rescore with four rows per wavefront, for up to 16 candidates per row
// (parts <= 4) and D % 4 == 0: lanes 16 r .. 16 r + 15 hold the candidates of
// row r, so each of the four selection rounds is one 4-step butterfly within
// rows of 16 lanes serving all four rows; the 16 FP32 distances (4 rows x 4
// picks) are summed by one reduce-scatter instead of 16 full wavefront sums.
// Same candidates, same picks and the same per-lane partial sums as the
// one-row form; only the order of the final cross-lane additions differs.
template <bool CONF>
__global__ void __launch_bounds__(256) vq_rescore4_kernel(const float* __restrict__ X, int64_t N, int D,
                                                         const float* __restrict__ E,
                                                         const int2* __restrict__ cand, int parts,
                                                         int32_t* __restrict__ idx, float* __restrict__ dist,
                                                         const float2* __restrict__ lse,
                                                         float* __restrict__ conf) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;
    if (row0 >= N) return;  // uniform per wave
    const int grp = lane >> 4, j = lane & 15;
    const int64_t myrow = row0 + grp;
    const int nc = 4 * parts;
    const int2 v = (j < nc && myrow < N) ? cand[myrow * nc + j] : make_int2(0x7FFFFFFF, -1);
    int ck = v.x, cc = v.y;
    int pk[4];
    auto take = [&](int& bk, int& bc, int ok, int oc) {
        if (cand_before(ok, oc, bk, bc)) { bk = ok; bc = oc; }
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int bk = ck, bc = cc;
        take(bk, bc, xlane_partner<8>(bk, lane), xlane_partner<8>(bc, lane));
        take(bk, bc, xlane_partner<4>(bk, lane), xlane_partner<4>(bc, lane));
        take(bk, bc, xlane_partner<2>(bk, lane), xlane_partner<2>(bc, lane));
        take(bk, bc, xlane_partner<1>(bk, lane), xlane_partner<1>(bc, lane));
        pk[q] = bc;
        if (cc == bc) cc = -1;  // codewords are distinct across lists
    }
    int pick[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) pick[r][q] = __builtin_amdgcn_readlane(pk[q], 16 * r);
    float a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = 0.f;
    const int D4 = D / 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (row0 + r >= N) break;  // uniform
        const f32x4_t* xr = reinterpret_cast<const f32x4_t*>(X + (row0 + r) * D);
        const f32x4_t* er[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            er[q] = reinterpret_cast<const f32x4_t*>(E + (size_t)(pick[r][q] >= 0 ? pick[r][q] : 0) * D);
#pragma unroll 3
        for (int d4 = lane; d4 < D4; d4 += 64) {
            const f32x4_t xv = __builtin_nontemporal_load(xr + d4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4_t ev = er[q][d4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float df = xv[k] - ev[k];
                    a[4 * r + q] += df * df;
                }
            }
        }
    }
    int my_id = 0;
    bool my_own = false;
    rs_layout<16>(lane, &my_id, &my_own);
    reduce_scatter<16>(a, lane);
    // sum id = 4 r + q now sits in a[0] of its owning lane
    float sums[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint64_t m = __ballot(my_own && my_id == k);
        sums[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[0]), (int)__builtin_ctzll(m)));
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (row0 + r >= N) break;
        float bd = INFINITY;
        int bi = 0x7FFFFFFF;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (pick[r][q] >= 0 && better(sums[4 * r + q], pick[r][q], bd, bi)) { bd = sums[4 * r + q]; bi = pick[r][q]; }
        if (lane == r) {
            idx[row0 + r] = bi;
            dist[row0 + r] = bd;
        }
    }
    if constexpr (CONF) {
        // merge the parts' (m, s) of each row within its 16 lanes
        float2 q = (j < parts && myrow < N) ? lse[myrow * parts + j] : make_float2(-INFINITY, 0.f);
        float m = q.x;
        m = fmaxf(m, xlane_dpp<8>(m));
        m = fmaxf(m, xlane_dpp<4>(m));
        m = fmaxf(m, xlane_dpp<2>(m));
        m = fmaxf(m, xlane_dpp<1>(m));
        float sum = q.x > -INFINITY ? q.y * __expf(q.x - m) : 0.f;
        sum += xlane_dpp<8>(sum);
        sum += xlane_dpp<4>(sum);
        sum += xlane_dpp<2>(sum);
        sum += xlane_dpp<1>(sum);
        if (j == 0 && myrow < N) conf[myrow] = 1.f / sum;
    }
}

struct VqWs {
    uint16_t* xa;
    uint16_t* ea;
    int2* cand;
    float2* lse;
};

struct VqPlan {
    int tiles, tiles_part, parts, seq_bits;
};

static VqPlan vq_plan(int K) {
    VqPlan p;
    p.tiles = (K + Q_BN - 1) / Q_BN;
    // At least Q_MIN_PARTS parts when there are enough tiles: the parts of a
    // row block share its X chunks in one L2 (the sweep reads them once per
    // tile).
    p.parts = std::max((p.tiles + Q_MAX_TILES - 1) / Q_MAX_TILES, std::min(Q_MIN_PARTS, p.tiles));
    p.tiles_part = (p.tiles + p.parts - 1) / p.parts;
    p.parts = (p.tiles + p.tiles_part - 1) / p.tiles_part;
    int b = 0;
    while ((1 << b) < p.tiles_part) ++b;
    p.seq_bits = 6 + b;
    return p;
}

static int vq_dp(int D) { return (D + Q_BK - 1) / Q_BK * Q_BK; }
static int64_t vq_np(int64_t N) { return (N + VqCfg::ROWS - 1) / VqCfg::ROWS * VqCfg::ROWS; }

static VqWs carve_vq(void* base, int64_t N, int D, const VqPlan& plan, size_t* bytes) {
    Carve c(base);
    VqWs w;
    const int64_t n1 = N > 0 ? N : 1;
    const size_t dx = (size_t)vq_dp(D) + Q_BK;
    w.xa = c.take<uint16_t>((size_t)vq_np(n1) * dx);
    w.ea = c.take<uint16_t>((size_t)plan.parts * plan.tiles_part * Q_BN * dx);
    w.cand = c.take<int2>((size_t)n1 * plan.parts * 4);
    w.lse = c.take<float2>((size_t)n1 * plan.parts);
    *bytes = c.total();
    return w;
}

// ------------------------------------------------------------------- EMA
// Key = the assigned codeword; rows below the confidence threshold (App. C,
// Eq. (mask_confidence)) go to the extra segment K, which no codeword reads.
__global__ void ema_keys_kernel(const int32_t* __restrict__ idx, int64_t N, int K,
                                const float* __restrict__ conf, float gamma,
                                uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                int64_t* __restrict__ count) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0) *count = N;
    if (n >= N) return;
    int a = idx[n];
    a = a < 0 ? 0 : (a >= K ? K - 1 : a);
    if (conf && !(conf[n] >= gamma)) a = K;
    keys[n] = (uint64_t)(uint32_t)a;
    vals[n] = (uint32_t)n;
}

// Dead codes (App. C, Eq. (dead_code)): N_k < delta after the EMA step.  One
// workgroup ranks them in codeword order: rank[k] = j for the j-th dead code,
// -1 otherwise; *n_dead = their number.
__global__ void __launch_bounds__(1024) ema_dead_rank_kernel(const float* __restrict__ N_ema, int K, float delta,
                                                            int32_t* __restrict__ rank, int32_t* __restrict__ n_dead) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (K + 1023) / 1024;
    const int k0 = t * per, k1 = min(K, k0 + per);
    int c = 0;
    for (int k = k0; k < k1; ++k) c += N_ema[k] < delta;
    part[t] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan (Hillis-Steele)
        const int v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int j = part[t] - c;
    for (int k = k0; k < k1; ++k) rank[k] = N_ema[k] < delta ? j++ : -1;
    if (t == 1023 && n_dead) *n_dead = part[1023];
}

// M_k <- reservoir[(offset + rank_k) mod R], N_k <- 1 + eps for dead codes.
__global__ void __launch_bounds__(256) ema_dead_reinit_kernel(const int32_t* __restrict__ rank, int D,
                                                             const float* __restrict__ reservoir, int R,
                                                             int64_t offset, float eps, float* __restrict__ N_ema,
                                                             float* __restrict__ M_ema) {
    const int k = blockIdx.x;
    const int j = rank[k];
    if (j < 0) return;
    const int64_t r = (offset + j) % R;
    for (int d = threadIdx.x; d < D; d += 256) M_ema[(size_t)k * D + d] = reservoir[(size_t)r * D + d];
    if (threadIdx.x == 0) N_ema[k] = 1.f + eps;
}

__global__ void ema_zero_i32_kernel(int32_t* __restrict__ p) { *p = 0; }

// One workgroup per codeword: counts, row sums in ascending row order, EMA of
// N and M.  Row ids are staged in LDS; each thread owns up to 4 columns and
// issues the loads of 8 rows before adding them in order, so the sum order
// (and hence the result) does not depend on timing.
constexpr int EMA_COLS = 4, EMA_ROWS = 8;
// Rows per piece of the EMA sums: a code with n rows is summed as ceil(n / P)
// pieces (one workgroup each), so a popular code does not leave one long
// workgroup behind.
constexpr int EMA_PIECE = 128;

// One workgroup: the pieces of each code (ceil(n_l / P) for its n_l rows) and
// their exclusive prefix poff[0..K]; each thread takes a contiguous run of
// codes, so the pieces of a code are consecutive and in row order.
__global__ void __launch_bounds__(1024) ema_pieces_kernel(const uint32_t* __restrict__ ranges, int K,
                                                         uint32_t* __restrict__ poff) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (K + 1023) / 1024;
    const int k0 = min(K, t * per), k1 = min(K, k0 + per);
    uint32_t c = 0;
    for (int k = k0; k < k1; ++k) c += (ranges[2 * k + 1] - ranges[2 * k] + EMA_PIECE - 1) / EMA_PIECE;
    part[t] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - c;
    for (int k = k0; k < k1; ++k) {
        poff[k] = run;
        run += (ranges[2 * k + 1] - ranges[2 * k] + EMA_PIECE - 1) / EMA_PIECE;
    }
    if (t == 1023) poff[K] = part[1023];
}

// One workgroup per piece: the column sums of its (at most P) rows, added in
// row order, into partial[piece][:].  The piece's code comes from a binary
// search of poff.
__global__ void __launch_bounds__(256) ema_piece_sum_kernel(const float* __restrict__ X, int D,
                                                           const uint32_t* __restrict__ rows,
                                                           const uint32_t* __restrict__ ranges,
                                                           const uint32_t* __restrict__ poff, int K,
                                                           float* __restrict__ partial) {
    __shared__ uint32_t rid[EMA_PIECE];
    const uint32_t pc = blockIdx.x, t = threadIdx.x;
    if (pc >= poff[K]) return;
    int lo = 0, hi = K - 1;  // last code with poff <= pc (codes with no pieces share poff)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (poff[mid] <= pc) lo = mid; else hi = mid - 1;
    }
    const uint32_t b = ranges[2 * lo] + (pc - poff[lo]) * EMA_PIECE;
    const uint32_t e = min(b + (uint32_t)EMA_PIECE, ranges[2 * lo + 1]);
    if (t < e - b) rid[t] = rows[b + t];
    __syncthreads();
    const int cnt = (int)(e - b);
    float* out = partial + (size_t)pc * D;
    for (int d0 = 0; d0 < D; d0 += 256 * EMA_COLS) {
        float acc[EMA_COLS];
#pragma unroll
        for (int c = 0; c < EMA_COLS; ++c) acc[c] = 0.f;
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
#pragma unroll
        for (int c = 0; c < EMA_COLS; ++c) {
            const int d = d0 + t + 256 * c;
            if (d < D) out[d] = acc[c];
        }
    }
}

// One workgroup per code: the code's sum is its pieces' sums added in piece
// order (fixed by the row counts alone, so the result is reproducible), then
// the EMA step of Eq. (ema_update) on N and M.
__global__ void __launch_bounds__(256) ema_combine_kernel(const float* __restrict__ partial, int D,
                                                         const uint32_t* __restrict__ ranges,
                                                         const uint32_t* __restrict__ poff, float decay,
                                                         float* __restrict__ N_ema, float* __restrict__ M_ema,
                                                         float* __restrict__ counts) {
    const int l = blockIdx.x, t = threadIdx.x;
    const uint32_t p0 = poff[l], p1 = poff[l + 1];
    for (int d = t; d < D; d += 256) {
        float acc = 0.f;
        for (uint32_t q = p0; q < p1; ++q) acc += partial[(size_t)q * D + d];
        float* m = M_ema + (size_t)l * D + d;
        *m = decay * *m + (1.f - decay) * acc;
    }
    if (t == 0) {
        const float c = (float)(ranges[2 * l + 1] - ranges[2 * l]);
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
    int32_t* rank;
    uint32_t* poff;   // [K + 1] first piece of each code, poff[K] = number of pieces
    float* partial;   // [max pieces][D] per-piece column sums
};

inline int64_t ema_max_pieces(int64_t N, int K) { return (N + EMA_PIECE - 1) / EMA_PIECE + (K > 0 ? K : 1); }

static EmaWs carve_ema(void* base, int64_t N, int D, int K, size_t* bytes) {
    Carve c(base);
    EmaWs w;
    const int64_t n1 = N > 0 ? N : 1;
    w.keys = c.take<uint64_t>(n1);
    w.vals = c.take<uint32_t>(n1);
    w.keys_alt = c.take<uint64_t>(n1);
    w.vals_alt = c.take<uint32_t>(n1);
    w.hist = c.take<uint32_t>(radix_hist_words(n1));
    w.ranges = c.take<uint32_t>(2 * (size_t)(K > 0 ? K + 1 : 2));
    w.count = c.take<int64_t>(1);
    w.total = c.take<float>(1);
    w.rank = c.take<int32_t>((size_t)(K > 0 ? K : 1));
    w.poff = c.take<uint32_t>((size_t)(K > 0 ? K + 1 : 2));
    w.partial = c.take<float>((size_t)ema_max_pieces(N, K) * (size_t)(D > 0 ? D : 1));
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
    if (precision != XGS_VQ_BF16_RESCORE4 || D < 1 || K < 1) return 0;
    size_t bytes = 0;
    carve_vq(nullptr, N < 0 ? 0 : N, D, vq_plan(K), &bytes);
    return bytes;
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

// Checks the BF16 sizes and carves the workspace.
static xgs_status vq_bf16_setup(const char* who, int64_t N, int32_t D, int32_t K, void* ws, size_t ws_bytes,
                                VqPlan* plan, VqWs* w) {
    if (N < 0 || D < 1 || K < 1) return fail(XGS_ERR_INVALID_ARG, std::string(who) + ": bad sizes");
    if (D % 8 != 0) return fail(XGS_ERR_UNSUPPORTED, std::string(who) + ": BF16 path needs D % 8 == 0");
    if (N > (int64_t)1 << 40) return fail(XGS_ERR_UNSUPPORTED, std::string(who) + ": N too large");
    *plan = vq_plan(K);
    if (plan->parts > Q_MAX_PARTS) return fail(XGS_ERR_UNSUPPORTED, std::string(who) + ": K above 65536");
    const int64_t dx = vq_dp(D) + Q_BK;
    if ((int64_t)plan->parts * plan->tiles_part * Q_BN * dx >= ((int64_t)1 << 31) ||
        (int64_t)VqCfg::ROWS * dx >= ((int64_t)1 << 30))
        return fail(XGS_ERR_UNSUPPORTED, std::string(who) + ": codebook above 2^31 bf16 elements");
    if (((N + VqCfg::ROWS - 1) / VqCfg::ROWS + 7) / 8 * 8 * plan->parts >= ((int64_t)1 << 31))
        return fail(XGS_ERR_UNSUPPORTED, std::string(who) + ": N too large");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, std::string(who) + ": workspace must be 256-byte aligned");
    size_t need = 0;
    *w = carve_vq(ws, N, D, *plan, &need);
    if (!ws || ws_bytes < need) return fail(XGS_ERR_CAPACITY, std::string(who) + ": workspace too small");
    return XGS_OK;
}

extern "C" xgs_status xgs_vq_stage(const float* X, int64_t N, int32_t D, const uint16_t* E_bf16,
                                   const float* e_norm2, int32_t K, void* ws, size_t ws_bytes,
                                   xgs_stream_t stream) {
    clear_error();
    VqPlan plan;
    VqWs w;
    if (xgs_status s = vq_bf16_setup("xgs_vq_stage", N, D, K, ws, ws_bytes, &plan, &w)) return s;
    if ((N > 0 && !X) || !E_bf16 || !e_norm2) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_stage: null pointer");
    if (!aligned(X, 16) || !aligned(E_bf16, 16))
        return fail(XGS_ERR_INVALID_ARG, "xgs_vq_stage: X and E_bf16 must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int Dp = vq_dp(D), Dx = Dp + Q_BK;
    const int Kp = plan.parts * plan.tiles_part * Q_BN;
    if (N > 0)
        hipLaunchKernelGGL(vq_xprep_kernel, dim3((unsigned)((vq_np(N) + 3) / 4)), dim3(256), 0, st, X, N, vq_np(N), D, Dp,
                           Dx, VqCfg::ROWS, w.xa);
    hipLaunchKernelGGL(vq_eprep_kernel, dim3((unsigned)((Kp + 3) / 4)), dim3(256), 0, st, E_bf16, e_norm2, K, D, Kp,
                       Dp, Dx, w.ea);
    return check_launch("xgs_vq_stage");
}

extern "C" xgs_status xgs_vq_candidates(int64_t N, int32_t D, int32_t K, void* ws, size_t ws_bytes,
                                        xgs_stream_t stream) {
    clear_error();
    VqPlan plan;
    VqWs w;
    if (xgs_status s = vq_bf16_setup("xgs_vq_candidates", N, D, K, ws, ws_bytes, &plan, &w)) return s;
    if (N == 0) return XGS_OK;
    const int64_t blocks = ((N + VqCfg::ROWS - 1) / VqCfg::ROWS + 7) / 8 * 8 * plan.parts;
    hipLaunchKernelGGL((vq_gemm_ereg_kernel<VqRegCfg, false>), dim3((unsigned)blocks), dim3(VqRegCfg::THREADS), 0, (hipStream_t)stream, w.xa, N,
                       vq_dp(D) + Q_BK, w.ea, K, plan.parts, plan.tiles_part, plan.seq_bits, w.cand, 0.f, nullptr);
    return check_launch("xgs_vq_candidates");
}

// Four rows per wavefront when the rows have at most 16 candidates and the
// rows are float4-aligned; one row per wavefront otherwise.
template <bool CONF>
static void launch_rescore(const float* X, int64_t N, int D, const float* E, int K, const int2* cand, int parts,
                           int32_t* idx, float* dist, const float2* lse, float* conf, hipStream_t st) {
    const bool v4 = D % 4 == 0 && aligned(X, 16) && aligned(E, 16);
    if (v4 && parts <= 4) {
        const unsigned blocks = (unsigned)((N + 15) / 16);
        hipLaunchKernelGGL((vq_rescore4_kernel<CONF>), dim3(blocks), dim3(256), 0, st, X, N, D, E, cand, parts, idx,
                           dist, lse, conf);
        return;
    }
    const unsigned blocks = (unsigned)((N + 3) / 4);
    if (v4)
        hipLaunchKernelGGL((vq_rescore_kernel<true, CONF>), dim3(blocks), dim3(256), 0, st, X, N, D, E, K, cand, parts,
                           idx, dist, lse, conf);
    else
        hipLaunchKernelGGL((vq_rescore_kernel<false, CONF>), dim3(blocks), dim3(256), 0, st, X, N, D, E, K, cand,
                           parts, idx, dist, lse, conf);
}

extern "C" xgs_status xgs_vq_rescore(const float* X, int64_t N, int32_t D, const float* E, int32_t K,
                                     int32_t* idx, float* dist, void* ws, size_t ws_bytes, xgs_stream_t stream) {
    clear_error();
    VqPlan plan;
    VqWs w;
    if (xgs_status s = vq_bf16_setup("xgs_vq_rescore", N, D, K, ws, ws_bytes, &plan, &w)) return s;
    if (N == 0) return XGS_OK;
    if (!X || !E || !idx || !dist) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_rescore: null pointer");
    launch_rescore<false>(X, N, D, E, K, w.cand, plan.parts, idx, dist, nullptr, nullptr, (hipStream_t)stream);
    return check_launch("xgs_vq_rescore");
}

extern "C" xgs_status xgs_vq_assign_conf(const float* X, int64_t N, int32_t D, const float* E,
                                         const uint16_t* E_bf16, const float* e_norm2, int32_t K, float tau,
                                         int32_t* idx, float* dist, float* conf, void* ws, size_t ws_bytes,
                                         xgs_stream_t stream) {
    clear_error();
    VqPlan plan;
    VqWs w;
    if (xgs_status s = vq_bf16_setup("xgs_vq_assign_conf", N, D, K, ws, ws_bytes, &plan, &w)) return s;
    if (!(tau > 0.f)) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign_conf: tau must be positive");
    if (N == 0) return XGS_OK;
    if (!X || !E || !idx || !dist || !conf) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign_conf: null pointer");
    if (xgs_status s = xgs_vq_stage(X, N, D, E_bf16, e_norm2, K, ws, ws_bytes, stream)) return s;
    hipStream_t st = (hipStream_t)stream;
    const int64_t gb = ((N + VqCfg::ROWS - 1) / VqCfg::ROWS + 7) / 8 * 8 * plan.parts;
    hipLaunchKernelGGL((vq_gemm_kernel<VqCfg, true>), dim3((unsigned)gb), dim3(VqCfg::THREADS), 0, st, w.xa, N, vq_dp(D) + Q_BK, w.ea, K,
                       plan.parts, plan.tiles_part, plan.seq_bits, w.cand, 1.f / tau, w.lse);
    launch_rescore<true>(X, N, D, E, K, w.cand, plan.parts, idx, dist, w.lse, conf, st);
    return check_launch("xgs_vq_assign_conf");
}

extern "C" xgs_status xgs_vq_assign(const float* X, int64_t N, int32_t D, const float* E,
                                    const uint16_t* E_bf16, const float* e_norm2, int32_t K,
                                    int32_t precision, int32_t* idx, float* dist, void* ws,
                                    size_t ws_bytes, xgs_stream_t stream) {
    clear_error();
    if (N < 0 || D < 1 || K < 1) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: bad sizes");
    if (precision != XGS_VQ_FP32 && precision != XGS_VQ_BF16_RESCORE4)
        return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: unknown precision");
    if (N == 0) return XGS_OK;
    if (!X || !E || !idx || !dist) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: null pointer");
    if (N > (int64_t)1 << 40) return fail(XGS_ERR_UNSUPPORTED, "xgs_vq_assign: N too large");
    if (precision == XGS_VQ_FP32) {
        const int64_t blocks = (N + P_BM - 1) / P_BM;
        hipLaunchKernelGGL(vq_fp32_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, X, N, D, E, K,
                           idx, dist);
        return check_launch("xgs_vq_assign fp32");
    }
    if (!E_bf16 || !e_norm2) return fail(XGS_ERR_INVALID_ARG, "xgs_vq_assign: bf16 shadow or norms missing");
    if (xgs_status s = xgs_vq_stage(X, N, D, E_bf16, e_norm2, K, ws, ws_bytes, stream)) return s;
    if (xgs_status s = xgs_vq_candidates(N, D, K, ws, ws_bytes, stream)) return s;
    return xgs_vq_rescore(X, N, D, E, K, idx, dist, ws, ws_bytes, stream);
}

extern "C" size_t xgs_vq_ema_workspace(int64_t N, int32_t D, int32_t K) {
    size_t bytes = 0;
    carve_ema(nullptr, N < 0 ? 0 : N, D, K, &bytes);
    return bytes;
}

// One EMA step: optional confidence mask on the samples, optional dead-code
// reinitialisation after the decay step.
static xgs_status ema_impl(const char* who, const float* X, const int32_t* idx, const float* conf, float gamma,
                           int64_t N, int32_t D, int32_t K, float* N_ema, float* M_ema, float* E,
                           uint16_t* E_bf16, float* e_norm2, float* counts, float decay, float eps, int32_t mode,
                           float delta, const float* reservoir, int32_t R, int64_t offset, int32_t* n_dead,
                           void* ws, size_t ws_bytes, hipStream_t st) {
    const std::string w_ = who;
    if (N < 0 || D < 1 || K < 1) return fail(XGS_ERR_INVALID_ARG, w_ + ": bad sizes");
    if (N >= ((int64_t)1 << 32)) return fail(XGS_ERR_UNSUPPORTED, w_ + ": N must be below 2^32");
    if (K >= (1 << 30)) return fail(XGS_ERR_UNSUPPORTED, w_ + ": K too large");
    if (!(decay >= 0.f && decay < 1.f)) return fail(XGS_ERR_INVALID_ARG, w_ + ": decay must be in [0, 1)");
    if (mode != XGS_EMA_PAPER && mode != XGS_EMA_LAPLACE) return fail(XGS_ERR_INVALID_ARG, w_ + ": unknown mode");
    if ((N > 0 && (!X || !idx)) || !N_ema || !M_ema || !E) return fail(XGS_ERR_INVALID_ARG, w_ + ": null pointer");
    if ((E_bf16 == nullptr) != (e_norm2 == nullptr))
        return fail(XGS_ERR_INVALID_ARG, w_ + ": E_bf16 and e_norm2 go together");
    const bool dead_on = delta > 0.f;
    if (dead_on && (!reservoir || R < 1 || offset < 0))
        return fail(XGS_ERR_INVALID_ARG, w_ + ": dead-code reset needs a reservoir (R >= 1, offset >= 0)");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, w_ + ": workspace must be 256-byte aligned");
    size_t need = 0;
    EmaWs w = carve_ema(ws, N, D, K, &need);
    if (!ws || ws_bytes < need) return fail(XGS_ERR_CAPACITY, w_ + ": workspace too small");
    xgs_status s;
    if ((s = fill_u32(w.ranges, 2 * ((int64_t)K + 1), 0u, st))) return s;
    const int64_t n1 = N > 0 ? N : 1;
    hipLaunchKernelGGL(ema_keys_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, idx, N, K, conf, gamma,
                       w.keys, w.vals, w.count);
    if ((s = check_launch(who))) return s;
    const int bits = bits_for((int64_t)K + 1);
    if ((s = radix_sort(w.keys, w.vals, w.keys_alt, w.vals_alt, w.count, N, bits, w.hist, st))) return s;
    const bool even = radix_passes(bits, N) % 2 == 0;
    const uint64_t* sk = even ? w.keys : w.keys_alt;
    const uint32_t* sv = even ? w.vals : w.vals_alt;
    if ((s = segment_ranges(sk, w.count, N, 0, w.ranges, st))) return s;
    hipLaunchKernelGGL(ema_pieces_kernel, dim3(1), dim3(1024), 0, st, w.ranges, K, w.poff);
    hipLaunchKernelGGL(ema_piece_sum_kernel, dim3((unsigned)ema_max_pieces(N, K)), dim3(256), 0, st, X, D, sv,
                       w.ranges, w.poff, K, w.partial);
    hipLaunchKernelGGL(ema_combine_kernel, dim3((unsigned)K), dim3(256), 0, st, w.partial, D, w.ranges, w.poff,
                       decay, N_ema, M_ema, counts);
    if (dead_on) {
        hipLaunchKernelGGL(ema_dead_rank_kernel, dim3(1), dim3(1024), 0, st, N_ema, K, delta, w.rank, n_dead);
        hipLaunchKernelGGL(ema_dead_reinit_kernel, dim3((unsigned)K), dim3(256), 0, st, w.rank, D, reservoir, R, offset,
                           eps, N_ema, M_ema);
    } else if (n_dead) {
        hipLaunchKernelGGL(ema_zero_i32_kernel, dim3(1), dim3(1), 0, st, n_dead);
    }
    hipLaunchKernelGGL(ema_total_kernel, dim3(1), dim3(256), 0, st, N_ema, K, w.total);
    hipLaunchKernelGGL(ema_finalize_kernel, dim3((unsigned)K), dim3(256), 0, st, N_ema, M_ema, K, D, eps, mode,
                       w.total, E, E_bf16, e_norm2);
    return check_launch(who);
}

extern "C" xgs_status xgs_vq_ema_update(const float* X, const int32_t* idx, int64_t N, int32_t D,
                                        int32_t K, float* N_ema, float* M_ema, float* E,
                                        uint16_t* E_bf16, float* e_norm2, float* counts, float decay,
                                        float eps, int32_t mode, void* ws, size_t ws_bytes,
                                        xgs_stream_t stream) {
    clear_error();
    return ema_impl("xgs_vq_ema_update", X, idx, nullptr, 0.f, N, D, K, N_ema, M_ema, E, E_bf16, e_norm2, counts,
                    decay, eps, mode, 0.f, nullptr, 0, 0, nullptr, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" xgs_status xgs_vq_ema_update_robust(const float* X, const int32_t* idx, const float* conf, float gamma,
                                               int64_t N, int32_t D, int32_t K, float* N_ema, float* M_ema,
                                               float* E, uint16_t* E_bf16, float* e_norm2, float* counts,
                                               float decay, float eps, int32_t mode, float delta,
                                               const float* reservoir, int32_t R, int64_t offset,
                                               int32_t* n_dead, void* ws, size_t ws_bytes, xgs_stream_t stream) {
    clear_error();
    return ema_impl("xgs_vq_ema_update_robust", X, idx, conf, gamma, N, D, K, N_ema, M_ema, E, E_bf16, e_norm2,
                    counts, decay, eps, mode, delta, reservoir, R, offset, n_dead, ws, ws_bytes,
                    (hipStream_t)stream);
}
