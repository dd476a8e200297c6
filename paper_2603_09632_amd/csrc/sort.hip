// Scan and radix sort used by the binning step (and by the VQ EMA update to
// group rows by codeword).  All sizes that depend on data are read from device
// memory; grids are sized by the caller's capacity and idle blocks return.
#include "sort.h"

namespace xgs {

// ------------------------------------------------------------------ fill
__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

xgs_status fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream) {
    if (n <= 0) return XGS_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return check_launch("fill");
}

// Zero fill of up to four ranges in one launch (blockIdx.y picks the range):
// 16-byte stores for the aligned body, 4-byte stores for the ends.
__global__ void zero_ranges_kernel(ZeroRanges r) {
    uint32_t* p = r.p[blockIdx.y];
    const int64_t n = r.n[blockIdx.y];
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t head = (int64_t)(((16 - ((uintptr_t)p & 15)) & 15) / 4);  // words before 16-byte alignment
    const int64_t h = head < n ? head : n;
    const int64_t nv = (n - h) / 4;
    uint4* pv = reinterpret_cast<uint4*>(p + h);
    for (int64_t i = t0; i < nv; i += stride) pv[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t tail0 = h + 4 * nv;
    for (int64_t i = t0; i < h + (n - tail0); i += stride) p[i < h ? i : tail0 + (i - h)] = 0u;
}

xgs_status zero_ranges(const ZeroRanges& r, hipStream_t stream) {
    int64_t most = 0;
    for (int j = 0; j < r.k; ++j) most = r.n[j] > most ? r.n[j] : most;
    if (r.k <= 0 || most <= 0) return XGS_OK;
    int64_t blocks = (most / 4 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_ranges_kernel, dim3((unsigned)blocks, (unsigned)r.k), dim3(256), 0, stream, r);
    return check_launch("zero_ranges");
}

xgs_status fill_f32(float* p, int64_t n, float v, hipStream_t stream) {
    union { float f; uint32_t u; } c;
    c.f = v;
    return fill_u32(reinterpret_cast<uint32_t*>(p), n, c.u, stream);
}

// ------------------------------------------------------------------ scan
// Block-wide inclusive scan of one u64 per thread (256 threads).
__device__ __forceinline__ uint64_t block_incl_scan_256(uint64_t v, uint64_t* sh) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    if (lane == 63) sh[w] = v;
    __syncthreads();
    uint64_t add = 0;
    for (int k = 0; k < w; ++k) add += sh[k];
    __syncthreads();
    return v + add;
}

// zero_p (optional): zero_n words cleared by the same grid (a buffer the
// caller needs cleared before later stages, folded in to save a launch).
__global__ void __launch_bounds__(256) scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                         uint64_t* __restrict__ partials,
                                                         uint32_t* __restrict__ zero_p, int64_t zero_n) {
    __shared__ uint64_t sh[4];
    if (zero_p)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < zero_n; i += (int64_t)gridDim.x * 256)
            zero_p[i] = 0u;
    int64_t base = (int64_t)blockIdx.x * kScanItems;
    // every load is issued before the first add (a guarded add per load would
    // wait for each load in turn)
    uint32_t v[kScanItems / 256];
#pragma unroll
    for (int r = 0; r < kScanItems / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        v[r] = i < n ? in[i] : 0u;
    }
    uint64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems / 256; ++r) s += v[r];
    uint64_t incl = block_incl_scan_256(s, sh);
    if (threadIdx.x == 255) partials[blockIdx.x] = incl;
}

// One block: exclusive scan of the block partials in place, then the total.
__global__ void __launch_bounds__(256) scan_partials_kernel(uint64_t* partials, int64_t nb,
                                                           int64_t* total, int64_t cap,
                                                           int64_t* count, int32_t* status) {
    __shared__ uint64_t sh[4];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        int64_t i = b0 + threadIdx.x;
        uint64_t v = i < nb ? partials[i] : 0;
        uint64_t incl = block_incl_scan_256(v, sh);
        uint64_t c = carry;
        if (i < nb) partials[i] = c + incl - v;
        __syncthreads();
        if (threadIdx.x == 255) carry = c + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint64_t tot = carry;
        partials[nb] = tot;
        if (total) *total = (int64_t)tot;
        if (cap >= 0) {
            // on overflow nothing is sorted: the lists are empty and status says why
            *count = (int64_t)(tot > (uint64_t)cap ? 0 : tot);
            *status = tot > (uint64_t)cap ? 1 : 0;
        }
    }
}

__global__ void __launch_bounds__(256) scan_apply_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                        const uint64_t* __restrict__ partials,
                                                        uint64_t* __restrict__ out) {
    __shared__ uint64_t sh[4];
    constexpr int per = kScanItems / 256;  // consecutive items per thread
    int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * per;
    uint32_t v[per];
    uint64_t s = 0;
#pragma unroll
    for (int r = 0; r < per; ++r) {
        int64_t i = base + r;
        v[r] = i < n ? in[i] : 0u;
        s += v[r];
    }
    uint64_t incl = block_incl_scan_256(s, sh);
    uint64_t run = partials[blockIdx.x] + incl - s;
#pragma unroll
    for (int r = 0; r < per; ++r) {
        int64_t i = base + r;
        if (i < n) out[i] = run;
        run += v[r];
    }
}

// Apply without the separate partials pass: block b sums the block totals
// partials[0..b) itself (nb <= kFusedScanBlocks keeps that cheap), and the
// last block writes the total, count and status as scan_partials_kernel does.

__global__ void __launch_bounds__(256) scan_apply_fused_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                              const uint64_t* __restrict__ partials, int64_t nb,
                                                              uint64_t* __restrict__ out, int64_t* __restrict__ total,
                                                              int64_t cap, int64_t* __restrict__ count,
                                                              int32_t* __restrict__ status) {
    __shared__ uint64_t sh[4];
    __shared__ uint64_t red[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint64_t acc = 0;
    for (int64_t j = t; j < (int64_t)blockIdx.x; j += 256) acc += partials[j];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    const uint64_t base = (red[0] + red[1]) + (red[2] + red[3]);
    constexpr int per = kScanItems / 256;  // consecutive items per thread
    const int64_t first = (int64_t)blockIdx.x * kScanItems + (int64_t)t * per;
    uint32_t v[per];
    uint64_t s = 0;
#pragma unroll
    for (int r = 0; r < per; ++r) {
        const int64_t i = first + r;
        v[r] = i < n ? in[i] : 0u;
        s += v[r];
    }
    const uint64_t incl = block_incl_scan_256(s, sh);
    uint64_t run = base + incl - s;
#pragma unroll
    for (int r = 0; r < per; ++r) {
        const int64_t i = first + r;
        if (i < n) out[i] = run;
        run += v[r];
    }
    if (blockIdx.x == nb - 1 && t == 255) {
        const uint64_t tot = base + incl;  // thread 255's inclusive sum is the block total
        if (total) *total = (int64_t)tot;
        if (cap >= 0) {
            // on overflow nothing is sorted: the lists are empty and status says why
            *count = (int64_t)(tot > (uint64_t)cap ? 0 : tot);
            *status = tot > (uint64_t)cap ? 1 : 0;
        }
    }
}

xgs_status scan_block_totals(const uint32_t* in, int64_t n, uint64_t* partials, uint32_t* zero_p, int64_t zero_n,
                             hipStream_t stream) {
    const int64_t nb = scan_blocks(n);
    if (nb <= 0) return XGS_OK;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, stream, in, n, partials, zero_p, zero_n);
    return check_launch("scan_block_totals");
}

xgs_status exclusive_scan_u32(const uint32_t* in, int64_t n, uint64_t* out, uint64_t* partials,
                              int64_t* total, int64_t cap, int64_t* count, int32_t* status,
                              uint32_t* zero_p, int64_t zero_n, hipStream_t stream) {
    int64_t nb = scan_blocks(n);
    if (nb > 0 && nb <= kFusedScanBlocks) {
        hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, stream, in, n, partials, zero_p,
                           zero_n);
        hipLaunchKernelGGL(scan_apply_fused_kernel, dim3((unsigned)nb), dim3(256), 0, stream, in, n, partials, nb,
                           out, total, cap, count, status);
        return check_launch("scan");
    }
    if (zero_p) {
        if (xgs_status s = fill_u32(zero_p, zero_n, 0u, stream)) return s;
    }
    if (nb > 0)
        hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, stream, in, n, partials,
                           (uint32_t*)nullptr, (int64_t)0);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(256), 0, stream, partials, nb, total, cap,
                       count, status);
    if (nb > 0)
        hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, stream, in, n, partials, out);
    return check_launch("scan");
}

// ------------------------------------------------------------ radix sort
// The grids cover the capacity; only the ceil(count / kSortItems) blocks that
// hold keys take part (the others return at once and their histogram columns
// are never read), so the cost follows the instance count.
//
// Per block: digit histogram of its kSortItems keys (BINS digits), written
// digit-major (hist[d * nb + b], nb = the grid size).
template <int BINS>
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                 const int64_t* __restrict__ count,
                                                                 int shift, uint32_t mask,
                                                                 uint32_t* __restrict__ hist) {
    constexpr int DPT = BINS / kSortThreads;  // digits per thread
    __shared__ uint32_t h[BINS];
    const int64_t m = *count;
    const int64_t base = (int64_t)blockIdx.x * kSortItems;
    if (base >= m) return;  // uniform: a column no scan reads
#pragma unroll
    for (int j = 0; j < DPT; ++j) h[threadIdx.x + kSortThreads * j] = 0;
    // all of the block's keys are loaded before any is counted (a load per
    // count would wait a full memory latency each)
    uint64_t k[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * kSortThreads + threadIdx.x;
        k[r] = i < m ? keys[i] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < m) atomicAdd(&h[(uint32_t)(k[r] >> shift) & mask], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int d = threadIdx.x + kSortThreads * j;
        hist[(int64_t)d * gridDim.x + blockIdx.x] = h[d];
    }
}

// One workgroup per digit d: exclusive scan of d's per-block counts in place
// (the offset of block b among the keys with digit d), and totals[d], over
// the blocks that hold keys (row stride nb).
__global__ void __launch_bounds__(256) radix_scan_kernel(uint32_t* __restrict__ hist,
                                                        uint32_t* __restrict__ totals, int64_t nb,
                                                        const int64_t* __restrict__ count) {
    __shared__ uint32_t ws[4];
    const int d = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t* row = hist + (int64_t)d * nb;
    const int64_t m = *count;
    const int64_t nbe = m <= 0 ? 0 : min(nb, (m + kSortItems - 1) / kSortItems);
    uint32_t carry = 0;
    // the first four chunks of the row are loaded together
    constexpr int PRE = 4;
    uint32_t pv[PRE];
#pragma unroll
    for (int c = 0; c < PRE; ++c) {
        const int64_t i = (int64_t)c * 256 + t;
        pv[c] = i < nbe ? row[i] : 0u;
    }
    for (int64_t b0 = 0; b0 < nbe; b0 += 256) {
        const int64_t i = b0 + t;
        uint32_t v = 0u;
#pragma unroll
        for (int c = 0; c < PRE; ++c)
            if (b0 == (int64_t)c * 256) v = pv[c];
        if (b0 >= (int64_t)PRE * 256) v = i < nbe ? row[i] : 0u;
        const uint32_t incl = wave_incl_scan(v, lane);
        if (lane == 63) ws[w] = incl;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = ws[k];
            pre += k < w ? x : 0u;
            tot += x;
        }
        if (i < nbe) row[i] = carry + pre + incl - v;
        carry += tot;
        __syncthreads();
    }
    if (t == 0) totals[d] = carry;
}

// Stable scatter of BINS digits.  Wavefront w of the block owns the
// contiguous run of kSortRounds * 64 items that starts at base + w *
// kSortRounds * 64, so the block order of equal digits is (wave, round, lane)
// and the waves meet at a few barriers only (the digit bases, then two).
// Each wave first ranks every one of its items among the equal digits of its
// round (the lanes whose digit ballots agree) and counts its digits into its
// own LDS row; one barrier later thread t turns the four wave counts of each
// of its digits (t, t + 256, ...) into the wave bases (the digit's global
// base from the totals and the block's offset from the scanned histogram,
// plus the counts of the earlier waves); a second barrier later every wave
// walks its rounds again in order, each item going to its wave base plus its
// rank, the digit's first lane moving that base on by the round's count.  LDS
// operations of one wave complete in issue order, so a wave's own counter row
// needs no barrier.
template <int BINS>
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const int64_t* __restrict__ count, int shift, uint32_t mask,
    int nbits, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals) {
    constexpr int kWaves = kSortThreads / 64;
    constexpr int DPT = BINS / kSortThreads;  // digits per thread
    static_assert(kWaves == 4 && kSortRounds * 64 * kWaves == kSortItems, "four wavefronts per sort block");
    __shared__ uint32_t run[kWaves][BINS];
    __shared__ uint32_t ws[DPT][kWaves];
    const int64_t m = *count;
    const int64_t base = (int64_t)blockIdx.x * kSortItems;
    if (base >= m) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t wbase = base + (int64_t)w * (kSortRounds * 64) + lane;
    // every round's pair is loaded up front: a load issued per round would
    // put a full memory latency between consecutive rounds
    uint64_t rkey[kSortRounds];
    uint32_t rval[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = wbase + r * 64;
        rkey[r] = i < m ? kin[i] : 0ull;
        rval[r] = i < m ? vin[i] : 0u;
    }
    // digit d's base for this block (d = t + 256 j): exclusive prefix of the
    // digit totals plus the block's offset among the keys with digit d
    uint32_t g[DPT];
    {
        uint32_t tv[DPT], hv[DPT], incl[DPT];
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            tv[j] = totals[t + kSortThreads * j];
            hv[j] = hist[(int64_t)(t + kSortThreads * j) * gridDim.x + blockIdx.x];
        }
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            incl[j] = wave_incl_scan(tv[j], lane);
            if (lane == 63) ws[j][w] = incl[j];
        }
        __syncthreads();
        uint32_t carry = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            uint32_t pre = 0, tot = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) {
                const uint32_t x = ws[j][k];
                pre += k < w ? x : 0u;
                tot += x;
            }
            g[j] = carry + pre + incl[j] - tv[j] + hv[j];
            carry += tot;
        }
    }
#pragma unroll
    for (int k = 0; k < BINS / 64; ++k) run[w][lane + 64 * k] = 0u;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // rank among the round's equal digits (bits 0-7) and, for the digit's
    // first lane, the round's count of that digit (bits 8-15)
    uint32_t rc[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const bool valid = wbase + r * 64 < m;
        const uint32_t d = (uint32_t)(rkey[r] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const uint64_t bm = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bm : ~bm;
        }
        const uint32_t rank = __popcll(peers & lt), cnt = __popcll(peers);
        rc[r] = rank | (cnt << 8);
        if (valid && rank == 0) atomicAdd(&run[w][d], cnt);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int d = t + kSortThreads * j;
        const uint32_t c0 = run[0][d], c1 = run[1][d], c2 = run[2][d];
        run[0][d] = g[j];
        run[1][d] = g[j] + c0;
        run[2][d] = g[j] + c0 + c1;
        run[3][d] = g[j] + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        if (wbase + r * 64 < m) {
            const uint32_t d = (uint32_t)(rkey[r] >> shift) & mask;
            const uint32_t rank = rc[r] & 0xffu;
            const uint32_t dst = run[w][d] + rank;
            kout[dst] = rkey[r];
            vout[dst] = rval[r];
            if (rank == 0) atomicAdd(&run[w][d], rc[r] >> 8);
        }
    }
}

int radix_digit_bits(int key_bits, int64_t cap) {
    return (key_bits + 8) / 9 < (key_bits + 7) / 8 && sort_blocks(cap) <= kRadix9MaxBlocks ? 9 : 8;
}
int radix_passes(int key_bits, int64_t cap) {
    const int db = radix_digit_bits(key_bits, cap);
    return (key_bits + db - 1) / db;
}

template <int BINS>
static void radix_pass(const uint64_t* ki, const uint32_t* vi, uint64_t* ko, uint32_t* vo, const int64_t* count,
                       int64_t nb, int shift, int nbits, uint32_t* hist, hipStream_t stream) {
    const uint32_t mask = (1u << nbits) - 1u;
    uint32_t* totals = hist + (int64_t)BINS * nb;
    hipLaunchKernelGGL(radix_hist_kernel<BINS>, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, ki, count, shift,
                       mask, hist);
    hipLaunchKernelGGL(radix_scan_kernel, dim3(BINS), dim3(256), 0, stream, hist, totals, nb, count);
    hipLaunchKernelGGL(radix_scatter_kernel<BINS>, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, ki, vi, ko, vo,
                       count, shift, mask, nbits, hist, totals);
}

xgs_status radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, const int64_t* count,
                      int64_t cap, int key_bits, uint32_t* hist, hipStream_t stream) {
    int64_t nb = sort_blocks(cap);
    if (nb == 0) return XGS_OK;
    const int db = radix_digit_bits(key_bits, cap);
    const int passes = radix_passes(key_bits, cap);
    uint64_t* ki = k0; uint32_t* vi = v0; uint64_t* ko = k1; uint32_t* vo = v1;
    for (int p = 0; p < passes; ++p) {
        const int shift = db * p;
        const int nbits = key_bits - shift < db ? key_bits - shift : db;
        if (db == 9) radix_pass<512>(ki, vi, ko, vo, count, nb, shift, nbits, hist, stream);
        else radix_pass<256>(ki, vi, ko, vo, count, nb, shift, nbits, hist, stream);
        uint64_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    return check_launch("radix_sort");
}

// ---------------------------------------------------------------- ranges
__global__ void ranges_kernel(const uint64_t* __restrict__ keys, const int64_t* __restrict__ count,
                              int shift, uint32_t* __restrict__ ranges) {
    const int64_t m = *count;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    // the three keys are loaded together (in-bounds neighbours, ignored at the ends)
    const uint64_t s = keys[i] >> shift;
    const uint64_t sp = keys[i > 0 ? i - 1 : i] >> shift;
    const uint64_t sn = keys[i < m - 1 ? i + 1 : i] >> shift;
    if (i == 0 || sp != s) ranges[2 * s] = (uint32_t)i;
    if (i == m - 1 || sn != s) ranges[2 * s + 1] = (uint32_t)(i + 1);
}

xgs_status segment_ranges(const uint64_t* keys, const int64_t* count, int64_t cap, int shift,
                          uint32_t* ranges, hipStream_t stream) {
    if (cap <= 0) return XGS_OK;
    int64_t blocks = (cap + 255) / 256;
    hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, keys, count, shift,
                       ranges);
    return check_launch("ranges");
}

}  // namespace xgs
