// a2: binning of projected splats into 16x16 tiles and per-tile depth sort.
// Keys are (tile_id << 32) | bits(depth): camera depths are positive, and
// positive IEEE binary32 values order like their bit patterns.  Keys are
// emitted in Gaussian order and sorted with a stable LSD radix sort, so equal
// keys keep ascending Gaussian index.
#include <mutex>

#include "sort.h"

namespace xgs {

// Scratch of the allocation-free entry point: the library's own workspace
// for the sort, one copy per GPU (each device that runs the entry point holds
// it until the process ends).  In host code the name is a host-side stand-in:
// its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kSortScratchBytes = size_t(68) << 20;
static __device__ __align__(256) unsigned char scratch[kSortScratchBytes];
constexpr int kMaxScratchDevices = 64;
static void* g_scratch_ptr[kMaxScratchDevices];
static std::mutex g_scratch_mu;

// A wavefront's 64 consecutive Gaussians own one contiguous run of output
// positions (the offsets are their exclusive scan), so the wavefront writes
// that run together: lane l takes positions l, l + 64, ... of the run, finds
// the owning Gaussian by a 6-step search over the lanes' prefix counts and
// the tile as the row-major index within its rectangle.  Each store
// instruction then covers 64 consecutive keys.  Positions at or beyond cap
// are not written (on overflow the sort sees zero instances anyway).
//
// emit_wave: the wavefront's part, given the run's first position `base`,
// the lane's count and its inclusive prefix over the wavefront.
__device__ __forceinline__ void emit_wave(int64_t n, int64_t i0, uint64_t base, uint32_t cnt, uint32_t incl,
                                          uint32_t total, const uint2* __restrict__ tile_rect,
                                          const float4* __restrict__ splat, int64_t cap, int tiles_x,
                                          uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                          uint32_t* s_excl, uint2* s_rect, uint32_t* s_dbits) {
    const int lane = threadIdx.x & 63;
    const int64_t i = i0 + lane;
    uint2 r = make_uint2(0u, 0u);
    uint32_t dbits = 0;
    if (i < n && cnt > 0) {
        r = tile_rect[i];
        dbits = __float_as_uint(splat[2 * i + 1].z);
    }
    s_excl[lane] = incl - cnt;
    s_rect[lane] = r;
    s_dbits[lane] = dbits;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t t = lane; t < total; t += 64) {
        const uint64_t pos = base + t;
        if (pos >= (uint64_t)cap) break;  // positions only grow along the loop
        // owner: the last lane whose exclusive start is <= t (lanes with no
        // instances share their start with the next lane and are skipped)
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1)
            if (lo + step < 64 && s_excl[lo + step] <= t) lo += step;
        const uint32_t local = t - s_excl[lo];
        const uint2 rr = s_rect[lo];
        const uint32_t x0 = rr.x & 0xFFFFu, y0 = rr.x >> 16, x1 = rr.y & 0xFFFFu;
        const uint32_t wd = x1 - x0;
        const uint32_t y = y0 + local / wd, x = x0 + local - (local / wd) * wd;
        const uint64_t tile = (uint64_t)y * (uint32_t)tiles_x + x;
        keys[pos] = (tile << 32) | s_dbits[lo];
        vals[pos] = (uint32_t)(i0 + lo);
    }
}

__device__ __forceinline__ uint32_t wave_incl_scan_counts(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Emission after a full exclusive scan of the counts (offsets).
__global__ void __launch_bounds__(256) emit_keys_kernel(
    int64_t n, const uint2* __restrict__ tile_rect, const uint32_t* __restrict__ touched,
    const float4* __restrict__ splat, const uint64_t* __restrict__ offsets, int64_t cap, int tiles_x,
    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_excl[4][64];
    __shared__ uint2 s_rect[4][64];
    __shared__ uint32_t s_dbits[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x) + 64 * w;  // the wave's first Gaussian
    if (i0 >= n) return;  // uniform per wave
    const int64_t i = i0 + lane;
    const uint64_t base = offsets[i0];  // issued with the count load
    const uint32_t cnt = i < n ? touched[i] : 0u;
    const uint32_t incl = wave_incl_scan_counts(cnt, lane);
    const uint32_t total = __shfl(incl, 63, 64);
    if (total == 0) return;  // uniform
    emit_wave(n, i0, base, cnt, incl, total, tile_rect, splat, cap, tiles_x, keys, vals, s_excl[w], s_rect[w],
              s_dbits[w]);
}

// Emission with the scan's apply pass folded in (no offsets array): given
// the scan-block totals (partials[b], blocks of kScanItems counts),
// workgroup k (256 Gaussians, part k % 8 of scan block k / 8) starts at the
// totals of the scan blocks before its own plus the counts of the earlier
// workgroups of its scan block, and each wavefront adds the counts of the
// workgroup's earlier wavefronts.  The last workgroup writes the total, and
// count / status as the scan does (count 0 and status 1 past cap).
__global__ void __launch_bounds__(256) emit_scan_keys_kernel(
    int64_t n, const uint2* __restrict__ tile_rect, const uint32_t* __restrict__ touched,
    const float4* __restrict__ splat, const uint64_t* __restrict__ partials, int64_t cap, int tiles_x,
    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t* __restrict__ total_out,
    int64_t* __restrict__ count, int32_t* __restrict__ status) {
    constexpr int SUB = kScanItems / 256;  // workgroups per scan block
    __shared__ uint32_t s_excl[4][64];
    __shared__ uint2 s_rect[4][64];
    __shared__ uint32_t s_dbits[4][64];
    __shared__ uint64_t red[4];
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t sb = (int64_t)blockIdx.x / SUB;
    const int sub = (int)(blockIdx.x - sb * SUB);
    const int64_t i0 = (int64_t)blockIdx.x * 256 + 64 * w;
    const int64_t i = i0 + lane;
    // the counts of the scan block's earlier workgroups (in bounds: below
    // blockIdx.x * 256 < n; the others clamped and dropped) and the lane's own
    uint32_t pc[SUB - 1];
#pragma unroll
    for (int c = 0; c < SUB - 1; ++c) {
        const int64_t j = sb * kScanItems + c * 256 + t;
        const uint32_t x = touched[j < n ? j : n - 1];
        pc[c] = c < sub ? x : 0u;
    }
    const uint32_t cnt = i < n ? touched[i] : 0u;
    uint64_t acc = 0;
    for (int64_t j = t; j < sb; j += 256) acc += partials[j];
#pragma unroll
    for (int c = 0; c < SUB - 1; ++c) acc += pc[c];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    const uint32_t incl = wave_incl_scan_counts(cnt, lane);
    if (lane == 0) red[w] = acc;
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    const uint64_t block_base = (red[0] + red[1]) + (red[2] + red[3]);
    uint64_t base = block_base;
#pragma unroll
    for (int k = 0; k < 4; ++k) base += k < w ? (uint64_t)wsum[k] : 0ull;
    if (blockIdx.x == gridDim.x - 1 && t == 0) {
        const uint64_t tot = block_base + (uint64_t)wsum[0] + wsum[1] + wsum[2] + wsum[3];
        *total_out = (int64_t)tot;
        if (cap >= 0) {
            *count = (int64_t)(tot > (uint64_t)cap ? 0 : tot);
            *status = tot > (uint64_t)cap ? 1 : 0;
        }
    }
    if (i0 >= n) return;  // uniform per wave
    const uint32_t total = __shfl(incl, 63, 64);
    if (total == 0) return;  // uniform
    emit_wave(n, i0, base, cnt, incl, total, tile_rect, splat, cap, tiles_x, keys, vals, s_excl[w], s_rect[w],
              s_dbits[w]);
}

struct SortWs {
    uint64_t* offsets;
    uint64_t* partials;
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* hist;
    int64_t* total;
};

static SortWs carve_sort(void* base, int64_t n, int64_t cap, size_t* bytes) {
    Carve c(base);
    SortWs w;
    w.offsets = c.take<uint64_t>(n > 0 ? n : 1);
    w.partials = c.take<uint64_t>(scan_blocks(n) + 1);
    w.keys_alt = c.take<uint64_t>(cap > 0 ? cap : 1);
    w.vals_alt = c.take<uint32_t>(cap > 0 ? cap : 1);
    w.hist = c.take<uint32_t>(radix_hist_words(cap));
    w.total = c.take<int64_t>(1);
    *bytes = c.total();
    return w;
}

static int tile_bits(int64_t tiles) {
    int b = 0;
    while ((int64_t(1) << b) < tiles) ++b;
    return b;
}

// Tile processing order for the compositing kernels: tiles by descending
// list length (in buckets of 16 instances, capped at 255 buckets), ties by
// tile index, so the longest lists are dispatched first and the short ones
// fill the machine behind them.  One workgroup runs a stable counting sort on
// the key 255 - bucket: each of the 16 wavefronts owns a contiguous range of
// tile ids and walks it 64 tiles at a time; lanes with equal keys find each
// other with eight ballots (one per key bit), so a lane's rank among equal
// keys is a popcount and no atomics are needed.  The result is fully
// determined.  Up to kOrderMax tiles; beyond that the order is the identity.
constexpr int kOrderMax = 16384;
constexpr int kOrderWaves = 16;

// For a lane in `valid`: the lanes of `valid` whose key equals its own.
__device__ __forceinline__ uint64_t same_key_lanes(uint32_t key, uint64_t valid) {
    // one key across the valid lanes (runs of empty tiles): no bit ballots
    const uint32_t k0 = __builtin_amdgcn_readlane(key, valid ? __builtin_ctzll(valid) : 0);
    if (__ballot(((valid >> __lane_id()) & 1ull) && key != k0) == 0ull) return valid;
    uint64_t m = valid;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const bool on = (key >> bit) & 1u;
        const uint64_t bl = __ballot(on);
        m &= on ? bl : ~bl;
    }
    return m;
}

__global__ void __launch_bounds__(1024) tile_order_kernel(const uint32_t* __restrict__ ranges, int T,
                                                         uint32_t* __restrict__ order) {
    constexpr int kIters = kOrderMax / (kOrderWaves * 64);  // 64-tile steps per wavefront
    __shared__ uint32_t cnt[kOrderWaves][256];  // per wave and key: count, then next output slot
    __shared__ uint32_t ws[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int i = t; i < kOrderWaves * 256; i += 1024) (&cnt[0][0])[i] = 0;
    const int per = (T + kOrderWaves - 1) / kOrderWaves;
    const int lo = min(T, w * per), hi = min(T, lo + per);
    const uint64_t lt = (1ull << lane) - 1ull;
    // every key of the wavefront's range is loaded up front (in-bounds
    // clamped reads past the range, ignored): a load per 64-tile step would
    // put a full memory latency in front of each step, twice
    uint32_t key[kIters];
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int i = lo + it * 64 + lane;
        const int ic = min(i, T - 1);
        const uint32_t len = ranges[2 * ic + 1] - ranges[2 * ic];
        key[it] = i < hi ? 255u - min(len >> 4, 255u) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        if (lo + it * 64 >= hi) break;  // uniform across the wavefront
        const bool ok = lo + it * 64 + lane < hi;
        const uint64_t m = same_key_lanes(key[it], __ballot(ok));
        if (ok && (m & lt) == 0) cnt[w][key[it]] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    // exclusive prefix over keys of the totals (four wavefront scans), then
    // over waves within a key
    uint32_t s = 0, incl = 0;
    if (t < 256) {
#pragma unroll
        for (int v = 0; v < kOrderWaves; ++v) s += cnt[v][t];
        incl = wave_incl_scan(s, lane);
        if (lane == 63) ws[w] = incl;
    }
    __syncthreads();
    if (t < 256) {
        uint32_t pre = incl - s;  // tiles with a smaller key
#pragma unroll
        for (int k = 0; k < 4; ++k) pre += k < w ? ws[k] : 0u;
#pragma unroll
        for (int v = 0; v < kOrderWaves; ++v) {
            const uint32_t c = cnt[v][t];
            cnt[v][t] = pre;
            pre += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        if (lo + it * 64 >= hi) break;
        const int i = lo + it * 64 + lane;
        const bool ok = i < hi;
        const uint64_t m = same_key_lanes(key[it], __ballot(ok));
        const uint32_t base = ok ? cnt[w][key[it]] : 0u;
        const uint32_t pos = base + (uint32_t)__popcll(m & lt);
        if (ok && pos < (uint32_t)T) order[pos] = (uint32_t)i;
        // every lane has read its base before the group leader advances it
        if (ok && (m & lt) == 0) cnt[w][key[it]] = base + (uint32_t)__popcll(m);
    }
}

__global__ void __launch_bounds__(256) tile_order_identity_kernel(int64_t T, uint32_t* __restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < T) order[i] = (uint32_t)i;
}

}  // namespace xgs

using namespace xgs;

extern "C" size_t xgs_tile_sort_workspace(int64_t n, int64_t max_instances, int32_t num_tiles) {
    (void)num_tiles;
    size_t bytes = 0;
    carve_sort(nullptr, n < 0 ? 0 : n, max_instances < 0 ? 0 : max_instances, &bytes);
    return bytes;
}

extern "C" xgs_status xgs_tile_sort(const xgs_projected* p, const xgs_camera* cam, int64_t n,
                                    void* ws, size_t ws_bytes, xgs_binning* b, xgs_stream_t stream) {
    clear_error();
    if (!p || !cam || !b) return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort: null argument");
    if (xgs_status s = validate_camera(cam)) return s;
    if (n < 0 || b->max_instances < 0)
        return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort: negative size");
    if (b->max_instances >= (int64_t(1) << 32))
        return fail(XGS_ERR_UNSUPPORTED, "xgs_tile_sort: max_instances must be below 2^32");
    if (!b->keys || !b->vals || !b->ranges || !b->num_instances || !b->status)
        return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort: null binning array");
    if (n > 0 && (!p->splat || !p->tile_rect || !p->tiles_touched))
        return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort: null projected array");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort: workspace must be 256-byte aligned");
    size_t need = 0;
    SortWs w = carve_sort(ws, n, b->max_instances, &need);
    if (ws_bytes < need || !ws)
        return fail(XGS_ERR_CAPACITY, "xgs_tile_sort: workspace too small (need " + std::to_string(need) + " bytes)");
    hipStream_t st = (hipStream_t)stream;
    Grid g = grid_of(*cam);
    int64_t tiles = (int64_t)g.tx * g.ty;
    const int64_t cap = b->max_instances;
    int bits = 32 + tile_bits(tiles);
    bool even = radix_passes(bits, cap) % 2 == 0;
    uint64_t* k0 = even ? b->keys : w.keys_alt;
    uint32_t* v0 = even ? b->vals : w.vals_alt;
    uint64_t* k1 = even ? w.keys_alt : b->keys;
    uint32_t* v1 = even ? w.vals_alt : b->vals;
    xgs_status s = XGS_OK;
    if (n > 0 && scan_blocks(n) <= kFusedScanBlocks) {
        // block totals (clearing the per-tile ranges: empty tiles keep (0, 0)),
        // then the emission applies the prefix itself
        if ((s = scan_block_totals(p->tiles_touched, n, w.partials, b->ranges, 2 * tiles, st))) return s;
        hipLaunchKernelGGL(emit_scan_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                           reinterpret_cast<const uint2*>(p->tile_rect), p->tiles_touched,
                           reinterpret_cast<const float4*>(p->splat), w.partials, cap, g.tx, k0, v0, w.total,
                           b->num_instances, b->status);
        if ((s = check_launch("xgs_tile_sort emit"))) return s;
    } else {
        // the scan also clears the per-tile ranges (empty tiles keep (0, 0))
        if ((s = exclusive_scan_u32(p->tiles_touched, n, w.offsets, w.partials, w.total, cap, b->num_instances,
                                    b->status, b->ranges, 2 * tiles, st)))
            return s;
        if (n > 0) {
            hipLaunchKernelGGL(emit_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                               reinterpret_cast<const uint2*>(p->tile_rect), p->tiles_touched,
                               reinterpret_cast<const float4*>(p->splat), w.offsets, cap, g.tx, k0, v0);
            if ((s = check_launch("xgs_tile_sort emit"))) return s;
        }
    }
    if ((s = radix_sort(k0, v0, k1, v1, b->num_instances, cap, bits, w.hist, st))) return s;
    if ((s = segment_ranges(b->keys, b->num_instances, cap, 32, b->ranges, st))) return s;
    if (b->tile_order && tiles > 0) {
        if (tiles <= kOrderMax)
            hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, st, b->ranges, (int)tiles, b->tile_order);
        else
            hipLaunchKernelGGL(tile_order_identity_kernel, dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, st,
                               tiles, b->tile_order);
    }
    return check_launch("xgs_tile_sort order");
}

extern "C" size_t xgs_tile_sort_noalloc_max_bytes(void) { return kSortScratchBytes; }

extern "C" xgs_status xgs_tile_sort_noalloc(const xgs_projected* p, const xgs_camera* cam, int64_t n,
                                            xgs_binning* b, xgs_stream_t stream) {
    clear_error();
    if (!p || !cam || !b) return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort_noalloc: null argument");
    if (xgs_status s = validate_camera(cam)) return s;
    if (n < 0 || b->max_instances < 0)
        return fail(XGS_ERR_INVALID_ARG, "xgs_tile_sort_noalloc: negative size");
    const Grid g = grid_of(*cam);
    const size_t need = xgs_tile_sort_workspace(n, b->max_instances, g.tx * g.ty);
    if (need > kSortScratchBytes)
        return fail(XGS_ERR_CAPACITY, "xgs_tile_sort_noalloc: n = " + std::to_string(n) + " and max_instances = " +
                                          std::to_string(b->max_instances) + " need " + std::to_string(need) +
                                          " bytes of scratch, above the fixed " + std::to_string(kSortScratchBytes) +
                                          " (use xgs_tile_sort with a workspace)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(XGS_ERR_HIP, std::string("xgs_tile_sort_noalloc: hipGetDevice: ") +
                                                      hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(XGS_ERR_UNSUPPORTED, "xgs_tile_sort_noalloc: device index above 63");
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // with the device current: each GPU holds its own copy of the array
            e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                g_scratch_ptr[dev] = nullptr;
                return fail(XGS_ERR_HIP, std::string("xgs_tile_sort_noalloc: hipGetSymbolAddress: ") +
                                             hipGetErrorString(e));
            }
        }
        ws = g_scratch_ptr[dev];
    }
    // every kernel of the sort writes the scratch words it later reads, so
    // nothing has to be cleared between calls
    return xgs_tile_sort(p, cam, n, ws, kSortScratchBytes, b, stream);
}
