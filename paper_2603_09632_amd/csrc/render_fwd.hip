// a3: front-to-back alpha compositing of RGB, depth and semantic channels,
// Eq. (rendering) with the feature and depth substitutions (Sec. 3.1, App. B),
// evaluated only at the sampled grid pixels (App. D): the rasterizer never
// forms the dense map when stride > 1.
#include "render_common.h"

namespace xgs {

// CS: compile-time semantic channel count.  EXACT: csem == CS, so feature
// rows have a compile-time stride and merge into wide scalar loads; otherwise
// CS only bounds csem and channels >= csem are neither read nor written.
//
// A wavefront takes an 8x8 quadrant of a tile.  It reads the tile list 64
// entries at a time (one per lane: list entry and splat record), keeps the
// splats that can reach alpha >= 1/255 somewhere in its quadrant (quad_hit;
// the others would be skipped by all 64 pixels) and appends them to a ring in
// LDS; the walk then takes the ring 16 splats at a time.  The next 64 entries
// are in flight while the ring is walked.  For each splat every pixel
// evaluates alpha and updates T, giving the blend weight w_k(p) = alpha_k T_k
// (0 for skipped, terminated or absent pairs).  The weights go through LDS
// (row stride 17: conflict-free both ways) and the channel sums
// out[p][c] += sum_k w_k(p) chan_k[c] run as a 64 x 16 x 48 product on
// v_mfma_f32_16x16x4_f32, with the channel rows read as vectors (issued
// before the walk, consumed after it).  The accumulators hold the wave's
// 64 x (4 + CS) output block until the end.
//
// The walk is latency-bound (one dependent transmittance chain per pixel), so
// occupancy pays: at least 3 wavefronts per SIMD (the accumulators stay in
// VGPRs; no spills up to CS = 64) measured 16% faster than the 2 the default
// register allocation gives (at CS = 32 the kernel fits 4).  For the same
// reason the per-splat step has no branches and reads its ring record two
// splats ahead, so those LDS reads overlap the previous splats' chains.
//
// BATCH: the tiles of several requests in one launch (serving).  g then
// describes the virtual grid (tx = its width in tiles, tiles = all of it,
// order over it); each workgroup finds its request's slot, takes that slot's
// grid, colours, features and outputs, and reads the tile list of the global
// tile.  Splat records are indexed by global Gaussian index, colours and
// features by index within the slot's scene.
template <int CS, bool EXACT, bool BATCH = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CS > 32 ? 3 : 4))) render_fwd_mfma_kernel(
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float4* __restrict__ splat, const float* __restrict__ colors,
    const float* __restrict__ features, int csem, TileGrid g, float* __restrict__ out,
    float* __restrict__ final_T, int32_t* __restrict__ n_last, const xgs_batch_slot* __restrict__ slots = nullptr,
    int n_slots = 0) {
    constexpr int CH = 4 + CS;
    constexpr int NT = (CH + 15) / 16;
    __shared__ float wl[64 * 17];
    __shared__ Ring ring;
    QuadPix P;
    int rtile;  // tile whose list is read (the global tile when batched)
    if constexpr (BATCH) {
        const int slot = quad_slot();
        if (slot >= g.tiles) return;
        rtile = g.order ? (int)uniform(g.order[slot]) : slot;
        BatchTile bt;
        if (!batch_tile(slots, n_slots, g.tx, rtile, bt)) return;
        const xgs_batch_slot& sl = slots[bt.slot];
        // colours and features are indexed by global Gaussian index: shift
        // their bases by the slot's first global index
        const int64_t base = (int64_t)sl.gauss_base;
        colors = reinterpret_cast<const float*>(reinterpret_cast<uintptr_t>(sl.g.colors) -
                                                (uintptr_t)(base * 3 * (int64_t)sizeof(float)));
        features = reinterpret_cast<const float*>(reinterpret_cast<uintptr_t>(sl.g.features) -
                                                  (uintptr_t)(base * (EXACT ? CS : csem) * (int64_t)sizeof(float)));
        out = sl.out;
        final_T = sl.final_T;
        n_last = sl.n_last;
        g = bt.grid;
        P = quad_pixel_at(g, bt.tile, quad_index());
    } else {
        P = quad_pixel(g);
        rtile = P.tile;
    }
    if (P.tile >= g.tiles) return;
    const QuadRect qr = quad_rect(g, P);
    const int lane = threadIdx.x;
    // The first 16 channels of a splat (colour, depth, features 0-11) as one
    // lane-constant source and stride: channel lane % 16 of Gaussian i is
    // src0[i * str0], so that the batch's loads of those channels do not
    // branch on the channel.
    const int fstr = EXACT ? CS : csem;
    const int j0 = lane & 15;
    const float* const src0 = j0 < 3 ? colors + j0
                                     : j0 == 3 ? reinterpret_cast<const float*>(splat) + 6 : features + (j0 - 4);
    const int str0 = j0 < 3 ? 3 : j0 == 3 ? 8 : fstr;
    f32x4_t acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    float T = 1.f;
    int last = 0;
    bool done = !P.inside;
    const uint32_t start = uniform(ranges[2 * rtile]);
    const int len = (int)(uniform(ranges[2 * rtile + 1]) - start);
    // candidate registers: list entry and splat record of position cpos + lane
    int cg = -1;
    float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
    auto fetch = [&](int pos) {
        cg = -1;
        if (pos + lane < len) {
            cg = (int)vals[start + (uint32_t)(pos + lane)];
            c0 = splat[2 * (uint32_t)cg];
            c1 = splat[2 * (uint32_t)cg + 1];
        }
    };
    int cpos = 0, head = 0, tail = 0;
    fetch(0);
    for (;;) {
        if (__ballot(!done) == 0ull) break;
        // fill the ring to one batch (or the end of the list)
        while (tail - head < 16 && cpos < len) {
            tail = ring_push(ring, tail, cg >= 0 && quad_hit(c0, c1, qr), c0, c1, cg, cpos + lane);
            cpos += 64;
            fetch(cpos);
        }
        const int nb = min(16, tail - head);
        if (nb == 0) break;
        __syncthreads();
        // channel rows of this batch in B-operand layout (consumed after the walk)
        float b[4][NT];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int slot = 4 * kk + (lane >> 4);
            const int gs = slot < nb ? ring.gid[(head + slot) & (kRing - 1)] : -1;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = 16 * nt + (lane & 15);
                const bool use = gs >= 0 && c < CH && (EXACT || c < 4 + csem);
                if (nt == 0)
                    b[kk][nt] = use ? src0[(size_t)(uint32_t)gs * str0] : 0.f;
                else
                    b[kk][nt] = use ? features[(size_t)(uint32_t)gs * fstr + (c - 4)] : 0.f;
            }
        }
        // Branch-free per splat (selects only), so that the next splats' ring
        // reads can be issued while this one's chain runs; the list position of
        // the pixel's last contributing splat is read once per batch.
        uint32_t nz = 0;  // bit k: this pixel's weight for splat k is nonzero
        int lastk = -1;   // batch index of this pixel's last contributing splat
        // records of splats k + 1 and k + 2 are read while splat k is evaluated;
        // slots k >= nb hold stale records: read (in bounds) and masked
        float4 ra0 = ring.rec[head & (kRing - 1)][0], ra1 = ring.rec[head & (kRing - 1)][1];
        float4 rb0 = ring.rec[(head + 1) & (kRing - 1)][0], rb1 = ring.rec[(head + 1) & (kRing - 1)][1];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float4 s0 = ra0, s1 = ra1;
            ra0 = rb0; ra1 = rb1;
            if (k + 2 < 16) {
                const int an = (head + k + 2) & (kRing - 1);
                rb0 = ring.rec[an][0];
                rb1 = ring.rec[an][1];
            }
            const PairEval e = eval_pair(P.px, P.py, s0.x, s0.y, s0.z, s0.w, s1.x, s1.y);
            const bool ok = k < nb && !done && e.alpha >= kAlphaMin;
            const float Tn = T * (1.f - e.alpha);
            const bool stop = ok && Tn < kTStop;
            const bool contrib = ok && !stop;
            done = done || stop;
            const float w = contrib ? e.alpha * T : 0.f;
            T = contrib ? Tn : T;
            lastk = contrib ? k : lastk;
            nz |= contrib ? (1u << k) : 0u;
            wl[lane * 17 + k] = w;
        }
        if (lastk >= 0) last = ring.pos[(head + lastk) & (kRing - 1)] + 1;
        head += nb;
        __syncthreads();
        // a 16-pixel x 4-splat block of weights that is all zero adds nothing
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const uint64_t live = __ballot(((nz >> (4 * kk)) & 0xFu) != 0u);
            const int slot = 4 * kk + (lane >> 4);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                if (((live >> (16 * mt)) & 0xFFFFull) == 0ull) continue;
                const float a = wl[(16 * mt + (lane & 15)) * 17 + slot];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma16x16x4(a, b[kk][nt], acc[mt][nt]);
            }
        }
        __syncthreads();
    }
    const size_t hw = (size_t)g.hs * g.ws;
    if (P.inside) {
        const size_t pix = (size_t)P.m * g.ws + P.n;
        final_T[pix] = T;
        n_last[pix] = (int32_t)last;
    }
    // accumulator (mt, nt) holds pixel 16 mt + 4 (lane / 16) + r, channel 16 nt + lane % 16
    const int qx = P.n - (lane & 7), qy = P.m - (lane >> 3);  // quadrant origin
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * mt + 4 * (lane >> 4) + r;
            const int m = qy + (p >> 3), n = qx + (p & 7);
            if (m >= g.hs || n >= g.ws) continue;
            const size_t pix = (size_t)m * g.ws + n;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = 16 * nt + (lane & 15);
                if (c < CH && (EXACT || c < 4 + csem)) out[c * hw + pix] = acc[mt][nt][r];
            }
        }
}

template <int CS, bool EXACT = true>
static void launch_fwd(const xgs_gaussians* g, const xgs_projected* p, const xgs_binning* b,
                       const TileGrid& tg, float* out, float* final_T, int32_t* n_last,
                       hipStream_t st) {
    hipLaunchKernelGGL((render_fwd_mfma_kernel<CS, EXACT>), dim3(quad_blocks(tg)), dim3(64), 0, st, b->ranges,
                           b->vals, reinterpret_cast<const float4*>(p->splat), g->colors, g->features,
                           g->c_sem, tg, out, final_T, n_last);
}

template <int CS>
static void launch_fwd_batch(const xgs_batch_slot* slots, int n_slots, const xgs_projected* p,
                             const xgs_binning* b, const TileGrid& tg, hipStream_t st) {
    hipLaunchKernelGGL((render_fwd_mfma_kernel<CS, true, true>), dim3(quad_blocks(tg)), dim3(64), 0, st, b->ranges,
                       b->vals, reinterpret_cast<const float4*>(p->splat), nullptr, nullptr, CS, tg, nullptr,
                       nullptr, nullptr, slots, n_slots);
}

}  // namespace xgs

using namespace xgs;

extern "C" xgs_status xgs_batch_render_fwd(const xgs_batch_slot* d_slots, int32_t n_slots, int32_t c_sem,
                                           int32_t tiles_x, int32_t tile_rows, const xgs_projected* p,
                                           const xgs_binning* b, xgs_stream_t stream) {
    clear_error();
    if (!p || !b) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_render_fwd: null argument");
    if (n_slots < 0 || n_slots > XGS_BATCH_MAX_SLOTS)
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_render_fwd: n_slots must be in [0, 16]");
    if (n_slots > 0 && !d_slots) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_render_fwd: null slot table");
    if (tiles_x < 1 || tile_rows < 1 || tiles_x > 65535 || tile_rows > 65535 ||
        (int64_t)tiles_x * tile_rows >= (int64_t(1) << 31))
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_render_fwd: bad tile grid");
    if (!p->splat || !b->ranges || !b->vals) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_render_fwd: null array");
    if (!aligned(p->splat, 16)) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_render_fwd: splat must be 16-byte aligned");
    if (n_slots == 0) return XGS_OK;
    TileGrid tg;
    tg.tx = tiles_x; tg.ty = tile_rows; tg.tiles = tiles_x * tile_rows;
    tg.hs = 16 * tile_rows; tg.ws = 16 * tiles_x; tg.s = 1; tg.oy = 0; tg.ox = 0;
    tg.order = b->tile_order;
    hipStream_t st = (hipStream_t)stream;
    switch (c_sem) {
#define XGS_BFWD_CASE(n) case n: launch_fwd_batch<n>(d_slots, n_slots, p, b, tg, st); break;
        XGS_BFWD_CASE(0) XGS_BFWD_CASE(1) XGS_BFWD_CASE(2) XGS_BFWD_CASE(3) XGS_BFWD_CASE(4)
        XGS_BFWD_CASE(8) XGS_BFWD_CASE(16) XGS_BFWD_CASE(32)
#undef XGS_BFWD_CASE
        default:
            return fail(XGS_ERR_UNSUPPORTED, "xgs_batch_render_fwd: c_sem must be one of 0-4, 8, 16, 32");
    }
    return check_launch("xgs_batch_render_fwd");
}

extern "C" xgs_status xgs_render_fwd(const xgs_gaussians* g, const xgs_projected* p,
                                     const xgs_binning* b, const xgs_camera* cam, float* out,
                                     float* final_T, int32_t* n_last, xgs_stream_t stream) {
    clear_error();
    if (!g || !p || !b || !cam) return fail(XGS_ERR_INVALID_ARG, "xgs_render_fwd: null argument");
    if (xgs_status s = validate_camera(cam)) return s;
    if (!out || !final_T || !n_last) return fail(XGS_ERR_INVALID_ARG, "xgs_render_fwd: null output");
    if (g->c_sem < 0 || g->c_sem > XGS_MAX_C_SEM)
        return fail(XGS_ERR_UNSUPPORTED, "xgs_render_fwd: c_sem must be in [0, 64]");
    if (g->n > 0 && (!g->colors || (g->c_sem > 0 && !g->features) || !p->splat))
        return fail(XGS_ERR_INVALID_ARG, "xgs_render_fwd: null Gaussian array");
    if (!b->ranges || !b->vals) return fail(XGS_ERR_INVALID_ARG, "xgs_render_fwd: null binning array");
    if (!aligned(p->splat, 16)) return fail(XGS_ERR_INVALID_ARG, "xgs_render_fwd: splat must be 16-byte aligned");
    TileGrid tg = tile_grid(*cam, b->tile_order);
    hipStream_t st = (hipStream_t)stream;
    switch (g->c_sem) {
#define XGS_FWD_CASE(n) case n: launch_fwd<n>(g, p, b, tg, out, final_T, n_last, st); break;
        XGS_FWD_CASE(0) XGS_FWD_CASE(1) XGS_FWD_CASE(2) XGS_FWD_CASE(3) XGS_FWD_CASE(4)
        XGS_FWD_CASE(8) XGS_FWD_CASE(12) XGS_FWD_CASE(16) XGS_FWD_CASE(24) XGS_FWD_CASE(32)
        XGS_FWD_CASE(48) XGS_FWD_CASE(64)
#undef XGS_FWD_CASE
        default:
            if (g->c_sem <= 16) launch_fwd<16, false>(g, p, b, tg, out, final_T, n_last, st);
            else if (g->c_sem <= 32) launch_fwd<32, false>(g, p, b, tg, out, final_T, n_last, st);
            else launch_fwd<64, false>(g, p, b, tg, out, final_T, n_last, st);
    }
    return check_launch("xgs_render_fwd");
}
