// Shared launch geometry of the forward and backward compositing kernels.
#pragma once
#include "common.h"

namespace xgs {

// One wavefront (one 64-thread workgroup) renders an 8x8 quadrant of a 16x16
// tile.  Every wave walks its tile's list on its own, so waves never wait for
// each other and retire as soon as their 64 pixels are done.  Consecutive
// workgroups go round-robin to the 8 XCDs; the mapping below puts the four
// quadrants of a tile on the same XCD so that the tile's list and splat
// records are fetched into one L2.
// order: the tile processing order (slot -> tile id), nullptr for id order.
struct TileGrid {
    int hs, ws, tx, ty, tiles;
    int s, oy, ox;
    const uint32_t* order;
};

inline TileGrid tile_grid(const xgs_camera& cam, const uint32_t* order = nullptr) {
    Grid g = grid_of(cam);
    TileGrid t;
    t.hs = g.hs; t.ws = g.ws; t.tx = g.tx; t.ty = g.ty; t.tiles = g.tx * g.ty;
    t.s = cam.stride; t.oy = cam.off_y; t.ox = cam.off_x;
    t.order = order;
    return t;
}

inline unsigned quad_blocks(const TileGrid& t) {
    return (unsigned)(((t.tiles + 7) / 8) * 32);
}

struct QuadPix {
    int tile, m, n;
    bool inside;
    float px, py;
};

// Slots go round-robin over the eight XCDs (the four quadrants of a slot
// share one XCD and its L2); the order table maps slot -> tile.
__device__ __forceinline__ int quad_slot() {
    const int b = blockIdx.x;
    return ((b >> 3) >> 2) * 8 + (b & 7);
}
__device__ __forceinline__ int quad_index() { return (blockIdx.x >> 3) & 3; }

// Pixel of this lane in quadrant q of tile `tile` of grid g.
__device__ __forceinline__ QuadPix quad_pixel_at(const TileGrid& g, int tile, int q) {
    QuadPix r;
    r.tile = tile;
    const int lane = threadIdx.x;
    const int tx = r.tile % g.tx, ty = r.tile / g.tx;
    r.n = tx * kTile + (q & 1) * 8 + (lane & 7);
    r.m = ty * kTile + (q >> 1) * 8 + (lane >> 3);
    r.inside = r.tile < g.tiles && r.n < g.ws && r.m < g.hs;
    r.px = (float)g.ox + (float)r.n * (float)g.s + 0.5f;
    r.py = (float)g.oy + (float)r.m * (float)g.s + 0.5f;
    return r;
}

__device__ __forceinline__ QuadPix quad_pixel(const TileGrid& g) {
    const int b = blockIdx.x;
    const int xcd = b & 7, k = b >> 3;
    const int q = k & 3;
    QuadPix r;
    const int slot = (k >> 2) * 8 + xcd;
    r.tile = (g.order && slot < g.tiles) ? (int)__builtin_amdgcn_readfirstlane((int)g.order[slot]) : slot;
    const int lane = threadIdx.x;
    const int tx = r.tile % g.tx, ty = r.tile / g.tx;
    r.n = tx * kTile + (q & 1) * 8 + (lane & 7);
    r.m = ty * kTile + (q >> 1) * 8 + (lane >> 3);
    r.inside = r.tile < g.tiles && r.n < g.ws && r.m < g.hs;
    r.px = (float)g.ox + (float)r.n * (float)g.s + 0.5f;
    r.py = (float)g.oy + (float)r.m * (float)g.s + 0.5f;
    return r;
}

// Pixel-centre rectangle of a wavefront's 8x8 quadrant (clipped to nothing:
// pixels past the image edge only make the rectangle larger).
struct QuadRect {
    float x0, y0, x1, y1;
};

__device__ __forceinline__ QuadRect quad_rect(const TileGrid& g, const QuadPix& P) {
    const int lane = threadIdx.x;
    QuadRect r;
    r.x0 = P.px - (float)((lane & 7) * g.s);
    r.y0 = P.py - (float)((lane >> 3) * g.s);
    r.x1 = r.x0 + (float)(7 * g.s);
    r.y1 = r.y0 + (float)(7 * g.s);
    return r;
}

// Whether a splat can reach alpha >= 1/255 at any pixel centre of the
// quadrant.  alpha = min(0.99, o exp(-q/2)) >= 1/255 holds exactly where
// q <= t = 2 ln(255 o); q is convex, so its minimum over the rectangle is 0
// when the mean lies inside and otherwise lies on an edge, where it is the
// edge's 1D quadratic at its clamped vertex.  The test errs on the side of
// keeping: the margin (0.05 + 0.2% of t) is several times the rounding of
// the per-pixel q (|grad q| <= 2 sqrt(3.4 t) for conics of a Sigma' with the
// 0.3 dilation, times the ~1e-4 px rounding of dx, dy), so a splat it drops
// is skipped by every pixel of the quadrant in both passes.
__device__ __forceinline__ bool quad_hit(const float4 s0, const float4 s1, const QuadRect& r) {
    const float mx = s0.x, my = s0.y, A = s0.z, B = s0.w, C = s1.x, o = s1.y;
    const float ex0 = r.x0 - mx, ex1 = r.x1 - mx, ey0 = r.y0 - my, ey1 = r.y1 - my;
    if (ex0 <= 0.f && ex1 >= 0.f && ey0 <= 0.f && ey1 >= 0.f) return true;
    const float t = 2.f * __logf(255.f * o);
    const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
    auto q = [&](float dx, float dy) { return A * dx * dx + 2.f * B * dx * dy + C * dy * dy; };
    const float y0 = fminf(fmaxf(-B * ex0 * iC, ey0), ey1);
    const float y1 = fminf(fmaxf(-B * ex1 * iC, ey0), ey1);
    const float x0 = fminf(fmaxf(-B * ey0 * iA, ex0), ex1);
    const float x1 = fminf(fmaxf(-B * ey1 * iA, ex0), ex1);
    const float best = fminf(fminf(q(ex0, y0), q(ex1, y1)), fminf(q(x0, ey0), q(x1, ey1)));
    return best <= t * 1.002f + 0.05f;
}

// Ring of splats that survive the quadrant test, in walk order: the tile
// list is read 64 candidates at a time (one per lane), the survivors are
// appended with ballot ranks, and the walk takes them 16 at a time, so each
// batch of the walk and of its matrix-core channel product holds 16 splats
// that can touch the wavefront's pixels.
constexpr int kRing = 128;

struct Ring {
    float4 rec[kRing][2];
    int gid[kRing];
    int pos[kRing];  // list position (offset from the tile's start)
};

// Appends this lane's candidate when keep is set; returns the new tail.
__device__ __forceinline__ int ring_push(Ring& q, int tail, bool keep, float4 s0, float4 s1, int gid, int pos) {
    const uint64_t m = __ballot(keep);
    if (keep) {
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        const int at = (tail + below) & (kRing - 1);
        q.rec[at][0] = s0;
        q.rec[at][1] = s1;
        q.gid[at] = gid;
        q.pos[at] = pos;
    }
    return tail + __popcll(m);
}

// 16x16x4 FP32 matrix core op: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; the accumulator holds D[4 (l / 16) + r][l % 16], r = 0..3.
__device__ __forceinline__ f32x4_t mfma16x16x4(float a, float b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Wave-uniform value: the compiler keeps it in a scalar register, so loads
// indexed by it become scalar (constant-cache) loads.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Batched requests: the slot of a global tile and the slot's own tile grid.
// Slot s owns rows [row_base, row_base + tiles_y) of a virtual grid gtx tiles
// wide; tiles at columns >= the slot's tiles_x are empty.  Returns false when
// the tile belongs to no slot (or lies past its columns).
struct BatchTile {
    int slot, tile;  // slot index, tile index within the slot's grid
    TileGrid grid;   // the slot's grid (no order table)
};

__device__ __forceinline__ bool batch_tile(const xgs_batch_slot* __restrict__ slots, int n_slots, int gtx,
                                           int gtile, BatchTile& bt) {
    const int grow = gtile / gtx, gcol = gtile - (gtile / gtx) * gtx;
    for (int j = 0; j < n_slots; ++j) {
        const xgs_camera& c = slots[j].cam;
        const int rb = (int)uniform((uint32_t)slots[j].row_base);
        const int st = (int)uniform((uint32_t)c.stride);
        const int hs = ((int)uniform((uint32_t)c.height) + st - 1) / st;
        const int ws = ((int)uniform((uint32_t)c.width) + st - 1) / st;
        const int ty = (hs + kTile - 1) / kTile, tx = (ws + kTile - 1) / kTile;
        if (grow >= rb && grow < rb + ty) {
            if (gcol >= tx) return false;
            bt.slot = j;
            bt.tile = (grow - rb) * tx + gcol;
            bt.grid.hs = hs; bt.grid.ws = ws; bt.grid.tx = tx; bt.grid.ty = ty; bt.grid.tiles = tx * ty;
            bt.grid.s = st;
            bt.grid.oy = (int)uniform((uint32_t)c.off_y);
            bt.grid.ox = (int)uniform((uint32_t)c.off_x);
            bt.grid.order = nullptr;
            return true;
        }
    }
    return false;
}

}  // namespace xgs
