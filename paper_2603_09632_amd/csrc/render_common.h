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

__device__ __forceinline__ QuadPix quad_pixel(const TileGrid& g) {
    const int b = blockIdx.x;
    const int xcd = b & 7, k = b >> 3;
    const int q = k & 3;
    QuadPix r;
    // Slots go round-robin over the eight XCDs (the four quadrants of a slot
    // share one XCD and its L2); the order table maps slot -> tile.
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

// 16x16x4 FP32 matrix core op: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; the accumulator holds D[4 (l / 16) + r][l % 16], r = 0..3.
__device__ __forceinline__ f32x4_t mfma16x16x4(float a, float b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Channel c of Gaussian i: 0..2 colour, 3 camera depth (from the splat
// record), 4.. semantic features.
template <int CS, bool EXACT>
__device__ __forceinline__ float channel_of(const float* __restrict__ colors, const float4* __restrict__ splat,
                                            const float* __restrict__ features, int csem, uint32_t i, int c) {
    if (c < 3) return colors[3 * (size_t)i + c];
    if (c == 3) return splat[2 * (size_t)i + 1].z;
    return features[(size_t)i * (EXACT ? CS : csem) + (c - 4)];
}

// Wave-uniform value: the compiler keeps it in a scalar register, so loads
// indexed by it become scalar (constant-cache) loads.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

}  // namespace xgs
