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
struct TileGrid {
    int hs, ws, tx, ty, tiles;
    int s, oy, ox;
};

inline TileGrid tile_grid(const xgs_camera& cam) {
    Grid g = grid_of(cam);
    TileGrid t;
    t.hs = g.hs; t.ws = g.ws; t.tx = g.tx; t.ty = g.ty; t.tiles = g.tx * g.ty;
    t.s = cam.stride; t.oy = cam.off_y; t.ox = cam.off_x;
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
    r.tile = (k >> 2) * 8 + xcd;
    const int lane = threadIdx.x;
    const int tx = r.tile % g.tx, ty = r.tile / g.tx;
    r.n = tx * kTile + (q & 1) * 8 + (lane & 7);
    r.m = ty * kTile + (q >> 1) * 8 + (lane >> 3);
    r.inside = r.tile < g.tiles && r.n < g.ws && r.m < g.hs;
    r.px = (float)g.ox + (float)r.n * (float)g.s + 0.5f;
    r.py = (float)g.oy + (float)r.m * (float)g.s + 0.5f;
    return r;
}

// Wave-uniform value: the compiler keeps it in a scalar register, so loads
// indexed by it become scalar (constant-cache) loads.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

}  // namespace xgs
