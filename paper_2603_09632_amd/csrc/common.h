// Internal helpers shared by the HIP translation units of libxgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>

#include "xgs.h"

namespace xgs {

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Thresholds of the compositing rule (alpha clamp, skip, stop) and the
// dilation added to Sigma'.
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;
constexpr float kDilation = 0.3f;
constexpr float kGuard = 1.3f;
constexpr int kTile = XGS_TILE;

// Thread-local last-error text, returned by xgs_last_error().
void set_error(const std::string& msg);
void clear_error();

inline xgs_status fail(xgs_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

inline xgs_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return XGS_ERR_HIP;
    }
    return XGS_OK;
}

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

struct Grid {
    int hs, ws, ty, tx;
};

inline Grid grid_of(const xgs_camera& c) {
    Grid g;
    g.hs = (c.height + c.stride - 1) / c.stride;
    g.ws = (c.width + c.stride - 1) / c.stride;
    g.ty = (g.hs + kTile - 1) / kTile;
    g.tx = (g.ws + kTile - 1) / kTile;
    return g;
}

xgs_status validate_camera(const xgs_camera* c);

// Carves aligned sub-buffers out of a caller-provided workspace.
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(void* p) : base(static_cast<char*>(p)) {}
    template <class T>
    T* take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
    size_t total() const { return (used + 255) & ~size_t(255); }
};

// Per-pair opacity of a splat at a pixel: alpha = min(0.99, o exp(-q/2)),
// q = A dx^2 + 2B dx dy + C dy^2.  The forward and backward kernels both call
// this one function so that they take the same skip decisions.
struct PairEval {
    float G, alpha, dx, dy;
};

__device__ __forceinline__ PairEval eval_pair(float px, float py, float mx, float my, float A,
                                              float B, float C, float o) {
    PairEval r;
    r.dx = px - mx;
    r.dy = py - my;
    float q = A * r.dx * r.dx + 2.0f * B * r.dx * r.dy + C * r.dy * r.dy;
    r.G = __expf(-0.5f * q);
    r.alpha = fminf(kAlphaMax, o * r.G);
    return r;
}

}  // namespace xgs
