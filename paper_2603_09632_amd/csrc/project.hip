// a1: EWA projection of 3D Gaussians to screen-space splats (App. A), plus
// the opacity-aware tile rectangle.  One thread per Gaussian; every input row
// is read once with full cache lines (row-major [n][k] rows are contiguous
// across a wavefront) and each output record is written once.
#include "common.h"

namespace xgs {

struct CamDev {
    float fx, fy, cx, cy, near_, limx, limy;
    float R[9], t[3];
    int s, oy, ox, hs, ws;
};

// Projection of Gaussian i (input row) into output row o.  row_off shifts the
// tile rectangle's rows (the batched form places each request in its own band
// of a shared tile grid; 0 otherwise).  Products and sums are rounded one by
// one (no contraction into fused multiply-adds): whether the compiler fuses a
// product depends on where its operands live (kernel arguments or loads),
// and the single-request and batched kernels must give the same bits.
__device__ __forceinline__ void project_one(
    int64_t i, int64_t o_, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ opacity, const CamDev& c, uint32_t row_off,
    float4* __restrict__ splat, int32_t* __restrict__ radius, uint2* __restrict__ tile_rect,
    uint32_t* __restrict__ touched) {
#pragma clang fp contract(off)
    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    const float o = opacity[i];
    float px = c.R[0] * mx + c.R[1] * my + c.R[2] * mz + c.t[0];
    float py = c.R[3] * mx + c.R[4] * my + c.R[5] * mz + c.t[1];
    float pz = c.R[6] * mx + c.R[7] * my + c.R[8] * mz + c.t[2];

    float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = make_float4(0.f, o, pz, 0.f);
    uint2 rect = make_uint2(0u, 0u);
    int32_t rad = 0;
    uint32_t tt = 0;
    bool ok = pz > c.near_ && o >= kAlphaMin;
    if (ok) {
        // Sigma = M M^T with M = R(q) diag(exp l)
        float4 q = quats[i];
        float inv = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
        float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
        float R00 = 1.f - 2.f * (y * y + z * z), R01 = 2.f * (x * y - w * z), R02 = 2.f * (x * z + w * y);
        float R10 = 2.f * (x * y + w * z), R11 = 1.f - 2.f * (x * x + z * z), R12 = 2.f * (y * z - w * x);
        float R20 = 2.f * (x * z - w * y), R21 = 2.f * (y * z + w * x), R22 = 1.f - 2.f * (x * x + y * y);
        float sx = __expf(log_scales[3 * i]), sy = __expf(log_scales[3 * i + 1]),
              sz = __expf(log_scales[3 * i + 2]);
        // rows of T = Rv M  (camera-frame factor, Sigma_cam = T T^T)
        float M00 = R00 * sx, M01 = R01 * sy, M02 = R02 * sz;
        float M10 = R10 * sx, M11 = R11 * sy, M12 = R12 * sz;
        float M20 = R20 * sx, M21 = R21 * sy, M22 = R22 * sz;
        float T0[3], T1[3], T2[3];
        T0[0] = c.R[0] * M00 + c.R[1] * M10 + c.R[2] * M20;
        T0[1] = c.R[0] * M01 + c.R[1] * M11 + c.R[2] * M21;
        T0[2] = c.R[0] * M02 + c.R[1] * M12 + c.R[2] * M22;
        T1[0] = c.R[3] * M00 + c.R[4] * M10 + c.R[5] * M20;
        T1[1] = c.R[3] * M01 + c.R[4] * M11 + c.R[5] * M21;
        T1[2] = c.R[3] * M02 + c.R[4] * M12 + c.R[5] * M22;
        T2[0] = c.R[6] * M00 + c.R[7] * M10 + c.R[8] * M20;
        T2[1] = c.R[6] * M01 + c.R[7] * M11 + c.R[8] * M21;
        T2[2] = c.R[6] * M02 + c.R[7] * M12 + c.R[8] * M22;
        // J at the guarded point
        float iz = 1.f / pz;
        float u = px * iz, v = py * iz;
        float tx = fminf(fmaxf(u, -c.limx), c.limx) * pz;
        float ty = fminf(fmaxf(v, -c.limy), c.limy) * pz;
        float J00 = c.fx * iz, J02 = -c.fx * tx * iz * iz;
        float J11 = c.fy * iz, J12 = -c.fy * ty * iz * iz;
        // U = J T (2x3);  Sigma' = U U^T + 0.3 I
        float U0[3], U1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U0[k] = J00 * T0[k] + J02 * T2[k];
            U1[k] = J11 * T1[k] + J12 * T2[k];
        }
        float a = U0[0] * U0[0] + U0[1] * U0[1] + U0[2] * U0[2] + kDilation;
        float b = U0[0] * U1[0] + U0[1] * U1[1] + U0[2] * U1[2];
        float cc = U1[0] * U1[0] + U1[1] * U1[1] + U1[2] * U1[2] + kDilation;
        float det = a * cc - b * b;
        ok = det > 0.f;
        if (ok) {
            float id = 1.f / det;
            float mx2 = c.fx * u + c.cx, my2 = c.fy * v + c.cy;
            float tau = 2.f * __logf(255.f * o);
            float ex = sqrtf(tau * a), ey = sqrtf(tau * cc);
            // sampled-pixel index range whose centres lie in [m - e, m + e]
            float fs = (float)c.s;
            float nlo = ceilf((mx2 - ex - (float)c.ox - 0.5f) / fs);
            float nhi = floorf((mx2 + ex - (float)c.ox - 0.5f) / fs);
            float mlo = ceilf((my2 - ey - (float)c.oy - 0.5f) / fs);
            float mhi = floorf((my2 + ey - (float)c.oy - 0.5f) / fs);
            nlo = fmaxf(nlo, 0.f);
            mlo = fmaxf(mlo, 0.f);
            nhi = fminf(nhi, (float)(c.ws - 1));
            mhi = fminf(mhi, (float)(c.hs - 1));
            ok = (nlo <= nhi) && (mlo <= mhi);
            if (ok) {
                int x0 = (int)nlo / kTile, x1 = (int)nhi / kTile + 1;
                int y0 = (int)mlo / kTile, y1 = (int)mhi / kTile + 1;
                rect = make_uint2((uint32_t)x0 | (((uint32_t)y0 + row_off) << 16),
                                  (uint32_t)x1 | (((uint32_t)y1 + row_off) << 16));
                tt = (uint32_t)((x1 - x0) * (y1 - y0));
                rad = (int32_t)ceilf(fmaxf(ex, ey));
                if (rad < 1) rad = 1;
                s0 = make_float4(mx2, my2, cc * id, -b * id);
                s1 = make_float4(a * id, o, pz, 0.f);
            }
        }
    }
    splat[2 * o_] = s0;
    splat[2 * o_ + 1] = s1;
    radius[o_] = rad;
    tile_rect[o_] = rect;
    touched[o_] = tt;
}

// viewmat (optional): world->camera matrix in device memory, row-major 4x4;
// when given it replaces the rotation and translation in c.
__global__ void __launch_bounds__(256) project_kernel(
    int64_t n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ opacity, CamDev c,
    const float* __restrict__ viewmat, float4* __restrict__ splat, int32_t* __restrict__ radius,
    uint2* __restrict__ tile_rect, uint32_t* __restrict__ touched) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (viewmat) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int k = 0; k < 3; ++k) c.R[3 * r + k] = viewmat[4 * r + k];
            c.t[r] = viewmat[4 * r + 3];
        }
    }
    project_one(i, i, means, log_scales, quats, opacity, c, 0u, splat, radius, tile_rect, touched);
}

__host__ __device__ inline CamDev cam_dev(const xgs_camera& cam) {
    CamDev c;
    c.fx = cam.fx; c.fy = cam.fy; c.cx = cam.cx; c.cy = cam.cy; c.near_ = cam.near_plane;
    c.limx = kGuard * (0.5f * cam.width) / cam.fx;
    c.limy = kGuard * (0.5f * cam.height) / cam.fy;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) c.R[3 * r + k] = cam.viewmat[4 * r + k];
        c.t[r] = cam.viewmat[4 * r + 3];
    }
    c.s = cam.stride; c.oy = cam.off_y; c.ox = cam.off_x;
    c.hs = (cam.height + cam.stride - 1) / cam.stride;
    c.ws = (cam.width + cam.stride - 1) / cam.stride;
    return c;
}

// Batched projection: row i of the batch belongs to the slot whose
// [gauss_base, gauss_base + n) holds it.  Each block reads the slot bounds
// and builds every slot's camera once, in LDS; rows of no slot only get
// tiles_touched = 0 (nothing else of such a row is ever read).
__global__ void __launch_bounds__(256) project_batch_kernel(
    const xgs_batch_slot* __restrict__ slots, int n_slots, int64_t cap, float4* __restrict__ splat,
    int32_t* __restrict__ radius, uint2* __restrict__ tile_rect, uint32_t* __restrict__ touched) {
    __shared__ int64_t s_lo[XGS_BATCH_MAX_SLOTS], s_hi[XGS_BATCH_MAX_SLOTS];
    __shared__ CamDev s_cam[XGS_BATCH_MAX_SLOTS];
    if (threadIdx.x < n_slots) {
        const xgs_batch_slot& sl = slots[threadIdx.x];
        s_lo[threadIdx.x] = sl.gauss_base;
        s_hi[threadIdx.x] = sl.gauss_base + sl.g.n;
        s_cam[threadIdx.x] = cam_dev(sl.cam);
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    int s = -1;
    for (int j = 0; j < n_slots; ++j)
        if (i >= s_lo[j] && i < s_hi[j]) s = j;
    if (s < 0) {
        touched[i] = 0u;
        return;
    }
    const xgs_batch_slot& sl = slots[s];
    project_one(i - s_lo[s], i, sl.g.means, sl.g.log_scales, reinterpret_cast<const float4*>(sl.g.quats),
                sl.g.opacity, s_cam[s], (uint32_t)sl.row_base, splat, radius, tile_rect, touched);
}

}  // namespace xgs

using namespace xgs;

static xgs_status project_impl(const xgs_gaussians* g, const xgs_camera* cam, const float* d_viewmat,
                               xgs_projected* out, xgs_stream_t stream, const char* name) {
    clear_error();
    if (!g || !cam || !out) return fail(XGS_ERR_INVALID_ARG, std::string(name) + ": null argument");
    if (xgs_status s = validate_camera(cam)) return s;
    if (g->n < 0) return fail(XGS_ERR_INVALID_ARG, std::string(name) + ": n < 0");
    if (g->n == 0) return XGS_OK;
    if (!g->means || !g->log_scales || !g->quats || !g->opacity)
        return fail(XGS_ERR_INVALID_ARG, std::string(name) + ": null Gaussian array");
    if (!out->splat || !out->radius || !out->tile_rect || !out->tiles_touched)
        return fail(XGS_ERR_INVALID_ARG, std::string(name) + ": null output array");
    if (!aligned(g->quats, 16) || !aligned(out->splat, 16) || !aligned(out->tile_rect, 8))
        return fail(XGS_ERR_INVALID_ARG, std::string(name) + ": quats/splat need 16-byte, tile_rect 8-byte alignment");
    Grid gr = grid_of(*cam);
    if (gr.tx > 65535 || gr.ty > 65535)
        return fail(XGS_ERR_UNSUPPORTED, std::string(name) + ": more than 65535 tiles along an axis");
    CamDev c = cam_dev(*cam);
    int64_t blocks = (g->n + 255) / 256;
    hipLaunchKernelGGL(project_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       g->n, g->means, g->log_scales, reinterpret_cast<const float4*>(g->quats),
                       g->opacity, c, d_viewmat, reinterpret_cast<float4*>(out->splat), out->radius,
                       reinterpret_cast<uint2*>(out->tile_rect), out->tiles_touched);
    return check_launch(name);
}

extern "C" xgs_status xgs_project(const xgs_gaussians* g, const xgs_camera* cam,
                                  xgs_projected* out, xgs_stream_t stream) {
    return project_impl(g, cam, nullptr, out, stream, "xgs_project");
}

extern "C" xgs_status xgs_project_posed(const xgs_gaussians* g, const xgs_camera* cam,
                                        const float* d_viewmat, xgs_projected* out,
                                        xgs_stream_t stream) {
    if (!d_viewmat) return fail(XGS_ERR_INVALID_ARG, "xgs_project_posed: null device viewmat");
    return project_impl(g, cam, d_viewmat, out, stream, "xgs_project_posed");
}

extern "C" xgs_status xgs_batch_check(const xgs_batch_slot* h, int32_t n_slots, int64_t cap_gaussians,
                                      int32_t tiles_x, int32_t tile_rows, int32_t c_sem) {
    clear_error();
    if (n_slots < 0 || n_slots > XGS_BATCH_MAX_SLOTS)
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_check: n_slots must be in [0, 16]");
    if (n_slots > 0 && !h) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_check: null slot table");
    if (cap_gaussians < 0 || tiles_x < 1 || tile_rows < 1 || tiles_x > 65535 || tile_rows > 65535)
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_check: bad capacities");
    int64_t g_end = 0;
    int32_t r_end = 0;
    for (int s = 0; s < n_slots; ++s) {
        const xgs_batch_slot& sl = h[s];
        const std::string who = "xgs_batch_check: slot " + std::to_string(s);
        if (xgs_status st = validate_camera(&sl.cam)) return fail(st, who + ": " + xgs_last_error());
        Grid gr = grid_of(sl.cam);
        if (sl.g.n < 0 || sl.gauss_base < g_end || sl.gauss_base + sl.g.n > cap_gaussians)
            return fail(XGS_ERR_INVALID_ARG, who + ": Gaussian rows overlap or exceed cap_gaussians");
        if (sl.row_base < r_end || (int64_t)sl.row_base + gr.ty > tile_rows || gr.tx > tiles_x)
            return fail(XGS_ERR_INVALID_ARG, who + ": tile band overlaps or exceeds the grid");
        if (sl.g.c_sem != c_sem) return fail(XGS_ERR_INVALID_ARG, who + ": c_sem differs");
        if (!sl.out || !sl.final_T || !sl.n_last) return fail(XGS_ERR_INVALID_ARG, who + ": null output");
        if (sl.g.n > 0 && (!sl.g.means || !sl.g.log_scales || !sl.g.quats || !sl.g.opacity || !sl.g.colors ||
                           (c_sem > 0 && !sl.g.features)))
            return fail(XGS_ERR_INVALID_ARG, who + ": null Gaussian array");
        if (sl.g.n > 0 && !aligned(sl.g.quats, 16))
            return fail(XGS_ERR_INVALID_ARG, who + ": quats need 16-byte alignment");
        g_end = sl.gauss_base + sl.g.n;
        r_end = sl.row_base + gr.ty;
    }
    return XGS_OK;
}

extern "C" xgs_status xgs_batch_project(const xgs_batch_slot* d_slots, int32_t n_slots, int64_t cap_gaussians,
                                        int32_t tiles_x, int32_t tile_rows, xgs_projected* out,
                                        xgs_stream_t stream) {
    clear_error();
    if (!out) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_project: null argument");
    if (n_slots < 0 || n_slots > XGS_BATCH_MAX_SLOTS)
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_project: n_slots must be in [0, 16]");
    if (n_slots > 0 && !d_slots) return fail(XGS_ERR_INVALID_ARG, "xgs_batch_project: null slot table");
    if (cap_gaussians < 0 || tiles_x < 1 || tile_rows < 1 || tiles_x > 65535 || tile_rows > 65535)
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_project: bad capacities");
    if (cap_gaussians == 0) return XGS_OK;
    if (!out->splat || !out->radius || !out->tile_rect || !out->tiles_touched)
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_project: null output array");
    if (!aligned(out->splat, 16) || !aligned(out->tile_rect, 8))
        return fail(XGS_ERR_INVALID_ARG, "xgs_batch_project: splat needs 16-byte, tile_rect 8-byte alignment");
    const int64_t blocks = (cap_gaussians + 255) / 256;
    hipLaunchKernelGGL(project_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, d_slots,
                       (int)n_slots, cap_gaussians, reinterpret_cast<float4*>(out->splat), out->radius,
                       reinterpret_cast<uint2*>(out->tile_rect), out->tiles_touched);
    return check_launch("xgs_batch_project");
}
