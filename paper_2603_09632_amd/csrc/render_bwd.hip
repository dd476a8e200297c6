// a4: backward of the compositing step and of the EWA projection.
//
// Pixel pass: each wavefront takes an 8x8 quadrant of a tile and walks the
// tile list back to front from the largest n_last of its pixels.  A pixel
// recovers the transmittance in front of Gaussian k as T_k = T_{k+1}/(1-a_k),
// starting from final_T, so nothing per (pixel, Gaussian) is stored by the
// forward pass.  With S_k = sum_{j>k} a_j T_j (g . c_j), the derivative of
// Eq. (rendering) is dL/da_k = T_k (g . c_k) - S_k / (1 - a_k).  The per-pixel
// contributions of one Gaussian are summed over the wavefront by a
// reduce-scatter (each exchange halves the number of live values per lane), so
// one atomic instruction per Gaussian and wave carries all of its sums.
//
// Gaussian pass: gradients of (mean2d, conic, depth) are carried back through
// conic = Sigma'^-1, Sigma' = J Sigma_cam J^T + 0.3 I, Sigma_cam = Rv Sigma Rv^T,
// Sigma = (R S)(R S)^T, p = Rv mu + t (App. A).
#include "render_common.h"
#include "sort.h"
#include "wave.h"

namespace xgs {

// Geometry workspace row per Gaussian (8 floats).
enum { GW_MX = 0, GW_MY = 1, GW_A = 2, GW_B = 3, GW_C = 4, GW_DEPTH = 5, GW_STRIDE = 8 };

// The walk runs back to front.  The tile list is read 64 entries at a time
// (one per lane: list entry and splat record, the next 64 in flight), the
// splats that can reach alpha >= 1/255 somewhere in the wavefront's quadrant
// are appended to a ring in LDS (quad_hit; the others are skipped by all 64
// pixels) and the walk takes the ring 16 at a time, with the channel rows of
// the next batch in flight.  Per Gaussian each pixel recovers T_k, forms
// w_k = a_k T_k and dL/da_k; the six geometric sums (opacity, conic A B C,
// mean x y) are reduced over the wavefront at once (reduce-scatter, 6 values)
// and added atomically.  The channel gradients dL/dc_k = sum_p w_k(p) g(p) of
// the batch are one 16 x 64 x 48 product W^T G on v_mfma_f32_16x16x4_f32:
// W goes through LDS, G (the wave's upstream gradients in operand layout) is
// loaded once.
template <int CS, bool GEO, bool EXACT>
__global__ void __launch_bounds__(64) render_bwd_mfma_kernel(
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float4* __restrict__ splat, const float* __restrict__ colors,
    const float* __restrict__ features, int csem, TileGrid g, const float* __restrict__ d_out,
    const float* __restrict__ final_T, const int32_t* __restrict__ n_last,
    float* __restrict__ d_colors, float* __restrict__ d_features, float* __restrict__ d_opacity,
    float* __restrict__ geo) {
    constexpr int CH = 4 + CS;
    constexpr int CHP = (CH + 3) / 4 * 4;           // LDS row stride (float4 rows)
    constexpr int NT = (CH + 15) / 16;
    constexpr int VG = 6;
    __shared__ float wl[64 * 17];
    __shared__ Ring ring;
    __shared__ __align__(16) float chl[16 * CHP];
    __shared__ float sdl[GEO ? 64 * 17 : 1];
    const QuadPix P = quad_pixel(g);
    if (P.tile >= g.tiles) return;
    const QuadRect qr = quad_rect(g, P);
    const int lane = threadIdx.x;
    int my_id = 0;
    bool my_own = false;
    if (GEO) rs_layout<2 * VG>(lane, &my_id, &my_own);
    const int my_split = my_id / VG, my_v = my_id - VG * (my_id / VG);  // splat of the pair, sum
    // the array and stride that this lane's sum goes to (lane-constant, so the
    // walk adds without branching on the destination)
    float* const g_base = my_v == 0 ? d_opacity
                                    : geo + (my_v == 1 ? GW_A : my_v == 2 ? GW_B : my_v == 3 ? GW_C
                                                        : my_v == 4 ? GW_MX : GW_MY);
    const int g_stride = my_v == 0 ? 1 : GW_STRIDE;
    const size_t hw = (size_t)g.hs * g.ws;
    const int fstride = EXACT ? CS : csem;
    const int qx = P.n - (lane & 7), qy = P.m - (lane >> 3);  // quadrant origin
    // upstream gradients in B-operand layout: pixel 4 kk + lane / 16, channel 16 nt + lane % 16
    float bg[NT][16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int p = 4 * kk + (lane >> 4);
        const int m = qy + (p >> 3), n = qx + (p & 7);
        const bool in = m < g.hs && n < g.ws;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int c = 16 * nt + (lane & 15);
            const bool use = in && c < CH && (GEO || c >= 4) && (EXACT || c < 4 + csem);
            bg[nt][kk] = use ? d_out[c * hw + (size_t)m * g.ws + n] : 0.f;
        }
    }
    // Upstream gradients as the B operand of S = C G^T (channel 4 kc + lane / 16,
    // pixel 16 nt + lane % 16): S[k][p] = g(p) . c_k for the batch's 16 splats.
    constexpr int KC = CHP / 4;
    float gt[GEO ? KC : 1][4];
    if constexpr (GEO) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int p = 16 * nt + (lane & 15), c = 4 * kc + (lane >> 4);
                const int m = qy + (p >> 3), n = qx + (p & 7);
                const bool use = m < g.hs && n < g.ws && c < CH && (EXACT || c < 4 + csem);
                gt[kc][nt] = use ? d_out[c * hw + (size_t)m * g.ws + n] : 0.f;
            }
    }
    float T = 1.f;
    int nl = 0;
    if (P.inside) {
        const size_t pix = (size_t)P.m * g.ws + P.n;
        T = final_T[pix];
        nl = n_last[pix];
    }
    int jmax = nl;
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) jmax = max(jmax, __shfl_xor(jmax, k, 64));
    const uint32_t start = uniform(ranges[2 * P.tile]);
    const int top = (int)uniform((uint32_t)jmax);

    // candidate registers: list entry and splat record of position cpos - 1 - lane
    int cg = -1;
    float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
    auto fetch = [&](int pos) {
        const int j = pos - 1 - lane;
        cg = -1;
        if (j >= 0) {
            cg = (int)vals[start + (uint32_t)j];
            c0 = splat[2 * (uint32_t)cg];
            c1 = splat[2 * (uint32_t)cg + 1];
        }
    };
    int cpos = top, head = 0, tail = 0;
    // keeps at least two batches in the ring (or everything that is left);
    // the slots written lie past the two batches being read
    auto fill = [&]() {
        while (tail - head < 32 && cpos > 0) {
            tail = ring_push(ring, tail, cg >= 0 && quad_hit(c0, c1, qr), c0, c1, cg, cpos - 1 - lane);
            cpos -= 64;
            fetch(cpos);
        }
    };
    // Channel rows of a batch (only the S = C G^T product reads them): the
    // colour and depth of splat lane / 4 (channel lane % 4) in one load, then
    // the feature rows as 64 consecutive (splat, feature) pairs per load, so
    // that every load reads one array and feature rows are read contiguously.
    // Slots past the batch hold zeros.
    constexpr int PERF = (16 * CS + 63) / 64;
    constexpr int CSD = CS > 0 ? CS : 1;  // divisor (no feature loads when CS = 0)
    float cv[GEO ? 1 + PERF : 1];
    auto fetch_channels = [&](int base, int n) {
        if constexpr (GEO) {
            {
                const int k = lane >> 2, c = lane & 3;
                const int gk = k < n ? ring.gid[(base + k) & (kRing - 1)] : -1;
                const uint32_t i = (uint32_t)(gk >= 0 ? gk : 0);
                const float* src = c < 3 ? colors + 3 * (size_t)i + c
                                         : reinterpret_cast<const float*>(splat) + 8 * (size_t)i + 6;  // depth
                cv[0] = gk >= 0 ? *src : 0.f;
            }
#pragma unroll
            for (int t = 1; t <= PERF; ++t) {
                const int e = lane + 64 * (t - 1);
                const int k = e / CSD, f = e - k * CSD;
                const int gk = k < n ? ring.gid[(base + k) & (kRing - 1)] : -1;
                cv[t] = (gk >= 0 && (EXACT || f < csem)) ? features[(size_t)gk * fstride + f] : 0.f;
            }
        }
    };
    auto store_channels = [&]() {
        if constexpr (GEO) {
            chl[(lane >> 2) * CHP + (lane & 3)] = cv[0];
#pragma unroll
            for (int t = 1; t <= PERF; ++t) {
                const int e = lane + 64 * (t - 1);
                const int k = e / CSD, f = e - k * CSD;
                if (k < 16) chl[k * CHP + 4 + f] = cv[t];
            }
        }
    };
    if constexpr (GEO && CHP > CH) {  // padding columns, read as zeros by the product
        for (int i = lane; i < 16 * (CHP - CH); i += 64) chl[(i / (CHP - CH)) * CHP + CH + i % (CHP - CH)] = 0.f;
    }
    fetch(top);
    fill();
    __syncthreads();
    int nb = min(16, tail - head);
    fetch_channels(head, nb);
    float S = 0.f;
    while (nb > 0) {
        store_channels();
        fill();
        __syncthreads();
        if constexpr (GEO) {
            // S = C G^T on the matrix cores (A: splat lane % 16, channel 4 kc + lane / 16),
            // stored as sdl[pixel][splat] for the walk
            f32x4_t sacc[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) sacc[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const float a = chl[(lane & 15) * CHP + 4 * kc + (lane >> 4)];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) sacc[nt] = mfma16x16x4(a, gt[kc][nt], sacc[nt]);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) sdl[(16 * nt + (lane & 15)) * 17 + 4 * (lane >> 4) + r] = sacc[nt][r];
        }
        const int nb2 = min(16, tail - head - nb);
        fetch_channels(head + nb, nb2);
        if constexpr (GEO) __syncthreads();
        // Splats are taken in pairs: the twelve sums of a pair share one
        // reduce-scatter and one atomic instruction.
#pragma unroll
        for (int k2 = 0; k2 < 16; k2 += 2) {
            float a[2 * VG];
#pragma unroll
            for (int v = 0; v < 2 * VG; ++v) a[v] = 0.f;
            bool any = false;
            int gp[2] = {-1, -1};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                // branch-free: slots past the batch are read (in bounds) and
                // every result is selected, so stale records change nothing
                const int k = k2 + u;
                const int at = (head + k) & (kRing - 1);
                const float4 s0 = ring.rec[at][0];
                const float4 s1 = ring.rec[at][1];
                gp[u] = k < nb ? ring.gid[at] : -1;
                const int j = ring.pos[at];
                const PairEval e = eval_pair(P.px, P.py, s0.x, s0.y, s0.z, s0.w, s1.x, s1.y);
                const bool contrib = k < nb && j < nl && e.alpha >= kAlphaMin;
                const float om = 1.f - e.alpha;  // >= 0.01
                const float rom = __builtin_amdgcn_rcpf(om);
                const float Tk = T * rom;
                const float wv = e.alpha * Tk;
                if (GEO) {
                    const float sd = sdl[lane * 17 + k];
                    const float dalpha = Tk * sd - S * rom;
                    const bool live = contrib && s1.y * e.G < kAlphaMax;
                    const float dq = dalpha * s1.y * e.G * -0.5f;
                    a[VG * u + 0] = live ? dalpha * e.G : 0.f;
                    a[VG * u + 1] = live ? dq * e.dx * e.dx : 0.f;
                    a[VG * u + 2] = live ? 2.f * dq * e.dx * e.dy : 0.f;
                    a[VG * u + 3] = live ? dq * e.dy * e.dy : 0.f;
                    a[VG * u + 4] = live ? -2.f * dq * (s0.z * e.dx + s0.w * e.dy) : 0.f;
                    a[VG * u + 5] = live ? -2.f * dq * (s0.w * e.dx + s1.x * e.dy) : 0.f;
                    S = contrib ? S + wv * sd : S;
                }
                T = contrib ? Tk : T;
                const float w = contrib ? wv : 0.f;
                any = any || contrib;
                wl[lane * 17 + k] = w;
            }
            if (GEO && k2 < nb && __ballot(any) != 0ull) {
                reduce_scatter<2 * VG>(a, lane);
                const int gid = my_split ? gp[1] : gp[0];
                if (my_own && gid >= 0) unsafeAtomicAdd(g_base + (size_t)gid * g_stride, a[0]);
            }
        }
        __syncthreads();
        f32x4_t acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const float a = wl[(4 * kk + (lane >> 4)) * 17 + (lane & 15)];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16x16x4(a, bg[nt][kk], acc[nt]);
        }
        // acc[nt][r]: Gaussian slot 4 (lane / 16) + r, channel 16 nt + lane % 16
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int slot = 4 * (lane >> 4) + r;
            const int gs = slot < nb ? ring.gid[(head + slot) & (kRing - 1)] : -1;
            if (gs < 0) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                // channel c of this lane: colour, depth (workspace row) or feature
                const int c = 16 * nt + (lane & 15);
                const bool ok = c < CH && (EXACT || c < 4 + csem) && (GEO || c >= 4);
                float* const base = c < 3 ? d_colors + c : c == 3 ? geo + GW_DEPTH : d_features + (c - 4);
                const int stride = c < 3 ? 3 : c == 3 ? (int)GW_STRIDE : fstride;
                const float v = acc[nt][r];
                if (ok && v != 0.f) unsafeAtomicAdd(base + (size_t)gs * stride, v);
            }
        }
        __syncthreads();
        head += nb;
        nb = nb2;
    }
}

struct CamDevB {
    float fx, fy, limx, limy, near_;
    float R[9], t[3];
};

// Adjoint of one Gaussian's projection down to the camera frame (App. A):
// recomputes p = Rv mu + t, R(q), the scales, M = R S, Sigma_cam = (Rv M)
// (Rv M)^T and J at the guarded p, then carries dL/dmean2d, dL/dconic and
// dL/ddepth (the workspace row) to dL/dp and dL/dSigma_cam.
struct CamAdj {
    float p[3];
    float R[3][3], s[3], M[3][3], Sc[3][3];
    float dSc[3][3], dp[3];
    float q[4], inv;
};

__device__ __forceinline__ void cam_adjoint(int64_t i, const float* __restrict__ means,
                                            const float* __restrict__ log_scales,
                                            const float4* __restrict__ quats, const float4* __restrict__ splat,
                                            const float* __restrict__ gw, const CamDevB& c, CamAdj& a) {
    const float gmx = gw[GW_MX], gmy = gw[GW_MY];
    const float gA = gw[GW_A], gB = gw[GW_B], gC = gw[GW_C], gd = gw[GW_DEPTH];
    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    const float px = c.R[0] * mx + c.R[1] * my + c.R[2] * mz + c.t[0];
    const float py = c.R[3] * mx + c.R[4] * my + c.R[5] * mz + c.t[1];
    const float pz = c.R[6] * mx + c.R[7] * my + c.R[8] * mz + c.t[2];
    a.p[0] = px; a.p[1] = py; a.p[2] = pz;
    float4 q = quats[i];
    const float qn = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    a.inv = 1.f / qn;
    const float w = q.x * a.inv, x = q.y * a.inv, y = q.z * a.inv, z = q.w * a.inv;
    a.q[0] = w; a.q[1] = x; a.q[2] = y; a.q[3] = z;
    const float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                           {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                           {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) a.R[r][k] = R[r][k];
    a.s[0] = __expf(log_scales[3 * i]); a.s[1] = __expf(log_scales[3 * i + 1]); a.s[2] = __expf(log_scales[3 * i + 2]);
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) a.M[r][k] = R[r][k] * a.s[k];
    // Sigma_cam = (Rv M)(Rv M)^T
    float TM[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            TM[r][k] = c.R[3 * r] * a.M[0][k] + c.R[3 * r + 1] * a.M[1][k] + c.R[3 * r + 2] * a.M[2][k];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) a.Sc[r][k] = TM[r][0] * TM[k][0] + TM[r][1] * TM[k][1] + TM[r][2] * TM[k][2];
    const float iz = 1.f / pz;
    const float u = px * iz, v = py * iz;
    const bool clx = u < -c.limx || u > c.limx, cly = v < -c.limy || v > c.limy;
    const float tx = fminf(fmaxf(u, -c.limx), c.limx) * pz;
    const float ty = fminf(fmaxf(v, -c.limy), c.limy) * pz;
    const float J[2][3] = {{c.fx * iz, 0.f, -c.fx * tx * iz * iz}, {0.f, c.fy * iz, -c.fy * ty * iz * iz}};
    // conic = (A, B, C) from the splat record; dSigma' = -K Ghat K
    const float4 s0 = splat[2 * i], s1 = splat[2 * i + 1];
    const float K00 = s0.z, K01 = s0.w, K11 = s1.x;
    const float G00 = gA, G01 = 0.5f * gB, G11 = gC;
    const float KG00 = K00 * G00 + K01 * G01, KG01 = K00 * G01 + K01 * G11;
    const float KG10 = K01 * G00 + K11 * G01, KG11 = K01 * G01 + K11 * G11;
    const float dS00 = -(KG00 * K00 + KG01 * K01);
    const float dS01 = -(KG00 * K01 + KG01 * K11);
    const float dS11 = -(KG10 * K01 + KG11 * K11);
    const float dS[2][2] = {{dS00, dS01}, {dS01, dS11}};
    // dSc = J^T dS J ; dJ = 2 dS J Sc
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            float acc = 0.f;
            for (int aa = 0; aa < 2; ++aa)
                for (int bb = 0; bb < 2; ++bb) acc += J[aa][r] * dS[aa][bb] * J[bb][k];
            a.dSc[r][k] = acc;
        }
    float JSc[2][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) JSc[r][k] = J[r][0] * a.Sc[0][k] + J[r][1] * a.Sc[1][k] + J[r][2] * a.Sc[2][k];
    float dJ[2][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) dJ[r][k] = 2.f * (dS[r][0] * JSc[0][k] + dS[r][1] * JSc[1][k]);
    // J(p), mean2d(p), depth(p) -> p
    const float iz2 = iz * iz, iz3 = iz2 * iz;
    const float dtx_dpx = clx ? 0.f : 1.f, dtx_dpz = clx ? tx * iz : 0.f;
    const float dty_dpy = cly ? 0.f : 1.f, dty_dpz = cly ? ty * iz : 0.f;
    a.dp[0] = dJ[0][2] * (-c.fx * iz2) * dtx_dpx + gmx * c.fx * iz;
    a.dp[1] = dJ[1][2] * (-c.fy * iz2) * dty_dpy + gmy * c.fy * iz;
    a.dp[2] = dJ[0][0] * (-c.fx * iz2) + dJ[1][1] * (-c.fy * iz2) +
              dJ[0][2] * (-c.fx * iz2 * dtx_dpz + 2.f * c.fx * tx * iz3) +
              dJ[1][2] * (-c.fy * iz2 * dty_dpz + 2.f * c.fy * ty * iz3) - gmx * c.fx * px * iz2 -
              gmy * c.fy * py * iz2 + gd;
}

// Per-Gaussian chain rule from (mean2d, conic, depth) to (mean, log-scale,
// quaternion); the forward quantities are recomputed from the parameters.
__global__ void __launch_bounds__(256) project_bwd_kernel(
    int64_t n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const int32_t* __restrict__ radius,
    const float4* __restrict__ splat, const float* __restrict__ geo, CamDevB c,
    float* __restrict__ d_means, float* __restrict__ d_ls, float4* __restrict__ d_quats) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gm[3] = {0.f, 0.f, 0.f}, gl[3] = {0.f, 0.f, 0.f};
    float4 gq = make_float4(0.f, 0.f, 0.f, 0.f);
    if (radius[i] > 0) {
        CamAdj a;
        cam_adjoint(i, means, log_scales, quats, splat, geo + (size_t)i * GW_STRIDE, c, a);
        // dSigma = Rv^T dSc Rv
        float tmp[3][3], dSig[3][3];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                tmp[r][k] = c.R[r] * a.dSc[0][k] + c.R[3 + r] * a.dSc[1][k] + c.R[6 + r] * a.dSc[2][k];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                dSig[r][k] = tmp[r][0] * c.R[k] + tmp[r][1] * c.R[3 + k] + tmp[r][2] * c.R[6 + k];
        // dM = 2 dSig M ; dR = dM diag(s) ; ds = diag(R^T dM)
        float dR[3][3];
        for (int k = 0; k < 3; ++k) {
            float ds = 0.f;
            for (int r = 0; r < 3; ++r) {
                const float dM = 2.f * (dSig[r][0] * a.M[0][k] + dSig[r][1] * a.M[1][k] + dSig[r][2] * a.M[2][k]);
                ds += dM * a.R[r][k];
                dR[r][k] = dM * a.s[k];
            }
            gl[k] = ds * a.s[k];
        }
        const float w = a.q[0], x = a.q[1], y = a.q[2], z = a.q[3];
        float g0 = 2.f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
        float g1 = 2.f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.f * x * dR[1][1] - w * dR[1][2] +
                          z * dR[2][0] + w * dR[2][1] - 2.f * x * dR[2][2]);
        float g2 = 2.f * (-2.f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                          w * dR[2][0] + z * dR[2][1] - 2.f * y * dR[2][2]);
        float g3 = 2.f * (-2.f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.f * z * dR[1][1] +
                          y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
        const float dot = w * g0 + x * g1 + y * g2 + z * g3;
        gq = make_float4((g0 - w * dot) * a.inv, (g1 - x * dot) * a.inv, (g2 - y * dot) * a.inv,
                         (g3 - z * dot) * a.inv);
        // p -> mu
        for (int k = 0; k < 3; ++k) gm[k] = c.R[k] * a.dp[0] + c.R[3 + k] * a.dp[1] + c.R[6 + k] * a.dp[2];
    }
    d_means[3 * i] = gm[0]; d_means[3 * i + 1] = gm[1]; d_means[3 * i + 2] = gm[2];
    d_ls[3 * i] = gl[0]; d_ls[3 * i + 1] = gl[1]; d_ls[3 * i + 2] = gl[2];
    d_quats[i] = gq;
}

// Camera-pose gradient (Eq. (tracking): extrinsics optimised with the map
// frozen) for the left perturbation T(xi) = exp(xi^) T, xi = (rho, phi):
// p -> p + rho + phi x p and Sigma_cam -> Sigma_cam + phi^ Sigma_cam -
// Sigma_cam phi^, so per Gaussian dL/drho = dL/dp and
// dL/dphi = p x dL/dp + axial(Sc G - G Sc), G = dL/dSigma_cam,
// axial(A) = (A_23 - A_32, A_31 - A_13, A_12 - A_21).  Each workgroup sums
// its 256 Gaussians in a fixed tree order into partial[block][6].
__global__ void __launch_bounds__(256) pose_grad_kernel(
    int64_t n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const int32_t* __restrict__ radius, const float4* __restrict__ splat,
    const float* __restrict__ geo, CamDevB c, float* __restrict__ partial) {
    __shared__ float red[4][6];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < n && radius[i] > 0) {
        CamAdj a;
        cam_adjoint(i, means, log_scales, quats, splat, geo + (size_t)i * GW_STRIDE, c, a);
        float A[3][3];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) {
                float acc = 0.f;
                for (int m = 0; m < 3; ++m) acc += a.Sc[r][m] * a.dSc[m][k] - a.dSc[r][m] * a.Sc[m][k];
                A[r][k] = acc;
            }
        const float* p = a.p;
        const float* dp = a.dp;
        v[0] = dp[0]; v[1] = dp[1]; v[2] = dp[2];
        v[3] = p[1] * dp[2] - p[2] * dp[1] + (A[1][2] - A[2][1]);
        v[4] = p[2] * dp[0] - p[0] * dp[2] + (A[2][0] - A[0][2]);
        v[5] = p[0] * dp[1] - p[1] * dp[0] + (A[0][1] - A[1][0]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
        for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 6; ++k) red[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6)
        partial[(size_t)blockIdx.x * 6 + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// Thread j sums the partials of blocks j, j + 256, ... in order, then a
// fixed tree combines the 256 sums: deterministic.
__global__ void __launch_bounds__(256) pose_total_kernel(const float* __restrict__ partial, int64_t nb,
                                                        float* __restrict__ d_pose) {
    __shared__ float red[6][256];
    const int t = threadIdx.x;
    float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t b = t; b < nb; b += 256)
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] += partial[(size_t)b * 6 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) red[k][t] = s[k];
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (t < o)
#pragma unroll
            for (int k = 0; k < 6; ++k) red[k][t] += red[k][t + o];
        __syncthreads();
    }
    if (t < 6) d_pose[t] = red[t][0];
}

template <int CS, bool GEO, bool EXACT = true>
static void launch_bwd(const xgs_gaussians* g, const xgs_projected* p, const xgs_binning* b,
                       const TileGrid& tg, const float* d_out, const float* final_T,
                       const int32_t* n_last, xgs_gaussians_grad* gr, float* geo, hipStream_t st) {
    hipLaunchKernelGGL((render_bwd_mfma_kernel<CS, GEO, EXACT>), dim3(quad_blocks(tg)), dim3(64), 0, st, b->ranges,
                       b->vals, reinterpret_cast<const float4*>(p->splat), g->colors, g->features, g->c_sem, tg,
                       d_out, final_T, n_last, gr->colors, gr->features, gr->opacity, geo);
}

template <bool GEO>
static void dispatch_bwd(const xgs_gaussians* g, const xgs_projected* p, const xgs_binning* b,
                         const TileGrid& tg, const float* d_out, const float* final_T,
                         const int32_t* n_last, xgs_gaussians_grad* gr, float* geo, hipStream_t st) {
    const int cs = g->c_sem;
    if (!GEO && cs == 0) return;
    switch (cs) {
#define XGS_BWD_CASE(n) case n: launch_bwd<n, GEO>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st); return;
        XGS_BWD_CASE(1) XGS_BWD_CASE(2) XGS_BWD_CASE(3) XGS_BWD_CASE(4) XGS_BWD_CASE(8)
        XGS_BWD_CASE(12) XGS_BWD_CASE(16) XGS_BWD_CASE(24) XGS_BWD_CASE(32) XGS_BWD_CASE(48)
#undef XGS_BWD_CASE
        default: break;
    }
    if constexpr (GEO) {
        if (cs == 0) launch_bwd<0, true>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        else if (cs <= 16) launch_bwd<16, true, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        else if (cs <= 32) launch_bwd<32, true, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        else launch_bwd<54, true, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
    } else {
        if (cs == 64) launch_bwd<64, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        else if (cs <= 16) launch_bwd<16, false, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        else if (cs <= 32) launch_bwd<32, false, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        else launch_bwd<64, false, false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
    }
}

static CamDevB cam_dev_b(const xgs_camera& cam) {
    CamDevB c;
    c.fx = cam.fx; c.fy = cam.fy; c.near_ = cam.near_plane;
    c.limx = kGuard * (0.5f * cam.width) / cam.fx;
    c.limy = kGuard * (0.5f * cam.height) / cam.fy;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) c.R[3 * r + k] = cam.viewmat[4 * r + k];
        c.t[r] = cam.viewmat[4 * r + 3];
    }
    return c;
}

}  // namespace xgs

using namespace xgs;

static size_t pose_blocks(int64_t n) { return (size_t)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

extern "C" size_t xgs_render_bwd_workspace(int64_t n) {
    Carve c(nullptr);
    c.take<float>((size_t)(n > 0 ? n : 1) * GW_STRIDE);
    c.take<float>(pose_blocks(n) * 6);
    return c.total();
}

// The accumulated gradients (features; with the geometry also colours,
// opacity) and the geometry workspace rows start at zero: one launch.
static xgs_status zero_accumulated(const xgs_gaussians* g, bool geo_on, xgs_gaussians_grad* gr, float* geo,
                                   hipStream_t st) {
    ZeroRanges zr{};
    if (g->c_sem > 0) { zr.p[zr.k] = reinterpret_cast<uint32_t*>(gr->features); zr.n[zr.k++] = g->n * g->c_sem; }
    if (geo_on) {
        zr.p[zr.k] = reinterpret_cast<uint32_t*>(gr->colors); zr.n[zr.k++] = 3 * g->n;
        zr.p[zr.k] = reinterpret_cast<uint32_t*>(gr->opacity); zr.n[zr.k++] = g->n;
        zr.p[zr.k] = reinterpret_cast<uint32_t*>(geo); zr.n[zr.k++] = GW_STRIDE * g->n;
    }
    return zero_ranges(zr, st);
}

extern "C" xgs_status xgs_render_bwd_zero(const xgs_gaussians* g, int32_t flags, xgs_gaussians_grad* gr, void* ws,
                                          size_t ws_bytes, xgs_stream_t stream) {
    clear_error();
    if (!g || !gr) return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd_zero: null argument");
    if ((flags & ~XGS_BWD_PREZEROED) != XGS_BWD_ALL && (flags & ~XGS_BWD_PREZEROED) != XGS_BWD_FEATURES_ONLY)
        return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd_zero: unknown flags");
    const bool geo_on = (flags & ~XGS_BWD_PREZEROED) == XGS_BWD_ALL;
    if (g->n < 0 || g->c_sem < 0 || g->c_sem > XGS_MAX_C_SEM || gr->n != g->n || gr->c_sem != g->c_sem)
        return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd_zero: gradient shapes differ from the Gaussians");
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd_zero: workspace must be 256-byte aligned");
    if (!ws || ws_bytes < xgs_render_bwd_workspace(g->n))
        return fail(XGS_ERR_CAPACITY, "xgs_render_bwd_zero: workspace too small");
    if (g->n == 0) return XGS_OK;
    if ((g->c_sem > 0 && !gr->features) || (geo_on && (!gr->colors || !gr->opacity)))
        return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd_zero: null gradient array");
    xgs_status s = zero_accumulated(g, geo_on, gr, static_cast<float*>(ws), (hipStream_t)stream);
    if (s) return s;
    return check_launch("xgs_render_bwd_zero");
}

extern "C" xgs_status xgs_render_bwd(const xgs_gaussians* g, const xgs_projected* p,
                                     const xgs_binning* b, const xgs_camera* cam, const float* d_out,
                                     const float* final_T, const int32_t* n_last, int32_t flags,
                                     xgs_gaussians_grad* gr, void* ws, size_t ws_bytes,
                                     xgs_stream_t stream) {
    clear_error();
    if (!g || !p || !b || !cam || !gr) return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: null argument");
    if (xgs_status s = validate_camera(cam)) return s;
    const bool prezeroed = (flags & XGS_BWD_PREZEROED) != 0;
    flags &= ~XGS_BWD_PREZEROED;
    if (flags != XGS_BWD_ALL && flags != XGS_BWD_FEATURES_ONLY)
        return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: unknown flags");
    const bool geo_on = flags == XGS_BWD_ALL;
    if (g->c_sem < 0 || g->c_sem > XGS_MAX_C_SEM)
        return fail(XGS_ERR_UNSUPPORTED, "xgs_render_bwd: c_sem must be in [0, 64]");
    if (geo_on && g->c_sem > 54)
        return fail(XGS_ERR_UNSUPPORTED, "xgs_render_bwd: c_sem <= 54 (4 + c_sem + 6 sums per lane)");
    if (gr->n != g->n || gr->c_sem != g->c_sem)
        return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: gradient shapes differ from the Gaussians");
    if (!d_out || !final_T || !n_last) return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: null image buffer");
    if (g->n > 0) {
        if (!g->colors || (g->c_sem > 0 && !g->features) || !p->splat || !p->radius)
            return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: null Gaussian array");
        if (g->c_sem > 0 && !gr->features)
            return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: null feature gradient");
        if (geo_on && (!gr->means || !gr->log_scales || !gr->quats || !gr->opacity || !gr->colors ||
                       !g->means || !g->log_scales || !g->quats))
            return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: null gradient array");
        if (geo_on && !aligned(gr->quats, 16))
            return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: quats gradient must be 16-byte aligned");
    }
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_render_bwd: workspace must be 256-byte aligned");
    if (!ws || ws_bytes < xgs_render_bwd_workspace(g->n))
        return fail(XGS_ERR_CAPACITY, "xgs_render_bwd: workspace too small");
    if (g->n == 0) return XGS_OK;
    hipStream_t st = (hipStream_t)stream;
    float* geo = static_cast<float*>(ws);
    xgs_status s;
    // the accumulated gradients and the geometry workspace start at zero (one
    // launch), unless the caller had xgs_render_bwd_zero do it beforehand
    if (!prezeroed && (s = zero_accumulated(g, geo_on, gr, geo, st))) return s;
    TileGrid tg = tile_grid(*cam, b->tile_order);
    if (geo_on) {
        dispatch_bwd<true>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
        if ((s = check_launch("xgs_render_bwd pixels"))) return s;
        const CamDevB c = cam_dev_b(*cam);
        hipLaunchKernelGGL(project_bwd_kernel, dim3((unsigned)((g->n + 255) / 256)), dim3(256), 0, st, g->n,
                           g->means, g->log_scales, reinterpret_cast<const float4*>(g->quats), p->radius,
                           reinterpret_cast<const float4*>(p->splat), geo, c, gr->means, gr->log_scales,
                           reinterpret_cast<float4*>(gr->quats));
        return check_launch("xgs_render_bwd projection");
    }
    dispatch_bwd<false>(g, p, b, tg, d_out, final_T, n_last, gr, geo, st);
    return check_launch("xgs_render_bwd features");
}

extern "C" xgs_status xgs_pose_grad(const xgs_gaussians* g, const xgs_projected* p, const xgs_camera* cam,
                                    const void* ws, size_t ws_bytes, float* d_pose, xgs_stream_t stream) {
    clear_error();
    if (!g || !p || !cam || !d_pose) return fail(XGS_ERR_INVALID_ARG, "xgs_pose_grad: null argument");
    if (xgs_status s = validate_camera(cam)) return s;
    if (!aligned(ws, 256)) return fail(XGS_ERR_INVALID_ARG, "xgs_pose_grad: workspace must be 256-byte aligned");
    if (!ws || ws_bytes < xgs_render_bwd_workspace(g->n))
        return fail(XGS_ERR_CAPACITY, "xgs_pose_grad: workspace too small");
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !p->splat || !p->radius))
        return fail(XGS_ERR_INVALID_ARG, "xgs_pose_grad: null Gaussian array");
    Carve cv(const_cast<void*>(ws));
    const float* geo = cv.take<float>((size_t)(g->n > 0 ? g->n : 1) * GW_STRIDE);
    float* partial = cv.take<float>(pose_blocks(g->n) * 6);
    hipStream_t st = (hipStream_t)stream;
    if (g->n == 0) return fill_f32(d_pose, 6, 0.f, st);
    const size_t nb = pose_blocks(g->n);
    hipLaunchKernelGGL(pose_grad_kernel, dim3((unsigned)nb), dim3(256), 0, st, g->n, g->means, g->log_scales,
                       reinterpret_cast<const float4*>(g->quats), p->radius,
                       reinterpret_cast<const float4*>(p->splat), geo, cam_dev_b(*cam), partial);
    hipLaunchKernelGGL(pose_total_kernel, dim3(1), dim3(256), 0, st, partial, (int64_t)nb, d_pose);
    return check_launch("xgs_pose_grad");
}
