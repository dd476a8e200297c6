/*
 * FP64 CPU oracle for the X-GS Perceiver hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the bench's CPU-baseline leg may load this file's library.  It shares no code,
 * header, table or constant generator with the HIP path and is written straight
 * from the equations, with plain scalar loops and no blocking.
 *
 * Paper passages followed (arXiv 2603.09632):
 *   - Gaussian parameterisation Sigma = R S S^T R^T       (App. A, eq. after "scaling matrix")
 *   - EWA splat Sigma' = J W Sigma W^T J^T                (App. A)
 *   - front-to-back alpha blending, Eq. (rendering) / Eq. (discrete_render)
 *   - feature and depth maps by substituting f_i / d_i for c_i (Sec. 3.1, App. B)
 *   - sampled grid (u,v) = (o_h + m s, o_w + n s), Eq. (sampled_loc)
 *   - nearest-codeword assignment a_n = argmin_l ||x_n - E_l||, Sec. 3.2.2
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - 0.3 I dilation of Sigma', alpha = min(0.99, o G), skip alpha < 1/255,
 *     stop before adding when T(1-alpha) < 1e-4, background 0;
 *   - near-plane cull z <= near; the Jacobian is evaluated at the point whose
 *     x/z, y/z are clamped to +-1.3 * (W/2)/fx, (H/2)/fy;
 *   - the splat extent is the axis-aligned box of the ellipse on which
 *     o G = 1/255, i.e. half-widths sqrt(2 ln(255 o) Sigma'_xx) and
 *     sqrt(2 ln(255 o) Sigma'_yy); o < 1/255 is culled;
 *   - sampled pixel (m,n) has its centre at (o_w + n s + 0.5, o_h + m s + 0.5);
 *   - tiles are 16 x 16 sampled pixels; the depth channel is camera z of the
 *     mean; the sort key is (tile, binary32 depth, index).
 *
 * Camera array layout (double[26]):
 *   0 W, 1 H, 2 fx, 3 fy, 4 cx, 5 cy, 6 near, 7 stride, 8 off_y, 9 off_x,
 *   10..25 world->camera 4x4 row-major.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TILE 16

static const double ALPHA_MAX = 0.99;
static const double ALPHA_MIN = 1.0 / 255.0;
static const double T_STOP = 1e-4;
static const double DILATION = 0.3;
static const double GUARD = 1.3;

typedef struct {
    int W, H, s, oy, ox, Ws, Hs, tx, ty;
    double fx, fy, cx, cy, near_;
    double Rv[3][3], tv[3];
} cam_t;

static void read_cam(const double* c, cam_t* k) {
    k->W = (int)c[0]; k->H = (int)c[1];
    k->fx = c[2]; k->fy = c[3]; k->cx = c[4]; k->cy = c[5]; k->near_ = c[6];
    k->s = (int)c[7]; k->oy = (int)c[8]; k->ox = (int)c[9];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) k->Rv[i][j] = c[10 + 4 * i + j];
        k->tv[i] = c[10 + 4 * i + 3];
    }
    k->Hs = (k->H + k->s - 1) / k->s;
    k->Ws = (k->W + k->s - 1) / k->s;
    k->tx = (k->Ws + ORC_TILE - 1) / ORC_TILE;
    k->ty = (k->Hs + ORC_TILE - 1) / ORC_TILE;
}

int orc_grid_info(const double* cam, int32_t* out4) {
    cam_t k; read_cam(cam, &k);
    out4[0] = k.Hs; out4[1] = k.Ws; out4[2] = k.ty; out4[3] = k.tx;
    return 0;
}

/* ---------------------------------------------------------------- rotation */
static void quat_to_rot(const double qh[4], double R[3][3]) {
    double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

/* All intermediate quantities of one Gaussian's projection. */
typedef struct {
    double qn, qh[4], R[3][3], s[3], M[3][3], Sig[3][3];
    double p[3], u, v, tx, ty; int clx, cly;
    double J[2][3], Sc[3][3], a, b, c, det;
    double mean2d[2], conic[3], depth, ext[2];
    int culled;
} proj_t;

static void project_one(const double* mu, const double* ls, const double* q, double o,
                        const cam_t* k, proj_t* P) {
    memset(P, 0, sizeof(*P));
    P->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) P->qh[i] = q[i] / P->qn;
    quat_to_rot(P->qh, P->R);
    for (int j = 0; j < 3; ++j) P->s[j] = exp(ls[j]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P->M[i][j] = P->R[i][j] * P->s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += P->M[i][m] * P->M[j][m];
            P->Sig[i][j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        P->p[i] = k->Rv[i][0] * mu[0] + k->Rv[i][1] * mu[1] + k->Rv[i][2] * mu[2] + k->tv[i];
    P->depth = P->p[2];
    if (!(P->p[2] > k->near_)) { P->culled = 1; return; }
    double z = P->p[2];
    P->u = P->p[0] / z; P->v = P->p[1] / z;
    double limx = GUARD * (0.5 * k->W) / k->fx, limy = GUARD * (0.5 * k->H) / k->fy;
    double uc = P->u, vc = P->v;
    P->clx = (uc < -limx) || (uc > limx);
    P->cly = (vc < -limy) || (vc > limy);
    if (uc < -limx) uc = -limx; if (uc > limx) uc = limx;
    if (vc < -limy) vc = -limy; if (vc > limy) vc = limy;
    P->tx = uc * z; P->ty = vc * z;
    P->J[0][0] = k->fx / z; P->J[0][1] = 0; P->J[0][2] = -k->fx * P->tx / (z * z);
    P->J[1][0] = 0; P->J[1][1] = k->fy / z; P->J[1][2] = -k->fy * P->ty / (z * z);
    /* Sigma_cam = Rv Sigma Rv^T */
    double tmp[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += k->Rv[i][m] * P->Sig[m][j];
            tmp[i][j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += tmp[i][m] * k->Rv[j][m];
            P->Sc[i][j] = acc;
        }
    /* T = J Sc J^T */
    double JS[2][3], T2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += P->J[i][m] * P->Sc[m][j];
            JS[i][j] = acc;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += JS[i][m] * P->J[j][m];
            T2[i][j] = acc;
        }
    P->a = T2[0][0] + DILATION; P->b = T2[0][1]; P->c = T2[1][1] + DILATION;
    P->det = P->a * P->c - P->b * P->b;
    if (!(P->det > 0)) { P->culled = 1; return; }
    P->conic[0] = P->c / P->det; P->conic[1] = -P->b / P->det; P->conic[2] = P->a / P->det;
    P->mean2d[0] = k->fx * P->u + k->cx;
    P->mean2d[1] = k->fy * P->v + k->cy;
    if (o < ALPHA_MIN) { P->culled = 1; return; }
    double tau = 2.0 * log(255.0 * o);
    P->ext[0] = sqrt(tau * P->a);
    P->ext[1] = sqrt(tau * P->c);
}

/* Sampled-pixel index range [lo, hi] whose centres o + n s + 0.5 lie within
 * [centre - ext, centre + ext]; returns 0 if empty. */
static int pixel_range(double centre, double ext, int off, int s, int n_max, int* lo, int* hi) {
    double flo = ceil((centre - ext - off - 0.5) / s);
    double fhi = floor((centre + ext - off - 0.5) / s);
    if (flo < 0) flo = 0;
    if (fhi > n_max - 1) fhi = n_max - 1;
    if (flo > fhi) return 0;
    *lo = (int)flo; *hi = (int)fhi;
    return 1;
}

/*
 * Projection of n Gaussians.  Outputs (all [n]-major, row per Gaussian):
 *   mean2d[2], conic[3] (A,B,C of A dx^2 + 2B dx dy + C dy^2), depth, cov2d[3]
 *   (a,b,c of Sigma' incl. dilation), ext[2], rect[4] = tiles [x0,x1) x [y0,y1),
 *   touched = (x1-x0)(y1-y0), visible (0 = culled).
 */
int orc_project(int64_t n, const double* means, const double* log_scales, const double* quats,
                const double* opac, const double* cam, double* mean2d, double* conic,
                double* depth, double* cov2d, double* ext, int32_t* rect, int64_t* touched,
                int32_t* visible) {
    cam_t k; read_cam(cam, &k);
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opac[i], &k, &P);
        depth[i] = P.depth;
        mean2d[2 * i] = P.mean2d[0]; mean2d[2 * i + 1] = P.mean2d[1];
        for (int j = 0; j < 3; ++j) conic[3 * i + j] = P.conic[j];
        cov2d[3 * i] = P.a; cov2d[3 * i + 1] = P.b; cov2d[3 * i + 2] = P.c;
        ext[2 * i] = P.ext[0]; ext[2 * i + 1] = P.ext[1];
        int nlo, nhi, mlo, mhi;
        int ok = !P.culled &&
                 pixel_range(P.mean2d[0], P.ext[0], k.ox, k.s, k.Ws, &nlo, &nhi) &&
                 pixel_range(P.mean2d[1], P.ext[1], k.oy, k.s, k.Hs, &mlo, &mhi);
        if (!ok) {
            rect[4 * i] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = 0;
            touched[i] = 0; visible[i] = 0;
            continue;
        }
        rect[4 * i + 0] = nlo / ORC_TILE; rect[4 * i + 2] = nhi / ORC_TILE + 1;
        rect[4 * i + 1] = mlo / ORC_TILE; rect[4 * i + 3] = mhi / ORC_TILE + 1;
        touched[i] = (int64_t)(rect[4 * i + 2] - rect[4 * i + 0]) * (rect[4 * i + 3] - rect[4 * i + 1]);
        visible[i] = 1;
    }
    return 0;
}

/* ----------------------------------------------------------------- binning */
typedef struct { uint64_t key; uint32_t idx; } inst_t;

static int inst_cmp(const void* pa, const void* pb) {
    const inst_t* a = (const inst_t*)pa; const inst_t* b = (const inst_t*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/*
 * Every (tile, Gaussian) instance of the rectangles, keyed (tile << 32) | depth
 * bits, sorted by (key, index).  ranges[2t], ranges[2t+1] = [first, last+1) of
 * tile t in the sorted list, (0,0) if empty.  Returns the instance count, or -1
 * if it exceeds max_inst.
 */
int64_t orc_bin(int64_t n, const int32_t* rect, const uint32_t* depth_bits, int32_t tiles_x,
                int32_t tiles_y, int64_t max_inst, uint64_t* keys, uint32_t* vals, uint32_t* ranges) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        m += (int64_t)(rect[4 * i + 2] - rect[4 * i]) * (rect[4 * i + 3] - rect[4 * i + 1]);
    if (m > max_inst) return -1;
    inst_t* L = (inst_t*)malloc(sizeof(inst_t) * (m > 0 ? m : 1));
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int y = rect[4 * i + 1]; y < rect[4 * i + 3]; ++y)
            for (int x = rect[4 * i]; x < rect[4 * i + 2]; ++x) {
                uint64_t tile = (uint64_t)y * tiles_x + x;
                L[w].key = (tile << 32) | depth_bits[i];
                L[w].idx = (uint32_t)i;
                ++w;
            }
    qsort(L, (size_t)m, sizeof(inst_t), inst_cmp);
    int64_t T = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t < 2 * T; ++t) ranges[t] = 0;
    for (int64_t j = 0; j < m; ++j) {
        keys[j] = L[j].key; vals[j] = L[j].idx;
        uint64_t t = L[j].key >> 32;
        if (j == 0 || (L[j - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)j;
        ranges[2 * t + 1] = (uint32_t)(j + 1);
    }
    free(L);
    return m;
}

/* -------------------------------------------------------------- compositing */
/*
 * One pixel's front-to-back walk over the Gaussians list[0..len).  Channels of
 * Gaussian i are chan[i*C .. i*C+C).  Writes out[C] and returns T; *n_last is
 * the list position after the last Gaussian blended.  The three ambiguity
 * measures are minima over the walk of |255 o G - 1| (skip decision),
 * |T'/1e-4 - 1| (stop decision) and the relative depth gap between consecutive
 * blended Gaussians.  amb[3] is a signature of the blended sequence,
 * sum over blended Gaussians of (index + 1) * (ordinal + 1), exact in double;
 * it changes whenever a skip, stop or ordering decision changes.
 */
static double walk_pixel(double px, double py, const uint32_t* list, int64_t len,
                         const double* mean2d, const double* conic, const double* opac,
                         const double* chan, const double* depth, int C, double* out,
                         int64_t* n_last, double* amb) {
    double T = 1.0;
    for (int c = 0; c < C; ++c) out[c] = 0.0;
    *n_last = 0;
    double a_skip = INFINITY, a_stop = INFINITY, a_depth = INFINITY, prev_z = NAN, sig = 0.0;
    double ordinal = 0.0;
    for (int64_t j = 0; j < len; ++j) {
        uint32_t i = list[j];
        double dx = px - mean2d[2 * i], dy = py - mean2d[2 * i + 1];
        double A = conic[3 * i], B = conic[3 * i + 1], Cc = conic[3 * i + 2];
        double q = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
        double G = exp(-0.5 * q);
        double oG = opac[i] * G;
        double r = fabs(255.0 * oG - 1.0);
        if (r < a_skip) a_skip = r;
        double alpha = oG < ALPHA_MAX ? oG : ALPHA_MAX;
        if (alpha < ALPHA_MIN) continue;
        double Tn = T * (1.0 - alpha);
        double rs = fabs(Tn / T_STOP - 1.0);
        if (rs < a_stop) a_stop = rs;
        if (Tn < T_STOP) break;
        double w = alpha * T;
        for (int c = 0; c < C; ++c) out[c] += w * chan[(int64_t)i * C + c];
        if (depth) {
            if (!isnan(prev_z)) {
                double g = fabs(depth[i] - prev_z) / fmax(fabs(depth[i]), 1e-30);
                if (g < a_depth) a_depth = g;
            }
            prev_z = depth[i];
        }
        T = Tn;
        *n_last = j + 1;
        ordinal += 1.0;
        sig += ((double)i + 1.0) * ordinal;
    }
    if (amb) { amb[0] = a_skip; amb[1] = a_stop; amb[2] = a_depth; amb[3] = sig; }
    return T;
}

/*
 * Tiled forward composite over the sampled grid.  order/ranges come from
 * orc_bin.  Outputs out[C][Hs][Ws], final_T[Hs][Ws], n_last[Hs][Ws] (position
 * within the tile list), amb[4][Hs][Ws] (see walk_pixel).  tile_mask (optional, [T]) restricts
 * the work to tiles with a nonzero entry; other pixels are left untouched.
 */
int orc_composite_fwd(int64_t n, const double* mean2d, const double* conic, const double* opac,
                      const double* chan, const double* depth, int32_t C, const uint32_t* order,
                      const uint32_t* ranges, const double* cam, const uint8_t* tile_mask,
                      double* out, double* final_T, int64_t* n_last, double* amb) {
    (void)n;
    cam_t k; read_cam(cam, &k);
    int64_t HW = (int64_t)k.Hs * k.Ws;
    /* pixels are independent: rows of the grid may run on several threads */
#pragma omp parallel
    {
        double* acc = (double*)malloc(sizeof(double) * (C > 0 ? C : 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < k.Hs; ++m)
            for (int nn = 0; nn < k.Ws; ++nn) {
                int t = (m / ORC_TILE) * k.tx + nn / ORC_TILE;
                if (tile_mask && !tile_mask[t]) continue;
                double px = k.ox + (double)nn * k.s + 0.5, py = k.oy + (double)m * k.s + 0.5;
                uint32_t b = ranges[2 * t], e = ranges[2 * t + 1];
                double a3[4]; int64_t nl;
                double T = walk_pixel(px, py, order + b, (int64_t)e - b, mean2d, conic, opac, chan,
                                      depth, C, acc, &nl, a3);
                int64_t pix = (int64_t)m * k.Ws + nn;
                for (int c = 0; c < C; ++c) out[c * HW + pix] = acc[c];
                final_T[pix] = T; n_last[pix] = nl;
                if (amb) for (int j = 0; j < 4; ++j) amb[j * HW + pix] = a3[j];
            }
        free(acc);
    }
    return 0;
}

/*
 * Same walk as orc_composite_fwd for a list of tiles only, written compactly:
 * out[k][C][16][16], final_T[k][16][16], amb[k][4][16][16] (the measures of
 * walk_pixel) for tile k = tiles[k]; pixels past the grid edge are left 0.
 */
int orc_composite_tiles(const double* mean2d, const double* conic, const double* opac,
                        const double* chan, const double* depth, int32_t C, const uint32_t* order,
                        const uint32_t* ranges, const double* cam, const int32_t* tiles, int32_t nt,
                        double* out, double* final_T, double* amb) {
    cam_t k; read_cam(cam, &k);
#pragma omp parallel
    {
        double* acc = (double*)malloc(sizeof(double) * (C > 0 ? C : 1));
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < nt; ++q) {
            int t = tiles[q];
            int ty = t / k.tx, tx = t % k.tx;
            uint32_t b = ranges[2 * t], e = ranges[2 * t + 1];
            for (int r = 0; r < ORC_TILE; ++r)
                for (int c = 0; c < ORC_TILE; ++c) {
                    int m = ty * ORC_TILE + r, nn = tx * ORC_TILE + c;
                    if (m >= k.Hs || nn >= k.Ws) continue;
                    double px = k.ox + (double)nn * k.s + 0.5, py = k.oy + (double)m * k.s + 0.5;
                    double a4[4]; int64_t nl;
                    double T = walk_pixel(px, py, order + b, (int64_t)e - b, mean2d, conic, opac, chan,
                                          depth, C, acc, &nl, a4);
                    int64_t p = (int64_t)r * ORC_TILE + c;
                    for (int ch = 0; ch < C; ++ch) out[((int64_t)q * C + ch) * 256 + p] = acc[ch];
                    final_T[(int64_t)q * 256 + p] = T;
                    for (int j = 0; j < 4; ++j) amb[((int64_t)q * 4 + j) * 256 + p] = a4[j];
                }
        }
        free(acc);
    }
    return 0;
}

/*
 * Brute-force composite: every pixel walks the same global list (all visible
 * Gaussians in (depth, index) order), no tiles.  Same outputs as above.
 */
int orc_composite_list(const double* mean2d, const double* conic, const double* opac,
                       const double* chan, int32_t C, const uint32_t* list, int64_t len,
                       const double* cam, double* out, double* final_T) {
    cam_t k; read_cam(cam, &k);
    int64_t HW = (int64_t)k.Hs * k.Ws;
    double* acc = (double*)malloc(sizeof(double) * C);
    for (int m = 0; m < k.Hs; ++m)
        for (int nn = 0; nn < k.Ws; ++nn) {
            double px = k.ox + (double)nn * k.s + 0.5, py = k.oy + (double)m * k.s + 0.5;
            int64_t nl;
            double T = walk_pixel(px, py, list, len, mean2d, conic, opac, chan, NULL, C, acc, &nl, NULL);
            int64_t pix = (int64_t)m * k.Ws + nn;
            for (int c = 0; c < C; ++c) out[c * HW + pix] = acc[c];
            final_T[pix] = T;
        }
    free(acc);
    return 0;
}

/*
 * Analytic gradient of L = sum_x sum_c g[c][x] out[c][x] with respect to the
 * 2D splat parameters and channels.  Per pixel the forward walk is repeated,
 * recording each blended Gaussian's alpha, T and G; then, from the back,
 *   dL/dalpha_k = T_k (g . chan_k) - S_k / (1 - alpha_k),
 *   S_k = sum_{j>k} alpha_j T_j (g . chan_j),
 * which is the derivative of Eq. (rendering) with T_k = prod_{j<k}(1-alpha_j).
 * The chain continues through alpha = min(0.99, o G) (no gradient when
 * clamped), G = exp(-q/2), q = A dx^2 + 2B dx dy + C dy^2 and dx = px - mean.
 * Outputs are accumulated (+=) into d_mean2d[n][2], d_conic[n][3] (A,B,C),
 * d_opac[n], d_chan[n][C].  Skipped and terminated pairs contribute nothing.
 */
int orc_composite_bwd(int64_t n, const double* mean2d, const double* conic, const double* opac,
                      const double* chan, int32_t C, const uint32_t* order, const uint32_t* ranges,
                      const double* cam, const double* g, const uint8_t* tile_mask,
                      double* d_mean2d, double* d_conic, double* d_opac, double* d_chan) {
    (void)n;
    cam_t k; read_cam(cam, &k);
    int64_t HW = (int64_t)k.Hs * k.Ws;
    int64_t cap = 0;
    for (int64_t t = 0; t < (int64_t)k.tx * k.ty; ++t) {
        int64_t l = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
        if (l > cap) cap = l;
    }
    if (cap == 0) return 0;
    /* pixels are independent; rows of the grid may run on several threads,
       each accumulating into the per-Gaussian sums with atomic adds */
#pragma omp parallel
    {
        uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
        double* al = (double*)malloc(sizeof(double) * cap);
        double* Ts = (double*)malloc(sizeof(double) * cap);
        double* Gs = (double*)malloc(sizeof(double) * cap);
        double* gx = (double*)malloc(sizeof(double) * (C > 0 ? C : 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < k.Hs; ++m)
            for (int nn = 0; nn < k.Ws; ++nn) {
                int t = (m / ORC_TILE) * k.tx + nn / ORC_TILE;
                if (tile_mask && !tile_mask[t]) continue;
                double px = k.ox + (double)nn * k.s + 0.5, py = k.oy + (double)m * k.s + 0.5;
                int64_t pix = (int64_t)m * k.Ws + nn;
                for (int c = 0; c < C; ++c) gx[c] = g[c * HW + pix];
                /* forward walk, recording the blended Gaussians */
                uint32_t b = ranges[2 * t], e = ranges[2 * t + 1];
                double T = 1.0; int64_t cnt = 0;
                for (uint32_t j = b; j < e; ++j) {
                    uint32_t i = order[j];
                    double dx = px - mean2d[2 * i], dy = py - mean2d[2 * i + 1];
                    double q = conic[3 * i] * dx * dx + 2.0 * conic[3 * i + 1] * dx * dy +
                               conic[3 * i + 2] * dy * dy;
                    double G = exp(-0.5 * q);
                    double oG = opac[i] * G;
                    double alpha = oG < ALPHA_MAX ? oG : ALPHA_MAX;
                    if (alpha < ALPHA_MIN) continue;
                    double Tn = T * (1.0 - alpha);
                    if (Tn < T_STOP) break;
                    ids[cnt] = i; al[cnt] = alpha; Ts[cnt] = T; Gs[cnt] = G; ++cnt;
                    T = Tn;
                }
                /* backward over the recorded list */
                double S = 0.0;
                for (int64_t r = cnt - 1; r >= 0; --r) {
                    uint32_t i = ids[r];
                    double alpha = al[r], Ti = Ts[r], G = Gs[r];
                    double s = 0.0;
                    for (int c = 0; c < C; ++c) s += gx[c] * chan[(int64_t)i * C + c];
                    double dalpha = Ti * s - S / (1.0 - alpha);
                    S += alpha * Ti * s;
                    double w = alpha * Ti;
                    for (int c = 0; c < C; ++c) {
#pragma omp atomic
                        d_chan[(int64_t)i * C + c] += w * gx[c];
                    }
                    if (opac[i] * G < ALPHA_MAX) {
                        double dx = px - mean2d[2 * i], dy = py - mean2d[2 * i + 1];
                        double A = conic[3 * i], B = conic[3 * i + 1], Cc = conic[3 * i + 2];
                        double dq = dalpha * opac[i] * G * (-0.5); /* dL/dq */
#pragma omp atomic
                        d_opac[i] += dalpha * G;
#pragma omp atomic
                        d_conic[3 * i] += dq * dx * dx;
#pragma omp atomic
                        d_conic[3 * i + 1] += dq * 2.0 * dx * dy;
#pragma omp atomic
                        d_conic[3 * i + 2] += dq * dy * dy;
                        /* dq/dmean_x = -2 (A dx + B dy) */
#pragma omp atomic
                        d_mean2d[2 * i] += dq * (-2.0) * (A * dx + B * dy);
#pragma omp atomic
                        d_mean2d[2 * i + 1] += dq * (-2.0) * (B * dx + Cc * dy);
                    }
                }
            }
        free(ids); free(al); free(Ts); free(Gs); free(gx);
    }
    return 0;
}

/*
 * Chain rule from the splat gradients (d_mean2d, d_conic, d_depth) to the 3D
 * parameters, written out from the forward formulas of project_one:
 * conic = Sigma'^{-1}, Sigma' = J Sigma_cam J^T + 0.3 I, Sigma_cam = Rv Sigma Rv^T,
 * Sigma = (R S)(R S)^T, R = R(q/|q|), S = diag(exp l), p = Rv mu + t,
 * mean2d = f p_xy / p_z + c, depth = p_z.  The clamp of x/z, y/z in J is
 * differentiated as the piecewise function it is.  Culled Gaussians get 0.
 */
/* Adjoint of one Gaussian's projection down to the camera frame: from
 * dL/dmean2d, dL/dconic and dL/ddepth to dL/dp (camera-space mean, through
 * mean2d, J and the depth channel; clamped guard components pass nothing) and
 * dL/dSigma_cam (symmetric). */
static void adjoint_cam(const cam_t* k, const proj_t* P, const double* gcon, double gmx, double gmy,
                        double gdepth, double dp[3], double dSc[3][3]) {
    double z = P->p[2];
    /* conic -> Sigma' : dS = -K Ghat K with Ghat = [[gA, gB/2],[gB/2, gC]] */
    double K[2][2] = {{P->conic[0], P->conic[1]}, {P->conic[1], P->conic[2]}};
    double Gh[2][2] = {{gcon[0], 0.5 * gcon[1]}, {0.5 * gcon[1], gcon[2]}};
    double KG[2][2], dS[2][2];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) KG[r][c] = K[r][0] * Gh[0][c] + K[r][1] * Gh[1][c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) dS[r][c] = -(KG[r][0] * K[0][c] + KG[r][1] * K[1][c]);
    /* Sigma' = J Sc J^T (+0.3 I): dSc = J^T dS J ; dJ = 2 dS J Sc */
    double dJ[2][3], JSc[2][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc += P->J[a][r] * dS[a][b] * P->J[b][c];
            dSc[r][c] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += P->J[r][m] * P->Sc[m][c];
            JSc[r][c] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) dJ[r][c] = 2.0 * (dS[r][0] * JSc[0][c] + dS[r][1] * JSc[1][c]);
    /* J(p), mean2d(p), depth(p) -> p */
    dp[0] = dp[1] = dp[2] = 0;
    double dtx_dpx = P->clx ? 0.0 : 1.0, dtx_dpz = P->clx ? P->tx / z : 0.0;
    double dty_dpy = P->cly ? 0.0 : 1.0, dty_dpz = P->cly ? P->ty / z : 0.0;
    dp[2] += dJ[0][0] * (-k->fx / (z * z)) + dJ[1][1] * (-k->fy / (z * z));
    dp[0] += dJ[0][2] * (-k->fx / (z * z)) * dtx_dpx;
    dp[2] += dJ[0][2] * (-k->fx / (z * z) * dtx_dpz + 2.0 * k->fx * P->tx / (z * z * z));
    dp[1] += dJ[1][2] * (-k->fy / (z * z)) * dty_dpy;
    dp[2] += dJ[1][2] * (-k->fy / (z * z) * dty_dpz + 2.0 * k->fy * P->ty / (z * z * z));
    dp[0] += gmx * k->fx / z;
    dp[2] += -gmx * k->fx * P->p[0] / (z * z);
    dp[1] += gmy * k->fy / z;
    dp[2] += -gmy * k->fy * P->p[1] / (z * z);
    dp[2] += gdepth;
}

int orc_project_bwd(int64_t n, const double* means, const double* log_scales, const double* quats,
                    const double* opac, const double* cam, const double* d_mean2d,
                    const double* d_conic, const double* d_depth, double* d_means,
                    double* d_log_scales, double* d_quats) {
    cam_t k; read_cam(cam, &k);
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opac[i], &k, &P);
        for (int j = 0; j < 3; ++j) { d_means[3 * i + j] = 0; d_log_scales[3 * i + j] = 0; }
        for (int j = 0; j < 4; ++j) d_quats[4 * i + j] = 0;
        if (P.culled) continue;
        double dp[3], dSc[3][3];
        adjoint_cam(&k, &P, d_conic + 3 * i, d_mean2d[2 * i], d_mean2d[2 * i + 1], d_depth[i], dp, dSc);
        /* Sc = Rv Sig Rv^T : dSig = Rv^T dSc Rv */
        double dSig[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) acc += k.Rv[a][r] * dSc[a][b] * k.Rv[b][c];
                dSig[r][c] = acc;
            }
        /* Sig = M M^T : dM = 2 dSig M ; M = R diag(s) */
        double dM[3][3], dR[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += dSig[r][m] * P.M[m][c];
                dM[r][c] = 2.0 * acc;
            }
        for (int j = 0; j < 3; ++j) {
            double ds = 0;
            for (int r = 0; r < 3; ++r) { ds += dM[r][j] * P.R[r][j]; dR[r][j] = dM[r][j] * P.s[j]; }
            d_log_scales[3 * i + j] = ds * P.s[j];
        }
        /* R(qh) -> qh */
        double w = P.qh[0], x = P.qh[1], y = P.qh[2], zq = P.qh[3];
        double gq[4];
        gq[0] = 2 * (-zq * dR[0][1] + y * dR[0][2] + zq * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
        gq[1] = 2 * (y * dR[0][1] + zq * dR[0][2] + y * dR[1][0] - 2 * x * dR[1][1] - w * dR[1][2] +
                     zq * dR[2][0] + w * dR[2][1] - 2 * x * dR[2][2]);
        gq[2] = 2 * (-2 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + zq * dR[1][2] -
                     w * dR[2][0] + zq * dR[2][1] - 2 * y * dR[2][2]);
        gq[3] = 2 * (-2 * zq * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2 * zq * dR[1][1] +
                     y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
        double dot = 0;
        for (int j = 0; j < 4; ++j) dot += P.qh[j] * gq[j];
        for (int j = 0; j < 4; ++j) d_quats[4 * i + j] = (gq[j] - P.qh[j] * dot) / P.qn;
        for (int j = 0; j < 3; ++j)
            d_means[3 * i + j] = k.Rv[0][j] * dp[0] + k.Rv[1][j] * dp[1] + k.Rv[2][j] * dp[2];
    }
    return 0;
}

/*
 * Gradient with respect to the camera pose (Eq. (tracking): the map is frozen
 * and the extrinsics are optimised).  The world-to-camera pose T is perturbed
 * on the left, T(xi) = exp(xi^) T with xi = (rho, phi), so to first order
 * p -> p + rho + phi x p and Sigma_cam -> Sigma_cam + phi^ Sigma_cam -
 * Sigma_cam phi^.  Summed over the Gaussians:
 *   dL/drho = sum_i dL/dp_i,
 *   dL/dphi = sum_i [ p_i x dL/dp_i + axial(Sc_i G_i - G_i Sc_i) ],
 * G_i = dL/dSigma_cam,i, axial(A) = (A_23 - A_32, A_31 - A_13, A_12 - A_21).
 * d_pose[6] = (dL/drho, dL/dphi).
 */
int orc_pose_grad(int64_t n, const double* means, const double* log_scales, const double* quats,
                  const double* opac, const double* cam, const double* d_mean2d, const double* d_conic,
                  const double* d_depth, double* d_pose) {
    cam_t k; read_cam(cam, &k);
    for (int j = 0; j < 6; ++j) d_pose[j] = 0;
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opac[i], &k, &P);
        if (P.culled) continue;
        double dp[3], G[3][3];
        adjoint_cam(&k, &P, d_conic + 3 * i, d_mean2d[2 * i], d_mean2d[2 * i + 1], d_depth[i], dp, G);
        double A[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += P.Sc[r][m] * G[m][c] - G[r][m] * P.Sc[m][c];
                A[r][c] = acc;
            }
        const double* p = P.p;
        d_pose[0] += dp[0]; d_pose[1] += dp[1]; d_pose[2] += dp[2];
        d_pose[3] += p[1] * dp[2] - p[2] * dp[1] + (A[1][2] - A[2][1]);
        d_pose[4] += p[2] * dp[0] - p[0] * dp[2] + (A[2][0] - A[0][2]);
        d_pose[5] += p[0] * dp[1] - p[1] * dp[0] + (A[0][1] - A[1][0]);
    }
    return 0;
}

/* ---------------------------------------------------------------------- VQ */
/*
 * a_n = argmin_l sum_d (x_nd - E_ld)^2 in FP64 from the binary32 inputs; ties
 * go to the lowest l.  dist[n] is the minimum squared distance and dist2[n] the
 * second smallest (used to recognise near-ties).  Rows are independent, so the
 * loop over n may run on several threads.
 */
int orc_vq_assign(int64_t N, int32_t D, const float* X, int32_t K, const float* E,
                  int32_t* idx, double* dist, double* dist2) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t nrow = 0; nrow < N; ++nrow) {
        const float* x = X + nrow * D;
        double best = INFINITY, second = INFINITY; int32_t bi = -1;
        for (int32_t l = 0; l < K; ++l) {
            const float* e = E + (int64_t)l * D;
            double acc = 0.0;
            for (int32_t d = 0; d < D; ++d) {
                double t = (double)x[d] - (double)e[d];
                acc += t * t;
            }
            if (acc < best) { second = best; best = acc; bi = l; }
            else if (acc < second) { second = acc; }
        }
        idx[nrow] = bi; dist[nrow] = best; dist2[nrow] = second;
    }
    return 0;
}

/*
 * Confidence of App. C, Eq. (confidence_score): p_nk = softmax_k(-|x_n - e_k| / tau)
 * with the unsquared distance; conf[n] = max_k p_nk = 1 / sum_j exp(-(d_j - d_min) / tau),
 * FP64 over every codeword (the shifted sum cannot overflow).
 */
int orc_vq_confidence(int64_t N, int32_t D, const float* X, int32_t K, const float* E, double tau,
                      double* conf) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t nrow = 0; nrow < N; ++nrow) {
        const float* x = X + nrow * D;
        double dmin = INFINITY;
        double* dist = (double*)malloc(sizeof(double) * (size_t)K);
        for (int32_t l = 0; l < K; ++l) {
            const float* e = E + (int64_t)l * D;
            double acc = 0.0;
            for (int32_t d = 0; d < D; ++d) {
                double t = (double)x[d] - (double)e[d];
                acc += t * t;
            }
            dist[l] = sqrt(acc);
            if (dist[l] < dmin) dmin = dist[l];
        }
        double s = 0.0;
        for (int32_t l = 0; l < K; ++l) s += exp(-(dist[l] - dmin) / tau);
        conf[nrow] = 1.0 / s;
        free(dist);
    }
    return 0;
}

/* Threads used by the parallel loops above (rows of the grid, rows of X);
   returns the count now in effect. */
int orc_set_threads(int32_t n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
