// Status strings, the thread-local error text and camera validation.
#include "common.h"
#include "render_common.h"

namespace xgs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

xgs_status validate_camera(const xgs_camera* c) {
    if (!c) return fail(XGS_ERR_INVALID_ARG, "camera: null");
    if (c->width < 1 || c->height < 1) return fail(XGS_ERR_INVALID_ARG, "camera: width and height must be positive");
    if (!(c->fx > 0.f) || !(c->fy > 0.f)) return fail(XGS_ERR_INVALID_ARG, "camera: focal lengths must be positive");
    if (c->stride < 1) return fail(XGS_ERR_INVALID_ARG, "camera: stride must be >= 1");
    if (c->off_y < 0 || c->off_x < 0 || c->off_y >= c->stride || c->off_x >= c->stride)
        return fail(XGS_ERR_INVALID_ARG, "camera: grid offsets must lie in [0, stride)");
    if (!(c->near_plane > 0.f)) return fail(XGS_ERR_INVALID_ARG, "camera: near_plane must be positive");
    Grid g = grid_of(*c);
    if ((int64_t)g.tx * g.ty >= (int64_t(1) << 31))
        return fail(XGS_ERR_UNSUPPORTED, "camera: too many tiles");
    return XGS_OK;
}

}  // namespace xgs

using namespace xgs;

extern "C" const char* xgs_status_string(xgs_status s) {
    switch (s) {
        case XGS_OK: return "ok";
        case XGS_ERR_INVALID_ARG: return "invalid argument";
        case XGS_ERR_CAPACITY: return "buffer or workspace too small";
        case XGS_ERR_HIP: return "HIP runtime error";
        case XGS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* xgs_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t xgs_version(void) { return 1; }

extern "C" xgs_status xgs_grid_dims(const xgs_camera* cam, int32_t* hs, int32_t* ws, int32_t* tiles_y,
                                    int32_t* tiles_x) {
    clear_error();
    if (xgs_status s = validate_camera(cam)) return s;
    Grid g = grid_of(*cam);
    if (hs) *hs = g.hs;
    if (ws) *ws = g.ws;
    if (tiles_y) *tiles_y = g.ty;
    if (tiles_x) *tiles_x = g.tx;
    return XGS_OK;
}
