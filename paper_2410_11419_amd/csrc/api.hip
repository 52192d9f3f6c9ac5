// Host side of the C-ABI (include/gs3.h): argument checks, workspace
// layout, view set-up in double precision, kernel launch order.
#include <vector>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "gs3_internal.h"

namespace gs3 {

static thread_local std::string g_last_error;

static int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int set_error(int status, const char* msg) { return fail(status, "%s", msg); }

static int hip_fail(hipError_t e, const char* where) {
    return fail(GS3_HIP_ERROR, "%s: %s", where, hipGetErrorString(e));
}

#define GS3_CHECK_HIP(expr)                                  \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(_e, #expr);    \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool make_layout(int64_t n, int32_t width, int32_t height, int64_t capacity, Layout* L) {
    if (n < 0 || n >= (int64_t(1) << 31) || width <= 0 || height <= 0 || width > 16384 || height > 16384 ||
        capacity < 0 || capacity >= (int64_t(1) << 31))
        return false;
    Layout l;
    l.n = n;
    l.width = width;
    l.height = height;
    l.tiles_x = (width + kTile - 1) / kTile;
    l.tiles_y = (height + kTile - 1) / kTile;
    l.n_tiles = (int64_t)l.tiles_x * l.tiles_y;
    {
        const int64_t groups = (int64_t)((l.tiles_x + kGroupTiles - 1) / kGroupTiles) *
                               ((l.tiles_y + kGroupTiles - 1) / kGroupTiles);
        l.n_slots = groups <= kMaxGroups ? 8 * ((groups + 7) / 8) * kGroupTiles * kGroupTiles : l.n_tiles;
        if (l.n_slots < l.n_tiles) l.n_slots = l.n_tiles;
    }
    l.capacity = capacity;
    l.nblk_n = (n + kSortItemsN - 1) / kSortItemsN;
    l.nblk_p = (capacity + kSortItems - 1) / kSortItems;
    const int64_t nblk = l.nblk_n > l.nblk_p ? l.nblk_n : l.nblk_p;
    l.table_len = nblk * kRadixBins;
    const int64_t longest = l.table_len > n + 1 ? l.table_len : n + 1;
    l.scan_sums = (longest + kSortItems - 1) / kSortItems + 1;
    if (l.scan_sums < kRadixBins) l.scan_sums = kRadixBins;   // also the radix passes' digit totals
    if (l.scan_sums < (n + 255) / 256) l.scan_sums = (n + 255) / 256;   // 256-splat count sums
    {
        int tile_bits = 0, id_bits = 1;
        while ((int64_t(1) << tile_bits) < l.n_tiles) ++tile_bits;
        while ((int64_t(1) << id_bits) < n) ++id_bits;
        l.id_bits = tile_bits + id_bits <= 32 ? id_bits : 0;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.hdr = take(sizeof(ViewHeader));
    l.rec0 = take(sizeof(float4) * n);
    l.rec1 = take(sizeof(float4) * n);
    l.rec2 = take(sizeof(float4) * n);
    l.depth = take(sizeof(float) * n);
    l.ext = take(sizeof(int4) * n);
    l.drec = take(sizeof(int4) * n);
    l.cnt = take(sizeof(uint32_t) * n);
    l.num = take(sizeof(unsigned long long) * n);
    l.col0 = take(sizeof(float4) * n);
    l.col1 = take(sizeof(float4) * n);
    l.keys_a = take(sizeof(uint32_t) * n);
    l.vals_a = take(sizeof(uint32_t) * n);
    l.keys_b = take(sizeof(uint32_t) * n);
    l.vals_b = take(sizeof(uint32_t) * n);
    l.offs = take(sizeof(uint32_t) * (n + 1));
    l.pk_a = take(sizeof(uint32_t) * capacity);
    l.pv_a = take(sizeof(uint32_t) * capacity);
    l.pk_b = take(sizeof(uint32_t) * capacity);
    l.pv_b = take(sizeof(uint32_t) * capacity);
    l.table = take(sizeof(uint32_t) * l.table_len);
    l.sums = take(sizeof(uint32_t) * l.scan_sums);
    l.ranges = take(sizeof(int2) * l.n_tiles);
    l.order = take(sizeof(uint32_t) * l.n_slots);
    l.total = off;
    *L = l;
    return true;
}

static int check_vb(const gs3_viewbuf* vb, Layout* L) {
    if (!vb) return fail(GS3_INVALID_ARG, "viewbuf is NULL");
    if (!make_layout(vb->n, vb->width, vb->height, vb->pair_capacity, L))
        return fail(GS3_INVALID_ARG, "invalid view buffer sizes (n=%lld, %dx%d, capacity=%lld)",
                    (long long)vb->n, vb->width, vb->height, (long long)vb->pair_capacity);
    if (!vb->ws) return fail(GS3_INVALID_ARG, "viewbuf.ws is NULL");
    if ((reinterpret_cast<uintptr_t>(vb->ws) & 255) != 0) return fail(GS3_INVALID_ARG, "viewbuf.ws not 256-byte aligned");
    if (vb->ws_bytes < L->total)
        return fail(GS3_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", vb->ws_bytes, L->total);
    return GS3_OK;
}

// Binning status block (gs3_viewbuf.status): the host-side generation in
// status[0], the device-written packed outcome in status[1].
constexpr int kGenBits = 24;
constexpr unsigned long long kGenMask = (1ull << kGenBits) - 1ull;

static void read_status(const gs3_viewbuf* vb, int32_t* state, int64_t* required) {
    const volatile int64_t* st = vb->status;
    const unsigned long long gen = (unsigned long long)st[0];
    const unsigned long long word = (unsigned long long)__atomic_load_n(&vb->status[1], __ATOMIC_ACQUIRE);
    if (gen == 0 || (word >> 40) != (gen & kGenMask)) {
        *state = GS3_VIEW_PENDING;
        *required = -1;
        return;
    }
    *required = (int64_t)(word & ((1ull << 39) - 1ull));
    *state = (word >> 39) & 1ull ? GS3_VIEW_OVERFLOW : GS3_VIEW_OK;
}

// Calls that read a workspace's lists: refuse, enqueueing nothing, once the
// latest binning is known (from the status block) to have overflowed.
static int check_lists(const gs3_viewbuf* vb) {
    if (!vb->status) return GS3_OK;
    int32_t state;
    int64_t req;
    read_status(vb, &state, &req);
    if (state == GS3_VIEW_OVERFLOW)
        return fail(GS3_PAIR_CAPACITY_EXCEEDED, "the last binning of this workspace needed %lld pairs, capacity is %lld",
                    (long long)req, (long long)vb->pair_capacity);
    return GS3_OK;
}

// A binning into `vb`: the device address of the status block (NULL when
// there is none), checked before anything is enqueued.
static int status_target(const gs3_viewbuf* vb, int64_t** dev) {
    *dev = nullptr;
    if (!vb->status) return GS3_OK;
    if ((reinterpret_cast<uintptr_t>(vb->status) & 7) != 0)
        return fail(GS3_INVALID_ARG, "viewbuf.status is not 8-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, vb->status) != hipSuccess || attr.devicePointer == nullptr) {
        (void)hipGetLastError();
        return fail(GS3_INVALID_ARG, "viewbuf.status is not host-pinned memory the device can write");
    }
    *dev = reinterpret_cast<int64_t*>(attr.devicePointer);
    return GS3_OK;
}

// Before a binning is enqueued: the next generation of the view's status
// block (word 0, written by the host) and where the binning reports it.
static StatusReq next_status(const gs3_viewbuf* vb, int64_t* dev) {
    volatile int64_t* gen = vb->status;
    const long long g = (long long)gen[0] + 1;
    gen[0] = g;
    return StatusReq{g, dev + 1};
}

static int check_consts(const gs3_consts* k) {
    if (!k) return fail(GS3_INVALID_ARG, "consts is NULL");
    if (!(k->near_plane > 0.f) || !(k->clamp_frac > 0.f) || !(k->dilation >= 0.f) || !(k->cutoff > 0.f) ||
        !(k->alpha_min >= 0.f) || !(k->alpha_max > 0.f) || !(k->alpha_max <= 1.f) || !(k->t_min >= 0.f) ||
        !(k->shadow_bias >= 0.f) || !std::isfinite(k->shadow_bias))
        return fail(GS3_INVALID_ARG, "invalid rasteriser constants");
    return GS3_OK;
}

static int check_scene(const gs3_scene* s, bool need_shading) {
    if (!s) return fail(GS3_INVALID_ARG, "scene is NULL");
    if (s->n < 0 || s->n >= (int64_t(1) << 31)) return fail(GS3_INVALID_ARG, "scene.n out of range");
    if (s->k < 0 || s->k > kMaxLobes) return fail(GS3_INVALID_ARG, "scene.k out of range (0..%d)", kMaxLobes);
    if (s->n == 0) return GS3_OK;
    if (!s->mean || !s->log_scale || !s->rot || !s->opacity_logit)
        return fail(GS3_INVALID_ARG, "scene geometry pointer is NULL");
    if (s->appearance != GS3_APPEARANCE_LOBES && s->appearance != GS3_APPEARANCE_BASIS)
        return fail(GS3_INVALID_ARG, "scene.appearance must be GS3_APPEARANCE_LOBES or GS3_APPEARANCE_BASIS");
    if (!need_shading) return GS3_OK;
    if (s->appearance == GS3_APPEARANCE_BASIS) {
        if (!s->shade_rot || !s->albedo || !s->spec_albedo || !s->latent ||
            (s->k > 0 && (!s->basis_weight || !s->basis_rot || !s->basis_log_sigma)))
            return fail(GS3_INVALID_ARG, "scene appearance pointer is NULL (basis appearance)");
        return GS3_OK;
    }
    if (!s->shade_rot || !s->albedo || !s->feat || (s->k > 0 && (!s->lobe_axis || !s->lobe_log_sharp || !s->lobe_amp)))
        return fail(GS3_INVALID_ARG, "scene appearance pointer is NULL");
    return GS3_OK;
}

static SceneDev scene_dev(const gs3_scene* s) {
    SceneDev d;
    d.mean = s->mean;
    d.log_scale = s->log_scale;
    d.rot = s->rot;
    d.opacity_logit = s->opacity_logit;
    d.shade_rot = s->shade_rot;
    d.albedo = s->albedo;
    d.lobe_axis = s->lobe_axis;
    d.lobe_log_sharp = s->lobe_log_sharp;
    d.lobe_amp = s->lobe_amp;
    d.feat = s->feat;
    d.n = (int32_t)s->n;
    d.k = s->k;
    d.appearance = s->appearance;
    d.spec_albedo = s->spec_albedo;
    d.basis_weight = s->basis_weight;
    d.latent = s->latent;
    d.basis_rot = s->basis_rot;
    d.basis_log_sigma = s->basis_log_sigma;
    return d;
}

// Pinhole view in double: world-to-camera rows (right, down, forward).
static int view_params(const gs3_view* v, const Layout& L, int depth_mode, ViewParams* vp) {
    if (!v) return fail(GS3_INVALID_ARG, "view is NULL");
    if (v->width != L.width || v->height != L.height)
        return fail(GS3_INVALID_ARG, "view size %dx%d does not match the view buffer %dx%d", v->width, v->height,
                    L.width, L.height);
    if (v->projection != GS3_PERSPECTIVE && v->projection != GS3_ORTHOGRAPHIC)
        return fail(GS3_INVALID_ARG, "bad projection");
    const bool ortho = v->projection == GS3_ORTHOGRAPHIC;
    if (ortho && !(v->ortho_width > 0.0 && std::isfinite(v->ortho_width)))
        return fail(GS3_INVALID_ARG, "ortho_width must be positive");
    if (!ortho && !(v->fov > 0.0 && v->fov < M_PI)) return fail(GS3_INVALID_ARG, "fov must be in (0, pi)");
    if (depth_mode != GS3_DEPTH_Z && depth_mode != GS3_DEPTH_DIST) return fail(GS3_INVALID_ARG, "bad depth_mode");
    double f[3] = {v->target[0] - v->eye[0], v->target[1] - v->eye[1], v->target[2] - v->eye[2]};
    const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fn > 0.0) || !std::isfinite(fn)) return fail(GS3_INVALID_ARG, "eye and target coincide");
    for (double& x : f) x /= fn;
    const double up[3] = {0.0, std::fabs(f[2]) <= 0.99 ? 0.0 : 1.0, std::fabs(f[2]) <= 0.99 ? 1.0 : 0.0};
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (double& x : r) x /= rn;
    const double d[3] = {f[1] * r[2] - f[2] * r[1], f[2] * r[0] - f[0] * r[2], f[0] * r[1] - f[1] * r[0]};
    for (int i = 0; i < 3; ++i) {
        vp->R[i] = r[i];
        vp->R[3 + i] = d[i];
        vp->R[6 + i] = f[i];
        vp->eye[i] = v->eye[i];
    }
    vp->ortho = ortho ? 1 : 0;
    vp->scale = ortho ? v->width / v->ortho_width : 0.0;
    vp->focal = ortho ? vp->scale : (v->width / 2.0) / std::tan(v->fov / 2.0);
    vp->cx = v->width / 2.0;
    vp->cy = v->height / 2.0;
    vp->width = L.width;
    vp->height = L.height;
    vp->tiles_x = L.tiles_x;
    vp->tiles_y = L.tiles_y;
    vp->depth_mode = depth_mode;
    return GS3_OK;
}

static int check_mlp(const gs3_mlp* m, int n_in, int n_out, const char* name) {
    if (!m) return GS3_OK;
    if (m->n_in != n_in || m->n_out != n_out)
        return fail(GS3_INVALID_ARG, "%s must take %d inputs and give %d outputs (got n_in=%d, n_out=%d)", name, n_in,
                    n_out, m->n_in, m->n_out);
    for (int i = 0; i < 4; ++i)
        if (!m->w[i] || !m->b[i]) return fail(GS3_INVALID_ARG, "%s weight pointer %d is NULL", name, i);
    return GS3_OK;
}

// Phi and Psi shapes of the scene's appearance model.
static int check_mlps(const gs3_scene* scene, const gs3_mlp* phi, const gs3_mlp* psi) {
    const bool basis = scene->appearance == GS3_APPEARANCE_BASIS;
    int st = check_mlp(phi, basis ? kPhiBasisIn : 17, 1, "phi");
    if (st != GS3_OK) return st;
    return check_mlp(psi, basis ? kPsiBasisIn : 22, 3, "psi");
}

static hipError_t shade_launch(const gs3_scene* scene, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                               const gs3_mlp* psi, const Layout& L, void* ws, float* colour, int parts,
                               hipStream_t st) {
    if (scene->appearance == GS3_APPEARANCE_BASIS)
        return launch_basis_shade(scene_dev(scene), sp, T, phi, psi, L, ws, colour, parts, st);
    return launch_shade_mlp(scene_dev(scene), sp, T, phi, psi, L, ws, colour, parts, st);
}

}  // namespace gs3

using namespace gs3;

extern "C" {

void gs3_consts_default(gs3_consts* out) {
    if (!out) return;
    out->near_plane = 0.2f;
    out->clamp_frac = 1.3f;
    out->dilation = 0.3f;
    out->cutoff = 4.5f;
    out->alpha_min = 1.0f / 255.0f;
    out->alpha_max = 0.99f;
    out->t_min = 1e-4f;
    out->shadow_bias = 0.015f;
}

const char* gs3_status_string(int status) {
    switch (status) {
        case GS3_OK: return "GS3_OK";
        case GS3_INVALID_ARG: return "GS3_INVALID_ARG";
        case GS3_WORKSPACE_TOO_SMALL: return "GS3_WORKSPACE_TOO_SMALL";
        case GS3_PAIR_CAPACITY_EXCEEDED: return "GS3_PAIR_CAPACITY_EXCEEDED";
        case GS3_HIP_ERROR: return "GS3_HIP_ERROR";
        case GS3_UNSUPPORTED: return "GS3_UNSUPPORTED";
        default: return "GS3_UNKNOWN_STATUS";
    }
}

const char* gs3_last_error(void) { return g_last_error.c_str(); }

int gs3_device_ok(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

int gs3_view_workspace_size(int64_t n, int32_t width, int32_t height, int64_t pair_capacity, size_t* bytes) {
    if (!bytes) return fail(GS3_INVALID_ARG, "bytes is NULL");
    Layout L;
    if (!make_layout(n, width, height, pair_capacity, &L))
        return fail(GS3_INVALID_ARG, "invalid sizes (n=%lld, %dx%d, capacity=%lld)", (long long)n, width, height,
                    (long long)pair_capacity);
    *bytes = L.total;
    return GS3_OK;
}

int gs3_project(const gs3_scene* scene, const gs3_view* view, const gs3_consts* consts, int32_t depth_mode,
                const gs3_viewbuf* vb, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    if ((st = check_scene(scene, false)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if (scene->n != vb->n) return fail(GS3_INVALID_ARG, "scene.n != viewbuf.n");
    ViewParams vp;
    if ((st = view_params(view, L, depth_mode, &vp)) != GS3_OK) return st;
    const double tx = (view->width / 2.0) / vp.focal, ty = (view->height / 2.0) / vp.focal;
    vp.lim_x = consts->clamp_frac * tx;
    vp.lim_y = consts->clamp_frac * ty;
    GS3_CHECK_HIP(launch_project(scene_dev(scene), vp, *consts, L, vb->ws, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_bin(const int32_t* ix, const int32_t* iy, const int32_t* rx, const int32_t* ry, const float* depth,
            const gs3_viewbuf* vb, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    if (L.n > 0 && (!ix || !iy || !rx || !ry || !depth)) return fail(GS3_INVALID_ARG, "extent/depth pointer is NULL");
    int64_t* sdev;
    if ((st = status_target(vb, &sdev)) != GS3_OK) return st;
    GS3_CHECK_HIP(launch_extent_keys(ix, iy, rx, ry, depth, L, vb->ws, (hipStream_t)stream));
    StatusReq r{};
    if (sdev) r = next_status(vb, sdev);
    GS3_CHECK_HIP(launch_bin(L, vb->ws, (hipStream_t)stream, sdev ? &r : nullptr));
    return GS3_OK;
}

int gs3_sort(const gs3_viewbuf* vb, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    int64_t* sdev;
    if ((st = status_target(vb, &sdev)) != GS3_OK) return st;
    StatusReq r{};
    if (sdev) r = next_status(vb, sdev);
    GS3_CHECK_HIP(launch_bin(L, vb->ws, (hipStream_t)stream, sdev ? &r : nullptr));
    return GS3_OK;
}

int gs3_preprocess(const gs3_scene* scene, const gs3_view* view, const gs3_consts* consts, int32_t depth_mode,
                   const gs3_viewbuf* vb, gs3_stream_t stream) {
    return gs3_preprocess_views(scene, view, &depth_mode, 1, consts, vb, stream);
}

int gs3_preprocess_views(const gs3_scene* scene, const gs3_view* views, const int32_t* depth_modes,
                         int32_t n_views, const gs3_consts* consts, const gs3_viewbuf* vbs, gs3_stream_t stream) {
    if (n_views < 1) return fail(GS3_INVALID_ARG, "n_views must be at least 1");
    if (!views || !depth_modes || !vbs) return fail(GS3_INVALID_ARG, "views, depth_modes or viewbufs is NULL");
    int st;
    if ((st = check_scene(scene, false)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    std::vector<Layout> L(n_views);
    std::vector<ViewParams> vp(n_views);
    std::vector<int64_t*> sdev(n_views);
    for (int v = 0; v < n_views; ++v) {
        const gs3_viewbuf* vb = &vbs[v];
        if ((st = check_vb(vb, &L[v])) != GS3_OK) return st;
        if (scene->n != vb->n) return fail(GS3_INVALID_ARG, "scene.n != viewbufs[%d].n", v);
        if ((st = view_params(&views[v], L[v], depth_modes[v], &vp[v])) != GS3_OK) return st;
        const double tx = (views[v].width / 2.0) / vp[v].focal, ty = (views[v].height / 2.0) / vp[v].focal;
        vp[v].lim_x = consts->clamp_frac * tx;
        vp[v].lim_y = consts->clamp_frac * ty;
        if ((st = status_target(vb, &sdev[v])) != GS3_OK) return st;
        // views of one call share a launch: their workspaces must not overlap
        const char* a0 = static_cast<const char*>(vb->ws);
        for (int u = 0; u < v; ++u) {
            const char* b0 = static_cast<const char*>(vbs[u].ws);
            if (a0 < b0 + L[u].total && b0 < a0 + L[v].total)
                return fail(GS3_INVALID_ARG, "viewbufs[%d] and viewbufs[%d] share workspace memory", u, v);
        }
    }
    std::vector<const Layout*> Lp(n_views);
    std::vector<void*> ws(n_views);
    for (int v = 0; v < n_views; ++v) {
        Lp[v] = &L[v];
        ws[v] = vbs[v].ws;
    }
    const hipStream_t s = (hipStream_t)stream;
    GS3_CHECK_HIP(launch_project_batch(scene_dev(scene), vp.data(), *consts, Lp.data(), ws.data(), n_views, s));
    std::vector<StatusReq> req(n_views);
    std::vector<const StatusReq*> reqp(n_views, nullptr);
    for (int v = 0; v < n_views; ++v) {
        if (!sdev[v]) continue;
        req[v] = next_status(&vbs[v], sdev[v]);
        reqp[v] = &req[v];
    }
    GS3_CHECK_HIP(launch_bin_batch(Lp.data(), ws.data(), n_views, s, reqp.data()));
    return GS3_OK;
}

int gs3_view_pair_count(const gs3_viewbuf* vb, int64_t* n_pairs, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    if (!n_pairs) return fail(GS3_INVALID_ARG, "n_pairs is NULL");
    ViewHeader h;
    GS3_CHECK_HIP(hipMemcpyAsync(&h, at<ViewHeader>(vb->ws, L.hdr), sizeof h, hipMemcpyDeviceToHost,
                                 (hipStream_t)stream));
    GS3_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream));
    *n_pairs = (int64_t)h.required_pairs;
    if (h.overflow)
        return fail(GS3_PAIR_CAPACITY_EXCEEDED, "binning needs %llu pairs, capacity is %lld", h.required_pairs,
                    (long long)L.capacity);
    return GS3_OK;
}

int gs3_view_poll(const gs3_viewbuf* vb, int32_t* state, int64_t* required_pairs) {
    if (!vb || !vb->status) return fail(GS3_INVALID_ARG, "viewbuf or its status block is NULL");
    if (!state || !required_pairs) return fail(GS3_INVALID_ARG, "state / required_pairs is NULL");
    read_status(vb, state, required_pairs);
    return GS3_OK;
}

int gs3_view_lists(const gs3_viewbuf* vb, int32_t* tile_start, int32_t* tile_end, int32_t* ids, uint64_t* keys,
                   gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    if ((st = check_lists(vb)) != GS3_OK) return st;
    GS3_CHECK_HIP(launch_export_lists(L, vb->ws, tile_start, tile_end, ids, keys, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_view_splats(const gs3_viewbuf* vb, float* mean2d, float* conic, float* opacity, float* depth, int32_t* extent,
                    gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    GS3_CHECK_HIP(launch_export_splats(L, vb->ws, mean2d, conic, opacity, depth, extent, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_view_count_hits(const gs3_consts* consts, const gs3_viewbuf* vb, int32_t stop_early, int64_t* hits,
                        gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(vb, &L)) != GS3_OK) return st;
    if ((st = check_lists(vb)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if (!hits) return fail(GS3_INVALID_ARG, "hits is NULL");
    if ((reinterpret_cast<uintptr_t>(hits) & 7) != 0) return fail(GS3_INVALID_ARG, "hits not 8-byte aligned");
    GS3_CHECK_HIP(launch_count_hits(*consts, L, vb->ws, stop_early ? 1 : 0,
                                    reinterpret_cast<unsigned long long*>(hits), (hipStream_t)stream));
    return GS3_OK;
}

int gs3_shadow_splat(const gs3_consts* consts, const gs3_viewbuf* light_vb, float* num_den, float* T,
                     gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(light_vb, &L)) != GS3_OK) return st;
    if ((st = check_lists(light_vb)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if (L.n > 0 && (!num_den || !T)) return fail(GS3_INVALID_ARG, "num_den / T is NULL");
    GS3_CHECK_HIP(launch_shadow(*consts, L, light_vb->ws, num_den, T, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_shadow_den(const gs3_consts* consts, const gs3_viewbuf* light_vb, float* num_den, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(light_vb, &L)) != GS3_OK) return st;
    if ((st = check_lists(light_vb)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if (L.n > 0 && !num_den) return fail(GS3_INVALID_ARG, "num_den is NULL");
    GS3_CHECK_HIP(launch_shadow_den(*consts, L, light_vb->ws, num_den, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_shadow_num(const gs3_consts* consts, const gs3_viewbuf* light_vb, float* num_den, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(light_vb, &L)) != GS3_OK) return st;
    if ((st = check_lists(light_vb)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if (L.n > 0 && !num_den) return fail(GS3_INVALID_ARG, "num_den is NULL");
    GS3_CHECK_HIP(launch_shadow_num(*consts, L, light_vb->ws, num_den, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_shadow_resolve(const gs3_viewbuf* light_vb, float* num_den, float* T, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = check_vb(light_vb, &L)) != GS3_OK) return st;
    if ((st = check_lists(light_vb)) != GS3_OK) return st;
    if (L.n > 0 && (!num_den || !T)) return fail(GS3_INVALID_ARG, "num_den / T is NULL");
    GS3_CHECK_HIP(launch_shadow_resolve(L, light_vb->ws, num_den, T, (hipStream_t)stream));
    return GS3_OK;
}

static int render_args(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light,
                       const gs3_consts* consts, const gs3_viewbuf* cam_vb, Layout* L) {
    int st;
    if ((st = check_vb(cam_vb, L)) != GS3_OK) return st;
    if ((st = check_lists(cam_vb)) != GS3_OK) return st;
    if ((st = check_scene(scene, true)) != GS3_OK) return st;
    if (consts && (st = check_consts(consts)) != GS3_OK) return st;
    if (scene->n != cam_vb->n) return fail(GS3_INVALID_ARG, "scene.n != viewbuf.n");
    if (!cam || cam->width != L->width || cam->height != L->height)
        return fail(GS3_INVALID_ARG, "camera view missing or its size differs from the view buffer");
    if (!light) return fail(GS3_INVALID_ARG, "light view is NULL");
    if (light->projection == GS3_ORTHOGRAPHIC) {
        const double d[3] = {light->eye[0] - light->target[0], light->eye[1] - light->target[1],
                             light->eye[2] - light->target[2]};
        if (!(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > 0.0)) return fail(GS3_INVALID_ARG, "light eye and target coincide");
    } else if (light->projection != GS3_PERSPECTIVE) {
        return fail(GS3_INVALID_ARG, "bad light projection");
    }
    return GS3_OK;
}

// The light of the shading: a point light at the eye of a perspective light
// view, or (orthographic light view) a directional light whose unit
// direction toward the light is stored instead (Sec. 4.5).
static void shade_light(const gs3_view* light, ShadeParams* sp) {
    if (light->projection == GS3_ORTHOGRAPHIC) {
        double d[3] = {light->eye[0] - light->target[0], light->eye[1] - light->target[1],
                       light->eye[2] - light->target[2]};
        const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int i = 0; i < 3; ++i) sp->light[i] = (float)(d[i] / dn);
        sp->light_dir = 1;
    } else {
        for (int i = 0; i < 3; ++i) sp->light[i] = (float)light->eye[i];
        sp->light_dir = 0;
    }
}

static ShadeParams shade_params(const gs3_view* cam, const gs3_view* light, const gs3_mlp* phi,
                                const gs3_mlp* psi) {
    ShadeParams sp;
    shade_light(light, &sp);
    for (int i = 0; i < 3; ++i) sp.eye[i] = (float)cam->eye[i];
    sp.use_phi = phi != nullptr;
    sp.use_psi = psi != nullptr;
    return sp;
}

int gs3_render(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light, const gs3_consts* consts,
               const float* T, const gs3_mlp* phi, const gs3_mlp* psi, const gs3_viewbuf* cam_vb,
               const gs3_images* out, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = render_args(scene, cam, light, consts, cam_vb, &L)) != GS3_OK) return st;
    if (!consts) return fail(GS3_INVALID_ARG, "consts is NULL");
    if (!out || !out->final_rgb || !out->shading || !out->shadow || !out->residual || !out->t_final ||
        !out->n_contrib || !out->colour)
        return fail(GS3_INVALID_ARG, "an output pointer is NULL");
    if (L.n > 0 && !T) return fail(GS3_INVALID_ARG, "T is NULL");
    if ((st = check_mlps(scene, phi, psi)) != GS3_OK) return st;
    const ShadeParams sp = shade_params(cam, light, phi, psi);
    hipStream_t s = (hipStream_t)stream;
    GS3_CHECK_HIP(shade_launch(scene, sp, T, phi, psi, L, cam_vb->ws, out->colour, 3, s));
    GS3_CHECK_HIP(launch_render(*consts, L, cam_vb->ws, *out, s));
    return GS3_OK;
}

int gs3_shade(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light, const gs3_mlp* psi,
              const gs3_viewbuf* cam_vb, float* colour, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = render_args(scene, cam, light, nullptr, cam_vb, &L)) != GS3_OK) return st;
    if (!colour) return fail(GS3_INVALID_ARG, "colour is NULL");
    if ((st = check_mlps(scene, nullptr, psi)) != GS3_OK) return st;
    const ShadeParams sp = shade_params(cam, light, nullptr, psi);
    GS3_CHECK_HIP(shade_launch(scene, sp, nullptr, nullptr, psi, L, cam_vb->ws, colour, 1, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_render_shaded(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light,
                      const gs3_consts* consts, const float* T, const gs3_mlp* phi, const gs3_viewbuf* cam_vb,
                      const gs3_images* out, gs3_stream_t stream) {
    Layout L;
    int st;
    if ((st = render_args(scene, cam, light, consts, cam_vb, &L)) != GS3_OK) return st;
    if (!consts) return fail(GS3_INVALID_ARG, "consts is NULL");
    if (!out || !out->final_rgb || !out->shading || !out->shadow || !out->residual || !out->t_final ||
        !out->n_contrib || !out->colour)
        return fail(GS3_INVALID_ARG, "an output pointer is NULL");
    if (L.n > 0 && !T) return fail(GS3_INVALID_ARG, "T is NULL");
    if ((st = check_mlps(scene, phi, nullptr)) != GS3_OK) return st;
    const ShadeParams sp = shade_params(cam, light, phi, nullptr);
    hipStream_t s = (hipStream_t)stream;
    GS3_CHECK_HIP(shade_launch(scene, sp, T, phi, nullptr, L, cam_vb->ws, out->colour, 2, s));
    GS3_CHECK_HIP(launch_render(*consts, L, cam_vb->ws, *out, s));
    return GS3_OK;
}

// Views of one batched call: each workspace valid, with lists that are not
// from an overflowed binning, and no two sharing memory.
static int check_batch_vbs(const gs3_viewbuf* vbs, int32_t n_views, std::vector<Layout>* L) {
    int st;
    L->resize(n_views);
    for (int v = 0; v < n_views; ++v) {
        const gs3_viewbuf* vb = &vbs[v];
        if ((st = check_vb(vb, &(*L)[v])) != GS3_OK) return st;
        if ((st = check_lists(vb)) != GS3_OK) return st;
        const char* a0 = static_cast<const char*>(vb->ws);
        for (int u = 0; u < v; ++u) {
            const char* b0 = static_cast<const char*>(vbs[u].ws);
            if (a0 < b0 + (*L)[u].total && b0 < a0 + (*L)[v].total)
                return fail(GS3_INVALID_ARG, "viewbufs[%d] and viewbufs[%d] share workspace memory", u, v);
        }
    }
    return GS3_OK;
}

int gs3_shadow_splat_views(const gs3_consts* consts, const gs3_viewbuf* light_vbs, int32_t n_views,
                           float* const* num_den, float* const* T, gs3_stream_t stream) {
    if (n_views < 1) return fail(GS3_INVALID_ARG, "n_views must be at least 1");
    if (!light_vbs || !num_den || !T) return fail(GS3_INVALID_ARG, "light_vbs, num_den or T is NULL");
    int st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    std::vector<Layout> L;
    if ((st = check_batch_vbs(light_vbs, n_views, &L)) != GS3_OK) return st;
    std::vector<const Layout*> Lp(n_views);
    std::vector<void*> ws(n_views);
    for (int v = 0; v < n_views; ++v) {
        if (L[v].n != L[0].n) return fail(GS3_INVALID_ARG, "light_vbs[%d].n differs from light_vbs[0].n", v);
        if (L[v].n > 0 && (!num_den[v] || !T[v])) return fail(GS3_INVALID_ARG, "num_den[%d] / T[%d] is NULL", v, v);
        Lp[v] = &L[v];
        ws[v] = light_vbs[v].ws;
    }
    const hipStream_t s = (hipStream_t)stream;
    GS3_CHECK_HIP(launch_shadow_den_batch(*consts, Lp.data(), ws.data(), num_den, n_views, s));
    GS3_CHECK_HIP(launch_shadow_num_batch(*consts, Lp.data(), ws.data(), num_den, n_views, s));
    GS3_CHECK_HIP(launch_shadow_resolve_batch(Lp.data(), ws.data(), num_den, T, n_views, s));
    return GS3_OK;
}

int gs3_render_views(const gs3_scene* scene, const gs3_view* cams, const gs3_view* lights, int32_t n_views,
                     const gs3_consts* consts, const float* const* T, const gs3_mlp* phi, const gs3_mlp* psi,
                     const gs3_viewbuf* cam_vbs, const gs3_images* outs, gs3_stream_t stream) {
    if (n_views < 1) return fail(GS3_INVALID_ARG, "n_views must be at least 1");
    if (!cams || !lights || !T || !cam_vbs || !outs) return fail(GS3_INVALID_ARG, "an array argument is NULL");
    int st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if ((st = check_scene(scene, true)) != GS3_OK) return st;
    if ((st = check_mlps(scene, phi, psi)) != GS3_OK) return st;
    std::vector<Layout> L;
    if ((st = check_batch_vbs(cam_vbs, n_views, &L)) != GS3_OK) return st;
    std::vector<const Layout*> Lp(n_views);
    std::vector<void*> ws(n_views);
    std::vector<ShadeParams> sp(n_views);
    std::vector<float*> colour(n_views);
    for (int v = 0; v < n_views; ++v) {
        Layout Lv;
        if ((st = render_args(scene, &cams[v], &lights[v], consts, &cam_vbs[v], &Lv)) != GS3_OK) return st;
        const gs3_images* o = &outs[v];
        if (!o->final_rgb || !o->shading || !o->shadow || !o->residual || !o->t_final || !o->n_contrib || !o->colour)
            return fail(GS3_INVALID_ARG, "an output pointer of outs[%d] is NULL", v);
        if (L[v].n > 0 && !T[v]) return fail(GS3_INVALID_ARG, "T[%d] is NULL", v);
        Lp[v] = &L[v];
        ws[v] = cam_vbs[v].ws;
        sp[v] = shade_params(&cams[v], &lights[v], phi, psi);
        colour[v] = o->colour;
    }
    const hipStream_t s = (hipStream_t)stream;
    const SceneDev sd = scene_dev(scene);
    if (scene->appearance == GS3_APPEARANCE_BASIS)
        GS3_CHECK_HIP(launch_basis_shade_batch(sd, sp.data(), T, phi, psi, Lp.data(), ws.data(), colour.data(), 3,
                                               n_views, s));
    else
        GS3_CHECK_HIP(launch_shade_mlp_batch(sd, sp.data(), T, phi, psi, Lp.data(), ws.data(), colour.data(), 3,
                                             n_views, s));
    GS3_CHECK_HIP(launch_render_batch(*consts, Lp.data(), ws.data(), outs, n_views, s));
    return GS3_OK;
}

// Backward workspace: per-Gaussian splat gradients of both views, colour
// gradients, dL/dT, dL/dnum, per-light-pixel sums, the MLP scratch rows and
// the weight-gradient partial sums.
struct BwdLayout {
    size_t gcam, gcol, glight, dT, dnum, gray, rows, partial, total;
};
static bool bwd_layout(int32_t appearance, int64_t n, int32_t lw, int32_t lh, BwdLayout* B) {
    if (n < 0 || n >= (int64_t(1) << 31) || lw <= 0 || lh <= 0 || lw > 16384 || lh > 16384) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t nn = (size_t)n;
    const int64_t chunks = (n + kWgChunkHost - 1) / kWgChunkHost;
    B->gcam = take(4 * 6 * nn);
    B->gcol = take(4 * 7 * nn);
    B->glight = take(4 * 6 * nn);
    B->dT = take(4 * nn);
    B->dnum = take(4 * nn);
    B->gray = take(4 * (size_t)lw * lh);
    if (appearance == GS3_APPEARANCE_BASIS) {
        B->rows = take(4 * (size_t)basis_scratch_rows() * nn);
        B->partial = take(4 * ((size_t)basis_partial_floats(kMaxLobes) +
                               (size_t)chunks * basis_wgrad_total_params()));
    } else {
        B->rows = take(4 * (size_t)mlp_scratch_rows() * nn);
        B->partial = take(4 * (size_t)chunks * wgrad_total_params(true, true));
    }
    B->total = off;
    return true;
}

int gs3_backward_workspace_size_for(int32_t appearance, int64_t n, int32_t light_width, int32_t light_height,
                                    size_t* bytes) {
    if (!bytes) return fail(GS3_INVALID_ARG, "bytes is NULL");
    if (appearance != GS3_APPEARANCE_LOBES && appearance != GS3_APPEARANCE_BASIS)
        return fail(GS3_INVALID_ARG, "bad appearance");
    BwdLayout B;
    if (!bwd_layout(appearance, n, light_width, light_height, &B))
        return fail(GS3_INVALID_ARG, "invalid sizes (n=%lld, light %dx%d)", (long long)n, light_width, light_height);
    *bytes = B.total;
    return GS3_OK;
}

int gs3_backward_workspace_size(int64_t n, int32_t light_width, int32_t light_height, size_t* bytes) {
    return gs3_backward_workspace_size_for(GS3_APPEARANCE_LOBES, n, light_width, light_height, bytes);
}

static int proj_params(const gs3_view* v, const Layout& L, int depth_mode, const gs3_consts* k, ViewParams* vp) {
    int st = view_params(v, L, depth_mode, vp);
    if (st != GS3_OK) return st;
    vp->lim_x = k->clamp_frac * ((v->width / 2.0) / vp->focal);
    vp->lim_y = k->clamp_frac * ((v->height / 2.0) / vp->focal);
    return GS3_OK;
}

int gs3_render_backward(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light,
                        const gs3_consts* consts, const float* T, const float* num_den, const gs3_mlp* phi,
                        const gs3_mlp* psi, const gs3_viewbuf* light_vb, const gs3_viewbuf* cam_vb,
                        const gs3_images* fwd, const float* dL_dfinal, const gs3_grads* grads, void* ws,
                        size_t ws_bytes, gs3_stream_t stream) {
    Layout Lc, Ll;
    int st;
    if ((st = check_vb(cam_vb, &Lc)) != GS3_OK) return st;
    if ((st = check_vb(light_vb, &Ll)) != GS3_OK) return st;
    if ((st = check_lists(cam_vb)) != GS3_OK) return st;
    if ((st = check_lists(light_vb)) != GS3_OK) return st;
    if ((st = check_scene(scene, true)) != GS3_OK) return st;
    if ((st = check_consts(consts)) != GS3_OK) return st;
    if (scene->n != cam_vb->n || scene->n != light_vb->n)
        return fail(GS3_INVALID_ARG, "scene.n differs from a view buffer's n");
    ViewParams vpc, vpl;
    if ((st = proj_params(cam, Lc, GS3_DEPTH_Z, consts, &vpc)) != GS3_OK) return st;
    if ((st = proj_params(light, Ll, GS3_DEPTH_DIST, consts, &vpl)) != GS3_OK) return st;
    if ((st = check_mlps(scene, phi, psi)) != GS3_OK) return st;
    if (!fwd || !fwd->shading || !fwd->shadow || !fwd->residual)
        return fail(GS3_INVALID_ARG, "forward images (shading, shadow, residual) missing");
    if (scene->n > 0 && (!T || !num_den)) return fail(GS3_INVALID_ARG, "T / num_den is NULL");
    if (!dL_dfinal) return fail(GS3_INVALID_ARG, "dL_dfinal is NULL");
    const bool basis = scene->appearance == GS3_APPEARANCE_BASIS;
    if (!grads || !grads->mean || !grads->log_scale || !grads->rot || !grads->opacity_logit || !grads->shade_rot ||
        !grads->albedo)
        return fail(GS3_INVALID_ARG, "a scene gradient pointer is NULL");
    if (!basis && (!grads->lobe_axis || !grads->lobe_log_sharp || !grads->lobe_amp || !grads->feat))
        return fail(GS3_INVALID_ARG, "a lobe or feature gradient pointer is NULL");
    if (basis && (!grads->spec_albedo || !grads->latent ||
                  (scene->k > 0 && (!grads->basis_weight || !grads->basis_rot || !grads->basis_log_sigma))))
        return fail(GS3_INVALID_ARG, "a basis-appearance gradient pointer is NULL");
    for (int i = 0; i < 4; ++i) {
        if (phi && (!grads->phi_w[i] || !grads->phi_b[i])) return fail(GS3_INVALID_ARG, "phi gradient pointer is NULL");
        if (psi && (!grads->psi_w[i] || !grads->psi_b[i])) return fail(GS3_INVALID_ARG, "psi gradient pointer is NULL");
    }
    BwdLayout B;
    if (!bwd_layout(scene->appearance, scene->n, light->width, light->height, &B))
        return fail(GS3_INVALID_ARG, "invalid sizes");
    if (!ws) return fail(GS3_INVALID_ARG, "ws is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(GS3_INVALID_ARG, "ws not 256-byte aligned");
    if (ws_bytes < B.total)
        return fail(GS3_WORKSPACE_TOO_SMALL, "backward workspace has %zu bytes, needs %zu", ws_bytes, B.total);
    if (scene->n == 0) return GS3_OK;
    hipStream_t s = (hipStream_t)stream;
    float* gcam = at<float>(ws, B.gcam);
    float* gcol = at<float>(ws, B.gcol);
    float* glight = at<float>(ws, B.glight);
    float* dT = at<float>(ws, B.dT);
    float* dnum = at<float>(ws, B.dnum);
    float* gray = at<float>(ws, B.gray);
    float* rows = at<float>(ws, B.rows);
    float* partial = at<float>(ws, B.partial);
    const int64_t n = scene->n;
    GS3_CHECK_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(gcam), 0u, 6 * n, s));
    GS3_CHECK_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(gcol), 0u, 7 * n, s));
    GradDev g;
    g.mean = grads->mean;
    g.log_scale = grads->log_scale;
    g.rot = grads->rot;
    g.opacity_logit = grads->opacity_logit;
    g.shade_rot = grads->shade_rot;
    g.albedo = grads->albedo;
    g.lobe_axis = grads->lobe_axis;
    g.lobe_log_sharp = grads->lobe_log_sharp;
    g.lobe_amp = grads->lobe_amp;
    g.feat = grads->feat;
    g.spec_albedo = grads->spec_albedo;
    g.basis_weight = grads->basis_weight;
    g.latent = grads->latent;
    g.basis_rot = grads->basis_rot;
    g.basis_log_sigma = grads->basis_log_sigma;
    ShadeParams sp;
    shade_light(light, &sp);
    for (int i = 0; i < 3; ++i) sp.eye[i] = (float)cam->eye[i];
    sp.use_phi = phi != nullptr;
    sp.use_psi = psi != nullptr;
    const SceneDev sd = scene_dev(scene);
    GS3_CHECK_HIP(launch_render_bwd(*consts, Lc, cam_vb->ws, *fwd, dL_dfinal, gcam, gcol, s));
    if (basis)
        GS3_CHECK_HIP(launch_basis_shade_bwd(sd, sp, T, phi, psi, gcol, dT, g, rows, partial, grads, s));
    else
        GS3_CHECK_HIP(launch_shade_bwd(sd, sp, T, phi, psi, gcol, dT, g, rows, partial, grads, s));
    GS3_CHECK_HIP(launch_shadow_bwd(*consts, Ll, light_vb->ws, T, num_den, dT, dnum, gray, glight, s));
    GS3_CHECK_HIP(launch_project_bwd(sd, vpc, vpl, *consts, gcam, glight, g, s));
    return GS3_OK;
}

int gs3_l1_loss_workspace_size(int64_t count, size_t* bytes) {
    if (!bytes) return fail(GS3_INVALID_ARG, "bytes is NULL");
    if (count < 0) return fail(GS3_INVALID_ARG, "count < 0");
    const int64_t chunks = l1_chunks(count);
    *bytes = align256(sizeof(double) * (size_t)(chunks > 0 ? chunks : 1));
    return GS3_OK;
}

int gs3_l1_loss(const float* pred, const float* target, int64_t count, float scale, float* loss, float* dL_dpred,
                void* ws, size_t ws_bytes, gs3_stream_t stream) {
    if (count < 0) return fail(GS3_INVALID_ARG, "count < 0");
    if (!loss || (count > 0 && (!pred || !target))) return fail(GS3_INVALID_ARG, "pred / target / loss is NULL");
    if (!ws) return fail(GS3_INVALID_ARG, "ws is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(GS3_INVALID_ARG, "ws not 256-byte aligned");
    size_t need;
    gs3_l1_loss_workspace_size(count, &need);
    if (ws_bytes < need) return fail(GS3_WORKSPACE_TOO_SMALL, "loss workspace has %zu bytes, needs %zu", ws_bytes, need);
    GS3_CHECK_HIP(launch_l1_loss(pred, target, count, scale, loss, dL_dpred, static_cast<double*>(ws),
                                 (hipStream_t)stream));
    return GS3_OK;
}

int gs3_dssim_loss_workspace_size(int32_t channels, int32_t height, int32_t width, size_t* bytes) {
    if (!bytes) return fail(GS3_INVALID_ARG, "bytes is NULL");
    if (channels <= 0 || height <= 0 || width <= 0 || channels > 64 || height > 16384 || width > 16384)
        return fail(GS3_INVALID_ARG, "invalid image size %d x %d x %d", channels, height, width);
    *bytes = ssim_layout(channels, height, width).total;
    return GS3_OK;
}

int gs3_dssim_loss(const float* pred, const float* target, int32_t channels, int32_t height, int32_t width,
                   float scale, float* loss, float* dL_dpred, int32_t accumulate, void* ws, size_t ws_bytes,
                   gs3_stream_t stream) {
    size_t need;
    int st;
    if ((st = gs3_dssim_loss_workspace_size(channels, height, width, &need)) != GS3_OK) return st;
    if (!pred || !target || !loss) return fail(GS3_INVALID_ARG, "pred / target / loss is NULL");
    if (!ws) return fail(GS3_INVALID_ARG, "ws is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(GS3_INVALID_ARG, "ws not 256-byte aligned");
    if (ws_bytes < need) return fail(GS3_WORKSPACE_TOO_SMALL, "D-SSIM workspace has %zu bytes, needs %zu", ws_bytes, need);
    GS3_CHECK_HIP(launch_dssim(pred, target, channels, height, width, scale, loss, dL_dpred, accumulate ? 1 : 0, ws,
                               (hipStream_t)stream));
    return GS3_OK;
}

int gs3_adam_step(float* param, const float* grad, float* m, float* v, int64_t count, int32_t step, float lr,
                  float beta1, float beta2, float eps, gs3_stream_t stream) {
    if (count < 0 || (count > 0 && (!param || !grad || !m || !v))) return fail(GS3_INVALID_ARG, "bad Adam buffers");
    if (step < 1) return fail(GS3_INVALID_ARG, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f) || !std::isfinite(lr))
        return fail(GS3_INVALID_ARG, "invalid Adam hyper-parameters");
    GS3_CHECK_HIP(launch_adam(param, grad, m, v, count, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_image_accumulate(float* dst, const float* src, float weight, int64_t count, gs3_stream_t stream) {
    if (count < 0 || (count > 0 && (!dst || !src))) return fail(GS3_INVALID_ARG, "bad image buffers");
    if (!std::isfinite(weight)) return fail(GS3_INVALID_ARG, "weight is not finite");
    GS3_CHECK_HIP(launch_accumulate_scaled(dst, src, weight, count, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_grads_clear(float* g, int64_t count, gs3_stream_t stream) {
    if (count < 0 || (count > 0 && !g)) return fail(GS3_INVALID_ARG, "bad gradient buffer");
    GS3_CHECK_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(g), 0u, count, (hipStream_t)stream));
    return GS3_OK;
}

int gs3_grads_accumulate(float* dst, const float* src, int64_t count, gs3_stream_t stream) {
    if (count < 0 || (count > 0 && (!dst || !src))) return fail(GS3_INVALID_ARG, "bad gradient buffers");
    GS3_CHECK_HIP(launch_accumulate(dst, src, count, (hipStream_t)stream));
    return GS3_OK;
}

}  // extern "C"
