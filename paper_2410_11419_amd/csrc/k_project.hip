// Projection of spatial Gaussians to 2D splats (Sec. 3, Eq. 1; EWA splatting
// as in the Gaussian-splatting pipeline the paper builds on).
//
// One lane per Gaussian, evaluated in double precision: this is per-Gaussian
// work (a few hundred flops each, negligible next to the per-pixel passes),
// and doing it in double keeps splat centres and depth keys accurate to well
// below a float32 ulp of the pixel coordinate, so the float32 per-pixel
// threshold decisions downstream agree with an exact evaluation except on a
// vanishing set of pixels.
#include "splat_common.h"

namespace gs3 {

__device__ inline int64_t floor_clamped(double x) {
    x = fmin(fmax(x, -1073741824.0), 1073741824.0);
    return (int64_t)floor(x);
}

// Integer tile rectangle of a splat (shared by projection and explicit
// binning): pixel columns ix-rx..ix+rx, rows iy-ry..iy+ry, 16x16 tiles.
__device__ inline bool tile_rect(int64_t ix, int64_t iy, int64_t rx, int64_t ry, int tiles_x,
                                 int tiles_y, int* x0, int* x1, int* y0, int* y1) {
    if (rx <= 0 || ry <= 0) return false;
    auto fdiv = [](int64_t a) -> int64_t { return a >= 0 ? a / kTile : -((-a + kTile - 1) / kTile); };
    int64_t a0 = fdiv(ix - rx), a1 = fdiv(ix + rx);
    int64_t b0 = fdiv(iy - ry), b1 = fdiv(iy + ry);
    a0 = a0 < 0 ? 0 : a0;
    b0 = b0 < 0 ? 0 : b0;
    a1 = a1 > tiles_x - 1 ? tiles_x - 1 : a1;
    b1 = b1 > tiles_y - 1 ? tiles_y - 1 : b1;
    if (a0 > a1 || b0 > b1) return false;
    *x0 = (int)a0; *x1 = (int)a1; *y0 = (int)b0; *y1 = (int)b1;
    return true;
}

// Output buffers of one view's projection (in its workspace).
struct ProjDesc {
    ViewParams vp;
    float4* rec0;
    float4* rec1;
    float4* rec2;
    float* depth_out;
    int4* ext;
    int4* drec;
    uint32_t* cnt;
    uint32_t* keys;
    uint32_t* vals;
    unsigned long long* num;
};
struct ProjBatch {
    int32_t nv;
    uint32_t blocks_per_view;
    ProjDesc d[kMaxBatch];
};
static_assert(sizeof(ProjBatch) <= 3072, "projection batch exceeds the kernel argument budget");

// One lane per (view, Gaussian): the views of the batch share the scene,
// block b projects Gaussians of view b / blocks_per_view.
__global__ __launch_bounds__(256) void k_project(SceneDev sc, gs3_consts kc, ProjBatch B) {
    const int view = (int)(blockIdx.x / B.blocks_per_view);
    const ProjDesc& D = B.d[view];
    const ViewParams& vp = D.vp;
    float4* __restrict__ rec0 = D.rec0;
    float4* __restrict__ rec1 = D.rec1;
    float4* __restrict__ rec2 = D.rec2;
    float* __restrict__ depth_out = D.depth_out;
    int4* __restrict__ ext = D.ext;
    int4* __restrict__ drec = D.drec;
    uint32_t* __restrict__ cnt = D.cnt;
    uint32_t* __restrict__ keys = D.keys;
    uint32_t* __restrict__ vals = D.vals;
    const int i = (int)(blockIdx.x - view * B.blocks_per_view) * blockDim.x + threadIdx.x;
    const int n = sc.n;
    if (i >= n) return;
    D.num[i] = 0ull;   // the shadow numerator's accumulator starts empty for every projection
    const double mx = sc.mean[i], my = sc.mean[n + i], mz = sc.mean[2 * n + i];
    const double s0 = exp((double)sc.log_scale[i]);
    const double s1 = exp((double)sc.log_scale[n + i]);
    const double s2 = exp((double)sc.log_scale[2 * n + i]);
    double qw = sc.rot[i], qx = sc.rot[n + i], qy = sc.rot[2 * n + i], qz = sc.rot[3 * n + i];
    const double qn = rsqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    // R (Eq. 1) and M = R diag(s): Sigma = M M^T
    const double R00 = 1 - 2 * (qy * qy + qz * qz), R01 = 2 * (qx * qy - qw * qz), R02 = 2 * (qx * qz + qw * qy);
    const double R10 = 2 * (qx * qy + qw * qz), R11 = 1 - 2 * (qx * qx + qz * qz), R12 = 2 * (qy * qz - qw * qx);
    const double R20 = 2 * (qx * qz - qw * qy), R21 = 2 * (qy * qz + qw * qx), R22 = 1 - 2 * (qx * qx + qy * qy);
    const double M00 = R00 * s0, M01 = R01 * s1, M02 = R02 * s2;
    const double M10 = R10 * s0, M11 = R11 * s1, M12 = R12 * s2;
    const double M20 = R20 * s0, M21 = R21 * s1, M22 = R22 * s2;
    // view-space centre
    const double dx = mx - vp.eye[0], dy = my - vp.eye[1], dz = mz - vp.eye[2];
    const double tx = vp.R[0] * dx + vp.R[1] * dy + vp.R[2] * dz;
    const double ty = vp.R[3] * dx + vp.R[4] * dy + vp.R[5] * dz;
    const double tz = vp.R[6] * dx + vp.R[7] * dy + vp.R[8] * dz;
    // distance key: to the light's position (perspective), or along the
    // light's direction (orthographic: a directional light, Sec. 4.5)
    const double dep = vp.depth_mode == GS3_DEPTH_DIST && !vp.ortho ? sqrt(dx * dx + dy * dy + dz * dz) : tz;

    bool ok = tz > (double)kc.near_plane;
    const double tzs = ok ? tz : 1.0;
    const double f = vp.focal;
    const double xr = fmin(fmax(tx / tzs, -vp.lim_x), vp.lim_x);
    const double yr = fmin(fmax(ty / tzs, -vp.lim_y), vp.lim_y);
    // A = J R_v (2x3) with J = [[f/z, 0, -f xr/z], [0, f/z, -f yr/z]], or
    // for a parallel projection J = [[s, 0, 0], [0, s, 0]]
    const double j0 = vp.ortho ? vp.scale : f / tzs;
    const double j2x = vp.ortho ? 0.0 : -f * xr / tzs, j2y = vp.ortho ? 0.0 : -f * yr / tzs;
    const double A00 = j0 * vp.R[0] + j2x * vp.R[6], A01 = j0 * vp.R[1] + j2x * vp.R[7], A02 = j0 * vp.R[2] + j2x * vp.R[8];
    const double A10 = j0 * vp.R[3] + j2y * vp.R[6], A11 = j0 * vp.R[4] + j2y * vp.R[7], A12 = j0 * vp.R[5] + j2y * vp.R[8];
    // B = A M (2x3); Sigma' = B B^T
    const double B00 = A00 * M00 + A01 * M10 + A02 * M20;
    const double B01 = A00 * M01 + A01 * M11 + A02 * M21;
    const double B02 = A00 * M02 + A01 * M12 + A02 * M22;
    const double B10 = A10 * M00 + A11 * M10 + A12 * M20;
    const double B11 = A10 * M01 + A11 * M11 + A12 * M21;
    const double B12 = A10 * M02 + A11 * M12 + A12 * M22;
    const double ca = B00 * B00 + B01 * B01 + B02 * B02 + (double)kc.dilation;
    const double cb = B00 * B10 + B01 * B11 + B02 * B12;
    const double cc = B10 * B10 + B11 * B11 + B12 * B12 + (double)kc.dilation;
    const double det = ca * cc - cb * cb;
    ok = ok && det > 0.0;
    const double u = (vp.ortho ? vp.scale * tx : f * tx / tzs) + vp.cx;
    const double v = (vp.ortho ? vp.scale * ty : f * ty / tzs) + vp.cy;
    const double logit = sc.opacity_logit[i];
    const double opac = 1.0 / (1.0 + exp(-logit));
    // hit ellipse: power >= -p with p = min(cutoff, ln(opacity / alpha_min))
    double p = (double)kc.cutoff;
    if (kc.alpha_min > 0.f) p = fmin(p, log(opac / (double)kc.alpha_min));
    ok = ok && p > 0.0;
    int64_t rx = -1, ry = -1, ix = 0, iy = 0;
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    if (ok) {
        const double big = 1048576.0;
        const double ex = sqrt(2.0 * p * ca), ey = sqrt(2.0 * p * cc);
        rx = (int64_t)fmin(ceil(ex), big);
        ry = (int64_t)fmin(ceil(ey), big);
        ix = floor_clamped(u);
        iy = floor_clamped(v);
        ok = tile_rect(ix, iy, rx, ry, vp.tiles_x, vp.tiles_y, &x0, &x1, &y0, &y1);
    }
    if (ok) {
        const double id = 1.0 / det;
        const double fu = floor(u), fv = floor(v);
        rec0[i] = make_float4((float)fu, (float)fv, (float)(u - fu), (float)(v - fv));
        const float4 r1 = make_float4((float)(cc * id), (float)(-cb * id), (float)(ca * id), (float)opac);
        rec1[i] = r1;
        // the float32 hit threshold and bounding box every splat kernel uses
        const float4 r2 = splat_bounds(r1, kc.cutoff, kc.alpha_min);
        rec2[i] = r2;
        drec[i] = den_ranges(make_float4((float)fu, (float)fv, (float)(u - fu), (float)(v - fv)), r1, r2, x0, x1, y0,
                             y1);
        ext[i] = make_int4((int)ix, (int)iy, (int)rx, (int)ry);
        const float d32 = (float)dep;
        depth_out[i] = d32;
        cnt[i] = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
        keys[i] = __float_as_uint(d32);
    } else {
        rec0[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        rec1[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        rec2[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        drec[i] = make_int4(1, 1, 0, 0);
        ext[i] = make_int4((int)floor_clamped(u), (int)floor_clamped(v), -1, -1);
        depth_out[i] = (float)dep;
        cnt[i] = 0u;
        keys[i] = 0xFFFFFFFFu;
    }
    vals[i] = (uint32_t)i;
}

// Explicit binning input: extents and depths given by the caller.
__global__ __launch_bounds__(256) void k_extent_keys(const int32_t* __restrict__ ix, const int32_t* __restrict__ iy,
                                                      const int32_t* __restrict__ rx, const int32_t* __restrict__ ry,
                                                      const float* __restrict__ depth, int n, int tiles_x, int tiles_y,
                                                      int4* __restrict__ ext, uint32_t* __restrict__ cnt,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                      float* __restrict__ depth_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int x0, x1, y0, y1;
    const bool ok = tile_rect(ix[i], iy[i], rx[i], ry[i], tiles_x, tiles_y, &x0, &x1, &y0, &y1);
    ext[i] = make_int4(ix[i], iy[i], ok ? rx[i] : -1, ok ? ry[i] : -1);
    cnt[i] = ok ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;
    keys[i] = ok ? __float_as_uint(depth[i]) : 0xFFFFFFFFu;
    vals[i] = (uint32_t)i;
    depth_out[i] = depth[i];
}

hipError_t launch_project_batch(const SceneDev& sc, const ViewParams* vps, const gs3_consts& k,
                                const Layout* const* Ls, void* const* wss, int nv, hipStream_t st) {
    if (sc.n == 0 || nv <= 0) return hipSuccess;
    const uint32_t per = (uint32_t)((sc.n + 255) / 256);
    for (int c0 = 0; c0 < nv; c0 += kMaxBatch) {
        ProjBatch B;
        B.nv = 0;
        B.blocks_per_view = per;
        for (int v = c0; v < nv && v < c0 + kMaxBatch; ++v) {
            const Layout& L = *Ls[v];
            void* ws = wss[v];
            ProjDesc& d = B.d[B.nv++];
            d.vp = vps[v];
            d.rec0 = at<float4>(ws, L.rec0);
            d.rec1 = at<float4>(ws, L.rec1);
            d.rec2 = at<float4>(ws, L.rec2);
            d.depth_out = at<float>(ws, L.depth);
            d.ext = at<int4>(ws, L.ext);
            d.drec = at<int4>(ws, L.drec);
            d.cnt = at<uint32_t>(ws, L.cnt);
            d.keys = at<uint32_t>(ws, L.keys_a);
            d.vals = at<uint32_t>(ws, L.vals_a);
            d.num = at<unsigned long long>(ws, L.num);
        }
        hipLaunchKernelGGL(k_project, dim3(per * (uint32_t)B.nv), dim3(256), 0, st, sc, k, B);
    }
    return hipGetLastError();
}

hipError_t launch_project(const SceneDev& sc, const ViewParams& vp, const gs3_consts& k,
                          const Layout& L, void* ws, hipStream_t st) {
    const Layout* Lp = &L;
    return launch_project_batch(sc, &vp, k, &Lp, &ws, 1, st);
}

hipError_t launch_extent_keys(const int32_t* ix, const int32_t* iy, const int32_t* rx,
                              const int32_t* ry, const float* depth, const Layout& L,
                              void* ws, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    const int grid = (int)((L.n + 255) / 256);
    hipLaunchKernelGGL(k_extent_keys, dim3(grid), dim3(256), 0, st, ix, iy, rx, ry, depth, (int)L.n,
                       L.tiles_x, L.tiles_y, at<int4>(ws, L.ext), at<uint32_t>(ws, L.cnt),
                       at<uint32_t>(ws, L.keys_a), at<uint32_t>(ws, L.vals_a), at<float>(ws, L.depth));
    // records are unused by the explicit binning path; zero them for readers
    hipError_t e = launch_fill_u32(at<uint32_t>(ws, L.rec0), 0u, 4 * L.n, st);
    if (e == hipSuccess) e = launch_fill_u32(at<uint32_t>(ws, L.rec1), 0u, 4 * L.n, st);
    if (e == hipSuccess) e = launch_fill_u32(at<uint32_t>(ws, L.rec2), 0u, 4 * L.n, st);
    // no denominator work: the empty range {1, 1, 0, 0} in every word pair
    if (e == hipSuccess) e = launch_fill_u32(at<uint32_t>(ws, L.drec), 1u, 4 * L.n, st);
    if (e == hipSuccess) e = launch_fill_u32(at<uint32_t>(ws, L.num), 0u, 2 * L.n, st);
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace gs3
