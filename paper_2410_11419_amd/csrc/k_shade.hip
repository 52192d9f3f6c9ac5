// Per-Gaussian appearance: the first splat (Sec. 4.1, Eq. 4-7), the shadow
// refinement MLP Phi (Sec. 4.2, Eq. 8) and the residual MLP Psi (Sec. 4.3).
//
// k_shade_c evaluates the shading one Gaussian per lane. k_shade_mlp runs
// the MLPs: a wave handles 16 Gaussians, four lanes per Gaussian (lane l:
// Gaussian l % 16, quarter q = l / 16), which is the operand layout of the
// MFMA MLPs (mlp_common.h). The one- and three-wide output layers run on
// the VALU (16 FMAs per lane and a cross-lane sum over the four quarters).
#include "mlp_common.h"

namespace gs3 {

// Which parts a launch computes: the shading c and Psi's residual r (they do
// not depend on the shadow values) and/or Phi's refined shadow T'.
enum ShadeParts { kShadePsi = 1, kShadePhi = 2 };

// Scene, MLPs and the views of one launch (blockIdx.y selects the view).
struct ShadeArgs {
    SceneDev sc;
    int use_phi, use_psi;
    int parts;
    MlpArgs phi, psi;
    ShadeView v[kMaxBatch];
};

// Shading c (Eq. 4-7) of the view blockIdx.y, one Gaussian per lane over
// all its lobes. Writes c to col0.xyz and colour rows 0..2; k_shade_mlp
// adds T' (col0.w, row 3) and r (col1, rows 4..7).
__global__ __launch_bounds__(256) void k_shade_c(ShadeArgs a) {
    const SceneDev& sc = a.sc;
    const ShadeView vw = a.v[blockIdx.y];
    const int n = sc.n;
    const float kd = 0.01f * (1.f - 0.36787944117144233f);   // eps (1 - 1/e), Eq. 5
    const float fd_norm = 1.f / ((1.f + kd) * 3.14159265358979f);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        // w_i: toward a point light, or a directional light's fixed direction
        const float lm = vw.light_dir ? 0.f : 1.f;
        float wix = vw.light[0] - lm * mx, wiy = vw.light[1] - lm * my, wiz = vw.light[2] - lm * mz;
        float r = rsqrtf(wix * wix + wiy * wiy + wiz * wiz);
        wix *= r; wiy *= r; wiz *= r;
        float wox = vw.eye[0] - mx, woy = vw.eye[1] - my, woz = vw.eye[2] - mz;
        r = rsqrtf(wox * wox + woy * woy + woz * woz);
        wox *= r; woy *= r; woz *= r;
        float qw = sc.shade_rot[g], qx = sc.shade_rot[n + g], qy = sc.shade_rot[2 * n + g], qz = sc.shade_rot[3 * n + g];
        r = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= r; qx *= r; qy *= r; qz *= r;
        const float R00 = 1 - 2 * (qy * qy + qz * qz), R01 = 2 * (qx * qy - qw * qz), R02 = 2 * (qx * qz + qw * qy);
        const float R10 = 2 * (qx * qy + qw * qz), R11 = 1 - 2 * (qx * qx + qz * qz), R12 = 2 * (qy * qz - qw * qx);
        const float R20 = 2 * (qx * qz - qw * qy), R21 = 2 * (qy * qz + qw * qx), R22 = 1 - 2 * (qx * qx + qy * qy);
        const float lix = R00 * wix + R01 * wiy + R02 * wiz;
        const float liy = R10 * wix + R11 * wiy + R12 * wiz;
        const float liz = R20 * wix + R21 * wiy + R22 * wiz;
        const float lox = R00 * wox + R01 * woy + R02 * woz;
        const float loy = R10 * wox + R11 * woy + R12 * woz;
        const float loz = R20 * wox + R21 * woy + R22 * woz;
        // modified Lambertian (Eq. 5), normal = +z of the shading frame
        const float elu = liz > 0.f ? liz : 0.01f * (expf(fminf(liz, 0.f)) - 1.f);
        const float fd = (elu + kd) * fd_norm;
        // half vector (Eq. 6)
        float hx = lix + lox, hy = liy + loy, hz = liz + loz;
        const float hn2 = hx * hx + hy * hy + hz * hz;
        if (hn2 > 1e-24f) {
            r = rsqrtf(hn2);
            hx *= r; hy *= r; hz *= r;
        } else {
            hx = 0.f; hy = 0.f; hz = 1.f;
        }
        // isotropic angular Gaussians (Eq. 7 with sigma_x = sigma_y):
        // G = lambda exp(-(lambda theta)^2 / 2), theta = angle(h', z_k)
        float sp0 = 0.f, sp1 = 0.f, sp2 = 0.f;
        for (int kl = 0; kl < sc.k; ++kl) {
            const float* ax = sc.lobe_axis + (size_t)kl * 3 * n;
            float zx = ax[g], zy = ax[n + g], zz = ax[2 * n + g];
            r = rsqrtf(zx * zx + zy * zy + zz * zz);
            zx *= r; zy *= r; zz *= r;
            const float cz = hx * zx + hy * zy + hz * zz;
            const float cx = hy * zz - hz * zy, cy = hz * zx - hx * zz, cw = hx * zy - hy * zx;
            const float theta = atan2f(sqrtf(cx * cx + cy * cy + cw * cw), cz);
            const float lam = expf(sc.lobe_log_sharp[(size_t)kl * n + g]);
            const float t = lam * theta;
            const float G = lam * expf(-0.5f * t * t);
            const float* am = sc.lobe_amp + (size_t)kl * 3 * n;
            sp0 = fmaf(am[g], G, sp0);
            sp1 = fmaf(am[n + g], G, sp1);
            sp2 = fmaf(am[2 * n + g], G, sp2);
        }
        const float c0 = fmaf(sc.albedo[g], fd, sp0);
        const float c1 = fmaf(sc.albedo[n + g], fd, sp1);
        const float c2 = fmaf(sc.albedo[2 * n + g], fd, sp2);
        float* c0p = reinterpret_cast<float*>(vw.col0 + g);
        c0p[0] = c0;
        c0p[1] = c1;
        c0p[2] = c2;
        vw.colour[g] = c0;
        vw.colour[(size_t)n + g] = c1;
        vw.colour[(size_t)2 * n + g] = c2;
    }
}

__global__ __launch_bounds__(512, 4) void k_shade_mlp(ShadeArgs a) {
    __shared__ __align__(16) float sm[kShadeSmem];
    const SceneDev& sc = a.sc;
    const ShadeView vw = a.v[blockIdx.y];
    const int n = sc.n;
    // only the MLPs this launch evaluates
    if (a.use_phi && (a.parts & kShadePhi)) load_mlp(sm, kPhiS, kPhiKR, kPhiIn, 1, a.phi);
    if (a.use_psi && (a.parts & kShadePsi)) load_mlp(sm, kPsiS, kPsiKR, kPsiIn, 3, a.psi);
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4;
    const int waves = blockDim.x >> 6;
    for (int base = (blockIdx.x * waves + w) * 16; base < n; base += gridDim.x * waves * 16) {
        const int g_raw = base + (lane & 15);
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        // ---- directions, Psi's inputs (the shading c is k_shade_c's)
        float wix = 0.f, wiy = 0.f, wiz = 0.f, wox = 0.f, woy = 0.f, woz = 0.f;
        if ((a.parts & kShadePsi) && a.use_psi) {
            const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
            const float lm = vw.light_dir ? 0.f : 1.f;
            wix = vw.light[0] - lm * mx; wiy = vw.light[1] - lm * my; wiz = vw.light[2] - lm * mz;
            float r = rsqrtf(wix * wix + wiy * wiy + wiz * wiz);
            wix *= r; wiy *= r; wiz *= r;
            wox = vw.eye[0] - mx; woy = vw.eye[1] - my; woz = vw.eye[2] - mz;
            r = rsqrtf(wox * wox + woy * woy + woz * woz);
            wox *= r; woy *= r; woz *= r;
        }
        // ---- shadow refinement Phi([T, feat]) (Eq. 8)
        float tp = 0.f;
        if (a.parts & kShadePhi) tp = vw.T[g];
        if ((a.parts & kShadePhi) && a.use_phi) {
            const float Tg = tp;
            floatx4 h[4];
            auto xin = [&](int k) -> float {
                if (k == 0) return Tg;
                if (k <= kFeat) return sc.feat[(size_t)(k - 1) * n + g];
                return 0.f;
            };
            mlp_hidden<kPhiKR>(sm, kPhiS, lane, xin, h);
            tp = mlp_out(sm, kPhiS, lane, h, 0);
        }
        // ---- residual Psi([feat, w_i, w_o]) (Sec. 4.3)
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if ((a.parts & kShadePsi) && a.use_psi) {
            floatx4 h[4];
            auto xin = [&](int k) -> float {
                if (k < kFeat) return sc.feat[(size_t)k * n + g];
                switch (k - kFeat) {
                    case 0: return wix;
                    case 1: return wiy;
                    case 2: return wiz;
                    case 3: return wox;
                    case 4: return woy;
                    case 5: return woz;
                    default: return 0.f;
                }
            };
            mlp_hidden<kPsiKR>(sm, kPsiS, lane, xin, h);
            r0 = mlp_out(sm, kPsiS, lane, h, 0);
            r1 = mlp_out(sm, kPsiS, lane, h, 1);
            r2 = mlp_out(sm, kPsiS, lane, h, 2);
        }
        if (valid) {
            // r: col1 and colour rows 4..7 (row 7 = 0); T': col0.w and row 3
            if (a.parts & kShadePsi) {
                if (q == 0) vw.col1[g] = make_float4(r0, r1, r2, 0.f);
                vw.colour[(size_t)(4 + q) * n + g] = q == 0 ? r0 : (q == 1 ? r1 : (q == 2 ? r2 : 0.f));
            }
            if ((a.parts & kShadePhi) && q == 0) {
                reinterpret_cast<float*>(vw.col0 + g)[3] = tp;
                vw.colour[(size_t)3 * n + g] = tp;
            }
        }
    }
}

hipError_t launch_shade_mlp_batch(const SceneDev& sc, const ShadeParams* sps, const float* const* T,
                                  const gs3_mlp* phi, const gs3_mlp* psi, const Layout* const* Ls,
                                  void* const* wss, float* const* colour, int parts, int nv, hipStream_t st) {
    if (sc.n == 0) return hipSuccess;
    ShadeArgs a;
    a.sc = sc;
    a.parts = parts;
    a.use_phi = phi != nullptr;
    a.use_psi = psi != nullptr;
    for (int i = 0; i < 4; ++i) {
        a.phi.w[i] = phi ? phi->w[i] : nullptr;
        a.phi.b[i] = phi ? phi->b[i] : nullptr;
        a.psi.w[i] = psi ? psi->w[i] : nullptr;
        a.psi.b[i] = psi ? psi->b[i] : nullptr;
    }
    const int per_block = 8 * 16;
    int grid = (int)((sc.n + per_block - 1) / per_block);
    if (grid > 512) grid = 512;
    for (int v0 = 0; v0 < nv; v0 += kMaxBatch) {
        const int m = nv - v0 < kMaxBatch ? nv - v0 : kMaxBatch;
        for (int i = 0; i < m; ++i) {
            const ShadeParams& sp = sps[v0 + i];
            ShadeView& w = a.v[i];
            for (int c = 0; c < 3; ++c) {
                w.light[c] = sp.light[c];
                w.eye[c] = sp.eye[c];
            }
            w.light_dir = sp.light_dir;
            w.T = T ? T[v0 + i] : nullptr;
            w.col0 = at<float4>(wss[v0 + i], Ls[v0 + i]->col0);
            w.col1 = at<float4>(wss[v0 + i], Ls[v0 + i]->col1);
            w.colour = colour[v0 + i];
        }
        if (parts & kShadePsi) {
            const int64_t gc = (sc.n + 255) / 256;
            hipLaunchKernelGGL(k_shade_c, dim3((unsigned)(gc < 2048 ? gc : 2048), m), dim3(256), 0, st, a);
        }
        hipLaunchKernelGGL(k_shade_mlp, dim3(grid, m), dim3(512), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_shade_mlp(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                            const gs3_mlp* psi, const Layout& L, void* ws, float* colour_out, int parts,
                            hipStream_t st) {
    const Layout* Ls[1] = {&L};
    return launch_shade_mlp_batch(sc, &sp, &T, phi, psi, Ls, &ws, &colour_out, parts, 1, st);
}

}  // namespace gs3
