// Per-Gaussian adjoints: shading (Sec. 4.1, Eq. 4-7), the MLPs Phi (Sec.
// 4.2, Eq. 8) and Psi (Sec. 4.3), their weight gradients, and the EWA
// projection (Sec. 3, Eq. 1) of both views.
#include "mlp_common.h"

namespace gs3 {

constexpr float kLog2eF = 1.4426950408889634f;

// Rows of the per-Gaussian MLP scratch ([row][n] floats): each MLP's input
// and the gradient of its output pre-activation. The weight-gradient kernel
// recomputes the hidden activations and the hidden pre-activation gradients
// from these on the matrix cores, so the scratch stays small (43 rows).
struct MlpRows {
    int x, dout, size;
};
__host__ __device__ constexpr MlpRows mlp_rows(int base, int n_in, int n_out) {
    return MlpRows{base, base + n_in, n_in + n_out};
}
constexpr MlpRows kPhiRows = mlp_rows(0, kPhiIn, 1);
constexpr MlpRows kPsiRows = mlp_rows(kPhiRows.size, kPsiIn, 3);
constexpr int kMlpRows = kPhiRows.size + kPsiRows.size;
// after the MLP rows: Psi's gradient of its direction inputs w_i, w_o (6
// rows), from k_shade_bwd to k_shade_bwd_geom
constexpr int kDwRow = kMlpRows;
int mlp_scratch_rows() { return kMlpRows + 6; }

// LDS of one MLP's adjoint launch (PART 1: Phi, 2: Psi): its packed forward
// weights, then its transposed ones
template <int PART>
struct BwdLds {
    static constexpr MlpSmem S = PART == 1 ? mlp_smem(0, kPhiKR, 1) : mlp_smem(0, kPsiKR, 3);
    static constexpr MlpTSmem T = mlp_tsmem(S.size);
    static constexpr int size = S.size + T.size;
};
static_assert(BwdLds<1>::size * 4 <= 80 * 1024 && BwdLds<2>::size * 4 <= 80 * 1024,
              "each MLP adjoint fits half the LDS (two workgroups per CU)");

struct ShadeBwdArgs {
    SceneDev sc;
    float light[3];      // point light, or (light_dir) unit direction toward the light
    float eye[3];
    int use_phi, use_psi;
    int light_dir;
    const float* T;
    MlpArgs phi, psi;
    const float* gcol;   // [7][n] dL/d{c.rgb, T', r.rgb}
    float* dT;           // [n] = dL/dT
    GradDev g;           // += scene gradients (shading part)
    float* rows;         // [kMlpRows][n] MLP scratch (inputs, output-layer gradients)
};

// The shading adjoint outside the MLPs, one Gaussian per lane at full
// occupancy, after k_shade_bwd: the lobes (Eq. 7: amplitude, sharpness and
// axis gradients), the Lambertian term (Eq. 5, albedo), the half vector and
// shading frame (Eq. 6, shading quaternion) and the directions, with Psi's
// gradient of its w_i, w_o inputs from the scratch rows (mean).
__global__ __launch_bounds__(256) void k_shade_bwd_geom(ShadeBwdArgs a) {
    const SceneDev& sc = a.sc;
    const int n = sc.n;
    const float kd = 0.01f * (1.f - 0.36787944117144233f);
    const float fd_norm = 1.f / ((1.f + kd) * 3.14159265358979f);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
        // ---- forward recompute of the shading inputs
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        // w_i: toward a point light, or a directional light's fixed direction
        const float lm = a.light_dir ? 0.f : 1.f;
        float wix = a.light[0] - lm * mx, wiy = a.light[1] - lm * my, wiz = a.light[2] - lm * mz;
        const float ri = rsqrtf(wix * wix + wiy * wiy + wiz * wiz);
        wix *= ri; wiy *= ri; wiz *= ri;
        float wox = a.eye[0] - mx, woy = a.eye[1] - my, woz = a.eye[2] - mz;
        const float ro = rsqrtf(wox * wox + woy * woy + woz * woz);
        wox *= ro; woy *= ro; woz *= ro;
        float qw = sc.shade_rot[g], qx = sc.shade_rot[n + g], qy = sc.shade_rot[2 * n + g], qz = sc.shade_rot[3 * n + g];
        const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        const float rq = 1.f / qn;
        qw *= rq; qx *= rq; qy *= rq; qz *= rq;
        const float R00 = 1 - 2 * (qy * qy + qz * qz), R01 = 2 * (qx * qy - qw * qz), R02 = 2 * (qx * qz + qw * qy);
        const float R10 = 2 * (qx * qy + qw * qz), R11 = 1 - 2 * (qx * qx + qz * qz), R12 = 2 * (qy * qz - qw * qx);
        const float R20 = 2 * (qx * qz - qw * qy), R21 = 2 * (qy * qz + qw * qx), R22 = 1 - 2 * (qx * qx + qy * qy);
        const float lix = R00 * wix + R01 * wiy + R02 * wiz;
        const float liy = R10 * wix + R11 * wiy + R12 * wiz;
        const float liz = R20 * wix + R21 * wiy + R22 * wiz;
        const float lox = R00 * wox + R01 * woy + R02 * woz;
        const float loy = R10 * wox + R11 * woy + R12 * woz;
        const float loz = R20 * wox + R21 * woy + R22 * woz;
        const float elu = liz > 0.f ? liz : 0.01f * (expf(fminf(liz, 0.f)) - 1.f);
        const float delu = liz > 0.f ? 1.f : 0.01f * expf(fminf(liz, 0.f));
        const float fd = (elu + kd) * fd_norm;
        float hx = lix + lox, hy = liy + loy, hz = liz + loz;
        const float hn2 = hx * hx + hy * hy + hz * hz;
        const bool hok = hn2 > 1e-24f;
        float rh = 0.f;
        if (hok) {
            rh = rsqrtf(hn2);
            hx *= rh; hy *= rh; hz *= rh;
        } else {
            hx = 0.f; hy = 0.f; hz = 1.f;
        }
        const float dc0 = a.gcol[g], dc1 = a.gcol[(size_t)n + g], dc2 = a.gcol[(size_t)2 * n + g];
        // ---- lobes (Eq. 7): G = lambda exp(-(lambda theta)^2 / 2)
        float dhx = 0.f, dhy = 0.f, dhz = 0.f;
        for (int kl = 0; kl < sc.k; ++kl) {
            const size_t ab = (size_t)kl * 3 * n;
            const float ax = sc.lobe_axis[ab + g], ay = sc.lobe_axis[ab + n + g], az = sc.lobe_axis[ab + 2 * n + g];
            const float ra = rsqrtf(ax * ax + ay * ay + az * az);
            const float zx = ax * ra, zy = ay * ra, zz = az * ra;
            const float cz = hx * zx + hy * zy + hz * zz;
            const float cx = hy * zz - hz * zy, cy = hz * zx - hx * zz, cw = hx * zy - hy * zx;
            const float sn = sqrtf(cx * cx + cy * cy + cw * cw);
            const float theta = atan2f(sn, cz);
            const float lam = expf(sc.lobe_log_sharp[(size_t)kl * n + g]);
            const float t = lam * theta;
            const float ex = expf(-0.5f * t * t);
            const float G = lam * ex;
            const float am0 = sc.lobe_amp[ab + g], am1 = sc.lobe_amp[ab + n + g], am2 = sc.lobe_amp[ab + 2 * n + g];
            const float dG = fmaf(dc0, am0, fmaf(dc1, am1, dc2 * am2));
            // dtheta/dh = -(z - cz h)/sin(theta); dG/dtheta = -lam^3 theta ex
            const float ratio = sn > 1e-6f ? theta / sn : 1.f;
            const float coef = dG * lam * lam * lam * ex * ratio;
            dhx = fmaf(coef, zx - cz * hx, dhx);
            dhy = fmaf(coef, zy - cz * hy, dhy);
            dhz = fmaf(coef, zz - cz * hz, dhz);
            float dzx = coef * (hx - cz * zx), dzy = coef * (hy - cz * zy), dzz = coef * (hz - cz * zz);
            const float dzd = dzx * zx + dzy * zy + dzz * zz;
            dzx = (dzx - dzd * zx) * ra;
            dzy = (dzy - dzd * zy) * ra;
            dzz = (dzz - dzd * zz) * ra;
            a.g.lobe_amp[ab + g] += dc0 * G;
            a.g.lobe_amp[ab + n + g] += dc1 * G;
            a.g.lobe_amp[ab + 2 * n + g] += dc2 * G;
            a.g.lobe_log_sharp[(size_t)kl * n + g] += dG * ex * (1.f - t * t) * lam;
            a.g.lobe_axis[ab + g] += dzx;
            a.g.lobe_axis[ab + n + g] += dzy;
            a.g.lobe_axis[ab + 2 * n + g] += dzz;
        }
        // ---- Lambertian, half vector, frames and directions
        const float alb0 = sc.albedo[g], alb1 = sc.albedo[n + g], alb2 = sc.albedo[2 * n + g];
        const float dfd = fmaf(dc0, alb0, fmaf(dc1, alb1, dc2 * alb2));
        float dhsx = 0.f, dhsy = 0.f, dhsz = 0.f;
        if (hok) {
            const float dd = dhx * hx + dhy * hy + dhz * hz;
            dhsx = (dhx - dd * hx) * rh;
            dhsy = (dhy - dd * hy) * rh;
            dhsz = (dhz - dd * hz) * rh;
        }
        const float dlix = dhsx, dliy = dhsy, dliz = dhsz + dfd * fd_norm * delu;
        const float dlox = dhsx, dloy = dhsy, dloz = dhsz;
        const float dR[9] = {dlix * wix + dlox * wox, dlix * wiy + dlox * woy, dlix * wiz + dlox * woz,
                             dliy * wix + dloy * wox, dliy * wiy + dloy * woy, dliy * wiz + dloy * woz,
                             dliz * wix + dloz * wox, dliz * wiy + dloz * woy, dliz * wiz + dloz * woz};
        float dq[4];
        quat_grad(qw, qx, qy, qz, qn, dR, dq);
        // world directions: R^T dl plus Psi's direct inputs
        const float* pw = a.rows + (size_t)kDwRow * n + g;
        const float dwx = R00 * dlix + R10 * dliy + R20 * dliz + pw[0];
        const float dwy = R01 * dlix + R11 * dliy + R21 * dliz + pw[(size_t)n];
        const float dwz = R02 * dlix + R12 * dliy + R22 * dliz + pw[(size_t)2 * n];
        const float dox = R00 * dlox + R10 * dloy + R20 * dloz + pw[(size_t)3 * n];
        const float doy = R01 * dlox + R11 * dloy + R21 * dloz + pw[(size_t)4 * n];
        const float doz = R02 * dlox + R12 * dloy + R22 * dloz + pw[(size_t)5 * n];
        // w = (p - mu)/|p - mu|: dmu = -(dw - (dw.w) w) / |p - mu|; a
        // directional light's w_i does not depend on mu
        const float wd = dwx * wix + dwy * wiy + dwz * wiz;
        const float od = dox * wox + doy * woy + doz * woz;
        const float rim = lm * ri;
        a.g.albedo[g] += dc0 * fd;
        a.g.albedo[n + g] += dc1 * fd;
        a.g.albedo[2 * n + g] += dc2 * fd;
        a.g.shade_rot[g] += dq[0];
        a.g.shade_rot[n + g] += dq[1];
        a.g.shade_rot[2 * n + g] += dq[2];
        a.g.shade_rot[3 * n + g] += dq[3];
        a.g.mean[g] += -(dwx - wd * wix) * rim - (dox - od * wox) * ro;
        a.g.mean[n + g] += -(dwy - wd * wiy) * rim - (doy - od * woy) * ro;
        a.g.mean[2 * n + g] += -(dwz - wd * wiz) * rim - (doz - od * woz) * ro;
    }
}

template <int PART>
__global__ __launch_bounds__(512, 4) void k_shade_bwd(ShadeBwdArgs a) {
    using L = BwdLds<PART>;
    __shared__ __align__(16) float sm[L::size];
    const SceneDev& sc = a.sc;
    const int n = sc.n;
    if (PART == 1 && a.use_phi) {
        load_mlp(sm, L::S, kPhiKR, kPhiIn, 1, a.phi);
        load_mlp_t(sm, L::T, kPhiIn, a.phi);
    }
    if (PART == 2 && a.use_psi) {
        load_mlp(sm, L::S, kPsiKR, kPsiIn, 3, a.psi);
        load_mlp_t(sm, L::T, kPsiIn, a.psi);
    }
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4, l16 = lane & 15;
    const int waves = blockDim.x >> 6;
    for (int base = (blockIdx.x * waves + w) * 16; base < n; base += gridDim.x * waves * 16) {
        // keeps the weight operands' LDS reads inside the loop: hoisted out of
        // it they would need several hundred registers
        asm volatile("" ::: "memory");
        const int g_raw = base + l16;
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        // ---- directions, Psi's inputs
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        const float lm = a.light_dir ? 0.f : 1.f;
        float wix = a.light[0] - lm * mx, wiy = a.light[1] - lm * my, wiz = a.light[2] - lm * mz;
        const float ri = rsqrtf(wix * wix + wiy * wiy + wiz * wiz);
        wix *= ri; wiy *= ri; wiz *= ri;
        float wox = a.eye[0] - mx, woy = a.eye[1] - my, woz = a.eye[2] - mz;
        const float ro = rsqrtf(wox * wox + woy * woy + woz * woz);
        wox *= ro; woy *= ro; woz *= ro;
        // ---- upstream gradients
        const float dtp = a.gcol[(size_t)3 * n + g];
        const float dr0 = a.gcol[(size_t)4 * n + g], dr1 = a.gcol[(size_t)5 * n + g], dr2 = a.gcol[(size_t)6 * n + g];
        // ---- Phi([T, feat]) adjoint
        const float Tg = a.T[g];
        float dTg = dtp;
        float phi_dx0[4] = {0.f, 0.f, 0.f, 0.f}, phi_dx1[4] = {0.f, 0.f, 0.f, 0.f};
        if (PART == 1 && a.use_phi) {
            floatx4 h[3][4];
            auto xin = [&](int k) -> float {
                if (k == 0) return Tg;
                if (k <= kFeat) return sc.feat[(size_t)(k - 1) * n + g];
                return 0.f;
            };
            mlp_hidden_all<kPhiKR>(sm, L::S, lane, xin, h);
            const float tp = mlp_out(sm, L::S, lane, h[2], 0);
            // the input goes to the scratch now; the adjoint needs only the
            // ReLU patterns of h (fewer live registers)
            if (valid) {
                float* R = a.rows;
                for (int k = q; k < kPhiIn; k += 4) R[(size_t)(kPhiRows.x + k) * n + g] = xin(k);
            }
            const uint32_t hmask[3] = {relu_mask(h[0]), relu_mask(h[1]), relu_mask(h[2])};
            const float d4 = dtp * tp * (1.f - tp);
            floatx4 dh3[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) dh3[m][i] = sm[L::S.w4 + 16 * m + 4 * q + i] * d4;
            floatx4 dx[2];
            mlp_backward_masked(sm, L::T, lane, hmask, dh3, [](int, const floatx4*) {}, dx);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                phi_dx0[i] = dx[0][i];
                phi_dx1[i] = dx[1][i];
            }
            if (valid && q == 0) a.rows[(size_t)kPhiRows.dout * n + g] = d4;
            // dL/dT = dx row 0 (tile 0, quarter 0, i = 0)
            dTg = __shfl(phi_dx0[0], l16, 64);
        }
        // ---- Psi([feat, w_i, w_o]) adjoint
        float psi_dx0[4] = {0.f, 0.f, 0.f, 0.f};
        float pdwx = 0.f, pdwy = 0.f, pdwz = 0.f, pdox = 0.f, pdoy = 0.f, pdoz = 0.f;
        if (PART == 2 && a.use_psi) {
            floatx4 h[3][4];
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
            mlp_hidden_all<kPsiKR>(sm, L::S, lane, xin, h);
            const float r0 = mlp_out(sm, L::S, lane, h[2], 0);
            const float r1 = mlp_out(sm, L::S, lane, h[2], 1);
            const float r2 = mlp_out(sm, L::S, lane, h[2], 2);
            if (valid) {
                float* R = a.rows;
                for (int k = q; k < kPsiIn; k += 4) R[(size_t)(kPsiRows.x + k) * n + g] = xin(k);
            }
            const uint32_t hmask[3] = {relu_mask(h[0]), relu_mask(h[1]), relu_mask(h[2])};
            const float d40 = dr0 * r0 * (1.f - r0), d41 = dr1 * r1 * (1.f - r1), d42 = dr2 * r2 * (1.f - r2);
            floatx4 dh3[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * m + 4 * q + i;
                    dh3[m][i] = fmaf(sm[L::S.w4 + r], d40,
                                     fmaf(sm[L::S.w4 + 64 + r], d41, sm[L::S.w4 + 128 + r] * d42));
                }
            floatx4 dx[2];
            mlp_backward_masked(sm, L::T, lane, hmask, dh3, [](int, const floatx4*) {}, dx);
#pragma unroll
            for (int i = 0; i < 4; ++i) psi_dx0[i] = dx[0][i];
            // rows 16..21 = w_i, w_o live in tile 1, quarters 0 and 1
            const float t10 = __shfl(dx[1][0], l16, 64), t11 = __shfl(dx[1][1], l16, 64);
            const float t12 = __shfl(dx[1][2], l16, 64), t13 = __shfl(dx[1][3], l16, 64);
            const float t20 = __shfl(dx[1][0], l16 + 16, 64), t21 = __shfl(dx[1][1], l16 + 16, 64);
            pdwx = t10; pdwy = t11; pdwz = t12; pdox = t13; pdoy = t20; pdoz = t21;
            if (valid) {
                float* R = a.rows;
                if (q == 0) {
                    R[(size_t)kPsiRows.dout * n + g] = d40;
                    R[(size_t)(kPsiRows.dout + 1) * n + g] = d41;
                    R[(size_t)(kPsiRows.dout + 2) * n + g] = d42;
                }
            }
        }
        // ---- features: Phi row r + 1 (PART 1) or Psi row r (PART 2) of dx
        // feeds feat r
        if (PART == 1 && a.use_phi) {
            const float up0 = __shfl(phi_dx0[0], l16 + 16 * ((q + 1) & 3), 64);
            const float up1 = __shfl(phi_dx1[0], l16, 64);
            const float nxt = q < 3 ? up0 : up1;
            if (valid) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    a.g.feat[(size_t)(4 * q + i) * n + g] += i < 3 ? phi_dx0[i + 1] : nxt;
            }
        }
        if (PART == 2 && a.use_psi && valid) {
#pragma unroll
            for (int i = 0; i < 4; ++i) a.g.feat[(size_t)(4 * q + i) * n + g] += psi_dx0[i];
        }
        // ---- dT (PART 1); Psi's direction gradients for k_shade_bwd_geom
        // (PART 2)
        if (valid && q == 0) {
            if (PART == 1) a.dT[g] = dTg;
            if (PART == 2) {
                float* pw = a.rows + (size_t)kDwRow * n + g;
                pw[0] = pdwx;
                pw[(size_t)n] = pdwy;
                pw[(size_t)2 * n] = pdwz;
                pw[(size_t)3 * n] = pdox;
                pw[(size_t)4 * n] = pdoy;
                pw[(size_t)5 * n] = pdoz;
            }
        }
    }
}

// --------------------------------------------------------------------------
// MLP weight gradients from stored rows: dW_l = sum_g dz_l[:, g] in_l[:, g]^T
// and db_l = sum_g dz_l[:, g] over all Gaussians, as split-K partial sums
// (one workgroup per (chunk of Gaussians, layer)) and one reduction. The
// basis appearance's MLPs use this (their adjoint stores every layer's
// input and gradient); the lobes model's are recomputed by k_mlp_wgrad
// below, which shares the reduction.

constexpr int kWgChunk = kWgChunkHost;

struct WgProblem {
    int dz_row, in_row, O, J, off;   // scratch rows, output/input widths, offset in the flat vector
    int ldw;                         // row stride of dW
    float* dW;                       // [O][ldw] +=
    float* db;                       // [O] += (NULL: bias not accumulated by this problem)
};
constexpr int kWgMaxProblems = 16;
struct WgArgs {
    WgProblem p[kWgMaxProblems];
    int count, total;                // problems, flat parameter count
    const float* rows;
    int n;
    float* partial;                  // [chunks][total]
};

// One workgroup per (chunk of Gaussians, problem): C[O x J] = D[O x chunk] .
// H[J x chunk]^T on mfma_f32_16x16x4f32, the Gaussians being the
// contraction, for O, J <= R (R = 64 or 128). The chunk goes through LDS 32
// Gaussians at a time (zero padded to R x R); wave w owns output rows
// R/4 w .. R/4 w + R/4 - 1 (R/64 tiles of 16 rows) and all R/16 column
// blocks. A-operand lane l: D[row0 + l % 16][4s + l / 16]; B-operand lane l:
// H[16c + l % 16][4s + l / 16]; the result lane l holds rows
// row0 + 4 (l / 16) + i, column 16c + l % 16. Bias sums come from the same
// D tile.
template <int R>
__global__ __launch_bounds__(256) void k_wgrad(WgArgs a) {
    constexpr int KB = 32;
    constexpr int RT = R / 64;        // row tiles per wave
    constexpr int CB = R / 16;        // column blocks
    __shared__ float sD[R][KB + 1];
    __shared__ float sH[R][KB + 1];
    // workgroup = chunk * count + problem: the problems of one chunk, which
    // share its rows, run side by side and meet them in the caches
    const int chunk = blockIdx.x / a.count;
    const WgProblem P = a.p[blockIdx.x - chunk * a.count];
    const int n = a.n;
    const int k0 = chunk * kWgChunk, k1 = min(n, k0 + kWgChunk);
    const float* D = a.rows + (size_t)P.dz_row * n;
    const float* H = a.rows + (size_t)P.in_row * n;
    const int t = threadIdx.x, lane = __lane_id();
    const int w = t >> 6, r16 = lane & 15, kq = lane >> 4;
    floatx4 acc[RT][CB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[rt][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bacc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) bacc[rt] = 0.f;
    // the next tile's loads are in flight while the current one is multiplied
    constexpr int kPer = R * KB / 256;
    float pd[kPer], ph[kPer];
    auto fetch = [&](int kb) {
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const int idx = t + 256 * m, r = idx / KB, gg = kb + idx % KB;
            pd[m] = (r < P.O && gg < k1) ? D[(size_t)r * n + gg] : 0.f;
            ph[m] = (r < P.J && gg < k1) ? H[(size_t)r * n + gg] : 0.f;
        }
    };
    if (k0 < k1) fetch(k0);
    for (int kb = k0; kb < k1; kb += KB) {
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const int idx = t + 256 * m;
            sD[idx / KB][idx % KB] = pd[m];
            sH[idx / KB][idx % KB] = ph[m];
        }
        __syncthreads();
        if (kb + KB < k1) fetch(kb + KB);
#pragma unroll
        for (int s4 = 0; s4 < KB / 4; ++s4) {
            float av[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                av[rt] = sD[(R / 4) * w + 16 * rt + r16][4 * s4 + kq];
                bacc[rt] += av[rt];
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const float bv = sH[16 * c + r16][4 * s4 + kq];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt], bv, acc[rt][c], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float* part = a.partial + (size_t)chunk * a.total + P.off;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int row0 = (R / 4) * w + 16 * rt;
        // bias: lanes r16, r16 + 16, r16 + 32, r16 + 48 hold row row0 + r16
        float bs = bacc[rt];
        bs += __shfl_xor(bs, 16, 64);
        bs += __shfl_xor(bs, 32, 64);
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int j = 16 * c + r16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = row0 + 4 * kq + i;
                if (o < P.O && j < P.J) part[o * P.J + j] = acc[rt][c][i];
            }
        }
        if (kq == 0 && row0 + r16 < P.O) part[P.O * P.J + row0 + r16] = bs;
    }
}

// Sum of the per-chunk partials of 64 consecutive parameters per
// workgroup: each of the four waves takes every fourth chunk with eight
// loads in flight, then one wave adds the four wave sums (fixed order, so
// the result is deterministic).
__global__ __launch_bounds__(256) void k_wgrad_reduce(WgArgs a, int chunks) {
    __shared__ float s_part[4][64];
    const int lp = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lp;
    float s = 0.f;
    if (p < a.total) {
        const float* src = a.partial + p;
        const size_t ld = (size_t)a.total;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int c = grp;
        for (; c + 28 < chunks; c += 32) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += src[(size_t)(c + 4 * u) * ld];
        }
        for (; c < chunks; c += 4) acc[0] += src[(size_t)c * ld];
        s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    }
    s_part[grp][lp] = s;
    __syncthreads();
    if (grp != 0 || p >= a.total) return;
    s = (s_part[0][lp] + s_part[1][lp]) + (s_part[2][lp] + s_part[3][lp]);
    for (int i = 0; i < a.count; ++i) {
        const WgProblem& P = a.p[i];
        const int rel = p - P.off;
        if (rel >= 0 && rel < P.O * P.J) {
            P.dW[(size_t)(rel / P.J) * P.ldw + rel % P.J] += s;
            return;
        }
        if (rel >= P.O * P.J && rel < P.O * P.J + P.O) {
            if (P.db) P.db[rel - P.O * P.J] += s;
            return;
        }
    }
}

// --------------------------------------------------------------------------
// Weight gradients of Phi and Psi from the small scratch: one workgroup per
// (run of Gaussians, MLP), 8 waves of 16 Gaussians per step. Each wave
// recomputes its Gaussians' hidden activations with the forward's split
// half-precision products (the same routine as the shading adjoint, so the
// same ReLU patterns) and the hidden pre-activation gradients from the
// output-layer gradient on float32 products; the workgroup stages each
// layer's gradient and input for its 128 Gaussians in LDS and adds
// dW_l += dZ_l IN_l^T (Gaussians as the contraction) on
// mfma_f32_16x16x4f32. The per-workgroup sums go to the partial buffer in
// the layout k_wgrad_reduce sums (per layer: O x J weights, then O biases).

constexpr int kWgGroup = 128;          // Gaussians per step (8 waves x 16)
constexpr int kWgLd = kWgGroup + 4;    // staging row stride (floats)

struct MlpWgArgs {
    MlpArgs m[2];                      // Phi, Psi
    int mlp[2];                        // blockIdx.y -> 0 (Phi) or 1 (Psi)
    int off[2];                        // each MLP's first parameter in the flat partial vector
    const float* rows;                 // [kMlpRows][n]
    int n;
    int total;                         // flat parameter count (partial row length)
    float* partial;                    // [gridDim.x][total]
};

constexpr int mlp_wgrad_smem(int kr, int n_out) {
    return mlp_smem(0, kr, n_out).size + mlp_tsmem(0).size + 2 * 64 * kWgLd;
}
constexpr int kMlpWgSmem = mlp_wgrad_smem(kPhiKR, 1) > mlp_wgrad_smem(kPsiKR, 3) ? mlp_wgrad_smem(kPhiKR, 1)
                                                                                     : mlp_wgrad_smem(kPsiKR, 3);
static_assert(kMlpWgSmem * 4 <= 160 * 1024, "weight-gradient LDS exceeds 160 KiB");
static_assert(kWgLd % 4 == 0 && kWgGroup == 128, "staging rows are read as 16-byte vectors, 32 Gaussians per lane group");

// acc += DZ[row0 .. +15][0 .. 127] . IN[col0 .. +15][0 .. 127]^T; rows at
// or past o_rows read as 0; bias (when given) += the lane's DZ values.
__device__ inline void wg_tile(const float* dz, const float* in, int row0, int col0, int o_rows, int lane,
                               floatx4* acc, float* bias) {
    // lane group kq takes the Gaussians 32 kq .. 32 kq + 31, four per
    // 16-byte read
    const int r16 = lane & 15, kq = lane >> 4;
    const bool row_ok = row0 + r16 < o_rows;
    const float4* pa = reinterpret_cast<const float4*>(dz + (row0 + r16) * kWgLd + 32 * kq);
    const float4* pb = reinterpret_cast<const float4*>(in + (col0 + r16) * kWgLd + 32 * kq);
    float bs = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float4 av = row_ok ? pa[u] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 bv = pb[u];
        bs += (av.x + av.y) + (av.z + av.w);
        *acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, *acc, 0, 0, 0);
        *acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, *acc, 0, 0, 0);
        *acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, *acc, 0, 0, 0);
        *acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, *acc, 0, 0, 0);
    }
    if (bias) *bias += bs;
}

// The workgroup's sums of one layer (O x J weights at P, then O biases)
// into its partial row; lane layout of wg_tile's result.
__device__ inline void wg_store(float* P, int O, int J, int row0, int col0, int lane, const floatx4& acc,
                                const float* bias) {
    const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = row0 + 4 * kq + i, j = col0 + r16;
        if (o < O && j < J) P[o * J + j] = acc[i];
    }
    if (bias) {
        float b = *bias;
        b += __shfl_xor(b, 16, 64);
        b += __shfl_xor(b, 32, 64);
        if (kq == 0 && row0 + r16 < O) P[O * J + row0 + r16] = b;
    }
}

template <int KR, int N_IN, int N_OUT>
__device__ inline void mlp_wgrad(float* sm, const MlpArgs& mw, const float* rows, int n, MlpRows R, float* part) {
    constexpr MlpSmem S = mlp_smem(0, KR, N_OUT);
    constexpr MlpTSmem T = mlp_tsmem(S.size);
    constexpr int kDz = S.size + T.size, kIn = kDz + 64 * kWgLd;
    static_assert(N_IN <= 32 && N_OUT <= 16, "input rows are staged as two 16-row tiles, outputs as one");
    load_mlp(sm, S, KR, N_IN, N_OUT, mw);
    load_mlp_t(sm, T, N_IN, mw);
    __syncthreads();
    float* sdz = sm + kDz;
    float* sin_ = sm + kIn;
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4, l16 = lane & 15;
    const int col = 16 * w + l16;   // the lane's Gaussian in the staging tiles
    // accumulators: layer 0 one tile (rows 16 (w/2), input cols 16 (w%2));
    // layers 1, 2 tiles w and w + 8 of the 4 x 4 grid; layer 3 (waves 0-3)
    // output rows 0..15, hidden cols 16 w
    floatx4 a0 = {0.f, 0.f, 0.f, 0.f}, a1[2], a2[2], a3 = {0.f, 0.f, 0.f, 0.f};
    float b0 = 0.f, b1[2] = {0.f, 0.f}, b2[2] = {0.f, 0.f}, b3 = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t) a1[t] = a2[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto put = [&](float* tile, const floatx4 v[4]) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) tile[(16 * m + 4 * q + i) * kWgLd + col] = v[m][i];
    };
    for (int base = blockIdx.x * kWgGroup; base < n; base += gridDim.x * kWgGroup) {
        asm volatile("" ::: "memory");
        const int g_raw = base + col;
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        auto xin = [&](int k) -> float { return k < N_IN ? rows[(size_t)(R.x + k) * n + g] : 0.f; };
        floatx4 h[3][4];
        mlp_hidden_all<KR>(sm, S, lane, xin, h);
        // output-layer gradient (0 for the padding Gaussians), and dL/dh3 as
        // the shading adjoint forms it
        float d4[N_OUT];
#pragma unroll
        for (int o = 0; o < N_OUT; ++o) d4[o] = valid ? rows[(size_t)(R.dout + o) * n + g] : 0.f;
        floatx4 dh3[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * m + 4 * q + i;
                float v = sm[S.w4 + (N_OUT - 1) * 64 + r] * d4[N_OUT - 1];
#pragma unroll
                for (int o = N_OUT - 2; o >= 0; --o) v = fmaf(sm[S.w4 + o * 64 + r], d4[o], v);
                dh3[m][i] = v;
            }
        // layer 3: dW4 = d4 h3^T
        put(sin_, h[2]);
        if (q == 0) {
#pragma unroll
            for (int o = 0; o < N_OUT; ++o) sdz[o * kWgLd + col] = d4[o];
        }
        __syncthreads();
        if (w < 4) wg_tile(sdz, sin_, 0, 16 * w, N_OUT, lane, &a3, w == 0 ? &b3 : nullptr);
        __syncthreads();
        // hidden layers, last to first: dz_l gated by the forward's ReLU
        // pattern, staged with the layer's input
        floatx4 dz[4], d[4];
        auto gate = [&](const floatx4 hl[4], const floatx4 in[4]) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) dz[m][i] = hl[m][i] > 0.f ? in[m][i] : 0.f;
        };
        gate(h[2], dh3);
        put(sdz, dz);
        put(sin_, h[1]);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int tt = w + 8 * t;
            wg_tile(sdz, sin_, 16 * (tt >> 2), 16 * (tt & 3), 64, lane, &a2[t], (tt & 3) == 0 ? &b2[t] : nullptr);
        }
        __syncthreads();
        mlp_back_layer<4>(sm, T.t3, lane, dz, d);
        gate(h[1], d);
        put(sdz, dz);
        put(sin_, h[0]);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int tt = w + 8 * t;
            wg_tile(sdz, sin_, 16 * (tt >> 2), 16 * (tt & 3), 64, lane, &a1[t], (tt & 3) == 0 ? &b1[t] : nullptr);
        }
        __syncthreads();
        mlp_back_layer<4>(sm, T.t2, lane, dz, d);
        gate(h[0], d);
        put(sdz, dz);
        // the input rows 0..31 (0 past N_IN)
#pragma unroll
        for (int t = 0; t < 8; ++t) sin_[(4 * t + q) * kWgLd + col] = xin(4 * t + q);
        __syncthreads();
        wg_tile(sdz, sin_, 16 * (w >> 1), 16 * (w & 1), 64, lane, &a0, (w & 1) == 0 ? &b0 : nullptr);
        __syncthreads();
    }
    // partial sums, per layer: O x J weights then O biases
    constexpr int o1 = 64 * N_IN + 64, o2 = o1 + 64 * 64 + 64, o3 = o2 + 64 * 64 + 64;
    wg_store(part, 64, N_IN, 16 * (w >> 1), 16 * (w & 1), lane, a0, (w & 1) == 0 ? &b0 : nullptr);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int tt = w + 8 * t;
        wg_store(part + o1, 64, 64, 16 * (tt >> 2), 16 * (tt & 3), lane, a1[t], (tt & 3) == 0 ? &b1[t] : nullptr);
        wg_store(part + o2, 64, 64, 16 * (tt >> 2), 16 * (tt & 3), lane, a2[t], (tt & 3) == 0 ? &b2[t] : nullptr);
    }
    if (w < 4) wg_store(part + o3, N_OUT, 64, 0, 16 * w, lane, a3, w == 0 ? &b3 : nullptr);
}

__global__ __launch_bounds__(512) void k_mlp_wgrad(MlpWgArgs a) {
    __shared__ __align__(16) float sm[kMlpWgSmem];
    const int which = a.mlp[blockIdx.y];
    float* part = a.partial + (size_t)blockIdx.x * a.total + a.off[which];
    if (which == 0)
        mlp_wgrad<kPhiKR, kPhiIn, 1>(sm, a.m[0], a.rows, a.n, kPhiRows, part);
    else
        mlp_wgrad<kPsiKR, kPsiIn, 3>(sm, a.m[1], a.rows, a.n, kPsiRows, part);
}

// --------------------------------------------------------------------------
// Projection adjoint (both views), in double like the forward projection.

struct ProjBwdArgs {
    SceneDev sc;
    ViewParams v[2];          // camera, light
    const float* gs[2];       // [6][n] {u, v, A, B, C, opacity} per view
    gs3_consts kc;
    GradDev g;
};

__global__ __launch_bounds__(256) void k_project_bwd(ProjBwdArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.sc.n;
    if (i >= n) return;
    const SceneDev& sc = a.sc;
    const double mx = sc.mean[i], my = sc.mean[n + i], mz = sc.mean[2 * n + i];
    const double s[3] = {exp((double)sc.log_scale[i]), exp((double)sc.log_scale[n + i]),
                         exp((double)sc.log_scale[2 * n + i])};
    double qw = sc.rot[i], qx = sc.rot[n + i], qy = sc.rot[2 * n + i], qz = sc.rot[3 * n + i];
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                         2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                         2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = R[3 * r + c] * s[c];
    double gmean[3] = {0, 0, 0}, gM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gop = 0.0;
    for (int vi = 0; vi < 2; ++vi) {
        const float* G = a.gs[vi];
        const double gu = G[i], gv = G[(size_t)n + i], gA = G[(size_t)2 * n + i], gB = G[(size_t)3 * n + i],
                     gC = G[(size_t)4 * n + i];
        gop += G[(size_t)5 * n + i];
        if (gu == 0.0 && gv == 0.0 && gA == 0.0 && gB == 0.0 && gC == 0.0) continue;
        const ViewParams& vp = a.v[vi];
        const double dx = mx - vp.eye[0], dy = my - vp.eye[1], dz = mz - vp.eye[2];
        const double tx = vp.R[0] * dx + vp.R[1] * dy + vp.R[2] * dz;
        const double ty = vp.R[3] * dx + vp.R[4] * dy + vp.R[5] * dz;
        const double tz = vp.R[6] * dx + vp.R[7] * dy + vp.R[8] * dz;
        if (!(tz > (double)a.kc.near_plane)) continue;
        const double f = vp.focal;
        const bool ortho = vp.ortho != 0;
        const double xs = tx / tz, ys = ty / tz;
        const bool cx_ = xs < -vp.lim_x || xs > vp.lim_x, cy_ = ys < -vp.lim_y || ys > vp.lim_y;
        const double xr = fmin(fmax(xs, -vp.lim_x), vp.lim_x);
        const double yr = fmin(fmax(ys, -vp.lim_y), vp.lim_y);
        // J of the forward projection: pinhole, or the constant scale of a
        // parallel projection (no dependence on the position)
        const double j0 = ortho ? vp.scale : f / tz;
        const double j2x = ortho ? 0.0 : -f * xr / tz, j2y = ortho ? 0.0 : -f * yr / tz;
        double A[6];
        for (int c = 0; c < 3; ++c) {
            A[c] = j0 * vp.R[c] + j2x * vp.R[6 + c];
            A[3 + c] = j0 * vp.R[3 + c] + j2y * vp.R[6 + c];
        }
        double B[6];
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 3; ++k)
                B[3 * r + k] = A[3 * r] * M[k] + A[3 * r + 1] * M[3 + k] + A[3 * r + 2] * M[6 + k];
        const double ca = B[0] * B[0] + B[1] * B[1] + B[2] * B[2] + (double)a.kc.dilation;
        const double cb = B[0] * B[3] + B[1] * B[4] + B[2] * B[5];
        const double cc = B[3] * B[3] + B[4] * B[4] + B[5] * B[5] + (double)a.kc.dilation;
        const double det = ca * cc - cb * cb;
        if (!(det > 0.0)) continue;
        // (A, B, C) of the kernels -> conic (a, b, c) -> Sigma' entries
        const double ga = gA * (-0.5 * (double)kLog2eF), gb = gB * (-(double)kLog2eF), gc = gC * (-0.5 * (double)kLog2eF);
        const double id = 1.0 / det, id2 = id * id;
        const double gca = ga * (-cc * cc) * id2 + gb * (cb * cc) * id2 + gc * (id - ca * cc * id2);
        const double gcc = ga * (id - cc * ca * id2) + gb * (cb * ca) * id2 + gc * (-ca * ca) * id2;
        const double gcb = ga * (2.0 * cc * cb) * id2 + gb * (-id - 2.0 * cb * cb * id2) + gc * (2.0 * ca * cb) * id2;
        double gB_[6];
        for (int k = 0; k < 3; ++k) {
            gB_[k] = 2.0 * gca * B[k] + gcb * B[3 + k];
            gB_[3 + k] = gcb * B[k] + 2.0 * gcc * B[3 + k];
        }
        double gA_[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                gA_[3 * r + c] = gB_[3 * r] * M[3 * c] + gB_[3 * r + 1] * M[3 * c + 1] + gB_[3 * r + 2] * M[3 * c + 2];
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) gM[3 * c + k] += A[c] * gB_[k] + A[3 + c] * gB_[3 + k];
        double gj0 = 0.0, gj2x = 0.0, gj2y = 0.0;
        for (int c = 0; c < 3; ++c) {
            gj0 += gA_[c] * vp.R[c] + gA_[3 + c] * vp.R[3 + c];
            gj2x += gA_[c] * vp.R[6 + c];
            gj2y += gA_[3 + c] * vp.R[6 + c];
        }
        double gtx = 0.0, gty = 0.0, gtz = 0.0;
        if (ortho) {
            // u = s t_x + cx, v = s t_y + cy; J constant
            gtx = gu * vp.scale;
            gty = gv * vp.scale;
            for (int c = 0; c < 3; ++c) gmean[c] += vp.R[c] * gtx + vp.R[3 + c] * gty;
            continue;
        }
        gtz += gj0 * (-f / (tz * tz));
        if (cx_) {
            gtz += gj2x * (f * xr / (tz * tz));
        } else {
            gtx += gj2x * (-f / (tz * tz));
            gtz += gj2x * (2.0 * f * tx / (tz * tz * tz));
        }
        if (cy_) {
            gtz += gj2y * (f * yr / (tz * tz));
        } else {
            gty += gj2y * (-f / (tz * tz));
            gtz += gj2y * (2.0 * f * ty / (tz * tz * tz));
        }
        gtx += gu * f / tz;
        gtz += -gu * f * tx / (tz * tz);
        gty += gv * f / tz;
        gtz += -gv * f * ty / (tz * tz);
        for (int c = 0; c < 3; ++c) gmean[c] += vp.R[c] * gtx + vp.R[3 + c] * gty + vp.R[6 + c] * gtz;
    }
    // M = R diag(s)
    double gR[9], gls[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            gR[3 * r + c] = gM[3 * r + c] * s[c];
            gls[c] += gM[3 * r + c] * R[3 * r + c] * s[c];
        }
    const double dw = 2.0 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    const double dxq = 2.0 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.0 * qx * gR[4] - qw * gR[5] + qz * gR[6] +
                              qw * gR[7] - 2.0 * qx * gR[8]);
    const double dyq = 2.0 * (-2.0 * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] +
                              qz * gR[7] - 2.0 * qy * gR[8]);
    const double dzq = 2.0 * (-2.0 * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.0 * qz * gR[4] +
                              qy * gR[5] + qx * gR[6] + qy * gR[7]);
    const double dot = dw * qw + dxq * qx + dyq * qy + dzq * qz;
    const double logit = sc.opacity_logit[i];
    const double op = 1.0 / (1.0 + exp(-logit));
    a.g.mean[i] += (float)gmean[0];
    a.g.mean[n + i] += (float)gmean[1];
    a.g.mean[2 * n + i] += (float)gmean[2];
    a.g.log_scale[i] += (float)gls[0];
    a.g.log_scale[n + i] += (float)gls[1];
    a.g.log_scale[2 * n + i] += (float)gls[2];
    a.g.rot[i] += (float)((dw - dot * qw) / qn);
    a.g.rot[n + i] += (float)((dxq - dot * qx) / qn);
    a.g.rot[2 * n + i] += (float)((dyq - dot * qy) / qn);
    a.g.rot[3 * n + i] += (float)((dzq - dot * qz) / qn);
    a.g.opacity_logit[i] += (float)(gop * op * (1.0 - op));
}

// --------------------------------------------------------------------------

int wgrad_total_params(bool phi, bool psi) {
    int t = 0;
    if (phi) t += 64 * kPhiIn + 64 + 2 * (64 * 64 + 64) + 64 + 1;
    if (psi) t += 64 * kPsiIn + 64 + 2 * (64 * 64 + 64) + 3 * 64 + 3;
    return t;
}

hipError_t launch_shade_bwd(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                            const gs3_mlp* psi, const float* gcol, float* dT, const GradDev& g, float* rows,
                            float* partial, const gs3_grads* gr, hipStream_t st) {
    if (sc.n == 0) return hipSuccess;
    ShadeBwdArgs a;
    a.sc = sc;
    for (int i = 0; i < 3; ++i) {
        a.light[i] = sp.light[i];
        a.eye[i] = sp.eye[i];
    }
    a.use_phi = phi != nullptr;
    a.use_psi = psi != nullptr;
    a.light_dir = sp.light_dir;
    a.T = T;
    for (int i = 0; i < 4; ++i) {
        a.phi.w[i] = phi ? phi->w[i] : nullptr;
        a.phi.b[i] = phi ? phi->b[i] : nullptr;
        a.psi.w[i] = psi ? psi->w[i] : nullptr;
        a.psi.b[i] = psi ? psi->b[i] : nullptr;
    }
    a.gcol = gcol;
    a.dT = dT;
    a.g = g;
    a.rows = rows;
    // each MLP's adjoint in its own launch with half the LDS: two 512-thread
    // workgroups per CU (four waves per SIMD, 128 registers each)
    const int per_block = 8 * 16;
    int grid = (int)((sc.n + per_block - 1) / per_block);
    if (grid > 512) grid = 512;
    hipLaunchKernelGGL(k_shade_bwd<1>, dim3(grid), dim3(512), 0, st, a);
    hipLaunchKernelGGL(k_shade_bwd<2>, dim3(grid), dim3(512), 0, st, a);
    const int64_t gl = (sc.n + 255) / 256;
    hipLaunchKernelGGL(k_shade_bwd_geom, dim3((unsigned)(gl < 2048 ? gl : 2048)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || (!phi && !psi)) return e;
    // weight gradients: per-workgroup partial sums, then one fixed-order
    // reduction into the gradient buffers
    MlpWgArgs wa;
    WgArgs ra;
    int ny = 0, off = 0;
    ra.count = 0;
    auto add_mlp = [&](int which, const gs3_mlp* m, int n_in, int n_out, float* const* gw, float* const* gb) {
        for (int i = 0; i < 4; ++i) {
            wa.m[which].w[i] = m->w[i];
            wa.m[which].b[i] = m->b[i];
        }
        wa.mlp[ny++] = which;
        wa.off[which] = off;
        const int O[4] = {64, 64, 64, n_out}, J[4] = {n_in, 64, 64, 64};
        for (int l = 0; l < 4; ++l) {
            WgProblem& P = ra.p[ra.count++];
            P.dz_row = P.in_row = 0;
            P.O = O[l];
            P.J = J[l];
            P.off = off;
            P.ldw = J[l];
            P.dW = gw[l];
            P.db = gb[l];
            off += O[l] * J[l] + O[l];
        }
    };
    if (phi) add_mlp(0, phi, kPhiIn, 1, gr->phi_w, gr->phi_b);
    if (psi) add_mlp(1, psi, kPsiIn, 3, gr->psi_w, gr->psi_b);
    ra.total = wa.total = off;
    ra.rows = wa.rows = rows;
    ra.n = wa.n = sc.n;
    ra.partial = wa.partial = partial;
    // one run of Gaussians per workgroup and MLP; at most as many runs as
    // the partial buffer has rows (one per kWgChunk Gaussians)
    const int chunks = (sc.n + kWgChunk - 1) / kWgChunk;
    const int runs = chunks < 128 ? chunks : 128;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(runs, ny), dim3(512), 0, st, wa);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((ra.total + 63) / 64), dim3(256), 0, st, ra, runs);
    return hipGetLastError();
}

int wgrad_partial_floats(const WgSpec* specs, int count) {
    int t = 0;
    for (int i = 0; i < count; ++i) t += specs[i].O * specs[i].J + specs[i].O;
    return t;
}

hipError_t launch_wgrad(const WgSpec* specs, int count, const float* rows, int n, float* partial, hipStream_t st) {
    if (count <= 0 || n <= 0) return hipSuccess;
    if (count > kWgMaxProblems) return hipErrorInvalidValue;
    WgArgs w;
    w.count = count;
    int off = 0;
    int widest = 0;
    for (int i = 0; i < count; ++i) {
        const WgSpec& S = specs[i];
        if (S.O > 128 || S.J > 128 || S.O <= 0 || S.J <= 0) return hipErrorInvalidValue;
        widest = max(widest, max(S.O, S.J));
        WgProblem& P = w.p[i];
        P.dz_row = S.dz_row; P.in_row = S.in_row; P.O = S.O; P.J = S.J; P.off = off;
        P.ldw = S.ldw; P.dW = S.dW; P.db = S.db;
        off += S.O * S.J + S.O;
    }
    w.total = off;
    w.rows = rows;
    w.n = n;
    w.partial = partial;
    const int chunks = (n + kWgChunk - 1) / kWgChunk;
    const dim3 grid(chunks * w.count);
    if (widest > 64)
        hipLaunchKernelGGL(k_wgrad<128>, grid, dim3(256), 0, st, w);
    else
        hipLaunchKernelGGL(k_wgrad<64>, grid, dim3(256), 0, st, w);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((w.total + 63) / 64), dim3(256), 0, st, w, chunks);
    return hipGetLastError();
}

hipError_t launch_project_bwd(const SceneDev& sc, const ViewParams& cam, const ViewParams& light,
                              const gs3_consts& k, const float* gcam, const float* glight, const GradDev& g,
                              hipStream_t st) {
    if (sc.n == 0) return hipSuccess;
    ProjBwdArgs a;
    a.sc = sc;
    a.v[0] = cam;
    a.v[1] = light;
    a.gs[0] = gcam;
    a.gs[1] = glight;
    a.kc = k;
    a.g = g;
    hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)((sc.n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace gs3
