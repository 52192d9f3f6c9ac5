// Per-Gaussian appearance: the first splat (Sec. 4.1, Eq. 4-7), the shadow
// refinement MLP Phi (Sec. 4.2, Eq. 8) and the residual MLP Psi (Sec. 4.3).
//
// A wave handles 16 Gaussians, four lanes per Gaussian: lane l works on
// Gaussian l % 16 and lobe quarter q = l / 16 (lobes q, q+4, ...), which is
// exactly the operand layout of v_mfma_f32_16x16x4_f32. The MLPs are
// evaluated transposed, H^T = W X^T, so Gaussians are the N dimension:
//   B operand of k-step kk: lane l supplies X[g = l%16][4 kk + l/16]
//   A operand: W[16 mt + l%16][4 kk + l/16]
//   D: lane l holds H^T[16 mt + 4 (l/16) + i][l%16], i = 0..3.
// Because the contraction order over the hidden index is free, the D
// registers of one layer are fed directly as the B operand of the next
// (k-step (m, i) <-> hidden 16 m + 4 (l/16) + i) and the weights are packed
// in LDS in that permuted order, so no transposes are needed between layers.
// The one- and three-wide output layers run on the VALU (16 FMAs per lane
// and a cross-lane sum over the four quarters).
#include "gs3_internal.h"

namespace gs3 {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kPhiIn = 1 + kFeat;        // [T, feat]
constexpr int kPsiIn = kFeat + 6;        // [feat, w_i, w_o]
constexpr int kPhiK1 = (kPhiIn + 3) / 4; // k-steps of the input layer
constexpr int kPsiK1 = (kPsiIn + 3) / 4;
// LDS layout (floats) of one packed MLP
constexpr int kLH = 4 * 16 * 64;          // a 64x64 hidden layer
struct MlpSmem {
    int l1, l2, l3, w4, b1, b2, b3, b4, size;
};
__host__ __device__ constexpr MlpSmem mlp_smem(int base, int k1, int n_out) {
    return MlpSmem{base,
                   base + 4 * k1 * 64,
                   base + 4 * k1 * 64 + kLH,
                   base + 4 * k1 * 64 + 2 * kLH,
                   base + 4 * k1 * 64 + 2 * kLH + n_out * 64,
                   base + 4 * k1 * 64 + 2 * kLH + n_out * 64 + 64,
                   base + 4 * k1 * 64 + 2 * kLH + n_out * 64 + 128,
                   base + 4 * k1 * 64 + 2 * kLH + n_out * 64 + 192,
                   4 * k1 * 64 + 2 * kLH + n_out * 64 + 192 + 4};
}
constexpr MlpSmem kPhiS = mlp_smem(0, kPhiK1, 1);
constexpr MlpSmem kPsiS = mlp_smem(kPhiS.size, kPsiK1, 3);
constexpr int kShadeSmem = kPhiS.size + kPsiS.size;

struct MlpArgs {
    const float* w[4];
    const float* b[4];
};

struct ShadeArgs {
    SceneDev sc;
    float light[3];
    float eye[3];
    int use_phi, use_psi;
    const float* T;
    MlpArgs phi, psi;
    float4* col0;
    float4* col1;
    float* colour;   // [8][n]
};

// Copy one MLP into LDS in the permuted A-operand order.
__device__ inline void load_mlp(float* sm, const MlpSmem& S, int k1, int n_in, int n_out, const MlpArgs& m) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < 4 * k1 * 64; idx += nt) {
        const int mt = idx / (k1 * 64), rem = idx % (k1 * 64), kk = rem / 64, l = rem % 64;
        const int row = 16 * mt + (l & 15), col = 4 * kk + (l >> 4);
        sm[S.l1 + idx] = col < n_in ? m.w[0][row * n_in + col] : 0.f;
    }
    for (int idx = tid; idx < kLH; idx += nt) {
        const int mt = idx / 1024, rem = idx % 1024, ks = rem / 64, l = rem % 64;
        const int row = 16 * mt + (l & 15), col = 16 * (ks >> 2) + 4 * (l >> 4) + (ks & 3);
        sm[S.l2 + idx] = m.w[1][row * kHidden + col];
        sm[S.l3 + idx] = m.w[2][row * kHidden + col];
    }
    for (int idx = tid; idx < n_out * 64; idx += nt) sm[S.w4 + idx] = m.w[3][idx];
    for (int idx = tid; idx < 64; idx += nt) {
        sm[S.b1 + idx] = m.b[0][idx];
        sm[S.b2 + idx] = m.b[1][idx];
        sm[S.b3 + idx] = m.b[2][idx];
    }
    for (int idx = tid; idx < n_out; idx += nt) sm[S.b4 + idx] = m.b[3][idx];
}

__device__ inline float relu(float x) { return fmaxf(x, 0.f); }

// Three hidden layers on MFMA; returns the last hidden activations in D
// layout (h[m][i] = hidden 16 m + 4 q + i of Gaussian l % 16).
template <int K1, typename InFn>
__device__ inline void mlp_hidden(const float* sm, const MlpSmem& S, int lane, InFn x_of_k, floatx4 h[4]) {
    const int q = lane >> 4;
    floatx4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < K1; ++kk) {
        const float bx = x_of_k(4 * kk + q);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sm[S.l1 + (mt * K1 + kk) * 64 + lane], bx, acc[mt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mt][i] = relu(acc[mt][i] + sm[S.b1 + 16 * mt + 4 * q + i]);
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const int wl = layer == 0 ? S.l2 : S.l3;
        const int bl = layer == 0 ? S.b2 : S.b3;
        floatx4 nxt[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) nxt[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ks = 4 * m + i;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    nxt[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sm[wl + (mt * 16 + ks) * 64 + lane], acc[m][i],
                                                                   nxt[mt], 0, 0, 0);
            }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[mt][i] = relu(nxt[mt][i] + sm[bl + 16 * mt + 4 * q + i]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) h[mt] = acc[mt];
}

// Output unit o: sigmoid(w4[o] . h + b4[o]), summed over the lane quarters.
__device__ inline float mlp_out(const float* sm, const MlpSmem& S, int lane, const floatx4 h[4], int o) {
    const int q = lane >> 4;
    float part = 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) part = fmaf(sm[S.w4 + o * 64 + 16 * m + 4 * q + i], h[m][i], part);
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    const float z = part + sm[S.b4 + o];
    return 1.f / (1.f + expf(-z));
}

__global__ __launch_bounds__(512) void k_shade_mlp(ShadeArgs a) {
    __shared__ float sm[kShadeSmem];
    const SceneDev& sc = a.sc;
    const int n = sc.n;
    if (a.use_phi) load_mlp(sm, kPhiS, kPhiK1, kPhiIn, 1, a.phi);
    if (a.use_psi) load_mlp(sm, kPsiS, kPsiK1, kPsiIn, 3, a.psi);
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4;
    const int waves = blockDim.x >> 6;
    const float kd = 0.01f * (1.f - 0.36787944117144233f);   // eps (1 - 1/e), Eq. 5
    const float fd_norm = 1.f / ((1.f + kd) * 3.14159265358979f);
    for (int base = (blockIdx.x * waves + w) * 16; base < n; base += gridDim.x * waves * 16) {
        const int g_raw = base + (lane & 15);
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        // ---- shading (Eq. 4-7)
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        float wix = a.light[0] - mx, wiy = a.light[1] - my, wiz = a.light[2] - mz;
        float r = rsqrtf(wix * wix + wiy * wiy + wiz * wiz);
        wix *= r; wiy *= r; wiz *= r;
        float wox = a.eye[0] - mx, woy = a.eye[1] - my, woz = a.eye[2] - mz;
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
        for (int kl = q; kl < sc.k; kl += 4) {
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
        sp0 += __shfl_xor(sp0, 16, 64); sp0 += __shfl_xor(sp0, 32, 64);
        sp1 += __shfl_xor(sp1, 16, 64); sp1 += __shfl_xor(sp1, 32, 64);
        sp2 += __shfl_xor(sp2, 16, 64); sp2 += __shfl_xor(sp2, 32, 64);
        const float c0 = fmaf(sc.albedo[g], fd, sp0);
        const float c1 = fmaf(sc.albedo[n + g], fd, sp1);
        const float c2 = fmaf(sc.albedo[2 * n + g], fd, sp2);
        // ---- shadow refinement Phi([T, feat]) (Eq. 8)
        const float Tg = a.T[g];
        float tp = Tg;
        if (a.use_phi) {
            floatx4 h[4];
            auto xin = [&](int k) -> float {
                if (k == 0) return Tg;
                if (k <= kFeat) return sc.feat[(size_t)(k - 1) * n + g];
                return 0.f;
            };
            mlp_hidden<kPhiK1>(sm, kPhiS, lane, xin, h);
            tp = mlp_out(sm, kPhiS, lane, h, 0);
        }
        // ---- residual Psi([feat, w_i, w_o]) (Sec. 4.3)
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if (a.use_psi) {
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
            mlp_hidden<kPsiK1>(sm, kPsiS, lane, xin, h);
            r0 = mlp_out(sm, kPsiS, lane, h, 0);
            r1 = mlp_out(sm, kPsiS, lane, h, 1);
            r2 = mlp_out(sm, kPsiS, lane, h, 2);
        }
        if (valid) {
            if (q == 0) {
                a.col0[g] = make_float4(c0, c1, c2, tp);
                a.col1[g] = make_float4(r0, r1, r2, 0.f);
            }
            const float v0 = q == 0 ? c0 : (q == 1 ? c2 : (q == 2 ? r0 : r2));
            const float v1 = q == 0 ? c1 : (q == 1 ? tp : (q == 2 ? r1 : 0.f));
            a.colour[(size_t)(2 * q) * n + g] = v0;
            a.colour[(size_t)(2 * q + 1) * n + g] = v1;
        }
    }
}

hipError_t launch_shade_mlp(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                            const gs3_mlp* psi, const Layout& L, void* ws, float* colour_out, hipStream_t st) {
    if (sc.n == 0) return hipSuccess;
    ShadeArgs a;
    a.sc = sc;
    for (int i = 0; i < 3; ++i) {
        a.light[i] = sp.light[i];
        a.eye[i] = sp.eye[i];
    }
    a.use_phi = phi != nullptr;
    a.use_psi = psi != nullptr;
    a.T = T;
    for (int i = 0; i < 4; ++i) {
        a.phi.w[i] = phi ? phi->w[i] : nullptr;
        a.phi.b[i] = phi ? phi->b[i] : nullptr;
        a.psi.w[i] = psi ? psi->w[i] : nullptr;
        a.psi.b[i] = psi ? psi->b[i] : nullptr;
    }
    a.col0 = at<float4>(ws, L.col0);
    a.col1 = at<float4>(ws, L.col1);
    a.colour = colour_out;
    const int per_block = 8 * 16;
    int grid = (int)((sc.n + per_block - 1) / per_block);
    if (grid > 512) grid = 512;
    hipLaunchKernelGGL(k_shade_mlp, dim3(grid), dim3(512), 0, st, a);
    return hipGetLastError();
}

}  // namespace gs3
