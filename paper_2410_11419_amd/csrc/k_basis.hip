// The paper's own appearance model and MLP form, forward and adjoint:
//  - shading with K basis angular Gaussians shared by every spatial Gaussian
//    (Sec. 4.1, Eq. 4-7 and the shared-basis paragraph): c = rho_d f_d +
//    rho_s sum_j alpha_j G_j(h'), G_j the anisotropic Eq. 7 in basis j's
//    frame;
//  - Phi(T, w_i; mu, l) (Sec. 4.2, Eq. 8): 61 -> 32 -> 32 -> 32 -> 1 and
//    Psi(w_o; mu, l) (Sec. 4.3): 60 -> 128 -> 128 -> 128 -> 3, leaky ReLU
//    hidden layers, sigmoid outputs, inputs [T, PE(w_i), PE(mu), l] and
//    [PE(w_o), PE(mu), l] with the 4-band positional encoding PE.
//
// The MLPs are dense contractions over the Gaussians and run on MFMA with
// the split half-precision products of mlp_common.h (x = hi + lo / 2048,
// three 16x16x32 products per 32-wide k-block). Each column (Gaussian) of the
// B operand is first scaled by a power of two that brings its largest
// entry to [128, 256), so the halves keep their precision for any
// magnitude (gradients included); outputs are scaled back exactly.
//
// A wave handles 16 Gaussians, four lanes per Gaussian (lane l: Gaussian
// l % 16, quarter q = l / 16); the D layout of a 16k-wide activation gives
// lane l the units 16 m + 4 q + i, i = 0..3, of tile m.
//
// Forward: k_basis_psi (shading + Psi, whose three layers of split weights
// fill the 160 KiB of LDS: one workgroup per CU) and k_basis_phi. Adjoint:
// the same two kernels in STORE mode recompute the forward, store every
// layer's input and output and the last hidden layer's pre-activation
// gradient in per-Gaussian scratch rows; k_mlp_layer_bwd steps the
// gradient back one layer at a time (W^T dz with the leaky-ReLU mask) down
// to the inputs; k_basis_shade_bwd turns the input gradients and the colour
// gradient into scene gradients (encoding, directions, shading frame,
// albedos, weights, latent) and per-wave sums for the shared basis, which
// k_basis_finish adds up in a fixed order; the weight gradients come from
// k_wgrad over the scratch rows.
#include "mlp_common.h"

namespace gs3 {

constexpr int kPE = 27;           // PE of a 3-vector: v, then sin/cos of 2^j pi v, j = 0..3
constexpr int kXin = 64;          // MLP inputs padded to four 16-wide k-blocks
constexpr int kMaxBasis = 16;

// Scratch rows ([row][n] floats) of the adjoint of one MLP with hidden width H:
// layer inputs x (kXin rows), hidden outputs h1..h3, pre-activation
// gradients dz1..dz3 (H rows each), output-layer gradient dz4 (n_out) and
// the gradient of the inputs dx (kXin).
struct BRows {
    int x, h1, h2, h3, dz1, dz2, dz3, dz4, dx, size;
};
__host__ __device__ constexpr BRows brows(int base, int H, int n_out) {
    return BRows{base,
                 base + kXin,
                 base + kXin + H,
                 base + kXin + 2 * H,
                 base + kXin + 3 * H,
                 base + kXin + 4 * H,
                 base + kXin + 5 * H,
                 base + kXin + 6 * H,
                 base + kXin + 6 * H + n_out,
                 2 * kXin + 6 * H + n_out};
}
constexpr BRows kPsiB = brows(0, kPsiBasisHidden, 3);
constexpr BRows kPhiB = brows(kPsiB.size, kPhiBasisHidden, 1);
constexpr int kBasisRows = kPsiB.size + kPhiB.size;
int basis_scratch_rows() { return kBasisRows; }

// LDS images (floats) of the split weights: a layer of M outputs and K
// (padded) inputs takes M K floats.
constexpr int kPsiL1 = 0, kPsiL2 = kPsiBasisHidden * kXin, kPsiL3 = kPsiL2 + kPsiBasisHidden * kPsiBasisHidden;
constexpr int kPsiSmem = kPsiL3 + kPsiBasisHidden * kPsiBasisHidden;
constexpr int kPhiL1 = 0, kPhiL2 = kPhiBasisHidden * kXin, kPhiL3 = kPhiL2 + kPhiBasisHidden * kPhiBasisHidden;
constexpr int kPhiSmem = kPhiL3 + kPhiBasisHidden * kPhiBasisHidden;
static_assert(kPsiSmem * 4 <= 160 * 1024, "Psi weights exceed the LDS");

// ---------------------------------------------------------------- helpers

__device__ inline float leaky(float z) { return z > 0.f ? z : kLeakySlope * z; }

// h = leaky(z + b) in place, b the layer's bias (global memory, tiny and hot)
template <int MT>
__device__ inline void bias_leaky(floatx4* z, const float* b, int q) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) z[mt][i] = leaky(z[mt][i] + b[16 * mt + 4 * q + i]);
}

// Output unit o of the last layer: sigmoid(w4[o] . h + b4[o]), the
// four quarters' partial sums combined.
template <int MT>
__device__ inline float out_unit(const float* w4, const float* b4, int o, const floatx4* h, int q) {
    float part = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) part = fmaf(w4[o * 16 * MT + 16 * mt + 4 * q + i], h[mt][i], part);
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    return 1.f / (1.f + expf(-(part + b4[o])));
}

// Rows row0 + 16 m + 4 q + i of Gaussian g (D-layout store).
template <int MT>
__device__ inline void store_d(float* rows, int row0, int q, int g, int n, const floatx4* v) {
    float* p = rows + (size_t)(row0 + 4 * q) * n + g;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) p[(size_t)(16 * mt + i) * n] = v[mt][i];
}
template <int MT>
__device__ inline void load_d(const float* rows, int row0, int q, int g, int n, floatx4* v) {
    const float* p = rows + (size_t)(row0 + 4 * q) * n + g;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[mt][i] = p[(size_t)(16 * mt + i) * n];
}

// sin and cos of 2^j pi v. With x = 2^(j - 1) v the angle is 2 pi x; x less
// its nearest integer (an exact difference) lies in [-1/2, 1/2], where the
// hardware sine and cosine, which take their argument in revolutions, are
// accurate to about 1e-7.
__device__ inline float pe_turns(float v, int j) {
    const float x = ldexpf(v, j - 1);
    return x - rintf(x);
}
__device__ inline float pe_sin(float v, int j) { return __builtin_amdgcn_sinf(pe_turns(v, j)); }
__device__ inline float pe_cos(float v, int j) { return __builtin_amdgcn_cosf(pe_turns(v, j)); }

// The MLP inputs in the order the lanes form them. Lane group q < 3 takes
// component q of both encoded vectors: k-block 0 holds the sines of the
// first vector's bands 0..3, k-block 1 their cosines, k-blocks 2 and 3 the
// same for mu. Lane group 3 holds the raw entries [T,] v, mu, l and zero
// padding. Every lane so runs one branch-free sequence; the weights' input
// columns are packed in the same order. in_index(c) is the position of
// packed column c in the MLP's own input order ([T,] PE(v), PE(mu), l),
// -1 for padding; t_first = 1 when T leads the inputs (Phi).
__device__ inline int in_index(int c, int t_first) {
    const int kb = c >> 4, q = (c >> 2) & 3, i = c & 3;
    if (q < 3) return t_first + (kb < 2 ? 0 : kPE) + ((kb & 1) ? 6 : 3) + 6 * i + q;
    const int r = 4 * kb + i;
    if (r < t_first) return 0;
    const int s = r - t_first;
    if (s < 3) return t_first + s;
    if (s < 6) return t_first + kPE + s - 3;
    if (s < 6 + kLatent) return t_first + 2 * kPE + s - 6;
    return -1;
}

// The lane's 16 inputs x[kb][i] (packed column 16 kb + 4 q + i) for the
// encoded vector v, the mean m, the Gaussian's latent and (t_first) T.
__device__ inline void form_inputs(int q, int t_first, float Tg, const float v[3], const float m[3],
                                   const SceneDev& sc, int g, floatx4 x[4]) {
    if (q < 3) {
        const float vq = q == 0 ? v[0] : (q == 1 ? v[1] : v[2]);
        const float mq = q == 0 ? m[0] : (q == 1 ? m[1] : m[2]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float fv = pe_turns(vq, i), fm = pe_turns(mq, i);
            x[0][i] = __builtin_amdgcn_sinf(fv);
            x[1][i] = __builtin_amdgcn_cosf(fv);
            x[2][i] = __builtin_amdgcn_sinf(fm);
            x[3][i] = __builtin_amdgcn_cosf(fm);
        }
    } else {
        float raw[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) raw[r] = 0.f;
        const int o = t_first;
        if (o) raw[0] = Tg;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            raw[o + c] = v[c];
            raw[o + 3 + c] = m[c];
        }
#pragma unroll
        for (int l = 0; l < kLatent; ++l) raw[o + 6 + l] = sc.latent[(size_t)l * sc.n + g];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) x[kb][i] = raw[4 * kb + i];
    }
}

// Rotation matrix (row-major) of a quaternion (w, x, y, z), normalised.
__device__ inline void quat_mat(float qw, float qx, float qy, float qz, float R[9]) {
    const float r = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= r; qx *= r; qy *= r; qz *= r;
    R[0] = 1 - 2 * (qy * qy + qz * qz); R[1] = 2 * (qx * qy - qw * qz); R[2] = 2 * (qx * qz + qw * qy);
    R[3] = 2 * (qx * qy + qw * qz); R[4] = 1 - 2 * (qx * qx + qz * qz); R[5] = 2 * (qy * qz - qw * qx);
    R[6] = 2 * (qx * qz - qw * qy); R[7] = 2 * (qy * qz + qw * qx); R[8] = 1 - 2 * (qx * qx + qy * qy);
}

// Eq. 7 in the basis frame: h' has coordinates (a, b, c) there; theta is
// the angle to z, rho = |(a, b)|, S = (a^2/sx^2 + b^2/sy^2) / rho^2 (the
// squared anisotropy factor, 1 when rho = 0), E = theta^2 S / sz^2 and
// G = exp(-E / 2) / sz.
struct AsgEval {
    float theta, rho2, S, E, G;
};
__device__ inline AsgEval asg_eval(float a, float b, float c, float isx2, float isy2, float isz2, float isz) {
    AsgEval r;
    r.rho2 = a * a + b * b;
    r.theta = atan2f(sqrtf(r.rho2), c);
    r.S = r.rho2 > 1e-30f ? (a * a * isx2 + b * b * isy2) / r.rho2 : 1.f;
    r.E = r.theta * r.theta * r.S * isz2;
    r.G = expf(-0.5f * r.E) * isz;
    return r;
}

struct BasisConst {
    float R[kMaxBasis][9];     // shading -> basis frame (rows x, y, z)
    float isx2[kMaxBasis], isy2[kMaxBasis], isz2[kMaxBasis], isz[kMaxBasis];
};

__device__ inline void load_basis(const SceneDev& sc, int j, float R[9], float* isx2, float* isy2, float* isz2,
                                  float* isz) {
    quat_mat(sc.basis_rot[4 * j], sc.basis_rot[4 * j + 1], sc.basis_rot[4 * j + 2], sc.basis_rot[4 * j + 3], R);
    const float sx = expf(sc.basis_log_sigma[3 * j]), sy = expf(sc.basis_log_sigma[3 * j + 1]);
    const float sz = expf(sc.basis_log_sigma[3 * j + 2]);
    *isx2 = 1.f / (sx * sx);
    *isy2 = 1.f / (sy * sy);
    *isz = 1.f / sz;
    *isz2 = *isz * *isz;
}

// Unit directions from the centre toward the light (or a directional
// light's fixed direction) and toward the camera; returns the inverse
// distances (0 for a directional light's w_i).
__device__ inline void directions(const float light[3], int light_dir, const float eye[3], float mx, float my,
                                  float mz, float wi[3], float wo[3], float* ri, float* ro) {
    const float lm = light_dir ? 0.f : 1.f;
    wi[0] = light[0] - lm * mx; wi[1] = light[1] - lm * my; wi[2] = light[2] - lm * mz;
    const float r = rsqrtf(wi[0] * wi[0] + wi[1] * wi[1] + wi[2] * wi[2]);
    wi[0] *= r; wi[1] *= r; wi[2] *= r;
    *ri = lm * r;
    wo[0] = eye[0] - mx; wo[1] = eye[1] - my; wo[2] = eye[2] - mz;
    const float s = rsqrtf(wo[0] * wo[0] + wo[1] * wo[1] + wo[2] * wo[2]);
    wo[0] *= s; wo[1] *= s; wo[2] *= s;
    *ro = s;
}

// ---------------------------------------------------------------- forward

// Scene, MLPs and the views of one launch (blockIdx.y selects the view;
// STORE launches take one view).
struct BasisArgs {
    SceneDev sc;
    int use_phi, use_psi;
    MlpArgs phi, psi;
    const float* gcol;   // STORE: [7][n] dL/d{c.rgb, T', r.rgb}
    float* rows;         // STORE: scratch rows
    ShadeView v[kMaxBatch];
};

// Shading c (Eq. 4-7 with the shared basis) of the view blockIdx.y, one
// Gaussian per lane; the basis frames and inverse scales are formed once per
// workgroup in LDS. Writes c to col0.xyz and colour rows 0..2.
__global__ __launch_bounds__(256) void k_basis_c(BasisArgs a) {
    const ShadeView vw = a.v[blockIdx.y];
    __shared__ BasisConst B;
    const SceneDev& sc = a.sc;
    const int n = sc.n, K = sc.k;
    for (int j = threadIdx.x; j < K; j += blockDim.x)
        load_basis(sc, j, B.R[j], &B.isx2[j], &B.isy2[j], &B.isz2[j], &B.isz[j]);
    __syncthreads();
    const float kd = 0.01f * (1.f - 0.36787944117144233f);   // eps (1 - 1/e), Eq. 5
    const float fd_norm = 1.f / ((1.f + kd) * 3.14159265358979f);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        float wi[3], wo[3], ri, ro;
        directions(vw.light, vw.light_dir, vw.eye, mx, my, mz, wi, wo, &ri, &ro);
        float Rs[9];
        quat_mat(sc.shade_rot[g], sc.shade_rot[n + g], sc.shade_rot[2 * n + g], sc.shade_rot[3 * n + g], Rs);
        const float lix = Rs[0] * wi[0] + Rs[1] * wi[1] + Rs[2] * wi[2];
        const float liy = Rs[3] * wi[0] + Rs[4] * wi[1] + Rs[5] * wi[2];
        const float liz = Rs[6] * wi[0] + Rs[7] * wi[1] + Rs[8] * wi[2];
        const float lox = Rs[0] * wo[0] + Rs[1] * wo[1] + Rs[2] * wo[2];
        const float loy = Rs[3] * wo[0] + Rs[4] * wo[1] + Rs[5] * wo[2];
        const float loz = Rs[6] * wo[0] + Rs[7] * wo[1] + Rs[8] * wo[2];
        const float elu = liz > 0.f ? liz : 0.01f * (expf(fminf(liz, 0.f)) - 1.f);
        const float fd = (elu + kd) * fd_norm;
        float hx = lix + lox, hy = liy + loy, hz = liz + loz;
        const float hn2 = hx * hx + hy * hy + hz * hz;
        if (hn2 > 1e-24f) {
            const float r = rsqrtf(hn2);
            hx *= r; hy *= r; hz *= r;
        } else {
            hx = 0.f; hy = 0.f; hz = 1.f;
        }
        // Eq. 6 over the shared basis
        float fs = 0.f;
        for (int j = 0; j < K; ++j) {
            const float* Rb = B.R[j];
            const float ba = Rb[0] * hx + Rb[1] * hy + Rb[2] * hz;
            const float bb = Rb[3] * hx + Rb[4] * hy + Rb[5] * hz;
            const float bc = Rb[6] * hx + Rb[7] * hy + Rb[8] * hz;
            const AsgEval ev = asg_eval(ba, bb, bc, B.isx2[j], B.isy2[j], B.isz2[j], B.isz[j]);
            fs = fmaf(sc.basis_weight[(size_t)j * n + g], ev.G, fs);
        }
        const float c0 = fmaf(sc.albedo[g], fd, sc.spec_albedo[g] * fs);
        const float c1 = fmaf(sc.albedo[n + g], fd, sc.spec_albedo[n + g] * fs);
        const float c2 = fmaf(sc.albedo[2 * n + g], fd, sc.spec_albedo[2 * n + g] * fs);
        // col0.w is Phi's T', written by k_basis_phi
        float* c0p = reinterpret_cast<float*>(vw.col0 + g);
        c0p[0] = c0;
        c0p[1] = c1;
        c0p[2] = c2;
        vw.colour[g] = c0;
        vw.colour[(size_t)n + g] = c1;
        vw.colour[(size_t)2 * n + g] = c2;
    }
}

// The residual r = Psi(w_o; mu, l) (Sec. 4.3). STORE: no colours; Psi's
// layer inputs/outputs and its last hidden layer's pre-activation gradient
// go to the scratch rows.
// The forward runs 12 waves a CU (three a SIMD within its register
// budget); STORE keeps more live and runs 8.
constexpr int psi_threads(bool store) { return store ? 512 : 768; }
template <bool STORE>
__global__ __launch_bounds__(psi_threads(STORE)) void k_basis_psi(BasisArgs a) {
    const ShadeView vw = a.v[blockIdx.y];
    __shared__ __align__(16) float sm[kPsiSmem];
    const SceneDev& sc = a.sc;
    const int n = sc.n;
    if (a.use_psi) {
        const MlpArgs& m = a.psi;
        pack_split(sm + kPsiL1, kPsiBasisHidden, kXin,
                   [&](int r, int c) {
                       const int k = in_index(c, 0);
                       return k >= 0 ? m.w[0][r * kPsiBasisIn + k] : 0.f;
                   });
        pack_split(sm + kPsiL2, kPsiBasisHidden, kPsiBasisHidden,
                   [&](int r, int c) { return m.w[1][r * kPsiBasisHidden + c]; });
        pack_split(sm + kPsiL3, kPsiBasisHidden, kPsiBasisHidden,
                   [&](int r, int c) { return m.w[2][r * kPsiBasisHidden + c]; });
    }
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4;
    const int waves = blockDim.x >> 6;
    constexpr int MT = kPsiBasisHidden / 16;
    for (int base = (blockIdx.x * waves + w) * 16; base < n; base += gridDim.x * waves * 16) {
        asm volatile("" ::: "memory");
        const int g_raw = base + (lane & 15);
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        float wi[3], wo[3], ri, ro;
        directions(vw.light, vw.light_dir, vw.eye, mx, my, mz, wi, wo, &ri, &ro);
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if (a.use_psi) {
            // inputs [PE(w_o), PE(mu), l] in the lane-grouped order
            floatx4 x[4];
            const float mu[3] = {mx, my, mz};
            form_inputs(q, 0, 0.f, wo, mu, sc, g, x);
            floatx4 h1[MT], h2[MT], h3[MT];
            split_gemm<MT, 4>(sm + kPsiL1, lane, x, h1);
            bias_leaky<MT>(h1, a.psi.b[0], q);
            split_gemm<MT, MT>(sm + kPsiL2, lane, h1, h2);
            bias_leaky<MT>(h2, a.psi.b[1], q);
            if (STORE && valid) {
                float* R = a.rows;
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = in_index(16 * kb + 4 * q + i, 0);
                        if (k >= 0) R[(size_t)(kPsiB.x + k) * n + g] = x[kb][i];
                    }
                store_d<MT>(R, kPsiB.h1, q, g, n, h1);
                store_d<MT>(R, kPsiB.h2, q, g, n, h2);
            }
            split_gemm<MT, MT>(sm + kPsiL3, lane, h2, h3);
            bias_leaky<MT>(h3, a.psi.b[2], q);
            r0 = out_unit<MT>(a.psi.w[3], a.psi.b[3], 0, h3, q);
            r1 = out_unit<MT>(a.psi.w[3], a.psi.b[3], 1, h3, q);
            r2 = out_unit<MT>(a.psi.w[3], a.psi.b[3], 2, h3, q);
            if (STORE) {
                const float d0 = a.gcol[(size_t)4 * n + g] * r0 * (1.f - r0);
                const float d1 = a.gcol[(size_t)5 * n + g] * r1 * (1.f - r1);
                const float d2 = a.gcol[(size_t)6 * n + g] * r2 * (1.f - r2);
                const float* w4 = a.psi.w[3];
                floatx4 dz[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int u = 16 * mt + 4 * q + i;
                        const float dh = fmaf(w4[u], d0, fmaf(w4[kPsiBasisHidden + u], d1, w4[2 * kPsiBasisHidden + u] * d2));
                        dz[mt][i] = h3[mt][i] > 0.f ? dh : kLeakySlope * dh;
                    }
                if (valid) {
                    store_d<MT>(a.rows, kPsiB.h3, q, g, n, h3);
                    store_d<MT>(a.rows, kPsiB.dz3, q, g, n, dz);
                    if (q == 0) {
                        a.rows[(size_t)kPsiB.dz4 * n + g] = d0;
                        a.rows[(size_t)(kPsiB.dz4 + 1) * n + g] = d1;
                        a.rows[(size_t)(kPsiB.dz4 + 2) * n + g] = d2;
                    }
                }
            }
        }
        if (!STORE && valid) {
            // r: col1 and colour rows 4..6, row 7 = 0
            if (q == 0) vw.col1[g] = make_float4(r0, r1, r2, 0.f);
            vw.colour[(size_t)(4 + q) * n + g] = q == 0 ? r0 : (q == 1 ? r1 : (q == 2 ? r2 : 0.f));
        }
    }
}

// Refined shadow T' = Phi(T, w_i; mu, l) (Sec. 4.2, Eq. 8), or T' = T
// without Phi. STORE: Phi's layer inputs/outputs and its last hidden
// layer's pre-activation gradient go to the scratch rows.
template <bool STORE>
__global__ __launch_bounds__(256) void k_basis_phi(BasisArgs a) {
    const ShadeView vw = a.v[blockIdx.y];
    __shared__ __align__(16) float sm[kPhiSmem];
    const SceneDev& sc = a.sc;
    const int n = sc.n;
    if (a.use_phi) {
        const MlpArgs& m = a.phi;
        pack_split(sm + kPhiL1, kPhiBasisHidden, kXin,
                   [&](int r, int c) {
                       const int k = in_index(c, 1);
                       return k >= 0 ? m.w[0][r * kPhiBasisIn + k] : 0.f;
                   });
        pack_split(sm + kPhiL2, kPhiBasisHidden, kPhiBasisHidden,
                   [&](int r, int c) { return m.w[1][r * kPhiBasisHidden + c]; });
        pack_split(sm + kPhiL3, kPhiBasisHidden, kPhiBasisHidden,
                   [&](int r, int c) { return m.w[2][r * kPhiBasisHidden + c]; });
    }
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4;
    const int waves = blockDim.x >> 6;
    constexpr int MT = kPhiBasisHidden / 16;
    for (int base = (blockIdx.x * waves + w) * 16; base < n; base += gridDim.x * waves * 16) {
        const int g_raw = base + (lane & 15);
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        const float Tg = vw.T[g];
        float tp = Tg;
        if (a.use_phi) {
            const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
            float wi[3], wo[3], ri, ro;
            directions(vw.light, vw.light_dir, vw.eye, mx, my, mz, wi, wo, &ri, &ro);
            // inputs [T, PE(w_i), PE(mu), l] in the lane-grouped order
            floatx4 x[4];
            const float mu[3] = {mx, my, mz};
            form_inputs(q, 1, Tg, wi, mu, sc, g, x);
            floatx4 h1[MT], h2[MT], h3[MT];
            split_gemm<MT, 4>(sm + kPhiL1, lane, x, h1);
            bias_leaky<MT>(h1, a.phi.b[0], q);
            split_gemm<MT, MT>(sm + kPhiL2, lane, h1, h2);
            bias_leaky<MT>(h2, a.phi.b[1], q);
            split_gemm<MT, MT>(sm + kPhiL3, lane, h2, h3);
            bias_leaky<MT>(h3, a.phi.b[2], q);
            tp = out_unit<MT>(a.phi.w[3], a.phi.b[3], 0, h3, q);
            if (STORE && valid) {
                float* R = a.rows;
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = in_index(16 * kb + 4 * q + i, 1);
                        if (k >= 0) R[(size_t)(kPhiB.x + k) * n + g] = x[kb][i];
                    }
                store_d<MT>(R, kPhiB.h1, q, g, n, h1);
                store_d<MT>(R, kPhiB.h2, q, g, n, h2);
                store_d<MT>(R, kPhiB.h3, q, g, n, h3);
                const float d4 = a.gcol[(size_t)3 * n + g] * tp * (1.f - tp);
                floatx4 dz[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float dh = a.phi.w[3][16 * mt + 4 * q + i] * d4;
                        dz[mt][i] = h3[mt][i] > 0.f ? dh : kLeakySlope * dh;
                    }
                store_d<MT>(R, kPhiB.dz3, q, g, n, dz);
                if (q == 0) R[(size_t)kPhiB.dz4 * n + g] = d4;
            }
        }
        if (!STORE && valid && q == 0) {
            reinterpret_cast<float*>(vw.col0 + g)[3] = tp;
            vw.colour[(size_t)3 * n + g] = tp;
        }
    }
}

// ---------------------------------------------------------------- adjoint

struct LayerBwdArgs {
    const float* W;      // [n_out][n_in] row-major
    int n_in, n_out;
    float* rows;
    int dz_row;          // gradient of the layer's pre-activations (16 KB rows)
    int h_row;           // MASK: the layer's inputs (previous hidden outputs)
    int out_row;         // written: 16 MT rows
    int n;
};

// One layer back: out = W^T dz, times the leaky-ReLU derivative of the
// layer's inputs when they are hidden activations (MASK), giving the
// previous layer's pre-activation gradient; without MASK the gradient of
// the MLP inputs.
template <int MT, int KB, bool MASK>
__global__ __launch_bounds__(256) void k_mlp_layer_bwd(LayerBwdArgs a) {
    __shared__ __align__(16) float sm[16 * MT * 16 * KB];
    pack_split(sm, 16 * MT, 16 * KB,
               [&](int r, int c) { return (r < a.n_in && c < a.n_out) ? a.W[(size_t)c * a.n_in + r] : 0.f; });
    __syncthreads();
    const int n = a.n;
    const int lane = __lane_id(), w = threadIdx.x >> 6, q = lane >> 4;
    const int waves = blockDim.x >> 6;
    for (int base = (blockIdx.x * waves + w) * 16; base < n; base += gridDim.x * waves * 16) {
        const int g_raw = base + (lane & 15);
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        SplitB<KB> b;
        {
            floatx4 dz[KB];
            load_d<KB>(a.rows, a.dz_row, q, g, n, dz);
            split_cols<KB>(dz, b);
        }
        // two output tiles at a time: their products, mask and stores
#pragma unroll 1
        for (int mt = 0; mt < MT; mt += 2) {
            floatx4 out[2];
            split_tiles<KB, 2>(sm, lane, mt, b, out);
            if (MASK) {
                floatx4 h[2];
                load_d<2>(a.rows, a.h_row + 16 * mt, q, g, n, h);
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int i = 0; i < 4; ++i) out[c][i] = h[c][i] > 0.f ? out[c][i] : kLeakySlope * out[c][i];
            }
            if (valid) store_d<2>(a.rows, a.out_row + 16 * mt, q, g, n, out);
        }
    }
}

struct ShadeBwdBasisArgs {
    SceneDev sc;
    float light[3], eye[3];
    int light_dir;
    int use_phi, use_psi;
    const float* gcol;   // [7][n]
    const float* rows;   // dx rows of both MLPs
    float* dT;           // [n]
    GradDev g;
    float* partial;      // [waves][12 k] per-wave sums of dR_j (9) and d log sigma_j (3)
};

// Adjoint of the encoding: d/dv of PE(v) given dPE (27 entries at
// rows[row0 ..]).
__device__ inline void pe_adjoint(const float* rows, int row0, int n, int g, float v0, float v1, float v2,
                                  float dv[3]) {
    const float v[3] = {v0, v1, v2};
    for (int c = 0; c < 3; ++c) dv[c] = rows[(size_t)(row0 + c) * n + g];
    for (int j = 0; j < 4; ++j) {
        const float f = ldexpf(3.14159265358979f, j);
        for (int c = 0; c < 3; ++c) {
            const float sn = pe_sin(v[c], j), cs = pe_cos(v[c], j);
            const float ds = rows[(size_t)(row0 + 3 + 6 * j + c) * n + g];
            const float dc = rows[(size_t)(row0 + 6 + 6 * j + c) * n + g];
            dv[c] = fmaf(f, ds * cs - dc * sn, dv[c]);
        }
    }
}

__global__ __launch_bounds__(256) void k_basis_shade_bwd(ShadeBwdBasisArgs a) {
    __shared__ BasisConst B;
    const SceneDev& sc = a.sc;
    const int n = sc.n, K = sc.k;
    for (int j = threadIdx.x; j < K; j += blockDim.x)
        load_basis(sc, j, B.R[j], &B.isx2[j], &B.isy2[j], &B.isz2[j], &B.isz[j]);
    __syncthreads();
    const int lane = __lane_id();
    const float kd = 0.01f * (1.f - 0.36787944117144233f);
    const float fd_norm = 1.f / ((1.f + kd) * 3.14159265358979f);
    // per-wave sums of the shared-basis gradients: value v = 12 j + t is
    // kept by lane v % 64 in acc[v / 64]
    float acc[3] = {0.f, 0.f, 0.f};
    const int stride = gridDim.x * blockDim.x;
    const int start = blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int base = start; base < n; base += stride) {
        const int g_raw = base + lane;
        const bool valid = g_raw < n;
        const int g = valid ? g_raw : n - 1;
        const float mx = sc.mean[g], my = sc.mean[n + g], mz = sc.mean[2 * n + g];
        float wi[3], wo[3], ri, ro;
        directions(a.light, a.light_dir, a.eye, mx, my, mz, wi, wo, &ri, &ro);
        float qw = sc.shade_rot[g], qx = sc.shade_rot[n + g], qy = sc.shade_rot[2 * n + g], qz = sc.shade_rot[3 * n + g];
        const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        float Rs[9];
        quat_mat(qw, qx, qy, qz, Rs);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const float lix = Rs[0] * wi[0] + Rs[1] * wi[1] + Rs[2] * wi[2];
        const float liy = Rs[3] * wi[0] + Rs[4] * wi[1] + Rs[5] * wi[2];
        const float liz = Rs[6] * wi[0] + Rs[7] * wi[1] + Rs[8] * wi[2];
        const float lox = Rs[0] * wo[0] + Rs[1] * wo[1] + Rs[2] * wo[2];
        const float loy = Rs[3] * wo[0] + Rs[4] * wo[1] + Rs[5] * wo[2];
        const float loz = Rs[6] * wo[0] + Rs[7] * wo[1] + Rs[8] * wo[2];
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
        const float dc0 = valid ? a.gcol[g] : 0.f, dc1 = valid ? a.gcol[(size_t)n + g] : 0.f;
        const float dc2 = valid ? a.gcol[(size_t)2 * n + g] : 0.f;
        const float rs0 = sc.spec_albedo[g], rs1 = sc.spec_albedo[n + g], rs2 = sc.spec_albedo[2 * n + g];
        const float dGs = fmaf(dc0, rs0, fmaf(dc1, rs1, dc2 * rs2));   // dL/d(sum_j alpha_j G_j)
        float fs = 0.f, dhx = 0.f, dhy = 0.f, dhz = 0.f;
        for (int j = 0; j < K; ++j) {
            const float* Rb = B.R[j];
            const float ba = Rb[0] * hx + Rb[1] * hy + Rb[2] * hz;
            const float bb = Rb[3] * hx + Rb[4] * hy + Rb[5] * hz;
            const float bc = Rb[6] * hx + Rb[7] * hy + Rb[8] * hz;
            const float isx2 = B.isx2[j], isy2 = B.isy2[j], isz2 = B.isz2[j];
            const AsgEval ev = asg_eval(ba, bb, bc, isx2, isy2, isz2, B.isz[j]);
            const float al = sc.basis_weight[(size_t)j * n + g];
            fs = fmaf(al, ev.G, fs);
            if (valid) a.g.basis_weight[(size_t)j * n + g] += dGs * ev.G;
            const float dG = dGs * al;
            const float dE = -0.5f * ev.G * dG;
            // E = theta^2 S / sz^2: with P = theta / rho and r^2 = rho^2 + c^2,
            // dE/da = 2 (P a c S / r^2 + P^2 a (1/sx^2 - S)) / sz^2, likewise b,
            // dE/dc = -2 theta rho S / (r^2 sz^2)
            const float r2 = ev.rho2 + bc * bc;
            float da = 0.f, db = 0.f, dcz = 0.f, P2 = 1.f;
            if (ev.rho2 > 1e-30f) {
                const float rho = sqrtf(ev.rho2);
                const float P = ev.theta / rho;
                P2 = P * P;
                const float t1 = 2.f * P * bc * ev.S / r2;
                da = (t1 * ba + 2.f * P2 * ba * (isx2 - ev.S)) * isz2;
                db = (t1 * bb + 2.f * P2 * bb * (isy2 - ev.S)) * isz2;
                dcz = -2.f * ev.theta * rho * ev.S / r2 * isz2;
            }
            da *= dE; db *= dE; dcz *= dE;
            dhx += Rb[0] * da + Rb[3] * db + Rb[6] * dcz;
            dhy += Rb[1] * da + Rb[4] * db + Rb[7] * dcz;
            dhz += Rb[2] * da + Rb[5] * db + Rb[8] * dcz;
            // shared-basis sums: dR_j = d(a, b, c) h'^T and d log sigma_j
            const float gsc = dG * ev.G * P2 * isz2;
            float val[12] = {da * hx, da * hy, da * hz, db * hx, db * hy, db * hz, dcz * hx, dcz * hy, dcz * hz,
                             gsc * ba * ba * isx2, gsc * bb * bb * isy2, dG * ev.G * (ev.E - 1.f)};
            if (!valid) {
#pragma unroll
                for (int t = 0; t < 12; ++t) val[t] = 0.f;
            }
#pragma unroll
            for (int t = 0; t < 12; ++t) {
                float s = val[t];
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
                const int v = 12 * j + t;
                if (lane == (v & 63)) {
                    const int slot = v >> 6;
                    if (slot == 0) acc[0] += s;
                    else if (slot == 1) acc[1] += s;
                    else acc[2] += s;
                }
            }
        }
        // Lambertian and half vector
        const float al0 = sc.albedo[g], al1 = sc.albedo[n + g], al2 = sc.albedo[2 * n + g];
        const float dfd = fmaf(dc0, al0, fmaf(dc1, al1, dc2 * al2));
        float dhsx = 0.f, dhsy = 0.f, dhsz = 0.f;
        if (hok) {
            const float dd = dhx * hx + dhy * hy + dhz * hz;
            dhsx = (dhx - dd * hx) * rh;
            dhsy = (dhy - dd * hy) * rh;
            dhsz = (dhz - dd * hz) * rh;
        }
        const float dlix = dhsx, dliy = dhsy, dliz = dhsz + dfd * fd_norm * delu;
        const float dlox = dhsx, dloy = dhsy, dloz = dhsz;
        const float dR[9] = {dlix * wi[0] + dlox * wo[0], dlix * wi[1] + dlox * wo[1], dlix * wi[2] + dlox * wo[2],
                             dliy * wi[0] + dloy * wo[0], dliy * wi[1] + dloy * wo[1], dliy * wi[2] + dloy * wo[2],
                             dliz * wi[0] + dloz * wo[0], dliz * wi[1] + dloz * wo[1], dliz * wi[2] + dloz * wo[2]};
        float dq[4];
        quat_grad(qw, qx, qy, qz, qn, dR, dq);
        float dwi[3] = {Rs[0] * dlix + Rs[3] * dliy + Rs[6] * dliz, Rs[1] * dlix + Rs[4] * dliy + Rs[7] * dliz,
                        Rs[2] * dlix + Rs[5] * dliy + Rs[8] * dliz};
        float dwo[3] = {Rs[0] * dlox + Rs[3] * dloy + Rs[6] * dloz, Rs[1] * dlox + Rs[4] * dloy + Rs[7] * dloz,
                        Rs[2] * dlox + Rs[5] * dloy + Rs[8] * dloz};
        float dmu[3] = {0.f, 0.f, 0.f};
        float dTg = valid ? a.gcol[(size_t)3 * n + g] : 0.f;   // T' = T without Phi
        float dlat[kLatent] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (a.use_phi) {
            dTg = a.rows[(size_t)kPhiB.dx * n + g];
            float d[3];
            pe_adjoint(a.rows, kPhiB.dx + 1, n, g, wi[0], wi[1], wi[2], d);
            for (int c = 0; c < 3; ++c) dwi[c] += d[c];
            pe_adjoint(a.rows, kPhiB.dx + 1 + kPE, n, g, mx, my, mz, d);
            for (int c = 0; c < 3; ++c) dmu[c] += d[c];
            for (int c = 0; c < kLatent; ++c) dlat[c] += a.rows[(size_t)(kPhiB.dx + 1 + 2 * kPE + c) * n + g];
        }
        if (a.use_psi) {
            float d[3];
            pe_adjoint(a.rows, kPsiB.dx, n, g, wo[0], wo[1], wo[2], d);
            for (int c = 0; c < 3; ++c) dwo[c] += d[c];
            pe_adjoint(a.rows, kPsiB.dx + kPE, n, g, mx, my, mz, d);
            for (int c = 0; c < 3; ++c) dmu[c] += d[c];
            for (int c = 0; c < kLatent; ++c) dlat[c] += a.rows[(size_t)(kPsiB.dx + 2 * kPE + c) * n + g];
        }
        // w = (p - mu) / |p - mu|: dmu -= (dw - (dw . w) w) / |p - mu| (no
        // dependence for a directional light's w_i)
        const float wd = dwi[0] * wi[0] + dwi[1] * wi[1] + dwi[2] * wi[2];
        const float od = dwo[0] * wo[0] + dwo[1] * wo[1] + dwo[2] * wo[2];
        for (int c = 0; c < 3; ++c) dmu[c] -= (dwi[c] - wd * wi[c]) * ri + (dwo[c] - od * wo[c]) * ro;
        if (valid) {
            a.g.albedo[g] += dc0 * fd;
            a.g.albedo[n + g] += dc1 * fd;
            a.g.albedo[2 * n + g] += dc2 * fd;
            a.g.spec_albedo[g] += dc0 * fs;
            a.g.spec_albedo[n + g] += dc1 * fs;
            a.g.spec_albedo[2 * n + g] += dc2 * fs;
            for (int c = 0; c < 4; ++c) a.g.shade_rot[(size_t)c * n + g] += dq[c];
            for (int c = 0; c < 3; ++c) a.g.mean[(size_t)c * n + g] += dmu[c];
            for (int c = 0; c < kLatent; ++c) a.g.latent[(size_t)c * n + g] += dlat[c];
            a.dT[g] = dTg;
        }
    }
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    float* part = a.partial + (size_t)wave * 12 * kMaxBasis;
    for (int s = 0; s < 3; ++s) {
        const int v = 64 * s + lane;
        if (v < 12 * K) part[v] = acc[s];
    }
}

// Sum the per-wave basis sums in a fixed order and apply the adjoint of the
// basis quaternions (dR_j -> dq_j) and sigmas. Workgroup j handles basis j
// with 12 waves, one per value: lane l adds every 64th wave's partial from
// wave l on, the lanes are combined by a butterfly (fixed order), and the
// first thread applies the quaternion adjoint.
__global__ __launch_bounds__(768) void k_basis_finish(SceneDev sc, const float* partial, int waves, GradDev g) {
    __shared__ float tot[12];
    const int j = blockIdx.x, v = threadIdx.x >> 6, lane = __lane_id();
    float s = 0.f;
    for (int w = lane; w < waves; w += 64) s += partial[(size_t)w * 12 * kMaxBasis + 12 * j + v];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) tot[v] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float qw = sc.basis_rot[4 * j], qx = sc.basis_rot[4 * j + 1], qy = sc.basis_rot[4 * j + 2],
              qz = sc.basis_rot[4 * j + 3];
        const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const float dR[9] = {tot[0], tot[1], tot[2], tot[3], tot[4], tot[5], tot[6], tot[7], tot[8]};
        float dq[4];
        quat_grad(qw, qx, qy, qz, qn, dR, dq);
        for (int c = 0; c < 4; ++c) g.basis_rot[4 * j + c] += dq[c];
        for (int c = 0; c < 3; ++c) g.basis_log_sigma[3 * j + c] += tot[9 + c];
    }
}

// ---------------------------------------------------------------- launchers

static BasisArgs basis_args(const SceneDev& sc, const gs3_mlp* phi, const gs3_mlp* psi) {
    BasisArgs a;
    a.sc = sc;
    a.use_phi = phi != nullptr;
    a.use_psi = psi != nullptr;
    for (int i = 0; i < 4; ++i) {
        a.phi.w[i] = phi ? phi->w[i] : nullptr;
        a.phi.b[i] = phi ? phi->b[i] : nullptr;
        a.psi.w[i] = psi ? psi->w[i] : nullptr;
        a.psi.b[i] = psi ? psi->b[i] : nullptr;
    }
    a.gcol = nullptr;
    a.rows = nullptr;
    return a;
}

static void set_view(ShadeView& w, const ShadeParams& sp, const float* T, float4* col0, float4* col1,
                     float* colour) {
    for (int c = 0; c < 3; ++c) {
        w.light[c] = sp.light[c];
        w.eye[c] = sp.eye[c];
    }
    w.light_dir = sp.light_dir;
    w.T = T;
    w.col0 = col0;
    w.col1 = col1;
    w.colour = colour;
}

// Workgroups of a grid-stride launch over n Gaussians, `per` per workgroup.
static int grid_for(int64_t n, int per, int cap) {
    int64_t g = (n + per - 1) / per;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// Workgroups of `threads` threads of a kernel (no dynamic LDS) that the
// device holds at once: one round of a grid-stride launch, so that each
// workgroup packs its weights into LDS once.
template <typename Kernel>
static int resident_blocks(Kernel kernel, int threads) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess)
        return 2048;
    return (per < 1 ? 1 : per) * (cus < 1 ? 1 : cus);
}

hipError_t launch_basis_shade_batch(const SceneDev& sc, const ShadeParams* sps, const float* const* T,
                                    const gs3_mlp* phi, const gs3_mlp* psi, const Layout* const* Ls,
                                    void* const* wss, float* const* colour, int parts, int nv, hipStream_t st) {
    if (sc.n == 0) return hipSuccess;
    BasisArgs a = basis_args(sc, phi, psi);
    for (int v0 = 0; v0 < nv; v0 += kMaxBatch) {
        const int m = nv - v0 < kMaxBatch ? nv - v0 : kMaxBatch;
        for (int i = 0; i < m; ++i)
            set_view(a.v[i], sps[v0 + i], T ? T[v0 + i] : nullptr, at<float4>(wss[v0 + i], Ls[v0 + i]->col0),
                     at<float4>(wss[v0 + i], Ls[v0 + i]->col1), colour[v0 + i]);
        if (parts & 1) {
            hipLaunchKernelGGL(k_basis_c, dim3(grid_for(sc.n, 256, 2048), m), dim3(256), 0, st, a);
            // the Psi weights take the whole LDS: one workgroup per CU
            constexpr int T = psi_threads(false);
            hipLaunchKernelGGL(k_basis_psi<false>, dim3(grid_for(sc.n, T / 4, 256), m), dim3(T), 0, st, a);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (parts & 2) {
            static const int round = resident_blocks(k_basis_phi<false>, 256);
            hipLaunchKernelGGL(k_basis_phi<false>, dim3(grid_for(sc.n, 4 * 16, round), m), dim3(256), 0, st, a);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_basis_shade(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                              const gs3_mlp* psi, const Layout& L, void* ws, float* colour_out, int parts,
                              hipStream_t st) {
    const Layout* Ls[1] = {&L};
    return launch_basis_shade_batch(sc, &sp, &T, phi, psi, Ls, &ws, &colour_out, parts, 1, st);
}

int basis_partial_floats(int k) {
    (void)k;
    return 1024 * 4 * 12 * kMaxBasis;   // waves of k_basis_shade_bwd (grid <= 1024 x 4)
}

// The weight-gradient problems (at most 64 x 64 each) of both MLPs; with
// gr == NULL only the shapes (for sizing the partial sums).
static int basis_wgrad_specs(const gs3_grads* gr, bool phi, bool psi, WgSpec* spec) {
    int count = 0;
    auto ptr = [&](float* const* arr, int i, size_t off) -> float* { return gr ? arr[i] + off : nullptr; };
    auto add = [&](int dz_row, int in_row, int O, int J, int ldw, float* dW, float* db) {
        spec[count++] = WgSpec{dz_row, in_row, O, J, ldw, dW, db};
    };
    if (phi) {
        const int H = kPhiBasisHidden;
        add(kPhiB.dz1, kPhiB.x, H, kPhiBasisIn, kPhiBasisIn, ptr(gr ? gr->phi_w : nullptr, 0, 0),
            ptr(gr ? gr->phi_b : nullptr, 0, 0));
        add(kPhiB.dz2, kPhiB.h1, H, H, H, ptr(gr ? gr->phi_w : nullptr, 1, 0), ptr(gr ? gr->phi_b : nullptr, 1, 0));
        add(kPhiB.dz3, kPhiB.h2, H, H, H, ptr(gr ? gr->phi_w : nullptr, 2, 0), ptr(gr ? gr->phi_b : nullptr, 2, 0));
        add(kPhiB.dz4, kPhiB.h3, 1, H, H, ptr(gr ? gr->phi_w : nullptr, 3, 0), ptr(gr ? gr->phi_b : nullptr, 3, 0));
    }
    if (psi) {
        const int H = kPsiBasisHidden;
        float* const* W = gr ? gr->psi_w : nullptr;
        float* const* B = gr ? gr->psi_b : nullptr;
        // 64 x 64 problems (twice the workgroups of 128-wide ones, which
        // measured slower for all that they read each row once)
        for (int o = 0; o < H; o += 64)
            add(kPsiB.dz1 + o, kPsiB.x, 64, kPsiBasisIn, kPsiBasisIn, ptr(W, 0, (size_t)o * kPsiBasisIn), ptr(B, 0, o));
        for (int o = 0; o < H; o += 64)
            for (int j = 0; j < H; j += 64) {
                add(kPsiB.dz2 + o, kPsiB.h1 + j, 64, 64, H, ptr(W, 1, (size_t)o * H + j), j == 0 ? ptr(B, 1, o) : nullptr);
                add(kPsiB.dz3 + o, kPsiB.h2 + j, 64, 64, H, ptr(W, 2, (size_t)o * H + j), j == 0 ? ptr(B, 2, o) : nullptr);
            }
        for (int j = 0; j < H; j += 64) add(kPsiB.dz4, kPsiB.h3 + j, 3, 64, H, ptr(W, 3, j), j == 0 ? ptr(B, 3, 0) : nullptr);
    }
    return count;
}

int basis_wgrad_total_params() {
    WgSpec spec[16];
    const int count = basis_wgrad_specs(nullptr, true, true, spec);
    return wgrad_partial_floats(spec, count);
}

template <int MT, int KB, bool MASK>
static hipError_t layer_bwd(const float* W, int n_in, int n_out, float* rows, int dz_row, int h_row, int out_row,
                            int n, hipStream_t st) {
    LayerBwdArgs a{W, n_in, n_out, rows, dz_row, h_row, out_row, n};
    hipLaunchKernelGGL((k_mlp_layer_bwd<MT, KB, MASK>), dim3(grid_for(n, 4 * 16, 2048)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_basis_shade_bwd(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                                  const gs3_mlp* psi, const float* gcol, float* dT, const GradDev& g, float* rows,
                                  float* partial, const gs3_grads* gr, hipStream_t st) {
    if (sc.n == 0) return hipSuccess;
    const int n = sc.n;
    BasisArgs a = basis_args(sc, phi, psi);
    set_view(a.v[0], sp, T, nullptr, nullptr, nullptr);
    a.gcol = gcol;
    a.rows = rows;
    hipError_t e;
    // forward recompute with stored activations, output layers' adjoint
    if (psi) {
        constexpr int T = psi_threads(true);
        hipLaunchKernelGGL(k_basis_psi<true>, dim3(grid_for(n, T / 4, 256)), dim3(T), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        constexpr int P = kPsiBasisHidden / 16;
        if ((e = layer_bwd<P, P, true>(psi->w[2], kPsiBasisHidden, kPsiBasisHidden, rows, kPsiB.dz3, kPsiB.h2,
                                       kPsiB.dz2, n, st)) != hipSuccess)
            return e;
        if ((e = layer_bwd<P, P, true>(psi->w[1], kPsiBasisHidden, kPsiBasisHidden, rows, kPsiB.dz2, kPsiB.h1,
                                       kPsiB.dz1, n, st)) != hipSuccess)
            return e;
        if ((e = layer_bwd<kXin / 16, P, false>(psi->w[0], kPsiBasisIn, kPsiBasisHidden, rows, kPsiB.dz1, 0,
                                                kPsiB.dx, n, st)) != hipSuccess)
            return e;
    }
    if (phi) {
        static const int round = resident_blocks(k_basis_phi<true>, 256);
        hipLaunchKernelGGL(k_basis_phi<true>, dim3(grid_for(n, 4 * 16, round)), dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        constexpr int P = kPhiBasisHidden / 16;
        if ((e = layer_bwd<P, P, true>(phi->w[2], kPhiBasisHidden, kPhiBasisHidden, rows, kPhiB.dz3, kPhiB.h2,
                                       kPhiB.dz2, n, st)) != hipSuccess)
            return e;
        if ((e = layer_bwd<P, P, true>(phi->w[1], kPhiBasisHidden, kPhiBasisHidden, rows, kPhiB.dz2, kPhiB.h1,
                                       kPhiB.dz1, n, st)) != hipSuccess)
            return e;
        if ((e = layer_bwd<kXin / 16, P, false>(phi->w[0], kPhiBasisIn, kPhiBasisHidden, rows, kPhiB.dz1, 0,
                                                kPhiB.dx, n, st)) != hipSuccess)
            return e;
    }
    // scene gradients of the shading, encoding and directions
    ShadeBwdBasisArgs b;
    b.sc = sc;
    for (int i = 0; i < 3; ++i) {
        b.light[i] = sp.light[i];
        b.eye[i] = sp.eye[i];
    }
    b.light_dir = sp.light_dir;
    b.use_phi = phi != nullptr;
    b.use_psi = psi != nullptr;
    b.gcol = gcol;
    b.rows = rows;
    b.dT = dT;
    b.g = g;
    b.partial = partial;
    const int grid = grid_for(n, 256, 1024);
    hipLaunchKernelGGL(k_basis_shade_bwd, dim3(grid), dim3(256), 0, st, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sc.k > 0) {
        hipLaunchKernelGGL(k_basis_finish, dim3(sc.k), dim3(768), 0, st, sc, (const float*)partial, grid * 4, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!phi && !psi) return hipSuccess;
    // weight gradients, their partial sums after the per-wave basis sums
    WgSpec spec[16];
    const int count = basis_wgrad_specs(gr, phi != nullptr, psi != nullptr, spec);
    return launch_wgrad(spec, count, rows, n, partial + basis_partial_floats(sc.k), st);
}

}  // namespace gs3
