// MLP helpers shared by the shading kernel and its adjoint: the shadow
// refinement MLP Phi (Sec. 4.2, Eq. 8) and the residual MLP Psi (Sec. 4.3),
// each n_in -> 64 -> 64 -> 64 -> n_out with ReLU and a sigmoid output.
//
// A wave evaluates 16 Gaussians, four lanes per Gaussian (lane l: Gaussian
// l % 16, quarter q = l / 16), transposed, H^T = W X^T, on
// v_mfma_f32_16x16x4_f32, so Gaussians are the N dimension:
//   B operand of k-step kk: lane l supplies X[g = l%16][4 kk + l/16]
//   A operand: W[16 mt + l%16][4 kk + l/16]
//   D: lane l holds H^T[16 mt + 4 (l/16) + i][l%16], i = 0..3.
// Because the contraction order over the hidden index is free, the D
// registers of one layer are fed directly as the B operand of the next
// (k-step (m, i) <-> hidden 16 m + 4 (l/16) + i) and the weights are packed
// in LDS in that permuted order, so no transposes are needed between layers.
// The adjoint runs the same scheme with W^T packed the same way.
#pragma once

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


// All three hidden layers of the forward, in D layout (h[l][m][i] = layer
// l + 1, hidden unit 16 m + 4 q + i of Gaussian lane % 16), for the adjoint.
template <int K1, typename InFn>
__device__ inline void mlp_hidden_all(const float* sm, const MlpSmem& S, int lane, InFn x_of_k, floatx4 h[3][4]) {
    const int q = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) h[0][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < K1; ++kk) {
        const float bx = x_of_k(4 * kk + q);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            h[0][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sm[S.l1 + (mt * K1 + kk) * 64 + lane], bx, h[0][mt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h[0][mt][i] = relu(h[0][mt][i] + sm[S.b1 + 16 * mt + 4 * q + i]);
#pragma unroll
    for (int layer = 1; layer < 3; ++layer) {
        const int wl = layer == 1 ? S.l2 : S.l3;
        const int bl = layer == 1 ? S.b2 : S.b3;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h[layer][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ks = 4 * m + i;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    h[layer][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sm[wl + (mt * 16 + ks) * 64 + lane],
                                                                        h[layer - 1][m][i], h[layer][mt], 0, 0, 0);
            }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) h[layer][mt][i] = relu(h[layer][mt][i] + sm[bl + 16 * mt + 4 * q + i]);
    }
}

// LDS layout (floats) of one MLP's transposed weights for the adjoint:
// W1^T as two 16-row tiles (input rows 0..31, zero past n_in), W2^T, W3^T.
struct MlpTSmem {
    int t1, t2, t3, size;
};
__host__ __device__ constexpr MlpTSmem mlp_tsmem(int base) {
    return MlpTSmem{base, base + 2 * 16 * 64, base + 2 * 16 * 64 + kLH, 2 * 16 * 64 + 2 * kLH};
}

// Copy W^T into LDS in the A-operand order of the adjoint: for output tile
// mt (rows j = 16 mt + l%16 of the layer's input) and k-step ks = 4 m + i
// (contraction over the layer's output o = 16 m + 4 (l/16) + i), lane l
// holds W[o][j].
__device__ inline void load_mlp_t(float* sm, const MlpTSmem& T, int n_in, const MlpArgs& m) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < 2 * 16 * 64; idx += nt) {
        const int mt = idx / 1024, rem = idx % 1024, ks = rem / 64, l = rem % 64;
        const int j = 16 * mt + (l & 15), o = 16 * (ks >> 2) + 4 * (l >> 4) + (ks & 3);
        sm[T.t1 + idx] = j < n_in ? m.w[0][o * n_in + j] : 0.f;
    }
    for (int idx = tid; idx < kLH; idx += nt) {
        const int mt = idx / 1024, rem = idx % 1024, ks = rem / 64, l = rem % 64;
        const int j = 16 * mt + (l & 15), o = 16 * (ks >> 2) + 4 * (l >> 4) + (ks & 3);
        sm[T.t2 + idx] = m.w[1][o * kHidden + j];
        sm[T.t3 + idx] = m.w[2][o * kHidden + j];
    }
}

// d = W^T g for a 64-wide g in D layout, TILES output tiles of 16 rows.
template <int TILES>
__device__ inline void mlp_back_layer(const float* sm, int off, int lane, const floatx4 g[4], floatx4 d[TILES]) {
#pragma unroll
    for (int mt = 0; mt < TILES; ++mt) d[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ks = 4 * m + i;
#pragma unroll
            for (int mt = 0; mt < TILES; ++mt)
                d[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sm[off + (mt * 16 + ks) * 64 + lane], g[m][i], d[mt], 0,
                                                             0, 0);
        }
}

// Adjoint of the hidden layers. In: dh3 = dL/dh3 (D layout) and the
// forward's h. Each pre-activation gradient dz_l (D layout) is handed to
// store(l, dz) as soon as it is formed (l = 0, 1, 2 for layers 1..3); out:
// dx = dL/dinput, two 16-row tiles in D layout.
template <typename StoreFn>
__device__ inline void mlp_backward(const float* sm, const MlpTSmem& T, int lane, const floatx4 h[3][4],
                                    const floatx4 dh3[4], StoreFn store, floatx4 dx[2]) {
    floatx4 dz[4], d[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) dz[m][i] = h[2][m][i] > 0.f ? dh3[m][i] : 0.f;
    store(2, dz);
    mlp_back_layer<4>(sm, T.t3, lane, dz, d);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) dz[m][i] = h[1][m][i] > 0.f ? d[m][i] : 0.f;
    store(1, dz);
    mlp_back_layer<4>(sm, T.t2, lane, dz, d);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) dz[m][i] = h[0][m][i] > 0.f ? d[m][i] : 0.f;
    store(0, dz);
    mlp_back_layer<2>(sm, T.t1, lane, dz, dx);
}

// ReLU pattern of a 64-wide activation in D layout: bit 4 m + i set when
// h[m][i] > 0 (the lane's 16 values).
__device__ inline uint32_t relu_mask(const floatx4 h[4]) {
    uint32_t b = 0u;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) b |= (h[m][i] > 0.f ? 1u : 0u) << (4 * m + i);
    return b;
}

// mlp_backward with the forward's activations given only by their ReLU
// patterns (relu_mask of h1, h2, h3), which is all the adjoint reads of them.
template <typename StoreFn>
__device__ inline void mlp_backward_masked(const float* sm, const MlpTSmem& T, int lane, const uint32_t mask[3],
                                           const floatx4 dh3[4], StoreFn store, floatx4 dx[2]) {
    floatx4 dz[4], d[4];
    auto gate = [&](uint32_t mk, const floatx4 in[4]) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) dz[m][i] = ((mk >> (4 * m + i)) & 1u) ? in[m][i] : 0.f;
    };
    gate(mask[2], dh3);
    store(2, dz);
    mlp_back_layer<4>(sm, T.t3, lane, dz, d);
    gate(mask[1], d);
    store(1, dz);
    mlp_back_layer<4>(sm, T.t2, lane, dz, d);
    gate(mask[0], d);
    store(0, dz);
    mlp_back_layer<2>(sm, T.t1, lane, dz, dx);
}

}  // namespace gs3
