// MLP helpers shared by the shading kernel and its adjoint: the shadow
// refinement MLP Phi (Sec. 4.2, Eq. 8) and the residual MLP Psi (Sec. 4.3),
// each n_in -> 64 -> 64 -> 64 -> n_out with ReLU and a sigmoid output.
//
// A wave evaluates 16 Gaussians, four lanes per Gaussian (lane l: Gaussian
// l % 16, quarter q = l / 16), transposed, H^T = W X^T, so Gaussians are the
// N dimension. The hidden layers run on half-precision MFMA with every
// float32 operand split into two halves, x = hi + lo / 2048 (hi = x rounded
// to half, lo = the remainder scaled by 2048 so that it stays a normal
// half): W X = Wh Xh + (Wh Xl + Wl Xh) / 2048, the dropped Wl Xl / 2048^2
// term and the halves' rounding leave a relative error near 2^-22 per
// product, below the float32 accumulation's own. Three half-precision
// products cost far less than the four float32 ones (16x16x4) they replace.
// Operand layout of one 16x16x16 product (the input layer's first k-block
// kb, output tile mt):
//   A: lane l supplies W[16 mt + l%16][16 kb + 4 (l/16) + i], i = 0..3
//   B: lane l supplies X[g = l%16][16 kb + 4 (l/16) + i]
//   D: lane l holds H^T[16 mt + 4 (l/16) + i][l%16], i = 0..3,
// so the D registers of output tile m are exactly a 16-wide B operand of
// the next layer. The 64x64 hidden layers take 16x16x32 products (twice the
// rate of 16x16x16 on gfx950) over two 32-wide k-blocks, each pairing the D
// tiles 2 kb and 2 kb + 1 (kcol below), again with no transposes between
// layers. Activations above the half range (65504) are outside this
// scheme's domain.
// The adjoint recomputes the forward activations with the same routine (so
// its ReLU masks are the forward's); its products W^T dz use the same split
// form, each Gaussian's gradient column first scaled by a power of two.
#pragma once

#include "gs3_internal.h"

namespace gs3 {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int kPhiIn = 1 + kFeat;          // [T, feat]
constexpr int kPsiIn = kFeat + 6;          // [feat, w_i, w_o]
// The input layer's first 16 inputs form one split 16-wide k-block; the
// remaining ones run as float32 16x16x4 steps (padding them to a second
// 16-wide block would not fit the adjoint's LDS).
constexpr int kPhiKR = (kPhiIn - 16 + 3) / 4;   // float32 k-steps of the input layer
constexpr int kPsiKR = (kPsiIn - 16 + 3) / 4;
static_assert(kPhiIn >= 16 && kPsiIn >= 16, "the input layer's first k-block is full");
// LDS layout (floats) of one packed MLP: the input layer's first k-block per
// (output tile, lane) four floats holding the A operand's hi and lo halves,
// its float32 remainder per (output tile, k-step, lane) one float; a hidden
// layer per (output tile, 32-wide k-block) 512 floats (the 64 lanes' hi
// halves, then their lo halves)
constexpr int kLH = 4 * 4 * 64 * 4;          // a 64x64 hidden layer
struct MlpSmem {
    int l1, l1r, l2, l3, w4, b1, b2, b3, b4, size;
};
__host__ __device__ constexpr MlpSmem mlp_smem(int base, int kr, int n_out) {
    return MlpSmem{base,
                   base + 4 * 64 * 4,
                   base + 4 * 64 * 4 + 4 * kr * 64,
                   base + 4 * 64 * 4 + 4 * kr * 64 + kLH,
                   base + 4 * 64 * 4 + 4 * kr * 64 + 2 * kLH,
                   base + 4 * 64 * 4 + 4 * kr * 64 + 2 * kLH + n_out * 64,
                   base + 4 * 64 * 4 + 4 * kr * 64 + 2 * kLH + n_out * 64 + 64,
                   base + 4 * 64 * 4 + 4 * kr * 64 + 2 * kLH + n_out * 64 + 128,
                   base + 4 * 64 * 4 + 4 * kr * 64 + 2 * kLH + n_out * 64 + 192,
                   (4 * 64 * 4 + 4 * kr * 64 + 2 * kLH + n_out * 64 + 192 + 4 + 3) / 4 * 4};
}
constexpr MlpSmem kPhiS = mlp_smem(0, kPhiKR, 1);
constexpr MlpSmem kPsiS = mlp_smem(kPhiS.size, kPsiKR, 3);
constexpr int kShadeSmem = kPhiS.size + kPsiS.size;
static_assert(kPhiS.size % 4 == 0 && kPsiS.l1 % 4 == 0, "packed operands are read as 16-byte vectors");

struct MlpArgs {
    const float* w[4];
    const float* b[4];
};



// Adjoint of the quaternion -> rotation map (q normalised inside): dR -> dq.
__device__ inline void quat_grad(float qw, float qx, float qy, float qz, float qn, const float dR[9], float dq[4]) {
    // (qw..qz) is the normalised quaternion, qn the raw norm
    const float g00 = dR[0], g01 = dR[1], g02 = dR[2], g10 = dR[3], g11 = dR[4], g12 = dR[5], g20 = dR[6],
                g21 = dR[7], g22 = dR[8];
    const float dw = 2.f * (-qz * g01 + qy * g02 + qz * g10 - qx * g12 - qy * g20 + qx * g21);
    const float dx = 2.f * (qy * g01 + qz * g02 + qy * g10 - 2.f * qx * g11 - qw * g12 + qz * g20 + qw * g21 -
                            2.f * qx * g22);
    const float dy = 2.f * (-2.f * qy * g00 + qx * g01 + qw * g02 + qx * g10 + qz * g12 - qw * g20 + qz * g21 -
                            2.f * qy * g22);
    const float dz = 2.f * (-2.f * qz * g00 - qw * g01 + qx * g02 + qw * g10 - 2.f * qz * g11 + qy * g12 +
                            qx * g20 + qy * g21);
    const float dot = dw * qw + dx * qx + dy * qy + dz * qz;
    const float inv = 1.f / qn;
    dq[0] = (dw - dot * qw) * inv;
    dq[1] = (dx - dot * qx) * inv;
    dq[2] = (dy - dot * qy) * inv;
    dq[3] = (dz - dot * qz) * inv;
}

// x = hi + lo / 2048 with both parts half precision.
__device__ inline void split_half(float x, _Float16* hi, _Float16* lo) {
    const _Float16 h = (_Float16)x;
    *hi = h;
    *lo = (_Float16)((x - (float)h) * 2048.f);
}

// A 32-wide k-block pairs two 16-wide ones: slot j (0..7) of lane group g
// in block kb is column kcol(kb, g, j) = 32 kb + 16 (j / 4) + 4 g + j % 4,
// the entry that the D layout of tile 2 kb + j / 4 gives the lane. The
// 16x16x32 product takes slot j of lane group g of A and of B as the same
// k, so the activations of one layer feed the next one without a shuffle.
__device__ inline int kcol(int kb, int g, int j) { return 32 * kb + 16 * (j >> 2) + 4 * g + (j & 3); }

// One split product step over a 32-wide k-block: D += A B, the A halves
// read from a packed entry (hi halves of the 64 lanes, then the lo halves)
// at sm + off, the lane's offset included.
__device__ inline void mfma_split32(const float* sm, int off, halfx8 bh, halfx8 bl, floatx4* d, floatx4* dc) {
    const float4 vh = *reinterpret_cast<const float4*>(sm + off);
    const float4 vl = *reinterpret_cast<const float4*>(sm + off + 256);
    halfx8 ah, al;
    __builtin_memcpy(&ah, &vh, sizeof ah);
    __builtin_memcpy(&al, &vl, sizeof al);
    *d = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, *d, 0, 0, 0);
    *dc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, *dc, 0, 0, 0);
    *dc = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, *dc, 0, 0, 0);
}

// Pack A[r][c] (r < M a multiple of 16, c < K a multiple of 32) as split
// MFMA A operands: entry (mt, kb) holds 512 floats, first the hi halves of
// every lane (eight per lane, four floats) and then the lo halves, lane l
// holding A[16 mt + l % 16][kcol(kb, l / 16, j)], j = 0..7.
template <typename ElemFn>
__device__ inline void pack_split(float* sm, int M, int K, ElemFn elem) {
    const int KB = K / 32;
    for (int idx = threadIdx.x; idx < (M / 16) * KB * 64; idx += blockDim.x) {
        const int l = idx & 63, rest = idx >> 6, kb = rest % KB, mt = rest / KB;
        _Float16 hv[16];
#pragma unroll
        for (int j = 0; j < 8; ++j) split_half(elem(16 * mt + (l & 15), kcol(kb, l >> 4, j)), &hv[j], &hv[8 + j]);
        float4 v[2];
        __builtin_memcpy(v, hv, sizeof v);
        float* e = sm + 512 * rest + 4 * l;
        *reinterpret_cast<float4*>(e) = v[0];
        *reinterpret_cast<float4*>(e + 256) = v[1];
    }
}

// The B operand of a split product for the 16 Gaussians of the wave (x in
// D layout, KB 16-wide k-blocks, KB even): each Gaussian's column scaled by
// a power of two that brings its largest entry to [128, 256) and split
// into halves, two 16-wide blocks per 32-wide one; `down` undoes the
// scaling.
template <int KB>
struct SplitB {
    static_assert(KB % 2 == 0, "k is a multiple of 32");
    halfx8 h[KB / 2], l[KB / 2];
    float down;
};
template <int KB>
__device__ inline void split_cols(const floatx4* x, SplitB<KB>& b) {
    float m = 0.f;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) m = fmaxf(m, fabsf(x[kb][i]));
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    // m = f 2^e with f in [0.5, 1): the scale 2^(8 - e) (none for a zero
    // or infinite column, which then passes through as in float32)
    const int e = (m > 0.f && m < __builtin_inff()) ? max(ilogbf(m) + 1, -100) : 0;
    const float up = ldexpf(1.f, 8 - e);
    b.down = ldexpf(1.f, e - 8);
#pragma unroll
    for (int kb = 0; kb < KB / 2; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            _Float16 hi, lo;
            split_half(x[2 * kb + (j >> 2)][j & 3] * up, &hi, &lo);
            b.h[kb][j] = hi;
            b.l[kb][j] = lo;
        }
}

// Output tiles mt0 .. mt0 + CH - 1 of A x (A packed by pack_split from KB
// 16-wide k-blocks per row of tiles), D layout.
template <int KB, int CH>
__device__ inline void split_tiles(const float* sm, int lane, int mt0, const SplitB<KB>& b, floatx4* out) {
    floatx4 cor[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) out[c] = cor[c] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB / 2; ++kb)
#pragma unroll
        for (int c = 0; c < CH; ++c)
            mfma_split32(sm, 512 * ((mt0 + c) * (KB / 2) + kb) + 4 * lane, b.h[kb], b.l[kb], &out[c], &cor[c]);
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[c][i] = fmaf(cor[c][i], 1.f / 2048.f, out[c][i]) * b.down;
}

// out = A x for the 16 Gaussians of the wave (MT output tiles), two tiles
// at a time so that only the split operand and two tiles' accumulators are
// live beside the result.
template <int MT, int KB>
__device__ inline void split_gemm(const float* sm, int lane, const floatx4* x, floatx4* out) {
    SplitB<KB> b;
    split_cols<KB>(x, b);
    constexpr int CH = MT % 2 == 0 ? 2 : 1;
#pragma unroll
    for (int mt = 0; mt < MT; mt += CH) split_tiles<KB, CH>(sm, lane, mt, b, out + mt);
}

// Copy one MLP into LDS: hidden-layer and input-layer weights as split A
// operands, the output layer and biases as float32.
__device__ inline void load_mlp(float* sm, const MlpSmem& S, int kr, int n_in, int n_out, const MlpArgs& m) {
    const int tid = threadIdx.x, nt = blockDim.x;
    auto put = [&](int off, const float* W, int ld, int row, int col0, int ncol) {
        _Float16 hv[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int col = col0 + i;
            split_half(col < ncol ? W[row * ld + col] : 0.f, &hv[i], &hv[4 + i]);
        }
        float4 v;
        __builtin_memcpy(&v, hv, sizeof v);
        *reinterpret_cast<float4*>(sm + off) = v;
    };
    for (int idx = tid; idx < 4 * 64; idx += nt) {
        const int mt = idx / 64, l = idx % 64;
        put(S.l1 + 4 * idx, m.w[0], n_in, 16 * mt + (l & 15), 4 * (l >> 4), n_in);
    }
    for (int idx = tid; idx < 4 * kr * 64; idx += nt) {
        const int mt = idx / (kr * 64), rem = idx % (kr * 64), kk = rem / 64, l = rem % 64;
        const int row = 16 * mt + (l & 15), col = 16 + 4 * kk + (l >> 4);
        sm[S.l1r + idx] = col < n_in ? m.w[0][row * n_in + col] : 0.f;
    }
    // hidden layers as 16x16x32 operands: entry (mt, kb) of 512 floats, the
    // hi halves of the 64 lanes and then their lo halves
    auto put32 = [&](int off, const float* W, int row, int kb, int g) {
        _Float16 hv[16];
#pragma unroll
        for (int j = 0; j < 8; ++j) split_half(W[row * kHidden + kcol(kb, g, j)], &hv[j], &hv[8 + j]);
        float4 v[2];
        __builtin_memcpy(v, hv, sizeof v);
        *reinterpret_cast<float4*>(sm + off) = v[0];
        *reinterpret_cast<float4*>(sm + off + 256) = v[1];
    };
    for (int idx = tid; idx < 4 * 2 * 64; idx += nt) {
        const int l = idx & 63, rest = idx >> 6, kb = rest & 1, mt = rest >> 1;
        put32(S.l2 + 512 * rest + 4 * l, m.w[1], 16 * mt + (l & 15), kb, l >> 4);
        put32(S.l3 + 512 * rest + 4 * l, m.w[2], 16 * mt + (l & 15), kb, l >> 4);
    }
    for (int idx = tid; idx < n_out * 64; idx += nt) sm[S.w4 + idx] = m.w[3][idx];
    for (int idx = tid; idx < 64; idx += nt) {
        sm[S.b1 + idx] = m.b[0][idx];
        sm[S.b2 + idx] = m.b[1][idx];
        sm[S.b3 + idx] = m.b[2][idx];
    }
    for (int idx = tid; idx < n_out; idx += nt) sm[S.b4 + idx] = m.b[3][idx];
}

// One split product step: D += A B over a 16-wide k-block, with the A
// operand's halves read from LDS and B given as hi/lo halves.
__device__ inline void mfma_split(const float* sm, int off, halfx4 bh, halfx4 bl, floatx4* d, floatx4* dc) {
    const float4 v = *reinterpret_cast<const float4*>(sm + off);
    halfx4 ah, al;
    __builtin_memcpy(&ah, &v.x, sizeof ah);
    __builtin_memcpy(&al, &v.z, sizeof al);
    *d = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, *d, 0, 0, 0);
    *dc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl, *dc, 0, 0, 0);
    *dc = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh, *dc, 0, 0, 0);
}

__device__ inline void split_b(const float x[4], halfx4* bh, halfx4* bl) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        _Float16 h, l;
        split_half(x[i], &h, &l);
        (*bh)[i] = h;
        (*bl)[i] = l;
    }
}

__device__ inline float relu(float x) { return fmaxf(x, 0.f); }

// The three hidden layers of the forward; h[l][m][i] = layer l + 1, hidden
// unit 16 m + 4 q + i of Gaussian lane % 16 (D layout). Only the last layer
// is kept when ALL is false.
template <int KR, bool ALL, typename InFn>
__device__ inline void mlp_layers(const float* sm, const MlpSmem& S, int lane, InFn x_of_k,
                                  floatx4 (*h)[4]) {
    const int q = lane >> 4;
    floatx4 acc[4], cor[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = cor[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
    {
        float xv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[i] = x_of_k(4 * q + i);
        halfx4 bh, bl;
        split_b(xv, &bh, &bl);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) mfma_split(sm, S.l1 + 4 * (mt * 64 + lane), bh, bl, &acc[mt], &cor[mt]);
    }
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
        const float bx = x_of_k(16 + 4 * kk + q);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sm[S.l1r + (mt * KR + kk) * 64 + lane], bx, acc[mt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc[mt][i] = relu(fmaf(cor[mt][i], 1.f / 2048.f, acc[mt][i]) + sm[S.b1 + 16 * mt + 4 * q + i]);
    if (ALL) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h[0][mt] = acc[mt];
    }
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const int wl = layer == 0 ? S.l2 : S.l3;
        const int bl = layer == 0 ? S.b2 : S.b3;
        floatx4 nxt[4], ncor[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) nxt[mt] = ncor[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            halfx8 bh, bq;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                _Float16 hi, lo;
                split_half(acc[2 * kb + (j >> 2)][j & 3], &hi, &lo);
                bh[j] = hi;
                bq[j] = lo;
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) mfma_split32(sm, wl + 512 * (mt * 2 + kb) + 4 * lane, bh, bq, &nxt[mt], &ncor[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc[mt][i] = relu(fmaf(ncor[mt][i], 1.f / 2048.f, nxt[mt][i]) + sm[bl + 16 * mt + 4 * q + i]);
        if (ALL || layer == 1) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) h[ALL ? layer + 1 : 0][mt] = acc[mt];
        }
    }
}

// Three hidden layers; returns the last hidden activations in D layout.
template <int KR, typename InFn>
__device__ inline void mlp_hidden(const float* sm, const MlpSmem& S, int lane, InFn x_of_k, floatx4 h[4]) {
    mlp_layers<KR, false>(sm, S, lane, x_of_k, reinterpret_cast<floatx4(*)[4]>(h));
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
template <int KR, typename InFn>
__device__ inline void mlp_hidden_all(const float* sm, const MlpSmem& S, int lane, InFn x_of_k, floatx4 h[3][4]) {
    mlp_layers<KR, true>(sm, S, lane, x_of_k, h);
}

// LDS layout (floats) of one MLP's transposed weights for the adjoint, as
// split operands packed by pack_split: W1^T as two 16-row tiles (input rows
// 0..31, zero past n_in), W2^T, W3^T.
struct MlpTSmem {
    int t1, t2, t3, size;
};
__host__ __device__ constexpr MlpTSmem mlp_tsmem(int base) {
    return MlpTSmem{base, base + 2 * 16 * 64, base + 2 * 16 * 64 + kLH, 2 * 16 * 64 + 2 * kLH};
}

// Pack W^T into LDS: row j of the product is the layer's input j, the
// contraction runs over the layer's outputs o.
__device__ inline void load_mlp_t(float* sm, const MlpTSmem& T, int n_in, const MlpArgs& m) {
    pack_split(sm + T.t1, 32, kHidden, [&](int j, int o) { return j < n_in ? m.w[0][o * n_in + j] : 0.f; });
    pack_split(sm + T.t2, kHidden, kHidden, [&](int j, int o) { return m.w[1][o * kHidden + j]; });
    pack_split(sm + T.t3, kHidden, kHidden, [&](int j, int o) { return m.w[2][o * kHidden + j]; });
}

// d = W^T g for a 64-wide g in D layout, TILES output tiles of 16 rows: the
// split product of the forward, each Gaussian's gradient column scaled by a
// power of two before the split (gradients can be of any size).
template <int TILES>
__device__ inline void mlp_back_layer(const float* sm, int off, int lane, const floatx4 g[4], floatx4 d[TILES]) {
    split_gemm<TILES, 4>(sm + off, lane, g, d);
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
