// D-SSIM term of the training loss (Sec. 4.4, Eq. 9) and its gradient.
//
// Per channel and pixel p, with G the 11x11 Gaussian window (sigma 1.5,
// separable, zero outside the image):
//   mu_x = G*x, mu_y = G*y, Exx = G*(x x), Eyy = G*(y y), Exy = G*(x y),
//   s = (2 mu_x mu_y + C1)(2 (Exy - mu_x mu_y) + C2) /
//       ((mu_x^2 + mu_y^2 + C1)(Exx - mu_x^2 + Eyy - mu_y^2 + C2)),
// and the loss is scale * sum (1 - s). Only the prediction x is
// differentiated. s at q depends on x(p) through mu_x(q), Exx(q) and
// Exy(q), each a window sum around q, so
//   dL/dx(p) = (G*a)(p) + 2 x(p) (G*b)(p) + y(p) (G*c)(p)
// with the per-pixel maps a = -scale ds/dmu_x, b = -scale ds/dExx,
// c = -scale ds/dExy (G is symmetric, so the adjoint of the window sum is
// the same window sum).
//
// Two kernels, each over 16x16 output tiles with a 5-pixel halo staged in
// LDS and the window applied as a horizontal then a vertical 11-tap pass:
//   k_ssim_fwd  the five window sums, s, one float64 partial sum of 1 - s per
//               tile, and the maps a, b, c (workspace);
//   k_ssim_bwd  the three window sums of a, b, c and the gradient.
// A final one-workgroup kernel adds the partial sums in tile order (a fixed
// order: the same bits on every run).
#include "gs3_internal.h"

namespace gs3 {

constexpr int kSsimR = 5;                      // window radius
constexpr int kSsimT = 16;                     // output tile edge
constexpr int kSsimE = kSsimT + 2 * kSsimR;    // staged edge, 26
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct SsimWin {
    float w[2 * kSsimR + 1];
};

// Horizontal 11-tap pass over the staged rows: out[r][c] for the 26 staged
// rows and the 16 output columns.
template <int NM>
__device__ inline void hpass(const float (*in)[kSsimE][kSsimE], float (*out)[kSsimE][kSsimT], const SsimWin& W) {
    for (int i = threadIdx.x; i < kSsimE * kSsimT; i += 256) {
        const int r = i / kSsimT, c = i % kSsimT;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t <= 2 * kSsimR; ++t) acc = fmaf(W.w[t], in[m][r][c + t], acc);
            out[m][r][c] = acc;
        }
    }
}

__device__ inline double block_sum_256(double x, double* s_part) {
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_part[w] = x;
    __syncthreads();
    const double t = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
    __syncthreads();
    return t;
}

// grid (tiles_x, tiles_y, channels); 256 threads, one per output pixel.
__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                   int W, float scale, SsimWin win, float* __restrict__ amap,
                                                   float* __restrict__ bmap, float* __restrict__ cmap,
                                                   double* __restrict__ partial) {
    __shared__ float s_in[5][kSsimE][kSsimE];     // x, y, xx, yy, xy with halo
    __shared__ float s_h[5][kSsimE][kSsimT];      // after the horizontal pass
    __shared__ double s_part[4];
    const int ch = blockIdx.z;
    const int ox = blockIdx.x * kSsimT - kSsimR, oy = blockIdx.y * kSsimT - kSsimR;
    const size_t plane = (size_t)H * W;
    const float* xc = x + ch * plane;
    const float* yc = y + ch * plane;
    for (int i = threadIdx.x; i < kSsimE * kSsimE; i += 256) {
        const int r = i / kSsimE, c = i % kSsimE;
        const int gy = oy + r, gx = ox + c;
        float xv = 0.f, yv = 0.f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            xv = xc[(size_t)gy * W + gx];
            yv = yc[(size_t)gy * W + gx];
        }
        s_in[0][r][c] = xv;
        s_in[1][r][c] = yv;
        s_in[2][r][c] = xv * xv;
        s_in[3][r][c] = yv * yv;
        s_in[4][r][c] = xv * yv;
    }
    __syncthreads();
    hpass<5>(s_in, s_h, win);
    __syncthreads();
    const int tx = threadIdx.x % kSsimT, ty = threadIdx.x / kSsimT;
    const int px = blockIdx.x * kSsimT + tx, py = blockIdx.y * kSsimT + ty;
    float st[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) acc = fmaf(win.w[t], s_h[m][ty + t][tx], acc);
        st[m] = acc;
    }
    double loss = 0.0;
    if (px < W && py < H) {
        const float mx = st[0], my = st[1];
        const float sxx = st[2] - mx * mx, syy = st[3] - my * my, sxy = st[4] - mx * my;
        const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
        const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
        const float s = (A1 * A2) / (B1 * B2);
        loss = 1.0 - (double)s;
        const size_t p = ch * plane + (size_t)py * W + px;
        // ds/dmu_x = s (2 mu_y / A1 - 2 mu_y / A2 - 2 mu_x / B1 + 2 mu_x / B2),
        // ds/dExx = -s / B2, ds/dExy = 2 s / A2
        const float dmu = s * (2.f * my / A1 - 2.f * my / A2 - 2.f * mx / B1 + 2.f * mx / B2);
        amap[p] = -scale * dmu;
        bmap[p] = scale * s / B2;
        cmap[p] = -scale * 2.f * s / A2;
    }
    const double t = block_sum_256(loss, s_part);
    if (threadIdx.x == 0)
        partial[((size_t)ch * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                   int W, SsimWin win, const float* __restrict__ amap,
                                                   const float* __restrict__ bmap, const float* __restrict__ cmap,
                                                   float* __restrict__ grad, int accumulate) {
    __shared__ float s_in[3][kSsimE][kSsimE];
    __shared__ float s_h[3][kSsimE][kSsimT];
    const int ch = blockIdx.z;
    const int ox = blockIdx.x * kSsimT - kSsimR, oy = blockIdx.y * kSsimT - kSsimR;
    const size_t plane = (size_t)H * W;
    for (int i = threadIdx.x; i < kSsimE * kSsimE; i += 256) {
        const int r = i / kSsimE, c = i % kSsimE;
        const int gy = oy + r, gx = ox + c;
        float av = 0.f, bv = 0.f, cv = 0.f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const size_t p = ch * plane + (size_t)gy * W + gx;
            av = amap[p];
            bv = bmap[p];
            cv = cmap[p];
        }
        s_in[0][r][c] = av;
        s_in[1][r][c] = bv;
        s_in[2][r][c] = cv;
    }
    __syncthreads();
    hpass<3>(s_in, s_h, win);
    __syncthreads();
    const int tx = threadIdx.x % kSsimT, ty = threadIdx.x / kSsimT;
    const int px = blockIdx.x * kSsimT + tx, py = blockIdx.y * kSsimT + ty;
    if (px >= W || py >= H) return;
    float st[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) acc = fmaf(win.w[t], s_h[m][ty + t][tx], acc);
        st[m] = acc;
    }
    const size_t p = ch * plane + (size_t)py * W + px;
    const float g = st[0] + 2.f * x[p] * st[1] + y[p] * st[2];
    grad[p] = accumulate ? grad[p] + g : g;
}

__global__ __launch_bounds__(256) void k_ssim_final(const double* __restrict__ partial, int64_t count, float scale,
                                                     float* __restrict__ loss) {
    __shared__ double s_part[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) acc += partial[i];
    const double t = block_sum_256(acc, s_part);
    if (threadIdx.x == 0) *loss = (float)(t * (double)scale);
}

SsimLayout ssim_layout(int channels, int height, int width) {
    SsimLayout L;
    const size_t plane = (size_t)channels * height * width;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    L.tiles_x = (width + kSsimT - 1) / kSsimT;
    L.tiles_y = (height + kSsimT - 1) / kSsimT;
    L.amap = 0;
    L.bmap = up(4 * plane);
    L.cmap = L.bmap + up(4 * plane);
    L.partial = L.cmap + up(4 * plane);
    L.total = L.partial + up(8 * (size_t)channels * L.tiles_x * L.tiles_y + 8);
    return L;
}

hipError_t launch_dssim(const float* pred, const float* target, int channels, int height, int width, float scale,
                        float* loss, float* grad, int accumulate, void* ws, hipStream_t st) {
    const SsimLayout L = ssim_layout(channels, height, width);
    // the normalised window in double, rounded once to float
    SsimWin win;
    double g[2 * kSsimR + 1], sum = 0.0;
    for (int t = -kSsimR; t <= kSsimR; ++t) sum += (g[t + kSsimR] = exp(-(double)(t * t) / (2.0 * 1.5 * 1.5)));
    for (int t = 0; t <= 2 * kSsimR; ++t) win.w[t] = (float)(g[t] / sum);
    float* amap = at<float>(ws, L.amap);
    float* bmap = at<float>(ws, L.bmap);
    float* cmap = at<float>(ws, L.cmap);
    double* partial = at<double>(ws, L.partial);
    const dim3 grid((unsigned)L.tiles_x, (unsigned)L.tiles_y, (unsigned)channels);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, st, pred, target, height, width, scale, win, amap, bmap, cmap,
                       partial);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, st, partial,
                       (int64_t)channels * L.tiles_x * L.tiles_y, scale, loss);
    if (grad)
        hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, st, pred, target, height, width, win, amap, bmap, cmap,
                           grad, accumulate);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Adam
//
// One Adam update per element (the optimiser of Sec. 4.4): m and v are the
// first and second moment estimates, c1 = 1 / (1 - b1^t), c2 =
// 1 / (1 - b2^t) the bias corrections (computed on the host in double).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                               float* __restrict__ m, float* __restrict__ v, int64_t count, float lr,
                                               float b1, float b2, float eps, float c1, float c2) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
        const float gi = g[i];
        const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, int step, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const float c1 = (float)(1.0 / (1.0 - pow((double)b1, step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)b2, step)));
    int64_t grid = (count + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)grid), dim3(256), 0, st, p, g, m, v, count, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace gs3
