// Shadow splatting (Sec. 4.2, Fig. 3): the second of the three splats.
//
// For Gaussian j, T_j = num_j / den_j with
//   num_j = sum_m beta_jm T_m(j),   den_j = sum_m beta_jm
// over the light pixels m (shadow rays) it hits, where T_m(j) is the
// product of (1 - alpha_km) over the Gaussians k hit at m with
// dist_k < dist_j - bias (Eq. 3 with the shadow bias of Sec. 4.2).
//
// The two sums are computed by two kernels:
//  - den does not depend on occlusion, so k_shadow_den sums beta over each
//    Gaussian's own footprint (one wave per Gaussian, one reduction per
//    Gaussian instead of one per tile and splat);
//  - num needs the depth order: k_shadow walks each 16x16 light tile's
//    distance-sorted list. A tile-uniform trailing pointer follows the
//    leading one and multiplies the per-pixel T_trail by (1 - alpha_k) as k
//    falls more than `bias` behind; records of the last two batches stay in
//    an LDS ring, older ones are re-staged from global memory. Once a
//    pixel's T_trail is below kShadowEps every later term of that pixel is
//    below kShadowEps * beta, so dropping them moves T_j by less than
//    kShadowEps; a wave whose 64 pixels are all there stops, and so does the
//    workgroup. In an opaque scene this leaves only the splats near the
//    lit surface to evaluate.
// Both kernels test pixels with the same float32 arithmetic (stage_coeffs,
// rel_centre, quad_q), so num and den see exactly the same hits.
#include "splat_common.h"

namespace gs3 {

constexpr float kShadowEps = 9.5367431640625e-07f;   // 2^-20

struct ShadowArgs {
    const int2* ranges;
    const uint32_t* list;
    const float4* rec0;
    const float4* rec1;
    const float* depth;
    const int4* ext;
    uint32_t n;
    int width, height, tiles_x;
    float cutoff, alpha_min, alpha_max, bias;
    float* num;
    float* den;
};

__global__ __launch_bounds__(256) void k_shadow(ShadowArgs a) {
    __shared__ Staged s_rec[512];      // ring: list position (p - s) & 511
    __shared__ uint32_t s_mask[512];
    __shared__ uint32_t s_id[256];
    __shared__ float s_part[4][256];
    const int tile = blockIdx.x;
    const int2 rg = a.ranges[tile];
    const int s = rg.x, e = rg.y;
    if (e <= s) return;  // uniform
    const int tid = threadIdx.x, w = tid >> 6, lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int lx = (w & 1) * 8 + (lane & 7), ly = (w >> 1) * 8 + (lane >> 3);
    const bool inside = (tx * kTile + lx < a.width) && (ty * kTile + ly < a.height);
    const float pxc = lx + 0.5f, pyc = ly + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    const uint32_t wbit = 1u << w;
    float t_trail = 1.f;
    bool alive = inside;
    int trail = s;
    for (int b = s; b < e; b += 256) {
        if (__syncthreads_count(alive) == 0) break;   // every pixel of the tile is dark
        const int m = min(256, e - b);
        const int base = (b - s) & 511;
        if (tid < m) {
            const uint32_t id = safe_id(a.list[b + tid], a.n);
            uint32_t mk;
            s_rec[base + tid] = stage_splat(id, a.rec0, a.rec1, a.depth, tile_x0, tile_y0, a.cutoff, a.alpha_min, &mk);
            s_mask[base + tid] = mk;
            s_id[tid] = id;
        }
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) s_part[ww][tid] = 0.f;
        __syncthreads();
        if (__ballot(alive)) {
            for (int j = 0; j < m; ++j) {
                const float thr_d = s_rec[base + j].g1.w - a.bias;
                // trailing pointer: every k with dist_k < dist_j - bias shadows j
                while (trail < b + j) {
                    Staged tk;
                    uint32_t tm;
                    if (trail >= b - 256) {
                        tk = s_rec[(trail - s) & 511];
                        tm = s_mask[(trail - s) & 511];
                    } else {
                        tk = stage_splat(safe_id(a.list[trail], a.n), a.rec0, a.rec1, a.depth, tile_x0, tile_y0,
                                         a.cutoff, a.alpha_min, &tm);
                    }
                    if (!(tk.g1.w < thr_d)) break;
                    if (tm & wbit) {
                        const float q = splat_q(tk, pxc, pyc);
                        if (alive && q >= tk.g1.y) t_trail *= 1.f - fminf(a.alpha_max, tk.g1.z * fast_exp2(q));
                    }
                    ++trail;
                }
                alive = alive && t_trail >= kShadowEps;
                if (!__ballot(alive)) break;       // the wave's pixels are all dark
                const Staged sj = s_rec[base + j];
                const uint32_t mj = s_mask[base + j];
                if (mj & wbit) {
                    const float q = splat_q(sj, pxc, pyc);
                    const bool hit = alive && q >= sj.g1.y;
                    if (__ballot(hit)) {
                        const float vn = hit ? fast_exp2(q) * t_trail : 0.f;
                        const float sn = wave_sum_lane63(vn);
                        if (lane == 63) s_part[w][j] = sn;
                    }
                }
            }
        }
        __syncthreads();
        if (tid < m) {
            const float v = (s_part[0][tid] + s_part[1][tid]) + (s_part[2][tid] + s_part[3][tid]);
            if (v > 0.f) atomicAdd(&a.num[s_id[tid]], v);
        }
    }
}

// den_j = sum of beta over the pixels of the light image Gaussian j hits.
// One wave per Gaussian walks the 16x4 pixel blocks of the tiles it is
// binned to (the same pixels the tile kernel tests), skipping blocks outside
// the hit ellipse's bounding box. The centre is formed relative to each
// tile's origin exactly as in stage_splat, so every pixel test is
// bit-identical to the one k_shadow makes.
__global__ __launch_bounds__(256) void k_shadow_den(ShadowArgs a) {
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const int lx = lane & 15, ly = lane >> 4;
    const int n = (int)a.n;
    const int tiles_y = (a.height + kTile - 1) / kTile;
    for (int g = blockIdx.x * 4 + w; g < n; g += gridDim.x * 4) {
        const int4 ex = a.ext[g];
        float acc = 0.f;
        int x0, x1, y0, y1;
        if (tile_rect_i(ex.x, ex.y, ex.z, ex.w, a.tiles_x, tiles_y, &x0, &x1, &y0, &y1)) {
            const float4 r0 = a.rec0[g];
            const float4 r1 = a.rec1[g];
            float A, B, C, thr;
            const float p = stage_coeffs(r1, a.cutoff, a.alpha_min, &A, &B, &C, &thr);
            float hx = 3.0e38f, hy = 3.0e38f;
            if (!isinf(p)) {
                const float det = r1.x * r1.z - r1.y * r1.y;
                hx = sqrtf(fmaxf(2.f * p * r1.z / det, 0.f)) * 1.01f + 0.01f;
                hy = sqrtf(fmaxf(2.f * p * r1.x / det, 0.f)) * 1.01f + 0.01f;
            }
            if (p > 0.f) {
                for (int ty = y0; ty <= y1; ++ty) {
                    const float oy = (float)(ty * kTile);
                    const float v = rel_centre(r0.y, r0.w, oy);
                    for (int tx = x0; tx <= x1; ++tx) {
                        const float ox = (float)(tx * kTile);
                        const float u = rel_centre(r0.x, r0.z, ox);
                        if (u + hx < 0.5f || u - hx > 15.5f) continue;
                        const float dx = (float)lx + 0.5f - u;
                        const bool in_x = tx * kTile + lx < a.width;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float yb = (float)(4 * r);
                            if (v + hy < yb + 0.5f || v - hy > yb + 3.5f) continue;
                            const float dy = (float)(4 * r + ly) + 0.5f - v;
                            const float q = quad_q(dx, dy, A, B, C);
                            const bool hit = in_x && (ty * kTile + 4 * r + ly < a.height) && q >= thr;
                            acc += hit ? fast_exp2(q) : 0.f;
                        }
                    }
                }
            }
        }
        const float sum = wave_sum_lane63(acc);
        if (lane == 63) a.den[g] = sum;
    }
}

__global__ __launch_bounds__(256) void k_shadow_finish(const float* __restrict__ num, const float* __restrict__ den,
                                                        float* __restrict__ T, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) T[i] = den[i] > 0.f ? num[i] / den[i] : 1.f;
}

hipError_t launch_shadow(const gs3_consts& k, const Layout& L, const void* ws, float* num_den, float* T,
                         hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(num_den), 0u, L.n, st);
    if (e != hipSuccess) return e;
    ShadowArgs a;
    a.ranges = at<int2>(ws, L.ranges);
    a.list = at<uint32_t>(ws, L.pv_a);
    a.rec0 = at<float4>(ws, L.rec0);
    a.rec1 = at<float4>(ws, L.rec1);
    a.depth = at<float>(ws, L.depth);
    a.ext = at<int4>(ws, L.ext);
    a.n = (uint32_t)L.n;
    a.width = L.width;
    a.height = L.height;
    a.tiles_x = L.tiles_x;
    a.cutoff = k.cutoff;
    a.alpha_min = k.alpha_min;
    a.alpha_max = k.alpha_max;
    a.bias = k.shadow_bias;
    a.num = num_den;
    a.den = num_den + L.n;
    int den_grid = (int)((L.n + 3) / 4);
    if (den_grid > 8192) den_grid = 8192;
    hipLaunchKernelGGL(k_shadow_den, dim3(den_grid), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_shadow, dim3((unsigned)L.n_tiles), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_shadow_finish, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, a.num, a.den, T,
                       (int)L.n);
    return hipGetLastError();
}

}  // namespace gs3
