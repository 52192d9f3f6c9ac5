// Shadow splatting (Sec. 4.2, Fig. 3): the second of the three splats.
//
// One workgroup per 16x16 tile of the light image, one lane per light pixel
// (shadow ray m), wave w owning the 8x8 quadrant w. The tile's splats arrive
// sorted by distance to the light. For each splat j hit at pixel m the
// transmittance in front of it is T_m(j) = prod (1 - alpha_km) over the
// splats k hit at m with dist_k < dist_j - bias (Eq. 3 with the shadow bias
// of Sec. 4.2). A tile-uniform trailing pointer walks the same list behind
// the leading one and multiplies a per-pixel T_trail by (1 - alpha_k) as k
// falls more than `bias` behind; records of the last two batches stay in an
// LDS ring, older ones are re-staged from global memory.
//
// Per splat the workgroup reduces sum_m beta_jm T_m(j) and sum_m beta_jm
// over its 256 pixels (DPP wave sums, then the four waves in LDS) and adds
// them to num[j], den[j] with one atomic each. The denominator needs every
// hit, so there is no early termination here.
#include "splat_common.h"

namespace gs3 {

struct ShadowArgs {
    const int2* ranges;
    const uint32_t* list;
    const float4* rec0;
    const float4* rec1;
    const float* depth;
    uint32_t n;
    int width, height, tiles_x;
    float cutoff, alpha_min, alpha_max, bias;
    float* num;
    float* den;
};

__global__ __launch_bounds__(256) void k_shadow(ShadowArgs a) {
    __shared__ Staged s_rec[2][256];
    __shared__ uint32_t s_mask[2][256];
    __shared__ uint32_t s_id[256];
    __shared__ float2 s_part[4][256];
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
    int trail = s;
    int slot = 0;
    for (int b = s; b < e; b += 256, slot ^= 1) {
        const int m = min(256, e - b);
        if (tid < m) {
            const uint32_t id = safe_id(a.list[b + tid], a.n);
            uint32_t mk;
            s_rec[slot][tid] = stage_splat(id, a.rec0, a.rec1, a.depth, tile_x0, tile_y0, a.cutoff, a.alpha_min, &mk);
            s_mask[slot][tid] = mk;
            s_id[tid] = id;
        }
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) s_part[ww][tid] = make_float2(0.f, 0.f);
        __syncthreads();
        for (int j = 0; j < m; ++j) {
            const float thr_d = s_rec[slot][j].g1.w - a.bias;
            // trailing pointer: every k with dist_k < dist_j - bias has shadowed j
            while (trail < b + j) {
                Staged tk;
                uint32_t tm;
                if (trail >= b) {
                    tk = s_rec[slot][trail - b];
                    tm = s_mask[slot][trail - b];
                } else if (trail >= b - 256) {
                    tk = s_rec[slot ^ 1][trail - (b - 256)];
                    tm = s_mask[slot ^ 1][trail - (b - 256)];
                } else {
                    tk = stage_splat(safe_id(a.list[trail], a.n), a.rec0, a.rec1, a.depth, tile_x0, tile_y0, a.cutoff,
                                     a.alpha_min, &tm);
                }
                if (!(tk.g1.w < thr_d)) break;
                if (tm & wbit) {
                    const float q = splat_q(tk, pxc, pyc);
                    if (inside && q >= tk.g1.y) {
                        const float al = fminf(a.alpha_max, tk.g1.z * exp2f(q));
                        t_trail *= 1.f - al;
                    }
                }
                ++trail;
            }
            if (s_mask[slot][j] & wbit) {
                const Staged sj = s_rec[slot][j];
                const float q = splat_q(sj, pxc, pyc);
                const bool hit = inside && q >= sj.g1.y;
                if (__ballot(hit)) {
                    const float beta = exp2f(q);
                    const float vn = hit ? beta * t_trail : 0.f;
                    const float vd = hit ? beta : 0.f;
                    const float sn = wave_sum_lane63(vn);
                    const float sd = wave_sum_lane63(vd);
                    if (lane == 63) s_part[w][j] = make_float2(sn, sd);
                }
            }
        }
        __syncthreads();
        if (tid < m) {
            const float2 p0 = s_part[0][tid], p1 = s_part[1][tid], p2 = s_part[2][tid], p3 = s_part[3][tid];
            const float dn = (p0.y + p1.y) + (p2.y + p3.y);
            if (dn > 0.f) {
                const uint32_t id = s_id[tid];
                atomicAdd(&a.num[id], (p0.x + p1.x) + (p2.x + p3.x));
                atomicAdd(&a.den[id], dn);
            }
        }
        __syncthreads();
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
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(num_den), 0u, 2 * L.n, st);
    if (e != hipSuccess) return e;
    ShadowArgs a;
    a.ranges = at<int2>(ws, L.ranges);
    a.list = at<uint32_t>(ws, L.pv_a);
    a.rec0 = at<float4>(ws, L.rec0);
    a.rec1 = at<float4>(ws, L.rec1);
    a.depth = at<float>(ws, L.depth);
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
    hipLaunchKernelGGL(k_shadow, dim3((unsigned)L.n_tiles), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_shadow_finish, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, a.num, a.den, T,
                       (int)L.n);
    return hipGetLastError();
}

}  // namespace gs3
