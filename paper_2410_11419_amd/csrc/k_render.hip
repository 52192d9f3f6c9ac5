// Camera splatting (Sec. 3 Eq. 2-3; Sec. 4 and Fig. 2): the third splat.
//
// One workgroup per 16x16 tile of the camera image, one lane per pixel, wave
// w owning the 8x8 quadrant w. Splats arrive sorted by view depth and are
// blended front to back into three images at once: the shading image S
// (colour c from Eq. 4), the shadow image Sh (refined shadow value T',
// Eq. 8) and the residual image R (Psi's RGB, Sec. 4.3). A pixel stops before
// the splat that would take its transmittance below t_min; the workgroup
// stops when all its pixels have. Output final = S * Sh + R per pixel.
#include "splat_common.h"

namespace gs3 {

struct RenderArgs {
    const int2* ranges;
    const uint32_t* order;   // launch order of the tiles
    const uint32_t* list;
    const float4* rec0;
    const float4* rec1;
    const float4* rec2;   // {thr, hx, hy, p}
    const float4* col0;   // {c.r, c.g, c.b, T'}
    const float4* col1;   // {r.r, r.g, r.b, 0}
    const ViewHeader* hdr;
    uint32_t n;
    int width, height, tiles_x, n_tiles;
    int n_slots;             // entries of order (some may be kNoTile)
    float alpha_max, t_min;
    gs3_images out;
};

// The views of one launch: blockIdx.y selects the view, blockIdx.x its
// tile (the x extent is the largest view's tile count; the surplus
// workgroups of smaller views exit).
struct RenderBatch {
    RenderArgs v[kMaxBatch];
};

template <bool ONE>
__global__ __launch_bounds__(256) void k_render(RenderBatch B) {
    // ONE: a single view (static argument offsets)
    const RenderArgs a = ONE ? B.v[0] : B.v[blockIdx.y];
    if ((int)blockIdx.x >= a.n_slots) return;
    const uint32_t ot = a.order[blockIdx.x];
    if (ot == kNoTile) return;
    __shared__ Staged s_rec[256];
    __shared__ float4 s_c0[256];
    __shared__ float4 s_c1[256];
    __shared__ uint32_t s_mask[256];
    const int tile = (int)ot;
    const int tid = threadIdx.x, w = tid >> 6, lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int lx = (w & 1) * 8 + (lane & 7), ly = (w >> 1) * 8 + (lane >> 3);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    const bool inside = px < a.width && py < a.height;
    const float pxc = lx + 0.5f, pyc = ly + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    const uint32_t wbit = 1u << w;
    const int2 rg = a.ranges[tile];
    const int s = rg.x, e = rg.y;
    float T = 1.f;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, Sh = 0.f, R0 = 0.f, R1 = 0.f, R2 = 0.f;
    int last = 0;
    bool done = !inside;
    for (int b = s; b < e; b += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const int m = min(256, e - b);
        if (tid < m) {
            const uint32_t id = safe_id(a.list[b + tid], a.n);
            uint32_t mk;
            s_rec[tid] = stage_splat(id, a.rec0, a.rec1, a.rec2, nullptr, tile_x0, tile_y0, &mk);
            s_mask[tid] = mk;
            s_c0[tid] = a.col0[id];
            s_c1[tid] = a.col1[id];
        }
        __syncthreads();
        // the entries that can hit a pixel centre of this wave's quadrant, as
        // four 64-bit sets (bounding box, then the hit ellipse itself)
        unsigned long long set[4] = {0ull, 0ull, 0ull, 0ull};
        if (__builtin_amdgcn_ballot_w64(!done)) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int jj = 64 * h + lane;
                set[h] = __builtin_amdgcn_ballot_w64(jj < m && (s_mask[jj] & wbit) && quad_reach(s_rec[jj], w));
            }
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          unsigned long long todo = set[h];
          while (todo) {
            const int j = 64 * h + __builtin_ctzll(todo);
            todo &= todo - 1ull;
            if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
            const Staged sj = s_rec[j];
            const float q = splat_q(sj, pxc, pyc);
            bool hit = !done && q >= sj.g1.y;
            const float al = fminf(a.alpha_max, sj.g1.z * fast_exp2(q));
            const float tn = T * (1.f - al);
            if (hit && tn < a.t_min) {
                done = true;
                hit = false;
            }
            if (hit) {
                const float wgt = al * T;
                const float4 c0 = s_c0[j];
                const float4 c1 = s_c1[j];
                S0 = fmaf(wgt, c0.x, S0);
                S1 = fmaf(wgt, c0.y, S1);
                S2 = fmaf(wgt, c0.z, S2);
                Sh = fmaf(wgt, c0.w, Sh);
                R0 = fmaf(wgt, c1.x, R0);
                R1 = fmaf(wgt, c1.y, R1);
                R2 = fmaf(wgt, c1.z, R2);
                T = tn;
                last = b + j - s + 1;
            }
          }
        }
        __syncthreads();
    }
    if (a.hdr->overflow) {
        // the binning overflowed its pair capacity and left every list
        // empty: mark the pixels instead of writing an empty-scene image
        const float nan = __builtin_nanf("");
        S0 = S1 = S2 = Sh = R0 = R1 = R2 = T = nan;
    }
    if (inside) {
        const int64_t hw = (int64_t)a.width * a.height;
        const int64_t p = (int64_t)py * a.width + px;
        a.out.shading[p] = S0;
        a.out.shading[hw + p] = S1;
        a.out.shading[2 * hw + p] = S2;
        a.out.shadow[p] = Sh;
        a.out.residual[p] = R0;
        a.out.residual[hw + p] = R1;
        a.out.residual[2 * hw + p] = R2;
        a.out.final_rgb[p] = fmaf(S0, Sh, R0);
        a.out.final_rgb[hw + p] = fmaf(S1, Sh, R1);
        a.out.final_rgb[2 * hw + p] = fmaf(S2, Sh, R2);
        a.out.t_final[p] = T;
        a.out.n_contrib[p] = last;
    }
}

static RenderArgs render_args(const gs3_consts& k, const Layout& L, const void* ws, const gs3_images& out) {
    RenderArgs a;
    a.ranges = at<int2>(ws, L.ranges);
    a.order = at<uint32_t>(ws, L.order);
    a.list = at<uint32_t>(ws, L.pv_a);
    a.rec0 = at<float4>(ws, L.rec0);
    a.rec1 = at<float4>(ws, L.rec1);
    a.rec2 = at<float4>(ws, L.rec2);
    a.col0 = at<float4>(ws, L.col0);
    a.col1 = at<float4>(ws, L.col1);
    a.hdr = at<ViewHeader>(ws, L.hdr);
    a.n = (uint32_t)L.n;
    a.width = L.width;
    a.height = L.height;
    a.tiles_x = L.tiles_x;
    a.n_tiles = (int)L.n_tiles;
    a.n_slots = (int)L.n_slots;
    a.alpha_max = k.alpha_max;
    a.t_min = k.t_min;
    a.out = out;
    return a;
}

hipError_t launch_render_batch(const gs3_consts& k, const Layout* const* Ls, void* const* wss,
                               const gs3_images* outs, int nv, hipStream_t st) {
    for (int v0 = 0; v0 < nv; v0 += kMaxBatch) {
        const int m = nv - v0 < kMaxBatch ? nv - v0 : kMaxBatch;
        RenderBatch B;
        int64_t gx = 0;
        for (int i = 0; i < m; ++i) {
            B.v[i] = render_args(k, *Ls[v0 + i], wss[v0 + i], outs[v0 + i]);
            gx = Ls[v0 + i]->n_slots > gx ? Ls[v0 + i]->n_slots : gx;
        }
        if (m == 1)
            hipLaunchKernelGGL(k_render<true>, dim3((unsigned)gx), dim3(256), 0, st, B);
        else
            hipLaunchKernelGGL(k_render<false>, dim3((unsigned)gx, m), dim3(256), 0, st, B);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_render(const gs3_consts& k, const Layout& L, const void* ws, const gs3_images& out,
                         hipStream_t st) {
    const Layout* Ls[1] = {&L};
    void* w = const_cast<void*>(ws);
    return launch_render_batch(k, Ls, &w, &out, 1, st);
}

}  // namespace gs3
