// Export kernels: unpack a view workspace into the plain arrays of the
// C-ABI (tile lists, sort keys, projected splats).
#include "splat_common.h"

namespace gs3 {

__global__ __launch_bounds__(256) void k_export_ranges(const int2* __restrict__ rg, int64_t tiles,
                                                        int32_t* __restrict__ start, int32_t* __restrict__ end) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= tiles) return;
    const int2 r = rg[t];
    if (start) start[t] = r.x;
    if (end) end[t] = r.y;
}

__global__ __launch_bounds__(256) void k_export_pairs(const uint32_t* __restrict__ pk, const uint32_t* __restrict__ pv,
                                                       const float* __restrict__ depth, const ViewHeader* __restrict__ hdr,
                                                       uint32_t n, int32_t* __restrict__ ids,
                                                       uint64_t* __restrict__ keys) {
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= hdr->n_pairs) return;
    const uint32_t id = pv[p];
    if (ids) ids[p] = (int32_t)id;
    if (keys) keys[p] = ((uint64_t)pk[p] << 32) | (uint64_t)__float_as_uint(depth[id < n ? id : 0u]);
}

// Keys of packed binnings, where the sorted tile indices are not kept: one
// thread per tile writes its range's keys.
__global__ __launch_bounds__(256) void k_export_tile_keys(const int2* __restrict__ rg, int64_t tiles,
                                                           const uint32_t* __restrict__ pv,
                                                           const float* __restrict__ depth, uint32_t n,
                                                           uint64_t* __restrict__ keys) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= tiles) return;
    const int2 r = rg[t];
    for (int p = r.x; p < r.y; ++p) {
        const uint32_t id = pv[p];
        keys[p] = ((uint64_t)t << 32) | (uint64_t)__float_as_uint(depth[id < n ? id : 0u]);
    }
}

__global__ __launch_bounds__(256) void k_export_splats(const float4* __restrict__ rec0, const float4* __restrict__ rec1,
                                                        const float* __restrict__ depth, const int4* __restrict__ ext,
                                                        int n, float* __restrict__ mean2d, float* __restrict__ conic,
                                                        float* __restrict__ opacity, float* __restrict__ depth_out,
                                                        int32_t* __restrict__ extent) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 r0 = rec0[i], r1 = rec1[i];
    const int4 e = ext[i];
    if (mean2d) {
        mean2d[i] = r0.x + r0.z;
        mean2d[n + i] = r0.y + r0.w;
    }
    if (conic) {
        conic[i] = r1.x;
        conic[n + i] = r1.y;
        conic[2 * n + i] = r1.z;
    }
    if (opacity) opacity[i] = r1.w;
    if (depth_out) depth_out[i] = depth[i];
    if (extent) {
        extent[i] = e.x;
        extent[n + i] = e.y;
        extent[2 * n + i] = e.z;
        extent[3 * n + i] = e.w;
    }
}

hipError_t launch_export_lists(const Layout& L, const void* ws, int32_t* start, int32_t* end, int32_t* ids,
                               uint64_t* keys, hipStream_t st) {
    if ((start || end) && L.n_tiles > 0)
        hipLaunchKernelGGL(k_export_ranges, dim3((unsigned)((L.n_tiles + 255) / 256)), dim3(256), 0, st,
                           at<int2>(ws, L.ranges), L.n_tiles, start, end);
    const bool packed = L.id_bits > 0;
    if ((ids || (keys && !packed)) && L.capacity > 0)
        hipLaunchKernelGGL(k_export_pairs, dim3((unsigned)((L.capacity + 255) / 256)), dim3(256), 0, st,
                           at<uint32_t>(ws, L.pk_a), at<uint32_t>(ws, L.pv_a), at<float>(ws, L.depth),
                           at<ViewHeader>(ws, L.hdr), (uint32_t)L.n, ids, packed ? nullptr : keys);
    if (keys && packed && L.n_tiles > 0)
        hipLaunchKernelGGL(k_export_tile_keys, dim3((unsigned)((L.n_tiles + 255) / 256)), dim3(256), 0, st,
                           at<int2>(ws, L.ranges), L.n_tiles, at<uint32_t>(ws, L.pv_a), at<float>(ws, L.depth),
                           (uint32_t)L.n, keys);
    return hipGetLastError();
}

hipError_t launch_export_splats(const Layout& L, const void* ws, float* mean2d, float* conic, float* opacity,
                                float* depth, int32_t* extent, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_splats, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st,
                       at<float4>(ws, L.rec0), at<float4>(ws, L.rec1), at<float>(ws, L.depth), at<int4>(ws, L.ext),
                       (int)L.n, mean2d, conic, opacity, depth, extent);
    return hipGetLastError();
}

}  // namespace gs3

namespace gs3 {

// Number of (pixel, splat) hits of a binned view: pixels where
// power >= -cutoff and alpha >= alpha_min. With stop_early the camera rule
// applies (a pixel stops before the hit that would take its transmittance
// below t_min) and only the hits that are blended are counted.
__global__ __launch_bounds__(256) void k_count_hits(const int2* __restrict__ ranges, const uint32_t* __restrict__ list,
                                                     const float4* __restrict__ rec0, const float4* __restrict__ rec1,
                                                     const float4* __restrict__ rec2, uint32_t n, int width,
                                                     int height, int tiles_x, float alpha_max, float t_min, int stop_early,
                                                     unsigned long long* __restrict__ out) {
    const int tile = blockIdx.x;
    const int2 rg = ranges[tile];
    const int tid = threadIdx.x, w = tid >> 6, lane = __lane_id();
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int lx = (w & 1) * 8 + (lane & 7), ly = (w >> 1) * 8 + (lane >> 3);
    const bool inside = (tx * kTile + lx < width) && (ty * kTile + ly < height);
    const float pxc = lx + 0.5f, pyc = ly + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    unsigned long long cnt = 0;
    float T = 1.f;
    bool done = !inside;
    for (int i = rg.x; i < rg.y; ++i) {
        uint32_t mk;
        const Staged s = stage_splat(safe_id(list[i], n), rec0, rec1, rec2, nullptr, tile_x0, tile_y0, &mk);
        const float q = splat_q(s, pxc, pyc);
        if (!done && q >= s.g1.y) {
            if (stop_early) {
                const float al = fminf(alpha_max, s.g1.z * fast_exp2(q));
                const float tn = T * (1.f - al);
                if (tn < t_min) {
                    done = true;
                    continue;
                }
                T = tn;
            }
            ++cnt;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if (lane == 0 && cnt) atomicAdd(out, cnt);
}

hipError_t launch_count_hits(const gs3_consts& k, const Layout& L, const void* ws, int stop_early,
                             unsigned long long* out, hipStream_t st) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(out), 0u, 2, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_hits, dim3((unsigned)L.n_tiles), dim3(256), 0, st, at<int2>(ws, L.ranges),
                       at<uint32_t>(ws, L.pv_a), at<float4>(ws, L.rec0), at<float4>(ws, L.rec1),
                       at<float4>(ws, L.rec2), (uint32_t)L.n, L.width, L.height, L.tiles_x, k.alpha_max, k.t_min,
                       stop_early, out);
    return hipGetLastError();
}

}  // namespace gs3
