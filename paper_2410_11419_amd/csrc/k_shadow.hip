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
// list entries staged at a time: 64 keeps a wave's LDS (two batches of
// records, ids, lead sums) near 5 KB, so twice as many of these
// latency-bound waves fit on a CU as with 128 (0.72 -> 0.57 ms per 1024^2
// light view); 32 makes the ring too short for the bias lag
constexpr int kShadowBatch = 64;
constexpr int kRingMask = 2 * kShadowBatch - 1;       // the LDS ring holds two batches

struct ShadowArgs {
    const int2* ranges;
    const uint32_t* order;   // launch order of the tiles
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

// 128-bit set of batch entries (two 64-bit halves).
// The lists, pointers and distances a wave walks are the same in every
// lane; reading such a value through readfirstlane tells the compiler so,
// which keeps the pointer arithmetic and loop control in scalar registers
// and scalar branches.
__device__ inline float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ inline uint32_t uniform_u(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }

struct Bits128 {
    unsigned long long lo, hi;
};
__device__ inline Bits128 range_bits(int lo, int hi) {   // entries lo .. hi-1, 0 <= lo <= hi <= 128
    auto upto = [](int k) -> unsigned long long { return k >= 64 ? ~0ull : ((1ull << k) - 1ull); };
    Bits128 b;
    b.lo = upto(min(hi, 64)) & ~upto(min(lo, 64));
    b.hi = upto(max(hi - 64, 0)) & ~upto(max(lo - 64, 0));
    return b;
}
__device__ inline int first_bit(const Bits128& b) {
    return b.lo ? __builtin_ctzll(b.lo) : 64 + __builtin_ctzll(b.hi);
}
__device__ inline void clear_bit(Bits128& b, int k) {
    if (k < 64) b.lo &= ~(1ull << k); else b.hi &= ~(1ull << (k - 64));
}

// One wave per (tile, 8x8 quadrant): the four quadrants of a light tile run
// as independent single-wave workgroups, one pixel per lane. The wave stages
// its tile's list a batch at a time into an LDS ring that also keeps the
// previous batch for the trailing pointer; a ballot marks the entries whose
// hit ellipse can reach the quadrant, and both pointers visit only those, so
// the wave's sequential chain is as short as its quadrant allows. For each
// lead entry j, L(j) (the first list position not more than `bias` closer to
// the light) comes from a binary search over the ring's distances; when it
// lies before the ring the trailing pointer walks and compares instead. The
// wave exits when all its pixels are dark.
__global__ __launch_bounds__(64) void k_shadow(ShadowArgs a) {
    __shared__ Staged s_rec[2 * kShadowBatch];
    __shared__ uint32_t s_id[2 * kShadowBatch];
    __shared__ float s_sum[kShadowBatch];        // lead sums of the current batch
    const int tile = (int)a.order[blockIdx.x >> 2];
    const int qd = blockIdx.x & 3;
    const int2 rg = a.ranges[tile];
    const int s = rg.x, e = rg.y;
    if (e <= s) return;
    const int lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int lx = (qd & 1) * 8 + (lane & 7), ly = (qd >> 1) * 8 + (lane >> 3);
    const float pxc = lx + 0.5f, pyc = ly + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    bool alive = (tx * kTile + lx < a.width) && (ty * kTile + ly < a.height);
    if (!__ballot(alive)) return;
    const uint32_t qbit = 1u << qd;
    float tt = 1.f;
    Bits128 cur{0ull, 0ull}, prv{0ull, 0ull};
    int trail = s;
    // multiply (1 - alpha) of occluder k into tt where it hits
    auto occlude = [&](const Staged& k) {
        const float q = splat_q(k, pxc, pyc);
        if (alive && q >= k.g1.y) tt *= 1.f - fminf(a.alpha_max, k.g1.z * fast_exp2(q));
    };
    // A global atomic without a returned value still counts as an
    // outstanding vector memory operation, so the next wait for a load would
    // wait for it too: the lead sums of a batch collect in LDS and go out
    // in one burst of atomics when the batch ends.
    auto flush = [&](int base, int m) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jj = lane + 64 * h;
            if (jj < m) {
                const float v = s_sum[jj];
                if (v != 0.f) atomicAdd(&a.num[s_id[base + jj]], v);
            }
        }
    };
    for (int b = s; b < e; b += kShadowBatch) {
        const int m = min(kShadowBatch, e - b);
        const int base = (b - s) & kRingMask;          // ring slot of entry b
        bool qm[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jj = lane + 64 * h;
            qm[h] = false;
            if (jj < m) {
                uint32_t mk;
                const uint32_t id = safe_id(a.list[b + jj], a.n);
                s_rec[base + jj] = stage_splat(id, a.rec0, a.rec1, a.depth, tile_x0, tile_y0, a.cutoff,
                                               a.alpha_min, &mk);
                s_id[base + jj] = id;
                qm[h] = (mk & qbit) != 0u;
            }
            if (jj < kShadowBatch) s_sum[jj] = 0.f;
        }
        cur.lo = __ballot(qm[0]);
        cur.hi = __ballot(qm[1]);
        __syncthreads();
        // L(j) for the lane's two entries: the first position in
        // [lo_pos, b + j) whose distance is not below dist_j - bias (b + j
        // if none); -1 when it lies before the ring
        const int lo_pos = max(s, b - kShadowBatch);
        int Lh[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jj = lane + 64 * h;
            Lh[h] = b + min(jj, m);
            if (jj < m) {
                const float thr = s_rec[base + jj].g1.w - a.bias;
                if (lo_pos > s && !(s_rec[(lo_pos - s) & kRingMask].g1.w < thr)) {
                    Lh[h] = -1;
                } else {
                    int lo = lo_pos, hi = b + jj;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_rec[(mid - s) & kRingMask].g1.w < thr) lo = mid + 1; else hi = mid;
                    }
                    Lh[h] = lo;
                }
            }
        }
        Bits128 todo = cur;
        while (todo.lo | todo.hi) {
            const int j = first_bit(todo);
            clear_bit(todo, j);
            const Staged sj = s_rec[base + j];
            const int L0 = __builtin_amdgcn_readlane(Lh[0], j & 63);
            const int L1 = __builtin_amdgcn_readlane(Lh[1], j & 63);
            const int Lj = j < 64 ? L0 : L1;
            const float thr_d = uniform_f(sj.g1.w) - a.bias;
            const int stop = Lj >= 0 ? Lj : b + j;
            while (trail < stop) {
                if (trail < lo_pos) {
                    // older than the ring: re-stage from global memory
                    uint32_t mk;
                    const Staged tk = stage_splat(safe_id(a.list[trail], a.n), a.rec0, a.rec1, a.depth, tile_x0,
                                                  tile_y0, a.cutoff, a.alpha_min, &mk);
                    if (Lj < 0 && !(uniform_f(tk.g1.w) < thr_d)) break;
                    if (uniform_u(mk) & qbit) occlude(tk);
                    ++trail;
                    continue;
                }
                // ring entries of one batch, only those that reach the quadrant
                const bool in_cur = trail >= b;
                const int bstart = in_cur ? b : b - kShadowBatch;
                const int lo = trail - bstart, hi = min(stop - bstart, kShadowBatch);
                Bits128 rel = range_bits(lo, hi);
                const Bits128 msk = in_cur ? cur : prv;
                rel.lo &= msk.lo;
                rel.hi &= msk.hi;
                bool stopped = false;
                while (rel.lo | rel.hi) {
                    const int k = first_bit(rel);
                    clear_bit(rel, k);
                    const Staged tk = s_rec[(bstart + k - s) & kRingMask];
                    if (Lj < 0 && !(uniform_f(tk.g1.w) < thr_d)) {
                        trail = bstart + k;
                        stopped = true;
                        break;
                    }
                    occlude(tk);
                }
                if (stopped) break;
                trail = bstart + hi;
            }
            alive = alive && tt >= kShadowEps;
            if (!__ballot(alive)) {                // every pixel of the quadrant is dark
                flush(base, m);
                return;
            }
            const float q = splat_q(sj, pxc, pyc);
            const bool hit = alive && q >= sj.g1.y;
            if (__ballot(hit)) {
                const float v = hit ? fast_exp2(q) * tt : 0.f;
                const float sn = wave_sum_lane63(v);
                if (lane == 63) s_sum[j] = sn;
            }
        }
        flush(base, m);
        prv = cur;
        __syncthreads();
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

static ShadowArgs shadow_args(const gs3_consts& k, const Layout& L, const void* ws, float* num_den) {
    ShadowArgs a;
    a.ranges = at<int2>(ws, L.ranges);
    a.order = at<uint32_t>(ws, L.order);
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
    return a;
}

hipError_t launch_shadow_den(const gs3_consts& k, const Layout& L, const void* ws, float* num_den, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    int grid = (int)((L.n + 3) / 4);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_shadow_den, dim3(grid), dim3(256), 0, st, shadow_args(k, L, ws, num_den));
    return hipGetLastError();
}

hipError_t launch_shadow_num(const gs3_consts& k, const Layout& L, const void* ws, float* num_den, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(num_den), 0u, L.n, st);
    if (e != hipSuccess) return e;
    if (L.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shadow, dim3((unsigned)(4 * L.n_tiles)), dim3(64), 0, st, shadow_args(k, L, ws, num_den));
    return hipGetLastError();
}

hipError_t launch_shadow_resolve(const Layout& L, const float* num_den, float* T, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shadow_finish, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, num_den,
                       num_den + L.n, T, (int)L.n);
    return hipGetLastError();
}

hipError_t launch_shadow(const gs3_consts& k, const Layout& L, const void* ws, float* num_den, float* T,
                         hipStream_t st) {
    hipError_t e = launch_shadow_den(k, L, ws, num_den, st);
    if (e == hipSuccess) e = launch_shadow_num(k, L, ws, num_den, st);
    if (e == hipSuccess) e = launch_shadow_resolve(L, num_den, T, st);
    return e;
}

}  // namespace gs3
