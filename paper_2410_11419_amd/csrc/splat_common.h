// Device helpers shared by the per-tile splatting kernels (shadow, camera
// and their adjoints): staging of splat records into tile-relative form,
// wave64 reductions.
#pragma once

#include "gs3_internal.h"

namespace gs3 {

constexpr float kLog2e = 1.4426950408889634f;

// A splat staged for one tile. The conic is pre-scaled by -log2(e)/2 so that
// q = A dx^2 + B dx dy + C dy^2 equals power * log2(e) and exp2(q) is the
// splat density beta = exp(power) at the pixel. A pixel is hit iff q >= thr,
// with thr = log2(e) * max(-cutoff, ln(alpha_min / opacity)) -- the cut-off
// and the alpha >= alpha_min test in one comparison.
struct Staged {
    float4 g0;  // {u_rel, v_rel, A, B}  centre relative to the tile origin
    float4 g1;  // {C, thr, opacity, depth}
};

// Ids come from the view's own binning and are < n; the clamp only keeps a
// corrupted list (never produced by a successful binning) inside the arrays.
__device__ inline uint32_t safe_id(uint32_t id, uint32_t n) { return id < n ? id : 0u; }

// Scaled conic and hit threshold of a splat record (shared by every kernel
// that tests pixels against a splat, so they take identical decisions).
// Returns p, the power threshold (hit iff power >= -p); p <= 0 never hits.
__device__ inline float stage_coeffs(const float4 r1, float cutoff, float alpha_min, float* A, float* B, float* C,
                                     float* thr) {
    float p = cutoff;
    if (alpha_min > 0.f) p = fminf(p, logf(r1.w / alpha_min));
    *A = -0.5f * kLog2e * r1.x;
    *B = -kLog2e * r1.y;
    *C = -0.5f * kLog2e * r1.z;
    *thr = -p * kLog2e;
    return p;
}

// Per-splat constants of the hit test from record r1 = {conic a, b, c,
// opacity}, computed once per view by the projection and stored as rec2:
// {thr, hx, hy, p} with thr and p as stage_coeffs gives them, and hx, hy the
// half-widths sqrt(2 p Sigma'_xx), sqrt(2 p Sigma'_yy) of the hit ellipse's
// bounding box (Sigma' = conic^-1), padded so that the box is conservative
// with respect to the per-pixel float32 test (3e38 when p is infinite).
__device__ inline float4 splat_bounds(const float4 r1, float cutoff, float alpha_min) {
    float A, B, C, thr;
    const float p = stage_coeffs(r1, cutoff, alpha_min, &A, &B, &C, &thr);
    float hx = 3.0e38f, hy = 3.0e38f;
    if (p > 0.f && !isinf(p)) {
        const float det = r1.x * r1.z - r1.y * r1.y;
        hx = sqrtf(fmaxf(2.f * p * r1.z / det, 0.f)) * 1.01f + 0.01f;
        hy = sqrtf(fmaxf(2.f * p * r1.x / det, 0.f)) * 1.01f + 0.01f;
    }
    return make_float4(thr, hx, hy, p);
}

// The conic scaled by -log2(e)/2 (see Staged), from record r1.
__device__ inline void scaled_conic(const float4 r1, float* A, float* B, float* C) {
    *A = -0.5f * kLog2e * r1.x;
    *B = -kLog2e * r1.y;
    *C = -0.5f * kLog2e * r1.z;
}

// q = power * log2(e) for offset (dx, dy) from the splat centre; written with
// explicit fmaf so that every kernel rounds it the same way.
__device__ inline float quad_q(float dx, float dy, float A, float B, float C) {
    return fmaf(dx, fmaf(B, dy, A * dx), (C * dy) * dy);
}

// Tile-relative centre of a splat for the tile whose origin is (x0, y0).
__device__ inline float rel_centre(float hi, float lo, float origin) { return (hi - origin) + lo; }

// Tile-relative staging of Gaussian `id`. `mask` gets bit w set when the
// hit ellipse's bounding box reaches wave w's 8x8 quadrant (quadrant w
// covers tile pixels x in [8 (w & 1), +8), y in [8 (w >> 1), +8)).
__device__ inline Staged stage_splat(uint32_t id, const float4* __restrict__ rec0,
                                     const float4* __restrict__ rec1, const float4* __restrict__ rec2,
                                     const float* __restrict__ depth, float tile_x0, float tile_y0,
                                     uint32_t* mask) {
    const float4 r0 = rec0[id];
    const float4 r1 = rec1[id];
    const float4 r2 = rec2[id];
    Staged s;
    const float u = rel_centre(r0.x, r0.z, tile_x0);
    const float v = rel_centre(r0.y, r0.w, tile_y0);
    float A, B, C;
    scaled_conic(r1, &A, &B, &C);
    const float p = r2.w;
    s.g0 = make_float4(u, v, A, B);
    s.g1 = make_float4(C, r2.x, r1.w, depth ? depth[id] : 0.f);
    // the hit ellipse's bounding box (rec2) against each quadrant
    uint32_t m = 0u;
    if (p > 0.f) {
        if (isinf(p)) {
            m = 0xFu;
        } else {
            const float hx = r2.y, hy = r2.z;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const float qx = 8.f * (w & 1), qy = 8.f * (w >> 1);
                const bool ox = (u + hx >= qx + 0.5f) && (u - hx <= qx + 7.5f);
                const bool oy = (v + hy >= qy + 0.5f) && (v - hy <= qy + 7.5f);
                if (ox && oy) m |= 1u << w;
            }
        }
    }
    *mask = m;
    return s;
}

// Whether the hit region q >= thr of staged splat s can reach a pixel centre
// of the 8x8 quadrant qd of its tile: the maximum of the concave quadratic q
// over the rectangle spanned by the quadrant's pixel centres (the value at
// the splat centre when that lies inside, else the best point of each edge,
// a one-dimensional concave maximum clamped to the edge), compared with thr
// less a slack that covers the float32 rounding of the per-pixel test. False
// only when no pixel centre of the quadrant is hit, so skipping the splat
// there changes no result.
__device__ inline bool quad_reach(const Staged& s, int qd) {
    const float A = s.g0.z, B = s.g0.w, C = s.g1.x, thr = s.g1.y;
    if (!(A < 0.f && C < 0.f)) return true;
    const float x0 = (8.f * (qd & 1) + 0.5f) - s.g0.x, x1 = x0 + 7.f;     // dx over the quadrant
    const float y0 = (8.f * (qd >> 1) + 0.5f) - s.g0.y, y1 = y0 + 7.f;    // dy over the quadrant
    if (x0 <= 0.f && 0.f <= x1 && y0 <= 0.f && 0.f <= y1) return true;
    const float kx = -0.5f * B / A, ky = -0.5f * B / C;   // argmax of q in dx for fixed dy, in dy for fixed dx
    auto on_x_edge = [&](float dx) { return quad_q(dx, fminf(fmaxf(ky * dx, y0), y1), A, B, C); };
    auto on_y_edge = [&](float dy) { return quad_q(fminf(fmaxf(kx * dy, x0), x1), dy, A, B, C); };
    const float best = fmaxf(fmaxf(on_x_edge(x0), on_x_edge(x1)), fmaxf(on_y_edge(y0), on_y_edge(y1)));
    const float mx = fmaxf(fabsf(x0), fabsf(x1)), my = fmaxf(fabsf(y0), fabsf(y1));
    const float mag = (-A * mx) * mx + (fabsf(B) * mx) * my + (-C * my) * my;
    return best >= thr - (1e-5f * mag + 1e-3f * fabsf(thr) + 1e-6f);
}

// x-extent of the hit region q >= thr per band of rows. For fixed dy the
// region is the interval xc(dy) -+ w(dy), xc = -B dy / (2A),
// w = sqrt(4A thr - K dy^2) / (2|A|), K = 4AC - B^2 > 0. Its left end is
// smallest at the ellipse's leftmost point, which lies at dy = B xmax / (2C)
// (xmax^2 = 4C thr / K); when that row is outside a band, the convex left
// end is smallest at a band edge. The right end likewise.
struct RowExtent {
    float A, B, K, fourAthr, ymax, xmax, inv2a, yl;
    bool valid;
};
__device__ inline RowExtent row_extent(float A, float B, float C, float thr) {
    RowExtent e;
    e.A = A;
    e.B = B;
    e.K = 4.f * A * C - B * B;
    e.valid = A < 0.f && C < 0.f && e.K > 0.f && thr < 0.f && !isinf(thr);
    // hardware reciprocal and square root (about 1 ulp): the result is
    // padded by far more than their error
    const float rK = __builtin_amdgcn_rcpf(e.K);
    e.fourAthr = 4.f * A * thr;
    e.ymax = __builtin_amdgcn_sqrtf(e.fourAthr * rK) * 1.01f + 0.02f;
    e.xmax = __builtin_amdgcn_sqrtf(4.f * C * thr * rK);
    e.inv2a = 0.5f * __builtin_amdgcn_rcpf(A);  // negative
    e.yl = 0.5f * B * e.xmax * __builtin_amdgcn_rcpf(C);   // row of the leftmost point; the rightmost is at -yl
    return e;
}
// Range [lo, hi] of dx (offset from the splat centre) that the hit region
// covers within the band of rows dy0 <= dy <= dy1 (e.valid required); false
// when the band misses it. Widened by 1 % of xmax + 0.02 px for float32
// rounding, so it contains every pixel offset the per-pixel test can hit.
__device__ inline bool band_x_range(const RowExtent& e, float dy0, float dy1, float* lo, float* hi) {
    dy0 = fmaxf(dy0, -e.ymax);
    dy1 = fminf(dy1, e.ymax);
    if (dy0 > dy1) return false;
    auto w = [&](float dy) { return __builtin_amdgcn_sqrtf(fmaxf(e.fourAthr - e.K * dy * dy, 0.f)) * (-e.inv2a); };
    const float w0 = w(dy0), w1 = w(dy1);
    const float c0 = -e.B * dy0 * e.inv2a, c1 = -e.B * dy1 * e.inv2a;
    const float l = (e.yl >= dy0 && e.yl <= dy1) ? -e.xmax : fminf(c0 - w0, c1 - w1);
    const float h = (-e.yl >= dy0 && -e.yl <= dy1) ? e.xmax : fmaxf(c0 + w0, c1 + w1);
    const float pad = 0.01f * e.xmax + 0.02f;
    *lo = l - pad;
    *hi = h + pad;
    return true;
}

// q = power * log2(e) at tile-relative pixel centre (px, py)
__device__ inline float splat_q(const Staged& s, float px, float py) {
    return quad_q(px - s.g0.x, py - s.g0.y, s.g0.z, s.g0.w, s.g1.x);
}

// 2^q on the hardware exp unit (q >= thr > -126 wherever the value is used)
__device__ inline float fast_exp2(float q) { return __builtin_amdgcn_exp2f(q); }

// Sum of x over the 64 lanes of a wave; valid in lane 63 (DPP butterfly in
// quads, half-rows and rows, then row broadcasts across the wave).
__device__ inline float wave_sum_lane63(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, true));  // row_half_mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, true));  // row_mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, false)); // row_bcast:15
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xC, 0xF, false)); // row_bcast:31
    return x;
}

// The lists, pointers and distances a wave walks are the same in every
// lane; reading such a value through readfirstlane tells the compiler so,
// which keeps the pointer arithmetic and loop control in scalar registers
// and scalar branches.
__device__ inline float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ inline uint32_t uniform_u(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
// The shadow denominator's per-Gaussian culls, computed once per view by the
// projection (one lane per Gaussian) instead of by a whole wave per Gaussian
// in every denominator pass. From the stored records: the bounding box's tile
// columns [x_lo, x_hi] clipped to the splat's tile rectangle [x0, x1] x
// [y0, y1], and its 4-row groups [g_lo, g_hi] (absolute index 4 ty + r)
// clipped to the rectangle's rows, with 0.05 px of slack on top of the box's
// padding for the rounding of the absolute centre; bit 31 of .x flags a
// large elongated splat whose columns are narrowed per tile row (16 tiles or
// more, bounding box over 2.5x the ellipse); iu, iv = (int) of rec0.x,
// rec0.y (floor of the centre, exact below 2^24). Packed as
//   {x_lo | x_hi << 16 | banded << 31, g_lo | g_hi << 16, iu, iv};
// an empty range (no denominator work) has x_lo > x_hi, as {1, 1, 0, 0}.
// The tile rows to visit are ceil((g_lo - 3) / 4) .. floor(g_hi / 4).
__device__ inline int4 den_ranges(float4 r0, float4 r1, float4 r2, int x0, int x1, int y0, int y1) {
    const int4 empty = make_int4(1, 1, 0, 0);
    const float hx = r2.y, hy = r2.z, p = r2.w;
    if (!(p > 0.f)) return empty;
    const float U = r0.x + r0.z, V = r0.y + r0.w;
    auto toi = [](float x) { return (int)fminf(fmaxf(x, -16777216.f), 16777216.f); };
    const int x_lo = max(x0, toi(ceilf((U - hx - 15.55f) * (1.f / kTile))));
    const int x_hi = min(x1, toi(floorf((U + hx - 0.45f) * (1.f / kTile))));
    // clipping the row groups to the rectangle's rows changes no tile row's
    // [max(0, g_lo - 4 ty), min(3, g_hi - 4 ty)] inside the rectangle
    const int g_lo = max(4 * y0, toi(ceilf((V - hy - 3.55f) * 0.25f)));
    const int g_hi = min(4 * y1 + 3, toi(floorf((V + hy - 0.45f) * 0.25f)));
    if (x_lo > x_hi || g_lo > g_hi) return empty;
    bool banded = false;
    if (!isinf(p)) {
        const float det = r1.x * r1.z - r1.y * r1.y;
        banded = (x1 - x0 + 1) * (y1 - y0 + 1) >= 16 && r1.x * r1.z > 4.f * det;
    }
    return make_int4(x_lo | (x_hi << 16) | (banded ? (int)0x80000000u : 0), g_lo | (g_hi << 16), toi(r0.x),
                     toi(r0.y));
}

// A wave-uniform int pinned to a scalar register. The builtin above is
// dropped when the compiler already knows the value is uniform, and a
// float-to-int conversion (a vector instruction) then leaves the loop bounds
// and indices derived from it in vector registers, compared and stepped with
// vector instructions.
__device__ inline int sgpr_i(int x) {
    int s;
    asm("v_readfirstlane_b32 %0, %1" : "=s"(s) : "v"(x));
    return s;
}

// Bits lo .. hi-1 of a 64-bit set (lo and hi clamped to [0, 64]).
__device__ inline unsigned long long range_mask64(int lo, int hi) {
    lo = lo < 0 ? 0 : lo;
    hi = hi > 64 ? 64 : hi;
    if (hi <= lo) return 0ull;
    const unsigned long long up = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return up & ~((1ull << lo) - 1ull);
}

// A lane's 64-bit value as seen by lane j (j wave-uniform).
__device__ inline unsigned long long readlane64(unsigned long long x, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((unsigned long long)hi << 32) | lo;
}

// Sum of x over each 16-lane row, in every lane of the row (DPP butterfly in
// quads, then half-row and row mirrors).
__device__ inline float row_sum16(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, true));  // row_half_mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, true));  // row_mirror
    return x;
}

// Row sums (as row_sum16) of N values at once, the DPP steps interleaved
// across the values so that no step waits on the one before it.
template <int N>
__device__ inline void row_sums16(float (&x)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x[c]), 0xB1, 0xF, 0xF, true));
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x[c]), 0x4E, 0xF, 0xF, true));
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x[c]), 0x141, 0xF, 0xF, true));
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x[c]), 0x140, 0xF, 0xF, true));
}

// Launch slot of the per-(tile, quadrant) waves. Consecutive workgroups go
// to the 8 XCDs in turn, each with its own L2, so workgroup 32k + 8q + x
// takes quadrant q of tile slot 8k + x: the four waves that stage the same
// tile list run on one XCD and share its L2. The grid is 32 ceil(tiles / 8);
// false for the slots past the last tile.
__device__ inline bool xcd_tile_quadrant(int n_tiles, int* slot, int* qd) {
    const int b = (int)blockIdx.x;
    *slot = 8 * (b >> 5) + (b & 7);
    *qd = (b >> 3) & 3;
    return *slot < n_tiles;
}
inline unsigned quadrant_grid(int64_t n_tiles) { return (unsigned)(32 * ((n_tiles + 7) / 8)); }

}  // namespace gs3
