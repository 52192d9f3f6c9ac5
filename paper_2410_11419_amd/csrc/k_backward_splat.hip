// Adjoints of the two per-tile splats: the camera splat (Sec. 3 Eq. 2-3,
// Fig. 2) and the shadow splat (Sec. 4.2, Fig. 3). Nothing per (pixel,
// splat) pair is stored by the forward: each kernel walks the same tile
// lists again with the same float32 arithmetic, so every hit, alpha,
// transmittance and stop decision is the forward's.
//
// Per-splat gradients are kept in the kernels' own parametrisation:
//   q = A dx^2 + B dx dy + C dy^2  (= power * log2 e),  dx = px - u,
// so the outputs are dL/du, dL/dv, dL/dA, dL/dB, dL/dC and dL/dopacity;
// the projection adjoint converts (A, B, C) to the conic (a, b, c).
#include "splat_common.h"

namespace gs3 {

constexpr float kLn2 = 0.69314718055994531f;
constexpr float kBwdEps = 9.5367431640625e-07f;   // 2^-20, the forward numerator's dark-ray bound

// Gradient of q with respect to the splat parameters at offset (dx, dy),
// scaled by dq: {u, v, A, B, C}.
struct QGrad {
    float u, v, A, B, C;
};
__device__ inline QGrad q_grad(float dq, float dx, float dy, float A, float B, float C) {
    QGrad g;
    g.u = -dq * fmaf(2.f * A, dx, B * dy);
    g.v = -dq * fmaf(B, dx, 2.f * C * dy);
    g.A = dq * dx * dx;
    g.B = dq * dx * dy;
    g.C = dq * dy * dy;
    return g;
}

// --------------------------------------------------------------------------
// Camera splat adjoint.
//
// Per pixel the forward composites 7 channels f_j = (c_j, T'_j, r_j):
// F = sum_j f_j alpha_j T_j. With C_j the value composited through hit j,
//   dF/df_j     = alpha_j T_j
//   dF/dalpha_j = T_j f_j - (F - C_j) / (1 - alpha_j)
// F is the forward's stored image; the walk recomputes C_j with the
// forward's operations in the forward's order, so F - C_j is the exact
// remainder up to rounding. The upstream gradient of the 7 channels follows
// from final = S * Sh + R.

struct RenderBwdArgs {
    const int2* ranges;
    const uint32_t* order;
    const uint32_t* list;
    const float4* rec0;
    const float4* rec1;
    const float4* rec2;   // {thr, hx, hy, p}
    const float4* col0;
    const float4* col1;
    uint32_t n;
    int width, height, tiles_x;
    float alpha_max, t_min;
    const float* S;      // [3][H][W]
    const float* Sh;     // [H][W]
    const float* R;      // [3][H][W]
    const float* dF;     // dL/dfinal [3][H][W]
    float* gsplat;       // [6][n] += {u, v, A, B, C, opacity}
    float* gcol;         // [7][n] += {c.rgb, T', r.rgb}
};

constexpr int kCamGrads = 13;

__global__ __launch_bounds__(256) void k_render_bwd(RenderBwdArgs a) {
    __shared__ Staged s_rec[256];
    __shared__ float4 s_c0[256];
    __shared__ float4 s_c1[256];
    __shared__ uint32_t s_mask[256];
    __shared__ uint32_t s_id[256];
    __shared__ float s_g[kCamGrads][256];
    const uint32_t ot = a.order[blockIdx.x];
    if (ot == kNoTile) return;
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
    // stored forward values and upstream gradient of the 7 channels
    float F[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float G[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (inside) {
        const int64_t hw = (int64_t)a.width * a.height;
        const int64_t p = (int64_t)py * a.width + px;
        F[0] = a.S[p]; F[1] = a.S[hw + p]; F[2] = a.S[2 * hw + p];
        F[3] = a.Sh[p];
        F[4] = a.R[p]; F[5] = a.R[hw + p]; F[6] = a.R[2 * hw + p];
        const float d0 = a.dF[p], d1 = a.dF[hw + p], d2 = a.dF[2 * hw + p];
        G[0] = d0 * F[3]; G[1] = d1 * F[3]; G[2] = d2 * F[3];
        G[3] = fmaf(d0, F[0], fmaf(d1, F[1], d2 * F[2]));
        G[4] = d0; G[5] = d1; G[6] = d2;
    }
    float T = 1.f;
    float Cc[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    bool done = !inside;
    for (int i = tid; i < kCamGrads * 256; i += 256) (&s_g[0][0])[i] = 0.f;
    for (int b = s; b < e; b += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const int m = min(256, e - b);
        if (tid < m) {
            const uint32_t id = safe_id(a.list[b + tid], a.n);
            uint32_t mk;
            s_rec[tid] = stage_splat(id, a.rec0, a.rec1, a.rec2, nullptr, tile_x0, tile_y0, &mk);
            s_mask[tid] = mk;
            s_id[tid] = id;
            s_c0[tid] = a.col0[id];
            s_c1[tid] = a.col1[id];
        }
        __syncthreads();
        // the forward's sets of entries that can hit this wave's quadrant
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
            const float dx = pxc - sj.g0.x, dy = pyc - sj.g0.y;
            const float q = quad_q(dx, dy, sj.g0.z, sj.g0.w, sj.g1.x);
            bool hit = !done && q >= sj.g1.y;
            const float beta = fast_exp2(q);
            const float ob = sj.g1.z * beta;
            const float al = fminf(a.alpha_max, ob);
            const float tn = T * (1.f - al);
            if (hit && tn < a.t_min) {
                done = true;
                hit = false;
            }
            float gv[kCamGrads];
#pragma unroll
            for (int c = 0; c < kCamGrads; ++c) gv[c] = 0.f;
            if (hit) {
                const float wgt = al * T;
                const float4 c0 = s_c0[j];
                const float4 c1 = s_c1[j];
                const float f[7] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z};
                // the forward's blend, in its order
                Cc[0] = fmaf(wgt, f[0], Cc[0]);
                Cc[1] = fmaf(wgt, f[1], Cc[1]);
                Cc[2] = fmaf(wgt, f[2], Cc[2]);
                Cc[3] = fmaf(wgt, f[3], Cc[3]);
                Cc[4] = fmaf(wgt, f[4], Cc[4]);
                Cc[5] = fmaf(wgt, f[5], Cc[5]);
                Cc[6] = fmaf(wgt, f[6], Cc[6]);
                const float inv = __builtin_amdgcn_rcpf(1.f - al);   // about 1 ulp
                float dal = 0.f;
#pragma unroll
                for (int c = 0; c < 7; ++c) {
                    gv[6 + c] = G[c] * wgt;
                    dal = fmaf(G[c], fmaf(T, f[c], -(F[c] - Cc[c]) * inv), dal);
                }
                if (ob < a.alpha_max) {
                    const float dq = dal * al * kLn2;
                    const QGrad g = q_grad(dq, dx, dy, sj.g0.z, sj.g0.w, sj.g1.x);
                    gv[0] = g.u; gv[1] = g.v; gv[2] = g.A; gv[3] = g.B; gv[4] = g.C;
                    gv[5] = dal * beta;
                }
                T = tn;
            }
            if (__builtin_amdgcn_ballot_w64(hit)) {
                // per-row sums, added into the entry by one lane of each row
                row_sums16<kCamGrads>(gv);
                if ((lane & 15) == 15) {
#pragma unroll
                    for (int c = 0; c < kCamGrads; ++c)
                        if (gv[c] != 0.f) atomicAdd(&s_g[c][j], gv[c]);
                }
            }
          }
        }
        __syncthreads();
        if (tid < m) {
            const uint32_t id = s_id[tid];
#pragma unroll
            for (int c = 0; c < kCamGrads; ++c) {
                const float v = s_g[c][tid];
                if (v != 0.f) {
                    float* dst = c < 6 ? a.gsplat + (size_t)c * a.n : a.gcol + (size_t)(c - 6) * a.n;
                    atomicAdd(dst + id, v);
                    s_g[c][tid] = 0.f;
                }
            }
        }
    }
}

// --------------------------------------------------------------------------
// Shadow splat adjoint.
//
// T_j = num_j / den_j gives dL/dnum_j = g_j / den_j and
// dL/dden_j = -g_j T_j / den_j (g_j = dL/dT_j; both 0 where den_j = 0).
//  - den_j = sum_m beta_jm: k_shadow_den_bwd, one wave per Gaussian over its
//    footprint, like k_shadow_den.
//  - num_j = sum_m beta_jm T_m(j): for a ray m let w_jm = dL/dnum_j beta_jm
//    T_m(j) and G_m = sum_j w_jm. Occluder k enters T_m(j) for exactly the
//    leads j from the point where the forward's trailing pointer multiplies
//    it in, so dL/dalpha_km = -(G_m - P_m) / (1 - alpha_km), P_m being the
//    sum of w over the leads before that point. k_shadow_bwd<0> computes G_m
//    (same walk as the forward numerator), k_shadow_bwd<1> repeats the walk
//    with the running P_m. Terms the forward numerator drops (ray
//    transmittance below 2^-20) are dropped here too.

struct ShadowBwdArgs {
    const int2* ranges;
    const uint32_t* order;
    const uint32_t* list;
    const float4* rec0;
    const float4* rec1;
    const float4* rec2;   // {thr, hx, hy, p}
    const float* depth;
    const int4* drec;      // den_ranges per Gaussian (written by the projection)
    uint32_t n;
    int width, height, tiles_x, n_tiles;
    int n_slots;           // entries of order (some may be kNoTile)
    float alpha_max, bias;
    const float* T;        // [n] forward shadow values
    const float* num_den;  // [2][n]
    const float* dT;       // [n] dL/dT
    float* dnum;           // [n] dL/dnum (written by the den kernel)
    float* gray;           // [H][W] G_m per light pixel
    float* gsplat;         // [6][n] {u, v, A, B, C, opacity}
};

// den part: writes gsplat (=, the numerator sweeps then add) and dnum.
__global__ __launch_bounds__(256) void k_shadow_den_bwd(ShadowBwdArgs a) {
    // the Gaussian and its records are wave-uniform (scalar loop control)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = __lane_id();
    const int lx = lane & 15, ly = lane >> 4;
    const int n = (int)a.n;
    const int tiles_y = (a.height + kTile - 1) / kTile;
    // the forward denominator's pixel-centre offsets and partial-edge masks
    const float cx = (float)lx + 0.5f;
    float cy[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) cy[r] = (float)(4 * r + ly) + 0.5f;
    const int last_tx = (a.width & (kTile - 1)) ? a.tiles_x - 1 : -1;
    const int last_ty = (a.height & (kTile - 1)) ? tiles_y - 1 : -1;
    const bool lane_x_last = lx < (a.width & (kTile - 1));
    bool lane_y_last[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) lane_y_last[r] = 4 * r + ly < (a.height & (kTile - 1));
    auto uf4 = [](float4 x) { return make_float4(uniform_f(x.x), uniform_f(x.y), uniform_f(x.z), uniform_f(x.w)); };
    for (int g = blockIdx.x * 4 + w; g < n; g += gridDim.x * 4) {
        const float den = uniform_f(a.num_den[n + g]);
        const float dTg = uniform_f(a.dT[g]);
        const float dden = den > 0.f ? -dTg * uniform_f(a.T[g]) / den : 0.f;
        const int4 drv = a.drec[g];
        const int4 dr = make_int4(__builtin_amdgcn_readfirstlane(drv.x), __builtin_amdgcn_readfirstlane(drv.y),
                                  __builtin_amdgcn_readfirstlane(drv.z), __builtin_amdgcn_readfirstlane(drv.w));
        float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        // the forward denominator's culls (den_ranges, from the projection)
        const int box_lo = dr.x & 0xFFFF, box_hi = (dr.x >> 16) & 0x7FFF;
        const int g_lo = dr.y & 0xFFFF, g_hi = (dr.y >> 16) & 0xFFFF;
        const int y0 = -((3 - g_lo) >> 2), y1 = g_hi >> 2;   // rows with a group in [g_lo, g_hi]
        if (dden != 0.f && box_lo <= box_hi) {
            const float4 r0 = uf4(a.rec0[g]);
            const float4 r1 = uf4(a.rec1[g]);
            const float4 r2 = uf4(a.rec2[g]);
            float A, B, C;
            scaled_conic(r1, &A, &B, &C);
            const float thr = r2.x, hx = r2.y;
            bool banded = dr.x < 0;
            RowExtent rows;
            if (banded) {
                rows = row_extent(A, B, C, thr);
                banded = rows.valid;
            }
            {
                const float U = r0.x + r0.z;
                auto toi = [](float x) { return sgpr_i((int)fminf(fmaxf(x, -16777216.f), 16777216.f)); };
                auto col_range = [&](float lo, float hi, int* t_lo, int* t_hi) {
                    *t_lo = max(box_lo, toi(ceilf((U + lo - 15.55f) * (1.f / kTile))));
                    *t_hi = min(box_hi, toi(floorf((U + hi - 0.45f) * (1.f / kTile))));
                };
                const int iu = dr.z, iv = dr.w;
                for (int ty = y0; ty <= y1; ++ty) {
                    const int r_lo = max(0, g_lo - 4 * ty), r_hi = min(3, g_hi - 4 * ty);
                    if (r_lo > r_hi) continue;
                    const float v = (float)(iv - ty * kTile) + r0.w;
                    int t_lo = box_lo, t_hi = box_hi;
                    if (banded) {
                        // the ellipse's x-range within this tile row's pixel rows
                        float bl, bh;
                        if (!band_x_range(rows, 0.5f - v, 15.5f - v, &bl, &bh)) continue;
                        int b_lo, b_hi;
                        col_range(fmaxf(-hx, bl), fminf(hx, bh), &b_lo, &b_hi);
                        t_lo = max(t_lo, b_lo);
                        t_hi = min(t_hi, b_hi);
                    }
                    const bool row_full = ty != last_ty;
                    for (int tx = t_lo; tx <= t_hi; ++tx) {
                        const float u = (float)(iu - tx * kTile) + r0.z;
                        const float dx = cx - u;
                        const bool in_x = (tx != last_tx) | lane_x_last;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if (r < r_lo || r > r_hi) continue;
                            const float dy = cy[r] - v;
                            const float q = quad_q(dx, dy, A, B, C);
                            const bool hit = in_x & (row_full | lane_y_last[r]) & (q >= thr);
                            if (hit) {
                                const float dq = dden * fast_exp2(q) * kLn2;
                                const QGrad gq = q_grad(dq, dx, dy, A, B, C);
                                acc[0] += gq.u; acc[1] += gq.v; acc[2] += gq.A; acc[3] += gq.B; acc[4] += gq.C;
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const float sum = wave_sum_lane63(acc[c]);
            if (lane == 63) a.gsplat[(size_t)c * n + g] = sum;
        }
        if (lane == 63) {
            a.gsplat[(size_t)5 * n + g] = 0.f;
            a.dnum[g] = den > 0.f ? dTg / den : 0.f;
        }
    }
}

constexpr int kBwdBatch = 64;                    // list entries staged at a time: one per lane
constexpr int kBwdRingMask = 2 * kBwdBatch - 1;

// The forward numerator's walk (one wave per (tile, 8x8 quadrant), an LDS
// ring of two 64-entry batches, quadrant-masked leads, per-lead occluder
// segments [L(previous lead), L(j)) as sets of ring entries, older entries
// walked from global memory), carrying the adjoint. PASS 0: G_m per pixel.
// PASS 1: per-splat gradients.
template <int PASS>
__global__ __launch_bounds__(64) void k_shadow_bwd(ShadowBwdArgs a) {
    __shared__ Staged s_rec[2 * kBwdBatch];
    __shared__ uint32_t s_id[2 * kBwdBatch];
    __shared__ float s_dn[kBwdBatch];               // dL/dnum of the current batch's entries
    // PASS 1: gradients of the ring's entries collect here and go out in
    // bursts of atomics (a global atomic still counts as an outstanding
    // memory operation that the next load would wait for)
    __shared__ float s_acc[PASS == 1 ? 6 : 1][2 * kBwdBatch];
    int slot, qd;
    if (!xcd_tile_quadrant(a.n_slots, &slot, &qd)) return;
    const uint32_t ot = a.order[slot];
    if (ot == kNoTile) return;
    const int tile = (int)ot;
    const int2 rg = a.ranges[tile];
    const int s = rg.x, e = rg.y;
    const int lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int lx = (qd & 1) * 8 + (lane & 7), ly = (qd >> 1) * 8 + (lane >> 3);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    const float pxc = lx + 0.5f, pyc = ly + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    const bool inside = px < a.width && py < a.height;
    const int64_t pix = (int64_t)py * a.width + px;
    bool alive = inside;
    float gm = 0.f;                  // PASS 0: G_m; PASS 1: G_m - P_m
    if (PASS == 1 && inside) gm = a.gray[pix];
    const uint32_t qbit = 1u << qd;
    float tt = 1.f;
    unsigned long long prv = 0ull;
    int trail = s;
    bool finished = e <= s || !__builtin_amdgcn_ballot_w64(alive);
    if (PASS == 1) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            s_acc[c][lane] = 0.f;
            s_acc[c][lane + 64] = 0.f;
        }
    }
    // add the gradients of the `count` ring entries from slot `first` to
    // global memory and clear them (PASS 1)
    auto flush = [&](int first, int count) {
        if (lane < count) {
            const int slot = first + lane;
            const uint32_t id = s_id[slot];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const float v = s_acc[c][slot];
                if (v != 0.f) {
                    atomicAdd(&a.gsplat[(size_t)c * a.n + id], v);
                    s_acc[c][slot] = 0.f;
                }
            }
        }
    };
    // occluder k: T *= (1 - alpha); PASS 1 also its gradient, into ring slot
    // `slot`, or straight to global memory when k is older than the ring (-1)
    auto occlude = [&](const Staged& k, uint32_t kid, int slot) {
        const float dx = pxc - k.g0.x, dy = pyc - k.g0.y;
        const float q = quad_q(dx, dy, k.g0.z, k.g0.w, k.g1.x);
        const bool hit = alive && q >= k.g1.y;
        // the first sweep takes no branch on the ballot (its latency-bound
        // walk loses more to the branch than the unused evaluation costs)
        if (PASS == 1 && !__builtin_amdgcn_ballot_w64(hit)) return;
        const float beta = fast_exp2(q);
        const float ob = k.g1.z * beta;
        const float al = fminf(a.alpha_max, ob);
        if (PASS == 1) {
            float g[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (hit && gm != 0.f && ob < a.alpha_max) {
                // hardware reciprocal (about 1 ulp) instead of a division
                const float dal = -gm * __builtin_amdgcn_rcpf(1.f - al);
                const QGrad gq = q_grad(dal * al * kLn2, dx, dy, k.g0.z, k.g0.w, k.g1.x);
                g[0] = gq.u; g[1] = gq.v; g[2] = gq.A; g[3] = gq.B; g[4] = gq.C;
                g[5] = dal * beta;
            }
            if (__builtin_amdgcn_ballot_w64(g[5] != 0.f)) {
                if (slot >= 0) {
                    // per-row sums, added into the slot by one lane of each row
                    row_sums16<6>(g);
                    if ((lane & 15) == 15) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) atomicAdd(&s_acc[c][slot], g[c]);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        const float sum = wave_sum_lane63(g[c]);
                        if (lane == 63) atomicAdd(&a.gsplat[(size_t)c * a.n + kid], sum);
                    }
                }
            }
        }
        if (hit) tt *= 1.f - al;
    };
    // the occluders of one set of ring entries in order, each record read
    // from LDS while the previous one is being applied
    auto occlude_set = [&](unsigned long long m, int slot0) {
        if (!m) return;
        int k = slot0 + __builtin_ctzll(m);
        Staged cur_rec = s_rec[k];
        m &= m - 1ull;
        while (m) {
            const int k2 = slot0 + __builtin_ctzll(m);
            const Staged nxt = s_rec[k2];
            m &= m - 1ull;
            occlude(cur_rec, 0u, k);
            cur_rec = nxt;
            k = k2;
        }
        occlude(cur_rec, 0u, k);
    };
    int last_base = 0, last_m = 0;
    for (int b = s; b < e && !finished; b += kBwdBatch) {
        const int m = min(kBwdBatch, e - b);
        const int base = (b - s) & kBwdRingMask;
        const int pbase = base ^ kBwdBatch;
        last_base = base;
        last_m = m;
        bool qm = false;
        if (lane < m) {
            uint32_t mk;
            const uint32_t id = safe_id(a.list[b + lane], a.n);
            const Staged rec = stage_splat(id, a.rec0, a.rec1, a.rec2, a.depth, tile_x0, tile_y0, &mk);
            s_rec[base + lane] = rec;
            s_id[base + lane] = id;
            s_dn[lane] = a.dnum[id];
            qm = (mk & qbit) != 0u && quad_reach(rec, qd);
        }
        const unsigned long long cur = __builtin_amdgcn_ballot_w64(qm);
        __syncthreads();
        const int lo_pos = max(s, b - kBwdBatch);
        int L = b + min(lane, m);
        if (lane < m) {
            const float thr = s_rec[base + lane].g1.w - a.bias;
            if (lo_pos > s && !(s_rec[(lo_pos - s) & kBwdRingMask].g1.w < thr)) {
                L = -1;
            } else {
                int lo = lo_pos, hi = b + lane;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_rec[(mid - s) & kBwdRingMask].g1.w < thr) lo = mid + 1; else hi = mid;
                }
                L = lo;
            }
        }
        const unsigned long long before = __builtin_amdgcn_ballot_w64(L < 0);
        // lead j: false when every pixel of the quadrant is dark
        auto lead_eval = [&](int j, const Staged& sj) {
            alive = alive && tt >= kBwdEps;
            if (!__builtin_amdgcn_ballot_w64(alive)) return false;
            const float dx = pxc - sj.g0.x, dy = pyc - sj.g0.y;
            const float q = quad_q(dx, dy, sj.g0.z, sj.g0.w, sj.g1.x);
            const bool hit = alive && q >= sj.g1.y;
            if (PASS == 0 || __builtin_amdgcn_ballot_w64(hit)) {
                const float dn = s_dn[j];
                const float beta = fast_exp2(q);
                const float wv = hit ? dn * beta * tt : 0.f;
                if (PASS == 0) {
                    gm += wv;
                } else {
                    if (dn != 0.f) {
                        float g[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
                        if (hit) {
                            const QGrad gq = q_grad(wv * kLn2, dx, dy, sj.g0.z, sj.g0.w, sj.g1.x);
                            g[0] = gq.u; g[1] = gq.v; g[2] = gq.A; g[3] = gq.B; g[4] = gq.C;
                        }
                        row_sums16<5>(g);
                        if ((lane & 15) == 15) {
#pragma unroll
                            for (int c = 0; c < 5; ++c) atomicAdd(&s_acc[c][base + j], g[c]);
                        }
                    }
                    gm -= wv;
                }
            }
            return true;
        };
        // leads whose L lies before the ring: walk older entries from global
        // memory up to L, comparing distances
        unsigned long long todo = cur & before;
        while (todo) {
            const int j = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            const float thr_d = uniform_f(s_rec[base + j].g1.w) - a.bias;
            while (trail < lo_pos) {
                uint32_t mk;
                const uint32_t kid = safe_id(a.list[trail], a.n);
                const Staged tk = stage_splat(kid, a.rec0, a.rec1, a.rec2, a.depth, tile_x0, tile_y0, &mk);
                if (!(uniform_f(tk.g1.w) < thr_d)) break;
                if (uniform_u(mk) & qbit) occlude(tk, uniform_u(kid), -1);
                ++trail;
            }
            if (!lead_eval(j, s_rec[base + j])) {
                finished = true;
                break;
            }
        }
        todo = cur & ~before;
        if (!finished && todo) {
            // entries before the ring precede every remaining lead's L
            while (trail < lo_pos) {
                uint32_t mk;
                const uint32_t kid = safe_id(a.list[trail], a.n);
                const Staged tk = stage_splat(kid, a.rec0, a.rec1, a.rec2, a.depth, tile_x0, tile_y0, &mk);
                if (uniform_u(mk) & qbit) occlude(tk, uniform_u(kid), -1);
                ++trail;
            }
            // the lane's segment [max(trail, L(previous lead)), L) as sets of
            // ring entries of the previous and the current batch
            const unsigned long long below = todo & ((1ull << lane) - 1ull);
            const int prev = below ? 63 - __builtin_clzll(below) : 0;
            const int Lprev = __builtin_amdgcn_ds_bpermute(prev << 2, L);
            const int lo_abs = below ? max(Lprev, trail) : trail;
            unsigned long long mp = 0ull, mc = 0ull;
            if ((todo >> lane) & 1ull) {
                mp = range_mask64(lo_abs - (b - kBwdBatch), L - (b - kBwdBatch)) & prv;
                mc = range_mask64(lo_abs - b, L - b) & cur;
            }
            const int last = 63 - __builtin_clzll(todo);
            while (todo) {
                const int j = __builtin_ctzll(todo);
                todo &= todo - 1ull;
                // the lead's record is read while its occluders are applied
                const Staged sj = s_rec[base + j];
                occlude_set(readlane64(mp, j), pbase);
                occlude_set(readlane64(mc, j), base);
                if (!lead_eval(j, sj)) {
                    finished = true;
                    break;
                }
            }
            trail = __builtin_amdgcn_readlane(L, last);
        }
        // the previous batch leaves the ring: its gradients are final
        if (PASS == 1 && b - kBwdBatch >= s) flush(pbase, kBwdBatch);
        prv = cur;
        __syncthreads();
    }
    if (PASS == 1 && last_m > 0) flush(last_base, last_m);
    if (PASS == 0 && inside) a.gray[pix] = gm;
}

// --------------------------------------------------------------------------

hipError_t launch_render_bwd(const gs3_consts& k, const Layout& L, const void* ws, const gs3_images& fwd,
                             const float* dF, float* gsplat, float* gcol, hipStream_t st) {
    if (L.n == 0 || L.n_tiles == 0) return hipSuccess;
    RenderBwdArgs a;
    a.ranges = at<int2>(ws, L.ranges);
    a.order = at<uint32_t>(ws, L.order);
    a.list = at<uint32_t>(ws, L.pv_a);
    a.rec0 = at<float4>(ws, L.rec0);
    a.rec1 = at<float4>(ws, L.rec1);
    a.rec2 = at<float4>(ws, L.rec2);
    a.col0 = at<float4>(ws, L.col0);
    a.col1 = at<float4>(ws, L.col1);
    a.n = (uint32_t)L.n;
    a.width = L.width;
    a.height = L.height;
    a.tiles_x = L.tiles_x;
    a.alpha_max = k.alpha_max;
    a.t_min = k.t_min;
    a.S = fwd.shading;
    a.Sh = fwd.shadow;
    a.R = fwd.residual;
    a.dF = dF;
    a.gsplat = gsplat;
    a.gcol = gcol;
    hipLaunchKernelGGL(k_render_bwd, dim3((unsigned)L.n_slots), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_shadow_bwd(const gs3_consts& k, const Layout& L, const void* ws, const float* T,
                             const float* num_den, const float* dT, float* dnum, float* gray, float* gsplat,
                             hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    ShadowBwdArgs a;
    a.ranges = at<int2>(ws, L.ranges);
    a.order = at<uint32_t>(ws, L.order);
    a.list = at<uint32_t>(ws, L.pv_a);
    a.rec0 = at<float4>(ws, L.rec0);
    a.rec1 = at<float4>(ws, L.rec1);
    a.rec2 = at<float4>(ws, L.rec2);
    a.depth = at<float>(ws, L.depth);
    a.drec = at<int4>(ws, L.drec);
    a.n = (uint32_t)L.n;
    a.width = L.width;
    a.height = L.height;
    a.tiles_x = L.tiles_x;
    a.n_tiles = (int)L.n_tiles;
    a.n_slots = (int)L.n_slots;
    a.alpha_max = k.alpha_max;
    a.bias = k.shadow_bias;
    a.T = T;
    a.num_den = num_den;
    a.dT = dT;
    a.dnum = dnum;
    a.gray = gray;
    a.gsplat = gsplat;
    int grid = (int)((L.n + 3) / 4);
    if (grid > 32768) grid = 32768;
    hipLaunchKernelGGL(k_shadow_den_bwd, dim3(grid), dim3(256), 0, st, a);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(gray), 0u, (int64_t)L.width * L.height, st);
    if (e != hipSuccess) return e;
    if (L.n_tiles == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_shadow_bwd<0>, dim3(quadrant_grid(L.n_slots)), dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_shadow_bwd<1>, dim3(quadrant_grid(L.n_slots)), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace gs3
