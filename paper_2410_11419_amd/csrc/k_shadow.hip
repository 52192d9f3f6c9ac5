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
// Both kernels test pixels with the same per-splat float32 threshold (the
// view's rec2, written by the projection) and the same float32 arithmetic
// (rel_centre, quad_q), so num and den see exactly the same hits.
#include "splat_common.h"
#include <type_traits>

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
    const float4* rec2;   // {thr, hx, hy, p}
    const float* depth;
    const int4* drec;   // den_ranges per Gaussian (written by the projection)
    uint32_t n;
    int width, height, tiles_x, n_tiles;
    int n_slots;             // entries of order (some may be kNoTile)
    float alpha_max, bias;
    unsigned long long* num;   // fixed point (kNumScale)
    float* den;
};

static_assert(kShadowBatch == 64, "the walk stages one list entry per lane per batch");

// The views of one launch: blockIdx.y selects the view, blockIdx.x runs
// over that view's work as in a launch of the view alone (the x extent is
// the largest view's; the surplus workgroups of smaller views exit).
struct ShadowBatch {
    ShadowArgs v[kMaxBatch];
};

// One wave per (tile, 8x8 quadrant): the four quadrants of a light tile run
// as independent single-wave workgroups, one pixel per lane. The wave stages
// its tile's list 64 entries at a time (one per lane) into an LDS ring that
// also keeps the previous batch; a ballot marks the entries whose hit
// ellipse can reach the quadrant, and only those are visited.
//
// For lead entry j, L(j) = the first list position whose distance is not
// below dist_j - bias; T_m(j) is the product of (1 - alpha) over the marked
// entries before L(j). L is non-decreasing along the list (distances are
// sorted), so the occluders that enter between two consecutive leads form
// the segment [L(previous lead), L(j)) of the list. Each lane finds L for
// its entry by a binary search over the ring's distances and turns its
// segment into two 64-bit sets (previous batch, current batch); the walk
// then reads the lead's two sets and multiplies in their entries, with no
// per-lead position arithmetic. Leads whose L lies before the ring (always
// the first leads of a batch) walk older entries from global memory
// instead, comparing distances; entries before the ring that precede every
// remaining lead are walked once. The lead's beta T_m(j) is summed per
// 16-lane row (DPP) into four partial sums per entry, which go to num_j in
// one burst of atomics per batch. The wave exits when all its pixels are
// dark.
template <bool ONE>
__global__ __launch_bounds__(64) void k_shadow(ShadowBatch B) {
    // ONE: a single view (static argument offsets)
    const ShadowArgs a = ONE ? B.v[0] : B.v[blockIdx.y];
    __shared__ Staged s_rec[2 * kShadowBatch];
    __shared__ uint32_t s_id[2 * kShadowBatch];
    __shared__ float s_sum[4][kShadowBatch];     // lead sums of the current batch, per 16-lane row
    int slot, qd;
    if (!xcd_tile_quadrant(a.n_slots, &slot, &qd)) return;
    const uint32_t ot = a.order[slot];
    if (ot == kNoTile) return;
    const int tile = (int)ot;
    const int2 rg = a.ranges[tile];
    const int s = rg.x, e = rg.y;
    if (e <= s) return;
    const int lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int lx = (qd & 1) * 8 + (lane & 7), ly = (qd >> 1) * 8 + (lane >> 3);
    const float pxc = lx + 0.5f, pyc = ly + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    bool alive = (tx * kTile + lx < a.width) && (ty * kTile + ly < a.height);
    if (!__builtin_amdgcn_ballot_w64(alive)) return;
    const uint32_t qbit = 1u << qd;
    float tt = 1.f;
    unsigned long long prv = 0ull;
    int trail = s;
    // multiply (1 - alpha) of occluder k into tt where it hits (the same
    // rounding as the adjoint's replay: the fminf keeps 1 - alpha from being
    // fused with the product)
    auto occlude = [&](const Staged& k) {
        const float q = splat_q(k, pxc, pyc);
        const bool hit = alive && q >= k.g1.y;
        // no branch on the ballot: a latency-bound walk loses more to the
        // branch than the unused evaluation costs
        const float f = 1.f - fminf(a.alpha_max, k.g1.z * fast_exp2(q));
        tt = hit ? tt * f : tt;
    };
    // the occluders of one set in order, each record read from LDS while
    // the previous one is being applied
    auto occlude_set = [&](unsigned long long m, int slot0) {
        if (!m) return;
        Staged cur_rec = s_rec[slot0 + __builtin_ctzll(m)];
        m &= m - 1ull;
        while (m) {
            const Staged nxt = s_rec[slot0 + __builtin_ctzll(m)];
            m &= m - 1ull;
            occlude(cur_rec);
            cur_rec = nxt;
        }
        occlude(cur_rec);
    };
    // A global atomic without a returned value still counts as an
    // outstanding vector memory operation, so the next wait for a load would
    // wait for it too: the lead sums of a batch collect in LDS and go out
    // in one burst of atomics when the batch ends.
    auto flush = [&](int base, int m) {
        if (lane < m) {
            const float v = (s_sum[0][lane] + s_sum[1][lane]) + (s_sum[2][lane] + s_sum[3][lane]);
            // v * 2^36 is exact in float; rounded to an integer it goes into
            // the fixed-point sum (order-independent)
            const unsigned long long u = __float2ull_rn(v * kNumScale);
            if (u != 0ull) atomicAdd(&a.num[s_id[base + lane]], u);
        }
    };
    for (int b = s; b < e; b += kShadowBatch) {
        const int m = min(kShadowBatch, e - b);
        const int base = (b - s) & kRingMask;          // ring slot of entry b
        const int pbase = base ^ kShadowBatch;         // ring slot of entry b - 64
        bool qm = false;
        if (lane < m) {
            uint32_t mk;
            const uint32_t id = safe_id(a.list[b + lane], a.n);
            const Staged rec = stage_splat(id, a.rec0, a.rec1, a.rec2, a.depth, tile_x0, tile_y0, &mk);
            s_rec[base + lane] = rec;
            s_id[base + lane] = id;
            qm = (mk & qbit) != 0u && quad_reach(rec, qd);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) s_sum[r][lane] = 0.f;
        const unsigned long long cur = __builtin_amdgcn_ballot_w64(qm);
        __syncthreads();
        // L for the lane's entry: the first position in [lo_pos, b + lane)
        // whose distance is not below dist - bias (b + lane if none); -1 when
        // it lies before the ring
        const int lo_pos = max(s, b - kShadowBatch);
        int L = b + min(lane, m);
        if (lane < m) {
            const float thr = s_rec[base + lane].g1.w - a.bias;
            if (lo_pos > s && !(s_rec[(lo_pos - s) & kRingMask].g1.w < thr)) {
                L = -1;
            } else {
                int lo = lo_pos, hi = b + lane;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_rec[(mid - s) & kRingMask].g1.w < thr) lo = mid + 1; else hi = mid;
                }
                L = lo;
            }
        }
        const unsigned long long before = __builtin_amdgcn_ballot_w64(L < 0);
        auto lead_eval = [&](int j, const Staged& sj) {
            alive = alive && tt >= kShadowEps;
            if (!__builtin_amdgcn_ballot_w64(alive)) return false;
            const float q = splat_q(sj, pxc, pyc);
            const bool hit = alive && q >= sj.g1.y;
            const float v = row_sum16(hit ? fast_exp2(q) * tt : 0.f);
            if ((lane & 15) == 15) s_sum[lane >> 4][j] = v;
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
                const Staged tk = stage_splat(safe_id(a.list[trail], a.n), a.rec0, a.rec1, a.rec2, a.depth, tile_x0, tile_y0, &mk);
                if (!(uniform_f(tk.g1.w) < thr_d)) break;
                if (uniform_u(mk) & qbit) occlude(tk);
                ++trail;
            }
            if (!lead_eval(j, s_rec[base + j])) {
                flush(base, m);
                return;
            }
        }
        todo = cur & ~before;
        if (todo) {
            // entries before the ring precede every remaining lead's L
            while (trail < lo_pos) {
                uint32_t mk;
                const Staged tk = stage_splat(safe_id(a.list[trail], a.n), a.rec0, a.rec1, a.rec2, a.depth, tile_x0, tile_y0, &mk);
                if (uniform_u(mk) & qbit) occlude(tk);
                ++trail;
            }
            // the lane's segment [max(trail, L(previous lead)), L) as sets of
            // ring entries: previous batch (positions b-64 ..) and current
            // batch (positions b ..)
            const unsigned long long below = todo & ((1ull << lane) - 1ull);
            const int prev = below ? 63 - __builtin_clzll(below) : 0;
            const int Lprev = __builtin_amdgcn_ds_bpermute(prev << 2, L);
            const int lo_abs = below ? max(Lprev, trail) : trail;
            const int W0 = b - kShadowBatch;
            unsigned long long mp = 0ull, mc = 0ull;
            if ((todo >> lane) & 1ull) {
                mp = range_mask64(lo_abs - W0, L - W0) & prv;
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
                    flush(base, m);
                    return;
                }
            }
            trail = __builtin_amdgcn_readlane(L, last);
        }
        flush(base, m);
        prv = cur;
        __syncthreads();
    }
}

// den_j = sum of beta over the pixels of the light image Gaussian j hits.
// One wave per Gaussian walks the 16x4 pixel blocks of the tiles it is
// binned to (the same pixels the tile kernel tests), skipping blocks outside
// the hit ellipse's bounding box; those culls come precomputed from the
// projection (den_ranges). The centre is formed relative to each tile's
// origin exactly as in stage_splat, so every pixel test is bit-identical to
// the one k_shadow makes.
// Everything but the pixel is the same in all lanes of the wave; the
// readfirstlane reads say so, which keeps the loops and the block culls in
// scalar registers and scalar branches.
template <bool ONE>
__global__ __launch_bounds__(256) void k_shadow_den(ShadowBatch B) {
    const ShadowArgs a = ONE ? B.v[0] : B.v[blockIdx.y];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = __lane_id();
    const int lx = lane & 15, ly = lane >> 4;
    const int n = (int)a.n;
    const int tiles_y = (a.height + kTile - 1) / kTile;
    // pixel-centre offsets of the lane, and the partial last tile column /
    // row (when the image size is not a multiple of 16) as lane masks
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
    const int stride = gridDim.x * 4;
    int g = blockIdx.x * 4 + w;
    // the next Gaussian's ranges and records are loaded while the current
    // one is evaluated
    int4 nx_dr = make_int4(1, 1, 0, 0);
    float4 nx_r0 = make_float4(0.f, 0.f, 0.f, 0.f), nx_r1 = nx_r0, nx_r2 = nx_r0;
    if (g < n) {
        nx_dr = a.drec[g];
        nx_r0 = a.rec0[g];
        nx_r1 = a.rec1[g];
        nx_r2 = a.rec2[g];
    }
    for (; g < n; g += stride) {
        const int4 dr = make_int4(__builtin_amdgcn_readfirstlane(nx_dr.x), __builtin_amdgcn_readfirstlane(nx_dr.y),
                                  __builtin_amdgcn_readfirstlane(nx_dr.z), __builtin_amdgcn_readfirstlane(nx_dr.w));
        const float4 r0 = uf4(nx_r0);
        const float4 r1 = uf4(nx_r1);
        const float4 r2 = uf4(nx_r2);
        if (g + stride < n) {
            nx_dr = a.drec[g + stride];
            nx_r0 = a.rec0[g + stride];
            nx_r1 = a.rec1[g + stride];
            nx_r2 = a.rec2[g + stride];
        }
        float acc = 0.f;
        // the culls computed by the projection (den_ranges)
        const int box_lo = dr.x & 0xFFFF, box_hi = (dr.x >> 16) & 0x7FFF;
        const int g_lo = dr.y & 0xFFFF, g_hi = (dr.y >> 16) & 0xFFFF;
        const int y0 = -((3 - g_lo) >> 2), y1 = g_hi >> 2;   // rows with a group in [g_lo, g_hi]
        if (box_lo <= box_hi) {
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
                // integer loop bounds and centre offsets in scalar registers
                auto toi = [](float x) { return sgpr_i((int)fminf(fmaxf(x, -16777216.f), 16777216.f)); };
                auto col_range = [&](float lo, float hi, int* t_lo, int* t_hi) {
                    *t_lo = max(box_lo, toi(ceilf((U + lo - 15.55f) * (1.f / kTile))));
                    *t_hi = min(box_hi, toi(floorf((U + hi - 0.45f) * (1.f / kTile))));
                };
                // the centre's integer part (rec0.x, rec0.y hold floor(u),
                // floor(v)); (float)(iu - ox) equals rec0.x - ox exactly
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
                    if (row_full && t_hi != last_tx) {
                        // no partial image edge in this tile row: row groups
                        // r_lo..r_hi of every column with the compare feeding
                        // the select directly (no masks, no per-block skips)
                        auto rows_of = [&](auto nr_c) {
                            constexpr int NR = decltype(nr_c)::value;
                            // cy[0] + 4 (r_lo + j) is exact, and is cy[j] when
                            // all four groups are taken (r_lo = 0)
                            float dyv[NR];
                            const float base = NR == 4 ? cy[0] : cy[0] + (float)(4 * r_lo);
#pragma unroll
                            for (int j = 0; j < NR; ++j) dyv[j] = (NR == 4 ? cy[j] : base + (float)(4 * j)) - v;
                            for (int k = iu - t_lo * kTile; k >= iu - t_hi * kTile; k -= kTile) {
                                const float dx = cx - ((float)k + r0.z);
#pragma unroll
                                for (int j = 0; j < NR; ++j) {
                                    const float q = quad_q(dx, dyv[j], A, B, C);
                                    float e = fast_exp2(q);
                                    asm volatile("" : "+v"(e));
                                    // acc += e where q >= thr, as a compare that
                                    // narrows the lane mask and a masked add: one
                                    // vector instruction fewer per block than
                                    // compare, select and add. The scalar moves
                                    // that save and restore the mask issue beside
                                    // other waves' vector work. thr is
                                    // wave-uniform; a NaN q fails both forms.
                                    float sum = acc;
                                    const float th = thr;
                                    unsigned long long saved;
                                    asm volatile(
                                        "s_mov_b64 %1, exec\n\t"
                                        "v_cmpx_le_f32_e32 vcc, %3, %2\n\t"
                                        "v_add_f32_e32 %0, %0, %4\n\t"
                                        "s_mov_b64 exec, %1"
                                        : "+v"(sum), "=&s"(saved)
                                        : "v"(q), "s"(th), "v"(e)
                                        : "vcc");
                                    acc = sum;
                                }
                            }
                        };
                        switch (r_hi - r_lo) {
                            case 3: rows_of(std::integral_constant<int, 4>{}); break;
                            case 2: rows_of(std::integral_constant<int, 3>{}); break;
                            case 1: rows_of(std::integral_constant<int, 2>{}); break;
                            default: rows_of(std::integral_constant<int, 1>{}); break;
                        }
                        continue;
                    }
                    for (int tx = t_lo; tx <= t_hi; ++tx) {
                        const float u = (float)(iu - tx * kTile) + r0.z;
                        const float dx = cx - u;
                        const bool in_x = (tx != last_tx) | lane_x_last;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if (r < r_lo || r > r_hi) continue;
                            const float dy = cy[r] - v;
                            const float q = quad_q(dx, dy, A, B, C);
                            // evaluated in every lane (no branch around it)
                            float e = fast_exp2(q);
                            asm volatile("" : "+v"(e));
                            const bool hit = (q >= thr) & in_x & (row_full | lane_y_last[r]);
                            acc += hit ? e : 0.f;
                        }
                    }
                }
            }
        }
        const float sum = wave_sum_lane63(acc);
        if (lane == 63) a.den[g] = sum;
    }
}

// T = num / den (1 where den = 0), with num taken from the view's
// accumulator, which is handed to the caller's num_den and cleared for the
// next numerator pass. A binning that overflowed its pair capacity left the
// tile lists empty, so num is missing every term: T is then NaN, not a
// plausible value.
struct FinishArgs {
    unsigned long long* acc;   // fixed point (kNumScale)
    float* num;
    const float* den;
    const ViewHeader* hdr;
    float* T;
};
struct FinishBatch {
    FinishArgs v[kMaxBatch];
};
__global__ __launch_bounds__(256) void k_shadow_finish(FinishBatch B, int n) {
    const FinishArgs f = B.v[blockIdx.y];
    unsigned long long* __restrict__ acc = f.acc;
    float* __restrict__ num = f.num;
    const float* __restrict__ den = f.den;
    const ViewHeader* __restrict__ hdr = f.hdr;
    float* __restrict__ T = f.T;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float nu = (float)((double)acc[i] * (1.0 / (double)kNumScale));
    acc[i] = 0ull;
    num[i] = nu;
    const float t = den[i] > 0.f ? nu / den[i] : 1.f;
    T[i] = hdr->overflow ? __builtin_nanf("") : t;
}

static ShadowArgs shadow_args(const gs3_consts& k, const Layout& L, void* ws, float* num_den) {
    ShadowArgs a;
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
    a.num = at<unsigned long long>(ws, L.num);   // the view's accumulator
    a.den = num_den + L.n;
    return a;
}

// Launches over nv views in chunks of kMaxBatch (blockIdx.y = view).
template <typename Fill>
static hipError_t batched(int nv, Fill fill) {
    for (int v0 = 0; v0 < nv; v0 += kMaxBatch) {
        const int m = nv - v0 < kMaxBatch ? nv - v0 : kMaxBatch;
        hipError_t e = fill(v0, m);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_shadow_den_batch(const gs3_consts& k, const Layout* const* Ls, void* const* wss,
                                   float* const* num_den, int nv, hipStream_t st) {
    return batched(nv, [&](int v0, int m) {
        ShadowBatch B;
        int64_t gx = 0;
        for (int i = 0; i < m; ++i) {
            B.v[i] = shadow_args(k, *Ls[v0 + i], wss[v0 + i], num_den[v0 + i]);
            gx = Ls[v0 + i]->n > gx ? Ls[v0 + i]->n : gx;
        }
        if (gx == 0) return hipSuccess;
        int grid = (int)((gx + 3) / 4);
        if (grid > 32768) grid = 32768;
        if (m == 1)
            hipLaunchKernelGGL(k_shadow_den<true>, dim3(grid), dim3(256), 0, st, B);
        else
            hipLaunchKernelGGL(k_shadow_den<false>, dim3(grid, m), dim3(256), 0, st, B);
        return hipGetLastError();
    });
}

hipError_t launch_shadow_num_batch(const gs3_consts& k, const Layout* const* Ls, void* const* wss,
                                   float* const* num_den, int nv, hipStream_t st) {
    return batched(nv, [&](int v0, int m) {
        ShadowBatch B;
        unsigned gx = 0;
        for (int i = 0; i < m; ++i) {
            const Layout& L = *Ls[v0 + i];
            B.v[i] = shadow_args(k, L, wss[v0 + i], num_den[v0 + i]);
            // a view without Gaussians has no list to walk
            if (L.n == 0) B.v[i].n_slots = 0;
            const unsigned g = L.n == 0 ? 0u : quadrant_grid(L.n_slots);
            gx = g > gx ? g : gx;
        }
        if (gx == 0) return hipSuccess;
        if (m == 1)
            hipLaunchKernelGGL(k_shadow<true>, dim3(gx), dim3(64), 0, st, B);
        else
            hipLaunchKernelGGL(k_shadow<false>, dim3(gx, m), dim3(64), 0, st, B);
        return hipGetLastError();
    });
}

hipError_t launch_shadow_resolve_batch(const Layout* const* Ls, void* const* wss, float* const* num_den,
                                       float* const* T, int nv, hipStream_t st) {
    return batched(nv, [&](int v0, int m) {
        FinishBatch B;
        const int64_t n = Ls[v0]->n;
        for (int i = 0; i < m; ++i) {
            const Layout& L = *Ls[v0 + i];
            void* ws = wss[v0 + i];
            B.v[i] = FinishArgs{at<unsigned long long>(ws, L.num), num_den[v0 + i], num_den[v0 + i] + L.n,
                                at<ViewHeader>(ws, L.hdr), T[v0 + i]};
        }
        if (n == 0) return hipSuccess;
        hipLaunchKernelGGL(k_shadow_finish, dim3((unsigned)((n + 255) / 256), m), dim3(256), 0, st, B, (int)n);
        return hipGetLastError();
    });
}

hipError_t launch_shadow_den(const gs3_consts& k, const Layout& L, void* ws, float* num_den, hipStream_t st) {
    const Layout* Ls[1] = {&L};
    return launch_shadow_den_batch(k, Ls, &ws, &num_den, 1, st);
}

hipError_t launch_shadow_num(const gs3_consts& k, const Layout& L, void* ws, float* num_den, hipStream_t st) {
    if (L.n_tiles == 0) return hipSuccess;
    const Layout* Ls[1] = {&L};
    return launch_shadow_num_batch(k, Ls, &ws, &num_den, 1, st);
}

hipError_t launch_shadow_resolve(const Layout& L, void* ws, float* num_den, float* T, hipStream_t st) {
    const Layout* Ls[1] = {&L};
    return launch_shadow_resolve_batch(Ls, &ws, &num_den, &T, 1, st);
}

hipError_t launch_shadow(const gs3_consts& k, const Layout& L, void* ws, float* num_den, float* T,
                         hipStream_t st) {
    hipError_t e = launch_shadow_den(k, L, ws, num_den, st);
    if (e == hipSuccess) e = launch_shadow_num(k, L, ws, num_den, st);
    if (e == hipSuccess) e = launch_shadow_resolve(L, ws, num_den, T, st);
    return e;
}

}  // namespace gs3
