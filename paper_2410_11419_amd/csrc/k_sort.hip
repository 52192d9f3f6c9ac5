// Tile binning and depth ordering (Sec. 3: splats are sorted per pixel;
// Sec. 4.2: toward the light they are sorted by distance).
//
// Every tile's list must be ordered by (float32 depth bits, Gaussian index).
// Instead of a radix sort over 64-bit (tile, depth) keys of all P pairs, the
// N splats are first put in depth order (a 32-bit LSD radix sort of N keys,
// stable, so equal depths stay in index order), pairs are emitted in that
// order, and a stable LSD radix sort by tile index alone (ceil(log2 tiles)
// bits) then leaves each tile's pairs in depth order. Same lists, far fewer
// bytes moved per pair than sorting 64-bit keys.
#include "gs3_internal.h"
#include <climits>

namespace gs3 {

__device__ inline int lane_id() { return __lane_id(); }

// exclusive block scan of one u32 per thread (blockDim.x == 256)
__device__ inline uint32_t block_excl_scan_256(uint32_t v, uint32_t* total, uint32_t* s_wave) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t t = s_wave[i];
        wpre += (i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return wpre + x - v;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = value;
}

// ---------------------------------------------------------------- scan

// With gather given, element i of the scanned sequence is in[gather[i]].
__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, const uint32_t* __restrict__ gather,
                                                      int64_t len, uint32_t* __restrict__ sums) {
    __shared__ uint32_t s_wave[4];
    const int64_t base = (int64_t)blockIdx.x * kSortItems + threadIdx.x * 16;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t i = base + j;
        acc += (i < len) ? in[gather ? gather[i] : i] : 0u;
    }
    uint32_t tot;
    block_excl_scan_256(acc, &tot, s_wave);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of m block sums in place; the grand
// total (64-bit) optionally goes to the view header.
__global__ __launch_bounds__(256) void k_scan_top(uint32_t* __restrict__ sums, int64_t m,
                                                   ViewHeader* __restrict__ hdr, int64_t capacity,
                                                   uint32_t* __restrict__ tail_out) {
    __shared__ uint32_t s_wave[4];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < m; base += 256) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < m ? sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_256(v, &tot, s_wave);
        if (i < m) sums[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (hdr) {
            hdr->required_pairs = carry;
            const unsigned long long cap = (unsigned long long)capacity;
            hdr->n_pairs = (uint32_t)(carry < cap ? carry : cap);
            hdr->overflow = carry > cap ? 1u : 0u;
        }
        if (tail_out) *tail_out = (uint32_t)carry;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* __restrict__ in, const uint32_t* __restrict__ gather,
                                                    int64_t len, const uint32_t* __restrict__ sums,
                                                    uint32_t* __restrict__ out) {
    __shared__ uint32_t s_wave[4];
    const int64_t base = (int64_t)blockIdx.x * kSortItems + threadIdx.x * 16;
    uint32_t vals[16];
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t i = base + j;
        vals[j] = (i < len) ? in[gather ? gather[i] : i] : 0u;
        acc += vals[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan_256(acc, &tot, s_wave) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t i = base + j;
        if (i < len) out[i] = run;
        run += vals[j];
    }
}

static hipError_t exclusive_scan(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t len,
                                 uint32_t* sums, ViewHeader* hdr, int64_t capacity, uint32_t* tail_out,
                                 hipStream_t st) {
    const int64_t nb = (len + kSortItems - 1) / kSortItems;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, sums, (int64_t)0, hdr, capacity, tail_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, st, in, gather, len, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, sums, nb, hdr, capacity, tail_out);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(256), 0, st, in, gather, len, sums, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix

// Per-block digit histogram of keys[base .. base+ITEMS), written digit-major
// into table[digit * nblk + block]. n is read from *n_dev when given.
template <int ITEMS>
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                                                     uint32_t n_host, int shift, uint32_t* __restrict__ table, int nblk) {
    __shared__ uint32_t h[4][kRadixBins];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int i = tid; i < 4 * kRadixBins; i += 256) (&h[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t base = blockIdx.x * (uint32_t)ITEMS;
    if (base < n) {
#pragma unroll 4
        for (int r = 0; r < ITEMS / 256; ++r) {
            const uint32_t idx = base + r * 256 + tid;
            if (idx < n) atomicAdd(&h[w][(keys[idx] >> shift) & (kRadixBins - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < kRadixBins; d += 256) table[d * nblk + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Exclusive scan of each digit's row of the digit-major table, in place:
// workgroup d scans table[d nblk, (d + 1) nblk) and writes the row total
// (the digit's count over all blocks) to totals[d].
__global__ __launch_bounds__(256) void k_radix_rowscan(uint32_t* __restrict__ table, int nblk,
                                                        uint32_t* __restrict__ totals) {
    __shared__ uint32_t s_wave[4];
    uint32_t* row = table + (size_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int base = 0; base < nblk; base += 256 * 4) {
        const int i0 = base + threadIdx.x * 4;
        uint32_t v[4], acc = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = (i0 + j < nblk) ? row[i0 + j] : 0u;
            acc += v[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl_scan_256(acc, &tot, s_wave);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < nblk) row[i0 + j] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter. Wave w of the block owns the contiguous items
// [w ITEMS/4, (w + 1) ITEMS/4) and ranks them 64 at a time against its own
// running per-digit counts (ballot multisplit; no barrier between rounds).
// After one barrier the per-digit totals give each wave's offset within its
// digit and the block's digit starts; items are staged digit-sorted in LDS
// and each digit run goes to its global offset: the digit's start (the
// exclusive scan of the 256 digit totals, done here) plus the digit's count
// in earlier blocks (the row-scanned table). An item's rank counts exactly
// the earlier items of its block with the same digit, so ties keep input
// order.
template <int ITEMS, bool VALS, bool FINAL>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                        uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                        const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift,
                                                        const uint32_t* __restrict__ table,
                                                        const uint32_t* __restrict__ totals, int nblk, int id_bits,
                                                        int* __restrict__ ranges) {
    constexpr int PER_WAVE = ITEMS / 4;
    constexpr int R = PER_WAVE / 64;
    static_assert(R * 64 * 4 == ITEMS, "ITEMS must be a multiple of 256");
    __shared__ uint32_t s_key[ITEMS];
    __shared__ uint32_t s_val[VALS ? ITEMS : 1];
    __shared__ uint32_t s_cnt[4][kRadixBins];   // per-wave digit counts, then each wave's offset in its digit
    __shared__ uint32_t s_lstart[kRadixBins];
    __shared__ uint32_t s_gstart[kRadixBins];
    __shared__ uint32_t s_wave[4];
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t base = blockIdx.x * (uint32_t)ITEMS;
    if (base >= n) return;   // whole block beyond the data: uniform exit
    const uint32_t count = (n - base) < (uint32_t)ITEMS ? (n - base) : (uint32_t)ITEMS;
    for (int i = tid; i < 4 * kRadixBins; i += 256) (&s_cnt[0][0])[i] = 0u;
    {
        const int d = tid;   // 256 threads, 256 digits
        uint32_t all;
        const uint32_t dstart = block_excl_scan_256(totals[d], &all, s_wave);
        s_gstart[d] = dstart + table[d * nblk + blockIdx.x];
    }
    __syncthreads();
    uint32_t key[R], val[R], rank[R];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = (uint32_t)(w * PER_WAVE + r * 64 + lane);
        const bool valid = idx < count;
        key[r] = valid ? kin[base + idx] : 0u;
        val[r] = (VALS && valid) ? vin[base + idx] : 0u;
        const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        // every lane reads its digit's count before the first lane of each
        // digit group advances it (program order within the wave)
        const uint32_t run = valid ? s_cnt[w][d] : 0u;
        rank[r] = run + before;
        if (valid && before == 0) s_cnt[w][d] = run + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: each wave's offset within the digit, and the block's digit
    // starts (exclusive scan of the totals)
    {
        const int d = tid;   // 256 threads, 256 digits
        const uint32_t c0 = s_cnt[0][d], c1 = s_cnt[1][d], c2 = s_cnt[2][d], c3 = s_cnt[3][d];
        s_cnt[0][d] = 0u;
        s_cnt[1][d] = c0;
        s_cnt[2][d] = c0 + c1;
        s_cnt[3][d] = c0 + c1 + c2;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_256(c0 + c1 + c2 + c3, &tot, s_wave);
        s_lstart[d] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = (uint32_t)(w * PER_WAVE + r * 64 + lane);
        if (idx < count) {
            const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
            const uint32_t p = s_lstart[d] + s_cnt[w][d] + rank[r];
            s_key[p] = key[r];
            if (VALS) s_val[p] = val[r];
        }
    }
    __syncthreads();
    for (uint32_t p = tid; p < count; p += 256) {
        const uint32_t k = s_key[p];
        const uint32_t d = (k >> shift) & (kRadixBins - 1);
        const uint32_t g = s_gstart[d] + (p - s_lstart[d]);
        if (FINAL) {
            // last pass over packed pairs: the block's staged keys are in
            // final order, so a run of one tile is contiguous here and in
            // the output; its ends widen the tile's range (atomics across
            // the blocks holding parts of the tile), and only the id is kept
            const uint32_t t = k >> id_bits;
            kout[g] = k & ((1u << id_bits) - 1u);
            if (p == 0 || (s_key[p - 1] >> id_bits) != t) atomicMin(&ranges[2 * t], (int)g);
            if (p == count - 1 || (s_key[p + 1] >> id_bits) != t) atomicMax(&ranges[2 * t + 1], (int)(g + 1));
        } else {
            kout[g] = k;
            if (VALS) vout[g] = s_val[p];
        }
    }
}

// One stable LSD pass over 8 bits: block histograms, row scan, scatter.
// ITEMS per workgroup: the table has ceil(max_items / ITEMS) * 256 entries
// (the layout sizes it for both sorts); sums holds the 256 digit totals.
// Without VALS only the keys move (values packed into their low bits);
// FINAL (last pass over packed pairs) writes the ids and the tile ranges.
template <int ITEMS, bool VALS, bool FINAL = false>
static hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                             const uint32_t* n_dev, uint32_t n_host, int64_t max_items, int shift,
                             uint32_t* table, uint32_t* sums, hipStream_t st, int id_bits = 0,
                             int2* ranges = nullptr) {
    const int nblk = (int)((max_items + ITEMS - 1) / ITEMS);
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_radix_hist<ITEMS>, dim3(nblk), dim3(256), 0, st, kin, n_dev, n_host, shift, table, nblk);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(kRadixBins), dim3(256), 0, st, table, nblk, sums);
    hipLaunchKernelGGL((k_radix_scatter<ITEMS, VALS, FINAL>), dim3(nblk), dim3(256), 0, st, kin, vin, kout, vout,
                       n_dev, n_host, shift, table, sums, nblk, id_bits, reinterpret_cast<int*>(ranges));
    return hipGetLastError();
}

// ---------------------------------------------------------------- emit

// Pairs of 256 depth-sorted splats per workgroup, one pair slot per lane.
// With id_bits > 0 a pair is one word, (tile << id_bits) | id, and pv is
// unused; otherwise the tile goes to pk and the id to pv. The grid also
// resets the per-tile ranges to (INT_MAX, 0): the range pass (or the last
// tile pass) fills in the tiles that have pairs, and k_tile_order turns the
// untouched ones into empty (0, 0) ranges.
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ offs,
                                               const int4* __restrict__ ext, int n, int tiles_x, uint32_t capacity,
                                               uint32_t* __restrict__ pk, uint32_t* __restrict__ pv,
                                               int2* __restrict__ ranges, int n_tiles, int id_bits) {
    __shared__ uint32_t s_lo[257];
    __shared__ int s_x0[256], s_y0[256], s_w[256];
    __shared__ uint32_t s_id[256];
    const int tid = threadIdx.x;
    for (int t = blockIdx.x * 256 + tid; t < n_tiles; t += gridDim.x * 256) ranges[t] = make_int2(INT_MAX, 0);
    const int s0 = blockIdx.x * 256;
    const int m = min(256, n - s0);
    const uint32_t base = offs[s0];
    if (tid < m) {
        const uint32_t g = ids[s0 + tid];
        s_id[tid] = g;
        s_lo[tid] = offs[s0 + tid] - base;
        const int4 e = ext[g];
        int x0 = 0, y0 = 0, w = 1;
        if (e.z > 0 && e.w > 0) {
            auto fdiv = [](int a) -> int { return a >= 0 ? a / kTile : -((-a + kTile - 1) / kTile); };
            x0 = max(fdiv(e.x - e.z), 0);
            y0 = max(fdiv(e.y - e.w), 0);
            const int x1 = min(fdiv(e.x + e.z), tiles_x - 1);
            w = x1 - x0 + 1;
            if (w < 1) w = 1;
        }
        s_x0[tid] = x0; s_y0[tid] = y0; s_w[tid] = w;
    }
    if (tid == 0) s_lo[m] = offs[s0 + m] - base;
    __syncthreads();
    const uint32_t total = s_lo[m];
    if (base >= capacity) return;
    const uint32_t room = capacity - base;              // slots left in the pair arrays
    const uint32_t lim = total < room ? total : room;
    for (uint32_t j = tid; j < lim; j += 256) {
        // last i with s_lo[i] <= j (s_lo is non-decreasing, s_lo[0] = 0)
        int lo = 0, hi = m - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_lo[mid] <= j) lo = mid; else hi = mid - 1;
        }
        const uint32_t k = j - s_lo[lo];
        const int w = s_w[lo];
        const uint32_t tile = (uint32_t)(s_y0[lo] + (int)(k / w)) * (uint32_t)tiles_x + (uint32_t)(s_x0[lo] + (int)(k % w));
        if (id_bits > 0) {
            pk[base + j] = (tile << id_bits) | s_id[lo];   // packed: tile above the id
        } else {
            pk[base + j] = tile;
            pv[base + j] = s_id[lo];
        }
    }
}

// Per-tile [start, end) of the sorted pairs. With packed pairs
// (id_bits > 0) the tile is the word's high part, and the ids are written
// to ids for the splatting kernels.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ pk, const ViewHeader* __restrict__ hdr,
                                                 int2* __restrict__ ranges, uint32_t n_tiles, int id_bits,
                                                 uint32_t* __restrict__ ids) {
    const uint32_t n = hdr->n_pairs;
    if (hdr->overflow) return;   // an overflowed binning leaves every tile empty
    const uint32_t id_mask = id_bits > 0 ? (1u << id_bits) - 1u : 0u;
    for (uint32_t p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256) {
        const uint32_t w = pk[p];
        const uint32_t t = w >> id_bits;
        if (id_bits > 0) ids[p] = w & id_mask;
        if (t >= n_tiles) continue;
        if (p == 0 || (pk[p - 1] >> id_bits) != t) ranges[t].x = (int)p;
        if (p == n - 1 || (pk[p + 1] >> id_bits) != t) ranges[t].y = (int)(p + 1);
    }
}

// Final per-tile ranges, then the launch order of the tiles: longest list
// first (lengths bucketed by 8), so the few long tiles start early instead
// of forming the tail of the splatting kernels. Only the schedule depends on
// the order, not any result.
__global__ __launch_bounds__(1024) void k_tile_order(int2* __restrict__ ranges, int n_tiles,
                                                      const ViewHeader* __restrict__ hdr,
                                                      uint32_t* __restrict__ order) {
    __shared__ uint32_t hist[1024];
    __shared__ uint32_t s_wave[16];
    const int tid = threadIdx.x;
    hist[tid] = 0u;
    // tiles without pairs (still (INT_MAX, 0)) and every tile of an
    // overflowed binning become empty ranges; each thread later reads back
    // only the tiles it wrote here
    const bool overflow = hdr->overflow != 0u;
    for (int t = tid; t < n_tiles; t += 1024) {
        const int2 r = ranges[t];
        if (overflow || r.x >= r.y) ranges[t] = make_int2(0, 0);
    }
    __syncthreads();
    auto bucket = [&](int t) -> int {
        const int2 r = ranges[t];
        const int len = r.y - r.x;
        return 1023 - min(1023, max(len, 0) >> 3);
    };
    for (int t = tid; t < n_tiles; t += 1024) atomicAdd(&hist[bucket(t)], 1u);
    __syncthreads();
    // exclusive scan of the 1024 bucket counts
    const uint32_t v = hist[tid];
    uint32_t x = v;
    const int lane = __lane_id(), w = tid >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    uint32_t pre = 0;
    for (int i = 0; i < w; ++i) pre += s_wave[i];
    __syncthreads();
    hist[tid] = pre + x - v;
    __syncthreads();
    for (int t = tid; t < n_tiles; t += 1024) order[atomicAdd(&hist[bucket(t)], 1u)] = (uint32_t)t;
}

// The binning's outcome into the caller's host-pinned status word (see
// gs3_viewbuf.status): (generation mod 2^24) << 40 | overflow << 39 |
// required pairs, one 64-bit store, made visible to the host at once.
__global__ __launch_bounds__(64) void k_write_status(const ViewHeader* __restrict__ hdr, long long generation,
                                                      unsigned long long* __restrict__ status) {
    if (threadIdx.x != 0) return;
    const unsigned long long req = hdr->required_pairs;
    const unsigned long long req39 = req < (1ull << 39) ? req : (1ull << 39) - 1ull;
    const unsigned long long v = ((unsigned long long)(generation & 0xFFFFFF) << 40) |
                                 ((unsigned long long)(hdr->overflow ? 1u : 0u) << 39) | req39;
    __hip_atomic_store(status, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
}

hipError_t launch_write_status(const Layout& L, const void* ws, long long generation, int64_t* status_dev,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_write_status, dim3(1), dim3(64), 0, st, at<ViewHeader>(ws, L.hdr), generation,
                       reinterpret_cast<unsigned long long*>(status_dev));
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, value, count);
    return hipGetLastError();
}

// Depth sort of the splats, pair emission in depth order, stable sort of
// the pairs by tile, per-tile ranges. Inputs: keys_a/vals_a (depth bits /
// index), cnt, ext from the projection (or the explicit extents).
hipError_t launch_bin(const Layout& L, void* ws, hipStream_t st) {
    ViewHeader* hdr = at<ViewHeader>(ws, L.hdr);
    uint32_t* keys_a = at<uint32_t>(ws, L.keys_a);
    uint32_t* vals_a = at<uint32_t>(ws, L.vals_a);
    uint32_t* keys_b = at<uint32_t>(ws, L.keys_b);
    uint32_t* vals_b = at<uint32_t>(ws, L.vals_b);
    uint32_t* table = at<uint32_t>(ws, L.table);
    uint32_t* sums = at<uint32_t>(ws, L.sums);
    uint32_t* offs = at<uint32_t>(ws, L.offs);
    const uint32_t n = (uint32_t)L.n;
    hipError_t e;
    // 1. depth order: 4 stable 8-bit passes over the 32-bit depth keys, 1024
    //    keys per workgroup (N is small next to the pair count: more, shorter
    //    workgroups)
    for (int pass = 0; pass < 4; ++pass) {
        const bool even = (pass & 1) == 0;
        e = radix_pass<kSortItemsN, true>(even ? keys_a : keys_b, even ? vals_a : vals_b, even ? keys_b : keys_a,
                       even ? vals_b : vals_a, nullptr, n, L.n, pass * 8, table, sums, st);
        if (e != hipSuccess) return e;
    }
    // 2. pair offsets in depth order (the counts gathered through the order)
    e = exclusive_scan(at<uint32_t>(ws, L.cnt), vals_a, offs, L.n, sums, hdr, L.capacity, offs + L.n, st);
    if (e != hipSuccess) return e;
    // 3. emit (tile, id) pairs, packed into one word when tile and id bits
    // fit in 32 (only the keys then move through the tile passes); the
    // number of tile passes decides which buffer they start in so that the
    // sorted result lands in pk_a / pv_a
    int tile_bits = 0;
    while ((1ll << tile_bits) < L.n_tiles) ++tile_bits;
    const int tile_passes = tile_bits == 0 ? 0 : (tile_bits + kRadixBits - 1) / kRadixBits;
    uint32_t* pk_a = at<uint32_t>(ws, L.pk_a);
    uint32_t* pv_a = at<uint32_t>(ws, L.pv_a);
    uint32_t* pk_b = at<uint32_t>(ws, L.pk_b);
    uint32_t* pv_b = at<uint32_t>(ws, L.pv_b);
    const bool packed = L.id_bits > 0;
    // packed pairs start in pk_a and alternate with pk_b; the last pass
    // writes the ids to pv_a. Unpacked pairs start where the sorted result
    // lands in pk_a / pv_a.
    const bool start_b = !packed && (tile_passes & 1) == 1;
    {
        const unsigned emit_grid = n > 0 ? (n + 255) / 256 : 1u;
        hipLaunchKernelGGL(k_emit, dim3(emit_grid), dim3(256), 0, st, vals_a, offs, at<int4>(ws, L.ext), (int)n,
                           L.tiles_x, (uint32_t)L.capacity, start_b ? pk_b : pk_a, start_b ? pv_b : pv_a,
                           at<int2>(ws, L.ranges), (int)L.n_tiles, L.id_bits);
    }
    // 4. stable passes by tile index
    const uint32_t* n_dev = &hdr->n_pairs;
    for (int pass = 0; pass < tile_passes; ++pass) {
        const bool from_b = ((pass & 1) == 0) == start_b;
        const int shift = L.id_bits + pass * kRadixBits;
        if (packed && pass == tile_passes - 1) {
            e = radix_pass<kSortItems, false, true>(from_b ? pk_b : pk_a, nullptr, pv_a, nullptr, n_dev, 0u,
                                                    L.capacity, shift, table, sums, st, L.id_bits,
                                                    at<int2>(ws, L.ranges));
        } else if (packed) {
            e = radix_pass<kSortItems, false>(from_b ? pk_b : pk_a, nullptr, from_b ? pk_a : pk_b, nullptr, n_dev, 0u,
                                              L.capacity, shift, table, sums, st);
        } else {
            e = radix_pass<kSortItems, true>(from_b ? pk_b : pk_a, from_b ? pv_b : pv_a, from_b ? pk_a : pk_b,
                                             from_b ? pv_a : pv_b, n_dev, 0u, L.capacity, shift, table, sums, st);
        }
        if (e != hipSuccess) return e;
    }
    // 5. per-tile [start, end) (already done by the last pass over packed
    //    pairs)
    if (L.capacity > 0 && !(packed && tile_passes > 0)) {
        int64_t grid = (L.capacity + 255) / 256;
        if (grid > 1024) grid = 1024;
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)grid), dim3(256), 0, st, pk_a, hdr, at<int2>(ws, L.ranges),
                           (uint32_t)L.n_tiles, L.id_bits, pv_a);
    }
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, st, at<int2>(ws, L.ranges), (int)L.n_tiles, hdr,
                       at<uint32_t>(ws, L.order));
    return hipGetLastError();
}

}  // namespace gs3
