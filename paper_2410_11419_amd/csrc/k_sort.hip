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

// ---------------------------------------------------------------- batches
//
// Every kernel below runs over a batch of up to kMaxBatch views in one
// launch: the grid is the concatenation of each view's own grid, block b
// belongs to view v with blk0[v] <= b < blk0[v + 1], and each view's
// descriptor carries its own buffers and sizes. A single view is a batch of
// one. Views with an empty grid take no blocks.

__device__ inline int batch_view(const uint32_t* blk0, int nv, uint32_t b) {
    int v = 0;
    while (v + 1 < nv && b >= blk0[v + 1]) ++v;
    return v;
}

__device__ inline uint32_t digit_of(uint32_t k, int shift) {
    return shift < 32 ? (k >> shift) & (kRadixBins - 1) : 0u;
}

template <class D>
struct Batch {
    int32_t nv = 0;
    uint32_t blk0[kMaxBatch + 1] = {};
    D d[kMaxBatch];
};

// Appends view descriptor `d` with `blocks` workgroups; returns the grid.
template <class D>
static void batch_add(Batch<D>& b, const D& d, uint32_t blocks) {
    b.d[b.nv] = d;
    b.blk0[b.nv + 1] = b.blk0[b.nv] + blocks;
    ++b.nv;
}

// ---------------------------------------------------------------- scan

// Exclusive scan of len u32 counts per view; with gather given, element i of
// the scanned sequence is in[gather[i]]. The grand total goes to the view
// header (required pairs, clamped count, overflow flag) and to tail_out.
// With per256 (gather given), k_scan_reduce alone runs, over 1024 elements
// per workgroup: sums[c] = the sum over elements [256 c, 256 c + 256)
// (k_emit forms the offsets from these).
struct ScanDesc {
    const uint32_t* in;
    const uint32_t* gather;
    uint32_t* out;
    uint32_t* sums;
    ViewHeader* hdr;
    uint32_t* tail_out;
    int64_t len;
    int64_t capacity;
    int64_t nb;
    int32_t per256;
};

__global__ __launch_bounds__(256) void k_scan_reduce(Batch<ScanDesc> B) {
    __shared__ uint32_t s_wave[4];
    const int v = batch_view(B.blk0, B.nv, blockIdx.x);
    const ScanDesc& D = B.d[v];
    const uint32_t blk = blockIdx.x - B.blk0[v];
    if (D.per256) {
        // 1024 elements per workgroup, 4 per thread: each wave sums one
        // 256-element chunk
        const int64_t c = (int64_t)blk * 4 + (threadIdx.x >> 6);
        const int64_t i0 = c * 256 + (threadIdx.x & 63) * 4;
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j;
            acc += (i < D.len) ? D.in[D.gather[i]] : 0u;
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) acc += __shfl_xor(acc, d, 64);
        if ((threadIdx.x & 63) == 0 && c * 256 < D.len) D.sums[c] = acc;
        return;
    }
    const int64_t base = (int64_t)blk * kSortItems + threadIdx.x * 16;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t i = base + j;
        acc += (i < D.len) ? D.in[D.gather ? D.gather[i] : i] : 0u;
    }
    uint32_t tot;
    block_excl_scan_256(acc, &tot, s_wave);
    if (threadIdx.x == 0) D.sums[blk] = tot;
}

// one workgroup per view: exclusive scan of the view's nb block sums in
// place, then the grand total (64-bit) to the header and the tail
__global__ __launch_bounds__(256) void k_scan_top(Batch<ScanDesc> B) {
    __shared__ uint32_t s_wave[4];
    const ScanDesc& D = B.d[blockIdx.x];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < D.nb; base += 256) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < D.nb ? D.sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_256(v, &tot, s_wave);
        if (i < D.nb) D.sums[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) {
        ViewHeader* hdr = D.hdr;
        hdr->required_pairs = carry;
        const unsigned long long cap = (unsigned long long)D.capacity;
        hdr->n_pairs = (uint32_t)(carry < cap ? carry : cap);
        hdr->overflow = carry > cap ? 1u : 0u;
        *D.tail_out = (uint32_t)carry;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(Batch<ScanDesc> B) {
    __shared__ uint32_t s_wave[4];
    const int v = batch_view(B.blk0, B.nv, blockIdx.x);
    const ScanDesc& D = B.d[v];
    const uint32_t blk = blockIdx.x - B.blk0[v];
    const int64_t base = (int64_t)blk * kSortItems + threadIdx.x * 16;
    uint32_t vals[16];
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t i = base + j;
        vals[j] = (i < D.len) ? D.in[D.gather ? D.gather[i] : i] : 0u;
        acc += vals[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan_256(acc, &tot, s_wave) + D.sums[blk];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t i = base + j;
        if (i < D.len) D.out[i] = run;
        run += vals[j];
    }
}

// ---------------------------------------------------------------- radix

// One stable LSD pass of a view: kin (+ vin) -> kout (+ vout) by the 8-bit
// digit at `shift` (digits at or above bit 32 are 0). n items, read from
// *n_dev when given; nblk workgroups of ITEMS items; table holds the
// digit-major per-block counts, totals the 256 digit totals. FINAL (last
// pass over packed pairs) writes ids to kout and the tile ranges.
struct RadixDesc {
    const uint32_t* kin;
    const uint32_t* vin;
    uint32_t* kout;
    uint32_t* vout;
    const uint32_t* n_dev;
    uint32_t* table;
    uint32_t* totals;
    int* ranges;
    uint32_t n_host;
    int32_t shift;
    int32_t nblk;
    int32_t id_bits;
};

// Per-block digit histogram of the block's keys, written digit-major into
// table[digit * nblk + block].
template <int ITEMS>
__global__ __launch_bounds__(256) void k_radix_hist(Batch<RadixDesc> B) {
    __shared__ uint32_t h[4][kRadixBins];
    const int v = batch_view(B.blk0, B.nv, blockIdx.x);
    const RadixDesc& D = B.d[v];
    const uint32_t blk = blockIdx.x - B.blk0[v];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int i = tid; i < 4 * kRadixBins; i += 256) (&h[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t n = D.n_dev ? *D.n_dev : D.n_host;
    const uint32_t base = blk * (uint32_t)ITEMS;
    const uint32_t* keys = D.kin;
    const int shift = D.shift;
    if (base < n) {
#pragma unroll 4
        for (int r = 0; r < ITEMS / 256; ++r) {
            const uint32_t idx = base + r * 256 + tid;
            if (idx < n) atomicAdd(&h[w][digit_of(keys[idx], shift)], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < kRadixBins; d += 256)
        D.table[d * D.nblk + blk] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Exclusive scan of each digit's row of a view's digit-major table, in
// place: workgroup (v, d) scans view v's row d and writes the row total
// (the digit's count over all blocks) to totals[d].
__global__ __launch_bounds__(256) void k_radix_rowscan(Batch<RadixDesc> B) {
    __shared__ uint32_t s_wave[4];
    const RadixDesc& D = B.d[blockIdx.x / kRadixBins];
    const int digit = blockIdx.x % kRadixBins;
    const int nblk = D.nblk;
    uint32_t* row = D.table + (size_t)digit * nblk;
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
    if (threadIdx.x == 0) D.totals[digit] = carry;
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
__global__ __launch_bounds__(256) void k_radix_scatter(Batch<RadixDesc> B) {
    constexpr int PER_WAVE = ITEMS / 4;
    constexpr int R = PER_WAVE / 64;
    static_assert(R * 64 * 4 == ITEMS, "ITEMS must be a multiple of 256");
    __shared__ uint32_t s_key[ITEMS];
    __shared__ uint32_t s_val[VALS ? ITEMS : 1];
    __shared__ uint32_t s_cnt[4][kRadixBins];   // per-wave digit counts, then each wave's offset in its digit
    __shared__ uint32_t s_lstart[kRadixBins];
    __shared__ uint32_t s_gstart[kRadixBins];
    __shared__ uint32_t s_wave[4];
    const int v = batch_view(B.blk0, B.nv, blockIdx.x);
    const RadixDesc& D = B.d[v];
    const uint32_t blk = blockIdx.x - B.blk0[v];
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const uint32_t n = D.n_dev ? *D.n_dev : D.n_host;
    const uint32_t base = blk * (uint32_t)ITEMS;
    if (base >= n) return;   // whole block beyond the data: uniform exit
    const int shift = D.shift;
    const int nblk = D.nblk;
    const uint32_t count = (n - base) < (uint32_t)ITEMS ? (n - base) : (uint32_t)ITEMS;
    for (int i = tid; i < 4 * kRadixBins; i += 256) (&s_cnt[0][0])[i] = 0u;
    {
        const int d = tid;   // 256 threads, 256 digits
        const uint32_t total = D.totals[d];
        const uint32_t earlier = D.table[d * nblk + blk];
        uint32_t all;
        const uint32_t dstart = block_excl_scan_256(total, &all, s_wave);
        s_gstart[d] = dstart + earlier;
    }
    __syncthreads();
    uint32_t key[R], val[R], rank[R];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = (uint32_t)(w * PER_WAVE + r * 64 + lane);
        const bool valid = idx < count;
        key[r] = valid ? D.kin[base + idx] : 0u;
        val[r] = (VALS && valid) ? D.vin[base + idx] : 0u;
        const uint32_t d = digit_of(key[r], shift);
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
            const uint32_t d = digit_of(key[r], shift);
            const uint32_t p = s_lstart[d] + s_cnt[w][d] + rank[r];
            s_key[p] = key[r];
            if (VALS) s_val[p] = val[r];
        }
    }
    __syncthreads();
    uint32_t* kout = D.kout;
    for (uint32_t p = tid; p < count; p += 256) {
        const uint32_t k = s_key[p];
        const uint32_t d = digit_of(k, shift);
        const uint32_t g = s_gstart[d] + (p - s_lstart[d]);
        if (FINAL) {
            // last pass over packed pairs: the block's staged keys are in
            // final order, so a run of one tile is contiguous here and in
            // the output; its ends widen the tile's range (atomics across
            // the blocks holding parts of the tile), and only the id is kept
            const int id_bits = D.id_bits;
            const uint32_t t = k >> id_bits;
            kout[g] = k & ((1u << id_bits) - 1u);
            if (p == 0 || (s_key[p - 1] >> id_bits) != t) atomicMin(&D.ranges[2 * t], (int)g);
            if (p == count - 1 || (s_key[p + 1] >> id_bits) != t) atomicMax(&D.ranges[2 * t + 1], (int)(g + 1));
        } else {
            kout[g] = k;
            if (VALS) D.vout[g] = s_val[p];
        }
    }
}

// One stable LSD pass over 8 bits for every view of the batch: block
// histograms, row scans, scatter. Each view's table has nblk * 256 entries
// (the layout sizes it for both sorts); totals holds its 256 digit totals.
template <int ITEMS, bool VALS, bool FINAL = false>
static hipError_t radix_pass(const Batch<RadixDesc>& B, hipStream_t st) {
    const uint32_t grid = B.blk0[B.nv];
    if (B.nv == 0 || grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_radix_hist<ITEMS>, dim3(grid), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_radix_rowscan, dim3((unsigned)(kRadixBins * B.nv)), dim3(256), 0, st, B);
    hipLaunchKernelGGL((k_radix_scatter<ITEMS, VALS, FINAL>), dim3(grid), dim3(256), 0, st, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------- emit

// Pairs of 256 depth-sorted splats per workgroup, one pair slot per lane.
// With id_bits > 0 a pair is one word, (tile << id_bits) | id, and pv is
// unused; otherwise the tile goes to pk and the id to pv. The view's blocks
// also reset its per-tile ranges to (INT_MAX, 0): the range pass (or the
// last tile pass) fills in the tiles that have pairs, and k_tile_order turns
// the untouched ones into empty (0, 0) ranges.
// offs == nullptr: the offsets are formed here from the 256-element chunk
// sums of the depth-ordered counts (sums, nb256 of them; k_scan_reduce with
// per256), and workgroup 0 writes the view header.
struct EmitDesc {
    const uint32_t* ids;
    const uint32_t* offs;
    const uint32_t* cnt;
    const uint32_t* sums;
    ViewHeader* hdr;
    int32_t nb256;
    const int4* ext;
    uint32_t* pk;
    uint32_t* pv;
    int2* ranges;
    int32_t n;
    int32_t tiles_x;
    uint32_t capacity;
    int32_t n_tiles;
    int32_t id_bits;
    int32_t nblk;
};

// sum over the workgroup of one u64 per thread (blockDim.x == 256)
__device__ inline unsigned long long block_sum_u64_256(unsigned long long x, unsigned long long* s_red) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) x += __shfl_xor(x, d, 64);
    if (lane_id() == 0) s_red[threadIdx.x >> 6] = x;
    __syncthreads();
    const unsigned long long t = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_emit(Batch<EmitDesc> B) {
    __shared__ uint32_t s_lo[257];
    __shared__ int s_x0[256], s_y0[256], s_w[256];
    __shared__ uint32_t s_id[256];
    __shared__ uint32_t s_wave[4];
    __shared__ unsigned long long s_red[4];
    const int v = batch_view(B.blk0, B.nv, blockIdx.x);
    const EmitDesc& D = B.d[v];
    const int blk = (int)(blockIdx.x - B.blk0[v]);
    const int tid = threadIdx.x;
    const int n = D.n, tiles_x = D.tiles_x, id_bits = D.id_bits;
    for (int t = blk * 256 + tid; t < D.n_tiles; t += D.nblk * 256) D.ranges[t] = make_int2(INT_MAX, 0);
    const int s0 = blk * 256;
    const int m = min(256, n - s0);
    unsigned long long base64;
    if (D.offs) {
        base64 = D.offs[s0];
    } else {
        // the offset of the workgroup's first pair: the chunk sums before
        // it (chunk c holds depth positions [256 c, 256 c + 256), so this
        // workgroup is chunk blk); workgroup 0 also forms the grand total
        unsigned long long pre = 0ull, all = 0ull;
        for (int c = tid; c < D.nb256; c += 256) {
            const uint32_t x = D.sums[c];
            pre += c < blk ? x : 0u;
            all += x;
        }
        base64 = block_sum_u64_256(pre, s_red);
        if (blk == 0) {
            const unsigned long long total = block_sum_u64_256(all, s_red);
            if (tid == 0) {
                ViewHeader* hdr = D.hdr;
                hdr->required_pairs = total;
                hdr->n_pairs = (uint32_t)(total < D.capacity ? total : D.capacity);
                hdr->overflow = total > D.capacity ? 1u : 0u;
            }
        }
    }
    // offsets within the workgroup (these fit in 32 bits: at most 256
    // splats, each over at most 2^24 tiles)
    uint32_t lo_own = 0u;
    if (!D.offs) {
        const uint32_t c = tid < m ? D.cnt[D.ids[s0 + tid]] : 0u;
        uint32_t tot;
        lo_own = block_excl_scan_256(c, &tot, s_wave);
        if (tid == 0) s_lo[m > 0 ? m : 0] = tot;
    }
    const uint32_t base = (uint32_t)base64;
    if (tid < m) {
        const uint32_t g = D.ids[s0 + tid];
        s_id[tid] = g;
        s_lo[tid] = D.offs ? D.offs[s0 + tid] - base : lo_own;
        const int4 e = D.ext[g];
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
    if (D.offs && tid == 0) s_lo[m > 0 ? m : 0] = D.offs[s0 + (m > 0 ? m : 0)] - base;
    __syncthreads();
    const uint32_t total = s_lo[m > 0 ? m : 0];
    if (base64 >= D.capacity) return;
    const uint32_t room = D.capacity - base;              // slots left in the pair arrays
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
            D.pk[base + j] = (tile << id_bits) | s_id[lo];   // packed: tile above the id
        } else {
            D.pk[base + j] = tile;
            D.pv[base + j] = s_id[lo];
        }
    }
}

// Per-tile [start, end) of the sorted pairs. With packed pairs
// (id_bits > 0) the tile is the word's high part, and the ids are written
// to ids for the splatting kernels.
struct RangesDesc {
    const uint32_t* pk;
    const ViewHeader* hdr;
    int2* ranges;
    uint32_t* ids;
    uint32_t n_tiles;
    int32_t id_bits;
    int32_t nblk;
};

__global__ __launch_bounds__(256) void k_ranges(Batch<RangesDesc> B) {
    const int v = batch_view(B.blk0, B.nv, blockIdx.x);
    const RangesDesc& D = B.d[v];
    const uint32_t blk = blockIdx.x - B.blk0[v];
    const uint32_t n = D.hdr->n_pairs;
    if (D.hdr->overflow) return;   // an overflowed binning leaves every tile empty
    const int id_bits = D.id_bits;
    const uint32_t id_mask = id_bits > 0 ? (1u << id_bits) - 1u : 0u;
    const uint32_t* pk = D.pk;
    for (uint32_t p = blk * 256 + threadIdx.x; p < n; p += (uint32_t)D.nblk * 256) {
        const uint32_t w = pk[p];
        const uint32_t t = w >> id_bits;
        if (id_bits > 0) D.ids[p] = w & id_mask;
        if (t >= D.n_tiles) continue;
        if (p == 0 || (pk[p - 1] >> id_bits) != t) D.ranges[t].x = (int)p;
        if (p == n - 1 || (pk[p + 1] >> id_bits) != t) D.ranges[t].y = (int)(p + 1);
    }
}

// Final per-tile ranges, then the launch order of the tiles. Only the
// schedule depends on the order, not any result. One workgroup per view.
// The order has n_slots entries; slot 8 k + x goes to XCD x (workgroups
// are dealt to the XCDs round-robin):
// - tiles are grouped in 8x8 blocks; the groups, sorted by their pairs,
//   are dealt to the eight XCDs in snake order (0..7, 7..0, ...), so each
//   XCD gets whole neighbourhoods (their splats' records stay in its L2)
//   and about an eighth of the work;
// - within an XCD the tiles go longest list first (lengths bucketed by
//   32), so its few long tiles start early instead of forming the tail;
// - slots an XCD does not fill hold kNoTile.
// Views with more than kMaxGroups groups take the longest-first order
// alone (lengths bucketed by 8) in slots 0 .. n_tiles - 1.
// With status given, the workgroup also reports the binning's outcome into
// the caller's host-pinned status word (see gs3_viewbuf.status):
// (generation mod 2^24) << 40 | overflow << 39 | required pairs, one 64-bit
// store, made visible to the host at once.
struct OrderDesc {
    int2* ranges;
    const ViewHeader* hdr;
    uint32_t* order;
    int32_t n_tiles;
    int32_t tiles_x;
    int32_t n_slots;
    unsigned long long* status;
    long long generation;
};

__global__ __launch_bounds__(1024) void k_tile_order(Batch<OrderDesc> B) {
    __shared__ uint32_t hist[1024];
    __shared__ uint32_t s_wave[16];
    __shared__ unsigned long long s_key[kMaxGroups];
    __shared__ uint8_t s_xcd[kMaxGroups];
    __shared__ uint32_t s_xstart[8];
    const OrderDesc& D = B.d[blockIdx.x];
    int2* ranges = D.ranges;
    const int n_tiles = D.n_tiles, tiles_x = D.tiles_x;
    const int tid = threadIdx.x;
    const int lane = __lane_id(), w = tid >> 6;
    // tiles without pairs (still (INT_MAX, 0)) and every tile of an
    // overflowed binning become empty ranges
    const bool overflow = D.hdr->overflow != 0u;
    if (tid == 0 && D.status) {
        const unsigned long long req = D.hdr->required_pairs;
        const unsigned long long req39 = req < (1ull << 39) ? req : (1ull << 39) - 1ull;
        const unsigned long long word = ((unsigned long long)(D.generation & 0xFFFFFF) << 40) |
                                        ((unsigned long long)(overflow ? 1u : 0u) << 39) | req39;
        __hip_atomic_store(D.status, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __threadfence_system();
    }
    for (int t = tid; t < n_tiles; t += 1024) {
        const int2 r = ranges[t];
        if (overflow || r.x >= r.y) ranges[t] = make_int2(0, 0);
    }
    for (int i = tid; i < D.n_slots; i += 1024) D.order[i] = kNoTile;
    hist[tid] = 0u;
    __syncthreads();
    auto len_of = [&](int t) -> uint32_t {
        const int2 r = ranges[t];
        return (uint32_t)max(r.y - r.x, 0);
    };
    const int ngx = (tiles_x + kGroupTiles - 1) / kGroupTiles;
    const int tiles_y = n_tiles / tiles_x;
    const int n_groups = ngx * ((tiles_y + kGroupTiles - 1) / kGroupTiles);
    const bool grouped = n_groups <= kMaxGroups;
    auto group_of = [&](int t) { return (t / tiles_x / kGroupTiles) * ngx + (t % tiles_x) / kGroupTiles; };
    if (grouped) {
        // pairs per group, then the groups sorted by them (descending; a
        // bitonic sort of (~pairs, group) keys) and dealt out in snake order
        for (int t = tid; t < n_tiles; t += 1024) atomicAdd(&hist[group_of(t)], len_of(t));
        __syncthreads();
        s_key[tid] = tid < n_groups ? ((unsigned long long)(~hist[tid]) << 32) | (unsigned)tid : ~0ull;
        __syncthreads();
        int span = 2;   // the sort's size: the power of two at or above n_groups
        while (span < n_groups) span <<= 1;
        for (int k = 2; k <= span; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int o = tid ^ j;
                if (tid < span && o > tid) {
                    const unsigned long long a = s_key[tid], b = s_key[o];
                    if ((a > b) == ((tid & k) == 0)) {
                        s_key[tid] = b;
                        s_key[o] = a;
                    }
                }
                __syncthreads();
            }
        if (tid < n_groups) {
            const int round = tid >> 3, pos = tid & 7;
            s_xcd[(uint32_t)s_key[tid]] = (uint8_t)((round & 1) ? 7 - pos : pos);
        }
        hist[tid] = 0u;
        __syncthreads();
    }
    auto bucket = [&](int t) -> int {
        const uint32_t len = len_of(t);
        return grouped ? (int)s_xcd[group_of(t)] * 128 + 127 - (int)min(127u, len >> 5)
                       : 1023 - (int)min(1023u, len >> 3);
    };
    for (int t = tid; t < n_tiles; t += 1024) atomicAdd(&hist[bucket(t)], 1u);
    __syncthreads();
    // exclusive scan of the 1024 bucket counts
    const uint32_t v = hist[tid];
    uint32_t x = v;
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
    if ((tid & 127) == 0) s_xstart[tid >> 7] = pre + x - v;   // first position of XCD tid / 128
    __syncthreads();
    for (int t = tid; t < n_tiles; t += 1024) {
        const int b = bucket(t);
        const uint32_t pos = atomicAdd(&hist[b], 1u);
        const uint32_t slot = grouped ? 8u * (pos - s_xstart[b >> 7]) + (uint32_t)(b >> 7) : pos;
        D.order[slot] = (uint32_t)t;
    }
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, value, count);
    return hipGetLastError();
}

static int tile_passes_of(const Layout& L) {
    int tile_bits = 0;
    while ((1ll << tile_bits) < L.n_tiles) ++tile_bits;
    return tile_bits == 0 ? 0 : (tile_bits + kRadixBits - 1) / kRadixBits;
}

// Binning of up to kMaxBatch views in one launch sequence: depth order of
// the splats, pair offsets, pair emission in depth order, stable passes by
// tile index, per-tile ranges and the tile launch order. Inputs of each
// view: keys_a / vals_a (depth bits / index), cnt and ext from the
// projection (or the explicit extents). Views with packed pairs and views
// without run their tile passes as two sub-batches; within one, every view
// takes the largest pass count (a pass over digits that are all 0 keeps the
// order), so the sorted result lands where the view's readers expect it.
static hipError_t bin_chunk(const Layout* const* Ls, void* const* wss, const StatusReq* const* status, int nv,
                            hipStream_t st) {
    hipError_t e;
    // Views of up to kEmitScanMaxN splats take the short form of step 2: the
    // pair offsets are formed inside k_emit from 256-splat sums (two launches
    // instead of four; every k_emit workgroup reads all nb256 sums).
    bool short_form = true;
    for (int v = 0; v < nv; ++v)
        if (Ls[v]->n > kEmitScanMaxN) short_form = false;
    // 1. depth order: 4 stable 8-bit passes over the 32-bit depth keys, 1024
    //    keys per workgroup (N is small next to the pair count: more, shorter
    //    workgroups)
    for (int pass = 0; pass < 4; ++pass) {
        const bool even = (pass & 1) == 0;
        Batch<RadixDesc> B;
        for (int v = 0; v < nv; ++v) {
            const Layout& L = *Ls[v];
            void* ws = wss[v];
            RadixDesc d{};
            d.kin = at<uint32_t>(ws, even ? L.keys_a : L.keys_b);
            d.vin = at<uint32_t>(ws, even ? L.vals_a : L.vals_b);
            d.kout = at<uint32_t>(ws, even ? L.keys_b : L.keys_a);
            d.vout = at<uint32_t>(ws, even ? L.vals_b : L.vals_a);
            d.n_dev = nullptr;
            d.n_host = (uint32_t)L.n;
            d.shift = pass * 8;
            d.table = at<uint32_t>(ws, L.table);
            d.totals = at<uint32_t>(ws, L.sums);
            d.nblk = (int32_t)L.nblk_n;
            batch_add(B, d, (uint32_t)L.nblk_n);
        }
        if ((e = radix_pass<kSortItemsN, true>(B, st)) != hipSuccess) return e;
    }
    // tile pass counts of the two sub-batches
    int passes[2] = {0, 0};   // [unpacked, packed]
    for (int v = 0; v < nv; ++v) {
        const int p = tile_passes_of(*Ls[v]);
        const int g = Ls[v]->id_bits > 0 ? 1 : 0;
        if (p > passes[g]) passes[g] = p;
    }
    // 2. pair offsets in depth order (the counts gathered through the order)
    if (short_form) {
        Batch<ScanDesc> B;
        for (int v = 0; v < nv; ++v) {
            const Layout& L = *Ls[v];
            void* ws = wss[v];
            ScanDesc d{};
            d.in = at<uint32_t>(ws, L.cnt);
            d.gather = at<uint32_t>(ws, L.vals_a);
            d.sums = at<uint32_t>(ws, L.sums);
            d.len = L.n;
            d.per256 = 1;
            d.nb = (L.n + 1023) / 1024;
            batch_add(B, d, (uint32_t)d.nb);
        }
        const uint32_t grid = B.blk0[B.nv];
        if (grid > 0) hipLaunchKernelGGL(k_scan_reduce, dim3(grid), dim3(256), 0, st, B);
    } else {
        Batch<ScanDesc> B;
        for (int v = 0; v < nv; ++v) {
            const Layout& L = *Ls[v];
            void* ws = wss[v];
            ScanDesc d{};
            d.in = at<uint32_t>(ws, L.cnt);
            d.gather = at<uint32_t>(ws, L.vals_a);
            d.out = at<uint32_t>(ws, L.offs);
            d.sums = at<uint32_t>(ws, L.sums);
            d.hdr = at<ViewHeader>(ws, L.hdr);
            d.tail_out = at<uint32_t>(ws, L.offs) + L.n;
            d.len = L.n;
            d.capacity = L.capacity;
            d.nb = (L.n + kSortItems - 1) / kSortItems;
            batch_add(B, d, (uint32_t)d.nb);
        }
        const uint32_t grid = B.blk0[B.nv];
        if (grid > 0) hipLaunchKernelGGL(k_scan_reduce, dim3(grid), dim3(256), 0, st, B);
        hipLaunchKernelGGL(k_scan_top, dim3((unsigned)nv), dim3(256), 0, st, B);
        if (grid > 0) hipLaunchKernelGGL(k_scan_down, dim3(grid), dim3(256), 0, st, B);
    }
    // 3. emit (tile, id) pairs, packed into one word when tile and id bits
    //    fit in 32 (only the keys then move through the tile passes). Packed
    //    pairs start in pk_a and alternate with pk_b, the last pass writing
    //    the ids to pv_a; unpacked pairs start where an odd or even number
    //    of passes leaves the result in pk_a / pv_a.
    {
        Batch<EmitDesc> B;
        for (int v = 0; v < nv; ++v) {
            const Layout& L = *Ls[v];
            void* ws = wss[v];
            const bool packed = L.id_bits > 0;
            const bool start_b = !packed && (passes[0] & 1) == 1;
            EmitDesc d{};
            d.ids = at<uint32_t>(ws, L.vals_a);
            d.offs = short_form ? nullptr : at<uint32_t>(ws, L.offs);
            d.cnt = at<uint32_t>(ws, L.cnt);
            d.sums = at<uint32_t>(ws, L.sums);
            d.hdr = at<ViewHeader>(ws, L.hdr);
            d.nb256 = (int32_t)((L.n + 255) / 256);
            d.ext = at<int4>(ws, L.ext);
            d.pk = at<uint32_t>(ws, start_b ? L.pk_b : L.pk_a);
            d.pv = at<uint32_t>(ws, start_b ? L.pv_b : L.pv_a);
            d.ranges = at<int2>(ws, L.ranges);
            d.n = (int32_t)L.n;
            d.tiles_x = L.tiles_x;
            d.capacity = (uint32_t)L.capacity;
            d.n_tiles = (int32_t)L.n_tiles;
            d.id_bits = L.id_bits;
            d.nblk = L.n > 0 ? (int32_t)((L.n + 255) / 256) : 1;
            batch_add(B, d, (uint32_t)d.nblk);
        }
        hipLaunchKernelGGL(k_emit, dim3(B.blk0[B.nv]), dim3(256), 0, st, B);
    }
    // 4. stable passes by tile index, per sub-batch
    for (int g = 0; g < 2; ++g) {
        const bool packed = g == 1;
        const int P = passes[g];
        const bool start_b = !packed && (P & 1) == 1;
        for (int pass = 0; pass < P; ++pass) {
            const bool from_b = ((pass & 1) == 0) == start_b;
            const bool final_pass = packed && pass == P - 1;
            Batch<RadixDesc> B;
            for (int v = 0; v < nv; ++v) {
                const Layout& L = *Ls[v];
                if ((L.id_bits > 0) != packed) continue;
                void* ws = wss[v];
                RadixDesc d{};
                d.kin = at<uint32_t>(ws, from_b ? L.pk_b : L.pk_a);
                d.vin = packed ? nullptr : at<uint32_t>(ws, from_b ? L.pv_b : L.pv_a);
                d.kout = at<uint32_t>(ws, final_pass ? L.pv_a : (from_b ? L.pk_a : L.pk_b));
                d.vout = packed ? nullptr : at<uint32_t>(ws, from_b ? L.pv_a : L.pv_b);
                d.n_dev = &at<ViewHeader>(ws, L.hdr)->n_pairs;
                d.n_host = 0u;
                d.shift = L.id_bits + pass * kRadixBits;
                d.table = at<uint32_t>(ws, L.table);
                d.totals = at<uint32_t>(ws, L.sums);
                d.ranges = reinterpret_cast<int*>(at<int2>(ws, L.ranges));
                d.nblk = (int32_t)L.nblk_p;
                d.id_bits = L.id_bits;
                batch_add(B, d, (uint32_t)L.nblk_p);
            }
            if (final_pass) e = radix_pass<kSortItems, false, true>(B, st);
            else if (packed) e = radix_pass<kSortItems, false>(B, st);
            else e = radix_pass<kSortItems, true>(B, st);
            if (e != hipSuccess) return e;
        }
    }
    // 5. per-tile [start, end), unless the last pass over packed pairs
    //    already wrote them
    {
        Batch<RangesDesc> B;
        for (int v = 0; v < nv; ++v) {
            const Layout& L = *Ls[v];
            const bool packed = L.id_bits > 0;
            if (L.capacity == 0 || (packed && passes[1] > 0)) continue;
            void* ws = wss[v];
            RangesDesc d{};
            d.pk = at<uint32_t>(ws, L.pk_a);
            d.hdr = at<ViewHeader>(ws, L.hdr);
            d.ranges = at<int2>(ws, L.ranges);
            d.ids = at<uint32_t>(ws, L.pv_a);
            d.n_tiles = (uint32_t)L.n_tiles;
            d.id_bits = L.id_bits;
            int64_t grid = (L.capacity + 255) / 256;
            d.nblk = (int32_t)(grid > 1024 ? 1024 : grid);
            batch_add(B, d, (uint32_t)d.nblk);
        }
        if (B.nv > 0) hipLaunchKernelGGL(k_ranges, dim3(B.blk0[B.nv]), dim3(256), 0, st, B);
    }
    {
        Batch<OrderDesc> B;
        for (int v = 0; v < nv; ++v) {
            const Layout& L = *Ls[v];
            void* ws = wss[v];
            OrderDesc d{};
            d.ranges = at<int2>(ws, L.ranges);
            d.hdr = at<ViewHeader>(ws, L.hdr);
            d.order = at<uint32_t>(ws, L.order);
            d.n_tiles = (int32_t)L.n_tiles;
            d.tiles_x = L.tiles_x;
            d.n_slots = (int32_t)L.n_slots;
            const StatusReq* r = status ? status[v] : nullptr;
            d.status = r ? reinterpret_cast<unsigned long long*>(r->status_dev) : nullptr;
            d.generation = r ? r->generation : 0;
            batch_add(B, d, 1u);
        }
        hipLaunchKernelGGL(k_tile_order, dim3((unsigned)nv), dim3(1024), 0, st, B);
    }
    return hipGetLastError();
}

hipError_t launch_bin_batch(const Layout* const* Ls, void* const* wss, int nv, hipStream_t st,
                            const StatusReq* const* status) {
    for (int c0 = 0; c0 < nv; c0 += kMaxBatch) {
        const int m = nv - c0 < kMaxBatch ? nv - c0 : kMaxBatch;
        const hipError_t e = bin_chunk(Ls + c0, wss + c0, status ? status + c0 : nullptr, m, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_bin(const Layout& L, void* ws, hipStream_t st, const StatusReq* status) {
    const Layout* Lp = &L;
    return launch_bin_batch(&Lp, &ws, 1, st, &status);
}

}  // namespace gs3
