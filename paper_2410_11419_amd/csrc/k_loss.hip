// Training-step kernels around the adjoint (Sec. 4.4): the L1 image loss
// with its gradient, and gradient-set upkeep (clear, accumulate).
//
// The L1 term of Eq. 9 is a plain reduction over the image. Its value is
// formed in a fixed order: each workgroup sums one 8192-element chunk in
// float64 (a fixed per-lane order, then a fixed tree over the workgroup) and
// writes one partial sum; a single workgroup then adds the partial sums in
// chunk order. The same input therefore gives the same float64 sum on every
// run and for every caller of these kernels. Bound by HBM: 8 B read and (with
// the gradient) 4 B written per element.
#include <mutex>

#include "gs3_internal.h"

namespace gs3 {

constexpr int kL1Chunk = 8192;   // elements per partial sum (256 lanes x 32)

__device__ inline double block_sum_f64_256(double x, double* s_part) {
    // wave64 butterfly, then the four wave totals in wave order
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_part[w] = x;
    __syncthreads();
    const double t = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
    __syncthreads();
    return t;
}

// One workgroup per chunk: partial[c] = sum of |pred - target| over chunk c;
// the gradient of each element is written on the way.
__global__ __launch_bounds__(256) void k_l1_partial(const float* __restrict__ pred, const float* __restrict__ target,
                                                     int64_t count, float scale, float* __restrict__ grad,
                                                     double* __restrict__ partial) {
    __shared__ double s_part[4];
    const int64_t c0 = (int64_t)blockIdx.x * kL1Chunk;
    double acc = 0.0;
#pragma unroll 4
    for (int r = 0; r < kL1Chunk / 256; ++r) {
        const int64_t i = c0 + (int64_t)r * 256 + threadIdx.x;
        if (i < count) {
            const float d = pred[i] - target[i];
            acc += (double)fabsf(d);
            if (grad) grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
        }
    }
    const double t = block_sum_f64_256(acc, s_part);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Single workgroup: the partial sums in chunk order (lane i takes chunks
// i, i + 256, ... in turn, then the fixed tree of block_sum_f64_256).
__global__ __launch_bounds__(256) void k_l1_final(const double* __restrict__ partial, int64_t chunks, float scale,
                                                   float* __restrict__ loss) {
    __shared__ double s_part[4];
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < chunks; c += 256) acc += partial[c];
    const double t = block_sum_f64_256(acc, s_part);
    if (threadIdx.x == 0) *loss = (float)(t * (double)scale);
}

// ceil(count / kL1Chunk) for count >= 0, without overflow near INT64_MAX
int64_t l1_chunks(int64_t count) { return count / kL1Chunk + (count % kL1Chunk != 0 ? 1 : 0); }

hipError_t launch_l1_loss(const float* pred, const float* target, int64_t count, float scale, float* loss,
                          float* grad, double* partial, hipStream_t st) {
    const int64_t chunks = l1_chunks(count);
    if (chunks > 0)
        hipLaunchKernelGGL(k_l1_partial, dim3((unsigned)chunks), dim3(256), 0, st, pred, target, count, scale, grad,
                           partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(256), 0, st, partial, chunks, scale, loss);
    return hipGetLastError();
}

// g += src, four floats per lane where both are 16-byte aligned.
__global__ __launch_bounds__(256) void k_accumulate(float* __restrict__ dst, const float* __restrict__ src,
                                                     int64_t count, int vec) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    if (vec) {
        const int64_t n4 = count >> 2;
        float4* d4 = reinterpret_cast<float4*>(dst);
        const float4* s4 = reinterpret_cast<const float4*>(src);
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
            float4 a = d4[i];
            const float4 b = s4[i];
            a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
            d4[i] = a;
        }
        for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) dst[i] += src[i];
    } else {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) dst[i] += src[i];
    }
}

hipError_t launch_accumulate(float* dst, const float* src, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const bool vec = ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0;
    int64_t grid = ((vec ? count / 4 : count) + 255) / 256;
    if (grid < 1) grid = 1;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)grid), dim3(256), 0, st, dst, src, count, vec ? 1 : 0);
    return hipGetLastError();
}

// dst += w * src (the weighted sum of an environment light's renders).
__global__ __launch_bounds__(256) void k_accumulate_scaled(float* __restrict__ dst, const float* __restrict__ src,
                                                            float w, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) dst[i] = fmaf(w, src[i], dst[i]);
}

hipError_t launch_accumulate_scaled(float* dst, const float* src, float w, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t grid = (count + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_accumulate_scaled, dim3((unsigned)grid), dim3(256), 0, st, dst, src, w, count);
    return hipGetLastError();
}

// ------------------------------------------------ no-allocation variant
//
// gs3_l1_loss_noalloc keeps its partial sums in this file-scope array
// instead of a caller workspace. Each device the library runs on holds its
// own copy until the process ends. Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): its device
// address is looked up once per device with hipGetSymbolAddress and kept.
constexpr int64_t kL1NoAllocChunks = 4096;   // 32 KiB: up to 4096 * 8192 = 33,554,432 elements
static __device__ __align__(256) double scratch[kL1NoAllocChunks];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there).
static hipError_t scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace gs3

using namespace gs3;

extern "C" int gs3_l1_loss_noalloc(const float* pred, const float* target, int64_t count, float scale, float* loss,
                                   float* dL_dpred, gs3_stream_t stream) {
    if (count < 0) return set_error(GS3_INVALID_ARG, "count < 0");
    if (!loss || (count > 0 && (!pred || !target))) return set_error(GS3_INVALID_ARG, "pred / target / loss is NULL");
    if (l1_chunks(count) > kL1NoAllocChunks)
        return set_error(GS3_INVALID_ARG,
                         "count exceeds the no-allocation scratch (at most 33554432 elements; use gs3_l1_loss)");
    double* partial = nullptr;
    hipError_t e = scratch_address(&partial);
    if (e == hipSuccess) e = launch_l1_loss(pred, target, count, scale, loss, dL_dpred, partial, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(GS3_HIP_ERROR, hipGetErrorString(e));
    return GS3_OK;
}
