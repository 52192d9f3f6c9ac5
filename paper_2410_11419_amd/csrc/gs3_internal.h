// Internal declarations of libgs3: workspace layout, splat record format,
// kernel launchers. Not part of the public ABI (see include/gs3.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/gs3.h"

namespace gs3 {

constexpr int kTile = 16;          // tile edge in pixels
constexpr int kBlock = 256;        // threads per tile workgroup (4 wave64)
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortItems = 4096;   // items per radix (pair sort) / scan workgroup
constexpr int kSortItemsN = 1024;  // items per radix workgroup of the depth sort of the N splats
constexpr int64_t kEmitScanMaxN = 1 << 19;  // views of at most this many splats form pair offsets inside the emission
constexpr int kFeat = 16;          // per-Gaussian MLP feature size
constexpr int kHidden = 64;        // MLP hidden width
constexpr int kMaxLobes = 16;
constexpr int kMaxBatch = 8;       // views per batched launch (longer batches run in chunks)
// The shadow numerator is summed as unsigned 64-bit fixed point with 36
// fraction bits: integer addition does not depend on the order of the
// atomics, so num (and T) are the same bits on every run. A term is
// rounded to 2^-36; num_j >= 0 is below 2^28 for any image this library
// takes (each term is at most alpha_max < 1, one per pixel of at most
// 16384^2).
constexpr float kNumScale = 68719476736.0f;   // 2^36
// Tile-walking kernels take their tiles from a launch order of n_slots
// entries: slot 8 k + x runs on XCD x (workgroups are dealt to the XCDs
// round-robin), and kNoTile marks an empty slot.
constexpr uint32_t kNoTile = 0xFFFFFFFFu;
constexpr int kGroupTiles = 8;     // tiles per side of a group kept on one XCD
constexpr int kMaxGroups = 1024;   // above this many groups the order is LPT alone

// Device-side counters at the head of every view workspace.
struct ViewHeader {
    unsigned long long required_pairs;  // unclamped pair total of the last binning
    uint32_t n_pairs;                   // min(required, capacity)
    uint32_t overflow;                  // 1 if required > capacity
    uint32_t pad[60];
};

// Projected splat record, two float4 per Gaussian:
//   rec0 = {floor(u), floor(v), u - floor(u), v - floor(v)}  (pixel centre,
//          split so a tile-relative centre can be formed without rounding)
//   rec1 = {a, b, c, opacity}  conic (inverse 2D covariance) and sigmoid opacity
//   rec2 = {thr, hx, hy, p}    hit threshold of q (float32, the one every kernel
//                              tests), padded bounding-box half-widths of the hit
//                              ellipse and the power threshold p (p <= 0: no hits)
// Culled Gaussians have ext.z = ext.w = -1 and zero records.
struct Layout {
    int64_t n = 0;
    int32_t width = 0, height = 0, tiles_x = 0, tiles_y = 0;
    int64_t n_tiles = 0;
    int64_t n_slots = 0;   // entries of the tile launch order (>= n_tiles)
    int64_t capacity = 0;
    int64_t nblk_n = 0, nblk_p = 0, table_len = 0, scan_sums = 0;
    int32_t id_bits = 0;   // > 0: pairs are packed (tile << id_bits) | id while sorting
    size_t hdr = 0, rec0 = 0, rec1 = 0, rec2 = 0, depth = 0, ext = 0, drec = 0, cnt = 0, col0 = 0, col1 = 0;
    size_t num = 0;   // shadow numerator accumulator [n], u64 fixed point (kNumScale): cleared by the projection and by the resolve
    size_t keys_a = 0, vals_a = 0, keys_b = 0, vals_b = 0, offs = 0;
    size_t pk_a = 0, pv_a = 0, pk_b = 0, pv_b = 0, table = 0, sums = 0, ranges = 0, order = 0;
    size_t total = 0;
};

// Records `msg` as the calling thread's last error (gs3_last_error) and
// returns `status`.
int set_error(int status, const char* msg);

// Compute the workspace layout; returns false on invalid sizes.
bool make_layout(int64_t n, int32_t width, int32_t height, int64_t capacity, Layout* L);

template <typename T>
inline T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }
template <typename T>
inline const T* at(const void* base, size_t off) {
    return reinterpret_cast<const T*>(static_cast<const char*>(base) + off);
}

// View parameters for the projection kernel (all derived on the host in double).
struct ViewParams {
    double R[9];        // world -> camera rotation, row-major (rows: right, down, forward)
    double eye[3];
    double focal;       // pixels
    double cx, cy;      // principal point
    double lim_x, lim_y;  // clamp of x/z, y/z in the Jacobian
    int32_t width, height, tiles_x, tiles_y;
    int32_t depth_mode;
    int32_t ortho;      // 1: orthographic (x_pixel = scale x_view + cx), 0: pinhole
    double scale;       // orthographic: pixels per world unit
};

struct SceneDev {
    const float* mean;
    const float* log_scale;
    const float* rot;
    const float* opacity_logit;
    const float* shade_rot;
    const float* albedo;
    const float* lobe_axis;
    const float* lobe_log_sharp;
    const float* lobe_amp;
    const float* feat;
    int32_t n;
    int32_t k;
    int32_t appearance;          // GS3_APPEARANCE_LOBES / GS3_APPEARANCE_BASIS
    const float* spec_albedo;    // basis appearance (Sec. 4.1 shared basis)
    const float* basis_weight;
    const float* latent;
    const float* basis_rot;
    const float* basis_log_sigma;
};

// Launchers (return hipError_t of the launch).
hipError_t launch_project(const SceneDev& sc, const ViewParams& vp, const gs3_consts& k,
                          const Layout& L, void* ws, hipStream_t st);
hipError_t launch_extent_keys(const int32_t* ix, const int32_t* iy, const int32_t* rx,
                              const int32_t* ry, const float* depth, const Layout& L,
                              void* ws, hipStream_t st);
// A binning outcome to report into a host-pinned status block.
struct StatusReq {
    long long generation;
    int64_t* status_dev;   // device address of the block's word 1
};
// status (optional): where to report the outcome (the last kernel of the
// binning writes it).
hipError_t launch_bin(const Layout& L, void* ws, hipStream_t st, const StatusReq* status = nullptr);
// One launch sequence bins all nv views (any nv; chunks of kMaxBatch);
// status (optional) holds one entry per view, nullptr for none.
hipError_t launch_bin_batch(const Layout* const* Ls, void* const* wss, int nv, hipStream_t st,
                            const StatusReq* const* status = nullptr);
// Projection of one scene into nv views (ViewParams vps[v], workspace
// wss[v] with layout Ls[v]); chunks of kMaxBatch views per launch.
hipError_t launch_project_batch(const SceneDev& sc, const ViewParams* vps, const gs3_consts& k,
                                const Layout* const* Ls, void* const* wss, int nv, hipStream_t st);
hipError_t launch_shadow(const gs3_consts& k, const Layout& L, void* ws,
                         float* num_den, float* T, hipStream_t st);
hipError_t launch_shadow_den(const gs3_consts& k, const Layout& L, void* ws, float* num_den, hipStream_t st);
hipError_t launch_shadow_num(const gs3_consts& k, const Layout& L, void* ws, float* num_den, hipStream_t st);
hipError_t launch_shadow_resolve(const Layout& L, void* ws, float* num_den, float* T, hipStream_t st);
struct ShadeParams {
    float light[3];     // point light position, or (light_dir) unit direction toward the light
    float eye[3];
    int32_t use_phi, use_psi;
    int32_t light_dir;  // 1: directional light (w_i = light for every Gaussian)
};
// Per-view inputs and outputs of the per-Gaussian shading kernels (one
// entry per view of a batched launch; blockIdx.y selects it).
struct ShadeView {
    float light[3];     // point light position, or (light_dir) unit direction toward the light
    float eye[3];
    int32_t light_dir;
    const float* T;     // shadow values (Phi's input)
    float4* col0;       // splat colours in the camera view's workspace
    float4* col1;
    float* colour;      // [8][n] caller copy
};
// parts: 1 = shading c and Psi's r, 2 = Phi's T', 3 = both
hipError_t launch_shade_mlp(const SceneDev& sc, const ShadeParams& sp, const float* T,
                            const gs3_mlp* phi, const gs3_mlp* psi, const Layout& L,
                            void* ws, float* colour_out, int parts, hipStream_t st);
// The same for nv views of one scene (any nv; chunks of kMaxBatch views per
// launch): view v has shading parameters sps[v], shadow values T[v] and the
// camera workspace wss[v] with layout Ls[v].
hipError_t launch_shade_mlp_batch(const SceneDev& sc, const ShadeParams* sps, const float* const* T,
                                  const gs3_mlp* phi, const gs3_mlp* psi, const Layout* const* Ls,
                                  void* const* wss, float* const* colour, int parts, int nv, hipStream_t st);
hipError_t launch_basis_shade_batch(const SceneDev& sc, const ShadeParams* sps, const float* const* T,
                                    const gs3_mlp* phi, const gs3_mlp* psi, const Layout* const* Ls,
                                    void* const* wss, float* const* colour, int parts, int nv, hipStream_t st);
hipError_t launch_render(const gs3_consts& k, const Layout& L, const void* ws,
                         const gs3_images& out, hipStream_t st);
hipError_t launch_render_batch(const gs3_consts& k, const Layout* const* Ls, void* const* wss,
                               const gs3_images* outs, int nv, hipStream_t st);
hipError_t launch_shadow_den_batch(const gs3_consts& k, const Layout* const* Ls, void* const* wss,
                                   float* const* num_den, int nv, hipStream_t st);
hipError_t launch_shadow_num_batch(const gs3_consts& k, const Layout* const* Ls, void* const* wss,
                                   float* const* num_den, int nv, hipStream_t st);
hipError_t launch_shadow_resolve_batch(const Layout* const* Ls, void* const* wss, float* const* num_den,
                                       float* const* T, int nv, hipStream_t st);
// Device pointers of the scene gradients (+=), mirror of SceneDev.
struct GradDev {
    float* mean;
    float* log_scale;
    float* rot;
    float* opacity_logit;
    float* shade_rot;
    float* albedo;
    float* lobe_axis;
    float* lobe_log_sharp;
    float* lobe_amp;
    float* feat;
    float* spec_albedo;
    float* basis_weight;
    float* latent;
    float* basis_rot;
    float* basis_log_sigma;
};
int mlp_scratch_rows();
int wgrad_total_params(bool phi, bool psi);
constexpr int kWgChunkHost = 1024;   // Gaussians per weight-gradient partial sum
hipError_t launch_render_bwd(const gs3_consts& k, const Layout& L, const void* ws, const gs3_images& fwd,
                             const float* dF, float* gsplat, float* gcol, hipStream_t st);
hipError_t launch_shadow_bwd(const gs3_consts& k, const Layout& L, const void* ws, const float* T,
                             const float* num_den, const float* dT, float* dnum, float* gray, float* gsplat,
                             hipStream_t st);
hipError_t launch_shade_bwd(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                            const gs3_mlp* psi, const float* gcol, float* dT, const GradDev& g, float* rows,
                            float* partial, const gs3_grads* gr, hipStream_t st);
// Shared-basis appearance (Sec. 4.1) with the paper's MLP form (Sec. 4.2,
// 4.3): forward shading + Psi, forward Phi, and the adjoint of both.
constexpr int kLatent = 6;
constexpr int kPhiBasisIn = 61, kPsiBasisIn = 60;     // [T, PE(w_i), PE(mu), l] / [PE(w_o), PE(mu), l]
constexpr int kPhiBasisHidden = 32, kPsiBasisHidden = 128;
constexpr float kLeakySlope = 0.01f;
hipError_t launch_basis_shade(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                              const gs3_mlp* psi, const Layout& L, void* ws, float* colour_out, int parts,
                              hipStream_t st);
int basis_scratch_rows();
int basis_wgrad_total_params();
int basis_partial_floats(int k);
hipError_t launch_basis_shade_bwd(const SceneDev& sc, const ShadeParams& sp, const float* T, const gs3_mlp* phi,
                                  const gs3_mlp* psi, const float* gcol, float* dT, const GradDev& g, float* rows,
                                  float* partial, const gs3_grads* gr, hipStream_t st);
// Weight gradients dW += sum_g dz[:, g] in[:, g]^T (and db += sum_g dz)
// over problems of at most 128 x 128 (scratch rows [row][n]); dW has row
// stride ldw, db may be NULL.
struct WgSpec {
    int dz_row, in_row, O, J, ldw;
    float* dW;
    float* db;
};
hipError_t launch_wgrad(const WgSpec* specs, int count, const float* rows, int n, float* partial, hipStream_t st);
int wgrad_partial_floats(const WgSpec* specs, int count);
hipError_t launch_project_bwd(const SceneDev& sc, const ViewParams& cam, const ViewParams& light,
                              const gs3_consts& k, const float* gcam, const float* glight, const GradDev& g,
                              hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st);
int64_t l1_chunks(int64_t count);
hipError_t launch_l1_loss(const float* pred, const float* target, int64_t count, float scale, float* loss,
                          float* grad, double* partial, hipStream_t st);
hipError_t launch_accumulate(float* dst, const float* src, int64_t count, hipStream_t st);
hipError_t launch_accumulate_scaled(float* dst, const float* src, float w, int64_t count, hipStream_t st);
// D-SSIM workspace: the adjoint maps a, b, c and the per-tile partial sums.
struct SsimLayout {
    int tiles_x = 0, tiles_y = 0;
    size_t amap = 0, bmap = 0, cmap = 0, partial = 0, total = 0;
};
SsimLayout ssim_layout(int channels, int height, int width);
hipError_t launch_dssim(const float* pred, const float* target, int channels, int height, int width, float scale,
                        float* loss, float* grad, int accumulate, void* ws, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, int step, float lr, float b1,
                       float b2, float eps, hipStream_t st);
hipError_t launch_export_lists(const Layout& L, const void* ws, int32_t* start, int32_t* end, int32_t* ids,
                               uint64_t* keys, hipStream_t st);
hipError_t launch_count_hits(const gs3_consts& k, const Layout& L, const void* ws, int stop_early,
                             unsigned long long* out, hipStream_t st);
hipError_t launch_export_splats(const Layout& L, const void* ws, float* mean2d, float* conic, float* opacity,
                                float* depth, int32_t* extent, hipStream_t st);

}  // namespace gs3
