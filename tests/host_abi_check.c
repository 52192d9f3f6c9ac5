/*
 * Host-layer check of libgs3 under AddressSanitizer and UndefinedBehavior-
 * Sanitizer: every call below is decided on the host (argument checks, size
 * queries, status-block decoding, refusals before anything is enqueued), so
 * it runs without a GPU. The library's host code is built with the
 * sanitizers (the device code is not); any memory error or undefined
 * behaviour in it aborts this program with the sanitizer's report.
 * Device pointers passed here are never dereferenced: each call fails its
 * checks first. Exit status 0 and the line "host ABI checks passed" mean
 * every expectation held.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gs3.h"

static int failures = 0;

#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "%s:%d: expectation failed: %s (last error: %s)\n", \
                    __FILE__, __LINE__, #cond, gs3_last_error());           \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static void* fake(uintptr_t a) { return (void*)a; }

static gs3_view pinhole(int w, int h) {
    gs3_view v;
    memset(&v, 0, sizeof v);
    v.eye[2] = 4.0;
    v.width = w;
    v.height = h;
    v.fov = 0.7;
    v.projection = GS3_PERSPECTIVE;
    return v;
}

static gs3_scene scene_of(int64_t n, int k, int appearance) {
    gs3_scene s;
    memset(&s, 0, sizeof s);
    s.n = n;
    s.k = k;
    s.appearance = appearance;
    s.mean = s.log_scale = s.rot = s.opacity_logit = fake(4096);
    s.shade_rot = s.albedo = s.feat = fake(4096);
    return s;
}

static void check_constants_and_strings(void) {
    gs3_consts k;
    gs3_consts_default(&k);
    EXPECT(k.cutoff > 4.49f && k.cutoff < 4.51f);
    EXPECT(k.shadow_bias > 0.0149f && k.shadow_bias < 0.0151f);
    const int codes[] = {0, -1, -2, -3, -4, -5, -6, 1, 99, -2147483647 - 1, 2147483647};
    for (size_t i = 0; i < sizeof codes / sizeof codes[0]; ++i) {
        const char* s = gs3_status_string(codes[i]);
        EXPECT(s != NULL && strlen(s) > 0);
    }
    EXPECT(strcmp(gs3_status_string(-3), "GS3_PAIR_CAPACITY_EXCEEDED") == 0);
    EXPECT(gs3_last_error() != NULL);
}

static void check_size_queries(void) {
    size_t a = 0, b = 0;
    EXPECT(gs3_view_workspace_size(1000, 128, 96, 50000, &a) == GS3_OK && a > 50000 * 16);
    EXPECT(gs3_view_workspace_size(1000, 128, 96, 100000, &b) == GS3_OK && b > a);
    EXPECT(gs3_view_workspace_size(0, 1, 1, 0, &a) == GS3_OK);
    /* the largest accepted sizes must not wrap the byte count */
    EXPECT(gs3_view_workspace_size(2147483647LL, 16384, 16384, 2147483647LL, &a) == GS3_OK);
    EXPECT(a > (size_t)2147483647LL * 16);
    EXPECT(gs3_view_workspace_size(-1, 128, 96, 10, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_view_workspace_size(10, 0, 96, 10, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_view_workspace_size(10, 128, -5, 10, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_view_workspace_size(10, 128, 96, -1, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_view_workspace_size(10, 128, 96, 10, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_view_workspace_size(10, 1 << 30, 1 << 30, 10, &a) != GS3_OK);
    EXPECT(gs3_view_workspace_size(INT64_MAX, 128, 96, INT64_MAX, &a) != GS3_OK);

    EXPECT(gs3_backward_workspace_size_for(GS3_APPEARANCE_LOBES, 300000, 1024, 1024, &a) == GS3_OK);
    EXPECT(gs3_backward_workspace_size_for(GS3_APPEARANCE_BASIS, 300000, 1024, 1024, &b) == GS3_OK && b > a);
    EXPECT(gs3_backward_workspace_size(300000, 1024, 1024, &b) == GS3_OK && b == a);
    EXPECT(gs3_backward_workspace_size_for(GS3_APPEARANCE_BASIS, 2147483647LL, 16384, 16384, &a) == GS3_OK);
    EXPECT(a > (size_t)2147483647LL * 64);
    EXPECT(gs3_backward_workspace_size_for(5, 10, 8, 8, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_backward_workspace_size_for(GS3_APPEARANCE_LOBES, -1, 8, 8, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_backward_workspace_size_for(GS3_APPEARANCE_LOBES, 10, 0, 8, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_backward_workspace_size_for(GS3_APPEARANCE_LOBES, INT64_MAX, 8, 8, &a) != GS3_OK);

    EXPECT(gs3_l1_loss_workspace_size(0, &a) == GS3_OK && a >= 8);
    EXPECT(gs3_l1_loss_workspace_size(3 * 800 * 800, &a) == GS3_OK && a % 256 == 0);
    EXPECT(gs3_l1_loss_workspace_size(-1, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_l1_loss_workspace_size(INT64_MAX, &a) != GS3_OK || a > 0);
    EXPECT(gs3_dssim_loss_workspace_size(3, 800, 800, &a) == GS3_OK && a > 3 * 800 * 800 * 4);
    EXPECT(gs3_dssim_loss_workspace_size(3, 16384, 16384, &a) == GS3_OK);
    EXPECT(gs3_dssim_loss_workspace_size(0, 8, 8, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_dssim_loss_workspace_size(65, 8, 8, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_dssim_loss_workspace_size(3, 16385, 8, &a) == GS3_INVALID_ARG);
    EXPECT(gs3_dssim_loss_workspace_size(3, 8, -8, &a) == GS3_INVALID_ARG);
}

static void check_status_block(void) {
    size_t size = 0;
    EXPECT(gs3_view_workspace_size(100, 64, 64, 1000, &size) == GS3_OK);
    gs3_consts k;
    gs3_consts_default(&k);
    int64_t blk[2];
    blk[0] = 3;
    blk[1] = (int64_t)(((uint64_t)(3 & 0xFFFFFF) << 40) | (1ull << 39) | 12345ull);
    gs3_viewbuf vb = {fake(256), size, 100, 64, 64, 1000, blk};
    int32_t st = 0;
    int64_t req = 0;
    EXPECT(gs3_view_poll(&vb, &st, &req) == GS3_OK && req == 12345);
    EXPECT(gs3_shadow_splat(&k, &vb, fake(512), fake(512), NULL) == GS3_PAIR_CAPACITY_EXCEEDED);
    EXPECT(strstr(gs3_last_error(), "12345") != NULL);
    EXPECT(gs3_shadow_den(&k, &vb, fake(512), NULL) == GS3_PAIR_CAPACITY_EXCEEDED);
    EXPECT(gs3_shadow_num(&k, &vb, fake(512), NULL) == GS3_PAIR_CAPACITY_EXCEEDED);
    EXPECT(gs3_shadow_resolve(&vb, fake(512), fake(512), NULL) == GS3_PAIR_CAPACITY_EXCEEDED);
    EXPECT(gs3_view_lists(&vb, NULL, NULL, NULL, NULL, NULL) == GS3_PAIR_CAPACITY_EXCEEDED);
    EXPECT(gs3_view_count_hits(&k, &vb, 0, fake(1024), NULL) == GS3_PAIR_CAPACITY_EXCEEDED);
    gs3_scene sc = scene_of(100, 0, GS3_APPEARANCE_LOBES);
    gs3_view cam = pinhole(64, 64), light = pinhole(64, 64);
    light.eye[1] = 4.0;
    light.eye[2] = 0.0;
    gs3_images im = {fake(512), fake(512), fake(512), fake(512), fake(512), fake(512), fake(512)};
    EXPECT(gs3_render(&sc, &cam, &light, &k, fake(512), NULL, NULL, &vb, &im, NULL) ==
           GS3_PAIR_CAPACITY_EXCEEDED);
    blk[0] = 4;   /* a newer binning still pending */
    EXPECT(gs3_view_poll(&vb, &st, &req) == GS3_OK && req == -1);
    int64_t fresh[2] = {0, 0};
    vb.status = fresh;
    EXPECT(gs3_view_poll(&vb, &st, &req) == GS3_OK);
    vb.status = NULL;
    EXPECT(gs3_view_poll(&vb, &st, &req) == GS3_INVALID_ARG);
    EXPECT(gs3_view_poll(NULL, &st, &req) == GS3_INVALID_ARG);
}

static void check_argument_refusals(void) {
    gs3_consts k;
    gs3_consts_default(&k);
    size_t size = 0;
    EXPECT(gs3_view_workspace_size(10, 64, 64, 1000, &size) == GS3_OK);
    /* views: orthographic without a width, an unknown projection */
    gs3_viewbuf vb = {fake(256), size, 10, 64, 64, 1000, NULL};
    gs3_scene sc = scene_of(10, 0, GS3_APPEARANCE_LOBES);
    gs3_view v = pinhole(64, 64);
    v.projection = GS3_ORTHOGRAPHIC;
    v.ortho_width = 0.0;
    EXPECT(gs3_project(&sc, &v, &k, 1, &vb, NULL) == GS3_INVALID_ARG);
    v.projection = 7;
    EXPECT(gs3_project(&sc, &v, &k, 1, &vb, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_project(NULL, &v, &k, 1, &vb, NULL) == GS3_INVALID_ARG);
    /* a too small or misaligned workspace */
    gs3_viewbuf small = {fake(256), 1000, 100, 64, 64, 1000, NULL};
    int64_t n = 0;
    EXPECT(gs3_view_pair_count(&small, &n, NULL) == GS3_WORKSPACE_TOO_SMALL);
    gs3_viewbuf odd = {fake(257), (size_t)1 << 30, 100, 64, 64, 1000, NULL};
    EXPECT(gs3_view_pair_count(&odd, &n, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_view_pair_count(NULL, NULL, NULL) == GS3_INVALID_ARG);
    /* view arrays: none, NULL, two views sharing one workspace */
    gs3_viewbuf big = {fake(256), (size_t)1 << 30, 100, 64, 64, 1000, NULL};
    gs3_viewbuf two[2] = {big, big};
    float* arr[2] = {fake(512), fake(1024)};
    EXPECT(gs3_shadow_splat_views(&k, two, 0, arr, arr, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_shadow_splat_views(&k, NULL, 1, arr, arr, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_shadow_splat_views(&k, two, 2, arr, arr, NULL) == GS3_INVALID_ARG);
    const float* const* carr = (const float* const*)arr;
    gs3_view views[2] = {pinhole(64, 64), pinhole(32, 64)};
    int32_t modes[2] = {0, 1};
    gs3_viewbuf pre[2] = {{fake(1 << 20), size, 10, 64, 64, 1000, NULL},
                          {fake((uintptr_t)1 << 30), size, 10, 64, 64, 1000, NULL}};
    EXPECT(gs3_preprocess_views(&sc, views, modes, 0, &k, pre, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_preprocess_views(&sc, views, modes, 2, &k, pre, NULL) == GS3_INVALID_ARG);
    modes[1] = 5;
    views[1] = pinhole(64, 64);
    EXPECT(gs3_preprocess_views(&sc, views, modes, 2, &k, pre, NULL) == GS3_INVALID_ARG);
    /* appearance models */
    gs3_scene bad = scene_of(100, 2, 7);
    gs3_view cams[1] = {pinhole(64, 64)};
    gs3_images ims[1];
    memset(ims, 0, sizeof ims);
    gs3_viewbuf vbs[1] = {big};
    EXPECT(gs3_render_views(&bad, cams, cams, 1, &k, carr, NULL, NULL, vbs, ims, NULL) == GS3_INVALID_ARG);
    bad.appearance = GS3_APPEARANCE_BASIS;   /* without the basis pointers */
    EXPECT(gs3_render_views(&bad, cams, cams, 1, &k, carr, NULL, NULL, vbs, ims, NULL) == GS3_INVALID_ARG);
    bad.appearance = GS3_APPEARANCE_LOBES;
    bad.k = 17;
    EXPECT(gs3_render_views(&bad, cams, cams, 1, &k, carr, NULL, NULL, vbs, ims, NULL) == GS3_INVALID_ARG);
    /* losses, optimiser, gradient sets, image sums */
    void* p = fake(256);
    EXPECT(gs3_l1_loss(NULL, p, 10, 1.0f, p, NULL, p, 1 << 20, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_l1_loss(p, p, -1, 1.0f, p, NULL, p, 1 << 20, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_l1_loss(p, p, 10, 1.0f, p, NULL, fake(260), 1 << 20, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_l1_loss(p, p, 1 << 24, 1.0f, p, NULL, p, 8, NULL) == GS3_WORKSPACE_TOO_SMALL);
    EXPECT(gs3_l1_loss_noalloc(p, p, -1, 1.0f, p, NULL, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_l1_loss_noalloc(p, p, 10, 1.0f, NULL, NULL, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_l1_loss_noalloc(p, p, (int64_t)1 << 40, 1.0f, p, NULL, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_dssim_loss(NULL, p, 3, 8, 8, 1.0f, p, NULL, 0, p, 1 << 20, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_dssim_loss(p, p, 3, 8, 8, 1.0f, p, NULL, 0, p, 8, NULL) == GS3_WORKSPACE_TOO_SMALL);
    EXPECT(gs3_adam_step(NULL, p, p, p, 10, 1, 1e-3f, 0.9f, 0.999f, 1e-8f, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_adam_step(p, p, p, p, 10, 0, 1e-3f, 0.9f, 0.999f, 1e-8f, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_adam_step(p, p, p, p, 10, 1, 1e-3f, 1.0f, 0.999f, 1e-8f, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_grads_clear(NULL, 5, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_grads_clear(p, -1, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_grads_accumulate(p, NULL, 5, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_image_accumulate(p, NULL, 1.0f, 5, NULL) == GS3_INVALID_ARG);
    EXPECT(gs3_image_accumulate(p, p, 1.0f, -5, NULL) == GS3_INVALID_ARG);
}

int main(void) {
    check_constants_and_strings();
    check_size_queries();
    check_status_block();
    check_argument_refusals();
    if (failures) {
        fprintf(stderr, "%d host ABI expectations failed\n", failures);
        return 1;
    }
    printf("host ABI checks passed\n");
    return 0;
}
