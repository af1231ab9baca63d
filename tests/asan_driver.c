/* Drives the library's host code, built with host-only AddressSanitizer,
 * through every entry point's validation paths, the plan and batch
 * lifecycles and the status strings, without a GPU: every call must return
 * cleanly (an error status where the arguments or the missing device call
 * for one), with no invalid access and no leak. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include "psfs.h"

static int calls = 0;
/* every call's status is allowed; the sanitizer is the check */
#define CALL(x) do { int rc_ = (int)(x); (void)rc_; ++calls; const char *m = psfs_last_error(); (void)strlen(m); } while (0)

int main(void)
{
    for (int s = -10; s <= 2; ++s) (void)strlen(psfs_status_str(s));
    psfs_plan *p = NULL;
    CALL(psfs_plan_create(NULL));
    CALL(psfs_plan_create(&p));
    psfs_camera cams[17];
    memset(cams, 0, sizeof(cams));
    for (int k = 0; k < 17; ++k) { cams[k].width = 8 + k; cams[k].height = 6 + k; cams[k].P[0] = 1.f; cams[k].P[5] = 1.f; cams[k].P[10] = 1.f; cams[k].P[11] = 2.f; }
    psfs_grid g = {5, 6, 7, {0.f, 0.f, 0.f}, 0.1f}, bad = {-1, 2, 3, {0.f, 0.f, 0.f}, 0.1f};
    psfs_params prm;
    psfs_default_params(&prm);
    float fake4[4];
    void *fk = (void *)(uintptr_t)0x100000;
    const uint8_t *imgs[16]; const float *maps[16]; float *gm[16];
    for (int k = 0; k < 16; ++k) { imgs[k] = (const uint8_t *)fk; maps[k] = (const float *)fk; gm[k] = (float *)fk; }
    /* before cameras */
    CALL(psfs_lmap_floats(p)); CALL(psfs_lmap_offset(p, 0)); CALL(psfs_workspace_bytes(p));
    CALL(psfs_likelihood(p, imgs, (float *)fk, NULL));
    CALL(psfs_particle_weights(p, (const float *)fk, 4, maps, maps, 1.0, (double *)fk, NULL, NULL, NULL));
    CALL(psfs_set_cameras(p, 17, cams));
    CALL(psfs_set_cameras(p, -1, cams));
    CALL(psfs_set_cameras(p, 2, NULL));
    cams[3].P[2] = NAN;
    CALL(psfs_set_cameras(p, 4, cams));
    cams[3].P[2] = 0.f;
    cams[2].width = 0;
    CALL(psfs_set_cameras(p, 4, cams));
    cams[2].width = 10;
    CALL(psfs_set_cameras(p, 16, cams));
    CALL(psfs_set_grid(p, &bad)); CALL(psfs_set_grid(p, NULL)); CALL(psfs_set_grid(p, &g));
    prm.prior = 2.f; CALL(psfs_set_params(p, &prm)); psfs_default_params(&prm); prm.sampling = 7; CALL(psfs_set_params(p, &prm));
    psfs_default_params(&prm); CALL(psfs_set_params(p, &prm));
    CALL(psfs_set_background(p, 16, (const float *)fk, (const float *)fk));
    CALL(psfs_set_background(p, 0, NULL, (const float *)fk));
    CALL(psfs_set_background(p, 0, (const float *)((char *)fk + 4), (const float *)fk));
    for (int k = 0; k < 16; ++k) CALL(psfs_set_background(p, k, (const float *)fk, (const float *)fk));
    CALL(psfs_set_input_check(NULL, NULL));
    CALL(psfs_set_input_check(p, (uint32_t *)((char *)fk + 2)));
    CALL(psfs_input_status(NULL));
    CALL(psfs_input_status(p));
    for (int k = -1; k <= 16; ++k) CALL(psfs_lmap_offset(p, k));
    CALL(psfs_lmap_floats(p)); CALL(psfs_workspace_bytes(p)); CALL(psfs_diff_workspace_bytes(p));
    CALL(psfs_surface_workspace_bytes(p)); CALL(psfs_colour_workspace_bytes(p));
    CALL(psfs_likelihood(p, NULL, (float *)fk, NULL));
    CALL(psfs_fuse(p, NULL, NULL, NULL, NULL));
    CALL(psfs_fuse(p, (const float *)fk, (float *)((char *)fk + 4), NULL, NULL));
    CALL(psfs_reconstruct(p, imgs, (float *)fk, NULL, fk, 16, NULL));
    CALL(psfs_reconstruct_static(p, imgs, (float *)fk, NULL, NULL));
    CALL(psfs_reconstruct_static(NULL, imgs, (float *)fk, NULL, NULL));
    CALL(psfs_tune(p, imgs, fk, 16, NULL, 0, NULL));
    CALL(psfs_tune(NULL, imgs, fk, 16, NULL, 1, NULL));
    CALL((int)psfs_tune_workspace_bytes(p));
    CALL(psfs_get_tile(p));
    CALL(psfs_pipeline_step(p, imgs, (float *)fk, (const float *)fk, (float *)fk, NULL, NULL));
    CALL(psfs_pipeline_step(p, NULL, NULL, NULL, NULL, (uint8_t *)fk, NULL));
    CALL(psfs_threshold(NULL, -3, 0.5f, NULL, NULL));
    CALL(psfs_surface(p, (const float *)fk, NULL, NULL, NULL, 0, NULL, NULL, 0, NULL));
    CALL(psfs_surface(p, (const float *)fk, NULL, (uint8_t *)fk, (int32_t *)fk, 10, (int64_t *)fk, fk, 1, NULL));
    CALL(psfs_colour(p, imgs, (const int32_t *)fk, -1, NULL, NULL, NULL, 0, NULL));
    CALL(psfs_colour(p, imgs, (const int32_t *)fk, 5, (float *)fk, (int32_t *)fk, fk, 8, NULL));
    CALL(psfs_foreground_model(p, imgs, NULL, NULL, (float *)fk, fk, 16384, NULL));
    CALL(psfs_set_foreground(p, (const float *)((char *)fk + 2)));
    CALL(psfs_set_foreground(p, NULL));
    const int32_t sub[6] = {0, 99, 0, 1, 0, 1};
    CALL(psfs_diff_forward(p, imgs, (const uint8_t *)fk, sub, (float *)fk, (float *)fk, fk, 16, NULL));
    CALL(psfs_diff_backward(p, imgs, (const uint8_t *)fk, NULL, (const float *)fk, (const float *)fk, gm, gm, (float *)fk, fk, 16, NULL));
    CALL(psfs_particle_weights(p, (const float *)fk, -1, maps, maps, 1.0, (double *)fk, NULL, NULL, NULL));
    CALL(psfs_particle_weights(p, (const float *)fk, 4, maps, maps, NAN, (double *)fk, (double *)fk, NULL, NULL));
    CALL(psfs_particle_weights(p, (const float *)((char *)fk + 8), 4, maps, maps, 1.0, (double *)fk, NULL, NULL, NULL));
    CALL(psfs_particle_weights(p, (const float *)fk, 4, NULL, maps, 1.0, (double *)fk, NULL, NULL, NULL));
    CALL(psfs_particle_weights(p, (const float *)fk, 4, maps, maps, 1.0, (double *)fk, NULL, NULL, NULL));
    CALL(psfs_particle_weights(p, NULL, 0, NULL, NULL, 1.0, NULL, NULL, NULL, NULL));
    CALL(psfs_set_cameras(p, 0, NULL));
    CALL(psfs_reconstruct(p, NULL, (float *)fk, NULL, NULL, 0, NULL));
    psfs_plan_destroy(p);
    psfs_plan_destroy(NULL);
    /* batches */
    psfs_batch *b = NULL;
    psfs_frame fr[3];
    memset(fr, 0, sizeof(fr));
    for (int f = 0; f < 3; ++f) {
        fr[f].grid = g; fr[f].n = 2; fr[f].cams = cams; fr[f].images_dev = imgs;
        fr[f].mean_dev = maps; fr[f].var_dev = maps; fr[f].posterior_dev = (float *)fk; fr[f].occ_dev = NULL;
    }
    CALL(psfs_batch_create(NULL, &prm, 3, fr));
    CALL(psfs_batch_create(&b, &prm, 0, fr));
    CALL(psfs_batch_create(&b, &prm, 3, NULL));
    fr[1].n = 17;
    CALL(psfs_batch_create(&b, &prm, 3, fr));
    fr[1].n = 2; fr[2].grid = bad;
    CALL(psfs_batch_create(&b, &prm, 3, fr));
    fr[2].grid = g;
    CALL(psfs_batch_create(&b, &prm, 3, fr));
    CALL(psfs_batch_workspace_bytes(b));
    CALL(psfs_batch_run(b, NULL, 0, NULL));
    CALL(psfs_batch_update(b, 3, fr));
    psfs_batch_destroy(b);
    psfs_batch_destroy(NULL);
    for (int t = -1; t <= psfs_tile_count(); ++t) { int32_t a, bq, c; CALL(psfs_tile_describe(t, &a, &bq, &c)); CALL(psfs_tile_describe(t, NULL, NULL, NULL)); }
    CALL(psfs_batch_set_tile(NULL, 0)); CALL(psfs_batch_get_tile(NULL));
    CALL(psfs_set_tile(NULL, 0));
    printf("calls %d, last error '%s'\nOK\n", calls, psfs_last_error());
    return 0;
}
