/* Compiles the public header as C and exercises the validation paths that
 * never touch a device. Prints struct sizes for the Python-side layout check. */
#include <stdio.h>
#include <string.h>
#include "psfs.h"

#define EXPECT(cond) do { if (!(cond)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); return 1; } } while (0)

int main(void)
{
    psfs_plan *p = NULL;
    psfs_camera cam;
    psfs_grid g = {4, 4, 4, {0.f, 0.f, 0.f}, 0.1f};
    psfs_params prm;
    memset(&cam, 0, sizeof(cam));
    cam.width = 8; cam.height = 6; cam.P[11] = 1.f;
    EXPECT(psfs_version() == PSFS_VERSION);
    EXPECT(psfs_plan_create(&p) == PSFS_OK && p);
    EXPECT(psfs_set_cameras(p, 17, &cam) == PSFS_E_RANGE);
    EXPECT(strlen(psfs_last_error()) > 0);
    EXPECT(psfs_set_cameras(p, 1, &cam) == PSFS_OK);
    EXPECT(psfs_set_grid(p, &g) == PSFS_OK);
    psfs_default_params(&prm);
    prm.prior = 1.5f;
    EXPECT(psfs_set_params(p, &prm) == PSFS_E_RANGE);
    EXPECT(psfs_lmap_floats(p) == 64);
    EXPECT(psfs_workspace_bytes(p) == 256);
    EXPECT(psfs_fuse(p, NULL, NULL, NULL, NULL) == PSFS_E_ARG);
    psfs_plan_destroy(p);
    psfs_plan_destroy(NULL);
    printf("sizes %zu %zu %zu\n", sizeof(psfs_camera), sizeof(psfs_grid), sizeof(psfs_params));
    printf("OK\n");
    return 0;
}
