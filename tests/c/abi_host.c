/* A plain C99 caller of the library's host-side calls: the header compiles
 * as C, the library links and its set-up calls run without a GPU.  Prints
 * the node-class counts of a D2Q9 disk box (the caller compares them with
 * its own count) and exits 0 when every check holds. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define CHECK(cond)                                                  \
    do {                                                             \
        if (!(cond)) {                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                \
        }                                                            \
    } while (0)

int main(void) {
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.abi_version = LBM_ABI_VERSION;
    p.lattice = LBM_D2Q9;
    p.precision = LBM_FP64;
    p.ghost_rule = LBM_GHOST_EQ9;
    p.n[0] = 64;
    p.n[1] = 48;
    p.n[2] = 1;
    p.rho_l = 1000.0;
    p.rho_g = 1.0;
    p.mu_l = 10.0;
    p.mu_g = 0.1;
    p.sigma = 0.01;
    p.W = 4.0;
    p.mobility = 0.02;

    lbm_ctx* ctx = NULL;
    p.W = 3.0;   /* below 4: rejected with a message */
    CHECK(lbm_create(&p, &ctx) == LBM_EINVAL && ctx == NULL);
    CHECK(lbm_last_error(NULL) != NULL && strlen(lbm_last_error(NULL)) > 0);
    p.W = 4.0;
    CHECK(lbm_create(&p, &ctx) == LBM_OK && ctx != NULL);

    size_t bytes = 0;
    CHECK(lbm_device_bytes(ctx, &bytes) == LBM_ESTATE);   /* geometry first */
    lbm_solid disk;
    memset(&disk, 0, sizeof disk);
    disk.kind = 0;
    disk.center[0] = 32.0;
    disk.center[1] = 20.0;
    disk.radius = 9.5;
    CHECK(lbm_set_geometry(ctx, &disk, 1) == LBM_OK);
    CHECK(lbm_device_bytes(ctx, &bytes) == LBM_OK && bytes > 0);
    CHECK(lbm_step(ctx, 1) == LBM_ESTATE);                 /* not bound, not started */

    int32_t c[19 * 3], q = 0;
    CHECK(lbm_lattice(LBM_D2Q9, c, &q) == LBM_OK && q == 9);

    const size_t n = 64 * 48;
    double* flags = (double*)malloc(n * sizeof(double));
    CHECK(flags != NULL);
    CHECK(lbm_read_field(ctx, LBM_FIELD_FLAGS, flags, n) == LBM_OK);
    long solid = 0, ghost = 0, near = 0;
    for (size_t k = 0; k < n; k++) {
        const int f = (int)flags[k];
        solid += (f & 1) != 0;
        near += (f & 2) != 0;
        ghost += (f & 4) != 0;
    }
    CHECK(solid > 0 && ghost > 0 && near > 0);
    printf("solid %ld ghost %ld near %ld device_bytes %zu\n", solid, ghost, near, bytes);
    free(flags);
    CHECK(lbm_destroy(ctx) == LBM_OK);
    return 0;
}
