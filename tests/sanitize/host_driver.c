/* Drives the host-side paths of librbe that need no GPU (the normaliser,
 * parameter validation, creation without a device, the tile cache, the
 * no-allocation entry point's argument checks, error messages), for an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the host code. */
#include <stdio.h>
#include <string.h>

#include "rbe.h"

int main(void)
{
    int bad = 0;
    double H = 0, S = 0;
    bad |= rbe_normalizer(1.0, 10.0, &H, &S) != RBE_OK;
    bad |= rbe_normalizer(-1.0, 10.0, &H, &S) != RBE_ERR_INVALID;
    rbe_params p;
    memset(&p, 0, sizeof p);
    p.n = 100;
    p.p = 10;
    p.box = 10.0;
    p.alpha = 1.0;
    p.r_cut = 3.5;
    p.coulomb = 1.0;
    p.mass = 1.0;
    p.lj_sigma = 1.0;
    p.lj_rcut = 2.5;
    rbe_ctx *ctx = NULL;
    p.r_cut = 6.0;
    bad |= rbe_create(&p, NULL, &ctx) != RBE_ERR_CUTOFF || ctx != NULL;
    bad |= strlen(rbe_last_error(NULL)) == 0;
    p.r_cut = 3.5;
    p.n_fixed = 101;
    bad |= rbe_create(&p, NULL, &ctx) != RBE_ERR_INVALID;
    p.n_fixed = 0;
    double d[100];
    for (int i = 0; i < 100; ++i) d[i] = i == 5 ? -1.0 : 1.0;
    p.diameter = d;
    p.lj_eps = 1.0;
    bad |= rbe_create(&p, NULL, &ctx) != RBE_ERR_INVALID;
    p.diameter = NULL;
    /* valid parameters: fails cleanly without a device */
    rbe_status st = rbe_create(&p, NULL, &ctx);
    bad |= !(st == RBE_ERR_NO_DEVICE || st == RBE_OK);
    if (ctx) rbe_destroy(ctx);
    rbe_tiles t;
    bad |= rbe_tune_lookup(NULL, 0, 100, 10, 1, &t) != RBE_ERR_INVALID;
    (void)rbe_tune_lookup("gfx950", 0, 100, 10, 1, &t);
    int dummy = 0;
    p.n = (1 << 20) + 1;
    bad |= rbe_kspace_forces_noalloc(&p, &dummy, &dummy, &dummy, &dummy, 0, NULL) != RBE_ERR_INVALID;
    bad |= strstr(rbe_last_error(NULL), "fixed workspace") == NULL;
    bad |= rbe_kspace_forces_noalloc(NULL, NULL, NULL, NULL, NULL, 0, NULL) != RBE_ERR_INVALID;
    bad |= rbe_check(NULL) != RBE_ERR_INVALID;
    bad |= rbe_sample_k(NULL, 0, NULL) != RBE_ERR_INVALID;
    printf("host driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
