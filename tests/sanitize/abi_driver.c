/* Exercises the host-side paths of the C ABI (argument checks, workspace sizing, engine
 * configuration, error strings) in a build of the library with AddressSanitizer and
 * UndefinedBehaviorSanitizer on its host code (tests/test_sanitizers.py). No GPU is needed:
 * every call here is rejected or answered before any device work. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "gsk.h"

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, gsk_last_error()); return 1; } } while (0)

int main(void) {
    CHECK(gsk_version() > 0);
    gsk_options o;
    gsk_default_options(&o);
    CHECK(o.maxit == 10000 && o.check_every > 0);
    CHECK(gsk_workspace_bytes(GSK_METHOD_BICGSTAB, 1000, 0) > 7 * 8 * 1000);
    CHECK(gsk_workspace_bytes(GSK_METHOD_GMRES, 1000, 30) > 32 * 8 * 1000);
    CHECK(gsk_workspace_bytes(GSK_METHOD_GMRES, 1000, 0) == 0);
    CHECK(gsk_workspace_bytes(GSK_METHOD_GMRES, 0, 30) == 0);
    CHECK(gsk_workspace_bytes(99, 1000, 30) == 0);
    /* a stencil matrix description (no device memory is touched by sizing or rejection) */
    static double dummy[1];
    gsk_matrix S;
    memset(&S, 0, sizeof S);
    S.kind = GSK_MATRIX_STENCIL;
    S.stencil.nx = 10;
    S.stencil.ny = 10;
    S.stencil.nz = 10;
    S.stencil.coef = dummy;
    CHECK(gsk_workspace_bytes_for(&S, GSK_METHOD_GMRES_MIXED, 20) > 0);
    S.stencil.nx = 1;
    CHECK(gsk_workspace_bytes_for(&S, GSK_METHOD_GMRES, 20) == 0);
    CHECK(strlen(gsk_last_error()) > 0);
    S.stencil.nx = 10;
    gsk_info info;
    CHECK(gsk_gmres(NULL, dummy, dummy, 30, 1e-8, NULL, &info, dummy, 8, NULL) ==
          GSK_ERR_INVALID_ARG);
    CHECK(gsk_gmres(&S, dummy, dummy, 0, 1e-8, NULL, &info, dummy, 8, NULL) ==
          GSK_ERR_INVALID_ARG);
    CHECK(gsk_bicgstab(&S, dummy, dummy, -1.0, NULL, &info, dummy, 8, NULL) ==
          GSK_ERR_INVALID_ARG);
    CHECK(gsk_bicgstab(&S, dummy, dummy, 1e-8, NULL, &info, NULL, 0, NULL) ==
          GSK_ERR_WORKSPACE);
    gsk_options bad = o;
    bad.check_every = 0;
    CHECK(gsk_bicgstab(&S, dummy, dummy, 1e-8, &bad, &info, dummy, 8, NULL) ==
          GSK_ERR_INVALID_ARG);
    /* the no-allocation entry point rejects systems beyond its scratch array before any
     * device work */
    S.stencil.nx = S.stencil.ny = S.stencil.nz = 100;
    CHECK(gsk_bicgstab_noalloc(&S, dummy, dummy, 1e-8, NULL, &info, NULL) == GSK_ERR_WORKSPACE);
    CHECK(gsk_bicgstab_noalloc_max_bytes() > 0);
    /* engine configurations */
    gsk_engine_config c;
    memset(&c, 0, sizeof c);
    c.max_rows = 1 << 20;
    c.max_systems = 64;
    c.method = GSK_METHOD_BICGSTAB;
    c.precision = GSK_PRECISION_FP64;
    c.check_every = 8;
    CHECK(gsk_engine_workspace_bytes_ex(&c) > 7 * 8 * (size_t)(1 << 20));
    c.precision = GSK_PRECISION_MIXED;
    CHECK(gsk_engine_workspace_bytes_ex(&c) > 0);
    c.run_cap = -2;
    CHECK(gsk_engine_workspace_bytes_ex(&c) == 0);
    c.run_cap = 0;
    c.method = GSK_METHOD_GMRES;
    c.m = 0;
    CHECK(gsk_engine_workspace_bytes_ex(&c) == 0);
    c.m = 65;
    CHECK(gsk_engine_workspace_bytes_ex(&c) == 0);
    c.m = 20;
    c.tile_units = 2;
    CHECK(gsk_engine_workspace_bytes_ex(&c) == 0);
    c.tile_units = 0;
    CHECK(gsk_engine_workspace_bytes_ex(&c) > 0);
    c.class_shapes = 0x321;   /* per-class shapes: FP64 Bi-CGSTAB only */
    CHECK(gsk_engine_workspace_bytes_ex(&c) == 0);
    c.method = GSK_METHOD_BICGSTAB;
    c.precision = GSK_PRECISION_FP64;
    CHECK(gsk_engine_workspace_bytes_ex(&c) > 0);
    c.class_shapes = 0x5;
    CHECK(gsk_engine_workspace_bytes_ex(&c) == 0);
    c.class_shapes = 0;
    c.method = GSK_METHOD_GMRES;
    gsk_engine* e = NULL;
    CHECK(gsk_engine_create_ex(NULL, dummy, 8, NULL, &e) == GSK_ERR_INVALID_ARG && e == NULL);
    CHECK(gsk_engine_create_ex(&c, dummy, 8, NULL, &e) == GSK_ERR_WORKSPACE && e == NULL);
    CHECK(gsk_stream_mix_bytes(11, 2, 1000) > 13 * 8 * 1000);
    CHECK(gsk_stream_mix_bytes(2, 2, 1000) == 0);
    float ms = 0.0f;
    CHECK(gsk_stream_mix_ms(2, 2, 1000, dummy, 8, 1, &ms, NULL) == GSK_ERR_INVALID_ARG);
    CHECK(gsk_stream_mix_ms(11, 2, 1000, dummy, 8, 1, &ms, NULL) == GSK_ERR_WORKSPACE);
    CHECK(gsk_probe_begin(99, 1) == GSK_ERR_INVALID_ARG);
    CHECK(gsk_probe_begin(GSK_KCLASS_BATCH_P, 0) == GSK_ERR_INVALID_ARG);
    printf("abi driver: ok\n");
    return 0;
}
