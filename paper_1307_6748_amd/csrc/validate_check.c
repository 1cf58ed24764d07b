/*
 * Address- and undefined-behaviour-sanitizer run of the library's host-side
 * validation (test infrastructure): tests/test_sanitizers.py builds the
 * library's host code (no device code) under -fsanitize=address,undefined
 * and links this driver, which calls every entry point of the C ABI with
 * arguments each check must reject -- NULL, misaligned and unaligned
 * pointers, bad sizes, non-finite parameters -- plus the host-only size and
 * layout queries, and checks the status codes and error messages.  No call
 * here reaches a GPU.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/isis_mg.h"

static int fails = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            printf("FAIL line %d: %s\n", __LINE__, #cond);                 \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

static void expect_msg(const char* m)
{
    EXPECT(m != NULL && strlen(m) > 0 && strlen(m) < 512);
}

int main(void)
{
    isis_model_params p;
    memset(&p, 0, sizeof(p));
    p.model = ISIS_SYMMETRON;
    p.lambda0 = 1.0;
    p.a_ssb = 0.5;
    p.beta = 1.0;
    p.omega_m = 0.27;
    isis_model_params bad = p;
    bad.lambda0 = NAN;
    /* fake device pointers: never dereferenced, every call fails validation */
    double* ok = (double*)(uintptr_t)4096;
    double* mis = (double*)(uintptr_t)(4096 + 8);

    isis_mg_desc d;
    memset(&d, 0, sizeof(d));
    d.N = 64;
    d.box = 64.0;
    d.nu_pre = d.nu_post = 2;
    d.nu_coarse = 32;
    d.max_cycles = 50;
    d.restriction = -1;
    d.prolongation = -1;
    size_t w64 = isis_mg_workspace_size(&d);
    EXPECT(w64 > 0);
    d.precision = ISIS_MIXED;
    EXPECT(isis_mg_workspace_size(&d) > w64);
    EXPECT(isis_mg_workspace_size(NULL) == 0);
    isis_mg_desc e = d;
    e.N = 48;
    EXPECT(isis_mg_workspace_size(&e) == 0);
    e = d;
    e.box = NAN;
    EXPECT(isis_mg_workspace_size(&e) == 0);
    e = d;
    e.max_cycles = ISIS_MG_MAX_HIST;
    EXPECT(isis_mg_workspace_size(&e) == 0);
    e = d;
    e.judge_skip = 3;
    EXPECT(isis_mg_workspace_size(&e) == 0);
    e = d;
    e.guess_accept = 2.0;
    EXPECT(isis_mg_workspace_size(&e) == 0);
    e = d;
    e.prolongation = 2;
    EXPECT(isis_mg_workspace_size(&e) == 0);

    isis_mg_t* h = (isis_mg_t*)1;
    EXPECT(isis_mg_create(&d, &h) == ISIS_ERR_INVALID_ARG && h == NULL);  /* no workspace */
    expect_msg(isis_mg_last_error(NULL));
    d.workspace = (void*)(uintptr_t)(4096 + 16);
    d.workspace_bytes = w64 * 4;
    EXPECT(isis_mg_create(&d, &h) == ISIS_ERR_INVALID_ARG);               /* misaligned */
    EXPECT(isis_mg_create(NULL, &h) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_create(&d, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_solve(NULL, ok, ok, &p, 1.0, 1e-8, 0, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_residual(NULL, ok, ok, &p, 1.0, NULL, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_set_profiling(NULL, 1) == ISIS_ERR_INVALID_ARG);
    isis_mg_destroy(NULL);

    double rms = 0.0;
    EXPECT(isis_mg_residual_noalloc(&p, 1.0, 8192, 1.0, ok, ok, NULL, &rms, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_residual_noalloc(&p, 1.0, 24, 1.0, ok, ok, NULL, &rms, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_residual_noalloc(&p, 1.0, 8, -1.0, ok, ok, NULL, &rms, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_residual_noalloc(&p, 1.0, 8, 1.0, mis, ok, NULL, &rms, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_residual_noalloc(&bad, 1.0, 8, 1.0, ok, ok, NULL, &rms, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_mg_residual_noalloc(NULL, 1.0, 8, 1.0, ok, ok, NULL, &rms, NULL) ==
           ISIS_ERR_INVALID_ARG);
    expect_msg(isis_mg_last_error(NULL));

    EXPECT(isis_op_halfsweep(&p, 1.0, 7, 1.0, ok, ok, NULL, 0, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_halfsweep(&p, 1.0, 8, 1.0, ok, ok, NULL, 2, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_halfsweep(&bad, 1.0, 8, 1.0, ok, ok, NULL, 0, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_sweeps(&p, 1.0, 8, 1.0, ok, mis, ok, NULL, 1, 0, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_sweeps(&p, 1.0, 8, 1.0, ok, ok, ok, NULL, 1, 3, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_prolong_sweeps(&p, 1.0, 8, 1.0, ok, ok, ok, NULL, ok, NULL, 1, 1, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_prolong_sweeps(&p, 1.0, 2, 1.0, ok, ok, ok, NULL, ok, ok, 1, 1, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_prolong_sweeps(&p, 1.0, 8, 1.0, ok, ok, ok, NULL, mis, ok, 1, 1, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_defect(&p, 0.0, 8, 1.0, ok, ok, NULL, ok, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_defect(&p, 1.0, 8, 1.0, ok, ok, NULL, NULL, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_restrict(9, ok, ok, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_restrict_fw(8, ok, mis, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_fas_descend(&p, 1.0, 8, 1.0, ok, ok, NULL, ok, ok, ok, ok, ok, mis, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_fas_descend(&p, 1.0, 2, 1.0, ok, ok, NULL, ok, ok, ok, ok, ok, NULL, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_prolong_correct(8, ok, NULL, ok, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_prolong_correct_w(8, ok, ok, NULL, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_prolong_correct_w(8, ok, ok, mis, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_coarse_solve(&p, 1.0, -1.0, ok, ok, NULL, 4, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_cold_start(&p, 1.0, -1, ok, ok, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_cold_start(&p, 1.0, 0, NULL, NULL, NULL) == ISIS_OK);
    EXPECT(isis_force(&p, 1.0, 8, 1.0, NULL, NULL, ok, ok, ok, NULL) == ISIS_ERR_INVALID_ARG);
    isis_model_params cham = p;
    cham.model = ISIS_CHAMELEON;
    cham.cham_alpha = cham.cham_mu = 1.0;
    cham.cham_n = 1.0;
    EXPECT(isis_force(&cham, 1.0, 8, 1.0, ok, NULL, ok, ok, ok, NULL) == ISIS_ERR_UNSUPPORTED);
    isis_model_params nomodel = p;
    nomodel.model = 9;
    EXPECT(isis_op_defect(&nomodel, 1.0, 8, 1.0, ok, ok, NULL, ok, NULL) == ISIS_ERR_INVALID_ARG);
    isis_model_params pu = p;
    pu.paper_u = 1;
    EXPECT(isis_op_defect(&pu, 1.0, 8, 1.0, ok, ok, NULL, ok, NULL) == ISIS_ERR_INVALID_ARG);

    EXPECT(isis_op_masked_defect(&p, 1.0, 8, 1.0, ok, ok, NULL, ok, ok, NULL, ok, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_op_masked_halfsweep(&p, 1.0, 8, 1.0, ok, ok, NULL, ok, ok, ok, 5, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_patch_workspace_size(7) == 0 && isis_patch_workspace_size(8) > 8 * 8 * 8 * 8);
    int sweeps = -1;
    EXPECT(isis_patch_solve(&p, 1.0, 8, 1.0, ok, ok, ok, ok, 0, 10, 1e-8, ok, 1 << 20, &sweeps,
                            &rms, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_patch_solve(&p, 1.0, 8, 1.0, ok, ok, ok, ok, 2, 10, 1e-8, ok, 16, &sweeps,
                            &rms, NULL) == ISIS_ERR_INVALID_ARG);

    /* the network's host-side checks and layout */
    EXPECT(isis_unet_param_count() > 900000);
    EXPECT(isis_unet_workspace_size(24, 0) == 0 && isis_unet_workspace_size(32, 1) >
                                                       isis_unet_workspace_size(32, 0));
    EXPECT(isis_unet_forward(NULL, ok, ok, 1.0, 32, NULL, ok, 1u << 30, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_unet_backward((const float*)ok, NULL, ok, 32, ok, 1u << 30, NULL, NULL, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_unet_adam_step(NULL, (const float*)ok, (float*)ok, (float*)ok, 10, 1, 1e-3f,
                               NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_unet_train_step((float*)ok, (float*)ok, (float*)ok, 0, 1e-3f, ok, ok, ok, 1.0, 32,
                                ok, 1u << 30, NULL, NULL, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_unet_predict((const float*)ok, ok, ok, 1.0, 12, NULL, NULL, ok, 1u << 30, NULL) ==
           ISIS_ERR_INVALID_ARG);
    expect_msg(isis_unet_last_error());
    void* ptr = NULL;
    long vox = 0;
    int ch = 0;
    EXPECT(isis_unet_tensor((void*)(uintptr_t)(1 << 20), 32, 22, &ptr, &vox, &ch) ==
           ISIS_ERR_INVALID_ARG);
    for (int id = 0; id < 22; ++id)
        EXPECT(isis_unet_tensor((void*)(uintptr_t)(1 << 20), 32, id, &ptr, &vox, &ch) == ISIS_OK &&
               vox > 0 && ch > 0);
    EXPECT(isis_conv3_fwd(NULL, 8, 16, NULL, NULL, 16, 0, NULL, NULL, NULL) ==
           ISIS_ERR_INVALID_ARG);
    EXPECT(isis_conv3_bwd_weight_workspace(3, 16, 16) == 0);
    EXPECT(isis_conv3_bwd_weight((const uint16_t*)ok, 16, 16, (const uint16_t*)ok, 16,
                                 (float*)ok, (float*)ok, ok, 8, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_conv3_bwd_weight(NULL, 16, 16, (const uint16_t*)ok, 16, (float*)ok, NULL, ok,
                                 1u << 30, NULL) == ISIS_ERR_INVALID_ARG);
    EXPECT(isis_conv3_flip_weights(NULL, 16, 16, NULL, NULL) == ISIS_ERR_INVALID_ARG);

    printf("sanitized validation run: %d failures\n", fails);
    return fails ? 1 : 0;
}
