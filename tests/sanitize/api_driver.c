/* Calls the library's host-side paths that run without a GPU (argument validation, workspace sizes,
 * pitches, error messages, NULL contexts) for the host sanitizer test (tests/test_host_sanitizers.py),
 * which links it against a host-only build of the library compiled with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Prints one line per check and "ok <n>" at the end; exits 1 on the first
 * unexpected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/lbm.h"

static int checks = 0;

static int expect(const char *what, int got, int want)
{
    ++checks;
    const char *msg = lbm_last_error();
    if (!msg || strlen(msg) > 4096) {
        printf("FAIL %s: bad error message\n", what);
        return 1;
    }
    if (got != want) {
        printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, msg);
        return 1;
    }
    printf("%s: %d (%s)\n", what, got, msg);
    return 0;
}

static lbm_params base(int32_t nx, int32_t ny)
{
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.dx = 1.0 / nx;
    p.dt = 1e-4;
    p.lambda = 0.25;
    p.D_const = 1e-3;
    p.store = LBM_STORE_F64;
    p.math = LBM_MATH_F64;
    p.aux = LBM_AUX_LOCAL;
    p.scale_log2 = 15;
    p.boundary = LBM_BC_PERIODIC;
    p.lattice = LBM_LATTICE_D2Q9;
    return p;
}

int main(void)
{
    int bad = 0;
    size_t bytes = 0;
    int64_t pitch = 0;
    bad |= expect("abi version", lbm_abi_version(), LBM_ABI_VERSION);

    /* valid parameter sets: every store, math, aux, boundary and lattice */
    const int stores[4][2] = {{LBM_STORE_F64, LBM_MATH_F64}, {LBM_STORE_F64, LBM_MATH_F32},
                              {LBM_STORE_F32, LBM_MATH_F32}, {LBM_STORE_F16S, LBM_MATH_F32}};
    for (int s = 0; s < 4; ++s)
        for (int aux = 0; aux < 3; ++aux)
            for (int bc = 0; bc < 3; ++bc) {
                lbm_params p = base(37, 29);
                p.store = stores[s][0];
                p.math = stores[s][1];
                p.aux = aux;
                p.boundary = bc;
                char what[96];
                snprintf(what, sizeof what, "workspace store %d math %d aux %d bc %d", p.store, p.math, aux, bc);
                /* the flux form is periodic only */
                const int want = aux == LBM_AUX_FLUX && bc != LBM_BC_PERIODIC ? LBM_E_UNSUPPORTED : LBM_OK;
                bad |= expect(what, lbm_workspace_size(1, &p, &bytes), want);
                if (want != LBM_OK) continue;
                bad |= expect("pitch", lbm_pitch(&p, &pitch), LBM_OK);
                if (pitch < p.nx) bad |= expect("pitch >= nx", 0, 1);
            }
    {
        lbm_params p = base(64, 64);
        p.store = LBM_STORE_F16SR;
        p.math = LBM_MATH_F32;
        p.round_seed = 12345;
        bad |= expect("workspace f16sr", lbm_workspace_size(1, &p, &bytes), LBM_OK);
        p.store = LBM_STORE_F32;
        bad |= expect("round_seed without f16sr", lbm_workspace_size(1, &p, &bytes), LBM_E_ARG);
    }
    for (int lat = 1; lat <= 2; ++lat) {
        lbm_params p = base(17, 13);
        p.lattice = lat;
        p.nz = 11;
        bad |= expect("workspace 3D", lbm_workspace_size(1, &p, &bytes), LBM_OK);
        p.nz = 2;
        bad |= expect("3D nz < 3", lbm_workspace_size(1, &p, &bytes), LBM_E_ARG);
    }
    {
        lbm_params ps[3] = {base(40, 40), base(100, 7), base(3, 3)};
        bad |= expect("workspace batch", lbm_workspace_size(3, ps, &bytes), LBM_OK);
    }

    /* invalid parameters: each rejected with LBM_E_ARG before anything is allocated */
    struct {
        const char *what;
        int field;
        double v;
    } cases[] = {
        {"nx < 3", 0, 2},          {"ny < 3", 1, 2},           {"nx > 2^24", 0, 16777217.0},
        {"nodes > 2^31", 2, 0},    {"dx = 0", 3, 0.0},         {"dt NaN", 4, NAN},
        {"lambda <= 0", 5, -1.0},  {"store 7", 7, 7},
        {"math 5", 8, 5},          {"aux 9", 9, 9},            {"scale_log2 25", 10, 25},
        {"boundary 3", 11, 3},     {"tau3 0.5", 12, 0.5},      {"lattice 3", 13, 3},
        {"phi_ref NaN", 14, NAN},  {"FP64 math, FP32 store", 6, 0},
    };
    for (size_t k = 0; k < sizeof cases / sizeof cases[0]; ++k) {
        lbm_params p = base(32, 32);
        switch (cases[k].field) {
        case 0: p.nx = (int32_t)cases[k].v; break;
        case 1: p.ny = (int32_t)cases[k].v; break;
        case 2: p.nx = 1 << 16; p.ny = (1 << 15) + 1; break;
        case 3: p.dx = cases[k].v; break;
        case 4: p.dt = cases[k].v; break;
        case 5: p.lambda = cases[k].v; break;
        case 6: p.store = LBM_STORE_F32; break;
        case 7: p.store = (int32_t)cases[k].v; break;
        case 8: p.math = (int32_t)cases[k].v; break;
        case 9: p.aux = (int32_t)cases[k].v; break;
        case 10: p.store = LBM_STORE_F16S; p.math = LBM_MATH_F32; p.scale_log2 = (int32_t)cases[k].v; break;
        case 11: p.boundary = (int32_t)cases[k].v; break;
        case 12: p.tau3 = cases[k].v; break;
        case 13: p.lattice = (int32_t)cases[k].v; break;
        case 14: p.store = LBM_STORE_F16S; p.math = LBM_MATH_F32; p.phi_ref = cases[k].v; break;
        }
        bad |= expect(cases[k].what, lbm_workspace_size(1, &p, &bytes), LBM_E_ARG);
    }
    bad |= expect("n_inst 0", lbm_workspace_size(0, NULL, &bytes), LBM_E_ARG);
    bad |= expect("n_inst -1", lbm_workspace_size(-1, NULL, &bytes), LBM_E_ARG);
    {
        lbm_params p = base(32, 32);
        bad |= expect("bytes NULL", lbm_workspace_size(1, &p, NULL), LBM_E_ARG);
        bad |= expect("pitch NULL", lbm_pitch(&p, NULL), LBM_E_ARG);
    }

    /* lbm_init argument errors (host checks before any device work) */
    {
        lbm_params p = base(32, 32);
        lbm_fields f;
        memset(&f, 0, sizeof f);
        lbm_ctx *ctx = (lbm_ctx *)&bytes;
        bad |= expect("init out NULL", lbm_init(NULL, 1, &p, &f, NULL, 0, NULL), LBM_E_ARG);
        bad |= expect("init fields NULL", lbm_init(&ctx, 1, &p, NULL, NULL, 0, NULL), LBM_E_ARG);
        if (ctx != NULL) bad |= expect("init clears ctx", 0, 1);
        bad |= expect("init phi0 NULL", lbm_init(&ctx, 1, &p, &f, NULL, 0, NULL), LBM_E_ARG);
        double dummy[4];
        f.phi0 = f.ux = f.uy = dummy;
        lbm_params p3 = base(8, 8);
        p3.lattice = LBM_LATTICE_D3Q19;
        p3.nz = 8;
        bad |= expect("init 3D without uz", lbm_init(&ctx, 1, &p3, &f, NULL, 0, NULL), LBM_E_ARG);
        lbm_params pd = base(32, 32);
        pd.D_const = INFINITY;
        bad |= expect("init D_const inf without D", lbm_init(&ctx, 1, &pd, &f, NULL, 0, NULL), LBM_E_ARG);
        pd.D_const = 0.0;
        bad |= expect("init D_const 0 without D", lbm_init(&ctx, 1, &pd, &f, NULL, 0, NULL), LBM_E_ARG);
        char ws[512];
        bad |= expect("init workspace too small", lbm_init(&ctx, 1, &p, &f, ws, sizeof ws, NULL), LBM_E_ARG);
        bad |= expect("init n_inst 0", lbm_init(&ctx, 0, &p, &f, NULL, 0, NULL), LBM_E_ARG);
    }

    /* calls on a NULL context */
    {
        lbm_launch lc;
        memset(&lc, 0, sizeof lc);
        lc.rows = 1;
        lbm_batch b;
        memset(&b, 0, sizeof b);
        lbm_stats st;
        bad |= expect("step NULL ctx", lbm_step(NULL, 1, NULL, NULL, NULL, NULL), LBM_E_STATE);
        bad |= expect("set_launch NULL ctx", lbm_set_launch(NULL, -1, &lc), LBM_E_STATE);
        bad |= expect("get_launch NULL ctx", lbm_get_launch(NULL, 0, &lc), LBM_E_STATE);
        bad |= expect("set_batch NULL ctx", lbm_set_batch(NULL, &b), LBM_E_STATE);
        bad |= expect("macros NULL ctx", lbm_macros(NULL, 0, NULL, NULL, &st), LBM_E_STATE);
        bad |= expect("state_bytes NULL ctx", lbm_state_bytes(NULL, 0, &bytes), LBM_E_STATE);
        bad |= expect("free NULL", lbm_free(NULL), LBM_OK);
    }
    if (bad) return 1;
    printf("ok %d\n", checks);
    return 0;
}
