/*
 * A plain C consumer of the liblbm C ABI (include/lbm.h): no Python, no PyTorch.
 *
 * Reads a run configuration from stdin as `name=value` lines (the lbm_config field names), a line
 * `steps=N` and optionally `precision=...` among them; allocates the device workspace and a stream
 * with HIP, creates a handle, advances it N steps and prints, as C99 hex floats (exact), the mass,
 * the heat-flux triple and the fields rho, ux, uy, T of run 0 (one value per line, row-major).
 * Exit status: 0 on success, 1 on a library error (message on stderr), 2 on bad input.
 *
 * Built by the package build into tests/c_abi_example.bin; used by tests/test_gpu_c_abi.py.
 */
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define FIELD_I(name) {#name, offsetof(lbm_config, name), 0}
#define FIELD_D(name) {#name, offsetof(lbm_config, name), 1}

static const struct {
    const char *name;
    size_t off;
    int is_double;
} kFields[] = {
    FIELD_I(nx), FIELD_I(ny), FIELD_I(bc_x), FIELD_I(rk_stages), FIELD_I(warmup_steps),
    FIELD_I(cyl_x), FIELD_I(cyl_y), FIELD_I(cyl_r), FIELD_I(upwind_kind), FIELD_I(diag_every),
    FIELD_D(nu), FIELD_D(eos_a), FIELD_D(eos_b), FIELD_D(eos_R), FIELD_D(acentric), FIELD_D(Tr_sat),
    FIELD_D(dTr_wall), FIELD_D(G), FIELD_D(sigma), FIELD_D(gx), FIELD_D(gy), FIELD_D(rho_gref),
    FIELD_D(rho_l), FIELD_D(rho_v), FIELD_D(rho_wall), FIELD_D(u_in), FIELD_D(alpha_T), FIELD_D(cv),
    FIELD_I(precision), FIELD_I(check_every), FIELD_D(rho_ref_shift), FIELD_D(nu_vapor),
    FIELD_D(alpha_vapor), FIELD_I(outlet_kind), FIELD_I(pad_),
};

static int fail_lib(const lbm_handle *h, const char *what, int rc)
{
    fprintf(stderr, "%s failed (%d): %s\n", what, rc, lbm_last_error(h));
    return 1;
}

int main(void)
{
    lbm_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    long steps = -1;
    char line[256];
    while (fgets(line, sizeof(line), stdin)) {
        char *eq = strchr(line, '=');
        if (!eq) continue;
        *eq = '\0';
        const char *key = line, *val = eq + 1;
        if (strcmp(key, "steps") == 0) {
            steps = strtol(val, NULL, 10);
            continue;
        }
        size_t k;
        for (k = 0; k < sizeof(kFields) / sizeof(kFields[0]); ++k)
            if (strcmp(key, kFields[k].name) == 0) break;
        if (k == sizeof(kFields) / sizeof(kFields[0])) {
            fprintf(stderr, "unknown field %s\n", key);
            return 2;
        }
        char *p = (char *)&cfg + kFields[k].off;
        if (kFields[k].is_double) *(double *)p = strtod(val, NULL);
        else *(int32_t *)p = (int32_t)strtol(val, NULL, 10);
    }
    if (steps < 0) {
        fprintf(stderr, "missing steps=N\n");
        return 2;
    }

    const size_t bytes = lbm_workspace_bytes(&cfg, 1);
    if (bytes == 0) return fail_lib(NULL, "lbm_workspace_bytes", LBM_EINVAL);
    void *ws = NULL;
    hipStream_t stream = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
        fprintf(stderr, "HIP allocation failed\n");
        return 1;
    }
    lbm_handle *h = NULL;
    int rc = lbm_create(&cfg, 1, ws, bytes, stream, &h);
    if (rc) return fail_lib(NULL, "lbm_create", rc);
    if ((rc = lbm_step(h, (int)steps))) return fail_lib(h, "lbm_step", rc);

    const size_t n = (size_t)cfg.nx * (size_t)cfg.ny;
    double *f = (double *)malloc(4 * n * sizeof(double));
    if (!f) return 2;
    double mass = 0, q = 0, nu = 0, nu_avg = 0;
    if ((rc = lbm_total_mass(h, 0, &mass))) return fail_lib(h, "lbm_total_mass", rc);
    if ((rc = lbm_wall_heat_flux(h, 0, &q, &nu, &nu_avg))) return fail_lib(h, "lbm_wall_heat_flux", rc);
    if ((rc = lbm_fields(h, 0, f, f + n, f + 2 * n, f + 3 * n, NULL))) return fail_lib(h, "lbm_fields", rc);
    printf("mass %a\nq %a\nnu %a\nnu_avg %a\n", mass, q, nu, nu_avg);
    for (size_t k = 0; k < 4 * n; ++k) printf("%a\n", f[k]);
    free(f);
    lbm_destroy(h);
    (void)hipStreamDestroy(stream);
    (void)hipFree(ws);
    return 0;
}
