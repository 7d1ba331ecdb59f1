/* A plain C caller of the library's C ABI: no Python anywhere on the path.
 * It draws the KL coefficients of R realizations with the library's own
 * generator, allocates the two state buffers of one jet level with the HIP
 * runtime, creates the ensemble, takes a given number of steps, and writes
 * the state (double [4 var][5 slot][R][ny][nx], vlbm_get_state's layout),
 * each realization's time and step count to a binary file.
 *
 *   abi_c_caller NX NY R STEPS OUT_FILE
 *
 * Exit status 0 on success; a failed call prints vlbm_last_error(). */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "vlbm.h"

#define CHECK(call)                                                                    \
    do {                                                                               \
        const vlbm_status rc_ = (call);                                                \
        if (rc_ != VLBM_OK) {                                                          \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)rc_, vlbm_last_error()); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 6) {
        fprintf(stderr, "usage: %s NX NY R STEPS OUT_FILE\n", argv[0]);
        return 2;
    }
    const int nx = atoi(argv[1]), ny = atoi(argv[2]), R = atoi(argv[3]), steps = atoi(argv[4]);
    const vlbm_params p = {5.0 / 3.0, 1.0 / 3.0, 1.0, 0.1, 1e-2, 0.5, 0.4127, 5.0, 800.0, 0.05, 0.1,
                           10, 2, VLBM_BC_JET, VLBM_LIMITER_RLMP, VLBM_FP64, 0};
    double *coefs = malloc(sizeof(double) * (size_t)R * 20);
    CHECK(vlbm_kl_coefficients(2605, 0, R, 10, coefs));
    size_t bytes = 0;
    CHECK(vlbm_state_bytes(&p, nx, ny, R, &bytes));
    vlbm_level lv = {nx, ny, 1.0 / nx, -0.25, {NULL, NULL}};
    if (hipMalloc(&lv.state[0], bytes) != hipSuccess || hipMalloc(&lv.state[1], bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    vlbm_ensemble *e = NULL;
    CHECK(vlbm_init_ensemble(&p, &lv, 1, coefs, R, NULL, &e));
    int32_t done = 0;
    CHECK(vlbm_step(e, 1e30, steps, &done));
    const size_t n = (size_t)20 * R * ny * nx;
    double *d_out = NULL;
    if (hipMalloc((void **)&d_out, n * sizeof(double)) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    CHECK(vlbm_get_state(e, 0, d_out));
    double *h_out = malloc(n * sizeof(double));
    double *t = malloc(sizeof(double) * R);
    int64_t *s = malloc(sizeof(int64_t) * R);
    if (hipMemcpy(h_out, d_out, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        fprintf(stderr, "hipMemcpy failed\n");
        return 1;
    }
    CHECK(vlbm_times(e, 0, t, s, NULL, NULL));
    FILE *f = fopen(argv[5], "wb");
    if (!f || fwrite(h_out, sizeof(double), n, f) != n || fwrite(t, sizeof(double), R, f) != (size_t)R ||
        fwrite(s, sizeof(int64_t), R, f) != (size_t)R) {
        fprintf(stderr, "writing %s failed\n", argv[5]);
        return 1;
    }
    fclose(f);
    CHECK(vlbm_destroy(e));
    hipFree(d_out);
    hipFree(lv.state[0]);
    hipFree(lv.state[1]);
    free(coefs);
    free(h_out);
    free(t);
    free(s);
    return 0;
}
