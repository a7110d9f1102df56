/* Exercises the host-only entry points of the C ABI (no device needed)
 * under AddressSanitizer and UndefinedBehaviorSanitizer; built against the
 * library's sources by tests/test_sanitizers.py. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/mpr.h"

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

int main(void)
{
    int64_t n = 0;
    CHECK(mpr_transfer_size(9, &n) == MPR_OK && n == 21909);
    CHECK(mpr_transfer_size(0, &n) == MPR_EINVAL);
    CHECK(mpr_transfer_size(12, &n) == MPR_OK);
    uint8_t *w = (uint8_t *)malloc((size_t)(33 * 3));
    CHECK(mpr_transfer_words(3, w, 33) == MPR_OK);
    CHECK(mpr_transfer_words(3, w, 32) == MPR_ENOMEM);
    free(w);
    /* m = 9 period (22, 5, 20) with gamma = 4n / 4n + 2 */
    int64_t tr[27];
    for (int k = 0; k < 27; k++) tr[k] = (k % 5 == 0) ? 4 * k : 4 * k + 2;
    int64_t g = 0, numer[5];
    CHECK(mpr_gamma_from_period(22, 5, 20, tr, 26, 1000000, &g) == MPR_OK && g == 4000000);
    CHECK(mpr_gamma_from_period(22, 5, 20, tr, 20, 100, &g) == MPR_EINVAL);
    CHECK(mpr_period_formula(22, 5, 20, tr, 26, numer) == MPR_OK);
    CHECK(numer[0] == 0 && numer[1] == 10);
    size_t bytes = 0;
    CHECK(mpr_power_workspace_size(1000, 10, MPR_CHAIN_SPARSE, &bytes) == MPR_OK && bytes > 0);
    CHECK(mpr_period_workspace_size_ex(100, 4, MPR_PERIOD_SPARSE, &bytes) == MPR_OK);
    CHECK(mpr_period_workspace_size_ex(100, 4, MPR_PERIOD_PIPELINE, &bytes) == MPR_OK);
    CHECK(mpr_period_workspace_size_ex(100, 4, MPR_PERIOD_PIPELINE | MPR_PERIOD_REUSE_A, &bytes) == MPR_EINVAL);
    CHECK(mpr_period_workspace_size_ex(100, 4, 16, &bytes) == MPR_EINVAL);
    CHECK(mpr_power_workspace_size(300, 10, MPR_CHAIN, &bytes) == MPR_OK && bytes >= 300 * 304 * 2 + 256);
    for (int s = 0; s < 9; s++) CHECK(mpr_status_string(s) != NULL);
    CHECK(mpr_gemm_config_count() > 0 && mpr_batch_config_count() > 0);
    CHECK(mpr_server_ladder_bytes(9, 32, 1000, 0) > mpr_server_ladder_bytes(9, 32, 1000, 1));
    CHECK(mpr_server_ladder_bytes(9, 32, 1000, 1) > 0 && mpr_server_ladder_bytes(0, 32, 1000, 0) < 0);
    printf("abi host sanitizer run ok\n");
    return 0;
}
