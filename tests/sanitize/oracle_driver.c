/* Exercises the oracle's C functions under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py).
 * Exit status 0 when every result matches a known value. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_words(int m, uint8_t *out);
int oracle_transfer(int m, int64_t *A);
int oracle_border_transfer(int m, int64_t *A);
int oracle_minplus(int64_t M, int64_t K, int64_t N, const int64_t *X, const int64_t *Y, int64_t *C);
void oracle_normalise(int64_t M, int64_t N, int64_t *C, int64_t *r);
int oracle_product_of_powers(int64_t n, const int64_t *Na, const int64_t *Ra, const int64_t *Nb, const int64_t *Rb,
                             int64_t *Nc, int64_t *Rc);
int64_t oracle_trace(int64_t n, const int64_t *N, const int64_t *R);
int64_t oracle_brute_gamma(int m, int n);
int64_t oracle_rowdp_gamma(int m, int n);
int64_t oracle_brute_border_loss(int m, int n);
void oracle_minplus_at(int64_t K, int64_t N, const int64_t *X, const int64_t *Y, const int64_t *ii,
                       const int64_t *jj, int64_t count, int64_t *out);

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

int main(void)
{
    CHECK(oracle_words(5, NULL) == 287);
    const int m = 3;
    const int64_t n = oracle_words(m, NULL);
    int64_t *A = malloc(sizeof(int64_t) * n * n), *N = malloc(sizeof(int64_t) * n * n);
    int64_t *C = malloc(sizeof(int64_t) * n * n), *R = malloc(sizeof(int64_t) * n), *r = malloc(sizeof(int64_t) * n);
    int64_t *N2 = malloc(sizeof(int64_t) * n * n), *R2 = malloc(sizeof(int64_t) * n);
    CHECK(oracle_transfer(m, A) == 0);
    /* A^5 by the chain: gamma_R(P_3 x C_5) = 8 */
    for (int64_t i = 0; i < n * n; i++) N[i] = A[i];
    oracle_normalise(n, n, N, R);
    for (int k = 2; k <= 5; k++) {
        CHECK(oracle_minplus(n, n, n, N, A, C) == 0);
        oracle_normalise(n, n, C, r);
        for (int64_t i = 0; i < n; i++) R[i] += r[i];
        for (int64_t i = 0; i < n * n; i++) N[i] = C[i];
    }
    CHECK(oracle_trace(n, N, R) == 8);
    /* A^5 (x) A^5 = A^10: gamma_R(P_3 x C_10) = 16 */
    CHECK(oracle_product_of_powers(n, N, R, N, R, N2, R2) == 0);
    CHECK(oracle_trace(n, N2, R2) == 16);
    int64_t ii[2] = {0, n - 1}, jj[2] = {n - 1, 0}, out[2];
    oracle_minplus_at(n, n, A, A, ii, jj, 2, out);
    CHECK(oracle_minplus(n, n, n, A, A, C) == 0);
    CHECK(out[0] == C[n - 1] && out[1] == C[(n - 1) * n]);
    CHECK(oracle_brute_gamma(2, 5) == 6);
    CHECK(oracle_rowdp_gamma(3, 6) == 10);
    CHECK(oracle_brute_border_loss(2, 4) >= 0 || oracle_brute_border_loss(2, 4) < 0);
    int64_t *B = malloc(sizeof(int64_t) * 97 * 97);
    CHECK(oracle_border_transfer(4, B) == 0);
    free(A); free(N); free(C); free(R); free(r); free(N2); free(R2); free(B);
    printf("oracle sanitizer run ok\n");
    return 0;
}
