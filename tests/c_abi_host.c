/* Plain C99 consumer of the C-ABI (no GPU needed): the headers compile as C,
 * the library links, and the host-only entry points work. */
#include <stdio.h>
#include <string.h>

#include "scaled_ilu.h"
#include "silu_factor.h"

int main(void)
{
    /* tridiagonal (2, -1) path of 5 rows: the relabeling of a path from its
     * end is the reversed natural order */
    int32_t rp[6] = {0, 2, 5, 8, 11, 13};
    int32_t col[13] = {0, 1, 0, 1, 2, 1, 2, 3, 2, 3, 4, 3, 4};
    double val[13] = {2, -1, -1, 2, -1, -1, 2, -1, -1, 2, -1, -1, 2};
    int32_t order[5];
    int st = silu_reorder_rcm(5, rp, col, val, 0.25, order);
    if (st != SILU_OK) {
        printf("silu_reorder_rcm: %s\n", silu_status_string(st));
        return 1;
    }
    for (int k = 0; k < 5; k++)
        if (order[k] != 4 - k) {
            printf("order[%d] = %d\n", k, (int)order[k]);
            return 1;
        }
    if (silu_reorder_rcm(5, rp, col, val, -1.0, order) != SILU_ERR_ARG) return 1;
    if (strcmp(silu_status_string(SILU_ERR_ZERO_PIVOT), "zero or non-finite pivot") != 0) return 1;
    /* host ILU(0) of the same matrix: the exact LU, u_ii = (i+2)/(i+1) */
    silu_host_csr A = {5, 13, rp, col, val}, L, U;
    int64_t bad = -1;
    memset(&L, 0, sizeof L);
    memset(&U, 0, sizeof U);
    if (silu_factor_iluk(&A, 0, &L, &U, &bad) != SILU_OK) return 1;
    for (int i = 0; i < 5; i++) {
        const double want = (double)(i + 2) / (double)(i + 1);
        const double got = U.val[U.row_ptr[i]];
        if (!(got > want * (1.0 - 1e-15) && got < want * (1.0 + 1e-15))) {
            printf("u_%d%d = %.17g, want %.17g\n", i, i, got, want);
            return 1;
        }
    }
    silu_host_csr_free(&L);
    silu_host_csr_free(&U);
    printf("c-abi ok\n");
    return 0;
}
