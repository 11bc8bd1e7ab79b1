/*
 * silu_factor.h -- host-side incomplete LU factorizations that produce the
 * factors the scaled-ILU smoother reads (libscaledilu.so).
 *
 * This is set-up, run once per matrix, on the host; the smoother's solve phase
 * (scaled_ilu.h) then runs entirely on the GPU.  The paper factors on the host
 * as well (Matlab's ilu, hypre's ILU set-up) and separates a symbolic phase,
 * which fixes the pattern, from a numeric phase (Section 3.1).
 *
 * All pointers here are HOST pointers.  Output matrices are allocated by the
 * library with malloc and released with silu_host_csr_free.
 *
 *   L  strictly lower part of the unit lower factor (the 1s are implied)
 *   U  upper factor with its diagonal stored as the FIRST entry of each row
 *
 * Return codes are those of scaled_ilu.h.  On SILU_ERR_ZERO_PIVOT or
 * SILU_ERR_PATTERN, *bad_row (if non-NULL) receives the offending row.
 */
#ifndef SILU_FACTOR_H
#define SILU_FACTOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n;
    int64_t nnz;
    int32_t *row_ptr; /* [n + 1] */
    int32_t *col_idx; /* [nnz]   */
    double *val;      /* [nnz]   */
} silu_host_csr;

/*
 * ILU(k), level of fill k >= 0 (Section 1, Saad's ILU(k); ILU(0) is the
 * 'nofill' factorization of Table 1).  Symbolic phase: stored entries of A
 * have level 0; eliminating row i with its lower entries k in increasing
 * order proposes level lev_ik + lev_kj + 1 for (i, j), j > k, and an entry
 * is kept when its level is <= k.  Numeric phase: Gaussian elimination
 * without pivoting restricted to that pattern.  A must store its diagonal.
 */
int silu_factor_iluk(const silu_host_csr *A, int k, silu_host_csr *L, silu_host_csr *U, int64_t *bad_row);

/*
 * ILUT(tau, p), the dual-threshold factorization (Sections 4.2 and 6.1:
 * drop tolerance and fill per row).  Row i with tau_i = tau * ||a_i*||_2:
 * lower entries are visited in increasing column order; an entry whose value
 * v (before division by the pivot) satisfies |v| < tau_i is dropped,
 * otherwise l_ik = v / u_kk eliminates with U's row k.  Upper entries with
 * |w_j| < tau_i are dropped.  At most p entries are kept in each of the L and
 * U parts, the largest by |l_ik u_kk| and by |u_ij| respectively, ties to the
 * smaller column; the diagonal is always kept.
 */
int silu_factor_ilut(const silu_host_csr *A, double tau, int p, silu_host_csr *L, silu_host_csr *U,
                     int64_t *bad_row);

void silu_host_csr_free(silu_host_csr *m);

#ifdef __cplusplus
}
#endif

#endif /* SILU_FACTOR_H */
