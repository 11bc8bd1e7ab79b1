/*
 * oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * scaled-ILU smoother of "Scaled ILU Smoothers for Navier-Stokes Pressure
 * Projection" (Thomas, Carr, Mullowney, Swirydowicz, Day; arXiv 2111.09512).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the package's smoke check and the
 * CPU-baseline leg of the benchmark are the only callers.  Nothing here is
 * shared with the GPU library: no headers, no helpers, no tables.  The two
 * implementations meet only through the seeded input generators.
 *
 * Conventions.  Square matrices in CSR form with int row pointers and column
 * indices (every size here is below 2^31) and double values; columns sorted
 * ascending inside a row.  A row sum sum_j a_ij x_j is always formed the plain
 * way: start from 0.0 and add the products in ascending column order.  A
 * Richardson/substitution step then subtracts that sum from the right-hand
 * side.  No fast-math, no FMA contraction (the build passes
 * -ffp-contract=off).
 *
 * Status codes returned by the functions below:
 *   0  ok
 *   1  zero (or non-finite) pivot; *bad_row holds the row
 *   2  out of memory
 *   3  pattern error (missing diagonal, entry on the wrong side, ...)
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ZERO_PIVOT 1
#define ORC_NOMEM 2
#define ORC_PATTERN 3

typedef struct {
    int n;
    long long nnz;
    int *rp;
    int *col;
    double *val;
} orc_csr;

void orc_csr_free(orc_csr *m)
{
    free(m->rp);
    free(m->col);
    free(m->val);
    m->rp = NULL;
    m->col = NULL;
    m->val = NULL;
    m->nnz = 0;
}

/* growable arrays used while a factor is being built row by row */
typedef struct {
    long long len, cap;
    int *col;
    double *val;
    int *lev;
} orc_rowbuf;

static int rb_push(orc_rowbuf *b, int c, double v, int lev)
{
    if (b->len == b->cap) {
        long long nc = b->cap ? 2 * b->cap : 1024;
        int *nc_col = (int *)realloc(b->col, (size_t)nc * sizeof(int));
        if (!nc_col) return ORC_NOMEM;
        b->col = nc_col;
        double *nv = (double *)realloc(b->val, (size_t)nc * sizeof(double));
        if (!nv) return ORC_NOMEM;
        b->val = nv;
        int *nl = (int *)realloc(b->lev, (size_t)nc * sizeof(int));
        if (!nl) return ORC_NOMEM;
        b->lev = nl;
        b->cap = nc;
    }
    b->col[b->len] = c;
    b->val[b->len] = v;
    b->lev[b->len] = lev;
    b->len++;
    return ORC_OK;
}

static void rb_free(orc_rowbuf *b)
{
    free(b->col);
    free(b->val);
    free(b->lev);
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Insert c into the ascending array a[0..*len) (c not present).  Used for the
 * list of lower-part columns still to be eliminated in the current row. */
static void insert_sorted(int *a, int *len, int c)
{
    int k = *len;
    while (k > 0 && a[k - 1] > c) {
        a[k] = a[k - 1];
        k--;
    }
    a[k] = c;
    (*len)++;
}

/* =========================================================================
 * ILU(k): level-of-fill incomplete LU without pivoting (Section 1 cites
 * Saad's ILU(k); Section 3.1 splits the factorization into a symbolic phase,
 * which fixes the pattern, and a numeric phase on that pattern).
 *
 * Symbolic phase: every stored entry of A has level 0.  Row i is processed by
 * eliminating its lower-part columns k in increasing order; each stored U
 * entry (k,j), j>k, of level lev_kj proposes level lev_ik + lev_kj + 1 for
 * (i,j); the smaller level is kept and an entry enters the pattern only when
 * its level is <= K.  Numeric phase: IKJ Gaussian elimination restricted to
 * that pattern: l_ik = w_ik / u_kk, then w_ij -= l_ik u_kj for every (i,j) in
 * the pattern.  ILU(0) is K = 0 (pattern of A; Table 1's 'nofill').
 *
 * Output: L strictly lower (the unit diagonal is implied), U upper with its
 * diagonal stored first in each row.  A must store every diagonal entry.
 * ========================================================================= */
int orc_iluk(int n, const int *Arp, const int *Acol, const double *Aval, int K,
             orc_csr *L, orc_csr *U, int *bad_row)
{
    int st = ORC_OK;
    orc_rowbuf lb = {0}, ub = {0};
    int *Lrp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *Urp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *lev = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int *touched = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int *low = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int *pos = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    double *w = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int *udiag = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    *bad_row = -1;
    if (!Lrp || !Urp || !lev || !touched || !low || !pos || !w || !udiag) {
        st = ORC_NOMEM;
        goto done;
    }
    for (int j = 0; j < n; j++) {
        lev[j] = INT32_MAX;
        pos[j] = -1;
    }

    /* ---- symbolic phase ---- */
    for (int i = 0; i < n; i++) {
        int nt = 0, nlow = 0, has_diag = 0;
        for (int p = Arp[i]; p < Arp[i + 1]; p++) {
            int j = Acol[p];
            lev[j] = 0;
            touched[nt++] = j;
            if (j < i) low[nlow++] = j; /* A's row is sorted, so low is ascending */
            if (j == i) has_diag = 1;
        }
        if (!has_diag) {
            st = ORC_PATTERN;
            *bad_row = i;
            goto done;
        }
        for (int q = 0; q < nlow; q++) {
            int k = low[q];
            int lik = lev[k];
            /* strict upper part of row k of U: entries after its diagonal */
            for (long long p = (long long)Urp[k] + 1; p < Urp[k + 1]; p++) {
                int j = ub.col[p];
                int nl = lik + ub.lev[p] + 1;
                if (nl > K) continue;
                if (lev[j] == INT32_MAX) {
                    touched[nt++] = j;
                    if (j < i) insert_sorted(low, &nlow, j);
                    lev[j] = nl;
                } else if (nl < lev[j]) {
                    lev[j] = nl;
                }
            }
        }
        qsort(touched, (size_t)nt, sizeof(int), cmp_int);
        for (int t = 0; t < nt; t++) {
            int j = touched[t];
            if (j < i) {
                if ((st = rb_push(&lb, j, 0.0, lev[j]))) goto done;
            } else {
                if ((st = rb_push(&ub, j, 0.0, lev[j]))) goto done;
            }
            lev[j] = INT32_MAX;
        }
        Lrp[i + 1] = (int)lb.len;
        Urp[i + 1] = (int)ub.len;
    }

    /* ---- numeric phase (IKJ on the fixed pattern) ---- */
    for (int i = 0; i < n; i++) {
        /* scatter the pattern of row i and the values of A into w */
        for (long long p = Lrp[i]; p < Lrp[i + 1]; p++) {
            pos[lb.col[p]] = (int)p;
            w[lb.col[p]] = 0.0;
        }
        for (long long p = Urp[i]; p < Urp[i + 1]; p++) {
            pos[ub.col[p]] = (int)p;
            w[ub.col[p]] = 0.0;
        }
        for (int p = Arp[i]; p < Arp[i + 1]; p++) w[Acol[p]] = Aval[p];
        /* eliminate with the lower-part columns in increasing order */
        for (long long p = Lrp[i]; p < Lrp[i + 1]; p++) {
            int k = lb.col[p];
            double lik = w[k] / ub.val[udiag[k]];
            w[k] = lik;
            for (long long q = (long long)Urp[k] + 1; q < Urp[k + 1]; q++) {
                int j = ub.col[q];
                if (pos[j] >= 0) w[j] = w[j] - lik * ub.val[q];
            }
        }
        for (long long p = Lrp[i]; p < Lrp[i + 1]; p++) {
            lb.val[p] = w[lb.col[p]];
            pos[lb.col[p]] = -1;
            w[lb.col[p]] = 0.0;
        }
        for (long long p = Urp[i]; p < Urp[i + 1]; p++) {
            ub.val[p] = w[ub.col[p]];
            pos[ub.col[p]] = -1;
            w[ub.col[p]] = 0.0;
        }
        udiag[i] = Urp[i]; /* the diagonal is the first entry of U's row */
        double piv = ub.val[udiag[i]];
        if (ub.col[udiag[i]] != i) {
            st = ORC_PATTERN;
            *bad_row = i;
            goto done;
        }
        if (piv == 0.0 || !isfinite(piv)) {
            st = ORC_ZERO_PIVOT;
            *bad_row = i;
            goto done;
        }
    }

    L->n = n;
    L->nnz = lb.len;
    L->rp = Lrp;
    L->col = lb.col;
    L->val = lb.val;
    U->n = n;
    U->nnz = ub.len;
    U->rp = Urp;
    U->col = ub.col;
    U->val = ub.val;
    free(lb.lev);
    free(ub.lev);
    Lrp = Urp = NULL;
    lb.col = ub.col = NULL;
    lb.val = ub.val = NULL;
    lb.lev = ub.lev = NULL;
done:
    free(Lrp);
    free(Urp);
    rb_free(&lb);
    rb_free(&ub);
    free(lev);
    free(touched);
    free(low);
    free(pos);
    free(w);
    free(udiag);
    return st;
}

/* =========================================================================
 * ILUT(tau, p): dual-threshold incomplete LU without pivoting, the threshold
 * variant the paper uses with a drop tolerance and a fill limit per row
 * (Sections 4.2 and 6.1; Matlab's ilutp with pivoting off, hypre's ILUT).
 *
 * The paper gives no formula; this follows Saad's row-wise ILUT, with every
 * magnitude measured in the units of A (the reading is documented with the
 * package):
 *   w = a_i*, tau_i = tau * ||a_i*||_2.
 *   For the lower-part columns k of w in increasing order (fill included):
 *     v = w_k; if |v| < tau_i the entry is dropped (w_k = 0, no elimination);
 *     else l_ik = v / u_kk and w_j -= l_ik u_kj for every stored j > k of
 *     U's row k (fill appears where w had no entry).
 *   Upper-part entries j > i with |w_j| < tau_i are dropped.
 *   Of the surviving entries at most p are kept in the L part (largest
 *   |l_ik u_kk| = |v|) and at most p in the U part (largest |w_j|); ties go to
 *   the smaller column.  The diagonal is always kept.
 * ========================================================================= */
typedef struct {
    double key;
    int col;
} orc_cand;

static int cmp_cand(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->col > y->col) - (x->col < y->col);
}

static int cmp_cand_col(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    return (x->col > y->col) - (x->col < y->col);
}

int orc_ilut(int n, const int *Arp, const int *Acol, const double *Aval, double tau, int p,
             orc_csr *L, orc_csr *U, int *bad_row)
{
    int st = ORC_OK;
    orc_rowbuf lb = {0}, ub = {0};
    size_t nn = (size_t)(n > 0 ? n : 1);
    int *Lrp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *Urp = (int *)calloc((size_t)n + 1, sizeof(int));
    double *w = (double *)calloc(nn, sizeof(double));
    double *pre = (double *)calloc(nn, sizeof(double));
    char *in = (char *)calloc(nn, 1);
    char *dropped = (char *)calloc(nn, 1);
    int *touched = (int *)malloc(nn * sizeof(int));
    int *low = (int *)malloc(nn * sizeof(int));
    orc_cand *cand = (orc_cand *)malloc(nn * sizeof(orc_cand));
    *bad_row = -1;
    if (!Lrp || !Urp || !w || !pre || !in || !dropped || !touched || !low || !cand) {
        st = ORC_NOMEM;
        goto done;
    }
    for (int i = 0; i < n; i++) {
        int nt = 0, nlow = 0;
        double nrm2 = 0.0;
        for (int q = Arp[i]; q < Arp[i + 1]; q++) {
            int j = Acol[q];
            w[j] = Aval[q];
            in[j] = 1;
            touched[nt++] = j;
            if (j < i) low[nlow++] = j;
            nrm2 = nrm2 + Aval[q] * Aval[q];
        }
        double tau_i = tau * sqrt(nrm2);
        if (!in[i]) { /* the diagonal position always exists in the row */
            w[i] = 0.0;
            in[i] = 1;
            touched[nt++] = i;
        }
        for (int q = 0; q < nlow; q++) {
            int k = low[q];
            double v = w[k];
            if (fabs(v) < tau_i) {
                w[k] = 0.0;
                dropped[k] = 1;
                continue;
            }
            double lik = v / ub.val[Urp[k]];
            w[k] = lik;
            pre[k] = v;
            for (long long r = (long long)Urp[k] + 1; r < Urp[k + 1]; r++) {
                int j = ub.col[r];
                if (!in[j]) {
                    in[j] = 1;
                    w[j] = 0.0;
                    touched[nt++] = j;
                    if (j < i) insert_sorted(low, &nlow, j);
                }
                w[j] = w[j] - lik * ub.val[r];
            }
        }
        /* L part: surviving multipliers, at most p by |l_ik u_kk| */
        int nc = 0;
        for (int q = 0; q < nlow; q++) {
            int k = low[q];
            if (dropped[k]) continue;
            cand[nc].key = fabs(pre[k]);
            cand[nc].col = k;
            nc++;
        }
        qsort(cand, (size_t)nc, sizeof(orc_cand), cmp_cand);
        if (nc > p) nc = p;
        qsort(cand, (size_t)nc, sizeof(orc_cand), cmp_cand_col);
        for (int q = 0; q < nc; q++)
            if ((st = rb_push(&lb, cand[q].col, w[cand[q].col], 0))) goto done;
        Lrp[i + 1] = (int)lb.len;
        /* U part: diagonal, then at most p off-diagonal entries by |w_j| */
        double piv = w[i];
        if (piv == 0.0 || !isfinite(piv)) {
            st = ORC_ZERO_PIVOT;
            *bad_row = i;
            goto done;
        }
        nc = 0;
        for (int t = 0; t < nt; t++) {
            int j = touched[t];
            if (j <= i) continue;
            if (fabs(w[j]) < tau_i) continue;
            cand[nc].key = fabs(w[j]);
            cand[nc].col = j;
            nc++;
        }
        qsort(cand, (size_t)nc, sizeof(orc_cand), cmp_cand);
        if (nc > p) nc = p;
        qsort(cand, (size_t)nc, sizeof(orc_cand), cmp_cand_col);
        if ((st = rb_push(&ub, i, piv, 0))) goto done;
        for (int q = 0; q < nc; q++)
            if ((st = rb_push(&ub, cand[q].col, w[cand[q].col], 0))) goto done;
        Urp[i + 1] = (int)ub.len;
        for (int t = 0; t < nt; t++) {
            int j = touched[t];
            w[j] = 0.0;
            pre[j] = 0.0;
            in[j] = 0;
            dropped[j] = 0;
        }
    }
    L->n = n;
    L->nnz = lb.len;
    L->rp = Lrp;
    L->col = lb.col;
    L->val = lb.val;
    U->n = n;
    U->nnz = ub.len;
    U->rp = Urp;
    U->col = ub.col;
    U->val = ub.val;
    free(lb.lev);
    free(ub.lev);
    Lrp = Urp = NULL;
    lb.col = ub.col = NULL;
    lb.val = ub.val = NULL;
    lb.lev = ub.lev = NULL;
done:
    free(Lrp);
    free(Urp);
    rb_free(&lb);
    rb_free(&ub);
    free(w);
    free(pre);
    free(in);
    free(dropped);
    free(touched);
    free(low);
    free(cand);
    return st;
}

/* =========================================================================
 * Row scaling of the U factor (Section 5.1, eqs. extractD and newD):
 * D = diag(U), U~ = D^{-1} U.  Writes d_i = u_ii, dinv_i = 1/u_ii and the
 * strictly upper part of U~, u~_ij = u_ij / u_ii (one division per entry).
 * U's diagonal must be the first stored entry of each row.  The output CSR
 * (Us_rp[n+1], Us_col, Us_val with nnz(U)-n entries) is caller-allocated.
 * ========================================================================= */
int orc_scale_rows(int n, const int *Urp, const int *Ucol, const double *Uval,
                   double *d, double *dinv, int *Us_rp, int *Us_col, double *Us_val, int *bad_row)
{
    long long o = 0;
    *bad_row = -1;
    Us_rp[0] = 0;
    for (int i = 0; i < n; i++) {
        if (Urp[i + 1] <= Urp[i] || Ucol[Urp[i]] != i) {
            *bad_row = i;
            return ORC_PATTERN;
        }
        double uii = Uval[Urp[i]];
        if (uii == 0.0 || !isfinite(uii)) {
            *bad_row = i;
            return ORC_ZERO_PIVOT;
        }
        d[i] = uii;
        dinv[i] = 1.0 / uii;
        for (int p = Urp[i] + 1; p < Urp[i + 1]; p++) {
            if (Ucol[p] <= i) {
                *bad_row = i;
                return ORC_PATTERN;
            }
            Us_col[o] = Ucol[p];
            Us_val[o] = Uval[p] / uii;
            o++;
        }
        Us_rp[i + 1] = (int)o;
    }
    return ORC_OK;
}

/* =========================================================================
 * Row/column scaling of the U factor (Section 5.1, eq. rowcolScale:
 * L D_r U D_c x = b, the Richardson iteration running on D_r U D_c, which
 * has a unit diagonal).  The paper names Ruiz scaling (Table 2) without a
 * formula; the reading here: `iters` Ruiz steps on U in the max norm,
 *   r_i = 1/sqrt(max_j |u^_ij|), c_j = 1/sqrt(max_i |u^_ij|),
 *   d_r <- d_r * r, d_c <- d_c * c, with u^_ij = (|u_ij| * d_r,i) * d_c,j,
 * starting from d_r = d_c = 1; then the row factor is replaced so that the
 * diagonal is exactly the unit one the paper requires, d_r,i = 1/(u_ii d_c,i),
 * and the strictly upper part of U^ = D_r U D_c is written,
 * u^_ij = (u_ij * d_r,i) * d_c,j.  Us_rp/col/val as in orc_scale_rows.
 * dr_ruiz (optional, may be NULL) receives the row factors before the
 * unit-diagonal step.
 * ========================================================================= */
int orc_scale_rowcol(int n, const int *Urp, const int *Ucol, const double *Uval, int iters,
                     double *dr, double *dc, double *dr_ruiz, int *Us_rp, int *Us_col, double *Us_val,
                     int *bad_row)
{
    double *cm = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *r = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    *bad_row = -1;
    if (!cm || !r) {
        free(cm);
        free(r);
        return ORC_NOMEM;
    }
    for (int i = 0; i < n; i++) {
        if (Urp[i + 1] <= Urp[i] || Ucol[Urp[i]] != i) {
            *bad_row = i;
            free(cm);
            free(r);
            return ORC_PATTERN;
        }
        double uii = Uval[Urp[i]];
        if (uii == 0.0 || !isfinite(uii)) {
            *bad_row = i;
            free(cm);
            free(r);
            return ORC_ZERO_PIVOT;
        }
        dr[i] = 1.0;
        dc[i] = 1.0;
    }
    for (int it = 0; it < iters; it++) {
        for (int j = 0; j < n; j++) cm[j] = 0.0;
        for (int i = 0; i < n; i++) {
            double rm = 0.0;
            for (int p = Urp[i]; p < Urp[i + 1]; p++) {
                double a = (fabs(Uval[p]) * dr[i]) * dc[Ucol[p]];
                if (a > rm) rm = a;
                if (a > cm[Ucol[p]]) cm[Ucol[p]] = a;
            }
            r[i] = 1.0 / sqrt(rm);
        }
        for (int i = 0; i < n; i++) dr[i] = dr[i] * r[i];
        for (int j = 0; j < n; j++) dc[j] = dc[j] * (1.0 / sqrt(cm[j]));
    }
    if (dr_ruiz)
        for (int i = 0; i < n; i++) dr_ruiz[i] = dr[i];
    long long o = 0;
    Us_rp[0] = 0;
    for (int i = 0; i < n; i++) {
        dr[i] = 1.0 / (Uval[Urp[i]] * dc[i]);
        for (int p = Urp[i] + 1; p < Urp[i + 1]; p++) {
            Us_col[o] = Ucol[p];
            Us_val[o] = (Uval[p] * dr[i]) * dc[Ucol[p]];
            o++;
        }
        Us_rp[i + 1] = (int)o;
    }
    free(cm);
    free(r);
    return ORC_OK;
}

/* y = N x, each row summed from 0.0 in ascending column order. */
void orc_spmv(int n, const int *rp, const int *col, const double *val, const double *x, double *y)
{
    for (int i = 0; i < n; i++) {
        double t = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; p++) t = t + val[p] * x[col[p]];
        y[i] = t;
    }
}

/* Residual r = b - A x (the argument of M^{-1} in eq. ILUsplit). */
void orc_residual(int n, const int *Arp, const int *Acol, const double *Aval,
                  const double *b, const double *x, double *r)
{
    orc_spmv(n, Arp, Acol, Aval, x, r);
    for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
}

/* =========================================================================
 * Richardson iteration for (I + N) y = rhs with N strictly triangular
 * (Algorithm 2's loops; eq. richard; G_L = I - L and G_U = U_s~ in eq.
 * LUiterMat): y_0 = 0 and y_k = rhs - N y_{k-1} for k = 1..m.  After m steps
 * y_m is the m-term truncated Neumann series sum_{j<m} (-N)^j rhs (eqs.
 * Neumann and Neuman); N is nilpotent, so m >= depth(N) gives the exact
 * solution.  The same routine runs the unscaled variant, where N = U - I
 * carries a diagonal.  tmp: caller scratch of n doubles.
 * ========================================================================= */
void orc_richardson(int n, const int *rp, const int *col, const double *val,
                    const double *rhs, int m, double *y, double *tmp)
{
    for (int i = 0; i < n; i++) y[i] = 0.0;
    for (int k = 1; k <= m; k++) {
        orc_spmv(n, rp, col, val, y, tmp);
        for (int i = 0; i < n; i++) y[i] = rhs[i] - tmp[i];
    }
}

/* =========================================================================
 * Direct triangular solve by substitution (Section 4: the sequential solve
 * the iteration replaces).  uplo: 0 = lower (rows in increasing order),
 * 1 = upper (decreasing order).  unit: 1 = the diagonal is taken as 1 and
 * stored diagonal entries are not read; 0 = the diagonal must be stored and
 * the row is divided by it.  out_i = (rhs_i - sum_{j != i} t_ij out_j) [/ t_ii].
 * ========================================================================= */
int orc_trisolve(int n, const int *rp, const int *col, const double *val, int uplo, int unit,
                 const double *rhs, double *out, int *bad_row)
{
    *bad_row = -1;
    for (int s = 0; s < n; s++) {
        int i = uplo == 0 ? s : n - 1 - s;
        double t = 0.0, dii = 0.0;
        int has_d = 0;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            int j = col[p];
            if (j == i) {
                has_d = 1;
                dii = val[p];
                continue;
            }
            if ((uplo == 0 && j > i) || (uplo == 1 && j < i)) {
                *bad_row = i;
                return ORC_PATTERN;
            }
            t = t + val[p] * out[j];
        }
        double v = rhs[i] - t;
        if (!unit) {
            if (!has_d) {
                *bad_row = i;
                return ORC_PATTERN;
            }
            if (dii == 0.0 || !isfinite(dii)) {
                *bad_row = i;
                return ORC_ZERO_PIVOT;
            }
            v = v / dii;
        }
        out[i] = v;
    }
    return ORC_OK;
}

/* =========================================================================
 * The ILU smoother with row-scaled U (eq. ILUsplit with M = L D U~;
 * Algorithm 2), one call = `outer` smoothing steps on x (in/out):
 *   r = b - A x
 *   y = m_L Richardson steps on L y = r            (direct: substitution)
 *   s = D^{-1} y   (dinv_i * y_i)
 *   z = m_U Richardson steps on U~ z = s           (direct: substitution)
 *   x = x + z
 * Ls: strict lower part of L; Us: strict upper part of U~ (scaled).
 * direct = 1 replaces both Richardson loops by exact substitution.
 * ws: caller scratch of 5n doubles.
 * ========================================================================= */
void orc_smooth(int n, const int *Arp, const int *Acol, const double *Aval,
                const int *Lrp, const int *Lcol, const double *Lval,
                const int *Urp, const int *Ucol, const double *Uval, const double *dinv,
                const double *b, double *x, int outer, int mL, int mU, int direct, double *ws)
{
    double *r = ws, *y = ws + n, *s = ws + 2 * (size_t)n, *z = ws + 3 * (size_t)n,
           *tmp = ws + 4 * (size_t)n;
    int bad;
    for (int it = 0; it < outer; it++) {
        orc_residual(n, Arp, Acol, Aval, b, x, r);
        if (direct)
            orc_trisolve(n, Lrp, Lcol, Lval, 0, 1, r, y, &bad);
        else
            orc_richardson(n, Lrp, Lcol, Lval, r, mL, y, tmp);
        for (int i = 0; i < n; i++) s[i] = dinv[i] * y[i];
        if (direct)
            orc_trisolve(n, Urp, Ucol, Uval, 1, 1, s, z, &bad);
        else
            orc_richardson(n, Urp, Ucol, Uval, s, mU, z, tmp);
        for (int i = 0; i < n; i++) x[i] = x[i] + z[i];
    }
}

/* =========================================================================
 * The same smoother step (iterative form only) with the row loops split
 * among OpenMP threads: the residual, every Richardson update and the two
 * vector updates.  A Richardson update reads only the previous iterate, so
 * the rows of one update are independent; each row is still summed from 0.0
 * in ascending column order by one thread, and the result equals orc_smooth
 * bit for bit whatever the thread count.  Used to time the CPU baseline on
 * all host cores (a substitution would not split this way: row i needs the
 * rows before it).  ws: 5n doubles.
 * ========================================================================= */
static void orc_spmv_omp(int n, const int *rp, const int *col, const double *val, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double t = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; p++) t = t + val[p] * x[col[p]];
        y[i] = t;
    }
}

static void orc_richardson_omp(int n, const int *rp, const int *col, const double *val,
                               const double *rhs, int m, double *y, double *tmp)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) y[i] = 0.0;
    for (int k = 1; k <= m; k++) {
        orc_spmv_omp(n, rp, col, val, y, tmp);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++) y[i] = rhs[i] - tmp[i];
    }
}

void orc_smooth_omp(int n, const int *Arp, const int *Acol, const double *Aval,
                    const int *Lrp, const int *Lcol, const double *Lval,
                    const int *Urp, const int *Ucol, const double *Uval, const double *dinv,
                    const double *b, double *x, int outer, int mL, int mU, double *ws)
{
    double *r = ws, *y = ws + n, *s = ws + 2 * (size_t)n, *z = ws + 3 * (size_t)n,
           *tmp = ws + 4 * (size_t)n;
    for (int it = 0; it < outer; it++) {
        orc_spmv_omp(n, Arp, Acol, Aval, x, r);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
        orc_richardson_omp(n, Lrp, Lcol, Lval, r, mL, y, tmp);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++) s[i] = dinv[i] * y[i];
        orc_richardson_omp(n, Urp, Ucol, Uval, s, mU, z, tmp);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++) x[i] = x[i] + z[i];
    }
}

/* Threads orc_smooth_omp uses (OMP_NUM_THREADS, else the host's). */
int orc_omp_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

/* =========================================================================
 * The unscaled variant the paper reports as failing (Section 6.1): plain
 * Richardson (step 1) on U z = y without the row scaling, z_k = y - (U - I)
 * z_{k-1}.  Nu is U - I with the diagonal entry u_ii - 1 stored (built by
 * orc_unit_shift).  ws: 5n doubles.
 * ========================================================================= */
void orc_unit_shift(int n, const int *Urp, const int *Ucol, const double *Uval, double *Nval)
{
    for (int i = 0; i < n; i++)
        for (int p = Urp[i]; p < Urp[i + 1]; p++) Nval[p] = Ucol[p] == i ? Uval[p] - 1.0 : Uval[p];
}

void orc_smooth_unscaled(int n, const int *Arp, const int *Acol, const double *Aval,
                         const int *Lrp, const int *Lcol, const double *Lval,
                         const int *Urp, const int *Ucol, const double *Nval,
                         const double *b, double *x, int outer, int mL, int mU, double *ws)
{
    double *r = ws, *y = ws + n, *z = ws + 3 * (size_t)n, *tmp = ws + 4 * (size_t)n;
    for (int it = 0; it < outer; it++) {
        orc_residual(n, Arp, Acol, Aval, b, x, r);
        orc_richardson(n, Lrp, Lcol, Lval, r, mL, y, tmp);
        orc_richardson(n, Urp, Ucol, Nval, y, mU, z, tmp);
        for (int i = 0; i < n; i++) x[i] = x[i] + z[i];
    }
}

/* =========================================================================
 * Mixed-precision emulation of the smoother: the two Richardson loops run on
 * FP32 copies of the factor values (round to nearest even) with FP32
 * iterates and FP32 accumulation; the residual r = b - A x, the diagonal
 * scaling s = dinv * y and the update of x stay FP64:
 *   r   = b - A x                              (double)
 *   y_0 = 0, y_k = (float)r - Lf y_{k-1}        (float)
 *   s   = (float)(dinv * (double)y_mL)
 *   z_0 = 0, z_k = s - Uf z_{k-1}               (float)
 *   x   = x + (double)z_mU
 * ws: 2n doubles; fws: 4n floats.
 * ========================================================================= */
static void orc_richardson_f32(int n, const int *rp, const int *col, const double *val64,
                               const float *rhs, int m, float *y, float *tmp)
{
    for (int i = 0; i < n; i++) y[i] = 0.0f;
    for (int k = 1; k <= m; k++) {
        for (int i = 0; i < n; i++) {
            float t = 0.0f;
            for (int p = rp[i]; p < rp[i + 1]; p++) t = t + (float)val64[p] * y[col[p]];
            tmp[i] = t;
        }
        for (int i = 0; i < n; i++) y[i] = rhs[i] - tmp[i];
    }
}

void orc_smooth_mixed(int n, const int *Arp, const int *Acol, const double *Aval,
                      const int *Lrp, const int *Lcol, const double *Lval,
                      const int *Urp, const int *Ucol, const double *Uval, const double *dinv,
                      const double *b, double *x, int outer, int mL, int mU, double *ws, float *fws)
{
    double *r = ws;
    float *rf = fws, *y = fws + n, *z = fws + 2 * (size_t)n, *tmp = fws + 3 * (size_t)n;
    for (int it = 0; it < outer; it++) {
        orc_residual(n, Arp, Acol, Aval, b, x, r);
        for (int i = 0; i < n; i++) rf[i] = (float)r[i];
        orc_richardson_f32(n, Lrp, Lcol, Lval, rf, mL, y, tmp);
        for (int i = 0; i < n; i++) rf[i] = (float)(dinv[i] * (double)y[i]);
        orc_richardson_f32(n, Urp, Ucol, Uval, rf, mU, z, tmp);
        for (int i = 0; i < n; i++) x[i] = x[i] + (double)z[i];
    }
}

/* =========================================================================
 * The smoother with row/column-scaled U (eq. rowcolScale): U z = y is solved
 * as U^ v = D_r y, z = D_c v, on U^ = D_r U D_c (unit diagonal; Us holds its
 * strict upper part):
 *   r = b - A x;  y = m_L steps on L y = r;  s = d_r * y;
 *   v = m_U steps on U^ v = s;  x = x + d_c * v.
 * mode 0: FP64 Richardson.  mode 1: the two Richardson loops in FP32 as in
 * orc_smooth_mixed, s = (float)(d_r * (double)y), x = x + d_c * (double)v.
 * mode 2: both solves by substitution.
 * ws: 5n doubles; fws: 4n floats (mode 1 only, else may be NULL).
 * ========================================================================= */
void orc_smooth_rowcol(int n, const int *Arp, const int *Acol, const double *Aval,
                       const int *Lrp, const int *Lcol, const double *Lval,
                       const int *Urp, const int *Ucol, const double *Uval, const double *dr, const double *dc,
                       const double *b, double *x, int outer, int mL, int mU, int mode, double *ws, float *fws)
{
    double *r = ws, *y = ws + n, *s = ws + 2 * (size_t)n, *v = ws + 3 * (size_t)n, *tmp = ws + 4 * (size_t)n;
    int bad;
    for (int it = 0; it < outer; it++) {
        orc_residual(n, Arp, Acol, Aval, b, x, r);
        if (mode == 1) {
            float *rf = fws, *yf = fws + n, *vf = fws + 2 * (size_t)n, *tf = fws + 3 * (size_t)n;
            for (int i = 0; i < n; i++) rf[i] = (float)r[i];
            orc_richardson_f32(n, Lrp, Lcol, Lval, rf, mL, yf, tf);
            for (int i = 0; i < n; i++) rf[i] = (float)(dr[i] * (double)yf[i]);
            orc_richardson_f32(n, Urp, Ucol, Uval, rf, mU, vf, tf);
            for (int i = 0; i < n; i++) x[i] = x[i] + dc[i] * (double)vf[i];
            continue;
        }
        if (mode == 2)
            orc_trisolve(n, Lrp, Lcol, Lval, 0, 1, r, y, &bad);
        else
            orc_richardson(n, Lrp, Lcol, Lval, r, mL, y, tmp);
        for (int i = 0; i < n; i++) s[i] = dr[i] * y[i];
        if (mode == 2)
            orc_trisolve(n, Urp, Ucol, Uval, 1, 1, s, v, &bad);
        else
            orc_richardson(n, Urp, Ucol, Uval, s, mU, v, tmp);
        for (int i = 0; i < n; i++) x[i] = x[i] + dc[i] * v[i];
    }
}

/* =========================================================================
 * ILU(0) by fixed-point sweeps (Section 7 names the fixed-point ILU of Chow
 * and Patel as the way to factor on the GPU).  The unknowns are the entries
 * of L (unit lower, strict part) and U (upper) on the pattern S of A; they
 * satisfy, for every (i,j) in S,
 *   u_ij = a_ij - sum_{k < i} l_ik u_kj            (j >= i)
 *   l_ij = (a_ij - sum_{k < j} l_ik u_kj) / u_jj    (j <  i)
 * with k over the entries (i,k) and (k,j) that are both in S.  A sweep
 * evaluates every equation from the previous sweep's values (synchronous,
 * so the result is independent of the order rows are visited), subtracting
 * the products from a_ij in ascending k -- the order in which the row-wise
 * (IKJ) elimination of orc_iluk applies them, so the fixed point equals that
 * ILU(0) bit for bit.  Initial guess: u_ij = a_ij, l_ij = a_ij / a_jj.
 * LU: values aligned with A's CSR (entry p holds l_ij or u_ij); ws: nnz(A)
 * doubles + n ints.  Returns the number of sweeps after which the values
 * stopped changing (sweeps + 1 if they still changed), or -1 (a row without
 * its diagonal).
 * ========================================================================= */
static int orc_find(const int *rp, const int *col, int row, int c)
{
    int lo = rp[row], hi = rp[row + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

int orc_ilu0_fixed_point(int n, const int *Arp, const int *Acol, const double *Aval, int sweeps, double *LU,
                         double *ws)
{
    const int nnz = Arp[n];
    double *old = ws;
    int *dpos = (int *)(ws + nnz);
    for (int i = 0; i < n; i++) {
        dpos[i] = orc_find(Arp, Acol, i, i);
        if (dpos[i] < 0) return -1;
    }
    for (int i = 0; i < n; i++)
        for (int p = Arp[i]; p < Arp[i + 1]; p++) {
            const int j = Acol[p];
            LU[p] = j < i ? Aval[p] / Aval[dpos[j]] : Aval[p];
        }
    for (int sw = 1; sw <= sweeps; sw++) {
        for (int p = 0; p < nnz; p++) old[p] = LU[p];
        int changed = 0;
        for (int i = 0; i < n; i++)
            for (int p = Arp[i]; p < Arp[i + 1]; p++) {
                const int j = Acol[p];
                const int kmax = j < i ? j : i;
                double s = Aval[p];
                for (int q = Arp[i]; q < Arp[i + 1] && Acol[q] < kmax; q++) {
                    const int pk = orc_find(Arp, Acol, Acol[q], j);
                    if (pk >= 0) s = s - old[q] * old[pk];
                }
                const double v = j < i ? s / old[dpos[j]] : s;
                if (v != old[p]) changed = 1;
                LU[p] = v;
            }
        if (!changed) return sw - 1;
    }
    return sweeps + 1;
}

/* =========================================================================
 * Polynomial Gauss-Seidel smoother (Section 2: the polynomial smoother the
 * ILU smoother is compared with).  Gauss-Seidel's (D + L)^{-1}, with D the
 * diagonal and L the strictly lower part of A, is written (I + D^{-1}L)^{-1}
 * D^{-1} and the inverse replaced by a truncated Neumann series:
 *   x <- x + sum_{j<m} (-D^{-1} L)^j D^{-1} (b - A x)      (m terms).
 * orc_gs_split: Gs = D^{-1} L (strictly lower CSR, g_ij = a_ij / a_ii, one
 * division each; Gs_col/Gs_val need room for nnz(A) entries) and
 * dinv_i = 1 / a_ii.  Errors: PATTERN (a row without its diagonal),
 * ZERO_PIVOT (a_ii == 0 or not finite).
 * ========================================================================= */
int orc_gs_split(int n, const int *Arp, const int *Acol, const double *Aval, int *Gs_rp, int *Gs_col,
                 double *Gs_val, double *dinv, int *bad_row)
{
    int o = 0;
    *bad_row = -1;
    Gs_rp[0] = 0;
    for (int i = 0; i < n; i++) {
        double aii = 0.0;
        int has = 0;
        for (int p = Arp[i]; p < Arp[i + 1]; p++)
            if (Acol[p] == i) {
                aii = Aval[p];
                has = 1;
            }
        if (!has) {
            *bad_row = i;
            return ORC_PATTERN;
        }
        if (aii == 0.0 || !isfinite(aii)) {
            *bad_row = i;
            return ORC_ZERO_PIVOT;
        }
        dinv[i] = 1.0 / aii;
        for (int p = Arp[i]; p < Arp[i + 1]; p++) {
            if (Acol[p] >= i) continue;
            Gs_col[o] = Acol[p];
            Gs_val[o] = Aval[p] / aii;
            o++;
        }
        Gs_rp[i + 1] = o;
    }
    return ORC_OK;
}

/* The smoother, `outer` steps on x (in/out):
 *   r = b - A x;  s = dinv * r;  y = m Richardson steps on (I + Gs) y = s;
 *   x = x + y.
 * mixed = 1: r stays FP64 and is rounded to FP32, s = (float)(dinv *
 * (double)(float)r), the Richardson loop runs in FP32 on FP32 copies of the
 * Gs values (as in orc_smooth_mixed), x = x + (double)y.
 * ws: 3n doubles; fws: 3n floats (mixed only, else may be NULL). */
void orc_gs_smooth(int n, const int *Arp, const int *Acol, const double *Aval, const int *Grp, const int *Gcol,
                   const double *Gval, const double *dinv, const double *b, double *x, int outer, int m, int mixed,
                   double *ws, float *fws)
{
    double *r = ws, *y = ws + n, *tmp = ws + 2 * (size_t)n;
    for (int it = 0; it < outer; it++) {
        orc_residual(n, Arp, Acol, Aval, b, x, r);
        if (mixed) {
            float *sf = fws, *yf = fws + n, *tf = fws + 2 * (size_t)n;
            for (int i = 0; i < n; i++) sf[i] = (float)(dinv[i] * (double)(float)r[i]);
            orc_richardson_f32(n, Grp, Gcol, Gval, sf, m, yf, tf);
            for (int i = 0; i < n; i++) x[i] = x[i] + (double)yf[i];
        } else {
            for (int i = 0; i < n; i++) r[i] = dinv[i] * r[i];
            orc_richardson(n, Grp, Gcol, Gval, r, m, y, tmp);
            for (int i = 0; i < n; i++) x[i] = x[i] + y[i];
        }
    }
}

/* Euclidean norm, summed in index order. */
double orc_nrm2(int n, const double *v)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s = s + v[i] * v[i];
    return sqrt(s);
}

/* =========================================================================
 * Outer convergence: repeat one smoothing step until the relative residual
 * ||b - A x||_2 / ||b||_2 (eq. relres) drops below tol, at most max_outer
 * steps.  mixed = 1 uses the FP32-inner form.  hist[k] receives the relative
 * residual after k steps (hist[0] for the initial x).  Returns the number of
 * steps taken (max_outer + 1 if the tolerance was not reached).
 * ws: 6n doubles; fws: 4n floats.
 * ========================================================================= */
int orc_smooth_until(int n, const int *Arp, const int *Acol, const double *Aval,
                     const int *Lrp, const int *Lcol, const double *Lval,
                     const int *Urp, const int *Ucol, const double *Uval, const double *dinv,
                     const double *b, double *x, int mL, int mU, int mixed, double tol, int max_outer,
                     double *hist, double *ws, float *fws)
{
    double *r = ws + 5 * (size_t)n;
    double nb = orc_nrm2(n, b);
    orc_residual(n, Arp, Acol, Aval, b, x, r);
    hist[0] = orc_nrm2(n, r) / nb;
    if (hist[0] < tol) return 0;
    for (int k = 1; k <= max_outer; k++) {
        if (mixed)
            orc_smooth_mixed(n, Arp, Acol, Aval, Lrp, Lcol, Lval, Urp, Ucol, Uval, dinv, b, x, 1, mL, mU,
                             ws, fws);
        else
            orc_smooth(n, Arp, Acol, Aval, Lrp, Lcol, Lval, Urp, Ucol, Uval, dinv, b, x, 1, mL, mU, 0, ws);
        orc_residual(n, Arp, Acol, Aval, b, x, r);
        hist[k] = orc_nrm2(n, r) / nb;
        if (hist[k] < tol) return k;
    }
    return max_outer + 1;
}

/* =========================================================================
 * FGMRES(m) with the ILU smoother as right preconditioner (Section 6: the
 * paper's Krylov solver is flexible GMRES [Saad03], stopped on the relative
 * residual of eq. relres).  Arnoldi with modified Gram-Schmidt; the small
 * least-squares problem is solved with Givens rotations, whose last entry
 * |g_{j+1}| is the residual norm of the current iterate:
 *   r0 = b - A x0, beta = ||r0||, v1 = r0 / beta, g = beta e1
 *   for j = 1..m:
 *     z_j = M^{-1} v_j            (one smoother call from z = 0: `outer`
 *                                  steps of orc_smooth with m_L, m_U)
 *     w = A z_j
 *     for i = 1..j: h_ij = (w, v_i); w = w - h_ij v_i
 *     h_{j+1,j} = ||w||; v_{j+1} = w / h_{j+1,j}
 *     apply the previous rotations to column j, make the new one, update g
 *     stop when |g_{j+1}| / (||b|| + norm_a ||x_j||) < tol (or h_{j+1,j} == 0)
 *   y = the solution of the triangular system H y = g;  x = x0 + sum_i y_i z_i
 *   restart from x while not converged and fewer than max_iters steps.
 * |g_{j+1}| is the residual norm of the iterate x_j = x0 + Z_j y_j that the
 * first j steps define.  norm_a = 0 gives the relative residual of eq. relres;
 * norm_a = ||A||_2 the norm-wise relative backward error of eq. nbre, whose
 * ||x_j|| is taken from x_j formed explicitly after every step.
 * Dot products and norms are summed in index order.  hist[k] receives the
 * estimate after k steps (hist[0] from the true residual of x0); returns the
 * number of steps taken.  ws: (2m + 8) n + (m + 1)(m + 4) doubles.
 * ========================================================================= */
static double orc_dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

/* y = the solution of the leading j x j upper-triangular block of H (column-
 * major with leading dimension m + 1) against g, by back substitution. */
static void orc_fgmres_solve(int m, int j, const double *H, const double *g, double *y)
{
    for (int i = j - 1; i >= 0; i--) {
        double t = g[i];
        for (int c2 = i + 1; c2 < j; c2++) t = t - H[i + (size_t)(m + 1) * c2] * y[c2];
        y[i] = t / H[i + (size_t)(m + 1) * i];
    }
}

int orc_fgmres(int n, const int *Arp, const int *Acol, const double *Aval,
               const int *Lrp, const int *Lcol, const double *Lval,
               const int *Urp, const int *Ucol, const double *Uval, const double *dinv,
               int outer, int mL, int mU, const double *b, double *x, int m, int max_iters, double tol,
               double norm_a, double *hist, double *ws)
{
    const size_t N = (size_t)n;
    double *V = ws;                          /* (m + 1) n */
    double *Z = V + (size_t)(m + 1) * N;     /* m n */
    double *w = Z + (size_t)m * N;           /* n */
    double *sws = w + N;                     /* 5 n for the smoother */
    double *H = sws + 5 * N;                 /* (m + 1) m, column-major: H[i + (m + 1) j] */
    double *cs = H + (size_t)(m + 1) * m;    /* m */
    double *sn = cs + m;                     /* m */
    double *g = sn + m;                      /* m + 1 */
    double *y = g + m + 1;                   /* m */
    double *xj = y + m;                      /* n: the iterate after each step (norm_a > 0) */
    const double nb = orc_nrm2(n, b);
    int k = 0;
    orc_residual(n, Arp, Acol, Aval, b, x, V);
    double beta = orc_nrm2(n, V);
    hist[0] = beta / (nb + norm_a * orc_nrm2(n, x));
    if (!(hist[0] >= tol)) return 0;
    while (k < max_iters) {
        for (int i = 0; i < n; i++) V[i] = V[i] / beta;
        for (int i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        int j = 0, done = 0;
        for (; j < m && k < max_iters; j++) {
            double *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N, *vn = V + (size_t)(j + 1) * N;
            for (int i = 0; i < n; i++) zj[i] = 0.0;
            orc_smooth(n, Arp, Acol, Aval, Lrp, Lcol, Lval, Urp, Ucol, Uval, dinv, vj, zj, outer, mL, mU, 0, sws);
            orc_spmv(n, Arp, Acol, Aval, zj, w);
            double *h = H + (size_t)(m + 1) * j;
            for (int i = 0; i <= j; i++) {
                const double *vi = V + (size_t)i * N;
                h[i] = orc_dot(n, w, vi);
                for (int t = 0; t < n; t++) w[t] = w[t] - h[i] * vi[t];
            }
            h[j + 1] = orc_nrm2(n, w);
            if (h[j + 1] != 0.0)
                for (int t = 0; t < n; t++) vn[t] = w[t] / h[j + 1];
            /* previous rotations, then the new one */
            for (int i = 0; i < j; i++) {
                const double a = h[i], c = h[i + 1];
                h[i] = cs[i] * a + sn[i] * c;
                h[i + 1] = -sn[i] * a + cs[i] * c;
            }
            const double den = sqrt(h[j] * h[j] + h[j + 1] * h[j + 1]);
            cs[j] = h[j] / den;
            sn[j] = h[j + 1] / den;
            h[j] = den;
            h[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k++;
            double xn = 0.0;
            if (norm_a > 0.0) {
                /* x_j = x0 + Z y from the first j + 1 columns of H and g */
                orc_fgmres_solve(m, j + 1, H, g, y);
                for (int t = 0; t < n; t++) xj[t] = x[t];
                for (int i = 0; i <= j; i++) {
                    const double *zi = Z + (size_t)i * N;
                    for (int t = 0; t < n; t++) xj[t] = xj[t] + y[i] * zi[t];
                }
                xn = orc_nrm2(n, xj);
            }
            hist[k] = fabs(g[j + 1]) / (nb + norm_a * xn);
            if (hist[k] < tol || den == 0.0) {
                done = 1;
                j++;
                break;
            }
        }
        /* y = H^{-1} g (upper triangular, j x j), x = x + Z y */
        orc_fgmres_solve(m, j, H, g, y);
        for (int i = 0; i < j; i++) {
            const double *zi = Z + (size_t)i * N;
            for (int t = 0; t < n; t++) x[t] = x[t] + y[i] * zi[t];
        }
        if (done) break;
        orc_residual(n, Arp, Acol, Aval, b, x, V);
        beta = orc_nrm2(n, V);
    }
    return k;
}

/* =========================================================================
 * Level sets of a triangular factor's elimination DAG (Section 4: level-set
 * scheduling).  level_i = 0 when row i depends on no other row, else
 * 1 + max level of the rows it reads.  uplo 0: lower (j < i), 1: upper.
 * Diagonal entries are ignored.  Returns the depth (number of levels), or -1
 * on an entry on the wrong side.
 * ========================================================================= */
int orc_levels(int n, const int *rp, const int *col, int uplo, int *level)
{
    int depth = 0;
    for (int s = 0; s < n; s++) {
        int i = uplo == 0 ? s : n - 1 - s;
        int lv = 0;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            int j = col[p];
            if (j == i) continue;
            if ((uplo == 0 && j > i) || (uplo == 1 && j < i)) return -1;
            if (level[j] + 1 > lv) lv = level[j] + 1;
        }
        level[i] = lv;
        if (lv + 1 > depth) depth = lv + 1;
    }
    return depth;
}

/* =========================================================================
 * Henrici's departure from normality (Section 4.1, eq. depB),
 * dep(T) = sqrt(||T||_F^2 - ||Lambda||_F^2).  For a triangular T the
 * eigenvalues are its diagonal entries, so dep(T) = ||T - diag(T)||_F; with
 * no off-diagonal entries it is 0 (eq. diagDep).  Entries are summed in
 * storage order.
 * ========================================================================= */
double orc_dep_triangular(int n, const int *rp, const int *col, const double *val)
{
    double s = 0.0;
    for (int i = 0; i < n; i++)
        for (int p = rp[i]; p < rp[i + 1]; p++)
            if (col[p] != i) s = s + val[p] * val[p];
    return sqrt(s);
}
