/*
 * oracle.c -- plain, slow, exact CPU oracle for the (min,+) power method of
 * Martinez, Garzon and Puertas, "Powers of large matrices on GPU platforms to
 * compute the Roman domination number of cylindrical graphs" (arXiv 2409.17658).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, import or
 * call this file: it exists so that the tests, the smoke check and the CPU
 * baseline of the benchmark can check the HIP library against an independent
 * definition.  It shares no source with the HIP library.
 *
 * Arithmetic: every value is an exact int64.  A missing arc / infinite entry
 * is the sentinel ORACLE_INF and is never added: each sum below is guarded by
 * an explicit finiteness test, so no wrap-around can occur.
 *
 * Letters of a column word: a=0 (label 2), b=1 (label 1), c=2 (label 0,
 * dominated in its own or the previous column), d=3 (label 0, not yet
 * dominated) -- Section 4.1, the labelling list before Remark 3.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF INT64_MAX
#define LA 0
#define LB 1
#define LC 2
#define LD 3

int64_t oracle_inf(void) { return ORACLE_INF; }

/* ------------------------------------------------------------------ */
/* Definition 4: a correct word contains none of ad, da, ab, ba, bb.   */
/* ------------------------------------------------------------------ */
static int bad_adjacent(int x, int y)
{
    if (x == LA && y == LD) return 1; /* ad */
    if (x == LD && y == LA) return 1; /* da */
    if (x == LA && y == LB) return 1; /* ab */
    if (x == LB && y == LA) return 1; /* ba */
    if (x == LB && y == LB) return 1; /* bb */
    return 0;
}

/*
 * Enumerate every word of length m over {a,b,c,d} in increasing base-4 order
 * (row 1 is the most significant letter) and keep the correct ones.  The
 * state index of a word is its rank in this order.  Returns the number of
 * correct words; when out != NULL the letters are written there, m per word.
 */
int64_t oracle_words(int m, uint8_t *out)
{
    if (m < 1 || m > 12) return -1;
    int64_t total = 1;
    for (int i = 0; i < m; i++) total *= 4;
    int64_t count = 0;
    uint8_t w[16];
    for (int64_t code = 0; code < total; code++) {
        for (int i = 0; i < m; i++) w[i] = (uint8_t)((code >> (2 * (m - 1 - i))) & 3);
        int ok = 1;
        for (int i = 0; i + 1 < m; i++)
            if (bad_adjacent(w[i], w[i + 1])) ok = 0;
        if (!ok) continue;
        if (out) memcpy(out + count * m, w, (size_t)m);
        count++;
    }
    return count;
}

/* ------------------------------------------------------------------ */
/* "p can follow q" (Section 4.1, the three rule lists for the first,  */
/* intermediate and last rows).                                        */
/* ------------------------------------------------------------------ */
/*
 * One row of the rule lists.  nb_a says whether a vertical neighbour of p_i
 * inside the new column carries the letter a (p_2 for the first row,
 * p_{i-1} or p_{i+1} for an intermediate row, p_{m-1} for the last row; a
 * neighbour that does not exist is not an a).  The intermediate-row list
 * prints "p_1 = d" where p_i = d is meant; this follows the first- and
 * last-row lists, which say p_1 = d and p_m = d for their own row.
 */
static int row_rule(int qi, int pi, int nb_a)
{
    switch (qi) {
    case LA: /* q_i = a: p_i = a or p_i = c */
        return pi == LA || pi == LC;
    case LB: /* q_i = b: (p_i = c and a vertical a) or p_i = d */
        return (pi == LC && nb_a) || pi == LD;
    case LC: /* q_i = c: p_i = a, b, d, or (c and a vertical a) */
        return pi == LA || pi == LB || (pi == LC && nb_a) || pi == LD;
    default: /* q_i = d: p_i = a */
        return pi == LA;
    }
}

int oracle_follows(const uint8_t *q, const uint8_t *p, int m)
{
    for (int i = 0; i < m; i++) {
        int nb_a = 0;
        if (i > 0 && p[i - 1] == LA) nb_a = 1;
        if (i + 1 < m && p[i + 1] == LA) nb_a = 1;
        if (!row_rule(q[i], p[i], nb_a)) return 0;
    }
    return 1;
}

/* Label of the arc q->p: 2 p(a) + p(b), the weight of the new column. */
static int64_t column_weight(const uint8_t *p, int m)
{
    int64_t w = 0;
    for (int i = 0; i < m; i++) {
        if (p[i] == LA) w += 2;
        if (p[i] == LB) w += 1;
    }
    return w;
}

/*
 * Corollary 7's matrix A(G): row q (previous column), column p (next column);
 * entry = 2 p(a) + p(b) when p can follow q, infinite otherwise.
 * A must hold count*count int64 values, count = oracle_words(m, NULL).
 */
int oracle_transfer(int m, int64_t *A)
{
    int64_t n = oracle_words(m, NULL);
    if (n < 0) return -1;
    uint8_t *w = (uint8_t *)malloc((size_t)(n * m));
    if (!w) return -2;
    oracle_words(m, w);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < n; qi++) {
        for (int64_t pi = 0; pi < n; pi++) {
            const uint8_t *q = w + qi * m, *p = w + pi * m;
            A[qi * n + pi] = oracle_follows(q, p, m) ? column_weight(p, m) : ORACLE_INF;
        }
    }
    free(w);
    return 0;
}

/* ------------------------------------------------------------------ */
/* (min,+) product, Section 3: c_ij = min_k (x_ik + y_kj), taken over  */
/* the k for which both entries are finite; infinite if there is none. */
/* ------------------------------------------------------------------ */
/* The same product with Y given by its finite entries only, row by row:
 * row k of Y holds the values val[t] in the columns col[t] for
 * start[k] <= t < start[k + 1]; every other entry of Y is infinite.
 * Skipping infinite entries is the definition's "over the k for which both
 * entries are finite", nothing more. */
int oracle_minplus_rows(int64_t M, int64_t K, int64_t N, const int64_t *X,
                        const int64_t *start, const int32_t *col, const int64_t *val, int64_t *C)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; i++) {
        int64_t *c = C + i * N;
        for (int64_t j = 0; j < N; j++) c[j] = ORACLE_INF;
        for (int64_t k = 0; k < K; k++) {
            int64_t x = X[i * K + k];
            if (x == ORACLE_INF) continue;
            for (int64_t t = start[k]; t < start[k + 1]; t++) {
                int64_t s = x + val[t];
                if (s < c[col[t]]) c[col[t]] = s;
            }
        }
    }
    return 0;
}

int oracle_minplus(int64_t M, int64_t K, int64_t N,
                   const int64_t *X, const int64_t *Y, int64_t *C)
{
    /* The finite entries of each row of Y, listed once. */
    int64_t *start = (int64_t *)malloc((size_t)(K + 1) * sizeof(int64_t));
    if (!start) return -2;
    start[0] = 0;
    for (int64_t k = 0; k < K; k++) {
        int64_t c = 0;
        for (int64_t j = 0; j < N; j++)
            if (Y[k * N + j] != ORACLE_INF) c++;
        start[k + 1] = start[k] + c;
    }
    const size_t nnz = (size_t)(start[K] > 0 ? start[K] : 1);
    int32_t *col = (int32_t *)malloc(nnz * sizeof(int32_t));
    int64_t *val = (int64_t *)malloc(nnz * sizeof(int64_t));
    if (!col || !val) { free(col); free(val); free(start); return -2; }
    for (int64_t k = 0; k < K; k++) {
        int64_t t = start[k];
        for (int64_t j = 0; j < N; j++)
            if (Y[k * N + j] != ORACLE_INF) {
                col[t] = (int32_t)j;
                val[t++] = Y[k * N + j];
            }
    }
    int rc = oracle_minplus_rows(M, K, N, X, start, col, val, C);
    free(val);
    free(col);
    free(start);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Row-min normalisation (canonical form of a power): r_i = min of the */
/* finite entries of row i, N_ij = C_ij - r_i, infinite entries stay   */
/* infinite; an all-infinite row gets r_i = ORACLE_INF ("none").       */
/* In place on C.                                                      */
/* ------------------------------------------------------------------ */
void oracle_normalise(int64_t M, int64_t N, int64_t *C, int64_t *r)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; i++) {
        int64_t mn = ORACLE_INF;
        for (int64_t j = 0; j < N; j++)
            if (C[i * N + j] < mn) mn = C[i * N + j];
        r[i] = mn;
        if (mn == ORACLE_INF) continue;
        for (int64_t j = 0; j < N; j++)
            if (C[i * N + j] != ORACLE_INF) C[i * N + j] -= mn;
    }
}

/*
 * Product of two powers kept in canonical form, X = Ra (+) Na and
 * Y = Rb (+) Nb (row offsets added to every finite entry of the row).
 * By the scalar rule of Section 3, (alpha (x) Y) pulls out of a product, so
 * with s = min_l Rb[l]:  X (x) Y = Ra + s + (Na (x) B'),  where
 * B'[l][j] = Nb[l][j] + (Rb[l] - s).  The result is normalised.
 */
int oracle_product_of_powers(int64_t n,
                             const int64_t *Na, const int64_t *Ra,
                             const int64_t *Nb, const int64_t *Rb,
                             int64_t *Nc, int64_t *Rc)
{
    int64_t s = ORACLE_INF;
    for (int64_t l = 0; l < n; l++)
        if (Rb[l] < s) s = Rb[l];
    int64_t *Bp = (int64_t *)malloc((size_t)(n * n) * sizeof(int64_t));
    int64_t *r = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!Bp || !r) { free(Bp); free(r); return -2; }
    for (int64_t l = 0; l < n; l++)
        for (int64_t j = 0; j < n; j++) {
            int64_t b = Nb[l * n + j];
            Bp[l * n + j] = (b == ORACLE_INF || Rb[l] == ORACLE_INF) ? ORACLE_INF : b + (Rb[l] - s);
        }
    int rc = oracle_minplus(n, n, n, Na, Bp, Nc);
    if (rc == 0) {
        oracle_normalise(n, n, Nc, r);
        for (int64_t i = 0; i < n; i++)
            Rc[i] = (Ra[i] == ORACLE_INF || r[i] == ORACLE_INF || s == ORACLE_INF)
                        ? ORACLE_INF : Ra[i] + s + r[i];
    }
    free(Bp);
    free(r);
    return rc;
}

/* Corollary 7: gamma = min_p (A^n)_pp = min_i (R_i + N_ii) over finite terms. */
int64_t oracle_trace(int64_t n, const int64_t *N, const int64_t *R)
{
    int64_t g = ORACLE_INF;
    for (int64_t i = 0; i < n; i++) {
        if (R[i] == ORACLE_INF || N[i * n + i] == ORACLE_INF) continue;
        int64_t v = R[i] + N[i * n + i];
        if (v < g) g = v;
    }
    return g;
}

/* ------------------------------------------------------------------ */
/* Independent checks of gamma_R(P_m x C_n), no word encoding at all.  */
/* ------------------------------------------------------------------ */

/*
 * Exhaustive search over all f: V -> {0,1,2} of the cylinder (m rows that
 * are cycles of length n, columns are paths; Section 4.1's encoding).
 * f is a Roman dominating function when every vertex with f = 0 has a
 * neighbour with f = 2 (Section 1).  Returns the minimum weight.
 * Feasible for m*n <= 16.
 */
int64_t oracle_brute_gamma(int m, int n)
{
    int V = m * n;
    if (m < 1 || n < 3 || V > 18) return -1;
    int64_t total = 1;
    for (int v = 0; v < V; v++) total *= 3;
    int64_t best = ORACLE_INF;
    uint8_t f[32];
#pragma omp parallel for schedule(static) private(f) reduction(min : best)
    for (int64_t code = 0; code < total; code++) {
        int64_t c = code, w = 0;
        for (int v = 0; v < V; v++) { f[v] = (uint8_t)(c % 3); c /= 3; w += f[v]; }
        if (w >= best) continue;
        int ok = 1;
        for (int i = 0; i < m && ok; i++)
            for (int j = 0; j < n && ok; j++) {
                if (f[i * n + j] != 0) continue;
                int dom = 0;
                if (f[i * n + (j + 1) % n] == 2) dom = 1;
                if (f[i * n + (j + n - 1) % n] == 2) dom = 1;
                if (i > 0 && f[(i - 1) * n + j] == 2) dom = 1;
                if (i + 1 < m && f[(i + 1) * n + j] == 2) dom = 1;
                if (!dom) ok = 0;
            }
        if (ok && w < best) best = w;
    }
    return best;
}

/*
 * Exact dynamic programme along the path P_m instead of the cycle: process
 * the rows (each a cycle C_n) one at a time.  State after row i: which
 * vertices of row i carry 2, and which zeros of row i are still undominated
 * (only the vertex below can still dominate them).  Cost ~ m * 9^n.
 */
int64_t oracle_rowdp_gamma(int m, int n)
{
    if (m < 1 || n < 3 || n > 9) return -1;
    int64_t L = 1;
    for (int j = 0; j < n; j++) L *= 3;
    int S = 1 << (2 * n); /* state = twos | (pending << n) */
    uint32_t *two = (uint32_t *)malloc((size_t)L * sizeof(uint32_t));
    uint32_t *zero = (uint32_t *)malloc((size_t)L * sizeof(uint32_t));
    uint32_t *self = (uint32_t *)malloc((size_t)L * sizeof(uint32_t));
    int32_t *wt = (int32_t *)malloc((size_t)L * sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc((size_t)S * sizeof(int64_t));
    int64_t *nxt = (int64_t *)malloc((size_t)S * sizeof(int64_t));
    if (!two || !zero || !self || !wt || !cur || !nxt) return -2;
    for (int64_t lab = 0; lab < L; lab++) {
        int64_t c = lab;
        uint32_t t = 0, z = 0;
        int32_t w = 0;
        for (int j = 0; j < n; j++) {
            int v = (int)(c % 3);
            c /= 3;
            if (v == 2) t |= 1u << j;
            if (v == 0) z |= 1u << j;
            w += v;
        }
        uint32_t s = 0; /* zeros dominated by a 2 next to them in the row */
        for (int j = 0; j < n; j++)
            if ((z >> j) & 1u)
                if (((t >> ((j + 1) % n)) & 1u) || ((t >> ((j + n - 1) % n)) & 1u)) s |= 1u << j;
        two[lab] = t; zero[lab] = z; self[lab] = s; wt[lab] = w;
    }
    for (int s = 0; s < S; s++) cur[s] = ORACLE_INF;
    for (int64_t lab = 0; lab < L; lab++) {
        uint32_t pend = zero[lab] & ~self[lab];
        int st = (int)(two[lab] | (pend << n));
        if (wt[lab] < cur[st]) cur[st] = wt[lab];
    }
    uint32_t full = (1u << n) - 1u;
    for (int row = 1; row < m; row++) {
        for (int s = 0; s < S; s++) nxt[s] = ORACLE_INF;
#pragma omp parallel
        {
            /* each thread keeps its own copy of the next row's table */
            int64_t *loc = (int64_t *)malloc((size_t)S * sizeof(int64_t));
            for (int s = 0; s < S; s++) loc[s] = ORACLE_INF;
#pragma omp for schedule(dynamic, 64)
            for (int64_t lab = 0; lab < L; lab++) {
                for (int s = 0; s < S; s++) {
                    if (cur[s] == ORACLE_INF) continue;
                    uint32_t t_prev = (uint32_t)s & full, pend_prev = ((uint32_t)s >> n) & full;
                    if (pend_prev & ~two[lab]) continue; /* a pending zero above needs a 2 below */
                    uint32_t pend = zero[lab] & ~self[lab] & ~t_prev;
                    int st = (int)(two[lab] | (pend << n));
                    int64_t v = cur[s] + wt[lab];
                    if (v < loc[st]) loc[st] = v;
                }
            }
#pragma omp critical
            for (int s = 0; s < S; s++)
                if (loc[s] < nxt[s]) nxt[s] = loc[s];
            free(loc);
        }
        int64_t *tmp = cur; cur = nxt; nxt = tmp;
    }
    int64_t best = ORACLE_INF;
    for (int s = 0; s < S; s++)
        if ((((uint32_t)s >> n) & full) == 0 && cur[s] < best) best = cur[s];
    free(two); free(zero); free(self); free(wt); free(cur); free(nxt);
    return best;
}

/* ------------------------------------------------------------------ */
/* Entry-wise forms for parity checks at sizes where a whole product   */
/* is too slow for the host.                                           */
/* ------------------------------------------------------------------ */

/* out[t] = (X (x) Y)[i[t]][j[t]] = min_k X[i][k] + Y[k][j] (finite k only).
 * X is rows x K (row stride K), Y is K x N (row stride N). */
void oracle_minplus_at(int64_t K, int64_t N, const int64_t *X, const int64_t *Y,
                       const int64_t *ii, const int64_t *jj, int64_t count, int64_t *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < count; t++) {
        int64_t best = ORACLE_INF;
        for (int64_t k = 0; k < K; k++) {
            int64_t x = X[ii[t] * K + k], y = Y[k * N + jj[t]];
            if (x == ORACLE_INF || y == ORACLE_INF) continue;
            if (x + y < best) best = x + y;
        }
        out[t] = best;
    }
}

/* Rows rows[0..count-1] of A(G) (Corollary 7), count x C_m values. */
int oracle_transfer_rows(int m, const int64_t *rows, int64_t count, int64_t *out)
{
    int64_t n = oracle_words(m, NULL);
    if (n < 0) return -1;
    uint8_t *w = (uint8_t *)malloc((size_t)(n * m));
    if (!w) return -2;
    oracle_words(m, w);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < count; t++)
        for (int64_t pi = 0; pi < n; pi++) {
            const uint8_t *q = w + rows[t] * m, *p = w + pi * m;
            out[t * n + pi] = oracle_follows(q, p, m) ? column_weight(p, m) : ORACLE_INF;
        }
    free(w);
    return 0;
}

/* A(G) of Corollary 7 by its finite entries (the arcs), row by row, for
 * sizes whose dense matrix would not fit: the same double loop over (q, p)
 * and the same rule and weight as oracle_transfer.  First call with
 * col == NULL: count[q] = number of p that can follow q.  Second call with
 * start[q] = sum of the counts before q: the columns p (ascending) and the
 * weights of row q go to col / val from start[q] on. */
int oracle_transfer_arcs(int m, int64_t *count, const int64_t *start, int32_t *col, int64_t *val)
{
    int64_t n = oracle_words(m, NULL);
    if (n < 0) return -1;
    uint8_t *w = (uint8_t *)malloc((size_t)(n * m));
    if (!w) return -2;
    oracle_words(m, w);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < n; qi++) {
        int64_t t = col ? start[qi] : 0;
        for (int64_t pi = 0; pi < n; pi++) {
            const uint8_t *q = w + qi * m, *p = w + pi * m;
            if (!oracle_follows(q, p, m)) continue;
            if (col) {
                col[t] = (int32_t)pi;
                val[t] = column_weight(p, m);
            }
            t++;
        }
        if (!col) count[qi] = t;
    }
    free(w);
    return 0;
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the OpenMP loops above use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Border ("loss") matrix of the appendix (proof of Lemma 10).         */
/* ------------------------------------------------------------------ */

/* Last-row rule of the border version: the m-th row need not be
 * dominated, so after q_m = d every label the other cases allow is
 * allowed.  (The printed q_m = b case says "p_3 = d"; read p_m = d, as in
 * the main text.) */
static int last_row_rule_border(int qm, int pm, int nb_a)
{
    if (qm == LD) return pm == LA || pm == LB || (pm == LC && nb_a) || pm == LD;
    return row_rule(qm, pm, nb_a);
}

int oracle_follows_border(const uint8_t *q, const uint8_t *p, int m)
{
    for (int i = 0; i < m; i++) {
        int nb_a = 0;
        if (i > 0 && p[i - 1] == LA) nb_a = 1;
        if (i + 1 < m && p[i + 1] == LA) nb_a = 1;
        int ok = (i == m - 1) ? last_row_rule_border(q[i], p[i], nb_a) : row_rule(q[i], p[i], nb_a);
        if (!ok) return 0;
    }
    return 1;
}

/* Algorithm 3: newly dominated vertices nd(q, p), rows 1..m, then one more
 * when p_m = a (the vertex below the border, outside it, is dominated). */
int64_t oracle_newly_dominated(const uint8_t *q, const uint8_t *p, int m)
{
    int64_t nd = 0;
    for (int i = 0; i < m; i++) {
        int qi = q[i], pi = p[i];
        if (qi == LA && pi == LA) nd += 1;
        else if (qi == LB && pi == LC) nd += 1;
        else if (qi == LC && pi == LA) nd += 2;
        else if ((qi == LC || qi == LD) && (pi == LB || pi == LC)) nd += 1;
        else if (qi == LD && pi == LA) nd += 3;
    }
    if (p[m - 1] == LA) nd += 1;
    return nd;
}

/* Border matrix: label 10 p(a) + 5 p(b) - 2 nd(q, p) on arcs, else
 * infinite.  Entries may be negative. */
int oracle_border_transfer(int m, int64_t *A)
{
    int64_t n = oracle_words(m, NULL);
    if (n < 0) return -1;
    uint8_t *w = (uint8_t *)malloc((size_t)(n * m));
    if (!w) return -2;
    oracle_words(m, w);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < n; qi++)
        for (int64_t pi = 0; pi < n; pi++) {
            const uint8_t *q = w + qi * m, *p = w + pi * m;
            int64_t v = ORACLE_INF;
            if (oracle_follows_border(q, p, m)) {
                int64_t na = 0, nb = 0;
                for (int i = 0; i < m; i++) { na += p[i] == LA; nb += p[i] == LB; }
                v = 10 * na + 5 * nb - 2 * oracle_newly_dominated(q, p, m);
            }
            A[qi * n + pi] = v;
        }
    free(w);
    return 0;
}

/*
 * Exhaustive minimum of 5 g(P_m x C_n) - 2 |D(g)| over almost Roman
 * dominating functions g of the border strip (Definition 14): every zero
 * outside the m-th row has a neighbour with 2; D(g) = R1 u N[R2] taken in
 * the larger cylinder, so a 2 in the m-th row also dominates the vertex
 * below the strip.  Feasible for m*n <= 20.
 */
int64_t oracle_brute_border_loss(int m, int n)
{
    int V = m * n;
    if (m < 1 || n < 3 || V > 20) return INT64_MIN;
    int64_t total = 1;
    for (int v = 0; v < V; v++) total *= 3;
    int64_t best = ORACLE_INF;
#pragma omp parallel for schedule(static) reduction(min : best)
    for (int64_t code = 0; code < total; code++) {
        uint8_t f[32];
        int64_t c = code, g = 0;
        for (int v = 0; v < V; v++) { f[v] = (uint8_t)(c % 3); c /= 3; g += f[v]; }
        int ok = 1;
        int64_t D = 0;
        for (int i = 0; i < m; i++)
            for (int j = 0; j < n; j++) {
                int nb2 = 0;
                if (f[i * n + (j + 1) % n] == 2) nb2 = 1;
                if (f[i * n + (j + n - 1) % n] == 2) nb2 = 1;
                if (i > 0 && f[(i - 1) * n + j] == 2) nb2 = 1;
                if (i + 1 < m && f[(i + 1) * n + j] == 2) nb2 = 1;
                int v = f[i * n + j];
                if (v == 0 && !nb2 && i < m - 1) ok = 0;
                if (v > 0 || nb2) D++;
                if (i == m - 1 && v == 2) D++; /* the vertex below the strip */
            }
        if (!ok) continue;
        int64_t loss = 5 * g - 2 * D;
        if (loss < best) best = loss;
    }
    return best;
}
