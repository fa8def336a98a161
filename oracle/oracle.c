/*
 * oracle.c -- plain, slow, single-threaded CPU reference for the assignment
 * and integer transportation problems.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP solver.
 *
 * What it computes (problem statement, Eq. (1) of the paper):
 *   transport:  min <C, X>  s.t.  X 1 = r,  X^T 1 = c,  X >= 0 integer
 *   assignment: the special case r = c = 1 (n = m), i.e.
 *               OPT(C) = min over permutations s of sum_i C[i, s(i)].
 *
 * The exact optimum has a plain definition, so the oracle is an exact
 * algorithm of a different family than the GPU path: the classical
 * Kuhn-Munkres method in its O(n^3) shortest-augmenting-path form (one new
 * row per stage, Dijkstra-like growth of a single alternating tree).  The
 * transport case reduces to assignment by giving every supply/demand unit its
 * own vertex (the S = sum r unit expansion the paper uses for the
 * Gabow-Tarjan transportation bound, Section 2.3.1), solving, and summing
 * the unit plan back onto bins.
 *
 * All arithmetic is exact in int64.  Every function returns 0 on success or a
 * negative code for invalid input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL (-1)
#define ORC_EUNBALANCED (-3)
#define ORC_ENEGMASS (-4)
#define ORC_ENOMEM (-6)

static const int64_t BIG = INT64_MAX / 4;

/* ------------------------------------------------------------------------- */
/* Assignment: shortest-augmenting-path Kuhn-Munkres (Kuhn 1955, Munkres 1957) */
/* ------------------------------------------------------------------------- */
/*
 * Duals start at zero (a feasible start for any C since we only ever raise a
 * row potential or lower a column potential by the smallest slack).  Rows
 * are added one at a time.  For the new root row r we grow one alternating
 * tree: `dist[j]` is the smallest reduced cost C[i][j] - u[i] - v[j] from any
 * tree row i to column j, `via[j]` the row attaining it.  Each step settles
 * the unsettled column with the smallest dist (ties -> smaller index), shifts
 * the duals by that amount so the column becomes tight while every tree edge
 * stays tight, and either stops (column unowned: augmenting path found) or
 * adds the column's owner row to the tree.  Then the path is flipped.
 */
int oracle_assign(const int32_t *C, int32_t n, int32_t *plan, int64_t *u_out, int64_t *v_out,
                  int64_t *cost_out)
{
    if (!C || n <= 0) return ORC_EINVAL;
    int64_t *u = calloc((size_t)n, sizeof *u);
    int64_t *v = calloc((size_t)n, sizeof *v);
    int64_t *dist = malloc((size_t)n * sizeof *dist);
    int32_t *via = malloc((size_t)n * sizeof *via);
    int32_t *owner = malloc((size_t)n * sizeof *owner);   /* column -> row, -1 free */
    int32_t *colof = malloc((size_t)n * sizeof *colof);   /* row -> column, -1 free */
    int32_t *tree = malloc((size_t)n * sizeof *tree);     /* rows in the current tree */
    unsigned char *settled = malloc((size_t)n);
    int rc = 0;
    if (!u || !v || !dist || !via || !owner || !colof || !tree || !settled) { rc = ORC_ENOMEM; goto out; }
    for (int32_t j = 0; j < n; ++j) owner[j] = -1;
    for (int32_t i = 0; i < n; ++i) colof[i] = -1;

    for (int32_t r = 0; r < n; ++r) {
        for (int32_t j = 0; j < n; ++j) { dist[j] = BIG; via[j] = -1; settled[j] = 0; }
        int32_t ntree = 0;
        tree[ntree++] = r;
        int32_t newest = r;     /* the row whose edges have not been relaxed yet */
        int32_t end = -1;       /* the free column that ends the augmenting path */
        for (;;) {
            const int32_t *Crow = C + (size_t)newest * (size_t)n;
            for (int32_t j = 0; j < n; ++j) {
                if (settled[j]) continue;
                int64_t s = (int64_t)Crow[j] - u[newest] - v[j];
                if (s < dist[j]) { dist[j] = s; via[j] = newest; }
            }
            int32_t best = -1;
            for (int32_t j = 0; j < n; ++j)
                if (!settled[j] && (best < 0 || dist[j] < dist[best])) best = j;
            int64_t delta = dist[best];
            for (int32_t t = 0; t < ntree; ++t) u[tree[t]] += delta;
            for (int32_t j = 0; j < n; ++j) {
                if (settled[j]) v[j] -= delta;
                else dist[j] -= delta;
            }
            settled[best] = 1;
            if (owner[best] < 0) { end = best; break; }
            newest = owner[best];
            tree[ntree++] = newest;
        }
        /* flip the path: every row on it takes the column it was reached through */
        for (int32_t j = end;;) {
            int32_t i = via[j];
            int32_t before = colof[i];
            owner[j] = i;
            colof[i] = j;
            if (i == r) break;
            j = before;
        }
    }

    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i) total += C[(size_t)i * (size_t)n + (size_t)colof[i]];
    if (plan) memcpy(plan, colof, (size_t)n * sizeof *plan);
    if (u_out) memcpy(u_out, u, (size_t)n * sizeof *u);
    if (v_out) memcpy(v_out, v, (size_t)n * sizeof *v);
    if (cost_out) *cost_out = total;
out:
    free(u); free(v); free(dist); free(via); free(owner); free(colof); free(tree); free(settled);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Brute force over all n! permutations (n <= 10)                             */
/* ------------------------------------------------------------------------- */
/* Depth-first enumeration of injective row -> column maps.  Returns the
 * minimum cost and how many permutations attain it. */
static void bf_rec(const int32_t *C, int32_t n, int32_t i, unsigned used, int64_t acc,
                   int64_t *best, int64_t *count)
{
    if (i == n) {
        if (acc < *best) { *best = acc; *count = 1; }
        else if (acc == *best) { *count += 1; }
        return;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (used & (1u << j)) continue;
        bf_rec(C, n, i + 1, used | (1u << j), acc + C[(size_t)i * (size_t)n + (size_t)j], best, count);
    }
}

int oracle_brute_force(const int32_t *C, int32_t n, int64_t *best, int64_t *num_optimal)
{
    if (!C || n <= 0 || n > 10 || !best) return ORC_EINVAL;
    int64_t b = INT64_MAX, cnt = 0;
    bf_rec(C, n, 0, 0u, 0, &b, &cnt);
    *best = b;
    if (num_optimal) *num_optimal = cnt;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* LP-duality certificate for the assignment problem                         */
/* ------------------------------------------------------------------------- */
/*
 * Returns 0 when (plan, u, v) is a proof of optimality:
 *   1  plan is a permutation of 0..n-1
 *   2  u_i + v_j <= C_ij for every (i, j)            (dual feasibility)
 *   3  u_i + v_plan(i) == C_i,plan(i) for every i     (complementary slackness)
 *   4  sum_i C_i,plan(i) == sum u + sum v             (equal objectives)
 * By weak duality 1-3 already imply optimality; 4 catches overflow.
 * The return value names the first condition that fails.
 */
int oracle_certify_assign(const int32_t *C, int32_t n, const int32_t *plan, const int64_t *u,
                          const int64_t *v)
{
    if (!C || n <= 0 || !plan || !u || !v) return ORC_EINVAL;
    unsigned char *seen = calloc((size_t)n, 1);
    if (!seen) return ORC_ENOMEM;
    for (int32_t i = 0; i < n; ++i) {
        if (plan[i] < 0 || plan[i] >= n || seen[plan[i]]) { free(seen); return 1; }
        seen[plan[i]] = 1;
    }
    free(seen);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            if (u[i] + v[j] > (int64_t)C[(size_t)i * (size_t)n + (size_t)j]) return 2;
    int64_t primal = 0, dual = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t cij = C[(size_t)i * (size_t)n + (size_t)plan[i]];
        if (u[i] + v[plan[i]] != cij) return 3;
        primal += cij;
        dual += u[i] + v[i];
    }
    return primal == dual ? 0 : 4;
}

/* ------------------------------------------------------------------------- */
/* Integer transportation by unit expansion                                  */
/* ------------------------------------------------------------------------- */
/*
 * Row bin i with mass r_i becomes r_i unit rows, column bin j with mass c_j
 * becomes c_j unit columns (zero-mass bins get no units).  The S x S unit
 * problem is solved exactly, and X[i][j] counts the unit pairs matched
 * between bins i and j.  Bin duals: every copy of a bin carries the same
 * dual in an optimal unit solution (two copies i, i' of one row bin see the
 * same costs, so feasibility against each other's partner forces u_i <= u_i'
 * and u_i' <= u_i), so a bin takes its first copy's dual.  Zero-mass bins
 * have no copy; they get the tightest feasible value: a zero-mass row takes
 * min over columns with mass of C_ij - v_j, then a zero-mass column takes
 * min over all rows of C_ij - u_i.
 */
int oracle_transport(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m,
                     int32_t *X, int64_t *u_out, int64_t *v_out, int64_t *cost_out)
{
    if (!C || !r || !c || n <= 0 || m <= 0) return ORC_EINVAL;
    int64_t sr = 0, sc = 0;
    for (int32_t i = 0; i < n; ++i) { if (r[i] < 0) return ORC_ENEGMASS; sr += r[i]; }
    for (int32_t j = 0; j < m; ++j) { if (c[j] < 0) return ORC_ENEGMASS; sc += c[j]; }
    if (sr != sc || sr < 1) return ORC_EUNBALANCED;
    if (sr > 46340) return ORC_EINVAL; /* S*S must stay addressable in int32 units */
    int32_t S = (int32_t)sr;
    int32_t *rowbin = malloc((size_t)S * sizeof *rowbin);
    int32_t *colbin = malloc((size_t)S * sizeof *colbin);
    int32_t *Cx = malloc((size_t)S * (size_t)S * sizeof *Cx);
    int32_t *px = malloc((size_t)S * sizeof *px);
    int64_t *U = malloc((size_t)S * sizeof *U);
    int64_t *V = malloc((size_t)S * sizeof *V);
    int64_t *ub = malloc((size_t)n * sizeof *ub);
    int64_t *vb = malloc((size_t)m * sizeof *vb);
    int rc = 0;
    if (!rowbin || !colbin || !Cx || !px || !U || !V || !ub || !vb) { rc = ORC_ENOMEM; goto out; }
    {
        int32_t a = 0;
        for (int32_t i = 0; i < n; ++i) for (int32_t k = 0; k < r[i]; ++k) rowbin[a++] = i;
        a = 0;
        for (int32_t j = 0; j < m; ++j) for (int32_t k = 0; k < c[j]; ++k) colbin[a++] = j;
    }
    for (int32_t a = 0; a < S; ++a)
        for (int32_t b = 0; b < S; ++b)
            Cx[(size_t)a * (size_t)S + (size_t)b] = C[(size_t)rowbin[a] * (size_t)m + (size_t)colbin[b]];
    rc = oracle_assign(Cx, S, px, U, V, NULL);
    if (rc) goto out;

    if (X) memset(X, 0, (size_t)n * (size_t)m * sizeof *X);
    int64_t total = 0;
    for (int32_t a = 0; a < S; ++a) {
        int32_t i = rowbin[a], j = colbin[px[a]];
        if (X) X[(size_t)i * (size_t)m + (size_t)j] += 1;
        total += C[(size_t)i * (size_t)m + (size_t)j];
    }
    for (int32_t i = 0; i < n; ++i) ub[i] = 0;
    for (int32_t j = 0; j < m; ++j) vb[j] = 0;
    for (int32_t a = S - 1; a >= 0; --a) ub[rowbin[a]] = U[a];   /* ends on the first copy */
    for (int32_t b = S - 1; b >= 0; --b) vb[colbin[b]] = V[b];
    for (int32_t i = 0; i < n; ++i) {
        if (r[i] > 0) continue;
        int64_t best = BIG;
        for (int32_t j = 0; j < m; ++j) {
            if (c[j] == 0) continue;
            int64_t s = (int64_t)C[(size_t)i * (size_t)m + (size_t)j] - vb[j];
            if (s < best) best = s;
        }
        ub[i] = best;
    }
    for (int32_t j = 0; j < m; ++j) {
        if (c[j] > 0) continue;
        int64_t best = BIG;
        for (int32_t i = 0; i < n; ++i) {
            int64_t s = (int64_t)C[(size_t)i * (size_t)m + (size_t)j] - ub[i];
            if (s < best) best = s;
        }
        vb[j] = best;
    }
    if (u_out) memcpy(u_out, ub, (size_t)n * sizeof *ub);
    if (v_out) memcpy(v_out, vb, (size_t)m * sizeof *vb);
    if (cost_out) *cost_out = total;
out:
    free(rowbin); free(colbin); free(Cx); free(px); free(U); free(V); free(ub); free(vb);
    return rc;
}

/*
 * Transport certificate.  Returns 0 when:
 *   1  X >= 0
 *   2  row sums of X equal r and column sums equal c
 *   3  u_i + v_j <= C_ij everywhere
 *   4  u_i + v_j == C_ij wherever X_ij > 0
 *   5  sum C X == sum r u + sum c v
 */
int oracle_certify_transport(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n,
                             int32_t m, const int32_t *X, const int64_t *u, const int64_t *v)
{
    if (!C || !r || !c || !X || !u || !v || n <= 0 || m <= 0) return ORC_EINVAL;
    int64_t *colsum = calloc((size_t)m, sizeof *colsum);
    if (!colsum) return ORC_ENOMEM;
    int64_t primal = 0, dual = 0;
    int rc = 0;
    for (int32_t i = 0; i < n && !rc; ++i) {
        int64_t rs = 0;
        for (int32_t j = 0; j < m; ++j) {
            int64_t x = X[(size_t)i * (size_t)m + (size_t)j];
            int64_t cij = C[(size_t)i * (size_t)m + (size_t)j];
            if (x < 0) { rc = 1; break; }
            rs += x;
            colsum[j] += x;
            primal += cij * x;
            if (u[i] + v[j] > cij) { rc = 3; break; }
            if (x > 0 && u[i] + v[j] != cij) { rc = 4; break; }
        }
        if (!rc && rs != r[i]) rc = 2;
    }
    for (int32_t j = 0; j < m && !rc; ++j)
        if (colsum[j] != c[j]) rc = 2;
    free(colsum);
    if (rc) return rc;
    for (int32_t i = 0; i < n; ++i) dual += (int64_t)r[i] * u[i];
    for (int32_t j = 0; j < m; ++j) dual += (int64_t)c[j] * v[j];
    return primal == dual ? 0 : 5;
}
