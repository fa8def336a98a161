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
 * Rectangular matrices (n != m, unit masses) are solved by the same
 * shortest-augmenting-path method over the longer side (oracle_assign_rect).
 *
 * oracle_auction is the auction algorithm with epsilon-scaling (Section
 * 2.3.3), one bidder at a time, in exact integer arithmetic; its pins are the
 * KM oracle's optimal cost, brute force and the paper's n * eps bound.
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
 *
 * The core takes n rows and m >= n columns (C row-major with stride m); the
 * square problem is m = n.  On return every row is matched (colof), and the
 * columns that were never matched still have v_j = 0.
 */
static int sap_rows_le_cols(const int32_t *C, int32_t n, int32_t m, int32_t *colof,
                             int64_t *u, int64_t *v)
{
    int64_t *dist = malloc((size_t)m * sizeof *dist);
    int32_t *via = malloc((size_t)m * sizeof *via);
    int32_t *owner = malloc((size_t)m * sizeof *owner);
    int32_t *tree = malloc((size_t)n * sizeof *tree);
    unsigned char *settled = malloc((size_t)m);
    int rc = 0;
    if (!dist || !via || !owner || !tree || !settled) { rc = ORC_ENOMEM; goto out; }
    for (int32_t i = 0; i < n; ++i) { colof[i] = -1; u[i] = 0; }
    for (int32_t j = 0; j < m; ++j) { owner[j] = -1; v[j] = 0; }

    for (int32_t r = 0; r < n; ++r) {
        for (int32_t j = 0; j < m; ++j) { dist[j] = BIG; via[j] = -1; settled[j] = 0; }
        int32_t ntree = 0;
        tree[ntree++] = r;
        int32_t newest = r;
        int32_t end = -1;
        for (;;) {
            const int32_t *Crow = C + (size_t)newest * (size_t)m;
            for (int32_t j = 0; j < m; ++j) {
                if (settled[j]) continue;
                int64_t s = (int64_t)Crow[j] - u[newest] - v[j];
                if (s < dist[j]) { dist[j] = s; via[j] = newest; }
            }
            int32_t best = -1;
            for (int32_t j = 0; j < m; ++j)
                if (!settled[j] && (best < 0 || dist[j] < dist[best])) best = j;
            int64_t delta = dist[best];
            for (int32_t t = 0; t < ntree; ++t) u[tree[t]] += delta;
            for (int32_t j = 0; j < m; ++j) {
                if (settled[j]) v[j] -= delta;
                else dist[j] -= delta;
            }
            settled[best] = 1;
            if (owner[best] < 0) { end = best; break; }
            newest = owner[best];
            tree[ntree++] = newest;
        }
        for (int32_t j = end;;) {
            int32_t i = via[j];
            int32_t before = colof[i];
            owner[j] = i;
            colof[i] = j;
            if (i == r) break;
            j = before;
        }
    }
out:
    free(dist); free(via); free(owner); free(tree); free(settled);
    return rc;
}

int oracle_assign(const int32_t *C, int32_t n, int32_t *plan, int64_t *u_out, int64_t *v_out,
                  int64_t *cost_out)
{
    if (!C || n <= 0) return ORC_EINVAL;
    int32_t *colof = malloc((size_t)n * sizeof *colof);
    int64_t *u = malloc((size_t)n * sizeof *u);
    int64_t *v = malloc((size_t)n * sizeof *v);
    int rc = (!colof || !u || !v) ? ORC_ENOMEM : sap_rows_le_cols(C, n, n, colof, u, v);
    if (!rc) {
        int64_t total = 0;
        for (int32_t i = 0; i < n; ++i) total += C[(size_t)i * (size_t)n + (size_t)colof[i]];
        if (plan) memcpy(plan, colof, (size_t)n * sizeof *plan);
        if (u_out) memcpy(u_out, u, (size_t)n * sizeof *u);
        if (v_out) memcpy(v_out, v, (size_t)n * sizeof *v);
        if (cost_out) *cost_out = total;
    }
    free(colof); free(u); free(v);
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

/* ------------------------------------------------------------------------- */
/* Transport on bins: successive shortest paths (no unit expansion)          */
/* ------------------------------------------------------------------------- */
/*
 * Eq. (1) as a min-cost flow: source -> row bin i (capacity r_i), row i ->
 * column bin j (unbounded, cost C_ij), column j -> sink (capacity c_j), the
 * textbook successive-shortest-path method with potentials.  The potentials
 * are the LP duals u (rows) and v (columns); they start at the reduction
 * u_i = min_j C_ij, v_j = min_i (C_ij - u_i), which is feasible.
 *
 * Each stage runs Dijkstra on reduced costs from every row that still has
 * supply: a row reaches column j at cost C_ij - u_i - v_j >= 0, and a column
 * reaches back, at cost 0, every row that already ships to it (the residual
 * arc of a positive flow, which is tight).  The first column settled that
 * still has demand ends the stage at distance D.  Every settled row gains
 * D - dist and every settled column loses D - dist: the duals stay feasible
 * and the whole path becomes tight.  The path then ships the largest amount
 * it can: the root's supply left, the end's demand left, and the flow on
 * every backward arc.  When all supply has shipped, flows sit on tight edges
 * only, so X and (u, v) are both optimal.  Zero-mass bins get the convention
 * of oracle_transport.  Masses may sum to 2^31 - 1.
 */
int oracle_transport_ssp(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m,
                         int32_t *X, int64_t *u_out, int64_t *v_out, int64_t *cost_out)
{
    if (!C || !r || !c || !X || n <= 0 || m <= 0) return ORC_EINVAL;
    int64_t sr = 0, sc = 0;
    for (int32_t i = 0; i < n; ++i) { if (r[i] < 0) return ORC_ENEGMASS; sr += r[i]; }
    for (int32_t j = 0; j < m; ++j) { if (c[j] < 0) return ORC_ENEGMASS; sc += c[j]; }
    if (sr != sc || sr < 1) return ORC_EUNBALANCED;
    if (sr > INT32_MAX) return ORC_EINVAL;
    const size_t N = (size_t)n, M = (size_t)m;
    int64_t *u = malloc(N * sizeof *u), *v = malloc(M * sizeof *v);
    int64_t *rs = malloc(N * sizeof *rs), *rd = malloc(M * sizeof *rd);
    int64_t *dr = malloc(N * sizeof *dr), *dc = malloc(M * sizeof *dc);
    char *sr_done = malloc(N), *sc_done = malloc(M);
    int32_t *pr = malloc(N * sizeof *pr), *pc = malloc(M * sizeof *pc);
    int rc = 0;
    if (!u || !v || !rs || !rd || !dr || !dc || !sr_done || !sc_done || !pr || !pc) { rc = ORC_ENOMEM; goto out; }
    memset(X, 0, N * M * sizeof *X);
    for (int32_t i = 0; i < n; ++i) {
        int64_t mn = BIG;
        for (int32_t j = 0; j < m; ++j) if (C[(size_t)i * M + (size_t)j] < mn) mn = C[(size_t)i * M + (size_t)j];
        u[i] = mn;
        rs[i] = r[i];
    }
    for (int32_t j = 0; j < m; ++j) {
        int64_t mn = BIG;
        for (int32_t i = 0; i < n; ++i) {
            int64_t s = (int64_t)C[(size_t)i * M + (size_t)j] - u[i];
            if (s < mn) mn = s;
        }
        v[j] = mn;
        rd[j] = c[j];
    }
    for (int64_t left = sr; left > 0;) {
        for (int32_t i = 0; i < n; ++i) { dr[i] = rs[i] > 0 ? 0 : BIG; sr_done[i] = 0; pr[i] = -1; }
        for (int32_t j = 0; j < m; ++j) { dc[j] = BIG; sc_done[j] = 0; pc[j] = -1; }
        int32_t end = -1;
        int64_t D = 0;
        for (;;) {
            /* the unsettled vertex of smallest distance (rows before columns on a tie) */
            int32_t bi = -1, bj = -1;
            int64_t best = BIG;
            for (int32_t i = 0; i < n; ++i) if (!sr_done[i] && dr[i] < best) { best = dr[i]; bi = i; }
            for (int32_t j = 0; j < m; ++j) if (!sc_done[j] && dc[j] < best) { best = dc[j]; bj = j; bi = -1; }
            if (bi < 0 && bj < 0) { rc = ORC_EINVAL; goto out; } /* unreachable when balanced */
            if (bi >= 0) {
                sr_done[bi] = 1;
                const int32_t *Crow = C + (size_t)bi * M;
                for (int32_t j = 0; j < m; ++j) {
                    if (sc_done[j]) continue;
                    int64_t d = dr[bi] + (int64_t)Crow[j] - u[bi] - v[j];
                    if (d < dc[j]) { dc[j] = d; pc[j] = bi; }
                }
            } else {
                sc_done[bj] = 1;
                if (rd[bj] > 0) { end = bj; D = dc[bj]; break; }
                for (int32_t i = 0; i < n; ++i) {
                    if (sr_done[i] || X[(size_t)i * M + (size_t)bj] == 0) continue;
                    if (dc[bj] < dr[i]) { dr[i] = dc[bj]; pr[i] = bj; }
                }
            }
        }
        for (int32_t i = 0; i < n; ++i) if (sr_done[i]) u[i] += D - dr[i];
        for (int32_t j = 0; j < m; ++j) if (sc_done[j]) v[j] -= D - dc[j];
        /* bottleneck along end <- row <- column <- row ... <- root */
        int64_t amt = rd[end];
        for (int32_t i = pc[end];;) {
            if (pr[i] < 0) { if (rs[i] < amt) amt = rs[i]; break; }
            int32_t j = pr[i];
            if (X[(size_t)i * M + (size_t)j] < amt) amt = X[(size_t)i * M + (size_t)j];
            i = pc[j];
        }
        rd[end] -= amt;
        X[(size_t)pc[end] * M + (size_t)end] += (int32_t)amt;
        for (int32_t i = pc[end];;) {
            if (pr[i] < 0) { rs[i] -= amt; break; }
            int32_t j = pr[i];
            X[(size_t)i * M + (size_t)j] -= (int32_t)amt;
            i = pc[j];
            X[(size_t)i * M + (size_t)j] += (int32_t)amt;
        }
        left -= amt;
    }
    {
        int64_t total = 0;
        for (size_t k = 0; k < N * M; ++k) total += (int64_t)C[k] * X[k];
        for (int32_t i = 0; i < n; ++i) {
            if (r[i] > 0) continue;
            int64_t best = BIG;
            for (int32_t j = 0; j < m; ++j) {
                if (c[j] == 0) continue;
                int64_t s = (int64_t)C[(size_t)i * M + (size_t)j] - v[j];
                if (s < best) best = s;
            }
            u[i] = best;
        }
        for (int32_t j = 0; j < m; ++j) {
            if (c[j] > 0) continue;
            int64_t best = BIG;
            for (int32_t i = 0; i < n; ++i) {
                int64_t s = (int64_t)C[(size_t)i * M + (size_t)j] - u[i];
                if (s < best) best = s;
            }
            v[j] = best;
        }
        if (u_out) memcpy(u_out, u, N * sizeof *u);
        if (v_out) memcpy(v_out, v, M * sizeof *v);
        if (cost_out) *cost_out = total;
    }
out:
    free(u); free(v); free(rs); free(rd); free(dr); free(dc); free(sr_done); free(sc_done); free(pr); free(pc);
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

/* ------------------------------------------------------------------------- */
/* Rectangular assignment (n x m, n != m allowed)                             */
/* ------------------------------------------------------------------------- */
/*
 * Eq. (1) is stated for an n x m cost matrix; with unit masses and n != m it
 * is not balanced, and the reading taken here is the usual one: the smaller
 * side is matched completely, every vertex of the larger side at most once,
 * at minimum total cost.
 *
 * For n <= m this is the shortest-augmenting-path core above over all m
 * columns.  A column's dual is lowered only while
 * it is settled inside a tree, and every settled column except the path's end
 * is matched, so duals start at 0, columns never matched keep v_j = 0 and all
 * v_j <= 0: exactly the dual of the rectangular LP (rows = 1, columns <= 1).
 *
 * For n > m the problem is solved on the transpose (columns become the rows
 * that must all be matched) and the answer is read back: plan[i] = -1 for the
 * n - m rows left unmatched; u and v swap roles (u_i <= 0, u_i = 0 when row i
 * is unmatched).
 */
int oracle_assign_rect(const int32_t *C, int32_t n, int32_t m, int32_t *plan, int64_t *u_out,
                       int64_t *v_out, int64_t *cost_out)
{
    if (!C || n <= 0 || m <= 0 || !plan || !u_out || !v_out || !cost_out) return ORC_EINVAL;
    int rc = 0;
    if (n <= m) {
        rc = sap_rows_le_cols(C, n, m, plan, u_out, v_out);
    } else {
        int32_t *CT = malloc((size_t)n * (size_t)m * sizeof *CT);
        int32_t *rowof = malloc((size_t)m * sizeof *rowof);   /* column -> row */
        if (!CT || !rowof) { free(CT); free(rowof); return ORC_ENOMEM; }
        for (int32_t i = 0; i < n; ++i)
            for (int32_t j = 0; j < m; ++j)
                CT[(size_t)j * (size_t)n + (size_t)i] = C[(size_t)i * (size_t)m + (size_t)j];
        rc = sap_rows_le_cols(CT, m, n, rowof, v_out, u_out);
        if (!rc) {
            for (int32_t i = 0; i < n; ++i) plan[i] = -1;
            for (int32_t j = 0; j < m; ++j) plan[rowof[j]] = j;
        }
        free(CT); free(rowof);
    }
    if (rc) return rc;
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i)
        if (plan[i] >= 0) total += C[(size_t)i * (size_t)m + (size_t)plan[i]];
    *cost_out = total;
    return 0;
}

/*
 * Certificate of the rectangular LP.  With k = min(n, m), the primal is
 * min sum C x over x >= 0 with every vertex of the smaller side covered
 * exactly once and every vertex of the larger side at most once; its dual
 * maximises sum u + sum v subject to u_i + v_j <= C_ij, with the potentials
 * of the larger side <= 0.  Returns 0 when:
 *   1  plan matches k distinct pairs, covering the smaller side (plan[i] = -1
 *      marks an unmatched row, allowed only when n > m)
 *   2  u_i + v_j <= C_ij everywhere
 *   3  equality on every matched pair
 *   4  larger-side potentials are <= 0, and == 0 where unmatched
 *   5  sum of matched costs == sum u + sum v
 * 1-4 imply optimality by weak duality; 5 catches overflow.
 */
int oracle_certify_rect(const int32_t *C, int32_t n, int32_t m, const int32_t *plan,
                        const int64_t *u, const int64_t *v)
{
    if (!C || n <= 0 || m <= 0 || !plan || !u || !v) return ORC_EINVAL;
    unsigned char *seen = calloc((size_t)m, 1);
    if (!seen) return ORC_ENOMEM;
    int32_t matched = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t j = plan[i];
        if (j == -1 && n > m) continue;
        if (j < 0 || j >= m || seen[j]) { free(seen); return 1; }
        seen[j] = 1;
        ++matched;
    }
    if (matched != (n < m ? n : m)) { free(seen); return 1; }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < m; ++j)
            if (u[i] + v[j] > (int64_t)C[(size_t)i * (size_t)m + (size_t)j]) { free(seen); return 2; }
    int64_t primal = 0, dual = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (plan[i] < 0) continue;
        int64_t cij = C[(size_t)i * (size_t)m + (size_t)plan[i]];
        if (u[i] + v[plan[i]] != cij) { free(seen); return 3; }
        primal += cij;
    }
    if (n <= m) {
        for (int32_t j = 0; j < m; ++j)
            if (v[j] > 0 || (!seen[j] && v[j] != 0)) { free(seen); return 4; }
    } else {
        for (int32_t i = 0; i < n; ++i)
            if (u[i] > 0 || (plan[i] < 0 && u[i] != 0)) { free(seen); return 4; }
    }
    free(seen);
    for (int32_t i = 0; i < n; ++i) dual += u[i];
    for (int32_t j = 0; j < m; ++j) dual += v[j];
    return primal == dual ? 0 : 5;
}

/* ------------------------------------------------------------------------- */
/* Sparse assignment on a bipartite graph given in CSR                         */
/* ------------------------------------------------------------------------- */
/*
 * Rows 0..n-1 and columns 0..m-1 with n <= m; row i's edges are the columns
 * idx[ptr[i] .. ptr[i+1]) with costs cst[...] (a column at most once per row).
 * Minimise the total cost over matchings that cover every row using edges of
 * the graph only: Eq. (1) with unit masses on a cost graph where missing
 * entries are not allowed (the sparse, possibly rectangular form of the
 * problem).  The LP's dual maximises sum u + sum v subject to u_i + v_j <= c_e
 * on every edge e = (i, j) and v_j <= 0.
 *
 * Same shortest-augmenting-path method as sap_rows_le_cols, one new row per
 * stage; a tree row relaxes only its own edges, so a column that no tree
 * edge reaches keeps dist = BIG.  When every unsettled column has dist = BIG
 * the tree cannot grow and holds a free column nowhere: its rows have fewer
 * neighbours than rows (Hall's condition fails) and no matching covers all
 * rows: ORC_EINFEASIBLE.  Duals start at zero and column duals only fall
 * after their column is settled; the first step of a stage may lower the new
 * root's u below zero (its edges can be cheaper than anything so far), and
 * every later step has delta >= 0, so v_j <= 0 and columns never matched keep
 * v_j = 0.
 */
#define ORC_EINFEASIBLE (-10)

static int sparse_validate(const int64_t *ptr, const int32_t *idx, int32_t n, int32_t m)
{
    if (ptr[0] != 0) return ORC_EINVAL;
    int32_t *mark = malloc((size_t)m * sizeof *mark);
    if (!mark) return ORC_ENOMEM;
    for (int32_t j = 0; j < m; ++j) mark[j] = -1;
    int rc = 0;
    for (int32_t i = 0; i < n && !rc; ++i) {
        if (ptr[i + 1] < ptr[i]) { rc = ORC_EINVAL; break; }
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            int32_t j = idx[e];
            if (j < 0 || j >= m || mark[j] == i) { rc = ORC_EINVAL; break; }
            mark[j] = i;
        }
    }
    free(mark);
    return rc;
}

int oracle_assign_sparse(const int64_t *ptr, const int32_t *idx, const int32_t *cst, int32_t n,
                         int32_t m, int32_t *plan, int64_t *u, int64_t *v, int64_t *cost_out)
{
    if (!ptr || !plan || !u || !v || !cost_out || n <= 0 || m < n) return ORC_EINVAL;
    if (ptr[n] > 0 && (!idx || !cst)) return ORC_EINVAL;
    int rc = sparse_validate(ptr, idx, n, m);
    if (rc) return rc;
    int64_t *dist = malloc((size_t)m * sizeof *dist);
    int32_t *via = malloc((size_t)m * sizeof *via);
    int32_t *owner = malloc((size_t)m * sizeof *owner);
    int32_t *trow = malloc((size_t)n * sizeof *trow);
    unsigned char *done = malloc((size_t)m);
    if (!dist || !via || !owner || !trow || !done) { rc = ORC_ENOMEM; goto out; }
    for (int32_t i = 0; i < n; ++i) { plan[i] = -1; u[i] = 0; }
    for (int32_t j = 0; j < m; ++j) { owner[j] = -1; v[j] = 0; }

    for (int32_t r = 0; r < n && !rc; ++r) {
        for (int32_t j = 0; j < m; ++j) { dist[j] = BIG; via[j] = -1; done[j] = 0; }
        int32_t ntree = 0;
        trow[ntree++] = r;
        int32_t newest = r;
        int32_t end = -1;
        for (;;) {
            for (int64_t e = ptr[newest]; e < ptr[newest + 1]; ++e) {
                int32_t j = idx[e];
                if (done[j]) continue;
                int64_t s = (int64_t)cst[e] - u[newest] - v[j];
                if (s < dist[j]) { dist[j] = s; via[j] = newest; }
            }
            int32_t best = -1;
            for (int32_t j = 0; j < m; ++j)
                if (!done[j] && dist[j] < BIG && (best < 0 || dist[j] < dist[best])) best = j;
            if (best < 0) { rc = ORC_EINFEASIBLE; break; }
            int64_t delta = dist[best];
            for (int32_t t = 0; t < ntree; ++t) u[trow[t]] += delta;
            for (int32_t j = 0; j < m; ++j) {
                if (done[j]) v[j] -= delta;
                else if (dist[j] < BIG) dist[j] -= delta;
            }
            done[best] = 1;
            if (owner[best] < 0) { end = best; break; }
            newest = owner[best];
            trow[ntree++] = newest;
        }
        if (rc) break;
        for (int32_t j = end;;) {
            int32_t i = via[j];
            int32_t before = plan[i];
            owner[j] = i;
            plan[i] = j;
            if (i == r) break;
            j = before;
        }
    }
    if (!rc) {
        int64_t total = 0;
        for (int32_t i = 0; i < n; ++i)
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
                if (idx[e] == plan[i]) total += cst[e];
        *cost_out = total;
    }
out:
    free(dist); free(via); free(owner); free(trow); free(done);
    return rc;
}

/*
 * Certificate of the sparse LP above.  Returns 0 when:
 *   1  plan maps the rows to distinct columns, each along an edge of its row
 *   2  u_i + v_j <= c_e on every edge
 *   3  equality on every matched edge
 *   4  v_j <= 0, and v_j == 0 on columns left unmatched
 *   5  sum of matched costs == sum u + sum v
 * 1-4 give optimality by weak duality; 5 catches overflow.
 */
int oracle_certify_sparse(const int64_t *ptr, const int32_t *idx, const int32_t *cst, int32_t n,
                          int32_t m, const int32_t *plan, const int64_t *u, const int64_t *v)
{
    if (!ptr || !plan || !u || !v || n <= 0 || m < n) return ORC_EINVAL;
    unsigned char *seen = calloc((size_t)m, 1);
    if (!seen) return ORC_ENOMEM;
    int64_t primal = 0, dual = 0;
    int rc = 0;
    for (int32_t i = 0; i < n && !rc; ++i) {
        int32_t j = plan[i];
        if (j < 0 || j >= m || seen[j]) { rc = 1; break; }
        seen[j] = 1;
        int found = 0;
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            if (u[i] + v[idx[e]] > (int64_t)cst[e]) { rc = 2; break; }
            if (idx[e] == j) {
                found = 1;
                if (u[i] + v[j] != (int64_t)cst[e]) { rc = 3; break; }
                primal += cst[e];
            }
        }
        if (!rc && !found) rc = 1;
    }
    for (int32_t j = 0; j < m && !rc; ++j)
        if (v[j] > 0 || (!seen[j] && v[j] != 0)) rc = 4;
    free(seen);
    if (rc) return rc;
    for (int32_t i = 0; i < n; ++i) dual += u[i];
    for (int32_t j = 0; j < m; ++j) dual += v[j];
    return primal == dual ? 0 : 5;
}

/* ------------------------------------------------------------------------- */
/* Auction with epsilon-scaling (Section 2.3.3; Bertsekas 1989)              */
/* ------------------------------------------------------------------------- */
/*
 * Rows are bidders, columns are objects, the reward of row i for column j is
 * R_ij = -C_ij.  Arithmetic is exact integer: rewards are multiplied by
 * (n + 1), so a slack of eps = 1 on that scale is eps < 1/n on the costs,
 * where the paper notes that the auction's result is exact for integer
 * weights (a result within n * eps of the optimum).  eps_final > 1 gives a
 * plan within floor(n * eps_final / (n + 1)) of the optimal cost.
 *
 * Each phase (eps = eps0, then eps / theta, ..., down to eps_final) starts
 * with every row unassigned and the prices of the previous phase.  Bidding
 * is one bidder at a time (Gauss-Seidel), first in first out: the bidder
 * finds its best value v1 = R_ij1 - p_j1 and the best value v2 over the
 * other columns, raises p_j1 by v1 - v2 + eps, takes j1 and evicts j1's
 * previous owner, who queues again.  Ties among best columns go to the
 * smaller column index.  n = 1: v2 is taken as v1 (the raise is eps).
 *
 * Outputs: plan[i] = column of row i, price[j] (scaled units), *cost =
 * sum_i C[i][plan[i]], *bids = total bids.  Returns 0, ORC_EINVAL, or
 * ORC_ENOMEM.
 */
int oracle_auction(const int32_t *C, int32_t n, int64_t eps0, int32_t theta, int64_t eps_final,
                   int32_t *plan, int64_t *price, int64_t *cost, int64_t *bids)
{
    if (!C || !plan || !price || !cost || n <= 0 || eps_final < 1 || eps0 < eps_final || theta < 2)
        return ORC_EINVAL;
    const int64_t scale = (int64_t)n + 1;
    int32_t *owner = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = malloc(sizeof(int32_t) * (size_t)n);
    if (!owner || !queue) { free(owner); free(queue); return ORC_ENOMEM; }
    for (int32_t j = 0; j < n; ++j) price[j] = 0;
    int64_t nb = 0;
    int64_t eps = eps0;
    for (;;) {
        for (int32_t i = 0; i < n; ++i) { plan[i] = -1; owner[i] = -1; queue[i] = i; }
        /* circular FIFO of unassigned rows: at most n are queued at once */
        int32_t head = 0, count = n;
        while (count > 0) {
            const int32_t i = queue[head];
            head = (head + 1) % n;
            --count;
            const int32_t *row = C + (size_t)i * (size_t)n;
            int32_t j1 = 0;
            int64_t v1 = -(int64_t)row[0] * scale - price[0], v2 = INT64_MIN;
            for (int32_t j = 1; j < n; ++j) {
                const int64_t val = -(int64_t)row[j] * scale - price[j];
                if (val > v1) { v2 = v1; v1 = val; j1 = j; }
                else if (val > v2) v2 = val;
            }
            if (n == 1) v2 = v1;
            price[j1] += v1 - v2 + eps;
            const int32_t prev = owner[j1];
            owner[j1] = i;
            plan[i] = j1;
            ++nb;
            if (prev >= 0) {
                plan[prev] = -1;
                queue[(head + count) % n] = prev;
                ++count;
            }
        }
        if (eps == eps_final) break;
        eps = eps / theta;
        if (eps < eps_final) eps = eps_final;
    }
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i) total += C[(size_t)i * (size_t)n + (size_t)plan[i]];
    *cost = total;
    if (bids) *bids = nb;
    free(owner);
    free(queue);
    return 0;
}
