/*
 * tg_oracle.c -- plain FP64 CPU oracle for batched Galerkin assembly.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this file;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no header, helper, table or constant with the HIP path.
 *
 * What it computes (TensorGalerkin, arXiv 2602.05052):
 *   K_ij = a(phi_j, phi_i),  F_i = l(phi_i)                  (Sec. 2, eq. matpde1)
 * assembled by the classical element loop with scatter-add
 *   K[g_e(a), g_e(b)] += (K_e)_ab   for e = 0, 1, ..., E-1  (Sec. 2, eq. scatter_add)
 * into a CSR matrix whose pattern is the set of DoF pairs that share an element.
 *
 * The configured coefficients are constant per element and every map is
 * affine, so the exact element integrals are polynomial integrals over a
 * simplex.  The oracle evaluates them in closed form with the barycentric
 * monomial rule
 *   int_T prod_i lambda_i^{e_i} dx = d! prod_i e_i! / (d + sum_i e_i)! * |T|
 * and uses no quadrature rule at all.  (The paper's Map uses a quadrature rule,
 * Sec. 2 Alg. 1 and eq. kloc1 / SM A.2 eq. matlclquad; for these degrees a
 * sufficient rule is exact, so both reach the same numbers up to rounding.)
 *
 * Element formulas:
 *   P1 Laplace  (SM A.2):  (K_e)_ab = a_e |T| grad(l_a).grad(l_b),  (F_e)_a = f_e int_T l_a
 *   P1 mass     (SM A.1, the mass inner product): (M_e)_ab = int_T l_a l_b
 *   P2 elasticity (Sec. B.1.1, Hooke's law sigma = lam tr(eps) I + 2 mu eps):
 *     row DoF (a, c) = test phi_a e_c, column DoF (b, c') = trial phi_b e_c',
 *     (K_e)_(a,c),(b,c') = lam D_ab[c][c'] + mu (D_ab[c'][c] + delta_cc' tr D_ab)
 *     with D_ab = int_T grad(phi_a) grad(phi_b)^T, and (F_e)_(a,c) = b_c int_T phi_a.
 *
 * Conventions that fix the global numbering (not stated in the paper):
 *   P2 local nodes: vertices 0..3, then edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3);
 *   P2 global nodes: the mesh vertices first, then every edge ranked by its
 *   (min vertex, max vertex) pair in lexicographic order;
 *   vector DoF = 3 * node + component.
 *   CSR: sorted columns, both triangles, entries that cancel to 0 kept.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_DEGENERATE (-2)
#define ORC_E_NOMEM (-4)

/* ------------------------------------------------------------------ */
/* Simplex geometry                                                    */
/* ------------------------------------------------------------------ */

static double fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

/* Barycentric monomial rule on a d-simplex of measure vol. */
double oracle_monomial(int dim, const int *e, double vol)
{
    int s = 0;
    double num = fact(dim);
    for (int i = 0; i <= dim; ++i) {
        s += e[i];
        num *= fact(e[i]);
    }
    return num / fact(dim + s) * vol;
}

/*
 * Geometry of the affine simplex with vertices X[0..d] (row-major [d+1][d]).
 * J has columns x_1 - x_0, ..., x_d - x_0 (Sec. 2 Alg. 1 "Geometry"; SM A.2,
 * where J_e is constant because the map is affine).  lambda_a for a >= 1 are
 * the components of J^{-1}(x - x_0), so grad(lambda_a) is row a-1 of J^{-1};
 * grad(lambda_0) = -sum of the others.  J^{-1} = adj(J) / det J with the
 * adjugate written out by cofactors.  grad is [d+1][d]; vol = |det J| / d!.
 * Returns ORC_E_DEGENERATE when det J is zero or not finite.
 */
int oracle_simplex_geometry(int dim, const double *X, double *grad, double *vol)
{
    double J[3][3];
    double inv[3][3];
    double det;
    if (dim != 2 && dim != 3) return ORC_E_ARG;
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            J[r][c] = X[(c + 1) * dim + r] - X[r]; /* column c = x_{c+1} - x_0 */
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (!(det != 0.0) || !isfinite(det)) return ORC_E_DEGENERATE;
        inv[0][0] = J[1][1] / det;
        inv[0][1] = -J[0][1] / det;
        inv[1][0] = -J[1][0] / det;
        inv[1][1] = J[0][0] / det;
    } else {
        double C[3][3]; /* cofactor matrix */
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        if (!(det != 0.0) || !isfinite(det)) return ORC_E_DEGENERATE;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                inv[r][c] = C[c][r] / det; /* adj = cofactor^T */
    }
    for (int c = 0; c < dim; ++c) grad[c] = 0.0;
    for (int a = 1; a <= dim; ++a)
        for (int c = 0; c < dim; ++c) {
            grad[a * dim + c] = inv[a - 1][c];
            grad[c] -= inv[a - 1][c];
        }
    *vol = fabs(det) / fact(dim);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Element matrices                                                    */
/* ------------------------------------------------------------------ */

/* P1 Laplace element: K [(d+1)^2] and F [d+1] (either may be NULL). */
int oracle_p1_laplace_element(int dim, const double *X, double a, double f, double *K, double *F)
{
    double g[4 * 3], vol;
    int k = dim + 1;
    int rc = oracle_simplex_geometry(dim, X, g, &vol);
    if (rc) return rc;
    if (K)
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                double s = 0.0;
                for (int c = 0; c < dim; ++c) s += g[i * dim + c] * g[j * dim + c];
                K[i * k + j] = a * vol * s;
            }
    if (F)
        for (int i = 0; i < k; ++i) {
            int e[4] = {0, 0, 0, 0};
            e[i] = 1;
            F[i] = f * oracle_monomial(dim, e, vol);
        }
    return ORC_OK;
}

/* P1 mass element M [(d+1)^2]: M_ab = int_T lambda_a lambda_b. */
int oracle_p1_mass_element(int dim, const double *X, double *M)
{
    double g[4 * 3], vol;
    int k = dim + 1;
    int rc = oracle_simplex_geometry(dim, X, g, &vol);
    if (rc) return rc;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            int e[4] = {0, 0, 0, 0};
            e[i] += 1;
            e[j] += 1;
            M[i * k + j] = oracle_monomial(dim, e, vol);
        }
    return ORC_OK;
}

/* P2 local edge list on the tetrahedron. */
static const int P2_EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

/*
 * grad(phi_a) = sum_p c_{a,p}(lambda) grad(lambda_p) with c_{a,p} affine in
 * lambda, stored as coef[a][p][0..4] = (constant, coefficient of lambda_0..3).
 *   vertex p: phi = lambda_p (2 lambda_p - 1)  => c_{a,p} = 4 lambda_p - 1
 *   edge (p,q): phi = 4 lambda_p lambda_q      => c_{a,p} = 4 lambda_q, c_{a,q} = 4 lambda_p
 */
static void p2_gradient_coefficients(double coef[10][4][5])
{
    memset(coef, 0, sizeof(double) * 10 * 4 * 5);
    for (int p = 0; p < 4; ++p) {
        coef[p][p][0] = -1.0;
        coef[p][p][1 + p] = 4.0;
    }
    for (int m = 0; m < 6; ++m) {
        int p = P2_EDGE[m][0], q = P2_EDGE[m][1];
        coef[4 + m][p][1 + q] = 4.0;
        coef[4 + m][q][1 + p] = 4.0;
    }
}

/* int_T u v for affine u = u0 + sum u_i lambda_i, v likewise (monomial rule). */
static double integrate_affine_product(const double *u, const double *v, double vol)
{
    double s = u[0] * v[0] * vol;
    for (int i = 0; i < 4; ++i) {
        int e[4] = {0, 0, 0, 0};
        e[i] = 1;
        s += (u[0] * v[1 + i] + v[0] * u[1 + i]) * oracle_monomial(3, e, vol);
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            int e[4] = {0, 0, 0, 0};
            e[i] += 1;
            e[j] += 1;
            s += u[1 + i] * v[1 + j] * oracle_monomial(3, e, vol);
        }
    return s;
}

/* int_T phi_a for the P2 basis. */
static double p2_basis_integral(int a, double vol)
{
    int e[4] = {0, 0, 0, 0};
    if (a < 4) {
        double s;
        e[a] = 2;
        s = 2.0 * oracle_monomial(3, e, vol);
        e[a] = 1;
        return s - oracle_monomial(3, e, vol);
    }
    e[P2_EDGE[a - 4][0]] = 1;
    e[P2_EDGE[a - 4][1]] = 1;
    return 4.0 * oracle_monomial(3, e, vol);
}

/*
 * P2 linear-elasticity tetrahedron: K [30][30], F [30] (F may be NULL),
 * local DoF 3 * node + component.  b is the body force (3 values).
 */
int oracle_p2_elasticity_element(const double *X, double lam, double mu, const double *b, double *K, double *F)
{
    double g[4][3], vol;
    double coef[10][4][5];
    int rc = oracle_simplex_geometry(3, X, &g[0][0], &vol);
    if (rc) return rc;
    p2_gradient_coefficients(coef);
    for (int a = 0; a < 10; ++a)
        for (int bb = 0; bb < 10; ++bb) {
            double D[3][3] = {{0}};
            double tr;
            for (int p = 0; p < 4; ++p)
                for (int r = 0; r < 4; ++r) {
                    double w = integrate_affine_product(coef[a][p], coef[bb][r], vol);
                    if (w == 0.0) continue;
                    for (int c = 0; c < 3; ++c)
                        for (int cc = 0; cc < 3; ++cc) D[c][cc] += w * g[p][c] * g[r][cc];
                }
            tr = D[0][0] + D[1][1] + D[2][2];
            for (int c = 0; c < 3; ++c)
                for (int cc = 0; cc < 3; ++cc)
                    K[(3 * a + c) * 30 + 3 * bb + cc] =
                        lam * D[c][cc] + mu * (D[cc][c] + (c == cc ? tr : 0.0));
        }
    if (F)
        for (int a = 0; a < 10; ++a) {
            double ia = p2_basis_integral(a, vol);
            for (int c = 0; c < 3; ++c) F[3 * a + c] = b[c] * ia;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Numbering and CSR pattern                                           */
/* ------------------------------------------------------------------ */

static int cmp_i64(const void *x, const void *y)
{
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

/*
 * P2 node numbering: nodes10 [E][10] receives the global node of each local
 * node (vertices keep their ids, edge m of element e becomes nv + rank of its
 * (min, max) vertex pair).  *n_nodes = nv + number of edges.
 */
int oracle_p2_numbering(int64_t nv, int64_t E, const int32_t *conn, int64_t *nodes10, int64_t *n_nodes)
{
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(6 * E + 1));
    int64_t nedge = 0;
    if (!keys) return ORC_E_NOMEM;
    for (int64_t e = 0; e < E; ++e)
        for (int m = 0; m < 6; ++m) {
            int64_t p = conn[e * 4 + P2_EDGE[m][0]], q = conn[e * 4 + P2_EDGE[m][1]];
            int64_t lo = p < q ? p : q, hi = p < q ? q : p;
            keys[e * 6 + m] = lo * nv + hi;
        }
    qsort(keys, (size_t)(6 * E), sizeof(int64_t), cmp_i64);
    for (int64_t t = 0; t < 6 * E; ++t)
        if (t == 0 || keys[t] != keys[t - 1]) keys[nedge++] = keys[t];
    for (int64_t e = 0; e < E; ++e) {
        for (int v = 0; v < 4; ++v) nodes10[e * 10 + v] = conn[e * 4 + v];
        for (int m = 0; m < 6; ++m) {
            int64_t p = conn[e * 4 + P2_EDGE[m][0]], q = conn[e * 4 + P2_EDGE[m][1]];
            int64_t key = (p < q ? p : q) * nv + (p < q ? q : p);
            int64_t *hit = (int64_t *)bsearch(&key, keys, (size_t)nedge, sizeof(int64_t), cmp_i64);
            nodes10[e * 10 + 4 + m] = nv + (hit - keys);
        }
    }
    free(keys);
    *n_nodes = nv + nedge;
    return ORC_OK;
}

/*
 * CSR pattern of the matrix whose element e couples the kd DoFs dofs[e][0..kd-1]:
 * row i holds every DoF that shares an element with i, sorted, without repeats.
 * row_ptr [ndof+1] is filled by the caller-provided buffer; col_idx is malloc'ed
 * and returned (free with oracle_free).
 */
int oracle_csr_pattern(int64_t ndof, int64_t E, int kd, const int64_t *dofs, int64_t *row_ptr, int64_t **col_idx_out,
                       int64_t *nnz_out)
{
    int64_t *cnt = (int64_t *)calloc((size_t)ndof + 1, sizeof(int64_t));
    int64_t *inc, *fill, *cols = NULL, *tmp = NULL;
    int64_t nnz = 0, cap = 0, tmpcap = 0;
    if (!cnt) return ORC_E_NOMEM;
    for (int64_t t = 0; t < E * kd; ++t) {
        if (dofs[t] < 0 || dofs[t] >= ndof) {
            free(cnt);
            return ORC_E_ARG;
        }
        cnt[dofs[t] + 1]++;
    }
    for (int64_t i = 0; i < ndof; ++i) cnt[i + 1] += cnt[i];
    inc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E * kd + 1));
    fill = (int64_t *)calloc((size_t)ndof + 1, sizeof(int64_t));
    if (!inc || !fill) return ORC_E_NOMEM;
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < kd; ++a) {
            int64_t i = dofs[e * kd + a];
            inc[cnt[i] + fill[i]++] = e; /* elements incident to DoF i */
        }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < ndof; ++i) {
        int64_t n = 0, need = (cnt[i + 1] - cnt[i]) * kd;
        if (need > tmpcap) {
            tmpcap = need * 2;
            tmp = (int64_t *)realloc(tmp, sizeof(int64_t) * (size_t)tmpcap);
            if (!tmp) return ORC_E_NOMEM;
        }
        for (int64_t t = cnt[i]; t < cnt[i + 1]; ++t)
            for (int b = 0; b < kd; ++b) tmp[n++] = dofs[inc[t] * kd + b];
        qsort(tmp, (size_t)n, sizeof(int64_t), cmp_i64);
        for (int64_t t = 0; t < n; ++t) {
            if (t > 0 && tmp[t] == tmp[t - 1]) continue;
            if (nnz == cap) {
                cap = cap ? cap * 2 : 1024;
                cols = (int64_t *)realloc(cols, sizeof(int64_t) * (size_t)cap);
                if (!cols) return ORC_E_NOMEM;
            }
            cols[nnz++] = tmp[t];
        }
        row_ptr[i + 1] = nnz;
    }
    free(tmp);
    free(inc);
    free(fill);
    free(cnt);
    *col_idx_out = cols;
    *nnz_out = nnz;
    return ORC_OK;
}

void oracle_free(void *p) { free(p); }

/* position of column j in CSR row i (binary search over the sorted columns) */
static int64_t csr_find(const int64_t *row_ptr, const int64_t *col_idx, int64_t i, int64_t j)
{
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] == j) return mid;
        if (col_idx[mid] < j) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Global assembly by scatter-add, elements in ascending order          */
/* ------------------------------------------------------------------ */

static void gather_vertices(int dim, const double *coords, const int32_t *vids, int nvtx, double *X)
{
    for (int a = 0; a < nvtx; ++a)
        for (int c = 0; c < dim; ++c) X[a * dim + c] = coords[(int64_t)vids[a] * dim + c];
}

/*
 * P1 scalar assembly.  form 0 = Laplace (coef a[E], load f[E]; load may be
 * NULL), form 1 = mass (coef, load ignored).  coords [nv][dim], conn [E][dim+1].
 * vals [nnz] and rhs [nv] must be zeroed by the caller (rhs may be NULL).
 * On a degenerate element, returns ORC_E_DEGENERATE and stores its index in *bad.
 */
int oracle_assemble_p1(int dim, int form, int64_t nv, const double *coords, int64_t E, const int32_t *conn,
                       const double *coef, const double *load, const int64_t *row_ptr, const int64_t *col_idx,
                       double *vals, double *rhs, int64_t *bad)
{
    int k = dim + 1;
    double X[4 * 3], Ke[16], Fe[4];
    (void)nv;
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *g = conn + e * k;
        int rc;
        gather_vertices(dim, coords, g, k, X);
        if (form == 0) rc = oracle_p1_laplace_element(dim, X, coef[e], load ? load[e] : 0.0, Ke, Fe);
        else rc = oracle_p1_mass_element(dim, X, Ke);
        if (rc) {
            if (bad) *bad = e;
            return rc;
        }
        for (int a = 0; a < k; ++a) {
            for (int b = 0; b < k; ++b) vals[csr_find(row_ptr, col_idx, g[a], g[b])] += Ke[a * k + b];
            if (rhs && form == 0 && load) rhs[g[a]] += Fe[a];
        }
    }
    return ORC_OK;
}

/*
 * The same P1 Laplace value and load assembly on several CPU threads, with the
 * same additions in the same order as oracle_assemble_p1, so the result is
 * bitwise identical to it (the multi-core CPU baseline):
 *   Map    : every element's K_e and F_e (independent; elements split among
 *            the threads) into Ke_all [E][k][k] and Fe_all [E][k];
 *   Reduce : every row i (rows split among the threads) adds, for its incident
 *            (element e, local node a) pairs in ascending e, K_e[a][b] into
 *            entry (i, g_e(b)) and F_e[a] into rhs[i].  Entry (i, j) thus
 *            receives its terms in ascending element order, exactly as the
 *            serial element loop adds them.
 * inc_ptr [nv+1] / inc [E k]: pair code e k + a of every row, ascending e.
 * Ke_all and Fe_all are caller scratch; vals and rhs need not be zeroed.
 * threads <= 0: the OpenMP default.
 */
int oracle_assemble_p1_parallel(int dim, int64_t nv, const double *coords, int64_t E, const int32_t *conn,
                                const double *coef, const double *load, const int64_t *row_ptr,
                                const int64_t *col_idx, const int64_t *inc_ptr, const int64_t *inc, double *Ke_all,
                                double *Fe_all, double *vals, double *rhs, int threads, int64_t *bad)
{
    const int k = dim + 1;
    int64_t first_bad = E;
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for num_threads(threads) schedule(static) reduction(min : first_bad)
    for (int64_t e = 0; e < E; ++e) {
        double X[4 * 3];
        gather_vertices(dim, coords, conn + e * k, k, X);
        if (oracle_p1_laplace_element(dim, X, coef[e], load ? load[e] : 0.0, Ke_all + e * k * k, Fe_all + e * k))
            first_bad = e < first_bad ? e : first_bad;
    }
    if (first_bad < E) {
        if (bad) *bad = first_bad;
        return ORC_E_DEGENERATE;
    }
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int64_t i = 0; i < nv; ++i) {
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) vals[q] = 0.0;
        double fi = 0.0;
        for (int64_t t = inc_ptr[i]; t < inc_ptr[i + 1]; ++t) {
            const int64_t e = inc[t] / k;
            const int a = (int)(inc[t] - e * k);
            const int32_t *g = conn + e * k;
            for (int b = 0; b < k; ++b) vals[csr_find(row_ptr, col_idx, i, g[b])] += Ke_all[(e * k + a) * k + b];
            fi += Fe_all[e * k + a];
        }
        if (rhs) rhs[i] = load ? fi : 0.0;
    }
    return ORC_OK;
}

/*
 * P2 elasticity assembly.  nodes10 [E][10] from oracle_p2_numbering; lam, mu [E];
 * body force b [E][3] (may be NULL).  DoF = 3 * node + component.
 */
int oracle_assemble_p2_elasticity(int64_t nv, const double *coords, int64_t E, const int32_t *conn,
                                  const int64_t *nodes10, const double *lam, const double *mu, const double *b,
                                  const int64_t *row_ptr, const int64_t *col_idx, double *vals, double *rhs,
                                  int64_t *bad)
{
    double X[12];
    double *Ke = (double *)malloc(sizeof(double) * 900);
    double Fe[30];
    const double zero[3] = {0.0, 0.0, 0.0};
    (void)nv;
    if (!Ke) return ORC_E_NOMEM;
    for (int64_t e = 0; e < E; ++e) {
        int64_t dof[30];
        int rc;
        gather_vertices(3, coords, conn + e * 4, 4, X);
        rc = oracle_p2_elasticity_element(X, lam[e], mu[e], b ? b + 3 * e : zero, Ke, Fe);
        if (rc) {
            if (bad) *bad = e;
            free(Ke);
            return rc;
        }
        for (int a = 0; a < 10; ++a)
            for (int c = 0; c < 3; ++c) dof[3 * a + c] = 3 * nodes10[e * 10 + a] + c;
        for (int r = 0; r < 30; ++r) {
            for (int s = 0; s < 30; ++s) vals[csr_find(row_ptr, col_idx, dof[r], dof[s])] += Ke[r * 30 + s];
            if (rhs) rhs[dof[r]] += Fe[r];
        }
    }
    free(Ke);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Adjoint of P1 assembly                                              */
/* ------------------------------------------------------------------ */

/*
 * For one P1 simplex, the element term of
 *   Phi = lam^T (A(c, x) u - M(x) w),   A = K(c) (mass = 0) or M + K(c) (mass = 1),
 * returns dPhi/d(log c) = lam^T K_e u (= c |T| g_lam . g_u with g_v = sum_b v_b grad(l_b))
 * in *dlogc, and dPhi/dx_a for every vertex a in dx [d+1][d]:
 *   K part:    c |T| [ G_a (g_lam.g_u) - g_lam (G_a.g_u) - g_u (G_a.g_lam) ]
 *   mass part: Phi_M G_a with Phi_M = lam^T M_e (mass u - w)
 * using d|T|/dx_a = |T| G_a and d(grad l_b)/dx_a = -grad(l_b) G_a^T (affine map),
 * G_a = grad(l_a).  w may be NULL (taken as 0).
 */
int oracle_p1_adjoint_element(int dim, const double *X, double c, const double *lam, const double *u,
                              const double *w, int mass, double *dlogc, double *dx)
{
    double G[4 * 3], vol, gl[3] = {0, 0, 0}, gu[3] = {0, 0, 0}, M[16], phim = 0.0, glu = 0.0;
    int k = dim + 1;
    int rc = oracle_simplex_geometry(dim, X, G, &vol);
    if (rc) return rc;
    for (int b = 0; b < k; ++b)
        for (int i = 0; i < dim; ++i) {
            gl[i] += lam[b] * G[b * dim + i];
            gu[i] += u[b] * G[b * dim + i];
        }
    for (int i = 0; i < dim; ++i) glu += gl[i] * gu[i];
    oracle_p1_mass_element(dim, X, M);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) phim += lam[a] * M[a * k + b] * ((mass ? u[b] : 0.0) - (w ? w[b] : 0.0));
    *dlogc = c * vol * glu;
    for (int a = 0; a < k; ++a) {
        double Ga_gu = 0.0, Ga_gl = 0.0;
        for (int i = 0; i < dim; ++i) {
            Ga_gu += G[a * dim + i] * gu[i];
            Ga_gl += G[a * dim + i] * gl[i];
        }
        for (int i = 0; i < dim; ++i)
            dx[a * dim + i] = c * vol * (G[a * dim + i] * glu - gl[i] * Ga_gu - gu[i] * Ga_gl) + phim * G[a * dim + i];
    }
    return ORC_OK;
}

/*
 * Global adjoint: dlogc [E] and dcoords [nv][dim] of Phi = lam^T (A u - M w), summed over
 * elements in ascending order (arrays are overwritten).
 */
int oracle_p1_adjoint(int dim, int64_t nv, const double *coords, int64_t E, const int32_t *conn, int mass,
                      const double *c, const double *lam, const double *u, const double *w, double *dlogc,
                      double *dcoords, int64_t *bad)
{
    int k = dim + 1;
    double X[12], le[4], ue[4], we[4], dx[12];
    for (int64_t t = 0; t < nv * dim; ++t) dcoords[t] = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *g = conn + e * k;
        int rc;
        gather_vertices(dim, coords, g, k, X);
        for (int a = 0; a < k; ++a) {
            le[a] = lam[g[a]];
            ue[a] = u[g[a]];
            we[a] = w ? w[g[a]] : 0.0;
        }
        rc = oracle_p1_adjoint_element(dim, X, c[e], le, ue, w ? we : NULL, mass, &dlogc[e], dx);
        if (rc) {
            if (bad) *bad = e;
            return rc;
        }
        for (int a = 0; a < k; ++a)
            for (int i = 0; i < dim; ++i) dcoords[(int64_t)g[a] * dim + i] += dx[a * dim + i];
    }
    return ORC_OK;
}
