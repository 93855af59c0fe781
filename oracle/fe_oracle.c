/*
 * fe_oracle.c -- plain FP64 CPU oracle for per-element weak-form evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: it builds its own
 * quadrature rules and basis tables from their definitions.
 *
 * What it computes follows the paper's element loops (the residual loop of
 * Algorithm "feloopv" and the matrix loop of Algorithm "feloopm"): for every
 * cell, for every quadrature point, add  (quadrature weight * |J|) * integrand.
 * The integrands are the weak forms of the table of example weak forms
 * (vector dot product / mass, weak Laplacian, linear elasticity, weighted
 * vector dot product, Navier-Stokes convection) written out element by
 * element, in FP64, with no blocking or reordering.
 *
 * Readings of the paper used here (the paper does not fix them):
 *   - reference hexahedron [0,1]^3; tensor Gauss-Legendre rule with p+1
 *     points per axis, i.e. (p+1)^3 points as in the cell/DOF count table;
 *   - equispaced Lagrange basis of order p, lexicographic local numbering
 *     a = i + (p+1)(j + (p+1)k); isoparametric geometry (same basis);
 *   - reference tetrahedron {xi>=0, sum xi<=1}; P1/P2 Lagrange basis with
 *     vertex then edge nodes, edges (0,1),(1,2),(0,2),(0,3),(1,3),(2,3);
 *     collapsed-coordinate (conical product) Gauss-Jacobi rule with
 *     p+1 points per collapsed direction (exact to degree 2p+1);
 *   - vector unknowns are stored component-major inside an element
 *     (row index r*n_b + a), the global DOF array is (n_nodes, n_comp);
 *   - symmetric storage of strain (Voigt) in the order 11,22,33,12,13,23
 *     with engineering shear (the ones of the symmetric-gradient extractor);
 *   - |J| is the determinant itself; a non-positive determinant is an error.
 *
 * Every function returns 0 on success or a negative status:
 *   -1 bad argument, -2 non-positive Jacobian, -3 node index out of range.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_HEX 0
#define ORC_TET 1

#define ORC_MASS 0
#define ORC_VMASS 1
#define ORC_LAPLACE 2
#define ORC_ELASTICITY 3
#define ORC_WDOT 4
#define ORC_CONVECT 5

#define ORC_MAT_NONE 0
#define ORC_MAT_ISO_CELL 1
#define ORC_MAT_ISO_QP 2
#define ORC_MAT_VOIGT_QP 3
#define ORC_MAT_TENSOR_QP 4

#define NB_MAX 216
#define NQ_MAX 216

#define ERR_ARG (-1)
#define ERR_DET (-2)
#define ERR_INDEX (-3)

/* ------------------------------------------------------------------------ */
/* 1-D building blocks                                                      */
/* ------------------------------------------------------------------------ */

/* Jacobi polynomial P_n^{(alpha,0)}(x) on [-1,1] by its three-term
 * recurrence (alpha = 0 gives Legendre). */
static double jacobi_poly(int n, double alpha, double x)
{
    const double beta = 0.0;
    double p0 = 1.0;
    if (n == 0) return p0;
    double p1 = (alpha + 1.0) + (alpha + beta + 2.0) * (x - 1.0) * 0.5;
    for (int k = 2; k <= n; k++) {
        double a = 2.0 * k + alpha + beta;
        double c1 = 2.0 * k * (k + alpha + beta) * (a - 2.0);
        double c2 = (a - 1.0) * (a * (a - 2.0) * x + alpha * alpha - beta * beta);
        double c3 = 2.0 * (k + alpha - 1.0) * (k + beta - 1.0) * a;
        double p2 = (c2 * p1 - c3 * p0) / c1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* Solve the small dense system A x = b (n <= 16) by Gaussian elimination
 * with partial pivoting. A is row-major and overwritten. */
static int solve_dense(int n, double *A, double *b)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return ERR_ARG;
        if (piv != c) {
            for (int k = 0; k < n; k++) {
                double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; r++) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; k++) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < n; k++) s -= A[r * n + k] * b[k];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* n-point Gauss rule on [0,1] for the weight (1-s)^alpha (alpha integer
 * >= 0).  Nodes: the n roots of the degree-n orthogonal polynomial for that
 * weight, i.e. of P_n^{(alpha,0)}(2s-1), bracketed on a fine grid and
 * bisected.  Weights: the unique solution of the moment equations
 * sum_i w_i s_i^k = int_0^1 s^k (1-s)^alpha ds, k = 0..n-1.  A Gauss rule is
 * then exact up to degree 2n-1. */
int orc_gauss_jacobi01(int n, int alpha, double *s, double *w)
{
    if (n < 1 || n > 16 || alpha < 0) return ERR_ARG;
    const int grid = 20000;
    int found = 0;
    double xl = -1.0, fl = jacobi_poly(n, alpha, xl);
    for (int g = 1; g <= grid && found < n; g++) {
        double xr = -1.0 + 2.0 * g / grid;
        double fr = jacobi_poly(n, alpha, xr);
        if (fl == 0.0) { s[found++] = 0.5 * (xl + 1.0); }
        else if (fl * fr < 0.0) {
            double a = xl, b = xr, fa = fl;
            for (int it = 0; it < 200; it++) {
                double m = 0.5 * (a + b);
                double fm = jacobi_poly(n, alpha, m);
                if (fm == 0.0) { a = b = m; break; }
                if (fa * fm < 0.0) { b = m; } else { a = m; fa = fm; }
                if (b - a < 1e-17) break;
            }
            s[found++] = 0.5 * (0.5 * (a + b) + 1.0);
        }
        xl = xr; fl = fr;
    }
    if (found != n) return ERR_ARG;
    double A[16 * 16], b[16];
    for (int k = 0; k < n; k++) {
        for (int i = 0; i < n; i++) A[k * n + i] = pow(s[i], k);
        /* int_0^1 s^k (1-s)^alpha ds = k! alpha! / (k+alpha+1)! */
        double m = 1.0;
        for (int t = 1; t <= alpha; t++) m *= (double)t / (double)(k + t);
        b[k] = m / (double)(k + alpha + 1);
    }
    if (solve_dense(n, A, b)) return ERR_ARG;
    for (int i = 0; i < n; i++) w[i] = b[i];
    return 0;
}

/* Equispaced 1-D Lagrange basis of order p on [0,1], nodes t_k = k/p:
 * phi_k(x) = prod_{m != k} (x - t_m)/(t_k - t_m) and its derivative by the
 * product rule. */
static void lagrange1d(int p, double x, double *val, double *der)
{
    for (int k = 0; k <= p; k++) {
        double tk = (double)k / p;
        double v = 1.0;
        for (int m = 0; m <= p; m++)
            if (m != k) v *= (x - (double)m / p) / (tk - (double)m / p);
        double d = 0.0;
        for (int l = 0; l <= p; l++) {
            if (l == k) continue;
            double t = 1.0 / (tk - (double)l / p);
            for (int m = 0; m <= p; m++)
                if (m != k && m != l) t *= (x - (double)m / p) / (tk - (double)m / p);
            d += t;
        }
        val[k] = v;
        der[k] = d;
    }
}

/* ------------------------------------------------------------------------ */
/* Reference element tables                                                 */
/* ------------------------------------------------------------------------ */

int orc_sizes(int cell, int p, int *n_basis, int *n_qp)
{
    if (cell == ORC_HEX) {
        if (p < 1 || p > 5) return ERR_ARG;
        *n_basis = (p + 1) * (p + 1) * (p + 1);
        *n_qp = (p + 1) * (p + 1) * (p + 1);
        return 0;
    }
    if (cell == ORC_TET) {
        if (p < 1 || p > 2) return ERR_ARG;
        *n_basis = (p == 1) ? 4 : 10;
        *n_qp = (p + 1) * (p + 1) * (p + 1);
        return 0;
    }
    return ERR_ARG;
}

/* Tetrahedron basis at reference point (x,y,z): values and gradients
 * d phi / d xi_j, vertex nodes first then edge nodes. */
static void tet_basis(int p, double x, double y, double z, double *val,
                      double (*grad)[NB_MAX] /* grad[j][a] */)
{
    double L[4] = {1.0 - x - y - z, x, y, z};
    double dL[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    if (p == 1) {
        for (int a = 0; a < 4; a++) {
            val[a] = L[a];
            for (int j = 0; j < 3; j++) grad[j][a] = dL[a][j];
        }
        return;
    }
    for (int a = 0; a < 4; a++) {
        val[a] = L[a] * (2.0 * L[a] - 1.0);
        for (int j = 0; j < 3; j++) grad[j][a] = (4.0 * L[a] - 1.0) * dL[a][j];
    }
    static const int edges[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
    for (int e = 0; e < 6; e++) {
        int i = edges[e][0], k = edges[e][1];
        val[4 + e] = 4.0 * L[i] * L[k];
        for (int j = 0; j < 3; j++)
            grad[j][4 + e] = 4.0 * (dL[i][j] * L[k] + L[i] * dL[k][j]);
    }
}

/* Quadrature weights w[q], points pts[q][3], basis values bf[q][a] and
 * reference gradients bfg[q][j][a]. */
int orc_tables(int cell, int p, double *w, double *pts, double *bf, double *bfg)
{
    int nb, nq;
    if (orc_sizes(cell, p, &nb, &nq)) return ERR_ARG;
    int n = p + 1;
    if (cell == ORC_HEX) {
        double s[16], sw[16];
        if (orc_gauss_jacobi01(n, 0, s, sw)) return ERR_ARG;
        double val[16][16], der[16][16]; /* [point][k] */
        for (int i = 0; i < n; i++) lagrange1d(p, s[i], val[i], der[i]);
        for (int q2 = 0; q2 < n; q2++)
            for (int q1 = 0; q1 < n; q1++)
                for (int q0 = 0; q0 < n; q0++) {
                    int q = q0 + n * (q1 + n * q2);
                    w[q] = sw[q0] * sw[q1] * sw[q2];
                    pts[3 * q + 0] = s[q0];
                    pts[3 * q + 1] = s[q1];
                    pts[3 * q + 2] = s[q2];
                    for (int k = 0; k < n; k++)
                        for (int j = 0; j < n; j++)
                            for (int i = 0; i < n; i++) {
                                int a = i + n * (j + n * k);
                                bf[q * nb + a] = val[q0][i] * val[q1][j] * val[q2][k];
                                bfg[(q * 3 + 0) * nb + a] = der[q0][i] * val[q1][j] * val[q2][k];
                                bfg[(q * 3 + 1) * nb + a] = val[q0][i] * der[q1][j] * val[q2][k];
                                bfg[(q * 3 + 2) * nb + a] = val[q0][i] * val[q1][j] * der[q2][k];
                            }
                }
        return 0;
    }
    /* tetrahedron: collapsed coordinates (a,b,c) in [0,1]^3,
     * x = a, y = (1-a) b, z = (1-a)(1-b) c, |d(x,y,z)/d(a,b,c)| = (1-a)^2 (1-b);
     * Gauss-Jacobi with weight (1-a)^2 in a, (1-b) in b, Legendre in c. */
    double sa[16], wa[16], sb[16], wb[16], sc[16], wc[16];
    if (orc_gauss_jacobi01(n, 2, sa, wa)) return ERR_ARG;
    if (orc_gauss_jacobi01(n, 1, sb, wb)) return ERR_ARG;
    if (orc_gauss_jacobi01(n, 0, sc, wc)) return ERR_ARG;
    double val[NB_MAX], grad[3][NB_MAX];
    for (int ic = 0; ic < n; ic++)
        for (int ib = 0; ib < n; ib++)
            for (int ia = 0; ia < n; ia++) {
                int q = ia + n * (ib + n * ic);
                double x = sa[ia];
                double y = (1.0 - sa[ia]) * sb[ib];
                double z = (1.0 - sa[ia]) * (1.0 - sb[ib]) * sc[ic];
                w[q] = wa[ia] * wb[ib] * wc[ic];
                pts[3 * q + 0] = x;
                pts[3 * q + 1] = y;
                pts[3 * q + 2] = z;
                tet_basis(p, x, y, z, val, grad);
                for (int a = 0; a < nb; a++) {
                    bf[q * nb + a] = val[a];
                    for (int j = 0; j < 3; j++) bfg[(q * 3 + j) * nb + a] = grad[j][a];
                }
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per element / per quadrature point geometry                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int cell, p, nb, nq;
    double w[NQ_MAX];
    double pts[NQ_MAX * 3];
    double *bf;   /* [nq][nb]    */
    double *bfg;  /* [nq][3][nb] */
} ref_t;

static int ref_init(ref_t *r, int cell, int p)
{
    if (orc_sizes(cell, p, &r->nb, &r->nq)) return ERR_ARG;
    r->cell = cell;
    r->p = p;
    r->bf = (double *)malloc(sizeof(double) * r->nq * r->nb);
    r->bfg = (double *)malloc(sizeof(double) * r->nq * 3 * r->nb);
    if (!r->bf || !r->bfg) return ERR_ARG;
    return orc_tables(cell, p, r->w, r->pts, r->bf, r->bfg);
}

static void ref_free(ref_t *r)
{
    free(r->bf);
    free(r->bfg);
}

/* Gather the element's node coordinates x[a][i] through the connectivity. */
static int gather_coords(const ref_t *r, int64_t e, int64_t n_nodes,
                         const double *coords, const int32_t *conn, double (*x)[3])
{
    for (int a = 0; a < r->nb; a++) {
        int64_t n = conn[e * r->nb + a];
        if (n < 0 || n >= n_nodes) return ERR_INDEX;
        for (int i = 0; i < 3; i++) x[a][i] = coords[3 * n + i];
    }
    return 0;
}

/* Geometry at quadrature point q (section on FE notation and the chain rule
 * below eq. fe2):
 *   J_ij   = sum_a x_a,i dphi_a/dxi_j           (Jacobian of the mapping)
 *   det    = det J (cofactor expansion)
 *   Jinv   = adj(J) / det
 *   wdet   = w_q det                             (weight folded into |J|)
 *   G[i][a]= sum_j dphi_a/dxi_j Jinv[j][i]      (physical gradients)      */
static int geometry(const ref_t *r, int q, double (*x)[3], double *wdet,
                    double (*G)[NB_MAX])
{
    const int nb = r->nb;
    const double *g = r->bfg + (size_t)q * 3 * nb;
    double J[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int a = 0; a < nb; a++) s += x[a][i] * g[j * nb + a];
            J[i][j] = s;
        }
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0)) return ERR_DET;
    double Ji[3][3];
    Ji[0][0] = c00 / det;
    Ji[1][0] = c01 / det;
    Ji[2][0] = c02 / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    *wdet = r->w[q] * det;
    for (int i = 0; i < 3; i++)
        for (int a = 0; a < nb; a++) {
            double s = 0.0;
            for (int j = 0; j < 3; j++) s += g[j * nb + a] * Ji[j][i];
            G[i][a] = s;
        }
    return 0;
}

/* Elastic coefficient matrix D (6x6 Voigt, engineering shear) of cell e at
 * quadrature point q.  Isotropic: D = lambda m m^T + mu diag(2,2,2,1,1,1). */
static int material_D(int kind, const double *mat, int64_t e, int q, int nq, double D[6][6])
{
    double lam, mu;
    if (kind == ORC_MAT_VOIGT_QP) {
        const double *d = mat + ((size_t)e * nq + q) * 36;
        for (int I = 0; I < 6; I++)
            for (int K = 0; K < 6; K++) D[I][K] = d[I * 6 + K];
        return 0;
    }
    if (kind == ORC_MAT_ISO_CELL) {
        lam = mat[2 * e];
        mu = mat[2 * e + 1];
    } else if (kind == ORC_MAT_ISO_QP) {
        lam = mat[2 * ((size_t)e * nq + q)];
        mu = mat[2 * ((size_t)e * nq + q) + 1];
    } else {
        return ERR_ARG;
    }
    for (int I = 0; I < 6; I++)
        for (int K = 0; K < 6; K++) D[I][K] = (I < 3 && K < 3) ? lam : 0.0;
    for (int I = 0; I < 6; I++) D[I][I] += (I < 3) ? 2.0 * mu : mu;
    return 0;
}

/* Strain-displacement matrix B[I][(r,a)] (6 x 3nb, column r*nb + a) of the
 * symmetric-gradient storage s(i:j)->I with engineering shear. */
static const int VOIGT_I[6] = {0, 1, 2, 0, 0, 1};
static const int VOIGT_J[6] = {0, 1, 2, 1, 2, 2};

static double B_entry(int I, int r, int a, double (*G)[NB_MAX])
{
    int i = VOIGT_I[I], j = VOIGT_J[I];
    double v = 0.0;
    if (r == i) v += G[j][a];
    if (r == j && i != j) v += G[i][a];
    return v;
}

static int n_comp_of(int form)
{
    return (form == ORC_MASS || form == ORC_LAPLACE) ? 1 : 3;
}

static int check_common(int cell, int p, int form, int mat_kind)
{
    int nb, nq;
    if (orc_sizes(cell, p, &nb, &nq)) return ERR_ARG;
    if (form < ORC_MASS || form > ORC_CONVECT) return ERR_ARG;
    if (form == ORC_ELASTICITY && (mat_kind < ORC_MAT_ISO_CELL || mat_kind > ORC_MAT_VOIGT_QP))
        return ERR_ARG;
    if (form == ORC_WDOT && mat_kind != ORC_MAT_TENSOR_QP) return ERR_ARG;
    return 0;
}

/* Weighted vector dot coefficient M_ij of cell e at quadrature point q
 * ('ij,i,j': a 3 x 3 matrix per point, row-major). */
static double wdot_M(const double *mat, int64_t e, int q, int nq, int i, int j)
{
    return mat[((size_t)e * nq + q) * 9 + i * 3 + j];
}

/* Values u_c(q) and physical gradients du_c/dx_j (q) of a vector field with
 * element DOFs ue[c][b] (component-major). */
static void field_at(const ref_t *r, int q, double (*G)[NB_MAX], const double *ue,
                     double uq[3], double gu[3][3])
{
    const int nb = r->nb;
    const double *phi = r->bf + (size_t)q * nb;
    for (int c = 0; c < 3; c++) {
        double v = 0.0;
        for (int b = 0; b < nb; b++) v += phi[b] * ue[c * nb + b];
        uq[c] = v;
        for (int j = 0; j < 3; j++) {
            double g = 0.0;
            for (int b = 0; b < nb; b++) g += G[j][b] * ue[c * nb + b];
            gu[c][j] = g;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Matrix mode: element matrices (Algorithm "feloopm")                      */
/* ------------------------------------------------------------------------ */

static int gather_dofs(const ref_t *r, int nc, int64_t e, const int32_t *conn,
                       const double *U, double *ue);

/* out: (n_cells, nc*nb, nc*nb) row-major, rows/cols component-major.
 * U (n_nodes, 3): the state the Navier-Stokes convection matrix is the
 * derivative at (eq. fe4); ignored by the linear forms. */
int orc_matrix_u(int cell, int p, int form, int64_t n_cells, int64_t n_nodes,
                 const double *coords, const int32_t *conn, int mat_kind,
                 const double *mat, const double *U, double *out)
{
    if (check_common(cell, p, form, mat_kind)) return ERR_ARG;
    if (form == ORC_CONVECT && !U) return ERR_ARG;
    ref_t r;
    if (ref_init(&r, cell, p)) { ref_free(&r); return ERR_ARG; }
    const int nb = r.nb, nq = r.nq, nc = n_comp_of(form), nd = nc * nb;
    int status = 0;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_cells; e++) {
        double x[NB_MAX][3];
        double G[3][NB_MAX];
        double ue[3 * NB_MAX];
        double *M = out + (size_t)e * nd * nd;
        for (int k = 0; k < nd * nd; k++) M[k] = 0.0;
        int st = gather_coords(&r, e, n_nodes, coords, conn, x);
        if (!st && form == ORC_CONVECT) gather_dofs(&r, 3, e, conn, U, ue);
        for (int q = 0; q < nq && !st; q++) {
            double wdet;
            st = geometry(&r, q, x, &wdet, G);
            if (st) break;
            const double *phi = r.bf + (size_t)q * nb;
            if (form == ORC_MASS || form == ORC_VMASS) {
                /* int phi_a phi_b |J|; vector form: delta_rs blocks (eq. fe3c) */
                for (int c = 0; c < nc; c++)
                    for (int a = 0; a < nb; a++)
                        for (int b = 0; b < nb; b++)
                            M[(c * nb + a) * nd + c * nb + b] += wdet * phi[a] * phi[b];
            } else if (form == ORC_WDOT) {
                /* int v_i M_ij u_j |J|: K[(i,a),(j,b)] = M_ij phi_a phi_b */
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        const double m = wdot_M(mat, e, q, nq, i, j);
                        for (int a = 0; a < nb; a++)
                            for (int b = 0; b < nb; b++)
                                M[(i * nb + a) * nd + j * nb + b] += wdet * m * phi[a] * phi[b];
                    }
            } else if (form == ORC_CONVECT) {
                /* derivative of int v_i (du_i/dx_j) u_j |J| w.r.t. u (eq. fe4):
                 * the two terms obtained by leaving out either u,
                 * K[(i,a),(c,m)] = phi_a (delta_ic u_j dphi_m/dx_j + du_i/dx_c phi_m) */
                double uq[3], gu[3][3];
                field_at(&r, q, G, ue, uq, gu);
                for (int i = 0; i < 3; i++)
                    for (int a = 0; a < nb; a++)
                        for (int c = 0; c < 3; c++)
                            for (int m = 0; m < nb; m++) {
                                double t = gu[i][c] * phi[m];
                                if (i == c) t += uq[0] * G[0][m] + uq[1] * G[1][m] + uq[2] * G[2][m];
                                M[(i * nb + a) * nd + c * nb + m] += wdet * phi[a] * t;
                            }
            } else if (form == ORC_LAPLACE) {
                /* int grad phi_a . grad phi_b |J|  ('cq,cqjd,cqje->cde') */
                for (int a = 0; a < nb; a++)
                    for (int b = 0; b < nb; b++) {
                        double s = 0.0;
                        for (int i = 0; i < 3; i++) s += G[i][a] * G[i][b];
                        M[a * nd + b] += wdet * s;
                    }
            } else {
                /* int e(v)^T D e(u) |J| = B^T D B  (linear elasticity form):
                 * B is the 6 x 3nb strain-displacement matrix at q */
                double D[6][6], Bm[6][3 * NB_MAX], DB[6][3 * NB_MAX];
                st = material_D(mat_kind, mat, e, q, nq, D);
                if (st) break;
                for (int I = 0; I < 6; I++)
                    for (int rr = 0; rr < 3; rr++)
                        for (int a = 0; a < nb; a++) Bm[I][rr * nb + a] = B_entry(I, rr, a, G);
                for (int I = 0; I < 6; I++)
                    for (int col = 0; col < nd; col++) {
                        double s = 0.0;
                        for (int K = 0; K < 6; K++) s += D[I][K] * Bm[K][col];
                        DB[I][col] = s;
                    }
                for (int row = 0; row < nd; row++)
                    for (int col = 0; col < nd; col++) {
                        double s = 0.0;
                        for (int I = 0; I < 6; I++) s += Bm[I][row] * DB[I][col];
                        M[row * nd + col] += wdet * s;
                    }
            }
        }
        if (st) {
#pragma omp critical
            if (!status || st == ERR_INDEX) status = st;
        }
    }
    ref_free(&r);
    return status;
}

int orc_matrix(int cell, int p, int form, int64_t n_cells, int64_t n_nodes,
               const double *coords, const int32_t *conn, int mat_kind,
               const double *mat, double *out)
{
    return orc_matrix_u(cell, p, form, n_cells, n_nodes, coords, conn, mat_kind, mat, NULL, out);
}

/* ------------------------------------------------------------------------ */
/* Residual mode: action on gathered DOFs (Algorithm "feloopv")             */
/* ------------------------------------------------------------------------ */

/* Gradient-first evaluation at one quadrature point: values/gradients of u at
 * the point, the flux, then the test-function contraction.  Also returns the
 * integrand of the eval mode (the energy density times wdet) in *energy. */
static int residual_qp(const ref_t *r, int form, int q, double wdet,
                       double (*G)[NB_MAX], const double *ue /*[nc][nb]*/,
                       int mat_kind, const double *mat, int64_t e,
                       double *re /*[nc][nb], accumulated*/, double *energy)
{
    const int nb = r->nb;
    const double *phi = r->bf + (size_t)q * nb;
    if (form == ORC_MASS || form == ORC_VMASS) {
        int nc = n_comp_of(form);
        for (int c = 0; c < nc; c++) {
            double uq = 0.0;
            for (int b = 0; b < nb; b++) uq += phi[b] * ue[c * nb + b];
            for (int a = 0; a < nb; a++) re[c * nb + a] += wdet * phi[a] * uq;
            *energy += wdet * uq * uq;
        }
        return 0;
    }
    if (form == ORC_WDOT) {
        /* test side phi_a, flux M u(q) */
        double uq[3];
        for (int c = 0; c < 3; c++) {
            double v = 0.0;
            for (int b = 0; b < nb; b++) v += phi[b] * ue[c * nb + b];
            uq[c] = v;
        }
        for (int i = 0; i < 3; i++) {
            double f = 0.0;
            for (int j = 0; j < 3; j++) f += wdot_M(mat, e, q, r->nq, i, j) * uq[j];
            for (int a = 0; a < nb; a++) re[i * nb + a] += wdet * phi[a] * f;
            *energy += wdet * uq[i] * f;
        }
        return 0;
    }
    if (form == ORC_CONVECT) {
        /* test side phi_a, flux (u . grad) u_i at the point */
        double uq[3], gu[3][3];
        field_at(r, q, G, ue, uq, gu);
        for (int i = 0; i < 3; i++) {
            const double f = gu[i][0] * uq[0] + gu[i][1] * uq[1] + gu[i][2] * uq[2];
            for (int a = 0; a < nb; a++) re[i * nb + a] += wdet * phi[a] * f;
            *energy += wdet * uq[i] * f;
        }
        return 0;
    }
    if (form == ORC_LAPLACE) {
        double gu[3] = {0, 0, 0};
        for (int i = 0; i < 3; i++)
            for (int b = 0; b < nb; b++) gu[i] += G[i][b] * ue[b];
        for (int a = 0; a < nb; a++)
            re[a] += wdet * (G[0][a] * gu[0] + G[1][a] * gu[1] + G[2][a] * gu[2]);
        *energy += wdet * (gu[0] * gu[0] + gu[1] * gu[1] + gu[2] * gu[2]);
        return 0;
    }
    /* elasticity: H[r][i] = du_r/dx_i, strain (Voigt), stress = D strain */
    double H[3][3];
    for (int rr = 0; rr < 3; rr++)
        for (int i = 0; i < 3; i++) {
            double s = 0.0;
            for (int b = 0; b < nb; b++) s += G[i][b] * ue[rr * nb + b];
            H[rr][i] = s;
        }
    double ev[6], sv[6], D[6][6];
    for (int I = 0; I < 6; I++) {
        int i = VOIGT_I[I], j = VOIGT_J[I];
        ev[I] = (i == j) ? H[i][i] : H[i][j] + H[j][i];
    }
    if (material_D(mat_kind, mat, e, q, r->nq, D)) return ERR_ARG;
    for (int I = 0; I < 6; I++) {
        double s = 0.0;
        for (int K = 0; K < 6; K++) s += D[I][K] * ev[K];
        sv[I] = s;
    }
    for (int rr = 0; rr < 3; rr++)
        for (int a = 0; a < nb; a++) {
            double s = 0.0;
            for (int I = 0; I < 6; I++) s += B_entry(I, rr, a, G) * sv[I];
            re[rr * nb + a] += wdet * s;
        }
    double en = 0.0;
    for (int I = 0; I < 6; I++) en += ev[I] * sv[I];
    *energy += wdet * en;
    return 0;
}

static int gather_dofs(const ref_t *r, int nc, int64_t e, const int32_t *conn,
                       const double *U, double *ue)
{
    for (int a = 0; a < r->nb; a++) {
        int64_t n = conn[e * r->nb + a];
        for (int c = 0; c < nc; c++) ue[c * r->nb + a] = U[n * nc + c];
    }
    return 0;
}

/* path 0: gradient-first (quadrature-point values first);
 * path 1: matrix-first (element matrix, then its product with u_e; linear
 * forms only: the convection matrix is a derivative, K(u) u = 2 r(u)).
 * out: (n_cells, nc, nb). */
int orc_residual(int cell, int p, int form, int64_t n_cells, int64_t n_nodes,
                 const double *coords, const int32_t *conn, int mat_kind,
                 const double *mat, const double *U, int path, double *out)
{
    if (check_common(cell, p, form, mat_kind) || (path != 0 && path != 1)) return ERR_ARG;
    if (form == ORC_CONVECT && path == 1) return ERR_ARG;
    ref_t r;
    if (ref_init(&r, cell, p)) { ref_free(&r); return ERR_ARG; }
    const int nb = r.nb, nq = r.nq, nc = n_comp_of(form), nd = nc * nb;
    int status = 0;
    double *Kbuf = NULL;
    if (path == 1) {
        Kbuf = (double *)malloc(sizeof(double) * (size_t)n_cells * nd * nd);
        if (!Kbuf) { ref_free(&r); return ERR_ARG; }
        status = orc_matrix(cell, p, form, n_cells, n_nodes, coords, conn, mat_kind, mat, Kbuf);
        if (status) { free(Kbuf); ref_free(&r); return status; }
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_cells; e++) {
        double x[NB_MAX][3], G[3][NB_MAX], ue[3 * NB_MAX];
        double *re = out + (size_t)e * nd;
        for (int k = 0; k < nd; k++) re[k] = 0.0;
        int st = gather_coords(&r, e, n_nodes, coords, conn, x);
        if (!st) gather_dofs(&r, nc, e, conn, U, ue);
        if (!st && path == 1) {
            const double *K = Kbuf + (size_t)e * nd * nd;
            for (int i = 0; i < nd; i++) {
                double s = 0.0;
                for (int j = 0; j < nd; j++) s += K[i * nd + j] * ue[j];
                re[i] = s;
            }
        }
        for (int q = 0; q < nq && !st && path == 0; q++) {
            double wdet, en = 0.0;
            st = geometry(&r, q, x, &wdet, G);
            if (!st) st = residual_qp(&r, form, q, wdet, G, ue, mat_kind, mat, e, re, &en);
        }
        if (st) {
#pragma omp critical
            if (!status || st == ERR_INDEX) status = st;
        }
    }
    free(Kbuf);
    ref_free(&r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Eval mode: per-element integral value u_e^T K_e u_e                      */
/* ------------------------------------------------------------------------ */

int orc_energy(int cell, int p, int form, int64_t n_cells, int64_t n_nodes,
               const double *coords, const int32_t *conn, int mat_kind,
               const double *mat, const double *U, double *out)
{
    if (check_common(cell, p, form, mat_kind)) return ERR_ARG;
    ref_t r;
    if (ref_init(&r, cell, p)) { ref_free(&r); return ERR_ARG; }
    const int nq = r.nq, nc = n_comp_of(form);
    int status = 0;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_cells; e++) {
        double x[NB_MAX][3], G[3][NB_MAX], ue[3 * NB_MAX], re[3 * NB_MAX];
        double en = 0.0;
        for (int k = 0; k < 3 * NB_MAX; k++) re[k] = 0.0;
        int st = gather_coords(&r, e, n_nodes, coords, conn, x);
        if (!st) gather_dofs(&r, nc, e, conn, U, ue);
        for (int q = 0; q < nq && !st; q++) {
            double wdet;
            st = geometry(&r, q, x, &wdet, G);
            if (!st) st = residual_qp(&r, form, q, wdet, G, ue, mat_kind, mat, e, re, &en);
        }
        out[e] = en;
        if (st) {
#pragma omp critical
            if (!status || st == ERR_INDEX) status = st;
        }
    }
    ref_free(&r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Gradient of J = sum_e u_e^T K_e u_e (linear elasticity, per-qp lambda/mu) */
/* ------------------------------------------------------------------------ */

/* g_mat:   (n_cells, nq, 2) dJ/dlambda, dJ/dmu at every quadrature point;
 *          J is linear in both: wdet (tr eps)^2 and 2 wdet eps:eps.
 * g_coords:(n_nodes, 3) dJ/dx, overwritten:
 *          dE/dx_{a,k} = sum_q wdet sum_l (W delta_kl - 2 (H^T sigma)_kl) G[l][a]
 *          with H = grad u, sigma = lambda tr(eps) I + 2 mu eps, W = eps:sigma;
 *          from d det = det sum_a G[:,a].dx_a and
 *          d(grad u) = -grad u sum_a dx_a (x) G[:,a].
 *          Element contributions are added to nodes in cell order. */
int orc_energy_grad(int cell, int p, int64_t n_cells, int64_t n_nodes,
                    const double *coords, const int32_t *conn, const double *lam_mu_qp,
                    const double *U, double *g_mat, double *g_coords)
{
    if (check_common(cell, p, ORC_ELASTICITY, ORC_MAT_ISO_QP)) return ERR_ARG;
    ref_t r;
    if (ref_init(&r, cell, p)) { ref_free(&r); return ERR_ARG; }
    const int nb = r.nb, nq = r.nq;
    int status = 0;
    double *part = NULL;
    if (g_coords) {
        part = (double *)calloc((size_t)n_cells * nb * 3, sizeof(double));
        if (!part) { ref_free(&r); return ERR_ARG; }
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_cells; e++) {
        double x[NB_MAX][3], G[3][NB_MAX], ue[3 * NB_MAX];
        int st = gather_coords(&r, e, n_nodes, coords, conn, x);
        if (!st) gather_dofs(&r, 3, e, conn, U, ue);
        for (int q = 0; q < nq && !st; q++) {
            double wdet;
            st = geometry(&r, q, x, &wdet, G);
            if (st) break;
            double lam = lam_mu_qp[2 * ((size_t)e * nq + q)];
            double mu = lam_mu_qp[2 * ((size_t)e * nq + q) + 1];
            double H[3][3], eps[3][3], sig[3][3];
            for (int rr = 0; rr < 3; rr++)
                for (int i = 0; i < 3; i++) {
                    double s = 0.0;
                    for (int b = 0; b < nb; b++) s += G[i][b] * ue[rr * nb + b];
                    H[rr][i] = s;
                }
            double tr = H[0][0] + H[1][1] + H[2][2];
            double ee = 0.0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    eps[i][j] = 0.5 * (H[i][j] + H[j][i]);
                    ee += eps[i][j] * eps[i][j];
                }
            if (g_mat) {
                g_mat[2 * ((size_t)e * nq + q)] = wdet * tr * tr;
                g_mat[2 * ((size_t)e * nq + q) + 1] = 2.0 * wdet * ee;
            }
            if (!part) continue;
            double W = 0.0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    sig[i][j] = 2.0 * mu * eps[i][j] + (i == j ? lam * tr : 0.0);
                    W += eps[i][j] * sig[i][j];
                }
            double Tm[3][3]; /* W delta - 2 H^T sigma */
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) {
                    double s = 0.0;
                    for (int rr = 0; rr < 3; rr++) s += H[rr][k] * sig[rr][l];
                    Tm[k][l] = (k == l ? W : 0.0) - 2.0 * s;
                }
            double *pe = part + (size_t)e * nb * 3;
            for (int a = 0; a < nb; a++)
                for (int k = 0; k < 3; k++) {
                    double s = 0.0;
                    for (int l = 0; l < 3; l++) s += Tm[k][l] * G[l][a];
                    pe[3 * a + k] += wdet * s;
                }
        }
        if (st) {
#pragma omp critical
            if (!status || st == ERR_INDEX) status = st;
        }
    }
    if (part && !status) {
        for (int64_t n = 0; n < 3 * n_nodes; n++) g_coords[n] = 0.0;
        for (int64_t e = 0; e < n_cells; e++)
            for (int a = 0; a < nb; a++) {
                int64_t n = conn[e * nb + a];
                for (int k = 0; k < 3; k++) g_coords[3 * n + k] += part[((size_t)e * nb + a) * 3 + k];
            }
    }
    free(part);
    ref_free(&r);
    return status;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel loops (the arithmetic does not depend on
 * it: every cell is computed by one thread, in the same order). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
