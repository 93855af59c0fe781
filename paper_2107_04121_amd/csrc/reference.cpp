// Reference-element tables built by the library itself (host code).
//
// Quadrature: Gauss rules from the Golub-Welsch construction -- the nodes are
// the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// orthogonal polynomials of the weight, the weights are mu0 times the squared
// first components of the normalised eigenvectors.  The small symmetric
// eigenproblem is solved with cyclic Jacobi rotations.
//
// Basis: hexahedra tensorise 1-D Lagrange polynomials on equispaced nodes,
// each held in Newton form (divided differences of its nodal values) and
// evaluated with its derivative by the nested Newton-Horner scheme in x87
// extended precision (64-bit significand) and rounded once; the monomial
// form through an inverted Vandermonde matrix lost about 1e-13 of the values
// and 2e-12 of the slopes at order 5, the Newton form in double 2e-13 of the
// slopes.  Tetrahedra (P1/P2) express
// the basis in monomials by inverting the small Vandermonde matrix of the
// vertex and edge-midpoint nodes.
#include "fe_internal.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace fe {

namespace {

// Cyclic Jacobi eigen-solver for a small symmetric matrix (row-major n x n).
// On return A's diagonal holds the eigenvalues and V's columns the
// orthonormal eigenvectors.
void jacobi_eigen(int n, std::vector<double> &A, std::vector<double> &V)
{
    V.assign(n * n, 0.0);
    for (int i = 0; i < n; i++) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = i + 1; j < n; j++) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-34) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) /
                           (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; k++) {  // A <- A R
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {  // A <- R^T A
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
}

// Gauss rule with n points on [0,1] for the weight (1-s)^alpha (beta = 0 in
// Jacobi terms on [-1,1]).  Sorted ascending.
void gauss_rule(int n, int alpha, double *s, double *w)
{
    const double a = alpha, b = 0.0;
    std::vector<double> T(n * n, 0.0), V;
    for (int k = 0; k < n; k++) {
        double den = (2.0 * k + a + b) * (2.0 * k + a + b + 2.0);
        T[k * n + k] = (k == 0) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / den;
        if (k + 1 < n) {
            double m = k + 1.0, c = 2.0 * m + a + b;
            double off = std::sqrt(4.0 * m * (m + a) * (m + b) * (m + a + b) /
                                   (c * c * (c + 1.0) * (c - 1.0)));
            T[k * n + k + 1] = T[(k + 1) * n + k] = off;
        }
    }
    jacobi_eigen(n, T, V);
    // mu0 on [-1,1] = 2^(a+b+1) Gamma(a+1) Gamma(b+1) / Gamma(a+b+2); mapping
    // to [0,1] multiplies by 2^-(a+1) (dx/2 and ((1-x)/2)^a).
    double mu0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) /
                 std::tgamma(a + b + 2.0);
    double scale = std::pow(2.0, -(a + 1.0));
    std::vector<std::pair<double, double>> nw(n);
    for (int i = 0; i < n; i++) {
        double v0 = V[0 * n + i];
        nw[i] = {0.5 * (T[i * n + i] + 1.0), mu0 * v0 * v0 * scale};
    }
    for (int i = 0; i < n; i++)  // insertion sort by node
        for (int j = i; j > 0 && nw[j].first < nw[j - 1].first; j--) std::swap(nw[j], nw[j - 1]);
    for (int i = 0; i < n; i++) { s[i] = nw[i].first; w[i] = nw[i].second; }
}

// Inverse of a small dense matrix by Gauss-Jordan with partial pivoting.
bool invert(int n, std::vector<double> A, std::vector<double> &Ainv)
{
    Ainv.assign(n * n, 0.0);
    for (int i = 0; i < n; i++) Ainv[i * n + i] = 1.0;
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        for (int k = 0; k < n; k++) {
            std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(Ainv[c * n + k], Ainv[piv * n + k]);
        }
        double d = A[c * n + c];
        for (int k = 0; k < n; k++) { A[c * n + k] /= d; Ainv[c * n + k] /= d; }
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; k++) {
                A[r * n + k] -= f * A[c * n + k];
                Ainv[r * n + k] -= f * Ainv[c * n + k];
            }
        }
    }
    return true;
}

// 1-D Lagrange basis phi_k on the equispaced nodes x_m = m/p, in Newton
// form: c[k][j] are the divided differences [x_0..x_j] of the nodal values
// delta_mk, so phi_k(x) = sum_j c[k][j] prod_{m<j} (x - x_m).
void lagrange_newton(int p, std::vector<long double> &c)
{
    const int n = p + 1;
    c.assign(n * n, 0.0L);
    for (int k = 0; k < n; k++) {
        long double *d = &c[k * n];
        for (int m = 0; m < n; m++) d[m] = (m == k) ? 1.0L : 0.0L;
        for (int j = 1; j < n; j++)          // column j of the difference table
            for (int m = n - 1; m >= j; m--)  // in place, from the bottom
                d[m] = (d[m] - d[m - 1]) * ((long double)p / j);  // x_m - x_{m-j} = j/p
    }
}

// phi_k(x) and phi_k'(x) by the nested Newton scheme.
void newton_eval(int p, const long double *ck, double x, double &v, double &dv)
{
    long double pv = ck[p], pd = 0.0L;
    for (int j = p - 1; j >= 0; j--) {
        const long double t = (long double)x - (long double)j / p;
        pd = pd * t + pv;
        pv = pv * t + ck[j];
    }
    v = (double)pv;
    dv = (double)pd;
}

}  // namespace

int reference_sizes(int cell, int order, int *nb, int *nq)
{
    if (cell == FE_CELL_HEX && order >= 1 && order <= 5) {
        *nb = (order + 1) * (order + 1) * (order + 1);
        *nq = *nb;
        return FE_OK;
    }
    if (cell == FE_CELL_TET && (order == 1 || order == 2)) {
        *nb = order == 1 ? 4 : 10;
        *nq = (order + 1) * (order + 1) * (order + 1);
        return FE_OK;
    }
    return FE_ERR_UNSUPPORTED;
}

int hex_tables_1d(int p, double *s, double *w, double *B, double *D)
{
    // B[q][k] = phi_k(s_q), D[q][k] = phi_k'(s_q) for the (p+1)-point rule.
    int n = p + 1;
    gauss_rule(n, 0, s, w);
    std::vector<long double> c;
    lagrange_newton(p, c);
    for (int q = 0; q < n; q++)
        for (int k = 0; k < n; k++) newton_eval(p, &c[k * n], s[q], B[q * n + k], D[q * n + k]);
    return FE_OK;
}

int hex_factor_tables(int order, RefTables &T, std::string &why)
{
    // With tensor-product tables, summing bf over the second and third axes
    // of both the point and the node index leaves B1[q0][i] s^2, where s is
    // the sum of all entries of B1; summing that once more gives s^3.  The
    // same sums of bfg_0 give D1 s^2, and w[(q0,0,0)] = w1[q0] w1[0]^2 with
    // w1[0] = cbrt(w[0]).  The factors are then checked entry by entry.
    const int n = order + 1, nb = n * n * n, nq = nb;
    std::vector<double> Mb(n * n, 0.0), Md(n * n, 0.0);
    for (int q = 0; q < nq; q++)
        for (int a = 0; a < nb; a++) {
            const int q0 = q % n, a0 = a % n;
            Mb[q0 * n + a0] += T.bf[(size_t)q * nb + a];
            Md[q0 * n + a0] += T.bfg[((size_t)q * 3 + 0) * nb + a];
        }
    double s3 = 0.0;
    for (double v : Mb) s3 += v;
    const double s = std::cbrt(s3);
    if (!(std::fabs(s) > 1e-8)) {
        why = "hexahedral tables do not factor into 1-D tables";
        return FE_ERR_UNSUPPORTED;
    }
    T.B1.assign(n * n, 0.0);
    T.D1.assign(n * n, 0.0);
    T.w1.assign(n, 0.0);
    T.s1.assign(n, 0.0);
    for (int k = 0; k < n * n; k++) {
        T.B1[k] = Mb[k] / (s * s);
        T.D1[k] = Md[k] / (s * s);
    }
    const double w0 = std::cbrt(T.w[0]);
    for (int q0 = 0; q0 < n; q0++) T.w1[q0] = T.w[q0] / (w0 * w0);
    double err = 0.0, big = 0.0, werr = 0.0, wbig = 0.0;
    for (int q = 0; q < nq; q++) {
        const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
        werr = std::fmax(werr, std::fabs(T.w[q] - T.w1[q0] * T.w1[q1] * T.w1[q2]));
        wbig = std::fmax(wbig, std::fabs(T.w[q]));
        for (int a = 0; a < nb; a++) {
            const int a0 = a % n, a1 = (a / n) % n, a2 = a / (n * n);
            const double bx = T.B1[q0 * n + a0], by = T.B1[q1 * n + a1], bz = T.B1[q2 * n + a2];
            const double dx = T.D1[q0 * n + a0], dy = T.D1[q1 * n + a1], dz = T.D1[q2 * n + a2];
            const double ref[4] = {bx * by * bz, dx * by * bz, bx * dy * bz, bx * by * dz};
            const double got[4] = {T.bf[(size_t)q * nb + a], T.bfg[((size_t)q * 3 + 0) * nb + a],
                                   T.bfg[((size_t)q * 3 + 1) * nb + a], T.bfg[((size_t)q * 3 + 2) * nb + a]};
            for (int k = 0; k < 4; k++) {
                err = std::fmax(err, std::fabs(got[k] - ref[k]));
                big = std::fmax(big, std::fabs(got[k]));
            }
        }
    }
    if (err > 1e-12 * std::fmax(big, 1.0) || werr > 1e-12 * wbig) {
        why = "hexahedral tables are not tensor products of one 1-D rule and basis in lexicographic order "
              "(x fastest)";
        return FE_ERR_UNSUPPORTED;
    }
    return FE_OK;
}

int reference_tables(int cell, int order, RefTables &T)
{
    int nb, nq;
    int st = reference_sizes(cell, order, &nb, &nq);
    if (st) return st;
    T.cell = cell;
    T.order = order;
    T.nb = nb;
    T.nq = nq;
    T.w.assign(nq, 0.0);
    T.pts.assign(nq * 3, 0.0);
    T.bf.assign((size_t)nq * nb, 0.0);
    T.bfg.assign((size_t)nq * 3 * nb, 0.0);
    const int n = order + 1;
    if (cell == FE_CELL_HEX) {
        T.s1.assign(n, 0.0);
        T.w1.assign(n, 0.0);
        T.B1.assign(n * n, 0.0);
        T.D1.assign(n * n, 0.0);
        hex_tables_1d(order, T.s1.data(), T.w1.data(), T.B1.data(), T.D1.data());
        for (int q2 = 0; q2 < n; q2++)
            for (int q1 = 0; q1 < n; q1++)
                for (int q0 = 0; q0 < n; q0++) {
                    int q = q0 + n * (q1 + n * q2);
                    T.w[q] = T.w1[q0] * T.w1[q1] * T.w1[q2];
                    T.pts[3 * q] = T.s1[q0];
                    T.pts[3 * q + 1] = T.s1[q1];
                    T.pts[3 * q + 2] = T.s1[q2];
                    for (int k = 0; k < n; k++)
                        for (int j = 0; j < n; j++)
                            for (int i = 0; i < n; i++) {
                                int a = i + n * (j + n * k);
                                double bx = T.B1[q0 * n + i], by = T.B1[q1 * n + j], bz = T.B1[q2 * n + k];
                                double dx = T.D1[q0 * n + i], dy = T.D1[q1 * n + j], dz = T.D1[q2 * n + k];
                                T.bf[(size_t)q * nb + a] = bx * by * bz;
                                T.bfg[((size_t)q * 3 + 0) * nb + a] = dx * by * bz;
                                T.bfg[((size_t)q * 3 + 1) * nb + a] = bx * dy * bz;
                                T.bfg[((size_t)q * 3 + 2) * nb + a] = bx * by * dz;
                            }
                }
        return FE_OK;
    }
    // Tetrahedron.  Quadrature: conical product over the collapsed cube,
    // x = a, y = (1-a) b, z = (1-a)(1-b) c, Jacobian (1-a)^2 (1-b) taken by
    // Gauss-Jacobi weights (alpha = 2, 1) and Gauss-Legendre in c.
    double sa[8], wa[8], sb[8], wb[8], sc[8], wc[8];
    gauss_rule(n, 2, sa, wa);
    gauss_rule(n, 1, sb, wb);
    gauss_rule(n, 0, sc, wc);
    // Basis: monomials of total degree <= order, Vandermonde at the nodes.
    static const int exps1[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    static const int exps2[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                     {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    const int(*ex)[3] = order == 1 ? exps1 : exps2;
    double nodes[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    static const int edges[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
    if (order == 2)
        for (int e = 0; e < 6; e++)
            for (int d = 0; d < 3; d++)
                nodes[4 + e][d] = 0.5 * (nodes[edges[e][0]][d] + nodes[edges[e][1]][d]);
    std::vector<double> Vd(nb * nb), C;
    for (int i = 0; i < nb; i++)
        for (int m = 0; m < nb; m++)
            Vd[i * nb + m] = std::pow(nodes[i][0], ex[m][0]) * std::pow(nodes[i][1], ex[m][1]) *
                             std::pow(nodes[i][2], ex[m][2]);
    if (!invert(nb, Vd, C)) return FE_ERR_INVALID_ARG;
    auto mono = [](double x, int e) { return e == 0 ? 1.0 : std::pow(x, e); };
    auto dmono = [](double x, int e) { return e == 0 ? 0.0 : e * (e == 1 ? 1.0 : std::pow(x, e - 1)); };
    for (int ic = 0; ic < n; ic++)
        for (int ib = 0; ib < n; ib++)
            for (int ia = 0; ia < n; ia++) {
                int q = ia + n * (ib + n * ic);
                double x = sa[ia], y = (1.0 - sa[ia]) * sb[ib], z = (1.0 - sa[ia]) * (1.0 - sb[ib]) * sc[ic];
                T.w[q] = wa[ia] * wb[ib] * wc[ic];
                T.pts[3 * q] = x;
                T.pts[3 * q + 1] = y;
                T.pts[3 * q + 2] = z;
                for (int a = 0; a < nb; a++) {
                    double v = 0, gx = 0, gy = 0, gz = 0;
                    for (int m = 0; m < nb; m++) {
                        double c = C[m * nb + a];
                        double px = mono(x, ex[m][0]), py = mono(y, ex[m][1]), pz = mono(z, ex[m][2]);
                        v += c * px * py * pz;
                        gx += c * dmono(x, ex[m][0]) * py * pz;
                        gy += c * px * dmono(y, ex[m][1]) * pz;
                        gz += c * px * py * dmono(z, ex[m][2]);
                    }
                    T.bf[(size_t)q * nb + a] = v;
                    T.bfg[((size_t)q * 3 + 0) * nb + a] = gx;
                    T.bfg[((size_t)q * 3 + 1) * nb + a] = gy;
                    T.bfg[((size_t)q * 3 + 2) * nb + a] = gz;
                }
            }
    return FE_OK;
}

}  // namespace fe
