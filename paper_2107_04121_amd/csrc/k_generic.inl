// Generic per-element kernels (any cell kind and order the library supports).
//
// Included by k_generic_f64.hip / k_generic_f32.hip with GEN_T set to the
// contraction type and GEN_SUFFIX naming the selector.  One workgroup holds E
// cells: it gathers their node coordinates through the connectivity into LDS,
// computes the geometry of every (cell, quadrature point) pair in FP64 (one
// lane per pair), keeps w_q det J and the physical basis gradients in LDS in
// the contraction type, then contracts:
//   matrix mode   -- one lane per (cell, row, chunk of CB columns), summing
//                    over quadrature points in registers (the paper's matrix
//                    loop, Algorithm "feloopm"), stores CB contiguous entries;
//   residual/eval -- gradient-first: values/gradients of u and the flux per
//                    quadrature point, then one lane per (cell, row) contracts
//                    with the test functions (Algorithm "feloopv").
// The weighted vector dot product and the Navier-Stokes convection test with
// basis values, like the mass forms; the convection matrix is the derivative
// at the given DOFs (eq. fe4), so its matrix kernel also gathers u and keeps
// u and grad u at every point in LDS.
#include "fe_device.h"

namespace fe {
namespace {

using T = GEN_T;

constexpr int pick_cb(int n)
{
    const int c[] = {12, 10, 9, 8, 6, 5, 4, 3, 2, 1};
    for (int i = 0; i < 10; i++)
        if (n % c[i] == 0) return c[i];
    return 1;
}

constexpr int LDS_SOFT = 64 * 1024;

template <int CELL, int P, int FORM>
struct Gen {
    static constexpr int NB = cell_nb(CELL, P);
    static constexpr int NQ = cell_nq(CELL, P);
    static constexpr int NC = form_nc(FORM);
    static constexpr int ND = NC * NB;
    static constexpr bool NEED_G = FORM == FE_FORM_LAPLACE || FORM == FE_FORM_ELASTICITY || FORM == FE_FORM_CONVECT;
    static constexpr int MATW = FORM == FE_FORM_ELASTICITY ? 36 : (FORM == FE_FORM_WDOT ? 9 : 0);
    // forms whose test side is the basis value (flux width NC), not its gradient
    static constexpr bool TESTVAL = FORM == FE_FORM_MASS || FORM == FE_FORM_VMASS || FORM == FE_FORM_WDOT ||
                                    FORM == FE_FORM_CONVECT;
    // convection matrix: u gathered per cell, u and grad u per point
    static constexpr int UW = FORM == FE_FORM_CONVECT ? 12 : 0;
    static constexpr int CB = pick_cb(NB);
    static constexpr int NCH = ND / CB;
    // matrix kernel LDS per cell
    static constexpr int M_BYTES = NB * 3 * 8 + (NEED_G ? NQ * 3 * NB * (int)sizeof(T) : 0) +
                                   NQ * (int)sizeof(T) + NQ * MATW * (int)sizeof(T) +
                                   (UW ? (3 * NB + NQ * UW) * (int)sizeof(T) : 0);
    // residual kernel LDS per cell: coords, u, flux, energy, material
    static constexpr int FW = TESTVAL ? NC : 3 * NC;
    static constexpr int R_BYTES = NB * 3 * 8 + NC * NB * (int)sizeof(T) + NQ * FW * (int)sizeof(T) +
                                   NQ * (int)sizeof(T) + NQ * MATW * (int)sizeof(T);
    static constexpr int work_m = (NQ > ND ? NQ : ND);
    static constexpr int choose(int bytes, int work)
    {
        int e = 512 / work;
        if (e < 1) e = 1;
        while (e > 1 && e * bytes > LDS_SOFT) e--;
        return e;
    }
    static constexpr int EM = choose(M_BYTES, work_m);
    static constexpr int ER = choose(R_BYTES, (NQ > NB ? NQ : NB));
};

// Material coefficients of cell e at quadrature point q into its LDS slot:
// ISO kinds store (lambda, mu) in m[0], m[1]; VOIGT stores D row-major
// (36); TENSOR stores the weighted dot product's M row-major (9).
__device__ __forceinline__ void load_material(const ExecArgs &A, int64_t e, int q, int NQ, T *m)
{
    const T *mat = static_cast<const T *>(A.mat);
    if (A.mat_kind == FE_MAT_TENSOR_QP) {
        const T *d = mat + (e * NQ + q) * 9;
        for (int k = 0; k < 9; k++) m[k] = d[k];
    } else if (A.mat_kind == FE_MAT_ISO_CELL) {
        m[0] = mat[2 * e];
        m[1] = mat[2 * e + 1];
    } else if (A.mat_kind == FE_MAT_ISO_QP) {
        m[0] = mat[2 * (e * NQ + q)];
        m[1] = mat[2 * (e * NQ + q) + 1];
    } else {
        const T *d = mat + (e * NQ + q) * 36;
        for (int k = 0; k < 36; k++) m[k] = d[k];
    }
}

// Voigt strain-displacement row entries of basis function with physical
// gradient g for displacement component r: b[I] = B[I][(r, a)].
__device__ __forceinline__ void voigt_b(int r, const T g[3], T b[6])
{
    b[0] = r == 0 ? g[0] : T(0);
    b[1] = r == 1 ? g[1] : T(0);
    b[2] = r == 2 ? g[2] : T(0);
    b[3] = r == 0 ? g[1] : (r == 1 ? g[0] : T(0));
    b[4] = r == 0 ? g[2] : (r == 2 ? g[0] : T(0));
    b[5] = r == 1 ? g[2] : (r == 2 ? g[1] : T(0));
}

template <int CELL, int P, int FORM>
__global__ __launch_bounds__(256) void k_matrix(ExecArgs A)
{
    using C = Gen<CELL, P, FORM>;
    constexpr int NB = C::NB, NQ = C::NQ, ND = C::ND, E = C::EM, CB = C::CB, NCH = C::NCH;
    extern __shared__ __align__(16) unsigned char smem[];
    double *xs = reinterpret_cast<double *>(smem);
    T *Gs = reinterpret_cast<T *>(xs + E * NB * 3);
    T *wd = Gs + (C::NEED_G ? E * NQ * 3 * NB : 0);
    T *ms = wd + E * NQ;
    T *ug = ms + E * NQ * C::MATW;  // CONVECT: u [E][3][NB], then u, grad u [E][NQ][12]
    T *uh = ug + (C::UW ? E * 3 * NB : 0);

    const int64_t e0 = logical_block(A.xcd_remap) * E;
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int i = tid; i < E * NB; i += nt) {
        const int el = i / NB, a = i - el * NB;
        const int64_t e = e0 + el;
        double x0 = 0.0, x1 = 0.0, x2 = 0.0;
        T u[3] = {T(0), T(0), T(0)};
        if (e < A.n_cells) {
            const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
            x0 = A.coords[3 * n];
            x1 = A.coords[3 * n + 1];
            x2 = A.coords[3 * n + 2];
            if constexpr (C::UW != 0) {
                const T *U = static_cast<const T *>(A.dofs);
#pragma unroll
                for (int c = 0; c < 3; c++) u[c] = U[n * 3 + c];
            }
        }
        xs[i * 3 + 0] = x0;
        xs[i * 3 + 1] = x1;
        xs[i * 3 + 2] = x2;
        if constexpr (C::UW != 0) {
#pragma unroll
            for (int c = 0; c < 3; c++) ug[(el * 3 + c) * NB + a] = u[c];
        }
    }
    if constexpr (C::MATW != 0) {
        for (int i = tid; i < E * NQ; i += nt) {
            const int el = i / NQ, q = i - el * NQ;
            const int64_t e = e0 + el;
            if (e < A.n_cells) load_material(A, e, q, NQ, ms + i * C::MATW);
        }
    }
    __syncthreads();

    for (int i = tid; i < E * NQ; i += nt) {
        const int el = i / NQ, q = i - el * NQ;
        if (e0 + el >= A.n_cells) continue;
        double J[3][3], Ji[3][3];
        jacobian_qp<NB, NQ>(xs + el * NB * 3, A.tab.bfgT, q, J);
        const double det = inverse3(J, Ji);
        if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
        wd[i] = static_cast<T>(A.tab.w[q] * det);
        if constexpr (C::NEED_G) {
            T *g = Gs + i * 3 * NB;
            for (int a = 0; a < NB; a++) {
                const double r0 = A.tab.bfgT[(a * 3 + 0) * NQ + q];
                const double r1 = A.tab.bfgT[(a * 3 + 1) * NQ + q];
                const double r2 = A.tab.bfgT[(a * 3 + 2) * NQ + q];
#pragma unroll
                for (int d = 0; d < 3; d++)
                    g[d * NB + a] = static_cast<T>(r0 * Ji[0][d] + r1 * Ji[1][d] + r2 * Ji[2][d]);
            }
            if constexpr (C::UW != 0) {
                // u and grad u at the point (the state of the derivative)
                const T *u = ug + el * 3 * NB;
                T v[3] = {T(0), T(0), T(0)}, h[3][3] = {};
                for (int b = 0; b < NB; b++) {
                    const T ph = static_cast<T>(A.tab.bf[q * NB + b]);
                    const T gb[3] = {g[b], g[NB + b], g[2 * NB + b]};
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const T uc = u[c * NB + b];
                        v[c] += ph * uc;
#pragma unroll
                        for (int d = 0; d < 3; d++) h[c][d] += gb[d] * uc;
                    }
                }
                T *o = uh + i * C::UW;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    o[c] = v[c];
#pragma unroll
                    for (int d = 0; d < 3; d++) o[3 + c * 3 + d] = h[c][d];
                }
            }
        }
    }
    __syncthreads();

    T *out = static_cast<T *>(A.out);
    for (int it = tid; it < E * ND * NCH; it += nt) {
        const int cc = it % NCH;
        const int row = (it / NCH) % ND;
        const int el = it / (NCH * ND);
        const int64_t e = e0 + el;
        if (e >= A.n_cells) continue;
        const int col0 = cc * CB;
        const int s = col0 / NB, b0 = col0 - s * NB;
        const int r = row / NB, a = row - r * NB;
        T acc[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) acc[c] = T(0);
        if (!(FORM == FE_FORM_VMASS && r != s)) {
            for (int q = 0; q < NQ; q++) {
                const T w = wd[el * NQ + q];
                if constexpr (FORM == FE_FORM_MASS || FORM == FE_FORM_VMASS) {
                    const double *phi = A.tab.bf + q * NB;
                    const T wa = w * static_cast<T>(phi[a]);
#pragma unroll
                    for (int c = 0; c < CB; c++) acc[c] += wa * static_cast<T>(phi[b0 + c]);
                } else if constexpr (FORM == FE_FORM_WDOT) {
                    // w M_rs phi_a phi_b
                    const double *phi = A.tab.bf + q * NB;
                    const T wa = w * ms[(el * NQ + q) * 9 + r * 3 + s] * static_cast<T>(phi[a]);
#pragma unroll
                    for (int c = 0; c < CB; c++) acc[c] += wa * static_cast<T>(phi[b0 + c]);
                } else if constexpr (FORM == FE_FORM_CONVECT) {
                    // w phi_a (delta_rs u . grad phi_b + du_r/dx_s phi_b)
                    const double *phi = A.tab.bf + q * NB;
                    const T *g = Gs + (el * NQ + q) * 3 * NB;
                    const T *o = uh + (el * NQ + q) * C::UW;
                    const T wa = w * static_cast<T>(phi[a]), hrs = o[3 + r * 3 + s];
                    const T u0 = r == s ? o[0] : T(0), u1 = r == s ? o[1] : T(0), u2 = r == s ? o[2] : T(0);
#pragma unroll
                    for (int c = 0; c < CB; c++)
                        acc[c] += wa * (hrs * static_cast<T>(phi[b0 + c]) + u0 * g[b0 + c] + u1 * g[NB + b0 + c] +
                                        u2 * g[2 * NB + b0 + c]);
                } else {
                    const T *g = Gs + (el * NQ + q) * 3 * NB;
                    const T ga[3] = {g[a], g[NB + a], g[2 * NB + a]};
                    if constexpr (FORM == FE_FORM_LAPLACE) {
                        const T w0 = w * ga[0], w1 = w * ga[1], w2 = w * ga[2];
#pragma unroll
                        for (int c = 0; c < CB; c++)
                            acc[c] += w0 * g[b0 + c] + w1 * g[NB + b0 + c] + w2 * g[2 * NB + b0 + c];
                    } else {
                        const T *m = ms + (el * NQ + q) * 36;
                        if (A.mat_kind == FE_MAT_VOIGT_QP) {
                            T bA[6], Db[6];
                            voigt_b(r, ga, bA);
#pragma unroll
                            for (int K = 0; K < 6; K++) {
                                T t = T(0);
#pragma unroll
                                for (int I = 0; I < 6; I++) t += bA[I] * m[I * 6 + K];
                                Db[K] = w * t;
                            }
#pragma unroll
                            for (int c = 0; c < CB; c++) {
                                const T gb[3] = {g[b0 + c], g[NB + b0 + c], g[2 * NB + b0 + c]};
                                T bB[6];
                                voigt_b(s, gb, bB);
                                T t = T(0);
#pragma unroll
                                for (int K = 0; K < 6; K++) t += Db[K] * bB[K];
                                acc[c] += t;
                            }
                        } else {
                            const T wl = w * m[0], wm = w * m[1];
                            const T lar = wl * sel3(r, ga[0], ga[1], ga[2]);
                            const T mas = wm * sel3(s, ga[0], ga[1], ga[2]);
                            const T dg = (r == s) ? wm : T(0);
#pragma unroll
                            for (int c = 0; c < CB; c++) {
                                const T gb0 = g[b0 + c], gb1 = g[NB + b0 + c], gb2 = g[2 * NB + b0 + c];
                                acc[c] += lar * sel3(s, gb0, gb1, gb2) + mas * sel3(r, gb0, gb1, gb2) +
                                          dg * (ga[0] * gb0 + ga[1] * gb1 + ga[2] * gb2);
                            }
                        }
                    }
                }
            }
        }
        T *o = out + (e * ND + row) * ND + col0;
#pragma unroll
        for (int c = 0; c < CB; c++) o[c] = acc[c];
    }
}

template <int CELL, int P, int FORM>
__global__ __launch_bounds__(256) void k_residual(ExecArgs A)
{
    using C = Gen<CELL, P, FORM>;
    constexpr int NB = C::NB, NQ = C::NQ, NC = C::NC, E = C::ER, FW = C::FW;
    constexpr bool MASSLIKE = FORM == FE_FORM_MASS || FORM == FE_FORM_VMASS;
    constexpr bool TESTVAL = C::TESTVAL;
    extern __shared__ __align__(16) unsigned char smem[];
    double *xs = reinterpret_cast<double *>(smem);
    T *us = reinterpret_cast<T *>(xs + E * NB * 3);  // [E][NC][NB]
    T *F = us + E * NC * NB;                           // [E][NQ][FW]
    T *en = F + E * NQ * FW;                           // [E][NQ]
    T *ms = en + E * NQ;                               // [E][NQ][MATW]

    const int64_t e0 = logical_block(A.xcd_remap) * E;
    const int tid = threadIdx.x, nt = blockDim.x;
    const T *U = static_cast<const T *>(A.dofs);

    for (int i = tid; i < E * NB; i += nt) {
        const int el = i / NB, a = i - el * NB;
        const int64_t e = e0 + el;
        double x0 = 0.0, x1 = 0.0, x2 = 0.0;
        T u[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) u[c] = T(0);
        if (e < A.n_cells) {
            const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
            x0 = A.coords[3 * n];
            x1 = A.coords[3 * n + 1];
            x2 = A.coords[3 * n + 2];
#pragma unroll
            for (int c = 0; c < NC; c++) u[c] = U[n * NC + c];
        }
        xs[i * 3 + 0] = x0;
        xs[i * 3 + 1] = x1;
        xs[i * 3 + 2] = x2;
#pragma unroll
        for (int c = 0; c < NC; c++) us[(el * NC + c) * NB + a] = u[c];
    }
    if constexpr (C::MATW != 0) {
        for (int i = tid; i < E * NQ; i += nt) {
            const int el = i / NQ, q = i - el * NQ;
            const int64_t e = e0 + el;
            if (e < A.n_cells) load_material(A, e, q, NQ, ms + i * C::MATW);
        }
    }
    __syncthreads();

    for (int i = tid; i < E * NQ; i += nt) {
        const int el = i / NQ, q = i - el * NQ;
        if (e0 + el >= A.n_cells) continue;
        double J[3][3], Ji[3][3];
        jacobian_qp<NB, NQ>(xs + el * NB * 3, A.tab.bfgT, q, J);
        const double det = inverse3(J, Ji);
        if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
        const T w = static_cast<T>(A.tab.w[q] * det);
        const T *u = us + el * NC * NB;
        T *f = F + i * FW;
        if constexpr (MASSLIKE) {
            T energy = T(0);
#pragma unroll
            for (int c = 0; c < NC; c++) {
                T v = T(0);
                for (int a = 0; a < NB; a++) v += static_cast<T>(A.tab.bf[q * NB + a]) * u[c * NB + a];
                f[c] = w * v;
                energy += w * v * v;
            }
            en[i] = energy;
        } else if constexpr (FORM == FE_FORM_WDOT) {
            // flux M u(q); energy u . M u
            T v[3] = {T(0), T(0), T(0)};
            for (int a = 0; a < NB; a++) {
                const T ph = static_cast<T>(A.tab.bf[q * NB + a]);
#pragma unroll
                for (int c = 0; c < 3; c++) v[c] += ph * u[c * NB + a];
            }
            const T *m = ms + i * 9;
            T energy = T(0);
#pragma unroll
            for (int r = 0; r < 3; r++) {
                const T fr = m[r * 3] * v[0] + m[r * 3 + 1] * v[1] + m[r * 3 + 2] * v[2];
                f[r] = w * fr;
                energy += w * v[r] * fr;
            }
            en[i] = energy;
        } else {
            // reference gradients of u, then physical ones through J^-1
            T Hx[NC][3];
#pragma unroll
            for (int c = 0; c < NC; c++) Hx[c][0] = Hx[c][1] = Hx[c][2] = T(0);
            for (int a = 0; a < NB; a++) {
                const T r0 = static_cast<T>(A.tab.bfgT[(a * 3 + 0) * NQ + q]);
                const T r1 = static_cast<T>(A.tab.bfgT[(a * 3 + 1) * NQ + q]);
                const T r2 = static_cast<T>(A.tab.bfgT[(a * 3 + 2) * NQ + q]);
#pragma unroll
                for (int c = 0; c < NC; c++) {
                    const T uc = u[c * NB + a];
                    Hx[c][0] += r0 * uc;
                    Hx[c][1] += r1 * uc;
                    Hx[c][2] += r2 * uc;
                }
            }
            T Jt[3][3];
#pragma unroll
            for (int j = 0; j < 3; j++)
#pragma unroll
                for (int d = 0; d < 3; d++) Jt[j][d] = static_cast<T>(Ji[j][d]);
            T H[NC][3];
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int d = 0; d < 3; d++) H[c][d] = Hx[c][0] * Jt[0][d] + Hx[c][1] * Jt[1][d] + Hx[c][2] * Jt[2][d];
            T S[NC][3];  // physical flux
            T energy = T(0);
            if constexpr (FORM == FE_FORM_CONVECT) {
                // flux (u . grad) u at the point, tested with basis values
                T v[3] = {T(0), T(0), T(0)};
                for (int a = 0; a < NB; a++) {
                    const T ph = static_cast<T>(A.tab.bf[q * NB + a]);
#pragma unroll
                    for (int c = 0; c < 3; c++) v[c] += ph * u[c * NB + a];
                }
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const T fc = H[c][0] * v[0] + H[c][1] * v[1] + H[c][2] * v[2];
                    f[c] = w * fc;
                    energy += w * v[c] * fc;
                }
                en[i] = energy;
                continue;
            } else if constexpr (FORM == FE_FORM_LAPLACE) {
#pragma unroll
                for (int d = 0; d < 3; d++) S[0][d] = H[0][d];
                energy = w * (H[0][0] * H[0][0] + H[0][1] * H[0][1] + H[0][2] * H[0][2]);
            } else {
                const T *m = ms + i * 36;
                if (A.mat_kind == FE_MAT_VOIGT_QP) {
                    const T ev[6] = {H[0][0], H[1][1], H[2][2], H[0][1] + H[1][0], H[0][2] + H[2][0],
                                     H[1][2] + H[2][1]};
                    T sv[6];
#pragma unroll
                    for (int I = 0; I < 6; I++) {
                        T t = T(0);
#pragma unroll
                        for (int K = 0; K < 6; K++) t += m[I * 6 + K] * ev[K];
                        sv[I] = t;
                    }
                    S[0][0] = sv[0]; S[1][1] = sv[1]; S[2][2] = sv[2];
                    S[0][1] = S[1][0] = sv[3];
                    S[0][2] = S[2][0] = sv[4];
                    S[1][2] = S[2][1] = sv[5];
                } else {
                    const T lam = m[0], mu = m[1];
                    const T tr = H[0][0] + H[1][1] + H[2][2];
#pragma unroll
                    for (int c = 0; c < 3; c++)
#pragma unroll
                        for (int d = 0; d < 3; d++)
                            S[c][d] = mu * (H[c][d] + H[d][c]) + (c == d ? lam * tr : T(0));
                }
                T ee = T(0);
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int d = 0; d < 3; d++) ee += H[c][d] * S[c][d];
                energy = w * ee;
            }
            en[i] = energy;
            // reference flux: f[c][j] = w sum_d Ji[j][d] S[c][d]
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    f[c * 3 + j] = w * (Jt[j][0] * S[c][0] + Jt[j][1] * S[c][1] + Jt[j][2] * S[c][2]);
        }
    }
    __syncthreads();

    T *out = static_cast<T *>(A.out);
    if (A.eval) {
        for (int el = tid; el < E; el += nt) {
            const int64_t e = e0 + el;
            if (e >= A.n_cells) continue;
            T s = T(0);
            for (int q = 0; q < NQ; q++) s += en[el * NQ + q];
            out[e] = s;
        }
        return;
    }
    for (int it = tid; it < E * NC * NB; it += nt) {
        const int el = it / (NC * NB), row = it - el * NC * NB;
        const int64_t e = e0 + el;
        if (e >= A.n_cells) continue;
        const int c = row / NB, a = row - c * NB;
        T acc = T(0);
        for (int q = 0; q < NQ; q++) {
            const T *f = F + (el * NQ + q) * FW;
            if constexpr (TESTVAL) {
                acc += static_cast<T>(A.tab.bf[q * NB + a]) * f[c];
            } else {
                acc += static_cast<T>(A.tab.bfgT[(a * 3 + 0) * NQ + q]) * f[c * 3 + 0] +
                       static_cast<T>(A.tab.bfgT[(a * 3 + 1) * NQ + q]) * f[c * 3 + 1] +
                       static_cast<T>(A.tab.bfgT[(a * 3 + 2) * NQ + q]) * f[c * 3 + 2];
            }
        }
        out[e * NC * NB + row] = acc;
    }
}

template <typename K>
int launch_kernel(K kernel, int64_t n_cells, int per_block, int lds, const ExecArgs &A, hipStream_t st)
{
    if (n_cells <= 0) return FE_OK;
    const int64_t blocks = (n_cells + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    if (lds > LDS_SOFT) FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), lds, st, A);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <int CELL, int P, int FORM>
int launch_matrix(const Plan &, const ExecArgs &A, hipStream_t st)
{
    using C = Gen<CELL, P, FORM>;
    return launch_kernel(k_matrix<CELL, P, FORM>, A.n_cells, C::EM, C::EM * C::M_BYTES, A, st);
}

template <int CELL, int P, int FORM>
int launch_residual(const Plan &, const ExecArgs &A, hipStream_t st)
{
    using C = Gen<CELL, P, FORM>;
    return launch_kernel(k_residual<CELL, P, FORM>, A.n_cells, C::ER, C::ER * C::R_BYTES, A, st);
}

template <int CELL, int P>
LaunchFn pick_form(int form, int mode)
{
    const bool m = mode == FE_MODE_MATRIX;
    switch (form) {
    case FE_FORM_MASS: return m ? launch_matrix<CELL, P, FE_FORM_MASS> : launch_residual<CELL, P, FE_FORM_MASS>;
    case FE_FORM_VMASS: return m ? launch_matrix<CELL, P, FE_FORM_VMASS> : launch_residual<CELL, P, FE_FORM_VMASS>;
    case FE_FORM_LAPLACE:
        return m ? launch_matrix<CELL, P, FE_FORM_LAPLACE> : launch_residual<CELL, P, FE_FORM_LAPLACE>;
    case FE_FORM_ELASTICITY:
        return m ? launch_matrix<CELL, P, FE_FORM_ELASTICITY> : launch_residual<CELL, P, FE_FORM_ELASTICITY>;
    case FE_FORM_WDOT: return m ? launch_matrix<CELL, P, FE_FORM_WDOT> : launch_residual<CELL, P, FE_FORM_WDOT>;
    case FE_FORM_CONVECT:
        return m ? launch_matrix<CELL, P, FE_FORM_CONVECT> : launch_residual<CELL, P, FE_FORM_CONVECT>;
    }
    return nullptr;
}

}  // namespace

LaunchFn GEN_SUFFIX(const Plan &p)
{
    if (p.cell == FE_CELL_HEX) {
        if (p.order == 1) return pick_form<FE_CELL_HEX, 1>(p.form, p.mode);
        if (p.order == 2) return pick_form<FE_CELL_HEX, 2>(p.form, p.mode);
        if (p.order == 3) return pick_form<FE_CELL_HEX, 3>(p.form, p.mode);
    } else {
        if (p.order == 1) return pick_form<FE_CELL_TET, 1>(p.form, p.mode);
        if (p.order == 2) return pick_form<FE_CELL_TET, 2>(p.form, p.mode);
    }
    return nullptr;
}

}  // namespace fe
