// Sum-factorized residual (action) and eval kernels for Q_p hexahedra.
//
// The residual mode of the paper's element loop (Algorithm "feloopv") on the
// DOFs gathered through the connectivity, gradient first: values/gradients
// of u at the quadrature points, the flux there, then the test-function
// contraction.  On a tensor-product cell every one of those contractions over
// the (p+1)^3 nodes factors into three one-dimensional ones:
//   dx_i/dxi_0 (q) = sum_a2 B[q2][a2] sum_a1 B[q1][a1] sum_a0 D[q0][a0] x_i[a]
// (B, D: 1-D basis values/derivatives at the 1-D Gauss points, [q][a]), and
// the transposed contraction
//   r[a] = sum_q0 ( D[q0][a0] W0 + B[q0][a0] W12 ),
//   W0 = sum_q1 B[q1][a1] sum_q2 B[q2][a2] F0,
//   W12 = sum_q1 ( D[q1][a1] sum_q2 B[q2][a2] F1 + B[q1][a1] sum_q2 D[q2][a2] F2 ),
// which cuts the work from O(p^6) to O(p^4) per cell.  The Jacobian, its
// determinant and inverse stay FP64; u, the flux and the residual use the
// plan's precision.
//
// Mapping: one lane per pencil, i.e. per line of N1 = p+1 points along one
// axis, so each 1-D contraction runs in the lane's registers; a cell takes
// N1^2 lanes of one wave (64 / N1^2 cells per wave).  Between the three axes
// the pencil values are transposed through the cell's LDS arrays; the lanes
// of a cell belong to one wave, so only wave-level ordering is needed, never
// a workgroup barrier.  The arrays are laid out so that these transposes
// hit distinct LDS banks (see idx).  The geometry is evaluated one
// coordinate component at a time and u one DOF component at a time, so a
// cell needs three stage arrays.
//
// Output layouts: cell-major [n_cells][n_comp][n_b] (default) or cell-minor
// [n_comp][n_b][n_cells].
//
// The weighted vector dot product and the convection use the same passes
// with value-type test functions: the flux at a point is w det J M u or
// w det J (u . grad) u, the latter from both the values and the gradients
// of u at the points.
//
// ADJ (elasticity only): the gradient of the eval value J = sum u^T K u.
// The same geometry and gradient passes, then at every point
//   dJ/dlambda = w det (tr eps)^2,  dJ/dmu = 2 w det eps:eps,
//   M = w det (W I - 2 H^T sigma),  W = eps:sigma,  H = grad u,
// and the transposed passes applied to the reference-space flux M J^-T give
// the per-(cell, node) partials of dJ/dx (the energy-momentum form), in the
// cell-major residual layout.
#include "cw_device.h"

namespace fe {
namespace {

using cw::ctab;
using cw::ctab_t;

// LDS writes of a wave before this point are seen by its LDS reads after it
// (a wave's LDS operations execute in order; this keeps the compiler from
// moving them across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P, int FORM, typename T>
struct SF {
    static constexpr int N1 = P + 1, NPL = N1 * N1, NP = N1 * NPL;
    static constexpr int CW = 64 / NPL;  // cells per wave
    static constexpr int CB = 4 * CW;    // cells per 256-thread workgroup
    static constexpr int NC = form_nc(FORM);
    // gradient test functions (and gradients of u); the other forms test
    // with values
    static constexpr bool GRAD = FORM == FE_FORM_LAPLACE || FORM == FE_FORM_ELASTICITY;
    static constexpr bool UGRAD = GRAD || FORM == FE_FORM_CONVECT;  // gradients of u at the points
    static constexpr bool UVAL = !GRAD;                            // values of u at the points
    // stage-array layout (see idx).  Q3: a dense XOR-swizzled 4x4x4 block,
    // no bank conflicts.  Q2: plane stride 20, array stride 49 and cell
    // stride 153 doubles, the best of a search over strides for the bank
    // conflicts of the nine transpose patterns (at most 2-way; 4-way with
    // the plain padded layout).  Other orders: planes and arrays padded by
    // one entry, the cell stride an odd multiple of 8 doubles.
    static constexpr int ZS = N1 == 3 ? 20 : NPL + 1;
    static constexpr int AS = N1 == 4 ? NP : (N1 == 3 ? 49 : N1 * ZS + 1);
    static constexpr int CELL = N1 == 3 ? 153
                                        : ((3 * AS + 7) / 8 % 2 == 0 ? (3 * AS + 7) / 8 + 1 : (3 * AS + 7) / 8) * 8;
};

// 1-D tables B[q][a], D[q][a]: FP64 through the scalar unit for the
// geometry, or converted once into registers in the contraction type.
struct TabC {
    const ctab_t *B, *D;
    __device__ __forceinline__ double b(int i) const { return B[i]; }
    __device__ __forceinline__ double d(int i) const { return D[i]; }
};
template <typename V, int NN>
struct TabR {
    V B[NN], D[NN];
    __device__ __forceinline__ V b(int i) const { return B[i]; }
    __device__ __forceinline__ V d(int i) const { return D[i]; }
};

// Position of (x0, x1, x2) in a stage array.  Every pass reads or writes
// with one coordinate fixed and the lanes of a cell spread over the other
// two.  For N1 = 4, (x0 ^ x2) + 4 (x1 ^ x2) + 16 x2 maps each of the three
// patterns onto 16 distinct double slots modulo 16, i.e. onto all 32
// four-byte LDS banks (16 lanes per pass for 8-byte accesses; two cells of
// 4-byte entries at an offset of 16 banks for 4-byte accesses): no bank
// conflicts.
template <int N1, int ZS>
__device__ __forceinline__ int idx(int x0, int x1, int x2)
{
    if constexpr (N1 == 4)
        return (x0 ^ x2) + 4 * (x1 ^ x2) + 16 * x2;
    else
        return x0 + N1 * x1 + ZS * x2;
}

// Three 1-D passes of one scalar field f given on the lane's axis-0 pencil
// (nodes (a0, p0, p1), a0 = 0..N1-1), through the cell's stage arrays L.
// GRAD: returns the reference gradient at the lane's axis-2 pencil of points
// (p0, p1, q2): g[q2][j] = d f / d xi_j; else the value v[q2].
template <int N1, int ZS, int AS, bool GRAD, typename V, typename TB>
__device__ __forceinline__ void forward3(const V (&f)[N1], V *L, const TB &tb, int p0, int p1, bool slot,
                                         V (&g)[N1][3], V (&v)[N1])
{
    V b0[N1], d0[N1];
#pragma unroll
    for (int q = 0; q < N1; q++) {
        V sb = V(0), sd = V(0);
#pragma unroll
        for (int a = 0; a < N1; a++) {
            sb += static_cast<V>(tb.b(q * N1 + a)) * f[a];
            if constexpr (GRAD) sd += static_cast<V>(tb.d(q * N1 + a)) * f[a];
        }
        b0[q] = sb;
        d0[q] = sd;
    }
    if (slot)
#pragma unroll
        for (int q = 0; q < N1; q++) {
            L[idx<N1, ZS>(q, p0, p1)] = b0[q];
            if constexpr (GRAD) L[AS + idx<N1, ZS>(q, p0, p1)] = d0[q];
        }
    wave_sync();
    // axis 1: lane = pencil (p0, *, p1)
    V gb[N1], gd[N1];
#pragma unroll
    for (int k = 0; k < N1; k++) {
        gb[k] = L[idx<N1, ZS>(p0, k, p1)];
        if constexpr (GRAD) gd[k] = L[AS + idx<N1, ZS>(p0, k, p1)];
    }
    V bb[N1], bd[N1], db[N1];
#pragma unroll
    for (int q = 0; q < N1; q++) {
        V s0 = V(0), s1 = V(0), s2 = V(0);
#pragma unroll
        for (int k = 0; k < N1; k++) {
            s0 += static_cast<V>(tb.b(q * N1 + k)) * gb[k];
            if constexpr (GRAD) {
                s1 += static_cast<V>(tb.d(q * N1 + k)) * gb[k];
                s2 += static_cast<V>(tb.b(q * N1 + k)) * gd[k];
            }
        }
        bb[q] = s0;
        bd[q] = s1;
        db[q] = s2;
    }
    // this lane's own pencil positions only: no other lane reads them now
    if (slot)
#pragma unroll
        for (int q = 0; q < N1; q++) {
            L[idx<N1, ZS>(p0, q, p1)] = bb[q];
            if constexpr (GRAD) {
                L[AS + idx<N1, ZS>(p0, q, p1)] = bd[q];
                L[2 * AS + idx<N1, ZS>(p0, q, p1)] = db[q];
            }
        }
    wave_sync();
    // axis 2: lane = pencil (p0, p1, *)
    V cb[N1], cd[N1], ce[N1];
#pragma unroll
    for (int k = 0; k < N1; k++) {
        cb[k] = L[idx<N1, ZS>(p0, p1, k)];
        if constexpr (GRAD) {
            cd[k] = L[AS + idx<N1, ZS>(p0, p1, k)];
            ce[k] = L[2 * AS + idx<N1, ZS>(p0, p1, k)];
        }
    }
    wave_sync();  // the arrays are rewritten by the next pass
#pragma unroll
    for (int q = 0; q < N1; q++) {
        V s0 = V(0), s1 = V(0), s2 = V(0);
#pragma unroll
        for (int k = 0; k < N1; k++) {
            if constexpr (GRAD) {
                s0 += static_cast<V>(tb.b(q * N1 + k)) * ce[k];  // D B B
                s1 += static_cast<V>(tb.b(q * N1 + k)) * cd[k];  // B D B
                s2 += static_cast<V>(tb.d(q * N1 + k)) * cb[k];  // B B D
            } else {
                s0 += static_cast<V>(tb.b(q * N1 + k)) * cb[k];
            }
        }
        if constexpr (GRAD) {
            g[q][0] = s0;
            g[q][1] = s1;
            g[q][2] = s2;
        } else {
            v[q] = s0;
        }
    }
}

template <int P, int FORM, typename T, bool ADJ, bool VOIGT = false>
__global__ __launch_bounds__(256) void k_sf(ExecArgs A, int cell_minor, T *gmat, double scale)
{
    using S = SF<P, FORM, T>;
    constexpr int N1 = S::N1, NPL = S::NPL, NP = S::NP, CW = S::CW, NC = S::NC, ZS = S::ZS, AS = S::AS;
    constexpr bool GRAD = S::GRAD, UGRAD = S::UGRAD, UVAL = S::UVAL;
    __shared__ double lds[S::CB * S::CELL];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int cw = lane / NPL, pp = lane - cw * NPL;
    const int p0 = pp % N1, p1 = pp / N1;
    const bool slot = cw < CW;  // lanes 64 - 64 % NPL .. 63 hold no cell
    const int cslot = slot ? cw : 0;
    const int64_t e = logical_block(A.xcd_remap) * S::CB + wave * CW + cslot;
    const bool live = slot && e < A.n_cells;
    double *Ld = lds + (wave * CW + cslot) * S::CELL;
    T *Lt = reinterpret_cast<T *>(Ld);
    const TabC tc{ctab(A.tab.B1), ctab(A.tab.D1)};
    TabR<T, N1 * N1> tt;
#pragma unroll
    for (int i = 0; i < N1 * N1; i++) {
        tt.B[i] = static_cast<T>(tc.b(i));
        tt.D[i] = static_cast<T>(tc.d(i));
    }
    unsigned fault = 0;

    // gather the lane's pencil of nodes a = a0 + N1 * pp (contiguous local
    // numbers): coordinates FP64, u in T
    double X[N1][3];
    T U[N1][NC];
    {
        int32_t nd[N1];
        const int32_t *cp = A.conn + (live ? e : 0) * NP + N1 * pp;
        if constexpr (N1 == 4) {
            const int4 v = *reinterpret_cast<const int4 *>(cp);
            nd[0] = v.x;
            nd[1] = v.y;
            nd[2] = v.z;
            nd[3] = v.w;
        } else if constexpr (N1 == 2) {
            const int2 v = *reinterpret_cast<const int2 *>(cp);
            nd[0] = v.x;
            nd[1] = v.y;
        } else {
#pragma unroll
            for (int a = 0; a < N1; a++) nd[a] = cp[a];
        }
        const T *Ug = static_cast<const T *>(A.dofs);
#pragma unroll
        for (int a = 0; a < N1; a++) {
            int64_t n = nd[a];
            if (n < 0 || n >= A.n_nodes) {
                if (live) fault |= FAULT_INDEX;
                n = 0;
            }
#pragma unroll
            for (int i = 0; i < 3; i++) X[a][i] = A.coords[3 * n + i];
#pragma unroll
            for (int c = 0; c < NC; c++) U[a][c] = Ug[n * NC + c];
        }
    }

    // ---- geometry (FP64), one coordinate component at a time
    double J[N1][3][3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        double f[N1], g[N1][3], v[N1];
#pragma unroll
        for (int a = 0; a < N1; a++) f[a] = X[a][i];
        forward3<N1, ZS, AS, true>(f, Ld, tc, p0, p1, slot, g, v);
#pragma unroll
        for (int q = 0; q < N1; q++)
#pragma unroll
            for (int j = 0; j < 3; j++) J[q][i][j] = g[q][j];
    }
    // det J, J^-1 and w det J at the lane's points (p0, p1, q2)
    T Ji[N1][3][3], wd[N1];
#pragma unroll
    for (int q = 0; q < N1; q++) {
        double Jid[3][3];
        const double det = inverse3(J[q], Jid);
        if (live && !(det > 0.0)) fault |= FAULT_DET;
        const int qi = pp + NPL * q;
        wd[q] = static_cast<T>(A.tab.w[qi] * det);
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int d = 0; d < 3; d++) Ji[q][j][d] = static_cast<T>(Jid[j][d]);
    }

    // ---- u at the points: reference gradients and/or values
    T gx[N1][NC][3], val[N1][NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
        T f[N1], g[N1][3], v[N1];
#pragma unroll
        for (int a = 0; a < N1; a++) f[a] = U[a][c];
        if constexpr (UGRAD) {
            forward3<N1, ZS, AS, true>(f, Lt, tt, p0, p1, slot, g, v);
#pragma unroll
            for (int q = 0; q < N1; q++)
#pragma unroll
                for (int j = 0; j < 3; j++) gx[q][c][j] = g[q][j];
        }
        if constexpr (UVAL) {
            forward3<N1, ZS, AS, false>(f, Lt, tt, p0, p1, slot, g, v);
#pragma unroll
            for (int q = 0; q < N1; q++) val[q][c] = v[q];
        }
    }

    // ---- flux at the points (reference space, weight folded in) and energy
    T F[N1][NC][3];
    T energy = T(0);
    T gsum[2] = {T(0), T(0)};  // ADJ with per-cell coefficients: this lane's dJ/dc
    const T *mat = static_cast<const T *>(A.mat);
    T lam = T(0), mu = T(0);
    if constexpr (FORM == FE_FORM_ELASTICITY)
        if (live && A.mat_kind == FE_MAT_ISO_CELL) {
            lam = mat[2 * e];
            mu = mat[2 * e + 1];
        }
#pragma unroll
    for (int q = 0; q < N1; q++) {
        if constexpr (GRAD) {
            T H[NC][3];  // physical gradient of u
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int d = 0; d < 3; d++)
                    H[c][d] = gx[q][c][0] * Ji[q][0][d] + gx[q][c][1] * Ji[q][1][d] + gx[q][c][2] * Ji[q][2][d];
            T Sg[NC][3];
            if constexpr (FORM == FE_FORM_LAPLACE) {
#pragma unroll
                for (int d = 0; d < 3; d++) Sg[0][d] = H[0][d];
                energy += wd[q] * (H[0][0] * H[0][0] + H[0][1] * H[0][1] + H[0][2] * H[0][2]);
            } else if constexpr (ADJ) {
                if (live && A.mat_kind == FE_MAT_ISO_QP) {
                    const int64_t k = e * NP + pp + NPL * q;
                    lam = mat[2 * k];
                    mu = mat[2 * k + 1];
                }
                const T tr = H[0][0] + H[1][1] + H[2][2];
                T eps[3][3], sig[3][3], ee = T(0), W = T(0);
#pragma unroll
                for (int r = 0; r < 3; r++)
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        eps[r][d] = T(0.5) * (H[r][d] + H[d][r]);
                        ee += eps[r][d] * eps[r][d];
                    }
#pragma unroll
                for (int r = 0; r < 3; r++)
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        sig[r][d] = T(2) * mu * eps[r][d] + (r == d ? lam * tr : T(0));
                        W += eps[r][d] * sig[r][d];
                    }
                const T g0 = wd[q] * tr * tr, g1 = T(2) * wd[q] * ee;
                if (A.mat_kind == FE_MAT_ISO_QP) {
                    if (live && gmat) {
                        const int64_t k = e * NP + pp + NPL * q;
                        gmat[2 * k] = static_cast<T>(scale * static_cast<double>(g0));
                        gmat[2 * k + 1] = static_cast<T>(scale * static_cast<double>(g1));
                    }
                } else {
                    gsum[0] += g0;
                    gsum[1] += g1;
                }
                // M[k][l] = w det (W delta_kl - 2 sum_r H[r][k] sig[r][l]); the
                // reference flux for the transposed passes is M J^-T
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    T Mk[3];
#pragma unroll
                    for (int l = 0; l < 3; l++) {
                        const T s2 = H[0][k] * sig[0][l] + H[1][k] * sig[1][l] + H[2][k] * sig[2][l];
                        Mk[l] = wd[q] * ((k == l ? W : T(0)) - T(2) * s2);
                    }
#pragma unroll
                    for (int j = 0; j < 3; j++) F[q][k][j] = Mk[0] * Ji[q][j][0] + Mk[1] * Ji[q][j][1] + Mk[2] * Ji[q][j][2];
                }
                continue;
            } else if constexpr (VOIGT) {
                // sigma = D eps in Voigt order 11,22,33,12,13,23 with
                // engineering shear; D row-major per point
                const T ev[6] = {H[0][0], H[1][1], H[2][2], H[0][1] + H[1][0], H[0][2] + H[2][0], H[1][2] + H[2][1]};
                T sv[6] = {};
                if (live) {
                    const T *D = mat + (e * NP + pp + NPL * q) * 36;
#pragma unroll
                    for (int I = 0; I < 6; I++) {
                        T x = T(0);
#pragma unroll
                        for (int K = 0; K < 6; K++) x += D[I * 6 + K] * ev[K];
                        sv[I] = x;
                    }
                }
                Sg[0][0] = sv[0];
                Sg[1][1] = sv[1];
                Sg[2][2] = sv[2];
                Sg[0][1] = Sg[1][0] = sv[3];
                Sg[0][2] = Sg[2][0] = sv[4];
                Sg[1][2] = Sg[2][1] = sv[5];
                T ee = T(0);
#pragma unroll
                for (int I = 0; I < 6; I++) ee += ev[I] * sv[I];
                energy += wd[q] * ee;
            } else {
                if (live && A.mat_kind == FE_MAT_ISO_QP) {
                    const int64_t k = e * NP + pp + NPL * q;
                    lam = mat[2 * k];
                    mu = mat[2 * k + 1];
                }
                const T tr = H[0][0] + H[1][1] + H[2][2];
                T ee = T(0);
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        Sg[c][d] = mu * (H[c][d] + H[d][c]) + (c == d ? lam * tr : T(0));
                        ee += H[c][d] * Sg[c][d];
                    }
                energy += wd[q] * ee;
            }
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    F[q][c][j] = wd[q] * (Ji[q][j][0] * Sg[c][0] + Ji[q][j][1] * Sg[c][1] + Ji[q][j][2] * Sg[c][2]);
        } else if constexpr (FORM == FE_FORM_WDOT) {
            // flux w det J M u (M row-major per point)
            T m[9] = {};
            if (live) {
                const T *mp = mat + (e * NP + pp + NPL * q) * 9;
#pragma unroll
                for (int k = 0; k < 9; k++) m[k] = mp[k];
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const T mu = m[3 * c] * val[q][0] + m[3 * c + 1] * val[q][1] + m[3 * c + 2] * val[q][2];
                F[q][c][0] = wd[q] * mu;
                energy += wd[q] * val[q][c] * mu;
            }
        } else if constexpr (FORM == FE_FORM_CONVECT) {
            // flux w det J (u . grad) u, grad u = (du/dxi) J^-1
#pragma unroll
            for (int c = 0; c < 3; c++) {
                T adv = T(0);
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    const T h = gx[q][c][0] * Ji[q][0][d] + gx[q][c][1] * Ji[q][1][d] + gx[q][c][2] * Ji[q][2][d];
                    adv += val[q][d] * h;
                }
                F[q][c][0] = wd[q] * adv;
                energy += wd[q] * val[q][c] * adv;
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                F[q][c][0] = wd[q] * val[q][c];
                energy += wd[q] * val[q][c] * val[q][c];
            }
        }
    }

    T *out = static_cast<T *>(A.out);
    if constexpr (ADJ) {
        if (A.mat_kind != FE_MAT_ISO_QP && gmat) {
            // per-cell dJ/dc: sum of the cell's lanes
            if (slot) {
                Lt[2 * pp] = gsum[0];
                Lt[2 * pp + 1] = gsum[1];
            }
            wave_sync();
            if (live && pp == 0) {
                double s0 = 0.0, s1 = 0.0;
                for (int k = 0; k < NPL; k++) {
                    s0 += static_cast<double>(Lt[2 * k]);
                    s1 += static_cast<double>(Lt[2 * k + 1]);
                }
                gmat[2 * e] = static_cast<T>(scale * s0);
                gmat[2 * e + 1] = static_cast<T>(scale * s1);
            }
            wave_sync();  // the arrays are rewritten below
        }
        if (!out) {
            if (fault) raise_fault(A.flags, fault);
            return;
        }
    }
    if (A.eval) {
        // cell sum of the lanes' point sums
        if (slot) Lt[pp] = energy;
        wave_sync();
        if (live && pp == 0) {
            T s = T(0);
            for (int k = 0; k < NPL; k++) s += Lt[k];
            out[e] = s;
        }
        if (fault) raise_fault(A.flags, fault);
        return;
    }

    // ---- transposed contraction with the test functions, per component
    T res[NC][N1];
#pragma unroll
    for (int c = 0; c < NC; c++) {
        // axis 2: lane = pencil (p0, p1, *) of points -> basis index a2
        if (slot)
#pragma unroll
            for (int a = 0; a < N1; a++) {
                T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
                for (int q = 0; q < N1; q++) {
                    s0 += tt.b(q * N1 + a) * F[q][c][0];
                    if constexpr (GRAD) {
                        s1 += tt.b(q * N1 + a) * F[q][c][1];
                        s2 += tt.d(q * N1 + a) * F[q][c][2];
                    }
                }
                Lt[idx<N1, ZS>(p0, p1, a)] = s0;
                if constexpr (GRAD) {
                    Lt[AS + idx<N1, ZS>(p0, p1, a)] = s1;
                    Lt[2 * AS + idx<N1, ZS>(p0, p1, a)] = s2;
                }
            }
        wave_sync();
        // axis 1: lane = pencil (p0, *, p1) -> a1
        {
            T r0[N1], r1[N1], r2[N1];
#pragma unroll
            for (int k = 0; k < N1; k++) {
                r0[k] = Lt[idx<N1, ZS>(p0, k, p1)];
                if constexpr (GRAD) {
                    r1[k] = Lt[AS + idx<N1, ZS>(p0, k, p1)];
                    r2[k] = Lt[2 * AS + idx<N1, ZS>(p0, k, p1)];
                }
            }
            if (slot)
#pragma unroll
                for (int a = 0; a < N1; a++) {
                    T s0 = T(0), s1 = T(0);
#pragma unroll
                    for (int k = 0; k < N1; k++) {
                        s0 += tt.b(k * N1 + a) * r0[k];
                        if constexpr (GRAD)
                            s1 += tt.d(k * N1 + a) * r1[k] + tt.b(k * N1 + a) * r2[k];
                    }
                    Lt[idx<N1, ZS>(p0, a, p1)] = s0;
                    if constexpr (GRAD) Lt[AS + idx<N1, ZS>(p0, a, p1)] = s1;
                }
        }
        wave_sync();
        // axis 0: lane = pencil (*, p0, p1) -> a0
        {
            T s0v[N1], s1v[N1];
#pragma unroll
            for (int k = 0; k < N1; k++) {
                s0v[k] = Lt[idx<N1, ZS>(k, p0, p1)];
                if constexpr (GRAD) s1v[k] = Lt[AS + idx<N1, ZS>(k, p0, p1)];
            }
#pragma unroll
            for (int a = 0; a < N1; a++) {
                T s = T(0);
#pragma unroll
                for (int k = 0; k < N1; k++) {
                    if constexpr (GRAD)
                        s += tt.d(k * N1 + a) * s0v[k] + tt.b(k * N1 + a) * s1v[k];
                    else
                        s += tt.b(k * N1 + a) * s0v[k];
                }
                res[c][a] = s;
            }
        }
        wave_sync();  // the arrays are rewritten for the next component
    }
    if (fault) raise_fault(A.flags, fault);
    if (live) {
        if (cell_minor) {
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int a = 0; a < N1; a++) out[(int64_t)(c * NP + N1 * pp + a) * A.n_cells + e] = res[c][a];
        } else {
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int a = 0; a < N1; a++) out[(e * NC + c) * NP + N1 * pp + a] = res[c][a];
        }
    }
}

template <int P, int FORM, typename T>
int launch_sf(const Plan &p, const ExecArgs &A, hipStream_t st)
{
    using S = SF<P, FORM, T>;
    if (A.n_cells <= 0) return FE_OK;
    const int64_t blocks = (A.n_cells + S::CB - 1) / S::CB;
    if (blocks > 0x7fffffff) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    const int minor = p.opts.layout == FE_LAYOUT_CELL_MINOR ? 1 : 0;
    // a separate instantiation for the per-point Voigt D keeps the
    // isotropic kernels' registers as they are
    if (FORM == FE_FORM_ELASTICITY && A.mat_kind == FE_MAT_VOIGT_QP)
        hipLaunchKernelGGL((k_sf<P, FORM, T, false, FORM == FE_FORM_ELASTICITY>), dim3((unsigned)blocks), dim3(256),
                           0, st, A, minor, static_cast<T *>(nullptr), 1.0);
    else
        hipLaunchKernelGGL((k_sf<P, FORM, T, false>), dim3((unsigned)blocks), dim3(256), 0, st, A, minor,
                           static_cast<T *>(nullptr), 1.0);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <int P, typename T>
LaunchFn pick(int form)
{
    switch (form) {
    case FE_FORM_MASS: return launch_sf<P, FE_FORM_MASS, T>;
    case FE_FORM_VMASS: return launch_sf<P, FE_FORM_VMASS, T>;
    case FE_FORM_LAPLACE: return launch_sf<P, FE_FORM_LAPLACE, T>;
    case FE_FORM_ELASTICITY: return launch_sf<P, FE_FORM_ELASTICITY, T>;
    case FE_FORM_WDOT: return launch_sf<P, FE_FORM_WDOT, T>;
    case FE_FORM_CONVECT: return launch_sf<P, FE_FORM_CONVECT, T>;
    }
    return nullptr;
}

template <typename T>
LaunchFn pick_order(int order, int form)
{
    if (order == 1) return pick<1, T>(form);
    if (order == 2) return pick<2, T>(form);
    if (order == 3) return pick<3, T>(form);
    if (order == 4) return pick<4, T>(form);
    if (order == 5) return pick<5, T>(form);
    return nullptr;
}

template <int P, typename T>
int launch_sf_adj(const ExecArgs &A, double scale, void *gmat, void *part, hipStream_t st)
{
    using S = SF<P, FE_FORM_ELASTICITY, T>;
    if (A.n_cells <= 0) return FE_OK;
    const int64_t blocks = (A.n_cells + S::CB - 1) / S::CB;
    if (blocks > 0x7fffffff) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    ExecArgs B = A;
    B.out = part;
    B.eval = 0;
    hipLaunchKernelGGL((k_sf<P, FE_FORM_ELASTICITY, T, true>), dim3((unsigned)blocks), dim3(256), 0, st, B, 0,
                       static_cast<T *>(gmat), scale);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <typename T>
int adj_order(int order, const ExecArgs &A, double scale, void *gmat, void *part, hipStream_t st)
{
    if (order == 1) return launch_sf_adj<1, T>(A, scale, gmat, part, st);
    if (order == 2) return launch_sf_adj<2, T>(A, scale, gmat, part, st);
    if (order == 3) return launch_sf_adj<3, T>(A, scale, gmat, part, st);
    if (order == 4) return launch_sf_adj<4, T>(A, scale, gmat, part, st);
    if (order == 5) return launch_sf_adj<5, T>(A, scale, gmat, part, st);
    return FE_ERR_UNSUPPORTED;
}

}  // namespace

int adjoint_sumfact(const Plan &p, const ExecArgs &A, double scale, void *gmat, void *part, hipStream_t st)
{
    if (p.cell != FE_CELL_HEX || p.form != FE_FORM_ELASTICITY ||
        (p.mat_kind != FE_MAT_ISO_CELL && p.mat_kind != FE_MAT_ISO_QP))
        return FE_ERR_UNSUPPORTED;
    if (p.prec == FE_PREC_FP64) return adj_order<double>(p.order, A, scale, gmat, part, st);
    if (p.prec == FE_PREC_FP32) return adj_order<float>(p.order, A, scale, gmat, part, st);
    return FE_ERR_UNSUPPORTED;
}

LaunchFn select_sumfact(const Plan &p)
{
    if (p.cell != FE_CELL_HEX || p.mode == FE_MODE_MATRIX) return nullptr;
    if (p.prec == FE_PREC_FP64) return pick_order<double>(p.order, p.form);
    if (p.prec == FE_PREC_FP32) return pick_order<float>(p.order, p.form);
    return nullptr;
}

}  // namespace fe
