// Sum-factorized residual (action) and eval kernels for Q_p hexahedra.
//
// The residual mode of the paper's element loop (Algorithm "feloopv") on the
// DOFs gathered through the connectivity, gradient first: values/gradients
// of u at the quadrature points, the flux there, then the test-function
// contraction.  On a tensor-product cell every one of those contractions over
// the (p+1)^3 nodes factors into three one-dimensional ones:
//   dx_i/dxi_0 (q) = sum_a2 B[q2][a2] sum_a1 B[q1][a1] sum_a0 D[q0][a0] x_i[a]
// (B, D: 1-D basis values/derivatives at the 1-D Gauss points), and the
// transposed contraction
//   r[a] = sum_q0 ( D[q0][a0] W0 + B[q0][a0] W12 ),
//   W0 = sum_q1 B[q1][a1] sum_q2 B[q2][a2] F0,
//   W12 = sum_q1 ( D[q1][a1] sum_q2 B[q2][a2] F1 + B[q1][a1] sum_q2 D[q2][a2] F2 ),
// which cuts the geometry work from 9 n_b n_q to about 48 (p+1)^4 FMA per
// component.  The Jacobian, its determinant and inverse stay FP64; u, the
// flux and the residual use the plan's precision.
//
// Mapping: one lane per point (node index and quadrature-point index share
// the lexicographic (i0, i1, i2) numbering), (p+1)^3 lanes per cell, as many
// cells per 256-thread workgroup as fit; each 1-D stage reads its 4 (or 3,
// 2) operands from LDS.  Output layouts: cell-major [n_cells][n_comp][n_b]
// (default) or cell-minor [n_comp][n_b][n_cells].
#include "fe_device.h"

namespace fe {
namespace {

template <int P, int FORM, typename T>
struct SF {
    static constexpr int N1 = P + 1, NP = N1 * N1 * N1;
    static constexpr int NC = form_nc(FORM);
    static constexpr int C = 256 / NP;  // cells per workgroup
    static constexpr bool GRAD = FORM == FE_FORM_LAPLACE || FORM == FE_FORM_ELASTICITY;
    // LDS per cell: coordinates, geometry stage buffers (FP64), u, u stage
    // buffers, residual stage buffers (T); phases reuse one scratch region
    static constexpr int GEO = (3 + 2 * 3 + 3 * 3) * NP * 8;
    static constexpr int UST = (NC + 2 * NC + 3 * NC) * NP * (int)sizeof(T);
    static constexpr int RST = (3 * NC + 3 * NC + 2 * NC) * NP * (int)sizeof(T);
    static constexpr int SCR = GEO > UST ? (GEO > RST ? GEO : RST) : (UST > RST ? UST : RST);
    static constexpr int PER = SCR + NP * (int)sizeof(T);  // + per-point energy
    static constexpr int BYTES = C * PER + 4 * N1 * N1 * 8;
};

// One 1-D contraction along axis AX for lane l = (i0, i1, i2):
//   out = sum_k M[k][idx] f(.., k at AX, ..)   when TR (transposed: sum over
//         the quadrature index k, the lane's AX index is the basis index)
//   out = sum_k M[idx][k] f(.., k at AX, ..)   otherwise
template <int N1, int AX, bool TR, typename T, typename M>
__device__ __forceinline__ T c1d(const T *f, const M *tab, int l, int idx)
{
    constexpr int S = AX == 0 ? 1 : (AX == 1 ? N1 : N1 * N1);
    const int base = l - idx * S;
    T s = T(0);
#pragma unroll
    for (int k = 0; k < N1; k++) s += static_cast<T>(TR ? tab[k * N1 + idx] : tab[idx * N1 + k]) * f[base + k * S];
    return s;
}

template <int P, int FORM, typename T>
__global__ __launch_bounds__(256) void k_sf(ExecArgs A, int cell_minor)
{
    using S = SF<P, FORM, T>;
    constexpr int N1 = S::N1, NP = S::NP, NC = S::NC, C = S::C;
    extern __shared__ __align__(16) unsigned char smem[];
    double *Bd = reinterpret_cast<double *>(smem);  // B[q][a], D[q][a] FP64
    double *Dd = Bd + N1 * N1;
    T *Bt = reinterpret_cast<T *>(Dd + N1 * N1);     // same in T
    T *Dt = Bt + N1 * N1;
    unsigned char *cells = smem + 4 * N1 * N1 * 8;

    const int tid = threadIdx.x;
    const int cs = tid / NP, l = tid - cs * NP;
    const int i0 = l % N1, i1 = (l / N1) % N1, i2 = l / (N1 * N1);
    const int64_t e = logical_block(A.xcd_remap) * C + cs;
    const bool live = cs < C && e < A.n_cells;
    unsigned char *mine = cells + (cs < C ? cs : 0) * S::PER;
    double *X = reinterpret_cast<double *>(mine);  // [3][NP] then stage buffers
    T *en = reinterpret_cast<T *>(mine + S::SCR);

    if (tid < N1 * N1) {
        Bd[tid] = A.tab.B1[tid];
        Dd[tid] = A.tab.D1[tid];
        Bt[tid] = static_cast<T>(A.tab.B1[tid]);
        Dt[tid] = static_cast<T>(A.tab.D1[tid]);
    }
    // gather coordinates and u of this lane's node (node index = l)
    T u[NC];
    if (live) {
        const int64_t n = checked_node(A.conn, e * NP + l, A.n_nodes, A.flags);
#pragma unroll
        for (int i = 0; i < 3; i++) X[i * NP + l] = A.coords[3 * n + i];
        const T *U = static_cast<const T *>(A.dofs);
#pragma unroll
        for (int c = 0; c < NC; c++) u[c] = U[n * NC + c];
    }
    __syncthreads();

    // ---- geometry (FP64): J[i][j] at quadrature point l by sum factorization
    double J[3][3] = {};
    if constexpr (S::GRAD || true) {
        double *tA = X + 3 * NP;       // [2][3][NP]  tB, tD
        double *tB = tA + 6 * NP;      // [3][3][NP]  uBB, uBD, uDB
        if (live) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                tA[(0 * 3 + i) * NP + l] = c1d<N1, 0, false>(X + i * NP, Bd, l, i0);
                tA[(1 * 3 + i) * NP + l] = c1d<N1, 0, false>(X + i * NP, Dd, l, i0);
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                tB[(0 * 3 + i) * NP + l] = c1d<N1, 1, false>(tA + (0 * 3 + i) * NP, Bd, l, i1);
                tB[(1 * 3 + i) * NP + l] = c1d<N1, 1, false>(tA + (0 * 3 + i) * NP, Dd, l, i1);
                tB[(2 * 3 + i) * NP + l] = c1d<N1, 1, false>(tA + (1 * 3 + i) * NP, Bd, l, i1);
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                J[i][0] = c1d<N1, 2, false>(tB + (2 * 3 + i) * NP, Bd, l, i2);
                J[i][1] = c1d<N1, 2, false>(tB + (1 * 3 + i) * NP, Bd, l, i2);
                J[i][2] = c1d<N1, 2, false>(tB + (0 * 3 + i) * NP, Dd, l, i2);
            }
        }
        __syncthreads();  // stage buffers are reused below
    }
    double Jid[3][3];
    const double det = inverse3(J, Jid);
    if (live && !(det > 0.0)) raise_fault(A.flags, FAULT_DET);
    const double wq = A.tab.w[l];
    const T w = static_cast<T>(wq * det);
    T Ji[3][3];
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
        for (int d = 0; d < 3; d++) Ji[j][d] = static_cast<T>(Jid[j][d]);

    // ---- values / reference gradients of u at the point, in T
    T *Us = reinterpret_cast<T *>(mine);  // [NC][NP], then stage buffers
    T *uA = Us + NC * NP;                 // [2][NC][NP]
    T *uB = uA + 2 * NC * NP;             // [3][NC][NP]
    if (live)
#pragma unroll
        for (int c = 0; c < NC; c++) Us[c * NP + l] = u[c];
    __syncthreads();
    T Hx[NC][3];
    T val[NC];
    if constexpr (S::GRAD) {
        if (live) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                uA[(0 * NC + c) * NP + l] = c1d<N1, 0, false>(Us + c * NP, Bt, l, i0);
                uA[(1 * NC + c) * NP + l] = c1d<N1, 0, false>(Us + c * NP, Dt, l, i0);
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                uB[(0 * NC + c) * NP + l] = c1d<N1, 1, false>(uA + (0 * NC + c) * NP, Bt, l, i1);
                uB[(1 * NC + c) * NP + l] = c1d<N1, 1, false>(uA + (0 * NC + c) * NP, Dt, l, i1);
                uB[(2 * NC + c) * NP + l] = c1d<N1, 1, false>(uA + (1 * NC + c) * NP, Bt, l, i1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; c++) {
            Hx[c][0] = live ? c1d<N1, 2, false>(uB + (2 * NC + c) * NP, Bt, l, i2) : T(0);
            Hx[c][1] = live ? c1d<N1, 2, false>(uB + (1 * NC + c) * NP, Bt, l, i2) : T(0);
            Hx[c][2] = live ? c1d<N1, 2, false>(uB + (0 * NC + c) * NP, Dt, l, i2) : T(0);
        }
    } else {
        if (live)
#pragma unroll
            for (int c = 0; c < NC; c++) uA[c * NP + l] = c1d<N1, 0, false>(Us + c * NP, Bt, l, i0);
        __syncthreads();
        if (live)
#pragma unroll
            for (int c = 0; c < NC; c++) uB[c * NP + l] = c1d<N1, 1, false>(uA + c * NP, Bt, l, i1);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; c++) val[c] = live ? c1d<N1, 2, false>(uB + c * NP, Bt, l, i2) : T(0);
    }
    __syncthreads();  // stage buffers are reused below

    // ---- flux at the point (reference space) and the energy density
    T F[NC][3];
    T energy = T(0);
    if constexpr (S::GRAD) {
        T H[NC][3];
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
            for (int d = 0; d < 3; d++) H[c][d] = Hx[c][0] * Ji[0][d] + Hx[c][1] * Ji[1][d] + Hx[c][2] * Ji[2][d];
        T Sg[NC][3];
        if constexpr (FORM == FE_FORM_LAPLACE) {
#pragma unroll
            for (int d = 0; d < 3; d++) Sg[0][d] = H[0][d];
            energy = w * (H[0][0] * H[0][0] + H[0][1] * H[0][1] + H[0][2] * H[0][2]);
        } else {
            const T *mat = static_cast<const T *>(A.mat);
            T lam = T(0), mu = T(0);
            if (live) {
                if (A.mat_kind == FE_MAT_ISO_QP) {
                    lam = mat[2 * (e * NP + l)];
                    mu = mat[2 * (e * NP + l) + 1];
                } else {
                    lam = mat[2 * e];
                    mu = mat[2 * e + 1];
                }
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
            energy = w * ee;
        }
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
            for (int j = 0; j < 3; j++) F[c][j] = w * (Ji[j][0] * Sg[c][0] + Ji[j][1] * Sg[c][1] + Ji[j][2] * Sg[c][2]);
    } else {
#pragma unroll
        for (int c = 0; c < NC; c++) {
            F[c][0] = w * val[c];
            energy += w * val[c] * val[c];
        }
    }

    T *out = static_cast<T *>(A.out);
    if (A.eval) {
        if (live) en[l] = energy;
        __syncthreads();
        if (live && l == 0) {
            T s = T(0);
            for (int k = 0; k < NP; k++) s += en[k];
            out[e] = s;
        }
        return;
    }

    // ---- transposed contraction with the test functions
    T *Fs = reinterpret_cast<T *>(mine);  // [NC][3][NP]
    T *rC = Fs + 3 * NC * NP;             // [3][NC][NP]
    T *rB = rC + 3 * NC * NP;             // [2][NC][NP]
    if (live)
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
            for (int j = 0; j < (S::GRAD ? 3 : 1); j++) Fs[(c * 3 + j) * NP + l] = F[c][j];
    __syncthreads();
    T res[NC];
    if constexpr (S::GRAD) {
        if (live) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                rC[(0 * NC + c) * NP + l] = c1d<N1, 2, true>(Fs + (c * 3 + 0) * NP, Bt, l, i2);
                rC[(1 * NC + c) * NP + l] = c1d<N1, 2, true>(Fs + (c * 3 + 1) * NP, Bt, l, i2);
                rC[(2 * NC + c) * NP + l] = c1d<N1, 2, true>(Fs + (c * 3 + 2) * NP, Dt, l, i2);
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                rB[(0 * NC + c) * NP + l] = c1d<N1, 1, true>(rC + (0 * NC + c) * NP, Bt, l, i1);
                rB[(1 * NC + c) * NP + l] = c1d<N1, 1, true>(rC + (1 * NC + c) * NP, Dt, l, i1) +
                                            c1d<N1, 1, true>(rC + (2 * NC + c) * NP, Bt, l, i1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; c++)
            res[c] = live ? c1d<N1, 0, true>(rB + (0 * NC + c) * NP, Dt, l, i0) +
                                c1d<N1, 0, true>(rB + (1 * NC + c) * NP, Bt, l, i0)
                          : T(0);
    } else {
        if (live)
#pragma unroll
            for (int c = 0; c < NC; c++) rC[c * NP + l] = c1d<N1, 2, true>(Fs + (c * 3) * NP, Bt, l, i2);
        __syncthreads();
        if (live)
#pragma unroll
            for (int c = 0; c < NC; c++) rB[c * NP + l] = c1d<N1, 1, true>(rC + c * NP, Bt, l, i1);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; c++) res[c] = live ? c1d<N1, 0, true>(rB + c * NP, Bt, l, i0) : T(0);
    }
    if (live) {
        if (cell_minor) {
#pragma unroll
            for (int c = 0; c < NC; c++) out[(c * NP + l) * A.n_cells + e] = res[c];
        } else {
#pragma unroll
            for (int c = 0; c < NC; c++) out[(e * NC + c) * NP + l] = res[c];
        }
    }
}

template <int P, int FORM, typename T>
int launch_sf(const Plan &p, const ExecArgs &A, hipStream_t st)
{
    using S = SF<P, FORM, T>;
    if (A.n_cells <= 0) return FE_OK;
    const int64_t blocks = (A.n_cells + S::C - 1) / S::C;
    if (blocks > 0x7fffffff) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    if (S::BYTES > 64 * 1024)
        FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(k_sf<P, FORM, T>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, S::BYTES));
    hipLaunchKernelGGL((k_sf<P, FORM, T>), dim3((unsigned)blocks), dim3(256), S::BYTES, st, A,
                       p.opts.layout == FE_LAYOUT_CELL_MINOR ? 1 : 0);
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
    }
    return nullptr;
}

template <typename T>
LaunchFn pick_order(int order, int form)
{
    if (order == 1) return pick<1, T>(form);
    if (order == 2) return pick<2, T>(form);
    if (order == 3) return pick<3, T>(form);
    return nullptr;
}

}  // namespace

LaunchFn select_sumfact(const Plan &p)
{
    if (p.cell != FE_CELL_HEX || p.mode == FE_MODE_MATRIX) return nullptr;
    if (p.form == FE_FORM_ELASTICITY && p.mat_kind == FE_MAT_VOIGT_QP) return nullptr;
    if (p.prec == FE_PREC_FP64) return pick_order<double>(p.order, p.form);
    if (p.prec == FE_PREC_FP32) return pick_order<float>(p.order, p.form);
    return nullptr;
}

}  // namespace fe
