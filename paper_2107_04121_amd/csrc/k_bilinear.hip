// Generic bilinear form kernel: any form  int v-operator . W . u-operator
// whose test and unknown operators are the basis values or the physical
// basis gradients of a scalar or vector variable and whose coupling W at
// each quadrature point is a constant matrix or P_test M(c, q) P_trial^T
// with M a per-point material matrix.  This is the shape of every bilinear
// term of the generalized notation once its identity and symmetric-gradient
// extractor operands are contracted (the divergence and the symmetric
// gradient are gradients with a particular coupling); the notation front-end
// derives the coupling tables, so a new bilinear form needs no new kernel.
//
// Rows of an operator are (component r, derivative j), component-major, with
// j absent for values: K_t = test_comp * (grad ? 3 : 1) rows for the test,
// K_u for the unknown.  Per cell and quadrature point q:
//   matrix   K[(r,a),(s,b)] += w det J  sum_{j,l} Phi_t[q][j][a] W_q[(r,j),(s,l)] Phi_u[q][l][b]
//   residual r[(r,a)]       += w det J  sum_j Phi_t[q][j][a] F_q[(r,j)],
//            F_q = W_q U_q,  U_q[(s,l)] = sum_b Phi_u[q][l][b] u_e[s][b]   (gradient first)
//   eval     E             += w det J  sum_(r,j) Ut_q[(r,j)] F_q[(r,j)]  (test bound to the same DOFs)
// Phi is the basis value phi_a(q) or the physical gradient G[q][j][a]
// (chain rule through J^-1, FP64 geometry).  One workgroup per cell at a
// time, a grid-stride loop over cells; the tables of one cell live in LDS.
#include "fe_device.h"

namespace fe {

// Everything the bilinear launcher passes to its kernel.
struct BilinearArgs {
    ExecArgs A;
    const double *coup;  // W0 [Kt][Ku], or P_test [Kt][n_a] followed by P_trial [Ku][n_b]
    int test_grad, test_comp, trial_grad, trial_comp;
    int Kt, Ku, n_a, n_b;
    int has_mat, mat_transpose;
    int mode;  // FE_MODE_*
};

namespace {

constexpr int BL_THREADS = 256;

template <int CELL, int P, typename T>
struct BL {
    static constexpr int NB = cell_nb(CELL, P);
    static constexpr int NQ = cell_nq(CELL, P);
};

template <int CELL, int P, typename T>
__global__ __launch_bounds__(BL_THREADS) void k_bilinear(BilinearArgs B)
{
    constexpr int NB = BL<CELL, P, T>::NB, NQ = BL<CELL, P, T>::NQ;
    __shared__ double xs[NB * 3];
    __shared__ double wd[NQ];
    __shared__ double Jis[NQ * 9];
    __shared__ T G[NQ * 3 * NB];
    __shared__ T Wq[NQ * 81];  // matrix: W_q scaled by w det J; residual/eval: U_q, F_q, Ut_q
    __shared__ T ub[3 * NB];
    __shared__ double red[BL_THREADS];
    const ExecArgs &A = B.A;
    const int tid = threadIdx.x;
    // Phi(q, j, a): the basis value (j = 0) or the physical gradient
    // component j (the LDS tables are indexed directly: no generic pointers
    // into LDS)
    // Both loads are issued and the values selected: a select between an
    // LDS and a global address would otherwise become one flat load.
    const __attribute__((address_space(1))) double *bfg1 = (const __attribute__((address_space(1))) double *)A.tab.bf;
    auto phi = [&](bool grad, int q, int j, int a) -> T {
        const T g = G[(q * 3 + j) * NB + a];
        const T v = static_cast<T>(bfg1[q * NB + a]);
        return grad ? g : v;
    };
    const bool any_grad = B.test_grad || B.trial_grad;
    const int Jt = B.test_grad ? 3 : 1, Ju = B.trial_grad ? 3 : 1;
    const int Kt = B.Kt, Ku = B.Ku;
    T *const out = static_cast<T *>(A.out);
    const T *const mat = static_cast<const T *>(A.mat);
    const T *const dofs = static_cast<const T *>(A.dofs);
    for (int64_t e = blockIdx.x; e < A.n_cells; e += gridDim.x) {
        unsigned fault = 0;
        // gather the node coordinates (and DOFs)
        for (int k = tid; k < NB * 3; k += BL_THREADS) {
            const int64_t n = checked_node(A.conn, e * NB + k / 3, A.n_nodes, A.flags);
            xs[k] = A.coords[3 * n + k % 3];
        }
        if (B.mode != FE_MODE_MATRIX)
            for (int k = tid; k < B.trial_comp * NB; k += BL_THREADS) {
                const int s = k / NB, b = k - s * NB;
                const int64_t n = checked_node(A.conn, e * NB + b, A.n_nodes, A.flags);
                ub[k] = dofs[n * B.trial_comp + s];
            }
        __syncthreads();
        // geometry, one thread per point (FP64)
        for (int q = tid; q < NQ; q += BL_THREADS) {
            double J[3][3], Ji[3][3];
            jacobian_qp<NB, NQ>(xs, A.tab.bfgT, q, J);
            const double det = inverse3(J, Ji);
            if (!(det > 0.0)) fault |= FAULT_DET;
            wd[q] = A.tab.w[q] * det;
#pragma unroll
            for (int k = 0; k < 3; k++)
#pragma unroll
                for (int i = 0; i < 3; i++) Jis[q * 9 + k * 3 + i] = Ji[k][i];
        }
        __syncthreads();
        // physical gradients G[q][i][a] = sum_k dphi_a/dxi_k (J^-1)_ki
        if (any_grad)
            for (int k = tid; k < NQ * NB; k += BL_THREADS) {
                const int q = k / NB, a = k - q * NB;
                const double g0 = A.tab.bfgT[(a * 3 + 0) * NQ + q], g1 = A.tab.bfgT[(a * 3 + 1) * NQ + q],
                             g2 = A.tab.bfgT[(a * 3 + 2) * NQ + q];
#pragma unroll
                for (int i = 0; i < 3; i++)
                    G[(q * 3 + i) * NB + a] =
                        static_cast<T>(g0 * Jis[q * 9 + i] + g1 * Jis[q * 9 + 3 + i] + g2 * Jis[q * 9 + 6 + i]);
            }
        if (B.mode == FE_MODE_MATRIX) {
            // W_q (scaled by w det J): constant W0 or P_test M P_trial^T
            for (int k = tid; k < NQ * Kt * Ku; k += BL_THREADS) {
                const int q = k / (Kt * Ku), rc = k - q * Kt * Ku, R = rc / Ku, C = rc - R * Ku;
                double w;
                if (!B.has_mat) {
                    w = B.coup[R * Ku + C];
                } else {
                    const double *Pt = B.coup, *Pu = B.coup + Kt * B.n_a;
                    const T *M = mat + (e * NQ + q) * (int64_t)(B.n_a * B.n_b);
                    w = 0.0;
                    for (int x = 0; x < B.n_a; x++) {
                        const double pt = Pt[R * B.n_a + x];
                        if (pt == 0.0) continue;
                        double m = 0.0;
                        for (int y = 0; y < B.n_b; y++) {
                            const double mxy = B.mat_transpose ? (double)M[y * B.n_a + x] : (double)M[x * B.n_b + y];
                            m += mxy * Pu[C * B.n_b + y];
                        }
                        w += pt * m;
                    }
                }
                Wq[k] = static_cast<T>(wd[q] * w);
            }
            __syncthreads();
            const int rows = B.test_comp * NB, cols = B.trial_comp * NB;
            for (int k = tid; k < rows * cols; k += BL_THREADS) {
                const int R = k / cols, C = k - R * cols;
                const int r = R / NB, a = R - r * NB, s = C / NB, b = C - s * NB;
                T acc = T(0);
                for (int q = 0; q < NQ; q++) {
                    const int w0 = q * Kt * Ku;
                    for (int j = 0; j < Jt; j++) {
                        const T pa = phi(B.test_grad, q, j, a);
                        const int wr = w0 + (r * Jt + j) * Ku + s * Ju;
                        T t = T(0);
                        for (int l = 0; l < Ju; l++) t += Wq[wr + l] * phi(B.trial_grad, q, l, b);
                        acc += pa * t;
                    }
                }
                out[e * (int64_t)rows * cols + k] = acc;
            }
        } else {
            __syncthreads();
            // Wq holds U_q at [q*9 + (s,l)], F_q at NQ*9 + [q*9 + (r,j)] and
            // the test operator on the DOFs (eval) at NQ*18 + [q*9 + (r,j)]
            constexpr int OF = NQ * 9, OT = NQ * 18;
            // U_q[(s,l)] = sum_b Phi_u[q][l][b] u[s][b]; in eval mode also the
            // test operator on the same DOFs
            for (int k = tid; k < NQ * Ku; k += BL_THREADS) {
                const int q = k / Ku, sl = k - q * Ku, s = sl / Ju, l = sl - s * Ju;
                T acc = T(0);
                for (int b = 0; b < NB; b++) acc += phi(B.trial_grad, q, l, b) * ub[s * NB + b];
                Wq[q * 9 + sl] = acc;
            }
            if (B.mode == FE_MODE_EVAL)
                for (int k = tid; k < NQ * Kt; k += BL_THREADS) {
                    const int q = k / Kt, rj = k - q * Kt, r = rj / Jt, j = rj - r * Jt;
                    T acc = T(0);
                    for (int a = 0; a < NB; a++) acc += phi(B.test_grad, q, j, a) * ub[r * NB + a];
                    Wq[OT + q * 9 + rj] = acc;
                }
            __syncthreads();
            // F_q = w det J W_q U_q
            for (int k = tid; k < NQ * Kt; k += BL_THREADS) {
                const int q = k / Kt, R = k - q * Kt;
                double f = 0.0;
                if (!B.has_mat) {
                    for (int C = 0; C < Ku; C++) f += B.coup[R * Ku + C] * (double)Wq[q * 9 + C];
                } else {
                    const double *Pt = B.coup, *Pu = B.coup + Kt * B.n_a;
                    const T *M = mat + (e * NQ + q) * (int64_t)(B.n_a * B.n_b);
                    for (int x = 0; x < B.n_a; x++) {
                        const double pt = Pt[R * B.n_a + x];
                        if (pt == 0.0) continue;
                        double m = 0.0;
                        for (int y = 0; y < B.n_b; y++) {
                            double v = 0.0;
                            for (int C = 0; C < Ku; C++) v += Pu[C * B.n_b + y] * (double)Wq[q * 9 + C];
                            const double mxy = B.mat_transpose ? (double)M[y * B.n_a + x] : (double)M[x * B.n_b + y];
                            m += mxy * v;
                        }
                        f += pt * m;
                    }
                }
                Wq[OF + q * 9 + R] = static_cast<T>(wd[q] * f);
            }
            __syncthreads();
            if (B.mode == FE_MODE_RESIDUAL) {
                for (int k = tid; k < B.test_comp * NB; k += BL_THREADS) {
                    const int r = k / NB, a = k - r * NB;
                    T acc = T(0);
                    for (int q = 0; q < NQ; q++)
                        for (int j = 0; j < Jt; j++)
                            acc += phi(B.test_grad, q, j, a) * Wq[OF + q * 9 + r * Jt + j];
                    out[e * (int64_t)B.test_comp * NB + k] = acc;
                }
            } else {
                double part = 0.0;
                for (int k = tid; k < NQ * Kt; k += BL_THREADS) {
                    const int q = k / Kt, R = k - q * Kt;
                    part += (double)Wq[OT + q * 9 + R] * (double)Wq[OF + q * 9 + R];
                }
                red[tid] = part;
                __syncthreads();
                for (int w = BL_THREADS / 2; w > 0; w >>= 1) {
                    if (tid < w) red[tid] += red[tid + w];
                    __syncthreads();
                }
                if (tid == 0) out[e] = static_cast<T>(red[0]);
            }
        }
        if (fault) raise_fault(A.flags, fault);
        __syncthreads();  // the LDS tables are rewritten for the next cell
    }
}

template <int CELL, int P, typename T>
int launch_bl(const Plan &p, const ExecArgs &A, hipStream_t st)
{
    if (A.n_cells <= 0) return FE_OK;
    BilinearArgs B{};
    B.A = A;
    B.coup = p.tab.coup;
    B.test_grad = p.bl.test_grad;
    B.test_comp = p.bl.test_comp;
    B.trial_grad = p.bl.trial_grad;
    B.trial_comp = p.bl.trial_comp;
    B.Kt = p.bl.Kt;
    B.Ku = p.bl.Ku;
    B.n_a = p.bl.n_a;
    B.n_b = p.bl.n_b;
    B.has_mat = p.mat_kind == FE_MAT_TENSOR_QP;
    B.mat_transpose = p.bl.mat_transpose;
    B.mode = p.mode;
    int dev = 0, cus = 256;
    FE_HIP_CHECK(hipGetDevice(&dev));
    FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t cap = (int64_t)cus * 8;
    const int64_t grid = A.n_cells < cap ? A.n_cells : cap;
    hipLaunchKernelGGL((k_bilinear<CELL, P, T>), dim3((unsigned)grid), dim3(BL_THREADS), 0, st, B);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <typename T>
LaunchFn select_bl_t(const Plan &p)
{
    if (p.cell == FE_CELL_HEX) {
        if (p.order == 1) return launch_bl<FE_CELL_HEX, 1, T>;
        if (p.order == 2) return launch_bl<FE_CELL_HEX, 2, T>;
        if (p.order == 3) return launch_bl<FE_CELL_HEX, 3, T>;
    } else {
        if (p.order == 1) return launch_bl<FE_CELL_TET, 1, T>;
        if (p.order == 2) return launch_bl<FE_CELL_TET, 2, T>;
    }
    return nullptr;
}

}  // namespace

LaunchFn select_bilinear(const Plan &p)
{
    if (p.form != FE_FORM_BILINEAR) return nullptr;
    if (p.prec == FE_PREC_FP64) return select_bl_t<double>(p);
    if (p.prec == FE_PREC_FP32) return select_bl_t<float>(p);
    return nullptr;
}

}  // namespace fe
