// Matrix-core element matrices of the two non-symmetric forms of the table
// of example weak forms on Q2 and Q3 hexahedra: the weighted vector dot
// product 'ij,i,j' and the Navier-Stokes convection matrix (the derivative
// of 'i,i.j,j', eq. fe4), in FP64 or FP32 with FP64 geometry.
//
// Both are, block by block (r, s = 0..2 the vector components),
//   K[(r,a),(s,b)] = sum_q phi_a(q) W_rs(q, b)
// with
//   weighted dot   W_rs(q, b) = w_q det J_q M_rs(q) phi_b(q)
//   convection     W_rs(q, b) = w_q det J_q (du_r/dx_s(q) phi_b(q)
//                                + delta_rs u(q) . grad phi_b(q))
// i.e. nine dense products Phi^T W_rs per cell, Phi (points x basis) being
// the basis values at the points, the same for every cell: it is built in
// LDS once per workgroup.
//
// One workgroup (8 waves) per cell at a time, persistent over an
// XCD-contiguous range of cells.  Per cell:
//   1. the reference derivatives of x (for the convection also those of u,
//      and u itself) at every point, by sum factorization over the 1-D
//      tables (FP64);
//   2. per point the nine block coefficients c_rs = w det J M_rs (weighted
//      dot) or w det J du_r/dx_s, with grad u = (du/dxi) J^-1 (convection),
//      and for the convection w det J v, v = J^-1 u the reference-space
//      velocity, so that u . grad phi_b = sum_j v_j dphi_b/dxi_j;
//   3. the W blocks in LDS in the contraction type (all nine for Q2, three
//      at a time for Q3), one (point, basis function) per item:
//      W_rs = c_rs phi_b (+ w det v . dphi_b/dxi on the diagonal blocks),
//      then every wave multiplies its 16x16 output tiles
//      (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32) over the points and
//      stores them.  Rows of 81 or 192 entries: Q2 tiles go out through the
//      L2 (their row segments straddle 128-byte lines), Q3 tiles
//      nontemporally.
#include "mm_device.h"

namespace fe {
namespace {

using mm::align_to;
using mm::op_stride;
using mm::store_tile;
using mm::valid;
using q2::cell_range;
using q2::MM_F32;
using q2::MM_F64;
using q2::MMT;

constexpr int GM_WAVES = 8;
constexpr int GM_THREADS = 64 * GM_WAVES;

template <int P, int FORM, int MM>
struct HexGM {
    static constexpr int N1 = P + 1, NB = N1 * N1 * N1, NQ = NB;
    static constexpr int ND = 3 * NB;  // output row length
    static constexpr int NBP = align_to(NB, 16), NT = NBP / 16;
    static constexpr bool RAGGED = NB % 16 != 0;
    static constexpr bool NT_STORE = ND % 16 == 0;
    using T = typename MMT<MM>::T;
    using ACC = typename MMT<MM>::acc;
    static constexpr int KP = align_to(NQ, 4), KS = op_stride(MM, KP);
    static constexpr int G = P <= 2 ? 9 : 3;  // blocks (r, s) per group
    static constexpr int NGRP = 9 / G;
    static constexpr int NTILE = G * NT * NT;                         // output tiles per group
    static constexpr int NJ = (NTILE + GM_WAVES - 1) / GM_WAVES;      // tiles per wave
    static constexpr bool CONV = FORM == FE_FORM_CONVECT;
    // entries per point from the sum factorization: dx_i/dxi_j (9); for the
    // convection also du_i/dxi_j (9) and u_i (3)
    static constexpr int NF = CONV ? 21 : 9;
    static constexpr int PS = CONV ? 12 : 9;  // per point: c_rs (9), then w det v (3)
    // LDS layout (bytes); the sum-factorization scratch F shares the space
    // of W, which is free between the last products of a cell and the
    // first W block of the next
    static constexpr int OFF_TB = 0;  // double B1[N1][N1], D1[N1][N1], w[NQ]
    // double xs[3][NB], then us[3][NB] (convection) or the cell's M[NQ][9]
    static constexpr int OFF_X = q2::align16(OFF_TB + (2 * N1 * N1 + NQ) * 8);
    static constexpr int OFF_P = q2::align16(OFF_X + (CONV ? 6 * NB : 3 * NB + 9 * NQ) * 8);  // double Pq[NQ][PS]
    static constexpr int OFF_A = q2::align16(OFF_P + NQ * PS * 8);               // T Phi[NBP][KS]
    static constexpr int OFF_W = q2::align16(OFF_A + NBP * KS * (int)sizeof(T));  // T W[G][NBP][KS]; double F[NF][NQ]
    static constexpr int W_BYTES = G * NBP * KS * (int)sizeof(T);
    static constexpr int F_BYTES = NF * NQ * 8;
    static constexpr int BYTES = q2::align16(OFF_W + (W_BYTES > F_BYTES ? W_BYTES : F_BYTES));
    // workgroups per CU the LDS allows (the launch bound asks for 2 MINB
    // waves per SIMD: 8 waves per workgroup over 4 SIMDs)
    static constexpr int MINB = P <= 2 ? 2 : 1;
    static_assert(BYTES * MINB <= 160 * 1024, "LDS");
};

template <int P, int FORM, int MM>
__global__ __launch_bounds__(GM_THREADS, (2 * HexGM<P, FORM, MM>::MINB)) void k_hexgm(ExecArgs A)
{
    using H = HexGM<P, FORM, MM>;
    using T = typename H::T;
    using ACC = typename H::ACC;
    constexpr int N1 = H::N1, NB = H::NB, NQ = H::NQ, NBP = H::NBP, NT = H::NT, KP = H::KP, KS = H::KS;
    constexpr int G = H::G, NF = H::NF, PS = H::PS, NJ = H::NJ;
    constexpr bool CONV = H::CONV;
    __shared__ __align__(16) unsigned char smem[H::BYTES];
    double *B1 = reinterpret_cast<double *>(smem + H::OFF_TB);
    double *D1 = B1 + N1 * N1;
    double *wq = D1 + N1 * N1;
    double *xs = reinterpret_cast<double *>(smem + H::OFF_X);  // [3][NB]
    double *us = xs + 3 * NB;                                  // [3][NB] (convection)
    double *Ms = xs + 3 * NB;                                  // [NQ][9] (weighted dot)
    double *Pq = reinterpret_cast<double *>(smem + H::OFF_P);  // [NQ][PS]
    T *Ph = reinterpret_cast<T *>(smem + H::OFF_A);            // [NBP][KS]
    T *W = reinterpret_cast<T *>(smem + H::OFF_W);             // [G][NBP][KS]
    double *F = reinterpret_cast<double *>(smem + H::OFF_W);   // [NF][NQ]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, grp = lane >> 4;

    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    if (e >= e_end) return;  // uniform over the workgroup
    const T *mat = static_cast<const T *>(A.mat);
    const T *Ug = static_cast<const T *>(A.dofs);

    for (int k = tid; k < N1 * N1; k += GM_THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < NQ; k += GM_THREADS) wq[k] = A.tab.w[k];
    __syncthreads();
    // Phi[b][q] = phi_b(q), zero in the padding rows and points
    for (int k = tid; k < NBP * KS; k += GM_THREADS) {
        const int b = k / KS, q = k - b * KS;
        double v = 0.0;
        if (b < NB && q < NQ) {
            const int b0 = b % N1, b1 = (b / N1) % N1, b2 = b / (N1 * N1);
            const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
            v = B1[q0 * N1 + b0] * B1[q1 * N1 + b1] * B1[q2 * N1 + b2];
        }
        Ph[k] = static_cast<T>(v);
    }

    for (; e < e_end; e += stride) {
        for (int k = tid; k < 3 * NB; k += GM_THREADS) {
            const int a = k / 3, c = k - 3 * a;
            const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
            xs[c * NB + a] = A.coords[3 * n + c];
            if constexpr (CONV) us[c * NB + a] = static_cast<double>(Ug[n * 3 + c]);
        }
        if constexpr (!CONV)
            for (int k = tid; k < NQ * 9; k += GM_THREADS) Ms[k] = static_cast<double>(mat[e * NQ * 9 + k]);
        __syncthreads();

        // 1. entry f at point q: f < 9: dx_i/dxi_j (i = f / 3, j = f % 3);
        //    9 <= f < 18: du_i/dxi_j; 18 <= f < 21: u_i
        for (int it = tid; it < NF * NQ; it += GM_THREADS) {
            const int q = it % NQ, f = it / NQ;
            const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
            const double *src = f < 9 ? xs + (f / 3) * NB : (f < 18 ? us + ((f - 9) / 3) * NB : us + (f - 18) * NB);
            const int j = f < 18 ? f % 3 : -1;
            const double *T0 = (j == 0 ? D1 : B1) + q0 * N1;
            const double *T1 = (j == 1 ? D1 : B1) + q1 * N1;
            const double *T2 = (j == 2 ? D1 : B1) + q2 * N1;
            double s2 = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < N1; a2++) {
                double s1 = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < N1; a1++) {
                    const double *xr = src + N1 * (a1 + N1 * a2);
                    double s0 = 0.0;
#pragma unroll
                    for (int a0 = 0; a0 < N1; a0++) s0 = fma(T0[a0], xr[a0], s0);
                    s1 = fma(T1[a1], s0, s1);
                }
                s2 = fma(T2[a2], s1, s2);
            }
            F[f * NQ + q] = s2;
        }
        __syncthreads();

        // 2. per point: the block coefficients c_rs and, for the convection,
        //    w det J v
        if (tid < NQ) {
            const int q = tid;
            double J[3][3], Ji[3][3];
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int c = 0; c < 3; c++) J[r][c] = F[(r * 3 + c) * NQ + q];
            const double det = inverse3(J, Ji);
            if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
            const double wd = wq[q] * det;
            double *pq = Pq + q * PS;
            if constexpr (CONV) {
                double u[3];
#pragma unroll
                for (int s = 0; s < 3; s++) u[s] = F[(18 + s) * NQ + q];
#pragma unroll
                for (int j = 0; j < 3; j++) pq[9 + j] = wd * (Ji[j][0] * u[0] + Ji[j][1] * u[1] + Ji[j][2] * u[2]);
#pragma unroll
                for (int r = 0; r < 3; r++)
#pragma unroll
                    for (int s = 0; s < 3; s++) {
                        double g = 0.0;
#pragma unroll
                        for (int j = 0; j < 3; j++) g = fma(F[(9 + r * 3 + j) * NQ + q], Ji[j][s], g);
                        pq[r * 3 + s] = wd * g;
                    }
            } else {
#pragma unroll
                for (int rs = 0; rs < 9; rs++) pq[rs] = wd * Ms[q * 9 + rs];
            }
        }
        __syncthreads();  // F (in W's space) is read for the last time above

        T *oc = static_cast<T *>(A.out) + e * static_cast<int64_t>(H::ND) * H::ND;
        for (int g = 0; g < H::NGRP; g++) {
            // 3a. W blocks rs = g G + bl, bl < G: item (b, q) writes row b,
            //     column q of each (zero at the padding rows and points)
            for (int it = tid; it < NBP * KP; it += GM_THREADS) {
                const int q = it % KP, b = it / KP;
                double phi = 0.0, adv = 0.0;
                const double *pq = Pq + (q < NQ ? q : 0) * PS;
                if (q < NQ && b < NB) {
                    const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
                    const int b0 = b % N1, b1 = (b / N1) % N1, b2 = b / (N1 * N1);
                    const double bx = B1[q0 * N1 + b0], by = B1[q1 * N1 + b1], bz = B1[q2 * N1 + b2];
                    phi = bx * by * bz;
                    if constexpr (CONV) {
                        const double dx = D1[q0 * N1 + b0], dy = D1[q1 * N1 + b1], dz = D1[q2 * N1 + b2];
                        adv = pq[9] * (dx * by * bz) + pq[10] * (bx * dy * bz) + pq[11] * (bx * by * dz);
                    }
                }
#pragma unroll
                for (int bl = 0; bl < G; bl++) {
                    const int rs = g * G + bl;
                    double x = pq[rs] * phi;
                    if (CONV && rs / 3 == rs % 3) x += adv;
                    W[(bl * NBP + b) * KS + q] = static_cast<T>(x);
                }
            }
            __syncthreads();

            // 3b. this wave's tiles t = wave + 8 u of the group: block bl,
            //     tile (ti, tj); slots past the last tile multiply tile 0
            //     and are not stored
            ACC acc[NJ];
            int ra[NJ], rb[NJ];
#pragma unroll
            for (int u = 0; u < NJ; u++) {
                acc[u] = ACC{};
                const int t = wave + GM_WAVES * u, tt = t < H::NTILE ? t : 0;
                const int bl = tt / (NT * NT), rem = tt - bl * (NT * NT), ti = rem / NT, tj = rem - ti * NT;
                ra[u] = 16 * ti;
                rb[u] = bl * NBP + 16 * tj;
            }
            // fragments of step k + 4 are loaded while step k multiplies
            // (the scheduling barriers keep the compiler from hoisting the
            // loads of every step ahead of the products)
            T a[2][NJ], b[2][NJ];
            auto load = [&](int buf, int k) {
#pragma unroll
                for (int u = 0; u < NJ; u++) {
                    a[buf][u] = Ph[(ra[u] + m) * KS + k + grp];
                    b[buf][u] = W[(rb[u] + m) * KS + k + grp];
                }
            };
            auto mfma = [&](int buf) {
#pragma unroll
                for (int u = 0; u < NJ; u++) {
                    if constexpr (MM == MM_F64)
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[buf][u], b[buf][u], acc[u], 0, 0, 0);
                    else
                        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[buf][u], b[buf][u], acc[u], 0, 0, 0);
                }
            };
            load(0, 0);
#pragma unroll
            for (int k = 0; k < KP; k += 4) {
                if (k + 4 < KP) load(((k >> 2) + 1) & 1, k + 4);
                __builtin_amdgcn_sched_barrier(0);
                mfma((k >> 2) & 1);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int u = 0; u < NJ; u++) {
                const int t = wave + GM_WAVES * u;
                if (t < H::NTILE) {
                    const int bl = t / (NT * NT), rem = t - bl * (NT * NT), ti = rem / NT, tj = rem - ti * NT;
                    const int rs = g * G + bl, r = rs / 3, s = rs - 3 * r;
                    store_tile<H>(oc, r * NB + 16 * ti, s * NB + 16 * tj, valid<H>(ti), valid<H>(tj), acc[u], lane);
                }
            }
            __syncthreads();  // W is rebuilt by the next group or cell
        }
    }
}

template <int P, int FORM, int MM>
int launch_hexgm(const Plan &, const ExecArgs &A, hipStream_t st)
{
    if (A.n_cells <= 0) return FE_OK;
    if (A.n_cells > 0x7fffffffLL) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    static int resident[64] = {0};
    int dev = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return FE_ERR_INVALID_ARG;
    if (!resident[dev]) {
        int per_cu = 0, cus = 0;
        FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hexgm<P, FORM, MM>, GM_THREADS, 0));
        FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        resident[dev] = per_cu * cus > 8 ? (per_cu * cus) & ~7 : 8;
    }
    const int64_t grid = A.n_cells < resident[dev] ? A.n_cells : resident[dev];
    hipLaunchKernelGGL((k_hexgm<P, FORM, MM>), dim3((unsigned)grid), dim3(GM_THREADS), 0, st, A);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <int P, int MM>
LaunchFn pick(const Plan &p)
{
    if (p.form == FE_FORM_WDOT && p.mat_kind == FE_MAT_TENSOR_QP) return launch_hexgm<P, FE_FORM_WDOT, MM>;
    if (p.form == FE_FORM_CONVECT) return launch_hexgm<P, FE_FORM_CONVECT, MM>;
    return nullptr;
}

template <int MM>
LaunchFn pick_order(const Plan &p)
{
    if (p.order == 2) return pick<2, MM>(p);
    if (p.order == 3) return pick<3, MM>(p);
    return nullptr;
}

}  // namespace

LaunchFn select_hexgm(const Plan &p)
{
    if (p.cell != FE_CELL_HEX || p.mode != FE_MODE_MATRIX) return nullptr;
    if (p.prec == FE_PREC_FP64) return pick_order<MM_F64>(p);
    if (p.prec == FE_PREC_FP32) return pick_order<MM_F32>(p);
    return nullptr;
}

}  // namespace fe
