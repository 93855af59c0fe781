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
//   3. Q3: the W blocks in LDS in the contraction type, three at a time,
//      one (point, basis function) per item: W_rs = c_rs phi_b (+ w det
//      v . dphi_b/dxi on the diagonal blocks); every wave multiplies its
//      16x16 output tiles (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32)
//      over the points and stores them nontemporally (rows of 192 entries:
//      whole 128-byte lines).
//      Q2: no W blocks.  A W fragment is c_rs times the Phi fragment of the
//      same rows (plus V = w det v . grad_xi phi, one matrix for the
//      convection's diagonal blocks), formed in registers; the weighted
//      dot's blocks are symmetric, so their (1,0) tiles are written as the
//      transposes of the (0,1) tiles.  The cell's matrix is staged in LDS
//      and leaves in linear 16-byte nontemporal stores (rows of 81 entries
//      straddle 128-byte lines).
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
    static constexpr bool ELAST = false;
    // entries per point from the sum factorization: dx_i/dxi_j (9); for the
    // convection also du_i/dxi_j (9) and u_i (3)
    static constexpr int NF = CONV ? 21 : 9;
    static constexpr int PS = CONV ? 12 : 9;  // per point: c_rs (9), then w det v (3)
    // Q2 (all nine blocks in one group): no W blocks.  The products take
    // W_rs = c_rs Phi (+ V on the diagonal blocks of the convection, V[b][q]
    // = w det v . grad_xi phi_b) straight from Phi, the point coefficients
    // and V, and the cell's matrix is staged in LDS after them and leaves in
    // linear 16-byte stores (its 81-entry rows straddle 128-byte lines, so
    // tile stores would write partial lines).
    static constexpr bool STAGE = G == 9;
    static constexpr int VEC = 16 / (int)sizeof(T);
    // LDS layout (bytes).  Region R holds, one after the other in a cell,
    // the sum-factorization scratch F, then W (Q3) or V (Q2 convection),
    // then (Q2) the staged matrix; F is free between the last products of a
    // cell and the first W block of the next.
    static constexpr int OFF_TB = 0;  // double B1[N1][N1], D1[N1][N1], w[NQ]
    // double xs[3][NB], then us[3][NB] (convection) or the cell's M[NQ][9]
    static constexpr int OFF_X = q2::align16(OFF_TB + (2 * N1 * N1 + NQ) * 8);
    // double Pq[KP][PS] (rows NQ.. are zero: the padding points)
    static constexpr int OFF_P = q2::align16(OFF_X + (CONV ? 6 * NB : 3 * NB + 9 * NQ) * 8);
    static constexpr int OFF_A = q2::align16(OFF_P + KP * PS * 8);               // T Phi[NBP][KS]
    static constexpr int OFF_W = q2::align16(OFF_A + NBP * KS * (int)sizeof(T));  // region R
    static constexpr int W_BYTES = STAGE ? (CONV ? NBP * KS * (int)sizeof(T) : 0) : G * NBP * KS * (int)sizeof(T);
    static constexpr int F_BYTES = NF * NQ * 8;
    static constexpr int K_BYTES = STAGE ? (ND * ND + VEC) * (int)sizeof(T) : 0;
    static constexpr int R_BYTES = q2::cmax(q2::cmax(W_BYTES, F_BYTES), K_BYTES);
    static constexpr int BYTES = q2::align16(OFF_W + R_BYTES);
    // workgroups per CU the LDS allows (the launch bound asks for 2 MINB
    // waves per SIMD: 8 waves per workgroup over 4 SIMDs)
    static constexpr int MINB = P <= 2 ? 2 : 1;
    static_assert(BYTES * MINB <= 160 * 1024, "LDS");
};

// The cell's coordinates into xs[3][NB], and its DOFs into us[3][NB]
// (convection) or its per-point M into Ms[NQ][9] (weighted dot).
template <class H>
__device__ __forceinline__ void gm_gather(const ExecArgs &A, int64_t e, double *xs, double *us, double *Ms, int tid)
{
    using T = typename H::T;
    constexpr int NB = H::NB, NQ = H::NQ;
    const T *mat = static_cast<const T *>(A.mat);
    const T *Ug = static_cast<const T *>(A.dofs);
    for (int k = tid; k < 3 * NB; k += GM_THREADS) {
        const int a = k / 3, c = k - 3 * a;
        const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
        xs[c * NB + a] = A.coords[3 * n + c];
        if constexpr (H::CONV) us[c * NB + a] = static_cast<double>(Ug[n * 3 + c]);
    }
    if constexpr (!H::CONV && !H::ELAST)
        for (int k = tid; k < NQ * 9; k += GM_THREADS) Ms[k] = static_cast<double>(mat[e * NQ * 9 + k]);
}

// Per-point data of the cell in Pq[NQ][PS] (F[NF][NQ]: scratch):
//   1. entry f at point q by sum factorization: f < 9: dx_i/dxi_j
//      (i = f / 3, j = f % 3); 9 <= f < 18: du_i/dxi_j; 18 <= f < 21: u_i;
//   2. the block coefficients c_rs and, for the convection, w det J v; for
//      elasticity J^-1 (row-major) and w det J.
// Contains one barrier, between the two steps.
template <class H>
__device__ __forceinline__ void gm_points(const ExecArgs &A, const double *B1, const double *D1, const double *wq,
                                          const double *xs, const double *us, const double *Ms, double *F, double *Pq,
                                          int tid)
{
    constexpr int N1 = H::N1, NB = H::NB, NQ = H::NQ, NF = H::NF, PS = H::PS;
    static_assert(NQ <= GM_THREADS, "one point per thread in step 2");
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
        if constexpr (H::ELAST) {
#pragma unroll
            for (int mm = 0; mm < 3; mm++)
#pragma unroll
                for (int j = 0; j < 3; j++) pq[mm * 3 + j] = Ji[mm][j];
            pq[9] = wd;
        } else if constexpr (H::CONV) {
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
}

template <int MM>
__device__ __forceinline__ typename MMT<MM>::acc gm_mma(typename MMT<MM>::T a, typename MMT<MM>::T b,
                                                      const typename MMT<MM>::acc &c)
{
    if constexpr (MM == MM_F64)
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Q2 (nine blocks of 2x2 tiles).  Weighted dot: every block is
// Phi^T diag(c_rs) Phi, symmetric, so its tiles (0,0), (0,1), (1,1) are
// computed and (1,0) is written as the transpose of (0,1): wave w takes
// those of block w (u = 0, 1, 2) and waves 0-2 one of block 8 (u = 3), 27
// tiles.  Convection (whose diagonal blocks add V): wave w takes the four
// tiles of block w (u = 0..3: ti = u % 2, tj = u / 2) and waves 0-3 tile
// (w % 2, w / 2) of block 8 (u = 4), 36 tiles.  (The symmetric plan for the
// convection's off-diagonal blocks, 30 tiles, measured slower.)
struct GmSlot {
    int bl, ti, tj;
    bool mirror, valid;
};

template <bool CONV>
__device__ __forceinline__ GmSlot gm_q2_slot(int wave, int u)
{
    if constexpr (CONV) {
        if (u < 4) return GmSlot{wave, u & 1, u >> 1, false, true};
        return GmSlot{8, wave & 1, wave >> 1, false, wave < 4};
    } else {
        if (u < 3) return GmSlot{wave, u == 2, u >= 1, u == 1, true};
        const int k = u == 3 && wave < 3 ? wave : -1;
        return GmSlot{8, k == 2, k >= 1, k == 1, k >= 0};
    }
}

// The Q2 products.  Both operands come from Phi: a fragment of W_rs (rows
// b, depth q) is c_rs(q) times the Phi fragment of the same rows, plus the
// V fragment on the diagonal blocks of the convection.  So a wave loads two
// Phi fragments (rows 0-15 and 16-31, the same for every block), its
// blocks' coefficients (one value per point: broadcast reads) and V where
// it needs it, per depth step.
template <class H>
__device__ __forceinline__ void gm_q2_products(const typename H::T *Ph, const double *Pq, const typename H::T *V,
                                               int wave, int m, int grp, typename H::ACC (&acc)[5])
{
    using T = typename H::T;
    constexpr int KS = H::KS, KP = H::KP, PS = H::PS, MM = sizeof(T) == 8 ? MM_F64 : MM_F32;
    static_assert(H::NT == 2 && H::G == 9 && H::NJ == 5, "Q2 tile plan");
    // wave-uniform: the tile of block 8, if any
    const GmSlot e = gm_q2_slot<H::CONV>(wave, H::CONV ? 4 : 3);
    const bool diag = H::CONV && (wave == 0 || wave == 4);
    const T *pa = Ph + m * KS + grp;
    const T *pv = V + m * KS + grp;
    const T *pve = V + (16 * e.tj + m) * KS + grp;
    const double *pc = Pq + grp * PS;
    T a0[2], a1[2], c[2], ce[2], v0[2], v1[2], ve[2];
    auto load = [&](int buf, int k) {
        a0[buf] = pa[k];
        a1[buf] = pa[16 * KS + k];
        c[buf] = static_cast<T>(pc[k * PS + wave]);
        if (e.valid) ce[buf] = static_cast<T>(pc[k * PS + 8]);
        if constexpr (H::CONV) {
            if (diag) {
                v0[buf] = pv[k];
                v1[buf] = pv[16 * KS + k];
            }
            if (e.valid) ve[buf] = pve[k];
        }
    };
    auto mfma = [&](int buf) {
        T b0 = c[buf] * a0[buf], b1 = c[buf] * a1[buf];
        if (diag) {
            b0 += v0[buf];
            b1 += v1[buf];
        }
        T ae = T(0), be = T(0);
        if (e.valid) {
            ae = e.ti ? a1[buf] : a0[buf];
            be = ce[buf] * (e.tj ? a1[buf] : a0[buf]);
            if constexpr (H::CONV) be += ve[buf];
        }
        if constexpr (H::CONV) {
            acc[0] = gm_mma<MM>(a0[buf], b0, acc[0]);
            acc[1] = gm_mma<MM>(a1[buf], b0, acc[1]);
            acc[2] = gm_mma<MM>(a0[buf], b1, acc[2]);
            acc[3] = gm_mma<MM>(a1[buf], b1, acc[3]);
            if (e.valid) acc[4] = gm_mma<MM>(ae, be, acc[4]);
        } else {
            acc[0] = gm_mma<MM>(a0[buf], b0, acc[0]);
            acc[1] = gm_mma<MM>(a0[buf], b1, acc[1]);
            acc[2] = gm_mma<MM>(a1[buf], b1, acc[2]);
            if (e.valid) acc[3] = gm_mma<MM>(ae, be, acc[3]);
        }
    };
    // fragments of step k + 4 are loaded while step k multiplies
    load(0, 0);
#pragma unroll
    for (int k = 0; k < KP; k += 4) {
        if (k + 4 < KP) load(((k >> 2) + 1) & 1, k + 4);
        __builtin_amdgcn_sched_barrier(0);
        mfma((k >> 2) & 1);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int P, int FORM, int MM>
__global__ __launch_bounds__(GM_THREADS, (2 * HexGM<P, FORM, MM>::MINB)) void k_hexgm(ExecArgs A)
{
    using H = HexGM<P, FORM, MM>;
    using T = typename H::T;
    using ACC = typename H::ACC;
    constexpr int N1 = H::N1, NB = H::NB, NQ = H::NQ, NBP = H::NBP, NT = H::NT, KP = H::KP, KS = H::KS;
    constexpr int G = H::G, PS = H::PS, NJ = H::NJ;
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

    for (int k = tid; k < N1 * N1; k += GM_THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < NQ; k += GM_THREADS) wq[k] = A.tab.w[k];
    __syncthreads();
    for (int k = tid; k < (KP - NQ) * PS; k += GM_THREADS) Pq[NQ * PS + k] = 0.0;
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

    // The next cell's data is prefetched in two hops and parked in xs / us /
    // Ms (free once gm_points is done) before this cell's stores: a wave's
    // loads complete only after its earlier stores, so a load issued after
    // the stores (the gather at the top of the next cell) would wait for
    // all of them.
    gm_gather<H>(A, e, xs, us, Ms, tid);
    __syncthreads();
    const T *mat = static_cast<const T *>(A.mat);
    const T *Ug = static_cast<const T *>(A.dofs);
    for (;;) {
        const int64_t en = e + stride;
        const bool has_next = en < e_end;
        // first hop: the next cell's connectivity (thread k < 3 nb: node k/3,
        // axis k%3) and its per-point M (weighted dot)
        constexpr int PM = (NQ * 9 + GM_THREADS - 1) / GM_THREADS;  // M entries per thread
        static_assert(3 * NB <= GM_THREADS, "one coordinate per thread");
        int32_t pn = 0;
        T pm[PM] = {};
        if (has_next) {
            if (tid < 3 * NB) pn = A.conn[en * NB + tid / 3];
            if constexpr (!CONV) {
#pragma unroll
                for (int k = 0; k < PM; k++)
                    if (tid + k * GM_THREADS < NQ * 9) pm[k] = mat[en * NQ * 9 + tid + k * GM_THREADS];
            }
        }
        gm_points<H>(A, B1, D1, wq, xs, us, Ms, F, Pq, tid);
        __syncthreads();  // F (in W's space) is read for the last time in gm_points
        // second hop: its coordinates (and DOFs); the empty asm keeps the
        // wait for the connectivity here
        double px = 0.0;
        T pu = T(0);
        if (has_next && tid < 3 * NB) {
            asm volatile("" : "+v"(pn));
            int64_t n = pn;
            if (n < 0 || n >= A.n_nodes) {
                raise_fault(A.flags, FAULT_INDEX);
                n = 0;
            }
            const int c = tid - 3 * (tid / 3);
            px = A.coords[3 * n + c];
            if constexpr (CONV) pu = Ug[n * 3 + c];
        }

        T *oc = static_cast<T *>(A.out) + e * static_cast<int64_t>(H::ND) * H::ND;
        for (int g = 0; g < H::NGRP; g++) {
            // 3a. W blocks rs = g G + bl, bl < G (Q2: V only): item (b, q)
            //     writes row b, column q of each (zero at the padding rows
            //     and points)
            if constexpr (H::STAGE) {
                if constexpr (CONV) {
                    for (int it = tid; it < NBP * KP; it += GM_THREADS) {
                        const int q = it % KP, b = it / KP;
                        double adv = 0.0;
                        if (q < NQ && b < NB) {
                            const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
                            const int b0 = b % N1, b1 = (b / N1) % N1, b2 = b / (N1 * N1);
                            const double bx = B1[q0 * N1 + b0], by = B1[q1 * N1 + b1], bz = B1[q2 * N1 + b2];
                            const double dx = D1[q0 * N1 + b0], dy = D1[q1 * N1 + b1], dz = D1[q2 * N1 + b2];
                            const double *pq = Pq + q * PS;
                            adv = pq[9] * (dx * by * bz) + pq[10] * (bx * dy * bz) + pq[11] * (bx * by * dz);
                        }
                        W[b * KS + q] = static_cast<T>(adv);
                    }
                    __syncthreads();
                }
            } else {
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
            }

            // 3b. this wave's tiles t = wave + 8 u of the group: block bl,
            //     tile (ti, tj); slots past the last tile multiply tile 0
            //     and are not stored (Q2: see gm_q2_products)
            ACC acc[NJ];
#pragma unroll
            for (int u = 0; u < NJ; u++) acc[u] = ACC{};
            if constexpr (H::STAGE) {
                gm_q2_products<H>(Ph, Pq, W, wave, m, grp, acc);
            } else {
                int ra[NJ], rb[NJ];
#pragma unroll
                for (int u = 0; u < NJ; u++) {
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
                    for (int u = 0; u < NJ; u++) acc[u] = gm_mma<MM>(a[buf][u], b[buf][u], acc[u]);
                };
                load(0, 0);
#pragma unroll
                for (int k = 0; k < KP; k += 4) {
                    if (k + 4 < KP) load(((k >> 2) + 1) & 1, k + 4);
                    __builtin_amdgcn_sched_barrier(0);
                    mfma((k >> 2) & 1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (g == 0 && has_next) {  // park the prefetched cell before the first stores
                if (tid < 3 * NB) {
                    const int a = tid / 3, c = tid - 3 * a;
                    xs[c * NB + a] = px;
                    if constexpr (CONV) us[c * NB + a] = static_cast<double>(pu);
                }
                if constexpr (!CONV) {
#pragma unroll
                    for (int k = 0; k < PM; k++)
                        if (tid + k * GM_THREADS < NQ * 9) Ms[tid + k * GM_THREADS] = static_cast<double>(pm[k]);
                }
            }
            if constexpr (H::STAGE) {
                // the cell's matrix row-major in W's space, shifted by h
                // entries so that LDS vectors line up with 16-byte aligned
                // output addresses (h from the address itself: the output
                // need only be aligned to its element size); then linear
                // 16-byte nontemporal stores
                const int64_t base = e * static_cast<int64_t>(H::ND) * H::ND;
                const int h = static_cast<int>(
                    (reinterpret_cast<uintptr_t>(static_cast<T *>(A.out) + base) / sizeof(T)) & (H::VEC - 1));
                T *Ks = W;
                __syncthreads();  // every wave is done reading W
#pragma unroll
                for (int u = 0; u < NJ; u++) {
                    const GmSlot t = gm_q2_slot<CONV>(wave, u);
                    if (t.valid) {
                        const int r = t.bl / 3, s = t.bl - 3 * r;
                        const int b = 16 * t.tj + m;
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int a = 16 * t.ti + mm::acc_row<MM>(lane, v);
                            if (a < NB && b < NB) {
                                Ks[h + (r * NB + a) * H::ND + s * NB + b] = acc[u][v];
                                if (t.mirror) Ks[h + (r * NB + b) * H::ND + s * NB + a] = acc[u][v];
                            }
                        }
                    }
                }
                __syncthreads();
                typedef T TV __attribute__((ext_vector_type(H::VEC)));
                constexpr int NK = H::ND * H::ND;
                const auto out = q2::gmem(static_cast<T *>(A.out));
                const auto aligned = (__attribute__((address_space(1))) TV *)(out + (base - h));
                const TV *k16 = reinterpret_cast<const TV *>(Ks);
                const int vf = h ? 1 : 0, vl = (NK + h) / H::VEC;  // whole vectors [vf, vl)
                constexpr int NV = ((NK + 2 * H::VEC - 1) / H::VEC + GM_THREADS - 1) / GM_THREADS;
                constexpr int BATCH = 4;
#pragma unroll
                for (int j0 = 0; j0 < NV; j0 += BATCH) {
                    TV buf[BATCH];
#pragma unroll
                    for (int j = 0; j < BATCH; j++) {
                        const int v = vf + tid + GM_THREADS * (j0 + j);
                        if (j0 + j < NV && v < vl) buf[j] = k16[v];
                    }
#pragma unroll
                    for (int j = 0; j < BATCH; j++) {
                        const int v = vf + tid + GM_THREADS * (j0 + j);
                        if (j0 + j < NV && v < vl) __builtin_nontemporal_store(buf[j], aligned + v);
                    }
                }
                // the entries before the first and after the last whole vector
                if (tid < 2 * H::VEC) {
                    const int f = tid < H::VEC ? tid : vl * H::VEC - h + (tid - H::VEC);
                    const bool head = tid < H::VEC && f < vf * H::VEC - h;
                    const bool tail = tid >= H::VEC && f < NK;
                    if (head || tail) out[base + f] = Ks[h + f];
                }
            } else {
#pragma unroll
                for (int u = 0; u < NJ; u++) {
                    const int t = wave + GM_WAVES * u;
                    if (t < H::NTILE) {
                        const int bl = t / (NT * NT), rem = t - bl * (NT * NT), ti = rem / NT, tj = rem - ti * NT;
                        const int rs = g * G + bl, r = rs / 3, s = rs - 3 * r;
                        store_tile<H>(oc, r * NB + 16 * ti, s * NB + 16 * tj, valid<H>(ti), valid<H>(tj), acc[u], lane);
                    }
                }
            }
            __syncthreads();  // W is rebuilt by the next group or cell
        }
        if (!has_next) break;
        e = en;
    }
}


// ---------------------------------------------------------------------------
// Q4 and Q5: the points in chunks.
//
// Phi (224 x 216 at Q5) and the nine W blocks no longer fit in LDS.  The
// per-point coefficients are computed once per cell as above; the output
// tiles (nine blocks of NT x NT) are taken in passes of 8 NJ tiles, NJ
// accumulators per wave (16 FP64 / 32 FP32 tiles) that stay in registers
// while the points go by in chunks of KC = 16:
//   for each pass: for each chunk: Phi chunk (read from the basis table,
//   the same for every cell) and the W chunks of the pass's blocks in LDS;
//   barrier; products; barrier; then the tiles are stored.
constexpr int gmc_cap(int mm) { return mm == MM_F64 ? 16 : 32; }

// Reference gradient d phi_b / d xi_m (m = 0..2) at point q from the 1-D
// value and derivative tables.
template <class H>
__device__ __forceinline__ void ref_grad(const double *B1, const double *D1, int b, int q, double (&g)[3])
{
    constexpr int N1 = H::N1;
    const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
    const int b0 = b % N1, b1 = (b / N1) % N1, b2 = b / (N1 * N1);
    const double bx = B1[q0 * N1 + b0], by = B1[q1 * N1 + b1], bz = B1[q2 * N1 + b2];
    g[0] = D1[q0 * N1 + b0] * by * bz;
    g[1] = bx * D1[q1 * N1 + b1] * bz;
    g[2] = bx * by * D1[q2 * N1 + b2];
}

// Voigt index of the symmetric pair (a, b): 11,22,33,12,13,23
__device__ __forceinline__ int voigt(int a, int b) { return a == b ? a : a + b + 2; }

// c[k] = C_rjsk at point kq = e n_q + q of the elasticity tensor written by
// the material: isotropic lambda delta_rj delta_sk + mu (delta_rs delta_jk +
// delta_rk delta_js) from ISO_QP, or D[voigt(r,j)][voigt(s,k)] from VOIGT_QP
// (engineering shear, so that sum C_rjsk du_s/dx_k is the stress).
template <typename T>
__device__ __forceinline__ void material_row(const ExecArgs &A, int64_t kq, int r, int j, int s, double (&c)[3])
{
    const T *mat = static_cast<const T *>(A.mat);
    if (A.mat_kind == FE_MAT_VOIGT_QP) {
        const T *D = mat + kq * 36 + voigt(r, j) * 6;
#pragma unroll
        for (int k = 0; k < 3; k++) c[k] = static_cast<double>(D[voigt(s, k)]);
    } else {
        const double lam = static_cast<double>(mat[2 * kq]), mu = static_cast<double>(mat[2 * kq + 1]);
#pragma unroll
        for (int k = 0; k < 3; k++)
            c[k] = (r == j && s == k ? lam : 0.0) + (r == s && j == k ? mu : 0.0) + (r == k && j == s ? mu : 0.0);
    }
}

template <int P, int FORM, int MM>
struct HexGMC {
    static constexpr int N1 = P + 1, NB = N1 * N1 * N1, NQ = NB;
    static constexpr int ND = 3 * NB;
    static constexpr int NBP = align_to(NB, 16), NT = NBP / 16, TPB = NT * NT;
    static constexpr bool RAGGED = NB % 16 != 0;
    static constexpr bool NT_STORE = ND % 16 == 0;
    using T = typename MMT<MM>::T;
    using ACC = typename MMT<MM>::acc;
    static constexpr bool CONV = FORM == FE_FORM_CONVECT;
    static constexpr bool ELAST = FORM == FE_FORM_ELASTICITY;  // per-point material
    // depth of the products: the points, or (point, gradient component)
    // pairs for elasticity
    static constexpr int DQ = ELAST ? 3 * NQ : NQ;
    static constexpr int KC = 16, NCH = (DQ + KC - 1) / KC, KS = op_stride(MM, KC);
    static constexpr int NTILES = 9 * TPB;
    // FP64 weighted dot: W_rs = c_rs Phi formed in registers from the Phi
    // chunk and the point coefficients (no W chunks), with fewer
    // accumulator tiles per wave to make room.  For the convection and in
    // FP32 the extra passes cost more than the W chunks save (measured).
    static constexpr bool REGW = FORM == FE_FORM_WDOT && MM == MM_F64;
    static constexpr int CAP = REGW ? 12 : gmc_cap(MM);
    static constexpr int NPASS = (NTILES + GM_WAVES * CAP - 1) / (GM_WAVES * CAP);
    static constexpr int NJ = (NTILES + GM_WAVES * NPASS - 1) / (GM_WAVES * NPASS);  // tiles per wave and pass
    static constexpr int PT = GM_WAVES * NJ;                                          // tiles per pass
    static constexpr int WB = (PT + TPB - 1) / TPB + 1 < 9 ? (PT + TPB - 1) / TPB + 1 : 9;  // blocks a pass touches
    static constexpr int NF = CONV ? 21 : 9;
    static constexpr int PS = ELAST ? 10 : (CONV ? 12 : 9);
    // LDS layout (bytes); F (sum-factorization scratch) shares the space of
    // the Phi and W chunks, free between the last products of a cell and the
    // first chunk of the next
    static constexpr int OFF_TB = 0;  // double B1[N1][N1], D1[N1][N1], w[NQ]
    static constexpr int OFF_X = q2::align16(OFF_TB + (2 * N1 * N1 + NQ) * 8);
    static constexpr int OFF_P = q2::align16(OFF_X + (CONV ? 6 * NB : (ELAST ? 3 * NB : 3 * NB + 9 * NQ)) * 8);  // double Pq[NQ][PS]
    // REGW: Pq rows NQ .. NCH KC - 1 are zero (the chunks' padding points)
    static constexpr int QPAD = REGW ? NCH * KC : NQ;
    static constexpr int OFF_A = q2::align16(OFF_P + QPAD * PS * 8);  // T Phi[NBP][KS] or G; double F[NF][NQ]
    static constexpr int OFF_W = q2::align16(OFF_A + NBP * KS * (int)sizeof(T));  // T W[WB][NBP][KS]
    static constexpr int CH_END = OFF_W + WB * NBP * KS * (int)sizeof(T);
    // elasticity: the material rows C_rjsk (k = 0..2) of a chunk's depth
    // values and the pass's blocks, double Cs[WB][KC][3]
    static constexpr int OFF_C = q2::align16(CH_END);
    static constexpr int C_END = OFF_C + (ELAST ? WB * KC * 3 * 8 : 0);
    static constexpr int F_END = OFF_A + NF * NQ * 8;
    static constexpr int BYTES = q2::align16(C_END > F_END ? C_END : F_END);
    static_assert(BYTES <= 160 * 1024, "LDS");
};

template <int P, int FORM, int MM>
__global__ __launch_bounds__(GM_THREADS, 2) void k_hexgmc(ExecArgs A)
{
    using H = HexGMC<P, FORM, MM>;
    using T = typename H::T;
    using ACC = typename H::ACC;
    constexpr int N1 = H::N1, NB = H::NB, NQ = H::NQ, NBP = H::NBP, NT = H::NT, TPB = H::TPB, KC = H::KC;
    constexpr int KS = H::KS, NJ = H::NJ, PT = H::PT, PS = H::PS;
    constexpr bool CONV = H::CONV, ELAST = H::ELAST;
    __shared__ __align__(16) unsigned char smem[H::BYTES];
    double *B1 = reinterpret_cast<double *>(smem + H::OFF_TB);
    double *D1 = B1 + N1 * N1;
    double *wq = D1 + N1 * N1;
    double *xs = reinterpret_cast<double *>(smem + H::OFF_X);  // [3][NB]
    double *us = xs + 3 * NB;                                  // [3][NB] (convection)
    double *Ms = xs + 3 * NB;                                  // [NQ][9] (weighted dot)
    double *Pq = reinterpret_cast<double *>(smem + H::OFF_P);  // [NQ][PS]
    T *Ph = reinterpret_cast<T *>(smem + H::OFF_A);            // [NBP][KS]: points of the chunk
    double *F = reinterpret_cast<double *>(smem + H::OFF_A);   // [NF][NQ]
    T *W = reinterpret_cast<T *>(smem + H::OFF_W);             // [WB][NBP][KS]
    double *Cs = reinterpret_cast<double *>(smem + H::OFF_C);  // [WB][KC][3] (elasticity)
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, grp = lane >> 4;

    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    if (e >= e_end) return;  // uniform over the workgroup

    for (int k = tid; k < N1 * N1; k += GM_THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < NQ; k += GM_THREADS) wq[k] = A.tab.w[k];
    for (int k = tid; k < (H::QPAD - NQ) * PS; k += GM_THREADS) Pq[NQ * PS + k] = 0.0;
    __syncthreads();

    for (; e < e_end; e += stride) {
        gm_gather<H>(A, e, xs, us, Ms, tid);
        __syncthreads();
        gm_points<H>(A, B1, D1, wq, xs, us, Ms, F, Pq, tid);
        __syncthreads();  // F (in the chunks' space) is read for the last time in gm_points

        T *oc = static_cast<T *>(A.out) + e * static_cast<int64_t>(H::ND) * H::ND;
        for (int ps = 0; ps < H::NPASS; ps++) {
            const int t0 = ps * PT;
            const int t1 = t0 + PT < H::NTILES ? t0 + PT : H::NTILES;
            const int blo = t0 / TPB, nbk = (t1 - 1) / TPB - blo + 1;
            // this wave's tiles t = t0 + wave + 8 u; slots past t1 multiply
            // the pass's first tile and are not stored
            ACC acc[NJ];
            int ra[NJ], rb[NJ];
#pragma unroll
            for (int u = 0; u < NJ; u++) {
                acc[u] = ACC{};
                const int t = t0 + wave + GM_WAVES * u, tt = t < t1 ? t : t0;
                const int blk = tt / TPB, rem = tt - blk * TPB, ti = rem / NT, tj = rem - ti * NT;
                ra[u] = 16 * ti;
                // the row of the block's W chunk, or (REGW) the Phi row of the
                // trial side
                rb[u] = H::REGW ? 16 * tj : (blk - blo) * NBP + 16 * tj;
            }
            // block of slot u (wave-uniform)
            auto slot_blk = [&](int u) {
                const int t = t0 + wave + GM_WAVES * u;
                return (t < t1 ? t : t0) / TPB;
            };
            for (int ch = 0; ch < H::NCH; ch++) {
                const int k0 = ch * KC;
                if constexpr (ELAST) {
                    // the material rows of the chunk and the pass's blocks,
                    // read from global memory once per chunk instead of by
                    // every basis function's item
                    if (tid < nbk * KC) {
                        const int dl = tid % KC, bk = tid / KC, d = k0 + dl, q = d / 3, j = d - 3 * (d / 3);
                        const int rs = blo + bk, r = rs / 3, s = rs - 3 * r;
                        double c[3] = {0.0, 0.0, 0.0};
                        if (q < NQ) material_row<T>(A, e * NQ + q, r, j, s, c);
#pragma unroll
                        for (int k = 0; k < 3; k++) Cs[(bk * KC + dl) * 3 + k] = c[k];
                    }
                    __syncthreads();
                    // G chunk: G_ja(q) at depth d = 3 q + j; W chunks:
                    // w det J sum_k C_rjsk(q) G_kb(q)
                    for (int it = tid; it < NBP * KC; it += GM_THREADS) {
                        const int b = it % NBP, dl = it / NBP, d = k0 + dl, q = d / 3, j = d - 3 * (d / 3);
                        double v = 0.0;
                        if (b < NB && q < NQ) {
                            double gx[3];
                            ref_grad<H>(B1, D1, b, q, gx);
                            const double *pq = Pq + q * PS;
                            v = gx[0] * pq[j] + gx[1] * pq[3 + j] + gx[2] * pq[6 + j];
                        }
                        Ph[b * KS + dl] = static_cast<T>(v);
                    }
                    for (int it = tid; it < nbk * NBP * KC; it += GM_THREADS) {
                        const int dl = it % KC, rest = it / KC, b = rest % NBP, bk = rest / NBP;
                        const int q = (k0 + dl) / 3;
                        double x = 0.0;
                        if (q < NQ && b < NB) {
                            double gx[3];
                            ref_grad<H>(B1, D1, b, q, gx);
                            const double *pq = Pq + q * PS;
                            const double *c = Cs + (bk * KC + dl) * 3;
#pragma unroll
                            for (int k = 0; k < 3; k++)
                                x += c[k] * (gx[0] * pq[k] + gx[1] * pq[3 + k] + gx[2] * pq[6 + k]);
                            x *= pq[9];
                        }
                        W[(bk * NBP + b) * KS + dl] = static_cast<T>(x);
                    }
                } else {
                // Phi chunk: basis b at the chunk's points (zero past NB / NQ),
                // from the 1-D tables in LDS: a global load here would wait
                // for the previous pass's tile stores (a wave's memory
                // operations complete in order)
                for (int it = tid; it < NBP * KC; it += GM_THREADS) {
                    const int b = it % NBP, ql = it / NBP, q = k0 + ql;
                    double v = 0.0;
                    if (b < NB && q < NQ) {
                        const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
                        const int b0 = b % N1, b1 = (b / N1) % N1, b2 = b / (N1 * N1);
                        v = B1[q0 * N1 + b0] * B1[q1 * N1 + b1] * B1[q2 * N1 + b2];
                    }
                    Ph[b * KS + ql] = static_cast<T>(v);
                }
                // W chunks of the pass's blocks (REGW: none)
                for (int it = tid; it < (H::REGW ? 0 : nbk) * NBP * KC; it += GM_THREADS) {
                    const int ql = it % KC, rest = it / KC, b = rest % NBP, bk = rest / NBP;
                    const int q = k0 + ql, rs = blo + bk;
                    double x = 0.0;
                    if (q < NQ && b < NB) {
                        const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
                        const int b0 = b % N1, b1 = (b / N1) % N1, b2 = b / (N1 * N1);
                        const double bx = B1[q0 * N1 + b0], by = B1[q1 * N1 + b1], bz = B1[q2 * N1 + b2];
                        const double *pq = Pq + q * PS;
                        x = pq[rs] * (bx * by * bz);
                        if (CONV && rs / 3 == rs % 3) {
                            const double dx = D1[q0 * N1 + b0], dy = D1[q1 * N1 + b1], dz = D1[q2 * N1 + b2];
                            x += pq[9] * (dx * by * bz) + pq[10] * (bx * dy * bz) + pq[11] * (bx * by * dz);
                        }
                    }
                    W[(bk * NBP + b) * KS + ql] = static_cast<T>(x);
                }
                }
                __syncthreads();
                // products over the chunk's points: k steps in a loop, the
                // slots in groups whose fragments are loaded while the
                // previous group multiplies
                constexpr int G = (sizeof(T) == 8 ? 4 : 8) / (H::REGW ? 2 : 1), NG = (NJ + G - 1) / G;
                T a[2][G], bb[2][G], cq[2][G];
                auto load = [&](int buf, int g, int k) {
#pragma unroll
                    for (int v = 0; v < G; v++)
                        if (g * G + v < NJ) {
                            a[buf][v] = Ph[(ra[g * G + v] + m) * KS + k];
                            if constexpr (H::REGW) {
                                bb[buf][v] = Ph[(rb[g * G + v] + m) * KS + k];
                                cq[buf][v] = static_cast<T>(Pq[(k0 + k) * PS + slot_blk(g * G + v)]);
                            } else {
                                bb[buf][v] = W[(rb[g * G + v] + m) * KS + k];
                            }
                        }
                };
                auto mfma = [&](int buf, int g) {
                    if constexpr (H::REGW) {
#pragma unroll
                        for (int v = 0; v < G; v++)
                            if (g * G + v < NJ) bb[buf][v] *= cq[buf][v];
                    }
#pragma unroll
                    for (int v = 0; v < G; v++)
                        if (g * G + v < NJ) {
                            if constexpr (MM == MM_F64)
                                acc[g * G + v] =
                                    __builtin_amdgcn_mfma_f64_16x16x4f64(a[buf][v], bb[buf][v], acc[g * G + v], 0, 0, 0);
                            else
                                acc[g * G + v] =
                                    __builtin_amdgcn_mfma_f32_16x16x4f32(a[buf][v], bb[buf][v], acc[g * G + v], 0, 0, 0);
                        }
                };
                for (int st = 0; st < KC / 4; st++) {
                    const int k = 4 * st + grp;
                    load(0, 0, k);
#pragma unroll
                    for (int g = 0; g < NG; g++) {
                        if (g + 1 < NG) load((g + 1) & 1, g + 1, k);
                        __builtin_amdgcn_sched_barrier(0);
                        mfma(g & 1, g);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                __syncthreads();  // the chunks are rebuilt next
            }
#pragma unroll
            for (int u = 0; u < NJ; u++) {
                const int t = t0 + wave + GM_WAVES * u;
                if (t < t1) {
                    const int blk = t / TPB, rem = t - blk * TPB, ti = rem / NT, tj = rem - ti * NT;
                    const int r = blk / 3, s = blk - 3 * r;
                    store_tile<H>(oc, r * NB + 16 * ti, s * NB + 16 * tj, valid<H>(ti), valid<H>(tj), acc[u], lane);
                }
            }
        }
    }
}

template <int P, int FORM, int MM>
int launch_hexgm(const Plan &, const ExecArgs &A, hipStream_t st)
{
    static std::atomic<int> resident[64];
    if constexpr (P <= 3 && FORM != FE_FORM_ELASTICITY)
        return launch_persistent(k_hexgm<P, FORM, MM>, GM_THREADS, A, st, resident);
    else
        return launch_persistent(k_hexgmc<P, FORM, MM>, GM_THREADS, A, st, resident);
}

template <int P, int MM>
LaunchFn pick(const Plan &p)
{
    if (p.form == FE_FORM_WDOT && p.mat_kind == FE_MAT_TENSOR_QP) return launch_hexgm<P, FE_FORM_WDOT, MM>;
    if (p.form == FE_FORM_CONVECT) return launch_hexgm<P, FE_FORM_CONVECT, MM>;
    // elasticity with per-point material at orders 4-5 (below, the generic
    // kernel keeps all points' gradients in LDS)
    if constexpr (P >= 4)
        if (p.form == FE_FORM_ELASTICITY && (p.mat_kind == FE_MAT_ISO_QP || p.mat_kind == FE_MAT_VOIGT_QP))
            return launch_hexgm<P, FE_FORM_ELASTICITY, MM>;
    return nullptr;
}

template <int MM>
LaunchFn pick_order(const Plan &p)
{
    if (p.order == 2) return pick<2, MM>(p);
    if (p.order == 3) return pick<3, MM>(p);
    if (p.order == 4) return pick<4, MM>(p);
    if (p.order == 5) return pick<5, MM>(p);
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
