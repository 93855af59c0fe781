// Cell-per-lane element-matrix kernels for low-order cells (Q1 hexahedra,
// P1/P2 tetrahedra): Algorithm "feloopm" with the cell loop spread over the
// lanes of a wave and the quadrature loop kept in each lane's registers.
//
//   k_cw_scalar  mass ('i,i', scalar and vector) and Laplace ('0.i,0.i'):
//                one wave of 64 lanes = 64 cells; each lane accumulates the
//                upper triangle of its cell's symmetric matrix.
//   k_cw_elast   isotropic linear elasticity: six waves per workgroup, wave w
//                computes block (r,s), r <= s, of the same 64 cells.  With
//                H = dphi/dxi adj J and s_q = w_q / det J (see cw_device.h):
//                  K_rs[a][b] = sum_q s_q (lambda H_r[a] H_s[b] + mu H_s[a] H_r[b])
//                  K_rr[a][b] = sum_q s_q ((lambda + mu) H_r[a] H_r[b] + mu H_a . H_b)
//                which is w det J B^T D B of section "Linear Elasticity
//                Expression" for the isotropic D, block by block; K_sr = K_rs^T.
//
// Output: every kernel stages a chunk of rows of its 64 cells in LDS (one
// padded row set per cell, so the lane-per-cell writes spread over the LDS
// banks) and then stores the chunk with consecutive threads on consecutive
// entries, so global stores are contiguous runs instead of one stream per
// lane.
#include "cw_device.h"

namespace fe {
namespace {

using namespace cw;

constexpr int SCALAR_STAGE = 12 * 1024;
constexpr int ELAST_STAGE = 28 * 1024;
constexpr int ELAST_THREADS = 384;

template <typename T>
__device__ __forceinline__ void st_nt(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

template <int CELL, int P, int FORM, typename T>
struct CwScalar {
    using S = Shape<CELL, P>;
    static constexpr int NB = S::NB, NQ = S::NQ, NP = NB * (NB + 1) / 2;
    static constexpr int ND = FORM == FE_FORM_VMASS ? 3 * NB : NB;
    static constexpr int RC = pick_rows(ND, ND, (int)sizeof(T), SCALAR_STAGE);
    static constexpr int SS = RC * ND + 1;
    // nontemporal stores when a cell's chunk of rows spans at least a
    // 128-byte line; shorter chunks (e.g. the FP32 vector mass of Q1, 96
    // bytes) go through the L2, which joins the parts written by neighbouring
    // cells (measured: Q1 FP32 vector mass 3.9 -> 2.2 ms at 128^3)
    static constexpr bool NT_STORE = RC * ND * (int)sizeof(T) >= 128;
    // coordinates in registers up to 8 nodes, in LDS beyond
    static constexpr bool X_LDS = NB > 8;
    using XT = typename std::conditional<X_LDS, XLds<NB>, XReg<NB>>::type;
};

template <int CELL, int P, int FORM, typename T>
__global__ __launch_bounds__(64, CELL == FE_CELL_HEX && sizeof(T) == 4 && FORM != FE_FORM_LAPLACE ? 4 : 1) void k_cw_scalar(ExecArgs A)
{
    using C = CwScalar<CELL, P, FORM, T>;
    constexpr int NB = C::NB, NP = C::NP, ND = C::ND, RC = C::RC, SS = C::SS;
    constexpr bool X_LDS = C::X_LDS;
    __shared__ T stage[64 * SS];
    __shared__ double xs[X_LDS ? 64 * XLds<NB>::STRIDE : 1];
    const int lane = threadIdx.x;
    const int64_t e0 = logical_block(A.xcd_remap) * 64;
    const int64_t e = e0 + lane;
    const bool valid = e < A.n_cells;
    const ctab_t *bfgT = ctab(A.tab.bfgT);
    const ctab_t *bf = ctab(A.tab.bf);
    const ctab_t *w = ctab(A.tab.w);

    using XT = typename C::XT;
    XT x;
    unsigned fault;
    if constexpr (X_LDS) {
        fault = gather_lds<NB>(A.conn, A.coords, e0, A.n_cells, A.n_nodes, xs, lane, 64);
        __syncthreads();
        x.row = xs + lane * XLds<NB>::STRIDE;
    } else {
        fault = gather<NB>(A.conn, A.coords, e, A.n_nodes, valid, x);
    }

    T acc[NP];
    if constexpr (CELL == FE_CELL_HEX && P == 1 && FORM == FE_FORM_LAPLACE) {
        // tensor-product sums in FP64, rounded once to the output type
        double accd[NP];
        acc_laplace_q1(x, ctab(A.tab.B1), ctab(A.tab.D1), w, valid, fault, accd);
#pragma unroll
        for (int p = 0; p < NP; p++) acc[p] = static_cast<T>(accd[p]);
    } else {
        acc_scalar<CELL, P, FORM == FE_FORM_VMASS ? FE_FORM_MASS : FORM, T>(x, w, bf, bfgT, valid, fault, acc);
    }

    if (fault) raise_fault(A.flags, fault);

    // staged, coalesced output of RC rows at a time
    T *out = static_cast<T *>(A.out);
    const int ncell = A.n_cells - e0 < 64 ? static_cast<int>(A.n_cells - e0) : 64;
#pragma unroll
    for (int c0 = 0; c0 < ND; c0 += RC) {
#pragma unroll
        for (int rr = 0; rr < RC; rr++) {
            const int row = c0 + rr, ra = row % NB, rc = row / NB;
#pragma unroll
            for (int col = 0; col < ND; col++) {
                const int cb = col % NB, cc = col / NB;
                const T v = (rc != cc) ? T(0) : (ra <= cb ? acc[tri(ra, cb, NB)] : acc[tri(cb, ra, NB)]);
                stage[lane * SS + rr * ND + col] = v;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int k = lane; k < 64 * RC * ND; k += 64) {
            const int cc = k / (RC * ND), off = k - cc * (RC * ND);
            if (cc < ncell) {
                T *dst = out + (e0 + cc) * (ND * ND) + c0 * ND + off;
                if constexpr (C::NT_STORE)
                    st_nt(dst, stage[cc * SS + off]);
                else
                    *dst = stage[cc * SS + off];
            }
        }
        __syncthreads();
    }
}

// Vector mass I3 (x) M of 64 cells per workgroup of 256 threads.  Wave 0
// evaluates the scalar mass matrix M (one lane per cell, upper triangle in
// LDS); then all four waves write the 3nb x 3nb matrices in sweeps of whole
// rows, a thread keeping its column: entry ((r,a),(s,b)) is M[a][b] when
// r == s and zero otherwise.  Two thirds of the output are zeros, so the
// kernel is a store stream; the sweeps make each one a contiguous run.
template <int CELL, int P, typename T>
__global__ __launch_bounds__(256) void k_cw_vmass(ExecArgs A)
{
    using S = Shape<CELL, P>;
    constexpr int NB = S::NB, NP = NB * (NB + 1) / 2, ND = 3 * NB, MSTR = NP + 1, RPS = 256 / ND;
    constexpr bool X_LDS = NB > 8;
    __shared__ T Mst[64 * MSTR];
    __shared__ double xs[X_LDS ? 64 * XLds<NB>::STRIDE : 1];
    const int tid = threadIdx.x;
    const int64_t e0 = logical_block(A.xcd_remap) * 64;
    const int ncell = A.n_cells - e0 < 64 ? static_cast<int>(A.n_cells - e0) : 64;
    unsigned fault = 0;
    if constexpr (X_LDS) {
        fault = gather_lds<NB>(A.conn, A.coords, e0, A.n_cells, A.n_nodes, xs, tid, 256);
        __syncthreads();
    }
    if (tid < 64) {
        const int64_t e = e0 + tid;
        const bool valid = e < A.n_cells;
        using XT = typename std::conditional<X_LDS, XLds<NB>, XReg<NB>>::type;
        XT x;
        if constexpr (X_LDS)
            x.row = xs + tid * XLds<NB>::STRIDE;
        else
            fault |= gather<NB>(A.conn, A.coords, e, A.n_nodes, valid, x);
        T acc[NP];
        acc_scalar<CELL, P, FE_FORM_MASS, T>(x, ctab(A.tab.w), ctab(A.tab.bf), ctab(A.tab.bfgT), valid, fault, acc);
#pragma unroll
        for (int p = 0; p < NP; p++) Mst[tid * MSTR + p] = acc[p];
    }
    if (fault) raise_fault(A.flags, fault);
    __syncthreads();
    if (tid < RPS * ND) {
        const int col = tid % ND, s = col / NB, b = col - s * NB;
        int row = (tid / ND) % ND, c = tid / (ND * ND);
        T *out = static_cast<T *>(A.out) + e0 * (ND * ND) + tid;
        for (int rr = tid / ND; rr < ncell * ND; rr += RPS) {
            const int r = row / NB, a = row - r * NB;
            const T v = r == s ? Mst[c * MSTR + (a <= b ? tri(a, b, NB) : tri(b, a, NB))] : T(0);
            st_nt(out, v);
            out += RPS * ND;
            row += RPS % ND;
            c += RPS / ND;
            if (row >= ND) {
                row -= ND;
                c++;
            }
        }
    }
}

template <int CELL, int P, typename T>
struct CwElast {
    using S = Shape<CELL, P>;
    static constexpr int NB = S::NB, NQ = S::NQ, ND = 3 * NB;
    static constexpr int RH = pick_rows(NB, ND, (int)sizeof(T), ELAST_STAGE);
    static constexpr int SS = RH * ND + 1;
};

// Block (R,S) of the isotropic elasticity matrix of the workgroup's 64 cells,
// computed by one wave (lane = cell) from the coordinates the workgroup
// gathered into LDS, then the staged row chunks written by the whole
// workgroup.  Every instantiation executes the same barriers.
template <int CELL, int P, typename T, int R, int S>
__device__ __forceinline__ void elast_block(const ExecArgs &A, int64_t e0, const double *xs, T *stage,
                                            unsigned fault)
{
    using C = CwElast<CELL, P, T>;
    constexpr int NB = C::NB, ND = C::ND, RH = C::RH, SS = C::SS;
    constexpr bool DIAG = R == S;
    constexpr int NACC = ElastAcc<NB, R, S>::N;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t e = e0 + lane;
    const bool valid = e < A.n_cells;
    const ctab_t *bfgT = ctab(A.tab.bfgT);
    const ctab_t *w = ctab(A.tab.w);
    const T *mat = static_cast<const T *>(A.mat);
    const bool per_qp = A.mat_kind == FE_MAT_ISO_QP;
    const XLds<NB> x{xs + lane * XLds<NB>::STRIDE};

    T acc[NACC];
    acc_elast<CELL, P, T, R, S>(x, w, bfgT, mat, per_qp, e, valid, fault, acc);

    if (fault) raise_fault(A.flags, fault);

    T *out = static_cast<T *>(A.out);
    const int ncell = A.n_cells - e0 < 64 ? static_cast<int>(A.n_cells - e0) : 64;
#pragma unroll
    for (int c = 0; c < 3; c++) {
#pragma unroll
        for (int h = 0; h < NB / RH; h++) {
            if (c == R) stage_block<NB, ND, RH, R, S, false>(acc, stage + lane * SS, h * RH, S * NB);
            if (!DIAG && c == S) stage_block<NB, ND, RH, R, S, true>(acc, stage + lane * SS, h * RH, R * NB);
            __syncthreads();
            const int64_t row0 = c * NB + h * RH;
            for (int k = tid; k < 64 * RH * ND; k += ELAST_THREADS) {
                const int cc = k / (RH * ND), off = k - cc * (RH * ND);
                if (cc < ncell) st_nt(out + (e0 + cc) * (ND * ND) + row0 * ND + off, stage[cc * SS + off]);
            }
            __syncthreads();
        }
    }
}

template <int CELL, int P, typename T>
__global__ __launch_bounds__(ELAST_THREADS) void k_cw_elast(ExecArgs A)
{
    constexpr int NB = CwElast<CELL, P, T>::NB;
    __shared__ T stage[64 * CwElast<CELL, P, T>::SS];
    __shared__ double xs[64 * XLds<NB>::STRIDE];
    const int64_t e0 = logical_block(A.xcd_remap) * 64;
    const unsigned fault = gather_lds<NB>(A.conn, A.coords, e0, A.n_cells, A.n_nodes, xs, threadIdx.x, ELAST_THREADS);
    __syncthreads();
    // the wave index, made visibly uniform so the six paths are separate
    // branches rather than one masked sequence
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: elast_block<CELL, P, T, 0, 0>(A, e0, xs, stage, fault); break;
    case 1: elast_block<CELL, P, T, 0, 1>(A, e0, xs, stage, fault); break;
    case 2: elast_block<CELL, P, T, 0, 2>(A, e0, xs, stage, fault); break;
    case 3: elast_block<CELL, P, T, 1, 1>(A, e0, xs, stage, fault); break;
    case 4: elast_block<CELL, P, T, 1, 2>(A, e0, xs, stage, fault); break;
    default: elast_block<CELL, P, T, 2, 2>(A, e0, xs, stage, fault); break;
    }
}

template <typename K>
int launch_cw(K kernel, int threads, const ExecArgs &A, hipStream_t st)
{
    if (A.n_cells <= 0) return FE_OK;
    const int64_t blocks = (A.n_cells + 63) / 64;
    if (blocks > 0x7fffffff) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(threads), 0, st, A);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <int CELL, int P, int FORM, typename T>
int launch_scalar(const Plan &, const ExecArgs &A, hipStream_t st)
{
    return launch_cw(k_cw_scalar<CELL, P, FORM, T>, 64, A, st);
}

template <int CELL, int P, typename T>
int launch_vmass(const Plan &, const ExecArgs &A, hipStream_t st)
{
    return launch_cw(k_cw_vmass<CELL, P, T>, 256, A, st);
}

template <int CELL, int P, typename T>
int launch_elast(const Plan &, const ExecArgs &A, hipStream_t st)
{
    return launch_cw(k_cw_elast<CELL, P, T>, ELAST_THREADS, A, st);
}

template <int CELL, int P, typename T>
LaunchFn pick(const Plan &p)
{
    switch (p.form) {
    case FE_FORM_MASS: return launch_scalar<CELL, P, FE_FORM_MASS, T>;
    case FE_FORM_VMASS: return launch_vmass<CELL, P, T>;
    case FE_FORM_LAPLACE: return launch_scalar<CELL, P, FE_FORM_LAPLACE, T>;
    case FE_FORM_ELASTICITY:
        if (p.mat_kind == FE_MAT_ISO_CELL || p.mat_kind == FE_MAT_ISO_QP) return launch_elast<CELL, P, T>;
        return nullptr;
    }
    return nullptr;
}

template <typename T>
LaunchFn pick_cell(const Plan &p)
{
    if (p.cell == FE_CELL_HEX && p.order == 1) return pick<FE_CELL_HEX, 1, T>(p);
    if (p.cell == FE_CELL_TET && p.order == 1) return pick<FE_CELL_TET, 1, T>(p);
    if (p.cell == FE_CELL_TET && p.order == 2) return pick<FE_CELL_TET, 2, T>(p);
    return nullptr;
}

}  // namespace

LaunchFn select_cellwise(const Plan &p)
{
    if (p.mode != FE_MODE_MATRIX) return nullptr;
    if (p.prec == FE_PREC_FP64) return pick_cell<double>(p);
    if (p.prec == FE_PREC_FP32) return pick_cell<float>(p);
    return nullptr;
}

}  // namespace fe
