// Matrix-core (MFMA) element-matrix kernel: linear elasticity on Q2
// hexahedra with per-cell isotropic coefficients.
//
// The linear elasticity form of the table of example weak forms, in matrix
// mode, is  K[(r,a),(s,b)] = sum_q w_q det J (lambda G_r[a] G_s[b]
// + mu G_s[a] G_r[b] + delta_rs mu G[a].G[b])  with G the physical basis
// gradients (the paper's 'cq,cqje,rjI,cqIK,cqlf,slK->cresf' with isotropic D).
// With lambda, mu constant over the cell all three terms come from ONE
// symmetric product per cell,
//     P[(r,a),(s,b)] = sum_q G[q][r][a] (w_q det J_q) G[q][s][b],
// a (3nb x nq) x (nq x 3nb) GEMM: K_rs = lambda P_rs + mu P_rs^T
// + delta_rs mu (P_00 + P_11 + P_22).  Only the 6 blocks r <= s of P are
// computed.  This is the dense contraction the paper's elasticity einsum
// performs, with the sparsity of the symmetric-gradient extractor (which the
// paper notes it does not exploit) folded away.
//
// One workgroup (4 waves) per cell:
//   1. gather the 27 node coordinates through the connectivity (FP64);
//   2. Jacobian columns from the tensor-product 1-D tables, then det J, J^-1
//      and w det J per quadrature point, all FP64;
//   3. G[q][(i,a)] = sum_j dphi_a/dxi_j Jinv[j][i] in FP64, stored in LDS in
//      the contraction type as the GEMM operand (K padded to the MFMA depth);
//   4. the products on the matrix cores, K, and a linear flush of the cell's
//      81x81 matrix from an LDS staging area with 16-byte stores.
// FP64 and FP32 (staged routine): the output tiles of 16x16 of the blocks
// r <= s of P (21: the diagonal blocks' tiles below the diagonal are left
// out; v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32) go to the staging
// area, and an in-place pass turns P into K there (every thread owns fixed
// (a,b) positions of the 27x27 blocks).  The split
// precision BF16X3 (v_mfma_f32_16x16x32_bf16 three times per tile on the
// hi/lo halves, FP32 accumulation) makes the products cheap, so it computes
// P_rs for all nine (r, s) at three tile positions, forms K in registers and
// stores K tiles (and the transposes that K's symmetry provides) to the
// staging area directly.  Prefetch of the next cell's data overlaps each
// cell's work.
#include "q2_device.h"

namespace fe {
namespace {

using namespace q2;

template <int MM>
__global__ __launch_bounds__(256, MM == MM_F64 ? 3 : 4) void k_elast_q2(ExecArgs A)
{
    __shared__ __align__(16) unsigned char smem[Q2Layout<MM>::BYTES];
    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    const Q2Job job{A.n_cells, A.n_nodes, A.coords, A.conn, A.mat, A.out, nullptr, nullptr, A.flags, A.tab};
    q2_run<MM, false>(job, e, e_end, stride, smem, threadIdx.x);
}

template <int MM>
int launch_elast_q2(const Plan &, const ExecArgs &A, hipStream_t st)
{
    if (A.n_cells <= 0) return FE_OK;
    if (reinterpret_cast<uintptr_t>(A.out) % 16 != 0) {
        set_error("out must be 16-byte aligned for the matrix-core kernel");
        return FE_ERR_INVALID_ARG;
    }
    static std::atomic<int> resident[64];
    return launch_persistent(k_elast_q2<MM>, 256, A, st, resident);
}

}  // namespace

LaunchFn select_mfma(const Plan &p)
{
    if (p.cell == FE_CELL_HEX && p.order == 2 && p.form == FE_FORM_ELASTICITY && p.mode == FE_MODE_MATRIX &&
        p.mat_kind == FE_MAT_ISO_CELL) {
        if (p.prec == FE_PREC_FP64) return launch_elast_q2<MM_F64>;
        if (p.prec == FE_PREC_FP32) return launch_elast_q2<MM_F32>;
        if (p.prec == FE_PREC_BF16X3) return launch_elast_q2<MM_BF16X3>;
    }
    if (LaunchFn f = select_hexgm(p)) return f;
    return select_hexmm(p);
}

}  // namespace fe
