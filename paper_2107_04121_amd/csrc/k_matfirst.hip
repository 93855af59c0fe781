// Matrix-first residual: form the element matrices of a chunk of cells (any
// matrix-mode kernel of the plan's cell, order, form and precision) in the
// workspace, then multiply each by its gathered DOF vector.  This is the
// other contraction order of the residual (K_e first, then K_e u_e); it does
// n_dof^2 work per quadrature point instead of n_dof and exists to be
// measured against the gradient-first kernels.
#include "fe_device.h"

namespace fe {
namespace {

// r[e][i] = sum_j K[e][i][j] u_e[j], u_e[s*nb + b] = U[conn[e][b]][s]
template <typename T>
__global__ __launch_bounds__(256) void k_matvec(const T *K, const int32_t *conn, const T *U, int64_t n_cells,
                                                int64_t n_nodes, int nb, int nc, T *out, unsigned *flags)
{
    const int nd = nb * nc;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_cells * nd) return;
    const int64_t e = t / nd;
    const int i = static_cast<int>(t - e * nd);
    const T *row = K + (e * nd + i) * nd;
    T s = T(0);
    for (int b = 0; b < nb; b++) {
        const int64_t n = checked_node(conn, e * nb + b, n_nodes, flags);
        for (int c = 0; c < nc; c++) s += row[c * nb + b] * U[n * nc + c];
    }
    out[t] = s;
}

}  // namespace

size_t matrix_first_bytes(const Plan &p, int64_t n_cells)
{
    const int64_t chunk = p.opts.chunk > 0 ? p.opts.chunk : 16384;
    const int64_t c = n_cells < chunk ? n_cells : chunk;
    const size_t nd = (size_t)p.nc * p.nb;
    return (size_t)c * nd * nd * (p.prec == FE_PREC_FP64 ? 8 : 4);
}

int launch_matrix_first(const Plan &p, const ExecArgs &A, hipStream_t st)
{
    if (A.n_cells <= 0) return FE_OK;
    const int64_t chunk = p.opts.chunk > 0 ? p.opts.chunk : 16384;
    const size_t esz = p.prec == FE_PREC_FP64 ? 8 : 4;
    const int nd = p.nc * p.nb;
    void *Kbuf = reinterpret_cast<char *>(A.flags) + 256;
    const int64_t mat_stride = material_entries_per_cell(p.mat_kind, p.nq);
    for (int64_t c0 = 0; c0 < A.n_cells; c0 += chunk) {
        const int64_t nc = A.n_cells - c0 < chunk ? A.n_cells - c0 : chunk;
        ExecArgs B = A;
        B.n_cells = nc;
        B.conn = A.conn + c0 * p.nb;
        B.mat = A.mat ? static_cast<const char *>(A.mat) + c0 * mat_stride * esz : nullptr;
        B.out = Kbuf;
        B.eval = 0;
        int rc = p.launch_mat(p, B, st);
        if (rc) return rc;
        const int64_t nt = nc * nd;
        const unsigned blocks = (unsigned)((nt + 255) / 256);
        if (p.prec == FE_PREC_FP64)
            hipLaunchKernelGGL(k_matvec<double>, dim3(blocks), dim3(256), 0, st, static_cast<const double *>(Kbuf),
                               B.conn, static_cast<const double *>(A.dofs), nc, A.n_nodes, p.nb, p.nc,
                               static_cast<double *>(A.out) + c0 * nd, A.flags);
        else
            hipLaunchKernelGGL(k_matvec<float>, dim3(blocks), dim3(256), 0, st, static_cast<const float *>(Kbuf),
                               B.conn, static_cast<const float *>(A.dofs), nc, A.n_nodes, p.nb, p.nc,
                               static_cast<float *>(A.out) + c0 * nd, A.flags);
        FE_HIP_CHECK(hipGetLastError());
    }
    return FE_OK;
}

}  // namespace fe
