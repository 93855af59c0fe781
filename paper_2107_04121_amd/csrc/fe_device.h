// Device-side helpers shared by the gfx950 kernels of this library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fe_internal.h"

namespace fe {

constexpr int hex_nb(int p) { return (p + 1) * (p + 1) * (p + 1); }
constexpr int cell_nb(int cell, int p) { return cell == FE_CELL_HEX ? hex_nb(p) : (p == 1 ? 4 : 10); }
constexpr int cell_nq(int cell, int p) { return (p + 1) * (p + 1) * (p + 1); }
constexpr int form_nc(int form) { return (form == FE_FORM_MASS || form == FE_FORM_LAPLACE) ? 1 : 3; }

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Remapping the hardware block id so that every XCD works
// on one contiguous range of logical blocks keeps neighbouring cells (which
// share nodes) in the same L2.  Bijective for any grid size.
__device__ __forceinline__ int64_t logical_block(int remap)
{
    const int64_t b = blockIdx.x, G = gridDim.x;
    if (!remap || G < 16) return b;
    const int64_t x = b & 7, i = b >> 3, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ void raise_fault(unsigned *flags, unsigned bit)
{
    atomicOr(flags, bit);
}

// Node number of local node a of cell e, checked against n_nodes; an invalid
// number raises FAULT_INDEX and is replaced by 0 so the access stays in bounds.
__device__ __forceinline__ int64_t checked_node(const int32_t *conn, int64_t idx, int64_t n_nodes,
                                                unsigned *flags)
{
    int64_t n = conn[idx];
    if (n < 0 || n >= n_nodes) {
        raise_fault(flags, FAULT_INDEX);
        n = 0;
    }
    return n;
}

// 3x3 determinant and inverse by cofactors, FP64.  Ji[j][i] = (J^-1)_{ji}.
__device__ __forceinline__ double inverse3(const double J[3][3], double Ji[3][3])
{
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    return det;
}

// Jacobian J_ij = sum_a x_a,i dphi_a/dxi_j at quadrature point q from node
// coordinates xs[a*3 + i] (LDS) and the transposed reference gradient table
// bfgT[(a*3 + j)*NQ + q].
template <int NB, int NQ>
__device__ __forceinline__ void jacobian_qp(const double *xs, const double *__restrict__ bfgT, int q,
                                            double J[3][3])
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) J[i][j] = 0.0;
#pragma unroll 4
    for (int a = 0; a < NB; a++) {
        const double g0 = bfgT[(a * 3 + 0) * NQ + q];
        const double g1 = bfgT[(a * 3 + 1) * NQ + q];
        const double g2 = bfgT[(a * 3 + 2) * NQ + q];
        const double x0 = xs[a * 3 + 0], x1 = xs[a * 3 + 1], x2 = xs[a * 3 + 2];
        J[0][0] = fma(x0, g0, J[0][0]);
        J[0][1] = fma(x0, g1, J[0][1]);
        J[0][2] = fma(x0, g2, J[0][2]);
        J[1][0] = fma(x1, g0, J[1][0]);
        J[1][1] = fma(x1, g1, J[1][1]);
        J[1][2] = fma(x1, g2, J[1][2]);
        J[2][0] = fma(x2, g0, J[2][0]);
        J[2][1] = fma(x2, g1, J[2][1]);
        J[2][2] = fma(x2, g2, J[2][2]);
    }
}

template <typename T>
__device__ __forceinline__ T sel3(int r, T a0, T a1, T a2)
{
    return r == 0 ? a0 : (r == 1 ? a1 : a2);
}

}  // namespace fe
