// Helpers shared by the matrix-core element-matrix kernels: operand padding
// and LDS strides, the 16x16 accumulator layout, masked tile stores.
#pragma once

#include "q2_device.h"

namespace fe {
namespace mm {

using q2::MM_BF16X3;
using q2::MM_F32;
using q2::MM_F64;

constexpr int align_to(int x, int a) { return (x + a - 1) / a * a; }

// LDS row stride (entries) of an operand for a padded depth KP, so that the
// fragment reads (16 rows x 4 points, or 16 rows x 8 points for bf16) hit
// distinct banks of the 32 four-byte LDS banks in every pass: FP64 odd,
// FP32 2 mod 4, bf16 8 mod 16 (measured with the LDS bank-conflict
// counter).
constexpr int op_stride(int mm, int kp)
{
    int ks = kp;
    if (mm == MM_F64)
        while (ks % 2 != 1) ks++;
    else if (mm == MM_F32)
        while (ks % 4 != 2) ks++;
    else
        while (ks % 16 != 8) ks++;
    return ks;
}

// accumulator row of element v for this lane (column = lane % 16)
template <int MM>
__device__ __forceinline__ int acc_row(int lane, int v)
{
    return MM == MM_F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

// store tile (output rows row0.., columns col0..) of one cell's matrix of
// row length H::ND; rl / cl = valid rows / columns of the tile (16 unless
// the block is ragged).  H::NT_STORE: nontemporal stores (for row segments
// that fill whole 128-byte lines), else through the L2.
template <class H>
__device__ __forceinline__ void store_tile(typename H::T *oc, int row0, int col0, int rl, int cl,
                                           const typename H::ACC &x, int lane)
{
    constexpr int MM = sizeof(typename H::T) == 8 ? MM_F64 : MM_F32;
    const int col = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int row = acc_row<MM>(lane, v);
        if (!H::RAGGED || (row < rl && col < cl)) {
            typename H::T *dst = oc + static_cast<int64_t>(row0 + row) * H::ND + col0 + col;
            if constexpr (H::NT_STORE)
                __builtin_nontemporal_store(x[v], dst);
            else
                *dst = x[v];
        }
    }
}

template <class H>
__device__ __forceinline__ int valid(int t)  // valid entries of tile t of a block of H::NB
{
    return H::NB - 16 * t < 16 ? H::NB - 16 * t : 16;
}

}  // namespace mm
}  // namespace fe
