// Node incidence (CSR), assembly by node-centric gather, and the gradient of
// the elasticity eval-mode value with respect to material coefficients and
// node coordinates.
//
// The coordinate gradient is produced in two deterministic steps: a per-cell
// kernel writes partials p[e][a][k] = dJ_e/dx_{conn[e][a],k} (geometry
// recomputed in FP64, nothing kept from the forward pass), then one thread
// per node sums the partials of its incident (cell, local node) pairs in the
// sorted incidence order.  No floating-point atomics, so results are bitwise
// repeatable.
#include <hipcub/hipcub.hpp>

#include "fe_device.h"


namespace fe {
namespace {

__global__ void k_inc_count(const int32_t *conn, int64_t n_items, int64_t n_nodes, int32_t *cnt, unsigned *flags)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const int64_t n = conn[i];
    if (n < 0 || n >= n_nodes) {
        raise_fault(flags, FAULT_INDEX);
        return;
    }
    atomicAdd(cnt + n, 1);
}

__global__ void k_inc_fill(const int32_t *conn, int64_t n_items, int64_t n_nodes, int32_t *cursor, int32_t *items)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const int64_t n = conn[i];
    if (n < 0 || n >= n_nodes) return;
    const int32_t pos = atomicAdd(cursor + n, 1);
    items[pos] = static_cast<int32_t>(i);
}

// Insertion sort of each node's (short) item list, in place.
__global__ void k_inc_sort(const int32_t *offsets, int64_t n_nodes, int32_t *items)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const int32_t b = offsets[n], e = offsets[n + 1];
    for (int32_t i = b + 1; i < e; i++) {
        const int32_t v = items[i];
        int32_t j = i - 1;
        while (j >= b && items[j] > v) {
            items[j + 1] = items[j];
            j--;
        }
        items[j + 1] = v;
    }
}

// out[n][c] = scale * sum_{item of n} vec[e][c][a] (FP64 accumulation)
template <typename TI, typename TO>
__global__ void k_gather(const int32_t *offsets, const int32_t *items, int64_t n_nodes, int nb, int nc,
                         const TI *vec, double scale, TO *out)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_nodes * nc) return;
    const int64_t n = t / nc;
    const int c = static_cast<int>(t - n * nc);
    double s = 0.0;
    for (int32_t k = offsets[n]; k < offsets[n + 1]; k++) {
        const int32_t it = items[k];
        const int32_t e = it / nb, a = it - e * nb;
        s += static_cast<double>(vec[((int64_t)e * nc + c) * nb + a]);
    }
    out[t] = static_cast<TO>(scale * s);
}

// Per-cell partials of dJ/dx laid out [n_cells][3][n_basis] so that the
// gather above (nc = 3) reads them like a vector-valued cell residual.
template <int CELL, int P, typename T>
struct GradCfg {
    static constexpr int NB = cell_nb(CELL, P), NQ = cell_nq(CELL, P);
    static constexpr int BYTES_EL = NB * 3 * 8 + 3 * NB * (int)sizeof(T) + NQ * 9 * (int)sizeof(T) +
                                    NQ * 2 * (int)sizeof(T);
    static constexpr int work = NQ > NB ? NQ : NB;
    static constexpr int choose()
    {
        int e = 512 / work;
        if (e < 1) e = 1;
        while (e > 1 && e * BYTES_EL > 64 * 1024) e--;
        return e;
    }
    static constexpr int E = choose();
};

template <int CELL, int P, typename T>
__global__ __launch_bounds__(256) void k_energy_grad(ExecArgs A, double scale, T *gmat, T *part)
{
    using C = GradCfg<CELL, P, T>;
    constexpr int NB = C::NB, NQ = C::NQ, E = C::E;
    extern __shared__ __align__(16) unsigned char smem[];
    double *xs = reinterpret_cast<double *>(smem);      // [E][NB][3]
    T *us = reinterpret_cast<T *>(xs + E * NB * 3);     // [E][3][NB]
    T *Nf = us + E * 3 * NB;                            // [E][NQ][9] reference-space flux of dJ/dx
    T *gq = Nf + E * NQ * 9;                            // [E][NQ][2] per-point dJ/dc (ISO_CELL sums)

    const int64_t e0 = logical_block(A.xcd_remap) * E;
    const int tid = threadIdx.x, nt = blockDim.x;
    const T *U = static_cast<const T *>(A.dofs);
    const T *mat = static_cast<const T *>(A.mat);

    for (int i = tid; i < E * NB; i += nt) {
        const int el = i / NB, a = i - el * NB;
        const int64_t e = e0 + el;
        double x0 = 0.0, x1 = 0.0, x2 = 0.0;
        T u0 = T(0), u1 = T(0), u2 = T(0);
        if (e < A.n_cells) {
            const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
            x0 = A.coords[3 * n];
            x1 = A.coords[3 * n + 1];
            x2 = A.coords[3 * n + 2];
            u0 = U[3 * n];
            u1 = U[3 * n + 1];
            u2 = U[3 * n + 2];
        }
        xs[i * 3 + 0] = x0;
        xs[i * 3 + 1] = x1;
        xs[i * 3 + 2] = x2;
        us[(el * 3 + 0) * NB + a] = u0;
        us[(el * 3 + 1) * NB + a] = u1;
        us[(el * 3 + 2) * NB + a] = u2;
    }
    __syncthreads();

    for (int i = tid; i < E * NQ; i += nt) {
        const int el = i / NQ, q = i - el * NQ;
        const int64_t e = e0 + el;
        if (e >= A.n_cells) continue;
        double J[3][3], Jid[3][3];
        jacobian_qp<NB, NQ>(xs + el * NB * 3, A.tab.bfgT, q, J);
        const double det = inverse3(J, Jid);
        if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
        const T w = static_cast<T>(A.tab.w[q] * det);
        T Ji[3][3];
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int d = 0; d < 3; d++) Ji[j][d] = static_cast<T>(Jid[j][d]);
        // reference then physical displacement gradient H[r][d] = du_r/dx_d
        T Hx[3][3] = {};
        const T *u = us + el * 3 * NB;
        for (int a = 0; a < NB; a++) {
            const T g0 = static_cast<T>(A.tab.bfgT[(a * 3 + 0) * NQ + q]);
            const T g1 = static_cast<T>(A.tab.bfgT[(a * 3 + 1) * NQ + q]);
            const T g2 = static_cast<T>(A.tab.bfgT[(a * 3 + 2) * NQ + q]);
#pragma unroll
            for (int r = 0; r < 3; r++) {
                const T ur = u[r * NB + a];
                Hx[r][0] += g0 * ur;
                Hx[r][1] += g1 * ur;
                Hx[r][2] += g2 * ur;
            }
        }
        T H[3][3];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int d = 0; d < 3; d++) H[r][d] = Hx[r][0] * Ji[0][d] + Hx[r][1] * Ji[1][d] + Hx[r][2] * Ji[2][d];
        T lam, mu;
        if (A.mat_kind == FE_MAT_ISO_QP) {
            lam = mat[2 * (e * NQ + q)];
            mu = mat[2 * (e * NQ + q) + 1];
        } else {
            lam = mat[2 * e];
            mu = mat[2 * e + 1];
        }
        const T tr = H[0][0] + H[1][1] + H[2][2];
        T eps[3][3], sig[3][3];
        T ee = T(0), W = T(0);
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
        gq[i * 2 + 0] = w * tr * tr;
        gq[i * 2 + 1] = T(2) * w * ee;
        // M = w (W I - 2 H^T sigma); reference flux N[k][j] = sum_l M[k][l] Jinv[j][l]
        T M[3][3];
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int l = 0; l < 3; l++) {
                T s = T(0);
#pragma unroll
                for (int r = 0; r < 3; r++) s += H[r][k] * sig[r][l];
                M[k][l] = w * ((k == l ? W : T(0)) - T(2) * s);
            }
        T *nf = Nf + i * 9;
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int j = 0; j < 3; j++) nf[k * 3 + j] = M[k][0] * Ji[j][0] + M[k][1] * Ji[j][1] + M[k][2] * Ji[j][2];
    }
    __syncthreads();

    if (gmat) {
        if (A.mat_kind == FE_MAT_ISO_QP) {
            for (int i = tid; i < E * NQ * 2; i += nt) {
                const int el = i / (NQ * 2);
                if (e0 + el < A.n_cells) gmat[e0 * NQ * 2 + i] = static_cast<T>(scale * static_cast<double>(gq[i]));
            }
        } else {
            for (int i = tid; i < E * 2; i += nt) {
                const int el = i / 2, c = i - 2 * el;
                if (e0 + el >= A.n_cells) continue;
                double s = 0.0;
                for (int q = 0; q < NQ; q++) s += static_cast<double>(gq[(el * NQ + q) * 2 + c]);
                gmat[(e0 + el) * 2 + c] = static_cast<T>(scale * s);
            }
        }
    }
    if (part) {
        for (int i = tid; i < E * 3 * NB; i += nt) {
            const int el = i / (3 * NB), rem = i - el * 3 * NB, k = rem / NB, a = rem - k * NB;
            const int64_t e = e0 + el;
            if (e >= A.n_cells) continue;
            T s = T(0);
            for (int q = 0; q < NQ; q++) {
                const T *nf = Nf + (el * NQ + q) * 9 + k * 3;
                s += static_cast<T>(A.tab.bfgT[(a * 3 + 0) * NQ + q]) * nf[0] +
                     static_cast<T>(A.tab.bfgT[(a * 3 + 1) * NQ + q]) * nf[1] +
                     static_cast<T>(A.tab.bfgT[(a * 3 + 2) * NQ + q]) * nf[2];
            }
            part[(e * 3 + k) * NB + a] = s;
        }
    }
}

template <int CELL, int P, typename T>
int launch_grad(const ExecArgs &A, double scale, void *gmat, void *part, hipStream_t st)
{
    using C = GradCfg<CELL, P, T>;
    if (A.n_cells <= 0) return FE_OK;
    const int64_t blocks = (A.n_cells + C::E - 1) / C::E;
    const int lds = C::E * C::BYTES_EL;
    if (lds > 64 * 1024)
        FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(k_energy_grad<CELL, P, T>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    hipLaunchKernelGGL((k_energy_grad<CELL, P, T>), dim3((unsigned)blocks), dim3(256), lds, st, A, scale,
                       static_cast<T *>(gmat), static_cast<T *>(part));
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

template <typename T>
int dispatch_grad(int cell, int order, const ExecArgs &A, double scale, void *gmat, void *part, hipStream_t st)
{
    if (cell == FE_CELL_HEX) {
        if (order == 1) return launch_grad<FE_CELL_HEX, 1, T>(A, scale, gmat, part, st);
        if (order == 2) return launch_grad<FE_CELL_HEX, 2, T>(A, scale, gmat, part, st);
        if (order == 3) return launch_grad<FE_CELL_HEX, 3, T>(A, scale, gmat, part, st);
    } else {
        if (order == 1) return launch_grad<FE_CELL_TET, 1, T>(A, scale, gmat, part, st);
        if (order == 2) return launch_grad<FE_CELL_TET, 2, T>(A, scale, gmat, part, st);
    }
    set_error("no gradient kernel for this cell/order");
    return FE_ERR_UNSUPPORTED;
}

int gather_launch(const fe_incidence_s *inc, int nc, bool fp64_in, bool fp64_out, const void *vec, double scale,
                  void *out, hipStream_t st)
{
    const int64_t n = inc->n_nodes * nc;
    if (n == 0) return FE_OK;
    const int64_t blocks = (n + 255) / 256;
    if (fp64_in && fp64_out)
        hipLaunchKernelGGL((k_gather<double, double>), dim3((unsigned)blocks), dim3(256), 0, st, inc->offsets,
                           inc->items, inc->n_nodes, inc->nb, nc, static_cast<const double *>(vec), scale,
                           static_cast<double *>(out));
    else if (!fp64_in && fp64_out)
        hipLaunchKernelGGL((k_gather<float, double>), dim3((unsigned)blocks), dim3(256), 0, st, inc->offsets,
                           inc->items, inc->n_nodes, inc->nb, nc, static_cast<const float *>(vec), scale,
                           static_cast<double *>(out));
    else if (!fp64_in && !fp64_out)
        hipLaunchKernelGGL((k_gather<float, float>), dim3((unsigned)blocks), dim3(256), 0, st, inc->offsets,
                           inc->items, inc->n_nodes, inc->nb, nc, static_cast<const float *>(vec), scale,
                           static_cast<float *>(out));
    else
        return FE_ERR_INVALID_ARG;
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

}  // namespace

size_t grad_part_bytes(const Plan &p, int64_t n_cells)
{
    return (size_t)n_cells * 3 * p.nb * (p.prec == FE_PREC_FP64 ? 8 : 4);
}

int energy_grad_impl(const Plan &p, const fe_incidence_s *inc, const ExecArgs &A, double scale, void *gmat,
                     double *gcoords, void *part, hipStream_t st)
{
    // hexahedra: the sum-factorized kernel; tetrahedra: the per-point kernel
    int rc = adjoint_sumfact(p, A, scale, gmat, gcoords ? part : nullptr, st);
    if (rc == FE_ERR_UNSUPPORTED) {
        if (p.prec == FE_PREC_FP64)
            rc = dispatch_grad<double>(p.cell, p.order, A, scale, gmat, gcoords ? part : nullptr, st);
        else
            rc = dispatch_grad<float>(p.cell, p.order, A, scale, gmat, gcoords ? part : nullptr, st);
    }
    if (rc || !gcoords) return rc;
    return gather_launch(inc, 3, p.prec == FE_PREC_FP64, true, part, scale, gcoords, st);
}

int assemble_impl(const fe_incidence_s *inc, int nc, int prec, const void *vec, double scale, void *out,
                  hipStream_t st)
{
    const bool f64 = prec == FE_PREC_FP64;
    return gather_launch(inc, nc, f64, f64, vec, scale, out, st);
}

int incidence_build(fe_incidence_s *inc, const int32_t *conn, hipStream_t st)
{
    const int64_t n_items = inc->n_cells * inc->nb;
    const int64_t nn = inc->n_nodes;
    int32_t *cnt = nullptr;
    unsigned *flags = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int rc = FE_OK;
    auto cleanup = [&]() {
        if (cnt) (void)hipFree(cnt);
        if (flags) (void)hipFree(flags);
        if (tmp) (void)hipFree(tmp);
    };
    if (hipMalloc(&inc->offsets, (nn + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&inc->items, (n_items > 0 ? n_items : 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&cnt, (nn + 1) * sizeof(int32_t)) != hipSuccess || hipMalloc(&flags, sizeof(unsigned)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("incidence allocation failed");
        return FE_ERR_OUT_OF_MEMORY;
    }
    if (hipMemsetAsync(cnt, 0, (nn + 1) * sizeof(int32_t), st) != hipSuccess ||
        hipMemsetAsync(flags, 0, sizeof(unsigned), st) != hipSuccess) {
        cleanup();
        set_error("hipMemsetAsync failed");
        return FE_ERR_HIP;
    }
    const unsigned gi = (unsigned)((n_items + 255) / 256), gn = (unsigned)((nn + 255) / 256);
    if (n_items > 0) hipLaunchKernelGGL(k_inc_count, dim3(gi), dim3(256), 0, st, conn, n_items, nn, cnt, flags);
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, inc->offsets, (int)(nn + 1), st) != hipSuccess ||
        hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1) != hipSuccess ||
        hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, inc->offsets, (int)(nn + 1), st) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("prefix sum failed");
        return FE_ERR_HIP;
    }
    // reuse cnt as the fill cursor
    if (hipMemcpyAsync(cnt, inc->offsets, (nn + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, st) != hipSuccess) {
        cleanup();
        set_error("copy failed");
        return FE_ERR_HIP;
    }
    if (n_items > 0) hipLaunchKernelGGL(k_inc_fill, dim3(gi), dim3(256), 0, st, conn, n_items, nn, cnt, inc->items);
    if (nn > 0) hipLaunchKernelGGL(k_inc_sort, dim3(gn), dim3(256), 0, st, inc->offsets, nn, inc->items);
    unsigned hflags = 0;
    if (hipMemcpyAsync(&hflags, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("incidence build failed");
        return FE_ERR_HIP;
    }
    if (hflags & FAULT_INDEX) {
        set_error("a connectivity entry is out of range");
        rc = FE_ERR_INDEX_OUT_OF_RANGE;
    }
    cleanup();
    return rc;
}

}  // namespace fe
