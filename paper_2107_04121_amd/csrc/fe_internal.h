// Internal declarations of the gfx950 weak-form library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fe_forms.h"

// Node-to-(cell, local node) incidence in CSR form (device arrays).
struct fe_incidence_s {
    int64_t n_cells = 0, n_nodes = 0;
    int nb = 0, device = -1;
    int32_t *offsets = nullptr;  // [n_nodes + 1]
    int32_t *items = nullptr;    // [n_cells * nb], item = e * nb + a, sorted per node
};

struct fe_batch_s;

namespace fe {

struct RefTables {
    int cell = 0, order = 0, nb = 0, nq = 0;
    std::vector<double> w, pts, bf, bfg;  // bf [nq][nb], bfg [nq][3][nb]
    std::vector<double> s1, w1, B1, D1;   // hex only: 1-D rule and basis [q][k]
};

int reference_sizes(int cell, int order, int *nb, int *nq);
int reference_tables(int cell, int order, RefTables &T);

// Device copy of the tables, laid out for the kernels:
//   w[nq] | bf[nq][nb] | bfgT[nb][3][nq] | B1[n][n] | D1[n][n] | coup  (FP64)
// coup: the coupling tables of a generic bilinear plan (else empty).
struct DevTables {
    const double *w, *bf, *bfgT, *B1, *D1, *coup;
};

// Hexahedral 1-D factors of tensor-product tables (w = w1 x w1 x w1,
// bf = B1 x B1 x B1, bfg_j with D1 in factor j), extracted from 3-D tables
// and checked against them; FE_ERR_UNSUPPORTED if they do not factor.
int hex_factor_tables(int order, RefTables &T, std::string &why);

// Operators and coupling of a generic bilinear plan (fe_bilinear).
struct BilinearDesc {
    int test_grad = 0, test_comp = 1, trial_grad = 0, trial_comp = 1;
    int Kt = 1, Ku = 1, n_a = 0, n_b = 0, mat_transpose = 0;
    std::vector<double> coup;  // W0 [Kt][Ku] or P_test [Kt][n_a] + P_trial [Ku][n_b]
};

// Fault bits written by kernels into the first word of the workspace.
// FAULT_REPEAT: a cell lists one node twice (refused by the pattern build).
enum : unsigned { FAULT_DET = 1u, FAULT_INDEX = 2u, FAULT_REPEAT = 4u };

// Everything a launcher needs for one fe_execute call.
struct ExecArgs {
    int64_t n_cells, n_nodes;
    const double *coords;
    const int32_t *conn;
    const void *mat;
    int mat_kind;
    const void *dofs;
    void *out;
    unsigned *flags;
    DevTables tab;
    int xcd_remap;
    int eval;  // residual-family kernels: 1 = write per-element energy
};

struct Plan;
using LaunchFn = int (*)(const Plan &, const ExecArgs &, hipStream_t);

struct Plan {
    int cell, order, form, mode, prec, mat_kind, variant;
    int nb, nq, nc;
    int device;
    RefTables ref;
    double *d_tab = nullptr;
    DevTables tab{};
    LaunchFn launch = nullptr;
    LaunchFn launch_mat = nullptr;  // MATRIX_FIRST: the matrix-mode kernel it uses
    fe_options opts{};
    BilinearDesc bl;                // FE_FORM_BILINEAR only
};

// thread-local error message
void set_error(const std::string &msg);

}  // namespace fe

// The ABI's opaque plan handle is the internal plan.
struct fe_plan_s : fe::Plan {};

namespace fe {

#define FE_HIP_CHECK(call)                                                     \
    do {                                                                       \
        hipError_t _e = (call);                                                \
        if (_e != hipSuccess) {                                                \
            ::fe::set_error(std::string(#call) + ": " + hipGetErrorString(_e)); \
            return FE_ERR_HIP;                                                 \
        }                                                                      \
    } while (0)

// Persistent launch of a kernel that walks XCD-contiguous cell ranges: as
// many workgroups as the device holds at once (a multiple of 8, at least 8,
// at most the number of cells).  The count is queried once per device and
// kernel and kept in resident[device] (0 = not yet known; concurrent first
// calls store the same value).
template <class K>
int launch_persistent(K kernel, int threads, const ExecArgs &A, hipStream_t st, std::atomic<int> *resident)
{
    if (A.n_cells <= 0) return FE_OK;
    if (A.n_cells > 0x7fffffffLL) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    int dev = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device index beyond 63");
        return FE_ERR_INVALID_ARG;
    }
    int r = resident[dev].load(std::memory_order_relaxed);
    if (!r) {
        int per_cu = 0, cus = 0;
        FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
        FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        r = per_cu * cus > 8 ? (per_cu * cus) & ~7 : 8;
        resident[dev].store(r, std::memory_order_relaxed);
    }
    const int64_t grid = A.n_cells < r ? A.n_cells : r;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), 0, st, A);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

// Kernel family selectors; each returns nullptr when it has no kernel for the
// plan (the caller then tries the next family).
LaunchFn select_generic(const Plan &p);
LaunchFn select_mfma(const Plan &p);
LaunchFn select_sumfact(const Plan &p);
LaunchFn select_cellwise(const Plan &p);
LaunchFn select_hexmm(const Plan &p);
LaunchFn select_hexgm(const Plan &p);
LaunchFn select_q2ws(const Plan &p);
LaunchFn select_bilinear(const Plan &p);
// deterministic sum of per-cell values (FP64 or FP32) into one FP64 value
int sum_cells(const void *vals, int prec, int64_t n, double *total, hipStream_t st);

// Gradient of the elasticity eval value on hexahedra by sum factorization
// (FE_ERR_UNSUPPORTED when the plan is not covered).
int adjoint_sumfact(const Plan &p, const ExecArgs &A, double scale, void *gmat, void *part, hipStream_t st);

int n_comp_of(int form);

// Material entries per cell of each material kind (the layouts of
// fe_material_kind): ISO_CELL 2, ISO_QP 2 n_qp, VOIGT_QP 36 n_qp,
// TENSOR_QP 9 n_qp, NONE 0.
inline int64_t material_entries_per_cell(int mat_kind, int nq)
{
    switch (mat_kind) {
    case FE_MAT_ISO_CELL: return 2;
    case FE_MAT_ISO_QP: return 2 * (int64_t)nq;
    case FE_MAT_VOIGT_QP: return 36 * (int64_t)nq;
    case FE_MAT_TENSOR_QP: return 9 * (int64_t)nq;
    default: return 0;
    }
}
size_t matrix_first_bytes(const Plan &p, int64_t n_cells);
// Workspace bytes of fe_execute: 256 bytes of fault bits, then the
// matrix-first chunk of element matrices when the plan uses it.
size_t workspace_bytes_of(const Plan &p, int64_t n_cells);
int execute_impl(const Plan *p, int64_t n_cells, int64_t n_nodes, const double *coords, const int32_t *conn,
                 const void *material, const void *dofs, void *out, void *workspace, size_t workspace_bytes,
                 hipStream_t stream);
int fail(int status, const std::string &msg);
int launch_matrix_first(const Plan &p, const ExecArgs &A, hipStream_t st);

}  // namespace fe
