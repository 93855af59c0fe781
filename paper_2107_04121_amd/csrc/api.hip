// C ABI of the gfx950 weak-form library: plans, validation, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "fe_internal.h"



namespace fe {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int n_comp_of(int form) { return (form == FE_FORM_MASS || form == FE_FORM_LAPLACE) ? 1 : 3; }

size_t grad_part_bytes(const Plan &p, int64_t n_cells);
int energy_grad_impl(const Plan &p, const fe_incidence_s *inc, const ExecArgs &A, double scale, void *gmat,
                     double *gcoords, void *part, hipStream_t st);
int assemble_impl(const fe_incidence_s *inc, int nc, int prec, const void *vec, double scale, void *out,
                  hipStream_t st);
int incidence_build(fe_incidence_s *inc, const int32_t *conn, hipStream_t st);

int batch_create(int n_groups, const fe_group *groups, int precision, int autotune, fe_batch_s **out);
int batch_execute(fe_batch_s *b, hipStream_t st);
int batch_check(fe_batch_s *b, hipStream_t st);
int batch_info(fe_batch_s *b, int *tiles, float *tune_ms, int *grid);
void batch_destroy(fe_batch_s *b);

LaunchFn select_generic_f64(const Plan &p);
LaunchFn select_generic_f32(const Plan &p);

LaunchFn select_generic(const Plan &p)
{
    if (p.prec == FE_PREC_FP64) return select_generic_f64(p);
    if (p.prec == FE_PREC_FP32) return select_generic_f32(p);
    return nullptr;
}

int fail(int status, const std::string &msg)
{
    set_error(msg);
    return status;
}

static constexpr size_t FLAG_BYTES = 256;

size_t workspace_bytes_of(const Plan &p, int64_t n_cells)
{
    return FLAG_BYTES + (p.variant == FE_VARIANT_MATRIX_FIRST ? matrix_first_bytes(p, n_cells) : 0);
}

}  // namespace fe

using namespace fe;

extern "C" {

const char *fe_status_string(int s)
{
    switch (s) {
    case FE_OK: return "FE_OK";
    case FE_ERR_INVALID_ARG: return "FE_ERR_INVALID_ARG";
    case FE_ERR_UNSUPPORTED: return "FE_ERR_UNSUPPORTED";
    case FE_ERR_NONPOSITIVE_JACOBIAN: return "FE_ERR_NONPOSITIVE_JACOBIAN";
    case FE_ERR_INDEX_OUT_OF_RANGE: return "FE_ERR_INDEX_OUT_OF_RANGE";
    case FE_ERR_OUT_OF_MEMORY: return "FE_ERR_OUT_OF_MEMORY";
    case FE_ERR_HIP: return "FE_ERR_HIP";
    case FE_ERR_NO_DEVICE: return "FE_ERR_NO_DEVICE";
    }
    return "FE_ERR_UNKNOWN";
}

const char *fe_last_error(void) { return g_last_error.c_str(); }

const char *fe_version(void) { return "fe_forms 0.1 (gfx950)"; }

int fe_reference_sizes(int cell, int order, int *n_basis, int *n_qp)
{
    int nb, nq;
    int st = reference_sizes(cell, order, &nb, &nq);
    if (st) return fail(st, "unsupported cell/order");
    if (n_basis) *n_basis = nb;
    if (n_qp) *n_qp = nq;
    return FE_OK;
}

int fe_reference_tables(int cell, int order, double *weights, double *points, double *bf, double *bfg)
{
    RefTables T;
    int st = reference_tables(cell, order, T);
    if (st) return fail(st, "unsupported cell/order");
    if (weights) std::memcpy(weights, T.w.data(), T.w.size() * sizeof(double));
    if (points) std::memcpy(points, T.pts.data(), T.pts.size() * sizeof(double));
    if (bf) std::memcpy(bf, T.bf.data(), T.bf.size() * sizeof(double));
    if (bfg) std::memcpy(bfg, T.bfg.data(), T.bfg.size() * sizeof(double));
    return FE_OK;
}

}  // extern "C"

namespace fe {

// Plan creation shared by fe_plan_create, fe_plan_create_ref and
// fe_plan_create_bilinear: caller (if not NULL) replaces the library's
// reference tables, bl (if not NULL) describes a generic bilinear form.
static int plan_create_impl(int cell, int order, int form, int mode, int precision, int material_kind,
                            const fe_options *opts, const RefTables *caller, const BilinearDesc *bl, fe_plan *out)
{
    if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (cell != FE_CELL_HEX && cell != FE_CELL_TET) return fail(FE_ERR_INVALID_ARG, "bad cell");
    if (form < FE_FORM_MASS || form > FE_FORM_BILINEAR) return fail(FE_ERR_INVALID_ARG, "bad form");
    if ((form == FE_FORM_BILINEAR) != (bl != nullptr))
        return fail(FE_ERR_INVALID_ARG, "generic bilinear plans are created by fe_plan_create_bilinear");
    if (mode < FE_MODE_MATRIX || mode > FE_MODE_EVAL) return fail(FE_ERR_INVALID_ARG, "bad mode");
    if (precision < FE_PREC_FP64 || precision > FE_PREC_BF16X3) return fail(FE_ERR_INVALID_ARG, "bad precision");
    if (form == FE_FORM_ELASTICITY) {
        if (material_kind < FE_MAT_ISO_CELL || material_kind > FE_MAT_VOIGT_QP)
            return fail(FE_ERR_INVALID_ARG, "elasticity needs a material kind");
    } else if (form == FE_FORM_WDOT) {
        if (material_kind != FE_MAT_TENSOR_QP)
            return fail(FE_ERR_INVALID_ARG, "the weighted dot product needs material kind TENSOR_QP");
    } else if (form == FE_FORM_BILINEAR) {
        if (material_kind != FE_MAT_NONE && material_kind != FE_MAT_TENSOR_QP)
            return fail(FE_ERR_INVALID_ARG, "a generic bilinear form takes material NONE or TENSOR_QP");
    } else if (material_kind != FE_MAT_NONE) {
        return fail(FE_ERR_INVALID_ARG, "only elasticity and the weighted dot product take a material");
    }
    int nb, nq;
    if (reference_sizes(cell, order, &nb, &nq)) return fail(FE_ERR_UNSUPPORTED, "unsupported cell/order");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return fail(FE_ERR_NO_DEVICE, "no HIP device");
    }
    fe_plan_s *p = new (std::nothrow) fe_plan_s();
    if (!p) return fail(FE_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->cell = cell;
    p->order = order;
    p->form = form;
    p->mode = mode;
    p->prec = precision;
    p->mat_kind = material_kind;
    p->nb = nb;
    p->nq = nq;
    p->nc = form == FE_FORM_BILINEAR ? bl->test_comp : n_comp_of(form);
    p->device = dev;
    if (bl) p->bl = *bl;
    if (opts) p->opts = *opts;
    else {
        p->opts.variant = FE_VARIANT_AUTO;
        p->opts.xcd_remap = -1;
    }
    if (p->opts.layout != FE_LAYOUT_CELL_MAJOR && p->opts.layout != FE_LAYOUT_CELL_MINOR) {
        delete p;
        return fail(FE_ERR_INVALID_ARG, "bad layout");
    }
    if (caller) {
        p->ref = *caller;
    } else if (reference_tables(cell, order, p->ref)) {
        delete p;
        return fail(FE_ERR_UNSUPPORTED, "reference tables");
    }
    // kernel choice
    const int want = p->opts.variant;
    LaunchFn fn = nullptr;
    int variant = FE_VARIANT_GENERIC;
    if (form == FE_FORM_BILINEAR) {
        if (want != FE_VARIANT_AUTO && want != FE_VARIANT_GENERIC) {
            delete p;
            return fail(FE_ERR_UNSUPPORTED, "generic bilinear forms run on the generic kernel only");
        }
        if (precision == FE_PREC_BF16X3 || !(fn = select_bilinear(*p))) {
            delete p;
            return fail(FE_ERR_UNSUPPORTED, "the generic bilinear kernel covers hex orders 1-3 and tets, FP64/FP32");
        }
        if (mode == FE_MODE_EVAL && (bl->test_comp != bl->trial_comp || bl->test_grad != bl->trial_grad)) {
            delete p;
            return fail(FE_ERR_UNSUPPORTED, "eval binds the test to the unknown's DOFs: operators must match");
        }
    }
    if (!fn && want == FE_VARIANT_MATRIX_FIRST) {
        if (mode != FE_MODE_RESIDUAL || p->opts.layout != FE_LAYOUT_CELL_MAJOR) {
            delete p;
            return fail(FE_ERR_UNSUPPORTED, "matrix-first is a cell-major residual variant");
        }
        if (form == FE_FORM_CONVECT) {
            delete p;
            return fail(FE_ERR_UNSUPPORTED, "the convection matrix is a derivative: K(u) u = 2 r(u)");
        }
        Plan pm = *p;
        pm.mode = FE_MODE_MATRIX;
        LaunchFn fm = select_mfma(pm);
        if (!fm) fm = select_cellwise(pm);
        if (!fm) fm = select_generic(pm);
        if (!fm) {
            delete p;
            return fail(FE_ERR_UNSUPPORTED, "no matrix kernel for matrix-first");
        }
        p->launch_mat = fm;
        fn = launch_matrix_first;
        variant = FE_VARIANT_MATRIX_FIRST;
    }
    if (!fn && (want == FE_VARIANT_AUTO || want == FE_VARIANT_MFMA)) {
        if (mode == FE_MODE_MATRIX && (fn = select_mfma(*p))) variant = FE_VARIANT_MFMA;
    }
    if (!fn && want == FE_VARIANT_MFMA_WS && mode == FE_MODE_MATRIX) {
        if ((fn = select_q2ws(*p))) variant = FE_VARIANT_MFMA_WS;
    }
    if (!fn && want == FE_VARIANT_MFMA_JOBS && mode == FE_MODE_MATRIX) {
        fn = select_hexgm(*p);
        if (!fn) fn = select_hexmm(*p);
        if (fn) variant = FE_VARIANT_MFMA_JOBS;
    }
    if (!fn && (want == FE_VARIANT_AUTO || want == FE_VARIANT_CELLWISE)) {
        if (mode == FE_MODE_MATRIX && (fn = select_cellwise(*p))) variant = FE_VARIANT_CELLWISE;
    }
    if (!fn && (want == FE_VARIANT_AUTO || want == FE_VARIANT_SUMFACT)) {
        if (mode != FE_MODE_MATRIX && (fn = select_sumfact(*p))) variant = FE_VARIANT_SUMFACT;
    }
    if (!fn && (want == FE_VARIANT_AUTO || want == FE_VARIANT_GENERIC)) {
        if ((fn = select_generic(*p))) variant = FE_VARIANT_GENERIC;
    }
    if (!fn) {
        delete p;
        return fail(FE_ERR_UNSUPPORTED, "no kernel for this cell/order/form/mode/precision/variant");
    }
    if (p->opts.layout == FE_LAYOUT_CELL_MINOR && (variant != FE_VARIANT_SUMFACT || mode != FE_MODE_RESIDUAL)) {
        delete p;
        return fail(FE_ERR_UNSUPPORTED, "cell-minor output exists for sum-factorized residuals only");
    }
    p->launch = fn;
    p->variant = variant;
    // device tables: w | bf | bfgT | B1 | D1 | coupling
    const int n1 = (cell == FE_CELL_HEX) ? (order + 1) * (order + 1) : 0;
    const size_t ncoup = p->bl.coup.size();
    const size_t nwords = nq + (size_t)nq * nb + (size_t)nb * 3 * nq + 2 * n1 + ncoup;
    std::vector<double> h(nwords, 0.0);
    double *w = h.data(), *bf = w + nq, *bfgT = bf + (size_t)nq * nb, *B1 = bfgT + (size_t)nb * 3 * nq,
           *D1 = B1 + n1, *coup = D1 + n1;
    for (int q = 0; q < nq; q++) {
        w[q] = p->ref.w[q];
        for (int a = 0; a < nb; a++) {
            bf[(size_t)q * nb + a] = p->ref.bf[(size_t)q * nb + a];
            for (int j = 0; j < 3; j++) bfgT[((size_t)a * 3 + j) * nq + q] = p->ref.bfg[((size_t)q * 3 + j) * nb + a];
        }
    }
    for (int i = 0; i < n1; i++) {
        B1[i] = p->ref.B1[i];
        D1[i] = p->ref.D1[i];
    }
    for (size_t i = 0; i < ncoup; i++) coup[i] = p->bl.coup[i];
    if (hipMalloc(&p->d_tab, nwords * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(FE_ERR_OUT_OF_MEMORY, "device table allocation failed");
    }
    if (hipMemcpy(p->d_tab, h.data(), nwords * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p->d_tab);
        delete p;
        return fail(FE_ERR_HIP, "device table copy failed");
    }
    p->tab.w = p->d_tab;
    p->tab.bf = p->d_tab + (bf - w);
    p->tab.bfgT = p->d_tab + (bfgT - w);
    p->tab.B1 = p->d_tab + (B1 - w);
    p->tab.D1 = p->d_tab + (D1 - w);
    p->tab.coup = ncoup ? p->d_tab + (coup - w) : nullptr;
    *out = p;
    return FE_OK;
}

static bool finite_all(const double *x, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// Caller tables: sizes, values, partition of unity, positive weights; the
// 1-D factors of hexahedral tables; constant gradients of P1 tetrahedra.
static int caller_tables(const fe_reference *r, RefTables &T)
{
    if (!r) return fail(FE_ERR_INVALID_ARG, "reference is NULL");
    int nb, nq;
    if (reference_sizes(r->cell, r->order, &nb, &nq)) return fail(FE_ERR_UNSUPPORTED, "unsupported cell/order");
    if (r->n_basis != nb || r->n_qp != nq)
        return fail(FE_ERR_UNSUPPORTED, "the kernels are compiled for " + std::to_string(nb) + " basis functions and " +
                                            std::to_string(nq) + " points for this cell and order");
    if (!r->weights || !r->bf || !r->bfg) return fail(FE_ERR_INVALID_ARG, "reference table pointer is NULL");
    T = RefTables();
    T.cell = r->cell;
    T.order = r->order;
    T.nb = nb;
    T.nq = nq;
    T.w.assign(r->weights, r->weights + nq);
    T.bf.assign(r->bf, r->bf + (size_t)nq * nb);
    T.bfg.assign(r->bfg, r->bfg + (size_t)nq * 3 * nb);
    if (!finite_all(T.w.data(), T.w.size()) || !finite_all(T.bf.data(), T.bf.size()) ||
        !finite_all(T.bfg.data(), T.bfg.size()))
        return fail(FE_ERR_INVALID_ARG, "reference tables hold non-finite values");
    for (int q = 0; q < nq; q++) {
        if (!(T.w[q] > 0.0)) return fail(FE_ERR_INVALID_ARG, "quadrature weights must be positive");
        double s = 0.0, g[3] = {0.0, 0.0, 0.0}, gm = 0.0;
        for (int a = 0; a < nb; a++) {
            s += T.bf[(size_t)q * nb + a];
            for (int j = 0; j < 3; j++) {
                const double v = T.bfg[((size_t)q * 3 + j) * nb + a];
                g[j] += v;
                gm = std::fmax(gm, std::fabs(v));
            }
        }
        if (std::fabs(s - 1.0) > 1e-12 || std::fabs(g[0]) > 1e-12 * (1.0 + gm) ||
            std::fabs(g[1]) > 1e-12 * (1.0 + gm) || std::fabs(g[2]) > 1e-12 * (1.0 + gm))
            return fail(FE_ERR_INVALID_ARG, "the basis must be a partition of unity (sum phi = 1, sum dphi = 0)");
    }
    if (r->cell == FE_CELL_HEX) {
        std::string why;
        if (hex_factor_tables(r->order, T, why)) return fail(FE_ERR_UNSUPPORTED, why);
    } else if (r->order == 1) {
        for (int q = 1; q < nq; q++)
            for (int k = 0; k < 3 * nb; k++)
                if (std::fabs(T.bfg[(size_t)q * 3 * nb + k] - T.bfg[k]) > 1e-12 * (1.0 + std::fabs(T.bfg[k])))
                    return fail(FE_ERR_UNSUPPORTED, "P1 tetrahedra need constant basis gradients");
    }
    return FE_OK;
}

}  // namespace fe

extern "C" {

int fe_plan_create(int cell, int order, int form, int mode, int precision, int material_kind,
                   const fe_options *opts, fe_plan *out)
{
    return plan_create_impl(cell, order, form, mode, precision, material_kind, opts, nullptr, nullptr, out);
}

int fe_plan_create_ref(const fe_reference *ref, int form, int mode, int precision, int material_kind,
                       const fe_options *opts, fe_plan *out)
{
    if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (form == FE_FORM_BILINEAR) return fail(FE_ERR_INVALID_ARG, "bilinear plans: fe_plan_create_bilinear");
    RefTables T;
    int rc = caller_tables(ref, T);
    if (rc) return rc;
    return plan_create_impl(ref->cell, ref->order, form, mode, precision, material_kind, opts, &T, nullptr, out);
}

int fe_plan_create_bilinear(int cell, int order, int mode, int precision, int material_kind,
                            const fe_bilinear *d, const fe_options *opts, fe_plan *out)
{
    if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d) return fail(FE_ERR_INVALID_ARG, "description is NULL");
    if ((d->test_grad != 0 && d->test_grad != 1) || (d->trial_grad != 0 && d->trial_grad != 1) ||
        (d->test_comp != 1 && d->test_comp != 3) || (d->trial_comp != 1 && d->trial_comp != 3))
        return fail(FE_ERR_INVALID_ARG, "operators: grad 0 or 1, components 1 or 3");
    BilinearDesc b;
    b.test_grad = d->test_grad;
    b.test_comp = d->test_comp;
    b.trial_grad = d->trial_grad;
    b.trial_comp = d->trial_comp;
    b.Kt = d->test_comp * (d->test_grad ? 3 : 1);
    b.Ku = d->trial_comp * (d->trial_grad ? 3 : 1);
    if (material_kind == FE_MAT_NONE) {
        if (!d->W0) return fail(FE_ERR_INVALID_ARG, "W0 is NULL (material NONE)");
        b.coup.assign(d->W0, d->W0 + b.Kt * b.Ku);
    } else if (material_kind == FE_MAT_TENSOR_QP) {
        if (!d->P_test || !d->P_trial || d->n_a < 1 || d->n_a > 9 || d->n_b < 1 || d->n_b > 9 ||
            (d->mat_transpose != 0 && d->mat_transpose != 1))
            return fail(FE_ERR_INVALID_ARG, "P_test/P_trial NULL or material shape outside 1..9");
        b.n_a = d->n_a;
        b.n_b = d->n_b;
        b.mat_transpose = d->mat_transpose;
        b.coup.assign(d->P_test, d->P_test + b.Kt * b.n_a);
        b.coup.insert(b.coup.end(), d->P_trial, d->P_trial + b.Ku * b.n_b);
    } else {
        return fail(FE_ERR_INVALID_ARG, "a generic bilinear form takes material NONE or TENSOR_QP");
    }
    if (!finite_all(b.coup.data(), b.coup.size())) return fail(FE_ERR_INVALID_ARG, "non-finite coupling tables");
    return plan_create_impl(cell, order, FE_FORM_BILINEAR, mode, precision, material_kind, opts, nullptr, &b, out);
}

int fe_plan_info(fe_plan p, int *n_basis, int *n_qp, int *n_comp, int *variant, int *n_dof)
{
    if (!p) return fail(FE_ERR_INVALID_ARG, "plan is NULL");
    if (n_basis) *n_basis = p->nb;
    if (n_qp) *n_qp = p->nq;
    if (n_comp) *n_comp = p->nc;
    if (variant) *variant = p->variant;
    if (n_dof) *n_dof = p->nc * p->nb;
    return FE_OK;
}

int fe_plan_workspace_size(fe_plan p, int64_t n_cells, size_t *bytes)
{
    if (!p || !bytes || n_cells < 0) return fail(FE_ERR_INVALID_ARG, "bad argument");
    *bytes = workspace_bytes_of(*p, n_cells);
    return FE_OK;
}

}  // extern "C"

namespace fe {

// Validation and launch shared by fe_execute and fe_execute_noalloc.
int execute_impl(const Plan *p, int64_t n_cells, int64_t n_nodes, const double *coords, const int32_t *conn,
                 const void *material, const void *dofs, void *out, void *workspace, size_t workspace_bytes,
                 hipStream_t stream)
{
    if (!p) return fail(FE_ERR_INVALID_ARG, "plan is NULL");
    if (n_cells < 0 || n_nodes < 0) return fail(FE_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0) return FE_OK;
    if (n_nodes == 0) return fail(FE_ERR_INVALID_ARG, "cells without nodes");
    if (!coords || !conn || !out) return fail(FE_ERR_INVALID_ARG, "coords/conn/out is NULL");
    if ((p->form == FE_FORM_ELASTICITY || p->form == FE_FORM_WDOT ||
         (p->form == FE_FORM_BILINEAR && p->mat_kind == FE_MAT_TENSOR_QP)) &&
        !material)
        return fail(FE_ERR_INVALID_ARG, "material is NULL");
    if ((p->mode != FE_MODE_MATRIX || p->form == FE_FORM_CONVECT) && !dofs)
        return fail(FE_ERR_INVALID_ARG, "dofs is NULL");
    const size_t need = workspace_bytes_of(*p, n_cells);
    if (!workspace || workspace_bytes < need) return fail(FE_ERR_INVALID_ARG, "workspace too small");
    if (n_nodes > 0x7fffffffLL) return fail(FE_ERR_INVALID_ARG, "n_nodes exceeds int32 node numbers");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(FE_ERR_INVALID_ARG, "plan was created on another device");
    ExecArgs A{};
    A.n_cells = n_cells;
    A.n_nodes = n_nodes;
    A.coords = coords;
    A.conn = conn;
    A.mat = material;
    A.mat_kind = p->mat_kind;
    A.dofs = dofs;
    A.out = out;
    A.flags = static_cast<unsigned *>(workspace);
    A.tab = p->tab;
    A.xcd_remap = p->opts.xcd_remap == 0 ? 0 : 1;
    A.eval = p->mode == FE_MODE_EVAL ? 1 : 0;
    return p->launch(*p, A, stream);
}

}  // namespace fe

extern "C" {

int fe_execute(fe_plan p, int64_t n_cells, int64_t n_nodes, const double *coords, const int32_t *conn,
               const void *material, const void *dofs, void *out, void *workspace, size_t workspace_bytes,
               void *stream)
{
    return execute_impl(p, n_cells, n_nodes, coords, conn, material, dofs, out, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

int fe_eval_sum(fe_plan p, int64_t n_cells, int64_t n_nodes, const double *coords, const int32_t *conn,
                const void *material, const void *dofs, void *cell_values, double *total, void *workspace,
                size_t workspace_bytes, void *stream)
{
    if (!p) return fail(FE_ERR_INVALID_ARG, "plan is NULL");
    if (p->mode != FE_MODE_EVAL) return fail(FE_ERR_INVALID_ARG, "fe_eval_sum needs an EVAL plan");
    if (!total || (n_cells > 0 && !cell_values)) return fail(FE_ERR_INVALID_ARG, "total/cell_values is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = execute_impl(p, n_cells, n_nodes, coords, conn, material, dofs, cell_values, workspace,
                          workspace_bytes, st);
    if (rc) return rc;
    return sum_cells(cell_values, p->prec, n_cells, total, st);
}

int fe_plan_check(fe_plan p, void *workspace, void *stream)
{
    if (!p || !workspace) return fail(FE_ERR_INVALID_ARG, "bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned flags = 0;
    FE_HIP_CHECK(hipMemcpyAsync(&flags, workspace, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    FE_HIP_CHECK(hipStreamSynchronize(st));
    if (flags) {
        const unsigned zero = 0;
        FE_HIP_CHECK(hipMemcpyAsync(workspace, &zero, sizeof(unsigned), hipMemcpyHostToDevice, st));
        FE_HIP_CHECK(hipStreamSynchronize(st));
    }
    if (flags & FAULT_INDEX) return fail(FE_ERR_INDEX_OUT_OF_RANGE, "a connectivity entry is out of range");
    if (flags & FAULT_DET) return fail(FE_ERR_NONPOSITIVE_JACOBIAN, "det J <= 0 at a quadrature point");
    return FE_OK;
}

int fe_incidence_create(int64_t n_cells, int64_t n_nodes, int n_basis, const int32_t *conn, void *stream,
                        fe_incidence *out)
{
    if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_cells < 0 || n_nodes < 0 || n_basis <= 0 || (n_cells > 0 && (!conn || n_nodes == 0)))
        return fail(FE_ERR_INVALID_ARG, "bad incidence arguments");
    if (n_cells * (int64_t)n_basis > 0x7fffffffLL || n_nodes > 0x7ffffffeLL)
        return fail(FE_ERR_INVALID_ARG, "mesh too large for int32 incidence");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return fail(FE_ERR_NO_DEVICE, "no HIP device");
    }
    fe_incidence_s *inc = new (std::nothrow) fe_incidence_s();
    if (!inc) return fail(FE_ERR_OUT_OF_MEMORY, "host allocation failed");
    inc->n_cells = n_cells;
    inc->n_nodes = n_nodes;
    inc->nb = n_basis;
    inc->device = dev;
    int rc = incidence_build(inc, conn, static_cast<hipStream_t>(stream));
    if (rc) {
        fe_incidence_destroy(inc);
        return rc;
    }
    *out = inc;
    return FE_OK;
}

int fe_incidence_destroy(fe_incidence inc)
{
    if (!inc) return FE_OK;
    if (inc->offsets) (void)hipFree(inc->offsets);
    if (inc->items) (void)hipFree(inc->items);
    delete inc;
    return FE_OK;
}

int fe_assemble(fe_incidence inc, int n_comp, int precision, const void *cell_vec, double scale, void *out,
                void *stream)
{
    if (!inc || !cell_vec || !out || n_comp < 1 || n_comp > 3) return fail(FE_ERR_INVALID_ARG, "bad argument");
    if (precision < FE_PREC_FP64 || precision > FE_PREC_BF16X3) return fail(FE_ERR_INVALID_ARG, "bad precision");
    return assemble_impl(inc, n_comp, precision, cell_vec, scale, out, static_cast<hipStream_t>(stream));
}

int fe_energy_grad_workspace_size(fe_plan p, int64_t n_cells, size_t *bytes)
{
    if (!p || !bytes || n_cells < 0) return fail(FE_ERR_INVALID_ARG, "bad argument");
    *bytes = FLAG_BYTES + grad_part_bytes(*p, n_cells);
    return FE_OK;
}

int fe_energy_grad(fe_plan p, fe_incidence inc, int64_t n_cells, int64_t n_nodes, const double *coords,
                   const int32_t *conn, const void *material, const void *dofs, double scale, void *grad_material,
                   double *grad_coords, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!p) return fail(FE_ERR_INVALID_ARG, "plan is NULL");
    if (p->form != FE_FORM_ELASTICITY || p->mode != FE_MODE_EVAL ||
        (p->mat_kind != FE_MAT_ISO_QP && p->mat_kind != FE_MAT_ISO_CELL) || p->prec == FE_PREC_BF16X3)
        return fail(FE_ERR_UNSUPPORTED, "needs an ELASTICITY/EVAL plan with ISO_QP or ISO_CELL material, FP64/FP32");
    if (n_cells < 0 || n_nodes < 0) return fail(FE_ERR_INVALID_ARG, "negative size");
    if (n_cells == 0) return FE_OK;
    if (!coords || !conn || !material || !dofs) return fail(FE_ERR_INVALID_ARG, "NULL input");
    if (grad_coords && (!inc || inc->n_cells != n_cells || inc->n_nodes != n_nodes || inc->nb != p->nb))
        return fail(FE_ERR_INVALID_ARG, "incidence does not match the mesh");
    size_t need;
    fe_energy_grad_workspace_size(p, n_cells, &need);
    if (!workspace || workspace_bytes < need) return fail(FE_ERR_INVALID_ARG, "workspace too small");
    ExecArgs A{};
    A.n_cells = n_cells;
    A.n_nodes = n_nodes;
    A.coords = coords;
    A.conn = conn;
    A.mat = material;
    A.mat_kind = p->mat_kind;
    A.dofs = dofs;
    A.out = nullptr;
    A.flags = static_cast<unsigned *>(workspace);
    A.tab = p->tab;
    A.xcd_remap = p->opts.xcd_remap == 0 ? 0 : 1;
    void *part = static_cast<char *>(workspace) + FLAG_BYTES;
    return energy_grad_impl(*p, inc, A, scale, grad_material, grad_coords, part, static_cast<hipStream_t>(stream));
}

int fe_batch_create(int n_groups, const fe_group *groups, int precision, int autotune, fe_batch *out)
{
    if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
    return batch_create(n_groups, groups, precision, autotune, out);
}

int fe_batch_execute(fe_batch b, void *stream)
{
    if (!b) return fail(FE_ERR_INVALID_ARG, "batch is NULL");
    return batch_execute(b, static_cast<hipStream_t>(stream));
}

int fe_batch_check(fe_batch b, void *stream)
{
    if (!b) return fail(FE_ERR_INVALID_ARG, "batch is NULL");
    return batch_check(b, static_cast<hipStream_t>(stream));
}

int fe_batch_tiles(fe_batch b, int *tiles, float *tune_ms, int *grid)
{
    if (!b) return fail(FE_ERR_INVALID_ARG, "batch is NULL");
    return batch_info(b, tiles, tune_ms, grid);
}

int fe_batch_destroy(fe_batch b)
{
    batch_destroy(b);
    return FE_OK;
}

int fe_plan_destroy(fe_plan p)
{
    if (!p) return FE_OK;
    if (p->d_tab) (void)hipFree(p->d_tab);
    delete p;
    return FE_OK;
}

}  // extern "C"
