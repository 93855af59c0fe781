/*
 * fe_forms.h -- C ABI of the MI355X (gfx950) per-element weak-form library.
 *
 * The library evaluates multilinear finite element weak forms element by
 * element and quadrature point by quadrature point, as in the paper's element
 * loops (Algorithm "feloopv": residual/action; Algorithm "feloopm": element
 * matrices) and its evaluation modes (section "Overview" of the weak form to
 * einsum transpiler: 'residual', 'matrix', 'eval').  The forms are those of
 * the table of example weak forms: vector dot product / mass ('i,i'), weak
 * Laplacian ('0.i,0.i') and linear elasticity ('IK,s(i:j)->I,s(k:l)->K').
 *
 * Conventions (fixed by this library where the paper leaves them open):
 *   - reference hexahedron [0,1]^3, tensor Gauss-Legendre rule with p+1
 *     points per axis ((p+1)^3 points, as in the paper's cell/DOF table);
 *     equispaced Lagrange basis of order p, isoparametric geometry;
 *     local numbering a = i + (p+1)(j + (p+1)k), x fastest;
 *   - reference tetrahedron {xi >= 0, xi_1+xi_2+xi_3 <= 1}, P1/P2 Lagrange
 *     basis, vertices then edge nodes on edges (0,1),(1,2),(0,2),(0,3),(1,3),
 *     (2,3); collapsed-coordinate Gauss-Jacobi rule, p+1 points per direction;
 *   - the geometry step (Jacobian J, det J, J^-1, w_q det J, physical basis
 *     gradients) is always computed in FP64 from FP64 node coordinates;
 *   - vector unknowns are component-major inside an element: row/column index
 *     r*n_basis + a (the reshape (j,k)->J below eq. fe1e); the global DOF
 *     array is (n_nodes, n_comp) row-major;
 *   - elasticity uses symmetric (Voigt) storage 11,22,33,12,13,23 with
 *     engineering shear (the extractor of section "Linear Elasticity
 *     Expression"), D is 6x6 in that order;
 *   - det J <= 0 at any quadrature point is an error (reported by
 *     fe_plan_check), never silently made positive.
 *
 * Ownership: every mesh, material, DOF, output and workspace buffer is a
 * DEVICE pointer owned by the caller.  A plan owns only its device copy of the
 * reference tables.  Nothing is allocated by fe_execute.  Calls enqueue work
 * on the given HIP stream (a hipStream_t passed as void*, NULL = default
 * stream) and return without synchronising, except fe_plan_check.
 *
 * Errors: every call returns an fe_status.  Host-side validation errors are
 * returned synchronously and nothing is enqueued.  Faults found by the
 * kernels (non-positive Jacobian, node index out of range) set sticky bits in
 * the workspace that fe_plan_check reads and clears; an out-of-range node
 * index is replaced by node 0 for the access so no kernel reads out of bounds.
 * fe_last_error() gives a thread-local message for the last failure.
 */
#ifndef FE_FORMS_H
#define FE_FORMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FE_OK = 0,
    FE_ERR_INVALID_ARG = 1,
    FE_ERR_UNSUPPORTED = 2,
    FE_ERR_NONPOSITIVE_JACOBIAN = 3,
    FE_ERR_INDEX_OUT_OF_RANGE = 4,
    FE_ERR_OUT_OF_MEMORY = 5,
    FE_ERR_HIP = 6,
    FE_ERR_NO_DEVICE = 7
} fe_status;

typedef enum { FE_CELL_HEX = 0, FE_CELL_TET = 1 } fe_cell;

/* Forms of the table of example weak forms.  MASS: scalar 'i,i' with one
 * component; VMASS: 'i,i' with three components (its matrix is D diagonal
 * blocks of the scalar one, eq. fe3c); LAPLACE: '0.i,0.i';
 * ELASTICITY: 'IK,s(i:j)->I,s(k:l)->K' with three components;
 * WDOT: the weighted vector dot product 'ij,i,j' (int v_i M_ij u_j, M a
 * 3 x 3 matrix per quadrature point, material kind TENSOR_QP);
 * CONVECT: the Navier-Stokes convection 'i,i.j,j' (int v_i du_i/dx_j u_j,
 * eq. fe2), non-linear: its residual is the action on the DOFs and its
 * matrix the derivative with respect to u at the DOFs passed (eq. fe4),
 *   K[(i,a),(c,m)] = int phi_a (delta_ic u . grad phi_m + du_i/dx_c phi_m),
 * so K(u) u = 2 r(u).
 * BILINEAR: any other bilinear form of the generalized notation, described
 * by its operators and coupling (fe_bilinear, fe_plan_create_bilinear). */
typedef enum {
    FE_FORM_MASS = 0,
    FE_FORM_VMASS = 1,
    FE_FORM_LAPLACE = 2,
    FE_FORM_ELASTICITY = 3,
    FE_FORM_WDOT = 4,
    FE_FORM_CONVECT = 5,
    FE_FORM_BILINEAR = 6
} fe_form;

/* MATRIX: element matrices (Algorithm "feloopm").  RESIDUAL: per-element
 * action on DOFs gathered through the connectivity, unassembled (Algorithm
 * "feloopv").  EVAL: per-element integral value u_e^T K_e u_e. */
typedef enum { FE_MODE_MATRIX = 0, FE_MODE_RESIDUAL = 1, FE_MODE_EVAL = 2 } fe_mode;

/* Arithmetic of the contraction.  The geometry step is FP64 in all three.
 * FP64: everything FP64, outputs/material/DOFs FP64.
 * FP32: contraction in FP32 (VALU or FP32 MFMA), FP32 outputs/material/DOFs.
 * BF16X3: each FP32 operand split as hi = bf16(a), lo = bf16(a - hi); the
 *         product is hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32
 *         accumulation; FP32 outputs/material/DOFs (matrix mode of the MFMA
 *         kernels only). */
typedef enum { FE_PREC_FP64 = 0, FE_PREC_FP32 = 1, FE_PREC_BF16X3 = 2 } fe_precision;

/* Material data layout (NONE for mass, Laplace and convection):
 * elasticity: ISO_CELL [n_cells][2] (lambda, mu); ISO_QP [n_cells][n_qp][2];
 * VOIGT_QP [n_cells][n_qp][6][6] (the per-quadrature-point D of the paper's
 * elasticity einsum, 'cqIK');
 * weighted dot product: TENSOR_QP [n_cells][n_qp][3][3] (M_ij, row-major).
 * FP64 in FP64 mode, FP32 otherwise. */
typedef enum {
    FE_MAT_NONE = 0,
    FE_MAT_ISO_CELL = 1,
    FE_MAT_ISO_QP = 2,
    FE_MAT_VOIGT_QP = 3,
    FE_MAT_TENSOR_QP = 4
} fe_material_kind;

/* Kernel variant (0 = automatic choice). */
typedef enum {
    FE_VARIANT_AUTO = 0,
    FE_VARIANT_GENERIC = 1,   /* reference-table VALU kernel, hex Q1-Q3 and tets */
    FE_VARIANT_MFMA = 2,      /* matrix mode: per-element GEMM on matrix cores */
    FE_VARIANT_SUMFACT = 3,   /* hex residual/eval: sum-factorized, gradient-first */
    FE_VARIANT_MATRIX_FIRST = 4, /* residual: form K_e then K_e u_e */
    FE_VARIANT_CELLWISE = 5,     /* matrix mode, Q1/P1/P2: one cell per lane, registers */
    FE_VARIANT_MFMA_JOBS = 6,    /* matrix mode, hex Q2-Q5: matrix-core tile jobs stored straight from the
                                    accumulators (no staging of the cell's matrix) */
    FE_VARIANT_MFMA_WS = 7       /* matrix mode, Q2 elasticity (ISO_CELL): tile jobs on consumer waves while
                                    producer waves build the next cell's operand */
} fe_variant;

/* Residual output layout: CELL_MAJOR [n_cells][n_comp][n_basis] (the
 * paper's default 'crd' order) or CELL_MINOR [n_comp][n_basis][n_cells]
 * (the cell axis last, as in the paper's layout study; sum-factorized
 * kernels only). */
typedef enum { FE_LAYOUT_CELL_MAJOR = 0, FE_LAYOUT_CELL_MINOR = 1 } fe_layout;

typedef struct {
    int variant;      /* fe_variant */
    int xcd_remap;    /* 1 = map contiguous element ranges to one XCD (default), 0 = off, -1 = default */
    int layout;       /* fe_layout of residual outputs */
    int chunk;        /* MATRIX_FIRST: cells per element-matrix chunk, 0 = default (16384) */
} fe_options;

typedef struct fe_plan_s *fe_plan;

/* Status name, e.g. "FE_ERR_INVALID_ARG". Never NULL. */
const char *fe_status_string(int status);
/* Thread-local detail message of the last failing call on this thread. */
const char *fe_last_error(void);
/* Library version string. */
const char *fe_version(void);

/* Number of basis functions and quadrature points of a reference element
 * (section "Notation": basis phi_k on the reference element, quadrature
 * points xi).  Host only. */
int fe_reference_sizes(int cell, int order, int *n_basis, int *n_qp);

/* The library's reference tables, written to HOST arrays of the caller:
 * weights[n_qp], points[n_qp][3], bf[n_qp][n_basis] (phi_a(xi_q)),
 * bfg[n_qp][3][n_basis] (d phi_a / d xi_j at xi_q).  Any pointer may be NULL.
 * Host only, no device needed. */
int fe_reference_tables(int cell, int order, double *weights, double *points,
                        double *bf, double *bfg);

/* Create a plan for one (cell, order, form, mode, precision, material kind)
 * on the current HIP device: builds the reference tables and copies them to
 * the device.  opts may be NULL.
 *
 * Supported (every other combination returns FE_ERR_UNSUPPORTED):
 *   cells and orders: HEX 1-5, TET 1-2;
 *   RESIDUAL, EVAL and MATRIX: every form and material kind, FP64 and
 *     FP32;
 *   MATRIX, BF16X3: MASS, VMASS, LAPLACE and ELASTICITY with ISO_CELL on
 *     HEX 2-5.
 * MATRIX_FIRST (a residual variant) needs a matrix kernel for the same
 * combination and is refused for CONVECT. */
int fe_plan_create(int cell, int order, int form, int mode, int precision,
                   int material_kind, const fe_options *opts, fe_plan *out);

/* Caller-supplied reference element (the paper's element loops take the
 * reference mappings as part of their data, Algorithms "feloopv" and
 * "feloopm"; the transpiler's evaluation function takes them with the FE
 * data, Algorithm "wfef").  HOST arrays, copied into the plan at creation:
 *   weights [n_qp]              quadrature weights on the reference cell;
 *   bf      [n_qp][n_basis]     phi_a at the points;
 *   bfg     [n_qp][3][n_basis]  d phi_a / d xi_j at the points.
 * n_basis and n_qp must equal the library's counts for the cell and order
 * (fe_reference_sizes: the kernels are compiled for them).  The basis must
 * be a partition of unity (sum_a phi_a = 1, sum_a d phi_a = 0, which the
 * isoparametric map needs to reproduce rigid translations) and the weights
 * positive.  Hexahedral tables must be tensor products of one 1-D rule and
 * one 1-D basis in the lexicographic order (point and node index
 * i + n(j + n k), x fastest): the sum-factorized and matrix-core kernels
 * work on the 1-D factors, which the library extracts and checks against
 * the given tables (relative 1e-12).  P1 tetrahedra need constant
 * gradients.  The reference cell itself is free: e.g. [-1,1]^3 tables
 * (weights x 8, gradients x 1/2) give the same element matrices. */
typedef struct {
    int cell, order, n_basis, n_qp;
    const double *weights;
    const double *bf;
    const double *bfg;
} fe_reference;

/* fe_plan_create with the caller's reference tables in place of the
 * library's (validated as above before any device query: FE_ERR_UNSUPPORTED
 * for sizes the kernels are not compiled for or hexahedral tables that do
 * not factor, FE_ERR_INVALID_ARG for non-finite values, weights <= 0 or a
 * basis that is not a partition of unity). */
int fe_plan_create_ref(const fe_reference *ref, int form, int mode, int precision, int material_kind,
                       const fe_options *opts, fe_plan *out);

/* A bilinear form  int (test operator) . W . (unknown operator)  for the
 * generic kernel (the shape every bilinear term of the generalized notation
 * takes once its identity and symmetric-gradient extractor operands are
 * contracted; the notation front-end derives these tables).
 *   test_grad / trial_grad: 0 = basis values, 1 = physical gradients;
 *   test_comp / trial_comp: 1 (scalar) or 3 (vector) components.
 * Operator rows are (component r, derivative j), component-major, j absent
 * for values: K_t = test_comp * (test_grad ? 3 : 1) rows, K_u likewise.
 * The coupling at every quadrature point is
 *   W0                                   [K_t][K_u]   (material NONE), or
 *   P_test M(c, q) P_trial^T             (material TENSOR_QP),
 * with P_test [K_t][n_a], P_trial [K_u][n_b] and the per-point material
 * matrix M read as material[cell][point][n_a][n_b] (mat_transpose = 0) or
 * [n_b][n_a] (1), 1 <= n_a, n_b <= 9.  HOST arrays, copied at creation.
 * Outputs: MATRIX [n_cells][test_comp n_basis][trial_comp n_basis];
 * RESIDUAL [n_cells][test_comp][n_basis] with DOFs [n_nodes][trial_comp];
 * EVAL [n_cells], the test bound to the same DOFs (test_comp == trial_comp
 * and test_grad == trial_grad). */
typedef struct {
    int test_grad, test_comp, trial_grad, trial_comp;
    const double *W0;
    const double *P_test;
    const double *P_trial;
    int n_a, n_b;
    int mat_transpose;
} fe_bilinear;

/* Plan of the generic bilinear kernel: hex orders 1-3 and tets 1-2, FP64 or
 * FP32, material_kind NONE (W0) or TENSOR_QP (P_test, P_trial).  Evaluated
 * by fe_execute like any plan (workspace: fe_plan_workspace_size). */
int fe_plan_create_bilinear(int cell, int order, int mode, int precision, int material_kind,
                            const fe_bilinear *desc, const fe_options *opts, fe_plan *out);

/* Plan facts: n_basis, n_qp, n_comp (1 or 3), the chosen variant and the
 * element matrix/vector row count n_comp*n_basis.  Any pointer may be NULL. */
int fe_plan_info(fe_plan plan, int *n_basis, int *n_qp, int *n_comp,
                 int *variant, int *n_dof);

/* Bytes of device workspace fe_execute needs for n_cells cells.  The
 * workspace holds the sticky fault bits (first 256 bytes); it must be
 * zero-filled once before first use and is cleared by fe_plan_check.  The
 * MATRIX_FIRST residual variant also keeps one chunk of element matrices
 * there (chunk * n_dof^2 entries). */
int fe_plan_workspace_size(fe_plan plan, int64_t n_cells, size_t *bytes);

/* Evaluate the plan's form on n_cells cells.
 *   coords [n_nodes][3] FP64        node coordinates
 *   conn   [n_cells][n_basis] int32 local-to-global node numbers
 *   material                        layout by the plan's material kind, or NULL
 *   dofs   [n_nodes][n_comp]        RESIDUAL/EVAL, and MATRIX of CONVECT (the
 *                                    state of the derivative); NULL otherwise
 *   out    MATRIX   [n_cells][n_dof][n_dof]
 *          RESIDUAL [n_cells][n_comp][n_basis]
 *          EVAL     [n_cells]
 * Element types follow the plan's precision (FP64 or FP32); coords are FP64
 * always.  All pointers are device pointers.  Asynchronous on `stream`. */
int fe_execute(fe_plan plan, int64_t n_cells, int64_t n_nodes,
               const double *coords, const int32_t *conn, const void *material,
               const void *dofs, void *out, void *workspace,
               size_t workspace_bytes, void *stream);

/* fe_execute for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same validation, kernels and outputs, but no workspace argument.  The fault
 * bits and the matrix-first chunk of element matrices live in a static
 * device array of 64 MiB that the library holds on every device it runs on
 * until the process ends; the call allocates nothing.
 *   fault_out: device pointer to one unsigned, or NULL; receives this call's
 *     fault bits (1 = det J <= 0, 2 = node index out of range), cleared at
 *     the start of the call.
 * A call whose workspace would exceed 64 MiB (a matrix-first plan whose
 * chunk of element matrices is larger) returns FE_ERR_INVALID_ARG and
 * enqueues nothing.  Every call on a device shares that device's array:
 * calls that overlap on one GPU (different streams, different host threads)
 * race on it.  Asynchronous on `stream`. */
int fe_execute_noalloc(fe_plan plan, int64_t n_cells, int64_t n_nodes,
                       const double *coords, const int32_t *conn,
                       const void *material, const void *dofs, void *out,
                       unsigned *fault_out, void *stream);

/* The eval mode summed over the cells: the library evaluates the per-cell
 * values u_e^T K_e u_e into cell_values [n_cells] (device, plan precision)
 * and adds them in a fixed order, in FP64, into total [1] (device, FP64) --
 * the integral value of the eval mode over the whole mesh (section
 * "Overview" of the transpiler: 'eval' returns the integral).  The plan
 * must be an EVAL plan; other arguments as fe_execute.  Asynchronous. */
int fe_eval_sum(fe_plan plan, int64_t n_cells, int64_t n_nodes, const double *coords, const int32_t *conn,
                const void *material, const void *dofs, void *cell_values, double *total, void *workspace,
                size_t workspace_bytes, void *stream);

/* Synchronise `stream`, read and clear the workspace fault bits.  Returns
 * FE_ERR_INDEX_OUT_OF_RANGE or FE_ERR_NONPOSITIVE_JACOBIAN if a kernel saw
 * one since the last check, FE_OK otherwise. */
int fe_plan_check(fe_plan plan, void *workspace, void *stream);

int fe_plan_destroy(fe_plan plan);

/* ---- node incidence, assembly and the adjoint of the eval mode ---------- */

typedef struct fe_incidence_s *fe_incidence;

/* Node-to-(cell, local node) incidence of a connectivity, in CSR form, built
 * on the current device (the gather step behind assembly and the coordinate
 * gradient).  Entries of each node are sorted by cell*n_basis + a, so every
 * sum over them has a fixed order and the results are bitwise repeatable.
 *   conn [n_cells][n_basis] int32, device; entries must lie in [0, n_nodes)
 *   (FE_ERR_INDEX_OUT_OF_RANGE otherwise).  Synchronises `stream`.  The
 *   handle owns its device arrays (allocated here, freed by
 *   fe_incidence_destroy). */
int fe_incidence_create(int64_t n_cells, int64_t n_nodes, int n_basis, const int32_t *conn,
                        void *stream, fe_incidence *out);
int fe_incidence_destroy(fe_incidence inc);

/* Assembly of per-cell vectors into nodal ones (the global residual the
 * paper leaves out of its timings, Algorithm "feloopv" returns the cell
 * parts):  out[n][c] = scale * sum over (e,a) with conn[e][a] = n of
 * cell_vec[e][c][a].
 *   cell_vec [n_cells][n_comp][n_basis], out [n_nodes][n_comp], both device,
 *   FP64 when precision == FE_PREC_FP64, FP32 otherwise; out is
 *   overwritten.  Asynchronous. */
int fe_assemble(fe_incidence inc, int n_comp, int precision, const void *cell_vec, double scale,
                void *out, void *stream);

/* Sparsity pattern of the global matrix of a connectivity (the matrix
 * assembly that follows the element loops): row node n couples to every node
 * m that shares a cell with n.  CSR over nodes with sorted column node
 * numbers, built on the current device from the cells' (n, m) node pairs by
 * a radix sort.
 *   conn [n_cells][n_basis] int32, device, entries in [0, n_nodes)
 *   (FE_ERR_INDEX_OUT_OF_RANGE otherwise), no node listed twice by one cell
 *   (FE_ERR_INVALID_ARG otherwise); n_cells * n_basis^2 pairs and the
 *   number of distinct pairs must stay below 2^31 (FE_ERR_INVALID_ARG).
 * Synchronises `stream`; the handle owns its device arrays. */
typedef struct fe_pattern_s *fe_pattern;
int fe_pattern_create(int64_t n_cells, int64_t n_nodes, int n_basis, const int32_t *conn, void *stream,
                      fe_pattern *out);
/* n_nodes and the number of stored node pairs nnz; either may be NULL. */
int fe_pattern_info(fe_pattern pat, int64_t *n_nodes, int64_t *nnz);
/* Copy the pattern into caller-owned device arrays row_ptr [n_nodes + 1] and
 * cols [nnz] (int32).  Asynchronous on `stream`. */
int fe_pattern_copy(fe_pattern pat, int32_t *row_ptr, int32_t *cols, void *stream);
int fe_pattern_destroy(fe_pattern pat);

/* Assembly of element matrices into the block-CSR global matrix of a pattern
 * (blocks n_comp x n_comp, global unknown (n, c) = node n, component c, as
 * the DOF array [n_nodes][n_comp]):
 *   values[k][c][d] = scale * sum over (e, a, b) with conn[e][a] = n,
 *                     conn[e][b] = m of K_e[c*n_basis + a][d*n_basis + b]
 * for the pattern entry k of (n, m).  cell_mats [n_cells][n_comp n_basis]^2
 * (component-major rows, the layout of the matrix mode) and values [nnz]
 * [n_comp][n_comp] are device arrays, FP64 when precision == FE_PREC_FP64,
 * FP32 otherwise; values is overwritten.  inc must be the incidence of the
 * same connectivity.  One thread sums each row node over its incidence list
 * in order, so results are bitwise repeatable.  Asynchronous. */
int fe_assemble_matrix(fe_pattern pat, fe_incidence inc, const int32_t *conn, int n_comp, int precision,
                       const void *cell_mats, double scale, void *values, void *stream);

/* Gradient of the eval-mode value of linear elasticity,
 *   J(c, x) = sum_e u_e^T K_e(c, x) u_e
 * (eval mode of the elasticity form; the derivative rules below follow from
 * differentiating the quadrature sum, as the paper differentiates forms with
 * respect to the DOFs), with respect to the material coefficients and the
 * node coordinates, recomputing the geometry (nothing is stored between the
 * forward and the backward pass):
 *   dJ/dlambda_{e,q} = w det J (tr eps)^2,   dJ/dmu_{e,q} = 2 w det J eps:eps,
 *   dJ/dx_n = sum_{(e,a): conn[e][a]=n} sum_q w det J
 *             sum_l (W delta_kl - 2 (H^T sigma)_kl) dphi_a/dx_l
 *   with H = grad u, sigma = lambda tr(eps) I + 2 mu eps, W = eps:sigma.
 * The plan must be ELASTICITY / EVAL with material ISO_QP or ISO_CELL.
 *   grad_material: [n_cells][n_qp][2] (ISO_QP) or [n_cells][2] (ISO_CELL),
 *                  plan precision, overwritten, or NULL;
 *   grad_coords:   [n_nodes][3] FP64, overwritten, or NULL (needs inc);
 *   scale multiplies both (the incoming gradient of a scalar loss).
 * The workspace must hold fe_energy_grad_workspace_size() bytes, the first
 * 256 of which are the fault bits of fe_plan_check.  Asynchronous. */
int fe_energy_grad_workspace_size(fe_plan plan, int64_t n_cells, size_t *bytes);
int fe_energy_grad(fe_plan plan, fe_incidence inc, int64_t n_cells, int64_t n_nodes, const double *coords,
                   const int32_t *conn, const void *material, const void *dofs, double scale,
                   void *grad_material, double *grad_coords, void *workspace, size_t workspace_bytes,
                   void *stream);

/* ---- batched evaluation of uneven groups in one persistent launch ------- */

/* One group of cells of a single kind and order with its own mesh arrays and
 * outputs (device pointers, caller-owned).  The paper's single-einsum
 * evaluation needs rectangular operands and so one call per cell kind and
 * order (grouping of mixed meshes is left open in its introduction); a batch
 * evaluates all groups and all their forms in one kernel launch.
 *   forms: bit mask of (1 << FE_FORM_MASS), (1 << FE_FORM_LAPLACE),
 *          (1 << FE_FORM_ELASTICITY); all of a group's forms share one
 *          geometry evaluation per cell;
 *   tile:  cells per work item, 0 = default (tuned when autotune is on);
 *          rounded up to a multiple of the group's pass (cells evaluated
 *          together: 256 for P1 tets, 8 for P2 tets, 16 for FP32 and 8 for
 *          FP64 Q1 hexahedra, 1 for Q2); the default is four passes;
 *   material: [n_cells][2] (lambda, mu) when ELASTICITY is requested;
 *   out_mass, out_laplace: [n_cells][n_basis][n_basis];
 *   out_elasticity: [n_cells][3 n_basis][3 n_basis] (16-byte aligned);
 *   a group with n_cells == 0 takes no work item and its arrays may be NULL;
 *   a group with cells needs n_nodes > 0 (FE_ERR_INVALID_ARG otherwise). */
typedef struct {
    int cell, order;
    int forms;
    int tile;
    int64_t n_cells, n_nodes;
    const double *coords;
    const int32_t *conn;
    const void *material;
    void *out_mass;
    void *out_laplace;
    void *out_elasticity;
} fe_group;

typedef struct fe_batch_s *fe_batch;

/* Build a batch of 1..16 groups (Q1/Q2 hexahedra, P1/P2 tetrahedra) in FP64
 * or FP32 on the current device: copies the group descriptions and the
 * reference tables to the device and captures the launch (a counter reset
 * and one persistent kernel that pulls (group, tile) work items) in a HIP
 * graph.  With autotune != 0 it then times the graph over tile candidates of
 * each group and keeps the fastest (this runs the batch, writing the
 * outputs).  Synchronous.  Errors: FE_ERR_INVALID_ARG, FE_ERR_UNSUPPORTED. */
int fe_batch_create(int n_groups, const fe_group *groups, int precision, int autotune, fe_batch *out);
/* Launch the captured graph on `stream` (asynchronous, allocates nothing).
 * The batch owns one work counter: executions of the same batch must not
 * overlap (enqueue them on one stream, or synchronise between streams);
 * different batches are independent. */
int fe_batch_execute(fe_batch b, void *stream);
/* Synchronise and report det J <= 0 / out-of-range node faults (then clear). */
int fe_batch_check(fe_batch b, void *stream);
/* Chosen tile per group (caller's order), the best tuned time in ms and the
 * persistent grid size.  Any pointer may be NULL. */
int fe_batch_tiles(fe_batch b, int *tiles, float *tune_ms, int *grid);
int fe_batch_destroy(fe_batch b);

#ifdef __cplusplus
}
#endif
#endif /* FE_FORMS_H */
