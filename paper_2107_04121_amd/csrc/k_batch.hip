// Batched evaluation of uneven cell groups in ONE persistent launch.
//
// The paper's einsum calls need rectangular operands, so a mesh with several
// cell kinds or orders takes one call per group, and grouping/sorting of
// mixed meshes is left open.  Here every group (cell kind, order, set of
// forms, its own mesh arrays and outputs) is cut into work items of `tile`
// cells; one persistent kernel pulls items from a device counter and runs
// the routine of the item's group.  All forms of a group share one geometry
// evaluation per cell:
//   - Q2 hexahedra: the matrix-core cell routine (elasticity GEMM P = G^T W G,
//     Laplace = P_00 + P_11 + P_22, mass on the matrix cores);
//   - P1/P2 tetrahedra and Q1 hexahedra: a fused VALU tile routine computing
//     the six blocks r <= s of P, the mass matrix, then all outputs.
// The counter reset and the kernel are captured once in a HIP graph; running
// the batch is one graph launch.  Tiles per group are tuned by timing the
// graph over a small candidate set.
#include <algorithm>
#include <vector>

#include "q2_device.h"

namespace fe {

enum { MAX_GROUPS = 16, FORM_BIT_MASS = 1, FORM_BIT_LAPLACE = 4, FORM_BIT_ELAST = 8 };

struct GroupDev {
    int cell, order, forms, tile;
    int64_t n_cells, n_nodes, item0, n_items;
    const double *coords;
    const int32_t *conn;
    const void *mat;
    void *out_mass, *out_lap, *out_el;
    DevTables tab;
};

struct BatchDev {
    int n_groups;
    int64_t n_items;
    GroupDev g[MAX_GROUPS];
};

namespace {

using namespace q2;

// Fused tile for small cells (any cell kind/order with NB <= 27): E cells per
// pass; mass, Laplace and isotropic elasticity element matrices from one
// geometry evaluation (FP64) and the six blocks P_rs = G_r^T W G_s, r <= s.
template <int CELL, int P, typename T>
struct Fused {
    static constexpr int NB = cell_nb(CELL, P), NQ = cell_nq(CELL, P), ND = 3 * NB;
    static constexpr int PER = NB * 3 * 8 + NQ * 3 * NB * (int)sizeof(T) + NQ * (int)sizeof(T) +
                               7 * NB * NB * (int)sizeof(T) + 2 * (int)sizeof(T);
    static constexpr int choose(int cap)
    {
        int e = 256 / (NQ > NB ? NQ : NB);
        if (e < 1) e = 1;
        while (e > 1 && e * PER > cap) e--;
        return e;
    }
    static constexpr int E = choose(48 * 1024);
    static constexpr int BYTES = E * PER;
};

template <int CELL, int P, typename T>
__device__ void fused_tile(const GroupDev &g, int64_t c0, int64_t c1, unsigned *flags, unsigned char *smem)
{
    using F = Fused<CELL, P, T>;
    constexpr int NB = F::NB, NQ = F::NQ, ND = F::ND, E = F::E, NN = NB * NB;
    double *xs = reinterpret_cast<double *>(smem);  // [E][NB][3]
    T *Gs = reinterpret_cast<T *>(xs + E * NB * 3);   // [E][NQ][3][NB]
    T *wd = Gs + E * NQ * 3 * NB;                     // [E][NQ]
    T *Ps = wd + E * NQ;                              // [E][7][NB][NB]: 6 blocks r <= s, then mass
    T *lm = Ps + E * 7 * NN;                          // [E][2]
    const int tid = threadIdx.x;
    const T *mat = static_cast<const T *>(g.mat);
    const bool want_el = g.forms & FORM_BIT_ELAST;

    for (int64_t e0 = c0; e0 < c1; e0 += E) {
        const int ne = static_cast<int>(c1 - e0 < E ? c1 - e0 : E);
        for (int i = tid; i < ne * NB; i += 256) {
            const int el = i / NB, a = i - el * NB;
            const int64_t n = checked_node(g.conn, (e0 + el) * NB + a, g.n_nodes, flags);
            xs[i * 3 + 0] = g.coords[3 * n];
            xs[i * 3 + 1] = g.coords[3 * n + 1];
            xs[i * 3 + 2] = g.coords[3 * n + 2];
        }
        if (want_el)
            for (int i = tid; i < ne * 2; i += 256) lm[i] = mat[2 * e0 + i];
        __syncthreads();
        for (int i = tid; i < ne * NQ; i += 256) {
            const int el = i / NQ, q = i - el * NQ;
            double J[3][3], Ji[3][3];
            jacobian_qp<NB, NQ>(xs + el * NB * 3, g.tab.bfgT, q, J);
            const double det = inverse3(J, Ji);
            if (!(det > 0.0)) raise_fault(flags, FAULT_DET);
            wd[i] = static_cast<T>(g.tab.w[q] * det);
            T *gq = Gs + i * 3 * NB;
            for (int a = 0; a < NB; a++) {
                const double r0 = g.tab.bfgT[(a * 3 + 0) * NQ + q];
                const double r1 = g.tab.bfgT[(a * 3 + 1) * NQ + q];
                const double r2 = g.tab.bfgT[(a * 3 + 2) * NQ + q];
#pragma unroll
                for (int d = 0; d < 3; d++) gq[d * NB + a] = static_cast<T>(r0 * Ji[0][d] + r1 * Ji[1][d] + r2 * Ji[2][d]);
            }
        }
        __syncthreads();
        // P_rs[a][b] = sum_q wd G_r[a] G_s[b] (6 blocks r <= s), block 6 = mass
        for (int i = tid; i < ne * 7 * NN; i += 256) {
            const int el = i / (7 * NN), rem = i - el * 7 * NN, blk = rem / NN, ab = rem - blk * NN;
            const int a = ab / NB, b = ab - a * NB;
            T s = T(0);
            if (blk == 6) {
                for (int q = 0; q < NQ; q++)
                    s += wd[el * NQ + q] * static_cast<T>(g.tab.bf[q * NB + a]) * static_cast<T>(g.tab.bf[q * NB + b]);
            } else {
                const int r = blk < 3 ? 0 : (blk < 5 ? 1 : 2);
                const int sc = blk < 3 ? blk : (blk < 5 ? blk - 2 : 2);
                for (int q = 0; q < NQ; q++) {
                    const T *gq = Gs + (el * NQ + q) * 3 * NB;
                    s += wd[el * NQ + q] * gq[r * NB + a] * gq[sc * NB + b];
                }
            }
            Ps[i] = s;
        }
        __syncthreads();
        // outputs, consecutive threads on consecutive entries of each cell
        if (g.forms & FORM_BIT_MASS) {
            T *om = static_cast<T *>(g.out_mass) + e0 * NN;
            for (int i = tid; i < ne * NN; i += 256) {
                const int el = i / NN, ab = i - el * NN;
                om[i] = Ps[(el * 7 + 6) * NN + ab];
            }
        }
        if (g.forms & FORM_BIT_LAPLACE) {
            T *ol = static_cast<T *>(g.out_lap) + e0 * NN;
            for (int i = tid; i < ne * NN; i += 256) {
                const int el = i / NN, ab = i - el * NN;
                const T *pe = Ps + el * 7 * NN;
                ol[i] = pe[0 * NN + ab] + pe[3 * NN + ab] + pe[5 * NN + ab];
            }
        }
        if (want_el) {
            T *oe = static_cast<T *>(g.out_el) + e0 * ND * ND;
            for (int i = tid; i < ne * ND * ND; i += 256) {
                const int el = i / (ND * ND), rem = i - el * ND * ND, row = rem / ND, col = rem - row * ND;
                const int r = row / NB, a = row - r * NB, s = col / NB, b = col - s * NB;
                const T *pe = Ps + el * 7 * NN;
                const int lo = r < s ? r : s, hi = r < s ? s : r;
                const int blk = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
                // P(r,s)[a][b] is stored for r <= s; P(s,r) = P(r,s)^T
                const T pab = r <= s ? pe[blk * NN + a * NB + b] : pe[blk * NN + b * NB + a];
                const T pba = r <= s ? pe[blk * NN + b * NB + a] : pe[blk * NN + a * NB + b];
                const T lam = lm[el * 2], mu = lm[el * 2 + 1];
                T v = lam * pab + mu * pba;
                if (r == s) v += mu * (pe[0 * NN + a * NB + b] + pe[3 * NN + a * NB + b] + pe[5 * NN + a * NB + b]);
                oe[i] = v;
            }
        }
        __syncthreads();
    }
}

template <typename T>
struct BatchLds {
    static constexpr int MM = sizeof(T) == 8 ? MM_F64 : MM_F32;
    static constexpr int v0 = Q2Layout<MM>::BYTES;
    static constexpr int v1 = Fused<FE_CELL_TET, 1, T>::BYTES;
    static constexpr int v2 = Fused<FE_CELL_TET, 2, T>::BYTES;
    static constexpr int v3 = Fused<FE_CELL_HEX, 1, T>::BYTES;
    static constexpr int m01 = v0 > v1 ? v0 : v1, m23 = v2 > v3 ? v2 : v3;
    static constexpr int BYTES = m01 > m23 ? m01 : m23;
};

__global__ void k_batch_reset(unsigned long long *ctr) { ctr[0] = 0ULL; }

template <typename T>
__global__ __launch_bounds__(256, 3) void k_batch(const BatchDev *B, unsigned long long *ctr, unsigned *flags)
{
    __shared__ __align__(16) unsigned char smem[BatchLds<T>::BYTES];
    __shared__ long long s_item;
    constexpr int MM = BatchLds<T>::MM;
    const int64_t n_items = B->n_items;
    const int ng = B->n_groups;
    for (;;) {
        if (threadIdx.x == 0) s_item = static_cast<long long>(atomicAdd(ctr, 1ULL));
        __syncthreads();
        const int64_t it = s_item;
        __syncthreads();
        if (it >= n_items) break;  // every workgroup leaves once the queue is drained
        int gi = 0;
        while (gi + 1 < ng && it >= B->g[gi + 1].item0) gi++;
        const GroupDev &g = B->g[gi];
        const int64_t c0 = (it - g.item0) * g.tile;
        const int64_t c1 = c0 + g.tile < g.n_cells ? c0 + g.tile : g.n_cells;
        if (g.cell == FE_CELL_HEX && g.order == 2) {
            const Q2Job job{g.n_cells, g.n_nodes, g.coords, g.conn, g.mat, g.out_el, g.out_mass, g.out_lap, flags, g.tab};
            q2_run<MM, true>(job, c0, c1, 1, smem);
        } else if (g.cell == FE_CELL_HEX && g.order == 1) {
            fused_tile<FE_CELL_HEX, 1, T>(g, c0, c1, flags, smem);
        } else if (g.cell == FE_CELL_TET && g.order == 1) {
            fused_tile<FE_CELL_TET, 1, T>(g, c0, c1, flags, smem);
        } else if (g.cell == FE_CELL_TET && g.order == 2) {
            fused_tile<FE_CELL_TET, 2, T>(g, c0, c1, flags, smem);
        }
    }
}

int group_pass_cells(int cell, int order, bool f64)
{
    if (cell == FE_CELL_HEX && order == 2) return 1;
    if (f64) {
        if (cell == FE_CELL_HEX) return Fused<FE_CELL_HEX, 1, double>::E;
        return order == 1 ? Fused<FE_CELL_TET, 1, double>::E : Fused<FE_CELL_TET, 2, double>::E;
    }
    if (cell == FE_CELL_HEX) return Fused<FE_CELL_HEX, 1, float>::E;
    return order == 1 ? Fused<FE_CELL_TET, 1, float>::E : Fused<FE_CELL_TET, 2, float>::E;
}

}  // namespace
}  // namespace fe

using namespace fe;

struct fe_batch_s {
    int device = -1, prec = 0, n_groups = 0;
    int orig[fe::MAX_GROUPS] = {};  // caller index of sorted group k
    BatchDev host{};
    BatchDev *dev = nullptr;
    unsigned long long *ctr = nullptr;
    unsigned *flags = nullptr;
    double *tables = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int grid = 0;
    float tune_ms = 0.0f;
};

namespace fe {
void batch_destroy(fe_batch_s *b);
namespace {

void assign_items(BatchDev &b)
{
    int64_t acc = 0;
    for (int i = 0; i < b.n_groups; i++) {
        GroupDev &g = b.g[i];
        g.item0 = acc;
        g.n_items = (g.n_cells + g.tile - 1) / g.tile;
        acc += g.n_items;
    }
    b.n_items = acc;
}

int upload(fe_batch_s *b)
{
    assign_items(b->host);
    FE_HIP_CHECK(hipMemcpy(b->dev, &b->host, sizeof(BatchDev), hipMemcpyHostToDevice));
    return FE_OK;
}

int time_graph(fe_batch_s *b, int reps, float *ms)
{
    hipEvent_t t0, t1;
    FE_HIP_CHECK(hipEventCreate(&t0));
    FE_HIP_CHECK(hipEventCreate(&t1));
    FE_HIP_CHECK(hipGraphLaunch(b->exec, b->cap));  // warm-up
    float best = 1e30f;
    for (int r = 0; r < reps; r++) {
        FE_HIP_CHECK(hipEventRecord(t0, b->cap));
        FE_HIP_CHECK(hipGraphLaunch(b->exec, b->cap));
        FE_HIP_CHECK(hipEventRecord(t1, b->cap));
        FE_HIP_CHECK(hipEventSynchronize(t1));
        float m = 0.0f;
        FE_HIP_CHECK(hipEventElapsedTime(&m, t0, t1));
        best = m < best ? m : best;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    *ms = best;
    return FE_OK;
}

}  // namespace

int batch_create(int n_groups, const fe_group *groups, int precision, int autotune, fe_batch_s **out)
{
    *out = nullptr;
    if (n_groups < 1 || n_groups > MAX_GROUPS || !groups) {
        set_error("1..16 groups required");
        return FE_ERR_INVALID_ARG;
    }
    if (precision != FE_PREC_FP64 && precision != FE_PREC_FP32) {
        set_error("batches run in FP64 or FP32");
        return FE_ERR_UNSUPPORTED;
    }
    const bool f64 = precision == FE_PREC_FP64;
    std::vector<int> order(n_groups);
    for (int i = 0; i < n_groups; i++) {
        const fe_group &g = groups[i];
        const bool ok_cell = (g.cell == FE_CELL_HEX && (g.order == 1 || g.order == 2)) ||
                             (g.cell == FE_CELL_TET && (g.order == 1 || g.order == 2));
        if (!ok_cell) {
            set_error("batch groups support Q1/Q2 hexahedra and P1/P2 tetrahedra");
            return FE_ERR_UNSUPPORTED;
        }
        const int bad_forms = g.forms & ~((1 << FE_FORM_MASS) | (1 << FE_FORM_LAPLACE) | (1 << FE_FORM_ELASTICITY));
        if (!g.forms || bad_forms || g.n_cells < 0 || g.n_nodes < 0 || (g.n_cells > 0 && (!g.coords || !g.conn)) ||
            ((g.forms & (1 << FE_FORM_MASS)) && !g.out_mass) || ((g.forms & (1 << FE_FORM_LAPLACE)) && !g.out_laplace) ||
            ((g.forms & (1 << FE_FORM_ELASTICITY)) && (!g.out_elasticity || !g.material)) || g.tile < 0) {
            set_error("bad group description");
            return FE_ERR_INVALID_ARG;
        }
        if (g.cell == FE_CELL_HEX && g.order == 2 && reinterpret_cast<uintptr_t>(g.out_elasticity) % 16) {
            set_error("Q2 elasticity output must be 16-byte aligned");
            return FE_ERR_INVALID_ARG;
        }
        order[i] = i;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        set_error("no HIP device");
        return FE_ERR_NO_DEVICE;
    }
    // heaviest cells first, so the tail of the queue holds the small items
    auto weight = [&](int i) { return groups[i].cell == FE_CELL_HEX ? groups[i].order * 4 : groups[i].order; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return weight(x) > weight(y); });

    fe_batch_s *b = new (std::nothrow) fe_batch_s();
    if (!b) return FE_ERR_OUT_OF_MEMORY;
    b->device = dev;
    b->prec = precision;
    b->n_groups = n_groups;
    b->host.n_groups = n_groups;
    // reference tables of every group, laid out like a plan's
    std::vector<double> tab;
    std::vector<size_t> toff(n_groups);
    for (int k = 0; k < n_groups; k++) {
        const fe_group &g = groups[order[k]];
        RefTables R;
        reference_tables(g.cell, g.order, R);
        toff[k] = tab.size();
        const int nq = R.nq, nb = R.nb, n1 = g.cell == FE_CELL_HEX ? (g.order + 1) * (g.order + 1) : 0;
        const size_t base = tab.size();
        tab.resize(base + nq + (size_t)nq * nb + (size_t)nb * 3 * nq + 2 * n1, 0.0);
        double *w = tab.data() + base, *bf = w + nq, *bfgT = bf + (size_t)nq * nb, *B1 = bfgT + (size_t)nb * 3 * nq,
               *D1 = B1 + n1;
        for (int q = 0; q < nq; q++) {
            w[q] = R.w[q];
            for (int a = 0; a < nb; a++) {
                bf[(size_t)q * nb + a] = R.bf[(size_t)q * nb + a];
                for (int j = 0; j < 3; j++) bfgT[((size_t)a * 3 + j) * nq + q] = R.bfg[((size_t)q * 3 + j) * nb + a];
            }
        }
        for (int i = 0; i < n1; i++) {
            B1[i] = R.B1[i];
            D1[i] = R.D1[i];
        }
    }
    auto fail_free = [&](int st, const char *msg) {
        set_error(msg);
        (void)hipGetLastError();
        batch_destroy(b);
        return st;
    };
    if (hipMalloc(&b->tables, tab.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&b->dev, sizeof(BatchDev)) != hipSuccess || hipMalloc(&b->ctr, 256) != hipSuccess ||
        hipMalloc(&b->flags, 256) != hipSuccess)
        return fail_free(FE_ERR_OUT_OF_MEMORY, "batch allocation failed");
    if (hipMemcpy(b->tables, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->flags, 0, 256) != hipSuccess || hipMemset(b->ctr, 0, 256) != hipSuccess)
        return fail_free(FE_ERR_HIP, "batch upload failed");
    for (int k = 0; k < n_groups; k++) {
        const fe_group &s = groups[order[k]];
        b->orig[k] = order[k];
        GroupDev &g = b->host.g[k];
        g.cell = s.cell;
        g.order = s.order;
        g.forms = (s.forms & (1 << FE_FORM_MASS) ? FORM_BIT_MASS : 0) |
                  (s.forms & (1 << FE_FORM_LAPLACE) ? FORM_BIT_LAPLACE : 0) |
                  (s.forms & (1 << FE_FORM_ELASTICITY) ? FORM_BIT_ELAST : 0);
        const int pass = group_pass_cells(s.cell, s.order, f64);
        g.tile = s.tile > 0 ? ((s.tile + pass - 1) / pass) * pass : pass * 4;
        g.n_cells = s.n_cells;
        g.n_nodes = s.n_nodes;
        g.coords = s.coords;
        g.conn = s.conn;
        g.mat = s.material;
        g.out_mass = s.out_mass;
        g.out_lap = s.out_laplace;
        g.out_el = s.out_elasticity;
        const int nq = (s.order + 1) * (s.order + 1) * (s.order + 1);
        const int nb = s.cell == FE_CELL_HEX ? nq : (s.order == 1 ? 4 : 10);
        const int n1 = s.cell == FE_CELL_HEX ? (s.order + 1) * (s.order + 1) : 0;
        const double *w = b->tables + toff[k];
        g.tab.w = w;
        g.tab.bf = w + nq;
        g.tab.bfgT = w + nq + (size_t)nq * nb;
        g.tab.B1 = g.tab.bfgT + (size_t)nb * 3 * nq;
        g.tab.D1 = g.tab.B1 + n1;
    }
    if (upload(b)) return fail_free(FE_ERR_HIP, "batch upload failed");
    // persistent grid
    int per_cu = 0, cus = 0;
    const void *kfn = f64 ? reinterpret_cast<const void *>(k_batch<double>) : reinterpret_cast<const void *>(k_batch<float>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail_free(FE_ERR_HIP, "occupancy query failed");
    b->grid = per_cu * cus > 0 ? per_cu * cus : 256;
    // capture: counter reset (a kernel, not a memset) + the persistent kernel
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return fail_free(FE_ERR_HIP, "stream creation failed");
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail_free(FE_ERR_HIP, "capture failed");
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, b->cap, b->ctr);
    if (f64)
        hipLaunchKernelGGL(k_batch<double>, dim3(b->grid), dim3(256), 0, b->cap, b->dev, b->ctr, b->flags);
    else
        hipLaunchKernelGGL(k_batch<float>, dim3(b->grid), dim3(256), 0, b->cap, b->dev, b->ctr, b->flags);
    if (hipStreamEndCapture(b->cap, &b->graph) != hipSuccess ||
        hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail_free(FE_ERR_HIP, "graph instantiation failed");
    // tile tuning: per group, coordinate-wise over multiples of its pass size
    if (autotune) {
        float best = 0.0f;
        if (time_graph(b, 3, &best)) return fail_free(FE_ERR_HIP, "tuning launch failed");
        for (int k = 0; k < n_groups; k++) {
            GroupDev &g = b->host.g[k];
            if (g.n_cells == 0) continue;
            const int pass = group_pass_cells(g.cell, g.order, f64);
            const int keep = g.tile;
            int best_tile = keep;
            for (int m : {1, 2, 4, 8, 16}) {
                const int t = pass * m;
                if (t == keep) continue;
                g.tile = t;
                float ms = 0.0f;
                if (upload(b) || time_graph(b, 3, &ms)) return fail_free(FE_ERR_HIP, "tuning launch failed");
                if (ms < best) {
                    best = ms;
                    best_tile = t;
                }
            }
            g.tile = best_tile;
            if (upload(b)) return fail_free(FE_ERR_HIP, "batch upload failed");
        }
        b->tune_ms = best;
    }
    unsigned hflags = 0;
    if (hipStreamSynchronize(b->cap) != hipSuccess ||
        hipMemcpy(&hflags, b->flags, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
        return fail_free(FE_ERR_HIP, "batch setup failed");
    *out = b;
    return FE_OK;
}

int batch_execute(fe_batch_s *b, hipStream_t st)
{
    FE_HIP_CHECK(hipGraphLaunch(b->exec, st));
    return FE_OK;
}

int batch_check(fe_batch_s *b, hipStream_t st)
{
    unsigned flags = 0;
    FE_HIP_CHECK(hipStreamSynchronize(st));
    FE_HIP_CHECK(hipStreamSynchronize(b->cap));
    FE_HIP_CHECK(hipMemcpy(&flags, b->flags, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (flags) FE_HIP_CHECK(hipMemset(b->flags, 0, sizeof(unsigned)));
    if (flags & FAULT_INDEX) {
        set_error("a connectivity entry is out of range");
        return FE_ERR_INDEX_OUT_OF_RANGE;
    }
    if (flags & FAULT_DET) {
        set_error("det J <= 0 at a quadrature point");
        return FE_ERR_NONPOSITIVE_JACOBIAN;
    }
    return FE_OK;
}

int batch_info(fe_batch_s *b, int *tiles, float *tune_ms, int *grid)
{
    if (tiles)
        for (int k = 0; k < b->n_groups; k++) tiles[b->orig[k]] = b->host.g[k].tile;
    if (tune_ms) *tune_ms = b->tune_ms;
    if (grid) *grid = b->grid;
    return FE_OK;
}

void batch_destroy(fe_batch_s *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->tables) (void)hipFree(b->tables);
    if (b->dev) (void)hipFree(b->dev);
    if (b->ctr) (void)hipFree(b->ctr);
    if (b->flags) (void)hipFree(b->flags);
    delete b;
}

}  // namespace fe
