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
//   - P2 tetrahedra and Q1 hexahedra: the same product on the matrix cores
//     for several cells per pass (see SmallMM);
//   - P1 tetrahedra: one geometry per cell and the factored quadrature sums
//     (see AffineTet).
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

// Low-order cells (P2 tetrahedra, Q1 hexahedra) on the matrix cores, CPP
// cells per pass: every (cell, quadrature point) pair's FP64 geometry is
// evaluated once by one thread, G = dphi/dxi J^-1 goes to LDS in the
// contraction type, and each wave forms, for CPW cells,
//   P = G_s^T diag(w det J) G_s   (3nb x 3nb, G_s = [G_x G_y G_z])
//   M = Phi^T diag(w det J) Phi   (nb x nb, the scalar mass matrix)
// on 16x16 MFMA tiles.  All outputs are then read off P and M in LDS:
//   K[(r,a),(s,b)] = lambda P[(r,a),(s,b)] + mu P[(s,a),(r,b)]
//                    + delta_rs mu sum_j P[(j,a),(j,b)]   (isotropic elasticity)
//   L[a][b] = sum_j P[(j,a),(j,b)]                        (Laplace)
// and stored with consecutive threads on consecutive entries of the pass's
// contiguous cells.
template <int CELL, int P, typename T>
struct SmallMM {
    static constexpr int NB = cell_nb(CELL, P), NQ = cell_nq(CELL, P), ND = 3 * NB;
    static constexpr int NQP = (NQ + 3) / 4 * 4;  // quadrature axis padded to the MFMA depth
    static constexpr int KS = NQP + 1;            // odd row stride of the operand
    static constexpr int NT = ND > 16 ? 2 : 1;    // 16x16 tiles per side of P
    static constexpr int RP = 16 * NT;            // operand rows, padded
    // cells per wave: 4 for FP32 Q1 hexahedra (16 cells per pass, 128
    // geometry threads), 2 otherwise (the FP64 records would not fit next
    // to a second workgroup)
    static constexpr int CPW = NB > 4 && (sizeof(T) == 8 || NQ > 8) ? 2 : 4;
    static constexpr int CPP = 4 * CPW;                       // cells per pass
    static constexpr int PS = ND + 1, MS = NB + 1;            // LDS row strides of P, M
    static constexpr int XB = CPP * NB * 3;                                    // doubles per x buffer
    static constexpr int OFF_X = 0;                                            // double x[2][CPP][NB*3]
    static constexpr int OFF_LM = align16(OFF_X + 2 * XB * 8);                 // T lm[2][CPP][2]
    static constexpr int OFF_WD = align16(OFF_LM + 2 * CPP * 2 * (int)sizeof(T));  // double wd[CPP][NQP]
    // a cell's operand G[RP][KS] and its product P[ND][PS] share one record
    // of CR entries: only the wave that owns the cell reads G, and it has
    // read all of it (its MFMA operands) before it writes P
    static constexpr int CR = RP * KS > ND * PS ? RP * KS : ND * PS;
    static constexpr int OFF_G = align16(OFF_WD + CPP * NQP * 8);                // T G[CPP][CR]
    static constexpr int OFF_P = OFF_G;                                          // T P[CPP][CR]
    static constexpr int OFF_M = align16(OFF_P + CPP * CR * (int)sizeof(T));     // T M[CPP][NB][MS]
    // the group's reference tables, copied once per work item: without them
    // the geometry and the products waited on global loads, and a wave's
    // loads complete only after its earlier stores (the previous pass's
    // outputs)
    static constexpr int TAB = NB * 3 * NQ + NQ * NB + NQ;                      // bfgT, bf, w
    static constexpr int OFF_TAB = align16(OFF_M + CPP * NB * MS * (int)sizeof(T));  // double tab[TAB]
    static constexpr int BYTES = align16(OFF_TAB + TAB * 8);
};

template <typename T>
__device__ __forceinline__ void mma4(T a, T b, typename MMT<sizeof(T) == 8 ? MM_F64 : MM_F32>::acc &c)
{
    if constexpr (sizeof(T) == 8) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Node coordinates (and coefficients) of cells e0 .. e0+n-1 into x buffer xb.
template <int CELL, int P, typename T>
__device__ __forceinline__ unsigned small_gather(const GroupDev &g, int64_t e0, int n, double *xb, T *lmb, int tid)
{
    using L = SmallMM<CELL, P, T>;
    constexpr int NB = L::NB, CPP = L::CPP;
    unsigned fault = 0;
    for (int t = tid; t < CPP * NB; t += 256) {
        const int c = t / NB, a = t - c * NB;
        double x0 = 0.0, x1 = 0.0, x2 = 0.0;
        if (c < n) {
            int64_t nd = gmem(g.conn)[(e0 + c) * NB + a];
            if (nd < 0 || nd >= g.n_nodes) {
                fault |= FAULT_INDEX;
                nd = 0;
            }
            x0 = gmem(g.coords)[3 * nd];
            x1 = gmem(g.coords)[3 * nd + 1];
            x2 = gmem(g.coords)[3 * nd + 2];
        }
        xb[t * 3] = x0;
        xb[t * 3 + 1] = x1;
        xb[t * 3 + 2] = x2;
    }
    if ((g.forms & FORM_BIT_ELAST) && tid < 2 * CPP)
        lmb[tid] = tid < 2 * n ? gmem(static_cast<const T *>(g.mat))[2 * e0 + tid] : T(0);
    return fault;
}

// Cells e0 .. e0+n-1 (n <= CPP) of a low-order group, their coordinates
// already in x buffer `buf`.  When nn_next > 0 the next pass (cells en ..
// en+nn_next-1) is prefetched into the other buffer in two hops: its
// connectivity during the geometry, its coordinates during the products,
// both parked in LDS before this pass's stores, so no load waits for those
// stores to drain (vector memory counters complete in order).
template <int CELL, int P, typename T>
__device__ void small_pass(const GroupDev &g, int64_t e0, int n, int buf, int64_t en, int nn_next, unsigned *flags,
                           unsigned char *smem, int tid)
{
    using L = SmallMM<CELL, P, T>;
    using ACC = typename MMT<sizeof(T) == 8 ? MM_F64 : MM_F32>::acc;
    constexpr int NB = L::NB, NQ = L::NQ, ND = L::ND, NQP = L::NQP, KS = L::KS, NT = L::NT, RP = L::RP;
    constexpr int CPP = L::CPP, CPW = L::CPW, PS = L::PS, MS = L::MS;
    double *xs = reinterpret_cast<double *>(smem + L::OFF_X) + buf * L::XB;
    double *xn = reinterpret_cast<double *>(smem + L::OFF_X) + (buf ^ 1) * L::XB;
    T *lm = reinterpret_cast<T *>(smem + L::OFF_LM) + buf * 2 * CPP;
    T *lmn = reinterpret_cast<T *>(smem + L::OFF_LM) + (buf ^ 1) * 2 * CPP;
    double *wd = reinterpret_cast<double *>(smem + L::OFF_WD);
    T *Gs = reinterpret_cast<T *>(smem + L::OFF_G);
    T *Ps = reinterpret_cast<T *>(smem + L::OFF_P);
    T *Ms = reinterpret_cast<T *>(smem + L::OFF_M);
    const double *bfgT = reinterpret_cast<const double *>(smem + L::OFF_TAB);
    const double *bf = bfgT + NB * 3 * NQ, *wq = bf + NQ * NB;
    const bool want_el = g.forms & FORM_BIT_ELAST;
    unsigned fault = 0;

    // 1. operand padding: rows nd..RP-1 and columns NQ..NQP-1 of every
    //    cell's operand, weights of the padding points
    constexpr int ZR = (RP - ND) * KS, ZC = ND * (NQP - NQ);
    if constexpr (ZR + ZC > 0)
        for (int t = tid; t < CPP * (ZR + ZC); t += 256) {
            const int c = t / (ZR + ZC), u = t - c * (ZR + ZC);
            T *G = Gs + c * L::CR;
            if (u < ZR) G[ND * KS + u] = T(0);
            else if constexpr (ZC > 0) G[((u - ZR) / (NQP - NQ)) * KS + NQ + (u - ZR) % (NQP - NQ)] = T(0);
        }
    if constexpr (NQP > NQ)
        if (tid < CPP * (NQP - NQ)) wd[(tid / (NQP - NQ)) * NQP + NQ + tid % (NQP - NQ)] = 0.0;

    // first prefetch hop: the next pass's connectivity and coefficients
    constexpr int PF = (CPP * NB + 255) / 256;  // prefetch slots per thread
    int32_t pn[PF];
    T plm = T(0);
#pragma unroll
    for (int k = 0; k < PF; k++) {
        const int t = tid + 256 * k, c = t / NB;
        pn[k] = (t < CPP * NB && c < nn_next) ? gmem(g.conn)[en * NB + t] : 0;
    }
    if (want_el && tid < 2 * nn_next) plm = gmem(static_cast<const T *>(g.mat))[2 * en + tid];

    // 2. FP64 geometry, one (cell, point) pair per thread
    for (int t = tid; t < CPP * NQ; t += 256) {
        const int c = t / NQ, q = t - c * NQ;
        const double *x = xs + c * NB * 3;
        double J[3][3] = {};
#pragma unroll
        for (int a = 0; a < NB; a++) {
            const double x0 = x[a * 3], x1 = x[a * 3 + 1], x2 = x[a * 3 + 2];
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const double gr = bfgT[(a * 3 + j) * NQ + q];
                J[0][j] = fma(x0, gr, J[0][j]);
                J[1][j] = fma(x1, gr, J[1][j]);
                J[2][j] = fma(x2, gr, J[2][j]);
            }
        }
        double Ji[3][3];
        const double det = inverse3(J, Ji);
        const bool live = c < n;
        if (live && !(det > 0.0)) fault |= FAULT_DET;
        wd[c * NQP + q] = live ? wq[q] * det : 0.0;
        T *G = Gs + c * L::CR + q;
#pragma unroll
        for (int a = 0; a < NB; a++) {
            const double r0 = bfgT[(a * 3 + 0) * NQ + q], r1 = bfgT[(a * 3 + 1) * NQ + q],
                         r2 = bfgT[(a * 3 + 2) * NQ + q];
#pragma unroll
            for (int i = 0; i < 3; i++)
                G[(i * NB + a) * KS] = live ? static_cast<T>(r0 * Ji[0][i] + r1 * Ji[1][i] + r2 * Ji[2][i]) : T(0);
        }
    }
    __syncthreads();

    // second prefetch hop: the next pass's coordinates (the empty asm keeps
    // the wait for the connectivity loads here, not next to the loads)
    double px[PF][3];
#pragma unroll
    for (int k = 0; k < PF; k++) {
        const int t = tid + 256 * k, c = t / NB;
        px[k][0] = px[k][1] = px[k][2] = 0.0;
        if (t < CPP * NB && c < nn_next) {
            asm volatile("" : "+v"(pn[k]));
            int64_t nd = pn[k];
            if (nd < 0 || nd >= g.n_nodes) {
                fault |= FAULT_INDEX;
                nd = 0;
            }
            px[k][0] = gmem(g.coords)[3 * nd];
            px[k][1] = gmem(g.coords)[3 * nd + 1];
            px[k][2] = gmem(g.coords)[3 * nd + 2];
        }
    }

    // 3. P and M on the matrix cores, wave w: cells w*CPW .. w*CPW+CPW-1
    {
        const int wave = tid >> 6, lane = tid & 63, col = lane & 15, grp = lane >> 4;
#pragma unroll
        for (int k = 0; k < CPW; k++) {
            const int c = wave * CPW + k;
            const T *G = Gs + c * L::CR;
            ACC acc[NT][NT], am{};
#pragma unroll
            for (int i = 0; i < NT; i++)
#pragma unroll
                for (int j = 0; j < NT; j++) acc[i][j] = ACC{};
#pragma unroll
            for (int kk = 0; kk < NQP / 4; kk++) {
                const int q = 4 * kk + grp;
                const T w = static_cast<T>(wd[c * NQP + q]);
                T a[NT], b[NT];
#pragma unroll
                for (int i = 0; i < NT; i++) {
                    b[i] = G[(i * 16 + col) * KS + q];
                    a[i] = b[i] * w;
                }
#pragma unroll
                for (int i = 0; i < NT; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++) mma4<T>(a[i], b[j], acc[i][j]);
                const T phi = (col < NB && q < NQ) ? static_cast<T>(bf[q * NB + col]) : T(0);
                mma4<T>(phi * w, phi, am);
            }
            // accumulator layout: column = lane % 16; FP32 rows 4*(lane/16)+v,
            // FP64 rows lane/16 + 4v
            T *Pc = Ps + c * L::CR;
#pragma unroll
            for (int i = 0; i < NT; i++)
#pragma unroll
                for (int j = 0; j < NT; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int r = i * 16 + (sizeof(T) == 8 ? grp + 4 * v : 4 * grp + v), cc = j * 16 + col;
                        if (r < ND && cc < ND) Pc[r * PS + cc] = static_cast<T>(acc[i][j][v]);
                    }
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = sizeof(T) == 8 ? grp + 4 * v : 4 * grp + v;
                if (r < NB && col < NB) Ms[(c * NB + r) * MS + col] = static_cast<T>(am[v]);
            }
        }
    }
    // park the prefetched pass in the other buffer (not read by this pass)
#pragma unroll
    for (int k = 0; k < PF; k++) {
        const int t = tid + 256 * k;
        if (t < CPP * NB) {
            xn[t * 3] = px[k][0];
            xn[t * 3 + 1] = px[k][1];
            xn[t * 3 + 2] = px[k][2];
        }
    }
    if (want_el && tid < 2 * CPP) lmn[tid] = plm;
    __syncthreads();

    // 4. outputs of the pass's n contiguous cells.  The rows of all n cells
    //    are contiguous in each output; a sweep covers RPS whole rows, a
    //    thread W adjacent columns (in one block: W divides nb) of one row
    //    per step with one W-wide store, so the stores of a sweep are one
    //    contiguous run.  A thread keeps its columns (and the block indices
    //    derived from them) and steps its row and cell: its LDS indices move
    //    by constant strides, corrected by selects at a block row and at a
    //    cell boundary, and the other columns' entries sit in the next words.
    //    Index work per entry is what bounds these loops, hence the column
    //    groups and the strides.
    constexpr int W = NB % 4 == 0 ? 4 : 2;
    static_assert(NB % W == 0, "column groups stay within a block");
    typedef T TW __attribute__((ext_vector_type(W)));
    if (want_el) {
        constexpr int HP = ND / W;  // column groups per row
        constexpr int RPS = 256 / HP, CS = RPS / ND, RR = RPS % ND, QS = RR / NB, MR = RR % NB;
        if (tid < RPS * HP) {
            const int col = W * (tid % HP), s = col / NB, b = col - s * NB;
            const int row = (tid / HP) % ND;
            int c = tid / (HP * ND), r = row / NB, a = row - r * NB;
            // P[(r,a),(s,b)], P[(s,a),(r,b)] and P_00[a][b] of cell c
            int i1 = c * L::CR + row * PS + col, i2 = c * L::CR + (s * NB + a) * PS + r * NB + b;
            int id = c * L::CR + a * PS + b;
            auto out = reinterpret_cast<__attribute__((address_space(1))) TW *>(
                gmem(static_cast<T *>(g.out_el)) + e0 * (ND * ND) + (tid / HP) * ND + col);
#pragma unroll 2
            for (int rr = tid / HP; rr < n * ND; rr += RPS) {
                const T lam = lm[2 * c], mu = lm[2 * c + 1];
                const T md = r == s ? mu : T(0);  // diagonal blocks only
                TW v;
#pragma unroll
                for (int j = 0; j < W; j++)
                    v[j] = lam * Ps[i1 + j] + mu * Ps[i2 + j] +
                           md * (Ps[id + j] + Ps[id + NB * PS + NB + j] + Ps[id + 2 * NB * PS + 2 * NB + j]);
                q2::out_store(v, out);
                out += RPS * HP;
                a += MR;
                r += QS;
                c += CS;
                i1 += CS * L::CR + RR * PS;
                i2 += CS * L::CR + MR * PS + QS * NB;
                id += CS * L::CR + MR * PS;
                const bool wa = a >= NB;  // next block row
                a = wa ? a - NB : a;
                r = wa ? r + 1 : r;
                i2 = wa ? i2 + NB - NB * PS : i2;
                id = wa ? id - NB * PS : id;
                const bool wc = r >= 3;  // next cell
                r = wc ? r - 3 : r;
                c = wc ? c + 1 : c;
                i1 = wc ? i1 + L::CR - ND * PS : i1;
                i2 = wc ? i2 + L::CR - 3 * NB : i2;
                id = wc ? id + L::CR : id;
            }
        }
    }
    constexpr int HB = NB / W, RPB = 256 / HB;  // column groups and rows per sweep of the nb x nb outputs
    constexpr int QB = RPB / NB, MB = RPB % NB;
    if ((g.forms & (FORM_BIT_LAPLACE | FORM_BIT_MASS)) && tid < RPB * HB) {
        const int b = W * (tid % HB);
        const bool lap = g.forms & FORM_BIT_LAPLACE, mass = g.forms & FORM_BIT_MASS;
        int a = (tid / HB) % NB, c = tid / (HB * NB);
        int il = c * L::CR + a * PS + b;  // P_00[a][b] of cell c
        const T *mp = Ms + (c * NB + a) * MS + b;
        const int o = (tid / HB) * NB + b;
        auto ol = reinterpret_cast<__attribute__((address_space(1))) TW *>(
            gmem(lap ? static_cast<T *>(g.out_lap) + e0 * (NB * NB) + o : nullptr));
        auto om = reinterpret_cast<__attribute__((address_space(1))) TW *>(
            gmem(mass ? static_cast<T *>(g.out_mass) + e0 * (NB * NB) + o : nullptr));
#pragma unroll 2
        for (int rr = tid / HB; rr < n * NB; rr += RPB) {
            if (lap) {
                TW v;
#pragma unroll
                for (int j = 0; j < W; j++) v[j] = Ps[il + j] + Ps[il + NB * PS + NB + j] + Ps[il + 2 * NB * PS + 2 * NB + j];
                q2::out_store(v, ol);
                ol += RPB * HB;
            }
            if (mass) {
                TW v;
#pragma unroll
                for (int j = 0; j < W; j++) v[j] = mp[j];
                q2::out_store(v, om);
                om += RPB * HB;
            }
            mp += RPB * MS;
            a += MB;
            il += MB * PS + QB * L::CR;
            const bool wc = a >= NB;  // next cell
            a = wc ? a - NB : a;
            il = wc ? il + L::CR - NB * PS : il;
        }
    }
    if (fault) raise_fault(flags, fault);
    __syncthreads();  // LDS is reused by the next pass
}

template <int CELL, int P, typename T>
__device__ void small_tile(const GroupDev &g, int64_t c0, int64_t c1, unsigned *flags, unsigned char *smem, int tid)
{
    using L = SmallMM<CELL, P, T>;
    constexpr int CPP = L::CPP, NB = L::NB, NQ = L::NQ;
    if (c0 >= c1) return;
    {
        double *tab = reinterpret_cast<double *>(smem + L::OFF_TAB);
        for (int t = tid; t < L::TAB; t += 256)
            tab[t] = t < NB * 3 * NQ ? gmem(g.tab.bfgT)[t]
                     : (t < NB * 3 * NQ + NQ * NB ? gmem(g.tab.bf)[t - NB * 3 * NQ]
                                                  : gmem(g.tab.w)[t - NB * 3 * NQ - NQ * NB]);
        const int n0 = c1 - c0 < CPP ? int(c1 - c0) : CPP;
        const unsigned f = small_gather<CELL, P, T>(g, c0, n0, reinterpret_cast<double *>(smem + L::OFF_X),
                                                    reinterpret_cast<T *>(smem + L::OFF_LM), tid);
        if (f) raise_fault(flags, f);
        __syncthreads();
    }
    int buf = 0;
    for (int64_t e0 = c0; e0 < c1; e0 += CPP, buf ^= 1) {
        const int n = c1 - e0 < CPP ? int(c1 - e0) : CPP;
        const int64_t en = e0 + CPP;
        const int nn = en < c1 ? (c1 - en < CPP ? int(c1 - en) : CPP) : 0;
        small_pass<CELL, P, T>(g, e0, n, buf, en, nn, flags, smem, tid);
    }
}

// P1 tetrahedra: the map is affine, so J, det J and the physical gradients
// G_i[a] = sum_j dphi_a/dxi_j (J^-1)_ji are the same at every quadrature
// point and each form's quadrature sum factors exactly into a per-cell
// geometry term times a reference sum:
//   K[(r,a),(s,b)] = det J (sum_q w_q) (lambda G_r[a] G_s[b] + mu G_s[a] G_r[b]
//                    + delta_rs mu G[a].G[b])
//   L[a][b] = det J (sum_q w_q) G[a].G[b],   M[a][b] = det J sum_q w_q phi_a phi_b.
// A pass takes 256 cells: one thread per cell evaluates the FP64 geometry and
// leaves G (in the output type), the two volume factors and the coefficients
// in LDS; then consecutive threads produce consecutive output entries of the
// pass's contiguous cells, so every store stream is contiguous.
template <typename T>
struct AffineTet {
    static constexpr int NB = 4, ND = 12, CPP = 256;
    static constexpr int SA = 17;  // per-cell LDS record (odd stride): G[12], vol, det, lambda, mu
    static constexpr int OFF_M = 0;  // double Mref[16] = sum_q w_q phi_a phi_b, then sum_q w_q
    static constexpr int OFF_C = align16(OFF_M + 17 * 8);
    static constexpr int BYTES = align16(OFF_C + CPP * SA * (int)sizeof(T));
};

template <typename T>
__device__ void affine_tile(const GroupDev &g, int64_t c0, int64_t c1, unsigned *flags, unsigned char *smem, int tid)
{
    using L = AffineTet<T>;
    constexpr int NB = L::NB, ND = L::ND, NQ = cell_nq(FE_CELL_TET, 1), SA = L::SA;
    double *Mref = reinterpret_cast<double *>(smem + L::OFF_M);
    T *rec = reinterpret_cast<T *>(smem + L::OFF_C);
    if (c0 >= c1) return;
    if (tid < NB * NB + 1) {
        const int a = tid / NB, b = tid - a * NB;
        double s = 0.0;
        for (int q = 0; q < NQ; q++)
            s += gmem(g.tab.w)[q] * (tid < NB * NB ? gmem(g.tab.bf)[q * NB + a] * gmem(g.tab.bf)[q * NB + b] : 1.0);
        Mref[tid] = s;
    }
    __syncthreads();
    const bool want_el = g.forms & FORM_BIT_ELAST;
    unsigned fault = 0;
    for (int64_t e0 = c0; e0 < c1; e0 += L::CPP) {
        const int n = c1 - e0 < L::CPP ? int(c1 - e0) : L::CPP;
        // 1. geometry of cell e0 + tid
        if (tid < n) {
            const int64_t e = e0 + tid;
            double J[3][3] = {};
            double gr[NB][3];
#pragma unroll
            for (int a = 0; a < NB; a++) {
                int64_t nd = gmem(g.conn)[e * NB + a];
                if (nd < 0 || nd >= g.n_nodes) {
                    fault |= FAULT_INDEX;
                    nd = 0;
                }
                const double x0 = gmem(g.coords)[3 * nd], x1 = gmem(g.coords)[3 * nd + 1], x2 = gmem(g.coords)[3 * nd + 2];
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    gr[a][j] = gmem(g.tab.bfgT)[(a * 3 + j) * NQ];  // constant over the cell
                    J[0][j] = fma(x0, gr[a][j], J[0][j]);
                    J[1][j] = fma(x1, gr[a][j], J[1][j]);
                    J[2][j] = fma(x2, gr[a][j], J[2][j]);
                }
            }
            double Ji[3][3];
            const double det = inverse3(J, Ji);
            if (!(det > 0.0)) fault |= FAULT_DET;
            T *r = rec + tid * SA;
#pragma unroll
            for (int a = 0; a < NB; a++)
#pragma unroll
                for (int i = 0; i < 3; i++)
                    r[i * NB + a] = static_cast<T>(gr[a][0] * Ji[0][i] + gr[a][1] * Ji[1][i] + gr[a][2] * Ji[2][i]);
            r[12] = static_cast<T>(det * Mref[NB * NB]);
            r[13] = static_cast<T>(det);
            if (want_el) {
                r[14] = gmem(static_cast<const T *>(g.mat))[2 * e];
                r[15] = gmem(static_cast<const T *>(g.mat))[2 * e + 1];
            }
        }
        __syncthreads();
        // 2. outputs, one thread per entry; the elasticity rows go in sweeps
        //    of RPS whole rows, so a thread keeps its column and steps its
        //    row and cell (one contiguous store run per sweep)
        if (want_el) {
            constexpr int RPS = 256 / ND;
            if (tid < RPS * ND) {
                const int col = tid % ND, s = col / NB, b = col - s * NB;
                int row = (tid / ND) % ND, c = tid / (ND * ND);
                auto out = gmem(static_cast<T *>(g.out_el)) + e0 * (ND * ND) + tid;
                for (int rr = tid / ND; rr < n * ND; rr += RPS) {
                    const int r = row / NB, a = row - r * NB;
                    const T *G = rec + c * SA;
                    const T lam = G[14], mu = G[15];
                    T v = lam * G[r * NB + a] * G[s * NB + b] + mu * G[s * NB + a] * G[r * NB + b];
                    if (r == s) v += mu * (G[a] * G[b] + G[NB + a] * G[NB + b] + G[2 * NB + a] * G[2 * NB + b]);
                    q2::out_store(G[12] * v, out);
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
        if (g.forms & FORM_BIT_LAPLACE) {
            const auto out = gmem(static_cast<T *>(g.out_lap)) + e0 * (NB * NB);
            for (int f = tid; f < n * NB * NB; f += 256) {
                const int c = f / (NB * NB), a = (f / NB) % NB, b = f % NB;
                const T *G = rec + c * SA;
                q2::out_store(G[12] * (G[a] * G[b] + G[NB + a] * G[NB + b] + G[2 * NB + a] * G[2 * NB + b]), out + f);
            }
        }
        if (g.forms & FORM_BIT_MASS) {
            const auto out = gmem(static_cast<T *>(g.out_mass)) + e0 * (NB * NB);
            for (int f = tid; f < n * NB * NB; f += 256) {
                const int c = f / (NB * NB), ab = f % (NB * NB);
                q2::out_store(static_cast<T>(static_cast<double>(rec[c * SA + 13]) * Mref[ab]), out + f);
            }
        }
        __syncthreads();  // the records are rewritten by the next pass
    }
    if (fault) raise_fault(flags, fault);
}

template <typename T>
struct BatchLds {
    static constexpr int MM = sizeof(T) == 8 ? MM_F64 : MM_F32;
    static constexpr int v0 = Q2Layout<MM>::BYTES;
    static constexpr int v1 = AffineTet<T>::BYTES;
    static constexpr int v2 = SmallMM<FE_CELL_TET, 2, T>::BYTES;
    static constexpr int v3 = SmallMM<FE_CELL_HEX, 1, T>::BYTES;
    static constexpr int m01 = v0 > v1 ? v0 : v1, m23 = v2 > v3 ? v2 : v3;
    static constexpr int BYTES = m01 > m23 ? m01 : m23;
};

// Q2 items.
template <int MM>
__device__ __forceinline__ void q2_item(const GroupDev &g, int64_t c0, int64_t c1, unsigned *flags, unsigned char *smem,
                                     int tid)
{
    const Q2Job job{g.n_cells, g.n_nodes, g.coords, g.conn, g.mat, g.out_el, g.out_mass, g.out_lap, flags, g.tab};
    q2_run<MM, true>(job, c0, c1, 1, smem, tid);
}

__global__ void k_batch_reset(unsigned long long *ctr) { ctr[0] = 0ULL; }

template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void k_batch(const BatchDev *__restrict__ B, unsigned long long *ctr, unsigned *flags)
{
    __shared__ __align__(16) unsigned char smem[BatchLds<T>::BYTES];
    __shared__ long long s_item;
    constexpr int MM = BatchLds<T>::MM;
    const int64_t n_items = B->n_items;
    const int ng = B->n_groups;
    for (;;) {
        if (threadIdx.x == 0) s_item = static_cast<long long>(atomicAdd(ctr, 1ULL));
        __syncthreads();
        // the item number is the same for the whole workgroup; saying so
        // (readfirstlane) keeps the group descriptor and every branch on it
        // in scalar registers instead of per-lane ones
        const long long sv = s_item;
        const int64_t it = static_cast<int64_t>(
            (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(sv >> 32)))) << 32) |
            static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(sv & 0xffffffff))));
        __syncthreads();
        if (it >= n_items) break;  // every workgroup leaves once the queue is drained
        // the thread index, re-read each item through an opaque move: the
        // per-thread offsets the item routines derive from it are then
        // recomputed per item instead of being hoisted out of this loop and
        // kept live (in registers the routines need) for the whole kernel
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(static_cast<int>(threadIdx.x)));
        int gi = 0;
        while (gi + 1 < ng && it >= B->g[gi + 1].item0) gi++;
        gi = __builtin_amdgcn_readfirstlane(gi);  // uniform: the descriptor loads stay scalar
        const GroupDev &g = B->g[gi];
        const int64_t c0 = (it - g.item0) * g.tile;
        const int64_t c1 = c0 + g.tile < g.n_cells ? c0 + g.tile : g.n_cells;
        if (g.cell == FE_CELL_HEX && g.order == 2) {
            q2_item<MM>(g, c0, c1, flags, smem, tid);
        } else if (g.cell == FE_CELL_HEX && g.order == 1) {
            small_tile<FE_CELL_HEX, 1, T>(g, c0, c1, flags, smem, tid);
        } else if (g.cell == FE_CELL_TET && g.order == 1) {
            affine_tile<T>(g, c0, c1, flags, smem, tid);
        } else if (g.cell == FE_CELL_TET && g.order == 2) {
            small_tile<FE_CELL_TET, 2, T>(g, c0, c1, flags, smem, tid);
        }
    }
}

int group_pass_cells(int cell, int order, bool f64)
{
    if (cell == FE_CELL_HEX && order == 2) return 1;
    if (cell == FE_CELL_HEX) return f64 ? SmallMM<FE_CELL_HEX, 1, double>::CPP : SmallMM<FE_CELL_HEX, 1, float>::CPP;
    if (order == 1) return AffineTet<double>::CPP;
    return f64 ? SmallMM<FE_CELL_TET, 2, double>::CPP : SmallMM<FE_CELL_TET, 2, float>::CPP;
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
        // an empty group needs no arrays at all
        const bool missing = g.n_cells > 0 && (!g.coords || !g.conn || ((g.forms & (1 << FE_FORM_MASS)) && !g.out_mass) ||
                                               ((g.forms & (1 << FE_FORM_LAPLACE)) && !g.out_laplace) ||
                                               ((g.forms & (1 << FE_FORM_ELASTICITY)) && (!g.out_elasticity || !g.material)));
        if (!g.forms || bad_forms || g.n_cells < 0 || g.n_nodes < 0 || (g.n_cells > 0 && g.n_nodes == 0) || missing ||
            g.tile < 0) {
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
