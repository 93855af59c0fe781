// Matrix-core (MFMA) element-matrix kernel for Q2 and Q3 hexahedra: scalar
// and vector mass, Laplace, and linear elasticity with per-cell isotropic
// coefficients, in FP64, FP32 or BF16X3, with FP64 geometry.
//
// Every form of the table of example weak forms in matrix mode is read off
// products of ONE operand per cell, built from the geometry:
//   Laplace / elasticity  g[q][(c,a)] = sqrt(w_q det J_q) G_c[q][a]  (c = 0..2)
//   mass                  g[q][a]     = sqrt(w_q det J_q) phi_a(q)
// (w_q > 0 and det J > 0, so the square root is real; a cell with det J <= 0
// raises the fault flag).  With P[(r,a),(s,b)] = sum_q g[q][(r,a)] g[q][(s,b)]:
//   mass        M = P                      vector mass = I_3 (x) M
//   Laplace     K = P_00 + P_11 + P_22
//   elasticity  K_rs = lambda P_rs + mu P_rs^T + delta_rs mu (P_00 + P_11 + P_22)
// which is w det B^T D B of the linear-elasticity expression for isotropic D
// (the same recombination the Q2 elasticity kernel uses).  Both MFMA
// operands come from the same array, so a diagonal tile is exactly symmetric.
//
// The output is cut into 16x16 tiles.  Per cell only tiles on or above the
// diagonal are multiplied, grouped into jobs whose outputs (including the
// mirrored tiles below the diagonal) need no other job's products:
//   DIAG(i,j)        elasticity, diagonal blocks: P_tt(i,j) for t = 0,1,2 ->
//                    K_tt(i,j) = (lambda + mu) P_tt(i,j) + mu sum_t' P_t't'(i,j)
//   PAIR(r,s,i<j)    elasticity, r < s: P_rs(i,j), P_rs(j,i) -> K_rs(i,j),
//                    K_rs(j,i) and their mirrors in K_sr
//   SINGLE(r,s,i)    elasticity, r < s: P_rs(i,i) -> K_rs(i,i), K_sr(i,i)
//   LAP(i,j)         Laplace: sum_t P_tt(i,j)
//   MASS(i,j)        mass: P(i,j) (vector mass: the three diagonal blocks,
//                    zeros in the six others)
// Jobs are spread over the waves of the workgroup by a static longest-first
// schedule.  A wave runs its jobs back to back with no workgroup barrier;
// mirrored tiles are transposed through a small per-wave LDS buffer, and
// every tile is stored straight from the accumulator layout (each store
// instruction writes four 16-entry row segments of the row-major output).
//
// One workgroup per cell at a time, persistent over an XCD-contiguous range
// of cells.  Per cell:
//   1. J entries at every quadrature point by sum factorization over the
//      tensor-product 1-D tables (FP64);
//   2. det J, J^-1 and sqrt(w det J) per point (FP64);
//   3. the operand g in LDS in the contraction type (two bf16 arrays, high
//      and low parts, for BF16X3), row (c,a) padded to a multiple of 16,
//      columns = quadrature points, row stride chosen so the 16 rows x 4
//      (or 4 x 8-point) fragment reads hit distinct LDS banks;
//   4. the jobs on the matrix cores:
//        FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32,
//        BF16X3: v_mfma_f32_16x16x32_bf16 on hi*hi + hi*lo + lo*hi.
// The next cell's connectivity is loaded during step 2, its coordinates
// during step 4, and parked in LDS at the end of step 4.
#include "mm_device.h"

namespace fe {
namespace {

using q2::bf8;
using q2::cell_range;
using q2::d4;
using q2::f4;
using q2::MM_BF16X3;
using q2::MM_F32;
using q2::MM_F64;
using q2::MMT;

constexpr int WAVES = 8;
constexpr int THREADS = 64 * WAVES;

enum : int { J_DIAG = 0, J_PAIR = 1, J_SINGLE = 2, J_LAP = 3, J_MASS = 4 };

using mm::acc_row;
using mm::align_to;
using mm::op_stride;
using mm::store_tile;
using mm::valid;

// Static schedule: jobs in order of decreasing weight (matrix-core tiles),
// each given to the least loaded wave.
struct Sched {
    uint32_t job[WAVES][32];
    int n[WAVES];
};

constexpr uint32_t enc(int kind, int r, int s, int i, int j)
{
    return static_cast<uint32_t>(kind | (r << 4) | (s << 6) | (i << 8) | (j << 12));
}

constexpr Sched make_sched(int form, int nt)
{
    Sched S{};
    uint32_t jobs[128] = {};
    int wt[128] = {};
    int nj = 0;
    if (form == FE_FORM_ELASTICITY) {
        for (int i = 0; i < nt; i++)
            for (int j = i; j < nt; j++) {
                jobs[nj] = enc(J_DIAG, 0, 0, i, j);
                wt[nj++] = 3;
            }
        for (int r = 0; r < 3; r++)
            for (int s = r + 1; s < 3; s++)
                for (int i = 0; i < nt; i++)
                    for (int j = i + 1; j < nt; j++) {
                        jobs[nj] = enc(J_PAIR, r, s, i, j);
                        wt[nj++] = 2;
                    }
        for (int r = 0; r < 3; r++)
            for (int s = r + 1; s < 3; s++)
                for (int i = 0; i < nt; i++) {
                    jobs[nj] = enc(J_SINGLE, r, s, i, i);
                    wt[nj++] = 1;
                }
    } else {
        const int kind = form == FE_FORM_LAPLACE ? J_LAP : J_MASS;
        for (int i = 0; i < nt; i++)
            for (int j = i; j < nt; j++) {
                jobs[nj] = enc(kind, 0, 0, i, j);
                wt[nj++] = kind == J_LAP ? 3 : 1;
            }
    }
    int load[WAVES] = {};
    for (int k = 0; k < nj; k++) {
        int w = 0;
        for (int v = 1; v < WAVES; v++)
            if (load[v] < load[w]) w = v;
        S.job[w][S.n[w]++] = jobs[k];
        load[w] += wt[k];
    }
    return S;
}

template <int P, int FORM, int MM>
struct HexMM {
    static constexpr int N1 = P + 1, NB = N1 * N1 * N1, NQ = NB;
    static constexpr bool MASSF = FORM == FE_FORM_MASS || FORM == FE_FORM_VMASS;
    static constexpr int NC = MASSF ? 1 : 3;  // operand components
    static constexpr int NCO = form_nc(FORM);  // output components
    static constexpr int ND = NCO * NB;        // output row length
    static constexpr int NBP = align_to(NB, 16), NT = NBP / 16;
    static constexpr bool RAGGED = NB % 16 != 0;
    using T = typename MMT<MM>::T;      // accumulation and output type
    using ACC = typename MMT<MM>::acc;  // 16x16 accumulator fragment
    using OPT = typename std::conditional<MM == MM_BF16X3, __bf16, T>::type;
    static constexpr int KP = align_to(NQ, MM == MM_BF16X3 ? 32 : 4);
    static constexpr int KS = op_stride(MM, KP);
    static constexpr int ROWS = NC * NBP;
    static constexpr int NOP = MM == MM_BF16X3 ? 2 : 1;  // operand arrays (hi, lo)
    static constexpr int TS = 17;  // transpose buffer row stride (conflict-free for FP64)
    // nontemporal stores when the tiles' row segments fill whole 128-byte
    // lines (Q3: rows of 64 or 192 entries); Q2 rows of 27 or 81 entries go
    // through the L2, which joins the halves of straddled lines
    static constexpr bool NT_STORE = ND % 16 == 0;
    // LDS layout (bytes)
    static constexpr int OFF_TB = 0;  // double B1[N1][N1], D1[N1][N1], w[NQ]
    static constexpr int OFF_X = q2::align16(OFF_TB + (2 * N1 * N1 + NQ) * 8);  // double xs[3][NB], T lm[2]
    static constexpr int OFF_OP = q2::align16(OFF_X + 3 * NB * 8 + 16);
    static constexpr int OP_BYTES = q2::align16(ROWS * KS * (int)sizeof(OPT));
    static constexpr int OFF_SC = OFF_OP + NOP * OP_BYTES;
    // scratch, used in turn by the geometry (J, then sqrt(wd) J^-1) and by
    // the per-wave transpose buffers of the job phase
    static constexpr int SC_GEO = NQ * 10 * 8;
    static constexpr int SC_TR = WAVES * 16 * TS * (int)sizeof(T);
    static constexpr int BYTES = q2::align16(OFF_SC + (SC_GEO > SC_TR ? SC_GEO : SC_TR));
    static constexpr Sched SCHED = make_sched(FORM == FE_FORM_VMASS ? FE_FORM_MASS : FORM, NT);
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc[u] += sum over k in [k0, k1) of g[rowsA[u] + m][k] g[rowsB[u] + n][k]
// (rows = operand row of the tile's first entry)
template <class H, int NU>
__device__ __forceinline__ void mma_run(typename H::ACC *acc, const typename H::OPT *op, const int *ra, const int *rb,
                                        int k0, int k1, int lane)
{
    using OPT = typename H::OPT;
    constexpr int KS = H::KS;
    const int m = lane & 15, grp = lane >> 4;
    if constexpr (H::NOP == 1) {
        // fragments double-buffered: step k + 4 is loaded while step k
        // multiplies, so the wave does not wait for LDS before every MFMA
        OPT a[2][NU], b[2][NU];
        auto load = [&](int buf, int k) {
#pragma unroll
            for (int u = 0; u < NU; u++) {
                a[buf][u] = op[(ra[u] + m) * KS + k + grp];
                b[buf][u] = op[(rb[u] + m) * KS + k + grp];
            }
        };
        auto mfma = [&](int buf) {
#pragma unroll
            for (int u = 0; u < NU; u++) {
                if constexpr (sizeof(OPT) == 8)
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[buf][u], b[buf][u], acc[u], 0, 0, 0);
                else
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[buf][u], b[buf][u], acc[u], 0, 0, 0);
            }
        };
        // (the scheduling barriers keep the compiler from regrouping the
        // loads after the products that do not need them)
        load(0, k0);
#pragma unroll
        for (int k = k0; k < k1; k += 8) {
            if (k + 4 < k1) load(1, k + 4);
            __builtin_amdgcn_sched_barrier(0);
            mfma(0);
            __builtin_amdgcn_sched_barrier(0);
            if (k + 4 < k1) {
                if (k + 8 < k1) load(0, k + 8);
                __builtin_amdgcn_sched_barrier(0);
                mfma(1);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        const OPT *lo = op + H::OP_BYTES / sizeof(OPT);
#pragma unroll 2
        for (int k = k0; k < k1; k += 32) {
            bf8 ah[NU], al[NU], bh[NU], bl[NU];
#pragma unroll
            for (int u = 0; u < NU; u++) {
                const int oa = (ra[u] + m) * KS + k + 8 * grp, ob = (rb[u] + m) * KS + k + 8 * grp;
                ah[u] = *reinterpret_cast<const bf8 *>(op + oa);
                al[u] = *reinterpret_cast<const bf8 *>(lo + oa);
                bh[u] = *reinterpret_cast<const bf8 *>(op + ob);
                bl[u] = *reinterpret_cast<const bf8 *>(lo + ob);
            }
#pragma unroll
            for (int u = 0; u < NU; u++) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[u], bh[u], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < NU; u++) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u], bl[u], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < NU; u++) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u], bh[u], acc[u], 0, 0, 0);
        }
    }
}

// x^T in the accumulator layout, through this wave's LDS buffer
template <class H>
__device__ __forceinline__ typename H::ACC transpose(const typename H::ACC &x, typename H::T *buf, int lane)
{
    constexpr int MM = sizeof(typename H::T) == 8 ? MM_F64 : MM_F32;
    const int col = lane & 15;
    typename H::ACC y;
#pragma unroll
    for (int v = 0; v < 4; v++) buf[acc_row<MM>(lane, v) * H::TS + col] = x[v];
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; v++) y[v] = buf[col * H::TS + acc_row<MM>(lane, v)];
    wave_sync();
    return y;
}

// The elasticity epilogues below evaluate lambda X + mu Y as
// fma(lambda, X, mu Y) in every copy, so that an entry and its mirror are
// rounded alike and the FP64/FP32 element matrices are exactly symmetric.
//
// Elasticity output of a DIAG job from c[t] = P_tt(i,j), t = 0,1,2:
// K_tt(i,j) = (lambda + mu) P_tt(i,j) + mu sum_t' P_t't'(i,j), and the
// mirrored tiles K_tt(j,i) = K_tt(i,j)^T when i != j.
template <class H>
__device__ __forceinline__ void epi_diag(const typename H::ACC *c, typename H::T *oc, typename H::T *buf,
                                         typename H::T lam, typename H::T mu, int i, int j, int lane)
{
    using T = typename H::T;
    using ACC = typename H::ACC;
    constexpr int NB = H::NB;
    const int vi = valid<H>(i), vj = valid<H>(j);
    ACC S;
#pragma unroll
    for (int v = 0; v < 4; v++) S[v] = c[0][v] + c[1][v] + c[2][v];
    const T lm = lam + mu;
#pragma unroll
    for (int t = 0; t < 3; t++) {
        ACC k;
#pragma unroll
        for (int v = 0; v < 4; v++) k[v] = fma(lm, c[t][v], mu * S[v]);
        store_tile<H>(oc, t * NB + 16 * i, t * NB + 16 * j, vi, vj, k, lane);
    }
    if (i != j) {
        const ACC St = transpose<H>(S, buf, lane);
#pragma unroll
        for (int t = 0; t < 3; t++) {
            const ACC ct = transpose<H>(c[t], buf, lane);
            ACC k;
#pragma unroll
            for (int v = 0; v < 4; v++) k[v] = fma(lm, ct[v], mu * St[v]);
            store_tile<H>(oc, t * NB + 16 * j, t * NB + 16 * i, vj, vi, k, lane);
        }
    }
}

// Elasticity output of a PAIR job from A = c[0] = P_rs(i,j), B = c[1] =
// P_rs(j,i) (r < s): K_rs(i,j) = lambda A + mu B^T, K_rs(j,i) = lambda B +
// mu A^T, and their transposes in block (s,r).
template <class H>
__device__ __forceinline__ void epi_pair(const typename H::ACC *c, typename H::T *oc, typename H::T *buf,
                                         typename H::T lam, typename H::T mu, int r, int s, int i, int j, int lane)
{
    using ACC = typename H::ACC;
    constexpr int NB = H::NB;
    const int vi = valid<H>(i), vj = valid<H>(j);
    const ACC Bt = transpose<H>(c[1], buf, lane);
    ACC x;
#pragma unroll
    for (int v = 0; v < 4; v++) x[v] = fma(lam, c[0][v], mu * Bt[v]);
    store_tile<H>(oc, r * NB + 16 * i, s * NB + 16 * j, vi, vj, x, lane);  // K_rs(i,j)
#pragma unroll
    for (int v = 0; v < 4; v++) x[v] = fma(lam, Bt[v], mu * c[0][v]);
    store_tile<H>(oc, s * NB + 16 * i, r * NB + 16 * j, vi, vj, x, lane);  // K_sr(i,j)
    const ACC At = transpose<H>(c[0], buf, lane);
#pragma unroll
    for (int v = 0; v < 4; v++) x[v] = fma(lam, c[1][v], mu * At[v]);
    store_tile<H>(oc, r * NB + 16 * j, s * NB + 16 * i, vj, vi, x, lane);  // K_rs(j,i)
#pragma unroll
    for (int v = 0; v < 4; v++) x[v] = fma(lam, At[v], mu * c[1][v]);
    store_tile<H>(oc, s * NB + 16 * j, r * NB + 16 * i, vj, vi, x, lane);  // K_sr(j,i)
}

// Elasticity output of a SINGLE job from a = P_rs(i,i) (r < s).
template <class H>
__device__ __forceinline__ void epi_single(const typename H::ACC &a, typename H::T *oc, typename H::T *buf,
                                           typename H::T lam, typename H::T mu, int r, int s, int i, int lane)
{
    using ACC = typename H::ACC;
    constexpr int NB = H::NB;
    const int vi = valid<H>(i);
    const ACC at = transpose<H>(a, buf, lane);
    ACC x;
#pragma unroll
    for (int v = 0; v < 4; v++) x[v] = fma(lam, a[v], mu * at[v]);
    store_tile<H>(oc, r * NB + 16 * i, s * NB + 16 * i, vi, vi, x, lane);
#pragma unroll
    for (int v = 0; v < 4; v++) x[v] = fma(lam, at[v], mu * a[v]);
    store_tile<H>(oc, s * NB + 16 * i, r * NB + 16 * i, vi, vi, x, lane);
}

// Laplace output of a LAP job from S = sum_t P_tt(i,j), and its mirror.
template <class H>
__device__ __forceinline__ void epi_lap(const typename H::ACC &S, typename H::T *oc, typename H::T *buf, int i, int j,
                                        int lane)
{
    const int vi = valid<H>(i), vj = valid<H>(j);
    store_tile<H>(oc, 16 * i, 16 * j, vi, vj, S, lane);
    if (i != j) store_tile<H>(oc, 16 * j, 16 * i, vj, vi, transpose<H>(S, buf, lane), lane);
}

// Mass output of a MASS job from a = P(i,j): scalar mass M(i,j) and its
// mirror, or for the vector mass the tile in the three diagonal blocks and
// zeros in the six others.
template <class H, int FORM>
__device__ __forceinline__ void epi_mass(const typename H::ACC &a, typename H::T *oc, typename H::T *buf, int i,
                                         int j, int lane)
{
    using ACC = typename H::ACC;
    const int vi = valid<H>(i), vj = valid<H>(j);
    if constexpr (FORM == FE_FORM_MASS) {
        store_tile<H>(oc, 16 * i, 16 * j, vi, vj, a, lane);
        if (i != j) store_tile<H>(oc, 16 * j, 16 * i, vj, vi, transpose<H>(a, buf, lane), lane);
    } else {
        constexpr int NB = H::NB;
        const ACC tt = i != j ? transpose<H>(a, buf, lane) : a;
        const ACC z = {};
#pragma unroll
        for (int rr = 0; rr < 3; rr++)
#pragma unroll
            for (int ss = 0; ss < 3; ss++) {
                store_tile<H>(oc, rr * NB + 16 * i, ss * NB + 16 * j, vi, vj, rr == ss ? a : z, lane);
                if (i != j) store_tile<H>(oc, rr * NB + 16 * j, ss * NB + 16 * i, vj, vi, rr == ss ? tt : z, lane);
            }
    }
}

// One job of the current cell.  oc = the cell's output matrix.
template <class H, int FORM>
__device__ __forceinline__ void run_job(uint32_t jb, const typename H::OPT *op, typename H::T *oc,
                                        typename H::T *buf, typename H::T lam, typename H::T mu, int lane)
{
    using ACC = typename H::ACC;
    constexpr int NBP = H::NBP, KP = H::KP;
    const int kind = jb & 15, r = (jb >> 4) & 3, s = (jb >> 6) & 3, i = (jb >> 8) & 15, j = (jb >> 12) & 15;
    if (kind == J_DIAG || kind == J_LAP) {
        ACC c[3] = {};
        const int ra[3] = {16 * i, NBP + 16 * i, 2 * NBP + 16 * i};
        const int rb[3] = {16 * j, NBP + 16 * j, 2 * NBP + 16 * j};
        mma_run<H, 3>(c, op, ra, rb, 0, KP, lane);
        if (kind == J_DIAG) {
            epi_diag<H>(c, oc, buf, lam, mu, i, j, lane);
            return;
        }
        ACC S;
#pragma unroll
        for (int v = 0; v < 4; v++) S[v] = c[0][v] + c[1][v] + c[2][v];
        epi_lap<H>(S, oc, buf, i, j, lane);
    } else if (kind == J_PAIR) {
        ACC c[2] = {};
        const int ra[2] = {r * NBP + 16 * i, r * NBP + 16 * j};
        const int rb[2] = {s * NBP + 16 * j, s * NBP + 16 * i};
        mma_run<H, 2>(c, op, ra, rb, 0, KP, lane);
        epi_pair<H>(c, oc, buf, lam, mu, r, s, i, j, lane);
    } else {
        // SINGLE / MASS: two half-depth products in flight, summed
        ACC c[2] = {};
        constexpr int KH = align_to(KP / 2, H::NOP == 2 ? 32 : 4);
        const int ra[1] = {kind == J_SINGLE ? r * NBP + 16 * i : 16 * i};
        const int rb[1] = {kind == J_SINGLE ? s * NBP + 16 * i : 16 * j};
        mma_run<H, 1>(c, op, ra, rb, 0, KH, lane);
        if constexpr (KH < KP) mma_run<H, 1>(c + 1, op, ra, rb, KH, KP, lane);
        ACC a;
#pragma unroll
        for (int v = 0; v < 4; v++) a[v] = c[0][v] + c[1][v];
        if (kind == J_SINGLE)
            epi_single<H>(a, oc, buf, lam, mu, r, s, i, lane);
        else
            epi_mass<H, FORM>(a, oc, buf, i, j, lane);
    }
}

template <int P, int FORM, int MM>
__global__ __launch_bounds__(THREADS, MM == MM_F64 ? 1 : 2) void k_hexmm(ExecArgs A)
{
    using H = HexMM<P, FORM, MM>;
    using T = typename H::T;
    using OPT = typename H::OPT;
    constexpr int N1 = H::N1, NB = H::NB, NQ = H::NQ, NC = H::NC, NBP = H::NBP, KS = H::KS;
    constexpr bool ELAST = FORM == FE_FORM_ELASTICITY;
    __shared__ __align__(16) unsigned char smem[H::BYTES];
    double *B1 = reinterpret_cast<double *>(smem + H::OFF_TB);
    double *D1 = B1 + N1 * N1;
    double *wq = D1 + N1 * N1;
    double *xs = reinterpret_cast<double *>(smem + H::OFF_X);  // [3][NB]
    T *lms = reinterpret_cast<T *>(xs + 3 * NB);
    OPT *op = reinterpret_cast<OPT *>(smem + H::OFF_OP);
    double *Jq = reinterpret_cast<double *>(smem + H::OFF_SC);  // [NQ][9]
    double *Mq = Jq;                                            // [NQ][10]: sqrt(wd) J^-1, sqrt(wd)
    T *tbuf = reinterpret_cast<T *>(smem + H::OFF_SC);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    T *buf = tbuf + wave * 16 * H::TS;

    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    if (e >= e_end) return;  // uniform over the workgroup
    const T *mat = static_cast<const T *>(A.mat);

    // tables, operand padding (never rewritten), the first cell's data
    for (int k = tid; k < N1 * N1; k += THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < NQ; k += THREADS) wq[k] = A.tab.w[k];
    for (int k = tid; k < H::NOP * H::OP_BYTES / (int)sizeof(OPT); k += THREADS) op[k] = OPT(0);
    const int ga = tid / 3, gc = tid - 3 * (tid / 3);  // node / axis of this thread's coordinate
    if (tid < 3 * NB) {
        const int64_t n = checked_node(A.conn, e * NB + ga, A.n_nodes, A.flags);
        xs[gc * NB + ga] = A.coords[3 * n + gc];
    }
    if constexpr (ELAST)
        if (tid < 2) lms[tid] = mat[2 * e + tid];
    __syncthreads();

    for (;;) {
        const int64_t en = e + stride;
        const bool has_next = en < e_end;
        T lam = T(0), mu = T(0);
        if constexpr (ELAST) {
            lam = lms[0];
            mu = lms[1];
        }

        // 1. J[i][j] at each point: sum over the tensor-product nodes with
        //    the 1-D value / derivative tables
        for (int it = tid; it < NQ * 9; it += THREADS) {
            const int q = it % NQ, ij = it / NQ, i = ij / 3, jj = ij - 3 * (ij / 3);
            const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
            const double *T0 = (jj == 0 ? D1 : B1) + q0 * N1;
            const double *T1 = (jj == 1 ? D1 : B1) + q1 * N1;
            const double *T2 = (jj == 2 ? D1 : B1) + q2 * N1;
            const double *x = xs + i * NB;
            double s2 = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < N1; a2++) {
                double s1 = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < N1; a1++) {
                    const double *xr = x + N1 * (a1 + N1 * a2);
                    double s0 = 0.0;
#pragma unroll
                    for (int a0 = 0; a0 < N1; a0++) s0 = fma(T0[a0], xr[a0], s0);
                    s1 = fma(T1[a1], s0, s1);
                }
                s2 = fma(T2[a2], s1, s2);
            }
            Jq[q * 9 + ij] = s2;
        }
        // first prefetch hop: the next cell's connectivity and coefficients
        int32_t nn = 0;
        T lamn = T(0);
        if (has_next) {
            if (tid < 3 * NB) nn = A.conn[en * NB + ga];
            if constexpr (ELAST)
                if (tid < 2) lamn = mat[2 * en + tid];
        }
        __syncthreads();

        // 2. det J, J^-1, sqrt(w det J) per point
        double Mv[10];
        const int q = tid;
        if (q < NQ) {
            double J[3][3], Ji[3][3];
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int c = 0; c < 3; c++) J[r][c] = Jq[q * 9 + r * 3 + c];
            const double det = inverse3(J, Ji);
            if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
            const double sw = sqrt(wq[q] * (det > 0.0 ? det : 0.0));
#pragma unroll
            for (int jj = 0; jj < 3; jj++)
#pragma unroll
                for (int i = 0; i < 3; i++) Mv[jj * 3 + i] = sw * Ji[jj][i];
            Mv[9] = sw;
        }
        __syncthreads();  // every J read before Mq (same space) is written
        if (q < NQ)
#pragma unroll
            for (int k = 0; k < 10; k++) Mq[q * 10 + k] = Mv[k];
        __syncthreads();

        // 3. the operand: item (q, a1, a2) writes g for a0 = 0..N1-1 and the
        //    NC components; consecutive threads take consecutive points
        for (int it = tid; it < NQ * N1 * N1; it += THREADS) {
            const int qq = it % NQ, a12 = it / NQ, a1 = a12 % N1, a2 = a12 / N1;
            const int q0 = qq % N1, q1 = (qq / N1) % N1, q2 = qq / (N1 * N1);
            const double by = B1[q1 * N1 + a1], bz = B1[q2 * N1 + a2];
            const double *M = Mq + qq * 10;
            double g[NC][N1];
            if constexpr (NC == 1) {
                const double f = M[9] * by * bz;
#pragma unroll
                for (int a0 = 0; a0 < N1; a0++) g[0][a0] = f * B1[q0 * N1 + a0];
            } else {
                // g_c = d0 m_c + d1 m_3+c + d2 m_6+c with d = (dx by bz, bx dy bz,
                // bx by dz), factored: dx (by bz m_c) + bx (dy bz m_3+c + by dz m_6+c)
                const double dy = D1[q1 * N1 + a1], dz = D1[q2 * N1 + a2];
                const double byz = by * bz, dyz = dy * bz, bdz = by * dz;
                double f[3], h[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    f[c] = byz * M[c];
                    h[c] = fma(dyz, M[3 + c], bdz * M[6 + c]);
                }
#pragma unroll
                for (int a0 = 0; a0 < N1; a0++) {
                    const double bx = B1[q0 * N1 + a0], dx = D1[q0 * N1 + a0];
#pragma unroll
                    for (int c = 0; c < 3; c++) g[c][a0] = fma(dx, f[c], bx * h[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int a0 = 0; a0 < N1; a0++) {
                    const int o = (c * NBP + a0 + N1 * a12) * KS + qq;
                    if constexpr (H::NOP == 1) {
                        op[o] = static_cast<OPT>(g[c][a0]);
                    } else {
                        const float x = static_cast<float>(g[c][a0]);
                        const __bf16 h = static_cast<__bf16>(x);
                        op[o] = h;
                        op[H::OP_BYTES / sizeof(OPT) + o] = static_cast<__bf16>(x - static_cast<float>(h));
                    }
                }
        }
        __syncthreads();

        // second prefetch hop: the next cell's coordinates (the empty asm
        // keeps the wait for the connectivity load here)
        double xnext = 0.0;
        if (has_next && tid < 3 * NB) {
            asm volatile("" : "+v"(nn));
            int64_t n = nn;
            if (n < 0 || n >= A.n_nodes) {
                raise_fault(A.flags, FAULT_INDEX);
                n = 0;
            }
            xnext = A.coords[3 * n + gc];
        }

        // 4. this wave's jobs
        {
            T *oc = static_cast<T *>(A.out) + e * static_cast<int64_t>(H::ND) * H::ND;
            const int nj = H::SCHED.n[wave];
            for (int jj = 0; jj < nj; jj++) run_job<H, FORM>(H::SCHED.job[wave][jj], op, oc, buf, lam, mu, lane);
        }

        // park the next cell's data (x is only read in step 1, the
        // coefficients at the top of the loop)
        if (has_next) {
            if (tid < 3 * NB) xs[gc * NB + ga] = xnext;
            if constexpr (ELAST)
                if (tid < 2) lms[tid] = lamn;
        }
        __syncthreads();
        if (!has_next) break;
        e = en;
    }
}

// ---------------------------------------------------------------------------
// Q3 elasticity (per-cell coefficients) with producer and consumer waves.
//
// The operand is split by quadrature points into two halves (points 0..31
// and 32..63), each in its own LDS buffer.  Eight consumer waves keep the
// accumulators of all their jobs' tiles across both halves; four producer
// waves build each half together, 8 points each (their Jacobians, inverses
// and operand columns), synchronising only inside their own wave, at raised
// wave priority since they are on the critical path.  Per cell, two phases
// separated by workgroup barriers:
//   A  consumers multiply on half 0; producers build half 1 of this cell and
//      load the next cell's coordinates and coefficients into the other
//      parity slot;
//   B  consumers multiply on half 1, then write the output of their even job
//      slots; producers build half 0 of the next cell.
// The odd slots' output is written at the start of the next phase A, so a
// cell's stores spread over both phases and drain while the matrix cores
// work.  Every wave executes the same barriers.
template <int MM>
struct Q3WS {
    static constexpr int N1 = 4, NB = 64, NQ = 64, NBP = 64, NT = 4, ND = 192;
    static constexpr bool RAGGED = false;
    using T = typename MMT<MM>::T;
    using ACC = typename MMT<MM>::acc;
    using OPT = typename std::conditional<MM == MM_BF16X3, __bf16, T>::type;
    static constexpr int KP = 32;  // points per half
    static constexpr int KS = op_stride(MM, KP);
    static constexpr int ROWS = 3 * NBP;
    static constexpr int NOP = MM == MM_BF16X3 ? 2 : 1;
    static constexpr int TS = 17;
    static constexpr bool NT_STORE = true;
    static constexpr int OP_BYTES = q2::align16(ROWS * KS * (int)sizeof(OPT));  // one array of one half
    static constexpr int CONS = WAVES, PROD = 4, THREADS = 64 * (CONS + PROD), QW = KP / PROD;
    static constexpr int OFF_TB = 0;                                   // double B1[16], D1[16], w[64]
    static constexpr int OFF_X = OFF_TB + (2 * N1 * N1 + NQ) * 8;      // double xs[2][3][64]
    static constexpr int OFF_LM = OFF_X + 2 * 3 * NB * 8;              // T lm[2][2]
    static constexpr int OFF_GEO = q2::align16(OFF_LM + 4 * 8);        // double geo[PROD][QW][10]
    static constexpr int OFF_OP = q2::align16(OFF_GEO + PROD * QW * 10 * 8);  // OPT op[2][NOP][ROWS][KS]
    static constexpr int OFF_TR = OFF_OP + 2 * NOP * OP_BYTES;         // T tbuf[CONS][16][TS]
    static constexpr int BYTES = q2::align16(OFF_TR + CONS * 16 * TS * (int)sizeof(T));
    static constexpr Sched SCHED = make_sched(FE_FORM_ELASTICITY, NT);
};

constexpr int sched_slots(const Sched &S)
{
    int m = 0;
    for (int w = 0; w < WAVES; w++) m = S.n[w] > m ? S.n[w] : m;
    return m;
}

// largest number of tiles any wave's job in slot jj multiplies
constexpr int slot_cap(const Sched &S, int jj)
{
    int m = 0;
    for (int w = 0; w < WAVES; w++)
        if (jj < S.n[w]) {
            const int k = S.job[w][jj] & 15, t = k == J_DIAG ? 3 : (k == J_PAIR ? 2 : 1);
            m = t > m ? t : m;
        }
    return m;
}

// one half of the depth for the tiles of the job in a slot of capacity CAP
template <int MM, int CAP>
__device__ __forceinline__ void ws_mma(typename Q3WS<MM>::ACC (&acc)[3], uint32_t jb, const typename Q3WS<MM>::OPT *op,
                                       int lane)
{
    using H = Q3WS<MM>;
    const int kind = jb & 15, r = (jb >> 4) & 3, s = (jb >> 6) & 3, i = (jb >> 8) & 15, j = (jb >> 12) & 15;
    if (kind == J_DIAG) {
        if constexpr (CAP >= 3) {
            const int ra[3] = {16 * i, 64 + 16 * i, 128 + 16 * i}, rb[3] = {16 * j, 64 + 16 * j, 128 + 16 * j};
            mma_run<H, 3>(acc, op, ra, rb, 0, H::KP, lane);
        }
    } else if (kind == J_PAIR) {
        if constexpr (CAP >= 2) {
            const int ra[2] = {r * 64 + 16 * i, r * 64 + 16 * j}, rb[2] = {s * 64 + 16 * j, s * 64 + 16 * i};
            mma_run<H, 2>(acc, op, ra, rb, 0, H::KP, lane);
        }
    } else {
        const int ra[1] = {r * 64 + 16 * i}, rb[1] = {s * 64 + 16 * i};
        mma_run<H, 1>(acc, op, ra, rb, 0, H::KP, lane);
    }
}

template <int MM, int CAP>
__device__ __forceinline__ void ws_epi(const typename Q3WS<MM>::ACC (&acc)[3], uint32_t jb, typename Q3WS<MM>::T *oc,
                                       typename Q3WS<MM>::T *buf, typename Q3WS<MM>::T lam, typename Q3WS<MM>::T mu,
                                       int lane)
{
    using H = Q3WS<MM>;
    const int kind = jb & 15, r = (jb >> 4) & 3, s = (jb >> 6) & 3, i = (jb >> 8) & 15, j = (jb >> 12) & 15;
    if (kind == J_DIAG) {
        if constexpr (CAP >= 3) epi_diag<H>(acc, oc, buf, lam, mu, i, j, lane);
    } else if (kind == J_PAIR) {
        if constexpr (CAP >= 2) epi_pair<H>(acc, oc, buf, lam, mu, r, s, i, j, lane);
    } else {
        epi_single<H>(acc[0], oc, buf, lam, mu, r, s, i, lane);
    }
}

// Consumer work of one phase over slots JJ.. of this wave:
//   PH = 0: (write the previous cell's odd slots,) zero, multiply on half 0;
//   PH = 1: multiply on half 1, write the even slots;
//   PH = 2: write the odd slots (after the last cell).
template <int MM, int PH, int JJ>
__device__ __forceinline__ void ws_slots(typename Q3WS<MM>::ACC (&acc)[sched_slots(Q3WS<MM>::SCHED)][3], int wave,
                                         const typename Q3WS<MM>::OPT *op, typename Q3WS<MM>::T *oc,
                                         typename Q3WS<MM>::T *oc_prev, typename Q3WS<MM>::T *buf,
                                         typename Q3WS<MM>::T lam, typename Q3WS<MM>::T mu, int lane)
{
    using H = Q3WS<MM>;
    constexpr int NS = sched_slots(H::SCHED);
    if constexpr (JJ < NS) {
        constexpr int CAP = slot_cap(H::SCHED, JJ);
        if (JJ < H::SCHED.n[wave]) {
            const uint32_t jb = H::SCHED.job[wave][JJ];
            if constexpr (PH == 0) {
                if ((JJ & 1) && oc_prev) ws_epi<MM, CAP>(acc[JJ], jb, oc_prev, buf, lam, mu, lane);
#pragma unroll
                for (int u = 0; u < 3; u++) acc[JJ][u] = typename H::ACC{};
                ws_mma<MM, CAP>(acc[JJ], jb, op, lane);
            } else if constexpr (PH == 1) {
                ws_mma<MM, CAP>(acc[JJ], jb, op, lane);
                if (!(JJ & 1)) ws_epi<MM, CAP>(acc[JJ], jb, oc, buf, lam, mu, lane);
            } else {
                if (JJ & 1) ws_epi<MM, CAP>(acc[JJ], jb, oc, buf, lam, mu, lane);
            }
        }
        ws_slots<MM, PH, JJ + 1>(acc, wave, op, oc, oc_prev, buf, lam, mu, lane);
    }
}

// Producer pw: geometry of the points 32 h + 8 pw .. + 7 of half h of the
// cell whose coordinates are x[3][64], and their columns of the operand
// half opd.
template <int MM>
__device__ __forceinline__ void ws_produce(int pw, int h, const double *x, const double *B1, const double *D1,
                                           const double *wq, double *geo, typename Q3WS<MM>::OPT *opd, int lane,
                                           unsigned *flags)
{
    using H = Q3WS<MM>;
    using OPT = typename H::OPT;
    constexpr int QW = H::QW, KS = H::KS;
    const int cb = QW * pw, qb = H::KP * h + cb;
    // J[i][0..2] at point qb + lane % QW for component i = lane / QW
    if (lane < 3 * QW) {
        const int ql = lane % QW, i = lane / QW, q = qb + ql;
        const int q0 = q & 3, q1 = (q >> 2) & 3, q2 = q >> 4;
        double b0[4], d0[4], b1[4], d1[4], b2[4], d2[4];
#pragma unroll
        for (int a = 0; a < 4; a++) {
            b0[a] = B1[q0 * 4 + a];
            d0[a] = D1[q0 * 4 + a];
            b1[a] = B1[q1 * 4 + a];
            d1[a] = D1[q1 * 4 + a];
            b2[a] = B1[q2 * 4 + a];
            d2[a] = D1[q2 * 4 + a];
        }
        const double *xi = x + 64 * i;
        double j0 = 0.0, j1 = 0.0, j2 = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < 4; a2++) {
            double tdb = 0.0, tbd = 0.0, tbb = 0.0;
#pragma unroll
            for (int a1 = 0; a1 < 4; a1++) {
                const double *xr = xi + 4 * a1 + 16 * a2;
                double sb = 0.0, sd = 0.0;
#pragma unroll
                for (int a0 = 0; a0 < 4; a0++) {
                    sb = fma(b0[a0], xr[a0], sb);
                    sd = fma(d0[a0], xr[a0], sd);
                }
                tdb = fma(b1[a1], sd, tdb);
                tbd = fma(d1[a1], sb, tbd);
                tbb = fma(b1[a1], sb, tbb);
            }
            j0 = fma(b2[a2], tdb, j0);
            j1 = fma(b2[a2], tbd, j1);
            j2 = fma(d2[a2], tbb, j2);
        }
        geo[ql * 10 + i * 3 + 0] = j0;
        geo[ql * 10 + i * 3 + 1] = j1;
        geo[ql * 10 + i * 3 + 2] = j2;
    }
    wave_sync();
    // sqrt(w det J) J^-1 and sqrt(w det J) per point (lane = point)
    if (lane < QW) {
        double J[3][3], Ji[3][3];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c < 3; c++) J[r][c] = geo[lane * 10 + r * 3 + c];
        const double det = inverse3(J, Ji);
        if (!(det > 0.0)) raise_fault(flags, FAULT_DET);
        const double sw = sqrt(wq[qb + lane] * (det > 0.0 ? det : 0.0));
#pragma unroll
        for (int jj = 0; jj < 3; jj++)
#pragma unroll
            for (int c = 0; c < 3; c++) geo[lane * 10 + jj * 3 + c] = sw * Ji[jj][c];
        geo[lane * 10 + 9] = sw;
    }
    wave_sync();
    // operand columns: item (point, a1, a2) writes a0 = 0..3, components 0..2
#pragma unroll
    for (int k = 0; k < QW * 16 / 64; k++) {
        const int it = lane + 64 * k, ql = it % QW, a12 = it / QW, a1 = a12 & 3, a2 = a12 >> 2;
        const int q = qb + ql, q0 = q & 3, q1 = (q >> 2) & 3, q2 = q >> 4;
        const double *M = geo + ql * 10;
        const double by = B1[q1 * 4 + a1], dy = D1[q1 * 4 + a1], bz = B1[q2 * 4 + a2], dz = D1[q2 * 4 + a2];
        double m[9];
#pragma unroll
        for (int t = 0; t < 9; t++) m[t] = M[t];
        const double byz = by * bz, dyz = dy * bz, bdz = by * dz;
#pragma unroll
        for (int a0 = 0; a0 < 4; a0++) {
            const double bx = B1[q0 * 4 + a0], dx = D1[q0 * 4 + a0];
            const double g0 = dx * byz, g1 = bx * dyz, g2 = bx * bdz;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double g = g0 * m[c] + g1 * m[3 + c] + g2 * m[6 + c];
                const int o = (c * 64 + a0 + 4 * a12) * KS + cb + ql;
                if constexpr (H::NOP == 1) {
                    opd[o] = static_cast<OPT>(g);
                } else {
                    const float xf = static_cast<float>(g);
                    const __bf16 h = static_cast<__bf16>(xf);
                    opd[o] = h;
                    opd[H::OP_BYTES / sizeof(OPT) + o] = static_cast<__bf16>(xf - static_cast<float>(h));
                }
            }
        }
    }
}

template <int MM>
__global__ __launch_bounds__(Q3WS<MM>::THREADS, 1) void k_elast_q3ws(ExecArgs A)
{
    using H = Q3WS<MM>;
    using T = typename H::T;
    using OPT = typename H::OPT;
    using ACC = typename H::ACC;
    constexpr int NS = sched_slots(H::SCHED);
    __shared__ __align__(16) unsigned char smem[H::BYTES];
    double *B1 = reinterpret_cast<double *>(smem + H::OFF_TB);
    double *D1 = B1 + 16;
    double *wq = D1 + 16;
    double *xs = reinterpret_cast<double *>(smem + H::OFF_X);  // [2][3][64]
    T *lms = reinterpret_cast<T *>(smem + H::OFF_LM);          // [2][2]
    OPT *op0 = reinterpret_cast<OPT *>(smem + H::OFF_OP);
    OPT *op1 = reinterpret_cast<OPT *>(smem + H::OFF_OP + H::NOP * H::OP_BYTES);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool consumer = wave < H::CONS;
    const int pw = wave - H::CONS;
    double *geo = reinterpret_cast<double *>(smem + H::OFF_GEO) + (consumer ? 0 : pw * H::QW * 10);
    T *buf = reinterpret_cast<T *>(smem + H::OFF_TR) + (consumer ? wave : 0) * 16 * H::TS;

    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    if (e >= e_end) return;  // uniform over the workgroup
    const T *mat = static_cast<const T *>(A.mat);
    T *out = static_cast<T *>(A.out);
    constexpr int64_t NK = 192 * 192;

    for (int k = tid; k < 16; k += H::THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < 64; k += H::THREADS) wq[k] = A.tab.w[k];
    const int pt = tid - 64 * H::CONS;  // producer thread 0..255
    if (!consumer) {
        if (pt < 192) {
            const int a = pt / 3, c = pt - 3 * (pt / 3);
            const int64_t n = checked_node(A.conn, e * 64 + a, A.n_nodes, A.flags);
            xs[c * 64 + a] = A.coords[3 * n + c];
        }
        if (pt < 2) lms[pt] = mat[2 * e + pt];
    }
    __syncthreads();
    if (!consumer) ws_produce<MM>(pw, 0, xs, B1, D1, wq, geo, op0, lane, A.flags);
    __syncthreads();

    // The two roles run separate loops with the same barriers in the same
    // order (the role is uniform per wave), so the consumers' accumulators
    // are not live in the producers' code.
    if (consumer) {
        ACC acc[NS][3];
        T lam = T(0), mu = T(0);
        T *oc_prev = nullptr;
        int par = 0;
        for (;;) {
            const bool has_next = e + stride < e_end;
            T *oc = out + e * NK;
            ws_slots<MM, 0, 0>(acc, wave, op0, oc, oc_prev, buf, lam, mu, lane);
            __syncthreads();
            lam = lms[par * 2];
            mu = lms[par * 2 + 1];
            ws_slots<MM, 1, 0>(acc, wave, op1, oc, nullptr, buf, lam, mu, lane);
            __syncthreads();
            oc_prev = oc;
            if (!has_next) break;
            e += stride;
            par ^= 1;
        }
        ws_slots<MM, 2, 0>(acc, wave, op0, oc_prev, nullptr, buf, lam, mu, lane);
    } else {
        __builtin_amdgcn_s_setprio(2);
        const int a0 = pt / 3, c0 = pt - 3 * (pt / 3);  // this thread's coordinate (pt < 192)
        int par = 0;
        for (;;) {
            const int64_t en = e + stride;
            const bool has_next = en < e_end;
            // the next cell's connectivity and coefficients now, its
            // coordinates after this phase's build; parked at the end
            int32_t nn = 0;
            T l = T(0);
            if (has_next) {
                if (pt < 192) nn = A.conn[en * 64 + a0];
                if (pt < 2) l = mat[2 * en + pt];
            }
            ws_produce<MM>(pw, 1, xs + par * 192, B1, D1, wq, geo, op1, lane, A.flags);
            if (has_next) {
                double xn = 0.0;
                if (pt < 192) {
                    asm volatile("" : "+v"(nn));
                    int64_t n = nn;
                    if (n < 0 || n >= A.n_nodes) {
                        raise_fault(A.flags, FAULT_INDEX);
                        n = 0;
                    }
                    xn = A.coords[3 * n + c0];
                    xs[(par ^ 1) * 192 + c0 * 64 + a0] = xn;
                }
                if (pt < 2) lms[(par ^ 1) * 2 + pt] = l;
            }
            __syncthreads();
            if (has_next) ws_produce<MM>(pw, 0, xs + (par ^ 1) * 192, B1, D1, wq, geo, op0, lane, A.flags);
            __syncthreads();
            if (!has_next) break;
            e = en;
            par ^= 1;
        }
    }
}

template <int MM>
int launch_q3ws(const Plan &, const ExecArgs &A, hipStream_t st)
{
    static std::atomic<int> resident[64];
    return launch_persistent(k_elast_q3ws<MM>, Q3WS<MM>::THREADS, A, st, resident);
}

// ---------------------------------------------------------------------------
// Q2 elasticity (per-cell coefficients) with producer and consumer waves.
//
// The Q2 operand (3 x 32 rows x 28 points) is small enough to keep two of
// them in LDS, so the producers build the WHOLE operand of the next cell
// while the consumers run this cell's jobs, and one workgroup barrier per
// cell hands it over:
//   consumers (8 waves): the k_hexmm jobs of the cell (21 tiles of the
//     blocks r <= s, longest first), each stored straight from the
//     accumulators with its mirrored tiles;
//   producers (4 waves): the geometry and operand columns of the next cell,
//     7 points per wave (J by sum factorization, J^-1, sqrt(w det J)), so
//     each wave synchronises only with itself; then the coordinates of the
//     cell after that are loaded into the other coordinate slot.
// Consumers issue no global loads, so their stores drain while they run the
// next cell (vector-memory counters complete in order: a load after stores
// would wait for them); producers issue no stores.  The operand padding is
// zeroed once, since nothing else is written there.
template <int MM>
struct Q2WS {
    using H = HexMM<2, FE_FORM_ELASTICITY, MM>;
    using T = typename H::T;
    using OPT = typename H::OPT;
    static constexpr int NB = 27, NQ = 27, N1 = 3;
    static constexpr int CONS = WAVES, PROD = 4, THREADS = 64 * (CONS + PROD), PPW = 7;
    static constexpr int OFF_TB = 0;                                  // double B1[9], D1[9], w[27]
    static constexpr int OFF_X = q2::align16(OFF_TB + 45 * 8);        // double xs[2][3][27]
    static constexpr int OFF_LM = q2::align16(OFF_X + 2 * 81 * 8);    // T lm[3][2]
    static constexpr int OFF_GEO = q2::align16(OFF_LM + 6 * 8);       // double geo[PROD][PPW][19]
    static constexpr int OFF_OP = q2::align16(OFF_GEO + PROD * PPW * 19 * 8);  // OPT op[2][NOP][ROWS][KS]
    static constexpr int OFF_TR = OFF_OP + 2 * H::NOP * H::OP_BYTES;  // T tbuf[CONS][16][TS]
    static constexpr int BYTES = q2::align16(OFF_TR + CONS * 16 * H::TS * (int)sizeof(T));
};

// Producer wave pw: geometry and operand columns of points 7 pw .. 7 pw + 6
// (6 for the last wave) of the cell with coordinates x[3][27].  geo holds
// this wave's J[7][9] then M[7][10] = sqrt(w det J) J^-1, sqrt(w det J).
template <int MM>
__device__ __forceinline__ void ws2_produce(int pw, const double *x, const double *B1, const double *D1,
                                            const double *wq, double *geo, typename Q2WS<MM>::OPT *opd, int lane,
                                            unsigned *flags)
{
    using W = Q2WS<MM>;
    using H = typename W::H;
    using OPT = typename W::OPT;
    constexpr int N1 = 3, NB = 27, NBP = H::NBP, KS = H::KS;
    const int np = pw < W::PROD - 1 ? W::PPW : W::NQ - W::PPW * (W::PROD - 1);
    const int qb = W::PPW * pw;
    double *geoJ = geo, *geoM = geo + W::PPW * 9;
    // 1. J[i][j] at point qb + ql: lane = ql + np (3 i + j)
    if (lane < 9 * np) {
        const int ql = lane % np, ij = lane / np, i = ij / 3, jj = ij - 3 * (ij / 3);
        const int q = qb + ql, q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
        const double *T0 = (jj == 0 ? D1 : B1) + q0 * N1;
        const double *T1 = (jj == 1 ? D1 : B1) + q1 * N1;
        const double *T2 = (jj == 2 ? D1 : B1) + q2 * N1;
        const double *xi = x + i * NB;
        double s2 = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < N1; a2++) {
            double s1 = 0.0;
#pragma unroll
            for (int a1 = 0; a1 < N1; a1++) {
                const double *xr = xi + N1 * (a1 + N1 * a2);
                s1 = fma(T1[a1], fma(T0[0], xr[0], fma(T0[1], xr[1], T0[2] * xr[2])), s1);
            }
            s2 = fma(T2[a2], s1, s2);
        }
        geoJ[ql * 9 + ij] = s2;
    }
    wave_sync();
    // 2. det J, J^-1, sqrt(w det J) per point (lane = point)
    if (lane < np) {
        double J[3][3], Ji[3][3];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c < 3; c++) J[r][c] = geoJ[lane * 9 + r * 3 + c];
        const double det = inverse3(J, Ji);
        if (!(det > 0.0)) raise_fault(flags, FAULT_DET);
        const double sw = sqrt(wq[qb + lane] * (det > 0.0 ? det : 0.0));
#pragma unroll
        for (int jj = 0; jj < 3; jj++)
#pragma unroll
            for (int i = 0; i < 3; i++) geoM[lane * 10 + jj * 3 + i] = sw * Ji[jj][i];
        geoM[lane * 10 + 9] = sw;
    }
    wave_sync();
    // 3. operand columns: item (point, a1, a2) writes a0 = 0..2 of the three
    //    components, g_c = dx (by bz m_c) + bx (dy bz m_3+c + by dz m_6+c)
    if (lane < 9 * np) {
        const int ql = lane % np, a12 = lane / np, a1 = a12 % N1, a2 = a12 / N1;
        const int q = qb + ql, q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
        const double *M = geoM + ql * 10;
        const double by = B1[q1 * N1 + a1], bz = B1[q2 * N1 + a2];
        const double dy = D1[q1 * N1 + a1], dz = D1[q2 * N1 + a2];
        const double byz = by * bz, dyz = dy * bz, bdz = by * dz;
        double f[3], h[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            f[c] = byz * M[c];
            h[c] = fma(dyz, M[3 + c], bdz * M[6 + c]);
        }
#pragma unroll
        for (int a0 = 0; a0 < N1; a0++) {
            const double bx = B1[q0 * N1 + a0], dx = D1[q0 * N1 + a0];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double g = fma(dx, f[c], bx * h[c]);
                const int o = (c * NBP + a0 + N1 * a12) * KS + q;
                if constexpr (H::NOP == 1) {
                    opd[o] = static_cast<OPT>(g);
                } else {
                    const float xf = static_cast<float>(g);
                    const __bf16 hb = static_cast<__bf16>(xf);
                    opd[o] = hb;
                    opd[H::OP_BYTES / sizeof(OPT) + o] = static_cast<__bf16>(xf - static_cast<float>(hb));
                }
            }
        }
    }
}

template <int MM>
__global__ __launch_bounds__(Q2WS<MM>::THREADS, 2) void k_elast_q2ws(ExecArgs A)
{
    using W = Q2WS<MM>;
    using H = typename W::H;
    using T = typename W::T;
    using OPT = typename W::OPT;
    constexpr int NB = W::NB;
    constexpr int64_t NK = 81 * 81;
    __shared__ __align__(16) unsigned char smem[W::BYTES];
    double *B1 = reinterpret_cast<double *>(smem + W::OFF_TB);
    double *D1 = B1 + 9;
    double *wq = D1 + 9;
    double *xs = reinterpret_cast<double *>(smem + W::OFF_X);  // [2][3][27]
    T *lms = reinterpret_cast<T *>(smem + W::OFF_LM);          // [3][2]
    OPT *op0 = reinterpret_cast<OPT *>(smem + W::OFF_OP);
    OPT *op1 = reinterpret_cast<OPT *>(smem + W::OFF_OP + H::NOP * H::OP_BYTES);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool consumer = wave < W::CONS;
    const int pw = wave - W::CONS;
    double *geo = reinterpret_cast<double *>(smem + W::OFF_GEO) + (consumer ? 0 : pw * W::PPW * 19);
    T *buf = reinterpret_cast<T *>(smem + W::OFF_TR) + (consumer ? wave : 0) * 16 * H::TS;

    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    if (e >= e_end) return;  // uniform over the workgroup
    const T *mat = static_cast<const T *>(A.mat);
    T *out = static_cast<T *>(A.out);

    for (int k = tid; k < 9; k += W::THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < W::NQ; k += W::THREADS) wq[k] = A.tab.w[k];
    for (int k = tid; k < 2 * H::NOP * H::OP_BYTES / (int)sizeof(OPT); k += W::THREADS) op0[k] = OPT(0);
    const int pt = tid - 64 * W::CONS;  // producer thread 0..255
    const int a0 = pt / 3, c0 = pt - 3 * (pt / 3);  // its coordinate (pt < 81)
    if (!consumer) {
        // the first two cells' coordinates and coefficients
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int64_t es = e + s * stride;
            if (es < e_end) {
                if (pt < 3 * NB) {
                    const int64_t n = checked_node(A.conn, es * NB + a0, A.n_nodes, A.flags);
                    xs[s * 81 + c0 * NB + a0] = A.coords[3 * n + c0];
                }
                if (pt < 2) lms[s * 2 + pt] = mat[2 * es + pt];
            }
        }
    }
    __syncthreads();
    if (!consumer) ws2_produce<MM>(pw, xs, B1, D1, wq, geo, op0, lane, A.flags);
    __syncthreads();

    // The two roles run separate loops with the same barriers in the same
    // order (the role is uniform per wave).  Cell k of this workgroup uses
    // operand slot k % 2, coordinate slot k % 2 and coefficient slot k % 3.
    int k = 0;
    if (consumer) {
        const int nj = H::SCHED.n[wave];
        for (;;) {
            const bool has_next = e + stride < e_end;
            const int slot = k % 3;
            const T lam = lms[slot * 2], mu = lms[slot * 2 + 1];
            const OPT *op = (k & 1) ? op1 : op0;
            T *oc = out + e * NK;
            for (int jj = 0; jj < nj; jj++)
                run_job<H, FE_FORM_ELASTICITY>(H::SCHED.job[wave][jj], op, oc, buf, lam, mu, lane);
            __syncthreads();
            if (!has_next) break;
            e += stride;
            k++;
        }
    } else {
        __builtin_amdgcn_s_setprio(2);
        for (;;) {
            const int64_t en = e + stride, enn = en + stride;
            const bool has_next = en < e_end, has_nn = enn < e_end;
            const int par = k & 1;
            // the connectivity and coefficients of cell k + 2 now, its
            // coordinates after the build (the empty asm keeps the wait for
            // the connectivity there)
            int32_t nn = 0;
            T l = T(0);
            if (has_nn) {
                if (pt < 3 * NB) nn = A.conn[enn * NB + a0];
                if (pt < 2) l = mat[2 * enn + pt];
            }
            if (has_next) ws2_produce<MM>(pw, xs + (par ^ 1) * 81, B1, D1, wq, geo, par ? op0 : op1, lane, A.flags);
            if (has_nn) {
                if (pt < 3 * NB) {
                    asm volatile("" : "+v"(nn));
                    int64_t n = nn;
                    if (n < 0 || n >= A.n_nodes) {
                        raise_fault(A.flags, FAULT_INDEX);
                        n = 0;
                    }
                    xs[par * 81 + c0 * NB + a0] = A.coords[3 * n + c0];
                }
                if (pt < 2) lms[((k + 2) % 3) * 2 + pt] = l;
            }
            __syncthreads();
            if (!has_next) break;
            e = en;
            k++;
        }
    }
}

template <int MM>
int launch_q2ws(const Plan &, const ExecArgs &A, hipStream_t st)
{
    static std::atomic<int> resident[64];
    return launch_persistent(k_elast_q2ws<MM>, Q2WS<MM>::THREADS, A, st, resident);
}

template <int P, int FORM, int MM>
int launch_hexmm(const Plan &, const ExecArgs &A, hipStream_t st)
{
    static std::atomic<int> resident[64];
    return launch_persistent(k_hexmm<P, FORM, MM>, THREADS, A, st, resident);
}

// ---------------------------------------------------------------------------
// Q4 and Q5: the same products with the quadrature points taken in chunks.
//
// At p = 4, 5 the operand g (3 (p+1)^3 rows x (p+1)^3 points) no longer fits
// in LDS (Q5, FP64: 1.2 MB), so only a chunk of KC points of it is built at a
// time (FP64 16, FP32 and BF16X3 32).  The geometry (sqrt(w det J) J^-1 at
// every point, FP64) is computed once per cell; the operand chunks are
// rebuilt from it.  The jobs are the tiles of k_hexmm, grouped by kind into
// passes small enough for their accumulators to stay in registers across
// all chunks (16 FP64 / 32 FP32 tiles per wave):
//   for each pass:  for each chunk: build it; barrier; every wave adds the
//                   chunk's products to its jobs' accumulators; barrier
//                   then every wave runs its jobs' epilogues
// Every wave of a pass carries the same number of job slots, so the
// products are straight-line code; slots beyond a wave's jobs multiply
// operand rows 0 and are never stored.  Laplace jobs sum the three
// gradient components into one accumulator.
constexpr int mc_cap(int mm) { return mm == MM_F32 ? 32 : 16; }  // accumulator tiles per wave
constexpr int mc_kc(int mm) { return mm == MM_F64 ? 16 : 32; }   // points per chunk
constexpr int kind_na(int kind) { return kind == J_DIAG ? 3 : (kind == J_PAIR ? 2 : 1); }
constexpr int kind_nprod(int kind) { return kind == J_DIAG || kind == J_LAP ? 3 : (kind == J_PAIR ? 2 : 1); }

constexpr int MC_PASSES = 12, MC_JOBS = 32;
struct MCSched {
    int ng;             // job kinds (groups of passes)
    int kind[3], nj[3];  // kind and job slots per wave of each group
    int p0[3], np[3];   // first pass and passes of each group
    uint8_t n[MC_PASSES][WAVES];
    uint32_t job[MC_PASSES][WAVES][MC_JOBS];
};

constexpr MCSched make_mc_sched(int form, int nt, int cap)
{
    MCSched S{};
    int kinds[3] = {J_LAP, 0, 0}, nk = 1;
    if (form == FE_FORM_ELASTICITY) {
        kinds[0] = J_DIAG;
        kinds[1] = J_PAIR;
        kinds[2] = J_SINGLE;
        nk = 3;
    } else if (form != FE_FORM_LAPLACE) {
        kinds[0] = J_MASS;
    }
    int npass = 0;
    for (int g = 0; g < nk; g++) {
        const int kind = kinds[g];
        uint32_t jobs[320] = {};
        int nj = 0;
        if (kind == J_PAIR) {
            for (int r = 0; r < 3; r++)
                for (int s = r + 1; s < 3; s++)
                    for (int i = 0; i < nt; i++)
                        for (int j = i + 1; j < nt; j++) jobs[nj++] = enc(J_PAIR, r, s, i, j);
        } else if (kind == J_SINGLE) {
            for (int r = 0; r < 3; r++)
                for (int s = r + 1; s < 3; s++)
                    for (int i = 0; i < nt; i++) jobs[nj++] = enc(J_SINGLE, r, s, i, i);
        } else {
            for (int i = 0; i < nt; i++)
                for (int j = i; j < nt; j++) jobs[nj++] = enc(kind, 0, 0, i, j);
        }
        const int capj = cap / kind_na(kind);
        const int np = (nj + WAVES * capj - 1) / (WAVES * capj);
        S.kind[g] = kind;
        S.np[g] = np;
        S.nj[g] = (nj + WAVES * np - 1) / (WAVES * np);
        S.p0[g] = npass;
        for (int p = 0; p < np; p++, npass++) {
            const int lo = p * nj / np, hi = (p + 1) * nj / np;
            for (int k = lo; k < hi; k++) {
                const int w = (k - lo) % WAVES;
                S.job[npass][w][S.n[npass][w]++] = jobs[k];
            }
        }
    }
    S.ng = nk;
    return S;
}

template <int P, int FORM, int MM>
struct HexMC {
    static constexpr int N1 = P + 1, NB = N1 * N1 * N1, NQ = NB;
    static constexpr bool MASSF = FORM == FE_FORM_MASS || FORM == FE_FORM_VMASS;
    static constexpr int NC = MASSF ? 1 : 3;
    static constexpr int NCO = form_nc(FORM);
    static constexpr int ND = NCO * NB;
    static constexpr int NBP = align_to(NB, 16), NT = NBP / 16;
    static constexpr bool RAGGED = NB % 16 != 0;
    using T = typename MMT<MM>::T;
    using ACC = typename MMT<MM>::acc;
    using OPT = typename std::conditional<MM == MM_BF16X3, __bf16, T>::type;
    static constexpr int KC = mc_kc(MM), NCH = (NQ + KC - 1) / KC;
    static constexpr int KSTEP = MM == MM_BF16X3 ? 32 : 4;
    static constexpr int KS = op_stride(MM, KC);
    static constexpr int ROWS = NC * NBP;
    static constexpr int NOP = MM == MM_BF16X3 ? 2 : 1;
    static constexpr int OP_N = ROWS * KS;  // entries of one operand array
    static constexpr int TS = 17;
    // plain stores: a 16-entry row segment of these matrices straddles two
    // 128-byte lines (rows of 375 or 648 entries, blocks starting at
    // multiples of 125 or 216), and the L2 joins the halves written by
    // neighbouring tiles before they go out (measured: Q4 elasticity 30 %
    // faster in FP32 than with nontemporal stores)
    static constexpr bool NT_STORE = false;
    static constexpr int OFF_TB = 0;  // double B1[N1][N1], D1[N1][N1], w[NQ]
    static constexpr int OFF_X = q2::align16(OFF_TB + (2 * N1 * N1 + NQ) * 8);  // double xs[3][NB], T lm[2]
    static constexpr int OFF_G = q2::align16(OFF_X + 3 * NB * 8 + 16);          // double [NQ][10] (J: [NQ][9])
    static constexpr int OFF_OP = q2::align16(OFF_G + NQ * 10 * 8);
    static constexpr int OFF_TR = q2::align16(OFF_OP + NOP * OP_N * (int)sizeof(OPT));
    static constexpr int BYTES = q2::align16(OFF_TR + WAVES * 16 * TS * (int)sizeof(T));
    static constexpr MCSched SCHED = make_mc_sched(FORM == FE_FORM_VMASS ? FE_FORM_MASS : FORM, NT, mc_cap(MM));
    static_assert(BYTES <= 160 * 1024, "LDS");
};

// Operand chunk ch: columns = points ch*KC .. ch*KC+KC-1 (zero beyond NQ),
// rows (c, a) for a < NB; item (point, a1, a2) writes a0 = 0..N1-1.
template <class H>
__device__ __forceinline__ void mc_build(typename H::OPT *op, const double *Mq, const double *B1, const double *D1,
                                         int ch, int tid)
{
    using OPT = typename H::OPT;
    constexpr int N1 = H::N1, NQ = H::NQ, NC = H::NC, NBP = H::NBP, KS = H::KS, KC = H::KC;
    auto put = [&](int c, int a0, int a12, int ql, double x) {
        const int o = (c * NBP + a0 + N1 * a12) * KS + ql;
        if constexpr (H::NOP == 1) {
            op[o] = static_cast<OPT>(x);
        } else {
            const float f = static_cast<float>(x);
            const __bf16 h = static_cast<__bf16>(f);
            op[o] = h;
            op[H::OP_N + o] = static_cast<__bf16>(f - static_cast<float>(h));
        }
    };
    for (int it = tid; it < KC * N1 * N1; it += THREADS) {
        const int ql = it % KC, a12 = it / KC, a1 = a12 % N1, a2 = a12 / N1;
        const int qq = ch * KC + ql;
        if (qq < NQ) {
            const int q0 = qq % N1, q1 = (qq / N1) % N1, q2 = qq / (N1 * N1);
            const double by = B1[q1 * N1 + a1], bz = B1[q2 * N1 + a2];
            const double *M = Mq + qq * 10;
            if constexpr (NC == 1) {
                const double f = M[9] * by * bz;
#pragma unroll
                for (int a0 = 0; a0 < N1; a0++) put(0, a0, a12, ql, f * B1[q0 * N1 + a0]);
            } else {
                // factored as in the one-pass build above
                const double dy = D1[q1 * N1 + a1], dz = D1[q2 * N1 + a2];
                const double byz = by * bz, dyz = dy * bz, bdz = by * dz;
                double f[3], h[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    f[c] = byz * M[c];
                    h[c] = fma(dyz, M[3 + c], bdz * M[6 + c]);
                }
#pragma unroll
                for (int a0 = 0; a0 < N1; a0++) {
                    const double bx = B1[q0 * N1 + a0], dx = D1[q0 * N1 + a0];
#pragma unroll
                    for (int c = 0; c < 3; c++) put(c, a0, a12, ql, fma(dx, f[c], bx * h[c]));
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int a0 = 0; a0 < N1; a0++) put(c, a0, a12, ql, 0.0);
        }
    }
}

// accumulator of product u = m * NJ + jj (m-th product of job slot jj)
template <int KIND, int NJ>
constexpr int mc_acc(int u)
{
    return KIND == J_DIAG ? (u % NJ) * 3 + u / NJ : (KIND == J_PAIR ? (u % NJ) * 2 + u / NJ : u % NJ);
}

// Operand rows of product u: a base row per job (two for PAIR, whose
// products differ in their tiles) plus, for DIAG and LAP, the component
// block m * NBP as a compile-time offset.
constexpr int mc_nbase(int kind) { return kind == J_PAIR ? 2 : 1; }
template <class H, int KIND, int NJ>
constexpr int mc_base(int u)
{
    return KIND == J_PAIR ? (u / NJ) * NJ + u % NJ : u % NJ;
}
template <class H, int KIND, int NJ>
constexpr int mc_ofs(int u)
{
    return KIND == J_DIAG || KIND == J_LAP ? (u / NJ) * H::NBP : 0;
}

// The products of one chunk: acc[mc_acc(u)] += g[ra[u]..][chunk] g[rb[u]..][chunk]^T
// for u < NS, in groups of G products whose fragments are loaded while the
// previous group multiplies.
template <class H, int KIND, int NJ>
__device__ __forceinline__ void mc_mma(typename H::ACC *acc, const typename H::OPT *op, const int *ra, const int *rb,
                                       int lane)
{
    using OPT = typename H::OPT;
    constexpr int NS = NJ * kind_nprod(KIND);
    constexpr int KS = H::KS, NSTEP = H::KC / H::KSTEP;
    const int m = lane & 15, grp = lane >> 4;
    if constexpr (H::NOP == 1) {
        // k steps in a loop, the groups of one step unrolled; the first
        // group of a step is loaded at its top
        constexpr int G = sizeof(OPT) == 8 ? 4 : 8;
        constexpr int NG = (NS + G - 1) / G;
        OPT a[2][G], b[2][G];
        auto load = [&](int buf, int g, int k) {
#pragma unroll
            for (int v = 0; v < G; v++)
                if (g * G + v < NS) {
                    const int u = g * G + v;
                    a[buf][v] = op[(ra[mc_base<H, KIND, NJ>(u)] + mc_ofs<H, KIND, NJ>(u) + m) * KS + k];
                    b[buf][v] = op[(rb[mc_base<H, KIND, NJ>(u)] + mc_ofs<H, KIND, NJ>(u) + m) * KS + k];
                }
        };
        auto mfma = [&](int buf, int g) {
#pragma unroll
            for (int v = 0; v < G; v++)
                if (g * G + v < NS) {
                    const int x = mc_acc<KIND, NJ>(g * G + v);
                    if constexpr (sizeof(OPT) == 8)
                        acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[buf][v], b[buf][v], acc[x], 0, 0, 0);
                    else
                        acc[x] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[buf][v], b[buf][v], acc[x], 0, 0, 0);
                }
        };
        for (int st = 0; st < NSTEP; st++) {
            const int k = 4 * st + grp;
            load(0, 0, k);
#pragma unroll
            for (int g = 0; g < NG; g++) {
                if (g + 1 < NG) load((g + 1) & 1, g + 1, k);
                __builtin_amdgcn_sched_barrier(0);
                mfma(g & 1, g);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        const OPT *lo = op + H::OP_N;
        constexpr int G = 2, NG = (NS + G - 1) / G;
        bf8 ah[2][G], al[2][G], bh[2][G], bl[2][G];
        auto load = [&](int buf, int it) {
            const int g0 = it * G;
#pragma unroll
            for (int v = 0; v < G; v++)
                if (g0 + v < NS) {
                    const int u = g0 + v;
                    const int oa = (ra[mc_base<H, KIND, NJ>(u)] + mc_ofs<H, KIND, NJ>(u) + m) * KS + 8 * grp;
                    const int ob = (rb[mc_base<H, KIND, NJ>(u)] + mc_ofs<H, KIND, NJ>(u) + m) * KS + 8 * grp;
                    ah[buf][v] = *reinterpret_cast<const bf8 *>(op + oa);
                    al[buf][v] = *reinterpret_cast<const bf8 *>(lo + oa);
                    bh[buf][v] = *reinterpret_cast<const bf8 *>(op + ob);
                    bl[buf][v] = *reinterpret_cast<const bf8 *>(lo + ob);
                }
        };
        auto mfma = [&](int buf, int it) {
            const int g0 = it * G;
#pragma unroll
            for (int v = 0; v < G; v++)
                if (g0 + v < NS) {
                    const int x = mc_acc<KIND, NJ>(g0 + v);
                    acc[x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[buf][v], bh[buf][v], acc[x], 0, 0, 0);
                    acc[x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[buf][v], bl[buf][v], acc[x], 0, 0, 0);
                    acc[x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[buf][v], bh[buf][v], acc[x], 0, 0, 0);
                }
        };
        load(0, 0);
#pragma unroll
        for (int it = 0; it < NG; it++) {
            if (it + 1 < NG) load((it + 1) & 1, it + 1);
            __builtin_amdgcn_sched_barrier(0);
            mfma(it & 1, it);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// One pass (jobs of one kind, NJ slots per wave) over all chunks of the cell.
template <class H, int FORM, int KIND, int NJ>
__device__ __forceinline__ void mc_pass(int ps, typename H::OPT *op, const double *Mq, const double *B1,
                                        const double *D1, typename H::T *oc, typename H::T *buf, typename H::T lam,
                                        typename H::T mu, int wave, int tid, int lane)
{
    using ACC = typename H::ACC;
    constexpr int NBP = H::NBP;
    const int nw = H::SCHED.n[ps][wave];
    constexpr int NBS = mc_nbase(KIND);
    int ra[NJ * NBS], rb[NJ * NBS];
#pragma unroll
    for (int jj = 0; jj < NJ; jj++) {
        const uint32_t jb = jj < nw ? H::SCHED.job[ps][wave][jj] : 0u;
        const int r = (jb >> 4) & 3, s = (jb >> 6) & 3, i = (jb >> 8) & 15, j = (jb >> 12) & 15;
        if constexpr (KIND == J_DIAG || KIND == J_LAP || KIND == J_MASS) {
            ra[jj] = 16 * i;
            rb[jj] = 16 * j;
        } else if constexpr (KIND == J_PAIR) {
            ra[jj] = r * NBP + 16 * i;
            rb[jj] = s * NBP + 16 * j;
            ra[NJ + jj] = r * NBP + 16 * j;
            rb[NJ + jj] = s * NBP + 16 * i;
        } else {
            ra[jj] = r * NBP + 16 * i;
            rb[jj] = s * NBP + 16 * i;
        }
    }
    ACC acc[NJ * kind_na(KIND)];
#pragma unroll
    for (int x = 0; x < NJ * kind_na(KIND); x++) acc[x] = ACC{};
    for (int ch = 0; ch < H::NCH; ch++) {
        mc_build<H>(op, Mq, B1, D1, ch, tid);
        __syncthreads();
        mc_mma<H, KIND, NJ>(acc, op, ra, rb, lane);
        __syncthreads();
    }
#pragma unroll
    for (int jj = 0; jj < NJ; jj++) {
        if (jj >= nw) continue;
        const uint32_t jb = H::SCHED.job[ps][wave][jj];
        const int r = (jb >> 4) & 3, s = (jb >> 6) & 3, i = (jb >> 8) & 15, j = (jb >> 12) & 15;
        if constexpr (KIND == J_DIAG) {
            epi_diag<H>(acc + 3 * jj, oc, buf, lam, mu, i, j, lane);
        } else if constexpr (KIND == J_PAIR) {
            epi_pair<H>(acc + 2 * jj, oc, buf, lam, mu, r, s, i, j, lane);
        } else if constexpr (KIND == J_SINGLE) {
            epi_single<H>(acc[jj], oc, buf, lam, mu, r, s, i, lane);
        } else if constexpr (KIND == J_LAP) {
            epi_lap<H>(acc[jj], oc, buf, i, j, lane);
        } else {
            epi_mass<H, FORM>(acc[jj], oc, buf, i, j, lane);
        }
    }
}

template <class H, int FORM, int G>
__device__ __forceinline__ void mc_group(typename H::OPT *op, const double *Mq, const double *B1, const double *D1,
                                         typename H::T *oc, typename H::T *buf, typename H::T lam, typename H::T mu,
                                         int wave, int tid, int lane)
{
    if constexpr (G < H::SCHED.ng) {
        constexpr int KIND = H::SCHED.kind[G], NJ = H::SCHED.nj[G];
        for (int p = 0; p < H::SCHED.np[G]; p++)
            mc_pass<H, FORM, KIND, NJ>(H::SCHED.p0[G] + p, op, Mq, B1, D1, oc, buf, lam, mu, wave, tid, lane);
    }
}

template <int P, int FORM, int MM>
__global__ __launch_bounds__(THREADS, 1) void k_hexmc(ExecArgs A)
{
    using H = HexMC<P, FORM, MM>;
    using T = typename H::T;
    using OPT = typename H::OPT;
    constexpr int N1 = H::N1, NB = H::NB, NQ = H::NQ, NC = H::NC, NBP = H::NBP, KS = H::KS;
    constexpr bool ELAST = FORM == FE_FORM_ELASTICITY;
    __shared__ __align__(16) unsigned char smem[H::BYTES];
    double *B1 = reinterpret_cast<double *>(smem + H::OFF_TB);
    double *D1 = B1 + N1 * N1;
    double *wq = D1 + N1 * N1;
    double *xs = reinterpret_cast<double *>(smem + H::OFF_X);  // [3][NB]
    T *lms = reinterpret_cast<T *>(xs + 3 * NB);
    double *Jq = reinterpret_cast<double *>(smem + H::OFF_G);  // [NQ][9]
    double *Mq = Jq;                                           // [NQ][10]: sqrt(wd) J^-1, sqrt(wd)
    OPT *op = reinterpret_cast<OPT *>(smem + H::OFF_OP);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    T *buf = reinterpret_cast<T *>(smem + H::OFF_TR) + wave * 16 * H::TS;

    int64_t e, e_end, stride;
    cell_range(A.xcd_remap, A.n_cells, e, e_end, stride);
    if (e >= e_end) return;  // uniform over the workgroup
    const T *mat = static_cast<const T *>(A.mat);

    for (int k = tid; k < N1 * N1; k += THREADS) {
        B1[k] = A.tab.B1[k];
        D1[k] = A.tab.D1[k];
    }
    for (int k = tid; k < NQ; k += THREADS) wq[k] = A.tab.w[k];
    // padding rows a = NB .. NBP-1 of every component stay zero
    for (int k = tid; k < H::NOP * NC * (NBP - NB) * KS; k += THREADS) {
        const int arr = k / (NC * (NBP - NB) * KS), rem = k - arr * (NC * (NBP - NB) * KS);
        const int rr = rem / KS, c = rr / (NBP - NB), a = NB + rr - c * (NBP - NB);
        op[arr * H::OP_N + (c * NBP + a) * KS + rem - rr * KS] = OPT(0);
    }

    for (; e < e_end; e += stride) {
        // coordinates relative to the cell's first node: J is unchanged (the
        // basis gradients sum to zero) but no longer formed by cancelling
        // terms of the size of |x| when the cell lies far from the origin
        for (int k = tid; k < 3 * NB; k += THREADS) {
            const int a = k / 3, c = k - 3 * a;
            const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
            const int64_t n0 = checked_node(A.conn, e * NB, A.n_nodes, A.flags);
            xs[c * NB + a] = A.coords[3 * n + c] - A.coords[3 * n0 + c];
        }
        if constexpr (ELAST)
            if (tid < 2) lms[tid] = mat[2 * e + tid];
        __syncthreads();
        T lam = T(0), mu = T(0);
        if constexpr (ELAST) {
            lam = lms[0];
            mu = lms[1];
        }
        // J[i][j] at each point by sum factorization over the 1-D tables
        for (int it = tid; it < NQ * 9; it += THREADS) {
            const int q = it % NQ, ij = it / NQ, i = ij / 3, jj = ij - 3 * (ij / 3);
            const int q0 = q % N1, q1 = (q / N1) % N1, q2 = q / (N1 * N1);
            const double *T0 = (jj == 0 ? D1 : B1) + q0 * N1;
            const double *T1 = (jj == 1 ? D1 : B1) + q1 * N1;
            const double *T2 = (jj == 2 ? D1 : B1) + q2 * N1;
            const double *x = xs + i * NB;
            double s2 = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < N1; a2++) {
                double s1 = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < N1; a1++) {
                    const double *xr = x + N1 * (a1 + N1 * a2);
                    double s0 = 0.0;
#pragma unroll
                    for (int a0 = 0; a0 < N1; a0++) s0 = fma(T0[a0], xr[a0], s0);
                    s1 = fma(T1[a1], s0, s1);
                }
                s2 = fma(T2[a2], s1, s2);
            }
            Jq[q * 9 + ij] = s2;
        }
        __syncthreads();
        // det J, J^-1, sqrt(w det J) per point
        double Mv[10];
        const int q = tid;
        if (q < NQ) {
            double J[3][3], Ji[3][3];
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int c = 0; c < 3; c++) J[r][c] = Jq[q * 9 + r * 3 + c];
            const double det = inverse3(J, Ji);
            if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
            const double sw = sqrt(wq[q] * (det > 0.0 ? det : 0.0));
#pragma unroll
            for (int jj = 0; jj < 3; jj++)
#pragma unroll
                for (int i = 0; i < 3; i++) Mv[jj * 3 + i] = sw * Ji[jj][i];
            Mv[9] = sw;
        }
        __syncthreads();  // every J read before Mq (same space) is written
        if (q < NQ)
#pragma unroll
            for (int k = 0; k < 10; k++) Mq[q * 10 + k] = Mv[k];
        __syncthreads();

        T *oc = static_cast<T *>(A.out) + e * static_cast<int64_t>(H::ND) * H::ND;
        mc_group<H, FORM, 0>(op, Mq, B1, D1, oc, buf, lam, mu, wave, tid, lane);
        mc_group<H, FORM, 1>(op, Mq, B1, D1, oc, buf, lam, mu, wave, tid, lane);
        mc_group<H, FORM, 2>(op, Mq, B1, D1, oc, buf, lam, mu, wave, tid, lane);
        // the last chunk's barrier has passed: x and Mq may be rewritten
    }
}

template <int P, int FORM, int MM>
int launch_hexmc(const Plan &, const ExecArgs &A, hipStream_t st)
{
    static std::atomic<int> resident[64];
    return launch_persistent(k_hexmc<P, FORM, MM>, THREADS, A, st, resident);
}

template <int P, int MM>
LaunchFn pick_form_mc(const Plan &p)
{
    switch (p.form) {
    case FE_FORM_MASS: return launch_hexmc<P, FE_FORM_MASS, MM>;
    case FE_FORM_VMASS: return launch_hexmc<P, FE_FORM_VMASS, MM>;
    case FE_FORM_LAPLACE: return launch_hexmc<P, FE_FORM_LAPLACE, MM>;
    case FE_FORM_ELASTICITY:
        if (p.mat_kind != FE_MAT_ISO_CELL) return nullptr;
        return launch_hexmc<P, FE_FORM_ELASTICITY, MM>;
    }
    return nullptr;
}

template <int P, int MM>
LaunchFn pick_form(const Plan &p)
{
    switch (p.form) {
    case FE_FORM_MASS: return launch_hexmm<P, FE_FORM_MASS, MM>;
    case FE_FORM_VMASS: return launch_hexmm<P, FE_FORM_VMASS, MM>;
    case FE_FORM_LAPLACE: return launch_hexmm<P, FE_FORM_LAPLACE, MM>;
    case FE_FORM_ELASTICITY:
        if (p.mat_kind != FE_MAT_ISO_CELL) return nullptr;
        if constexpr (P == 3) return launch_q3ws<MM>;
        return launch_hexmm<P, FE_FORM_ELASTICITY, MM>;
    }
    return nullptr;
}

template <int MM>
LaunchFn pick_order(const Plan &p)
{
    if (p.order == 2) return pick_form<2, MM>(p);
    if (p.order == 3) return pick_form<3, MM>(p);
    if (p.order == 4) return pick_form_mc<4, MM>(p);
    if (p.order == 5) return pick_form_mc<5, MM>(p);
    return nullptr;
}

}  // namespace

LaunchFn select_q2ws(const Plan &p)
{
    if (p.cell != FE_CELL_HEX || p.order != 2 || p.mode != FE_MODE_MATRIX || p.form != FE_FORM_ELASTICITY ||
        p.mat_kind != FE_MAT_ISO_CELL)
        return nullptr;
    if (p.prec == FE_PREC_FP64) return launch_q2ws<MM_F64>;
    if (p.prec == FE_PREC_FP32) return launch_q2ws<MM_F32>;
    if (p.prec == FE_PREC_BF16X3) return launch_q2ws<MM_BF16X3>;
    return nullptr;
}

LaunchFn select_hexmm(const Plan &p)
{
    if (p.cell != FE_CELL_HEX || p.mode != FE_MODE_MATRIX) return nullptr;
    if (p.prec == FE_PREC_FP64) return pick_order<MM_F64>(p);
    if (p.prec == FE_PREC_FP32) return pick_order<MM_F32>(p);
    if (p.prec == FE_PREC_BF16X3) return pick_order<MM_BF16X3>(p);
    return nullptr;
}

}  // namespace fe
