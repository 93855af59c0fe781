// Q2 hexahedron linear-elasticity cell routines on the matrix cores (shared
// by the single-form kernel and the batched kernel).  See k_mfma.hip for the
// method.
#pragma once

#include <type_traits>
#include <utility>

#include "fe_device.h"

namespace fe {
namespace q2 {


typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum { MM_F64 = 0, MM_F32 = 1, MM_BF16X3 = 2 };

template <int MM>
struct MMT {
    using T = float;
    using acc = f4;
};
template <>
struct MMT<MM_F64> {
    using T = double;
    using acc = d4;
};

constexpr int align16(int x) { return (x + 15) & ~15; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Q2 hexahedron
constexpr int NB = 27, NQ = 27, ND = 81, NK = ND * ND;

// ---------------------------------------------------------------------------
// Staged routine (FP64, FP32): the tiles of the blocks r <= s of P on the
// matrix cores, P to LDS, K from P in place, a linear flush.
template <int MM>
struct Q2Staged {
    using T = typename MMT<MM>::T;
    static constexpr int VEC = 16 / (int)sizeof(T);       // entries per 16-byte store
    static constexpr int KP = 28;                          // padded K (quadrature points)
    static_assert(MM == MM_F64 || MM == MM_F32, "the staged routine runs FP64 and FP32");
    // kept for the whole launch: 1-D tables and weights
    static constexpr int OFF_TB = 0;                      // double B1[9], D1[9], w[27]
    // the next cell's coordinates and coefficients, parked before the flush
    // (coordinates component-major: xn[3][28], node a of axis i at 28 i + a)
    static constexpr int OFF_N = align16(OFF_TB + (9 + 9 + NQ) * 8);  // double xn[3][28], T lmn[2]
    static constexpr int OFF_U = align16(OFF_N + 3 * 28 * 8 + 2 * 8);
    // JOUT: J and w det J lie outside the staging area, so a cell's J phase
    // may start while other waves still flush the previous cell (FP32; the
    // FP64 layout has no room for it within three workgroups per CU)
    static constexpr bool JOUT = MM == MM_F32;
    // phase A (per cell): geometry and GEMM operand
    static constexpr int OFF_J = OFF_U;                   // double J[27][9]
    static constexpr int OFF_WD = OFF_J + NQ * 9 * 8;     // double wd[28]
    // GEMM operand, transposed: row = i*33 + a (component i, basis a; rows
    // a = 27..32 are padding), column = quadrature point k, row stride KS.
    // Lanes of one MFMA fragment read 16 consecutive rows at four
    // consecutive k: with 32 four-byte LDS banks that is conflict-free for
    // an odd stride in FP64 and a stride of 2 mod 4 in FP32.
    static constexpr int KS = MM == MM_F64 ? KP + 1 : KP + 2;
    static constexpr int GROWS = 3 * 33;
    static constexpr int OFF_G = align16(OFF_WD + 28 * 8);  // T Gs[GROWS][KS]
    static constexpr int END_A = OFF_G + GROWS * KS * (int)sizeof(T);
    // phase B (aliases A, or only the operand with JOUT): the cell's matrix
    // row-major, shifted to the output alignment; it first holds the blocks
    // r <= s of P in their places
    static constexpr int OFF_K = JOUT ? OFF_G : OFF_U;
    static constexpr int END_B = OFF_K + (NK + VEC) * (int)sizeof(T);
    static constexpr int BYTES = align16(cmax(END_A, END_B));
    // 16-byte vectors of the staged matrix per thread in the flush
    static constexpr int NV = ((NK + 2 * VEC - 1) / VEC + 255) / 256;
};


// Persistent schedule: every workgroup walks a strided list of cells.  With
// XCD remapping, the 8 XCDs (hardware workgroup id modulo 8) own 8
// contiguous ranges of cells, so cells that share nodes meet in one L2.
__device__ __forceinline__ void cell_range(int remap, int64_t n, int64_t &first, int64_t &end, int64_t &stride)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (!remap || G < 8 || (G & 7)) {
        first = b;
        end = n;
        stride = G;
        return;
    }
    const int x = b & 7, j = b >> 3, per = G >> 3;
    const int64_t chunk = (n + 7) / 8;
    const int64_t lo = x * chunk;
    first = lo + j;
    end = lo + chunk < n ? lo + chunk : n;
    stride = per;
}

// Column c of adj J (J row-major at Jp) and det J: the column is the cross
// product of rows c+1 and c+2 (mod 3), det J its dot product with row c.
__device__ __forceinline__ void q2_adj_column(const double *Jp, int c, double (&adjc)[3], double &det)
{
    const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
    const double *R0 = Jp + 3 * c, *R1 = Jp + 3 * c1, *R2 = Jp + 3 * c2;
    const double x0 = R0[0], x1 = R0[1], x2 = R0[2];
    const double y0 = R1[0], y1 = R1[1], y2 = R1[2];
    const double z0 = R2[0], z1 = R2[1], z2 = R2[2];
    adjc[0] = y1 * z2 - y2 * z1;
    adjc[1] = y2 * z0 - y0 * z2;
    adjc[2] = y0 * z1 - y1 * z0;
    det = x0 * adjc[0] + x1 * adjc[1] + x2 * adjc[2];
}

// 6x6 grid of 16x16 output tiles; block (r,s) = tiles 2r..2r+1 x 2s..2s+1.
// The 24 tiles of blocks r <= s are split in 2-D rectangles, 6 per wave, so
// each wave loads few distinct operand fragments per k step (three of them
// are then left out, see skipped_tile):
//   wave 0: rows {0,1} x cols {0,1,2}   wave 1: rows {0,1} x cols {3,4,5}
//   wave 2: rows {2,3} x cols {2,3,4}   wave 3: rows {2,3} x {5}, {4,5} x {4,5}
// Wave w < 3 uses A rows AR[w][0..1], B cols BC[w][0..2], tile t = (t/3, t%3).
// Wave 3 uses A rows 2,3,4,5, B cols 4,5 with tiles (0,1),(1,1),(2,0),(2,1),
// (3,0),(3,1) in (A index, B index).
__device__ __forceinline__ void tile_of(int wave, int t, int &TM, int &TN)
{
    if (wave < 3) {
        const int r0 = wave == 2 ? 2 : 0;
        const int c0 = wave == 0 ? 0 : (wave == 1 ? 3 : 2);
        TM = r0 + t / 3;
        TN = c0 + t % 3;
    } else {
        const int ai[6] = {0, 1, 2, 2, 3, 3}, bi[6] = {1, 1, 0, 1, 0, 1};
        TM = 2 + ai[t];
        TN = 4 + bi[t];
    }
}

// The tile (1,0) of a diagonal block lies below its diagonal, where the
// in-place pass reads nothing (it writes both triangles from the upper
// one): waves 0, 2 and 3 leave theirs out (tile index 3, 3, 4), 21 tiles in
// all.
__host__ __device__ constexpr int skipped_tile(int wave) { return wave == 1 ? -1 : (wave == 3 ? 4 : 3); }

__device__ __forceinline__ int blk_id(int r, int s)  // r <= s
{
    return r == 0 ? s : (r == 1 ? 2 + s : 5);
}

// SKIP: a tile the wave leaves out (-1: none)
template <int MM, int NA, int NBF, int SKIP>
__device__ __forceinline__ void mma_rect(const typename MMT<MM>::T *Gs, const double *wd, const int (&ar)[NA],
                                         const int (&bc)[NBF], const int (&ta)[6], const int (&tb)[6], int lane,
                                         typename MMT<MM>::acc (&acc)[6])
{
    using T = typename MMT<MM>::T;
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int t = 0; t < 6; t++) acc[t] = typename MMT<MM>::acc{};
    constexpr int KS = Q2Staged<MM>::KS;
    // operand row of tile row TM for this lane: component TM/2, basis
    // 16*(TM%2) + lane%16
    int ra[NA], rb[NBF];
#pragma unroll
    for (int i = 0; i < NA; i++) ra[i] = ((ar[i] >> 1) * 33 + (ar[i] & 1) * 16 + col) * KS;
#pragma unroll
    for (int j = 0; j < NBF; j++) rb[j] = ((bc[j] >> 1) * 33 + (bc[j] & 1) * 16 + col) * KS;
#pragma unroll
    for (int kk = 0; kk < Q2Staged<MM>::KP / 4; kk++) {
        const int k = 4 * kk + grp;
        const T w = static_cast<T>(wd[k]);  // wd[27] == 0 (padding)
        T a[NA], b[NBF];
#pragma unroll
        for (int i = 0; i < NA; i++) a[i] = Gs[ra[i] + k] * w;
#pragma unroll
        for (int j = 0; j < NBF; j++) b[j] = Gs[rb[j] + k];
#pragma unroll
        for (int t = 0; t < 6; t++) {
            if (t == SKIP) continue;
            if constexpr (MM == MM_F64)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta[t]], b[tb[t]], acc[t], 0, 0, 0);
            else
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ta[t]], b[tb[t]], acc[t], 0, 0, 0);
        }
    }
}

template <int MM>
__device__ __forceinline__ void mma_wave(const typename MMT<MM>::T *Gs, const double *wd, int wave, int lane,
                                         typename MMT<MM>::acc (&acc)[6])
{
    const int ta[6] = {0, 0, 0, 1, 1, 1}, tb[6] = {0, 1, 2, 0, 1, 2};
    if (wave == 1) {
        const int ar[2] = {0, 1}, bc[3] = {3, 4, 5};
        mma_rect<MM, 2, 3, -1>(Gs, wd, ar, bc, ta, tb, lane, acc);
    } else if (wave != 3) {
        const int r0 = wave == 2 ? 2 : 0;
        const int ar[2] = {r0, r0 + 1}, bc[3] = {r0, r0 + 1, r0 + 2};
        mma_rect<MM, 2, 3, skipped_tile(0)>(Gs, wd, ar, bc, ta, tb, lane, acc);
    } else {
        const int ar[4] = {2, 3, 4, 5}, bc[2] = {4, 5};
        const int ta3[6] = {0, 1, 2, 2, 3, 3}, tb3[6] = {1, 1, 0, 1, 0, 1};
        mma_rect<MM, 4, 2, skipped_tile(3)>(Gs, wd, ar, bc, ta3, tb3, lane, acc);
    }
}

// 16x16 tile (TM, TN) of the scalar mass matrix sum_q wd[q] phi_a(q) phi_b(q)
// on the matrix cores, basis values built from the 1-D table B1.
template <int MM>
__device__ __forceinline__ typename MMT<MM>::acc mass_tile(const double *B1, const double *wd, int TM, int TN,
                                                           int lane)
{
    using T = typename MMT<MM>::T;
    typename MMT<MM>::acc acc{};
    const int col = lane & 15, grp = lane >> 4;
    const int a = TM * 16 + col, b = TN * 16 + col;
    auto phi = [&](int q, int f) -> double {
        if (f >= NB) return 0.0;
        return B1[(q % 3) * 3 + f % 3] * B1[((q / 3) % 3) * 3 + (f / 3) % 3] * B1[(q / 9) * 3 + f / 9];
    };
    // kept as a loop: unrolled, its table loads are all hoisted and stay
    // live next to the elasticity accumulators (the FP32 batched kernel then
    // spilled to scratch)
#pragma unroll 1
    for (int kk = 0; kk < 7; kk++) {
        const int k = 4 * kk + grp;
        const bool ok = k < NQ;
        const T x = ok ? static_cast<T>(wd[k] * phi(k, a)) : T(0);
        const T y = ok ? static_cast<T>(phi(k, b)) : T(0);
        if constexpr (MM == MM_F64)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
        else
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc, 0, 0, 0);
    }
    return acc;
}

template <typename V>
__device__ __forceinline__ void out_store(const V &v, V *p)
{
    __builtin_nontemporal_store(v, p);
}

// The global-memory view of a generic pointer.  Pointers that reach a kernel
// through a descriptor in memory (not as kernel arguments) are otherwise
// accessed with flat instructions, which also count against the LDS wait
// counter: every wait for an LDS read would then wait for the prefetch loads
// and output stores in flight as well.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

template <typename V>
__device__ __forceinline__ void out_store(const V &v, __attribute__((address_space(1))) V *p)
{
    __builtin_nontemporal_store(v, p);
}

// Everything one run of the Q2 cell routine reads and writes.
struct Q2Job {
    int64_t n_cells, n_nodes;
    const double *coords;
    const int32_t *conn;
    const void *mat;   // [n_cells][2] lambda, mu
    void *out;         // elasticity [n_cells][81][81]
    void *out_mass;    // MULTI only: scalar mass [n_cells][27][27] (or NULL)
    void *out_lap;     // MULTI only: Laplace [n_cells][27][27] (or NULL)
    unsigned *flags;
    DevTables tab;
};

// Q2 cells e, e + stride, ... < e_end, FP64 or FP32; see q2_run.
template <int MM, bool MULTI>
__device__ __forceinline__ void q2_run_staged(const Q2Job &A, int64_t e, int64_t e_end, int64_t stride, unsigned char *smem,
                                       int tid)
{
    using L = Q2Staged<MM>;
    using T = typename L::T;
    using ACC = typename MMT<MM>::acc;
    typedef T TV __attribute__((ext_vector_type(L::VEC)));
    double *B1 = reinterpret_cast<double *>(smem + L::OFF_TB);
    double *D1 = B1 + 9;
    double *wq = D1 + 9;
    double *xn = reinterpret_cast<double *>(smem + L::OFF_N);
    T *lmn = reinterpret_cast<T *>(xn + 3 * 28);
    double *Jq = reinterpret_cast<double *>(smem + L::OFF_J);
    double *wd = reinterpret_cast<double *>(smem + L::OFF_WD);
    T *Gs = reinterpret_cast<T *>(smem + L::OFF_G);
    T *Ks = reinterpret_cast<T *>(smem + L::OFF_K);
    // wave-uniform, and known to be so (scalar branches below)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    if (e >= e_end) return;  // uniform over the workgroup

    if (tid < 9) {
        B1[tid] = gmem(A.tab.B1)[tid];
        D1[tid] = gmem(A.tab.D1)[tid];
    } else if (tid >= 32 && tid < 32 + NQ) {
        wq[tid - 32] = gmem(A.tab.w)[tid - 32];
    }
    const auto mat = gmem(static_cast<const T *>(A.mat));
    const auto conn = gmem(A.conn);
    const auto coords = gmem(A.coords);
    // this thread's node coordinate (threads < 81: node a = tid/3, axis tid%3)
    const int ga = tid / 3, gc = tid - 3 * (tid / 3);
    // the first cell's coordinates and coefficients go to the parking slots
    // the loop reads every cell's data from (see the park step below)
    if (tid < NB * 3) {
        int64_t n = conn[e * NB + ga];
        if (n < 0 || n >= A.n_nodes) {
            raise_fault(A.flags, FAULT_INDEX);
            n = 0;
        }
        xn[gc * 28 + ga] = coords[3 * n + gc];
    }
    if (tid == 0) {
        lmn[0] = mat[2 * e];
        lmn[1] = mat[2 * e + 1];
    }
    __syncthreads();

    for (;;) {
        const int64_t en = e + stride;
        const bool has_next = en < e_end;
        const T lam = lmn[0], mu = lmn[1];  // read before the park step rewrites them

        // 1. (the cell's coordinates were parked component-major in LDS)
        // 2. J[i][j] at quadrature point q, one entry per thread (243
        //    threads), by sum factorization over the tensor-product basis
        if (tid < NQ * 9) {
            const int q = tid % NQ, ij = tid / NQ, i = ij / 3, j = ij - 3 * (ij / 3);
            const int q0 = q % 3, q1 = (q / 3) % 3, q2 = q / 9;
            const double *T0 = (j == 0 ? D1 : B1) + q0 * 3;
            const double *T1 = (j == 1 ? D1 : B1) + q1 * 3;
            const double *T2 = (j == 2 ? D1 : B1) + q2 * 3;
            const double f0[3] = {T0[0], T0[1], T0[2]}, f1[3] = {T1[0], T1[1], T1[2]},
                         f2[3] = {T2[0], T2[1], T2[2]};
            const double *x = xn + i * 28;
            double s2 = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < 3; a2++) {
                double s1 = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < 3; a1++) {
                    const double *xr = x + 3 * (a1 + 3 * a2);
                    s1 = fma(f1[a1], f0[0] * xr[0] + f0[1] * xr[1] + f0[2] * xr[2], s1);
                }
                s2 = fma(f2[a2], s1, s2);
            }
            Jq[q * 9 + i * 3 + j] = s2;
        }
        __syncthreads();

        // 3. det J and J^-1 per quadrature point (FP64, recomputed by each
        //    of the 9 threads of a point), w det J; then
        //    G[q][i][a] = sum_j dphi_a/dxi_j Jinv[j][i] (stored as T), one
        //    (q, i, a2) triple per thread, 9 basis functions each.
        //
        //    Prefetch of the next cell, in two hops that are each waited for
        //    one phase after they are issued: its connectivity and
        //    coefficients here, its coordinates after the GEMM, parked in LDS
        //    after the epilogue.  Every wait thus falls before this cell's
        //    flush; the previous cell's flush drains during phases 1-4.
        //
        //    The operand's depth padding (k = 27) of the real rows is zeroed
        //    here, after the barrier that follows the previous cell's flush
        //    reads.  The padding rows a = 27..32 keep what the staging area
        //    left there: they only reach output rows and columns that are
        //    never stored.
        static_assert(L::KP == NQ + 1, "one padding column");
        if (tid < NB * 3) Gs[((tid / NB) * 33 + tid % NB) * L::KS + NQ] = T(0);
        if (tid == 255) wd[NQ] = 0.0;
        int32_t nn = 0;
        T lamn = T(0), mun = T(0);
        if (has_next) {
            if (tid < NB * 3) nn = conn[en * NB + ga];
            if (tid == 0) {  // only the thread that parks them: a dead load would still be waited for
                lamn = mat[2 * en];
                mun = mat[2 * en + 1];
            }
        }
        if (tid < NQ * 9) {
            const int q = tid % NQ, r9 = tid / NQ, ci = r9 / 3, a2 = r9 - 3 * (r9 / 3);
            const int q0 = q % 3, q1 = (q / 3) % 3, q2 = q / 9;
            // column ci of J^-1 = adj J / det J.  That adjugate column is the
            // cross product of rows ci+1 and ci+2 of J (indices mod 3), and
            // det J = row ci . that column (cyclic), so the thread loads the
            // three rows in that order from addresses computed from ci.
            double adjc[3], det;
            q2_adj_column(Jq + q * 9, ci, adjc, det);
            // 1/det by the hardware reciprocal refined with two Newton steps
            // (r <- r + r (1 - det r)), accurate to ~1 ulp
            double rd = __builtin_amdgcn_rcp(det);
            rd = fma(rd, fma(-det, rd, 1.0), rd);
            rd = fma(rd, fma(-det, rd, 1.0), rd);
            if (r9 == 0) {
                if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
                wd[q] = wq[q] * det;
            }
            const double c0 = adjc[0] * rd, c1 = adjc[1] * rd, c2 = adjc[2] * rd;
            const double bz = B1[q2 * 3 + a2], dz = D1[q2 * 3 + a2];
            // G = c0 dx by bz + c1 bx dy bz + c2 bx by dz, factored over the
            // tensor indices: dx (c0 bz by) + bx (c1 bz dy + c2 dz by)
            T *dst = Gs + ci * 33 * L::KS + q;
            const double c0z = c0 * bz, c1z = c1 * bz, c2z = c2 * dz;
#pragma unroll
            for (int a1 = 0; a1 < 3; a1++) {
                const double by = B1[q1 * 3 + a1], dy = D1[q1 * 3 + a1];
                const double p0 = c0z * by, p12 = fma(c1z, dy, c2z * by);
#pragma unroll
                for (int a0 = 0; a0 < 3; a0++) {
                    const double bx = B1[q0 * 3 + a0], dx = D1[q0 * 3 + a0];
                    dst[(a0 + 3 * (a1 + 3 * a2)) * L::KS] = static_cast<T>(fma(p0, dx, p12 * bx));
                }
            }
        }
        __syncthreads();

        // 4. the per-cell GEMM on matrix cores
        ACC acc[6];
        mma_wave<MM>(Gs, wd, wave, lane, acc);
        if constexpr (MULTI) {
            // scalar mass M[a][b] = sum_q w_q det J_q phi_a(q) phi_b(q):
            // wave w takes tile (w/2, w%2) of the 2x2 tiles over 27x27
            if (A.out_mass) {
                ACC am = mass_tile<MM>(B1, wd, wave >> 1, wave & 1, lane);
                const auto om = gmem(static_cast<T *>(A.out_mass)) + e * (NB * NB);
                const int b = (wave & 1) * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int a = (wave >> 1) * 16 + (MM == MM_F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
                    if (a < NB && b < NB) om[a * NB + b] = static_cast<T>(am[v]);
                }
            }
        }
        __syncthreads();  // every wave is done reading the operands

        // second prefetch hop: the next cell's coordinates.  The empty asm
        // keeps the first use of the connectivity value (and so the wait for
        // its load) here instead of next to the load.
        double xnext = 0.0;
        if (has_next && tid < NB * 3) {
            asm volatile("" : "+v"(nn));
            int64_t n = nn;
            if (n < 0 || n >= A.n_nodes) {
                raise_fault(A.flags, FAULT_INDEX);
                n = 0;
            }
            xnext = coords[3 * n + gc];
        }

        // 5. the blocks r <= s of P go straight to their places in the
        //    staging area that holds the cell's matrix row-major, shifted by
        //    h entries so that LDS vectors line up with 16-byte aligned output
        const int64_t base = e * NK;
        const int h = static_cast<int>(base & (L::VEC - 1));
#pragma unroll
        for (int t = 0; t < 6; t++) {
            if (t == skipped_tile(wave)) continue;
            int TM, TN;
            tile_of(wave, t, TM, TN);
            const int r = TM >> 1, s = TN >> 1;
            // 16x16 accumulator layout: column = lane % 16; the f32 MFMAs
            // hold rows 4*(lane/16) + v, the f64 MFMA rows lane/16 + 4*v.
            const int b = (TN & 1) * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int a = (TM & 1) * 16 + (MM == MM_F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
                if (a < NB && b < NB) Ks[h + (r * NB + a) * ND + s * NB + b] = static_cast<T>(acc[t][v]);
            }
        }
        __syncthreads();

        // 6. K from P in place.  A thread owns an unordered pair {a,b}
        //    (a <= b) of block positions and touches only positions (a,b),
        //    (b,a) of the nine blocks, so no other thread reads its entries:
        //      K_rr = (lambda + mu) P_rr + mu (P_00 + P_11 + P_22)  (P_rr symmetric)
        //      K_rs[x][y] = lambda P_rs[x][y] + mu P_rs[y][x],  K_sr = K_rs^T.
        {
            T *K = Ks + h;
            const T lm = lam + mu;
#pragma unroll
            for (int it = 0; it < 2; it++) {
                const int p = tid + 256 * it;
                if (p >= NB * (NB + 1) / 2) break;
                // row a of the upper triangle starts at a*27 - a(a-1)/2
                int a = static_cast<int>((55.0f - sqrtf(3025.0f - 8.0f * p)) * 0.5f);
                a = a < 0 ? 0 : (a > NB - 1 ? NB - 1 : a);
                if (a > 0 && a * NB - a * (a - 1) / 2 > p) a--;
                if (a < NB - 1 && (a + 1) * NB - (a + 1) * a / 2 <= p) a++;
                const int b = a + (p - (a * NB - a * (a - 1) / 2));
                const int ab = a * ND + b, ba = b * ND + a;  // offsets inside a block
                const T d0 = K[ab], d1 = K[NB * ND + NB + ab], d2 = K[2 * NB * ND + 2 * NB + ab];
                T pab[3], pba[3];
#pragma unroll
                for (int o = 0; o < 3; o++) {
                    const int r = o == 2 ? 1 : 0, s = o == 0 ? 1 : 2;
                    const T *U = K + r * NB * ND + s * NB;
                    pab[o] = U[ab];
                    pba[o] = U[ba];
                }
                const T tr = mu * (d0 + d1 + d2);
                const T k0 = lm * d0 + tr, k1 = lm * d1 + tr, k2 = lm * d2 + tr;
                if constexpr (MULTI) {
                    if (A.out_lap) {
                        const auto ol = gmem(static_cast<T *>(A.out_lap)) + e * (NB * NB);
                        const T lv = d0 + d1 + d2;
                        ol[a * NB + b] = lv;
                        ol[b * NB + a] = lv;
                    }
                }
                K[ab] = k0;
                K[NB * ND + NB + ab] = k1;
                K[2 * NB * ND + 2 * NB + ab] = k2;
                K[ba] = k0;
                K[NB * ND + NB + ba] = k1;
                K[2 * NB * ND + 2 * NB + ba] = k2;
#pragma unroll
                for (int o = 0; o < 3; o++) {
                    const int r = o == 2 ? 1 : 0, s = o == 0 ? 1 : 2;
                    T *U = K + r * NB * ND + s * NB;  // block (r,s), holds P_rs
                    T *W = K + s * NB * ND + r * NB;  // block (s,r)
                    const T kab = lam * pab[o] + mu * pba[o], kba = lam * pba[o] + mu * pab[o];
                    U[ab] = kab;
                    W[ab] = kba;
                    U[ba] = kba;
                    W[ba] = kab;
                }
            }
        }
        // park the prefetched next-cell data in LDS: no loaded register stays
        // live across the flush, so nothing after the flush waits for its
        // stores to drain (vector memory counters complete in order)
        if (has_next) {
            if (tid < NB * 3) xn[gc * 28 + ga] = xnext;
            if (tid == 0) {
                lmn[0] = lamn;
                lmn[1] = mun;
            }
        }
        __syncthreads();

        // 7. linear flush: consecutive lanes store consecutive 16-byte vectors
        //    of the cell's contiguous output (LDS reads batched ahead of the
        //    stores); the few entries before the first and after the last
        //    whole vector go one by one
        {
            const auto out = gmem(static_cast<T *>(A.out));
            const auto aligned = (__attribute__((address_space(1))) TV *)(out + (base - h));
            const TV *k16 = reinterpret_cast<const TV *>(Ks);
            const int vf = h ? 1 : 0, vl = (NK + h) / L::VEC;  // whole vectors [vf, vl)
            constexpr int BATCH = 4;
#pragma unroll
            for (int j0 = 0; j0 < L::NV; j0 += BATCH) {
                TV buf[BATCH];
#pragma unroll
                for (int j = 0; j < BATCH; j++) {
                    const int v = vf + tid + 256 * (j0 + j);
                    if (v < vl) buf[j] = k16[v];
                }
#pragma unroll
                for (int j = 0; j < BATCH; j++) {
                    const int v = vf + tid + 256 * (j0 + j);
                    if (v < vl) out_store(buf[j], aligned + v);
                }
            }
            if (tid < 2 * L::VEC) {
                const int f = tid < L::VEC ? tid : vl * L::VEC - h + (tid - L::VEC);
                const bool head = tid < L::VEC && f < vf * L::VEC - h;
                const bool tail = tid >= L::VEC && f < NK;
                if (head || tail) out[base + f] = Ks[h + f];
            }
        }
        // the staging area is reused by the next cell: without JOUT its J
        // phase writes there; with JOUT the barrier after the J phase orders
        // the next writes after these reads
        if constexpr (!L::JOUT) __syncthreads();
        if (!has_next) break;
        e = en;
    }
    if constexpr (L::JOUT) __syncthreads();  // end synchronised
}
// ---------------------------------------------------------------------------
// Split routine (BF16X3: every operand a sum hi + lo of two bf16 values, the
// product hi*hi + hi*lo + lo*hi accumulated in FP32 on the bf16 matrix
// cores).  The products are cheap at this precision, so K is formed in
// registers instead of through an in-place pass over P: the operand is
// scaled symmetrically, Gt[27 i + a][k] = sqrt(w_k det J_k) dphi_a/dx_i (x_k),
// so that P_rs[a][b] = sum_k Gt[27 r + a][k] Gt[27 s + b][k], and with
// lambda, mu constant over the cell
//   K_rs = lambda P_rs + mu P_sr  (r != s),
//   K_rr = (lambda + mu) P_rr + mu (P_00 + P_11 + P_22).
// Each 27x27 block is covered by 2x2 tiles of 16x16 at positions (x, y).  K
// is symmetric, so its tiles at (1, 0) are the transposes of those at (0, 1)
// and only positions (0,0), (1,1) and (0,1) are computed: P_rs for all nine
// (r, s) at three positions, 27 tile products, 7 + 7 + 7 + 6 over the four
// waves.  Products are grouped so that K follows in registers: a diagonal
// group (P_00, P_11, P_22 at one position) gives K_00, K_11 and K_22 there,
// a pair group (P_rs, P_sr) gives K_rs and K_sr.
struct Q2Split {
    using T = float;
    static constexpr int VEC = 4;  // entries per 16-byte store
    // The staging area holds the cell's 81x81 matrix with every 27-entry
    // segment of a row padded to 28 (entry f at f + f/27), so that block
    // columns, and the four consecutive columns one lane holds, start on
    // 16-byte boundaries.
    static constexpr int SROW = 84, SBLK = 28;
    static constexpr int STAGE_BYTES = ND * SROW * 4;
    // operand halves hi[row][k], lo[row][k]: component i's rows start at
    // 27 i, rows 81..85 only pad the second tile of the last component; depth
    // padded with zeros to 32 (one bf16 step); a row stride of 40 entries
    // (8 mod 16) keeps the 16-byte fragment reads free of bank conflicts
    static constexpr int OROWS = 86, KP = 32, KS = 40;
    static constexpr int OP_BYTES = 2 * OROWS * KS * 2;
    // kept for the whole launch: 1-D tables and weights
    static constexpr int OFF_TB = 0;                                  // double B1[9], D1[9], w[27]
    // the next cell's coordinates and coefficients, parked before the flush
    // (coordinates component-major: xn[3][28], node a of axis i at 28 i + a)
    static constexpr int OFF_N = align16(OFF_TB + (9 + 9 + NQ) * 8);  // double xn[3][28], float lmn[2]
    // per cell, outside the staging area, so a cell's J phase may start while
    // other waves still flush the previous cell
    static constexpr int OFF_J = align16(OFF_N + 3 * 28 * 8 + 2 * 4);  // double J[27][9]
    static constexpr int OFF_S = align16(OFF_J + NQ * 9 * 8);          // staging
    // the operand halves, inside the staging area (written only after the
    // last operand read)
    static constexpr int OFF_OP = OFF_S;
    static constexpr int BYTES = align16(OFF_S + STAGE_BYTES);
    // 16-byte vectors of the staged matrix per thread in the flush
    static constexpr int NV = ((NK + 2 * VEC - 1) / VEC + 255) / 256;
    static_assert(OFF_OP + OP_BYTES <= OFF_S + STAGE_BYTES, "operand outside the staging area");
};

template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>)
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Work of wave W in the split routine.
//   F: operand fragments the wave loads, id 3 t + i = rows 27 i + 16 t ..
//   C: products (r, s, x, y);  G: groups (0 diagonal / 1 pair, first product)
template <int W>
struct WavePlan;
template <>
struct WavePlan<0> {  // position (0,0): everything but the pair (1,2)
    static constexpr int NF = 3, NC = 7, NG = 3;
    static constexpr int F[6] = {0, 1, 2};
    static constexpr int C[7][4] = {{0, 0, 0, 0}, {1, 1, 0, 0}, {2, 2, 0, 0}, {0, 1, 0, 0},
                                    {1, 0, 0, 0}, {0, 2, 0, 0}, {2, 0, 0, 0}};
    static constexpr int G[3][2] = {{0, 0}, {1, 3}, {1, 5}};
};
template <>
struct WavePlan<1> {  // pair (1,2) at (0,0); diagonal and pair (0,1) at (1,1)
    static constexpr int NF = 5, NC = 7, NG = 3;
    static constexpr int F[6] = {1, 2, 3, 4, 5};
    static constexpr int C[7][4] = {{1, 2, 0, 0}, {2, 1, 0, 0}, {0, 0, 1, 1}, {1, 1, 1, 1},
                                    {2, 2, 1, 1}, {0, 1, 1, 1}, {1, 0, 1, 1}};
    static constexpr int G[3][2] = {{1, 0}, {0, 2}, {1, 5}};
};
template <>
struct WavePlan<2> {  // pairs (0,2), (1,2) at (1,1); diagonal at (0,1)
    static constexpr int NF = 6, NC = 7, NG = 3;
    static constexpr int F[6] = {0, 1, 2, 3, 4, 5};
    static constexpr int C[7][4] = {{0, 2, 1, 1}, {2, 0, 1, 1}, {1, 2, 1, 1}, {2, 1, 1, 1},
                                    {0, 0, 0, 1}, {1, 1, 0, 1}, {2, 2, 0, 1}};
    static constexpr int G[3][2] = {{1, 0}, {1, 2}, {0, 4}};
};
template <>
struct WavePlan<3> {  // the three pairs at (0,1)
    static constexpr int NF = 6, NC = 6, NG = 3;
    static constexpr int F[6] = {0, 1, 2, 3, 4, 5};
    static constexpr int C[7][4] = {{0, 1, 0, 1}, {1, 0, 0, 1}, {0, 2, 0, 1},
                                    {2, 0, 0, 1}, {1, 2, 0, 1}, {2, 1, 0, 1}};
    static constexpr int G[3][2] = {{1, 0}, {1, 2}, {1, 4}};
};

template <typename WP>
constexpr int frag_slot(int id)
{
    for (int n = 0; n < WP::NF; n++)
        if (WP::F[n] == id) return n;
    return -1;
}

constexpr int frag_row(int id) { return (id % 3) * NB + (id / 3) * 16; }

// The wave's tile products.  The fragment of rows 27 s + 16 y .. goes in as
// the MFMA's first operand and that of rows 27 r + 16 x .. as the second, so
// the accumulator holds P_rs transposed: lane (g, c) = (lane / 16, lane % 16)
// owns row a = 16 x + c and columns b = 16 y + 4 g + v, v = 0..3.
template <typename WP>
__device__ __forceinline__ void split_gemm(const unsigned char *op, int lane, f4 (&acc)[7])
{
    using L = Q2Split;
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int m = 0; m < 7; m++) acc[m] = f4{};
    const __bf16 *hi = reinterpret_cast<const __bf16 *>(op);
    const __bf16 *lo = hi + L::OROWS * L::KS;
    bf8 fh[WP::NF], fl[WP::NF];
#pragma unroll
    for (int n = 0; n < WP::NF; n++) {
        const int o = (frag_row(WP::F[n]) + c) * L::KS + 8 * g;
        fh[n] = *reinterpret_cast<const bf8 *>(hi + o);
        fl[n] = *reinterpret_cast<const bf8 *>(lo + o);
    }
    // the small cross terms first, then hi * hi (FP32 accumulation)
    static_for<WP::NC>([&](auto m) {
        constexpr int ia = frag_slot<WP>(3 * WP::C[m][3] + WP::C[m][1]);
        constexpr int ib = frag_slot<WP>(3 * WP::C[m][2] + WP::C[m][0]);
        static_assert(ia >= 0 && ib >= 0, "fragment missing from the wave plan");
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl[ia], fh[ib], acc[m], 0, 0, 0);
    });
    static_for<WP::NC>([&](auto m) {
        constexpr int ia = frag_slot<WP>(3 * WP::C[m][3] + WP::C[m][1]);
        constexpr int ib = frag_slot<WP>(3 * WP::C[m][2] + WP::C[m][0]);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[ia], fl[ib], acc[m], 0, 0, 0);
    });
    static_for<WP::NC>([&](auto m) {
        constexpr int ia = frag_slot<WP>(3 * WP::C[m][3] + WP::C[m][1]);
        constexpr int ib = frag_slot<WP>(3 * WP::C[m][2] + WP::C[m][0]);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[ia], fh[ib], acc[m], 0, 0, 0);
    });
}

// One K tile (block (R, S), position (x, y), held as described at
// split_gemm) into the staging area; with TR also its transpose, tile (1, 0)
// of block (S, R) (only position (0, 1) is transposed, so x = 0 there).
template <bool TR>
__device__ __forceinline__ void put_tile(float *Ks, const f4 &k, int R, int S, int x, int y, int lane)
{
    using L = Q2Split;
    const int c = lane & 15, g = lane >> 4;
    const int a = 16 * x + c;
    // one 16-byte vector of columns 16 y + 4 g ..; for y = 1, g = 2 its
    // last entry falls on the segment's pad word, g = 3 is outside
    if (a < NB && (y == 0 || g < 3))
        *reinterpret_cast<f4 *>(Ks + (R * NB + a) * L::SROW + S * L::SBLK + 16 * y + 4 * g) = k;
    if constexpr (TR) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int b = 16 + 4 * g + v;
            if (b < NB) Ks[(S * NB + b) * L::SROW + R * L::SBLK + c] = k[v];
        }
    }
}

// K from the wave's tile products into the staging area.
template <typename WP>
__device__ __forceinline__ void split_epilogue(float *Ks, const f4 (&acc)[7], float lam, float mu, int lane)
{
    const float lm = lam + mu;
    static_for<WP::NG>([&](auto gi) {
        constexpr int kind = WP::G[gi][0], c0 = WP::G[gi][1];
        constexpr int x = WP::C[c0][2], y = WP::C[c0][3];
        constexpr bool TR = x == 0 && y == 1;
        if constexpr (kind == 0) {
            const f4 mtr = mu * (acc[c0] + acc[c0 + 1] + acc[c0 + 2]);
            put_tile<TR>(Ks, lm * acc[c0] + mtr, 0, 0, x, y, lane);
            put_tile<TR>(Ks, lm * acc[c0 + 1] + mtr, 1, 1, x, y, lane);
            put_tile<TR>(Ks, lm * acc[c0 + 2] + mtr, 2, 2, x, y, lane);
        } else {
            constexpr int r = WP::C[c0][0], s = WP::C[c0][1];
            put_tile<TR>(Ks, lam * acc[c0] + mu * acc[c0 + 1], r, s, x, y, lane);
            put_tile<TR>(Ks, lam * acc[c0 + 1] + mu * acc[c0], s, r, x, y, lane);
        }
    });
}

// Q2 cells e, e + stride, ... < e_end in the split precision; see q2_run.
__device__ __forceinline__ void q2_run_split(const Q2Job &A, int64_t e, int64_t e_end, int64_t stride,
                                             unsigned char *smem, int tid)
{
    using L = Q2Split;
    typedef float TV __attribute__((ext_vector_type(4)));
    double *B1 = reinterpret_cast<double *>(smem + L::OFF_TB);
    double *D1 = B1 + 9;
    double *wq = D1 + 9;
    double *xn = reinterpret_cast<double *>(smem + L::OFF_N);
    float *lmn = reinterpret_cast<float *>(xn + 3 * 28);
    double *Jq = reinterpret_cast<double *>(smem + L::OFF_J);
    float *Ks = reinterpret_cast<float *>(smem + L::OFF_S);
    unsigned char *op = smem + L::OFF_OP;
    __bf16 *ohi = reinterpret_cast<__bf16 *>(op);
    // wave-uniform, and known to be so (scalar branches below)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    if (e >= e_end) return;  // uniform over the workgroup

    if (tid < 9) {
        B1[tid] = gmem(A.tab.B1)[tid];
        D1[tid] = gmem(A.tab.D1)[tid];
    } else if (tid >= 32 && tid < 32 + NQ) {
        wq[tid - 32] = gmem(A.tab.w)[tid - 32];
    }
    const auto mat = gmem(static_cast<const float *>(A.mat));
    const auto conn = gmem(A.conn);
    const auto coords = gmem(A.coords);
    // this thread's node coordinate (threads < 81: node a = tid/3, axis tid%3)
    const int ga = tid / 3, gc = tid - 3 * (tid / 3);
    // the first cell's coordinates and coefficients go to the parking slots
    // the loop reads every cell's data from (see the park step below)
    if (tid < NB * 3) {
        int64_t n = conn[e * NB + ga];
        if (n < 0 || n >= A.n_nodes) {
            raise_fault(A.flags, FAULT_INDEX);
            n = 0;
        }
        xn[gc * 28 + ga] = coords[3 * n + gc];
    }
    if (tid == 0) {
        lmn[0] = mat[2 * e];
        lmn[1] = mat[2 * e + 1];
    }
    __syncthreads();

    for (;;) {
        const int64_t en = e + stride;
        const bool has_next = en < e_end;
        const float lam = lmn[0], mu = lmn[1];  // read before the park step rewrites them

        // 1. (the cell's coordinates were parked component-major in LDS)
        // 2. J[i][j] at quadrature point q, one entry per thread (243
        //    threads), by sum factorization over the tensor-product basis
        if (tid < NQ * 9) {
            const int q = tid % NQ, ij = tid / NQ, i = ij / 3, j = ij - 3 * (ij / 3);
            const int q0 = q % 3, q1 = (q / 3) % 3, q2 = q / 9;
            const double *T0 = (j == 0 ? D1 : B1) + q0 * 3;
            const double *T1 = (j == 1 ? D1 : B1) + q1 * 3;
            const double *T2 = (j == 2 ? D1 : B1) + q2 * 3;
            const double f0[3] = {T0[0], T0[1], T0[2]}, f1[3] = {T1[0], T1[1], T1[2]},
                         f2[3] = {T2[0], T2[1], T2[2]};
            const double *x = xn + i * 28;
            double s2 = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < 3; a2++) {
                double s1 = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < 3; a1++) {
                    const double *xr = x + 3 * (a1 + 3 * a2);
                    s1 = fma(f1[a1], f0[0] * xr[0] + f0[1] * xr[1] + f0[2] * xr[2], s1);
                }
                s2 = fma(f2[a2], s1, s2);
            }
            Jq[q * 9 + i * 3 + j] = s2;
        }
        __syncthreads();

        // 3. det J and J^-1 per quadrature point (FP64, recomputed by each
        //    of the 9 threads of a point); then the operand halves of
        //    Gt[27 i + a][q] = sqrt(w_q / det J) sum_j dphi_a/dxi_j adj(J)[j][i]
        //    (= sqrt(w_q det J) G[q][i][a]), one (q, i, a2) triple per
        //    thread, 9 basis functions each.  The next cell's connectivity
        //    and coefficients are prefetched here, its coordinates after the
        //    GEMM; both are parked in LDS before the flush.  The operand's
        //    depth padding is zeroed here, after the barrier that follows the
        //    previous cell's flush reads of the staging area.
        if (tid < 2 * ND) {
            __bf16 *p = ohi + (tid >= ND ? L::OROWS * L::KS : 0) + (tid >= ND ? tid - ND : tid) * L::KS;
#pragma unroll
            for (int k = NQ; k < L::KP; k++) p[k] = static_cast<__bf16>(0.0f);
        }
        int32_t nn = 0;
        float lamn = 0.0f, mun = 0.0f;
        if (has_next) {
            if (tid < NB * 3) nn = conn[en * NB + ga];
            if (tid == 0) {  // only the thread that parks them: a dead load would still be waited for
                lamn = mat[2 * en];
                mun = mat[2 * en + 1];
            }
        }
        if (tid < NQ * 9) {
            const int q = tid % NQ, r9 = tid / NQ, ci = r9 / 3, a2 = r9 - 3 * (r9 / 3);
            const int q0 = q % 3, q1 = (q / 3) % 3, q2 = q / 9;
            // column ci of the adjugate and det J (as in the staged routine);
            // 1/det by the hardware reciprocal refined with two Newton steps
            // (r <- r + r (1 - det r))
            double adjc[3], det;
            q2_adj_column(Jq + q * 9, ci, adjc, det);
            double rd = __builtin_amdgcn_rcp(det);
            rd = fma(rd, fma(-det, rd, 1.0), rd);
            rd = fma(rd, fma(-det, rd, 1.0), rd);
            if (r9 == 0 && !(det > 0.0)) raise_fault(A.flags, FAULT_DET);
            const double sc = sqrt(wq[q] * rd);
            const double bz = B1[q2 * 3 + a2], dz = D1[q2 * 3 + a2];
            // G = c0 dx by bz + c1 bx dy bz + c2 bx by dz, factored over the
            // tensor indices: dx (c0 bz by) + bx (c1 bz dy + c2 dz by)
            const double c0z = adjc[0] * sc * bz, c1z = adjc[1] * sc * bz, c2z = adjc[2] * sc * dz;
            const int o = (ci * NB + 9 * a2) * L::KS + q;
#pragma unroll
            for (int a1 = 0; a1 < 3; a1++) {
                const double by = B1[q1 * 3 + a1], dy = D1[q1 * 3 + a1];
                const double p0 = c0z * by, p12 = fma(c1z, dy, c2z * by);
#pragma unroll
                for (int a0 = 0; a0 < 3; a0++) {
                    const double bx = B1[q0 * 3 + a0], dx = D1[q0 * 3 + a0];
                    const double val = fma(p0, dx, p12 * bx);
                    const int oo = o + (a0 + 3 * a1) * L::KS;
                    // hi = bf16(x), lo = bf16(x - hi) of x = fl32(val): the
                    // residual is exact in FP32, and hi + lo carries 16 bits
                    const float x = static_cast<float>(val);
                    const __bf16 hb = static_cast<__bf16>(x);
                    ohi[oo] = hb;
                    ohi[L::OROWS * L::KS + oo] = static_cast<__bf16>(x - static_cast<float>(hb));
                }
            }
        }
        __syncthreads();

        // 4. the cell's tile products on the matrix cores
        f4 acc[7];
        if (wave == 0)
            split_gemm<WavePlan<0>>(op, lane, acc);
        else if (wave == 1)
            split_gemm<WavePlan<1>>(op, lane, acc);
        else if (wave == 2)
            split_gemm<WavePlan<2>>(op, lane, acc);
        else
            split_gemm<WavePlan<3>>(op, lane, acc);
        __syncthreads();  // every wave is done reading the operand

        // second prefetch hop: the next cell's coordinates.  The empty asm
        // keeps the first use of the connectivity value (and so the wait for
        // its load) here instead of next to the load.
        double xnext = 0.0;
        if (has_next && tid < NB * 3) {
            asm volatile("" : "+v"(nn));
            int64_t n = nn;
            if (n < 0 || n >= A.n_nodes) {
                raise_fault(A.flags, FAULT_INDEX);
                n = 0;
            }
            xnext = coords[3 * n + gc];
        }

        // 5. K tiles to the staging area
        if (wave == 0)
            split_epilogue<WavePlan<0>>(Ks, acc, lam, mu, lane);
        else if (wave == 1)
            split_epilogue<WavePlan<1>>(Ks, acc, lam, mu, lane);
        else if (wave == 2)
            split_epilogue<WavePlan<2>>(Ks, acc, lam, mu, lane);
        else
            split_epilogue<WavePlan<3>>(Ks, acc, lam, mu, lane);
        // park the prefetched next-cell data in LDS: no loaded register stays
        // live across the flush, so nothing after the flush waits for its
        // stores to drain (vector memory counters complete in order)
        if (has_next) {
            if (tid < NB * 3) xn[gc * 28 + ga] = xnext;
            if (tid == 0) {
                lmn[0] = lamn;
                lmn[1] = mun;
            }
        }
        __syncthreads();

        // 6. flush: consecutive lanes store consecutive 16-byte vectors of
        //    the cell's contiguous output, gathered from the padded staging
        //    rows (LDS reads batched ahead of the stores); the few entries
        //    before the first and after the last whole vector go one by one
        {
            const int64_t base = e * NK;
            const auto out = gmem(static_cast<float *>(A.out));
            const int ho = static_cast<int>(base & (L::VEC - 1));  // misalignment of the cell's output
            const auto aligned = (__attribute__((address_space(1))) TV *)(out + (base - ho));
            const int vf = ho ? 1 : 0, vl = (NK + ho) / L::VEC;  // whole vectors [vf, vl)
            constexpr int BATCH = 4;
#pragma unroll
            for (int j0 = 0; j0 < L::NV; j0 += BATCH) {
                TV buf[BATCH];
#pragma unroll
                for (int j = 0; j < BATCH; j++) {
                    const int v = vf + tid + 256 * (j0 + j);
                    if (v < vl) {
                        // entries f0..f0+3 sit at f + f/27: five words from
                        // f0 + f0/27 cover them, the one after a segment end
                        // skipped
                        const int f0 = L::VEC * v - ho;
                        const int d = static_cast<int>(fmaf(static_cast<float>(f0), 1.0f / 27.0f, 0.5f / 27.0f));
                        const int m = f0 - 27 * d;
                        const float *p = Ks + f0 + d;
                        const float w0 = p[0], w1 = p[1], w2 = p[2], w3 = p[3], w4 = p[4];
                        buf[j] = TV{w0, m >= 26 ? w2 : w1, m >= 25 ? w3 : w2, m >= 24 ? w4 : w3};
                    }
                }
#pragma unroll
                for (int j = 0; j < BATCH; j++) {
                    const int v = vf + tid + 256 * (j0 + j);
                    if (v < vl) out_store(buf[j], aligned + v);
                }
            }
            if (tid < 2 * L::VEC) {
                const int f = tid < L::VEC ? tid : vl * L::VEC - ho + (tid - L::VEC);
                const bool head = tid < L::VEC && f < vf * L::VEC - ho;
                const bool tail = tid >= L::VEC && f < NK;
                if (head || tail) out[base + f] = Ks[f + f / 27];
            }
        }
        // no barrier: the next cell's J phase writes outside the staging
        // area, and the barrier after it orders the next writes there after
        // these reads
        if (!has_next) break;
        e = en;
    }
    __syncthreads();  // end synchronised
}

template <int MM>
using Q2Layout = typename std::conditional<MM == MM_BF16X3, Q2Split, Q2Staged<MM>>::type;

// Q2 cells e, e + stride, ... < e_end with one workgroup of 256 threads.
// MULTI also emits the Laplace matrix P_00 + P_11 + P_22 (a by-product of
// the elasticity contraction) and the scalar mass matrix (one more small
// product on the matrix cores), sharing the geometry (FP64 and FP32 only).
// smem must hold Q2Layout<MM>::BYTES.  Ends with the workgroup synchronised.
template <int MM, bool MULTI>
__device__ __forceinline__ void q2_run(const Q2Job &A, int64_t e, int64_t e_end, int64_t stride, unsigned char *smem,
                                       int tid)
{
    if constexpr (MM == MM_BF16X3) {
        static_assert(!MULTI, "the split precision has no multi-form routine");
        q2_run_split(A, e, e_end, stride, smem, tid);
    } else {
        q2_run_staged<MM, MULTI>(A, e, e_end, stride, smem, tid);
    }
}

}  // namespace q2
}  // namespace fe
