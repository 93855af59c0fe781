// Matrix-core (MFMA) element-matrix kernel: linear elasticity on Q2
// hexahedra with per-cell isotropic coefficients.
//
// The linear elasticity form of the table of example weak forms, in matrix
// mode, is  K[(r,a),(s,b)] = sum_q w_q det J (lambda G_r[a] G_s[b]
// + mu G_s[a] G_r[b] + delta_rs mu G[a].G[b])  with G the physical basis
// gradients (the paper's 'cq,cqje,rjI,cqIK,cqlf,slK->cresf' with isotropic D).
// With lambda, mu constant over the cell all three terms come from ONE
// symmetric product per cell,
//     P[(r,a),(s,b)] = sum_q G[q][r][a] (w_q det J_q) G[q][s][b],
// a (3nb x nq) x (nq x 3nb) GEMM: K_rs = lambda P_rs + mu P_rs^T
// + delta_rs mu (P_00 + P_11 + P_22).  Only the 6 blocks r <= s of P are
// computed.  This is the dense contraction the paper's elasticity einsum
// performs, with the sparsity of the symmetric-gradient extractor (which the
// paper notes it does not exploit) folded away.
//
// One workgroup (4 waves) per cell:
//   1. gather the 27 node coordinates through the connectivity (FP64);
//   2. Jacobian columns from the tensor-product 1-D tables, then det J, J^-1
//      and w det J per quadrature point, all FP64;
//   3. G[q][(i,a)] = sum_j dphi_a/dxi_j Jinv[j][i] in FP64, stored in LDS in
//      the contraction type as the GEMM operand (rows padded 27 -> 32 per
//      component, K padded to the MFMA depth);
//   4. 24 output tiles of 16x16 (6 per wave) on MFMA:
//        FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32,
//        BF16X3: v_mfma_f32_16x16x32_bf16 three times per tile on the split
//        operands (hi*hi + hi*lo + lo*hi, FP32 accumulation);
//   5. P blocks to LDS (aliasing the operand area), L = P_00 + P_11 + P_22;
//   6. epilogue sweep over the 81x81 matrix: every lane writes consecutive
//      entries of the cell's contiguous output (non-temporal stores).
#include "fe_device.h"

namespace fe {
namespace {

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
constexpr int NB = 27, NQ = 27, NBP = 32, MROW = 3 * NBP, ND = 81;

template <int MM>
struct Q2Layout {
    using T = typename MMT<MM>::T;
    static constexpr int KP = MM == MM_BF16X3 ? 32 : 28;  // padded K (quadrature points)
    static constexpr int OFF_X = 0;                       // double xs[27][3]
    static constexpr int OFF_J = OFF_X + NB * 3 * 8;      // double J / Jinv [27][9]
    static constexpr int OFF_WD = OFF_J + NQ * 9 * 8;     // double wd[27]
    static constexpr int OFF_TB = OFF_WD + NQ * 8;        // double B1[9], D1[9], w[27]
    static constexpr int OFF_G = align16(OFF_TB + (9 + 9 + NQ) * 8);  // T Gs[KP][96]
    static constexpr int END_A = OFF_G + KP * MROW * (int)sizeof(T);
    static constexpr int OFF_P = 0;                        // T P[6][27][27] (aliases A)
    static constexpr int OFF_L = OFF_P + 6 * NB * NB * (int)sizeof(T);  // T L[27][27]
    static constexpr int END_B = OFF_L + NB * NB * (int)sizeof(T);
    static constexpr int BYTES = align16(cmax(END_A, END_B));
};

// 6x6 grid of 16x16 tiles; blocks (r,s) of 2x2 tiles; the 24 tiles of the
// blocks r <= s, 6 per wave.  Waves 0/1 take tile rows 0/1 (blocks (0,*)),
// waves 2/3 take tile rows 2/3 of blocks (1,1),(1,2) and 4/5 of block (2,2).
__device__ __forceinline__ void tile_of(int wave, int t, int &TM, int &TN)
{
    if (wave < 2) {
        TM = wave;
        TN = t;
    } else if (t < 4) {
        TM = wave;
        TN = 2 + t;
    } else {
        TM = wave + 2;
        TN = t;
    }
}

__device__ __forceinline__ int blk_id(int r, int s)  // r <= s
{
    return r == 0 ? s : (r == 1 ? 2 + s : 5);
}

template <typename T>
__device__ __forceinline__ void nt_store(T v, T *p)
{
    __builtin_nontemporal_store(v, p);
}

template <int MM>
__device__ __forceinline__ typename MMT<MM>::acc mma_tile(const typename MMT<MM>::T *Gs, const double *wd,
                                                          int TM, int TN, int lane,
                                                          typename MMT<MM>::acc acc)
{
    using T = typename MMT<MM>::T;
    const int col = lane & 15, grp = lane >> 4;
    if constexpr (MM == MM_F64 || MM == MM_F32) {
#pragma unroll
        for (int kk = 0; kk < Q2Layout<MM>::KP / 4; kk++) {
            const int k = 4 * kk + grp;
            const T a = Gs[k * MROW + TM * 16 + col];
            const T w = k < NQ ? static_cast<T>(wd[k]) : T(0);
            const T b = Gs[k * MROW + TN * 16 + col] * w;
            if constexpr (MM == MM_F64)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            else
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
    } else {
        bf8 ahi, alo, bhi, blo;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int k = 8 * grp + t;
            const float a = Gs[k * MROW + TM * 16 + col];
            const float w = k < NQ ? static_cast<float>(wd[k]) : 0.0f;
            const float b = Gs[k * MROW + TN * 16 + col] * w;
            const __bf16 ah = static_cast<__bf16>(a), bh = static_cast<__bf16>(b);
            ahi[t] = ah;
            bhi[t] = bh;
            alo[t] = static_cast<__bf16>(a - static_cast<float>(ah));
            blo[t] = static_cast<__bf16>(b - static_cast<float>(bh));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
    }
    return acc;
}

template <int MM>
__global__ __launch_bounds__(256) void k_elast_q2(ExecArgs A)
{
    using L = Q2Layout<MM>;
    using T = typename L::T;
    using ACC = typename MMT<MM>::acc;
    __shared__ __align__(16) unsigned char smem[L::BYTES];
    double *xs = reinterpret_cast<double *>(smem + L::OFF_X);
    double *Jq = reinterpret_cast<double *>(smem + L::OFF_J);
    double *wd = reinterpret_cast<double *>(smem + L::OFF_WD);
    double *B1 = reinterpret_cast<double *>(smem + L::OFF_TB);
    double *D1 = B1 + 9;
    double *wq = D1 + 9;
    T *Gs = reinterpret_cast<T *>(smem + L::OFF_G);

    const int64_t e = logical_block(A.xcd_remap);  // one cell per workgroup
    if (e >= A.n_cells) return;                     // uniform over the workgroup
    const int tid = threadIdx.x;

    // 1. gather coordinates; tables; zero the operand padding
    if (tid < NB * 3) {
        const int a = tid / 3, c = tid - 3 * a;
        const int64_t n = checked_node(A.conn, e * NB + a, A.n_nodes, A.flags);
        xs[tid] = A.coords[3 * n + c];
    } else if (tid < NB * 3 + 9) {
        B1[tid - NB * 3] = A.tab.B1[tid - NB * 3];
        D1[tid - NB * 3] = A.tab.D1[tid - NB * 3];
    } else if (tid < NB * 3 + 9 + NQ) {
        wq[tid - NB * 3 - 9] = A.tab.w[tid - NB * 3 - 9];
    }
    for (int i = tid; i < L::KP * MROW; i += 256) {
        const int k = i / MROW, m = i - k * MROW;
        if (k >= NQ || (m & (NBP - 1)) >= NB) Gs[i] = T(0);
    }
    const T *mat = static_cast<const T *>(A.mat);
    const T lam = mat[2 * e], mu = mat[2 * e + 1];
    __syncthreads();

    // 2a. Jacobian column j at quadrature point q: J[i][j] = sum_a x_a,i dphi_a/dxi_j
    if (tid < NQ * 3) {
        const int q = tid / 3, j = tid - 3 * q;
        const int q0 = q % 3, q1 = (q / 3) % 3, q2 = q / 9;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < 3; a2++)
#pragma unroll
            for (int a1 = 0; a1 < 3; a1++)
#pragma unroll
                for (int a0 = 0; a0 < 3; a0++) {
                    const double f0 = (j == 0 ? D1 : B1)[q0 * 3 + a0];
                    const double f1 = (j == 1 ? D1 : B1)[q1 * 3 + a1];
                    const double f2 = (j == 2 ? D1 : B1)[q2 * 3 + a2];
                    const double g = f0 * f1 * f2;
                    const int a = a0 + 3 * (a1 + 3 * a2);
                    c0 = fma(xs[a * 3 + 0], g, c0);
                    c1 = fma(xs[a * 3 + 1], g, c1);
                    c2 = fma(xs[a * 3 + 2], g, c2);
                }
        Jq[q * 9 + 0 + j] = c0;
        Jq[q * 9 + 3 + j] = c1;
        Jq[q * 9 + 6 + j] = c2;
    }
    __syncthreads();
    // 2b. det J, J^-1 (in place, stored as Ji[j][i]) and w det J
    if (tid < NQ) {
        double J[3][3], Ji[3][3];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) J[i][j] = Jq[tid * 9 + i * 3 + j];
        const double det = inverse3(J, Ji);
        if (!(det > 0.0)) raise_fault(A.flags, FAULT_DET);
        wd[tid] = wq[tid] * det;
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int i = 0; i < 3; i++) Jq[tid * 9 + j * 3 + i] = Ji[j][i];
    }
    __syncthreads();
    // 3. physical gradients G[q][i*32 + a] (FP64, stored as T)
    for (int p = tid; p < NQ * NB; p += 256) {
        const int q = p / NB, a = p - q * NB;
        const int q0 = q % 3, q1 = (q / 3) % 3, q2 = q / 9;
        const int a0 = a % 3, a1 = (a / 3) % 3, a2 = a / 9;
        const double bx = B1[q0 * 3 + a0], by = B1[q1 * 3 + a1], bz = B1[q2 * 3 + a2];
        const double g0 = D1[q0 * 3 + a0] * by * bz;
        const double g1 = bx * D1[q1 * 3 + a1] * bz;
        const double g2 = bx * by * D1[q2 * 3 + a2];
        const double *Ji = Jq + q * 9;
#pragma unroll
        for (int i = 0; i < 3; i++)
            Gs[q * MROW + i * NBP + a] = static_cast<T>(g0 * Ji[0 * 3 + i] + g1 * Ji[1 * 3 + i] + g2 * Ji[2 * 3 + i]);
    }
    __syncthreads();

    // 4. the per-cell GEMM on matrix cores
    const int wave = tid >> 6, lane = tid & 63;
    ACC acc[6];
#pragma unroll
    for (int t = 0; t < 6; t++) {
        int TM, TN;
        tile_of(wave, t, TM, TN);
        ACC z = {};
        acc[t] = mma_tile<MM>(Gs, wd, TM, TN, lane, z);
    }
    __syncthreads();  // every wave is done reading the operands

    // 5. P blocks to LDS, then L = P_00 + P_11 + P_22
    T *Ps = reinterpret_cast<T *>(smem + L::OFF_P);
    T *Ls = reinterpret_cast<T *>(smem + L::OFF_L);
#pragma unroll
    for (int t = 0; t < 6; t++) {
        int TM, TN;
        tile_of(wave, t, TM, TN);
        const int r = TM >> 1, s = TN >> 1, blk = blk_id(r, s);
        // 16x16 accumulator layout: column = lane % 16; the f32 MFMAs hold
        // rows 4*(lane/16) + v, the f64 MFMA holds rows lane/16 + 4*v.
        const int b = (TN & 1) * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int a = (TM & 1) * 16 + (MM == MM_F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
            if (a < NB && b < NB) Ps[blk * NB * NB + a * NB + b] = static_cast<T>(acc[t][v]);
        }
    }
    __syncthreads();
    for (int p = tid; p < NB * NB; p += 256) Ls[p] = Ps[p] + Ps[3 * NB * NB + p] + Ps[5 * NB * NB + p];
    __syncthreads();

    // 6. K_rs = lambda P_rs + mu P_rs^T + delta_rs mu L, coalesced stores
    T *out = static_cast<T *>(A.out) + e * (ND * ND);
    for (int f = tid; f < ND * ND; f += 256) {
        const int row = f / ND, col = f - row * ND;
        const int r = row / NB, a = row - r * NB, s = col / NB, b = col - s * NB;
        T pab, pba;
        if (r <= s) {
            const T *P = Ps + blk_id(r, s) * NB * NB;
            pab = P[a * NB + b];
            pba = P[b * NB + a];
        } else {
            const T *P = Ps + blk_id(s, r) * NB * NB;
            pab = P[b * NB + a];
            pba = P[a * NB + b];
        }
        T v = lam * pab + mu * pba;
        if (r == s) v += mu * Ls[a * NB + b];
        nt_store(v, out + f);
    }
}

template <int MM>
int launch_elast_q2(const Plan &, const ExecArgs &A, hipStream_t st)
{
    if (A.n_cells <= 0) return FE_OK;
    if (A.n_cells > 0x7fffffffLL) {
        set_error("too many cells for one launch");
        return FE_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_elast_q2<MM>, dim3((unsigned)A.n_cells), dim3(256), 0, st, A);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

}  // namespace

LaunchFn select_mfma(const Plan &p)
{
    if (p.cell == FE_CELL_HEX && p.order == 2 && p.form == FE_FORM_ELASTICITY && p.mode == FE_MODE_MATRIX &&
        p.mat_kind == FE_MAT_ISO_CELL) {
        if (p.prec == FE_PREC_FP64) return launch_elast_q2<MM_F64>;
        if (p.prec == FE_PREC_FP32) return launch_elast_q2<MM_F32>;
        if (p.prec == FE_PREC_BF16X3) return launch_elast_q2<MM_BF16X3>;
    }
    return nullptr;
}

}  // namespace fe
