// Global matrix assembly: the sparsity pattern of a connectivity and the
// block-CSR sum of element matrices (the assembly that follows the paper's
// element loops, which return per-cell matrices).
//
// Pattern: every cell contributes the node pairs (conn[e][a], conn[e][b]);
// the pairs are encoded as 64-bit keys n * n_nodes + m, radix-sorted and
// made unique on the device, so each row's column nodes come out sorted and
// the rows contiguous.
//
// Values: one wave per row node n walks the node's incidence list (cells and
// local numbers (e, a), sorted); at each step lane b adds the n_comp x n_comp
// block K_e[(., a), (., b)] into the row's LDS accumulator at the slot of
// conn[e][b] (binary search in the row's columns, staged in LDS).  Within a
// step the lanes hit distinct slots (the pattern build refuses a cell that
// lists one node twice), the steps run in incidence order, and
// lanes b read consecutive entries of the element matrix rows; the row is
// written once at the end.  No atomics: bitwise repeatable.
#include <hipcub/hipcub.hpp>

#include "fe_device.h"

struct fe_pattern_s {
    int64_t n_nodes = 0, nnz = 0;
    int nb = 0, device = -1, max_row = 0;
    int32_t *row_ptr = nullptr;  // [n_nodes + 1]
    int32_t *cols = nullptr;     // [nnz]
};

namespace fe {
namespace {

__global__ void k_pair_keys(const int32_t *conn, int64_t n_cells, int nb, int64_t n_nodes, uint64_t *keys,
                            unsigned *flags)
{
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_cells * nb2) return;
    const int64_t e = i / nb2;
    const int ab = static_cast<int>(i - e * nb2), a = ab / nb, b = ab - a * nb;
    int64_t n = conn[e * nb + a], m = conn[e * nb + b];
    if (n < 0 || n >= n_nodes || m < 0 || m >= n_nodes) {
        raise_fault(flags, FAULT_INDEX);
        n = m = 0;
    } else if (a != b && n == m) {
        // a cell listing one node twice would make two lanes of one
        // assembly step add into the same slot
        raise_fault(flags, FAULT_REPEAT);
    }
    keys[i] = static_cast<uint64_t>(n) * static_cast<uint64_t>(n_nodes) + static_cast<uint64_t>(m);
}

__global__ void k_pair_split(const uint64_t *keys, int64_t nnz, int64_t n_nodes, int32_t *cnt, int32_t *cols)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    const uint64_t k = keys[i];
    const int64_t row = static_cast<int64_t>(k / static_cast<uint64_t>(n_nodes));
    cols[i] = static_cast<int32_t>(k - static_cast<uint64_t>(row) * static_cast<uint64_t>(n_nodes));
    atomicAdd(&cnt[row], 1);  // integer counts: the result does not depend on the order
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS bytes of one row's columns and block accumulators
template <typename T, int NC>
constexpr size_t row_lds(int len)
{
    return ((size_t)len * 4 + 15) / 16 * 16 + (size_t)len * NC * NC * sizeof(T);
}

template <typename T, int NC>
__global__ __launch_bounds__(64) void k_asm_rows(const int32_t *row_ptr, const int32_t *cols,
                                                 const int32_t *inc_off, const int32_t *inc_items,
                                                 const int32_t *conn, int nb, const T *K, double scale, T *values)
{
    extern __shared__ __align__(16) unsigned char sm[];
    constexpr int B = NC * NC;
    const int64_t n = blockIdx.x;
    const int lane = threadIdx.x;
    const int r0 = row_ptr[n], len = row_ptr[n + 1] - r0;
    int32_t *sc = reinterpret_cast<int32_t *>(sm);
    T *acc = reinterpret_cast<T *>(sm + ((size_t)len * 4 + 15) / 16 * 16);
    for (int k = lane; k < len; k += 64) sc[k] = cols[r0 + k];
    for (int k = lane; k < len * B; k += 64) acc[k] = T(0);
    wave_sync();
    const int nd = NC * nb;
    const T s = static_cast<T>(scale);
    const int i1 = inc_off[n + 1];
    for (int it = inc_off[n]; it < i1; it++) {
        const int32_t item = inc_items[it];
        const int64_t e = item / nb;
        const int a = item - static_cast<int>(e) * nb;
        if (lane < nb) {
            const int32_t m = conn[e * nb + lane];
            int lo = 0, hi = len - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sc[mid] < m) lo = mid + 1;
                else hi = mid;
            }
            const T *Ke = K + e * (int64_t)nd * nd + a * nd + lane;
            T *v = acc + lo * B;
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int d = 0; d < NC; d++) v[c * NC + d] += s * Ke[(int64_t)c * nb * nd + d * nb];
        }
        wave_sync();  // the next step may add to a slot another lane wrote
    }
    T *out = values + (int64_t)r0 * B;
    for (int k = lane; k < len * B; k += 64) out[k] = acc[k];
}

int bits_for(uint64_t x)
{
    int b = 1;
    while (b < 64 && (x >> b) != 0) b++;
    return b;
}

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" {

int fe_pattern_create(int64_t n_cells, int64_t n_nodes, int n_basis, const int32_t *conn, void *stream,
                      fe_pattern *out)
{
    if (!out) {
        set_error("out is NULL");
        return FE_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (n_cells < 0 || n_nodes <= 0 || n_basis <= 0 || (n_cells > 0 && !conn)) {
        set_error("bad pattern arguments");
        return FE_ERR_INVALID_ARG;
    }
    const int64_t n_pairs = n_cells * (int64_t)n_basis * n_basis;
    if (n_pairs >= 0x7fffffffLL || n_nodes >= 0x7fffffffLL) {
        set_error("too many node pairs for one pattern (n_cells * n_basis^2 must stay below 2^31)");
        return FE_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        set_error("no HIP device");
        return FE_ERR_NO_DEVICE;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    fe_pattern_s *p = new (std::nothrow) fe_pattern_s();
    if (!p) {
        set_error("host allocation failed");
        return FE_ERR_OUT_OF_MEMORY;
    }
    p->n_nodes = n_nodes;
    p->nb = n_basis;
    p->device = dev;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    int32_t *cnt = nullptr, *nsel = nullptr;
    unsigned *flags = nullptr;
    void *tmp = nullptr;
    auto cleanup = [&]() {
        for (void *q : {(void *)k0, (void *)k1, (void *)cnt, (void *)nsel, (void *)flags, tmp})
            if (q) (void)hipFree(q);
    };
    auto fail_hip = [&](const char *what) {
        (void)hipGetLastError();
        cleanup();
        fe_pattern_destroy(p);
        set_error(what);
        return FE_ERR_HIP;
    };
    const int64_t np = n_pairs > 0 ? n_pairs : 1;
    if (hipMalloc(&k0, np * sizeof(uint64_t)) != hipSuccess || hipMalloc(&k1, np * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&cnt, (n_nodes + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&nsel, sizeof(int32_t)) != hipSuccess || hipMalloc(&flags, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&p->row_ptr, (n_nodes + 1) * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        fe_pattern_destroy(p);
        set_error("pattern allocation failed");
        return FE_ERR_OUT_OF_MEMORY;
    }
    if (hipMemsetAsync(cnt, 0, (n_nodes + 1) * sizeof(int32_t), st) != hipSuccess ||
        hipMemsetAsync(flags, 0, sizeof(unsigned), st) != hipSuccess ||
        hipMemsetAsync(nsel, 0, sizeof(int32_t), st) != hipSuccess)
        return fail_hip("hipMemsetAsync failed");
    const int items = static_cast<int>(n_pairs);
    if (items > 0) {
        hipLaunchKernelGGL(k_pair_keys, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, st, conn, n_cells,
                           n_basis, n_nodes, k0, flags);
        const int end_bit = bits_for(static_cast<uint64_t>(n_nodes) * static_cast<uint64_t>(n_nodes));
        size_t b_sort = 0, b_uniq = 0;
        if (hipcub::DeviceRadixSort::SortKeys(nullptr, b_sort, k0, k1, items, 0, end_bit, st) != hipSuccess ||
            hipcub::DeviceSelect::Unique(nullptr, b_uniq, k1, k0, nsel, items, st) != hipSuccess)
            return fail_hip("radix sort sizing failed");
        const size_t b_tmp = b_sort > b_uniq ? b_sort : b_uniq;
        if (hipMalloc(&tmp, b_tmp ? b_tmp : 1) != hipSuccess) return fail_hip("temporary allocation failed");
        size_t bs = b_tmp;
        if (hipcub::DeviceRadixSort::SortKeys(tmp, bs, k0, k1, items, 0, end_bit, st) != hipSuccess)
            return fail_hip("radix sort failed");
        bs = b_tmp;
        if (hipcub::DeviceSelect::Unique(tmp, bs, k1, k0, nsel, items, st) != hipSuccess)
            return fail_hip("unique failed");
    }
    int32_t h_nsel = 0;
    unsigned h_flags = 0;
    if (hipMemcpyAsync(&h_nsel, nsel, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&h_flags, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail_hip("pattern size read failed");
    if (h_flags & FAULT_INDEX) {
        cleanup();
        fe_pattern_destroy(p);
        set_error("a connectivity entry is out of range");
        return FE_ERR_INDEX_OUT_OF_RANGE;
    }
    if (h_flags & FAULT_REPEAT) {
        cleanup();
        fe_pattern_destroy(p);
        set_error("a cell lists the same node twice");
        return FE_ERR_INVALID_ARG;
    }
    p->nnz = h_nsel;
    if (hipMalloc(&p->cols, (p->nnz > 0 ? p->nnz : 1) * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        fe_pattern_destroy(p);
        set_error("pattern allocation failed");
        return FE_ERR_OUT_OF_MEMORY;
    }
    if (p->nnz > 0)
        hipLaunchKernelGGL(k_pair_split, dim3((unsigned)((p->nnz + 255) / 256)), dim3(256), 0, st, k0, p->nnz, n_nodes,
                           cnt, p->cols);
    size_t b_scan = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, b_scan, cnt, p->row_ptr, (int)(n_nodes + 1), st) != hipSuccess)
        return fail_hip("prefix sum sizing failed");
    if (tmp) (void)hipFree(tmp);
    tmp = nullptr;
    if (hipMalloc(&tmp, b_scan ? b_scan : 1) != hipSuccess) return fail_hip("temporary allocation failed");
    if (hipcub::DeviceScan::ExclusiveSum(tmp, b_scan, cnt, p->row_ptr, (int)(n_nodes + 1), st) != hipSuccess)
        return fail_hip("prefix sum failed");
    // the longest row sizes the LDS of the assembly kernel
    size_t b_max = 0;
    if (hipcub::DeviceReduce::Max(nullptr, b_max, cnt, nsel, (int)n_nodes, st) != hipSuccess)
        return fail_hip("row length sizing failed");
    if (tmp) (void)hipFree(tmp);
    tmp = nullptr;
    if (hipMalloc(&tmp, b_max ? b_max : 1) != hipSuccess) return fail_hip("temporary allocation failed");
    int32_t h_max = 0;
    if (hipcub::DeviceReduce::Max(tmp, b_max, cnt, nsel, (int)n_nodes, st) != hipSuccess ||
        hipMemcpyAsync(&h_max, nsel, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail_hip("row length reduction failed");
    p->max_row = h_max;
    cleanup();
    *out = p;
    return FE_OK;
}

int fe_pattern_info(fe_pattern p, int64_t *n_nodes, int64_t *nnz)
{
    if (!p) {
        set_error("pattern is NULL");
        return FE_ERR_INVALID_ARG;
    }
    if (n_nodes) *n_nodes = p->n_nodes;
    if (nnz) *nnz = p->nnz;
    return FE_OK;
}

int fe_pattern_copy(fe_pattern p, int32_t *row_ptr, int32_t *cols, void *stream)
{
    if (!p || (!row_ptr && !cols)) {
        set_error("bad argument");
        return FE_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (row_ptr)
        FE_HIP_CHECK(hipMemcpyAsync(row_ptr, p->row_ptr, (p->n_nodes + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (cols && p->nnz > 0)
        FE_HIP_CHECK(hipMemcpyAsync(cols, p->cols, p->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return FE_OK;
}

int fe_pattern_destroy(fe_pattern p)
{
    if (!p) return FE_OK;
    if (p->row_ptr) (void)hipFree(p->row_ptr);
    if (p->cols) (void)hipFree(p->cols);
    delete p;
    return FE_OK;
}

int fe_assemble_matrix(fe_pattern pat, fe_incidence inc, const int32_t *conn, int n_comp, int precision,
                       const void *cell_mats, double scale, void *values, void *stream)
{
    if (!pat || !inc || !conn || !cell_mats || !values || (n_comp != 1 && n_comp != 3) ||
        precision < FE_PREC_FP64 || precision > FE_PREC_BF16X3) {
        set_error("bad matrix assembly arguments");
        return FE_ERR_INVALID_ARG;
    }
    if (inc->n_nodes != pat->n_nodes || inc->nb != pat->nb) {
        set_error("incidence and pattern belong to different connectivities");
        return FE_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != pat->device || dev != inc->device) {
        set_error("pattern or incidence was created on another device");
        return FE_ERR_INVALID_ARG;
    }
    if (pat->n_nodes == 0 || inc->n_cells == 0) return FE_OK;
    if (pat->nb > 64) {
        set_error("matrix assembly takes at most 64 nodes per cell");
        return FE_ERR_UNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool f64 = precision == FE_PREC_FP64;
    const size_t lds = f64 ? (n_comp == 1 ? row_lds<double, 1>(pat->max_row) : row_lds<double, 3>(pat->max_row))
                           : (n_comp == 1 ? row_lds<float, 1>(pat->max_row) : row_lds<float, 3>(pat->max_row));
    if (lds > 160 * 1024) {
        set_error("a pattern row is too long for the LDS of the assembly kernel");
        return FE_ERR_UNSUPPORTED;
    }
    if (pat->n_nodes > 0x7fffffffLL) {
        set_error("too many rows for one launch");
        return FE_ERR_INVALID_ARG;
    }
    const dim3 grid((unsigned)pat->n_nodes), block(64);
    const int nb = pat->nb;
    auto go = [&](auto kernel, const auto *K, auto *V) -> int {
        if (lds > 64 * 1024)
            FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kernel, grid, block, lds, st, pat->row_ptr, pat->cols, inc->offsets, inc->items, conn, nb,
                           K, scale, V);
        return FE_OK;
    };
    int rc;
    if (f64)
        rc = n_comp == 1 ? go(k_asm_rows<double, 1>, static_cast<const double *>(cell_mats), static_cast<double *>(values))
                         : go(k_asm_rows<double, 3>, static_cast<const double *>(cell_mats), static_cast<double *>(values));
    else
        rc = n_comp == 1 ? go(k_asm_rows<float, 1>, static_cast<const float *>(cell_mats), static_cast<float *>(values))
                         : go(k_asm_rows<float, 3>, static_cast<const float *>(cell_mats), static_cast<float *>(values));
    if (rc) return rc;
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

}  // extern "C"
