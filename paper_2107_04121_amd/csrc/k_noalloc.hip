// fe_execute_noalloc: fe_execute without a caller workspace.  The fault bits
// and the matrix-first chunk of element matrices live in a file-scope device
// array instead, so the call allocates nothing and takes no workspace (for
// callers that cannot allocate device memory).
//
// Host code never passes the array's name to a kernel: on the host that name
// is only a stand-in.  The array's device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and kept; every
// kernel argument and clear uses that address.
#include "fe_device.h"

#include <atomic>
#include <string>

namespace fe {
namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;  // 64 MiB per device
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::atomic<void *> g_scratch_ptr[MAX_DEVICES];

__global__ void k_clear_fault_word(unsigned *flags) { flags[0] = 0u; }

__global__ void k_copy_fault_word(const unsigned *flags, unsigned *fault_out) { fault_out[0] = flags[0]; }

// Device address of this device's scratch array (looked up on first use).
int scratch_ptr(void **out)
{
    int dev = -1;
    FE_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(FE_ERR_INVALID_ARG, "device index beyond 63");
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        FE_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FE_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return FE_OK;
}

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" {

int fe_execute_noalloc(fe_plan p, int64_t n_cells, int64_t n_nodes, const double *coords, const int32_t *conn,
                       const void *material, const void *dofs, void *out, unsigned *fault_out, void *stream)
{
    if (!p) return fail(FE_ERR_INVALID_ARG, "plan is NULL");
    if (n_cells < 0) return fail(FE_ERR_INVALID_ARG, "negative size");
    const size_t need = workspace_bytes_of(*p, n_cells);
    if (need > SCRATCH_BYTES)
        return fail(FE_ERR_INVALID_ARG,
                    "this call needs " + std::to_string(need) + " bytes of scratch (fault bits and one matrix-first "
                    "chunk of element matrices), the static scratch holds " + std::to_string(SCRATCH_BYTES) +
                    "; create the plan with a smaller matrix-first chunk or use fe_execute with a workspace");
    void *ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned *flags = static_cast<unsigned *>(ws);
    hipLaunchKernelGGL(k_clear_fault_word, dim3(1), dim3(1), 0, st, flags);
    FE_HIP_CHECK(hipGetLastError());
    rc = execute_impl(p, n_cells, n_nodes, coords, conn, material, dofs, out, ws, SCRATCH_BYTES, st);
    if (rc) return rc;
    if (fault_out) {
        hipLaunchKernelGGL(k_copy_fault_word, dim3(1), dim3(1), 0, st, flags, fault_out);
        FE_HIP_CHECK(hipGetLastError());
    }
    return FE_OK;
}

}  // extern "C"
