// Static device scratch for the entry point that allocates nothing
// (hphi_lanczos_noalloc): a file-scope array each GPU holds from module
// load to process end. Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); the device
// address comes from hipGetSymbolAddress, taken once per device while that
// device is current, and everything else uses that address.
#include <atomic>
#include <mutex>

#include "internal.h"

namespace hphi {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
std::atomic<int> g_busy[kMaxDevices] = {};
} // namespace

int noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(HPHI_ERR_UNSUPPORTED, "device %d: no static scratch", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return HPHI_OK;
    int cur = -1;
    HPHI_HIP(hipGetDevice(&cur));
    if (cur != device) return fail(HPHI_ERR_DEVICE, "static scratch set-up on device %d while %d is current", device, cur);
    void *p = nullptr;
    HPHI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HPHI_ERR_DEVICE, "no device address for the static scratch");
    g_ptr[device] = p;
    return HPHI_OK;
}

int noalloc_scratch_acquire(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices || !g_ptr[device])
        return fail(HPHI_ERR_DEVICE, "static scratch of device %d not set up (hphi_init)", device);
    int expected = 0;
    if (!g_busy[device].compare_exchange_strong(expected, 1))
        return fail(HPHI_ERR_BUSY, "the static scratch of device %d is in use by another call", device);
    *ptr = g_ptr[device];
    return HPHI_OK;
}

void noalloc_scratch_release(int device)
{
    if (device >= 0 && device < kMaxDevices) g_busy[device].store(0);
}

// Zero `bytes` bytes (a multiple of 4, 4-byte aligned) with a kernel
// instead of a memset.
__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int launch_zero(void *p, size_t bytes, hipStream_t st)
{
    if (bytes % 4 || ((uintptr_t)p & 3u)) return fail(HPHI_ERR_INVALID_ARG, "zero fill of %zu bytes", bytes);
    const int64_t n = (int64_t)(bytes / 4);
    if (n == 0) return HPHI_OK;
    const int g = (int)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero_u32, dim3(g), dim3(256), 0, st, static_cast<uint32_t *>(p), n);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi
