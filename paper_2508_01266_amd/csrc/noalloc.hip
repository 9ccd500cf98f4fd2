// The static device array behind the no-allocation sigma entry point
// (lrcc_apply_sigma_dev_noalloc): the work tensors and launch tables of the sigma
// program live here instead of in memory the library allocates.  Each device the
// library runs on holds one copy until the process ends; every call on a device
// shares it (calls that overlap on one device race).
#include "common.hpp"
#include "plan.hpp"

namespace lrcc {

namespace {
constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;
}

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Address of `scratch` on device `dev` (which must be current): each device holds its own copy
// at its own address, so it is looked up once per device; the host-side name is not a device
// address and is never passed on.
void *noalloc_scratch(int dev, size_t *bytes) {
    static void *ptr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) throw LrccError(1, "device index beyond the static array table");
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw LrccError(5, std::string("hipGetSymbolAddress of the static array: ") + hipGetErrorString(e));
        ptr[dev] = p;
        arena_register(p, kScratchBytes);
    }
    *bytes = kScratchBytes;
    return ptr[dev];
}

}  // namespace lrcc
