// Scratch memory of evq_query_noalloc, the query entry point for callers that
// cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  It is one file-scope device array per
// GPU, held until the process ends.  Host code never names the array as an
// address: the first call on a device looks its device address up once (with
// that device current) and every later use goes through that pointer.  Every
// call on one GPU shares the array and finds whatever the last call left in
// it; the query clears what must start at zero with kernels of its own.
#include <mutex>

#include "evq_internal.h"

namespace evq {

namespace {

constexpr uint64_t kScratchBytes = 128ull << 20;  // 128 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

char* noalloc_scratch(int device, uint64_t* bytes) {
    if (device < 0 || device >= kMaxDevices) fail(EVQ_EDEVICE, "device id out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        EVQ_HIP(hipGetDevice(&cur));
        if (cur != device) fail(EVQ_EDEVICE, "scratch lookup with another device current");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(EVQ_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                  hipGetErrorString(e));
        }
        g_scratch_ptr[device] = static_cast<char*>(p);
    }
    if (bytes) *bytes = kScratchBytes;
    return g_scratch_ptr[device];
}

}  // namespace evq
