// noalloc.hip -- the fixed device scratch of the entry points that allocate nothing.
//
// kur_diagnostics folds per-chunk FP64 partial sums (3 per chunk of 256 rows) into three totals;
// it allocates that scratch for every call. kur_diagnostics_noalloc uses instead the file-scope
// array below, one copy per GPU for the life of the process, sized for n <= kNoAllocMaxN. Its
// device address is looked up once per device (hipGetSymbolAddress, with the device current)
// when the first context on that device is created, and only that address is handed to kernels
// and copies: in host code the array's name does not denote device memory.
//
// Every call on a GPU shares that GPU's array and leaves its contents behind. Nothing in it needs
// to start at zero: each call writes every partial it later reads. Calls that overlap in time on
// one GPU (two streams or two threads) race on the array and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kur_noalloc.hpp"

namespace kur {

namespace {

constexpr int64_t kChunksMax = kNoAllocMaxN / 256;
constexpr int64_t kScratchDoubles = 3 * kChunksMax + 4;  // partials, then the three totals (+ pad)

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        g_ptr[device] = p;
        g_err[device] = e;
        g_done[device] = true;
    }
    return g_err[device];
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_done[device] && g_err[device] == hipSuccess ? g_ptr[device] : nullptr;
}

size_t noalloc_scratch_bytes() { return sizeof(double) * (size_t)kScratchDoubles; }

int64_t noalloc_totals_offset() { return 3 * kChunksMax; }

}  // namespace kur
