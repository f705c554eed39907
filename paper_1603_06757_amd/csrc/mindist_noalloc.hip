// mindist_noalloc.hip -- mindist_run_noalloc: the single-code path (Section
// 2's information sets and Gamma_j, Algorithm 1's pair loop) with no device
// or pinned allocation.  Its device state lives in one static device buffer
// per GPU, of MINDIST_NOALLOC_BYTES, held until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/mindist.h"
#include "mindist_plan.h"

namespace md {
int noalloc_run(unsigned char *base, uint64_t bytes, bool *binom_ready, const uint64_t *G, int n, int k,
                hipStream_t stream, mindist_result *out, mindist_pair *pairs, int cap, int *n_pairs);
}

// The fixed buffer.  In host code this name is only a stand-in for the
// device symbol: its device address comes from hipGetSymbolAddress, per GPU.
static __device__ __align__(256) unsigned char scratch[MINDIST_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
struct PerDevice {
    std::mutex mu;                 // calls on one GPU share its buffer: one at a time
    unsigned char *ptr = nullptr;  // device address of scratch on this GPU
    bool binom_ready = false;      // the constant binomial table is in place
};
PerDevice g_dev[kMaxDevices];
}  // namespace

extern "C" int mindist_run_noalloc(const uint64_t *G, int n, int k, int64_t stream, mindist_result *out,
                                   mindist_pair *pairs, int pairs_cap, int *n_pairs) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return md::fail(MINDIST_E_HIP, "no HIP device");
    if (dev < 0 || dev >= kMaxDevices) return md::fail(MINDIST_E_LIMIT, "device index beyond 63");
    PerDevice &pd = g_dev[dev];
    std::lock_guard<std::mutex> lk(pd.mu);
    if (!pd.ptr) {
        // set-up, once per device with that device current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return md::fail(MINDIST_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        pd.ptr = static_cast<unsigned char *>(p);
    }
    return md::noalloc_run(pd.ptr, MINDIST_NOALLOC_BYTES, &pd.binom_ready, G, n, k, (hipStream_t)stream, out,
                           pairs, pairs_cap, n_pairs);
}
