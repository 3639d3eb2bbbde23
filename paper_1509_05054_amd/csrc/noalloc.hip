// The error ||Y - D X||_F / sqrt(p m) with its scratch in a static device
// array instead of a caller workspace, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).
//
// The scratch holds the error's control words (the non-finite counter) and
// its block partials.  The partial pass never uses more than
// kRmseMaxPartials workgroups, whatever the number of signals, so the array
// has a fixed size: every size dl_rmse accepts fits it.  Each GPU the library
// runs on holds its own copy of the array, whose address is looked up once
// per device (hipGetSymbolAddress) and kept; host code never passes the
// array's own name to a kernel.  Every call on a GPU shares that GPU's array:
// calls that overlap in time on one GPU race.
#include <mutex>

#include "dl_internal.h"

namespace dlk {
namespace {

constexpr size_t kScratchControl = 256;  // Control, padded to 256 bytes
constexpr size_t kScratchBytes = kScratchControl + sizeof(double) * kRmseMaxPartials;
static_assert(sizeof(Control) <= kScratchControl, "control words exceed their scratch slot");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The scratch address on the current device (looked up on first use), or
// null on failure.
void *scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

// Clears the control words (a fill kernel, not hipMemsetAsync, so that the
// call can be captured in a graph).
__global__ void clear_words(unsigned int *w, int words)
{
    for (int k = threadIdx.x; k < words; k += blockDim.x)
        w[k] = 0u;
}

bool aligned(const void *ptr, size_t a) { return ptr && ((uintptr_t)ptr % a) == 0; }

}  // namespace
}  // namespace dlk

using namespace dlk;

extern "C" {

dl_status dl_rmse_noalloc(const dl_params *prm, const float *Y, const float *D,
                          const int32_t *X_idx, const float *X_val, double *rmse_out,
                          dl_stream_t stream)
{
    if (!params_ok(prm) || !aligned(Y, 16) || !aligned(D, 16) || !aligned(X_idx, 4) ||
        !aligned(X_val, 4) || !aligned(rmse_out, 8))
        return DL_EINVAL;
    if (rmse_blocks(prm->m) > kRmseMaxPartials)
        return DL_EINVAL;  // more partials than the scratch holds (never for a valid m)
    char *base = (char *)scratch_ptr();
    if (!base)
        return DL_EHIP;
    hipStream_t st = (hipStream_t)stream;
    Control *ctl = reinterpret_cast<Control *>(base);
    hipLaunchKernelGGL(clear_words, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned int *>(ctl),
                       (int)(sizeof(Control) / sizeof(unsigned int)));
    if (hipGetLastError() != hipSuccess)
        return DL_EHIP;
    RmseArgs r;
    r.Y = Y;
    r.D = D;
    r.idx = X_idx;
    r.val = X_val;
    r.partial = reinterpret_cast<double *>(base + kScratchControl);
    r.out = rmse_out;
    r.ctl = ctl;
    r.p = prm->p;
    r.n = prm->n;
    r.m = prm->m;
    r.s = prm->s;
    if (launch_rmse_unprofiled(r, st) != hipSuccess)
        return DL_EHIP;
    return DL_OK;
}

}  // extern "C"
