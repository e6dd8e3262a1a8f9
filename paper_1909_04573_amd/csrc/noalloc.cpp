// Noise residuals for callers that cannot allocate device memory (code under
// stream capture, tight serving loops, hosts that forbid allocation): the
// scratch the denoiser needs (the wavelet pyramid of a batch of planes) is one
// file-scope device array per GPU instead of a caller workspace.
//
// Host code never passes the array's name to a kernel: the name is a host
// stand-in, not a device address.  The array's address on each device is
// looked up once, with that device current, and kept per device.

#include <mutex>

#include "host.h"
#include "internal.h"

namespace prnu {
constexpr size_t kStaticScratchBytes = PRNU_STATIC_SCRATCH_BYTES;  // one 4000 x 3000 plane's pyramid fits
constexpr int kMaxScratchDevices = 64;
}  // namespace prnu

static __device__ __align__(256) unsigned char scratch[prnu::kStaticScratchBytes];

namespace prnu {
namespace {

std::mutex g_scratch_mu;
void *g_scratch[kMaxScratchDevices];

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int scratch_address(void **out, const char *fn) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PRNU_E_HIP, "%s: hipGetDevice failed: %s", fn, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(PRNU_E_INVAL, "%s: device %d beyond the %d this library serves", fn, dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PRNU_E_HIP, "%s: hipGetSymbolAddress of the scratch array failed: %s", fn,
                        hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PRNU_OK;
}

}  // namespace
}  // namespace prnu

using namespace prnu;

extern "C" {

int prnu_denoise_residual_noalloc(const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                                  float *resid, void *stream) {
    const char *fn = "prnu_denoise_residual_noalloc";
    set_error("");
    if (!img || !resid) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (img == resid) return fail(PRNU_E_INVAL, "%s: resid may not alias img", fn);
    if (n_img < 1) return fail(PRNU_E_INVAL, "%s: n_img must be >= 1", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    const int nb = denoise_planes_fitting(H, W, p, kStaticScratchBytes);
    if (nb < 1)
        return fail(PRNU_E_INVAL, "%s: the wavelet pyramid of one %d x %d plane exceeds the %zu-byte static scratch",
                    fn, H, W, kStaticScratchBytes);
    void *ws = nullptr;
    PRNU_TRY(scratch_address(&ws, fn));
    return denoise_run(fn, img, n_img, H, W, p, resid, nullptr, ws, kStaticScratchBytes, stream, nb);
}

}  // extern "C"
