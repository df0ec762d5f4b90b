// y = A x for callers that cannot allocate device memory: the product of
// h2_matvec with its intermediate vectors (x^, y^, the near field and the
// partial sums of a split stream list) in a static device array instead of
// the handle's workspace.  Every call on a GPU uses that GPU's one copy of
// the array, so calls that overlap on one GPU race; nothing in it has to
// start at zero (every element the product reads, it has written before in
// the same call).
#include "h2_internal.h"

namespace {

constexpr int64_t kScratchBytes = int64_t(H2_NOALLOC_SCRATCH_BYTES);

// Module-scope device memory, one copy per GPU, held until the process ends.
// In host code this name is a stand-in for the symbol, not a device address:
// kernels receive the address hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of scratch (looked up at the first
// call on that GPU).
char *scratch_on_current_device() {
    int dev = 0;
    h2i::check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) h2i::fail(H2_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        h2i::check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<char *>(g_scratch_ptr[dev]);
}

}  // namespace

using namespace h2i;

extern "C" {

h2_status h2_matvec_noalloc(h2_handle A, const double *x, double *y, void *stream) {
    try {
        if (!A || !x || !y) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        int64_t part[4];
        workspace_bytes(*A, part);
        const int64_t need = part[0] + part[1] + part[2] + part[3];
        if (need > kScratchBytes)
            fail(H2_ERR_UNSUPPORTED, "h2_matvec_noalloc: the product needs " + std::to_string(need) +
                                         " bytes of scratch, more than the static " +
                                         std::to_string(kScratchBytes));
        char *base = scratch_on_current_device();
        const Workspace ws{base, base + part[0], base + part[0] + part[1], base + part[0] + part[1] + part[2]};
        run_product(*A, x, y, static_cast<hipStream_t>(stream), &ws);
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

}  // extern "C"
