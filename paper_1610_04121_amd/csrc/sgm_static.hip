// Allocation-free entry point (sgm_compute_noalloc, declared in
// include/sgm.h): the whole pipeline of sgm_compute, with the pair's
// workspace (cost volume, L_r planes, census words, raw maps) carved out of
// one file-scope device array instead of a hipMalloc'ed buffer.
//
// The array is a static __device__ variable, so every GPU the library runs on
// holds its own copy, at its own address, from the moment the code object is
// loaded until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host that name is only a stand-in): its
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and kept in a per-device table.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/sgm.h"
#include "sgm_plan.h"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // SGM_NOALLOC_MAX_BYTES
static_assert(kScratchBytes == SGM_NOALLOC_MAX_BYTES, "header and library disagree on the scratch size");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int fail(int code, const std::string& msg) {
    sgm::set_last_error(msg);
    return code;
}

// Device address of this device's copy of the scratch array (looked up on
// the first call on the device).  The current device is `dev`.
int scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(SGM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SGM_OK;
}

}  // namespace

extern "C" {

int sgm_compute_noalloc(int width, int height, int max_disp, int P1, int P2, int n_paths, int census_w,
                        int census_h, unsigned flags, int lr_threshold, const uint8_t* left, const uint8_t* right,
                        uint16_t* disp_out, sgm_stream_t stream) {
    if (flags & SGM_GRAPH) return fail(SGM_EINVAL, "SGM_GRAPH is not available without a context");
    sgm::Plan p;
    if (!sgm::plan_from_options(p, width, height, max_disp, P1, P2, n_paths, census_w, census_h, flags,
                                lr_threshold))
        return SGM_EINVAL;
    if (!left || !right || !disp_out) return fail(SGM_EINVAL, "null buffer pointer");
    if ((const void*)disp_out == (const void*)left || (const void*)disp_out == (const void*)right)
        return fail(SGM_EINVAL, "output aliases an input");
    const size_t need = sgm::workspace_bytes(p);
    if (need > kScratchBytes)
        return fail(SGM_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                    std::to_string(kScratchBytes) + "-byte static scratch of sgm_compute_noalloc");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SGM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SGM_EHIP, "device index out of range");
    void* base = nullptr;
    if (int rc = scratch_address(dev, &base)) return rc;
    // every buffer of the workspace is fully written before it is read in a
    // pass, so nothing needs clearing between calls
    const sgm::Workspace ws = sgm::workspace_carve(p, base);
    e = sgm::launch_pipeline(p, ws, left, right, disp_out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SGM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SGM_OK;
}

}  // extern "C"
