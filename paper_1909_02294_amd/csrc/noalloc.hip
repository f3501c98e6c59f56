// ivde_cost_volume_noalloc: the plain cost volume with its workspace in a
// fixed device array of the library instead of caller memory, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops that forbid allocation).  It runs the same kernels in the same order
// as ivde_cost_volume, so its results are bitwise those of that call.
//
// The array is one file-scope __device__ object: every GPU the library runs
// on holds its own copy until the process ends, at its own address.  In host
// code the array's name only stands in for the device object, so the device
// address is looked up once per device with hipGetSymbolAddress and only that
// address is ever passed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

namespace ivde {
namespace {

static __device__ __align__(256) unsigned char scratch[IVDE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call made with that device current.
ivde_status scratch_address(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index %d beyond the %d devices the scratch table covers", dev, kMaxDevices);
        return IVDE_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) {
            set_error("hipGetSymbolAddress(scratch) returned a null address");
            return IVDE_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_scratch_ptr[dev]);
    return IVDE_OK;
}

}  // namespace
}  // namespace ivde

using namespace ivde;

extern "C" ivde_status ivde_cost_volume_noalloc(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                                                const ivde_segmentation *segs, const ivde_label_range *labels,
                                                const ivde_options *opt, void *cost_out, ivde_stream stream)
{
    ivde_status st = validate_problem(n_views, cams, views, segs, labels, opt, true);
    if (st != IVDE_OK) return st;
    if (!cost_out) {
        set_error("null cost_out");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, labels, opt, views[0].bit_depth);
    if (ly.workspace_bytes > (size_t)IVDE_NOALLOC_SCRATCH_BYTES) {
        set_error("ivde_cost_volume_noalloc: the problem needs %zu bytes of workspace, more than the %zu bytes of "
                  "the library's fixed scratch array; call ivde_cost_volume with a workspace instead",
                  ly.workspace_bytes, (size_t)IVDE_NOALLOC_SCRATCH_BYTES);
        return IVDE_ENOMEM;
    }
    if ((st = check_tex_limits(ly)) != IVDE_OK) return st;
    char *ws = nullptr;
    if ((st = scratch_address(&ws)) != IVDE_OK) return st;
    return enqueue_cost_volume(n_views, cams, views, segs, labels, opt, ly, ws, cost_out,
                               static_cast<hipStream_t>(stream));
}
