// fof_label_noalloc: build + link + finalize of one box on a library-owned
// scratch array instead of a caller's workspace, for callers that cannot
// allocate memory. Same kernels and launch sequence as fof_build_cells +
// fof_link + fof_finalize.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/fof.h"
#include "fof_internal.h"

constexpr size_t kScratchBytes = (size_t)FOF_NOALLOC_SCRATCH_BYTES;

// The scratch: one copy per GPU, in the code object's device memory, held
// until the process ends. Its name is a host-side stand-in in host code: the
// device address of each GPU's copy comes from hipGetSymbolAddress (once per
// device, with that device current) and only that address is handed to
// kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the first call on
// that device; nullptr if the lookup fails.
void *scratch_address(int *device)
{
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices) return nullptr;
    *device = d;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[d]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch[d] = ptr;
    }
    return g_scratch[d];
}

}  // namespace

extern "C" fof_status fof_label_noalloc(const fof_options *opt, void *hip_stream, const float *d_pos, int64_t n,
                                        double box, double lx, int32_t *d_group_index, int32_t *d_group_size,
                                        int64_t *h_n_groups)
{
    fof_options o;
    if (opt) {
        o = *opt;
    } else {
        std::memset(&o, 0, sizeof(o));
        o.predicate = FOF_PRED_FP32_FILTER;
    }
    if (o.collect_timings) return FOF_ERR_INVALID_ARG;   // timing events are not kept here
    if (n > 0 && (!d_pos || !d_group_index || !d_group_size)) return FOF_ERR_INVALID_ARG;
    // validation and the size check come first, before any device call
    fof::Plan p{};
    size_t need = 0;
    fof_status st = fof::plan_one_box(o, n, box, lx, nullptr, kScratchBytes, &p, &need);
    if (st != FOF_OK) return st;
    if (need > kScratchBytes) return FOF_ERR_UNSUPPORTED;
    int device = -1;
    void *ws = scratch_address(&device);
    if (!ws) return FOF_ERR_DEVICE;
    st = fof::plan_one_box(o, n, box, lx, ws, kScratchBytes, &p, &need);
    if (st != FOF_OK) return st;
    p.pos = d_pos;
    p.label = d_group_index;
    p.size = d_group_size;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // every array the run reads is written by it first (k_clear zeroes the
    // counters, group counts and segment counts), so the previous call's
    // contents do not matter
    hipError_t e = fof::launch_clear(p, s, nullptr);
    if (e == hipSuccess) e = fof::launch_build(p, s, nullptr);
    if (e == hipSuccess) e = fof::launch_link(p, s, nullptr);
    if (e == hipSuccess) e = fof::launch_finalize(p, s, nullptr);
    if (e != hipSuccess) return FOF_ERR_DEVICE;
    if (!h_n_groups) return FOF_OK;
    unsigned long long groups = 0;
    unsigned int error = 0;
    if (hipMemcpyAsync(&groups, p.n_groups, sizeof(groups), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&error, &p.counters->error, sizeof(error), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FOF_ERR_DEVICE;
    *h_n_groups = (int64_t)groups;
    if (error & 2u) return FOF_ERR_DEVICE;
    return (error & 1u) ? FOF_ERR_OUT_OF_BOX : FOF_OK;
}
