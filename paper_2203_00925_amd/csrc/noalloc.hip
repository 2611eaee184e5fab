// mifvm_conservation_static: the conservation total of mifvm_conservation
// with its reduction scratch (per-block partials, per-mesh totals, the
// result) in a fixed device array of this library instead of the state's
// workspace and pinned host mirror, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mifvm.h"
#include "api_util.h"
#include "state.h"

using namespace mifvm;
using namespace mifvm_api;

namespace {

constexpr int kMaxDevices = 64;
// [0, kPartials): per-block partial sums (at most 1024 blocks per mesh);
// then SC_COUNT_ scalar slots for each of up to MIFVM_STATIC_MAX_MESHES meshes; then
// the total over the meshes
constexpr int64_t kPartials = 1024;
constexpr int64_t kScratchDoubles = kPartials + int64_t(MIFVM_STATIC_MAX_MESHES) * SC_COUNT_ + 8;
static_assert(kScratchDoubles * 8 == MIFVM_STATIC_SCRATCH_BYTES, "scratch size differs from the header's");

}  // namespace

// Every GPU holds its own copy until the process ends.  Host code never
// passes this name to a kernel or a copy: it is a host-side stand-in; the
// device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// the device address of this device's copy of `scratch`, looked up once per
// device with that device current
int scratch_ptr(double** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MIFVM_E_ARG, "device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MIFVM_E_HIP, "hipGetSymbolAddress returned a null address");
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return MIFVM_OK;
}

// the meshes' totals summed in mesh order from 0 (the order of the host sum
// of mifvm_conservation)
__global__ void k_sum_meshes(const double* __restrict__ scal, int nm, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t = 0.0;
    for (int m = 0; m < nm; ++m) t += scal[int64_t(m) * SC_COUNT_ + SC_CONS];
    *out = t;
}

}  // namespace

extern "C" int mifvm_conservation_static(mifvm_state* st, double* total_out, void* stream) {
    if (!st || !total_out) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    if (s.d.nm > MIFVM_STATIC_MAX_MESHES)
        return fail(MIFVM_E_ARG, "mifvm_conservation_static handles at most " +
                                     std::to_string(MIFVM_STATIC_MAX_MESHES) + " meshes; the state has " +
                                     std::to_string(s.d.nm));
    double* ptr = nullptr;
    int rc = scratch_ptr(&ptr);
    if (rc) return rc;
    hipStream_t hs = S(stream);
    // the same kernels, their partials and totals redirected into the array
    Dev d = s.d;
    d.partial = ptr;
    d.scal = ptr + kPartials;
    double* total = ptr + kPartials + int64_t(MIFVM_STATIC_MAX_MESHES) * SC_COUNT_;
    HIPCHK(launch_conservation(d, *s.mesh, s.fp32, hs));
    hipLaunchKernelGGL(k_sum_meshes, dim3(1), dim3(64), 0, hs, d.scal, int(d.nm), total);
    HIPCHK(hipGetLastError());
    double host = 0.0;
    HIPCHK(hipMemcpyAsync(&host, total, sizeof(double), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    *total_out = host;
    return MIFVM_OK;
}
