// Allocation-free projection: mac_project_static.
//
// The whole projection of mac_project (coefficients, right-hand side,
// compatibility check, V-cycles to rtol, velocity correction) on a hierarchy
// laid out in a fixed device array instead of hipMalloc'd memory, for callers
// that may not allocate: code under stream capture, tight serving loops,
// harnesses that forbid device allocation.
//
// The array is one per device: every GPU the library runs on holds its own
// copy from module load until the process ends.  Host code never passes the
// array's name to a kernel or a copy (in host code that name is a host-side
// stand-in, not a device address); it looks the device address up once per
// device with hipGetSymbolAddress, on the first call made with that device
// current, and uses that address from then on.  The host-side hierarchy
// object and its scalar readback buffer are static too, one per device.
//
// Calls on one device share its array and its hierarchy object: calls that
// overlap on one device (two host threads, or two streams in flight) race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "mg_internal.h"
#include "runtime.h"

namespace {
constexpr size_t kStaticScratchBytes = size_t(MG_STATIC_SCRATCH_BYTES);
constexpr int kMaxStaticDevices = 64;
}  // namespace

// The device scratch array (see above): every level array, the partial-sum
// rows, the scalars and the coarsest-level inverse of one problem.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

struct StaticSlot {
    bool ready = false;
    void* dev = nullptr;          // device address of `scratch` on this device
    mg_hierarchy H;               // host-side hierarchy object, rebuilt by every call
    double host[64] = {};         // scalar readbacks (ordinary host memory)
};

StaticSlot g_slots[kMaxStaticDevices];
std::mutex g_init_mu;

}  // namespace

extern "C" int mac_project_static(const mg_params* p, const double* rho, const double* beta0_cc,
                                  const double* beta0_edge, const double* S, double* u, double* v, double* w,
                                  double* phi, mg_stats* stats, void* stream) {
    using namespace mg;
    try {
        int rc = validate_params(p);
        if (rc) return rc;
        const size_t need = workspace_bytes(p);
        if (need > kStaticScratchBytes) {
            set_error("problem needs " + std::to_string(need) + " bytes of scratch; mac_project_static holds " +
                      std::to_string(kStaticScratchBytes));
            return MG_ERR_BAD_SIZE;
        }
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice", __LINE__);
        if (dev < 0 || dev >= kMaxStaticDevices) {
            set_error("mac_project_static supports devices 0.." + std::to_string(kMaxStaticDevices - 1));
            return MG_ERR_INVALID_ARG;
        }
        StaticSlot& s = g_slots[dev];
        {
            std::lock_guard<std::mutex> lock(g_init_mu);
            if (!s.ready) {
                void* ptr = nullptr;
                e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
                if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
                if (!ptr) {
                    set_error("hipGetSymbolAddress returned no address for the scratch array");
                    return MG_ERR_HIP;
                }
                s.dev = ptr;
                s.ready = true;
            }
        }
        rc = setup_static(p, s.dev, kStaticScratchBytes, s.host, &s.H);
        if (rc) return rc;
        hipStream_t st = (hipStream_t)stream;
        // the array keeps the previous call's contents: start from zeros (a
        // fill kernel, not a memset, so the call stays capturable)
        e = launch_fill<double>((double*)s.dev, need / sizeof(double), 0.0, st);
        if (e != hipSuccess) return hip_fail(e, "launch_fill(scratch)", __LINE__);
        return project(&s.H, rho, beta0_cc, beta0_edge, S, u, v, w, phi, stats, st);
    } catch (...) {
        set_error("internal error in mac_project_static");
        return MG_ERR_HIP;
    }
}
