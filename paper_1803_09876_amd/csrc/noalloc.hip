// Sweep entry point that allocates no device memory, for callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc).
//
// jsweep_sweep stages the per-cell product V s of the sweep in a buffer the
// graph allocates on first use.  The variant here stages it in `scratch`, a
// file-scope device array of fixed size that every GPU running the library
// holds until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels.  Everything else the
// sweep touches (level-position flux arrays, sigma_t cache, program,
// tickets) belongs to the graph and is allocated when the graph is built.
//
// All calls on one GPU share that GPU's array: calls that overlap in time on
// one GPU (two host threads, or two streams) race on it.  Nothing in the
// array has to start at zero: every call writes the entries it reads.
#include <mutex>

#include "common.hpp"

namespace jsw {

// V s of up to kNoAllocMaxCells cells (64 MiB)
constexpr int64_t kNoAllocMaxCells = (int64_t)1 << 23;
static __device__ __align__(256) double scratch[kNoAllocMaxCells];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's copy of `scratch`
void *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(JSWEEP_E_DEVICE, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            fail(JSWEEP_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

int64_t noalloc_max_cells() { return kNoAllocMaxCells; }

int sweep_noalloc(Graph &g, const double *sigma_t, const double *source, double *psi, double *phi, double psi_b,
                  hipStream_t s) {
    if (g.nc > kNoAllocMaxCells)
        fail(JSWEEP_E_INVALID_ARG, "jsweep_sweep_noalloc: " + std::to_string(g.nc) + " cells exceed its scratch of " +
                                       std::to_string(kNoAllocMaxCells) + " cells");
    int dev = -1;
    JSW_HIP(hipGetDevice(&dev));
    if (dev != g.device) fail(JSWEEP_E_INVALID_ARG, "jsweep_sweep_noalloc: the graph lives on another device");
    void *vs = scratch_address(dev);
    refresh_sigma(g, sigma_t, false, s);
    lag_snapshot64(g, psi, s);
    launch_sweep64_staged(g, source, psi, psi_b, vs, s);
    if (phi) scalar_flux(g, psi, phi, s);
    return check_sweep_status(g, s);
}

}  // namespace jsw
