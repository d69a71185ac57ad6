// Total energy without any allocation: the same kernels as gcmc_total_energy,
// with their scratch (workgroup partial sums, the particles in cell order, the
// scan of the cell counters) in a file-scope device array instead of the box's
// scratch, which gcmc_total_energy grows with hipMalloc.
//
// Every GPU the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and that address is what the kernels receive.
#include <mutex>

#include "gcmc_internal.h"

namespace gcmc {

// 16 MiB: enough for N + cells up to about 4.1 million (a cell-list pass needs
// N / 256 partials plus (N + cells) / 2 doubles of int32 order and offsets).
constexpr int64_t kNoAllocDoubles = (int64_t)1 << 21;
constexpr int kNoAllocDevices = 64;

}  // namespace gcmc

static __device__ __align__(256) double scratch[gcmc::kNoAllocDoubles];

namespace gcmc {

static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kNoAllocDevices];   // device address of `scratch`, per device

// The array's address on the current device (looked up on the first call on
// that device).  Returns GCMC_OK or an error code.
static int noalloc_scratch(int device, double** out) {
    if (device < 0 || device >= kNoAllocDevices) return set_error(GCMC_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_noalloc_ptr[device] = static_cast<double*>(p);
    }
    *out = g_noalloc_ptr[device];
    return GCMC_OK;
}

}  // namespace gcmc

using namespace gcmc;

extern "C" {

int gcmc_total_energy_noalloc(gcmc_box* box, int32_t all_pairs, double* d_U, double* d_e, void* stream) {
    if (!box || !d_U) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    int dev = -1;
    GCMC_HIP(hipGetDevice(&dev));
    if (dev != box->device) return set_error(GCMC_ERR_INVALID_ARG, "the box lives on another device than the current one");
    double* buf = nullptr;
    int rc = noalloc_scratch(dev, &buf);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    if ((rc = read_box_state(box, &h, s))) return rc;
    if (h.error) return set_error(GCMC_ERR_POISONED, "box holds a latched device error");
    const int64_t need = total_partials_needed(box->d, h.maxcount, all_pairs != 0, h.n);
    if (need > kNoAllocDoubles)
        return set_error(GCMC_ERR_INVALID_ARG, "the pass needs " + std::to_string(need) +
                                                   " doubles of scratch; the static buffer holds " +
                                                   std::to_string(kNoAllocDoubles));
    if (launch_total(box->d, box->d_desc, h.maxcount, all_pairs != 0, d_e, buf, kNoAllocDoubles, d_U, s, h.n))
        return set_error(GCMC_ERR_INVALID_ARG, "scratch too small");
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

}  // extern "C"
