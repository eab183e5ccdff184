// Allocation-free variant of the device update step: the same pipeline as
// hsma_energy_forces_device (same kernels and schedule), run in a static
// device scratch array instead of a caller workspace, every stage on the
// caller's stream.
#include <mutex>

#include "hsma_internal.h"
#include "solve.h"

namespace hsma {

// Scratch of the allocation-free entry point.  The name is a host-side
// stand-in for the array in host code: kernels and copies get the device
// address that hipGetSymbolAddress returns for the current device (each
// device holds its own copy of the array, at its own address).
static __device__ __align__(256) char scratch[HSMA_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
static hsma_status scratch_on(int device, char** out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(HSMA_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(HSMA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
        g_scratch_ptr[device] = (char*)p;
    }
    *out = g_scratch_ptr[device];
    return HSMA_OK;
}

}  // namespace hsma

using namespace hsma;

extern "C" hsma_status hsma_energy_forces_noalloc(hsma_plan pl, const double* x, const double* q,
                                                  int64_t N, void* stream, double* energy,
                                                  double* phi, double* forces) {
    hsma_status st = check_sizes(pl, N);
    if (st != HSMA_OK) return st;
    if (x == nullptr || q == nullptr || energy == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    Layout ly = make_layout(pl, N, false);
    ly.single_stream = true;
    if (ly.total > (size_t)HSMA_NOALLOC_SCRATCH_BYTES)
        return fail(HSMA_E_NOMEM, "N needs " + std::to_string(ly.total) +
                                      " bytes of scratch; the allocation-free entry point has " +
                                      std::to_string((size_t)HSMA_NOALLOC_SCRATCH_BYTES));
    HSMA_HIP(hipSetDevice(pl->device));
    char* ws = nullptr;
    st = scratch_on(pl->device, &ws);
    if (st != HSMA_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = forward(pl, ly, x, q, HSMA_DTYPE_F64, ws, s, phi, forces, nullptr);
    if (st != HSMA_OK) return st;
    return read_result(ly, ws, s, energy);
}
