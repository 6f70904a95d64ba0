// <psi|H|psi> of a Pauli sum on a caller's device buffer, for callers that
// cannot allocate device memory.  The term tables and the reduction partials
// live in `scratch`, a fixed array in device memory of every GPU the library
// runs on; the kernels are those of sv_expectation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.h"

namespace {

// Tables of SV_MAX_PAULI_TERMS terms take below 128 KiB; the partials of the
// first reduction stage and the result follow them.
constexpr size_t kScratchBytes = 192 * 1024;
constexpr size_t kTableBytes = kScratchBytes - 16 * 1024;
static_assert(size_t(sv::dev::kRedBlocks) * sizeof(double) + 256 <= kScratchBytes - kTableBytes, "partials");

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;                  // serialises set-up and the host staging buffer
void *g_scratch[kMaxDevices];     // scratch's device address on each device
alignas(256) char g_host[kTableBytes];  // host staging of the tables

// scratch's address on `dev` (the current device), looked up once per device
int scratch_on(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return sv::fail(SV_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sv::fail(SV_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = static_cast<char *>(g_scratch[dev]);
    return SV_OK;
}

}  // namespace

extern "C" int sv_expectation_noalloc(const void *dev_psi, int n, int dtype, void *hip_stream, const sv_pauli_sum *H,
                                      double *out)
{
    sv::clear_error();
    if (!dev_psi || !out) return sv::fail(SV_ERR_ARG, "NULL argument");
    if (dtype != SV_C64 && dtype != SV_C128) return sv::fail(SV_ERR_ARG, "dtype %d (SV_C64 or SV_C128)", dtype);
    const int nmax = dtype == SV_C64 ? SV_MAX_QUBITS_C64 : SV_MAX_QUBITS_C128;
    if (n < 1 || n > nmax) return sv::fail(SV_ERR_ARG, "n = %d outside 1..%d", n, nmax);
    if (reinterpret_cast<uintptr_t>(dev_psi) % 256) return sv::fail(SV_ERR_ARG, "state buffer not 256-byte aligned");
    if (int rc = sv::check_pauli(H, n)) return rc;
    if (H->n_terms == 0) {
        *out = 0.0;
        return SV_OK;
    }
    const size_t tables = sv::pauli_table_bytes(H);
    if (tables > kTableBytes)
        return sv::fail(SV_ERR_SIZE, "Pauli tables of %zu bytes exceed the %zu-byte scratch", tables, kTableBytes);
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return sv::fail(SV_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    char *base = nullptr;
    if (int rc = scratch_on(dev, &base)) return rc;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    sv::dev::PauliDev P;
    sv::pauli_table_fill(H, g_host, base, P);
    double *part = reinterpret_cast<double *>(base + kTableBytes);
    double *res = part + sv::dev::kRedBlocks;
    double host_res = 0.0;
    hipError_t e = hipMemcpyAsync(base, g_host, tables, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = sv::dev::launch_pauli_expect(dtype, dev_psi, n, P, part, res, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&host_res, res, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return sv::fail(SV_ERR_HIP, "sv_expectation_noalloc: %s", hipGetErrorString(e));
    *out = host_res;
    return SV_OK;
}
