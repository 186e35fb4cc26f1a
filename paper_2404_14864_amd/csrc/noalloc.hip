// The five-point grid solve of eq. (3.31) for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// kfbi_grid_solve keeps its two mode-space intermediates, the x-transformed
// right-hand side R^ and the solution U^ ((M-1)^2 elements each), in buffers
// the domain allocates.  This variant keeps them in `scratch`, a file-scope
// device array of a fixed size that every GPU the library runs on holds
// until the process ends; the call itself allocates nothing.  The kernels are
// the grid solve's own (x-DST, tridiagonal y-solves, inverse x-DST), given
// the array's device address where kfbi_grid_solve passes the domain's
// buffers, so both calls compute the same values.
//
// The array's device address is looked up once per device, at set-up
// (kfbi_domain_create, with the domain's device current), and kept per
// device; in host code the name `scratch` stands for a host-side shadow, so
// only the looked-up address is ever handed to a kernel.

#include <mutex>

#include "kfbi_internal.h"

namespace kfbi {

constexpr size_t kScratchBytes = (size_t)KFBI_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of 256 bytes");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int stream_device(hipStream_t s, int *dev) {
    if (s) KFBI_HIP(hipStreamGetDevice(s, dev));
    else KFBI_HIP(hipGetDevice(dev));
    if (*dev < 0 || *dev >= kMaxDevices) {
        set_error("device ordinal out of range for the no-allocation scratch table");
        return KFBI_EINVAL;
    }
    return KFBI_OK;
}

}  // namespace

// The device address of this device's copy of the scratch array (looked up
// on the first call for a device, with that device current).
int noalloc_scratch(hipStream_t s, void **out) {
    int dev = -1;
    KFBI_TRY(stream_device(s, &dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        KFBI_HIP(hipGetDevice(&cur));
        if (cur != dev) KFBI_HIP(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t r = hipSetDevice(cur);
            if (r != hipSuccess && e == hipSuccess) {
                set_error(std::string("hipSetDevice: ") + hipGetErrorString(r));
                return KFBI_EDEVICE;
            }
        }
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return KFBI_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KFBI_OK;
}

}  // namespace kfbi

using namespace kfbi;

extern "C" int kfbi_grid_solve_noalloc(kfbi_domain *d, double kre, double kim, const void *rhs, void *u_out) {
    if (!d || !rhs || !u_out) {
        set_error("null argument");
        return KFBI_EINVAL;
    }
    if (!d->cplx && kim != 0.0) {
        set_error("complex kappa needs a complex domain");
        return KFBI_EINVAL;
    }
    const size_t n = (size_t)d->M - 1, half = n * n * elem_size(d);
    // R^ at the start of the array, U^ at the next 256-byte boundary
    const size_t off = (half + 255) / 256 * 256;
    if (off + half > kScratchBytes) {
        set_error("grid too large for the no-allocation grid solve: needs " + std::to_string(off + half) +
                  " bytes of scratch, the library holds " + std::to_string(kScratchBytes) +
                  " per device (2 (M-1)^2 elements: M <= 1024 real, M <= 512 complex)");
        return KFBI_ENOTSUP;
    }
    void *base = nullptr;
    KFBI_TRY(noalloc_scratch(d->stream, &base));
    void *rhat = base;
    void *uhat = (unsigned char *)base + off;
    KFBI_TRY(dst_rows_dense(d, rhs, false, rhat));
    KFBI_TRY(ensure_coefficients(d, kre, kim));
    KFBI_TRY(tridiag_solve(d, rhat, nullptr, uhat));
    KFBI_TRY(idst_rows_dense(d, uhat, u_out));
    return KFBI_OK;
}
