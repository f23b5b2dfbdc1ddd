// fsd_apply_A_noalloc (include/fsd.h): the float64 matvec of fsd_apply_A
// with its device scratch in a file-scope array instead of the problem's
// workspace, for callers that cannot allocate device memory.
//
// The scratch (the packed input and output and the four pass intermediates,
// six vectors of Np doubles) lives in `scratch`, a static __device__ array of
// kScratchBytes.  Each GPU holds its own copy until the process ends; its
// device address is looked up once per device (hipGetSymbolAddress) on the
// first call with that device current, and only that address is handed to
// the kernels.  Every call clears the part it uses with a fill kernel (the
// passes rely on zero padding columns), so calls are independent; calls
// that overlap on one GPU share the array and race.
#include <cstdio>
#include <mutex>
#include <string>

#include "fsd_host.h"
#include "fsd_vec.h"

namespace fsd {
fsd_status matvec64_with(fsd_problem P, const double* x, double* y, double* const tmp[4]);
fsd_status require_bound(fsd_problem P);
}  // namespace fsd

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
fsd_status scratch_ptr(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fsd::set_error(FSD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fsd::set_error(FSD_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fsd::set_error(FSD_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                hipGetErrorString(e));
        g_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_ptr[dev];
    return FSD_OK;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

extern "C" {

size_t fsd_noalloc_scratch_bytes(void) { return kScratchBytes; }

fsd_status fsd_apply_A_noalloc(fsd_problem P, const double* d_x, double* d_y) {
    fsd_status st = fsd::require_bound(P);
    if (st != FSD_OK) return st;
    if (!d_x || !d_y) return fsd::set_error(FSD_EINVAL, "null vector");
    const size_t vbytes = align256((size_t)P->Np * sizeof(double));
    if (6 * vbytes > kScratchBytes) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "fsd_apply_A_noalloc: the grid needs %zu bytes of scratch, the static array "
                 "holds %zu (at most 6 padded vectors of %zu doubles)",
                 6 * vbytes, kScratchBytes, kScratchBytes / 6 / sizeof(double));
        return fsd::set_error(FSD_EUNSUPPORTED, buf);
    }
    char* base = nullptr;
    st = scratch_ptr(&base);
    if (st != FSD_OK) return st;
    double* v[6];
    for (int i = 0; i < 6; ++i) v[i] = reinterpret_cast<double*>(base + i * vbytes);
    hipStream_t s = P->stream;
    // zero the part used: the passes read the padding columns of their
    // inputs, which must hold zeros (the array keeps the last call's data)
    hipError_t e = fsd::vec_fill<double>(v[0], (long)(6 * vbytes / sizeof(double)), 0.0, s);
    if (e == hipSuccess)
        e = fsd::vec_pack<double>(d_x, v[0], P->ax[0].n, P->P1, P->rows, 1.0, s);
    if (e != hipSuccess) return fsd::set_error(FSD_EHIP, std::string("launch: ") + hipGetErrorString(e));
    double* const tmp[4] = {v[2], v[3], v[4], v[5]};
    st = fsd::matvec64_with(P, v[0], v[1], tmp);
    if (st != FSD_OK) return st;
    e = fsd::vec_unpack<double>(v[1], d_y, P->ax[0].n, P->P1, P->rows, s);
    if (e != hipSuccess) return fsd::set_error(FSD_EHIP, std::string("launch: ") + hipGetErrorString(e));
    return FSD_OK;
}

}  // extern "C"
