// Allocation-free form of steps (1)-(2) of Algorithm 1 (the singular-value soft threshold of
// the Casorati matrix and the singular-value prior), for callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// It runs the kernels of prior_ls_op_svt (Gram on MFMA, fixed-order FP64 reduction of the
// block partials, FP64 Jacobi eigensolve with the thresholds, back-projection L = C W) with
// every intermediate in one file-scope device array instead of handle-owned buffers.  The
// host takes that array's address once per device with hipGetSymbolAddress and passes the
// address to the kernels; the array's name itself is never used as a device address in host
// code.  The call only enqueues work on the caller's stream: no allocation, no
// synchronisation, no memset (every scratch entry a kernel reads was written by an earlier
// kernel of the same call).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "pls_kernels.hpp"
#include "prior_ls.h"

namespace pls {
void set_thread_error(const std::string& m);
}

namespace {

// Scratch layout (bytes).  The Gram is split over at most kNaGramBlocks workgroups whatever
// the voxel count, so the partials never exceed kNaGramBlocks x (tiles of nt <= 32) entries.
constexpr int kNaGramBlocks = 256;
constexpr int kNaEntries = 10 * 256;                  // gram_tiles(32): 4 x 4 tile pairs, 16 x 16
constexpr size_t kNaPart = 0;                         // double [256][2560] block partials
constexpr size_t kNaRed = kNaPart + (size_t)kNaGramBlocks * kNaEntries * 8;   // double [2560]
constexpr size_t kNaV = kNaRed + (size_t)kNaEntries * 8;                      // double2 [32][32]
constexpr size_t kNaWd = kNaV + 2 * 32 * 32 * 8;                              // double2 [32][32]
constexpr size_t kNaWop = kNaWd + 2 * 32 * 32 * 8;                            // float [64][64]
constexpr size_t kNaStat = kNaWop + 64 * 64 * 4;                              // double [64]
constexpr size_t kNaBytes = kNaStat + 64 * 8;

static_assert(PRIOR_LS_NOALLOC_SCRATCH_BYTES == kNaBytes, "header states the scratch size");

}  // namespace

// One copy per GPU, alive until the process ends.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
unsigned char* g_na_ptr[kMaxDevices] = {};

int na_fail(int code, const std::string& m) {
    pls::set_thread_error(m);
    return code;
}

bool na_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// Device address of the scratch array on the current device, taken once per device.
int na_scratch(unsigned char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return na_fail(PRIOR_LS_EHIP, "hipGetDevice failed");
    }
    if (dev < 0 || dev >= kMaxDevices) return na_fail(PRIOR_LS_EHIP, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return na_fail(PRIOR_LS_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                              hipGetErrorString(e));
        }
        g_na_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_na_ptr[dev];
    return PRIOR_LS_OK;
}

}  // namespace

extern "C" int prior_ls_svt_noalloc(const void* C, int64_t n_vox, int32_t nt, int32_t gram_mode,
                                    double lambda_L, int32_t lambda_L_relative, double lambda_p,
                                    const double* sigma_prev, void* L, double* sigma,
                                    void* stream) {
    pls::set_thread_error("");
    if (!C || !L) return na_fail(PRIOR_LS_EINVAL, "C and L are required");
    if (nt < 1 || nt > PRIOR_LS_NOALLOC_MAX_NT)
        return na_fail(PRIOR_LS_ESHAPE, "nt must be in [1, 32] (the scratch array holds the "
                                        "Gram tiles and eigenvectors of at most 32 frames)");
    if (n_vox < 64 || n_vox % 64 != 0)
        return na_fail(PRIOR_LS_ESHAPE, "n_vox must be a positive multiple of 64");
    if (n_vox * (int64_t)nt > (int64_t)INT32_MAX)
        return na_fail(PRIOR_LS_ESHAPE, "n_vox * nt must stay below 2^31 elements");
    if (gram_mode < PRIOR_LS_GRAM_FP64 || gram_mode > PRIOR_LS_GRAM_BF16X3)
        return na_fail(PRIOR_LS_EINVAL, "unknown gram_mode");
    if (!(lambda_L >= 0)) return na_fail(PRIOR_LS_EINVAL, "lambda_L must be >= 0");
    if (!(lambda_p >= 0 && lambda_p <= 1)) return na_fail(PRIOR_LS_EINVAL, "lambda_p must be in [0, 1]");
    if (lambda_p > 0 && !sigma_prev) return na_fail(PRIOR_LS_EINVAL, "sigma_prev is required when lambda_p > 0");
    if (!na_device_ptr(C) || !na_device_ptr(L))
        return na_fail(PRIOR_LS_EINVAL, "C and L must be device memory");
    if (lambda_p > 0 && !na_device_ptr(sigma_prev))
        return na_fail(PRIOR_LS_EINVAL, "sigma_prev must be device memory");
    if (sigma && !na_device_ptr(sigma)) return na_fail(PRIOR_LS_EINVAL, "sigma must be device memory");
    const char* c0 = static_cast<const char*>(C);
    const char* l0 = static_cast<const char*>(L);
    const int64_t bytes = n_vox * nt * 8;
    if (c0 < l0 + bytes && l0 < c0 + bytes) return na_fail(PRIOR_LS_EINVAL, "L must not overlap C");
    unsigned char* base = nullptr;
    int rc = na_scratch(&base);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = (int)n_vox;
    double* part = reinterpret_cast<double*>(base + kNaPart);
    double* red = reinterpret_cast<double*>(base + kNaRed);
    double* stat = reinterpret_cast<double*>(base + kNaStat);
    pls::GramArgs ga{static_cast<const float2*>(C), part, N, nt, 0, kNaGramBlocks};
    const int gb = pls::launch_gram(gram_mode, ga, s);
    pls::launch_gram_reduce(part, gb, pls::gram_tiles(nt) * 256, red, s);
    pls::EigArgs ea{};
    ea.gram = red;
    ea.V = reinterpret_cast<double*>(base + kNaV);
    ea.warm = 0;                       // Jacobi from the identity; V is written, not read
    ea.Wop = reinterpret_cast<float*>(base + kNaWop);
    ea.Wd = reinterpret_cast<double*>(base + kNaWd);
    ea.sigma_prev = lambda_p > 0 ? sigma_prev : nullptr;
    ea.stat = stat;
    ea.sigL = nullptr;
    ea.nt = nt;
    ea.lambda_L = lambda_L;
    ea.lambda_p = lambda_p;
    ea.relative = lambda_L_relative;
    pls::launch_eig(ea, s);
    pls::BpArgs ba{static_cast<const float2*>(C), static_cast<float2*>(L), ea.Wop, N, nt, 0};
    pls::launch_bp(ba, s);
    if (sigma) {
        const hipError_t e = hipMemcpyAsync(sigma, stat + 16, (size_t)nt * sizeof(double),
                                            hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return na_fail(PRIOR_LS_EHIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return na_fail(PRIOR_LS_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return PRIOR_LS_OK;
}
