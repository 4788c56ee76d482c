// Continuation estimates without device allocation, for callers that cannot
// call hipMalloc (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).  The spec tables and the per-job partial sums
// that bmc_estimate_continuation keeps in context buffers live here in one
// file-scope device array, `scratch`, whose address on each device is taken
// once (bmc_ctx_create) with hipGetSymbolAddress; host code uses only that
// address.  Every call on a device shares the device's array and leaves its
// contents behind: calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>

#include "bmc.h"
#include "internal.hpp"
#include "runtime.hpp"

namespace bmc {

// [DevSpec | spec staging | partial sums]
constexpr size_t NOALLOC_SPEC_OFF = 0;
constexpr size_t NOALLOC_PACK_OFF = (sizeof(DevSpec) + 255) & ~(size_t)255;
constexpr size_t NOALLOC_PART_OFF = (NOALLOC_PACK_OFF + sizeof(HostSpecPack) + 255) & ~(size_t)255;

}  // namespace bmc

static __device__ __align__(256) unsigned char scratch[BMC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};
}  // namespace

// Address of this device's scratch array (the current device must be
// `device`); taken once per device.
bmc_status bmc::noalloc_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(BMC_EINVAL, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return BMC_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch[device] = ptr;
    return BMC_OK;
}

extern "C" bmc_status bmc_estimate_continuation_noalloc(bmc_ctx* ctx, const bmc_spec* spec, const bmc_rules* rules,
                                                        int32_t date, const double* x, int64_t N, int64_t n,
                                                        uint64_t seed, int32_t precision, double* cont,
                                                        double* std_err, int64_t* steps)
{
    using namespace bmc;
    if (!ctx || !x || !cont || !std_err) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < MAX_DEVICES) base = g_scratch[ctx->device];
    }
    if (!base) return fail(BMC_EDEVICE, "no scratch address for device %d", ctx->device);
    bmc_status st = validate_spec(spec);
    if (st) return st;
    if (!rules || rules->d != spec->d || rules->n_dates != spec->n_dates || rules->payoff != spec->payoff)
        return fail(BMC_EINVAL, "rules do not match the spec");
    if (precision < BMC_FP64 || precision > BMC_FP32_KAHAN) return fail(BMC_EINVAL, "unknown precision %d", precision);
    if (seed > 0xFFFFFFFFull) return fail(BMC_EINVAL, "seed must fit in 32 bits");
    if (date < 0 || date >= spec->n_dates) return fail(BMC_EINVAL, "date %d outside 0..%d", date, spec->n_dates - 1);
    if (N < 1 || N > 0x7FFFFFFF) return fail(BMC_EINVAL, "N = %lld out of range", (long long)N);
    if (n < 2 || n > 0x7FFFFFFF) return fail(BMC_EINVAL, "n = %lld out of range", (long long)n);
    const int block = 256;
    const uint32_t per_wg = (uint32_t)block * choose_ppt(ctx, spec->d, precision, N, n, nullptr);
    const uint64_t nchunk = ((uint64_t)n + per_wg - 1) / per_wg;
    const uint64_t part_bytes = sizeof(double) * 3 * (uint64_t)N * nchunk;
    if (part_bytes > BMC_NOALLOC_SCRATCH_BYTES - NOALLOC_PART_OFF)
        return fail(BMC_ENOMEM,
                    "N = %lld points x %llu path chunks need %llu bytes of partial sums; the no-allocation "
                    "scratch holds %llu",
                    (long long)N, (unsigned long long)nchunk, (unsigned long long)part_bytes,
                    (unsigned long long)(BMC_NOALLOC_SCRATCH_BYTES - NOALLOC_PART_OFF));
    DevSpec* dspec = (DevSpec*)((char*)base + NOALLOC_SPEC_OFF);
    HostSpecPack* dpack = (HostSpecPack*)((char*)base + NOALLOC_PACK_OFF);
    double* part = (double*)((char*)base + NOALLOC_PART_OFF);
    // spec upload through the context's pinned staging; the setup status
    // comes back through its pinned result area
    hipError_t e;
    if ((e = hipStreamSynchronize(ctx->stream))) return hip_fail(e, "stream sync");   // staging and scratch free
    pack_spec(spec, ctx->pack_host);
    int32_t* status = (int32_t*)((char*)ctx->host_io + 120);
    if ((e = hipMemcpyAsync(dpack, ctx->pack_host, sizeof(HostSpecPack), hipMemcpyHostToDevice, ctx->stream)) ||
        (e = launch_setup(dpack, dspec, 1, ctx->stream)) ||
        (e = hipMemcpyAsync(status, (char*)dspec + offsetof(DevSpec, status), sizeof(int32_t), hipMemcpyDeviceToHost,
                            ctx->stream)) ||
        (e = hipStreamSynchronize(ctx->stream)))
        return hip_fail(e, "spec upload");
    if (*status != 0) return fail(BMC_ENOTSPD, "correlation matrix is not positive definite");
    return run_cont(ctx, dspec, spec->d, spec->n_dates, rules->method, rules->width, rules->w64, rules->w32, precision,
                    date, x, N, nullptr, nullptr, (uint32_t)n, (uint32_t)seed, key_hi(BMC_STREAM_INNER, date), cont,
                    std_err, steps, nullptr, nullptr, nullptr, 0, 0, nullptr, part);
}
