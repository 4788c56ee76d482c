// C ABI of the gfx950 nested continuation-value Monte Carlo: contexts, rule
// tables, spec validation/upload and the pricer drivers.  Declarations and
// contracts are in include/bmc.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bmc.h"
#include "internal.hpp"
#include "runtime.hpp"

using namespace bmc;

// ---------------------------------------------------------------------------
// Errors

static thread_local std::string g_last_error;

bmc_status bmc::fail(bmc_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

bmc_status bmc::hip_fail(hipError_t e, const char* where)
{
    return fail(BMC_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

extern "C" const char* bmc_last_error(void) { return g_last_error.c_str(); }
extern "C" int32_t bmc_version(void) { return 10000; }

// ---------------------------------------------------------------------------
// Device buffers

hipError_t DBuf::ensure(size_t n)
{
    if (n <= bytes) return hipSuccess;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = n < 256 ? 256 : n;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = want;
    return hipSuccess;
}

void DBuf::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// ---------------------------------------------------------------------------
// Spec validation and upload

bmc_status bmc::validate_spec(const bmc_spec* s)
{
    if (!s) return fail(BMC_EINVAL, "spec is NULL");
    if (s->d < 1 || s->d > BMC_D_MAX) return fail(BMC_EINVAL, "d = %d outside 1..%d", s->d, BMC_D_MAX);
    if (s->n_dates < 1 || s->n_dates > BMC_NT_MAX)
        return fail(BMC_EINVAL, "n_dates = %d outside 1..%d", s->n_dates, BMC_NT_MAX);
    if (!s->S0 || !s->delta || !s->sigma || !s->rho || !s->dates)
        return fail(BMC_EINVAL, "spec array pointer is NULL");
    if (!(s->K > 0.0) || !std::isfinite(s->K)) return fail(BMC_EINVAL, "K must be > 0");
    if (!(s->T > 0.0) || !std::isfinite(s->T)) return fail(BMC_EINVAL, "T must be > 0");
    if (!std::isfinite(s->r)) return fail(BMC_EINVAL, "r must be finite");
    if (s->payoff < BMC_PUT_BASKET || s->payoff > BMC_CALL_MIN)
        return fail(BMC_EINVAL, "unknown payoff %d", s->payoff);
    double prev = 0.0;
    for (int k = 0; k < s->n_dates; ++k) {
        if (!(s->dates[k] > prev) || !std::isfinite(s->dates[k]))
            return fail(BMC_EINVAL, "dates must be strictly increasing in (0, T]");
        prev = s->dates[k];
    }
    if (std::fabs(prev - s->T) > 1e-12 * s->T) return fail(BMC_EINVAL, "last date must equal T");
    const int d = s->d;
    for (int i = 0; i < d; ++i) {
        if (!(s->S0[i] > 0.0) || !std::isfinite(s->S0[i])) return fail(BMC_EINVAL, "S0[%d] must be > 0", i);
        if (!(s->sigma[i] >= 0.0) || !std::isfinite(s->sigma[i]))
            return fail(BMC_EINVAL, "sigma[%d] must be >= 0", i);
        if (!std::isfinite(s->delta[i])) return fail(BMC_EINVAL, "delta[%d] must be finite", i);
        if (std::fabs(s->rho[i * d + i] - 1.0) > 1e-12) return fail(BMC_EINVAL, "rho must have a unit diagonal");
        for (int j = 0; j < i; ++j) {
            const double a = s->rho[i * d + j], b = s->rho[j * d + i];
            if (!std::isfinite(a) || std::fabs(a - b) > 1e-12 || std::fabs(a) > 1.0)
                return fail(BMC_EINVAL, "rho must be symmetric with entries in [-1, 1]");
        }
    }
    return BMC_OK;
}

void bmc::pack_spec(const bmc_spec* s, HostSpecPack* p)
{
    std::memset(p, 0, sizeof(*p));
    p->d = s->d;
    p->n_dates = s->n_dates;
    p->payoff = s->payoff;
    p->K = s->K;
    p->r = s->r;
    p->T = s->T;
    for (int i = 0; i < s->d; ++i) {
        p->S0[i] = s->S0[i];
        p->delta[i] = s->delta[i];
        p->sigma[i] = s->sigma[i];
    }
    std::memcpy(p->rho, s->rho, sizeof(double) * s->d * s->d);
    std::memcpy(p->dates, s->dates, sizeof(double) * s->n_dates);
}

// Uploads and derives a spec into the context's spec slot; checks the
// Cholesky status (one stream synchronisation).
bmc_status bmc::upload_spec_async(bmc_ctx* ctx, const bmc_spec* s, DBuf& slot, int32_t* status_host)
{
    bmc_status st = validate_spec(s);
    if (st) return st;
    hipError_t e = slot.ensure(sizeof(DevSpec));
    if (e) return hip_fail(e, "spec allocation");
    if ((e = ctx->pack_dev.ensure(sizeof(HostSpecPack)))) return hip_fail(e, "spec staging");
    if ((e = hipStreamSynchronize(ctx->stream))) return hip_fail(e, "stream sync");   // staging free
    pack_spec(s, ctx->pack_host);
    // the setup kernel writes its status word straight into the pinned status_host
    int32_t* status_dev = (int32_t*)((char*)ctx->host_io_dev + ((char*)status_host - (char*)ctx->host_io));
    if ((e = hipMemcpyAsync(ctx->pack_dev.ptr, ctx->pack_host, sizeof(HostSpecPack), hipMemcpyHostToDevice,
                            ctx->stream)) ||
        (e = launch_setup((const HostSpecPack*)ctx->pack_dev.ptr, (DevSpec*)slot.ptr, 1, ctx->stream, nullptr,
                          status_dev)))
        return hip_fail(e, "spec upload");
    return BMC_OK;
}

bmc_status bmc::upload_spec(bmc_ctx* ctx, const bmc_spec* s, DBuf& slot)
{
    bmc_status st = validate_spec(s);
    if (st) return st;
    hipError_t e = slot.ensure(sizeof(DevSpec));
    if (e) return hip_fail(e, "spec allocation");
    if ((e = ctx->pack_dev.ensure(sizeof(HostSpecPack)))) return hip_fail(e, "spec staging");
    if ((e = hipStreamSynchronize(ctx->stream))) return hip_fail(e, "stream sync");
    pack_spec(s, ctx->pack_host);
    if ((e = hipMemcpyAsync(ctx->pack_dev.ptr, ctx->pack_host, sizeof(HostSpecPack),
                            hipMemcpyHostToDevice, ctx->stream)))
        return hip_fail(e, "spec upload");
    if ((e = launch_setup((const HostSpecPack*)ctx->pack_dev.ptr, (DevSpec*)slot.ptr, 1, ctx->stream)))
        return hip_fail(e, "setup launch");
    int32_t status = 0;
    if ((e = hipMemcpyAsync(&status, (char*)slot.ptr + offsetof(DevSpec, status), sizeof(int32_t),
                            hipMemcpyDeviceToHost, ctx->stream)))
        return hip_fail(e, "status read");
    if ((e = hipStreamSynchronize(ctx->stream))) return hip_fail(e, "stream sync");
    if (status != 0) return fail(BMC_ENOTSPD, "correlation matrix is not positive definite");
    return BMC_OK;
}

int32_t* bmc::fit_barrier_flag_dev(bmc_ctx* ctx) { return (int32_t*)((char*)ctx->host_io_dev + 136); }

bmc_status bmc::check_fit_barrier(bmc_ctx* ctx)
{
    volatile int32_t* flag = (volatile int32_t*)((char*)ctx->host_io + 136);
    if (*flag == 0) return BMC_OK;
    *flag = 0;
    // a barrier that gave up leaves its words in an unknown state
    if (ctx->gbar.ptr) {
        (void)hipMemsetAsync(ctx->gbar.ptr, 0, 256, ctx->stream);
        (void)hipStreamSynchronize(ctx->stream);
    }
    return fail(BMC_EDEVICE, "rule fit: a grid barrier timed out (its blocks were not all resident)");
}

const double* bmc::dev_S0(const void* devspec)
{
    return (const double*)((const char*)devspec + offsetof(DevSpec, f64) + offsetof(SpecT<double>, S0));
}

// ---------------------------------------------------------------------------
// Context

extern "C" bmc_status bmc_ctx_create(int32_t device, void* hip_stream, bmc_ctx** out)
{
    if (!out) return fail(BMC_EINVAL, "out is NULL");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(BMC_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(BMC_EINVAL, "device %d outside 0..%d", device, count - 1);
    if ((e = hipSetDevice(device))) return hip_fail(e, "hipSetDevice");
    bmc_status st = noalloc_setup(device);
    if (st) return st;
    bmc_ctx* c = new bmc_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if ((e = hipHostMalloc((void**)&c->pack_host, sizeof(HostSpecPack), hipHostMallocDefault))) {
        delete c;
        return hip_fail(e, "pinned staging");
    }
    if ((e = hipHostMalloc((void**)&c->host_io, 4096, hipHostMallocDefault)) ||
        (e = hipHostGetDevicePointer(&c->host_io_dev, c->host_io, 0))) {
        (void)hipHostFree(c->pack_host);
        c->pack_host = nullptr;
        delete c;   // frees host_io
        return hip_fail(e, "pinned staging");
    }
    *out = c;
    return BMC_OK;
}

bmc_ctx::~bmc_ctx()
{
    for (DBuf* b : {&spec, &spec2, &pack_dev, &part, &B, &x, &x2, &cont, &se, &steps, &fit, &iz,
                    &counters, &korobov, &rf, &order, &gbar, &bspec, &barena, &btab})
        b->release();
    if (pack_host) (void)hipHostFree(pack_host);
    if (bhost) (void)hipHostFree(bhost);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : poll_ev)
        if (e) (void)hipEventDestroy(e);
    srules.release();
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph_stream) (void)hipStreamDestroy(graph_stream);
    if (host_io) (void)hipHostFree(host_io);
}

extern "C" void bmc_ctx_destroy(bmc_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
}

extern "C" bmc_status bmc_ctx_set_graphs(bmc_ctx* ctx, int32_t enable)
{
    if (!ctx) return fail(BMC_EINVAL, "ctx is NULL");
    ctx->graphs = enable != 0;
    return BMC_OK;
}

extern "C" bmc_status bmc_ctx_graph_stats(bmc_ctx* ctx, int64_t* captures, int64_t* replays)
{
    if (!ctx || !captures || !replays) return fail(BMC_EINVAL, "NULL argument");
    *captures = ctx->graph_captures;
    *replays = ctx->graph_replays;
    return BMC_OK;
}

extern "C" bmc_status bmc_sync(bmc_ctx* ctx)
{
    if (!ctx) return fail(BMC_EINVAL, "ctx is NULL");
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(e, "stream sync");
    return BMC_OK;
}

// ---------------------------------------------------------------------------
// Rules

static double never_value(int method, int payoff)
{
    if (method != BMC_IZ) return 0.0;   // classifier rows of zeros: F = 0, never exercise
    return (payoff == BMC_CALL_MAX || payoff == BMC_CALL_MIN) ? 1e300 : -1e300;
}

static bmc_status rules_alloc(bmc_ctx* ctx, int method, int d, int n_dates, int payoff,
                              bmc_rules** out)
{
    bmc_rules* r = new bmc_rules();
    r->ctx = ctx;
    r->method = method;
    r->d = d;
    r->n_dates = n_dates;
    r->payoff = payoff;
    r->width = rule_row_width(method, d, payoff);
    const size_t rows = (size_t)(n_dates + 1) * r->width;
    const int block = method == BMC_IZ ? rule_width(method, d) : r->width;
    hipError_t e;
    if ((e = hipMalloc((void**)&r->w64, sizeof(double) * rows)) ||
        (e = hipMalloc((void**)&r->w32, sizeof(float) * rows))) {
        if (r->w64) (void)hipFree(r->w64);
        delete r;
        return fail(BMC_ENOMEM, "rule table allocation: %s", hipGetErrorString(e));
    }
    std::vector<double> h(rows, 0.0);
    std::vector<float> hf(rows, 0.0f);
    const double nv = never_value(method, payoff);
    for (size_t f = 0; f < rows; f += block) {   // every region's block starts "never"
        h[f] = nv;
        hf[f] = (float)nv;
    }
    if ((e = hipMemcpy(r->w64, h.data(), sizeof(double) * rows, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(r->w32, hf.data(), sizeof(float) * rows, hipMemcpyHostToDevice))) {
        bmc_rules_destroy(r);
        return hip_fail(e, "rule table init");
    }
    *out = r;
    return BMC_OK;
}

bmc_status bmc::scratch_rules(bmc_ctx* ctx, const bmc_spec* spec, int method, bmc_rules* r)
{
    r->ctx = ctx;
    r->method = method;
    r->d = spec->d;
    r->n_dates = spec->n_dates;
    r->payoff = spec->payoff;
    r->width = rule_row_width(method, spec->d, spec->payoff);
    const size_t rows = (size_t)(spec->n_dates + 1) * r->width;
    const size_t b64 = (sizeof(double) * rows + 255) & ~(size_t)255;
    hipError_t e = ctx->srules.ensure(b64 + sizeof(float) * rows);
    if (e) return hip_fail(e, "rule scratch");
    r->w64 = (double*)ctx->srules.ptr;
    r->w32 = (float*)((char*)ctx->srules.ptr + b64);
    // rows of one boundary block each: every I&Z region's block starts "never"
    const int block = method == BMC_IZ ? rule_width(method, spec->d) : r->width;
    if ((e = launch_rules_fill(r->w64, r->w32, (int)(rows / block), block, never_value(method, spec->payoff),
                               ctx->stream)))
        return hip_fail(e, "rule scratch");
    return BMC_OK;
}

extern "C" bmc_status bmc_rules_create(bmc_ctx* ctx, const bmc_spec* spec, int32_t method,
                                       bmc_rules** out)
{
    if (!ctx || !out) return fail(BMC_EINVAL, "NULL argument");
    bmc_status st = validate_spec(spec);
    if (st) return st;
    if (method != BMC_CMC && method != BMC_IZ && method != BMC_CMC_ADA)
        return fail(BMC_EINVAL, "unknown method %d", method);
    if (method == BMC_IZ && spec->d > IZ_D_MAX)
        return fail(BMC_EUNSUPPORTED, "I&Z supports d <= %d", IZ_D_MAX);
    (void)hipSetDevice(ctx->device);
    return rules_alloc(ctx, method, spec->d, spec->n_dates, spec->payoff, out);
}

extern "C" void bmc_rules_destroy(bmc_rules* r)
{
    if (!r) return;
    if (r->w64) (void)hipFree(r->w64);
    if (r->w32) (void)hipFree(r->w32);
    delete r;
}

extern "C" int32_t bmc_rules_width(const bmc_rules* r) { return r ? r->width : 0; }

extern "C" bmc_status bmc_rules_set(bmc_rules* r, int32_t date, const double* w)
{
    if (!r || !w) return fail(BMC_EINVAL, "NULL argument");
    if (date < 1 || date >= r->n_dates) return fail(BMC_EINVAL, "date %d outside 1..%d", date, r->n_dates - 1);
    (void)hipSetDevice(r->ctx->device);
    std::vector<float> wf(r->width);
    for (int f = 0; f < r->width; ++f) wf[f] = (float)w[f];
    hipError_t e;
    if ((e = hipStreamSynchronize(r->ctx->stream)) ||
        (e = hipMemcpy(r->w64 + (size_t)date * r->width, w, sizeof(double) * r->width, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(r->w32 + (size_t)date * r->width, wf.data(), sizeof(float) * r->width, hipMemcpyHostToDevice)))
        return hip_fail(e, "rule upload");
    return BMC_OK;
}

extern "C" bmc_status bmc_rules_get(const bmc_rules* r, int32_t date, double* w)
{
    if (!r || !w) return fail(BMC_EINVAL, "NULL argument");
    if (date < 0 || date > r->n_dates) return fail(BMC_EINVAL, "date %d outside 0..%d", date, r->n_dates);
    (void)hipSetDevice(r->ctx->device);
    hipError_t e;
    if ((e = hipStreamSynchronize(r->ctx->stream)) ||
        (e = hipMemcpy(w, r->w64 + (size_t)date * r->width, sizeof(double) * r->width, hipMemcpyDeviceToHost)))
        return hip_fail(e, "rule download");
    return BMC_OK;
}

struct RulesHeader {
    char magic[4];
    int32_t version, method, d, n_dates, width, payoff, pad;
};

extern "C" bmc_status bmc_rules_export(const bmc_rules* r, void* buf, size_t* bytes)
{
    if (!r || !bytes) return fail(BMC_EINVAL, "NULL argument");
    const size_t rows = (size_t)(r->n_dates + 1) * r->width;
    const size_t need = sizeof(RulesHeader) + sizeof(double) * rows;
    if (!buf) {
        *bytes = need;
        return BMC_OK;
    }
    if (*bytes < need) return fail(BMC_EINVAL, "buffer too small: %zu < %zu", *bytes, need);
    RulesHeader h;
    std::memcpy(h.magic, "BMCR", 4);
    h.version = 1;
    h.method = r->method;
    h.d = r->d;
    h.n_dates = r->n_dates;
    h.width = r->width;
    h.payoff = r->payoff;
    h.pad = 0;
    std::memcpy(buf, &h, sizeof(h));
    (void)hipSetDevice(r->ctx->device);
    hipError_t e;
    if ((e = hipStreamSynchronize(r->ctx->stream)) ||
        (e = hipMemcpy((char*)buf + sizeof(h), r->w64, sizeof(double) * rows, hipMemcpyDeviceToHost)))
        return hip_fail(e, "rule export");
    *bytes = need;
    return BMC_OK;
}

extern "C" bmc_status bmc_rules_import(bmc_ctx* ctx, const void* buf, size_t bytes, bmc_rules** out)
{
    if (!ctx || !buf || !out) return fail(BMC_EINVAL, "NULL argument");
    RulesHeader h;
    if (bytes < sizeof(h)) return fail(BMC_EINVAL, "buffer too small");
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "BMCR", 4) != 0 || h.version != 1) return fail(BMC_EINVAL, "not a rule table");
    if (h.d < 1 || h.d > BMC_D_MAX || h.n_dates < 1 || h.n_dates > BMC_NT_MAX ||
        (h.method != BMC_CMC && h.method != BMC_IZ && h.method != BMC_CMC_ADA) ||
        h.width != rule_row_width(h.method, h.d, h.payoff))
        return fail(BMC_EINVAL, "corrupt rule table header");
    const size_t rows = (size_t)(h.n_dates + 1) * h.width;
    if (bytes < sizeof(h) + sizeof(double) * rows) return fail(BMC_EINVAL, "truncated rule table");
    (void)hipSetDevice(ctx->device);
    bmc_rules* r = nullptr;
    bmc_status st = rules_alloc(ctx, h.method, h.d, h.n_dates, h.payoff, &r);
    if (st) return st;
    std::vector<double> w(rows);
    std::memcpy(w.data(), (const char*)buf + sizeof(h), sizeof(double) * rows);
    std::vector<float> wf(rows);
    for (size_t i = 0; i < rows; ++i) wf[i] = (float)w[i];
    hipError_t e;
    if ((e = hipMemcpy(r->w64, w.data(), sizeof(double) * rows, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(r->w32, wf.data(), sizeof(float) * rows, hipMemcpyHostToDevice))) {
        bmc_rules_destroy(r);
        return hip_fail(e, "rule import");
    }
    *out = r;
    return BMC_OK;
}

static bmc_status check_rules(const bmc_rules* r, const bmc_spec* s)
{
    if (!r) return fail(BMC_EINVAL, "rules is NULL");
    if (r->d != s->d || r->n_dates != s->n_dates)
        return fail(BMC_EINVAL, "rule table (d=%d, dates=%d) does not match the spec (d=%d, dates=%d)",
                    r->d, r->n_dates, s->d, s->n_dates);
    if (r->width != rule_row_width(r->method, s->d, s->payoff))
        return fail(BMC_EINVAL, "rule table rows (%d coefficients) do not fit this payoff's I&Z regions", r->width);
    return BMC_OK;
}

static bmc_status check_prec(int32_t prec)
{
    if (prec < BMC_FP64 || prec > BMC_FP32_KAHAN) return fail(BMC_EINVAL, "unknown precision %d", prec);
    return BMC_OK;
}

static bmc_status check_seed(uint64_t seed)
{
    if (seed > 0xFFFFFFFFull) return fail(BMC_EINVAL, "seed must fit in 32 bits");
    return BMC_OK;
}

// ---------------------------------------------------------------------------
// Continuation launches

int bmc::n_class(int64_t n)
{
    int c = 0;
    while (c < 40 && ((int64_t)1 << c) < n) ++c;
    return c + 1;   // 1 + ceil(log2 n); 0 is the wildcard
}

uint64_t bmc::ppt_key(int bucket, int prec_plus1, int nclass)
{
    return ((uint64_t)(uint32_t)bucket << 32) | ((uint64_t)(uint32_t)prec_plus1 << 16) | (uint64_t)(uint32_t)nclass;
}

uint32_t bmc::choose_ppt(const bmc_ctx* ctx, int d, int prec, int64_t points, int64_t n, const Tuning* tune)
{
    if (tune && tune->ppt > 0) return (uint32_t)tune->ppt;
    if (ctx && !ctx->ppt_table.empty()) {
        const int b = cont_bucket(d), pr = prec + 1, c = n_class(n);
        for (int mask = 0; mask < 8; ++mask) {   // exact key first, then wildcards
            const uint64_t k = ppt_key(mask & 4 ? 0 : b, mask & 2 ? 0 : pr, mask & 1 ? 0 : c);
            auto it = ctx->ppt_table.find(k);
            if (it != ctx->ppt_table.end()) return (uint32_t)it->second;
        }
    }
    // enough lanes to fill 256 CUs x 2048 resident lanes, then longer chunks
    const double lanes = 256.0 * 2048.0;
    const double per_lane = (double)points * (double)n / lanes;
    uint32_t ppt = 1;
    while (ppt < 16 && (double)(ppt * 2) <= per_lane) ppt *= 2;
    return ppt;
}

extern "C" bmc_status bmc_tuning_set(bmc_ctx* ctx, int32_t d, int32_t precision, int64_t n, int32_t ppt)
{
    if (!ctx) return fail(BMC_EINVAL, "NULL argument");
    if (d < 0 || d > BMC_D_MAX) return fail(BMC_EINVAL, "d = %d outside 0..%d", d, BMC_D_MAX);
    if (precision < -1 || precision > BMC_FP32_KAHAN) return fail(BMC_EINVAL, "unknown precision %d", precision);
    if (n < 0 || n > 0x7FFFFFFF) return fail(BMC_EINVAL, "n out of range");
    if (ppt < 0 || ppt > 64) return fail(BMC_EINVAL, "ppt = %d outside 0..64", ppt);
    const uint64_t k = ppt_key(d ? cont_bucket(d) : 0, precision + 1, n ? n_class(n) : 0);
    if (ppt == 0) ctx->ppt_table.erase(k);
    else ctx->ppt_table[k] = ppt;
    return BMC_OK;
}

// Autotuner: times the continuation kernel of this spec for each launch
// shape ppt = 1, 2, 4, .. up to one chunk per point (at most 64), on CMC
// training points at the first, middle and last dates under exercise rules
// from a small CMC pricing of the same spec (N <= 4096 points, n/8 paths),
// so that path and job lengths spread as in a real sweep, and
// stores the shape with the largest executed path-steps per second over the
// three dates in the context's table for the spec's (dimension bucket,
// precision, n class).  With a single date (or N = 1) it times date 0.
extern "C" bmc_status bmc_autotune(bmc_ctx* ctx, const bmc_spec* spec, int32_t precision, int64_t N, int64_t n,
                                   int32_t* ppt_out)
{
    if (!ctx || !spec) return fail(BMC_EINVAL, "NULL argument");
    if (precision < BMC_FP64 || precision > BMC_FP32_KAHAN) return fail(BMC_EINVAL, "unknown precision %d", precision);
    if (N < 1 || N > (1 << 24) || n < 2 || n > 0x7FFFFFFF) return fail(BMC_EINVAL, "N or n out of range");
    (void)hipSetDevice(ctx->device);
    bmc_status st;
    const int d = spec->d, NT = spec->n_dates;
    // exercise rules close to the real ones, so that path lengths (and the
    // spread of job lengths) are realistic: a small CMC pricing first
    bmc_rules* learned = nullptr;
    if (NT >= 2) {
        bmc_opts o;
        std::memset(&o, 0, sizeof(o));
        o.method = BMC_CMC;
        o.precision = precision;
        o.N = std::min<int64_t>(std::max<int64_t>(N, 1024), 4096);
        o.n = std::max<int64_t>(256, std::min<int64_t>(n, 4096) / 8);
        o.n_final = 2;
        o.seed = 7;
        bmc_result tmp;
        if ((st = bmc_price_impl(ctx, spec, &o, &learned, &tmp, nullptr))) return st;
    }
    if ((st = upload_spec(ctx, spec, ctx->spec))) {
        bmc_rules_destroy(learned);
        return st;
    }
    bmc_rules scratch;
    if (!learned && (st = scratch_rules(ctx, spec, BMC_CMC, &scratch))) return st;
    const bmc_rules& rules = learned ? *learned : scratch;
    struct Release {
        bmc_rules* r;
        ~Release() { bmc_rules_destroy(r); }
    } release_learned{learned};
    std::vector<int> dates;
    if (NT >= 2 && N > 1) {
        for (int m : {1, NT / 2, NT - 1})
            if (m >= 1 && (dates.empty() || dates.back() != m)) dates.push_back(m);
    } else {
        dates.push_back(0);
    }
    hipError_t e;
    if ((e = ctx->x.ensure(sizeof(double) * d * N * dates.size())) || (e = ctx->B.ensure(sizeof(double) * d * N)) ||
        (e = ctx->counters.ensure(64)))
        return fail(BMC_ENOMEM, "autotune buffers: %s", hipGetErrorString(e));
    std::vector<const double*> pts(dates.size());
    for (size_t i = 0; i < dates.size(); ++i) {
        if (dates[i] == 0) {
            pts[i] = dev_S0(ctx->spec.ptr);
            continue;
        }
        double* x = (double*)ctx->x.ptr + (size_t)d * N * i;
        if ((st = sample_points_impl(ctx, ctx->spec.ptr, spec, BMC_CMC, dates[i], N, 1u, x, (double*)ctx->B.ptr)))
            return st;
        pts[i] = x;
    }
    const int64_t npts = dates[0] == 0 ? 1 : N;
    unsigned long long* total = (unsigned long long*)ctx->counters.ptr;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1))) return hip_fail(e, "autotune events");
    int best = 1;
    double best_rate = -1.0;
    const int64_t max_ppt = std::min<int64_t>(64, std::max<int64_t>(1, (n + 255) / 256));
    for (int ppt = 1; ppt <= max_ppt && !st; ppt *= 2) {
        Tuning t;
        t.ppt = ppt;
        double secs = 0.0, steps_all = 0.0;
        for (int rep = 0; rep < 4 && !st; ++rep) {   // rep 0 warms up
            for (size_t i = 0; i < dates.size() && !st; ++i) {
                const int m = dates[i];
                if ((e = hipMemsetAsync(total, 0, sizeof(unsigned long long), ctx->stream)) ||
                    (e = hipEventRecord(e0, ctx->stream))) {
                    st = hip_fail(e, "autotune");
                    break;
                }
                st = run_cont(ctx, ctx->spec.ptr, d, NT, BMC_CMC, rules.width, rules.w64, rules.w32, precision, m,
                              pts[i], npts, nullptr, nullptr, (uint32_t)n, 1u,
                              key_hi(m == 0 ? BMC_STREAM_FINAL : BMC_STREAM_INNER, m), nullptr, nullptr, nullptr,
                              nullptr, total, &t);
                unsigned long long steps = 0;
                float ms = 0.f;
                if (!st && ((e = hipEventRecord(e1, ctx->stream)) ||
                            (e = hipMemcpyAsync(&steps, total, sizeof(steps), hipMemcpyDeviceToHost, ctx->stream)) ||
                            (e = hipStreamSynchronize(ctx->stream)) || (e = hipEventElapsedTime(&ms, e0, e1))))
                    st = hip_fail(e, "autotune");
                if (!st && rep > 0) {
                    secs += ms * 1e-3;
                    steps_all += (double)steps;
                }
            }
        }
        const double rate = secs > 0.0 ? steps_all / secs : 0.0;
        if (!st && rate > best_rate) {
            best_rate = rate;
            best = ppt;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    ctx->ppt_table[ppt_key(cont_bucket(d), precision + 1, n_class(n))] = best;
    if (ppt_out) *ppt_out = best;
    return BMC_OK;
}

extern "C" bmc_status bmc_tuning_get(bmc_ctx* ctx, int32_t d, int32_t precision, int64_t N, int64_t n, int32_t* ppt)
{
    if (!ctx || !ppt) return fail(BMC_EINVAL, "NULL argument");
    if (d < 1 || d > BMC_D_MAX) return fail(BMC_EINVAL, "d = %d outside 1..%d", d, BMC_D_MAX);
    if (precision < BMC_FP64 || precision > BMC_FP32_KAHAN) return fail(BMC_EINVAL, "unknown precision %d", precision);
    if (N < 1 || n < 1) return fail(BMC_EINVAL, "N and n must be positive");
    *ppt = (int32_t)choose_ppt(ctx, d, precision, N, n, nullptr);
    return BMC_OK;
}

// Launch shape, partial-sum buffer and arguments of one continuation pass
// over N points (ids/n_ids: the active ones, or null for all).  With an
// active list, max_active > 0 is a bound on its count known to the host: the
// grid then holds that many points' jobs (the jobs are slot-major, and the
// slots past the count return at once, so the results are unchanged).
static bmc_status prepare_cont(bmc_ctx* ctx, const void* devspec, int d, int n_dates, int method, int width,
                               const void* rules64, const void* rules32, int prec, int m, const double* x, int64_t N,
                               const int32_t* ids, const int32_t* n_ids, uint32_t n, uint32_t k0, uint32_t k1,
                               const Tuning* tune, uint32_t slot, uint32_t region_pts, ContArgs& a, int& block,
                               size_t& lds, int64_t& grid, double* part = nullptr, const IzFuse* fz = nullptr,
                               const JobOrder* ord = nullptr, int64_t max_active = 0)
{
    block = (tune && tune->block > 0) ? tune->block : 256;
    const uint32_t ppt = choose_ppt(ctx, d, prec, N, n, tune);
    const uint32_t per_wg = (uint32_t)block * ppt;
    const uint32_t nchunk = (n + per_wg - 1) / per_wg;
    if (!part) {
        const size_t part_bytes = sizeof(double) * 3 * (size_t)N * nchunk;
        hipError_t e = ctx->part.ensure(part_bytes);
        if (e) return hip_fail(e, "partials allocation");
    }
    lds = cont_lds_bytes(prec, d, n_dates, width);
    if (lds > cont_lds_limit()) return fail(BMC_EUNSUPPORTED, "rule table too large for LDS (%zu bytes)", lds);
    const int64_t cols = (ids && max_active > 0 && max_active < N) ? max_active : N;
    grid = cols * nchunk;
    if (grid > 0x7FFFFFFF) return fail(BMC_EINVAL, "too many jobs in one launch");
    a.spec = (const DevSpec*)devspec;
    a.rules = prec == BMC_FP64 ? rules64 : rules32;
    a.x = x;
    a.N = N;
    a.ids = ids;
    a.n_ids = n_ids;
    a.n = n;
    a.m = m;
    a.method = method;
    a.width = width;
    a.paths_per_wg = per_wg;
    a.nchunk = nchunk;
    a.k0 = k0;
    a.k1 = k1;
    a.slot = slot;
    a.region_pts = region_pts;
    a.part = part ? part : (double*)ctx->part.ptr;
    a.fz = fz ? *fz : IzFuse{};
    a.ord = (ord && !ids) ? *ord : JobOrder{};
    return BMC_OK;
}

// Chunks per point of a continuation pass (the split prepare_cont makes).
static uint32_t cont_nchunk(const bmc_ctx* ctx, int d, int prec, int64_t N, uint32_t n, const Tuning* tune)
{
    const int block = (tune && tune->block > 0) ? tune->block : 256;
    const uint32_t per_wg = (uint32_t)block * choose_ppt(ctx, d, prec, N, n, tune);
    return (n + per_wg - 1) / per_wg;
}

bmc_status bmc::run_cont(bmc_ctx* ctx, const void* devspec, int d, int n_dates, int method,
                         int width, const void* rules64, const void* rules32, int prec, int m,
                         const double* x, int64_t N, const int32_t* ids, const int32_t* n_ids,
                         uint32_t n, uint32_t k0, uint32_t k1, double* cont, double* se,
                         int64_t* steps, double* sums, unsigned long long* steps_total,
                         const Tuning* tune, uint32_t slot, uint32_t region_pts, uint32_t* nchunk_out,
                         double* part, const IzFuse* fz, const RefineSel* sel, const JobOrder* ord,
                         int64_t max_active)
{
    ContArgs a{};
    int block = 256;
    size_t lds = 0;
    int64_t grid = 0;
    bmc_status st = prepare_cont(ctx, devspec, d, n_dates, method, width, rules64, rules32, prec, m, x, N, ids,
                                 n_ids, n, k0, k1, tune, slot, region_pts, a, block, lds, grid, part, fz, ord,
                                 max_active);
    if (st) return st;
    const uint32_t nchunk = a.nchunk;
    hipError_t e;
    if ((e = launch_cont(d, prec, a, (int)grid, block, lds, ctx->stream))) return hip_fail(e, "continuation launch");
    if (nchunk_out) {   // the caller merges the partials (ctx->part) itself
        *nchunk_out = nchunk;
        return BMC_OK;
    }
    if ((e = launch_finalize(a.part, nchunk, n, N, ids, n_ids, cont, se, steps, sums, steps_total,
                             ctx->stream, sel)))
        return hip_fail(e, "finalize launch");
    return BMC_OK;
}

bool bmc::refine_supported(int prec, int d, int n_dates, int width)
{
    return prec != BMC_FP64 && cont_lds_bytes(BMC_FP64, d, n_dates, width) <= cont_lds_limit();
}

bmc_status bmc::refine_labels(bmc_ctx* ctx, const void* devspec, int d, int n_dates, const bmc_rules* rules, int m,
                              const double* x, int64_t N, uint32_t n, uint32_t seed, double* cont, const int32_t* ids,
                              const int32_t* n_ids)
{
    hipError_t e;
    ContArgs a{};
    int block = 256;
    size_t lds = 0;
    int64_t grid = 0;
    const Tuning one{256, REFINE_PPT};
    bmc_status st = prepare_cont(ctx, devspec, d, n_dates, rules->method, rules->width, rules->w64, rules->w32,
                                 BMC_FP64, m, x, N, ids, n_ids, n, seed, key_hi(BMC_STREAM_INNER, m), &one, 0, 0, a,
                                 block, lds, grid);
    if (st) return st;
    a.slot_stride = (uint32_t)std::min<int64_t>(N, REFINE_SLOTS);
    if ((e = launch_cont(d, BMC_FP64, a, (int)(a.slot_stride * a.nchunk), block, lds, ctx->stream)))
        return hip_fail(e, "refinement launch");
    if ((e = launch_finalize(a.part, a.nchunk, n, N, ids, n_ids, cont, nullptr, nullptr, nullptr, nullptr,
                             ctx->stream)))
        return hip_fail(e, "refinement finalize");
    return BMC_OK;
}

// ---------------------------------------------------------------------------
// Entry points on device arrays

extern "C" bmc_status bmc_estimate_continuation(bmc_ctx* ctx, const bmc_spec* spec, const bmc_rules* rules,
                                                int32_t date, const double* x, int64_t N, int64_t n,
                                                uint64_t seed, int32_t precision, double* cont,
                                                double* std_err, int64_t* steps)
{
    if (!ctx || !x || !cont || !std_err) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    bmc_status st;
    if ((st = upload_spec(ctx, spec, ctx->spec))) return st;
    if ((st = check_rules(rules, spec)) || (st = check_prec(precision)) || (st = check_seed(seed))) return st;
    if (date < 0 || date >= spec->n_dates) return fail(BMC_EINVAL, "date %d outside 0..%d", date, spec->n_dates - 1);
    if (N < 1 || N > 0x7FFFFFFF) return fail(BMC_EINVAL, "N = %lld out of range", (long long)N);
    if (n < 2 || n > 0x7FFFFFFF) return fail(BMC_EINVAL, "n = %lld out of range", (long long)n);
    return run_cont(ctx, ctx->spec.ptr, spec->d, spec->n_dates, rules->method, rules->width, rules->w64,
                    rules->w32, precision, date, x, N, nullptr, nullptr, (uint32_t)n, (uint32_t)seed,
                    key_hi(BMC_STREAM_INNER, date), cont, std_err, steps, nullptr, nullptr, nullptr);
}

bmc_status bmc::fit_rule_impl(bmc_ctx* ctx, const void* devspec, int d, bmc_rules* rules, int date,
                              const double* x, const double* values, int64_t N, int rounds, int region,
                              int64_t ld)
{
    hipError_t e;
    double* row64 = rules->w64 + (size_t)date * rules->width;
    float* row32 = rules->w32 + (size_t)date * rules->width;
    if (rules->method == BMC_CMC) {
        const int p = rules->width;
        if ((e = ctx->fit.ensure(sizeof(double) * fit_scratch_doubles(N, p, rounds))))
            return hip_fail(e, "fit scratch");
        FitScratch fs;
        fit_scratch_carve((double*)ctx->fit.ptr, N, p, rounds, &fs);
        if (!ctx->gbar.ptr) {   // barrier words: zero once; every launch leaves them zero
            if ((e = ctx->gbar.ensure(256)) || (e = hipMemsetAsync(ctx->gbar.ptr, 0, 256, ctx->stream)))
                return hip_fail(e, "fit barrier");
        }
        if ((e = launch_fit_cmc((const DevSpec*)devspec, d, x, values, N, rounds, fs, row64, row32, ctx->stream,
                                (unsigned*)ctx->gbar.ptr, fit_barrier_flag_dev(ctx))))
            return hip_fail(e, "fit launch");
    } else if (rules->method == BMC_CMC_ADA) {
        if ((e = ctx->fit.ensure(fit_ada_scratch_bytes(N, d)))) return hip_fail(e, "fit scratch");
        if ((e = launch_fit_ada((const DevSpec*)devspec, d, x, values, N, rounds, ctx->fit.ptr, row64, row32,
                                rules->width, ctx->stream)))
            return hip_fail(e, "fit launch");
    } else {
        const int p = rule_width(BMC_IZ, d);
        if ((e = ctx->fit.ensure(sizeof(double) * fitiz_scratch_doubles(N, p)))) return hip_fail(e, "fit scratch");
        if ((e = launch_fit_iz((const DevSpec*)devspec, d, region, x, N, ld > 0 ? ld : N, (double*)ctx->fit.ptr,
                               row64 + (size_t)region * p, row32 + (size_t)region * p, ctx->stream)))
            return hip_fail(e, "fit launch");
    }
    return BMC_OK;
}

static bmc_status check_region(int method, const bmc_spec* spec, int32_t region)
{
    const int regions = method == BMC_IZ ? iz_regions(spec->payoff, spec->d) : 1;
    if (region < 0 || region >= regions)
        return fail(BMC_EINVAL, "region %d outside 0..%d", region, regions - 1);
    return BMC_OK;
}

extern "C" int32_t bmc_iz_regions(const bmc_spec* spec)
{
    if (!spec || spec->d < 1) return 0;
    return iz_regions(spec->payoff, spec->d);
}

extern "C" bmc_status bmc_fit_rule(bmc_ctx* ctx, const bmc_spec* spec, bmc_rules* rules, int32_t date,
                                   int32_t region, const double* x, const double* values, int64_t N,
                                   int32_t rounds)
{
    if (!ctx || !x) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    bmc_status st;
    if ((st = upload_spec(ctx, spec, ctx->spec))) return st;
    if ((st = check_rules(rules, spec)) || (st = check_region(rules->method, spec, region))) return st;
    if (date < 1 || date >= spec->n_dates) return fail(BMC_EINVAL, "date %d outside 1..%d", date, spec->n_dates - 1);
    if (N < 1 || N > 0x7FFFFFFF) return fail(BMC_EINVAL, "N out of range");
    if (rules->method != BMC_IZ && !values) return fail(BMC_EINVAL, "CMC fit needs continuation values");
    if (rounds <= 0) rounds = rules->method == BMC_CMC_ADA ? ADA_TMAX : 8;
    if (rounds > 64) return fail(BMC_EINVAL, "rounds must be <= 64");
    if ((st = fit_rule_impl(ctx, ctx->spec.ptr, spec->d, rules, date, x, values, N, rounds, region))) return st;
    if (rules->method != BMC_CMC) return BMC_OK;
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(e, "stream sync");
    return check_fit_barrier(ctx);
}

bmc_status bmc::sample_points_impl(bmc_ctx* ctx, const void* devspec, const bmc_spec* spec, int method,
                                   int date, int64_t N, uint32_t seed, double* x, double* Bbuf, int region,
                                   int nreg)
{
    hipError_t e;
    const DevSpec* ds = (const DevSpec*)devspec;
    const int d = spec->d, NT = spec->n_dates;
    if (method != BMC_IZ) {
        if ((e = launch_bridge_end(ds, d, N, seed, Bbuf, ctx->stream))) return hip_fail(e, "bridge");
        for (int mm = NT - 1; mm >= date; --mm)
            if ((e = launch_bridge_back(ds, d, mm, N, seed, Bbuf, nullptr, 1, ctx->stream)))
                return hip_fail(e, "bridge");
        if ((e = launch_bridge_back(ds, d, date, N, seed, Bbuf, x, 0, ctx->stream))) return hip_fail(e, "points");
    } else {
        const unsigned long long* best = nullptr;
        if (d - 1 >= 2 && N > 2) {
            // the generator depends on (J, q) only: searched once, kept for
            // the following dates and calls
            if ((e = ctx->korobov.ensure(sizeof(unsigned long long)))) return hip_fail(e, "korobov");
            if (ctx->korobov_J != N || ctx->korobov_q != d - 1) {
                ctx->korobov_J = -1;
                if ((e = hipMemsetAsync(ctx->korobov.ptr, 0, sizeof(unsigned long long), ctx->stream)))
                    return hip_fail(e, "korobov");
                if ((e = launch_korobov(N, d - 1, (unsigned long long*)ctx->korobov.ptr, ctx->stream)))
                    return hip_fail(e, "korobov");
                ctx->korobov_J = N;
                ctx->korobov_q = d - 1;
            }
            best = (const unsigned long long*)ctx->korobov.ptr;
        }
        if ((e = launch_lattice(ds, d, date, region, nreg, N, best, x, ctx->stream))) return hip_fail(e, "lattice");
    }
    return BMC_OK;
}

extern "C" bmc_status bmc_sample_points(bmc_ctx* ctx, const bmc_spec* spec, int32_t method, int32_t date,
                                        int32_t region, int64_t N, uint64_t seed, double* x)
{
    if (!ctx || !x) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    bmc_status st;
    if ((st = upload_spec(ctx, spec, ctx->spec)) || (st = check_seed(seed))) return st;
    if (method != BMC_CMC && method != BMC_IZ && method != BMC_CMC_ADA)
        return fail(BMC_EINVAL, "unknown method %d", method);
    if ((st = check_region(method, spec, region))) return st;
    if (date < 1 || date > spec->n_dates) return fail(BMC_EINVAL, "date %d outside 1..%d", date, spec->n_dates);
    if (N < 1 || N > 0x7FFFFFFF) return fail(BMC_EINVAL, "N out of range");
    if (method == BMC_IZ && (spec->d > IZ_D_MAX || N > 65536))
        return fail(BMC_EUNSUPPORTED, "I&Z lattice supports d <= %d and J <= 65536", IZ_D_MAX);
    hipError_t e = ctx->B.ensure(sizeof(double) * spec->d * N);
    if (e) return hip_fail(e, "bridge buffer");
    return sample_points_impl(ctx, ctx->spec.ptr, spec, method, date, N, (uint32_t)seed, x, (double*)ctx->B.ptr,
                              region);
}

bmc_status bmc::iz_search_impl(bmc_ctx* ctx, const void* devspec, const bmc_spec* spec, const bmc_rules* rules,
                               int date, int region, int nreg, const double* x, int64_t J, uint32_t n,
                               uint32_t seed, int prec, double eps, int max_iter, int mode, double* s_out,
                               int32_t* iters, int64_t* steps_out, const Tuning* tune,
                               unsigned long long* tally, int32_t* ties, int again)
{
    const int d = spec->d;
    const int64_t Jr = J;   // points per region
    J *= nreg;              // columns of all regions
    hipError_t e;
    // FP32 searches with tie flags: the buffers also fit the FP64 search of
    // the flagged points that follows (again = 1), which keeps the others' results
    const double tau = (ties && !again) ? IZ_TIE_TAU * spec->K : 0.0;
    // Iteration it is one continuation launch over the columns active after
    // step it - 1, which also takes that step (IzFuse; iteration 0: a plain
    // pass over all columns); a last step launch follows the last pass.
    // Double-buffered across iterations: the partials P[it % 2] of pass it,
    // the search state St[t % 2] read by step t, the active lists A[it % 2].
    // Buffers: x_work [d][J], St 2 x [3][J], P 2 x [3 J nchunk], steps_acc [J],
    // ids 2 x [J].
    const Tuning research{256, IZ_RESEARCH_PPT};
    if (again) tune = &research;
    const uint32_t nch = cont_nchunk(ctx, d, prec, J, n, tune);
    const size_t part_n = (size_t)3 * J * (ties ? std::max(nch, cont_nchunk(ctx, d, BMC_FP64, J, n, &research)) : nch);
    const size_t need = sizeof(double) * ((size_t)d * J + 6 * J + 2 * part_n) + sizeof(unsigned long long) * J +
                        sizeof(int32_t) * 2 * J + 64;
    if ((e = ctx->iz.ensure(need))) return hip_fail(e, "search buffers");
    if ((e = ctx->counters.ensure(64))) return hip_fail(e, "counters");
    char* c = (char*)ctx->iz.ptr;
    double* x_work = (double*)c; c += sizeof(double) * d * J;
    double* St[2];
    St[0] = (double*)c; c += sizeof(double) * 3 * J;
    St[1] = (double*)c; c += sizeof(double) * 3 * J;
    double* P[2];
    P[0] = (double*)c; c += sizeof(double) * part_n;
    P[1] = (double*)c; c += sizeof(double) * part_n;
    unsigned long long* acc = (unsigned long long*)c; c += sizeof(unsigned long long) * J;
    int32_t* A[2];
    A[0] = (int32_t*)c; c += sizeof(int32_t) * J;
    A[1] = (int32_t*)c;
    // counters buffer: [0,8) step total, [16,40) final sums/steps, [48,60) three
    // rotating active counts: cnt[it % 3] counts A[it % 2]; the launch of
    // iteration it appends to it and clears cnt[(it + 1) % 3]
    int32_t* cnt = (int32_t*)((char*)ctx->counters.ptr + 48);
    const DevSpec* ds = (const DevSpec*)devspec;
    if (again && (e = hipMemsetAsync(cnt, 0, 3 * sizeof(int32_t), ctx->stream))) return hip_fail(e, "search init");
    if ((e = launch_iz_init(ds, x, d, region, nreg, Jr, x_work, St[0], s_out, iters, A[0], &cnt[0], acc,
                            ctx->stream, ties, again)))
        return hip_fail(e, "search init");
    const uint32_t k1 = key_hi(BMC_STREAM_INNER, date);
    // Progress polls without stalling the stream: every fourth launch writes
    // the active count it starts from (the previous pass's) to pinned memory
    // and an event follows it; the host reads the count once the event has
    // passed, with at most two polls outstanding.  Iterations enqueued after
    // the count reached zero find no active point and change nothing.
    for (hipEvent_t& ev : ctx->poll_ev)
        if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming))) return hip_fail(e, "search events");
    volatile int32_t* poll_host = (volatile int32_t*)((char*)ctx->host_io + 128);
    int32_t* poll_dev = (int32_t*)((char*)ctx->host_io_dev + 128);
    int polls_issued = 0, polls_read = 0;
    bool done = false;
    // a bound on the active count: the last count a poll returned (the lists
    // only shrink), which caps the grid of the launches enqueued after it
    int64_t active_max = J;
    auto read_poll = [&](bool wait) -> hipError_t {
        hipEvent_t ev = ctx->poll_ev[polls_read & 1];
        const hipError_t q = wait ? hipEventSynchronize(ev) : hipEventQuery(ev);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();   // not an error: keep it out of the next launch check
            return hipSuccess;
        }
        if (q != hipSuccess) return q;
        const int32_t v = poll_host[polls_read & 1];
        if (v == 0) done = true;
        else if (v > 0 && v < active_max) active_max = v;
        ++polls_read;
        return hipSuccess;
    };
    int last = -1;
    for (int it = 0; it < max_iter && !done; ++it) {
        IzFuse fz{};
        if (it > 0) {
            fz.on = 1;
            fz.it = it - 1;
            fz.max_iter = max_iter;
            fz.mode = mode;
            fz.eps = eps;
            fz.part = P[(it - 1) & 1];
            fz.st_r = St[(it - 1) & 1];
            fz.st_w = St[it & 1];
            fz.x_work = x_work;
            fz.s_out = s_out;
            fz.iters = iters;
            fz.steps_acc = acc;
            fz.ids_out = A[it & 1];
            fz.n_out = &cnt[it % 3];
            fz.n_next = &cnt[(it + 1) % 3];
            fz.ties = tau > 0.0 ? ties : nullptr;
            fz.tau = tau;
        }
        const int prev = it > 0 ? it - 1 : 0;
        // launch it >= 4 with it % 4 == 0 reports the count after pass it - 1;
        // the FP64 search of the near-tie points also reports its first count
        // (often zero), so that an empty one ends after a launch or two
        const bool poll = (it > 0 && (it & 3) == 0) || (again && it == 0);
        if (poll) {
            if (polls_issued - polls_read == 2 && (e = read_poll(true))) return hip_fail(e, "search progress");
            if (done) break;
            fz.poll = poll_dev + (polls_issued & 1);
        }
        uint32_t nchunk = 0;
        bmc_status st = run_cont(ctx, devspec, d, spec->n_dates, rules->method, rules->width, rules->w64,
                                 rules->w32, prec, date, x_work, J, A[prev & 1], &cnt[prev % 3], n, seed, k1,
                                 nullptr, nullptr, nullptr, nullptr, nullptr, tune, (uint32_t)region,
                                 nreg > 1 ? (uint32_t)Jr : 0u, &nchunk, P[it & 1], &fz, nullptr, nullptr,
                                 active_max);
        if (st) return st;
        if (nchunk != nch) return fail(BMC_EDEVICE, "search pass split %u chunks, expected %u", nchunk, nch);
        last = it;
        if (poll) {
            if ((e = hipEventRecord(ctx->poll_ev[polls_issued & 1], ctx->stream))) return hip_fail(e, "search progress");
            ++polls_issued;
        }
        while (!done && polls_read < polls_issued) {
            const int before = polls_read;
            if ((e = read_poll(false))) return hip_fail(e, "search progress");
            if (polls_read == before) break;   // the oldest poll has not passed yet
        }
    }
    // the step of the last pass
    if (last >= 0 &&
        (e = launch_iz_update(ds, d, region, nreg, Jr, P[last & 1], nch, n, A[last & 1], &cnt[last % 3],
                              A[(last + 1) & 1], &cnt[(last + 1) % 3], &cnt[(last + 2) % 3], St[last & 1],
                              St[(last + 1) & 1], x_work, s_out, iters, acc, eps, max_iter, mode, last,
                              ctx->stream, tau, tau > 0.0 ? ties : nullptr)))
        return hip_fail(e, "search update");
    if (tally && (e = launch_iz_tally(acc, s_out, iters, J, tally, ctx->stream))) return hip_fail(e, "search tally");
    if (steps_out) {
        std::vector<unsigned long long> h(J);
        if ((e = hipMemcpyAsync(h.data(), acc, sizeof(unsigned long long) * J, hipMemcpyDeviceToHost,
                                ctx->stream)) ||
            (e = hipStreamSynchronize(ctx->stream)))
            return hip_fail(e, "search steps");
        unsigned long long tot = 0;
        for (int64_t j = 0; j < J; ++j) tot += h[j];
        *steps_out = (int64_t)tot;
    }
    return BMC_OK;
}

extern "C" bmc_status bmc_iz_search(bmc_ctx* ctx, const bmc_spec* spec, const bmc_rules* rules, int32_t date,
                                    int32_t region, const double* x, int64_t J, int64_t n, uint64_t seed,
                                    int32_t precision, double eps, int32_t max_iter, int32_t mode,
                                    double* s_out, int32_t* iters, int64_t* steps)
{
    if (!ctx || !x || !s_out || !iters) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    bmc_status st;
    if ((st = upload_spec(ctx, spec, ctx->spec))) return st;
    if ((st = check_rules(rules, spec)) || (st = check_prec(precision)) || (st = check_seed(seed))) return st;
    if (rules->method != BMC_IZ) return fail(BMC_EINVAL, "I&Z search needs an I&Z rule table");
    if ((st = check_region(BMC_IZ, spec, region))) return st;
    if (date < 1 || date >= spec->n_dates) return fail(BMC_EINVAL, "date %d outside 1..%d", date, spec->n_dates - 1);
    if (J < 1 || J > 0x7FFFFFFF || n < 2 || n > 0x7FFFFFFF) return fail(BMC_EINVAL, "J or n out of range");
    if (!(eps > 0.0) || max_iter < 1) return fail(BMC_EINVAL, "eps must be > 0 and max_iter >= 1");
    if (mode != BMC_SEARCH_PLAIN && mode != BMC_SEARCH_SECANT) return fail(BMC_EINVAL, "unknown search mode %d", mode);
    st = iz_search_impl(ctx, ctx->spec.ptr, spec, rules, date, region, 1, x, J, (uint32_t)n, (uint32_t)seed,
                        precision, eps, max_iter, mode, s_out, iters, steps, nullptr);
    if (st) return st;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(e, "stream sync");
    return BMC_OK;
}

bmc_status bmc::final_price_impl(bmc_ctx* ctx, const void* devspec, const bmc_spec* spec, const bmc_rules* rules,
                                 int64_t n_final, uint32_t seed, int prec, double* host_sums,
                                 const Tuning* tune, bool sync)
{
    hipError_t e;
    // the finalize of the one point stores its sums and step count straight
    // into the pinned host_io (plain stores, visible once the stream is synchronized)
    double* sums = (double*)ctx->host_io_dev;                         // [2]
    int64_t* fsteps = (int64_t*)((char*)ctx->host_io_dev + 16);
    bmc_status st = run_cont(ctx, devspec, spec->d, spec->n_dates, rules->method, rules->width, rules->w64,
                             rules->w32, prec, 0, dev_S0(devspec), 1, nullptr, nullptr, (uint32_t)n_final,
                             seed, key_hi(BMC_STREAM_FINAL, 0), nullptr, nullptr, fsteps, sums, nullptr, tune);
    if (st) return st;
    if (!sync) return BMC_OK;
    if ((e = hipStreamSynchronize(ctx->stream))) return hip_fail(e, "final read");
    read_final_sums(ctx, host_sums);
    return BMC_OK;
}

void bmc::read_final_sums(const bmc_ctx* ctx, double* host_sums)
{
    std::memcpy(host_sums, ctx->host_io, 16);
    int64_t fs;
    std::memcpy(&fs, (const char*)ctx->host_io + 16, 8);
    host_sums[2] = (double)fs;
}

void bmc::fill_price(const double* sums, int64_t n_final, bmc_result* out)
{
    const double s = sums[0], q = sums[1], nn = (double)n_final;
    double var = (q - s * s / nn) / (nn - 1.0);
    if (var < 0.0) var = 0.0;
    out->price = s / nn;
    out->variance = var;
    out->std_err = std::sqrt(var / nn);
    out->ci95 = 1.96 * out->std_err;
    out->final_path_steps = (int64_t)sums[2];
}

extern "C" bmc_status bmc_final_price(bmc_ctx* ctx, const bmc_spec* spec, const bmc_rules* rules,
                                      int64_t n_final, uint64_t seed, int32_t precision, bmc_result* out)
{
    if (!ctx || !out) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    bmc_status st;
    if ((st = upload_spec(ctx, spec, ctx->spec))) return st;
    if ((st = check_rules(rules, spec)) || (st = check_prec(precision)) || (st = check_seed(seed))) return st;
    if (n_final < 2 || n_final > 0x7FFFFFFF) return fail(BMC_EINVAL, "n_final out of range");
    double sums[3];
    if ((st = final_price_impl(ctx, ctx->spec.ptr, spec, rules, n_final, (uint32_t)seed, precision, sums, nullptr)))
        return st;
    bmc_result r;
    std::memset(&r, 0, sizeof(r));
    fill_price(sums, n_final, &r);
    r.seconds = r.final_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = r;
    return BMC_OK;
}

extern "C" bmc_status bmc_philox(bmc_ctx* ctx, uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t M,
                                 uint32_t* out)
{
    if (!ctx || !ctr || !out || M < 0) return fail(BMC_EINVAL, "bad argument");
    (void)hipSetDevice(ctx->device);
    if (M == 0) return BMC_OK;
    hipError_t e = launch_philox(k0, k1, ctr, M, out, ctx->stream);
    return e ? hip_fail(e, "philox launch") : BMC_OK;
}

extern "C" bmc_status bmc_normals(bmc_ctx* ctx, uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t M,
                                  int32_t precision, double* out)
{
    if (!ctx || !ctr || !out || M < 0) return fail(BMC_EINVAL, "bad argument");
    bmc_status st = check_prec(precision);
    if (st) return st;
    (void)hipSetDevice(ctx->device);
    if (M == 0) return BMC_OK;
    hipError_t e = launch_normals(k0, k1, ctr, M, precision == BMC_FP64 ? 0 : 1, out, ctx->stream);
    return e ? hip_fail(e, "normals launch") : BMC_OK;
}
