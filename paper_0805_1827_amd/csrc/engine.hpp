// Round engine shared by batched pricing and the serving loop: many CMC
// pricings (Algorithm 2) advance together, one stage per round (a date to
// learn, or the final pricing), sharing every launch of the round.  Each
// pricing keeps the shapes of bmc_price (chunking, tiles, merge orders), so
// its price and rules are bit-identical to a standalone run on the same
// context.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"

namespace bmc {

// One pricing as the engine runs it.  Byte offsets locate its buffers in one
// contiguous device region: [rules64][rules32][counters][B][x][cont][part][fit];
// the first three (zero_bytes) start at zero.
// FP32 pricings also hold the list of their label refinement (refine: the
// FP64 tables fit the LDS), whose FP64 pass runs rnchunk chunks of rper_wg
// paths per point (REFINE_PPT paths per lane).
struct OptPlan {
    int d, NT, p, prec, rounds, bucket;
    int64_t N;
    uint32_t n, n_final, seed;
    uint32_t nchunk, per_wg, fnchunk, fper_wg, rnchunk, rper_wg;
    int refine;
    size_t lds, lds64;                                       // continuation LDS bytes
    size_t ow64, ow32, ocnt, oB, ox, ocont, opart, ofit, oids;
    size_t zero_bytes, bytes;
};

// Validates a CMC request and fills its plan (statuses as bmc_price).
bmc_status plan_option(const bmc_ctx* ctx, const bmc_spec* spec, const bmc_opts* opts, int index, OptPlan* q);

// Device view of one pricing.  cnt: [steps_total, sum, sum of squares,
// final path-steps] (u64, double, double, i64).
struct OptDev {
    const DevSpec* spec;
    double *B, *x, *cont, *part, *fit, *w64;
    float* w32;
    uint64_t* cnt;
    int32_t *ids, *n_ids;   // refinement list and its count (FP32 pricings)
    const int32_t* cancel;  // device cancel word of a served request (or null)
};
OptDev carve_option(const OptPlan& q, const DevSpec* spec, char* base);

// A pricing's work in one round: stage m >= 1 learns date m (the first one,
// m = N_T - 1, also draws the Brownian end points); stage 0 is the final pricing.
struct RoundItem {
    const OptPlan* q;
    const OptDev* dev;
    int stage;
};

enum StepKind { K_BRIDGE_END, K_BRIDGE_BACK, K_CONT, K_FIN, K_FIT, K_FIT_SINGLE, K_MARK };
enum { PH_CALC = 0, PH_FIT = 1, PH_FINAL = 2 };

struct Step {
    int kind = K_MARK;
    int bucket = 0, prec = 0, ntasks = 0, T = 0, phase = -1;
    bool stride = false;             // K_CONT: tasks with a slot stride (label refinement)
    uint32_t blocks = 0;             // grid (K_CONT: total jobs)
    size_t tasks = 0, prefix = 0;    // table offsets
    size_t lds = 0;
    OptPlan single_q;                // K_FIT_SINGLE: the pricing and its date
    OptDev single_dev;
    int date = 0;
};

// Host image of the task tables of one or more rounds.
struct Table {
    std::vector<char> bytes;
    template <class T>
    size_t put(const std::vector<T>& v)
    {
        const size_t off = (bytes.size() + 255) & ~(size_t)255;
        bytes.resize(off + sizeof(T) * v.size());
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), sizeof(T) * v.size());
        return off;
    }
};

// Appends the launches of one round (phase marks included) to steps.
bmc_status plan_round(const std::vector<RoundItem>& items, Table& tab, std::vector<Step>& steps);

// Enqueues steps on st with the tables at dtab (device copy of Table::bytes);
// mark(phase) is called at each phase mark.
template <class Mark>
hipError_t run_steps(const std::vector<Step>& steps, const char* dtab, hipStream_t st, Mark mark);
hipError_t run_step(const Step& s, const char* dtab, hipStream_t st);

template <class Mark>
hipError_t run_steps(const std::vector<Step>& steps, const char* dtab, hipStream_t st, Mark mark)
{
    for (const Step& s : steps) {
        if (s.kind == K_MARK) {
            mark(s.phase);
            continue;
        }
        const hipError_t e = run_step(s, dtab, st);
        if (e) return e;
    }
    return hipSuccess;
}

}  // namespace bmc
