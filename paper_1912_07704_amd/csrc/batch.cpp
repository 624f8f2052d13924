// Host core of the batched integer forward: buffer layout of the beams and
// the order of the persistent launch's work items (most expensive first, so
// the queue drains evenly).  Plain C++, no HIP.
#include <algorithm>
#include <new>
#include <string>

#include "plan.h"

namespace dd {

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

dd_status build_batch(const Plan *const *plans, int32_t nbeams, Batch *b, std::string *err)
{
    if (!plans || nbeams <= 0) {
        *err = "need at least one plan";
        return nbeams <= 0 ? DD_ERR_INVALID : DD_ERR_NULL;
    }
    try {
        b->plans.assign(plans, plans + nbeams);
        b->in_off.assign(size_t(nbeams), 0);
        b->out_off.assign(size_t(nbeams), 0);
        b->ws_off.assign(size_t(nbeams), 0);
        size_t in = 0, out = 0, ws = kBatchCounterBytes;
        size_t lds = 0;
        for (int32_t i = 0; i < nbeams; ++i) {
            const Plan *p = plans[i];
            if (!p) {
                *err = "plan " + std::to_string(i) + " is NULL";
                return DD_ERR_NULL;
            }
            if (p->dtype != DD_U8) {
                *err = "batches hold DD_U8 plans only";
                return DD_ERR_DTYPE;
            }
            if (p->subband) {
                *err = "batches hold variant 1 or 2 plans (variant 3 runs per plan)";
                return DD_ERR_INVALID;
            }
            b->in_off[i] = int64_t(in);
            in = align_up(in + size_t(p->nchans) * size_t(p->nsamp), 256);
            b->out_off[i] = int64_t(out);
            out = align_up(out + size_t(p->out_elems), 64);
            b->ws_off[i] = ws;
            ws = align_up(ws + p->ws_bytes, 256);
            lds = std::max(lds, p->lds_bytes);
            if (i == 0) {
                b->dedup = p->dedup;
                b->waves = p->waves;
            } else if (p->waves != b->waves) {
                *err = "all plans of a batch need the same DM tile";
                return DD_ERR_INVALID;
            }
        }
        b->in_bytes = int64_t(in);
        b->out_elems = int64_t(out);
        b->ws_bytes = ws;
        b->lds_bytes = lds;
        // Work items: every (beam, range) contributes time tiles x DM tiles
        // items of equal shape whose cost grows with the beam's channels.
        b->descs.clear();
        for (int32_t i = 0; i < nbeams; ++i)
            for (int32_t r = 0; r < int32_t(plans[i]->ranges.size()); ++r) {
                BatchDescHost d;
                d.beam = i;
                d.range = r;
                d.nitems = plans[i]->ranges[r].ntime_tiles * plans[i]->ranges[r].ndm_tiles;
                b->descs.push_back(d);
            }
        std::stable_sort(b->descs.begin(), b->descs.end(),
                         [&](const BatchDescHost &x, const BatchDescHost &y) {
                             return plans[x.beam]->nchans > plans[y.beam]->nchans;
                         });
        int64_t n = 0;
        for (BatchDescHost &d : b->descs) {
            d.item_start = n;
            n += d.nitems;
        }
        b->nitems = n;
    } catch (const std::bad_alloc &) {
        *err = "host allocation failed";
        return DD_ERR_NOMEM;
    }
    return DD_OK;
}

dd_status build_stream(const Plan *plan, int32_t time_major, Stream *s, std::string *err)
{
    if (!plan) {
        *err = "plan must not be NULL";
        return DD_ERR_NULL;
    }
    if (time_major != 0 && time_major != 1) {
        *err = "time_major must be 0 or 1";
        return DD_ERR_INVALID;
    }
    int64_t lcm = 1;
    int64_t limit = plan->nsamp;
    for (const RangeInfo &ri : plan->ranges) {
        int64_t a = lcm, b = ri.ds;
        while (b) {
            const int64_t t = a % b;
            a = b;
            b = t;
        }
        lcm = lcm / a * ri.ds;
        limit = std::min(limit, int64_t(ri.ds) * ri.nout);
    }
    const int64_t step = limit / lcm * lcm;
    if (step <= 0 || 2 * step < plan->nsamp) {
        *err = "chunk too short for streaming: need a step >= nsamp/2 that every downsample divides";
        return DD_ERR_INVALID;
    }
    s->plan = plan;
    s->time_major = time_major;
    s->step = step;
    s->overlap = plan->nsamp - step;
    s->chunks = 0;
    return DD_OK;
}

}  // namespace dd
