// Host core of the batched integer forward: buffer layout of the beams and
// the order of the persistent launch's work items (most expensive first, so
// the queue drains evenly).  Plain C++, no HIP.
#include <algorithm>
#include <cmath>
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
            b->in_off[i] = int64_t(in);
            in = align_up(in + size_t(p->nchans) * size_t(p->nsamp), 256);
            b->out_off[i] = int64_t(out);
            out = align_up(out + size_t(p->out_elems), 64);
            b->ws_off[i] = ws;
            ws = align_up(ws + p->ws_bytes, 256);
            lds = std::max(lds, p->lds_bytes);
            if (i == 0) {
                b->dedup = p->dedup;
                b->subband = p->subband;
                b->waves = p->waves;
                b->dm_tile = p->dm_tile;
            } else if (p->subband != b->subband || p->dm_tile != b->dm_tile ||
                       p->waves != b->waves) {
                *err = "all plans of a batch need the same kernel variant family (1/2 or 3) "
                       "and DM tile";
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
        double total = 0.0;
        for (BatchDescHost &d : b->descs) {
            d.item_start = n;
            n += d.nitems;
            total += double(d.nitems) * plans[d.beam]->nchans;
        }
        b->nitems = n;
        // Queue x starts at the first item whose preceding cost reaches
        // x/8 of the total: contiguous slices (neighbouring tiles share an
        // XCD's L2) of equal cost, whatever the mix of channel counts.
        b->queue_bounds[0] = 0;
        double before = 0.0;
        int q = 1;
        for (const BatchDescHost &d : b->descs) {
            const double w = plans[d.beam]->nchans;
            while (q < kBatchQueues && before + double(d.nitems) * w >= total * q / kBatchQueues) {
                const double need = total * q / kBatchQueues - before;
                const int64_t k = std::min<int64_t>(
                    d.nitems, std::max<int64_t>(0, int64_t(std::ceil(need / w))));
                b->queue_bounds[q++] = d.item_start + k;
            }
            before += double(d.nitems) * w;
        }
        while (q <= kBatchQueues)
            b->queue_bounds[q++] = n;
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
