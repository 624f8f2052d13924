// Host core of the batched forward: buffer layout of the beams, the kernel
// groups, and the order of each group's work items (most expensive first,
// so the queues, or the float32 launch's workgroups, drain evenly).  Plain
// C++, no HIP.
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
        b->dtype = plans[0] ? plans[0]->dtype : DD_U8;
        b->w_off.assign(size_t(nbeams), 0);
        b->in_off.assign(size_t(nbeams), 0);
        b->out_off.assign(size_t(nbeams), 0);
        b->ws_off.assign(size_t(nbeams), 0);
        b->groups.clear();
        std::vector<int32_t> group_of(size_t(nbeams), 0);
        size_t in = 0, out = 0, ws = kBatchCounterBytes;
        int64_t wn = 0;
        for (int32_t i = 0; i < nbeams; ++i) {
            const Plan *p = plans[i];
            if (!p) {
                *err = "plan " + std::to_string(i) + " is NULL";
                return DD_ERR_NULL;
            }
            if (p->dtype != b->dtype) {
                *err = "the plans of a batch share one dtype (plan " + std::to_string(i) +
                       " differs from plan 0)";
                return DD_ERR_DTYPE;
            }
            const bool f32 = p->dtype == DD_F32;
            b->in_off[i] = int64_t(in);
            in = align_up(in + size_t(p->nchans) * size_t(p->nsamp) * (f32 ? sizeof(float) : 1), 256);
            b->out_off[i] = int64_t(out);
            out = align_up(out + size_t(p->out_elems), 64);
            b->w_off[i] = wn;
            wn += p->nchans;
            // a beam's part of the workspace: what its forward uses
            b->ws_off[i] = ws;
            ws = align_up(ws + p->fwd_ws_bytes, 256);
            // plans that run the same kernel share a group (one launch); all
            // float32 plans run the generic shift-and-sum
            int32_t g = 0;
            while (g < int32_t(b->groups.size()) &&
                   !(f32 ? b->groups[g].f32
                         : (!b->groups[g].f32 && b->groups[g].subband == p->subband &&
                            b->groups[g].dedup == p->dedup && b->groups[g].dm_tile == p->dm_tile &&
                            b->groups[g].time_tile == p->time_tile)))
                ++g;
            if (g == int32_t(b->groups.size())) {
                if (g == kBatchMaxGroups) {
                    *err = "a batch runs at most " + std::to_string(kBatchMaxGroups) +
                           " kernels (variant, DM tile, time tile)";
                    return DD_ERR_INVALID;
                }
                BatchGroup G;
                G.f32 = f32;
                G.subband = p->subband;
                G.dedup = p->dedup;
                G.dm_tile = p->dm_tile;
                G.time_tile = p->time_tile;
                G.waves = p->waves;
                b->groups.push_back(G);
            }
            b->groups[g].lds_bytes = std::max(b->groups[g].lds_bytes, p->lds_bytes);
            group_of[size_t(i)] = g;
        }
        b->in_bytes = int64_t(in);
        b->out_elems = int64_t(out);
        b->w_elems = wn;
        b->ws_bytes = ws;
        // float32: the boxcar calls' part of the workspace
        b->gpad_off.assign(size_t(nbeams), std::vector<size_t>());
        b->dwp_off.assign(size_t(nbeams), 0);
        b->box_fused = b->dtype == DD_F32;
        b->loss_blocks = 0;
        if (b->dtype == DD_F32) {
            for (int32_t i = 0; i < nbeams; ++i) {
                const Plan *p = plans[i];
                for (const RangeInfo &ri : p->ranges) {
                    b->gpad_off[size_t(i)].push_back(ws);
                    ws = align_up(ws + size_t(ri.ndms) * size_t(ri.gpitch) * sizeof(float), 256);
                    b->loss_blocks += (ri.nout + kBoxLossStride - 1) / kBoxLossStride * ri.fwd.nout_tiles;
                }
                b->dwp_off[size_t(i)] = ws;
                ws = align_up(ws + size_t(p->nchans) * size_t(std::max(p->dw_tiles, 1)) * sizeof(float), 256);
                b->box_fused = b->box_fused && p->adj_fused;
            }
            b->loss_part_off = ws;
            ws = align_up(ws + size_t(b->loss_blocks) * sizeof(float), 256);
        }
        b->box_ws_bytes = ws;
        // Work items: every (beam, range) contributes time tiles x DM tiles
        // items of equal shape whose cost grows with the beam's channels.
        b->descs.clear();
        b->nitems = 0;
        for (size_t g = 0; g < b->groups.size(); ++g) {
            BatchGroup &G = b->groups[g];
            G.desc_begin = b->descs.size();
            for (int32_t i = 0; i < nbeams; ++i) {
                if (group_of[size_t(i)] != int32_t(g))
                    continue;
                for (int32_t r = 0; r < int32_t(plans[i]->ranges.size()); ++r) {
                    BatchDescHost d;
                    d.beam = i;
                    d.range = r;
                    const RangeInfo &ri = plans[i]->ranges[r];
                    // float32: the forward problem's workgroups (time tiles x
                    // output tiles); integer: time tiles x DM tiles
                    d.nitems = G.f32 ? ri.fwd.ntime_tiles * ri.fwd.nout_tiles
                                     : ri.ntime_tiles * ri.ndm_tiles;
                    b->descs.push_back(d);
                }
            }
            G.desc_end = b->descs.size();
            std::stable_sort(b->descs.begin() + G.desc_begin, b->descs.end(),
                             [&](const BatchDescHost &x, const BatchDescHost &y) {
                                 return plans[x.beam]->nchans > plans[y.beam]->nchans;
                             });
            // an item's cost: its channels plus a fixed part (staging of
            // the first stage, tables, output stores) worth kItemOverheadChans
            // channels, as the batch's kernels measure on beams of 1024 to
            // 4096 channels
            auto weight = [&](const BatchDescHost &d) {
                return double(plans[d.beam]->nchans) + kItemOverheadChans;
            };
            int64_t n = 0;
            double total = 0.0;
            for (size_t k = G.desc_begin; k < G.desc_end; ++k) {
                BatchDescHost &d = b->descs[k];
                d.item_start = n;
                n += d.nitems;
                total += double(d.nitems) * weight(d);
            }
            G.nitems = n;
            b->nitems += n;
            // Queue x starts at the first item whose preceding cost reaches
            // x/8 of the group's total: contiguous slices (neighbouring tiles
            // share an XCD's L2) of equal cost, whatever the mix of channel
            // counts.  (A workgroup whose queue is empty takes items from the
            // other queues, so an estimate off by a little costs only the
            // L2 locality of the items it takes.)
            G.queue_bounds[0] = 0;
            double before = 0.0;
            int q = 1;
            for (size_t k = G.desc_begin; k < G.desc_end; ++k) {
                const BatchDescHost &d = b->descs[k];
                const double w = weight(d);
                while (q < kBatchQueues &&
                       before + double(d.nitems) * w >= total * q / kBatchQueues) {
                    const double need = total * q / kBatchQueues - before;
                    const int64_t m = std::min<int64_t>(
                        d.nitems, std::max<int64_t>(0, int64_t(std::ceil(need / w))));
                    G.queue_bounds[q++] = d.item_start + m;
                }
                before += double(d.nitems) * w;
            }
            while (q <= kBatchQueues)
                G.queue_bounds[q++] = n;
        }
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
