// Host-only entry points of the C ABI: plan creation and queries, status
// text and the per-thread error detail (paper, "API Structure": immutable
// plans whose strategy fields the user may query, with error feedback).
#include <cstring>
#include <new>
#include <string>

#include "plan.h"

namespace dd {
const char *last_error();
}

using dd::clear_error;
using dd::set_error;

extern "C" {

dd_status dd_plan_create(const double *freqs_mhz, int32_t nchans, double tsamp_s, int64_t nsamp,
                         const dd_range *ranges, int32_t nranges, dd_dtype dtype, dd_plan **out)
{
    return dd_plan_create_ex(freqs_mhz, nchans, tsamp_s, nsamp, ranges, nranges, dtype, nullptr,
                             out);
}

dd_status dd_plan_create_ex(const double *freqs_mhz, int32_t nchans, double tsamp_s,
                            int64_t nsamp, const dd_range *ranges, int32_t nranges,
                            dd_dtype dtype, const dd_options *options, dd_plan **out)
{
    clear_error();
    if (!out) {
        set_error("out must not be NULL");
        return DD_ERR_NULL;
    }
    *out = nullptr;
    dd_plan *pl = new (std::nothrow) dd_plan;
    if (!pl) {
        set_error("host allocation failed");
        return DD_ERR_NOMEM;
    }
    std::string err;
    dd_status st;
    try {
        st = dd::build_plan(freqs_mhz, nchans, tsamp_s, nsamp, ranges, nranges, dtype, options,
                            &pl->p, &err);
    } catch (...) {
        st = DD_ERR_NOMEM;
        err = "unexpected host failure while building the plan";
    }
    if (st == DD_OK) {
        pl->p.device = dd::new_device_state();
        if (!pl->p.device) {
            st = DD_ERR_NOMEM;
            err = "host allocation failed";
        }
    }
    if (st != DD_OK) {
        delete pl;
        set_error(err);
        return st;
    }
    *out = pl;
    return DD_OK;
}

dd_status dd_plan_info(const dd_plan *plan, int32_t *ndms_total, int64_t *out_elems,
                       int64_t *overlap_samples)
{
    clear_error();
    if (!plan) {
        set_error("plan must not be NULL");
        return DD_ERR_NULL;
    }
    if (ndms_total)
        *ndms_total = int32_t(plan->p.dms.size());
    if (out_elems)
        *out_elems = plan->p.out_elems;
    if (overlap_samples)
        *overlap_samples = plan->p.overlap;
    return DD_OK;
}

dd_status dd_plan_nranges(const dd_plan *plan, int32_t *nranges)
{
    clear_error();
    if (!plan || !nranges) {
        set_error("plan and nranges must not be NULL");
        return DD_ERR_NULL;
    }
    *nranges = int32_t(plan->p.ranges.size());
    return DD_OK;
}

dd_status dd_plan_range(const dd_plan *plan, int32_t r, int32_t *ndms, int64_t *nout,
                        int64_t *out_offset, int32_t *max_shift, int32_t *downsample)
{
    clear_error();
    if (!plan) {
        set_error("plan must not be NULL");
        return DD_ERR_NULL;
    }
    if (r < 0 || r >= int32_t(plan->p.ranges.size())) {
        set_error("range index out of bounds");
        return DD_ERR_INVALID;
    }
    const dd::RangeInfo &ri = plan->p.ranges[r];
    if (ndms)
        *ndms = ri.ndms;
    if (nout)
        *nout = ri.nout;
    if (out_offset)
        *out_offset = ri.out_offset;
    if (max_shift)
        *max_shift = ri.max_shift;
    if (downsample)
        *downsample = ri.ds;
    return DD_OK;
}

dd_status dd_plan_dms(const dd_plan *plan, double *dms_out)
{
    clear_error();
    if (!plan || !dms_out) {
        set_error("plan and dms_out must not be NULL");
        return DD_ERR_NULL;
    }
    std::memcpy(dms_out, plan->p.dms.data(), plan->p.dms.size() * sizeof(double));
    return DD_OK;
}

dd_status dd_plan_shifts(const dd_plan *plan, int32_t *shifts_out)
{
    clear_error();
    if (!plan || !shifts_out) {
        set_error("plan and shifts_out must not be NULL");
        return DD_ERR_NULL;
    }
    std::memcpy(shifts_out, plan->p.shifts.data(), plan->p.shifts.size() * sizeof(int32_t));
    return DD_OK;
}

dd_status dd_plan_strategy(const dd_plan *plan, int32_t *time_tile, int32_t *dm_tile,
                           int32_t *chans_stage, int64_t *workgroups, int32_t *variant)
{
    clear_error();
    if (!plan) {
        set_error("plan must not be NULL");
        return DD_ERR_NULL;
    }
    const bool f32 = plan->p.dtype == DD_F32;
    int32_t st = 0;
    for (const dd::RangeInfo &ri : plan->p.ranges) {
        const int32_t c = f32 ? ri.fwd.stage_rows : ri.stage_chans;
        st = c > st ? c : st;
    }
    if (time_tile)
        *time_tile = f32 ? dd::kF32TimeTile : plan->p.time_tile;
    if (dm_tile)
        *dm_tile = f32 ? dd::kF32OutTile : plan->p.dm_tile;
    if (variant)
        *variant = plan->p.subband ? 3 : plan->p.dedup ? 2 : 1;
    if (chans_stage)
        *chans_stage = st;
    if (workgroups)
        *workgroups = plan->p.blocks;
    return DD_OK;
}

dd_status dd_workspace_bytes(const dd_plan *plan, size_t *bytes)
{
    clear_error();
    if (!plan || !bytes) {
        set_error("plan and bytes must not be NULL");
        return DD_ERR_NULL;
    }
    *bytes = plan->p.ws_bytes;
    return DD_OK;
}

dd_status dd_batch_create(const dd_plan *const *plans, int32_t nbeams, dd_batch **out)
{
    clear_error();
    if (!out) {
        set_error("out must not be NULL");
        return DD_ERR_NULL;
    }
    *out = nullptr;
    if (!plans) {
        set_error("plans must not be NULL");
        return DD_ERR_NULL;
    }
    dd_batch *bt = new (std::nothrow) dd_batch;
    if (!bt) {
        set_error("host allocation failed");
        return DD_ERR_NOMEM;
    }
    std::vector<const dd::Plan *> ps;
    dd_status st = DD_OK;
    std::string err;
    try {
        for (int32_t i = 0; i < nbeams; ++i)
            ps.push_back(plans[i] ? &plans[i]->p : nullptr);
        st = dd::build_batch(ps.data(), nbeams, &bt->b, &err);
        if (st == DD_OK) {
            bt->b.device = dd::new_batch_device_state();
            if (!bt->b.device) {
                st = DD_ERR_NOMEM;
                err = "host allocation failed";
            }
        }
    } catch (...) {
        st = DD_ERR_NOMEM;
        err = "host allocation failed";
    }
    if (st != DD_OK) {
        delete bt;
        set_error(err);
        return st;
    }
    *out = bt;
    return DD_OK;
}

dd_status dd_batch_info(const dd_batch *batch, int64_t *in_bytes, int64_t *out_elems,
                        size_t *ws_bytes, int64_t *work_items)
{
    clear_error();
    if (!batch) {
        set_error("batch must not be NULL");
        return DD_ERR_NULL;
    }
    if (in_bytes)
        *in_bytes = batch->b.in_bytes;
    if (out_elems)
        *out_elems = batch->b.out_elems;
    if (ws_bytes)
        *ws_bytes = batch->b.ws_bytes;
    if (work_items)
        *work_items = batch->b.nitems;
    return DD_OK;
}

dd_status dd_batch_groups(const dd_batch *batch, int32_t *ngroups)
{
    clear_error();
    if (!batch || !ngroups) {
        set_error("batch and ngroups must not be NULL");
        return DD_ERR_NULL;
    }
    *ngroups = int32_t(batch->b.groups.size());
    return DD_OK;
}

dd_status dd_batch_group(const dd_batch *batch, int32_t g, int32_t *variant, int32_t *dm_tile,
                         int64_t *work_items, int64_t *queue_bounds)
{
    clear_error();
    if (!batch) {
        set_error("batch must not be NULL");
        return DD_ERR_NULL;
    }
    if (g < 0 || g >= int32_t(batch->b.groups.size())) {
        set_error("group index out of bounds");
        return DD_ERR_INVALID;
    }
    const dd::BatchGroup &G = batch->b.groups[size_t(g)];
    if (variant)
        *variant = G.f32 ? 0 : G.subband ? 3 : (G.dedup ? 2 : 1);
    if (dm_tile)
        *dm_tile = G.f32 ? dd::kF32OutTile : G.dm_tile;
    if (work_items)
        *work_items = G.nitems;
    if (queue_bounds)
        for (int i = 0; i <= dd::kBatchQueues; ++i)
            queue_bounds[i] = G.queue_bounds[i];
    return DD_OK;
}

dd_status dd_batch_beam(const dd_batch *batch, int32_t beam, int64_t *in_offset,
                        int64_t *out_offset)
{
    clear_error();
    if (!batch) {
        set_error("batch must not be NULL");
        return DD_ERR_NULL;
    }
    if (beam < 0 || beam >= int32_t(batch->b.plans.size())) {
        set_error("beam index out of bounds");
        return DD_ERR_INVALID;
    }
    if (in_offset)
        *in_offset = batch->b.in_off[beam];
    if (out_offset)
        *out_offset = batch->b.out_off[beam];
    return DD_OK;
}

dd_status dd_stream_create(const dd_plan *plan, int32_t time_major, dd_stream **out)
{
    clear_error();
    if (!out || !plan) {
        set_error("plan and out must not be NULL");
        return DD_ERR_NULL;
    }
    *out = nullptr;
    dd_stream *st = new (std::nothrow) dd_stream;
    if (!st) {
        set_error("host allocation failed");
        return DD_ERR_NOMEM;
    }
    std::string err;
    const dd_status rc = dd::build_stream(&plan->p, time_major, &st->s, &err);
    st->s.handle = plan;
    if (rc != DD_OK) {
        delete st;
        set_error(err);
        return rc;
    }
    *out = st;
    return DD_OK;
}

void dd_stream_destroy(dd_stream *stream) { delete stream; }

dd_status dd_stream_info(const dd_stream *stream, int64_t *first, int64_t *step)
{
    clear_error();
    if (!stream) {
        set_error("stream must not be NULL");
        return DD_ERR_NULL;
    }
    if (first)
        *first = stream->s.plan->nsamp;
    if (step)
        *step = stream->s.step;
    return DD_OK;
}

dd_status dd_stream_reset(dd_stream *stream)
{
    clear_error();
    if (!stream) {
        set_error("stream must not be NULL");
        return DD_ERR_NULL;
    }
    stream->s.chunks = 0;
    return DD_OK;
}

const char *dd_status_str(dd_status status)
{
    switch (status) {
    case DD_OK: return "DD_OK";
    case DD_ERR_NULL: return "DD_ERR_NULL: a required pointer is NULL";
    case DD_ERR_INVALID: return "DD_ERR_INVALID: an argument is out of its domain";
    case DD_ERR_EMPTY_OUTPUT: return "DD_ERR_EMPTY_OUTPUT: a range has no valid output sample";
    case DD_ERR_OVERFLOW: return "DD_ERR_OVERFLOW: uint8 sums could overflow int32";
    case DD_ERR_CAPACITY: return "DD_ERR_CAPACITY: output buffer too small";
    case DD_ERR_DTYPE: return "DD_ERR_DTYPE: call does not apply to the plan's data type";
    case DD_ERR_HIP: return "DD_ERR_HIP: HIP runtime failure";
    case DD_ERR_NOMEM: return "DD_ERR_NOMEM: allocation failed";
    case DD_ERR_WORKSPACE: return "DD_ERR_WORKSPACE: workspace too small";
    }
    return "unknown dd_status";
}

const char *dd_last_error(void) { return dd::last_error(); }

}  // extern "C"
