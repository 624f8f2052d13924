/*
 * dd.h -- C ABI of the MI355X (gfx950) brute-force incoherent dedispersion
 * library.
 *
 * What is computed.  The paper names dedispersion as the first GPU analysis
 * module of the pipeline (Introduction) without printing its formula; this
 * library implements the standard brute-force incoherent operator:
 *   - a DM plan is a list of ranges; range r holds the trial DMs
 *     lo + i*step for i < round((hi - lo)/step)   (half-open [lo, hi));
 *   - channel c is delayed by
 *       s[d][c] = floor(K*DM_d*(f_c^-2 - f_ref^-2)/(tsamp*ds_r) + 1/2)
 *     samples of the range's binned series, K = 4.148808e3 s MHz^2 pc^-1
 *     cm^3, f_ref = the highest channel frequency (so every s >= 0); the
 *     table is computed once per plan in FP64 on the host;
 *   - a range with downsample ds_r > 1 works on the series binned by summing
 *     ds_r adjacent samples (bin 0 = samples [0, ds_r), partial bin dropped);
 *   - out_r[d][t] = sum_c w_c * x_r[c][t + s[d][c]] for the valid samples
 *     t < nout_r = floor(nsamp/ds_r) - max_{d in r, c} s[d][c];
 *   - the output holds the ranges in plan order, each DM-major
 *     [ndms_r][nout_r], starting at element out_offset_r.
 *
 * API shape (paper, "API Structure"): the caller describes the search in an
 * immutable plan; the library derives the GPU strategy from it (tile
 * shapes, workspace size) and exposes both for query; every call returns a
 * status code, and a failing call leaves the plan valid (paper, "Plan and
 * strategy" and "Pipeline").  Memory (paper, "Memory management", "Memory
 * ownership"): the caller asks how much workspace a plan needs before
 * allocating it; the caller owns the input (never modified), the output and
 * the workspace; the plan owns its host tables and its device copy of the
 * shift table, freed by dd_plan_destroy.  Unlike the paper's results
 * buffers, the output buffer here belongs to the caller.
 *
 * Pointers named d_* are device pointers on the current HIP device; all
 * other pointers are host pointers.  `stream` is a hipStream_t passed as
 * void* (NULL = the default stream).  Device work is enqueued asynchronously
 * on that stream; argument errors are reported synchronously, before
 * anything is enqueued.  Asynchronous device faults surface at the caller's
 * next synchronisation, as for any HIP launch.
 *
 * Thread safety: a plan is immutable after creation; calls on one plan
 * from several host threads or streams are safe as long as each in-flight
 * call has its own output and workspace.  dd_last_error() is per thread.
 */
#ifndef DD_MI355X_H
#define DD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (paper, "Pipeline": success or error per call). */
typedef enum {
    DD_OK = 0,
    DD_ERR_NULL = -1,          /* a required pointer is NULL */
    DD_ERR_INVALID = -2,       /* a value is out of its domain (see each call) */
    DD_ERR_EMPTY_OUTPUT = -3,  /* a range has nout_r <= 0: delays exceed the data */
    DD_ERR_OVERFLOW = -4,      /* uint8 sums could exceed int32: 255*nchans*ds >= 2^31 */
    DD_ERR_CAPACITY = -5,      /* output buffer smaller than dd_plan_info's out_elems */
    DD_ERR_DTYPE = -6,         /* the call does not apply to the plan's data type */
    DD_ERR_HIP = -7,           /* a HIP runtime call or launch failed */
    DD_ERR_NOMEM = -8,         /* host or device allocation failed */
    DD_ERR_WORKSPACE = -9      /* workspace smaller than dd_workspace_bytes */
} dd_status;

/* Input sample type.  DD_U8 input gives int32 output (exact sums);
 * DD_F32 input gives float32 output and accepts per-channel weights. */
typedef enum { DD_U8 = 0, DD_F32 = 1 } dd_dtype;

/* One DM range, half-open [dm_lo, dm_hi) with step dm_step (pc cm^-3), and
 * its time downsampling factor (1 = native resolution). */
typedef struct {
    double dm_lo;
    double dm_hi;
    double dm_step;
    int32_t downsample;
} dd_range;

/* Opaque, immutable plan. */
typedef struct dd_plan dd_plan;

/* Largest number of ranges one plan may hold. */
#define DD_MAX_RANGES 16

/*
 * Create a plan (paper, "Design of the API": one plan per module, strategy
 * derived by the library).  Host-only: it validates the arguments, expands
 * the DM ranges, computes the FP64 shift table, the per-range output sizes
 * and offsets, the workspace size and the tile strategy.  No device memory
 * is touched until dd_plan_prepare or the first compute call.
 *
 *   freqs_mhz  [nchans] channel centre frequencies in MHz, any order, all
 *              finite and > 0 (copied).
 *   tsamp_s    native sampling time in seconds, finite and > 0.
 *   nsamp      samples per channel of the input, > 0.
 *   ranges     [nranges] DM ranges (copied); 1 <= nranges <= DD_MAX_RANGES;
 *              each needs finite dm_lo >= 0, dm_hi > dm_lo, dm_step > 0,
 *              round((dm_hi - dm_lo)/dm_step) >= 1 and downsample >= 1
 *              (<= 256 for DD_U8, so a binned sample fits 16 bits).
 *   dtype      DD_U8 or DD_F32.
 *   out        receives the plan; set to NULL on failure.
 *
 * Errors: DD_ERR_NULL, DD_ERR_INVALID, DD_ERR_EMPTY_OUTPUT (a range whose
 * largest delay leaves no valid sample), DD_ERR_OVERFLOW (DD_U8 only),
 * DD_ERR_NOMEM.
 */
dd_status dd_plan_create(const double *freqs_mhz, int32_t nchans, double tsamp_s,
                         int64_t nsamp, const dd_range *ranges, int32_t nranges,
                         dd_dtype dtype, dd_plan **out);

/*
 * Strategy options for dd_plan_create_ex (paper, "Plan and strategy": the
 * strategy is configured once, then immutable).  Zero means "library
 * default" for every field.
 *   variant      DD_U8 shift-and-sum kernel: 1 = read a channel's words
 *                for every DM, 2 = re-read them only when the DM's delay
 *                differs from the previous DM's, 3 = exact sub-band reuse:
 *                DMs of a DM tile whose delays over a sub-band of 8
 *                channels differ from their smallest by the same pattern
 *                share that sub-band's partial sum (the same integer
 *                result; DD_ERR_INVALID when the patterns of a plan do not
 *                fit the LDS).  0 (the default) = variant 3 at the
 *                requested DM tile, or at 192 and then 128 when none is
 *                requested, if the patterns fit and a DM tile holds at
 *                most one distinct pattern per four DMs and sub-band
 *                (weighted over the ranges; denser plans run faster on the
 *                direct sum); variant 1 otherwise (at DM tile 32 when
 *                requested, else 64).  dd_plan_strategy reports the
 *                choice.
 *   stage_chans  channels staged in LDS at once (rounded down to even,
 *                or to a multiple of the sub-band for variant 3, and
 *                clamped to what the LDS and, for DD_U8, the exact 16-bit
 *                partial sums allow).
 *   dm_tile      DD_U8 trial DMs per workgroup: 32 (4 wavefronts) or 64 (8)
 *                for variants 1 and 2 (default 64); for variant 3, 192 (the
 *                default) or 128 (16 wavefronts), or 96 or 64 (8
 *                wavefronts); any of these for variant 0.
 *   time_tile    DD_U8 output samples per workgroup: 256 or 512 for variants
 *                1 and 2 (default 512, or 256 when 512-sample tiles would
 *                give the plan fewer than 512 workgroups) and for variant 3
 *                at DM tiles 96 and 64 (default 512); 256 only for variant 3
 *                at DM tiles 192 and 128.  DD_ERR_INVALID for other values.
 */
typedef struct {
    int32_t variant;
    int32_t stage_chans;
    int32_t dm_tile;
    int32_t time_tile;
} dd_options;

dd_status dd_plan_create_ex(const double *freqs_mhz, int32_t nchans, double tsamp_s,
                            int64_t nsamp, const dd_range *ranges, int32_t nranges,
                            dd_dtype dtype, const dd_options *options, dd_plan **out);

/* Release the plan, its host tables and every device copy it made.
 * NULL-safe.  No call on the plan may be in flight on any stream. */
void dd_plan_destroy(dd_plan *plan);

/*
 * Whole-plan sizes (paper, "Plan and strategy": the user may query the
 * strategy).  Any output pointer may be NULL.
 *   ndms_total       number of trial DMs over all ranges
 *   out_elems        output elements over all ranges (sum ndms_r*nout_r)
 *   overlap_samples  largest delay in native samples, max_r(ds_r*max shift):
 *                    the overlap a streaming run must keep between chunks
 */
dd_status dd_plan_info(const dd_plan *plan, int32_t *ndms_total, int64_t *out_elems,
                       int64_t *overlap_samples);

/*
 * Sizes of range r (paper, "Plan and strategy": the user may query the
 * configured plan and strategy).  0 <= r < nranges, else DD_ERR_INVALID;
 * DD_ERR_NULL for a NULL plan.  Any output pointer may be NULL.
 *   ndms        trial DMs of the range
 *   nout        valid output samples per DM (binned samples)
 *   out_offset  first output element of the range, in elements
 *   max_shift   largest delay of the range, in binned samples
 *   downsample  the range's ds_r
 */
dd_status dd_plan_range(const dd_plan *plan, int32_t r, int32_t *ndms, int64_t *nout,
                        int64_t *out_offset, int32_t *max_shift, int32_t *downsample);

/* Number of ranges of the plan. */
dd_status dd_plan_nranges(const dd_plan *plan, int32_t *nranges);

/* Copy the trial DMs the plan expanded (paper, "Plan and strategy": the
 * configured plan may be queried): dms_out is a caller-owned host array of
 * [ndms_total] doubles, filled with lo + i*step per range, ranges in plan
 * order.  DD_ERR_NULL for a NULL argument. */
dd_status dd_plan_dms(const dd_plan *plan, double *dms_out);

/* Copy the plan's FP64-derived shift table (paper, "Plan and strategy": the
 * configured plan may be queried): shifts_out is a caller-owned host array
 * of [ndms_total][nchans] int32, DM-major, each entry in binned samples of
 * its DM's range.  DD_ERR_NULL for a NULL argument. */
dd_status dd_plan_shifts(const dd_plan *plan, int32_t *shifts_out);

/*
 * Tile strategy the plan chose (paper, "Design of the API": the strategy
 * decides how input data are split and processed on the GPU).  Any output
 * pointer may be NULL.
 *   time_tile      output samples per workgroup
 *   dm_tile        trial DMs per workgroup
 *   chans_stage    largest number of channels staged in LDS at once
 *   workgroups     workgroups of one forward launch
 *   variant        kernel variant (see dd_options)
 */
dd_status dd_plan_strategy(const dd_plan *plan, int32_t *time_tile, int32_t *dm_tile,
                           int32_t *chans_stage, int64_t *workgroups, int32_t *variant);

/*
 * Device workspace a forward call needs, in bytes (paper, "Memory
 * management": modules request GPU memory before it is allocated).  For
 * DD_U8 it holds one 16-bit copy of the input per distinct downsample of
 * the plan (1 included): the samples, or the sums of ds adjacent samples,
 * in padded rows.  For DD_F32 it holds the weighted float32 copies and the
 * buffers of dd_adjoint.  The workspace passed to a compute call must be at least
 * this large and 256-byte aligned (DD_ERR_WORKSPACE otherwise).
 */
dd_status dd_workspace_bytes(const dd_plan *plan, size_t *bytes);

/*
 * Upload the plan's device tables to the current HIP device now (otherwise
 * the first compute call on a device does it).  Call it before capturing
 * compute calls in a HIP graph.  Errors: DD_ERR_NULL, DD_ERR_HIP,
 * DD_ERR_NOMEM.
 */
dd_status dd_plan_prepare(dd_plan *plan);

/*
 * Forward dedispersion of one filterbank: the dedispersion module of the
 * pipeline run on data already on the GPU (paper, Introduction: data are
 * dedispersed entirely on the GPU; "Design of the API": the run step of a
 * configured plan).
 *   d_in          [nchans][nsamp] channel-major, uint8 (DD_U8) or float32
 *                 (DD_F32); read only.
 *   d_weights     [nchans] float32 per-channel weights, DD_F32 only; NULL
 *                 means all ones.  Must be NULL for DD_U8 (else DD_ERR_DTYPE).
 *   d_out         int32 (DD_U8) or float32 (DD_F32), out_capacity elements;
 *                 elements [0, out_elems) are overwritten, the rest untouched.
 *   d_ws/ws_bytes workspace of at least dd_workspace_bytes bytes (contents
 *                 scratch; d_ws may be NULL when that size is 0).
 *   stream        hipStream_t as void*.
 * DD_U8 sums are exact in int32.  DD_F32 sums are formed in float32 in a
 * fixed, call-independent order (weights applied to each binned sample).
 * Errors: DD_ERR_NULL, DD_ERR_DTYPE, DD_ERR_CAPACITY, DD_ERR_WORKSPACE,
 * DD_ERR_HIP, DD_ERR_NOMEM.
 */
dd_status dd_forward(const dd_plan *plan, const void *d_in, const float *d_weights,
                     void *d_out, int64_t out_capacity, void *d_ws, size_t ws_bytes,
                     void *stream);

/*
 * The two steps of dd_forward, for callers that schedule or time them
 * separately:
 *   dd_forward_bin  writes into the workspace the copies of d_in the ranges
 *                   read: one per distinct downsample, binned by summing ds
 *                   samples (uint16 for DD_U8; float32 multiplied by
 *                   d_weights for DD_F32, NULL = ones).  Same argument rules
 *                   as dd_forward.
 *   dd_forward_sum  the shift-and-sum of every range into d_out, reading
 *                   only the workspace, which must hold what dd_forward_bin
 *                   wrote and be unchanged since.
 * dd_forward(...) is dd_forward_bin followed by dd_forward_sum on the same
 * stream.
 */
dd_status dd_forward_bin(const dd_plan *plan, const void *d_in, const float *d_weights,
                         void *d_ws, size_t ws_bytes, void *stream);
dd_status dd_forward_sum(const dd_plan *plan, void *d_out, int64_t out_capacity, void *d_ws,
                         size_t ws_bytes, void *stream);

/*
 * dd_forward for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * computes exactly what dd_forward computes (same kernels, same results) but
 * takes no workspace argument and calls no hipMalloc, hipFree or allocating
 * library routine: its workspace is a static device array of
 * DD_NOALLOC_WS_MAX bytes built into the library, one copy per GPU, held
 * until the process ends.  The caller still owns d_in, d_weights and d_out
 * (arguments as for dd_forward).
 *
 *   - The plan's tables must already be on the current device: call
 *     dd_plan_prepare on that device first (else DD_ERR_INVALID).
 *   - Plans whose forward needs more than DD_NOALLOC_WS_MAX bytes of
 *     workspace (the binned copies of the input, reported for DD_U8 plans by
 *     dd_workspace_bytes) are rejected with DD_ERR_WORKSPACE; use dd_forward.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (the forward overwrites everything it reads).  Calls
 *     that overlap in time on one GPU (two streams, two host threads) race:
 *     order them on one stream or serialise them.
 * Errors: as dd_forward, plus the two above.
 */
#define DD_NOALLOC_WS_MAX (64u << 20)

dd_status dd_forward_noalloc(const dd_plan *plan, const void *d_in, const float *d_weights,
                             void *d_out, int64_t out_capacity, void *stream);

/*
 * Adjoint of the DD_F32 forward (the transpose of the linear map x -> out
 * for fixed weights, and its derivative in the weights), for the gradient
 * of a loss L given g = dL/dout:
 *   G_r[c][tau] = sum_{d in r, 0 <= tau - s[d][c] < nout_r} g_r[d][tau - s[d][c]]
 *   d_grad_in[c][t] = w_c * sum_r G_r[c][floor(t/ds_r)]  (t < ds_r*nbin_r terms)
 *   d_grad_w[c]     = sum_t x[c][t] * sum_r G_r[c][floor(t/ds_r)]
 *   d_grad_out  [out_elems] float32, the layout of dd_forward's output.
 *   d_in        [nchans][nsamp] float32 input of the forward (needed when
 *               d_grad_w is not NULL).
 *   d_weights   [nchans] or NULL (ones).
 *   d_grad_in   [nchans][nsamp] float32, overwritten; NULL to skip.
 *   d_grad_w    [nchans] float32, overwritten; NULL to skip.
 *   d_ws        workspace as for dd_forward (the adjoint uses its own part).
 * Sums are formed in float32 in a fixed order (the weight gradient by
 * fixed-shape tree reductions), so results do not depend on scheduling.
 * Errors: DD_ERR_NULL, DD_ERR_DTYPE (DD_U8 plan), DD_ERR_WORKSPACE,
 * DD_ERR_HIP, DD_ERR_NOMEM.
 */
dd_status dd_adjoint(const dd_plan *plan, const float *d_grad_out, const float *d_in,
                     const float *d_weights, float *d_grad_in, float *d_grad_w, void *d_ws,
                     size_t ws_bytes, void *stream);

/*
 * Boxcar loss of DD_F32 plans (the single-pulse search's boxcar filters,
 * paper Introduction, recast as a differentiable loss):
 *   L = sum_beams sum_r sum_d sum_{w = 1, 2, 4, ..., max_width}
 *       sum_{t = 0}^{nout_r - w} ( sum_{k < w} out_r[d][t + k] )^2
 * with out = dd_forward(x_beam, weights).  The dedispersed output is never
 * stored: dd_boxcar_loss forms the windows inside each output tile, and
 * dd_boxcar_backward recomputes each tile to form dL/dout (one beam at a
 * time, in the workspace) and runs the adjoint, so
 *   d_grad_in[beam] = dL/dx_beam    and    d_grad_w = sum_beams dL/dw.
 *   d_in        [nbeams][nchans][nsamp] float32.
 *   d_weights   [nchans] shared by all beams, or NULL (ones).
 *   max_width   a power of two in [1, 32].
 *   d_loss      one float32 on the device (overwritten).
 *   d_grad_in   [nbeams][nchans][nsamp] float32 or NULL; d_grad_w [nchans]
 *               float32 or NULL.
 *   d_ws        the plan's workspace (dd_workspace_bytes).
 * Sums are float32 in a fixed order.  Errors: DD_ERR_NULL, DD_ERR_DTYPE,
 * DD_ERR_INVALID (nbeams < 1, max_width), DD_ERR_WORKSPACE, DD_ERR_HIP.
 */
dd_status dd_boxcar_loss(const dd_plan *plan, const float *d_in, int32_t nbeams,
                         const float *d_weights, int32_t max_width, float *d_loss, void *d_ws,
                         size_t ws_bytes, void *stream);
dd_status dd_boxcar_backward(const dd_plan *plan, const float *d_in, int32_t nbeams,
                             const float *d_weights, int32_t max_width, float *d_grad_in,
                             float *d_grad_w, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Batches (paper, "Design of the API": a strategy decides how the input is
 * split and processed on the GPU; here many beams share one).  Integer
 * plans (beams of uneven channel counts, lengths and DM plans) are summed
 * by persistent launches -- ONE per kernel the plans use (variant family,
 * DM tile and time tile; usually one) -- that take their work items (beam,
 * range, time tile, DM tile), most expensive first, from queues in the
 * workspace.  Float32 plans are summed by ONE launch of the float32
 * shift-and-sum over every (beam, range) problem, whose workgroups run the
 * beams with most channels first (each beam's weighted levels are formed
 * beam by beam before it).  The launch sequence allocates nothing and
 * contains no memset, so it can be captured in a HIP graph (call
 * dd_batch_prepare first).  Results equal dd_forward of each plan bit for
 * bit (the float32 sums run in the same order).
 *
 * dd_batch_create   plans: [nbeams] plans of one dtype (borrowed: they
 *                   must outlive the batch).  Integer plans that run the
 *                   same kernel form one group; a group's work items are
 *                   dealt to one queue per XCD in contiguous slices of equal
 *                   cost (an item weighs its beam's channel count); float32
 *                   plans form one group.  Host-only.  Errors: DD_ERR_NULL,
 *                   DD_ERR_INVALID (nbeams < 1), DD_ERR_DTYPE (mixed
 *                   dtypes), DD_ERR_NOMEM.
 * dd_batch_info     in_bytes: size of the batch input buffer (each beam's
 *                   [nchans][nsamp] uint8 or float32 block at its
 *                   in_offset); out_elems: int32 (DD_U8) or float32
 *                   (DD_F32) elements of the batch output (each beam's
 *                   dd_forward layout at its out_offset); ws_bytes:
 *                   workspace; work_items: items (float32: workgroups) of
 *                   all its launches.  Any pointer may be NULL.
 * dd_batch_beam     byte offset of beam b's input and element offset of its
 *                   output (both 256-byte aligned).
 * dd_batch_groups   the number of kernel groups (one persistent launch each).
 * dd_batch_group    group g's kernel (variant 1, 2 or 3 and DM tile; for
 *                   the float32 group variant 0 and its 32-output tile), its
 *                   work items, and the bounds of its per-XCD queues:
 *                   queue x holds items [queue_bounds[x], queue_bounds[x+1])
 *                   of the group (queue_bounds: 9 int64, or NULL).  Any
 *                   other pointer may be NULL; DD_ERR_INVALID for g out of
 *                   range.
 * dd_batch_prepare  upload the batch's and its plans' device tables to the
 *                   current device.
 * dd_batch_forward  d_in: batch input (256-byte aligned); d_out: int32 or
 *                   float32, out_capacity elements; d_ws: workspace (256-byte
 *                   aligned, ws_bytes >= dd_batch_info's).  Calls that
 *                   overlap in time need distinct workspaces.  Float32
 *                   batches run with unit channel weights.
 * dd_batch_forward_weighted  as dd_batch_forward, for DD_F32 batches, with
 *                   d_weights: each beam's [nchans] float32 channel weights
 *                   in beam order, concatenated (sum of nchans floats),
 *                   or NULL for unit weights.  DD_ERR_DTYPE for an integer
 *                   batch with weights.
 *
 * Boxcar loss and its backward over a float32 batch (the loss of
 * dd_boxcar_loss, each beam with its own plan):
 * dd_batch_boxcar_workspace  bytes of the workspace these two calls need
 *                   (more than dd_batch_info's: the padded gradient rows and
 *                   the partials of every beam).  DD_ERR_DTYPE for an
 *                   integer batch.
 * dd_batch_boxcar_loss  the beams' levels, ONE loss launch over every (beam,
 *                   range), ONE reduction: d_loss[b] = beam b's loss.
 *                   d_in: the batch input; d_weights: each beam's weights
 *                   concatenated (as dd_batch_forward_weighted), or NULL.
 * dd_batch_boxcar_backward  its gradients, for plans with one range at full
 *                   resolution (else DD_ERR_INVALID): the beams' levels, ONE
 *                   launch zeroing the padding of the gradient rows, ONE
 *                   gradient launch writing dL/dout into them, ONE adjoint
 *                   launch forming dX and the weight-gradient partials, ONE
 *                   reduction.  d_grad_in: dL/dx in the batch input's layout
 *                   (float32 at each beam's in_offset), or NULL; d_grad_w:
 *                   each beam's dL/dw concatenated like the weights, or NULL.
 *                   Once dd_batch_prepare has run on the device, both
 *                   calls allocate nothing and contain no memset (graph
 *                   capture); before it, the first call on a device
 *                   uploads the batch's descriptors.
 */
typedef struct dd_batch dd_batch;

dd_status dd_batch_create(const dd_plan *const *plans, int32_t nbeams, dd_batch **out);
void dd_batch_destroy(dd_batch *batch);
dd_status dd_batch_info(const dd_batch *batch, int64_t *in_bytes, int64_t *out_elems,
                        size_t *ws_bytes, int64_t *work_items);
dd_status dd_batch_groups(const dd_batch *batch, int32_t *ngroups);
dd_status dd_batch_group(const dd_batch *batch, int32_t g, int32_t *variant, int32_t *dm_tile,
                         int64_t *work_items, int64_t *queue_bounds);
dd_status dd_batch_beam(const dd_batch *batch, int32_t beam, int64_t *in_offset,
                        int64_t *out_offset);
dd_status dd_batch_prepare(dd_batch *batch);
dd_status dd_batch_forward(const dd_batch *batch, const void *d_in, void *d_out,
                           int64_t out_capacity, void *d_ws, size_t ws_bytes, void *stream);
dd_status dd_batch_forward_weighted(const dd_batch *batch, const void *d_in, const float *d_weights,
                                    void *d_out, int64_t out_capacity, void *d_ws, size_t ws_bytes,
                                    void *stream);
dd_status dd_batch_boxcar_workspace(const dd_batch *batch, size_t *bytes);
dd_status dd_batch_boxcar_loss(const dd_batch *batch, const void *d_in, const float *d_weights,
                               int32_t max_width, float *d_loss, void *d_ws, size_t ws_bytes,
                               void *stream);
dd_status dd_batch_boxcar_backward(const dd_batch *batch, const void *d_in, const float *d_weights,
                                   int32_t max_width, float *d_grad_in, float *d_grad_w, void *d_ws,
                                   size_t ws_bytes, void *stream);

/*
 * Streaming (paper, "Pipeline": the pipeline walks the input in chunks and
 * reports a status per iteration).  A stream processes a long series in
 * chunks of the plan's nsamp samples that start `step` samples apart, where
 * step is the largest multiple of every range's downsample not above any
 * range's ds_r * nout_r (so nsamp - step is the plan's largest delay,
 * rounded up to that multiple).  The first step/ds_r output samples of each
 * DM row of chunk k are the one-shot output samples k*step/ds_r + [0,
 * step/ds_r) of the whole series: concatenated, the chunks reproduce a
 * single forward over the series exactly (bit for bit for DD_U8).
 *
 * dd_stream_create  plan: borrowed, must outlive the stream.  time_major: 0
 *                   when pushed blocks are channel-major [nchans][samples],
 *                   1 when they are time-major [samples][nchans] (SIGPROC
 *                   filterbank order; transposed on the device).  Host-only.
 *                   DD_ERR_INVALID when step < nsamp/2.
 * dd_stream_info    first: samples the first push must supply (nsamp);
 *                   step: samples every later push supplies.
 * dd_stream_push    d_block: the next `samples` samples of the series in the
 *                   stream's layout (device, read only).  d_chunk: the
 *                   caller-owned chunk buffer [nchans][nsamp] of the plan's
 *                   input type, kept between pushes (it carries the
 *                   overlap).  Then runs dd_forward on the chunk into d_out
 *                   (d_weights, d_ws as for dd_forward).  *chunk_index (may
 *                   be NULL) receives the chunk's index.  DD_ERR_INVALID if
 *                   samples is not `first` (first push) or `step` (later).
 * dd_stream_reset   the next push is a first push again.
 */
typedef struct dd_stream dd_stream;

dd_status dd_stream_create(const dd_plan *plan, int32_t time_major, dd_stream **out);
void dd_stream_destroy(dd_stream *stream);
dd_status dd_stream_info(const dd_stream *stream, int64_t *first, int64_t *step);
dd_status dd_stream_reset(dd_stream *stream);
dd_status dd_stream_push(dd_stream *stream, const void *d_block, int64_t samples, void *d_chunk,
                         const float *d_weights, void *d_out, int64_t out_capacity, void *d_ws,
                         size_t ws_bytes, int64_t *chunk_index, void *hip_stream);

/*
 * Corner turn: out[c][t] = in[t][c] for t < nsamp, c < nchans (uint8 for
 * DD_U8, float32 for DD_F32), through LDS tiles.  d_out rows are out_pitch
 * elements apart.  Errors: DD_ERR_NULL, DD_ERR_INVALID, DD_ERR_HIP.
 */
dd_status dd_corner_turn(dd_dtype dtype, const void *d_in, int64_t nsamp, int32_t nchans,
                         void *d_out, int64_t out_pitch, void *stream);

/* Text of a status code (paper, "Design of the API": the API gives the user
 * feedback on errors; "Pipeline": a status code per call).  Returns a
 * static string, never NULL ("unknown dd_status" for values outside
 * dd_status). */
const char *dd_status_str(dd_status status);

/* Detail of the last failing call on this thread (paper, "Design of the
 * API": configuration errors are reported back to the user).  Returns a
 * thread-local string owned by the library, valid until the next failing
 * call on the same thread; "" if no call on this thread has failed. */
const char *dd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DD_MI355X_H */
