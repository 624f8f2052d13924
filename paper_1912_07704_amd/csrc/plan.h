// Host-side plan of the dedispersion library (internal).  No HIP types:
// the host core (plan.cpp) is plain C++ and builds with any host compiler.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dd.h"

namespace dd {

// Tile geometry of the integer forward kernel: each wavefront covers
// kWaveWords 32-bit words per lane (two samples per word) of one time tile,
// for kDmPerWave trial DMs; a workgroup holds 4 or 8 wavefronts (a plan
// option), one DM group each.
constexpr int kWaves = 8;                        // default; the float32 kernels always use 8
constexpr int kWaveWords = 4;                    // words per lane
constexpr int kDmPerWave = 8;
constexpr int kTimeTile = 128 * kWaveWords;      // samples per workgroup
constexpr int kDmTile = kWaves * kDmPerWave;     // default DMs per workgroup
constexpr int kMaxStageChans = 16;               // channels staged at once
constexpr int64_t kMinWorkgroups = 512;          // 2 per CU: below, default time tiles halve
constexpr size_t kMaxLdsBytes = 160 * 1024;
constexpr size_t kLdsTwoBlocks = 80 * 1024;      // LDS that still fits two workgroups per CU
constexpr int kLevelAlign = 64;                  // samples; row pitch granule of a level
// Exact sub-band reuse (integer variant 3).  Channels are grouped into
// sub-bands of up to kSubband consecutive channels.  Inside one DM tile the
// DMs whose delays over a sub-band differ from the sub-band's smallest delay
// by the same pattern share one partial sum of that sub-band, built once in
// LDS and added at each DM's own smallest delay.
constexpr int kSubband = 8;
// The default strategy takes sub-band reuse only when a DM tile holds at
// most this many distinct delay patterns per DM and sub-band (weighted by
// DM-trial samples over the ranges); denser plans build nearly a row per DM
// and run faster on the direct kernel (measured on gfx950: reuse won at
// densities up to 0.16 and lost from 0.37 on).
constexpr double kMaxPatternDensity = 0.25;
constexpr size_t kWsAlign = 256;

// Float32 path: one generic shift-and-sum over rows staged in LDS,
//   out[a][t] = sum_b rows[b][t + S[a][b]],  t < nt,
// used for the forward (a = DM, b = channel, rows = weighted binned input,
// S = s) and for the adjoint (a = channel, b = DM, rows = the output
// gradient with P zeros on both sides, S = P - s).  A workgroup owns
// kF32OutTile outputs (kF32PerWave per wave) by kF32TimeTile samples.
// Samples come from LDS in aligned 4-float granules (one 16-byte read
// each): lane l holds granules l + 63g (g < kF32Words/4) of the tile, i.e.
// samples 4(l + 63g) + j (j < 4).  A delay that is not a multiple of 4 takes
// the granule's tail from the lane itself and its head from the next lane
// (a cross-lane move fused into the add); lane 63 only supplies those heads,
// so a tile is 63 granules x 4 = 1008 samples wide and the lanes span 1024.
constexpr int kF32Words = 16;                    // samples per lane
constexpr int kF32PerWave = 4;
constexpr int kF32TileSpan = 64 * kF32Words;     // 1024: samples the lanes cover
constexpr int kF32TimeTile = 63 * kF32Words;     // 1008: samples a tile computes
constexpr int kF32OutTile = kWaves * kF32PerWave;
constexpr int kF32MaxStage = 16;
// Boxcar loss tiles: the loss tile counts windows starting in its first
// kBoxLossStride samples; the gradient tile writes dL/dout for its samples
// [kBoxLead, kBoxLead + kBoxGradStride).  Both keep the 31-sample reach of
// the widest (32-sample) window inside the 1008-sample tile.
constexpr int kBoxMaxWidth = 32;
constexpr int kBoxLossStride = kF32TimeTile - kBoxMaxWidth;          // 976
constexpr int kBoxLead = kBoxMaxWidth;                                // 32
constexpr int kBoxGradStride = kF32TimeTile - 2 * kBoxMaxWidth;      // 944

// Sub-band reuse in the float32 shift-and-sum (exact regrouping of the same
// sum): rows are taken in groups of kSbGroup; outputs of a tile whose delays
// on a group differ by one common offset (the same delay pattern) share a
// pattern row, PR[u] = sum_{b in group} rows[b][u0 + u + rel(b)], built once
// in LDS (level 1) and added by each of them at its own offset (level 2).
// A pattern row is computed over kSbPatWords samples in one pass of 5
// granules per lane (lane l: granules l + 63g, g < 5); a level-2 read of it
// at offset o reaches float 4*(o >> 2) + 1011, so patterns spread by at most
// kSbMaxSpread samples over their outputs.
constexpr int kSbGroup = 4;
constexpr int kSbStage = 8;                      // rows per stage (two groups)
constexpr int kSbPatWords = kF32TimeTile + kF32TimeTile / 4;     // 1260
constexpr int kSbMaxSpread = kSbPatWords - 1012;                 // 248
constexpr int kSbJobInts = 8;                    // dest, granules per lane, class ends, 4 entries, pad

struct SumProblem {
    int32_t nrows = 0;          // b: rows summed
    int32_t nouts = 0;          // a: output rows
    int64_t nt = 0;             // output samples per output row
    int32_t stage_rows = 0;     // rows staged in LDS at once
    int32_t row_words = 0;      // floats per staged row window (multiple of 4)
    int32_t span = 0;           // largest spread of S inside one output tile
    int32_t nout_tiles = 0;
    int32_t nouts_pad = 0;      // nout_tiles * kF32OutTile
    int64_t ntime_tiles = 0;
    int64_t block_start = 0;
    int32_t nstages = 0;        // ceil(nrows / stage_rows)
    int32_t tab_stride = 0;     // ints per output list: roundup(max entries + 1, 4)
    int32_t tab_block = 0;      // ints per (tile, stage) table block: the kF32OutTile lists,
                                // then (sub-band) the level-1 jobs and their count
    // sub-band reuse (0 patterns: every output adds the stage's rows directly)
    int32_t npat = 0;           // pattern-row slots per stage
    int32_t njobs_max = 0;      // level-1 jobs per stage (one per pattern row)
    // With m = min over the output tile of S[.][b], e = m & 3 and
    // o = e + S[a][b] - m (the delay inside the staged window):
    size_t base_offset = 0;     // baseF: [nout_tiles][nrows] = m - e
    size_t off_offset = 0;      // offF: [nout_tiles][nstages][kF32OutTile][tab_stride]:
                                // per output and stage, the stage's rows
                                // ordered by the class o & 3 (stable), each
                                // entry slot * row_words + 4 * (o >> 2) (slot
                                // = the row's place in the stage's LDS
                                // buffer); the last word holds the ends of
                                // the classes 0, 1, 2, 3 (one byte each, low
                                // byte first).  Sub-band problems: per
                                // (tile, stage) a block of tab_block ints,
                                // the lists (entries also name pattern rows,
                                // at stage_rows * row_words + slot *
                                // kSbPatWords + 4 * (o >> 2)), then njobs_max
                                // jobs of kSbJobInts {destination float,
                                // granules per lane (5), class ends, up to 4
                                // row entries}, then the job count
};

// One 16-bit copy of the input, binned by ds (ds = 1: the samples widened
// to 16 bits), held in the workspace as rows of `pitch` samples followed by
// a tail the staging loads may reach into.
struct BinLevel {
    int32_t ds = 1;          // total binning factor
    int32_t src = -1;        // index of the level it is binned from (-1 = raw input)
    int32_t factor = 1;      // ds / ds of the source
    int64_t nbin = 0;        // floor(nsamp / ds)
    int64_t pitch = 0;       // samples per row (multiple of kLevelAlign, > nbin)
    int64_t lead = 0;        // samples before row 0 (reads at small negative times land here)
    size_t ws_offset = 0;    // byte offset in the workspace (256-byte aligned)
    size_t bytes = 0;
};

struct RangeInfo {
    double lo = 0, hi = 0, step = 0;
    int32_t ds = 1;
    int32_t ndms = 0;
    int32_t dm_index = 0;        // first DM of the range in the plan's DM list
    int64_t nbin = 0;
    int64_t nout = 0;
    int64_t out_offset = 0;      // elements
    int32_t max_shift = 0;
    int32_t level = -1;          // 16-bit copy of the input this range reads
    // strategy
    int32_t stage_chans = 0;     // channels per LDS stage
    int32_t widen_every = 1;     // stages between widenings of the 16-bit sums
    int32_t span = 0;            // largest delay spread inside one DM tile
    int32_t row_words = 0;       // 32-bit words per staged channel copy (multiple of 4)
    int64_t ntime_tiles = 0;
    int32_t ndm_tiles = 0;
    int64_t block_start = 0;     // first workgroup of the range
    int32_t ndms_pad = 0;        // ndms rounded up to a multiple of kDmTile
    size_t off_offset = 0;       // element offset of this range in offT
    size_t base_offset = 0;      // element offset of this range in baseT
    // integer variant 3 (exact sub-band reuse)
    int32_t sb_spread = 0;       // largest spread of a pattern row's smallest delays
    int32_t sb_chans = 0;        // channels per sub-band (kSubband, fewer at large ds)
    int32_t sb_nsub = 0;         // sub-bands
    int32_t sb_jmax = 0;         // most delay patterns of one sub-band in one DM tile
    int32_t sb_span = 0;         // largest spread of one pattern's smallest delays
    int32_t sb_qwords = 0;       // words per copy of a partial-sum row (multiple of 4)
    int32_t sb_nslot = 0;        // sub-bands per stage
    int32_t sb_tb_words = 0;     // ints per LDS buffer of one stage's tables
    size_t sb_q_offset = 0;      // element offset of this range in qoffT
    size_t sb_n_offset = 0;      // element offset of this range in qcntT
    size_t sb_c_offset = 0;      // element offset of this range in offCT
    // float32 plans
    SumProblem fwd;              // forward of this range
    SumProblem adj;              // adjoint of this range (rows = DMs, outputs = channels)
    int64_t gpitch = 0;          // floats per padded output-gradient row
    size_t gpad_offset = 0;      // workspace bytes: padded gradient rows [ndms][gpitch]
    int64_t Gpitch = 0;          // floats per row of the channel gradient G_r
    size_t G_offset = 0;         // workspace bytes: G_r [nchans][Gpitch]
};

struct Plan {
    int32_t nchans = 0;
    double tsamp = 0;
    int64_t nsamp = 0;
    dd_dtype dtype = DD_U8;
    std::vector<double> freqs;
    std::vector<double> dms;               // [ndms_total]
    std::vector<int32_t> shifts;           // [ndms_total][nchans]
    // Device tables of the integer kernel, per range, concatenated.  With
    // b = s[d0][c] the delay of the first DM d0 of a DM tile, p = b & 1 and
    // e = ((b - p)/2) & 3:
    //  baseT[tile][c]  first 32-bit word of the staged window, relative to
    //                  sample t0 of the time tile: (b - p)/2 - e  (so the
    //                  window starts 16-byte aligned);
    //  offT[c][d]      word offset of DM d inside the staged channel:
    //                  ((o + p) & 1) * stage_chans * row_words + e + ((o + p) >> 1),
    //                  o = s[d][c] - b; the first term picks the odd-aligned
    //                  copy.  DMs past the last (up to ndms_pad) repeat the last.
    std::vector<int32_t> baseT;
    std::vector<int32_t> offT;
    // Variant 3 tables (offT unused; baseT as above).  For DM tile g,
    // sub-band b and delay pattern j of that tile and sub-band:
    //  qcntT[g][b]         number of patterns J;
    //  qoffT[g][b][j][k]   word offset, from the start of the stage's even
    //                      copy, of the staged window of the sub-band's k-th
    //                      channel at which pattern j's row starts (copy
    //                      select folded in, as in offT);
    //  offCT[g][b][d]      word offset, from the start of the partial-sum
    //                      region, of DM d's (d < dm_tile) row and delay:
    //                      ((s*jmax + j)*2 + (o & 1))*qwords + (o >> 1), with
    //                      s the sub-band's slot in its stage and o the DM's
    //                      smallest delay minus the pattern's smallest.
    std::vector<int32_t> qcntT;
    std::vector<int32_t> qoffT;
    std::vector<int32_t> offCT;
    bool subband = false;                  // integer variant 3
    double sb_density = 0;                 // variant 3: distinct patterns per DM and sub-band
    std::vector<RangeInfo> ranges;
    std::vector<BinLevel> levels;
    int64_t out_elems = 0;
    int64_t overlap = 0;
    size_t ws_bytes = 0;
    size_t fwd_ws_bytes = 0;               // the part of the workspace the forward uses (its levels)
    int64_t blocks = 0;                    // workgroups of one forward launch
    size_t lds_bytes = 0;                  // dynamic LDS of the forward kernel
    bool dedup = true;                     // integer kernel variant (dd_options.variant)
    int32_t waves = kWaves;                // integer kernel: wavefronts per workgroup (4 or 8)
    int32_t dm_tile = kDmTile;             // integer kernel: DMs per workgroup
    int32_t time_tile = kTimeTile;         // integer kernel: samples per workgroup
    // float32 plans: tables of the generic shift-and-sum (forward problems
    // then adjoint problems), and the adjoint's reduction buffer.
    std::vector<int32_t> offF;
    std::vector<int32_t> baseF;
    int64_t adj_blocks = 0;
    size_t adj_lds_bytes = 0;
    int32_t dw_chunks = 0;                 // time chunks of the weight-gradient reduction
    int64_t dw_chunk_len = 0;
    size_t dw_offset = 0;                  // workspace bytes: partials [nchans][dw_chunks], or
                                           // [nchans][dw_tiles] when the adjoint is fused
    // One range at full resolution: the adjoint kernel forms dX and the
    // weight-gradient partials itself, one per (channel, time tile).
    bool adj_fused = false;
    int32_t dw_tiles = 0;
    // boxcar loss (float32 plans): the loss partials of one launch and one
    // beam's weight gradient.
    size_t box_offset = 0;                 // [box_partials + 64] floats
    int64_t box_partials = 0;
    size_t dwb_offset = 0;                 // [nchans] floats
    void *device = nullptr;                // device-side state (owned by the HIP unit)
};

// Host core (plan.cpp).  On failure returns a negative status and writes a
// message into *err.
dd_status build_plan(const double *freqs_mhz, int32_t nchans, double tsamp_s, int64_t nsamp,
                     const dd_range *ranges, int32_t nranges, dd_dtype dtype,
                     const dd_options *opts, Plan *p, std::string *err);

// Device-side state of a plan (allocated by the HIP unit, freed by
// dd_plan_destroy).
void *new_device_state();
void *new_batch_device_state();

// Thread-local error text shared by every entry point.
void set_error(const std::string &msg);
void clear_error();

// A batch of integer plans (beams) summed by persistent launches, one per
// group of plans that share a kernel (variant family, DM tile, time tile).  Inputs and
// outputs of all beams share one buffer each, at fixed offsets.
struct BatchDescHost {
    int32_t beam = 0;
    int32_t range = 0;
    int64_t item_start = 0;      // first work item of this (beam, range) within its group
    int64_t nitems = 0;          // time tiles x DM tiles
};

constexpr int kBatchQueues = 8;                // one work queue per XCD
// fixed part of a batch item's cost, in channels: a 192-DM x 256-sample
// variant-3 item of a 1024-channel beam takes as long as 1024 + ~330
// channels' worth of a 4096-channel beam's item
constexpr double kItemOverheadChans = 330.0;
constexpr int kBatchMaxGroups = 8;             // kernels per batch

struct BatchGroup {
    bool f32 = false;                      // float32 plans: the generic shift-and-sum
    bool subband = false;                  // variant 3 (else the direct kernel)
    bool dedup = false;                    // direct kernel: variant 2
    int32_t dm_tile = kDmTile;
    int32_t time_tile = kTimeTile;
    int32_t waves = kWaves;
    size_t lds_bytes = 0;
    size_t desc_begin = 0, desc_end = 0;   // its (beam, range) descriptors in Batch::descs
    int64_t nitems = 0;
    // XCD x's queue holds items [queue_bounds[x], queue_bounds[x+1]): equal
    // shares of the group's cost (items weigh their beam's channel count)
    int64_t queue_bounds[kBatchQueues + 1] = {};
};

struct Batch {
    dd_dtype dtype = DD_U8;                // of every plan
    std::vector<const Plan *> plans;       // not owned
    std::vector<int64_t> w_off;            // float32: floats into the batch weights (beam b's
                                           // [nchans] weights)
    std::vector<int64_t> in_off;           // bytes into the batch input
    std::vector<int64_t> out_off;          // elements (int32 or float32) into the batch output
    std::vector<size_t> ws_off;            // bytes into the workspace (beam's own part)
    int64_t in_bytes = 0;
    int64_t out_elems = 0;
    int64_t w_elems = 0;                   // float32: weights of all beams
    size_t ws_bytes = 0;
    // float32 boxcar calls: after every beam's levels, per beam the
    // adjoint's padded gradient rows of each range and its weight-gradient
    // partials, then the loss partials of all beams
    std::vector<std::vector<size_t>> gpad_off;   // [beam][range] bytes
    std::vector<size_t> dwp_off;           // [beam] bytes: partials [nchans][dw_tiles]
    size_t loss_part_off = 0;              // bytes
    int64_t loss_blocks = 0;               // loss workgroups of all beams
    size_t box_ws_bytes = 0;
    bool box_fused = false;                // every plan's adjoint is fused (one range, ds 1)
    std::vector<BatchDescHost> descs;      // by group, most expensive items first in each
    std::vector<BatchGroup> groups;
    int64_t nitems = 0;                    // all groups
    void *device = nullptr;
};

constexpr size_t kBatchCounterBytes = 256;     // queue counters (kBatchQueues per group) at the
                                               // start of the workspace
static_assert(kBatchCounterBytes >= sizeof(int32_t) * kBatchQueues * kBatchMaxGroups, "counters");

// Streaming over a long series in chunks of the plan's nsamp samples.
// Consecutive chunks start `step` samples apart; step is the largest
// multiple of every range's downsample with step <= ds_r * nout_r for all r,
// so the first step/ds_r outputs of each chunk row tile the one-shot output.
struct Stream {
    const dd_plan *handle = nullptr;  // borrowed
    const Plan *plan = nullptr;       // the same plan
    int32_t time_major = 0;       // input blocks are [samples][nchans] (SIGPROC order)
    int64_t step = 0;
    int64_t overlap = 0;          // nsamp - step
    int64_t chunks = 0;           // chunks produced so far
};

dd_status build_stream(const Plan *plan, int32_t time_major, Stream *s, std::string *err);

dd_status build_batch(const Plan *const *plans, int32_t nbeams, Batch *b, std::string *err);

}  // namespace dd

struct dd_plan {
    dd::Plan p;
};

struct dd_batch {
    dd::Batch b;
};

struct dd_stream {
    dd::Stream s;
};
