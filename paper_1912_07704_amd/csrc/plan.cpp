// Host core of the dedispersion library: plan validation, DM expansion, the
// FP64 shift table, per-range sizes and the tile strategy.  Plain C++ with
// no HIP dependency (paper, "Separate compilation and linking": host code
// is built by the host compiler).  Build with -ffp-contract=off so the delay
// is evaluated exactly in the order written.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "plan.h"

namespace dd {

namespace {

constexpr double kDispersion = 4.148808e3;   // s MHz^2 pc^-1 cm^3

thread_local std::string g_last_error;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <typename... A>
std::string fmt(A &&...a)
{
    std::ostringstream os;
    (os << ... << a);
    return os.str();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// fn(begin, end) over contiguous slices of [0, n) on up to 16 host threads
// (one when the work is small).  Every element is computed by the same code
// whatever the slicing, so the tables do not depend on the thread count.
template <class F>
void parallel_for(int64_t n, int64_t work_per_item, F fn)
{
    const int64_t hw = std::max<int64_t>(1, std::thread::hardware_concurrency());
    const int64_t nt = std::min<int64_t>({hw, 16, n, std::max<int64_t>(1, n * work_per_item >> 20)});
    if (nt <= 1) {
        if (n > 0)
            fn(int64_t(0), n);
        return;
    }
    // a slice's exception (an allocation failure) is rethrown here after
    // every thread has joined
    std::vector<std::exception_ptr> fail(static_cast<size_t>(nt));
    auto run = [&](int64_t k) {
        try {
            fn(n * k / nt, n * (k + 1) / nt);
        } catch (...) {
            fail[size_t(k)] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve(size_t(nt - 1));
    for (int64_t k = 1; k < nt; ++k) {
        try {
            th.emplace_back(run, k);
        } catch (const std::system_error &) {
            run(k);                                  // no thread to spare: this one does it
        }
    }
    run(0);
    for (std::thread &t : th)
        t.join();
    for (const std::exception_ptr &e : fail)
        if (e)
            std::rethrow_exception(e);
}


// Sub-band reuse of one (output tile, stage): the pattern rows it builds
// and, per output and row group, the pattern the output adds (-1: the
// group's rows directly).
struct SbPattern {
    int32_t group = 0;              // row group inside the stage
    int32_t gn = 0;                 // rows in the group
    int32_t u0 = 0;                 // smallest pattern offset of its outputs
    std::vector<int32_t> rel;       // [gn] delay of each row minus the pattern offset
    int32_t nout = 0;               // outputs that add it
};

struct SbStagePlan {
    std::vector<SbPattern> pats;
    std::vector<int32_t> pat_of;    // [kF32OutTile][groups]
};

// Tables of one float32 shift-and-sum problem (see plan.h).  S(a, b) gives
// the delay of row b for output a; it must be >= 0.  sb_mode: 0 sub-band
// reuse where the work it saves passes a threshold, 1 never, 2 always
// (error when its tables do not fit the LDS).
template <typename SFn>
dd_status build_sum_problem(SumProblem &sp, int32_t nrows, int32_t nouts, int64_t nt, SFn S_,
                            std::vector<int32_t> &offF, std::vector<int32_t> &baseF,
                            int64_t *blocks, size_t *lds,
                            std::string *err, const char *what, int32_t want_stage, int32_t sb_mode)
{
    sp.nrows = nrows;
    sp.nouts = nouts;
    sp.nt = nt;
    sp.nout_tiles = (nouts + kF32OutTile - 1) / kF32OutTile;
    sp.nouts_pad = sp.nout_tiles * kF32OutTile;
    sp.ntime_tiles = (nt + kF32TimeTile - 1) / kF32TimeTile;
    int32_t span = 0;
    std::vector<int32_t> mins(size_t(sp.nout_tiles) * nrows);
    for (int32_t tile = 0; tile < sp.nout_tiles; ++tile) {
        const int32_t a0 = tile * kF32OutTile;
        const int32_t a1 = std::min(nouts, a0 + kF32OutTile);
        for (int32_t b = 0; b < nrows; ++b) {
            int32_t lo = S_(a0, b), hi = lo;
            for (int32_t a = a0 + 1; a < a1; ++a) {
                const int32_t v = S_(a, b);
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            mins[size_t(tile) * nrows + b] = lo;
            span = std::max(span, hi - lo);
        }
    }
    sp.span = span;
    // window start of row b in a tile (16-byte aligned)
    auto W0 = [&](int32_t tile, int32_t b) {
        const int32_t m = mins[size_t(tile) * nrows + b];
        return m - (m & 3);
    };
    // a delay o <= span + 3 inside the window; lane 63 reads its last
    // granule at 4*(o >> 2) + 4*63*G (G granules per lane), up to float
    // 4*(o >> 2) + 252*G + 3
    const int32_t direct_words = (span + 3 + 252 * (kF32Words / 4) + 3 + 1 + 3) / 4 * 4;
    auto stride_for = [&](int32_t st) { return (st + 1 + 3) / 4 * 4; };
    // one stage buffer: the rows, the pattern rows, then the table block
    auto bytes_for = [&](int32_t st, int32_t words, int32_t npat, int32_t tab_block) {
        return sizeof(float) * (size_t(st) * size_t(words) + size_t(npat) * kSbPatWords +
                                size_t(tab_block) + 16);
    };

    // ---- direct: every output adds every row of a stage
    int32_t stage = want_stage > 0 ? std::max(1, std::min(want_stage, kF32MaxStage)) : kF32MaxStage;
    if (stage > 1)
        stage &= ~1;
    auto direct_block = [&](int32_t st) { return kF32OutTile * stride_for(st); };
    while (stage > 1 && bytes_for(stage, direct_words, 0, direct_block(stage)) > kLdsTwoBlocks)
        stage = stage > 2 ? stage - 2 : 1;
    const bool direct_fits = bytes_for(stage, direct_words, 0, direct_block(stage)) <= kMaxLdsBytes;

    // ---- sub-band reuse
    const int32_t sb_nst = (nrows + kSbStage - 1) / kSbStage;
    const int32_t ngroups = kSbStage / kSbGroup;
    std::vector<SbStagePlan> sbs;
    int32_t sb_cap = 0, sb_words = 0;
    double cost_sb = 0.0, cost_direct = 0.0;
    bool sb_fits = false;
    if (sb_mode != 1 && nrows >= 2) {
        for (int32_t cap : {8, 6, 4, 2}) {
            sbs.assign(size_t(sp.nout_tiles) * sb_nst, SbStagePlan());
            int32_t words = direct_words;
            cost_sb = cost_direct = 0.0;
            for (int32_t tile = 0; tile < sp.nout_tiles; ++tile) {
                const int32_t a0 = tile * kF32OutTile;
                const int32_t na = std::min(nouts, a0 + kF32OutTile) - a0;
                cost_direct += double(na) * nrows;
                for (int32_t st = 0; st < sb_nst; ++st) {
                    SbStagePlan &P = sbs[size_t(tile) * sb_nst + st];
                    P.pat_of.assign(size_t(kF32OutTile) * ngroups, -1);
                    const int32_t b0 = st * kSbStage, bn = std::min(kSbStage, nrows - b0);
                    // candidate patterns of every group: delays minus their
                    // smallest, shared by two outputs or more
                    struct Cand {
                        int32_t group, gn, u0, spread_hi;
                        std::vector<int32_t> rel, outs;
                    };
                    std::vector<Cand> cands;
                    for (int32_t gi = 0; gi * kSbGroup < bn; ++gi) {
                        const int32_t gb = b0 + gi * kSbGroup;
                        const int32_t gn = std::min(kSbGroup, b0 + bn - gb);
                        std::map<std::vector<int32_t>, size_t> at;
                        for (int32_t al = 0; al < na; ++al) {
                            std::vector<int32_t> rel(static_cast<size_t>(gn));
                            int32_t base = S_(a0 + al, gb);
                            for (int32_t j = 1; j < gn; ++j)
                                base = std::min(base, S_(a0 + al, gb + j));
                            for (int32_t j = 0; j < gn; ++j)
                                rel[size_t(j)] = S_(a0 + al, gb + j) - base;
                            auto it = at.find(rel);
                            if (it == at.end()) {
                                Cand c;
                                c.group = gi;
                                c.gn = gn;
                                c.u0 = base;
                                c.spread_hi = base;
                                c.rel = rel;
                                c.outs.push_back(al);
                                at.emplace(rel, cands.size());
                                cands.push_back(std::move(c));
                            } else {
                                Cand &c = cands[it->second];
                                c.u0 = std::min(c.u0, base);
                                c.spread_hi = std::max(c.spread_hi, base);
                                c.outs.push_back(al);
                            }
                        }
                    }
                    std::vector<size_t> order;
                    for (size_t k = 0; k < cands.size(); ++k) {
                        const Cand &c = cands[k];
                        // sharing pays when the outputs' direct adds exceed
                        // the pattern row's (1.25 passes) plus one each
                        if (c.gn >= 2 && c.outs.size() >= 2 &&
                            c.spread_hi - c.u0 <= kSbMaxSpread &&
                            double(c.outs.size()) * c.gn > 1.25 * c.gn + double(c.outs.size()))
                            order.push_back(k);
                    }
                    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
                        return cands[x].outs.size() > cands[y].outs.size();
                    });
                    if (order.size() > size_t(cap))
                        order.resize(size_t(cap));
                    for (size_t k : order) {
                        const Cand &c = cands[k];
                        SbPattern pat;
                        pat.group = c.group;
                        pat.gn = c.gn;
                        pat.u0 = c.u0;
                        pat.rel = c.rel;
                        pat.nout = int32_t(c.outs.size());
                        const int32_t slot = int32_t(P.pats.size());
                        for (int32_t al : c.outs)
                            P.pat_of[size_t(al) * ngroups + c.group] = slot;
                        // level-1 reads of row b: the window offset e of
                        // the pattern's first sample, then 1260 + 4 floats
                        for (int32_t j = 0; j < c.gn; ++j) {
                            const int32_t b = b0 + c.group * kSbGroup + j;
                            const int32_t e = c.u0 + c.rel[size_t(j)] - W0(tile, b);
                            words = std::max(words, 4 * (e >> 2) + kSbPatWords + 4);
                        }
                        cost_sb += 1.25 * c.gn + double(c.outs.size());
                        P.pats.push_back(std::move(pat));
                    }
                    for (int32_t al = 0; al < na; ++al)
                        for (int32_t gi = 0; gi * kSbGroup < bn; ++gi)
                            if (P.pat_of[size_t(al) * ngroups + gi] < 0)
                                cost_sb += std::min(kSbGroup, bn - gi * kSbGroup);
                }
            }
            words = (words + 3) / 4 * 4;
            const int32_t block = kF32OutTile * stride_for(kSbStage) + kSbJobInts * cap + 4;
            if (bytes_for(kSbStage, words, cap, block) <= kLdsTwoBlocks) {
                sb_fits = true;
                sb_cap = cap;
                sb_words = words;
                break;
            }
        }
    }
    // (on the differentiable plans, 2.4-2.5x less work ran the forward
    // 1.11x and the adjoint 1.01x faster: the 8-row stages pay more for
    // their loads and barriers)
    const bool use_sb = sb_fits && (sb_mode == 2 || cost_sb < (2.0 / 3.0) * cost_direct);
    if (sb_mode == 2 && !sb_fits) {
        *err = fmt(what, ": the sub-band tables of this plan do not fit the LDS");
        return DD_ERR_INVALID;
    }
    if (!use_sb && !direct_fits) {
        *err = fmt(what, ": delay spread ", span,
                   " inside one tile needs more LDS than a workgroup has; use a finer DM step");
        return DD_ERR_INVALID;
    }
    if (use_sb) {
        sp.stage_rows = kSbStage;
        sp.row_words = sb_words;
        sp.npat = sb_cap;
        sp.njobs_max = sb_cap;
    } else {
        sp.stage_rows = stage;
        sp.row_words = direct_words;
        sp.npat = 0;
        sp.njobs_max = 0;
    }
    const int32_t C = sp.stage_rows, Wr = sp.row_words;
    sp.nstages = (nrows + C - 1) / C;
    sp.tab_stride = stride_for(C);
    sp.tab_block = kF32OutTile * sp.tab_stride + (use_sb ? kSbJobInts * sp.njobs_max + 4 : 0);
    *lds = std::max(*lds, bytes_for(C, Wr, sp.npat, sp.tab_block));
    sp.block_start = *blocks;
    *blocks += sp.ntime_tiles * sp.nout_tiles;
    sp.base_offset = baseF.size();
    baseF.resize(baseF.size() + size_t(sp.nout_tiles) * nrows);
    for (int32_t tile = 0; tile < sp.nout_tiles; ++tile)
        for (int32_t b = 0; b < nrows; ++b)
            baseF[sp.base_offset + size_t(tile) * nrows + b] = W0(tile, b);
    // Per (tile, stage): the output lists -- each output's entries ordered by
    // the class o & 3 of their offset (stable), the class ends in the list's
    // last word -- then (sub-band) the level-1 jobs and their count; the
    // kernel stages each block in LDS beside the rows.
    const int32_t TS = sp.tab_stride;
    const size_t nblocks = size_t(sp.nout_tiles) * size_t(sp.nstages);
    offF.resize((offF.size() + 3) / 4 * 4, 0);
    sp.off_offset = offF.size();
    offF.resize(offF.size() + nblocks * size_t(sp.tab_block), 0);
    std::vector<std::pair<int32_t, int32_t>> items;   // (entry, class)
    auto emit_sorted = [&](int32_t *out, int32_t *ends_out) {
        int32_t n = 0;
        uint32_t ends = 0;
        for (int32_t cls = 0; cls < 4; ++cls) {
            for (const auto &it : items)
                if (it.second == cls)
                    out[n++] = it.first;
            ends |= uint32_t(n) << (8 * cls);
        }
        *ends_out = int32_t(ends);
    };
    for (int32_t tile = 0; tile < sp.nout_tiles; ++tile)
        for (int32_t st = 0; st < sp.nstages; ++st) {
            int32_t *blk = &offF[sp.off_offset + (size_t(tile) * sp.nstages + st) * sp.tab_block];
            const int32_t b0 = st * C, bn = std::min(C, nrows - b0);
            const SbStagePlan *P = use_sb ? &sbs[size_t(tile) * sb_nst + st] : nullptr;
            for (int32_t al = 0; al < kF32OutTile; ++al) {
                const int32_t av = std::min(tile * kF32OutTile + al, nouts - 1);
                const int32_t alv = av - tile * kF32OutTile;
                items.clear();
                for (int32_t j = 0; j < bn; ++j) {
                    const int32_t b = b0 + j;
                    const int32_t gi = j / kSbGroup;
                    const int32_t pat = P ? P->pat_of[size_t(alv) * ngroups + gi] : -1;
                    if (pat >= 0) {
                        if (j % kSbGroup == 0) {
                            // the pattern row, at the output's offset
                            const SbPattern &pt = P->pats[size_t(pat)];
                            int32_t base = S_(av, b);
                            for (int32_t k = 1; k < pt.gn; ++k)
                                base = std::min(base, S_(av, b + k));
                            const int32_t o = base - pt.u0;
                            items.emplace_back(C * Wr + pat * kSbPatWords + 4 * (o >> 2), o & 3);
                        }
                        continue;
                    }
                    const int32_t o = S_(av, b) - W0(tile, b);
                    items.emplace_back(j * Wr + 4 * (o >> 2), o & 3);
                }
                emit_sorted(blk + size_t(al) * TS, blk + size_t(al) * TS + TS - 1);
            }
            if (!P)
                continue;
            int32_t *jobs = blk + size_t(kF32OutTile) * TS;
            const int32_t np = int32_t(P->pats.size());
            for (int32_t k = 0; k < np; ++k) {
                const SbPattern &pt = P->pats[size_t(k)];
                int32_t *J = jobs + size_t(k) * kSbJobInts;
                J[0] = C * Wr + k * kSbPatWords;
                J[1] = kSbPatWords / 252;         // granules per lane: the whole pattern row in one pass
                items.clear();
                for (int32_t j = 0; j < pt.gn; ++j) {
                    const int32_t slot = pt.group * kSbGroup + j;
                    const int32_t e = pt.u0 + pt.rel[size_t(j)] - W0(tile, b0 + slot);
                    items.emplace_back(slot * Wr + 4 * (e >> 2), e & 3);
                }
                emit_sorted(J + 3, J + 2);
            }
            jobs[size_t(sp.njobs_max) * kSbJobInts] = np;
        }
    return DD_OK;
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char *last_error() { return g_last_error.c_str(); }


// Float32 plans: weighted 32-bit level copies, forward and adjoint problems
// of the generic shift-and-sum, and the adjoint's workspace buffers.
dd_status build_f32(Plan *p, int32_t want_stage, int32_t sb_mode, std::string *err)
{
    const int32_t nchans = p->nchans;
    const int64_t nsamp = p->nsamp;
    size_t ws = 0;
    // levels (one per distinct downsample, cascaded like the integer path)
    std::vector<int32_t> dss;
    for (const RangeInfo &ri : p->ranges)
        dss.push_back(ri.ds);
    std::sort(dss.begin(), dss.end());
    dss.erase(std::unique(dss.begin(), dss.end()), dss.end());
    p->levels.clear();
    p->offF.clear();
    p->baseF.clear();
    int64_t blocks = 0, ablocks = 0;
    size_t lds = 0, alds = 0;
    for (int32_t r = 0; r < int32_t(p->ranges.size()); ++r) {
        RangeInfo &ri = p->ranges[r];
        const int32_t *sh = &p->shifts[size_t(ri.dm_index) * nchans];
        auto Sf = [&](int32_t a, int32_t b) { return sh[size_t(a) * nchans + b]; };
        dd_status st = build_sum_problem(ri.fwd, nchans, ri.ndms, ri.nout, Sf, p->offF, p->baseF,
                                         &blocks, &lds, err, "forward", want_stage, sb_mode);
        if (st != DD_OK)
            return st;
    }
    for (int32_t r = 0; r < int32_t(p->ranges.size()); ++r) {
        RangeInfo &ri = p->ranges[r];
        const int32_t *sh = &p->shifts[size_t(ri.dm_index) * nchans];
        const int32_t P = ri.max_shift;
        auto Sa = [&](int32_t a, int32_t b) { return P - sh[size_t(b) * nchans + a]; };
        dd_status st = build_sum_problem(ri.adj, ri.ndms, nchans, ri.nbin, Sa, p->offF, p->baseF,
                                         &ablocks, &alds, err, "adjoint", want_stage, sb_mode);
        if (st != DD_OK)
            return st;
    }
    p->blocks = blocks;
    p->lds_bytes = lds;
    p->adj_blocks = ablocks;
    p->adj_lds_bytes = alds;
    // reported as variant 3 when a forward problem uses sub-band reuse
    p->subband = false;
    p->dedup = true;
    for (const RangeInfo &ri : p->ranges)
        p->subband = p->subband || ri.fwd.npat > 0;
    for (int32_t ds : dss) {
        BinLevel lv;
        lv.ds = ds;
        lv.src = -1;
        lv.factor = ds;
        for (int32_t j = int32_t(p->levels.size()) - 1; j >= 0; --j)
            if (p->levels[j].ds > 1 && ds % p->levels[j].ds == 0) {
                lv.src = j;
                lv.factor = ds / p->levels[j].ds;
                break;
            }
        lv.nbin = nsamp / ds;
        lv.pitch = (lv.nbin + 8 + kLevelAlign - 1) / kLevelAlign * kLevelAlign;
        lv.lead = kLevelAlign;
        int32_t reach = 0;
        for (const RangeInfo &ri : p->ranges)
            if (ri.ds == ds)
                reach = std::max(reach, ri.fwd.row_words + 16);
        lv.ws_offset = ws;
        lv.bytes = (size_t(lv.lead) + size_t(nchans) * size_t(lv.pitch) + size_t(reach)) *
                   sizeof(float);
        ws = align_up(ws + lv.bytes, kWsAlign);
        p->levels.push_back(lv);
    }
    for (RangeInfo &ri : p->ranges)
        for (size_t j = 0; j < p->levels.size(); ++j)
            if (p->levels[j].ds == ri.ds)
                ri.level = int32_t(j);
    // adjoint buffers
    for (RangeInfo &ri : p->ranges) {
        const int64_t reach = ri.nbin + ri.max_shift + ri.adj.row_words + 16;
        ri.gpitch = (reach + kLevelAlign - 1) / kLevelAlign * kLevelAlign;
        ri.gpad_offset = ws;
        ws = align_up(ws + size_t(ri.ndms) * size_t(ri.gpitch) * sizeof(float), kWsAlign);
        ri.Gpitch = (ri.nbin + kLevelAlign - 1) / kLevelAlign * kLevelAlign;
        ri.G_offset = ws;
        ws = align_up(ws + size_t(nchans) * size_t(ri.Gpitch) * sizeof(float), kWsAlign);
    }
    p->dw_chunk_len = 4096;
    p->dw_chunks = int32_t((nsamp + p->dw_chunk_len - 1) / p->dw_chunk_len);
    p->adj_fused = p->ranges.size() == 1 && p->ranges[0].ds == 1;
    p->dw_tiles = p->adj_fused ? int32_t(p->ranges[0].adj.ntime_tiles) : 0;
    p->dw_offset = ws;
    ws = align_up(ws + size_t(nchans) * size_t(std::max(p->dw_chunks, p->dw_tiles)) * sizeof(float),
                  kWsAlign);
    // boxcar loss buffers (the backward writes dL/dout straight into the
    // adjoint's padded rows)
    int64_t lp = 0;
    for (const RangeInfo &ri : p->ranges)
        lp += (ri.nout + kBoxLossStride - 1) / kBoxLossStride * ri.fwd.nout_tiles;
    p->box_partials = lp;
    p->box_offset = ws;
    ws = align_up(ws + size_t(lp + 64) * sizeof(float), kWsAlign);
    p->dwb_offset = ws;
    ws = align_up(ws + size_t(nchans) * sizeof(float), kWsAlign);
    p->ws_bytes = ws;
    p->fwd_ws_bytes = 0;
    for (const BinLevel &lv : p->levels)
        p->fwd_ws_bytes = std::max(p->fwd_ws_bytes, lv.ws_offset + lv.bytes);
    return DD_OK;
}

// 16-bit copies of the input for the integer kernels: one per distinct
// downsample (1 included), each binned from the largest earlier level
// (ds > 1) that divides it, or from the raw input.  Each level's tail covers
// what the staging loads of its ranges may read past the last row.
void build_levels(Plan *p)
{
    std::vector<int32_t> dss;
    for (const RangeInfo &ri : p->ranges)
        dss.push_back(ri.ds);
    std::sort(dss.begin(), dss.end());
    dss.erase(std::unique(dss.begin(), dss.end()), dss.end());
    p->levels.clear();
    size_t ws = 0;
    for (int32_t ds : dss) {
        BinLevel lv;
        lv.ds = ds;
        lv.src = -1;
        lv.factor = ds;
        for (int32_t j = int32_t(p->levels.size()) - 1; j >= 0; --j)
            if (p->levels[j].ds > 1 && ds % p->levels[j].ds == 0) {
                lv.src = j;
                lv.factor = ds / p->levels[j].ds;
                break;
            }
        lv.nbin = p->nsamp / ds;
        lv.pitch = (lv.nbin + 8 + kLevelAlign - 1) / kLevelAlign * kLevelAlign;
        int32_t reach = 0;     // samples the staging may read past a row start + nbin
        for (const RangeInfo &ri : p->ranges)
            if (ri.ds == ds)
                reach = std::max(reach, 2 * ri.row_words + 16);
        lv.ws_offset = ws;
        lv.bytes = (size_t(p->nchans) * size_t(lv.pitch) + size_t(reach)) * sizeof(uint16_t);
        ws = align_up(ws + lv.bytes, kWsAlign);
        p->levels.push_back(lv);
    }
    for (RangeInfo &ri : p->ranges) {
        ri.level = -1;
        for (size_t j = 0; j < p->levels.size(); ++j)
            if (p->levels[j].ds == ri.ds)
                ri.level = int32_t(j);
    }
    p->ws_bytes = ws;
    p->fwd_ws_bytes = ws;
}

// Delay patterns of one sub-band (channels [c0, c0 + kb)) over the DMs
// [d0, d0 + nd) of a range.  a[i] is DM i's smallest delay over the
// sub-band; two DMs share a pattern when their delays minus a[i] agree on
// every channel of the sub-band, and then share one partial sum.
struct SbPatterns {
    int32_t J = 0;
    std::vector<int32_t> a, idx;          // per DM
    std::vector<int32_t> amin, amax, rep; // per pattern (rep: one of its DMs)
    std::vector<uint64_t> key;            // per DM: packed pattern (fast path)
};

void sb_patterns(const Plan &p, const RangeInfo &ri, int32_t d0, int32_t nd, int32_t c0,
                 int32_t kb, int32_t max_spread, SbPatterns &t, std::vector<int32_t> &order)
{
    const int32_t nch = p.nchans;
    const int32_t *s = &p.shifts[size_t(ri.dm_index + d0) * nch + c0];
    t.a.resize(size_t(nd));
    t.idx.resize(size_t(nd));
    order.resize(size_t(nd));
    t.key.resize(size_t(nd));
    int32_t umax = 0;
    for (int32_t i = 0; i < nd; ++i) {
        const int32_t *si = s + size_t(i) * nch;
        int32_t m = si[0];
        for (int32_t k = 1; k < kb; ++k)
            m = std::min(m, si[k]);
        t.a[i] = m;
        order[i] = i;
        uint64_t key = 0;
        for (int32_t k = 0; k < kSubband; ++k) {
            const int32_t u = k < kb ? si[k] - m : 0;
            umax = std::max(umax, u);
            key = (key << 8) | uint64_t(u & 0xff);
        }
        t.key[i] = key;
    }
    // Patterns in lexicographic order of their delays (channel c0 first),
    // ties in DM order.  With every delay difference below 256 the packed
    // key (channel c0 in the top byte) orders them the same way.
    const bool packed = umax < 256;
    auto cmp = [&](int32_t x, int32_t y) {
        if (packed)
            return t.key[x] == t.key[y] ? 0 : t.key[x] < t.key[y] ? -1 : 1;
        const int32_t *sx = s + size_t(x) * nch, *sy = s + size_t(y) * nch;
        for (int32_t k = 0; k < kb; ++k) {
            const int32_t u = sx[k] - t.a[x], v = sy[k] - t.a[y];
            if (u != v)
                return u < v ? -1 : 1;
        }
        return 0;
    };
    if (packed)
        std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            return t.key[x] != t.key[y] ? t.key[x] < t.key[y] : x < y;
        });
    else
        std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            const int c = cmp(x, y);
            return c != 0 ? c < 0 : x < y;
        });
    t.J = 0;
    t.amin.clear();
    t.amax.clear();
    t.rep.clear();
    // DMs of one pattern come in increasing DM order, so increasing a; a
    // pattern whose smallest delays would spread over more than max_spread
    // samples continues as a new pattern (a longer row costs every row).
    for (int32_t n = 0; n < nd; ++n) {
        const int32_t i = order[n];
        if (n == 0 || cmp(order[n - 1], i) != 0 || t.a[i] - t.amin[t.J - 1] > max_spread) {
            t.amin.push_back(t.a[i]);
            t.amax.push_back(t.a[i]);
            t.rep.push_back(i);
            ++t.J;
        }
        const int32_t j = t.J - 1;
        t.idx[i] = j;
        t.amin[j] = std::min(t.amin[j], t.a[i]);
        t.amax[j] = std::max(t.amax[j], t.a[i]);
    }
}

constexpr int32_t kWave64 = 64;    // lanes per wavefront

// Integer variant 3: exact sub-band reuse.  Per range: the channel windows
// of a DM tile (as in the direct kernel), the most patterns of one
// sub-band in one DM tile, the rows' sizes, the stage width that fits the
// LDS, then the tables documented in plan.h.
dd_status build_subband(Plan *p, int32_t want_stage, std::string *err)
{
    const int32_t nchans = p->nchans;
    const int32_t dmt = p->dm_tile;
    // dm_tile 128 and 192: 16 wavefronts of 8 or 12 DMs, 2 words (4 samples)
    // per lane; 64 and 96: 8 wavefronts of 8 or 12 DMs, 4 words per lane.
    const bool wide = dmt >= 128;
    const int32_t T = p->time_tile;
    if (wide && T != kTimeTile / 2) {
        *err = fmt("variant 3 at ", dmt, "-DM tiles runs ", kTimeTile / 2, "-sample time tiles only");
        return DD_ERR_INVALID;
    }
    p->waves = wide ? 2 * kWaves : kWaves;
    int64_t blocks = 0;
    size_t lds = 0;
    for (size_t r = 0; r < p->ranges.size(); ++r) {
        RangeInfo &ri = p->ranges[r];
        const int32_t cap = int32_t(65535 / (255 * ri.ds));
        const int32_t K = std::max(1, std::min(kSubband, cap));
        const int32_t nsub = (nchans + K - 1) / K;
        // pattern rows of at most 64*NW + 64 words (3 words per lane at
        // 256-sample tiles, 5 at 512), whose odd-aligned channels' partial
        // sum reaches one word further: a row's needed words stay below
        // 64*NW + 63, so (spread >> 1) <= 62
        const int32_t max_spread = 2 * (kWave64 - 2) + 1;
        // per DM tile: delay spread, most patterns of a sub-band, widest
        // pattern spread
        const int32_t ntiles = (ri.ndms + dmt - 1) / dmt;
        const size_t nt = size_t(ntiles);
        std::vector<int32_t> t_span(nt, 0), t_j(nt, 0), t_sj(nt, 0);
        parallel_for(ntiles, int64_t(nchans) * dmt, [&](int64_t g0, int64_t g1) {
            SbPatterns pt;
            std::vector<int32_t> order;
            for (int64_t g = g0; g < g1; ++g) {
                const int32_t d0 = int32_t(g) * dmt;
                const int32_t nd = std::min(dmt, ri.ndms - d0);
                const int32_t *s0 = &p->shifts[size_t(ri.dm_index + d0) * nchans];
                const int32_t *s1 = &p->shifts[size_t(ri.dm_index + d0 + nd - 1) * nchans];
                int32_t sp = 0, jm = 0, sj = 0;
                for (int32_t c = 0; c < nchans; ++c)
                    sp = std::max(sp, s1[c] - s0[c]);
                for (int32_t b = 0; b < nsub; ++b) {
                    sb_patterns(*p, ri, d0, nd, b * K, std::min(K, nchans - b * K), max_spread,
                                pt, order);
                    jm = std::max(jm, pt.J);
                    for (int32_t j = 0; j < pt.J; ++j)
                        sj = std::max(sj, pt.amax[j] - pt.amin[j]);
                }
                t_span[size_t(g)] = sp;
                t_j[size_t(g)] = jm;
                t_sj[size_t(g)] = sj;
            }
        });
        int32_t span = 0, jmax = 0, spanJ = 0;
        for (int32_t g = 0; g < ntiles; ++g) {
            span = std::max(span, t_span[size_t(g)]);
            jmax = std::max(jmax, t_j[size_t(g)]);
            spanJ = std::max(spanJ, t_sj[size_t(g)]);
        }
        // 64*NW < Wq <= 64*NW + 64 (NW = T/128 words per lane): the kernel
        // builds a row with NW + 1 words per lane
        const int32_t Wq = ((spanJ >> 1) + T / 2 + 1 + 3) / 4 * 4;
        if (Wq <= T / 2 || Wq > T / 2 + kWave64) {
            *err = fmt("variant 3, range ", r, ": pattern rows of ", Wq, " words");
            return DD_ERR_INVALID;
        }
        const int32_t Wr = (((span + 7) >> 1) + Wq + 1 + 3) / 4 * 4;
        // LDS: two stages of channel windows, the pattern rows of one stage
        // (even and odd copies), and two buffers of stage tables; one
        // workgroup per CU.
        auto slots_for = [&](int32_t st) { return (std::min(st, nchans) + K - 1) / K; };
        auto tb_words = [&](int32_t st) {
            const int32_t n = 4 + (st + 3) / 4 * 4 + slots_for(st) * (dmt + jmax * kSubband);
            return (n + 3) / 4 * 4;
        };
        auto bytes_for = [&](int32_t st) {
            return size_t(4) * (size_t(2) * st * Wr + size_t(slots_for(st)) * jmax * 2 * Wq + 4 +
                                size_t(2) * tb_words(st));
        };
        int32_t stage = std::min(cap >= 2 * K ? 2 * K : K, std::max(K, nchans));
        if (want_stage > 0)
            stage = std::max(K, std::min(stage, want_stage / K * K));
        // (the batch kernel keeps 16 bytes of static LDS beside the dynamic)
        const size_t target = kMaxLdsBytes - 64;
        if (stage > K && bytes_for(stage) > target)
            stage = K;
        if (bytes_for(stage) > target) {
            *err = fmt("variant 3, range ", r, ": ", jmax, " delay patterns per sub-band and a ",
                       span, "-sample delay spread per DM tile need ", bytes_for(stage),
                       " bytes of LDS");
            return DD_ERR_INVALID;
        }
        ri.sb_spread = max_spread;
        ri.sb_chans = K;
        ri.sb_nsub = nsub;
        ri.sb_jmax = jmax;
        ri.sb_span = spanJ;
        ri.sb_qwords = Wq;
        ri.sb_nslot = slots_for(stage);
        ri.sb_tb_words = tb_words(stage);
        ri.span = span;
        ri.row_words = Wr;
        ri.stage_chans = stage;
        ri.widen_every = std::max(1, cap / stage);
        lds = std::max(lds, bytes_for(stage));
        ri.ntime_tiles = (ri.nout + T - 1) / T;
        ri.ndm_tiles = (ri.ndms + dmt - 1) / dmt;
        ri.ndms_pad = ri.ndm_tiles * dmt;
        ri.block_start = blocks;
        blocks += ri.ntime_tiles * ri.ndm_tiles;
    }
    p->blocks = blocks;
    p->lds_bytes = lds;
    build_levels(p);

    size_t nbase = 0, nq = 0, nn = 0, nc = 0;
    for (RangeInfo &ri : p->ranges) {
        ri.base_offset = nbase;
        ri.sb_n_offset = nn;
        ri.sb_q_offset = nq;
        ri.sb_c_offset = nc;
        nbase += size_t(nchans) * ri.ndm_tiles;
        nn += size_t(ri.ndm_tiles) * ri.sb_nsub;
        nq += size_t(ri.ndm_tiles) * ri.sb_nsub * ri.sb_jmax * kSubband;
        nc += size_t(ri.ndm_tiles) * ri.sb_nsub * dmt;
    }
    p->offT.clear();
    p->baseT.assign(nbase, 0);
    p->qcntT.assign(nn, 0);
    p->qoffT.assign(nq, 0);
    p->offCT.assign(nc, 0);
    for (RangeInfo &ri : p->ranges) {
        const int32_t K = ri.sb_chans, S = ri.stage_chans, Wr = ri.row_words, Wq = ri.sb_qwords;
        const int32_t jmax = ri.sb_jmax;
        parallel_for(ri.ndm_tiles, int64_t(nchans) * dmt, [&](int64_t g0, int64_t g1) {
        SbPatterns pt;
        std::vector<int32_t> order;
        for (int32_t g = int32_t(g0); g < int32_t(g1); ++g) {
            const int32_t d0 = g * dmt;
            const int32_t nd = std::min(dmt, ri.ndms - d0);
            int32_t *base = &p->baseT[ri.base_offset + size_t(g) * nchans];
            for (int32_t c = 0; c < nchans; ++c) {
                const int32_t b = p->shifts[size_t(ri.dm_index + d0) * nchans + c];
                base[c] = (b >> 1) - ((b >> 1) & 3);
            }
            for (int32_t sb = 0; sb < ri.sb_nsub; ++sb) {
                const int32_t c0 = sb * K, kb = std::min(K, nchans - c0);
                const int32_t cs = c0 / S * S;            // first channel of the stage
                const int32_t slot = (c0 - cs) / K;
                sb_patterns(*p, ri, d0, nd, c0, kb, ri.sb_spread, pt, order);
                const size_t gb = size_t(g) * ri.sb_nsub + sb;
                p->qcntT[ri.sb_n_offset + gb] = pt.J;
                int32_t *q = &p->qoffT[ri.sb_q_offset + gb * jmax * kSubband];
                for (int32_t j = 0; j < pt.J; ++j) {
                    const int32_t *srep =
                        &p->shifts[size_t(ri.dm_index + d0 + pt.rep[j]) * nchans + c0];
                    // the word holding the first sample of pattern j's row in
                    // channel c0 + k, relative to the channel's staged
                    // window; channels whose first sample is odd come first,
                    // and entry 0 carries their count in bits 24-27
                    int32_t loc[kSubband], nodd = 0;
                    for (int32_t k = 0; k < kb; ++k) {
                        loc[k] = pt.amin[j] + (srep[k] - pt.a[pt.rep[j]]) - 2 * base[c0 + k];
                        nodd += loc[k] & 1;
                    }
                    for (int32_t k = 0, io = 0, ie = nodd; k < kb; ++k) {
                        const int32_t e = (loc[k] & 1) ? io++ : ie++;
                        q[j * kSubband + e] = (c0 + k - cs) * Wr + (loc[k] >> 1);
                    }
                    q[j * kSubband] |= nodd << 24;
                }
                int32_t *oc = &p->offCT[ri.sb_c_offset + gb * dmt];
                for (int32_t d = 0; d < dmt; ++d) {
                    const int32_t j = d < nd ? pt.idx[d] : 0;
                    const int32_t o = d < nd ? pt.a[d] - pt.amin[j] : 0;
                    oc[d] = ((slot * jmax + j) * 2 + (o & 1)) * Wq + (o >> 1);
                }
            }
        }
        });
    }
    // patterns per DM and sub-band, weighted by each range's DM-trial
    // samples; per real DM (the padding DMs of a range's last tile have no
    // patterns and no sums, so they do not dilute the density)
    double wsum = 0, dsum = 0;
    for (const RangeInfo &ri : p->ranges) {
        const size_t n = size_t(ri.ndm_tiles) * ri.sb_nsub;
        double J = 0;
        for (size_t i = 0; i < n; ++i)
            J += p->qcntT[ri.sb_n_offset + i];
        const double w = double(ri.ndms) * double(ri.nout);
        dsum += w * J / (double(ri.ndms) * ri.sb_nsub);
        wsum += w;
    }
    p->sb_density = wsum > 0 ? dsum / wsum : 0;
    return DD_OK;
}

// Integer variants 1 and 2 (the direct sum): windows, stage width and the
// per-DM offset tables.
dd_status build_direct(Plan *p, int32_t want_stage, std::string *err)
{
    const int32_t nchans = p->nchans;
    const int32_t nranges = int32_t(p->ranges.size());
    const dd_dtype dtype = p->dtype;
    const int32_t dmt = p->dm_tile;
    // Tile strategy: a time tile of kTimeTile samples by a DM tile of
    // kDmTile trials per workgroup.  Channels are staged in LDS in groups
    // (double-buffered, two copies each), and the 16-bit partial sums are
    // widened before 65535/(255*ds) channels have been added.
    int64_t blocks = 0;
    size_t lds = 0;
    for (int32_t r = 0; r < nranges; ++r) {
        RangeInfo &ri = p->ranges[r];
        int32_t span = 0;
        for (int32_t d0 = 0; d0 < ri.ndms; d0 += dmt) {
            const int32_t d1 = std::min(ri.ndms, d0 + dmt) - 1;
            const int32_t *s0 = &p->shifts[size_t(ri.dm_index + d0) * nchans];
            const int32_t *s1 = &p->shifts[size_t(ri.dm_index + d1) * nchans];
            for (int32_t c = 0; c < nchans; ++c)
                span = std::max(span, s1[c] - s0[c]);
        }
        ri.span = span;
        const int32_t imax = p->time_tile / 2 + 2 + ((span + 1) >> 1);
        ri.row_words = (imax + 2 + 3) / 4 * 4;
        const int32_t cap = dtype == DD_U8 ? int32_t(65535 / (255 * ri.ds)) : kMaxStageChans;
        int32_t stage = std::max(1, std::min(want_stage > 0 ? want_stage : kMaxStageChans, cap));
        if (stage > 1)
            stage &= ~1;
        auto bytes_for = [&](int32_t st) {
            return size_t(16) * size_t(st) * size_t(ri.row_words);
        };
        // LDS per workgroup that still lets 16 wavefronts share a CU.
        const size_t lds_target = kMaxLdsBytes * size_t(p->waves) / 16 - 1024;
        while (stage > 1 && bytes_for(stage) > lds_target)
            stage = stage > 2 ? stage - 2 : 1;
        if (bytes_for(stage) > kMaxLdsBytes) {
            *err = fmt("range ", r, ": delay spread ", span,
                       " inside one DM tile needs more LDS than a workgroup has; use a "
                       "finer DM step");
            return DD_ERR_INVALID;
        }
        ri.stage_chans = stage;
        ri.widen_every = std::max(1, cap / stage);
        lds = std::max(lds, bytes_for(stage));
        ri.ntime_tiles = (ri.nout + p->time_tile - 1) / p->time_tile;
        ri.ndm_tiles = (ri.ndms + dmt - 1) / dmt;
        ri.ndms_pad = ri.ndm_tiles * dmt;
        ri.block_start = blocks;
        blocks += ri.ntime_tiles * ri.ndm_tiles;
    }
    p->blocks = blocks;
    p->lds_bytes = lds;

    build_levels(p);

    // Device tables of the integer kernel (see plan.h).
    size_t noff = 0, nbase = 0;
    for (RangeInfo &ri : p->ranges) {
        ri.off_offset = noff;
        ri.base_offset = nbase;
        noff += size_t(nchans) * ri.ndms_pad;
        nbase += size_t(nchans) * ri.ndm_tiles;
    }
    p->offT.assign(noff, 0);
    p->baseT.assign(nbase, 0);
    for (RangeInfo &ri : p->ranges) {
        const int32_t copy_words = ri.stage_chans * ri.row_words;
        parallel_for(nchans, ri.ndms_pad, [&](int64_t c0, int64_t c1) {
        for (int32_t c = int32_t(c0); c < int32_t(c1); ++c) {
            int32_t *off = &p->offT[ri.off_offset + size_t(c) * ri.ndms_pad];
            for (int32_t tile = 0; tile < ri.ndm_tiles; ++tile) {
                const int32_t b = p->shifts[size_t(ri.dm_index + tile * dmt) * nchans + c];
                const int32_t par = b & 1;
                const int32_t e = ((b - par) / 2) & 3;
                p->baseT[ri.base_offset + size_t(tile) * nchans + c] = (b - par) / 2 - e;
                for (int32_t d = tile * dmt; d < (tile + 1) * dmt; ++d) {
                    const int32_t dv = std::min(d, ri.ndms - 1);
                    const int32_t o = p->shifts[size_t(ri.dm_index + dv) * nchans + c] - b;
                    off[d] = ((o + par) & 1) * copy_words + e + ((o + par) >> 1);
                }
            }
        }
        });
    }
    return DD_OK;
}

// Drops what a failed variant-3 attempt left in a plan.
void reset_subband(Plan *p)
{
    p->qcntT.clear();
    p->qoffT.clear();
    p->offCT.clear();
    p->baseT.clear();
    p->sb_density = 0;
    for (RangeInfo &ri : p->ranges) {
        ri.sb_spread = ri.sb_chans = ri.sb_nsub = ri.sb_jmax = ri.sb_span = 0;
        ri.sb_qwords = ri.sb_nslot = ri.sb_tb_words = 0;
        ri.sb_q_offset = ri.sb_n_offset = ri.sb_c_offset = 0;
    }
}

dd_status build_plan(const double *freqs, int32_t nchans, double tsamp, int64_t nsamp,
                     const dd_range *ranges, int32_t nranges, dd_dtype dtype,
                     const dd_options *opts, Plan *p, std::string *err)
{
    const int32_t want_variant = opts ? opts->variant : 0;
    const int32_t want_stage = opts ? opts->stage_chans : 0;
    const int32_t want_dm_tile = opts ? opts->dm_tile : 0;
    const int32_t want_time_tile = opts ? opts->time_tile : 0;
    if (want_time_tile != 0 && want_time_tile != kTimeTile / 2 && want_time_tile != kTimeTile) {
        *err = fmt("options: time_tile must be 0, ", kTimeTile / 2, " or ", kTimeTile);
        return DD_ERR_INVALID;
    }
    if (want_variant < 0 || want_variant > 3 || want_stage < 0) {
        *err = "options: variant must be 0 to 3 and stage_chans >= 0";
        return DD_ERR_INVALID;
    }
    const bool direct_tile = want_dm_tile == 32 || want_dm_tile == 64;
    const bool sb_tile = want_dm_tile == 64 || want_dm_tile == 96 || want_dm_tile == 128 ||
                         want_dm_tile == 192;
    const bool tile_ok = want_dm_tile == 0 ||
                         (want_variant == 3   ? sb_tile
                          : want_variant == 0 ? direct_tile || sb_tile
                                              : direct_tile);
    if (!tile_ok) {
        *err = "options: dm_tile must be 32 or 64 (variants 1, 2), 64, 96, 128 or 192 (variant 3), "
               "or any of these (variant 0)";
        return DD_ERR_INVALID;
    }
    if (!freqs || !ranges || !p) {
        *err = "freqs_mhz, ranges and out must not be NULL";
        return DD_ERR_NULL;
    }
    if (dtype != DD_U8 && dtype != DD_F32) {
        *err = fmt("unknown dtype ", int(dtype));
        return DD_ERR_DTYPE;
    }
    if (nchans <= 0) {
        *err = fmt("nchans must be > 0 (got ", nchans, ")");
        return DD_ERR_INVALID;
    }
    if (!finite_pos(tsamp)) {
        *err = "tsamp_s must be finite and > 0";
        return DD_ERR_INVALID;
    }
    if (nsamp <= 0 || nsamp >= (int64_t(1) << 31)) {
        *err = fmt("nsamp must be in [1, 2^31) (got ", nsamp, ")");
        return DD_ERR_INVALID;
    }
    if (nranges <= 0 || nranges > DD_MAX_RANGES) {
        *err = fmt("nranges must be in [1, ", DD_MAX_RANGES, "] (got ", nranges, ")");
        return DD_ERR_INVALID;
    }
    double f_ref = 0.0;
    for (int32_t c = 0; c < nchans; ++c) {
        if (!finite_pos(freqs[c])) {
            *err = fmt("channel ", c, " frequency must be finite and > 0");
            return DD_ERR_INVALID;
        }
        f_ref = std::max(f_ref, freqs[c]);
    }
    int32_t max_ds = 1;
    int64_t ndms_total = 0;
    for (int32_t r = 0; r < nranges; ++r) {
        const dd_range &g = ranges[r];
        if (!std::isfinite(g.dm_lo) || !std::isfinite(g.dm_hi) || !finite_pos(g.dm_step) ||
            g.dm_lo < 0.0 || !(g.dm_hi > g.dm_lo)) {
            *err = fmt("range ", r, ": need finite 0 <= dm_lo < dm_hi and dm_step > 0");
            return DD_ERR_INVALID;
        }
        const double n = std::floor((g.dm_hi - g.dm_lo) / g.dm_step + 0.5);
        if (!(n >= 1.0) || n > double(1 << 24)) {
            *err = fmt("range ", r, ": round((hi - lo)/step) must be in [1, 2^24]");
            return DD_ERR_INVALID;
        }
        if (g.downsample < 1 || (dtype == DD_U8 && g.downsample > 256) ||
            int64_t(g.downsample) > nsamp) {
            *err = fmt("range ", r, ": downsample must be in [1, ",
                       dtype == DD_U8 ? 256 : 1 << 30, "] and <= nsamp");
            return DD_ERR_INVALID;
        }
        max_ds = std::max(max_ds, g.downsample);
        ndms_total += int64_t(n);
    }
    if (dtype == DD_U8 && 255.0 * double(nchans) * double(max_ds) >= 2147483648.0) {
        *err = fmt("255 * nchans * downsample = ", 255.0 * nchans * max_ds,
                   " does not fit int32 output");
        return DD_ERR_OVERFLOW;
    }
    if (double(ndms_total) * double(nchans) > 1.5e9) {
        *err = "shift table larger than 1.5e9 entries";
        return DD_ERR_INVALID;
    }

    try {
        p->nchans = nchans;
        p->tsamp = tsamp;
        p->nsamp = nsamp;
        p->dtype = dtype;
        p->freqs.assign(freqs, freqs + nchans);
        p->dms.clear();
        p->dms.reserve(size_t(ndms_total));
        p->shifts.assign(size_t(ndms_total) * nchans, 0);
        p->ranges.assign(size_t(nranges), RangeInfo{});

        // Per-channel dispersion measure of the band: f_c^-2 - f_ref^-2.
        std::vector<double> delta(static_cast<size_t>(nchans));
        for (int32_t c = 0; c < nchans; ++c)
            delta[c] = 1.0 / (freqs[c] * freqs[c]) - 1.0 / (f_ref * f_ref);

        int64_t out_off = 0;
        int32_t dm_index = 0;
        p->overlap = 0;
        for (int32_t r = 0; r < nranges; ++r) {
            const dd_range &g = ranges[r];
            RangeInfo &ri = p->ranges[r];
            ri.lo = g.dm_lo;
            ri.hi = g.dm_hi;
            ri.step = g.dm_step;
            ri.ds = g.downsample;
            ri.ndms = int32_t(std::floor((g.dm_hi - g.dm_lo) / g.dm_step + 0.5));
            ri.dm_index = dm_index;
            ri.nbin = nsamp / ri.ds;
            for (int32_t i = 0; i < ri.ndms; ++i)
                p->dms.push_back(g.dm_lo + double(i) * g.dm_step);
            // per DM row: its largest delay, or -1 for a delay out of range
            std::vector<int32_t> row_max(size_t(ri.ndms), 0);
            parallel_for(ri.ndms, nchans, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i) {
                    const double dm = p->dms[size_t(dm_index + i)];
                    int32_t *row = &p->shifts[size_t(dm_index + i) * nchans];
                    int32_t m = 0;
                    for (int32_t c = 0; c < nchans; ++c) {
                        const double x = kDispersion * dm * delta[c] / (tsamp * ri.ds);
                        const double s = std::floor(x + 0.5);
                        if (!(s >= 0.0) || s > 2.0e9) {
                            m = -1;
                            break;
                        }
                        row[c] = int32_t(s);
                        m = std::max(m, row[c]);
                    }
                    row_max[size_t(i)] = m;
                }
            });
            int32_t smax = 0;
            for (int32_t i = 0; i < ri.ndms; ++i) {
                if (row_max[size_t(i)] < 0) {
                    *err = fmt("range ", r, ": delay out of range at DM ", p->dms[size_t(dm_index + i)]);
                    return DD_ERR_EMPTY_OUTPUT;
                }
                smax = std::max(smax, row_max[size_t(i)]);
            }
            ri.max_shift = smax;
            ri.nout = ri.nbin - smax;
            if (ri.nout <= 0) {
                *err = fmt("range ", r, ": largest delay ", smax, " leaves no valid sample of ",
                           ri.nbin, " binned samples");
                return DD_ERR_EMPTY_OUTPUT;
            }
            ri.out_offset = out_off;
            out_off += int64_t(ri.ndms) * ri.nout;
            p->overlap = std::max<int64_t>(p->overlap, int64_t(smax) * ri.ds);
            dm_index += ri.ndms;
        }
        p->out_elems = out_off;

        if (dtype == DD_F32) {
            p->dm_tile = kDmTile;
            p->waves = kWaves;
            p->time_tile = kTimeTile;
            // variant 0: sub-band reuse on the problems where it saves at
            // least a third of the work; 1 or 2: direct sums only; 3:
            // sub-band reuse on every problem
            const int32_t sb_mode = want_variant == 0 ? 0 : want_variant == 3 ? 2 : 1;
            return build_f32(p, want_stage, sb_mode, err);
        }
        auto use = [&](int32_t variant, int32_t dm_tile, std::string *e) {
            p->dedup = variant == 2;
            p->subband = variant == 3;
            p->dm_tile = dm_tile;
            p->waves = dm_tile / kDmPerWave;
            // variant 3 at 192- and 128-DM tiles: 256-sample tiles; else the
            // requested time tile, by default 512, or for the direct kernel
            // 256 when 512-sample tiles would leave fewer than
            // kMinWorkgroups workgroups (a small plan then fills the GPU
            // with twice as many)
            int64_t wg512 = 0;
            for (const RangeInfo &ri : p->ranges)
                wg512 += (ri.nout + kTimeTile - 1) / kTimeTile * ((ri.ndms + dm_tile - 1) / dm_tile);
            p->time_tile = want_time_tile                     ? want_time_tile
                           : (variant == 3 && dm_tile >= 128) ? kTimeTile / 2
                           : variant != 3 && wg512 < kMinWorkgroups ? kTimeTile / 2
                                                              : kTimeTile;
            return p->subband ? build_subband(p, want_stage, e) : build_direct(p, want_stage, e);
        };
        if (want_variant != 0)
            return use(want_variant,
                       want_dm_tile ? want_dm_tile : (want_variant == 3 ? 3 * kDmTile : kDmTile), err);
        // Variant 0: exact sub-band reuse (192-DM tiles, then 128) when the
        // plan's delay patterns fit the LDS and are few enough per DM to pay
        // (smaller tiles only hold more patterns per DM), else the direct
        // kernel.
        std::vector<int32_t> tiles;
        if (want_dm_tile == 0)
            tiles = {3 * kDmTile, 2 * kDmTile};
        else if (want_dm_tile != kDmTile / 2)
            tiles = {want_dm_tile};
        for (int32_t t : tiles) {
            std::string e;
            const dd_status st = use(3, t, &e);
            if (st == DD_OK && p->sb_density > kMaxPatternDensity)
                break;
            if (st != DD_ERR_INVALID) {
                if (st != DD_OK)
                    *err = e;
                return st;
            }
        }
        reset_subband(p);
        return use(1, want_dm_tile == kDmTile / 2 ? want_dm_tile : kDmTile, err);
    } catch (const std::bad_alloc &) {
        *err = "host allocation failed";
        return DD_ERR_NOMEM;
    }
    return DD_OK;
}

}  // namespace dd
