// CPU emulation of the float32 shift-and-sum tile (k_shiftsum_f32, output
// epilogue) on the host tables of float32 plans: forward problems (rows =
// binned input) and adjoint problems (rows = zero-padded gradient rows).
// It follows the kernel's lane layout -- lane l reads the 16-byte granules
// l and l + 63 of a row window at each output's delay, a delay that is not a
// multiple of 4 takes the granule head from lane l + 1 (lane 63 gets 0) --
// and checks every LDS and global index, the class lists (each stage row
// once per output, in class order, classes matching the delay), and every
// output of lanes 0..62 against the direct sum (integer-valued inputs, so
// the float sums are exact in any order).
#include "plan.h"
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <random>
#include <vector>
#include <algorithm>
using namespace dd;

static long fails = 0;
#define CHECK(c, ...)                                                   \
    do {                                                                \
        if (!(c)) {                                                     \
            if (fails++ < 30) {                                         \
                printf("FAIL %s:%d: ", __FILE__, __LINE__);             \
                printf(__VA_ARGS__);                                    \
                printf("\n");                                           \
            }                                                           \
        }                                                               \
    } while (0)

// The window sums of one entry as the kernel's lanes form them: lane l
// reads G granules at ent + 4*(l + 63g) of the stage buffer; a class-r
// entry takes floats r..3 of the lane's granule and the first r of lane
// l + 1's (lane 63 gets 0).  Values lanes 0..62 use (and lane 63's heads)
// must lie inside [lo, hi) and carry tag `want` (or any tag >= 0 when want
// is -1).
static void lane_windows(const std::vector<float> &lds, const std::vector<int> &tag, long lo, long hi,
                         int ent, int cls, int G, int want, double (*out)[20], const char *name,
                         const char *what)
{
    static double gr[64][5][4];
    for (int l = 0; l < 64; ++l)
        for (int k = 0; k < G; ++k)
            for (int j = 0; j < 4; ++j) {
                const long li = long(ent) + 4 * (l + 63 * k) + j;
                const bool used = l < 63 || j < cls;
                CHECK(li >= 0 && li < long(lds.size()), "[%s] %s: LDS read %ld of %zu", name, what, li, lds.size());
                if (used) {
                    CHECK(li >= lo && li < hi, "[%s] %s: read %ld outside [%ld, %ld) (lane %d)", name, what, li, lo, hi, l);
                    if (li >= 0 && li < long(tag.size()))
                        CHECK(want == -1 ? tag[li] >= 0 : tag[li] == want, "[%s] %s: word %ld tagged %d, want %d", name,
                              what, li, tag[li], want);
                }
                gr[l][k][j] = (li >= 0 && li < long(lds.size())) ? lds[li] : NAN;
            }
    for (int l = 0; l < 64; ++l)
        for (int k = 0; k < G; ++k)
            for (int j = 0; j < 4; ++j)
                out[l][4 * k + j] = j + cls < 4 ? gr[l][k][j + cls] : (l < 63 ? gr[l + 1][k][j + cls - 4] : 0.0);
}

template <class SFn>
static long emulate(const Plan &P, const SumProblem &sp, const std::vector<float> &src,
                    long src0, long pitch, SFn S, int block_stride, const char *name)
{
    const int C = sp.stage_rows, Wr = sp.row_words, nst = sp.nstages, nrows = sp.nrows;
    const long lds_floats = long(P.dtype == DD_F32 ? std::max(P.lds_bytes, P.adj_lds_bytes) : 0) / 4;
    const int TS = sp.tab_stride;
    const long rows_end = long(C) * Wr, pat_end = rows_end + long(sp.npat) * kSbPatWords;
    CHECK(TS % 4 == 0 && TS >= 2, "[%s] list stride %d", name, TS);
    CHECK(sp.tab_block % 4 == 0 && sp.tab_block == kF32OutTile * TS + (sp.npat ? kSbJobInts * sp.njobs_max + 4 : 0),
          "[%s] table block %d", name, sp.tab_block);
    CHECK(pat_end + sp.tab_block + 16 <= lds_floats, "[%s] stage buffer (%d x %d rows, %d patterns, %d table ints) past LDS %ld",
          name, C, Wr, sp.npat, sp.tab_block, lds_floats);
    CHECK(sp.off_offset % 4 == 0, "[%s] tables not 16-byte aligned", name);
    CHECK(Wr % 4 == 0, "[%s] row_words %d", name, Wr);
    CHECK(nst == (nrows + C - 1) / C, "[%s] nstages", name);
    CHECK(sp.off_offset + size_t(sp.nout_tiles) * nst * sp.tab_block <= P.offF.size(), "[%s] tables past offF", name);
    const long nblocks = sp.ntime_tiles * sp.nout_tiles;
    long checked = 0;
    // the stage buffer: rows, then pattern rows (tags: row b, or -2 - slot)
    std::vector<float> lds(static_cast<size_t>(pat_end));
    std::vector<int> tag(static_cast<size_t>(pat_end));
    static double win[64][20];
    for (long lb = 0; lb < nblocks; lb = lb + block_stride < nblocks ? lb + block_stride : (lb == nblocks - 1 ? nblocks : nblocks - 1)) {
        const long tt = lb / sp.nout_tiles;
        const int tile = int(lb - tt * sp.nout_tiles);
        const long t0 = tt * kF32TimeTile;
        std::vector<double> acc(size_t(kF32OutTile) * 64 * kF32Words, 0.0);
        for (int st = 0; st < nst; ++st) {
            const int b0 = st * C, bn = std::min(C, nrows - b0);
            std::fill(tag.begin(), tag.end(), -1);
            for (int j = 0; j < bn; ++j) {
                const size_t bi = sp.base_offset + size_t(tile) * nrows + b0 + j;
                CHECK(bi < P.baseF.size(), "[%s] baseF index", name);
                const int m = P.baseF[bi];
                CHECK(m % 4 == 0 && m >= 0, "[%s] window start %d", name, m);
                const long g = src0 + long(b0 + j) * pitch + t0 + m;
                CHECK(g % 4 == 0, "[%s] window not 16-byte aligned", name);
                for (int q = 0; q < Wr; ++q) {
                    const long gi = g + q;
                    CHECK(gi >= 0 && gi < long(src.size()), "[%s] window load %ld of %zu (row %d)", name, gi, src.size(), b0 + j);
                    lds[long(j) * Wr + q] = (gi >= 0 && gi < long(src.size())) ? src[gi] : NAN;
                    tag[long(j) * Wr + q] = b0 + j;
                }
            }
            const int32_t *blk = &P.offF[sp.off_offset + (size_t(tile) * nst + st) * sp.tab_block];
            // level 1: pattern rows from the jobs
            std::vector<std::vector<int>> pat_rows(static_cast<size_t>(sp.npat));
            if (sp.npat) {
                const int32_t *jobs = blk + kF32OutTile * TS;
                const int nj = jobs[kSbJobInts * sp.njobs_max];
                CHECK(nj >= 0 && nj <= sp.njobs_max, "[%s] %d jobs", name, nj);
                for (int jb = 0; jb < nj; ++jb) {
                    const int32_t *J = jobs + kSbJobInts * jb;
                    const int dest = J[0], G = J[1];
                    const uint32_t ends = uint32_t(J[2]);
                    const int pslot = (dest - int(rows_end)) / kSbPatWords;
                    const int pbase = int(rows_end) + pslot * kSbPatWords;
                    CHECK(G == 5, "[%s] job %d granules %d", name, jb, G);
                    CHECK(pslot >= 0 && pslot < sp.npat && dest == pbase, "[%s] job %d destination %d", name, jb, dest);
                    if (!(pslot >= 0 && pslot < sp.npat) || G != 5) continue;
                    int e[4] = {int(ends & 0xFF), int((ends >> 8) & 0xFF), int((ends >> 16) & 0xFF), int(ends >> 24)};
                    CHECK(e[0] <= e[1] && e[1] <= e[2] && e[2] <= e[3] && e[3] >= 1 && e[3] <= kSbGroup,
                          "[%s] job class ends %d %d %d %d", name, e[0], e[1], e[2], e[3]);
                    std::vector<double> pr(size_t(64) * 20, 0.0);
                    std::vector<int> rows_of;
                    int i = 0;
                    for (int cls = 0; cls < 4; ++cls)
                        for (; i < e[cls]; ++i) {
                            const int ent = J[3 + i];
                            const int slot = ent / Wr;
                            CHECK(slot >= 0 && slot < bn && ent % 4 == 0, "[%s] job entry %d", name, ent);
                            if (!(slot >= 0 && slot < bn)) continue;
                            rows_of.push_back(slot);
                            lane_windows(lds, tag, long(slot) * Wr, long(slot + 1) * Wr, ent, cls, G, b0 + slot, win,
                                         name, "level 1");
                            for (int l = 0; l < 64; ++l)
                                for (int k = 0; k < 4 * G; ++k)
                                    pr[size_t(l) * 20 + k] += win[l][k];
                        }
                    std::sort(rows_of.begin(), rows_of.end());
                    CHECK(pat_rows[size_t(pslot)].empty(), "[%s] pattern %d built twice", name, pslot);
                    pat_rows[size_t(pslot)] = rows_of;
                    for (int l = 0; l < 63; ++l)
                        for (int k = 0; k < G; ++k)
                            for (int j = 0; j < 4; ++j) {
                                const long li = long(dest) + 4 * (l + 63 * k) + j;
                                CHECK(li >= pbase && li < pbase + kSbPatWords, "[%s] pattern write %ld", name, li);
                                if (li >= pbase && li < pbase + kSbPatWords) {
                                    lds[li] = float(pr[size_t(l) * 20 + 4 * k + j]);
                                    tag[li] = -2 - pslot;
                                }
                            }
                }
            }
            // level 2: every output's list
            for (int al = 0; al < kF32OutTile; ++al) {
                const int a = tile * kF32OutTile + al;
                const int av = std::min(a, sp.nouts - 1);
                const int32_t *list = blk + al * TS;
                CHECK(al * TS + 16 <= kF32OutTile * TS + 16, "[%s] list read past the LDS block", name);
                const uint32_t ends = uint32_t(list[TS - 1]);
                int e[4] = {int(ends & 0xFF), int((ends >> 8) & 0xFF), int((ends >> 16) & 0xFF), int(ends >> 24)};
                CHECK(e[0] <= e[1] && e[1] <= e[2] && e[2] <= e[3] && e[3] <= bn && e[3] <= TS - 1 && e[3] <= 16,
                      "[%s] class ends %d %d %d %d bn %d", name, e[0], e[1], e[2], e[3], bn);
                std::vector<int> seen(bn, 0);
                int i = 0;
                for (int cls = 0; cls < 4; ++cls)
                    for (; i < e[cls]; ++i) {
                        const int ent = list[i];
                        CHECK(ent >= 0 && ent % 4 == 0 && ent < pat_end, "[%s] entry %d", name, ent);
                        if (!(ent >= 0 && ent < pat_end)) continue;
                        if (ent < rows_end) {
                            const int slot = ent / Wr, q4 = ent - slot * Wr;
                            if (slot >= bn) { CHECK(false, "[%s] entry row %d of %d", name, slot, bn); continue; }
                            seen[slot]++;
                            const int b = b0 + slot;
                            const int m = P.baseF[sp.base_offset + size_t(tile) * nrows + b];
                            CHECK(m + q4 + cls == S(av, b), "[%s] a %d b %d: window %d + %d != delay %d", name, av, b, m,
                                  q4 + cls, S(av, b));
                            lane_windows(lds, tag, long(slot) * Wr, long(slot + 1) * Wr, ent, cls, kF32Words / 4, b, win,
                                         name, "level 2 row");
                        } else {
                            const int pslot = int((ent - rows_end) / kSbPatWords);
                            const long pb = rows_end + long(pslot) * kSbPatWords;
                            for (int r : pat_rows[size_t(pslot)])
                                seen[r]++;
                            lane_windows(lds, tag, pb, pb + kSbPatWords, ent, cls, kF32Words / 4, -2 - pslot, win,
                                         name, "level 2 pattern");
                        }
                        for (int l = 0; l < 64; ++l)
                            for (int k = 0; k < kF32Words; ++k)
                                acc[(size_t(al) * 64 + l) * kF32Words + k] += win[l][k];
                    }
                for (int j = 0; j < bn; ++j)
                    CHECK(seen[j] == 1, "[%s] row %d of stage %d seen %d times by output %d", name, j, st, seen[j], a);
            }
        }
        // outputs of lanes 0..62 against the direct sum
        for (int al = 0; al < kF32OutTile; ++al) {
            const int a = tile * kF32OutTile + al;
            if (a >= sp.nouts) continue;
            for (int l = 0; l < 63; ++l)
                for (int k = 0; k < kF32Words / 4; ++k)
                    for (int j = 0; j < 4; ++j) {
                        const long t = t0 + 4 * (l + 63 * k) + j;
                        if (t >= sp.nt) continue;
                        double want = 0;
                        for (int b = 0; b < nrows; ++b) {
                            const long gi = src0 + long(b) * pitch + t + S(a, b);
                            want += src[gi];
                        }
                        const double got = acc[(size_t(al) * 64 + l) * kF32Words + 4 * k + j];
                        CHECK(got == want, "[%s] a %d t %ld: %g != %g", name, a, t, got, want);
                        ++checked;
                    }
        }
    }
    return checked;
}

static int run(const std::vector<double> &freqs, double tsamp, long nsamp, const std::vector<dd_range> &rg,
               int stage, int seed, int block_stride, const char *name, int variant = 0)
{
    Plan P; std::string err;
    dd_options o{variant, stage, 0, 0};
    dd_status st = build_plan(freqs.data(), int(freqs.size()), tsamp, nsamp, rg.data(), int(rg.size()), DD_F32, &o, &P, &err);
    if (st != DD_OK) { printf("[%s] plan: %d %s\n", name, int(st), err.c_str()); return 0; }
    const int nch = P.nchans;
    std::mt19937 gen(seed);
    std::uniform_int_distribution<int> u(-8, 8);
    std::vector<float> x(size_t(nch) * nsamp);
    for (auto &v : x) v = float(u(gen));
    long total = 0;
    for (size_t r = 0; r < P.ranges.size(); ++r) {
        const RangeInfo &R = P.ranges[r];
        const BinLevel &lv = P.levels[R.level];
        // the level buffer: lead, rows of pitch, tail; padding holds a value
        // that would spoil any sum it entered
        std::vector<float> lev(lv.bytes / 4, 1e30f);
        for (int c = 0; c < nch; ++c)
            for (long t = 0; t < lv.nbin; ++t) {
                float s = 0;
                for (int k = 0; k < lv.ds; ++k) s += x[size_t(c) * nsamp + t * lv.ds + k];
                lev[lv.lead + size_t(c) * lv.pitch + t] = s;
            }
        const int32_t *sh = &P.shifts[size_t(R.dm_index) * nch];
        auto Sf = [&](int a, int b) { return sh[size_t(a) * nch + b]; };
        char nm[128];
        snprintf(nm, sizeof nm, "%s fwd r%zu", name, r);
        long c1 = emulate(P, R.fwd, lev, lv.lead, lv.pitch, Sf, block_stride, nm);
        // adjoint rows: the gradient with max_shift zeros in front, zeros after
        std::vector<float> gp(size_t(R.ndms) * R.gpitch, 0.0f);
        for (int d = 0; d < R.ndms; ++d)
            for (long t = 0; t < R.nout; ++t) gp[size_t(d) * R.gpitch + R.max_shift + t] = float(u(gen));
        const int Pm = R.max_shift;
        auto Sa = [&](int a, int b) { return Pm - sh[size_t(b) * nch + a]; };
        snprintf(nm, sizeof nm, "%s adj r%zu", name, r);
        long c2 = emulate(P, R.adj, gp, 0, R.gpitch, Sa, block_stride, nm);
        printf("[%s] range %zu: stage %d/%d rows %d/%d, row words %d/%d, patterns %d/%d, checked %ld + %ld outputs\n",
               name, r, R.fwd.stage_rows, R.adj.stage_rows, R.fwd.nrows, R.adj.nrows, R.fwd.row_words, R.adj.row_words,
               R.fwd.npat, R.adj.npat, c1, c2);
        total += c1 + c2;
    }
    return total > 0;
}

static std::vector<double> band(double top, double bottom, int n) {
    std::vector<double> f(n);
    for (int c = 0; c < n; ++c) f[c] = top - c * (top - bottom) / n;
    return f;
}

int main(int argc, char **argv)
{
    (void)argc; (void)argv;
    int ok = 0, tried = 0;
    ++tried; ok += run(band(1500, 1200, 100), 2.56e-4, 3000, {{0, 20, 1, 1}, {20, 60, 2, 3}}, 0, 1, 1, "small");
    ++tried; ok += run(band(1500, 1200, 37), 2.56e-4, 1500, {{0, 9, 1, 1}}, 4, 2, 1, "odd stage");
    ++tried; ok += run(band(1500, 1200, 1), 2.56e-4, 2000, {{0, 5, 1, 1}}, 0, 3, 1, "one channel");
    ++tried; ok += run(band(1450, 1300, 64), 1e-3, 5000, {{0, 70, 1, 1}, {70, 100, 1, 2}}, 6, 4, 1, "wide");
    ++tried; ok += run(band(1500, 1200, 1024), 1.28e-4, 1 << 14, {{0, 512, 1, 1}}, 0, 5, 7, "diff 1024ch");
    std::vector<double> rnd; std::mt19937 g(9);
    for (int c = 0; c < 77; ++c) rnd.push_back(1200 + 300 * std::uniform_real_distribution<double>(0, 1)(g));
    ++tried; ok += run(rnd, 2.56e-4, 4000, {{0, 33, 1, 1}, {33, 40, 0.5, 2}}, 0, 6, 1, "permuted");
    // direct sums only (variant 1) and sub-band reuse on every problem (3)
    ++tried; ok += run(band(1500, 1200, 100), 2.56e-4, 3000, {{0, 20, 1, 1}, {20, 60, 2, 3}}, 0, 7, 1, "small sb", 3);
    ++tried; ok += run(band(1500, 1200, 37), 2.56e-4, 1500, {{0, 9, 1, 1}}, 0, 8, 1, "odd sb", 3);
    ++tried; ok += run(band(1500, 1200, 1024), 1.28e-4, 1 << 14, {{0, 512, 1, 1}}, 0, 9, 7, "diff direct", 1);
    ++tried; ok += run(band(1500, 1200, 1024), 1.28e-4, 1 << 14, {{0, 512, 1, 1}}, 0, 10, 7, "diff sb", 3);
    ++tried; ok += run(rnd, 2.56e-4, 4000, {{0, 33, 1, 1}, {33, 40, 0.5, 2}}, 0, 11, 1, "permuted sb", 3);
    ++tried; ok += run(band(1670, 1370, 4096), 6.4e-5, 1 << 13, {{0, 200, 1, 1}}, 0, 12, 13, "4096ch sb", 3);
    printf("plans %d of %d, fails %ld\n", ok, tried, fails);
    // random plans: band, sampling, length, one to three ranges of random
    // step and downsample, any strategy; a plan the library rejects (its
    // patterns do not fit, or no output is left) is counted, not failed
    std::mt19937 fz(20240611);
    auto uni = [&](double a, double b) { return std::uniform_real_distribution<double>(a, b)(fz); };
    auto pick = [&](int a, int b) { return std::uniform_int_distribution<int>(a, b)(fz); };
    int fuzz_ok = 0;
    const int fuzz_n = 24;
    for (int i = 0; i < fuzz_n; ++i) {
        const int nch = pick(1, 160);
        const double top = uni(1300, 1700);
        std::vector<double> f = band(top, top - uni(50, 400), nch);
        if (i % 3 == 1) std::shuffle(f.begin(), f.end(), fz);
        const double ts[4] = {6.4e-5, 1.28e-4, 2.56e-4, 1e-3};
        const double tsamp = ts[pick(0, 3)];
        const long nsamp = pick(1500, 6000);
        std::vector<dd_range> rg;
        double lo = 0;
        for (int r = pick(1, 3); r > 0; --r) {
            const double steps[4] = {0.25, 0.5, 1.0, 2.0};
            const double step = steps[pick(0, 3)];
            const double hi = lo + step * pick(3, 60);
            rg.push_back(dd_range{lo, hi, step, pick(1, 4)});
            lo = hi;
        }
        const int variants[3] = {0, 1, 3};
        const int variant = variants[i % 3];
        const int stage = i % 4 == 3 ? pick(1, 14) : 0;
        char nm[64];
        snprintf(nm, sizeof nm, "fuzz %d v%d", i, variant);
        fuzz_ok += run(f, tsamp, nsamp, rg, stage, 100 + i, 2, nm, variant);
    }
    printf("fuzz plans %d of %d accepted, fails %ld\n", fuzz_ok, fuzz_n, fails);
    return fails ? 1 : 0;
}
