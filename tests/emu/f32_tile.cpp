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

template <class SFn>
static long emulate(const Plan &P, const SumProblem &sp, const std::vector<float> &src,
                    long src0, long pitch, SFn S, int block_stride, const char *name)
{
    const int C = sp.stage_rows, Wr = sp.row_words, nst = sp.nstages, nrows = sp.nrows;
    const long lds_floats = long(P.dtype == DD_F32 ? std::max(P.lds_bytes, P.adj_lds_bytes) : 0) / 4;
    const int TS = sp.tab_stride;
    CHECK(TS % 4 == 0 && TS >= C + 1, "[%s] list stride %d for %d rows", name, TS, C);
    CHECK(long(C) * Wr + long(kF32OutTile) * TS + 16 <= lds_floats,
          "[%s] stage buffer (%d x %d rows + lists) past LDS %ld", name, C, Wr, lds_floats);
    CHECK(sp.off_offset % 4 == 0, "[%s] lists not 16-byte aligned", name);
    CHECK(Wr % 4 == 0, "[%s] row_words %d", name, Wr);
    CHECK(nst == (nrows + C - 1) / C, "[%s] nstages", name);
    const long nblocks = sp.ntime_tiles * sp.nout_tiles;
    long checked = 0;
    std::vector<float> lds(size_t(C) * Wr);
    std::vector<int> tag(size_t(C) * Wr);
    for (long lb = 0; lb < nblocks; lb = lb + block_stride < nblocks ? lb + block_stride : (lb == nblocks - 1 ? nblocks : nblocks - 1)) {
        const long tt = lb / sp.nout_tiles;
        const int tile = int(lb - tt * sp.nout_tiles);
        const long t0 = tt * kF32TimeTile;
        std::vector<double> acc(size_t(kF32OutTile) * 64 * kF32Words, 0.0);
        for (int st = 0; st < nst; ++st) {
            const int b0 = st * C, bn = std::min(C, nrows - b0);
            const long buf = 0;              // one stage buffer, refilled each stage
            std::fill(tag.begin() + buf, tag.begin() + buf + long(C) * Wr, -1);
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
                    lds[buf + long(j) * Wr + q] = (gi >= 0 && gi < long(src.size())) ? src[gi] : NAN;
                    tag[buf + long(j) * Wr + q] = b0 + j;
                }
            }
            for (int al = 0; al < kF32OutTile; ++al) {
                const int a = tile * kF32OutTile + al;
                const int av = std::min(a, sp.nouts - 1);
                // the stage's lists are staged whole ([nstages][outputs][TS] per
                // tile); each output reads 16 words of its list and its last
                // word (the LDS block holds 16 words past the last list)
                const size_t block = (size_t(tile) * nst + st) * kF32OutTile * TS;
                CHECK(sp.off_offset + block + size_t(kF32OutTile) * TS <= P.offF.size(),
                      "[%s] list block past offF", name);
                CHECK(al * TS + 16 <= kF32OutTile * TS + 16, "[%s] list read past the LDS block", name);
                const size_t list = sp.off_offset + block + size_t(al) * TS;
                const uint32_t ends = uint32_t(P.offF[list + TS - 1]);
                int e[4] = {int(ends & 0xFF), int((ends >> 8) & 0xFF), int((ends >> 16) & 0xFF), int(ends >> 24)};
                CHECK(e[0] <= e[1] && e[1] <= e[2] && e[2] <= e[3] && e[3] == bn, "[%s] class ends %d %d %d %d bn %d", name, e[0], e[1], e[2], e[3], bn);
                std::vector<int> seen(bn, 0);
                int i = 0;
                for (int cls = 0; cls < 4; ++cls)
                    for (; i < e[cls]; ++i) {
                        const int ent = P.offF[list + i];
                        const int slot = ent / Wr, q4 = ent - slot * Wr;
                        CHECK(slot >= 0 && slot < bn && q4 % 4 == 0, "[%s] entry %d", name, ent);
                        if (!(slot >= 0 && slot < bn)) continue;
                        seen[slot]++;
                        const int b = b0 + slot;
                        const int m = P.baseF[sp.base_offset + size_t(tile) * nrows + b];
                        const int o = q4 + cls;      // delay in the window
                        CHECK(m + o == S(av, b), "[%s] a %d b %d: window %d + %d != delay %d", name, av, b, m, o, S(av, b));
                        // the lanes' granules
                        double gr[64][kF32Words / 4][4];
                        for (int l = 0; l < 64; ++l)
                            for (int k = 0; k < kF32Words / 4; ++k)
                                for (int j = 0; j < 4; ++j) {
                                    const long li = buf + ent + 4 * (l + 63 * k) + j;
                                    CHECK(li >= buf && li < buf + long(C) * Wr, "[%s] LDS read %ld", name, li);
                                    const bool in_row = li < buf + long(slot + 1) * Wr;
                                    // lanes 0..62 use every value they read; lane 63 only
                                    // supplies heads to lane 62
                                    if (l < 63 || j < cls) {
                                        CHECK(in_row, "[%s] read past its row window (lane %d)", name, l);
                                        CHECK(tag[li] == b, "[%s] LDS word of row %d, want %d", name, tag[li], b);
                                    }
                                    gr[l][k][j] = lds[li];
                                }
                        for (int l = 0; l < 64; ++l)
                            for (int k = 0; k < kF32Words / 4; ++k)
                                for (int j = 0; j < 4; ++j) {
                                    double v;
                                    if (j + cls < 4) v = gr[l][k][j + cls];
                                    else v = l < 63 ? gr[l + 1][k][j + cls - 4] : 0.0;
                                    acc[(size_t(al) * 64 + l) * kF32Words + 4 * k + j] += v;
                                }
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
               int stage, int seed, int block_stride, const char *name)
{
    Plan P; std::string err;
    dd_options o{0, stage, 0};
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
        printf("[%s] range %zu: stage %d/%d rows %d/%d, row words %d/%d, checked %ld + %ld outputs\n", name, r,
               R.fwd.stage_rows, R.adj.stage_rows, R.fwd.nrows, R.adj.nrows, R.fwd.row_words, R.adj.row_words, c1, c2);
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
    printf("plans %d of %d, fails %ld\n", ok, tried, fails);
    return fails ? 1 : 0;
}
