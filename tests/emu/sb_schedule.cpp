// CPU emulation of the sub-band shift-and-sum tile (k_dedisp_u8_sb in
// dedisp.hip) on the host tables of variant-3 plans.  It follows the
// kernel's stage schedule -- direct loads of one stage's channel windows and
// tables, a wait and a barrier, the pattern rows (odd-aligned channels
// summed apart and realigned once), a barrier, the next stage's loads, the
// DM sums -- and checks:
//   * every LDS index against the plan's LDS size and every global index
//     against its table or binned level;
//   * that every LDS word a needed result reads was written for it (a tag
//     per stage) and, for direct loads, has landed (a wait and a barrier
//     since its issue);
//   * that no LDS word is written and read in the same phase (between two
//     barriers) by different wavefronts;
//   * that every output equals the direct sum over the shift table.
// Reads whose values are never used (lanes past the row or the output) are
// checked for bounds only.
#include "plan.h"
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include <algorithm>
using namespace dd;

static int fails = 0;
static long nodd_hist[9];
#define CHECK(c, ...)                                                                  \
    do {                                                                               \
        if (!(c)) {                                                                    \
            if (fails++ < 30) {                                                        \
                printf("FAIL %s:%d: ", __FILE__, __LINE__);                            \
                printf(__VA_ARGS__);                                                   \
                printf("\n");                                                          \
            }                                                                          \
        }                                                                              \
    } while (0)

struct Lds {
    std::vector<uint32_t> v; std::vector<int> tag, wph, rph; std::vector<char> pend;
    std::vector<long> pending;
    Lds(size_t n) : v(n, 0xDEADBEEF), tag(n, -1), wph(n, -1000), rph(n, -1000), pend(n, 0) {}
    bool ok(long i, const char *what) {
        bool g = i >= 0 && size_t(i) < v.size();
        CHECK(g, "%s LDS index %ld of %zu", what, i, v.size());
        return g;
    }
    void dma(long i, uint32_t x, int ph, int tg, const char *what) {
        if (!ok(i, what)) return;
        CHECK(rph[i] != ph, "%s: direct load to word %ld read in the same phase %d", what, i, ph);
        CHECK(!pend[i], "%s: word %ld already has a load in flight", what, i);
        v[i] = x; tag[i] = tg; wph[i] = ph; pend[i] = 1; pending.push_back(i);
    }
    void st(long i, uint32_t x, int ph, int tg, const char *what) {
        if (!ok(i, what)) return;
        CHECK(rph[i] != ph, "%s: write to word %ld read in the same phase %d", what, i, ph);
        CHECK(!pend[i], "%s: write to word %ld with a load in flight", what, i);
        v[i] = x; tag[i] = tg; wph[i] = ph;
    }
    uint32_t rd(long i, int ph, int tg, const char *what) {
        if (!ok(i, what)) return 0;
        CHECK(!pend[i], "%s: read of word %ld whose load has not landed (phase %d)", what, i, ph);
        CHECK(wph[i] < ph, "%s: read of word %ld written in the same phase %d", what, i, ph);
        CHECK(tag[i] == tg, "%s: word %ld has tag %d, want %d (phase %d)", what, i, tag[i], tg, ph);
        rph[i] = ph;
        return v[i];
    }
    uint32_t rd_any(long i, int ph, const char *what) {
        if (!ok(i, what)) return 0;
        return v[i];      // (its value is not used: a race with a write is harmless)
    }
    void wait_all() { for (long i : pending) pend[i] = 0; pending.clear(); }
};

static uint32_t alignbyte(uint32_t hi, uint32_t lo, int sh) {
    uint64_t x = (uint64_t(hi) << 32) | lo; return uint32_t(x >> (8 * sh));
}

enum { TAG_WIN = 1000000, TAG_TAB = 2000000, TAG_Q = 3000000 };

static int g_time_tile = 0;     // the time tile the runs ask for (0 = the tile's default)

int run(const std::vector<double> &freqs, double tsamp, int64_t nsamp, const std::vector<dd_range> &rg,
        int dm_tile, int stage, int seed, int block_stride, const char *name)
{
    Plan P; std::string err;
    dd_options o{3, stage, dm_tile, g_time_tile};
    dd_status stt = build_plan(freqs.data(), int(freqs.size()), tsamp, nsamp, rg.data(), int(rg.size()), DD_U8, &o, &P, &err);
    if (stt != DD_OK) { printf("[%s] plan: %d %s\n", name, int(stt), err.c_str()); return 0; }
    const int nch = P.nchans;
    std::mt19937 gen(seed);
    std::vector<uint8_t> x(size_t(nch) * nsamp);
    for (auto &v : x) v = uint8_t(gen());
    std::vector<std::vector<uint16_t>> lev(P.levels.size());
    for (size_t l = 0; l < P.levels.size(); ++l) {
        const BinLevel &lv = P.levels[l];
        lev[l].assign(lv.bytes / 2, 0xA5A5);
        for (int c = 0; c < nch; ++c)
            for (int64_t t = 0; t < lv.nbin; ++t) {
                uint32_t s = 0;
                for (int k = 0; k < lv.ds; ++k) s += x[size_t(c) * nsamp + t * lv.ds + k];
                lev[l][size_t(c) * lv.pitch + t] = uint16_t(s);
            }
    }
    const size_t ldsw = P.lds_bytes / 4;
    CHECK(P.lds_bytes <= kMaxLdsBytes - 64, "[%s] lds %zu", name, P.lds_bytes);
    int64_t checked = 0, mism = 0;
    for (size_t r = 0; r < P.ranges.size(); ++r) {
        const RangeInfo &R = P.ranges[r];
        const BinLevel &lv = P.levels[R.level];
        const std::vector<uint16_t> &L = lev[R.level];
        const int64_t Ln = int64_t(L.size());
        const int C = R.stage_chans, Wr = R.row_words, CW = C * Wr, K = R.sb_chans, Wq = R.sb_qwords;
        const int jmax = R.sb_jmax, nsub = R.sb_nsub, DT = P.dm_tile;
        const int NW = P.time_tile / 128, NQ = NW + 1, TT = P.time_tile;
        const int nst = (nch + C - 1) / C;
        const int nslot = R.sb_nslot;
        CHECK(nslot == 1 || nslot == 2, "nslot %d", nslot);
        CHECK(Wq > 64 * NW && Wq <= 64 * NQ, "[%s] Wq %d NW %d", name, Wq, NW);
        const long Qb = 2L * CW;
        const long Tb = Qb + long(nslot) * jmax * 2 * Wq + 4;
        const int offc = 4 + ((C + 3) & ~3), qoffs = offc + nslot * DT, tbw = R.sb_tb_words;
        const int ntb = 2;
        CHECK(Tb + long(ntb) * tbw <= long(ldsw), "[%s] tables past LDS: %ld + %d*%d > %zu", name, Tb, ntb, tbw, ldsw);
        CHECK(qoffs + nslot * jmax * 8 <= tbw, "[%s] table layout %d", name, tbw);
        CHECK(Tb % 4 == 0 && tbw % 4 == 0 && offc % 4 == 0 && qoffs % 4 == 0, "alignment");
        const bool issue_after = DT == 192;
        const int64_t nb = R.ntime_tiles * R.ndm_tiles;
        // every block_stride-th block, and always the last
        for (int64_t lb = 0; lb < nb;
             lb = lb + block_stride < nb ? lb + block_stride : (lb == nb - 1 ? nb : nb - 1)) {
            const int64_t tt = lb / R.ndm_tiles; const int tile = int(lb - tt * R.ndm_tiles);
            const int64_t t0 = tt * TT;
            const int nd = std::min(DT, R.ndms - tile * DT);
            Lds lds(ldsw);
            auto tbuf = [&](int k) -> long { return Tb + long(k & 1) * tbw; };
            const int nsb_last = (nch - (nst - 1) * C + K - 1) / K;
            auto nsb_of = [&](int k) { return k + 1 < nst ? nslot : nsb_last; };
            // direct loads of one stage's windows (starts from the host table or LDS)
            auto rows_issue = [&](int k, bool scalar, long tsrc, int ph) {
                const int cs = k * C, cn = std::min(C, nch - cs);
                const long buf = long(k & 1) * CW;
                for (int j = 0; j < cn; ++j) {
                    int w0;
                    if (scalar) {
                        const size_t gi = R.base_offset + size_t(tile) * nch + j;
                        CHECK(gi < P.baseT.size(), "baseT index");
                        w0 = P.baseT[gi];
                    } else w0 = int(lds.rd(tsrc + 4 + j, ph, TAG_TAB + k - 1, "window start"));
                    CHECK(w0 >= 0, "w0 %d", w0);
                    const int64_t g = int64_t(cs + j) * lv.pitch + t0 + 2 * int64_t(w0);
                    const int chunks = Wr >> 2;
                    for (int q = 0; q < chunks; ++q) {
                        CHECK(g + 8 * q + 8 <= Ln, "[%s] window load past level: r%zu c%d", name, r, cs + j);
                        for (int m = 0; m < 4; ++m) {
                            const int64_t e = g + 8 * q + 2 * m;
                            auto at = [&](int64_t i) -> uint32_t { return i < Ln ? L[i] : 0; };
                            lds.dma(buf + long(j) * Wr + 4 * q + m, at(e) | (at(e + 1) << 16), ph, TAG_WIN + k, "win");
                        }
                    }
                }
            };
            auto tables_issue = [&](int k, int nsb, int ph) {
                const long T = tbuf(k);
                const int c0 = k * C;
                const int64_t gsb = int64_t(tile) * nsub + int64_t(k) * nslot;
                for (int l = 0; l < nsb; ++l) {
                    const size_t gi = R.sb_n_offset + gsb + l;
                    CHECK(gi < P.qcntT.size() && gsb + l < int64_t(R.ndm_tiles) * nsub, "qcnt index");
                    lds.dma(T + l, uint32_t(P.qcntT[gi]), ph, TAG_TAB + k, "qcnt");
                }
                const int c1 = c0 + C, cn1 = std::min(C, nch - c1);
                for (int l = 0; l < cn1; ++l) {
                    const size_t gi = R.base_offset + size_t(tile) * nch + c1 + l;
                    CHECK(c1 + l < nch, "baseT next");
                    lds.dma(T + 4 + l, uint32_t(P.baseT[gi]), ph, TAG_TAB + k, "next starts");
                }
                const int n4 = nsb * DT / 4;
                CHECK(nsb * DT % 4 == 0, "offC chunks");
                for (int b = 0; b < n4; ++b)
                    for (int m = 0; m < 4; ++m) {
                        const int64_t gi = gsb * DT + 4 * b + m;
                        CHECK(gi < int64_t(R.ndm_tiles) * nsub * DT, "offC index");
                        lds.dma(T + offc + 4 * b + m, uint32_t(P.offCT[R.sb_c_offset + gi]), ph, TAG_TAB + k, "offC");
                    }
                const int q4 = nsb * jmax * kSubband / 4;
                for (int b = 0; b < q4; ++b)
                    for (int m = 0; m < 4; ++m) {
                        const int64_t gi = gsb * jmax * kSubband + 4 * b + m;
                        CHECK(gi < int64_t(R.ndm_tiles) * nsub * jmax * kSubband, "qoff index");
                        lds.dma(T + qoffs + 4 * b + m, uint32_t(P.qoffT[R.sb_q_offset + gi]), ph, TAG_TAB + k, "qoff");
                    }
            };
            std::vector<uint32_t> acc16(size_t(DT) * 64 * NW, 0);
            std::vector<int64_t> acc32(size_t(DT) * TT, 0);
            int widen_left = R.widen_every;
            int ph = 0;
            rows_issue(0, true, 0, ph);
            tables_issue(0, nsb_of(0), ph);
            for (int k = 0; k < nst; ++k) {
                // wait_loads + barrier
                ++ph; lds.wait_all();
                const long T = tbuf(k);
                const long A = long(k & 1) * CW;
                const int nsb = nsb_of(k);
                const int J0 = int(lds.rd(T, ph, TAG_TAB + k, "J0"));
                const int J1 = nsb > 1 ? int(lds.rd(T + 1, ph, TAG_TAB + k, "J1")) : 0;
                CHECK(J0 >= 1 && J0 <= jmax && J1 >= 0 && J1 <= jmax, "J %d %d", J0, J1);
                const int c0 = k * C;
                for (int row = 0; row < J0 + J1; ++row) {
                    const int s = row >= J0 ? 1 : 0;
                    const int rr = row + s * (jmax - J0);
                    const int kb = std::min(K, nch - (c0 + s * K));
                    int ov[8];
                    for (int m = 0; m < 8; ++m) ov[m] = int(lds.rd(T + qoffs + rr * 8 + m, ph, TAG_TAB + k, "ov"));
                    const int nodd = ov[0] >> 24;
                    ov[0] &= 0xffffff;
                    CHECK(nodd >= 0 && nodd <= kb, "nodd %d kb %d", nodd, kb);
                    if (nodd >= 0 && nodd <= 8) ++nodd_hist[nodd];
                    std::vector<uint32_t> se(64 * NQ, 0), so(64 * NQ, 0);
                    for (int w = 0; w < 64 * NQ; ++w)
                        for (int m = 0; m < kb; ++m) {
                            // needed: even channel words below Wq, odd channel words up to Wq
                            const bool need = m < nodd ? w <= Wq : w < Wq;
                            const uint32_t x = need ? lds.rd(A + ov[m] + w, ph, TAG_WIN + k, "row read")
                                                    : lds.rd_any(A + ov[m] + w, ph, "row read tail");
                            (m < nodd ? so : se)[w] += x;
                        }
                    std::vector<uint32_t> sv(64 * NQ);
                    for (int w = 0; w < 64 * NQ; ++w) {
                        const uint32_t nb = w + 1 < 64 * NQ ? so[w + 1] : 0;
                        sv[w] = se[w] + (nodd ? alignbyte(nb, so[w], 2) : 0);
                    }
                    const long qe = Qb + long(rr) * 2 * Wq;
                    for (int w = 0; w < 64 * NQ; ++w) {
                        const bool last = w >= 64 * (NQ - 1);
                        const uint32_t nb1 = w + 1 < 64 * NQ ? sv[w + 1] : 0;
                        if (!last || w < Wq) lds.st(qe + w, sv[w], ph, TAG_Q + k, "row even");
                        if (!last || w + 1 < Wq) lds.st(qe + Wq + w, alignbyte(nb1, sv[w], 2), ph, TAG_Q + k, "row odd");
                    }
                }
                auto issue_next = [&]() {
                    if (k + 1 < nst) {
                        rows_issue(k + 1, false, T, ph);
                        tables_issue(k + 1, nsb_of(k + 1), ph);
                    }
                };
                if (!issue_after) issue_next();
                ++ph;   // barrier
                if (issue_after) issue_next();
                const int DPW = DT / P.waves;
                for (int d = 0; d < DT; ++d) {
                    // a wavefront whose DMs all lie past the range's last skips its sums
                    if (tile * DT + (d / DPW) * DPW >= R.ndms)
                        continue;
                    for (int s = 0; s < nsb; ++s) {
                        const int o = int(lds.rd(T + offc + s * DT + d, ph, TAG_TAB + k, "offC read"));
                        for (int i = 0; i < NW; ++i)
                            for (int ln = 0; ln < 64; ++ln) {
                                const long wi = Qb + o + ln + 64 * i;
                                const int64_t t = t0 + 2 * (ln + 64 * i);
                                const bool need = d < nd && t < R.nout;
                                acc16[(size_t(d) * NW + i) * 64 + ln] += need ? lds.rd(wi, ph, TAG_Q + k, "sum read") : lds.rd_any(wi, ph, "sum read (unused)");
                            }
                    }
                }
                if (--widen_left == 0 || k + 1 == nst) {
                    widen_left = R.widen_every;
                    for (int d = 0; d < DT; ++d)
                        for (int i = 0; i < NW; ++i)
                            for (int ln = 0; ln < 64; ++ln) {
                                uint32_t &a = acc16[(size_t(d) * NW + i) * 64 + ln];
                                const int tl = 2 * (ln + 64 * i);
                                acc32[size_t(d) * TT + tl] += a & 0xffff;
                                acc32[size_t(d) * TT + tl + 1] += a >> 16;
                                a = 0;
                            }
                }
            }
            for (int d = 0; d < nd; ++d) {
                const int dm = tile * DT + d;
                const int32_t *shf = &P.shifts[size_t(R.dm_index + dm) * nch];
                for (int i = 0; i < TT; ++i) {
                    const int64_t t = t0 + i;
                    if (t >= R.nout) break;
                    int64_t want = 0;
                    for (int c = 0; c < nch; ++c) want += L[size_t(c) * lv.pitch + t + shf[c]];
                    ++checked;
                    if (acc32[size_t(d) * TT + i] != want) {
                        ++mism;
                        CHECK(false, "[%s] r%zu dm %d t %ld: got %ld want %ld", name, r, dm, long(t), long(acc32[size_t(d) * TT + i]), long(want));
                    }
                }
            }
        }
        printf("[%s] range %zu: ds %d ndms %d K %d stage %d nslot %d Wr %d Wq %d jmax %d widen %d lds %zu\n",
               name, r, R.ds, R.ndms, K, C, nslot, Wr, Wq, jmax, R.widen_every, P.lds_bytes);
    }
    printf("[%s] checked %ld outputs, %ld mismatches, fails %d\n", name, long(checked), long(mism), fails);
    return 0;
}

static std::vector<double> band(double fhi, double flo, int n) {
    std::vector<double> f(n); for (int c = 0; c < n; ++c) f[c] = fhi - c * (fhi - flo) / n; return f;
}

// sb_schedule small [STRIDE]: small plans at every DM tile (every STRIDE-th
// block of each range, and its last); sb_schedule ska [STRIDE [DM_TILE
// [STAGE]]]: the SKA-like beam's plan.
int main(int argc, char **argv)
{
    const char *which = argc > 1 ? argv[1] : "small";
    const int stride = argc > 2 ? std::max(1, atoi(argv[2])) : (strcmp(which, "small") ? 997 : 1);
    if (!strcmp(which, "small")) {
        // every DM tile at its default time tile, then the 8-wavefront tiles
        // (96 and 64 DMs) at 256-sample time tiles
        const int tiles[6][2] = {{192, 0}, {128, 0}, {96, 0}, {64, 0}, {96, 256}, {64, 256}};
        for (const auto &tl : tiles) {
            const int dt = tl[0];
            g_time_tile = tl[1];
            char nm[64];
            auto N = [&](const char *s) {
                snprintf(nm, sizeof nm, "%s-dt%d-tt%d", s, dt, g_time_tile);
                return nm;
            };
            const std::vector<dd_range> fine = {{0, 30, 0.1, 1}, {30, 60, 0.2, 2}};
            run(band(1500, 1200, 128), 256e-6, 65536 / 4, {{0, 100, 1, 1}}, dt, 0, 1, stride, N("128ch"));
            run(band(1670, 1370, 300), 64e-6, 20000, fine, dt, 0, 10, stride, N("300ch"));
            run(band(1670, 1370, 300), 64e-6, 20000, fine, dt, 8, 7, stride, N("300ch-stage8"));
            run(band(1500, 1300, 37), 2.56e-4, 5000, {{0, 20, 1, 1}, {20, 30, 2, 2}}, dt, 0, 11, stride, N("37ch"));
            run(band(1500, 1300, 5), 2.56e-4, 3000, {{0, 20, 1, 1}, {20, 40, 1, 4}}, dt, 0, 4, stride, N("5ch"));
            run(band(1500, 1300, 1), 2.56e-4, 3000, {{0, 20, 1, 1}}, dt, 0, 5, stride, N("1ch"));
            run(band(1500, 1300, 64), 2.56e-4, 40000, {{0, 20, 1, 32}, {20, 40, 1, 64}, {40, 60, 2, 256}},
                dt, 0, 6, stride, N("bigds"));
            run(band(1670, 1370, 257), 64e-6, 20000, {{0, 30, 0.1, 1}}, dt, 0, 18, stride, N("257ch"));
            run(band(1670, 1370, 24), 64e-6, 20000, {{0, 30, 0.1, 1}}, dt, 0, 19, stride, N("24ch"));
            run(band(1670, 1370, 17), 64e-6, 20000, {{0, 30, 0.1, 1}, {30, 60, 0.5, 16}}, dt, 0, 20, stride,
                N("17ch"));
        }
    } else if (!strcmp(which, "random")) {
        // random plans: band (possibly permuted), sampling, length, one to
        // three ranges of random step and downsample, every DM tile and time
        // tile; plans whose patterns do not fit the LDS are skipped
        std::mt19937 fz(7331);
        auto uni = [&](double a, double b) { return std::uniform_real_distribution<double>(a, b)(fz); };
        auto pick = [&](int a, int b) { return std::uniform_int_distribution<int>(a, b)(fz); };
        const int tiles[6][2] = {{192, 0}, {128, 0}, {96, 0}, {64, 0}, {96, 256}, {64, 256}};
        const int nplans = argc > 3 ? atoi(argv[3]) : 36;
        for (int i = 0; i < nplans; ++i) {
            const int nch = pick(1, 300);
            const double top = uni(1300, 1700);
            std::vector<double> f = band(top, top - uni(50, 400), nch);
            if (i % 4 == 2)
                std::shuffle(f.begin(), f.end(), fz);
            const double ts[3] = {6.4e-5, 1.28e-4, 2.56e-4};
            const double tsamp = ts[pick(0, 2)];
            const int64_t nsamp = pick(3000, 24000);
            std::vector<dd_range> rg;
            double lo = 0;
            for (int r = pick(1, 3); r > 0; --r) {
                const double steps[5] = {0.1, 0.2, 0.5, 1.0, 2.0};
                const double step = steps[pick(0, 4)];
                const double hi = lo + step * pick(5, 250);
                const int dss[6] = {1, 2, 3, 4, 8, 16};
                rg.push_back(dd_range{lo, hi, step, dss[pick(0, 5)]});
                lo = hi;
            }
            const int *tl = tiles[i % 6];
            g_time_tile = tl[1];
            const int stage = i % 5 == 4 ? 8 : 0;
            char nm[64];
            snprintf(nm, sizeof nm, "random%d-dt%d-tt%d", i, tl[0], g_time_tile);
            run(f, tsamp, nsamp, rg, tl[0], stage, 300 + i, stride, nm);
        }
    } else {
        const std::vector<dd_range> rg = {{0, 150, 0.1, 1}, {150, 300, 0.2, 2}, {300, 500, 0.5, 4},
                                          {500, 1000, 1, 8}, {1000, 2000, 2, 16}};
        run(band(1670, 1370, 4096), 64e-6, 262144, rg, argc > 3 ? atoi(argv[3]) : 192,
            argc > 4 ? atoi(argv[4]) : 0, 9, stride, "ska");
    }
    printf("rows by odd-aligned channels:");
    for (int i = 0; i < 9; ++i)
        printf(" %ld", nodd_hist[i]);
    printf("\n");
    return fails ? 1 : 0;
}
