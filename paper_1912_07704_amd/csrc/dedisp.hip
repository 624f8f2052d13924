// Device side of the dedispersion library for MI355X (gfx950): the binning
// kernels, the integer shift-and-sum kernels (direct, and exact sub-band
// reuse), their persistent batch forms, the float32 shift-and-sum (forward,
// adjoint, boxcar loss and its gradient) with its level and finalize
// kernels, the streaming and corner-turn copies, device copies of the plan
// tables, and the compute entry points of the C ABI.
//
// The operator (brute-force incoherent dedispersion; the paper names it as
// the pipeline's first GPU module in its Introduction):
//   out_r[d][t] = sum_c x_r[c][t + s[d][c]],  t < nout_r,
// with x_r the input binned by ds_r and s the FP64 delay table of the plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "plan.h"

namespace {

using dd::Plan;
using dd::RangeInfo;

constexpr int kWave = 64;
constexpr int kWavesPerBlock = dd::kWaves;
constexpr int kBlock = dd::kWaves * kWave;
constexpr int kDW = dd::kDmPerWave;
constexpr int kXcds = 8;     // workgroups are dealt to the XCDs round-robin
constexpr int kCusPerXcd = 32;

// Plan tables are read-only for the whole launch and read at wave-uniform
// addresses.  The compiler would use vector loads for them after the
// direct-to-LDS loads (which it treats as possible writes), and every such
// load's wait would also drain the in-flight staging loads; so eight table
// entries are fetched with one scalar load instead.
typedef int sgpr8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ sgpr8 table8(const int32_t *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
    const uint64_t addr = (uint64_t(hi) << 32) | lo;
    sgpr8 v;
    asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(addr));
    return v;
}

__device__ __forceinline__ int32_t table1(const int32_t *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
    const uint64_t addr = (uint64_t(hi) << 32) | lo;
    int32_t v;
    asm volatile("s_load_dword %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(addr));
    return v;
}

// ---------------------------------------------------------------------------
// Device-side plan state: the channel-major shift table, one copy per device.
// ---------------------------------------------------------------------------

struct DeviceTables {
    int32_t *offT = nullptr;     // start of the one allocation holding every table
    int32_t *baseT = nullptr;
    int32_t *qcnt = nullptr;     // integer variant 3 only
    int32_t *qoff = nullptr;
    int32_t *offC = nullptr;
};

struct DeviceState {
    std::mutex mu;
    std::map<int, DeviceTables> per_device;
};

DeviceState *state_of(const Plan &p) { return static_cast<DeviceState *>(p.device); }

bool fault_requested(const char *what)
{
    const char *f = std::getenv("DD_FAULT");
    return f && std::strcmp(f, what) == 0;
}

dd_status hip_fail(hipError_t e, const char *where)
{
    dd::set_error(std::string(where) + ": " + hipGetErrorString(e));
    return DD_ERR_HIP;
}

// Returns the tables of the current device, uploading them on first use.
dd_status device_tables(const Plan &p, DeviceTables **out)
{
    DeviceState *st = state_of(p);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(st->mu);
    auto it = st->per_device.find(dev);
    if (it != st->per_device.end()) {
        *out = &it->second;
        return DD_OK;
    }
    if (fault_requested("alloc")) {
        dd::set_error("device allocation failure forced by DD_FAULT=alloc");
        return DD_ERR_NOMEM;
    }
    DeviceTables t;
    // integer plans use offT/baseT (variant 3: baseT, qcntT, qoffT, offCT),
    // float plans offF/baseF; one allocation, each table 256-byte aligned
    const std::vector<int32_t> empty;
    const bool u8 = p.dtype == DD_U8;
    const std::vector<int32_t> *parts[5] = {u8 ? &p.offT : &p.offF, u8 ? &p.baseT : &p.baseF,
                                            p.subband ? &p.qcntT : &empty,
                                            p.subband ? &p.qoffT : &empty,
                                            p.subband ? &p.offCT : &empty};
    size_t at[5], total = 0;
    for (int i = 0; i < 5; ++i) {
        at[i] = total;
        total += (parts[i]->size() * sizeof(int32_t) + 255) / 256 * 256;
    }
    char *mem = nullptr;
    e = hipMalloc(&mem, total + 256);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dd::set_error(std::string("hipMalloc of the delay tables: ") + hipGetErrorString(e));
        return DD_ERR_NOMEM;
    }
    for (int i = 0; i < 5 && e == hipSuccess; ++i)
        if (!parts[i]->empty())
            e = hipMemcpy(mem + at[i], parts[i]->data(), parts[i]->size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "hipMemcpy of the delay tables");
    }
    t.offT = reinterpret_cast<int32_t *>(mem + at[0]);
    t.baseT = reinterpret_cast<int32_t *>(mem + at[1]);
    t.qcnt = reinterpret_cast<int32_t *>(mem + at[2]);
    t.qoff = reinterpret_cast<int32_t *>(mem + at[3]);
    t.offC = reinterpret_cast<int32_t *>(mem + at[4]);
    *out = &(st->per_device[dev] = t);
    return DD_OK;
}

// ---------------------------------------------------------------------------
// Binning into 16-bit rows: dst[c][t] = sum_{k<f} src[c][f*t + k], t < nbin.
// Each thread forms four consecutive bins.
// ---------------------------------------------------------------------------

template <typename Tin>
__global__ __launch_bounds__(256) void k_bin_u16(const Tin *__restrict__ src, int64_t src_pitch,
                                                 uint16_t *__restrict__ dst, int64_t dst_pitch,
                                                 int64_t nbin, int factor, int nchans)
{
    const int64_t nq = (nbin + 3) / 4;
    for (int64_t c = blockIdx.y; c < nchans; c += gridDim.y) {
        const Tin *row = src + c * src_pitch;
        uint16_t *out = dst + c * dst_pitch;
        for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < nq;
             q += int64_t(gridDim.x) * blockDim.x) {
            const int64_t t = 4 * q;
            uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (t + i < nbin) {
                    const Tin *p = row + (t + i) * factor;
                    for (int k = 0; k < factor; ++k)
                        v[i] += p[k];
                }
            }
            if (t + 4 <= nbin) {
                ushort4 w;
                w.x = uint16_t(v[0]);
                w.y = uint16_t(v[1]);
                w.z = uint16_t(v[2]);
                w.w = uint16_t(v[3]);
                *reinterpret_cast<ushort4 *>(out + t) = w;
            } else {
                for (int i = 0; i < 4 && t + i < nbin; ++i)
                    out[t + i] = uint16_t(v[i]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Integer shift-and-sum.
//
// A workgroup owns one (range, time tile of 128*NW samples, DM tile of
// kTileD trials).  Wave w handles kDW consecutive DMs; lane l handles the
// sample pairs t0 + 2*(l + 64k) + {0, 1}, k < NW, so a wave's LDS reads of
// one word index are 64 consecutive dwords (no bank conflict).
//
// The range reads a 16-bit copy of the input (binned by its downsample).
// Channels are staged in LDS in groups of C.  For channel c the staged
// window starts at the 16-byte aligned word t0/2 + baseT[tile][c] of its
// row, so it arrives by direct global-to-LDS loads; a second copy of the
// window, shifted by one sample, is then formed in LDS.  With the even
// (A) and odd (B) copies, the 32-bit word a lane needs for any delay is one
// aligned dword; offT[c][d] names it (copy, alignment and parity folded in
// on the host).  Stages are double-buffered: the loads of stage s+1 are in
// flight while stage s is summed.
//
// Each dword carries two 16-bit partial sums.  Two channels are added per
// instruction (v_add3_u32).  At most 65535/(255*ds) channels are added
// before the halves are widened into int32 accumulators, so no half can
// carry into the other and the int32 result is exact.
// ---------------------------------------------------------------------------

struct RangeArgs {
    const uint16_t *src;      // 16-bit rows of this range's level
    const int32_t *offT;      // [nchans][ndms_pad] word offsets of each DM
    const int32_t *baseT;     // [ndm_tiles][nchans] first word of each staged window
    int32_t *out;             // [ndms][nout] output rows of this range
    int64_t pitch;            // samples per row of src
    int64_t nout;
    int64_t block_start;
    int32_t nchans;
    int32_t ndms;
    int32_t ndms_pad;
    int32_t ndm_tiles;
    int32_t stage_chans;
    int32_t row_words;
    int32_t widen_every;
};

struct FwdArgs {
    RangeArgs r[DD_MAX_RANGES];
    int64_t nblocks;
    int64_t per_xcd;
    int32_t nranges;
};

// Barrier for LDS traffic only: outstanding global loads (the prefetch of
// the next stage) stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ void wait_loads()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Start the direct-to-LDS loads of the windows of channels [cs, cs + cn)
// into the A copy at `buf` (row j at buf + j*Wr).  One wave instruction
// moves 64 lanes x 16 bytes of one row.
template <int WAVES, class RA>
__device__ __forceinline__ int32_t stage_starts(const RA &R, int nchans, int tile, int cs, int cn, int lane)
{
    // the stage's window starts, lane j holding channel cs + j's
    return lane < cn ? R.baseT[int64_t(tile) * nchans + cs + lane] : 0;
}

// Wavefront w stages channels w, w + WAVES, ... of the stage (at most
// kMaxStageChans); their window starts are read out of ws (stage_starts,
// loaded a stage earlier) before the first direct load is issued, so that
// waiting for ws waits for nothing in flight.
template <int WAVES, class RA>
__device__ __forceinline__ void stage_issue(const RA &R, int nchans, int tile, int64_t t0,
                                            int cs, int cn, int32_t ws, uint32_t *buf, int wave,
                                            int lane)
{
    constexpr int kPer = (dd::kMaxStageChans + WAVES - 1) / WAVES;
    int32_t w0s[kPer];
#pragma unroll
    for (int h = 0; h < kPer; ++h)
        w0s[h] = __builtin_amdgcn_readlane(ws, min(wave + h * WAVES, kWave - 1));
    const int Wr = R.row_words;
    const int chunks = Wr >> 2;
    const int CW = R.stage_chans * Wr;
#pragma unroll
    for (int h = 0; h < kPer; ++h) {
        const int j = wave + h * WAVES;
        if (j >= cn)
            break;
        const int64_t c = cs + j;
        const uint16_t *g = R.src + c * R.pitch + t0 + 2 * int64_t(w0s[h]);
        for (int c0 = 0; c0 < chunks; c0 += kWave) {
            const int q = c0 + lane;
            if (q < chunks) {
                // even copy, and the odd-aligned copy: the same row one sample later
                __builtin_amdgcn_global_load_lds(g + 8 * q, buf + j * Wr + 4 * c0, 16, 0, 0);
                __builtin_amdgcn_global_load_lds(g + 8 * q + 1, buf + CW + j * Wr + 4 * c0, 16, 0, 0);
            }
        }
    }
}

// One work item: range R, item index lb inside the range (time tile major,
// DM tile minor).  `lds` holds two stages of two copies each.
// DEDUP: a channel's words are re-read from LDS only when a DM's offset
// differs from the previous DM's (consecutive DMs share a delay often).
template <bool DEDUP, int WAVES, int NW>
__device__ __forceinline__ void dedisp_tile_u8(const RangeArgs &R, int64_t lb, uint32_t *lds)
{
    constexpr int kTileDW = WAVES * kDW;
    const int64_t tt = lb / R.ndm_tiles;
    const int tile = int(lb - tt * R.ndm_tiles);
    const int d0 = tile * kTileDW;
    const int64_t t0 = tt * (2 * kWave * NW);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int ndms = R.ndms;
    const int dpad = R.ndms_pad;
    const int dw0 = d0 + wave * kDW;
    const int nchans = R.nchans;
    const int C = R.stage_chans;
    const int Wr = R.row_words;
    const int CW = C * Wr;              // words of one copy of a stage
    const int nst = (nchans + C - 1) / C;

    uint32_t acc16[kDW][NW];
    int32_t acc32[kDW][NW][2];
#pragma unroll
    for (int dd = 0; dd < kDW; ++dd)
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            acc16[dd][k] = 0u;
            acc32[dd][k][0] = 0;
            acc32[dd][k][1] = 0;
        }

    {
        const int32_t ws0 = stage_starts<WAVES>(R, nchans, tile, 0, min(C, nchans), lane);
        stage_issue<WAVES>(R, nchans, tile, t0, 0, min(C, nchans), ws0, lds, wave, lane);
    }
    // window starts of the next stage to issue, loaded one stage ahead
    int32_t ws_next = nst > 1 ? stage_starts<WAVES>(R, nchans, tile, C, min(C, nchans - C), lane) : 0;
    int widen_left = R.widen_every;
    for (int st = 0; st < nst; ++st) {
        const int c0 = st * C;
        const int cn = min(C, nchans - c0);
        uint32_t *A = lds + (st & 1) * (2 * CW);

        // Both copies of the stage's windows have landed (each wavefront
        // waits for its own loads, the barrier for everyone's).
        wait_loads();
        lds_barrier();
        if (st + 1 < nst) {
            const int cs = c0 + C;
            stage_issue<WAVES>(R, nchans, tile, t0, cs, min(C, nchans - cs), ws_next,
                               lds + ((st + 1) & 1) * (2 * CW), wave, lane);
            const int cs2 = cs + C;
            ws_next = st + 2 < nst ? stage_starts<WAVES>(R, nchans, tile, cs2, min(C, nchans - cs2), lane) : 0;
        }

        for (int jp = 0; jp < cn; jp += 2) {
            // Offsets of this wave's DMs in the two staged channels; the
            // table is padded so the 8 entries are aligned and in bounds.
            static_assert(kDW == 8, "offsets are loaded as one scalar octet per row");
            const int32_t *oa = R.offT + int64_t(c0 + jp) * dpad + dw0;
            const sgpr8 av = table8(oa);
            const int offa[kDW] = {av[0], av[1], av[2], av[3], av[4], av[5], av[6], av[7]};
            const uint32_t *rowa = A + jp * Wr + lane;
            if (jp + 1 < cn) {
                const sgpr8 bv = table8(oa + dpad);
                const int offb[kDW] = {bv[0], bv[1], bv[2], bv[3], bv[4], bv[5], bv[6], bv[7]};
                const uint32_t *rowb = rowa + Wr;
                if constexpr (DEDUP) {
                    uint32_t va[NW], vb[NW];
#pragma unroll
                    for (int dd = 0; dd < kDW; ++dd) {
                        if (dd == 0 || offa[dd] != offa[dd - 1]) {
#pragma unroll
                            for (int k = 0; k < NW; ++k)
                                va[k] = rowa[offa[dd] + kWave * k];
                        }
                        if (dd == 0 || offb[dd] != offb[dd - 1]) {
#pragma unroll
                            for (int k = 0; k < NW; ++k)
                                vb[k] = rowb[offb[dd] + kWave * k];
                        }
#pragma unroll
                        for (int k = 0; k < NW; ++k)
                            acc16[dd][k] += va[k] + vb[k];
                    }
                } else {
#pragma unroll
                    for (int dd = 0; dd < kDW; ++dd) {
                        const uint32_t *pa = rowa + offa[dd];
                        const uint32_t *pb = rowb + offb[dd];
#pragma unroll
                        for (int k = 0; k < NW; ++k)
                            acc16[dd][k] += pa[kWave * k] + pb[kWave * k];
                    }
                }
            } else {
#pragma unroll
                for (int dd = 0; dd < kDW; ++dd) {
                    const uint32_t *pa = rowa + offa[dd];
#pragma unroll
                    for (int k = 0; k < NW; ++k)
                        acc16[dd][k] += pa[kWave * k];
                }
            }
        }
        if (--widen_left == 0 || st + 1 == nst) {
            widen_left = R.widen_every;
#pragma unroll
            for (int dd = 0; dd < kDW; ++dd)
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    acc32[dd][k][0] += int32_t(acc16[dd][k] & 0xffffu);
                    acc32[dd][k][1] += int32_t(acc16[dd][k] >> 16);
                    acc16[dd][k] = 0u;
                }
        }
    }

#pragma unroll
    for (int dd = 0; dd < kDW; ++dd) {
        const int d = dw0 + dd;
        if (d >= ndms)
            break;
        int32_t *row = R.out + int64_t(d) * R.nout;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t t = t0 + 2 * (lane + kWave * k);
            if (t < R.nout)
                row[t] = acc32[dd][k][0];
            if (t + 1 < R.nout)
                row[t + 1] = acc32[dd][k][1];
        }
    }
}


template <bool DEDUP, int WAVES, int NW>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_dedisp_u8(const FwdArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];

    // Workgroups with consecutive logical index run on one XCD, so the DM
    // tiles of a time tile share that XCD's L2.
    const int64_t b = blockIdx.x;
    const int64_t L = (b % kXcds) * a.per_xcd + b / kXcds;
    if (L >= a.nblocks)
        return;
    int r = 0;
    for (int i = 1; i < a.nranges; ++i)
        if (L >= a.r[i].block_start)
            r = i;
    dedisp_tile_u8<DEDUP, WAVES, NW>(a.r[r], L - a.r[r].block_start, lds);
}

// ---------------------------------------------------------------------------
// Integer variant 3: exact sub-band reuse.
//
// Inside one DM tile, DMs whose delays over a sub-band of kSubband channels
// exceed their own smallest delay over that sub-band by the same pattern
// need the same partial sum of the sub-band, only read at different
// delays:
//   out[d][t] = sum_b Q_{b,j(d)}[t + a[d][b] - amin_j],
//   Q_{b,j}[u] = sum_{c in b} x[c][u + amin_j + v_j[c]].
// Per stage (stage_chans channels, one or two sub-bands) a workgroup stages
// one copy of each channel window (16-bit samples, two per word), builds
// every pattern row Q of its sub-bands in an even and an odd-aligned copy,
// and adds one row word per DM, sub-band and sample pair -- the same
// integer sums in another grouping, so exact.
// ---------------------------------------------------------------------------

struct SbRange {
    const uint16_t *src;      // 16-bit rows of this range's level
    const int32_t *baseT;     // [ndm_tiles][nchans] first word of each staged window
    const int32_t *qcnt;      // [ndm_tiles][nsub] patterns per sub-band
    const int32_t *qoff;      // [ndm_tiles][nsub][jmax][kSubband] pattern row starts
    const int32_t *offC;      // [ndm_tiles][nsub][dm_tile] per-DM row and delay
    int32_t *out;             // [ndms][nout] output rows of this range
    int64_t pitch;
    int64_t nout;
    int64_t block_start;
    int32_t nchans;
    int32_t ndms;
    int32_t ndm_tiles;
    int32_t stage_chans;
    int32_t row_words;
    int32_t widen_every;
    int32_t sb_chans;
    int32_t nsub;
    int32_t jmax;
    int32_t qwords;
    int32_t nslot;            // sub-bands per stage
    int32_t tb_words;         // ints per stage-table buffer
};

struct SbArgs {
    SbRange r[DD_MAX_RANGES];
    int64_t nblocks;
    int64_t per_xcd;
    int32_t nranges;
};

__device__ __forceinline__ void dma4(const void *g, void *l)
{
    __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
}

__device__ __forceinline__ void dma16(const void *g, void *l)
{
    __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
}

// Per-stage tables, staged in LDS one stage ahead by direct loads (ints):
//   [0, 4)             patterns of the stage's sub-bands
//   [4, tb_offc)       first staged word of the next stage's channel windows
//   [tb_offc, tb_qoff) per-DM row and delay, nslot x dm_tile
//   [tb_qoff, ...)     pattern row starts, nslot x jmax x kSubband (channels whose
//                      row starts odd first; bits 24-27 of entry 0 count them)
template <class RR>
__device__ __forceinline__ int tb_offc(const RR &R) { return 4 + ((R.stage_chans + 3) & ~3); }

// Direct loads of stage st's tables (its nsb sub-bands start at st*nslot).
template <int WAVES, int DT, class RR>
__device__ __forceinline__ void tables_issue(const RR &R, int tile, int st, int nsb,
                                             int32_t *T, int wave, int lane)
{
    const int C = R.stage_chans, nch = R.nchans;
    const int c0 = st * C;
    const int64_t gsb = int64_t(tile) * R.nsub + st * R.nslot;
    const int offc = tb_offc(R);
    if (wave == WAVES - 1) {
        if (lane < nsb)
            dma4(R.qcnt + gsb + lane, T);
        const int c1 = c0 + C;
        const int cn1 = min(C, nch - c1);
        if (lane < cn1)
            dma4(R.baseT + int64_t(tile) * nch + c1 + lane, T + 4);
    } else if (wave == WAVES - 2) {
        const int n4 = nsb * DT / 4;
        for (int b = 0; b < n4; b += kWave)
            if (b + lane < n4)
                dma16(R.offC + gsb * DT + 4 * (b + lane), T + offc + 4 * b);
    } else if (wave == WAVES - 3) {
        const int n4 = nsb * R.jmax * dd::kSubband / 4;
        const int32_t *g = R.qoff + gsb * R.jmax * dd::kSubband;
        int32_t *l = T + offc + R.nslot * DT;
        for (int b = 0; b < n4; b += kWave)
            if (b + lane < n4)
                dma16(g + 4 * (b + lane), l + 4 * b);
    }
}

// Direct loads of the channel windows this wavefront owns (rows j with
// j % WAVES == wave) of one stage; the window starts come from `base`
// (global or LDS stage tables).
template <int WAVES, bool SCALAR_BASE, class RR>
__device__ __forceinline__ void rows_issue(const RR &R, const uint16_t *src, const int32_t *base,
                                           int64_t t0, int cs, int cn, uint32_t *buf, int wave,
                                           int lane)
{
    const int Wr = R.row_words;
    const int chunks = Wr >> 2;
    for (int j = wave; j < cn; j += WAVES) {
        // (from LDS the start stays a VGPR: only the LDS destination of a
        // direct load has to be wave-uniform)
        const int32_t w0 = SCALAR_BASE ? table1(base + j) : base[j];
        const uint16_t *g = src + (cs + j) * R.pitch + t0 + 2 * int64_t(w0);
        for (int part = 0; part * kWave < chunks; ++part) {
            const int q = part * kWave + lane;
            if (q < chunks)
                dma16(g + 8 * q, buf + j * Wr + part * (4 * kWave));
        }
    }
}

__device__ __forceinline__ int lds_uniform(const int32_t *p)
{
    return __builtin_amdgcn_readfirstlane(*p);
}

// Whole-wavefront lane move (DPP): lane i receives lane i+1's value (lane
// 63 keeps `old`).
constexpr int kDppWaveShl1 = 0x130;

// One pattern row of NQ*64 words or fewer (Wq > 64 * (NQ - 1)), both
// copies; lane l builds words NQ*l .. NQ*l + NQ - 1 (a stride of NQ words
// between lanes, odd, so the LDS reads and writes stay conflict-free).
// Channel k's words at ov[k] + w hold its samples from an even position
// on; the rows of the first nodd (wave-uniform) channels start one sample
// later.  The even channels' words sum to sv, the odd channels' to so,
// realigned once: word w takes the upper half of so[w] and the lower half
// of so[w+1] (packed 16-bit halves never carry, so realigning the sum
// equals summing realigned words).  Word w+1 of a lane's last word is
// lane+1's first (lane 63: 0, past every needed word -- the plan keeps
// them below 64 * NQ - 1).  The odd copy of the row is realigned the same
// way.  All reads are in flight before the first sum; words past the row
// read other LDS data and are not stored.
template <int NQ, bool FULL>
__device__ __forceinline__ void qrow(const uint32_t *A, const int *ov, int nodd, int kb,
                                     uint32_t *qe, int Wq, int lane)
{
    const int wb = lane * NQ;
    uint32_t v[dd::kSubband][NQ];
#pragma unroll
    for (int k = 0; k < dd::kSubband; ++k)
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            v[k][i] = (FULL || k < kb) ? A[ov[k] + wb + i] : 0u;
    __builtin_amdgcn_sched_barrier(0);
    // running sums over the channels; the odd channels' sum is the one
    // after the first nodd (a register picked by a uniform index)
    uint32_t sv[NQ], so[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        uint32_t pre[dd::kSubband + 1];
        pre[0] = 0u;
#pragma unroll
        for (int k = 0; k < dd::kSubband; ++k)
            pre[k + 1] = pre[k] + v[k][i];
        so[i] = pre[nodd];
        sv[i] = pre[dd::kSubband] - so[i];
    }
    const uint32_t so_n = uint32_t(__builtin_amdgcn_update_dpp(0, int(so[0]), kDppWaveShl1, 0xF,
                                                               0xF, false));
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        sv[i] += __builtin_amdgcn_alignbyte(i + 1 < NQ ? so[i + 1] : so_n, so[i], 2);
    const uint32_t sv_n = uint32_t(__builtin_amdgcn_update_dpp(0, int(sv[0]), kDppWaveShl1, 0xF,
                                                               0xF, false));
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int w = wb + i;
        if (w < Wq)
            qe[w] = sv[i];
        if (w + 1 < Wq)
            qe[Wq + w] = __builtin_amdgcn_alignbyte(i + 1 < NQ ? sv[i + 1] : sv_n, sv[i], 2);
    }
}

template <int WAVES, int DPW, int NW, class RR>
__device__ __forceinline__ void dedisp_tile_sb(const RR &R, const uint16_t *src, int32_t *out,
                                               int64_t lb, uint32_t *lds)
{
    constexpr int DT = WAVES * DPW;
    const int64_t tt = lb / R.ndm_tiles;
    const int tile = int(lb - tt * R.ndm_tiles);
    const int64_t t0 = tt * (2 * kWave * NW);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int ndms = R.ndms;
    const int dw0 = tile * DT + wave * DPW;
    const int nchans = R.nchans;
    const int C = R.stage_chans;
    const int Wr = R.row_words;
    const int CW = C * Wr;
    const int K = R.sb_chans;
    const int Wq = R.qwords;
    const int jmax = R.jmax;
    const int nst = (nchans + C - 1) / C;
    uint32_t *Q = lds + 2 * CW;
    int32_t *Tb = reinterpret_cast<int32_t *>(Q + R.nslot * jmax * 2 * Wq + 4);
    const int offc = tb_offc(R);
    const int qoffs = offc + R.nslot * DT;

    uint32_t acc16[DPW][NW];
    int32_t acc32[DPW][NW][2];
#pragma unroll
    for (int dd = 0; dd < DPW; ++dd)
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            acc16[dd][k] = 0u;
            acc32[dd][k][0] = 0;
            acc32[dd][k][1] = 0;
        }

    // sub-bands per stage: nslot, and in the last stage whatever is left
    const int nsb_last = (nchans - (nst - 1) * C + K - 1) / K;
    rows_issue<WAVES, true>(R, src, R.baseT + int64_t(tile) * nchans, t0, 0, min(C, nchans), lds,
                            wave, lane);
    tables_issue<WAVES, DT>(R, tile, 0, nst > 1 ? R.nslot : nsb_last, Tb, wave, lane);
    int widen_left = R.widen_every;
    for (int st = 0; st < nst; ++st) {
        const int c0 = st * C;
        const int nsb = st + 1 < nst ? R.nslot : nsb_last;
        uint32_t *A = lds + (st & 1) * CW;
        const int32_t *T = Tb + (st & 1) * R.tb_words;

        // This wavefront's windows have landed.
        wait_loads();
        lds_barrier();

        const int J0 = lds_uniform(T);
        const int J1 = nsb > 1 ? lds_uniform(T + 1) : 0;
        // Pattern rows, one per wavefront at a time; row r = s * jmax + j
        // holds pattern j of the stage's sub-band s.  NW + 1 words per lane
        // cover a row (the plan keeps 64 * NW < Wq <= 64 * (NW + 1)); only
        // a band's last sub-band (or sub-bands of fewer than 8 channels at
        // large downsampling) sums fewer channels.
        const bool full = K == dd::kSubband && c0 + nsb * K <= nchans;
        for (int row = wave; row < J0 + J1; row += WAVES) {
            const int s = row >= J0 ? 1 : 0;
            const int r = row + s * (jmax - J0);
            const int32_t *qo = T + qoffs + r * dd::kSubband;
            // the row's 8 channel offsets: two broadcast 16-byte reads (the
            // wait the compiler puts before them finds none of this
            // wavefront's direct loads in flight: they are issued after its
            // rows)
            const int4 q0 = *reinterpret_cast<const int4 *>(qo);
            const int4 q1 = *reinterpret_cast<const int4 *>(qo + 4);
            // entry 0 carries the count of odd-aligned channels in bits 24-27
            const int nodd = __builtin_amdgcn_readfirstlane(q0.x) >> 24;
            const int ov[dd::kSubband] = {q0.x & 0xffffff, q0.y, q0.z, q0.w,
                                          q1.x, q1.y, q1.z, q1.w};
            uint32_t *qe = Q + r * 2 * Wq;
            if (full)
                qrow<NW + 1, true>(A, ov, nodd, dd::kSubband, qe, Wq, lane);
            else
                qrow<NW + 1, false>(A, ov, nodd, min(K, nchans - (c0 + s * K)), qe, Wq, lane);
        }
        // The next stage's loads go to the other buffers, whose last readers
        // (the previous stage's sums) finished before this stage's first
        // barrier.  At 192-DM tiles they are issued once every pattern row
        // is built and fly while this stage's (long) sums run: issued
        // earlier, their LDS writes compete with the rows' reads.  At the
        // smaller tiles the sums are too short to cover them, and each
        // wavefront issues its own right after its rows (measured).
        auto issue_next = [&]() {
            if (st + 1 < nst) {
                const int cs = c0 + C;
                rows_issue<WAVES, false>(R, src, T + 4, t0, cs, min(C, nchans - cs),
                                         lds + ((st + 1) & 1) * CW, wave, lane);
                tables_issue<WAVES, DT>(R, tile, st + 1, st + 2 < nst ? R.nslot : nsb_last,
                                        Tb + ((st + 1) & 1) * R.tb_words, wave, lane);
            }
        };
        constexpr bool issue_after = WAVES == 16 && DPW == 12;
        if constexpr (!issue_after)
            issue_next();
        lds_barrier();
        if constexpr (issue_after)
            issue_next();

        // One pattern-row word per DM, sub-band and sample pair; a wavefront
        // whose DMs all lie past the range's last (the last DM tile of a
        // range) has nothing to sum.
        if (dw0 < ndms) {
            const uint32_t *rowq = Q + lane;
            const int32_t *oc = T + offc + wave * DPW;
            int offa[DPW];
#pragma unroll
            for (int dd = 0; dd < DPW; ++dd)
                offa[dd] = oc[dd];
            if (nsb > 1) {
                int offb[DPW];
#pragma unroll
                for (int dd = 0; dd < DPW; ++dd)
                    offb[dd] = oc[DT + dd];
                // groups of 6 DMs bound the loads in flight (and the VGPRs they hold)
#pragma unroll
                for (int dd = 0; dd < DPW; ++dd) {
                    const uint32_t *pa = rowq + offa[dd];
                    const uint32_t *pb = rowq + offb[dd];
#pragma unroll
                    for (int k = 0; k < NW; ++k)
                        acc16[dd][k] += pa[kWave * k] + pb[kWave * k];
                    if (dd % 6 == 5 && dd + 1 < DPW)
                        __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int dd = 0; dd < DPW; ++dd) {
                    const uint32_t *pa = rowq + offa[dd];
#pragma unroll
                    for (int k = 0; k < NW; ++k)
                        acc16[dd][k] += pa[kWave * k];
                    if (dd % 6 == 5 && dd + 1 < DPW)
                        __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        if (--widen_left == 0 || st + 1 == nst) {
            widen_left = R.widen_every;
#pragma unroll
            for (int dd = 0; dd < DPW; ++dd)
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    acc32[dd][k][0] += int32_t(acc16[dd][k] & 0xffffu);
                    acc32[dd][k][1] += int32_t(acc16[dd][k] >> 16);
                    acc16[dd][k] = 0u;
                }
        }
    }

#pragma unroll
    for (int dd = 0; dd < DPW; ++dd) {
        const int d = dw0 + dd;
        if (d >= ndms)
            break;
        int32_t *row = out + int64_t(d) * R.nout;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t t = t0 + 2 * (lane + kWave * k);
            if (t < R.nout)
                row[t] = acc32[dd][k][0];
            if (t + 1 < R.nout)
                row[t + 1] = acc32[dd][k][1];
        }
    }
}

// One workgroup per CU: WAVES/4 wavefronts per SIMD, whose VGPRs hold the
// packed and the widened sums of DPW DMs x NW words without spilling.
template <int WAVES, int DPW, int NW>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(WAVES / 4, WAVES / 4))) void
k_dedisp_u8_sb(const SbArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int64_t b = blockIdx.x;
    const int64_t L = (b % kXcds) * a.per_xcd + b / kXcds;
    if (L >= a.nblocks)
        return;
    int r = 0;
    for (int i = 1; i < a.nranges; ++i)
        if (L >= a.r[i].block_start)
            r = i;
    dedisp_tile_sb<WAVES, DPW, NW>(a.r[r], a.r[r].src, a.r[r].out, L - a.r[r].block_start, lds);
}

// ---------------------------------------------------------------------------
// Float32 path.
//
// k_level_f32:     weighted (binned) 32-bit copies of the input,
//                  dst[c][t] = w_c * sum_{k<f} src[c][f*t + k].
// k_shiftsum_f32:  out[a][t] = sum_b rows[b][t + S[a][b]], the forward (a =
//                  DM, b = channel) and the adjoint (a = channel, b = DM over
//                  zero-padded output-gradient rows, S = P - s).  Staging by
//                  direct global-to-LDS loads into ONE stage buffer (two
//                  buffers of half the rows ran slower: the stage loop is
//                  bound by latency, which longer stages hide better, and a
//                  CU's other workgroup computes while this one waits for
//                  its loads), one float per sample.  Samples are read as
//                  aligned 16-byte granules (lane l: granules l + 63g, g <
//                  4); a delay that is not a multiple of 4 takes the
//                  granule's head from the next lane by a cross-lane move
//                  folded into the add.  Each output adds a stage's rows in a
//                  fixed order, grouped by delay mod 4 (a table per output and
//                  stage), so every group runs one fixed register pattern.
// k_pad_rows_f32:  the output gradient of one range with P zeros in front.
// k_adj_finalize:  dX[c][t] = w_c * G[c][t], G summed over ranges at each
//                  range's resolution, and per-chunk partials of
//                  dw_c = sum_t x[c][t] * G[c][t] (fixed-order tree sums).
// k_reduce_rows:   dw_c = sum of its chunk partials (fixed-order tree).
// ---------------------------------------------------------------------------

constexpr int kFW = dd::kF32Words;
constexpr int kFP = dd::kF32PerWave;
constexpr int kFTileT = dd::kF32TimeTile;      // samples computed per tile
constexpr int kFSpan = dd::kF32TileSpan;        // samples the lanes cover
// offset of accumulator k's sample from 4 * lane: granule k / 4 of the
// lane (63 granules apart), float k % 4 of it
__device__ __forceinline__ constexpr int ks(int k) { return 4 * (kWave - 1) * (k >> 2) + (k & 3); }
constexpr int kFTileA = dd::kF32OutTile;

// One thread per 4 consecutive outputs.  VEC: the source rows and the
// destination rows start on 16-byte boundaries, so a group's 4*factor
// source floats are `factor` aligned float4 loads and its outputs one
// float4 store; F (when nonzero) fixes the factor at compile time.
template <bool VEC, int F>
__global__ __launch_bounds__(256) void k_level_f32(const float *__restrict__ src, int64_t src_pitch,
                                                   const float *__restrict__ w,
                                                   float *__restrict__ dst, int64_t dst_pitch,
                                                   int64_t nbin, int factor, int nchans)
{
    const int f = F ? F : factor;
    const int64_t ngroups = (nbin + 3) >> 2;
    for (int64_t c = blockIdx.y; c < nchans; c += gridDim.y) {
        const float *row = src + c * src_pitch;
        float *out = dst + c * dst_pitch;
        const float wc = w ? w[c] : 1.0f;
        for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < ngroups;
             q += int64_t(gridDim.x) * blockDim.x) {
            const int64_t t = 4 * q;
            float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (VEC && t + 4 <= nbin) {
                const float4 *p = reinterpret_cast<const float4 *>(row + t * f);
                if (F == 1) {
                    const float4 v = p[0];
                    s[0] = v.x;
                    s[1] = v.y;
                    s[2] = v.z;
                    s[3] = v.w;
                } else if (F == 2) {
                    const float4 u = p[0], v = p[1];
                    s[0] = u.x + u.y;
                    s[1] = u.z + u.w;
                    s[2] = v.x + v.y;
                    s[3] = v.z + v.w;
                } else {
                    // other factors: sample by sample
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        for (int k = 0; k < f; ++k)
                            s[j] += row[(t + j) * f + k];
                }
                if (w) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        s[j] *= wc;
                }
                *reinterpret_cast<float4 *>(out + t) = make_float4(s[0], s[1], s[2], s[3]);
            } else {
                for (int j = 0; j < 4 && t + j < nbin; ++j) {
                    const float *p = row + (t + j) * f;
                    float acc = 0.0f;
                    for (int k = 0; k < f; ++k)
                        acc += p[k];
                    out[t + j] = w ? wc * acc : acc;
                }
            }
        }
    }
}

// The output gradient of one range with P zeros in front (and zeros up to
// the row pitch): 4 consecutive padded samples per thread, one aligned
// float4 store (the padded rows start on 16-byte boundaries, the gradient
// rows need not).
__global__ __launch_bounds__(256) void k_pad_rows_f32(const float *__restrict__ g, int64_t nout,
                                                      int64_t P, float *__restrict__ gpad,
                                                      int64_t gpitch, int nrows)
{
    const int64_t ngroups = gpitch >> 2;
    for (int64_t d = blockIdx.y; d < nrows; d += gridDim.y) {
        const float *row = g + d * nout;
        float *out = gpad + d * gpitch;
        for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < ngroups;
             q += int64_t(gridDim.x) * blockDim.x) {
            const int64_t i = 4 * q;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v[j] = (i + j >= P && i + j < P + nout) ? row[i + j - P] : 0.0f;
            *reinterpret_cast<float4 *>(out + i) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// The padding of one range's gradient rows: samples [0, P) and
// [P + nout, gpitch) of each row set to 0 (the boxcar backward writes the
// gradient between them itself).
__global__ __launch_bounds__(256) void k_zero_pads(float *__restrict__ gpad, int64_t gpitch, int64_t P,
                                                   int64_t nout, int nrows)
{
    const int64_t tail = gpitch - P - nout;
    for (int64_t d = blockIdx.y; d < nrows; d += gridDim.y) {
        float *row = gpad + d * gpitch;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < P + tail;
             i += int64_t(gridDim.x) * blockDim.x)
            row[i < P ? i : P + nout + (i - P)] = 0.0f;
    }
}

struct SumArgs {
    const float *src;         // rows, `pitch` floats apart
    const int32_t *off;       // [nout_tiles][nstages][tab_block] output lists (then level-1 jobs)
    const int32_t *base;      // [nout_tiles][nrows]
    float *dst;               // output rows, `dst_pitch` floats apart
    int64_t pitch;
    int64_t dst_pitch;
    int64_t nt;
    int64_t block_start;
    int32_t nrows;
    int32_t nouts;
    int32_t nouts_pad;
    int32_t nout_tiles;
    int32_t stage_rows;
    int32_t row_words;
    int32_t nstages;
    int32_t tab_stride;
    int32_t tab_block;        // ints per (tile, stage) table block
    int32_t pat_words;        // floats of pattern rows per stage (0: no sub-band reuse)
    int32_t njobs_max;        // level-1 job slots per stage
    int32_t w_off;            // kAdjFinal: this problem's first weight (floats from BoxArgs::w)
    int64_t x_off;            // kAdjFinal: this problem's x and dX rows (floats from BoxArgs::x, dX)
    int64_t x_pitch;          // kAdjFinal: floats between rows of x and dX
    int64_t part_off;         // kAdjFinal: its weight-gradient partials (floats from BoxArgs::partial)
};

struct SumBatch {
    SumArgs p[DD_MAX_RANGES];
    // a batch of beams: the problems' descriptors in device memory instead
    // of p (ordered by block_start), their src and dst holding byte offsets
    // from src_base and dst_base
    const SumArgs *pd;
    uintptr_t src_base;
    uintptr_t dst_base;
    int64_t nblocks;
    int64_t per_xcd;
    int32_t nprob;
    int32_t max_stage;        // largest stage_rows over the problems
};


// The fields of a problem the stage loop reads, held in registers (read
// through the kernel-argument reference they would be loaded again after
// every direct-to-LDS load, which the compiler takes for a possible write).
struct StageSrc {
    const float *src;
    const int32_t *base;
    const int32_t *tab;       // [nout_tiles][nstages][tab_block]
    int64_t pitch;
    int32_t nrows;
    int32_t row_words;
    int32_t nstages;
    int32_t tab_block;
};

// The window starts of a stage's rows, lane j holding row bs + j's: one
// vector load, issued a stage ahead so that its latency passes during the
// sums (which issue no vector memory operations of their own).
__device__ __forceinline__ int32_t stage_bases(const StageSrc &S, int tile, int bs, int bn, int lane)
{
    return lane < bn ? S.base[int64_t(tile) * S.nrows + bs + lane] : 0;
}

__device__ __forceinline__ void stage_issue_f32(const StageSrc &S, int tile, int64_t t0, int bs,
                                                int bn, int32_t mv, float *buf, int wave, int lane,
                                                int st, float *tbuf)
{
    // Wavefront w stages rows w and w + 8 of the stage (at most 16 rows).
    // Their window starts are read out of mv before any of the stage's
    // direct loads is issued, so that waiting for mv waits for nothing else
    // (the previous stage's loads were waited for before its sums).
    const int32_t m0 = __builtin_amdgcn_readlane(mv, wave);
    const int32_t m1 = __builtin_amdgcn_readlane(mv, wave + kWavesPerBlock);
    const int Wr = S.row_words;
    const int chunks = Wr >> 2;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = wave + h * kWavesPerBlock;
        if (j >= bn)
            break;
        const float *row = S.src + int64_t(bs + j) * S.pitch + t0 + (h ? m1 : m0);
        for (int c0 = 0; c0 < chunks; c0 += kWave) {
            const int q = c0 + lane;
            if (q < chunks)
                __builtin_amdgcn_global_load_lds(row + 4 * q, buf + j * Wr + 4 * c0, 16, 0, 0);
        }
    }
    {
        // the stage's table block (output lists, level-1 jobs), 16 bytes
        // per lane
        const int tchunks = S.tab_block / 4;
        const int32_t *blk = S.tab + (int64_t(tile) * S.nstages + st) * S.tab_block;
        for (int c0 = wave * kWave; c0 < tchunks; c0 += kBlock) {
            const int q = c0 + lane;
            if (q < tchunks)
                __builtin_amdgcn_global_load_lds(blk + 4 * q, tbuf + 4 * c0, 16, 0, 0);
        }
    }
}

// Epilogues of the float32 shift-and-sum:
//   kWrite    write the outputs;
//   kBoxLoss  sum over valid windows of (boxcar_w(out))^2 for w = 1, 2, 4,
//             ..., max_width, windows starting in the first t_stride samples
//             of the tile; one partial per workgroup (fixed-order tree);
//   kBoxGrad  dL/dout = 2 * sum_w sum_{j<w} B_w[t - j] (valid windows only)
//             for the tile's samples [t_lead, t_lead + t_stride).
// Boxcar sums are formed by doubling, B_2w[t] = B_w[t] + B_w[t + w], through
// one LDS row per wave; the window sums of the gradient likewise.
//   kAdjFinal the adjoint of a plan with one range at full resolution: its
//             outputs are the channels' G, so the epilogue writes
//             dX[c][t] = w_c * G[c][t] and one partial per (channel, time
//             tile) of dw_c = sum_t x[c][t] * G[c][t] (fixed-order sums);
//             G itself is never stored.
enum { kWrite = 0, kBoxLoss = 1, kBoxGrad = 2, kAdjFinal = 3 };

// LDS rows of kFSpan floats per wave that a boxcar epilogue uses
__host__ __device__ constexpr int box_rows(int mode) { return mode == kBoxGrad ? 2 : 1; }

struct BoxArgs {
    float *partial;           // kBoxLoss: one float per workgroup; kAdjFinal:
                              // per problem (at its part_off), [nouts][time tiles]
                              // weight-gradient partials
    int64_t t_stride;         // samples between consecutive time tiles
    int64_t t_lead;           // the first tile starts at sample -t_lead
    int32_t max_width;        // largest boxcar width (a power of two <= 32)
    int32_t pad_;
    const float *x;           // kAdjFinal: input rows (NULL: no weight gradient)
    const float *w;           // kAdjFinal: channel weights (NULL: all 1)
    float *dX;                // kAdjFinal: input-gradient rows (NULL: not wanted)
};

__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

typedef float f4v __attribute__((ext_vector_type(4)));

// One output's list of a stage (its entries and the class-ends word) from
// LDS, waited for in the same instruction block: NL 16-byte reads of 4
// entries each (2 when a stage has at most 8 rows, else 4).  Written out
// because the compiler, seeing LDS reads it cannot tell apart from the next
// stage's direct loads in flight, would put a wait for those loads before
// them and so undo the overlap of the staging with the sums.
template <int NL>
__device__ __forceinline__ void lds_list(const float *p, const float *pe, f4v (&q)[NL], float &e)
{
    const uint32_t la = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p));
    const uint32_t le = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(pe));
    if constexpr (NL == 2) {
        asm volatile("ds_read_b128 %0, %3\n\t"
                     "ds_read_b128 %1, %3 offset:16\n\t"
                     "ds_read_b32 %2, %4\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(q[0]), "=&v"(q[1]), "=&v"(e)
                     : "v"(la), "v"(le)
                     : "memory");
    } else {
        static_assert(NL == 4, "lists are read as 2 or 4 granules");
        asm volatile("ds_read_b128 %0, %5\n\t"
                     "ds_read_b128 %1, %5 offset:16\n\t"
                     "ds_read_b128 %2, %5 offset:32\n\t"
                     "ds_read_b128 %3, %5 offset:48\n\t"
                     "ds_read_b32 %4, %6\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(q[0]), "=&v"(q[1]), "=&v"(q[2]), "=&v"(q[3]), "=&v"(e)
                     : "v"(la), "v"(le)
                     : "memory");
    }
}

// Lane l receives lane l + 1's v (lane 63 receives 0); the compiler folds
// the move into the add that consumes it.
__device__ __forceinline__ float from_next_lane(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                  kDppWaveShl1, 0xF, 0xF, true));
}

// Sample j of a window that starts R floats into granule g: g[j + R] while
// inside it, else the head of the next lane's granule.
template <int R, int J>
__device__ __forceinline__ float window_at(const f4v g)
{
    if constexpr (J + R < 4)
        return g[J + R];
    else
        return from_next_lane(g[J + R - 4]);
}

template <int R>
__device__ __forceinline__ void add_window(float *acc, const f4v g)
{
    acc[0] += window_at<R, 0>(g);
    acc[1] += window_at<R, 1>(g);
    acc[2] += window_at<R, 2>(g);
    acc[3] += window_at<R, 3>(g);
}

// The rows of one class (delay mod 4 = R) of one output in one stage:
// entries [i, end) of its list, each the LDS float offset of the row's
// first granule; lane l adds granules l + 63g (g < kFG) of each.  Two rows
// per step when kFG is 2, one when it is 4.
constexpr int kFG = dd::kF32Words / 4;          // granules per lane and output

template <int R, int NE>
__device__ __forceinline__ void add_class(float *acc, const float *A, const int (&ent)[NE], int &i,
                                          int end, int lane)
{
    if constexpr (kFG <= 2) {
        for (; i + 1 < end; i += 2) {
            const f4v *p = reinterpret_cast<const f4v *>(A + ent[i]) + lane;
            const f4v *q = reinterpret_cast<const f4v *>(A + ent[i + 1]) + lane;
            f4v pv[kFG], qv[kFG];
#pragma unroll
            for (int g = 0; g < kFG; ++g) {
                pv[g] = p[(kWave - 1) * g];
                qv[g] = q[(kWave - 1) * g];
            }
#pragma unroll
            for (int g = 0; g < kFG; ++g)
                add_window<R>(acc + 4 * g, pv[g]);
#pragma unroll
            for (int g = 0; g < kFG; ++g)
                add_window<R>(acc + 4 * g, qv[g]);
        }
    }
    for (; i < end; ++i) {
        const f4v *p = reinterpret_cast<const f4v *>(A + ent[i]) + lane;
        f4v pv[kFG];
#pragma unroll
        for (int g = 0; g < kFG; ++g)
            pv[g] = p[(kWave - 1) * g];
#pragma unroll
        for (int g = 0; g < kFG; ++g)
            add_window<R>(acc + 4 * g, pv[g]);
    }
}

// Level 1 of sub-band reuse: one pattern row, the sum of its group's rows
// (up to kSbGroup entries, ordered by class) at their offsets, G = 5
// granules per lane (samples 4(l + 63g) + j of the row's 1260); lanes 0..62
// store their granules at the job's destination.
constexpr int kSbJobInts = dd::kSbJobInts;

template <int G>
__device__ __forceinline__ void pattern_pass(float *lds, const int (&e)[4], uint32_t ends, int dest,
                                             int lane)
{
    float acc[4 * G];
#pragma unroll
    for (int k = 0; k < 4 * G; ++k)
        acc[k] = 0.0f;
    int i = 0;
    auto entry = [&](int k) { return k == 0 ? e[0] : k == 1 ? e[1] : k == 2 ? e[2] : e[3]; };
    auto one = [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        const int end = int((ends >> (8 * R)) & 0xFF);
        for (; i < end; ++i) {
            const f4v *p = reinterpret_cast<const f4v *>(lds + entry(i)) + lane;
            f4v v[G];
#pragma unroll
            for (int g = 0; g < G; ++g)
                v[g] = p[(kWave - 1) * g];
#pragma unroll
            for (int g = 0; g < G; ++g)
                add_window<R>(acc + 4 * g, v[g]);
        }
    };
    one(std::integral_constant<int, 0>());
    one(std::integral_constant<int, 1>());
    one(std::integral_constant<int, 2>());
    one(std::integral_constant<int, 3>());
    if (lane < kWave - 1) {
        f4v *out = reinterpret_cast<f4v *>(lds + dest) + lane;
#pragma unroll
        for (int g = 0; g < G; ++g)
            out[(kWave - 1) * g] = f4v{acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]};
    }
}

__device__ __forceinline__ void build_pattern(float *lds, const float *job, int lane)
{
    const int *rec = reinterpret_cast<const int *>(job);
    const int dest = __builtin_amdgcn_readfirstlane(rec[0]);
    const uint32_t ends = uint32_t(__builtin_amdgcn_readfirstlane(rec[2]));
    const int e[4] = {__builtin_amdgcn_readfirstlane(rec[3]), __builtin_amdgcn_readfirstlane(rec[4]),
                      __builtin_amdgcn_readfirstlane(rec[5]), __builtin_amdgcn_readfirstlane(rec[6])};
    pattern_pass<dd::kSbPatWords / 252>(lds, e, ends, dest, lane);   // rec[1] is always 5
}

// NL: 16-byte granules per output list (2 when every problem's stage has at
// most 8 rows, else 4).  PD: the problems come from device descriptors (a
// batch of beams), found by binary search on block_start.
template <int MODE, int NL, bool PD>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void
k_shiftsum_f32(const SumBatch a, const BoxArgs bx)
{
    extern __shared__ __attribute__((aligned(16))) float ldsf[];
    const int64_t bid = blockIdx.x;
    const int64_t L = (bid % kXcds) * a.per_xcd + bid / kXcds;
    if (L >= a.nblocks)
        return;
    int r = 0;
    if constexpr (PD) {
        int hi = a.nprob - 1;
        while (r < hi) {
            const int mid = (r + hi + 1) >> 1;
            if (L >= a.pd[mid].block_start)
                r = mid;
            else
                hi = mid - 1;
        }
    } else {
        for (int i = 1; i < a.nprob; ++i)
            if (L >= a.p[i].block_start)
                r = i;
    }
    const SumArgs &R = PD ? a.pd[r] : a.p[r];
    const float *src_rows = reinterpret_cast<const float *>(a.src_base + reinterpret_cast<uintptr_t>(R.src));
    float *dst_rows = reinterpret_cast<float *>(a.dst_base + reinterpret_cast<uintptr_t>(R.dst));
    const int64_t lb = L - R.block_start;
    const int64_t tt = lb / R.nout_tiles;
    const int tile = int(lb - tt * R.nout_tiles);
    const int64_t t0 = tt * bx.t_stride - bx.t_lead;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int aw0 = tile * kFTileA + wave * kFP;
    const int C = R.stage_rows;
    const int Wr = R.row_words;
    const int CW = C * Wr;
    const int nrows = R.nrows;
    const int nst = R.nstages;
    const StageSrc S = {src_rows, R.base, R.off, R.pitch, nrows, Wr, nst, R.tab_block};
    const int TS = R.tab_stride;
    const int PW = R.pat_words;                 // pattern rows after the staged rows
    const int NJ = R.njobs_max;

    // acc[d][k*4 + j]: output aw0 + d at tile sample 4*(lane + 63k) + j
    float acc[kFP][kFW];
#pragma unroll
    for (int d = 0; d < kFP; ++d)
#pragma unroll
        for (int k = 0; k < kFW; ++k)
            acc[d][k] = 0.0f;

    stage_issue_f32(S, tile, t0, 0, min(C, nrows), stage_bases(S, tile, 0, min(C, nrows), lane), ldsf,
                    wave, lane, 0, ldsf + CW + PW);
    for (int st = 0; st < nst; ++st) {
        const float *A = ldsf;
        const float *T = A + CW + PW;
        wait_loads();
        lds_barrier();
        const int bs_next = (st + 1) * C;
        const int32_t mv_next = st + 1 < nst ? stage_bases(S, tile, bs_next, min(C, nrows - bs_next), lane) : 0;
        if (NJ > 0) {
            // level 1: this stage's pattern rows, one job per wavefront in
            // turn (nothing is in flight: plain LDS reads)
            const float *J = T + kFTileA * TS;
            const int njobs = __builtin_amdgcn_readfirstlane(__float_as_int(J[kSbJobInts * NJ]));
            for (int j = wave; j < njobs; j += kWavesPerBlock)
                build_pattern(ldsf, J + kSbJobInts * j, lane);
            lds_barrier();
        }
#pragma unroll
        for (int d = 0; d < kFP; ++d) {
            // this output's list from LDS: its entries, then the class ends
            // in the list's last word
            const float *Lp = T + (wave * kFP + d) * TS;
            f4v qs[NL];
            float ef;
            lds_list<NL>(Lp, Lp + (TS - 1), qs, ef);
            const uint32_t ends = uint32_t(__builtin_amdgcn_readfirstlane(__float_as_int(ef)));
            // 16 slots whatever NL: the compiler indexes an array this size
            // by relative register moves (a shorter one became chains of
            // selects per access)
            int ent[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ent[4 * k] = k < NL ? __float_as_int(qs[k].x) : 0;
                ent[4 * k + 1] = k < NL ? __float_as_int(qs[k].y) : 0;
                ent[4 * k + 2] = k < NL ? __float_as_int(qs[k].z) : 0;
                ent[4 * k + 3] = k < NL ? __float_as_int(qs[k].w) : 0;
            }
            int i = 0;
            add_class<0>(acc[d], A, ent, i, int(ends & 0xFF), lane);
            add_class<1>(acc[d], A, ent, i, int((ends >> 8) & 0xFF), lane);
            add_class<2>(acc[d], A, ent, i, int((ends >> 16) & 0xFF), lane);
            add_class<3>(acc[d], A, ent, i, int(ends >> 24), lane);
        }
        if (st + 1 < nst) {
            lds_barrier();          // every wave is done with this stage's rows and lists
            stage_issue_f32(S, tile, t0, bs_next, min(C, nrows - bs_next), mv_next, ldsf, wave, lane, st + 1,
                            ldsf + CW + PW);
        }
    }

    // lane 63 only supplied the next-lane heads: its sums are not outputs.
    // Accumulator k of a lane holds tile sample 4*lane + ks(k); bounds on
    // the series are taken as 32-bit bounds on the tile sample.
    const bool lane_ok = lane < kWave - 1;
    const int tb = 4 * lane;
    const int64_t nt = R.nt;
    const int t_lo = int(min<int64_t>(max<int64_t>(-t0, 0), kFSpan));   // tg >= 0
    const int t_end = int(min<int64_t>(max<int64_t>(nt - t0, -64), kFSpan + 64)); // tg < nt
    if constexpr (MODE == kAdjFinal) {
        const int64_t ntt = (R.nt + kFTileT - 1) / kFTileT;    // the partials' row length
#pragma unroll
        for (int d = 0; d < kFP; ++d) {
            const int c = aw0 + d;
            if (c >= R.nouts)
                break;
            const float wc = bx.w ? bx.w[R.w_off + c] : 1.0f;
            float *dx = bx.dX ? bx.dX + R.x_off + int64_t(c) * R.x_pitch + t0 : nullptr;
            const float *xs = bx.x ? bx.x + R.x_off + int64_t(c) * R.x_pitch + t0 : nullptr;
            float part = 0.0f;
            if (lane_ok) {
#pragma unroll
                for (int k = 0; k < kFW; ++k) {
                    const int t = tb + ks(k);
                    if (t >= t_lo && t < t_end) {
                        if (dx)
                            dx[t] = wc * acc[d][k];
                        if (xs)
                            part += xs[t] * acc[d][k];
                    }
                }
            }
            if (xs) {
                // fixed-order butterfly over the wavefront's lanes
#pragma unroll
                for (int h = kWave / 2; h > 0; h >>= 1)
                    part += __shfl_xor(part, h);
                if (lane == 0)
                    bx.partial[R.part_off + int64_t(c) * ntt + tt] = part;
            }
        }
    } else if constexpr (MODE == kWrite) {
        if (lane_ok) {
#pragma unroll
            for (int d = 0; d < kFP; ++d) {
                const int ao = aw0 + d;
                if (ao >= R.nouts)
                    break;
                float *row = dst_rows + int64_t(ao) * R.dst_pitch + t0;
#pragma unroll
                for (int k = 0; k < kFW; ++k) {
                    const int t = tb + ks(k);
                    if (t >= t_lo && t < t_end)
                        row[t] = acc[d][k];
                }
            }
        }
    } else {
        lds_barrier();                          // staging rows are no longer read
        // per wave: one exchange row (the doubling of B_w and the window
        // sums take turns on it, each pass ending in a wait for the wave's
        // LDS accesses) and, for the gradient, the running sum over widths,
        // of which each lane touches only its own samples
        float *rowR = ldsf + wave * (box_rows(MODE) * kFSpan);
        float *rowS = rowR;
        float *rowG = rowR + kFSpan;
        const int t_str = int(bx.t_stride);
        const int t_lead = int(bx.t_lead);
        float part = 0.0f;
        // one output at a time, its boxcar sums formed in place of its
        // accumulators (the loop is unrolled so that they stay in registers)
#pragma unroll
        for (int d = 0; d < kFP; ++d) {
            const int ao = aw0 + d;
            const bool dm_ok = ao < R.nouts && lane_ok;
            float *b = acc[d];
            if constexpr (MODE == kBoxGrad)
#pragma unroll
                for (int k = 0; k < kFW; ++k)
                    rowG[tb + ks(k)] = 0.0f;
            for (int w = 1; w <= bx.max_width; w *= 2) {
                // windows [t, t + w) inside the series
                const int t_hi = t_end - w;
                if constexpr (MODE == kBoxLoss) {
                    if (dm_ok)
#pragma unroll
                        for (int k = 0; k < kFW; ++k) {
                            const int t = tb + ks(k);
                            if (t < t_str && t >= t_lo && t <= t_hi)
                                part += b[k] * b[k];
                        }
                } else {
                    float c[kFW];
#pragma unroll
                    for (int k = 0; k < kFW; ++k) {
                        const int t = tb + ks(k);
                        c[k] = (dm_ok && t >= t_lo && t <= t_hi) ? b[k] : 0.0f;
                    }
                    for (int h = 1; h < w; h *= 2) {
                        if (lane_ok)
#pragma unroll
                            for (int k = 0; k < kFW; ++k)
                                rowS[tb + ks(k)] = c[k];
                        lds_wave_sync();
#pragma unroll
                        for (int k = 0; k < kFW; ++k) {
                            const int t = tb + ks(k);
                            c[k] += (t >= h && t - h < kFTileT) ? rowS[t - h] : 0.0f;
                        }
                        lds_wave_sync();
                    }
#pragma unroll
                    for (int k = 0; k < kFW; ++k)
                        rowG[tb + ks(k)] += c[k];
                }
                if (w < bx.max_width) {
                    if (lane_ok)
#pragma unroll
                        for (int k = 0; k < kFW; ++k)
                            rowR[tb + ks(k)] = b[k];
                    lds_wave_sync();
#pragma unroll
                    for (int k = 0; k < kFW; ++k) {
                        const int t = tb + ks(k);
                        b[k] += t + w < kFTileT ? rowR[t + w] : 0.0f;
                    }
                    lds_wave_sync();
                }
            }
            if constexpr (MODE == kBoxGrad) {
                if (dm_ok) {
                    float *row = dst_rows + int64_t(ao) * R.dst_pitch + t0;
#pragma unroll
                    for (int k = 0; k < kFW; ++k) {
                        const int t = tb + ks(k);
                        if (t >= t_lead && t < t_lead + t_str && t >= t_lo && t < t_end)
                            row[t] = 2.0f * rowG[t];
                    }
                }
            }
        }
        if constexpr (MODE == kBoxLoss) {
            float *red = ldsf + kWavesPerBlock * box_rows(MODE) * kFSpan;
            red[tid] = part;
            __syncthreads();
            for (int h = kBlock / 2; h > 0; h >>= 1) {
                if (tid < h)
                    red[tid] += red[tid + h];
                __syncthreads();
            }
            if (tid == 0)
                bx.partial[L] = red[0];
        }
    }
}

struct FinRange {
    const float *G;
    int64_t Gpitch;
    int64_t nbin;
    int32_t ds;
    int32_t pad_;
};

struct FinArgs {
    FinRange r[DD_MAX_RANGES];
    const float *x;
    const float *w;
    float *dX;
    float *partial;
    int64_t nsamp;
    int64_t chunk_len;
    int32_t nranges;
    int32_t nchunks;
};

// A thread handles 4 consecutive samples.  VEC: the rows of x and dX start
// on 16-byte boundaries, so those are float4 accesses; G rows always do.
// A range's bin index t / ds is stepped sample by sample after one division.
template <bool VEC>
__global__ __launch_bounds__(256) void k_adj_finalize(const FinArgs a)
{
    __shared__ float red[256];
    const int64_t c = blockIdx.y;
    const int chunk = blockIdx.x;
    const int64_t t_begin = int64_t(chunk) * a.chunk_len;   // a multiple of 4
    const int64_t t_end = min(a.nsamp, t_begin + a.chunk_len);
    const float wc = a.w ? a.w[c] : 1.0f;
    float acc = 0.0f;
    for (int64_t t = t_begin + 4 * int64_t(threadIdx.x); t < t_end; t += 4 * 256) {
        const int n = int(min<int64_t>(4, t_end - t));
        float g[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int r = 0; r < a.nranges; ++r) {
            const FinRange &R = a.r[r];
            const float *Gr = R.G + c * R.Gpitch;
            const int64_t lim = int64_t(R.ds) * R.nbin;      // samples inside a whole bin
            if (R.ds == 1 && t + 4 <= lim) {
                const float4 v = *reinterpret_cast<const float4 *>(Gr + t);
                g[0] += v.x;
                g[1] += v.y;
                g[2] += v.z;
                g[3] += v.w;
            } else {
                int64_t q = t < 0xFFFFFFFFll ? int64_t(uint32_t(t) / uint32_t(R.ds)) : t / R.ds;
                int rr = int(t - q * R.ds);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (t + j < lim)
                        g[j] += Gr[q];
                    if (++rr == R.ds) {
                        rr = 0;
                        ++q;
                    }
                }
            }
        }
        float *dx = a.dX ? a.dX + c * a.nsamp + t : nullptr;
        const float *xs = a.x ? a.x + c * a.nsamp + t : nullptr;
        if (VEC && n == 4) {
            if (dx)
                *reinterpret_cast<float4 *>(dx) = make_float4(wc * g[0], wc * g[1], wc * g[2], wc * g[3]);
            if (xs) {
                const float4 xv = *reinterpret_cast<const float4 *>(xs);
                acc += xv.x * g[0];
                acc += xv.y * g[1];
                acc += xv.z * g[2];
                acc += xv.w * g[3];
            }
        } else {
            for (int j = 0; j < n; ++j) {
                if (dx)
                    dx[j] = wc * g[j];
                if (xs)
                    acc += xs[j] * g[j];
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        a.partial[c * a.nchunks + chunk] = red[0];
}

__global__ __launch_bounds__(256) void k_reduce_rows(const float *__restrict__ partial, int n,
                                                     float *__restrict__ out)
{
    __shared__ float red[256];
    const int64_t c = blockIdx.x;
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256)
        acc += partial[c * n + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[c] = red[0];
}


// ---------------------------------------------------------------------------
// Batched integer forward: one persistent launch per kernel group over the
// work items of its beams.  Item L of the group's cost-ordered list belongs
// to the descriptor whose item_start is the largest not above L.  The list
// is cut into one contiguous queue per XCD of equal cost; a workgroup dealt
// to XCD x takes its next item from queue x (a counter in the workspace,
// reset by k_reset_counters before the launches), so the tiles of a time
// tile still share an L2.
// ---------------------------------------------------------------------------

struct BatchDesc {
    const int32_t *offT;
    const int32_t *baseT;
    int64_t src_off;          // bytes into the workspace
    int64_t out_off;          // elements into the batch output
    int64_t pitch;
    int64_t nout;
    int64_t item_start;
    int32_t nchans;
    int32_t ndms;
    int32_t ndms_pad;
    int32_t ndm_tiles;
    int32_t stage_chans;
    int32_t row_words;
    int32_t widen_every;
    int32_t pad_;
};

__global__ void k_reset_counters(int32_t *counters, int n)
{
    if (int(threadIdx.x) < n)
        counters[threadIdx.x] = 0;
}

// Item bounds of the per-XCD queues.
struct QueueBounds {
    int64_t b[dd::kBatchQueues + 1];
};
static_assert(dd::kBatchQueues == kXcds, "one queue per XCD");

// The next work item of a workgroup dealt to XCD x: from its own queue, and
// once that is empty from the other XCDs' queues in turn (the cheapest items
// of each sit at its end), or -1 when every queue is empty.  Counters only
// grow, so an item is taken exactly once.
__device__ __forceinline__ int64_t next_item(const QueueBounds &qb, int32_t *counters, int x)
{
    for (int k = 0; k < kXcds; ++k) {
        const int q = (x + k) % kXcds;
        const int64_t i = qb.b[q] + atomicAdd(&counters[q], 1);
        if (i < qb.b[q + 1])
            return i;
    }
    return -1;
}

template <bool DEDUP, int WAVES, int NW>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(4, 4))) void
k_dedisp_u8_batch(const BatchDesc *__restrict__ descs, const int64_t *__restrict__ starts,
                  int ndesc, const QueueBounds qb, const char *ws, int32_t *out,
                  int32_t *counters)
{
    // 16-byte rows: the staging loads and the odd-copy build move 16 bytes
    // per lane, so the dynamic region must not start at the static s_item's
    // 8-byte end.
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = next_item(qb, counters, blockIdx.x % kXcds);
        __syncthreads();
        const int64_t L = s_item;
        __syncthreads();
        if (L < 0)
            break;
        int lo = 0, hi = ndesc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (starts[mid] <= L)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchDesc &D = descs[lo];
        RangeArgs R;
        R.src = reinterpret_cast<const uint16_t *>(ws + D.src_off);
        R.offT = D.offT;
        R.baseT = D.baseT;
        R.out = out + D.out_off;
        R.pitch = D.pitch;
        R.nout = D.nout;
        R.block_start = 0;
        R.nchans = D.nchans;
        R.ndms = D.ndms;
        R.ndms_pad = D.ndms_pad;
        R.ndm_tiles = D.ndm_tiles;
        R.stage_chans = D.stage_chans;
        R.row_words = D.row_words;
        R.widen_every = D.widen_every;
        dedisp_tile_u8<DEDUP, WAVES, NW>(R, L - D.item_start, lds);
    }
}

// Variant 3 in a persistent launch of its own: each (beam, range) carries its
// whole sub-band range; the workspace and output pointers are the launch's
// own buffers plus the descriptor's offsets.
struct SbBatchDesc {
    SbRange R;                // src and out unset (set per launch from the offsets)
    int64_t src_off;          // bytes into the workspace
    int64_t out_off;          // elements into the batch output
    int64_t item_start;
    int64_t pad_[2];
};

static_assert(sizeof(SbBatchDesc) % 32 == 0, "descriptors are read 32 bytes at a time");

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// The descriptors and item starts do not change during a launch: read
// through the constant address space, they load into scalar registers (the
// item index is uniform) and the compiler may load a field again rather
// than hold it in a register through the whole item.
#define DD_CONST __attribute__((address_space(4)))

template <int WAVES, int DPW, int NW>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(WAVES / 4, WAVES / 4))) void
k_dedisp_u8_sb_batch(const SbBatchDesc *__restrict__ descs, const int64_t *__restrict__ starts,
                     int ndesc, const QueueBounds qb, const char *ws, int32_t *out,
                     int32_t *counters)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ int64_t s_item;
    for (;;) {
        // thread 0 takes the next item (-1: every queue empty), so that no
        // queue bound stays live through the item
        if (threadIdx.x == 0)
            s_item = next_item(qb, counters, blockIdx.x % kXcds);
        __syncthreads();
        // the item is the same for the whole workgroup: keep it (and with it
        // the descriptor's fields) in scalar registers
        const int64_t L = uniform64(s_item);
        __syncthreads();
        if (L < 0)
            break;
        const DD_CONST int64_t *cs = (const DD_CONST int64_t *)starts;
        int lo = 0, hi = ndesc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cs[mid] <= L)
                lo = mid;
            else
                hi = mid - 1;
        }
        const DD_CONST SbBatchDesc &D = ((const DD_CONST SbBatchDesc *)descs)[lo];
        dedisp_tile_sb<WAVES, DPW, NW>(D.R, reinterpret_cast<const uint16_t *>(ws + D.src_off),
                                       out + D.out_off, L - D.item_start, lds);
    }
}

dd_status launch_check(const char *what)
{
    if (fault_requested("launch")) {
        dd::set_error(std::string(what) + ": launch failure forced by DD_FAULT=launch");
        return DD_ERR_HIP;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, what);
    return DD_OK;
}

// The levels ds = 1, 2, 4, 8, 16 that a plan has, binned from the raw input
// in one pass: a thread reads 16 consecutive samples of one channel (one
// 16-byte load) and writes the 16/ds bins of each present level, from
// packed 16-bit sums (no half can carry: 16 * 255 < 65536).  Needs
// nsamp % 16 == 0 and a 16-byte aligned input.
struct FusedLevels {
    uint16_t *dst[5];         // ds = 1, 2, 4, 8, 16; nullptr when absent
    int64_t pitch[5];
};

__global__ __launch_bounds__(256) void k_bin_fused_u8(const uint8_t *__restrict__ src,
                                                      int64_t nsamp, FusedLevels L, int nchans)
{
    const int64_t ng = nsamp / 16;
    for (int64_t c = blockIdx.y; c < nchans; c += gridDim.y) {
        const uint4 *row = reinterpret_cast<const uint4 *>(src + c * nsamp);
        for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < ng;
             g += int64_t(gridDim.x) * blockDim.x) {
            const uint4 v = row[g];
            const uint32_t x[4] = {v.x, v.y, v.z, v.w};
            uint32_t l1[8], l2[4], l4[2], l8, l16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // bytes b0..b3 of word i: ds 1 as the pairs (b0, b1) and
                // (b2, b3); ds 2 as (b0 + b1, b2 + b3)
                l1[2 * i] = (x[i] & 0xffu) | ((x[i] & 0xff00u) << 8);
                l1[2 * i + 1] = ((x[i] >> 16) & 0xffu) | ((x[i] >> 8) & 0xff0000u);
                l2[i] = (x[i] & 0x00ff00ffu) + ((x[i] >> 8) & 0x00ff00ffu);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                // ds 4: one sum per input word, two words per output pair
                const uint32_t a = (l2[2 * i] & 0xffffu) + (l2[2 * i] >> 16);
                const uint32_t b = (l2[2 * i + 1] & 0xffffu) + (l2[2 * i + 1] >> 16);
                l4[i] = a | (b << 16);
            }
            {
                const uint32_t a = (l4[0] & 0xffffu) + (l4[0] >> 16);
                const uint32_t b = (l4[1] & 0xffffu) + (l4[1] >> 16);
                l8 = a | (b << 16);
                l16 = a + b;
            }
            if (L.dst[0]) {
                uint4 *o = reinterpret_cast<uint4 *>(L.dst[0] + c * L.pitch[0] + 16 * g);
                o[0] = make_uint4(l1[0], l1[1], l1[2], l1[3]);
                o[1] = make_uint4(l1[4], l1[5], l1[6], l1[7]);
            }
            if (L.dst[1])
                *reinterpret_cast<uint4 *>(L.dst[1] + c * L.pitch[1] + 8 * g) =
                    make_uint4(l2[0], l2[1], l2[2], l2[3]);
            if (L.dst[2])
                *reinterpret_cast<uint2 *>(L.dst[2] + c * L.pitch[2] + 4 * g) = make_uint2(l4[0], l4[1]);
            if (L.dst[3])
                *reinterpret_cast<uint32_t *>(L.dst[3] + c * L.pitch[3] + 2 * g) = l8;
            if (L.dst[4])
                L.dst[4][c * L.pitch[4] + g] = uint16_t(l16);
        }
    }
}

// ---------------------------------------------------------------------------
// Power-of-two levels (ds = 1, 2, 4, 8, 16) of rows of any length and any
// byte alignment, for many beams in one launch.  A block takes one segment
// of kBinSeg samples of one row: it copies the segment's bytes into LDS with
// aligned 4-byte loads from the aligned-down address (no load starts past
// the input's end), and each thread realigns its 16 samples with
// v_alignbyte and forms the levels as k_bin_fused_u8 does.  A row's last,
// partial group writes only the bins that lie inside the row.
// ---------------------------------------------------------------------------

constexpr int kBinSeg = 4096;
constexpr int kBinThreads = kBinSeg / 16;

struct BinJob {
    int64_t in_off;           // bytes into the input buffer: row 0 of this beam
    int64_t nsamp;
    int64_t ws_off[5];        // bytes into the workspace of level ds = 2^k, or -1
    int64_t pitch[5];         // samples per row of each level
    int64_t block_start;      // first block of this job in the launch
    int32_t nchans;
    int32_t nseg;             // segments per row
};

// Level K's bins of one 16-sample group: 16 >> K bins, two per word (K < 4)
// or one (K = 4).  A whole group is stored with one vector store; the row's
// last, partial group stores only the bins that lie inside the row.
template <int K>
__device__ __forceinline__ void store_level(const BinJob &J, char *ws, int64_t row, int64_t g0,
                                            bool full, const uint32_t *v)
{
    if (J.ws_off[K] < 0)
        return;
    uint16_t *o = reinterpret_cast<uint16_t *>(ws + J.ws_off[K]) + row * J.pitch[K] + (g0 >> K);
    if (full) {
        if constexpr (K == 0) {
            reinterpret_cast<uint4 *>(o)[0] = make_uint4(v[0], v[1], v[2], v[3]);
            reinterpret_cast<uint4 *>(o)[1] = make_uint4(v[4], v[5], v[6], v[7]);
        } else if constexpr (K == 1) {
            *reinterpret_cast<uint4 *>(o) = make_uint4(v[0], v[1], v[2], v[3]);
        } else if constexpr (K == 2) {
            *reinterpret_cast<uint2 *>(o) = make_uint2(v[0], v[1]);
        } else if constexpr (K == 3) {
            *reinterpret_cast<uint32_t *>(o) = v[0];
        } else {
            *o = uint16_t(v[0]);
        }
        return;
    }
    const int64_t nbin = J.nsamp >> K;
#pragma unroll
    for (int i = 0; i < (16 >> K); ++i)
        if ((g0 >> K) + i < nbin)
            o[i] = K == 4 ? uint16_t(v[0]) : uint16_t((i & 1) ? v[i >> 1] >> 16 : v[i >> 1] & 0xffffu);
}

__device__ __forceinline__ void bin_pow2_block(const BinJob &J, int64_t b, const uint8_t *in,
                                               const uint8_t *in_end, char *ws, uint32_t *lds)
{
    const int64_t row = b / J.nseg;
    const int seg = int(b - row * J.nseg);
    const int64_t t_seg = int64_t(seg) * kBinSeg;
    const uint8_t *p = in + J.in_off + row * J.nsamp + t_seg;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(p);
    const uint32_t *a = reinterpret_cast<const uint32_t *>(pa & ~uintptr_t(3));
    const uint32_t sh = uint32_t(pa & 3);
    // (a 4-byte load that starts before the input's end cannot cross a page
    // the input does not touch)
    for (int i = threadIdx.x; i <= kBinSeg / 4; i += kBinThreads)
        lds[i] = reinterpret_cast<const uint8_t *>(a + i) < in_end ? a[i] : 0u;
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t g0 = t_seg + 16 * t;
    if (g0 < J.nsamp) {
        uint32_t w[5];
#pragma unroll
        for (int k = 0; k < 5; ++k)
            w[k] = lds[4 * t + k];
        uint32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            x[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
        uint32_t l1[8], l2[4], l4[2], l8, l16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            l1[2 * i] = (x[i] & 0xffu) | ((x[i] & 0xff00u) << 8);
            l1[2 * i + 1] = ((x[i] >> 16) & 0xffu) | ((x[i] >> 8) & 0xff0000u);
            l2[i] = (x[i] & 0x00ff00ffu) + ((x[i] >> 8) & 0x00ff00ffu);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const uint32_t u = (l2[2 * i] & 0xffffu) + (l2[2 * i] >> 16);
            const uint32_t v = (l2[2 * i + 1] & 0xffffu) + (l2[2 * i + 1] >> 16);
            l4[i] = u | (v << 16);
        }
        {
            const uint32_t u = (l4[0] & 0xffffu) + (l4[0] >> 16);
            const uint32_t v = (l4[1] & 0xffffu) + (l4[1] >> 16);
            l8 = u | (v << 16);
            l16 = u + v;
        }
        const bool full = g0 + 16 <= J.nsamp;
        store_level<0>(J, ws, row, g0, full, l1);
        store_level<1>(J, ws, row, g0, full, l2);
        store_level<2>(J, ws, row, g0, full, l4);
        store_level<3>(J, ws, row, g0, full, &l8);
        store_level<4>(J, ws, row, g0, full, &l16);
    }
    __syncthreads();                                // the next block reuses the LDS
}

// One job by value (a single plan's input), blocks in a grid-stride loop.
__global__ __launch_bounds__(kBinThreads) void k_bin_pow2_u8(const BinJob job, const uint8_t *in,
                                                             const uint8_t *in_end, char *ws,
                                                             int64_t nblocks)
{
    __shared__ uint32_t lds[kBinSeg / 4 + 4];
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x)
        bin_pow2_block(job, b, in, in_end, ws, lds);
}

// Many jobs (the beams of a batch), in device memory ordered by
// block_start; each block finds its job by bisection.
__global__ __launch_bounds__(kBinThreads) void k_bin_pow2_u8_batch(const BinJob *__restrict__ jobs,
                                                                   int njobs, const uint8_t *in,
                                                                   const uint8_t *in_end, char *ws,
                                                                   int64_t nblocks)
{
    __shared__ uint32_t lds[kBinSeg / 4 + 4];
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].block_start <= b)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BinJob &J = jobs[lo];
        bin_pow2_block(J, b - J.block_start, in, in_end, ws, lds);
    }
}

// The power-of-two levels a plan has, as a job (ws offsets relative to the
// plan's workspace, input at in_off); returns whether it has any.
bool pow2_job(const Plan &p, int64_t in_off, size_t ws_off, BinJob &J)
{
    J.in_off = in_off;
    J.nsamp = p.nsamp;
    J.nchans = p.nchans;
    J.nseg = int32_t((p.nsamp + kBinSeg - 1) / kBinSeg);
    J.block_start = 0;
    bool any = false;
    for (int k = 0; k < 5; ++k) {
        J.ws_off[k] = -1;
        J.pitch[k] = 0;
    }
    for (const dd::BinLevel &lv : p.levels)
        for (int k = 0; k < 5; ++k)
            if (lv.ds == (1 << k)) {
                J.ws_off[k] = int64_t(ws_off + lv.ws_offset);
                J.pitch[k] = lv.pitch;
                any = true;
            }
    return any;
}

// Levels that are not powers of two up to 16, each from its source level
// (or the raw input), in increasing downsample order.
dd_status bin_u8_rest(const Plan &p, const uint8_t *d_in, char *d_ws, hipStream_t stream)
{
    for (size_t i = 0; i < p.levels.size(); ++i) {
        const dd::BinLevel &lv = p.levels[i];
        if (lv.ds <= 16 && (lv.ds & (lv.ds - 1)) == 0)
            continue;
        uint16_t *dst = reinterpret_cast<uint16_t *>(d_ws + lv.ws_offset);
        const dim3 grid(unsigned(std::min<int64_t>((lv.nbin + 1023) / 1024, 1024)),
                        unsigned(std::min<int32_t>(p.nchans, 65535)));
        if (lv.src < 0) {
            hipLaunchKernelGGL(k_bin_u16<uint8_t>, grid, dim3(256), 0, stream, d_in, p.nsamp,
                               dst, lv.pitch, lv.nbin, lv.factor, p.nchans);
        } else {
            const dd::BinLevel &sl = p.levels[lv.src];
            const uint16_t *src = reinterpret_cast<const uint16_t *>(d_ws + sl.ws_offset);
            hipLaunchKernelGGL(k_bin_u16<uint16_t>, grid, dim3(256), 0, stream, src, sl.pitch,
                               dst, lv.pitch, lv.nbin, lv.factor, p.nchans);
        }
        dd_status st = launch_check("k_bin_u16");
        if (st != DD_OK)
            return st;
    }
    return DD_OK;
}

dd_status bin_u8(const Plan &p, const uint8_t *d_in, char *d_ws, hipStream_t stream)
{
    // Levels ds = 1, 2, 4, 8, 16 in one pass over the raw input: 16-byte
    // loads when the rows allow them, else through LDS realignment; every
    // other level from its source level (or the raw input).
    BinJob J;
    if (pow2_job(p, 0, 0, J)) {
        if (p.nsamp % 16 == 0 && reinterpret_cast<uintptr_t>(d_in) % 16 == 0) {
            FusedLevels L;
            std::memset(&L, 0, sizeof(L));
            for (int k = 0; k < 5; ++k)
                if (J.ws_off[k] >= 0) {
                    L.dst[k] = reinterpret_cast<uint16_t *>(d_ws + J.ws_off[k]);
                    L.pitch[k] = J.pitch[k];
                }
            const int64_t ng = p.nsamp / 16;
            const dim3 grid(unsigned(std::min<int64_t>((ng + 255) / 256, 1024)),
                            unsigned(std::min<int32_t>(p.nchans, 65535)));
            hipLaunchKernelGGL(k_bin_fused_u8, grid, dim3(256), 0, stream, d_in, p.nsamp, L,
                               p.nchans);
            dd_status st = launch_check("k_bin_fused_u8");
            if (st != DD_OK)
                return st;
        } else {
            const int64_t nblocks = int64_t(p.nchans) * J.nseg;
            const uint8_t *end = d_in + int64_t(p.nchans) * p.nsamp;
            hipLaunchKernelGGL(k_bin_pow2_u8, dim3(unsigned(std::min<int64_t>(nblocks, 1 << 20))),
                               dim3(kBinThreads), 0, stream, J, d_in, end, d_ws, nblocks);
            dd_status st = launch_check("k_bin_pow2_u8");
            if (st != DD_OK)
                return st;
        }
    }
    return bin_u8_rest(p, d_in, d_ws, stream);
}

// A variant-3 range's fields apart from its input and output pointers.
void fill_sb_range(const Plan &p, const DeviceTables &t, const RangeInfo &ri, SbRange &R)
{
    const dd::BinLevel &lv = p.levels[ri.level];
    R.pitch = lv.pitch;
    R.baseT = t.baseT + ri.base_offset;
    R.qcnt = t.qcnt + ri.sb_n_offset;
    R.qoff = t.qoff + ri.sb_q_offset;
    R.offC = t.offC + ri.sb_c_offset;
    R.nout = ri.nout;
    R.block_start = ri.block_start;
    R.nchans = p.nchans;
    R.ndms = ri.ndms;
    R.ndm_tiles = ri.ndm_tiles;
    R.stage_chans = ri.stage_chans;
    R.row_words = ri.row_words;
    R.widen_every = ri.widen_every;
    R.sb_chans = ri.sb_chans;
    R.nsub = ri.sb_nsub;
    R.jmax = ri.sb_jmax;
    R.qwords = ri.sb_qwords;
    R.nslot = ri.sb_nslot;
    R.tb_words = ri.sb_tb_words;
}

// The direct kernel of a strategy: variant (re-read test), wavefronts and
// time tile (2 or 4 words of two samples per lane).
const void *direct_kernel(bool dedup, int waves, int time_tile)
{
    const bool w4 = waves == 4, t2 = time_tile == 2 * kWave * 2;
    if (dedup)
        return w4 ? (t2 ? reinterpret_cast<const void *>(k_dedisp_u8<true, 4, 2>)
                        : reinterpret_cast<const void *>(k_dedisp_u8<true, 4, 4>))
                  : (t2 ? reinterpret_cast<const void *>(k_dedisp_u8<true, 8, 2>)
                        : reinterpret_cast<const void *>(k_dedisp_u8<true, 8, 4>));
    return w4 ? (t2 ? reinterpret_cast<const void *>(k_dedisp_u8<false, 4, 2>)
                    : reinterpret_cast<const void *>(k_dedisp_u8<false, 4, 4>))
              : (t2 ? reinterpret_cast<const void *>(k_dedisp_u8<false, 8, 2>)
                    : reinterpret_cast<const void *>(k_dedisp_u8<false, 8, 4>));
}

// The sub-band kernel of a DM tile and time tile: 16 wavefronts of 12 or 8
// DMs at 256-sample tiles, or 8 wavefronts of 12 or 8 DMs at 256 or 512.
const void *subband_kernel(int dm_tile, int time_tile)
{
    const bool t2 = time_tile == 2 * kWave * 2;
    switch (dm_tile) {
    case 192: return reinterpret_cast<const void *>(k_dedisp_u8_sb<16, 12, 2>);
    case 128: return reinterpret_cast<const void *>(k_dedisp_u8_sb<16, 8, 2>);
    case 96:
        return t2 ? reinterpret_cast<const void *>(k_dedisp_u8_sb<8, 12, 2>)
                  : reinterpret_cast<const void *>(k_dedisp_u8_sb<8, 12, 4>);
    default:
        return t2 ? reinterpret_cast<const void *>(k_dedisp_u8_sb<8, 8, 2>)
                  : reinterpret_cast<const void *>(k_dedisp_u8_sb<8, 8, 4>);
    }
}

dd_status sum_u8_sb(const Plan &p, const DeviceTables &t, int32_t *d_out, const char *d_ws,
                    hipStream_t stream)
{
    SbArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nblocks = p.blocks;
    a.per_xcd = (p.blocks + kXcds - 1) / kXcds;
    a.nranges = int32_t(p.ranges.size());
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        const dd::BinLevel &lv = p.levels[ri.level];
        SbRange &R = a.r[i];
        fill_sb_range(p, t, ri, R);
        R.src = reinterpret_cast<const uint16_t *>(d_ws + lv.ws_offset);
        R.out = d_out + ri.out_offset;
    }
    const int64_t grid = a.per_xcd * kXcds;
    // dm_tile 192 and 128: 16 wavefronts of 12 or 8 DMs x 2 words; 96 and
    // 64: 8 wavefronts of 12 or 8 DMs x 4 words (the plan's time tile matches)
    const void *fn = subband_kernel(p.dm_tile, p.time_tile);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(dd::kMaxLdsBytes));
    void *args[] = {&a};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(unsigned(p.waves * kWave)),
                                   args, p.lds_bytes, stream);
    if (e != hipSuccess)
        return hip_fail(e, "k_dedisp_u8_sb");
    return launch_check("k_dedisp_u8_sb");
}

dd_status sum_u8(const Plan &p, const DeviceTables &t, int32_t *d_out, const char *d_ws,
                 hipStream_t stream)
{
    if (p.subband)
        return sum_u8_sb(p, t, d_out, d_ws, stream);
    FwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nblocks = p.blocks;
    a.per_xcd = (p.blocks + kXcds - 1) / kXcds;
    a.nranges = int32_t(p.ranges.size());
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        const dd::BinLevel &lv = p.levels[ri.level];
        RangeArgs &R = a.r[i];
        R.src = reinterpret_cast<const uint16_t *>(d_ws + lv.ws_offset);
        R.pitch = lv.pitch;
        R.offT = t.offT + ri.off_offset;
        R.baseT = t.baseT + ri.base_offset;
        R.out = d_out + ri.out_offset;
        R.nchans = p.nchans;
        R.nout = ri.nout;
        R.block_start = ri.block_start;
        R.ndms = ri.ndms;
        R.ndms_pad = ri.ndms_pad;
        R.ndm_tiles = ri.ndm_tiles;
        R.stage_chans = ri.stage_chans;
        R.row_words = ri.row_words;
        R.widen_every = ri.widen_every;
    }
    const int64_t grid = a.per_xcd * kXcds;
    const void *fn = direct_kernel(p.dedup, p.waves, p.time_tile);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(dd::kMaxLdsBytes));
    void *args[] = {&a};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(unsigned(p.waves * kWave)), args,
                                   p.lds_bytes, stream);
    if (e != hipSuccess)
        return hip_fail(e, "k_dedisp_u8");
    return launch_check("k_dedisp_u8");
}


// k_level_f32 for one level: the vector form when the source rows start on
// 16-byte boundaries (the level buffers' rows always do), factors 1 and 2
// compiled apart.
void launch_level_f32(const float *src, int64_t src_pitch, const float *w, float *dst,
                      int64_t dst_pitch, int64_t nbin, int factor, int nchans, hipStream_t stream)
{
    const dim3 grid(unsigned(std::min<int64_t>((nbin + 1023) / 1024, 1024)),
                    unsigned(std::min<int32_t>(nchans, 65535)));
    const bool vec = reinterpret_cast<uintptr_t>(src) % 16 == 0 && src_pitch % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(dst) % 16 == 0 && dst_pitch % 4 == 0;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, stream, src, src_pitch, w, dst, dst_pitch, nbin,
                           factor, nchans);
    };
    if (!vec)
        go(k_level_f32<false, 0>);
    else if (factor == 1)
        go(k_level_f32<true, 1>);
    else if (factor == 2)
        go(k_level_f32<true, 2>);
    else
        go(k_level_f32<true, 0>);
}

dd_status bin_f32(const Plan &p, const float *d_in, const float *d_w, char *d_ws, hipStream_t stream)
{
    for (const dd::BinLevel &lv : p.levels) {
        float *dst = reinterpret_cast<float *>(d_ws + lv.ws_offset) + lv.lead;
        if (lv.src < 0) {
            launch_level_f32(d_in, p.nsamp, d_w, dst, lv.pitch, lv.nbin, lv.factor, p.nchans, stream);
        } else {
            const dd::BinLevel &sl = p.levels[lv.src];
            const float *src = reinterpret_cast<const float *>(d_ws + sl.ws_offset) + sl.lead;
            launch_level_f32(src, sl.pitch, nullptr, dst, lv.pitch, lv.nbin, lv.factor, p.nchans,
                             stream);
        }
        dd_status st = launch_check("k_level_f32");
        if (st != DD_OK)
            return st;
    }
    return DD_OK;
}

SumArgs sum_args(const dd::SumProblem &sp, const DeviceTables &t, const float *src, int64_t pitch,
                 float *dst, int64_t dst_pitch)
{
    SumArgs R;
    std::memset(&R, 0, sizeof(R));
    R.src = src;
    R.off = t.offT + sp.off_offset;
    R.base = t.baseT + sp.base_offset;
    R.dst = dst;
    R.pitch = pitch;
    R.dst_pitch = dst_pitch;
    R.nt = sp.nt;
    R.block_start = sp.block_start;
    R.nrows = sp.nrows;
    R.nouts = sp.nouts;
    R.nouts_pad = sp.nouts_pad;
    R.nout_tiles = sp.nout_tiles;
    R.stage_rows = sp.stage_rows;
    R.row_words = sp.row_words;
    R.nstages = sp.nstages;
    R.tab_stride = sp.tab_stride;
    R.tab_block = sp.tab_block;
    R.pat_words = sp.npat * dd::kSbPatWords;
    R.njobs_max = sp.njobs_max;
    return R;
}

template <int MODE, bool PD = false>
dd_status launch_sum_mode(SumBatch &a, int64_t blocks, size_t lds, const BoxArgs &bx,
                          hipStream_t stream)
{
    a.nblocks = blocks;
    a.per_xcd = (blocks + kXcds - 1) / kXcds;
    if (!PD) {
        a.pd = nullptr;
        a.src_base = a.dst_base = 0;
        a.max_stage = 0;
        for (int i = 0; i < a.nprob; ++i)
            a.max_stage = std::max(a.max_stage, a.p[i].stage_rows);
    }
    const bool short_lists = a.max_stage <= 8;
    const void *fn = short_lists ? reinterpret_cast<const void *>(k_shiftsum_f32<MODE, 2, PD>)
                                 : reinterpret_cast<const void *>(k_shiftsum_f32<MODE, 4, PD>);
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        for (const void *f : {reinterpret_cast<const void *>(k_shiftsum_f32<MODE, 2, PD>),
                              reinterpret_cast<const void *>(k_shiftsum_f32<MODE, 4, PD>)})
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      int(dd::kMaxLdsBytes));
    });
    SumBatch a_arg = a;
    BoxArgs bx_arg = bx;
    void *args[] = {&a_arg, &bx_arg};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(a.per_xcd * kXcds)), dim3(kBlock), args, lds, stream);
    if (e != hipSuccess)
        return hip_fail(e, "k_shiftsum_f32");
    return launch_check("k_shiftsum_f32");
}

dd_status launch_sum(SumBatch &a, int64_t blocks, size_t lds, hipStream_t stream)
{
    BoxArgs bx;
    std::memset(&bx, 0, sizeof(bx));
    bx.t_stride = kFTileT;
    return launch_sum_mode<kWrite>(a, blocks, lds, bx, stream);
}

dd_status sum_f32(const Plan &p, const DeviceTables &t, float *d_out, const char *d_ws,
                  hipStream_t stream)
{
    SumBatch a;
    std::memset(&a, 0, sizeof(a));
    a.nprob = int32_t(p.ranges.size());
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        const dd::BinLevel &lv = p.levels[ri.level];
        a.p[i] = sum_args(ri.fwd, t, reinterpret_cast<const float *>(d_ws + lv.ws_offset) + lv.lead,
                          lv.pitch, d_out + ri.out_offset, ri.nout);
    }
    return launch_sum(a, p.blocks, p.lds_bytes, stream);
}

// The adjoint.  d_g: the output gradient in the plan's output layout, copied
// into the padded rows of the workspace; or NULL when the padded rows hold
// it already (the boxcar backward writes them itself).
dd_status adjoint_f32(const Plan &p, const DeviceTables &t, const float *d_g, const float *d_x,
                      const float *d_w, float *d_dx, float *d_dw, char *d_ws, hipStream_t stream)
{
    SumBatch a;
    std::memset(&a, 0, sizeof(a));
    a.nprob = int32_t(p.ranges.size());
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        float *gpad = reinterpret_cast<float *>(d_ws + ri.gpad_offset);
        if (d_g) {
            const dim3 grid(unsigned(std::min<int64_t>((ri.gpitch + 1023) / 1024, 1024)),
                            unsigned(std::min<int32_t>(ri.ndms, 65535)));
            hipLaunchKernelGGL(k_pad_rows_f32, grid, dim3(256), 0, stream, d_g + ri.out_offset,
                               ri.nout, int64_t(ri.max_shift), gpad, ri.gpitch, ri.ndms);
            dd_status st = launch_check("k_pad_rows_f32");
            if (st != DD_OK)
                return st;
        }
        a.p[i] = sum_args(ri.adj, t, gpad, ri.gpitch,
                          reinterpret_cast<float *>(d_ws + ri.G_offset), ri.Gpitch);
    }
    if (p.adj_fused) {
        // one range at full resolution: dX and the weight-gradient partials
        // come from the adjoint kernel's epilogue
        float *partial = reinterpret_cast<float *>(d_ws + p.dw_offset);
        BoxArgs fin;
        std::memset(&fin, 0, sizeof(fin));
        fin.t_stride = kFTileT;
        fin.partial = partial;
        fin.x = d_dw ? d_x : nullptr;
        fin.w = d_w;
        fin.dX = d_dx;
        a.p[0].x_pitch = p.nsamp;
        dd_status st = launch_sum_mode<kAdjFinal>(a, p.adj_blocks, p.adj_lds_bytes, fin, stream);
        if (st != DD_OK || !d_dw)
            return st;
        hipLaunchKernelGGL(k_reduce_rows, dim3(unsigned(p.nchans)), dim3(256), 0, stream, partial,
                           p.dw_tiles, d_dw);
        return launch_check("k_reduce_rows");
    }
    dd_status st = launch_sum(a, p.adj_blocks, p.adj_lds_bytes, stream);
    if (st != DD_OK)
        return st;
    FinArgs f;
    std::memset(&f, 0, sizeof(f));
    f.nranges = int32_t(p.ranges.size());
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        f.r[i].G = reinterpret_cast<const float *>(d_ws + ri.G_offset);
        f.r[i].Gpitch = ri.Gpitch;
        f.r[i].nbin = ri.nbin;
        f.r[i].ds = ri.ds;
    }
    float *partial = reinterpret_cast<float *>(d_ws + p.dw_offset);
    f.x = d_dw ? d_x : nullptr;
    f.w = d_w;
    f.dX = d_dx;
    f.partial = partial;
    f.nsamp = p.nsamp;
    f.chunk_len = p.dw_chunk_len;
    f.nchunks = p.dw_chunks;
    const bool vec = p.nsamp % 4 == 0 && reinterpret_cast<uintptr_t>(f.x) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(f.dX) % 16 == 0;
    const dim3 fgrid(unsigned(p.dw_chunks), unsigned(p.nchans));
    if (vec)
        hipLaunchKernelGGL(k_adj_finalize<true>, fgrid, dim3(256), 0, stream, f);
    else
        hipLaunchKernelGGL(k_adj_finalize<false>, fgrid, dim3(256), 0, stream, f);
    st = launch_check("k_adj_finalize");
    if (st != DD_OK || !d_dw)
        return st;
    hipLaunchKernelGGL(k_reduce_rows, dim3(unsigned(p.nchans)), dim3(256), 0, stream, partial,
                       p.dw_chunks, d_dw);
    return launch_check("k_reduce_rows");
}


__global__ void k_accumulate(float *__restrict__ dst, const float *__restrict__ src, int n,
                             int first)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = first ? src[i] : dst[i] + src[i];
}

// Forward problems of a plan relaunched with the boxcar tiling.
int64_t box_batch(const Plan &p, const DeviceTables &t, const char *d_ws, float *dst,
                  int64_t stride, SumBatch &a)
{
    std::memset(&a, 0, sizeof(a));
    a.nprob = int32_t(p.ranges.size());
    int64_t blocks = 0;
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        const dd::BinLevel &lv = p.levels[ri.level];
        a.p[i] = sum_args(ri.fwd, t, reinterpret_cast<const float *>(d_ws + lv.ws_offset) + lv.lead,
                          lv.pitch, dst ? dst + ri.out_offset : nullptr, ri.nout);
        a.p[i].block_start = blocks;
        blocks += (ri.nout + stride - 1) / stride * ri.fwd.nout_tiles;
    }
    return blocks;
}

size_t box_lds(const Plan &p, int mode)
{
    return std::max(p.lds_bytes, size_t(kWavesPerBlock * box_rows(mode) * kFSpan + kBlock) * sizeof(float));
}

dd_status boxcar_loss_f32(const Plan &p, const DeviceTables &t, const float *d_in, int32_t nbeams,
                          const float *d_w, int32_t max_width, float *d_loss, char *d_ws,
                          hipStream_t stream)
{
    float *partial = reinterpret_cast<float *>(d_ws + p.box_offset);
    float *beam_loss = partial + p.box_partials;
    for (int32_t b = 0; b < nbeams; ++b) {
        const float *x = d_in + int64_t(b) * p.nchans * p.nsamp;
        dd_status st = bin_f32(p, x, d_w, d_ws, stream);
        if (st != DD_OK)
            return st;
        SumBatch a;
        const int64_t blocks = box_batch(p, t, d_ws, nullptr, dd::kBoxLossStride, a);
        BoxArgs bx;
        std::memset(&bx, 0, sizeof(bx));
        bx.partial = partial;
        bx.t_stride = dd::kBoxLossStride;
        bx.t_lead = 0;
        bx.max_width = max_width;
        st = launch_sum_mode<kBoxLoss>(a, blocks, box_lds(p, kBoxLoss), bx, stream);
        if (st != DD_OK)
            return st;
        hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(256), 0, stream, partial, int(blocks),
                           beam_loss);
        st = launch_check("k_reduce_rows");
        if (st != DD_OK)
            return st;
        hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(64), 0, stream, d_loss, beam_loss, 1,
                           int(b == 0));
        st = launch_check("k_accumulate");
        if (st != DD_OK)
            return st;
    }
    return DD_OK;
}

dd_status boxcar_backward_f32(const Plan &p, const DeviceTables &t, const float *d_in,
                              int32_t nbeams, const float *d_w, int32_t max_width, float *d_dx,
                              float *d_dw, char *d_ws, hipStream_t stream)
{
    float *dwb = reinterpret_cast<float *>(d_ws + p.dwb_offset);
    for (int32_t b = 0; b < nbeams; ++b) {
        const int64_t xoff = int64_t(b) * p.nchans * p.nsamp;
        dd_status st = bin_f32(p, d_in + xoff, d_w, d_ws, stream);
        if (st != DD_OK)
            return st;
        // dL/dout straight into the adjoint's padded rows: their padding
        // zeroed, the gradient tiles written between
        SumBatch a;
        std::memset(&a, 0, sizeof(a));
        a.nprob = int32_t(p.ranges.size());
        int64_t blocks = 0;
        for (size_t i = 0; i < p.ranges.size(); ++i) {
            const RangeInfo &ri = p.ranges[i];
            const dd::BinLevel &lv = p.levels[ri.level];
            float *gpad = reinterpret_cast<float *>(d_ws + ri.gpad_offset);
            const int64_t P = ri.max_shift;
            const dim3 zgrid(unsigned(std::min<int64_t>((ri.gpitch - ri.nout + 255) / 256, 64)),
                             unsigned(std::min<int32_t>(ri.ndms, 65535)));
            hipLaunchKernelGGL(k_zero_pads, zgrid, dim3(256), 0, stream, gpad, ri.gpitch, P, ri.nout,
                               ri.ndms);
            st = launch_check("k_zero_pads");
            if (st != DD_OK)
                return st;
            a.p[i] = sum_args(ri.fwd, t, reinterpret_cast<const float *>(d_ws + lv.ws_offset) + lv.lead,
                              lv.pitch, gpad + P, ri.gpitch);
            a.p[i].block_start = blocks;
            blocks += (ri.nout + dd::kBoxGradStride - 1) / dd::kBoxGradStride * ri.fwd.nout_tiles;
        }
        BoxArgs bx;
        std::memset(&bx, 0, sizeof(bx));
        bx.t_stride = dd::kBoxGradStride;
        bx.t_lead = dd::kBoxLead;
        bx.max_width = max_width;
        st = launch_sum_mode<kBoxGrad>(a, blocks, box_lds(p, kBoxGrad), bx, stream);
        if (st != DD_OK)
            return st;
        st = adjoint_f32(p, t, nullptr, d_in + xoff, d_w, d_dx ? d_dx + xoff : nullptr,
                         d_dw ? dwb : nullptr, d_ws, stream);
        if (st != DD_OK)
            return st;
        if (d_dw) {
            hipLaunchKernelGGL(k_accumulate, dim3(unsigned((p.nchans + 255) / 256)), dim3(256), 0,
                               stream, d_dw, dwb, p.nchans, int(b == 0));
            st = launch_check("k_accumulate");
            if (st != DD_OK)
                return st;
        }
    }
    return DD_OK;
}


// ---------------------------------------------------------------------------
// Streaming helpers: corner turn of a time-major block into channel-major
// rows (32 x 32 tiles through LDS, coalesced on both sides), a pitched row
// copy, and the move of a chunk's last `overlap` samples to its front.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_corner_turn(const T *__restrict__ in, int64_t nsamp,
                                                     int nchans, T *__restrict__ out,
                                                     int64_t out_pitch, int64_t out_off)
{
    __shared__ T tile[32][33];
    const int64_t t0 = int64_t(blockIdx.x) * 32;
    const int c0 = int(blockIdx.y) * 32;
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int64_t t = t0 + j;
        const int c = c0 + int(threadIdx.x);
        if (t < nsamp && c < nchans)
            tile[j][threadIdx.x] = in[t * nchans + c];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int c = c0 + j;
        const int64_t t = t0 + threadIdx.x;
        if (t < nsamp && c < nchans)
            out[int64_t(c) * out_pitch + out_off + t] = tile[threadIdx.x][j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_rows(const T *__restrict__ in, int64_t n,
                                                   int nchans, T *__restrict__ out,
                                                   int64_t out_pitch, int64_t out_off)
{
    for (int64_t c = blockIdx.y; c < nchans; c += gridDim.y)
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
             i += int64_t(gridDim.x) * blockDim.x)
            out[c * out_pitch + out_off + i] = in[c * n + i];
}

// buf[c][i] = buf[c][i + step] for i < overlap (step >= overlap: no overlap
// between what is read and what is written).
template <typename T>
__global__ __launch_bounds__(256) void k_shift_rows(T *buf, int64_t pitch, int64_t step,
                                                    int64_t overlap, int nchans)
{
    for (int64_t c = blockIdx.y; c < nchans; c += gridDim.y)
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < overlap;
             i += int64_t(gridDim.x) * blockDim.x)
            buf[c * pitch + i] = buf[c * pitch + i + step];
}

template <typename T>
dd_status corner_turn_t(const T *in, int64_t nsamp, int nchans, T *out, int64_t pitch,
                        int64_t off, hipStream_t stream)
{
    const dim3 grid(unsigned((nsamp + 31) / 32), unsigned((nchans + 31) / 32));
    hipLaunchKernelGGL(k_corner_turn<T>, grid, dim3(32, 8), 0, stream, in, nsamp, nchans, out,
                       pitch, off);
    return launch_check("k_corner_turn");
}

template <typename T>
dd_status stream_fill(const dd::Stream &S, const T *block, int64_t samples, T *chunk,
                      hipStream_t stream)
{
    const Plan &p = *S.plan;
    const int64_t off = S.chunks == 0 ? 0 : S.overlap;
    const dim3 rows(unsigned(std::min<int64_t>((p.nsamp + 255) / 256, 1024)),
                    unsigned(std::min<int32_t>(p.nchans, 65535)));
    if (S.chunks > 0) {
        hipLaunchKernelGGL(k_shift_rows<T>, rows, dim3(256), 0, stream, chunk, p.nsamp, S.step,
                           S.overlap, p.nchans);
        dd_status st = launch_check("k_shift_rows");
        if (st != DD_OK)
            return st;
    }
    if (S.time_major)
        return corner_turn_t(block, samples, p.nchans, chunk, p.nsamp, off, stream);
    hipLaunchKernelGGL(k_copy_rows<T>, rows, dim3(256), 0, stream, block, samples, p.nchans, chunk,
                       p.nsamp, off);
    return launch_check("k_copy_rows");
}

dd_status forward_bin(const Plan &p, const void *d_in, const float *d_w, char *d_ws,
                      hipStream_t stream)
{
    if (p.dtype == DD_U8)
        return bin_u8(p, static_cast<const uint8_t *>(d_in), d_ws, stream);
    return bin_f32(p, static_cast<const float *>(d_in), d_w, d_ws, stream);
}

dd_status forward_sum(const Plan &p, const DeviceTables &t, void *d_out, const char *d_ws,
                      hipStream_t stream)
{
    if (p.dtype == DD_U8)
        return sum_u8(p, t, static_cast<int32_t *>(d_out), d_ws, stream);
    return sum_f32(p, t, static_cast<float *>(d_out), d_ws, stream);
}


// Device-side batch state, per device: one allocation holding, per kernel
// group, its descriptor array (BatchDesc or SbBatchDesc) and item starts.
struct ZeroDesc {              // one range's padded gradient rows (k_zero_pads_batch)
    int64_t off;              // floats from the workspace
    int64_t gpitch;
    int64_t P;
    int64_t nout;
    int64_t nrows;
};

struct SpanDesc {             // a beam's workgroups of a launch, or its channels' partials
    int64_t first;            // first partial (floats from the partial base)
    int64_t count;            // partials per output (k_reduce_spans: the whole span)
    int64_t out;              // output index (beam, or the beam's first channel)
    int64_t nrows;            // rows (channels) to reduce (1 for a loss span)
};

struct BatchDevice {
    void *mem = nullptr;
    std::vector<const void *> descs;       // per group
    std::vector<const int64_t *> starts;   // per group
    const BinJob *bin_jobs = nullptr;      // beams with power-of-two levels
    int32_t nbin_jobs = 0;
    int64_t bin_blocks = 0;
    // float32 boxcar calls: descriptors of the loss, gradient and adjoint
    // launches (same problem order as the forward's), the padded rows to
    // zero, and the reductions' spans
    const SumArgs *box_loss = nullptr, *box_grad = nullptr, *adj = nullptr;
    int64_t loss_blocks = 0, grad_blocks = 0, adj_blocks = 0;
    int32_t max_stage_fwd = 0, max_stage_adj = 0;
    const ZeroDesc *zero = nullptr;
    int32_t nzero = 0;
    const SpanDesc *loss_spans = nullptr, *dw_spans = nullptr;
};

struct BatchState {
    std::mutex mu;
    std::map<int, BatchDevice> per_device;
};

dd_status batch_device(const dd::Batch &b, BatchDevice **out)
{
    BatchState *st = static_cast<BatchState *>(b.device);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(st->mu);
    auto it = st->per_device.find(dev);
    if (it != st->per_device.end()) {
        *out = &it->second;
        return DD_OK;
    }
    // host image: per group, descriptors then starts, each 256-byte aligned
    std::vector<char> img;
    std::vector<size_t> off_desc(b.groups.size()), off_start(b.groups.size());
    auto grow = [&](size_t bytes) {
        const size_t at = (img.size() + 255) / 256 * 256;
        img.resize(at + bytes, 0);
        return at;
    };
    for (size_t g = 0; g < b.groups.size(); ++g) {
        const dd::BatchGroup &G = b.groups[g];
        const size_t n = G.desc_end - G.desc_begin;
        off_desc[g] = grow(n * (G.f32 ? sizeof(SumArgs) : G.subband ? sizeof(SbBatchDesc) : sizeof(BatchDesc)));
        off_start[g] = grow(n * sizeof(int64_t));
        for (size_t k = 0; k < n; ++k) {
            const dd::BatchDescHost &d = b.descs[G.desc_begin + k];
            const Plan &p = *b.plans[d.beam];
            DeviceTables *t = nullptr;
            dd_status s2 = device_tables(p, &t);
            if (s2 != DD_OK)
                return s2;
            const RangeInfo &ri = p.ranges[d.range];
            const dd::BinLevel &lv = p.levels[ri.level];
            reinterpret_cast<int64_t *>(img.data() + off_start[g])[k] = d.item_start;
            if (G.f32) {
                // src and dst as byte offsets from the call's workspace and
                // output (added in the kernel)
                const size_t src_off = b.ws_off[d.beam] + lv.ws_offset + size_t(lv.lead) * sizeof(float);
                const size_t dst_off = size_t(b.out_off[d.beam] + ri.out_offset) * sizeof(float);
                SumArgs R = sum_args(ri.fwd, *t, reinterpret_cast<const float *>(src_off), lv.pitch,
                                     reinterpret_cast<float *>(dst_off), ri.nout);
                R.block_start = d.item_start;
                reinterpret_cast<SumArgs *>(img.data() + off_desc[g])[k] = R;
                continue;
            }
            if (G.subband) {
                SbBatchDesc &S = reinterpret_cast<SbBatchDesc *>(img.data() + off_desc[g])[k];
                fill_sb_range(p, *t, ri, S.R);
                S.src_off = int64_t(b.ws_off[d.beam] + lv.ws_offset);
                S.out_off = b.out_off[d.beam] + ri.out_offset;
                S.item_start = d.item_start;
                continue;
            }
            BatchDesc &D = reinterpret_cast<BatchDesc *>(img.data() + off_desc[g])[k];
            D.offT = t->offT + ri.off_offset;
            D.baseT = t->baseT + ri.base_offset;
            D.src_off = int64_t(b.ws_off[d.beam] + lv.ws_offset);
            D.out_off = b.out_off[d.beam] + ri.out_offset;
            D.pitch = lv.pitch;
            D.nout = ri.nout;
            D.item_start = d.item_start;
            D.nchans = p.nchans;
            D.ndms = ri.ndms;
            D.ndms_pad = ri.ndms_pad;
            D.ndm_tiles = ri.ndm_tiles;
            D.stage_chans = ri.stage_chans;
            D.row_words = ri.row_words;
            D.widen_every = ri.widen_every;
        }
    }
    // float32 boxcar descriptors (problem order as the forward group's)
    size_t off_bl = 0, off_bg = 0, off_ad = 0, off_z = 0, off_ls = 0, off_dw = 0;
    int64_t nbl = 0, nbg = 0, nad = 0;
    int32_t ms_fwd = 0, ms_adj = 0, nz = 0;
    if (b.dtype == DD_F32 && !b.groups.empty()) {
        const dd::BatchGroup &G = b.groups[0];
        const size_t n = G.desc_end - G.desc_begin;
        std::vector<SumArgs> L(n), Gr(n), Ad(n);
        std::vector<ZeroDesc> Z;
        std::vector<SpanDesc> LS(b.plans.size()), DW(b.plans.size());
        std::vector<int64_t> first(b.plans.size(), -1), last(b.plans.size(), 0);
        for (size_t k = 0; k < n; ++k) {
            const dd::BatchDescHost &d = b.descs[G.desc_begin + k];
            const Plan &p = *b.plans[d.beam];
            DeviceTables *t = nullptr;
            dd_status s2 = device_tables(p, &t);
            if (s2 != DD_OK)
                return s2;
            const RangeInfo &ri = p.ranges[d.range];
            const dd::BinLevel &lv = p.levels[ri.level];
            const size_t src_off = b.ws_off[d.beam] + lv.ws_offset + size_t(lv.lead) * sizeof(float);
            const size_t gpad = b.gpad_off[d.beam][d.range];
            // loss: partial index = the launch's workgroup index
            L[k] = sum_args(ri.fwd, *t, reinterpret_cast<const float *>(src_off), lv.pitch, nullptr, ri.nout);
            L[k].block_start = nbl;
            if (first[d.beam] < 0)
                first[d.beam] = nbl;
            nbl += (ri.nout + dd::kBoxLossStride - 1) / dd::kBoxLossStride * ri.fwd.nout_tiles;
            last[d.beam] = nbl;
            // gradient: dL/dout into the padded rows, after their P zeros
            const size_t g_dst = gpad + size_t(ri.max_shift) * sizeof(float);
            Gr[k] = sum_args(ri.fwd, *t, reinterpret_cast<const float *>(src_off), lv.pitch,
                             reinterpret_cast<float *>(g_dst), ri.gpitch);
            Gr[k].block_start = nbg;
            nbg += (ri.nout + dd::kBoxGradStride - 1) / dd::kBoxGradStride * ri.fwd.nout_tiles;
            // adjoint over the padded rows; dX, x and the partials per beam
            Ad[k] = sum_args(ri.adj, *t, reinterpret_cast<const float *>(gpad), ri.gpitch, nullptr, ri.Gpitch);
            Ad[k].block_start = nad;
            Ad[k].x_off = b.in_off[d.beam] / int64_t(sizeof(float));
            Ad[k].x_pitch = p.nsamp;
            Ad[k].part_off = int64_t(b.dwp_off[d.beam] / sizeof(float));
            Ad[k].w_off = int32_t(b.w_off[d.beam]);
            nad += ri.adj.ntime_tiles * ri.adj.nout_tiles;
            ms_fwd = std::max(ms_fwd, ri.fwd.stage_rows);
            ms_adj = std::max(ms_adj, ri.adj.stage_rows);
            Z.push_back(ZeroDesc{int64_t(gpad / sizeof(float)), ri.gpitch, ri.max_shift, ri.nout, ri.ndms});
        }
        for (size_t i = 0; i < b.plans.size(); ++i) {
            LS[i] = SpanDesc{first[i], last[i] - first[i], int64_t(i), 1};
            const Plan &p = *b.plans[i];
            DW[i] = SpanDesc{int64_t(b.dwp_off[i] / sizeof(float)), std::max(p.dw_tiles, 1), b.w_off[i], p.nchans};
        }
        auto put = [&](const void *src, size_t bytes) {
            const size_t at = grow(std::max<size_t>(bytes, 1));
            std::memcpy(img.data() + at, src, bytes);
            return at;
        };
        off_bl = put(L.data(), n * sizeof(SumArgs));
        off_bg = put(Gr.data(), n * sizeof(SumArgs));
        off_ad = put(Ad.data(), n * sizeof(SumArgs));
        off_z = put(Z.data(), Z.size() * sizeof(ZeroDesc));
        off_ls = put(LS.data(), LS.size() * sizeof(SpanDesc));
        off_dw = put(DW.data(), DW.size() * sizeof(SpanDesc));
        nz = int32_t(Z.size());
    }
    // binning jobs: every beam's power-of-two levels, one launch
    std::vector<BinJob> jobs;
    int64_t bin_blocks = 0;
    for (size_t i = 0; i < b.plans.size() && b.dtype == DD_U8; ++i) {
        BinJob J;
        if (!pow2_job(*b.plans[i], b.in_off[i], b.ws_off[i], J))
            continue;
        J.block_start = bin_blocks;
        bin_blocks += int64_t(J.nchans) * J.nseg;
        jobs.push_back(J);
    }
    const size_t off_jobs = grow(std::max<size_t>(1, jobs.size()) * sizeof(BinJob));
    if (!jobs.empty())
        std::memcpy(img.data() + off_jobs, jobs.data(), jobs.size() * sizeof(BinJob));
    BatchDevice bd;
    e = hipMalloc(&bd.mem, img.size() + 256);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dd::set_error(std::string("hipMalloc of the batch descriptors: ") + hipGetErrorString(e));
        return DD_ERR_NOMEM;
    }
    e = hipMemcpy(bd.mem, img.data(), img.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(bd.mem);
        return hip_fail(e, "hipMemcpy of the batch descriptors");
    }
    bd.bin_jobs = reinterpret_cast<const BinJob *>(static_cast<const char *>(bd.mem) + off_jobs);
    bd.nbin_jobs = int32_t(jobs.size());
    bd.bin_blocks = bin_blocks;
    if (b.dtype == DD_F32) {
        const char *m = static_cast<const char *>(bd.mem);
        bd.box_loss = reinterpret_cast<const SumArgs *>(m + off_bl);
        bd.box_grad = reinterpret_cast<const SumArgs *>(m + off_bg);
        bd.adj = reinterpret_cast<const SumArgs *>(m + off_ad);
        bd.loss_blocks = nbl;
        bd.grad_blocks = nbg;
        bd.adj_blocks = nad;
        bd.max_stage_fwd = ms_fwd;
        bd.max_stage_adj = ms_adj;
        bd.zero = reinterpret_cast<const ZeroDesc *>(m + off_z);
        bd.nzero = nz;
        bd.loss_spans = reinterpret_cast<const SpanDesc *>(m + off_ls);
        bd.dw_spans = reinterpret_cast<const SpanDesc *>(m + off_dw);
    }
    for (size_t g = 0; g < b.groups.size(); ++g) {
        bd.descs.push_back(static_cast<const char *>(bd.mem) + off_desc[g]);
        bd.starts.push_back(
            reinterpret_cast<const int64_t *>(static_cast<const char *>(bd.mem) + off_start[g]));
    }
    *out = &(st->per_device[dev] = std::move(bd));
    return DD_OK;
}

// Persistent workgroups per XCD: two per CU of its 32.
constexpr int kPersistPerXcd = 64;

const void *direct_batch_kernel(bool dedup, int waves, int time_tile)
{
    const bool w4 = waves == 4, t2 = time_tile == 2 * kWave * 2;
    if (dedup)
        return w4 ? (t2 ? reinterpret_cast<const void *>(k_dedisp_u8_batch<true, 4, 2>)
                        : reinterpret_cast<const void *>(k_dedisp_u8_batch<true, 4, 4>))
                  : (t2 ? reinterpret_cast<const void *>(k_dedisp_u8_batch<true, 8, 2>)
                        : reinterpret_cast<const void *>(k_dedisp_u8_batch<true, 8, 4>));
    return w4 ? (t2 ? reinterpret_cast<const void *>(k_dedisp_u8_batch<false, 4, 2>)
                    : reinterpret_cast<const void *>(k_dedisp_u8_batch<false, 4, 4>))
              : (t2 ? reinterpret_cast<const void *>(k_dedisp_u8_batch<false, 8, 2>)
                    : reinterpret_cast<const void *>(k_dedisp_u8_batch<false, 8, 4>));
}

const void *subband_batch_kernel(int dm_tile, int time_tile)
{
    const bool t2 = time_tile == 2 * kWave * 2;
    switch (dm_tile) {
    case 192: return reinterpret_cast<const void *>(k_dedisp_u8_sb_batch<16, 12, 2>);
    case 128: return reinterpret_cast<const void *>(k_dedisp_u8_sb_batch<16, 8, 2>);
    case 96:
        return t2 ? reinterpret_cast<const void *>(k_dedisp_u8_sb_batch<8, 12, 2>)
                  : reinterpret_cast<const void *>(k_dedisp_u8_sb_batch<8, 12, 4>);
    default:
        return t2 ? reinterpret_cast<const void *>(k_dedisp_u8_sb_batch<8, 8, 2>)
                  : reinterpret_cast<const void *>(k_dedisp_u8_sb_batch<8, 8, 4>);
    }
}

// Float32 batch boxcar helpers.  k_zero_pads_batch: the padding of every
// (beam, range)'s gradient rows (one descriptor per blockIdx.y).
// k_reduce_spans: out[s.out] = fixed-order sum of partials [s.first,
// s.first + s.count) (one span per block: a beam's loss).  k_reduce_rows_spans:
// for span s and its channel c (blockIdx.x), out[s.out + c] = fixed-order sum
// of the c-th row of s.count partials (a beam's weight gradient).
__global__ __launch_bounds__(256) void k_zero_pads_batch(float *__restrict__ ws, const ZeroDesc *__restrict__ zd,
                                                         int nzd)
{
    for (int di = blockIdx.y; di < nzd; di += gridDim.y) {
        const ZeroDesc z = zd[di];
        const int64_t tail = z.gpitch - z.P - z.nout;
        const int64_t per_row = z.P + tail;
        const int64_t total = per_row * z.nrows;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
             i += int64_t(gridDim.x) * blockDim.x) {
            const int64_t r = i / per_row, k = i - r * per_row;
            ws[z.off + r * z.gpitch + (k < z.P ? k : z.P + z.nout + (k - z.P))] = 0.0f;
        }
    }
}

__device__ __forceinline__ float block_sum_256(float v, float *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(256) void k_reduce_spans(const float *__restrict__ partial,
                                                      const SpanDesc *__restrict__ spans,
                                                      float *__restrict__ out)
{
    __shared__ float red[256];
    const SpanDesc sp = spans[blockIdx.x];
    float acc = 0.0f;
    for (int64_t i = threadIdx.x; i < sp.count; i += 256)
        acc += partial[sp.first + i];
    const float total = block_sum_256(acc, red);
    if (threadIdx.x == 0)
        out[sp.out] = total;
}

__global__ __launch_bounds__(256) void k_reduce_rows_spans(const float *__restrict__ partial,
                                                           const SpanDesc *__restrict__ spans, int nspans,
                                                           float *__restrict__ out)
{
    __shared__ float red[256];
    for (int si = blockIdx.y; si < nspans; si += gridDim.y) {
        const SpanDesc sp = spans[si];
        for (int64_t c = blockIdx.x; c < sp.nrows; c += gridDim.x) {
            float acc = 0.0f;
            for (int64_t i = threadIdx.x; i < sp.count; i += 256)
                acc += partial[sp.first + c * sp.count + i];
            const float total = block_sum_256(acc, red);
            if (threadIdx.x == 0)
                out[sp.out + c] = total;
            __syncthreads();
        }
    }
}

// Float32 batch: every beam's weighted levels (k_level_f32, beam by beam),
// then one shift-and-sum launch over all (beam, range) problems, the most
// expensive beams' workgroups first.
dd_status batch_forward_f32(const dd::Batch &b, const BatchDevice &bd, const char *d_in,
                            const float *d_w, float *d_out, char *d_ws, hipStream_t stream)
{
    for (size_t i = 0; i < b.plans.size(); ++i) {
        dd_status st = bin_f32(*b.plans[i], reinterpret_cast<const float *>(d_in + b.in_off[i]),
                               d_w ? d_w + b.w_off[i] : nullptr, d_ws + b.ws_off[i], stream);
        if (st != DD_OK)
            return st;
    }
    const dd::BatchGroup &G = b.groups[0];
    SumBatch a;
    std::memset(&a, 0, sizeof(a));
    a.pd = static_cast<const SumArgs *>(bd.descs[0]);
    a.nprob = int32_t(G.desc_end - G.desc_begin);
    a.src_base = reinterpret_cast<uintptr_t>(d_ws);
    a.dst_base = reinterpret_cast<uintptr_t>(d_out);
    for (const dd::Plan *p : b.plans)
        for (const RangeInfo &ri : p->ranges)
            a.max_stage = std::max(a.max_stage, ri.fwd.stage_rows);
    BoxArgs bx;
    std::memset(&bx, 0, sizeof(bx));
    bx.t_stride = kFTileT;
    return launch_sum_mode<kWrite, true>(a, G.nitems, G.lds_bytes, bx, stream);
}

size_t batch_lds(const dd::Batch &b, int mode)
{
    size_t lds = 0;
    for (const dd::Plan *p : b.plans)
        lds = std::max(lds, mode == kAdjFinal ? p->adj_lds_bytes : box_lds(*p, mode));
    return lds;
}

// Float32 batch boxcar loss: the beams' levels, ONE loss launch over every
// (beam, range) problem, ONE reduction to the per-beam losses.
dd_status batch_boxcar_loss_f32(const dd::Batch &b, const BatchDevice &bd, const char *d_in,
                                const float *d_w, int32_t max_width, float *d_loss, char *d_ws,
                                hipStream_t stream)
{
    for (size_t i = 0; i < b.plans.size(); ++i) {
        dd_status st = bin_f32(*b.plans[i], reinterpret_cast<const float *>(d_in + b.in_off[i]),
                               d_w ? d_w + b.w_off[i] : nullptr, d_ws + b.ws_off[i], stream);
        if (st != DD_OK)
            return st;
    }
    float *partial = reinterpret_cast<float *>(d_ws + b.loss_part_off);
    SumBatch a;
    std::memset(&a, 0, sizeof(a));
    a.pd = bd.box_loss;
    a.nprob = int32_t(b.groups[0].desc_end - b.groups[0].desc_begin);
    a.src_base = reinterpret_cast<uintptr_t>(d_ws);
    a.max_stage = bd.max_stage_fwd;
    BoxArgs bx;
    std::memset(&bx, 0, sizeof(bx));
    bx.partial = partial;
    bx.t_stride = dd::kBoxLossStride;
    bx.max_width = max_width;
    dd_status st = launch_sum_mode<kBoxLoss, true>(a, bd.loss_blocks, batch_lds(b, kBoxLoss), bx, stream);
    if (st != DD_OK)
        return st;
    hipLaunchKernelGGL(k_reduce_spans, dim3(unsigned(b.plans.size())), dim3(256), 0, stream, partial,
                       bd.loss_spans, d_loss);
    return launch_check("k_reduce_spans");
}

// Float32 batch boxcar backward (plans with one full-resolution range):
// the beams' levels, ONE launch zeroing every padded row's padding, ONE
// gradient launch writing dL/dout into the padded rows, ONE adjoint launch
// forming dX and the weight-gradient partials, ONE reduction of those.
dd_status batch_boxcar_backward_f32(const dd::Batch &b, const BatchDevice &bd, const char *d_in,
                                    const float *d_w, int32_t max_width, float *d_dx, float *d_dw,
                                    char *d_ws, hipStream_t stream)
{
    for (size_t i = 0; i < b.plans.size(); ++i) {
        dd_status st = bin_f32(*b.plans[i], reinterpret_cast<const float *>(d_in + b.in_off[i]),
                               d_w ? d_w + b.w_off[i] : nullptr, d_ws + b.ws_off[i], stream);
        if (st != DD_OK)
            return st;
    }
    float *wsf = reinterpret_cast<float *>(d_ws);
    hipLaunchKernelGGL(k_zero_pads_batch, dim3(64, unsigned(std::min(bd.nzero, 65535))), dim3(256), 0, stream,
                       wsf, bd.zero, bd.nzero);
    dd_status st = launch_check("k_zero_pads_batch");
    if (st != DD_OK)
        return st;
    const int32_t nprob = int32_t(b.groups[0].desc_end - b.groups[0].desc_begin);
    SumBatch a;
    std::memset(&a, 0, sizeof(a));
    a.pd = bd.box_grad;
    a.nprob = nprob;
    a.src_base = a.dst_base = reinterpret_cast<uintptr_t>(d_ws);
    a.max_stage = bd.max_stage_fwd;
    BoxArgs bx;
    std::memset(&bx, 0, sizeof(bx));
    bx.t_stride = dd::kBoxGradStride;
    bx.t_lead = dd::kBoxLead;
    bx.max_width = max_width;
    st = launch_sum_mode<kBoxGrad, true>(a, bd.grad_blocks, batch_lds(b, kBoxGrad), bx, stream);
    if (st != DD_OK)
        return st;
    SumBatch j;
    std::memset(&j, 0, sizeof(j));
    j.pd = bd.adj;
    j.nprob = nprob;
    j.src_base = reinterpret_cast<uintptr_t>(d_ws);
    j.max_stage = bd.max_stage_adj;
    BoxArgs fin;
    std::memset(&fin, 0, sizeof(fin));
    fin.t_stride = kFTileT;
    fin.partial = wsf;
    fin.x = d_dw ? reinterpret_cast<const float *>(d_in) : nullptr;
    fin.w = d_w;
    fin.dX = d_dx;
    st = launch_sum_mode<kAdjFinal, true>(j, bd.adj_blocks, batch_lds(b, kAdjFinal), fin, stream);
    if (st != DD_OK || !d_dw)
        return st;
    int32_t max_ch = 1;
    for (const dd::Plan *p : b.plans)
        max_ch = std::max(max_ch, p->nchans);
    const int nspans = int(b.plans.size());
    hipLaunchKernelGGL(k_reduce_rows_spans, dim3(unsigned(std::min(max_ch, 4096)), unsigned(std::min(nspans, 65535))),
                       dim3(256), 0, stream, wsf, bd.dw_spans, nspans, d_dw);
    return launch_check("k_reduce_rows_spans");
}

dd_status batch_forward(const dd::Batch &b, const BatchDevice &bd, const char *d_in,
                        int32_t *d_out, char *d_ws, hipStream_t stream)
{
    // every beam's power-of-two levels in one launch, then the other levels
    // beam by beam
    if (bd.nbin_jobs > 0) {
        const uint8_t *in = reinterpret_cast<const uint8_t *>(d_in);
        hipLaunchKernelGGL(k_bin_pow2_u8_batch,
                           dim3(unsigned(std::min<int64_t>(bd.bin_blocks, 1 << 20))),
                           dim3(kBinThreads), 0, stream, bd.bin_jobs, bd.nbin_jobs, in,
                           in + b.in_bytes, d_ws, bd.bin_blocks);
        dd_status st = launch_check("k_bin_pow2_u8_batch");
        if (st != DD_OK)
            return st;
    }
    for (size_t i = 0; i < b.plans.size(); ++i) {
        dd_status st = bin_u8_rest(*b.plans[i], reinterpret_cast<const uint8_t *>(d_in + b.in_off[i]),
                                   d_ws + b.ws_off[i], stream);
        if (st != DD_OK)
            return st;
    }
    int32_t *counters = reinterpret_cast<int32_t *>(d_ws);
    const int ncounters = int(b.groups.size()) * dd::kBatchQueues;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, stream, counters, ncounters);
    dd_status st = launch_check("k_reset_counters");
    if (st != DD_OK)
        return st;
    for (size_t g = 0; g < b.groups.size(); ++g) {
        const dd::BatchGroup &G = b.groups[g];
        QueueBounds qb;
        for (int i = 0; i <= dd::kBatchQueues; ++i)
            qb.b[i] = G.queue_bounds[i];
        const void *fn = nullptr;
        // Persistent workgroups per XCD: two 8-wave (or four 4-wave) per CU
        // of its 32; variant 3 fills a CU's LDS with one workgroup.
        unsigned per_xcd = unsigned(kPersistPerXcd * (8 / G.waves));
        if (G.subband) {
            fn = subband_batch_kernel(G.dm_tile, G.time_tile);
            per_xcd = unsigned(kCusPerXcd);
        } else {
            fn = direct_batch_kernel(G.dedup, G.waves, G.time_tile);
        }
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(dd::kMaxLdsBytes - 64));
        const void *descs = bd.descs[g];
        const int64_t *starts = bd.starts[g];
        int ndesc = int(G.desc_end - G.desc_begin);
        const char *ws = d_ws;
        int32_t *cnt = counters + g * dd::kBatchQueues;
        void *args[] = {&descs, &starts, &ndesc, &qb, &ws, &d_out, &cnt};
        const char *name = G.subband ? "k_dedisp_u8_sb_batch" : "k_dedisp_u8_batch";
        hipError_t e = hipLaunchKernel(fn, dim3(kXcds * per_xcd), dim3(unsigned(G.waves * kWave)),
                                       args, G.lds_bytes, stream);
        if (e != hipSuccess)
            return hip_fail(e, name);
        st = launch_check(name);
        if (st != DD_OK)
            return st;
    }
    return DD_OK;
}

// Argument checks shared by the compute entry points (synchronous, before
// any HIP call).
dd_status check_forward_args(const dd_plan *plan, const void *d_in, const float *d_weights,
                             const void *d_out, int64_t out_capacity, const void *d_ws,
                             size_t ws_bytes, bool need_out, bool need_in = true,
                             size_t ws_need = SIZE_MAX)
{
    if (!plan || (need_in && !d_in) || (need_out && !d_out)) {
        dd::set_error("plan, d_in and d_out must not be NULL");
        return DD_ERR_NULL;
    }
    const Plan &p = plan->p;
    if (p.dtype == DD_U8 && d_weights) {
        dd::set_error("per-channel weights apply to DD_F32 plans only");
        return DD_ERR_DTYPE;
    }
    if (need_in && reinterpret_cast<uintptr_t>(d_in) % 4 != 0) {
        dd::set_error("d_in must be 4-byte aligned");
        return DD_ERR_INVALID;
    }
    if (need_out && out_capacity < p.out_elems) {
        dd::set_error("out_capacity " + std::to_string(out_capacity) + " < out_elems " +
                      std::to_string(p.out_elems));
        return DD_ERR_CAPACITY;
    }
    if (ws_need == SIZE_MAX)
        ws_need = p.ws_bytes;
    if (ws_bytes < ws_need || (ws_need > 0 && !d_ws)) {
        dd::set_error("workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                      std::to_string(ws_need));
        return DD_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        dd::set_error("workspace must be 256-byte aligned");
        return DD_ERR_WORKSPACE;
    }
    return DD_OK;
}

// Tables of the current device if they were uploaded already (never
// uploads: used by the entry point that allocates nothing).
DeviceTables *find_device_tables(const Plan &p)
{
    DeviceState *st = state_of(p);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return nullptr;
    std::lock_guard<std::mutex> lock(st->mu);
    auto it = st->per_device.find(dev);
    return it == st->per_device.end() ? nullptr : &it->second;
}

// Workspace bytes the forward itself touches: the binned levels (the rest of
// a float plan's workspace serves the adjoint and the boxcar loss).
size_t forward_ws_bytes(const Plan &p)
{
    size_t n = 0;
    for (const dd::BinLevel &lv : p.levels)
        n = std::max(n, lv.ws_offset + lv.bytes);
    return n;
}

}  // namespace

// Workspace of dd_forward_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  In host code `scratch` is only a
// host-side handle of the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (scratch_address), and only that address is passed to
// kernels.
static __device__ __align__(256) char scratch[DD_NOALLOC_WS_MAX];

namespace {

struct ScratchAddresses {
    std::mutex mu;
    std::map<int, char *> per_device;
};

ScratchAddresses &scratch_addresses()
{
    static ScratchAddresses s;
    return s;
}

// The current device's address of `scratch`, looked up once per device with
// that device current.
dd_status scratch_address(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    ScratchAddresses &sa = scratch_addresses();
    std::lock_guard<std::mutex> lock(sa.mu);
    auto it = sa.per_device.find(dev);
    if (it != sa.per_device.end()) {
        *out = it->second;
        return DD_OK;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return hip_fail(e, "hipGetSymbolAddress of the static workspace");
    }
    *out = sa.per_device[dev] = static_cast<char *>(ptr);
    return DD_OK;
}

}  // namespace

void *dd::new_device_state() { return new (std::nothrow) DeviceState; }
void *dd::new_batch_device_state() { return new (std::nothrow) BatchState; }

extern "C" {

void dd_plan_destroy(dd_plan *plan)
{
    if (!plan)
        return;
    DeviceState *st = state_of(plan->p);
    if (st) {
        int cur = -1;
        const bool have_cur = hipGetDevice(&cur) == hipSuccess;
        for (auto &kv : st->per_device) {
            if (hipSetDevice(kv.first) == hipSuccess)
                (void)hipFree(kv.second.offT);
        }
        if (have_cur)
            (void)hipSetDevice(cur);
        delete st;
    }
    delete plan;
}

void dd_batch_destroy(dd_batch *batch)
{
    if (!batch)
        return;
    BatchState *st = static_cast<BatchState *>(batch->b.device);
    if (st) {
        int cur = -1;
        const bool have_cur = hipGetDevice(&cur) == hipSuccess;
        for (auto &kv : st->per_device)
            if (hipSetDevice(kv.first) == hipSuccess)
                (void)hipFree(kv.second.mem);
        if (have_cur)
            (void)hipSetDevice(cur);
        delete st;
    }
    delete batch;
}

dd_status dd_batch_prepare(dd_batch *batch)
{
    dd::clear_error();
    if (!batch) {
        dd::set_error("batch must not be NULL");
        return DD_ERR_NULL;
    }
    BatchDevice *bd = nullptr;
    return batch_device(batch->b, &bd);
}

namespace {

dd_status batch_forward_any(const dd_batch *batch, const void *d_in, const float *d_weights,
                            void *d_out, int64_t out_capacity, void *d_ws, size_t ws_bytes,
                            void *stream)
{
    dd::clear_error();
    if (!batch || !d_in || !d_out || !d_ws) {
        dd::set_error("batch, d_in, d_out and d_ws must not be NULL");
        return DD_ERR_NULL;
    }
    const dd::Batch &b = batch->b;
    if (d_weights && b.dtype != DD_F32) {
        dd::set_error("per-channel weights apply to DD_F32 batches only");
        return DD_ERR_DTYPE;
    }
    if (out_capacity < b.out_elems) {
        dd::set_error("out_capacity " + std::to_string(out_capacity) + " < out_elems " +
                      std::to_string(b.out_elems));
        return DD_ERR_CAPACITY;
    }
    if (ws_bytes < b.ws_bytes || reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        dd::set_error("workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                      std::to_string(b.ws_bytes) + " or not 256-byte aligned");
        return DD_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(d_in) % 256 != 0) {
        dd::set_error("d_in must be 256-byte aligned");
        return DD_ERR_INVALID;
    }
    BatchDevice *bd = nullptr;
    dd_status st = batch_device(b, &bd);
    if (st != DD_OK)
        return st;
    if (b.dtype == DD_F32)
        return batch_forward_f32(b, *bd, static_cast<const char *>(d_in), d_weights,
                                 static_cast<float *>(d_out), static_cast<char *>(d_ws),
                                 static_cast<hipStream_t>(stream));
    return batch_forward(b, *bd, static_cast<const char *>(d_in), static_cast<int32_t *>(d_out),
                         static_cast<char *>(d_ws), static_cast<hipStream_t>(stream));
}

}  // namespace

dd_status dd_batch_forward(const dd_batch *batch, const void *d_in, void *d_out,
                           int64_t out_capacity, void *d_ws, size_t ws_bytes, void *stream)
{
    return batch_forward_any(batch, d_in, nullptr, d_out, out_capacity, d_ws, ws_bytes, stream);
}

dd_status dd_batch_forward_weighted(const dd_batch *batch, const void *d_in, const float *d_weights,
                                    void *d_out, int64_t out_capacity, void *d_ws, size_t ws_bytes,
                                    void *stream)
{
    return batch_forward_any(batch, d_in, d_weights, d_out, out_capacity, d_ws, ws_bytes, stream);
}

dd_status dd_plan_prepare(dd_plan *plan)
{
    dd::clear_error();
    if (!plan) {
        dd::set_error("plan must not be NULL");
        return DD_ERR_NULL;
    }
    DeviceTables *t = nullptr;
    return device_tables(plan->p, &t);
}

dd_status dd_forward_bin(const dd_plan *plan, const void *d_in, const float *d_weights,
                         void *d_ws, size_t ws_bytes, void *stream)
{
    dd::clear_error();
    dd_status st = check_forward_args(plan, d_in, d_weights, nullptr, 0, d_ws, ws_bytes, false);
    if (st != DD_OK)
        return st;
    return forward_bin(plan->p, d_in, d_weights, static_cast<char *>(d_ws),
                       static_cast<hipStream_t>(stream));
}

dd_status dd_forward_sum(const dd_plan *plan, void *d_out, int64_t out_capacity, void *d_ws,
                         size_t ws_bytes, void *stream)
{
    dd::clear_error();
    dd_status st = check_forward_args(plan, nullptr, nullptr, d_out, out_capacity, d_ws, ws_bytes,
                                      true, false);
    if (st != DD_OK)
        return st;
    DeviceTables *t = nullptr;
    st = device_tables(plan->p, &t);
    if (st != DD_OK)
        return st;
    return forward_sum(plan->p, *t, d_out, static_cast<const char *>(d_ws),
                       static_cast<hipStream_t>(stream));
}

dd_status dd_forward(const dd_plan *plan, const void *d_in, const float *d_weights, void *d_out,
                     int64_t out_capacity, void *d_ws, size_t ws_bytes, void *stream)
{
    dd::clear_error();
    dd_status st = check_forward_args(plan, d_in, d_weights, d_out, out_capacity, d_ws, ws_bytes,
                                      true);
    if (st != DD_OK)
        return st;
    DeviceTables *t = nullptr;
    st = device_tables(plan->p, &t);
    if (st != DD_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    st = forward_bin(plan->p, d_in, d_weights, static_cast<char *>(d_ws), s);
    if (st != DD_OK)
        return st;
    return forward_sum(plan->p, *t, d_out, static_cast<const char *>(d_ws), s);
}

dd_status dd_forward_noalloc(const dd_plan *plan, const void *d_in, const float *d_weights,
                             void *d_out, int64_t out_capacity, void *stream)
{
    dd::clear_error();
    if (!plan) {
        dd::set_error("plan must not be NULL");
        return DD_ERR_NULL;
    }
    const Plan &p = plan->p;
    const size_t need = forward_ws_bytes(p);
    if (need > size_t(DD_NOALLOC_WS_MAX)) {
        dd::set_error("the plan's forward needs " + std::to_string(need) +
                      " bytes of workspace, more than the static workspace's " +
                      std::to_string(size_t(DD_NOALLOC_WS_MAX)) + " (use dd_forward)");
        return DD_ERR_WORKSPACE;
    }
    DeviceTables *t = find_device_tables(p);
    if (!t) {
        dd::set_error("the plan's tables are not on the current device: call dd_plan_prepare "
                      "on it first (dd_forward_noalloc allocates nothing)");
        return DD_ERR_INVALID;
    }
    char *ws = nullptr;
    dd_status st = scratch_address(&ws);
    if (st != DD_OK)
        return st;
    st = check_forward_args(plan, d_in, d_weights, d_out, out_capacity, ws,
                            size_t(DD_NOALLOC_WS_MAX), true, true, need);
    if (st != DD_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    st = forward_bin(p, d_in, d_weights, ws, s);
    if (st != DD_OK)
        return st;
    return forward_sum(p, *t, d_out, ws, s);
}

dd_status dd_adjoint(const dd_plan *plan, const float *d_grad_out, const float *d_in,
                     const float *d_weights, float *d_grad_in, float *d_grad_w, void *d_ws,
                     size_t ws_bytes, void *stream)
{
    dd::clear_error();
    if (!plan || !d_grad_out || (d_grad_w && !d_in)) {
        dd::set_error("plan and d_grad_out must not be NULL, and d_in is needed for d_grad_w");
        return DD_ERR_NULL;
    }
    const Plan &p = plan->p;
    if (p.dtype != DD_F32) {
        dd::set_error("the adjoint is defined for DD_F32 plans");
        return DD_ERR_DTYPE;
    }
    if (ws_bytes < p.ws_bytes || !d_ws || reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        dd::set_error("workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                      std::to_string(p.ws_bytes) + " or not 256-byte aligned");
        return DD_ERR_WORKSPACE;
    }
    DeviceTables *t = nullptr;
    dd_status st = device_tables(p, &t);
    if (st != DD_OK)
        return st;
    return adjoint_f32(p, *t, d_grad_out, d_in, d_weights, d_grad_in, d_grad_w,
                       static_cast<char *>(d_ws), static_cast<hipStream_t>(stream));
}

static dd_status check_box_args(const dd_plan *plan, const float *d_in, int32_t nbeams,
                                int32_t max_width, const void *d_ws, size_t ws_bytes)
{
    if (!plan || !d_in) {
        dd::set_error("plan and d_in must not be NULL");
        return DD_ERR_NULL;
    }
    if (plan->p.dtype != DD_F32) {
        dd::set_error("the boxcar loss is defined for DD_F32 plans");
        return DD_ERR_DTYPE;
    }
    if (nbeams < 1 || max_width < 1 || max_width > dd::kBoxMaxWidth ||
        (max_width & (max_width - 1)) != 0) {
        dd::set_error("need nbeams >= 1 and max_width a power of two in [1, 32]");
        return DD_ERR_INVALID;
    }
    if (ws_bytes < plan->p.ws_bytes || !d_ws || reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        dd::set_error("workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                      std::to_string(plan->p.ws_bytes) + " or not 256-byte aligned");
        return DD_ERR_WORKSPACE;
    }
    return DD_OK;
}

namespace {

dd_status check_batch_box(const dd_batch *batch, const void *d_in, int32_t max_width, const void *d_ws,
                          size_t ws_bytes)
{
    if (!batch || !d_in || !d_ws) {
        dd::set_error("batch, d_in and d_ws must not be NULL");
        return DD_ERR_NULL;
    }
    const dd::Batch &b = batch->b;
    if (b.dtype != DD_F32) {
        dd::set_error("the boxcar calls take DD_F32 batches");
        return DD_ERR_DTYPE;
    }
    if (max_width < 1 || max_width > dd::kBoxMaxWidth || (max_width & (max_width - 1)) != 0) {
        dd::set_error("max_width must be a power of two in [1, 32]");
        return DD_ERR_INVALID;
    }
    if (ws_bytes < b.box_ws_bytes || reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        dd::set_error("workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                      std::to_string(b.box_ws_bytes) + " (dd_batch_boxcar_workspace) or not 256-byte aligned");
        return DD_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(d_in) % 256 != 0) {
        dd::set_error("d_in must be 256-byte aligned");
        return DD_ERR_INVALID;
    }
    return DD_OK;
}

}  // namespace

dd_status dd_batch_boxcar_workspace(const dd_batch *batch, size_t *bytes)
{
    dd::clear_error();
    if (!batch || !bytes) {
        dd::set_error("batch and bytes must not be NULL");
        return DD_ERR_NULL;
    }
    if (batch->b.dtype != DD_F32) {
        dd::set_error("the boxcar calls take DD_F32 batches");
        return DD_ERR_DTYPE;
    }
    *bytes = batch->b.box_ws_bytes;
    return DD_OK;
}

dd_status dd_batch_boxcar_loss(const dd_batch *batch, const void *d_in, const float *d_weights,
                               int32_t max_width, float *d_loss, void *d_ws, size_t ws_bytes,
                               void *stream)
{
    dd::clear_error();
    dd_status st = check_batch_box(batch, d_in, max_width, d_ws, ws_bytes);
    if (st != DD_OK)
        return st;
    if (!d_loss) {
        dd::set_error("d_loss must not be NULL");
        return DD_ERR_NULL;
    }
    BatchDevice *bd = nullptr;
    st = batch_device(batch->b, &bd);
    if (st != DD_OK)
        return st;
    return batch_boxcar_loss_f32(batch->b, *bd, static_cast<const char *>(d_in), d_weights, max_width,
                                 d_loss, static_cast<char *>(d_ws), static_cast<hipStream_t>(stream));
}

dd_status dd_batch_boxcar_backward(const dd_batch *batch, const void *d_in, const float *d_weights,
                                   int32_t max_width, float *d_grad_in, float *d_grad_w, void *d_ws,
                                   size_t ws_bytes, void *stream)
{
    dd::clear_error();
    dd_status st = check_batch_box(batch, d_in, max_width, d_ws, ws_bytes);
    if (st != DD_OK)
        return st;
    if (!batch->b.box_fused) {
        dd::set_error("the batched boxcar backward takes plans of one range at full resolution "
                      "(dd_boxcar_backward covers the others beam by beam)");
        return DD_ERR_INVALID;
    }
    BatchDevice *bd = nullptr;
    st = batch_device(batch->b, &bd);
    if (st != DD_OK)
        return st;
    return batch_boxcar_backward_f32(batch->b, *bd, static_cast<const char *>(d_in), d_weights,
                                     max_width, d_grad_in, d_grad_w, static_cast<char *>(d_ws),
                                     static_cast<hipStream_t>(stream));
}

dd_status dd_boxcar_loss(const dd_plan *plan, const float *d_in, int32_t nbeams,
                         const float *d_weights, int32_t max_width, float *d_loss, void *d_ws,
                         size_t ws_bytes, void *stream)
{
    dd::clear_error();
    dd_status st = check_box_args(plan, d_in, nbeams, max_width, d_ws, ws_bytes);
    if (st != DD_OK)
        return st;
    if (!d_loss) {
        dd::set_error("d_loss must not be NULL");
        return DD_ERR_NULL;
    }
    DeviceTables *t = nullptr;
    st = device_tables(plan->p, &t);
    if (st != DD_OK)
        return st;
    return boxcar_loss_f32(plan->p, *t, d_in, nbeams, d_weights, max_width, d_loss,
                           static_cast<char *>(d_ws), static_cast<hipStream_t>(stream));
}

dd_status dd_boxcar_backward(const dd_plan *plan, const float *d_in, int32_t nbeams,
                             const float *d_weights, int32_t max_width, float *d_grad_in,
                             float *d_grad_w, void *d_ws, size_t ws_bytes, void *stream)
{
    dd::clear_error();
    dd_status st = check_box_args(plan, d_in, nbeams, max_width, d_ws, ws_bytes);
    if (st != DD_OK)
        return st;
    DeviceTables *t = nullptr;
    st = device_tables(plan->p, &t);
    if (st != DD_OK)
        return st;
    return boxcar_backward_f32(plan->p, *t, d_in, nbeams, d_weights, max_width, d_grad_in,
                               d_grad_w, static_cast<char *>(d_ws),
                               static_cast<hipStream_t>(stream));
}


dd_status dd_corner_turn(dd_dtype dtype, const void *d_in, int64_t nsamp, int32_t nchans,
                         void *d_out, int64_t out_pitch, void *stream)
{
    dd::clear_error();
    if (!d_in || !d_out) {
        dd::set_error("d_in and d_out must not be NULL");
        return DD_ERR_NULL;
    }
    if (nsamp <= 0 || nchans <= 0 || out_pitch < nsamp || (dtype != DD_U8 && dtype != DD_F32) ||
        (nchans + 31) / 32 > 65535) {
        dd::set_error("need nsamp > 0, 0 < nchans <= 2096640, out_pitch >= nsamp, a known dtype");
        return DD_ERR_INVALID;
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == DD_U8)
        return corner_turn_t(static_cast<const uint8_t *>(d_in), nsamp, nchans,
                             static_cast<uint8_t *>(d_out), out_pitch, 0, s);
    return corner_turn_t(static_cast<const float *>(d_in), nsamp, nchans,
                         static_cast<float *>(d_out), out_pitch, 0, s);
}

dd_status dd_stream_push(dd_stream *stream, const void *d_block, int64_t samples, void *d_chunk,
                         const float *d_weights, void *d_out, int64_t out_capacity, void *d_ws,
                         size_t ws_bytes, int64_t *chunk_index, void *hip_stream)
{
    dd::clear_error();
    if (!stream || !d_block || !d_chunk || !d_out) {
        dd::set_error("stream, d_block, d_chunk and d_out must not be NULL");
        return DD_ERR_NULL;
    }
    dd::Stream &S = stream->s;
    const Plan &p = *S.plan;
    const int64_t want = S.chunks == 0 ? p.nsamp : S.step;
    if (samples != want) {
        dd::set_error("this push needs " + std::to_string(want) + " samples, got " +
                      std::to_string(samples));
        return DD_ERR_INVALID;
    }
    if ((p.nchans + 31) / 32 > 65535) {
        dd::set_error("too many channels for the corner turn");
        return DD_ERR_INVALID;
    }
    // The forward's own checks run before anything is enqueued.
    dd_status st = check_forward_args(S.handle, d_chunk, d_weights, d_out, out_capacity, d_ws,
                                      ws_bytes, true);
    if (st != DD_OK)
        return st;
    const hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    if (p.dtype == DD_U8)
        st = stream_fill(S, static_cast<const uint8_t *>(d_block), samples,
                         static_cast<uint8_t *>(d_chunk), hs);
    else
        st = stream_fill(S, static_cast<const float *>(d_block), samples,
                         static_cast<float *>(d_chunk), hs);
    if (st != DD_OK)
        return st;
    st = dd_forward(S.handle, d_chunk, d_weights, d_out, out_capacity, d_ws, ws_bytes, hip_stream);
    if (st != DD_OK)
        return st;
    if (chunk_index)
        *chunk_index = S.chunks;
    ++S.chunks;
    return DD_OK;
}

}  // extern "C"
