// Device side of the dedispersion library for MI355X (gfx950): the binning
// kernel, the integer shift-and-sum kernel, device copies of the plan
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

#include "plan.h"

namespace {

using dd::Plan;
using dd::RangeInfo;

constexpr int kWave = 64;
constexpr int kBlock = dd::kWaves * kWave;
constexpr int kNW = dd::kWaveWords;
constexpr int kDW = dd::kDmPerWave;
constexpr int kTileT = dd::kTimeTile;
constexpr int kTileD = dd::kDmTile;
constexpr int kXcds = 8;     // workgroups are dealt to the XCDs round-robin

// ---------------------------------------------------------------------------
// Device-side plan state: the channel-major shift table, one copy per device.
// ---------------------------------------------------------------------------

struct DeviceTables {
    int32_t *offT = nullptr;
    int32_t *baseT = nullptr;
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
    const size_t ob = p.offT.size() * sizeof(int32_t);
    const size_t bb = p.baseT.size() * sizeof(int32_t);
    e = hipMalloc(&t.offT, ob + bb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dd::set_error(std::string("hipMalloc of the delay tables: ") + hipGetErrorString(e));
        return DD_ERR_NOMEM;
    }
    t.baseT = t.offT + p.offT.size();
    e = hipMemcpy(t.offT, p.offT.data(), ob, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.baseT, p.baseT.data(), bb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(t.offT);
        return hip_fail(e, "hipMemcpy of the delay tables");
    }
    *out = &(st->per_device[dev] = t);
    return DD_OK;
}

// ---------------------------------------------------------------------------
// Binning: dst[c][t] = sum_{k<f} src[c][f*t + k], t < nbin (uint16 result).
// ---------------------------------------------------------------------------

template <typename Tin>
__global__ __launch_bounds__(256) void k_bin_u16(const Tin *__restrict__ src, int64_t src_stride,
                                                 uint16_t *__restrict__ dst, int64_t nbin,
                                                 int factor)
{
    const int64_t c = blockIdx.y;
    const Tin *row = src + c * src_stride;
    uint16_t *out = dst + c * nbin;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < nbin;
         t += int64_t(gridDim.x) * blockDim.x) {
        const Tin *p = row + t * factor;
        uint32_t s = 0;
        for (int k = 0; k < factor; ++k)
            s += p[k];
        out[t] = uint16_t(s);
    }
}

// ---------------------------------------------------------------------------
// Integer shift-and-sum.
//
// A workgroup owns one (range, time tile of kTileT samples, DM tile of
// kTileD trials).  Wave w handles kDW consecutive DMs; lane l handles the
// sample pairs t0 + 2*(l + 64k) + {0, 1}, k < kNW, so a wave's LDS reads of
// one word index are 64 consecutive dwords (no bank conflict).
//
// Channels are staged in LDS in groups.  Staged channel c holds the window
// v[i] = x_r[c][t0 + s[d0][c] + i] (d0 = first DM of the tile) twice: as
// even-aligned pairs P0[m] = v[2m] | v[2m+1] << 16 and odd-aligned pairs
// P1[m] = v[2m+1] | v[2m+2] << 16.  The pair a lane needs for a DM with
// relative delay o = s[d][c] - s[d0][c] is then one aligned dword,
// P_{o&1}[(o>>1) + l + 64k], whatever the parity of o.
//
// Each dword carries two 16-bit partial sums.  Two channels are added per
// instruction (v_add3_u32).  A stage holds at most 65535/(255*ds) channels,
// so no 16-bit half can carry into the other; after each stage the halves
// are widened into int32 accumulators, which hold the exact result.
// ---------------------------------------------------------------------------

struct RangeArgs {
    const void *src;          // uint8 [nchans][src_stride] or uint16 binned rows
    const int32_t *offT;      // [nchans][ndms_pad] LDS word offsets of each DM
    const int32_t *baseT;     // [nchans][ndm_tiles] delay of each tile's first DM
    int64_t src_stride;       // elements per channel row of src
    int64_t nbin;             // valid samples per row of src
    int64_t nout;
    int64_t out_offset;
    int64_t block_start;
    int32_t src_u16;
    int32_t ndms;
    int32_t stage_chans;
    int32_t row_words;
    int32_t ndm_tiles;
    int32_t ndms_pad;
};

struct FwdArgs {
    RangeArgs r[DD_MAX_RANGES];
    int32_t *out;
    int64_t nblocks;
    int64_t per_xcd;
    int32_t nranges;
    int32_t nchans;
};

__device__ __forceinline__ uint32_t sample_at(const RangeArgs &R, int64_t c, int64_t t)
{
    if (t >= R.nbin)
        return 0u;
    if (R.src_u16)
        return static_cast<const uint16_t *>(R.src)[c * R.src_stride + t];
    return static_cast<const uint8_t *>(R.src)[c * R.src_stride + t];
}

__global__ __launch_bounds__(kBlock) void k_dedisp_u8(const FwdArgs a)
{
    extern __shared__ uint32_t lds[];

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
    const RangeArgs &R = a.r[r];

    const int64_t lb = L - R.block_start;
    const int64_t tt = lb / R.ndm_tiles;
    const int tile = int(lb - tt * R.ndm_tiles);
    const int d0 = tile * kTileD;
    const int64_t t0 = tt * kTileT;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int ndms = R.ndms;
    const int dpad = R.ndms_pad;
    const int ntiles = R.ndm_tiles;
    const int dw0 = d0 + wave * kDW;
    const int nchans = a.nchans;
    const int C = R.stage_chans;
    const int Cp = (C + 1) & ~1;
    const int Lw = R.row_words;

    uint32_t acc16[kDW][kNW];
    int32_t acc32[kDW][kNW][2];
#pragma unroll
    for (int dd = 0; dd < kDW; ++dd)
#pragma unroll
        for (int k = 0; k < kNW; ++k) {
            acc16[dd][k] = 0u;
            acc32[dd][k][0] = 0;
            acc32[dd][k][1] = 0;
        }

    for (int c0 = 0; c0 < nchans; c0 += C) {
        const int cn = min(C, nchans - c0);
        // Stage the channel windows (rows past the last channel are zero).
        for (int j = 0; j < Cp; ++j) {
            uint32_t *P0 = lds + (2 * j) * Lw;
            uint32_t *P1 = P0 + Lw;
            if (j < cn) {
                const int64_t c = c0 + j;
                const int64_t tb = t0 + R.baseT[c * ntiles + tile];
                for (int m = tid; m < Lw; m += kBlock) {
                    const int64_t t = tb + 2 * m;
                    const uint32_t v0 = sample_at(R, c, t);
                    const uint32_t v1 = sample_at(R, c, t + 1);
                    const uint32_t v2 = sample_at(R, c, t + 2);
                    P0[m] = v0 | (v1 << 16);
                    P1[m] = v1 | (v2 << 16);
                }
            } else {
                for (int m = tid; m < Lw; m += kBlock) {
                    P0[m] = 0u;
                    P1[m] = 0u;
                }
            }
        }
        __syncthreads();

        for (int jp = 0; jp < Cp; jp += 2) {
            // Offsets of this wave's DMs in the two staged channels; the
            // table is padded so the 8 entries are aligned and in bounds.
            const int32_t *oa = R.offT + int64_t(c0 + jp) * dpad + dw0;
            const int32_t *ob = jp + 1 < cn ? oa + dpad : oa;
            const int4 a0 = *reinterpret_cast<const int4 *>(oa);
            const int4 a1 = *reinterpret_cast<const int4 *>(oa + 4);
            const int4 b0 = *reinterpret_cast<const int4 *>(ob);
            const int4 b1 = *reinterpret_cast<const int4 *>(ob + 4);
            const int offa[kDW] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const int offb[kDW] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
            const uint32_t *rowa = lds + (2 * jp) * Lw + lane;
            const uint32_t *rowb = rowa + 2 * Lw;
#pragma unroll
            for (int dd = 0; dd < kDW; ++dd) {
                const uint32_t *pa = rowa + offa[dd];
                const uint32_t *pb = rowb + offb[dd];
#pragma unroll
                for (int k = 0; k < kNW; ++k)
                    acc16[dd][k] += pa[kWave * k] + pb[kWave * k];
            }
        }
#pragma unroll
        for (int dd = 0; dd < kDW; ++dd)
#pragma unroll
            for (int k = 0; k < kNW; ++k) {
                acc32[dd][k][0] += int32_t(acc16[dd][k] & 0xffffu);
                acc32[dd][k][1] += int32_t(acc16[dd][k] >> 16);
                acc16[dd][k] = 0u;
            }
        __syncthreads();
    }

#pragma unroll
    for (int dd = 0; dd < kDW; ++dd) {
        const int d = dw0 + dd;
        if (d >= ndms)
            break;
        int32_t *row = a.out + R.out_offset + int64_t(d) * R.nout;
#pragma unroll
        for (int k = 0; k < kNW; ++k) {
            const int64_t t = t0 + 2 * (lane + kWave * k);
            if (t < R.nout)
                row[t] = acc32[dd][k][0];
            if (t + 1 < R.nout)
                row[t + 1] = acc32[dd][k][1];
        }
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

dd_status bin_u8(const Plan &p, const uint8_t *d_in, char *d_ws, hipStream_t stream)
{
    // Binned copies, each from its source level, in increasing order.
    for (const dd::BinLevel &lv : p.levels) {
        uint16_t *dst = reinterpret_cast<uint16_t *>(d_ws + lv.ws_offset);
        const dim3 grid(unsigned(std::min<int64_t>((lv.nbin + 255) / 256, 1024)),
                        unsigned(p.nchans));
        if (lv.src < 0) {
            hipLaunchKernelGGL(k_bin_u16<uint8_t>, grid, dim3(256), 0, stream, d_in, p.nsamp,
                               dst, lv.nbin, lv.factor);
        } else {
            const dd::BinLevel &sl = p.levels[lv.src];
            const uint16_t *src = reinterpret_cast<const uint16_t *>(d_ws + sl.ws_offset);
            hipLaunchKernelGGL(k_bin_u16<uint16_t>, grid, dim3(256), 0, stream, src, sl.nbin,
                               dst, lv.nbin, lv.factor);
        }
        dd_status st = launch_check("k_bin_u16");
        if (st != DD_OK)
            return st;
    }
    return DD_OK;
}

dd_status sum_u8(const Plan &p, const DeviceTables &t, const uint8_t *d_in, int32_t *d_out,
                 const char *d_ws, hipStream_t stream)
{
    FwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.out = d_out;
    a.nblocks = p.blocks;
    a.per_xcd = (p.blocks + kXcds - 1) / kXcds;
    a.nranges = int32_t(p.ranges.size());
    a.nchans = p.nchans;
    for (size_t i = 0; i < p.ranges.size(); ++i) {
        const RangeInfo &ri = p.ranges[i];
        RangeArgs &R = a.r[i];
        if (ri.level < 0) {
            R.src = d_in;
            R.src_stride = p.nsamp;
            R.src_u16 = 0;
        } else {
            const dd::BinLevel &lv = p.levels[ri.level];
            R.src = d_ws + lv.ws_offset;
            R.src_stride = lv.nbin;
            R.src_u16 = 1;
        }
        R.offT = t.offT + ri.off_offset;
        R.baseT = t.baseT + ri.base_offset;
        R.ndms_pad = ri.ndms_pad;
        R.nbin = ri.nbin;
        R.nout = ri.nout;
        R.out_offset = ri.out_offset;
        R.block_start = ri.block_start;
        R.ndms = ri.ndms;
        R.stage_chans = ri.stage_chans;
        R.row_words = ri.row_words;
        R.ndm_tiles = ri.ndm_tiles;
    }
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_dedisp_u8),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(dd::kMaxLdsBytes));
    });
    const int64_t grid = a.per_xcd * kXcds;
    hipLaunchKernelGGL(k_dedisp_u8, dim3(unsigned(grid)), dim3(kBlock), p.lds_bytes, stream, a);
    return launch_check("k_dedisp_u8");
}

// Argument checks shared by the compute entry points (synchronous, before
// any HIP call).
dd_status check_forward_args(const dd_plan *plan, const void *d_in, const float *d_weights,
                             const void *d_out, int64_t out_capacity, const void *d_ws,
                             size_t ws_bytes, bool need_out)
{
    if (!plan || !d_in || (need_out && !d_out)) {
        dd::set_error("plan, d_in and d_out must not be NULL");
        return DD_ERR_NULL;
    }
    const Plan &p = plan->p;
    if (p.dtype == DD_U8 && d_weights) {
        dd::set_error("per-channel weights apply to DD_F32 plans only");
        return DD_ERR_DTYPE;
    }
    if (p.dtype != DD_U8) {
        dd::set_error("this build computes DD_U8 plans only");
        return DD_ERR_DTYPE;
    }
    if (need_out && out_capacity < p.out_elems) {
        dd::set_error("out_capacity " + std::to_string(out_capacity) + " < out_elems " +
                      std::to_string(p.out_elems));
        return DD_ERR_CAPACITY;
    }
    if (ws_bytes < p.ws_bytes || (p.ws_bytes > 0 && !d_ws)) {
        dd::set_error("workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                      std::to_string(p.ws_bytes));
        return DD_ERR_WORKSPACE;
    }
    return DD_OK;
}

}  // namespace

void *dd::new_device_state() { return new (std::nothrow) DeviceState; }

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

dd_status dd_forward_bin(const dd_plan *plan, const void *d_in, void *d_ws, size_t ws_bytes,
                         void *stream)
{
    dd::clear_error();
    dd_status st = check_forward_args(plan, d_in, nullptr, nullptr, 0, d_ws, ws_bytes, false);
    if (st != DD_OK)
        return st;
    return bin_u8(plan->p, static_cast<const uint8_t *>(d_in), static_cast<char *>(d_ws),
                  static_cast<hipStream_t>(stream));
}

dd_status dd_forward_sum(const dd_plan *plan, const void *d_in, const float *d_weights,
                         void *d_out, int64_t out_capacity, void *d_ws, size_t ws_bytes,
                         void *stream)
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
    return sum_u8(plan->p, *t, static_cast<const uint8_t *>(d_in), static_cast<int32_t *>(d_out),
                  static_cast<const char *>(d_ws), static_cast<hipStream_t>(stream));
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
    st = bin_u8(plan->p, static_cast<const uint8_t *>(d_in), static_cast<char *>(d_ws), s);
    if (st != DD_OK)
        return st;
    return sum_u8(plan->p, *t, static_cast<const uint8_t *>(d_in), static_cast<int32_t *>(d_out),
                  static_cast<const char *>(d_ws), s);
}

}  // extern "C"
