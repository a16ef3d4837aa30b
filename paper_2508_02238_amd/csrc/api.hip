// api.hip -- the C ABI declared in include/esi.h: argument checks, state and
// scratch ownership, the per-call schedule, and stream-ordered launches.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "esi.h"
#include "esi_internal.hpp"

using namespace esi;

namespace {

// A named range on the calling thread for profilers (rocprofv3
// --marker-trace): the host time of an entry point and of each launch phase
// it enqueues.  The phases' GPU time is measured with HIP events instead
// (esi_profile_enable).
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

}  // namespace

// A pixel's run of more than this many events in one chunk of its tile is
// integrated by the scan of the whole wave rather than by one lane: below it
// the wave's fixed cost per 64 events (the scan's six composition steps)
// exceeds one lane's loop.
constexpr int kDefaultScanRun = 64;

// The scan threshold a call uses: the state's (set by esi_set_scan_run), or
// by default 64 for tiles of two or more pixels per thread and off for one
// pixel per thread, whose kernel the scan's code alone slows.
int effective_scan_run(int state_scan_run, int ppt)
{
    if (state_scan_run > 0)
        return state_scan_run;
    return ppt == 1 ? kScanOff : kDefaultScanRun;
}

struct esi_state {
    int32_t W = 0, H = 0;
    int64_t npix = 0;
    esi_params params{};
    int device = 0;
    // one allocation: S_hi f32, S_lo f32, T i64, N u32, P i32
    void* state_mem = nullptr;
    StateDev dev{};
    DiagDev* diag = nullptr;
    // scratch of integrate calls, grown on demand
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    // device address of the static scratch on this state's device (null if
    // the lookup failed: esi_integrate_window_noalloc then returns ESI_ERR_HIP)
    void* static_scratch = nullptr;
    int bucket_slots[2] = {1024, 1024};  // bucketing workgroups resident at once (narrow, wide)
    int integ_slots[4] = {1 << 30, 1 << 30, 1 << 30, 1 << 30};  // per ppt 1, 2, 4, 8
    int integ_slots_big = 1 << 30;  // two pixels per thread, 2048-record chunks
    int chunk = 0;                  // 2048: that form for tiles of 512 pixels
    int min_ppt = 1;          // smallest pixels per thread of the integration tiles
    int scan_run = 0;  // longer runs per chunk take the wave's scan (0: by tile size)
    bool state_in_range = true;  // every S in [s_min, s_max] (false after importing one outside)
    bool poisoned = false;
    uint64_t calls = 0;
    // profiling: HIP events around the two phases of recorded calls
    bool profiling = false;
    uint32_t prof_calls = 0;
    hipEvent_t* prof_ev = nullptr;  // [kProfMax][3]
};

// Descriptor staging of batched calls: pinned host copy and device copy.
struct esi_batch {
    int32_t max_items = 0;
    int device = 0;
    size_t bytes = 0;
    void* host = nullptr;
    void* dev = nullptr;
    hipEvent_t copied = nullptr;  // recorded after the last staging copy
    hipEvent_t used = nullptr;    // recorded after the last call's kernels
    bool pending = false;
    // frame times given in host memory, staged with the descriptors
    void* tf_host = nullptr;
    void* tf_dev = nullptr;
    size_t tf_cap = 0;
};

// Scratch of esi_integrate_window_noalloc, which allocates nothing: a fixed
// array in every GPU's memory that the library runs on (each device holds its
// own copy at its own address until the process ends).  Host code never
// passes this name to a kernel: it is a host-side stand-in, not a device
// address.  The device address is looked up once per device
// (static_scratch_address) and only that pointer is used.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_scratch[kMaxDevices] = {};

// The device address of `scratch` on device `dev`, which must be the current
// device; looked up on the first call for that device (esi_create_state),
// then cached.  Null if the lookup fails.
void* static_scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
            g_static_scratch[dev] = p;
        else
            (void)hipGetLastError();
    }
    return g_static_scratch[dev];
}

}  // namespace

namespace {

constexpr uint64_t kMagic = 0x3130495345ull;  // "ESI01"
constexpr uint32_t kProfMax = 1024;
// pixels of one pass of the kernels (kMaxTiles tiles of 2048 pixels); larger
// sensors are integrated in bands of rows, one pass each
constexpr int64_t kMaxPixels = (int64_t)kMaxTiles * 256 * 8;  // 4096000
constexpr int32_t kMaxSide = 65536;
constexpr int32_t kMaxBatch = 4096;  // streams per batched call

struct SerialHeader {
    uint64_t magic;
    int32_t W, H;
    uint64_t dropped, accepted;
    uint32_t flags, pad;
};

bool params_ok(const esi_params* p)
{
    return p && std::isfinite(p->C) && p->C > 0.0 && std::isfinite(p->k_per_us) &&
           p->k_per_us >= 0.0 && std::isfinite(p->b) && p->b > 0.0 && std::isfinite(p->s_min) &&
           std::isfinite(p->s_max) && p->s_min < p->s_max &&
           (p->flags & ~(uint32_t)(ESI_DECAY_THEN_ADD | ESI_SNAPSHOT_LAZY | ESI_DECAY_EXP)) == 0;
}

MethodParams method_params(const esi_params& p)
{
    MethodParams mp{};
    mp.scan_run = kDefaultScanRun;
    mp.C = p.C;
    mp.k = p.k_per_us;
    mp.b = p.b;
    mp.s_min = p.s_min;
    mp.s_max = p.s_max;
    mp.inv_range = 1.0 / (p.s_max - p.s_min);
    mp.f_off = -p.s_min * mp.inv_range;
    mp.sv_min = p.s_min * mp.inv_range;
    mp.sv_max = p.s_max * mp.inv_range;
    // a state in [s_min, s_max] decays towards 0, so it stays in range when
    // s_min <= 0 <= s_max
    mp.need_clamp = (p.s_min > 0.0 || p.s_max < 0.0) ? 1 : 0;
    mp.decay_then_add = (p.flags & ESI_DECAY_THEN_ADD) ? 1 : 0;
    mp.lazy = (p.flags & ESI_SNAPSHOT_LAZY) ? 1 : 0;
    mp.exp_decay = (p.flags & ESI_DECAY_EXP) ? 1 : 0;
    return mp;
}

// The split of one call into tiles and bucketing units: the smallest tile
// (most workgroups) with at most kMaxTiles tiles; the events split evenly over
// as many bucketing workgroups as the GPU holds at once (`slots`).
Schedule make_schedule(int64_t npix, int64_t n, int slots, int min_ppt = 1,
                       const int* integ_slots = nullptr)
{
    Schedule s{};
    for (int ppt = min_ppt; ppt <= 8; ppt *= 2) {
        s.ppt = ppt;
        s.tile_log = 8 + (ppt == 1 ? 0 : ppt == 2 ? 1 : ppt == 4 ? 2 : 3);
        s.ntiles = (int)((npix + (256 * ppt) - 1) / (256 * ppt));
        if (s.ntiles <= kMaxTiles)
            break;
    }
    const int pi = s.ppt == 1 ? 0 : s.ppt == 2 ? 1 : s.ppt == 4 ? 2 : 3;
    s.ordered = n > 0 && integ_slots && s.ntiles > integ_slots[pi];
    const int64_t per = (n + slots - 1) / std::max(slots, 1);
    s.unit_events = std::max<int64_t>(256, (per + 255) / 256 * 256);
    s.nunits = (n + s.unit_events - 1) / s.unit_events;
    return s;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev)
            (void)hipSetDevice(dev);
        else
            prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

esi_status hip_fail(esi_state* st)
{
    if (st)
        st->poisoned = true;
    return ESI_ERR_HIP;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Rows per pass of the kernels: the whole sensor when it fits one pass,
// else the most rows whose pixels fit.
int64_t band_rows(int32_t W, int32_t H)
{
    return ((int64_t)W * H <= kMaxPixels) ? (int64_t)H : kMaxPixels / W;
}

// Frame times given in host memory are staged on the device.
bool device_accessible(const void* p)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // plain pageable host memory
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

// The scratch layout of one call under schedule sc (n events; nf_stage
// frame times staged from host memory): frame times | table | segment sums |
// tile totals | tile order | total | records.  Every part is written by the call's own
// kernels before it is read (the tile totals are cleared by k_hist), so no
// part needs clearing between calls.
struct ScratchPlan {
    size_t o_tab, o_bs, o_tt, o_ord, o_tot, o_rec, need;
};

ScratchPlan scratch_plan(const Schedule& sc, int64_t n, int32_t nf_stage)
{
    ScratchPlan p{};
    const int64_t M = n > 0 ? (int64_t)sc.ntiles * sc.nunits : 0;
    const int64_t nseg = n > 0 ? (int64_t)scan_segments(sc.nunits) : 0;
    p.o_tab = align_up(8 * (size_t)nf_stage, 256);
    p.o_bs = p.o_tab + align_up(4 * (size_t)M, 256);
    p.o_tt = p.o_bs + align_up(4 * (size_t)(nseg * sc.ntiles), 256);
    p.o_ord = p.o_tt + align_up(4 * (size_t)sc.ntiles, 256);
    p.o_tot = p.o_ord + align_up(4 * (size_t)sc.ntiles, 256);
    p.o_rec = p.o_tot + 256;
    // records: n, and one spare slot that the bucketing writes for lanes
    // without a record
    p.need = p.o_rec + 8 * ((size_t)n + 1);
    return p;
}

void carve_scratch(char* base, const ScratchPlan& p, CallScratch& cs, int64_t** tf_stage)
{
    if (tf_stage)
        *tf_stage = (int64_t*)base;
    cs.table = (uint32_t*)(base + p.o_tab);
    cs.blocksum = (uint32_t*)(base + p.o_bs);
    cs.tile_tot = (uint32_t*)(base + p.o_tt);
    cs.order = (uint32_t*)(base + p.o_ord);
    cs.total = (uint32_t*)(base + p.o_tot);
    cs.records = (uint64_t*)(base + p.o_rec);
}

// The state's own scratch for one call, grown on demand (after the stream
// has finished with the old one).
esi_status call_scratch(esi_state* st, const Schedule& sc, int64_t n, int32_t nf_stage,
                        hipStream_t stream, CallScratch& cs, int64_t** tf_stage)
{
    const ScratchPlan p = scratch_plan(sc, n, nf_stage);
    if (p.need > st->scratch_bytes) {
        // the old scratch may still be read by work queued on this stream
        if (st->scratch && hipStreamSynchronize(stream) != hipSuccess)
            return hip_fail(st);
        if (st->scratch)
            (void)hipFree(st->scratch);
        st->scratch = nullptr;
        st->scratch_bytes = 0;
        const size_t bytes = p.need + p.need / 4;
        if (hipMalloc(&st->scratch, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return ESI_ERR_OUT_OF_MEMORY;
        }
        st->scratch_bytes = bytes;
    }
    carve_scratch((char*)st->scratch, p, cs, tf_stage);
    return ESI_OK;
}

// The state of rows [y0, y0 + rows) as a state of its own (one pass).
StateDev band_state(const StateDev& d, int64_t y0, int64_t rows)
{
    const int64_t off = y0 * d.W;
    StateDev b = d;
    b.S_hi += off;
    b.S_lo += off;
    b.T += off;
    b.N += off;
    b.P += off;
    b.H = (int)rows;
    b.npix = rows * d.W;
    return b;
}

}  // namespace

extern "C" {

const char* esi_status_string(esi_status s)
{
    switch (s) {
    case ESI_OK:
        return "ESI_OK";
    case ESI_ERR_INVALID_ARG:
        return "ESI_ERR_INVALID_ARG: an argument is out of its documented range";
    case ESI_ERR_OUT_OF_MEMORY:
        return "ESI_ERR_OUT_OF_MEMORY: device allocation failed";
    case ESI_ERR_HIP:
        return "ESI_ERR_HIP: a HIP runtime call failed; the state is poisoned";
    case ESI_ERR_POISONED:
        return "ESI_ERR_POISONED: an earlier HIP failure; call esi_reset or esi_import_state";
    case ESI_ERR_SCRATCH_LIMIT:
        return "ESI_ERR_SCRATCH_LIMIT: the call needs more scratch than the static 64 MiB of "
               "esi_integrate_window_noalloc";
    }
    return "ESI_ERR_UNKNOWN";
}

esi_status esi_create_state(int32_t width, int32_t height, const esi_params* params,
                            hipStream_t stream, esi_state** out)
{
    if (!out)
        return ESI_ERR_INVALID_ARG;
    *out = nullptr;
    if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide || !params_ok(params))
        return ESI_ERR_INVALID_ARG;
    const int64_t npix = (int64_t)width * height;
    esi_state* st = new (std::nothrow) esi_state();
    if (!st)
        return ESI_ERR_OUT_OF_MEMORY;
    st->W = width;
    st->H = height;
    st->npix = npix;
    st->params = *params;
    if (hipGetDevice(&st->device) != hipSuccess) {
        delete st;
        return ESI_ERR_HIP;
    }
    const size_t n = (size_t)npix;
    const size_t o_lo = align_up(4 * n, 256), o_T = o_lo + align_up(4 * n, 256);
    const size_t o_N = o_T + align_up(8 * n, 256), o_P = o_N + align_up(4 * n, 256);
    const size_t o_diag = o_P + align_up(4 * n, 256);
    const size_t bytes = o_diag + 256;
    if (hipMalloc(&st->state_mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete st;
        return ESI_ERR_OUT_OF_MEMORY;
    }
    char* base = (char*)st->state_mem;
    st->dev.S_hi = (float*)base;
    st->dev.S_lo = (float*)(base + o_lo);
    st->dev.T = (int64_t*)(base + o_T);
    st->dev.N = (uint32_t*)(base + o_N);
    st->dev.P = (int32_t*)(base + o_P);
    st->dev.W = width;
    st->dev.H = height;
    st->dev.npix = npix;
    st->diag = (DiagDev*)(base + o_diag);
    st->bucket_slots[0] = bucket_slots(1);
    st->bucket_slots[1] = bucket_slots(kMaxTiles);
    st->static_scratch = static_scratch_address(st->device);
    for (int i = 0; i < 4; ++i)
        st->integ_slots[i] = integrate_slots(1 << i);
    st->integ_slots_big = integrate_slots(2, true);
    if (launch_reset(st->dev, params->t0_us, st->diag, stream) != hipSuccess) {
        (void)hipFree(st->state_mem);
        delete st;
        return ESI_ERR_HIP;
    }
    *out = st;
    return ESI_OK;
}

esi_status esi_destroy_state(esi_state* st)
{
    if (!st)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(st->device);
    esi_status rc = ESI_OK;
    if (hipDeviceSynchronize() != hipSuccess)
        rc = ESI_ERR_HIP;
    if (st->scratch)
        (void)hipFree(st->scratch);
    if (st->state_mem)
        (void)hipFree(st->state_mem);
    if (st->prof_ev) {
        for (uint32_t i = 0; i < 3 * kProfMax; ++i)
            (void)hipEventDestroy(st->prof_ev[i]);
        delete[] st->prof_ev;
    }
    delete st;
    return rc;
}

esi_status esi_profile_enable(esi_state* st, int enable)
{
    if (!st)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(st->device);
    if (enable && !st->prof_ev) {
        st->prof_ev = new (std::nothrow) hipEvent_t[3 * kProfMax];
        if (!st->prof_ev)
            return ESI_ERR_OUT_OF_MEMORY;
        for (uint32_t i = 0; i < 3 * kProfMax; ++i)
            if (hipEventCreate(&st->prof_ev[i]) != hipSuccess) {
                for (uint32_t k = 0; k < i; ++k)
                    (void)hipEventDestroy(st->prof_ev[k]);
                delete[] st->prof_ev;
                st->prof_ev = nullptr;
                return hip_fail(st);
            }
    }
    st->profiling = enable != 0;
    st->prof_calls = 0;
    return ESI_OK;
}

esi_status esi_profile_read(esi_state* st, uint32_t* calls, double* bucket_ms,
                            double* integrate_ms)
{
    if (!st || !calls || !bucket_ms || !integrate_ms)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(st->device);
    *calls = st->prof_calls;
    *bucket_ms = 0.0;
    *integrate_ms = 0.0;
    for (uint32_t c = 0; c < st->prof_calls; ++c) {
        hipEvent_t* pe = st->prof_ev + 3 * c;
        float a = 0.f, b = 0.f;
        if (hipEventSynchronize(pe[2]) != hipSuccess || hipEventElapsedTime(&a, pe[0], pe[1]) ||
            hipEventElapsedTime(&b, pe[1], pe[2]))
            return hip_fail(st);
        *bucket_ms += a;
        *integrate_ms += b;
    }
    return ESI_OK;
}

esi_status esi_reset(esi_state* st, hipStream_t stream)
{
    if (!st)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(st->device);
    if (launch_reset(st->dev, st->params.t0_us, st->diag, stream) != hipSuccess)
        return hip_fail(st);
    st->poisoned = false;
    st->state_in_range = true;
    st->calls = 0;
    return ESI_OK;
}

}  // extern "C"

namespace {

// One integrate call (esi_integrate_window, esi_integrate_window_noalloc):
// argument checks, the schedule, scratch from the state's own buffer or from
// the device's static array, and the launches of every band.
esi_status integrate_window_impl(esi_state* st, const esi_events* ev, const int64_t* t_frames,
                                 int32_t n_frames, float* frames, uint8_t* frames_u8,
                                 hipStream_t stream, bool static_scratch)
{
    if (!st || !ev || n_frames < 0)
        return ESI_ERR_INVALID_ARG;
    if (ev->n > 0 && (!ev->x || !ev->y || !ev->t || !ev->p))
        return ESI_ERR_INVALID_ARG;
    if (ev->n >= ((size_t)1 << 31))
        return ESI_ERR_INVALID_ARG;
    if ((n_frames > 0) != (t_frames != nullptr))
        return ESI_ERR_INVALID_ARG;
    if (n_frames > 0 && !frames && !frames_u8)
        return ESI_ERR_INVALID_ARG;
    if (st->poisoned)
        return ESI_ERR_POISONED;
    Range range(static_scratch ? "esi_integrate_window_noalloc" : "esi_integrate_window");
    DeviceGuard g(st->device);
    const int64_t n = (int64_t)ev->n;
    MethodParams mp = method_params(st->params);
    if (!st->state_in_range)
        mp.need_clamp = 1;
    // the sensor in bands of rows, one pass of the kernels each (one band
    // unless the sensor is larger than a pass holds); the first band is the
    // largest, so its scratch serves every band
    const int64_t rows = band_rows(st->W, st->H);
    const bool stage_tf = n_frames > 0 && !device_accessible(t_frames);
    // ranges: the resident workgroups of the bucketing form the call's tile
    // count selects (the tile count does not depend on the ranges)
    const int slots =
        st->bucket_slots[bucket_wide(make_schedule(rows * st->W, n, 1, st->min_ppt).ntiles)];
    const Schedule sc0 = make_schedule(rows * st->W, n, slots, st->min_ppt);
    CallScratch cs{};
    int64_t* tf_dev = nullptr;
    if (static_scratch) {
        // frame times must already be device memory (nothing is staged), and
        // the call's scratch must fit the static array
        if (stage_tf)
            return ESI_ERR_INVALID_ARG;
        const ScratchPlan p = scratch_plan(sc0, n, 0);
        if (p.need > kStaticScratchBytes)
            return ESI_ERR_SCRATCH_LIMIT;
        if (!st->static_scratch)
            return ESI_ERR_HIP;
        carve_scratch((char*)st->static_scratch, p, cs, nullptr);
    } else if (n > 0 || stage_tf) {
        const esi_status rc =
            call_scratch(st, sc0, n, stage_tf ? n_frames : 0, stream, cs, &tf_dev);
        if (rc != ESI_OK)
            return rc;
    }
    const int64_t* tf = t_frames;
    if (stage_tf) {
        if (hipMemcpyAsync(tf_dev, t_frames, 8 * (size_t)n_frames, hipMemcpyHostToDevice,
                           stream) != hipSuccess)
            return hip_fail(st);
        tf = tf_dev;
    }
    hipEvent_t* pe = nullptr;
    if (st->profiling && st->prof_calls < kProfMax) {
        pe = st->prof_ev + 3 * st->prof_calls++;
        if (hipEventRecord(pe[0], stream) != hipSuccess)
            return hip_fail(st);
    }
    for (int64_t y0 = 0; y0 < st->H; y0 += rows) {
        const int64_t hb = std::min<int64_t>(rows, st->H - y0);
        const StateDev sd = band_state(st->dev, y0, hb);
        Schedule sc = make_schedule(sd.npix, n, slots, st->min_ppt, st->integ_slots);
        if (st->chunk == 2048 && sc.ppt == 2) {
            sc.big_chunk = true;
            sc.ordered = n > 0 && sc.ntiles > st->integ_slots_big;
        }
        const EventsDev evd{ev->x, ev->y, ev->t, ev->p, n, (int)y0, st->H};
        const int64_t off = y0 * st->W;
        const FrameOut fo{tf, n_frames, frames ? frames + off : nullptr,
                          frames_u8 ? frames_u8 + off : nullptr, st->npix};
        if (n > 0) {
            Range phase("bucketing");
            if (launch_bucket(evd, sd, sc, cs, st->diag, stream) != hipSuccess)
                return hip_fail(st);
        }
        // the bucketing time of a banded call is its first band's
        if (pe && y0 == 0 && hipEventRecord(pe[1], stream) != hipSuccess)
            return hip_fail(st);
        if (n > 0 || n_frames > 0) {
            Range phase("integration");
            mp.scan_run = effective_scan_run(st->scan_run, sc.ppt);
            if (launch_integrate(evd, sd, sc, cs, mp, fo, st->diag, stream) != hipSuccess)
                return hip_fail(st);
        }
    }
    if (pe && hipEventRecord(pe[2], stream) != hipSuccess)
        return hip_fail(st);
    st->calls++;
    return ESI_OK;
}

}  // namespace

extern "C" {

esi_status esi_integrate_window(esi_state* st, const esi_events* ev, const int64_t* t_frames,
                                int32_t n_frames, float* frames, uint8_t* frames_u8,
                                hipStream_t stream)
{
    return integrate_window_impl(st, ev, t_frames, n_frames, frames, frames_u8, stream, false);
}

esi_status esi_integrate_window_noalloc(esi_state* st, const esi_events* ev,
                                        const int64_t* t_frames, int32_t n_frames, float* frames,
                                        uint8_t* frames_u8, hipStream_t stream)
{
    return integrate_window_impl(st, ev, t_frames, n_frames, frames, frames_u8, stream, true);
}

esi_status esi_snapshot_frame(esi_state* st, int64_t t_frame_us, float* frame, uint8_t* u8,
                              hipStream_t stream)
{
    if (!st || (!frame && !u8))
        return ESI_ERR_INVALID_ARG;
    if (st->poisoned)
        return ESI_ERR_POISONED;
    Range range("esi_snapshot_frame");
    DeviceGuard g(st->device);
    if (launch_snapshot(st->dev, method_params(st->params), t_frame_us, frame, u8, stream) !=
        hipSuccess)
        return hip_fail(st);
    return ESI_OK;
}

esi_status esi_read_state(esi_state* st, float* S, int64_t* T, uint32_t* N, int32_t* P,
                          hipStream_t stream)
{
    if (!st)
        return ESI_ERR_INVALID_ARG;
    if (st->poisoned)
        return ESI_ERR_POISONED;
    DeviceGuard g(st->device);
    const size_t n = (size_t)st->npix;
    if ((S && hipMemcpyAsync(S, st->dev.S_hi, 4 * n, hipMemcpyDeviceToDevice, stream)) ||
        (T && hipMemcpyAsync(T, st->dev.T, 8 * n, hipMemcpyDeviceToDevice, stream)) ||
        (N && hipMemcpyAsync(N, st->dev.N, 4 * n, hipMemcpyDeviceToDevice, stream)) ||
        (P && hipMemcpyAsync(P, st->dev.P, 4 * n, hipMemcpyDeviceToDevice, stream)))
        return hip_fail(st);
    return ESI_OK;
}

size_t esi_state_bytes(const esi_state* st)
{
    return st ? sizeof(SerialHeader) + 24 * (size_t)st->npix : 0;
}

esi_status esi_export_state(esi_state* st, void* host_buf, size_t bytes)
{
    if (!st || !host_buf || bytes < esi_state_bytes(st))
        return ESI_ERR_INVALID_ARG;
    if (st->poisoned)
        return ESI_ERR_POISONED;
    DeviceGuard g(st->device);
    if (hipDeviceSynchronize() != hipSuccess)
        return hip_fail(st);
    const size_t n = (size_t)st->npix;
    SerialHeader h{};
    DiagDev d{};
    if (hipMemcpy(&d, st->diag, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess)
        return hip_fail(st);
    h.magic = kMagic;
    h.W = st->W;
    h.H = st->H;
    h.dropped = d.dropped;
    h.accepted = d.accepted;
    h.flags = d.flags;
    char* p = (char*)host_buf;
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    if (hipMemcpy(p, st->dev.S_hi, 4 * n, hipMemcpyDeviceToHost) ||
        hipMemcpy(p + 4 * n, st->dev.S_lo, 4 * n, hipMemcpyDeviceToHost) ||
        hipMemcpy(p + 8 * n, st->dev.T, 8 * n, hipMemcpyDeviceToHost) ||
        hipMemcpy(p + 16 * n, st->dev.N, 4 * n, hipMemcpyDeviceToHost) ||
        hipMemcpy(p + 20 * n, st->dev.P, 4 * n, hipMemcpyDeviceToHost))
        return hip_fail(st);
    return ESI_OK;
}

esi_status esi_import_state(esi_state* st, const void* host_buf, size_t bytes)
{
    if (!st || !host_buf || bytes < esi_state_bytes(st))
        return ESI_ERR_INVALID_ARG;
    SerialHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (h.magic != kMagic || h.W != st->W || h.H != st->H)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(st->device);
    if (hipDeviceSynchronize() != hipSuccess)
        return hip_fail(st);
    const size_t n = (size_t)st->npix;
    const char* p = (const char*)host_buf + sizeof(h);
    DiagDev d{};
    d.dropped = h.dropped;
    d.accepted = h.accepted;
    d.flags = h.flags;
    if (hipMemcpy(st->dev.S_hi, p, 4 * n, hipMemcpyHostToDevice) ||
        hipMemcpy(st->dev.S_lo, p + 4 * n, 4 * n, hipMemcpyHostToDevice) ||
        hipMemcpy(st->dev.T, p + 8 * n, 8 * n, hipMemcpyHostToDevice) ||
        hipMemcpy(st->dev.N, p + 16 * n, 4 * n, hipMemcpyHostToDevice) ||
        hipMemcpy(st->dev.P, p + 20 * n, 4 * n, hipMemcpyHostToDevice) ||
        hipMemcpy(st->diag, &d, sizeof(d), hipMemcpyHostToDevice))
        return hip_fail(st);
    // frames may skip the clamp of a decayed state only while every S is in
    // [s_min, s_max] (S = hi + lo, as the kernels read it)
    bool in_range = true;
    for (size_t q = 0; q < n && in_range; ++q) {
        float hi, lo;
        std::memcpy(&hi, p + 4 * q, 4);
        std::memcpy(&lo, p + 4 * n + 4 * q, 4);
        const double s = (double)hi + (double)lo;
        in_range = s >= st->params.s_min && s <= st->params.s_max;
    }
    st->state_in_range = in_range;
    st->poisoned = false;
    return ESI_OK;
}

esi_status esi_get_diagnostics(esi_state* st, esi_diag* out)
{
    if (!st || !out)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(st->device);
    std::memset(out, 0, sizeof(*out));
    out->poisoned = st->poisoned ? 1u : 0u;
    out->calls = st->calls;
    if (st->poisoned)
        return ESI_OK;
    DiagDev d{};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&d, st->diag, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) {
        st->poisoned = true;
        out->poisoned = 1u;
        return ESI_ERR_HIP;
    }
    out->dropped = d.dropped;
    out->accepted = d.accepted;
    out->flags = d.flags;
    return ESI_OK;
}

esi_status esi_set_tile_pixels(esi_state* st, int32_t tile_pixels)
{
    if (!st || !(tile_pixels == 0 || tile_pixels == 256 || tile_pixels == 512 ||
                 tile_pixels == 1024 || tile_pixels == 2048))
        return ESI_ERR_INVALID_ARG;
    st->min_ppt = tile_pixels ? tile_pixels / 256 : 1;
    return ESI_OK;
}

esi_status esi_scratch_bound(int32_t width, int32_t height, size_t n_events, size_t* bytes)
{
    if (!bytes || width < 1 || height < 1 || width > kMaxSide || height > kMaxSide ||
        n_events >= ((size_t)1 << 31))
        return ESI_ERR_INVALID_ARG;
    // the most bucketing ranges any call gives one state: the resident
    // bucketing workgroups of the smallest tile table
    const int64_t npix = band_rows(width, height) * width;
    // the larger range count of the two bucketing kernels (more ranges, a
    // larger table)
    const Schedule sc = make_schedule(npix, (int64_t)n_events,
                                      std::max(bucket_slots(1), bucket_slots_batch(1)));
    const ScratchPlan p = scratch_plan(sc, (int64_t)n_events, 0);
    *bytes = n_events > 0 ? p.need + p.need / 4 : 0;  // with the growth margin of call_scratch
    return ESI_OK;
}

esi_status esi_set_scan_run(esi_state* st, int32_t scan_run)
{
    if (!st || scan_run < 0)
        return ESI_ERR_INVALID_ARG;
    st->scan_run = scan_run;
    return ESI_OK;
}

esi_status esi_set_chunk(esi_state* st, int32_t records)
{
    if (!st || !(records == 0 || records == 1536 || records == 2048))
        return ESI_ERR_INVALID_ARG;
    st->chunk = records;
    return ESI_OK;
}

esi_status esi_get_size(const esi_state* st, int32_t* width, int32_t* height)
{
    if (!st || !width || !height)
        return ESI_ERR_INVALID_ARG;
    *width = st->W;
    *height = st->H;
    return ESI_OK;
}

}  // extern "C"

// ---- batched calls ----------------------------------------------------------

namespace {

size_t batch_items_bytes(int32_t m) { return align_up(sizeof(BatchItem) * (size_t)m, 256); }
size_t batch_base_bytes(int32_t m) { return align_up(sizeof(uint32_t) * ((size_t)m + 1), 256); }
size_t batch_bytes(int32_t m) { return batch_items_bytes(m) + 3 * batch_base_bytes(m); }

void batch_free(esi_batch* b)
{
    if (b->tf_dev)
        (void)hipFree(b->tf_dev);
    if (b->tf_host)
        (void)hipHostFree(b->tf_host);
    if (b->copied)
        (void)hipEventDestroy(b->copied);
    if (b->used)
        (void)hipEventDestroy(b->used);
    if (b->dev)
        (void)hipFree(b->dev);
    if (b->host)
        (void)hipHostFree(b->host);
    delete b;
}

}  // namespace

extern "C" {

esi_status esi_batch_create(int32_t max_items, esi_batch** out)
{
    if (!out)
        return ESI_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_items < 1 || max_items > kMaxBatch)
        return ESI_ERR_INVALID_ARG;
    esi_batch* b = new (std::nothrow) esi_batch();
    if (!b)
        return ESI_ERR_OUT_OF_MEMORY;
    b->max_items = max_items;
    b->bytes = batch_bytes(max_items);
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return ESI_ERR_HIP;
    }
    if (hipHostMalloc(&b->host, b->bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&b->dev, b->bytes) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return ESI_ERR_OUT_OF_MEMORY;
    }
    if (hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess) {
        b->copied = nullptr;
        batch_free(b);
        return ESI_ERR_HIP;
    }
    if (hipEventCreateWithFlags(&b->used, hipEventDisableTiming) != hipSuccess) {
        b->used = nullptr;
        batch_free(b);
        return ESI_ERR_HIP;
    }
    *out = b;
    return ESI_OK;
}

esi_status esi_batch_destroy(esi_batch* b)
{
    if (!b)
        return ESI_ERR_INVALID_ARG;
    DeviceGuard g(b->device);
    esi_status rc = ESI_OK;
    // kernels of earlier calls may still read the device descriptors
    if (hipDeviceSynchronize() != hipSuccess)
        rc = ESI_ERR_HIP;
    batch_free(b);
    return rc;
}

esi_status esi_integrate_batch(esi_batch* b, int32_t n_items, esi_state* const* states,
                               const esi_events* events, const int64_t* const* t_frames,
                               const int32_t* n_frames, float* const* frames,
                               uint8_t* const* frames_u8, hipStream_t stream)
{
    if (!b || !states || !events || n_items < 1 || n_items > b->max_items)
        return ESI_ERR_INVALID_ARG;
    // every item checked as esi_integrate_window checks its arguments
    int64_t n_all = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        const esi_state* st = states[i];
        const esi_events& ev = events[i];
        const int32_t nf = n_frames ? n_frames[i] : 0;
        const int64_t* tf = t_frames ? t_frames[i] : nullptr;
        const float* fr = frames ? frames[i] : nullptr;
        const uint8_t* u8 = frames_u8 ? frames_u8[i] : nullptr;
        if (!st || st->device != b->device || nf < 0)
            return ESI_ERR_INVALID_ARG;
        if (ev.n > 0 && (!ev.x || !ev.y || !ev.t || !ev.p))
            return ESI_ERR_INVALID_ARG;
        if (ev.n >= ((size_t)1 << 31))
            return ESI_ERR_INVALID_ARG;
        if ((nf > 0) != (tf != nullptr) || (nf > 0 && !fr && !u8))
            return ESI_ERR_INVALID_ARG;
        // a sensor larger than one pass of the kernels is integrated in bands
        // by esi_integrate_window only
        if (st->npix > kMaxPixels)
            return ESI_ERR_INVALID_ARG;
        n_all += (int64_t)ev.n;
    }
    {
        // one state at most once: its items would race
        std::vector<const esi_state*> seen(states, states + n_items);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            return ESI_ERR_INVALID_ARG;
    }
    for (int32_t i = 0; i < n_items; ++i)
        if (states[i]->poisoned)
            return ESI_ERR_POISONED;
    Range range("esi_integrate_batch");
    DeviceGuard g(b->device);

    // schedules: the bucketing ranges shared out by event count
    std::vector<Schedule> sc(n_items);
    int kmax = 1;
    for (int32_t i = 0; i < n_items; ++i) {
        sc[i] = make_schedule(states[i]->npix, 0, 1, states[i]->min_ppt);
        if (events[i].n > 0)
            kmax = std::max(kmax, sc[i].ntiles);
    }
    const int slots = bucket_slots_batch(kmax);
    std::vector<BatchItem> it(n_items);
    std::vector<int> cls(n_items);  // integration class: tile size and decay kind
    for (int32_t i = 0; i < n_items; ++i) {
        esi_state* st = states[i];
        const int64_t n = (int64_t)events[i].n;
        const int share =
            n > 0 ? std::max(1, (int)((double)slots * (double)n / (double)n_all)) : 1;
        sc[i] = make_schedule(st->npix, n, share, st->min_ppt);
        BatchItem& x = it[i];
        x = BatchItem{};
        x.ev = EventsDev{events[i].x, events[i].y, events[i].t, events[i].p, n, 0, st->H};
        x.st = st->dev;
        x.mp = method_params(st->params);
        x.mp.scan_run = effective_scan_run(st->scan_run, sc[i].ppt);
        if (!st->state_in_range)
            x.mp.need_clamp = 1;
        const int32_t nf = n_frames ? n_frames[i] : 0;
        x.fo = FrameOut{nf > 0 ? t_frames[i] : nullptr, nf,
                        (nf > 0 && frames) ? frames[i] : nullptr,
                        (nf > 0 && frames_u8) ? frames_u8[i] : nullptr, st->npix};
        x.diag = st->diag;
        x.tile_log = sc[i].tile_log;
        x.K = sc[i].ntiles;
        if (n > 0) {
            const esi_status rc = call_scratch(st, sc[i], n, 0, stream, x.cs, nullptr);
            if (rc != ESI_OK)
                return rc;
            x.E = sc[i].unit_events;
            x.B = sc[i].nunits;
            x.B_pad = (x.B + 7) / 8 * 8;
            x.nseg = (int)scan_segments(x.B);
            x.cols = (x.K + 255) / 256;
        }
        // integration class: tile size, scan compiled in or not, chunk form,
        // decay kind
        const int big = (st->chunk == 2048 && sc[i].ppt == 2) ? 1 : 0;
        cls[i] = ((sc[i].ppt * 2 + (x.mp.scan_run != kScanOff ? 1 : 0)) * 2 + big) * 8 +
                 decay_kind(x.mp);
    }
    // items ordered by class, so that each integration launch covers a range
    std::vector<int> order(n_items);
    for (int32_t i = 0; i < n_items; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cls[a] < cls[c]; });

    // the previous call's staging copy must have been read before reuse
    const bool earlier = b->pending;
    if (earlier && hipEventSynchronize(b->copied) != hipSuccess)
        return ESI_ERR_HIP;
    // frame times in host memory: packed into the batch's own staging and
    // copied with the descriptors
    size_t tf_bytes = 0;
    std::vector<size_t> tf_off(n_items, SIZE_MAX);
    for (int32_t i = 0; i < n_items; ++i)
        if (it[i].fo.nf > 0 && !device_accessible(it[i].fo.t_frames)) {
            tf_off[i] = tf_bytes;
            tf_bytes += align_up(8 * (size_t)it[i].fo.nf, 64);
        }
    if (tf_bytes > b->tf_cap) {
        // earlier calls' kernels may still read the device copy
        if (earlier && hipEventSynchronize(b->used) != hipSuccess)
            return ESI_ERR_HIP;
        if (b->tf_dev)
            (void)hipFree(b->tf_dev);
        if (b->tf_host)
            (void)hipHostFree(b->tf_host);
        b->tf_dev = b->tf_host = nullptr;
        b->tf_cap = 0;
        const size_t cap = tf_bytes + tf_bytes / 4;
        if (hipHostMalloc(&b->tf_host, cap, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&b->tf_dev, cap) != hipSuccess) {
            (void)hipGetLastError();
            return ESI_ERR_OUT_OF_MEMORY;
        }
        b->tf_cap = cap;
    }
    for (int32_t i = 0; i < n_items; ++i)
        if (tf_off[i] != SIZE_MAX) {
            std::memcpy((char*)b->tf_host + tf_off[i], it[i].fo.t_frames, 8 * (size_t)it[i].fo.nf);
            it[i].fo.t_frames = (const int64_t*)((char*)b->tf_dev + tf_off[i]);
        }
    char* h = (char*)b->host;
    BatchItem* hi = (BatchItem*)h;
    uint32_t* ub = (uint32_t*)(h + batch_items_bytes(b->max_items));
    uint32_t* sb = (uint32_t*)((char*)ub + batch_base_bytes(b->max_items));
    uint32_t* tb = (uint32_t*)((char*)sb + batch_base_bytes(b->max_items));
    ub[0] = sb[0] = tb[0] = 0;
    for (int32_t k = 0; k < n_items; ++k) {
        const BatchItem& x = it[order[k]];
        hi[k] = x;
        ub[k + 1] = ub[k] + (uint32_t)x.B_pad;
        sb[k + 1] = sb[k] + (uint32_t)(x.cols * x.nseg);
        tb[k + 1] = tb[k] + (uint32_t)x.K;
    }
    const char* d = (const char*)b->dev;
    BatchDev bd{};
    bd.items = (const BatchItem*)d;
    bd.unit_base = (const uint32_t*)(d + ((char*)ub - h));
    bd.seg_base = (const uint32_t*)(d + ((char*)sb - h));
    bd.tile_base = (const uint32_t*)(d + ((char*)tb - h));
    bd.n = n_items;
    auto fail = [&]() {
        for (int32_t i = 0; i < n_items; ++i)
            states[i]->poisoned = true;
        return ESI_ERR_HIP;
    };
    // the previous call's kernels (possibly on another stream) read the
    // device descriptors until they finish
    if ((earlier && hipStreamWaitEvent(stream, b->used, 0) != hipSuccess) ||
        hipMemcpyAsync(b->dev, b->host, b->bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        (tf_bytes > 0 && hipMemcpyAsync(b->tf_dev, b->tf_host, tf_bytes, hipMemcpyHostToDevice,
                                        stream) != hipSuccess) ||
        hipEventRecord(b->copied, stream) != hipSuccess)
        return fail();
    b->pending = true;
    if (n_all > 0) {
        Range phase("bucketing");
        if (launch_bucket_batch(bd, ub[n_items], sb[n_items], kmax, stream) != hipSuccess)
            return fail();
    }
    Range phase("integration");
    for (int32_t k0 = 0; k0 < n_items;) {
        int32_t k1 = k0 + 1;
        while (k1 < n_items && cls[order[k1]] == cls[order[k0]])
            ++k1;
        const int c = cls[order[k0]];
        if (launch_integrate_batch(bd, k0, k1, tb[k0], tb[k1] - tb[k0], c / 32, c % 8,
                                   (c / 16) % 2 == 1, (c / 8) % 2 == 1, stream) !=
            hipSuccess)
            return fail();
        k0 = k1;
    }
    if (hipEventRecord(b->used, stream) != hipSuccess)
        return fail();
    for (int32_t i = 0; i < n_items; ++i)
        states[i]->calls++;
    return ESI_OK;
}

}  // extern "C"

