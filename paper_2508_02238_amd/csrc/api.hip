// api.hip -- the C ABI declared in include/esi.h: argument checks, state and
// scratch ownership, the per-call schedule, and stream-ordered launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "esi.h"
#include "esi_internal.hpp"

using namespace esi;

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
    int bucket_slots = 1024;  // bucketing workgroups resident at once
    bool state_in_range = true;  // every S in [s_min, s_max] (false after importing one outside)
    bool poisoned = false;
    uint64_t calls = 0;
    // profiling: HIP events around the two phases of recorded calls
    bool profiling = false;
    uint32_t prof_calls = 0;
    hipEvent_t* prof_ev = nullptr;  // [kProfMax][3]
};

namespace {

constexpr uint64_t kMagic = 0x3130495345ull;  // "ESI01"
constexpr uint32_t kProfMax = 1024;
constexpr int64_t kMaxPixels = (int64_t)kMaxTiles * 256 * 8;  // 4096000

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
Schedule make_schedule(int64_t npix, int64_t n, int slots)
{
    Schedule s{};
    for (int ppt = 1; ppt <= 8; ppt *= 2) {
        s.ppt = ppt;
        s.tile_log = 8 + (ppt == 1 ? 0 : ppt == 2 ? 1 : ppt == 4 ? 2 : 3);
        s.ntiles = (int)((npix + (256 * ppt) - 1) / (256 * ppt));
        if (s.ntiles <= kMaxTiles)
            break;
    }
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
    }
    return "ESI_ERR_UNKNOWN";
}

esi_status esi_create_state(int32_t width, int32_t height, const esi_params* params,
                            hipStream_t stream, esi_state** out)
{
    if (!out)
        return ESI_ERR_INVALID_ARG;
    *out = nullptr;
    if (width < 1 || height < 1 || width > 65535 || height > 65535 || !params_ok(params))
        return ESI_ERR_INVALID_ARG;
    const int64_t npix = (int64_t)width * height;
    if (npix > kMaxPixels)
        return ESI_ERR_INVALID_ARG;
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
    st->bucket_slots = bucket_slots(make_schedule(npix, 0, 1).ntiles);
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

esi_status esi_integrate_window(esi_state* st, const esi_events* ev, const int64_t* t_frames,
                                int32_t n_frames, float* frames, uint8_t* frames_u8,
                                hipStream_t stream)
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
    DeviceGuard g(st->device);
    const int64_t n = (int64_t)ev->n;
    MethodParams mp = method_params(st->params);
    if (!st->state_in_range)
        mp.need_clamp = 1;
    const Schedule sc = make_schedule(st->npix, n, st->bucket_slots);
    EventsDev evd{ev->x, ev->y, ev->t, ev->p, n};
    CallScratch cs{};
    if (n > 0) {
        const int64_t M = (int64_t)sc.ntiles * sc.nunits;
        const int64_t nseg = (int64_t)scan_segments(sc.nunits);
        const size_t o_bs = align_up(4 * (size_t)M, 256);
        const size_t o_tt = o_bs + align_up(4 * (size_t)(nseg * sc.ntiles), 256);
        const size_t o_tot = o_tt + align_up(4 * (size_t)sc.ntiles, 256);
        const size_t o_rec = o_tot + 256;
        const size_t need = o_rec + 8 * (size_t)n;
        if (need > st->scratch_bytes) {
            // the old scratch may still be read by work queued on this stream
            if (hipStreamSynchronize(stream) != hipSuccess)
                return hip_fail(st);
            if (st->scratch)
                (void)hipFree(st->scratch);
            st->scratch = nullptr;
            st->scratch_bytes = 0;
            const size_t bytes = need + need / 4;
            if (hipMalloc(&st->scratch, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return ESI_ERR_OUT_OF_MEMORY;
            }
            st->scratch_bytes = bytes;
        }
        char* base = (char*)st->scratch;
        cs.table = (uint32_t*)base;
        cs.blocksum = (uint32_t*)(base + o_bs);
        cs.tile_tot = (uint32_t*)(base + o_tt);
        cs.total = (uint32_t*)(base + o_tot);
        cs.records = (uint64_t*)(base + o_rec);
    }
    hipEvent_t* pe = nullptr;
    if (st->profiling && st->prof_calls < kProfMax) {
        pe = st->prof_ev + 3 * st->prof_calls++;
        if (hipEventRecord(pe[0], stream) != hipSuccess)
            return hip_fail(st);
    }
    if (n > 0 && launch_bucket(evd, st->dev, sc, cs, st->diag, stream) != hipSuccess)
        return hip_fail(st);
    if (pe && hipEventRecord(pe[1], stream) != hipSuccess)
        return hip_fail(st);
    if (n > 0 || n_frames > 0) {
        if (launch_integrate(evd, st->dev, sc, cs, mp, t_frames, n_frames, frames, frames_u8,
                             st->diag, stream) != hipSuccess)
            return hip_fail(st);
    }
    if (pe && hipEventRecord(pe[2], stream) != hipSuccess)
        return hip_fail(st);
    st->calls++;
    return ESI_OK;
}

esi_status esi_snapshot_frame(esi_state* st, int64_t t_frame_us, float* frame, uint8_t* u8,
                              hipStream_t stream)
{
    if (!st || (!frame && !u8))
        return ESI_ERR_INVALID_ARG;
    if (st->poisoned)
        return ESI_ERR_POISONED;
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

esi_status esi_get_size(const esi_state* st, int32_t* width, int32_t* height)
{
    if (!st || !width || !height)
        return ESI_ERR_INVALID_ARG;
    *width = st->W;
    *height = st->H;
    return ESI_OK;
}

}  // extern "C"
