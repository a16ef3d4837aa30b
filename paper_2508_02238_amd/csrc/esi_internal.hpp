// esi_internal.hpp -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esi_device.hpp"

namespace esi {

// How one integrate call is split into work.
//   tile   = 256 * ppt consecutive pixels (row-major q), one workgroup each in
//            the integration kernel;
//   unit   = unit_events consecutive events (a multiple of 256), one
//            workgroup each when bucketing.
struct Schedule {
    int ppt;              // pixels per thread in the integration kernel: 1, 2, 4, 8
    int tile_log;         // log2(256 * ppt)
    int ntiles;           // K = ceil(P / tile)
    int64_t unit_events;  // E
    int64_t nunits;       // B = ceil(n / E)
    // the integration launch takes the tiles largest first (more tiles than
    // the GPU holds integration workgroups at once)
    bool ordered;
    // two pixels per thread: 2048-record chunks at three workgroups per CU
    bool big_chunk;
};

constexpr int kMaxTiles = 2000;  // bucketing LDS (staging + counters) stays near 32 KB

struct DiagDev {
    unsigned long long dropped;
    unsigned long long accepted;
    unsigned int flags;
    unsigned int pad;
};

// Scratch of one integrate call (device).
struct CallScratch {
    uint32_t* table;      // [B][K]: counts, then exclusive offsets in (tile, unit) order
    uint32_t* blocksum;   // [nseg][K]: per-segment sums
    uint32_t* tile_tot;   // [K]: events per tile
    uint32_t* total;      // [1]: number of accepted events
    uint64_t* records;    // [n + 1]: the last a spare slot
    uint32_t* order;      // [K]: tiles by size class of their event count, largest first
};

// Events of one call.  A sensor larger than one pass of the kernels holds is
// integrated in bands of rows: a pass takes the events with y in
// [y0, y0 + H) of the band's state (H = StateDev::H), passes over the other
// rows' events, and counts an event as dropped (x >= W or y >= H_all) only in
// the pass with y0 = 0.
struct EventsDev {
    const uint16_t* x;
    const uint16_t* y;
    const int64_t* t;
    const int8_t* p;
    int64_t n;
    int y0;     // first row of the pass
    int H_all;  // rows of the sensor
};

struct StateDev {
    float* S_hi;
    float* S_lo;
    int64_t* T;
    uint32_t* N;
    int32_t* P;
    int W, H;
    int64_t npix;
};

// Frames of one call: times (device), count, FP32 and 8-bit outputs (either
// may be null; they point at the pass's first pixel), and the pixels from
// one frame to the next (the whole sensor's W * H).
struct FrameOut {
    const int64_t* t_frames;
    int nf;
    float* frames;
    uint8_t* frames_u8;
    int64_t stride;
};

// One stream of a batched call: everything its kernels read, in device
// memory.  Work of one batched launch is laid out stream by stream; a
// stream's first work index in each launch is in the base arrays below.
struct BatchItem {
    EventsDev ev;
    StateDev st;
    MethodParams mp;
    FrameOut fo;
    CallScratch cs;  // null pointers when the stream has no events
    DiagDev* diag;
    int tile_log, K;  // tile size, tiles
    int nseg, cols;   // table scan: segments x columns of 256 tiles
    int64_t E, B;     // events per bucketing range, ranges
    int64_t B_pad;    // ranges rounded up to a multiple of the XCD count
};

struct BatchDev {
    const BatchItem* items;
    const uint32_t* unit_base;  // [n + 1]: bucketing ranges (padded), stream by stream
    const uint32_t* seg_base;   // [n + 1]: table-scan workgroups
    const uint32_t* tile_base;  // [n + 1]: tiles
    int n;
};

// Bucketing workgroups the current device holds at once for K tiles: of a
// single-stream call (k_bucket; its wide form from K tiles on, bucket_wide)
// and of a batched call (kb_bucket).
bool bucket_wide(int K);
int bucket_slots(int K);
int bucket_slots_batch(int K);
// integration workgroups of `ppt` pixels per thread resident at once (big:
// the 2048-record chunks of two pixels per thread)
int integrate_slots(int ppt, bool big = false);
// Segments of the column-wise table scan for B units.
size_t scan_segments(int64_t B);

// Kernel launchers (asynchronous on `stream`; return the launch error).
hipError_t launch_bucket(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                         const CallScratch& cs, DiagDev* diag, hipStream_t stream);
hipError_t launch_integrate(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                            const CallScratch& cs, const MethodParams& mp, const FrameOut& fo,
                            DiagDev* diag, hipStream_t stream);
hipError_t launch_snapshot(const StateDev& st, const MethodParams& mp, int64_t t_f, float* frame,
                           uint8_t* u8, hipStream_t stream);
hipError_t launch_reset(const StateDev& st, int64_t t0, DiagDev* diag, hipStream_t stream);

// Batched launches over items [i0, i1) of `b` (the integration launch covers
// items of one tile size and decay kind; kmax = largest K among them).
hipError_t launch_bucket_batch(const BatchDev& b, uint32_t units, uint32_t seg_blocks, int kmax,
                               hipStream_t stream);
// (scan: the launch's items have phase A's scan on; big: their tiles of two
// pixels per thread take 2048-record chunks)
hipError_t launch_integrate_batch(const BatchDev& b, int i0, int i1, uint32_t tile0,
                                  uint32_t tiles, int ppt, int bk, bool scan, bool big,
                                  hipStream_t stream);
int decay_kind(const MethodParams& mp);

}  // namespace esi
