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
    uint64_t* records;    // [n]
};

struct EventsDev {
    const uint16_t* x;
    const uint16_t* y;
    const int64_t* t;
    const int8_t* p;
    int64_t n;
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

// Bucketing workgroups the current device holds at once for K tiles.
int bucket_slots(int K);
// Segments of the column-wise table scan for B units.
size_t scan_segments(int64_t B);

// Kernel launchers (asynchronous on `stream`; return the launch error).
hipError_t launch_bucket(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                         const CallScratch& cs, DiagDev* diag, hipStream_t stream);
hipError_t launch_integrate(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                            const CallScratch& cs, const MethodParams& mp,
                            const int64_t* t_frames, int nf, float* frames, uint8_t* frames_u8,
                            DiagDev* diag, hipStream_t stream);
hipError_t launch_snapshot(const StateDev& st, const MethodParams& mp, int64_t t_f, float* frame,
                           uint8_t* u8, hipStream_t stream);
hipError_t launch_reset(const StateDev& st, int64_t t0, DiagDev* diag, hipStream_t stream);

}  // namespace esi
