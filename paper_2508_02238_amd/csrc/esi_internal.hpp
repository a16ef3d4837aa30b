// esi_internal.hpp -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esi_device.hpp"

namespace esi {

// How one integrate call is split into work.
//   tile   = 256 * ppt consecutive pixels (row-major q), one workgroup each in
//            the integration kernel;
//   unit   = 2^unit_log consecutive events, one workgroup each when bucketing.
struct Schedule {
    int ppt;          // pixels per thread in the integration kernel: 1, 2, 4, 8
    int tile_log;     // log2(256 * ppt)
    int ntiles;       // K = ceil(P / tile)
    int unit_log;     // log2(events per unit)
    int64_t nunits;   // B = ceil(n / unit)
    int chunk;        // records staged in LDS at a time by the integration kernel
};

constexpr int kMaxTiles = 2000;               // bucketing LDS (staging + tables) fits in 64 KB
constexpr int kUnitLog = 12;                  // events per bucketing unit (workgroup): 4096
constexpr int kChunk = 1792;

struct DiagDev {
    unsigned long long dropped;
    unsigned long long accepted;
    unsigned int flags;
    unsigned int pad;
};

// Scratch of one integrate call (device).
struct CallScratch {
    uint32_t* table;      // [B][K]: counts, then exclusive offsets in (tile, unit) order
    uint32_t* blocksum;   // [nseg][K]: per-segment sums, then offsets
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

// Units per segment of the column-wise table scan (at most 64 segments).
int scan_segment_units(int64_t B);
// LDS bytes of the bucketing kernel for K tiles.
size_t bucket_lds_bytes(int K);

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
