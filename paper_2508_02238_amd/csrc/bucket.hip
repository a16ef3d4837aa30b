// bucket.hip -- stable bucketing of a time-sorted event stream by pixel tile.
//
// Alg. 2 walks the events in array order and touches only the event's own
// pixel, so the order that matters is the order of the events of each pixel.
// These kernels regroup the events tile-major (a tile = a range of
// consecutive pixels) while keeping array order inside every tile (and so
// inside every pixel): a counting sort whose ranks are stable.
//
//   k_hist      one wave per unit of 2^unit_log consecutive events: per-tile
//               counts of the unit's valid events -> table[unit][tile];
//               out-of-range events are counted as dropped.
//   k_seg_sum,  exclusive scan of the table in (tile, unit) order, done
//   k_seg_scan, column-wise so every access is a coalesced row access:
//   k_seg_down  per-tile sums over segments of units, a scan over segments
//               and tiles, then a rescan of each segment writing offsets.
//   k_scatter   one wave per unit again: walks its events 64 at a time in
//               order (8 steps loaded ahead), ranks each event stably among
//               the same-tile events of the unit, writes a 64-bit record
//               (time offset, pixel in tile, polarity) to its slot.  Also
//               flags decreasing times and calls whose span the record cannot
//               hold.
//
// Workgroups are dispatched round-robin over the 8 XCDs; units are assigned
// so that the workgroups of one XCD take consecutive units.  Consecutive
// units write adjacent pieces of every tile bucket, so a cache line of a
// bucket is completed inside one XCD's L2 before it is written back.
#include <hip/hip_runtime.h>

#include "esi_internal.hpp"

namespace esi {
namespace {

constexpr int kXcds = 8;
constexpr int kBatch = 8;  // scatter: steps of 64 events loaded ahead

// Bijection blockIdx -> work index that gives each XCD a contiguous range.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t x = b % kXcds, i = b / kXcds;
    const int64_t q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ bool valid_q(uint32_t x, uint32_t y, int W, int H, uint32_t& q)
{
    q = y * (uint32_t)W + x;
    return x < (uint32_t)W && y < (uint32_t)H;
}

__global__ __launch_bounds__(kBlock) void k_hist(EventsDev ev, int W, int H, int tile_log, int K,
                                                 int unit_log, int64_t B, uint32_t* table,
                                                 DiagDev* diag)
{
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t unit = blk * kWavesPerBlock + wave;
    uint32_t* h = lds + wave * K;
    for (int k = lane; k < K; k += kWave)
        h[k] = 0;
    __syncthreads();
    uint32_t drop = 0;
    if (unit < B) {
        const int64_t lo = unit << unit_log;
        const int64_t hi = min(lo + ((int64_t)1 << unit_log), ev.n);
        const bool vec = (((uintptr_t)ev.x | (uintptr_t)ev.y) & 15u) == 0;
        int64_t i = lo;
        if (vec) {
            // 8 events per lane per step: 16-byte loads of x and y
            for (; i + 8 * kWave <= hi; i += 8 * kWave) {
                const int64_t e = i + 8 * lane;
                const uint4 xv = *(const uint4*)(ev.x + e);
                const uint4 yv = *(const uint4*)(ev.y + e);
                const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
                const uint32_t ys[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    uint32_t q;
                    if (valid_q(xs[m] & 0xFFFFu, ys[m] & 0xFFFFu, W, H, q))
                        atomicAdd(&h[q >> tile_log], 1u);
                    else
                        ++drop;
                    if (valid_q(xs[m] >> 16, ys[m] >> 16, W, H, q))
                        atomicAdd(&h[q >> tile_log], 1u);
                    else
                        ++drop;
                }
            }
        }
        for (int64_t e = i + lane; e < hi; e += kWave) {
            uint32_t q;
            if (valid_q(ev.x[e], ev.y[e], W, H, q))
                atomicAdd(&h[q >> tile_log], 1u);
            else
                ++drop;
        }
    }
    __syncthreads();
    if (unit < B) {
        uint32_t* row = table + unit * K;
        for (int k = lane; k < K; k += kWave)
            row[k] = h[k];
    }
    if (drop)
        atomicAdd(&diag->dropped, (unsigned long long)drop);
}

// ---- exclusive scan of table[u][k] in (k, u) order, column-wise -------------
// Segments of `seg` units.  segsum[s][k] = sum over the units of segment s.

__global__ __launch_bounds__(kBlock) void k_seg_sum(const uint32_t* table, int K, int64_t B,
                                                    int seg, uint32_t* segsum)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= K)
        return;
    const int64_t u0 = (int64_t)s * seg, u1 = min(u0 + seg, B);
    uint32_t sum = 0;
    for (int64_t u = u0; u < u1; ++u)
        sum += table[u * K + k];
    segsum[(int64_t)s * K + k] = sum;
}

// One workgroup: per tile, exclusive scan over segments; then the exclusive
// scan of tile totals gives each tile's start.  segsum[s][k] becomes the
// offset of (segment s, tile k) in the whole (tile, unit) order.  Each thread
// owns up to 4 consecutive tiles (K <= 4096).
__global__ __launch_bounds__(1024) void k_seg_scan(uint32_t* segsum, int K, int nseg,
                                                   uint32_t* total, DiagDev* diag)
{
    __shared__ uint32_t sw[1024 / kWave];
    const int per = (K + 1023) / 1024;
    const int k0 = threadIdx.x * per;
    uint32_t tot[4] = {0u, 0u, 0u, 0u};
    uint32_t mine = 0;
    for (int kk = 0; kk < per && kk < 4; ++kk) {
        const int k = k0 + kk;
        if (k >= K)
            break;
        uint32_t run = 0;
        for (int s = 0; s < nseg; ++s) {
            const uint32_t v = segsum[(int64_t)s * K + k];
            segsum[(int64_t)s * K + k] = run;
            run += v;
        }
        tot[kk] = run;
        mine += run;
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    uint32_t inc = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = (uint32_t)__shfl_up((int)inc, o);
        if (lane >= o)
            inc += n;
    }
    if (lane == kWave - 1)
        sw[wave] = inc;
    __syncthreads();
    uint32_t base = inc - mine, all = 0;
    for (int w = 0; w < 1024 / kWave; ++w) {
        base += (w < wave) ? sw[w] : 0u;
        all += sw[w];
    }
    for (int kk = 0; kk < per && kk < 4; ++kk) {
        const int k = k0 + kk;
        if (k >= K)
            break;
        for (int s = 0; s < nseg; ++s)
            segsum[(int64_t)s * K + k] += base;
        base += tot[kk];
    }
    if (threadIdx.x == 0) {
        *total = all;
        atomicAdd(&diag->accepted, (unsigned long long)all);
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_down(uint32_t* table, int K, int64_t B, int seg,
                                                     const uint32_t* segsum)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= K)
        return;
    const int64_t u0 = (int64_t)s * seg, u1 = min(u0 + seg, B);
    uint32_t run = segsum[(int64_t)s * K + k];
    for (int64_t u = u0; u < u1; ++u) {
        const uint32_t c = table[u * K + k];
        table[u * K + k] = run;
        run += c;
    }
}

// ---- stable scatter ----------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_scatter(EventsDev ev, int W, int H, int tile_log,
                                                    int K, int unit_log, int64_t B,
                                                    const uint32_t* table, uint64_t* records,
                                                    int64_t cap, DiagDev* diag)
{
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t unit = blk * kWavesPerBlock + wave;
    uint32_t* base = lds + wave * K;
    if (unit < B) {
        const uint32_t* row = table + unit * K;
        for (int k = lane; k < K; k += kWave)
            base[k] = row[k];
    }
    __syncthreads();
    if (unit >= B)
        return;  // whole wave leaves together

    const uint32_t tmask = (1u << tile_log) - 1u;
    const int kbits = key_bits_for((uint32_t)K);
    const int64_t t_ref = ev.t[0];
    const int64_t lo = unit << unit_log;
    const int64_t hi = min(lo + ((int64_t)1 << unit_log), ev.n);
    int64_t t_carry = (lo > 0) ? ev.t[lo - 1] : INT64_MIN;
    uint32_t flags = 0;
    for (int64_t b0 = lo; b0 < hi; b0 += kBatch * kWave) {
        uint32_t xs[kBatch], ys[kBatch];
        int64_t ts[kBatch];
        int ps[kBatch];
#pragma unroll
        for (int s = 0; s < kBatch; ++s) {
            // clamped index, no select on the loaded values: all loads of the
            // batch stay in flight together
            const int64_t i = min(b0 + s * kWave + lane, hi - 1);
            xs[s] = ev.x[i];
            ys[s] = ev.y[i];
            ts[s] = ev.t[i];
            ps[s] = ev.p[i];
        }
#pragma unroll
        for (int s = 0; s < kBatch; ++s) {
            const int64_t i = b0 + s * kWave + lane;
            const bool in = i < hi;
            uint32_t q;
            const bool ok = in && valid_q(xs[s], ys[s], W, H, q);
            const int64_t t = ts[s];
            // decreasing time versus the previous event in array order
            int64_t tprev = __shfl_up(t, 1);
            if (lane == 0)
                tprev = t_carry;
            if (in && t < tprev)
                flags |= 1u;  // ESI_DIAG_UNSORTED
            t_carry = __shfl(t, kWave - 1);
            const int64_t dt = t - t_ref;
            if (ok && (dt >= kMaxSpan || dt <= -kMaxSpan))
                flags |= 4u;  // ESI_DIAG_TIME_RANGE
            const uint32_t key = ok ? (q >> tile_log) : 0u;
            const uint32_t slot = wave_stable_rank(ok, key, kbits, base);
            if (ok) {
                if ((int64_t)slot < cap)
                    records[slot] = pack_record(dt, q & tmask, ps[s] > 0);
                else
                    flags |= 8u;  // ESI_DIAG_INTERNAL: never expected
            }
        }
    }
    // one atomic per wave with any flag
    if (__ballot(flags != 0)) {
        uint32_t f = flags;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            f |= (uint32_t)__shfl_xor((int)f, o);
        if (lane == 0)
            atomicOr(&diag->flags, f);
    }
}

}  // namespace

int scan_segment_units(int64_t B)
{
    int64_t seg = 64;
    while ((B + seg - 1) / seg > 64)
        seg *= 2;
    return (int)seg;
}

hipError_t launch_bucket(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                         const CallScratch& cs, DiagDev* diag, hipStream_t stream)
{
    const int K = sc.ntiles;
    const int64_t B = sc.nunits;
    const unsigned blocks_units = (unsigned)((B + kWavesPerBlock - 1) / kWavesPerBlock);
    const size_t lds_hist = sizeof(uint32_t) * kWavesPerBlock * K;
    hipLaunchKernelGGL(k_hist, dim3(blocks_units), dim3(kBlock), lds_hist, stream, ev, st.W, st.H,
                       sc.tile_log, K, sc.unit_log, B, cs.table, diag);
    const int seg = scan_segment_units(B);
    const int nseg = (int)((B + seg - 1) / seg);
    const dim3 grid((unsigned)((K + kBlock - 1) / kBlock), (unsigned)nseg);
    hipLaunchKernelGGL(k_seg_sum, grid, dim3(kBlock), 0, stream, cs.table, K, B, seg, cs.blocksum);
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, stream, cs.blocksum, K, nseg, cs.total,
                       diag);
    hipLaunchKernelGGL(k_seg_down, grid, dim3(kBlock), 0, stream, cs.table, K, B, seg,
                       cs.blocksum);
    const size_t lds_scatter = sizeof(uint32_t) * kWavesPerBlock * K;
    hipLaunchKernelGGL(k_scatter, dim3(blocks_units), dim3(kBlock), lds_scatter, stream, ev, st.W,
                       st.H, sc.tile_log, K, sc.unit_log, B, cs.table, cs.records, ev.n, diag);
    return hipGetLastError();
}

}  // namespace esi
