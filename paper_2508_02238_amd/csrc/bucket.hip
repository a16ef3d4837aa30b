// bucket.hip -- stable bucketing of a time-sorted event stream by pixel tile.
//
// Alg. 2 walks the events in array order and touches only the event's own
// pixel, so the order that matters is the order of the events of each pixel.
// These kernels regroup the events tile-major (a tile = a range of
// consecutive pixels) while keeping array order inside every tile (and so
// inside every pixel): a counting sort whose ranks are stable.
//
//   k_hist      one workgroup per unit of 2^unit_log consecutive events:
//               per-tile counts of the unit's valid events -> table[unit][tile];
//               out-of-range events are counted as dropped.
//   k_seg_sum,  exclusive scan of the table in (tile, unit) order, done
//   k_seg_scan, column-wise so every access is a coalesced row access:
//   k_seg_down  per-tile sums over segments of units, a scan over segments
//               and tiles, then a rescan of each segment writing offsets.
//   k_bucket    one workgroup per unit again: each wave ranks its quarter of
//               the unit stably by tile (wave-wide key match), a scan over
//               (tile, wave) gives every event its place in the unit sorted
//               by tile, the 64-bit records (time offset, pixel in tile,
//               polarity) are staged in LDS in that order, and each tile's run
//               is then written to its bucket in one burst.  Also flags
//               decreasing times and calls whose span the record cannot hold.
//
// Workgroups are dispatched round-robin over the 8 XCDs; units are assigned
// so that the workgroups of one XCD take consecutive units.  Consecutive
// units write adjacent runs of every tile bucket within a short time, so the
// cache lines of a bucket are completed in one XCD's L2 before they are
// written back (scattered 8-byte stores spread over the whole kernel would
// reach HBM as partial lines).
#include <hip/hip_runtime.h>

#include "esi_internal.hpp"

namespace esi {
namespace {

constexpr int kXcds = 8;

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
    extern __shared__ uint32_t h[];
    const int64_t unit = xcd_block(blockIdx.x, gridDim.x);
    for (int k = threadIdx.x; k < K; k += kBlock)
        h[k] = 0;
    __syncthreads();
    uint32_t drop = 0;
    const int64_t lo = unit << unit_log;
    const int64_t hi = min(lo + ((int64_t)1 << unit_log), ev.n);
    const bool vec = (((uintptr_t)ev.x | (uintptr_t)ev.y) & 15u) == 0;
    int64_t i = lo;
    if (vec) {
        // 8 events per thread per step: 16-byte loads of x and y
        for (; i + 8 * kBlock <= hi; i += 8 * kBlock) {
            const int64_t e = i + 8 * threadIdx.x;
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
    for (int64_t e = i + threadIdx.x; e < hi; e += kBlock) {
        uint32_t q;
        if (valid_q(ev.x[e], ev.y[e], W, H, q))
            atomicAdd(&h[q >> tile_log], 1u);
        else
            ++drop;
    }
    __syncthreads();
    uint32_t* row = table + unit * K;
    for (int k = threadIdx.x; k < K; k += kBlock)
        row[k] = h[k];
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

// ---- stable bucketing, staged in LDS ------------------------------------------

template <int UNIT_LOG>
__global__ __launch_bounds__(kBlock) void k_bucket(EventsDev ev, int W, int H, int tile_log,
                                                   int K, int64_t B, const uint32_t* table,
                                                   uint64_t* records, int64_t cap, DiagDev* diag)
{
    constexpr int U = 1 << UNIT_LOG;              // events per unit (workgroup)
    constexpr int PER_WAVE = U / kWavesPerBlock;  // events per wave
    constexpr int STEPS = PER_WAVE / kWave;       // steps of 64 per wave
    constexpr int BATCH = 8;                      // steps loaded ahead
    static_assert(STEPS % BATCH == 0, "unit size");
    extern __shared__ uint64_t smem[];
    uint64_t* staged = smem;                                   // [U]
    uint32_t* gbase = (uint32_t*)(staged + U);                 // [K] bucket offset of this unit
    uint16_t* cw = (uint16_t*)(gbase + K);                     // [4][K] per-wave counters
    uint16_t* skey = cw + kWavesPerBlock * K;                  // [U] tile of each staged record

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int64_t unit = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t* row = table + unit * K;
    for (int k = tid; k < K; k += kBlock)
        gbase[k] = row[k];
    for (int k = tid; k < kWavesPerBlock * K; k += kBlock)
        cw[k] = 0;
    __syncthreads();

    const uint32_t tmask = (1u << tile_log) - 1u;
    const int kbits = key_bits_for((uint32_t)K);
    const int64_t t_ref = ev.t[0];
    const int64_t lo = (unit << UNIT_LOG) + (int64_t)wave * PER_WAVE;
    const int64_t hi = min((unit << UNIT_LOG) + U, ev.n);
    int64_t t_carry = (lo > 0 && lo - 1 < ev.n) ? ev.t[lo - 1] : INT64_MIN;
    uint32_t flags = 0;
    uint64_t recs[STEPS];
    uint32_t packed[STEPS];  // rank | tile << 16, or ~0 for no event
    uint16_t* mycw = cw + wave * K;
#pragma unroll
    for (int b0 = 0; b0 < STEPS; b0 += BATCH) {
        uint32_t xs[BATCH], ys[BATCH];
        int64_t ts[BATCH];
        int ps[BATCH];
#pragma unroll
        for (int s = 0; s < BATCH; ++s) {
            // clamped index, no select on the loaded values: all loads of the
            // batch stay in flight together
            const int64_t i = max(min(lo + (b0 + s) * kWave + lane, hi - 1), (int64_t)0);
            xs[s] = ev.x[i];
            ys[s] = ev.y[i];
            ts[s] = ev.t[i];
            ps[s] = ev.p[i];
        }
#pragma unroll
        for (int s = 0; s < BATCH; ++s) {
            const int64_t i = lo + (b0 + s) * kWave + lane;
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
            const uint32_t rank = wave_stable_rank(ok, key, kbits, mycw);
            packed[b0 + s] = ok ? (rank | (key << 16)) : 0xFFFFFFFFu;
            recs[b0 + s] = pack_record(dt, q & tmask, ps[s] > 0);
        }
    }
    __syncthreads();

    // exclusive scan over (tile, wave), tile-major: start of each wave's run
    // of each tile inside the unit sorted by tile
    __shared__ uint32_t scan_w[kWavesPerBlock];
    __shared__ uint32_t unit_total;
    {
        const int kpt = (K + kBlock - 1) / kBlock;  // tiles per thread, consecutive
        const int k0 = tid * kpt;
        uint32_t sum = 0;
        for (int kk = 0; kk < kpt; ++kk) {
            const int k = k0 + kk;
            if (k < K)
                for (int w = 0; w < kWavesPerBlock; ++w)
                    sum += cw[w * K + k];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t n = (uint32_t)__shfl_up((int)inc, o);
            if (lane >= o)
                inc += n;
        }
        if (lane == kWave - 1)
            scan_w[wave] = inc;
        __syncthreads();
        uint32_t run = inc - sum;
        for (int w = 0; w < wave; ++w)
            run += scan_w[w];
        if (tid == kBlock - 1)
            unit_total = run + sum;
        for (int kk = 0; kk < kpt; ++kk) {
            const int k = k0 + kk;
            if (k < K)
                for (int w = 0; w < kWavesPerBlock; ++w) {
                    const uint32_t c = cw[w * K + k];
                    cw[w * K + k] = (uint16_t)run;
                    run += c;
                }
        }
    }
    __syncthreads();

    // stage the records in tile order
    bool bad = false;
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        if (packed[s] != 0xFFFFFFFFu) {
            const uint32_t key = packed[s] >> 16;
            const uint32_t pos = (uint32_t)mycw[key] + (packed[s] & 0xFFFFu);
            if (pos < (uint32_t)U) {
                staged[pos] = recs[s];
                skey[pos] = (uint16_t)key;
            } else {
                bad = true;
            }
        }
    }
    __syncthreads();

    // each tile's run of this unit goes to its bucket: consecutive staged
    // records of one tile land on consecutive addresses
    const uint32_t total = min(unit_total, (uint32_t)U);
    for (uint32_t p = tid; p < total; p += kBlock) {
        const uint32_t k = skey[p];
        const int64_t g = (int64_t)gbase[k] + (int64_t)(p - cw[k]);
        if (k < (uint32_t)K && g >= 0 && g < cap)
            records[g] = staged[p];
        else
            bad = true;
    }
    if (bad)
        flags |= 8u;  // ESI_DIAG_INTERNAL: never expected
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

size_t bucket_lds_bytes(int K)
{
    return sizeof(uint64_t) * ((size_t)1 << kUnitLog) + sizeof(uint32_t) * K +
           sizeof(uint16_t) * (kWavesPerBlock * K + ((size_t)1 << kUnitLog));
}

hipError_t launch_bucket(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                         const CallScratch& cs, DiagDev* diag, hipStream_t stream)
{
    const int K = sc.ntiles;
    const int64_t B = sc.nunits;
    const size_t lds_hist = sizeof(uint32_t) * K;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)B), dim3(kBlock), lds_hist, stream, ev, st.W, st.H,
                       sc.tile_log, K, sc.unit_log, B, cs.table, diag);
    const int seg = scan_segment_units(B);
    const int nseg = (int)((B + seg - 1) / seg);
    const dim3 grid((unsigned)((K + kBlock - 1) / kBlock), (unsigned)nseg);
    hipLaunchKernelGGL(k_seg_sum, grid, dim3(kBlock), 0, stream, cs.table, K, B, seg, cs.blocksum);
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, stream, cs.blocksum, K, nseg, cs.total,
                       diag);
    hipLaunchKernelGGL(k_seg_down, grid, dim3(kBlock), 0, stream, cs.table, K, B, seg,
                       cs.blocksum);
    hipLaunchKernelGGL(k_bucket<kUnitLog>, dim3((unsigned)B), dim3(kBlock), bucket_lds_bytes(K),
                       stream, ev, st.W, st.H, sc.tile_log, K, B, cs.table, cs.records, ev.n,
                       diag);
    return hipGetLastError();
}

}  // namespace esi
