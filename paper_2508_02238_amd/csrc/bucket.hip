// bucket.hip -- stable bucketing of a time-sorted event stream by pixel tile.
//
// Alg. 2 walks the events in array order and touches only the event's own
// pixel, so the order that matters is the order of the events of each pixel.
// These kernels regroup the events tile-major (a tile = a range of
// consecutive pixels) while keeping array order inside every tile (and so
// inside every pixel): a counting sort whose ranks are stable.
//
//   k_hist     one wave per unit of 2^unit_log events: per-tile counts of the
//              unit's valid events -> table[unit][tile].  Out-of-range events
//              are counted as dropped.
//   k_scan_*   exclusive scan of the table in (tile, unit) order: the offset
//              of each unit's run inside each tile's bucket.
//   k_scatter  one wave per unit again: walks its events 64 at a time in
//              order, ranks each event stably among the same-tile events of
//              the unit, writes a 64-bit record (time offset, pixel in tile,
//              polarity) to its slot.  Also flags decreasing times and calls
//              whose time span does not fit the record.
#include <hip/hip_runtime.h>

#include "esi_internal.hpp"

namespace esi {
namespace {

__device__ __forceinline__ bool decode(const EventsDev& ev, int64_t i, int W, int H, uint32_t& q)
{
    const uint32_t x = ev.x[i], y = ev.y[i];
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
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    uint32_t* h = lds + wave * K;
    for (int k = lane; k < K; k += kWave)
        h[k] = 0;
    __syncthreads();
    uint32_t drop = 0;
    if (unit < B) {
        const int64_t lo = unit << unit_log;
        const int64_t hi = min(lo + ((int64_t)1 << unit_log), ev.n);
        int64_t i = lo + lane;
        for (; i + 3 * kWave < hi; i += 4 * kWave) {
            uint32_t q0, q1, q2, q3;
            const bool v0 = decode(ev, i, W, H, q0);
            const bool v1 = decode(ev, i + kWave, W, H, q1);
            const bool v2 = decode(ev, i + 2 * kWave, W, H, q2);
            const bool v3 = decode(ev, i + 3 * kWave, W, H, q3);
            if (v0) atomicAdd(&h[q0 >> tile_log], 1u); else ++drop;
            if (v1) atomicAdd(&h[q1 >> tile_log], 1u); else ++drop;
            if (v2) atomicAdd(&h[q2 >> tile_log], 1u); else ++drop;
            if (v3) atomicAdd(&h[q3 >> tile_log], 1u); else ++drop;
        }
        for (; i < hi; i += kWave) {
            uint32_t q;
            if (decode(ev, i, W, H, q))
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

// ---- exclusive scan over the table in (tile, unit) order -------------------
// Element m = k * B + u lives at table[u * K + k].

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_waves,
                                                         uint32_t& block_total)
{
    // inclusive scan inside the wave
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = (uint32_t)__shfl_up((int)inc, o);
        if (lane >= o)
            inc += n;
    }
    if (lane == kWave - 1)
        lds_waves[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
        const uint32_t s = lds_waves[w];
        off += (w < wave) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    block_total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* table, int K, int64_t B,
                                                        int64_t M, uint32_t* blocksum)
{
    __shared__ uint32_t sw[kWavesPerBlock];
    const int64_t m0 = (int64_t)blockIdx.x * kScanBlockItems + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    if (m0 < M) {
        int64_t k = m0 / B, u = m0 - k * B;
        for (int j = 0; j < kScanItems && m0 + j < M; ++j) {
            s += table[u * K + k];
            if (++u == B) {
                u = 0;
                ++k;
            }
        }
    }
    uint32_t tot;
    block_exclusive_scan(s, sw, tot);
    if (threadIdx.x == 0)
        blocksum[blockIdx.x] = tot;
}

// One workgroup of 1024 threads: exclusive scan of nb <= 1024 block sums.
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* blocksum, int nb, uint32_t* total,
                                                      DiagDev* diag)
{
    __shared__ uint32_t sw[1024 / kWave];
    const uint32_t v = (threadIdx.x < (unsigned)nb) ? blocksum[threadIdx.x] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sw, tot);
    if (threadIdx.x < (unsigned)nb)
        blocksum[threadIdx.x] = ex;
    if (threadIdx.x == 0) {
        *total = tot;
        atomicAdd(&diag->accepted, (unsigned long long)tot);
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t* table, int K, int64_t B, int64_t M,
                                                      const uint32_t* blocksum)
{
    __shared__ uint32_t sw[kWavesPerBlock];
    const int64_t m0 = (int64_t)blockIdx.x * kScanBlockItems + (int64_t)threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t s = 0;
    int64_t k0 = 0, u0 = 0;
    if (m0 < M) {
        k0 = m0 / B;
        u0 = m0 - k0 * B;
        int64_t k = k0, u = u0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            vals[j] = (m0 + j < M) ? table[u * K + k] : 0u;
            s += vals[j];
            if (++u == B) {
                u = 0;
                ++k;
            }
        }
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, sw, tot) + blocksum[blockIdx.x];
    if (m0 < M) {
        int64_t k = k0, u = u0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            if (m0 + j < M)
                table[u * K + k] = run;
            run += vals[j];
            if (++u == B) {
                u = 0;
                ++k;
            }
        }
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
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    uint32_t* base = lds + wave * (K + 128);
    uint32_t* tag = base + K;
    if (unit < B) {
        const uint32_t* row = table + unit * K;
        for (int k = lane; k < K; k += kWave)
            base[k] = row[k];
    }
    for (int k = lane; k < 128; k += kWave)
        tag[k] = 0xFFFFFFFFu;
    __syncthreads();
    if (unit >= B)
        return;  // whole wave leaves together

    const uint32_t tmask = (1u << tile_log) - 1u;
    const int64_t t_ref = ev.t[0];
    const int64_t lo = unit << unit_log;
    const int64_t hi = min(lo + ((int64_t)1 << unit_log), ev.n);
    int64_t t_carry = (lo > 0) ? ev.t[lo - 1] : INT64_MIN;
    uint32_t flags = 0;
    for (int64_t i0 = lo; i0 < hi; i0 += kWave) {
        const int64_t i = i0 + lane;
        const bool in = i < hi;
        uint32_t q = 0;
        bool ok = false;
        int64_t t = 0;
        int pos = 0;
        if (in) {
            ok = decode(ev, i, W, H, q);
            t = ev.t[i];
            pos = ev.p[i] > 0;
        }
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
        const uint32_t key = q >> tile_log;
        uint32_t slot;
        const bool ranked = wave_stable_rank(ok, key, base, tag, slot);
        if (ok) {
            if (ranked && (int64_t)slot < cap)
                records[slot] = pack_record(dt, q & tmask, pos);
            else
                flags |= 8u;  // ESI_DIAG_INTERNAL: never expected
        }
    }
    // one atomic per wave with any flag
    const uint64_t any = __ballot(flags != 0);
    if (any) {
        uint32_t f = flags;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            f |= (uint32_t)__shfl_xor((int)f, o);
        if (lane == 0)
            atomicOr(&diag->flags, f);
    }
}

}  // namespace

hipError_t launch_bucket(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                         const CallScratch& cs, DiagDev* diag, hipStream_t stream)
{
    const int K = sc.ntiles;
    const int64_t B = sc.nunits;
    const int64_t M = (int64_t)K * B;
    const unsigned blocks_units = (unsigned)((B + kWavesPerBlock - 1) / kWavesPerBlock);
    const size_t lds_hist = sizeof(uint32_t) * kWavesPerBlock * K;
    hipLaunchKernelGGL(k_hist, dim3(blocks_units), dim3(kBlock), lds_hist, stream, ev, st.W, st.H,
                       sc.tile_log, K, sc.unit_log, B, cs.table, diag);
    const unsigned nb = (unsigned)((M + kScanBlockItems - 1) / kScanBlockItems);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, stream, cs.table, K, B, M,
                       cs.blocksum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, stream, cs.blocksum, (int)nb,
                       cs.total, diag);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, stream, cs.table, K, B, M,
                       cs.blocksum);
    const size_t lds_scatter = sizeof(uint32_t) * kWavesPerBlock * (K + 128);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_units), dim3(kBlock), lds_scatter, stream, ev, st.W,
                       st.H, sc.tile_log, K, sc.unit_log, B, cs.table, cs.records, ev.n, diag);
    return hipGetLastError();
}

}  // namespace esi
