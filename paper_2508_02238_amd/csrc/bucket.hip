// bucket.hip -- stable bucketing of a time-sorted event stream by pixel tile.
//
// Alg. 2 walks the events in array order and touches only the event's own
// pixel, so the order that matters is the order of the events of each pixel.
// These kernels regroup the events tile-major (a tile = a range of
// consecutive pixels) while keeping array order inside every tile (and so
// inside every pixel): a counting sort whose ranks are stable.
//
// The stream is split into G equal ranges of events, one per workgroup, with
// G = the number of bucketing workgroups the GPU holds at once, so every
// range is processed in a single round with no tail of late workgroups.
//
//   k_hist      per range: per-tile counts of its valid events ->
//               table[range][tile]; out-of-range events are counted as dropped.
//   k_seg_sum,  exclusive scan of the table in (tile, range) order, done
//   k_seg_down  column-wise so every access is a coalesced row access:
//               per-tile sums over segments of ranges (and per-tile totals),
//               then each segment rescanned into offsets.
//   k_bucket    per range again, in sub-batches of SUB events: each wave ranks
//               its share of the sub-batch stably by tile (wave-wide key
//               match), a scan over (tile, wave) gives every event its place
//               in the sub-batch sorted by tile, the 64-bit records (time
//               offset, pixel in tile, polarity) are staged in LDS in that
//               order, and each tile's run is appended to its bucket.  Also
//               flags decreasing times and calls whose span the record cannot
//               hold.
//
// Workgroups are dispatched round-robin over the 8 XCDs; ranges are assigned
// so that the workgroups of one XCD take consecutive ranges.  Neighbouring
// ranges append adjacent runs to every tile bucket within a short time, so the
// cache lines of a bucket are completed in one XCD's L2 before they are
// written back (scattered 8-byte stores spread over the whole kernel would
// reach HBM as partial lines).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "esi_internal.hpp"

namespace esi {
namespace {

constexpr int kXcds = 8;
constexpr int kSegRows = 16;  // table rows (ranges) per segment of the column scan
// Sub-batches of the bucketing: 4096 events over four waves (two workgroups
// per CU), and for calls of kWideTiles tiles or more 8192 events over eight
// waves (one workgroup per CU): twice the run per tile and write-out, and the
// per-sub-batch scan over the tiles spread over twice the events.  The
// batched kernel always takes the first.
constexpr int kSub = 4096;
constexpr int kSubWide = 8192;
constexpr int kWavesWide = 8;
constexpr int kWideTiles = 1536;

// Bijection blockIdx -> work index that gives each XCD a contiguous range.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t x = b % kXcds, i = b / kXcds;
    const int64_t q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// An event of this pass: x < W and y in the pass's rows [y0, y0 + H); q is
// its pixel inside the pass.  `drop`: the event is off the sensor.
__device__ __forceinline__ bool valid_q(uint32_t x, uint32_t y, int W, int H, const EventsDev& ev,
                                        uint32_t& q, bool& drop)
{
    const uint32_t yl = y - (uint32_t)ev.y0;
    q = yl * (uint32_t)W + x;
    drop = x >= (uint32_t)W || y >= (uint32_t)ev.H_all;
    return x < (uint32_t)W && yl < (uint32_t)H;
}

// Range `unit` holds events [unit E, min((unit + 1) E, n)); E is a multiple
// of kBlock.
// Workgroup 0 also clears the per-tile totals that k_seg_sum accumulates.
template <int NT>
__device__ __forceinline__ void hist_body(const EventsDev& ev, int W, int H, int tile_log, int K,
                                          int64_t E, uint32_t* table, uint32_t* tile_tot,
                                          DiagDev* diag, int64_t unit, bool first)
{
    extern __shared__ uint32_t h[];
    for (int k = threadIdx.x; k < K; k += NT) {
        h[k] = 0;
        if (first)
            tile_tot[k] = 0;
    }
    __syncthreads();
    uint32_t drop = 0;
    const int64_t lo = unit * E;
    const int64_t hi = min(lo + E, ev.n);
    const bool vec = (((uintptr_t)ev.x | (uintptr_t)ev.y) & 15u) == 0;
    int64_t i = lo;
    if (vec) {
        // 8 events per thread per step: 16-byte loads of x and y
        for (; i + 8 * NT <= hi; i += 8 * NT) {
            const int64_t e = i + 8 * threadIdx.x;
            const uint4 xv = *(const uint4*)(ev.x + e);
            const uint4 yv = *(const uint4*)(ev.y + e);
            const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
            const uint32_t ys[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                uint32_t q;
                bool off;
                if (valid_q(xs[m] & 0xFFFFu, ys[m] & 0xFFFFu, W, H, ev, q, off))
                    atomicAdd(&h[q >> tile_log], 1u);
                drop += off;
                if (valid_q(xs[m] >> 16, ys[m] >> 16, W, H, ev, q, off))
                    atomicAdd(&h[q >> tile_log], 1u);
                drop += off;
            }
        }
    }
    for (int64_t e = i + threadIdx.x; e < hi; e += NT) {
        uint32_t q;
        bool off;
        if (valid_q(ev.x[e], ev.y[e], W, H, ev, q, off))
            atomicAdd(&h[q >> tile_log], 1u);
        drop += off;
    }
    __syncthreads();
    uint32_t* row = table + unit * K;
    for (int k = threadIdx.x; k < K; k += NT)
        row[k] = h[k];
    if (drop && ev.y0 == 0)
        atomicAdd(&diag->dropped, (unsigned long long)drop);
}

// ---- exclusive scan of table[u][k] in (k, u) order, column-wise -------------
// Segments of kSegRows rows.  k_seg_sum: segsum[s][k] = sum over the rows of
// segment s, and tile_tot[k] += that sum.  k_seg_down: the offset of
// (unit u, tile k) = (tiles before k) + (segments before u's) + (rows of u's
// segment before u), written over table[u][k].

__device__ __forceinline__ void seg_sum_body(const uint32_t* table, int K, int64_t B,
                                             uint32_t* segsum, uint32_t* tile_tot, int bx, int s)
{
    const int k = bx * kBlock + threadIdx.x;
    if (k >= K)
        return;
    const int64_t u0 = (int64_t)s * kSegRows;
    uint32_t v[kSegRows];
#pragma unroll
    for (int r = 0; r < kSegRows; ++r)  // all loads in flight at once
        v[r] = (u0 + r < B) ? table[(u0 + r) * K + k] : 0u;
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kSegRows; ++r)
        sum += v[r];
    segsum[(int64_t)s * K + k] = sum;
    if (sum)
        atomicAdd(&tile_tot[k], sum);
}

__device__ __forceinline__ void seg_down_body(uint32_t* table, int K, int64_t B,
                                              const uint32_t* segsum, const uint32_t* tile_tot,
                                              uint32_t* total, DiagDev* diag, int bx, int s)
{
    constexpr int kBatch = 16;
    constexpr int kPer = (kMaxTiles + kBlock - 1) / kBlock;  // tile totals per thread
    __shared__ uint32_t base[kMaxTiles];
    __shared__ uint32_t sw[kWavesPerBlock];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    // exclusive scan of the tile totals (each workgroup for itself)
    uint32_t v[kPer], sum = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int k = tid * kPer + i;
        v[i] = (k < K) ? tile_tot[k] : 0u;
        sum += v[i];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = (uint32_t)__shfl_up((int)inc, o);
        if (lane >= o)
            inc += n;
    }
    if (lane == kWave - 1)
        sw[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum, all = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
        run += (w < wave) ? sw[w] : 0u;
        all += sw[w];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int k = tid * kPer + i;
        if (k < K)
            base[k] = run;
        run += v[i];
    }
    __syncthreads();
    if (bx == 0 && s == 0 && tid == 0) {
        *total = all;
        atomicAdd(&diag->accepted, (unsigned long long)all);
    }

    const int k = bx * kBlock + tid;
    if (k >= K)
        return;
    // segments before this one, loads in batches
    uint32_t off = base[k];
    for (int s0 = 0; s0 < s; s0 += kBatch) {
        uint32_t w[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            w[b] = (s0 + b < s) ? segsum[(int64_t)(s0 + b) * K + k] : 0u;
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            off += w[b];
    }
    const int64_t u0 = (int64_t)s * kSegRows;
    uint32_t c[kSegRows];
#pragma unroll
    for (int r = 0; r < kSegRows; ++r)
        c[r] = (u0 + r < B) ? table[(u0 + r) * K + k] : 0u;
#pragma unroll
    for (int r = 0; r < kSegRows; ++r) {
        if (u0 + r < B)
            table[(u0 + r) * K + k] = off;
        off += c[r];
    }
}

// ---- stable bucketing, staged in LDS ------------------------------------------

template <int SUB, int NW>
__device__ __forceinline__ void bucket_body(const EventsDev& ev, int W, int H, int tile_log, int K,
                                            int64_t E, const uint32_t* table, uint64_t* records,
                                            int64_t cap, DiagDev* diag, int64_t unit)
{
    constexpr int NT = NW * kWave;                  // threads of the workgroup
    constexpr int CW = NW / 4;                      // 64-bit counter words per tile
    static_assert(NW % 4 == 0, "four 16-bit wave counters per word");
    constexpr int PER_WAVE = SUB / NW;              // events per wave per sub-batch
    constexpr int STEPS = PER_WAVE / kWave;         // steps of 64 per wave
    constexpr int BATCH = STEPS < 8 ? STEPS : 8;    // steps loaded ahead
    static_assert(STEPS % BATCH == 0, "sub-batch size");
    static_assert(sizeof(uint64_t) * SUB >= sizeof(uint64_t) * NW * kWave + NW * kMaxTiles,
                  "the rank's scratch fits the staging area");
    extern __shared__ uint64_t smem[];
    // LDS: staged | cw | gbase | wd | skey.  While a sub-batch is ranked, the
    // staging area holds the rank's representative lanes and lane masks.
    uint64_t* staged = smem;                      // [SUB] records of the sub-batch by tile
    uint64_t* cw = staged + SUB;                  // [K][CW] NW x u16: per-wave counters, then run starts
    uint32_t* gbase = (uint32_t*)(cw + (size_t)K * CW);  // [K] next bucket position of each tile
    uint32_t* wd = gbase + K;                     // [K] bucket position minus staged position
    uint16_t* skey = (uint16_t*)(wd + K);         // [SUB] tile of each staged record
    uint64_t* group = staged;                     // [NW][64] lane masks of the rank
    uint8_t* rep = (uint8_t*)(staged + NW * kWave);  // [NW][K] representative lanes
    __shared__ uint32_t scan_w[NW];
    __shared__ uint32_t sub_total;

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const uint32_t* row = table + unit * K;
    for (int k = tid; k < K; k += NT)
        gbase[k] = row[k];
    for (int k = tid; k < K * CW; k += NT)
        cw[k] = 0;
    __syncthreads();

    const uint32_t tmask = (1u << tile_log) - 1u;
    const int64_t t_ref = ev.t[0];
    const int64_t u_lo = unit * E;
    const int64_t u_hi = min(u_lo + E, ev.n);
    uint16_t* mycw = (uint16_t*)cw + wave;
    uint8_t* myrep = rep + wave * K;
    uint64_t* mygroup = group + wave * kWave;
    uint32_t flags = 0;
    bool bad = false;

    // The sub-batches are software-pipelined: the first half of the next
    // sub-batch's events is loaded before this sub-batch's records are
    // written and the second half before the first is ranked, and the record
    // stores are a fixed sequence with no branch (a lane without a record
    // writes the spare slot records[cap]), so that the wait for a half leaves
    // the stores issued after it in flight: on CDNA one counter tracks vector
    // loads and stores, and a variable number of stores would make the
    // compiler wait for all of them.
    const int w0 = wave * PER_WAVE;
    constexpr int HALF = STEPS / 2;
    static_assert(STEPS % 2 == 0, "two halves of a sub-batch");
    uint32_t xs[STEPS], ys[STEPS];
    int64_t ts[STEPS];
    int ps[STEPS];
    int64_t tc = INT64_MIN;  // time of the event before this wave's first one
    // loads of steps [s0, s0 + HALF) of the sub-batch at sb: offsets clamped
    // into [u_lo, u_hi), so every load is valid and none depends on a select
    // of loaded values
    auto load_half = [&](int64_t sb, int s0) {
#pragma unroll
        for (int st = s0; st < s0 + HALF; ++st) {
            const int64_t o = min(sb + (int64_t)(w0 + st * kWave + lane), u_hi - 1);
            xs[st] = ev.x[o];
            ys[st] = ev.y[o];
            ts[st] = ev.t[o];
            ps[st] = ev.p[o];
        }
        if (s0 == 0)
            tc = ev.t[max(min(sb + (int64_t)w0, u_hi) - 1, (int64_t)0)];
    };
    if (u_lo < u_hi)
        load_half(u_lo, 0);

    for (int64_t sb = u_lo; sb < u_hi; sb += SUB) {
        // this sub-batch's events: [sb, sb + nsb); this wave's: from sb + w0
        const int nsb = (int)min((int64_t)SUB, u_hi - sb);
        load_half(sb, HALF);
        int64_t t_carry = (sb + w0 > 0 && w0 < nsb) ? tc : INT64_MIN;
        uint64_t recs[STEPS];
        uint32_t packed[STEPS];  // rank | tile << 16, or ~0 for no event
#pragma unroll
        for (int st = 0; st < STEPS; ++st) {
            const bool in = w0 + st * kWave + lane < nsb;
            const uint32_t yl = ys[st] - (uint32_t)ev.y0;
            const uint32_t q = yl * (uint32_t)W + xs[st];
            const bool ok = in && xs[st] < (uint32_t)W && yl < (uint32_t)H;
            const int64_t t = ts[st];
            // decreasing time versus the previous event in array order:
            // the previous lane's time (lane 0: the previous step's last)
            const uint64_t tu = (uint64_t)t, cu = (uint64_t)t_carry;
            const uint32_t plo = (uint32_t)__builtin_amdgcn_update_dpp(
                (int)(uint32_t)cu, (int)(uint32_t)tu, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
            const uint32_t phi = (uint32_t)__builtin_amdgcn_update_dpp(
                (int)(uint32_t)(cu >> 32), (int)(uint32_t)(tu >> 32), 0x138, 0xF, 0xF, false);
            const int64_t tprev = (int64_t)(((uint64_t)phi << 32) | plo);
            if (in && t < tprev)
                flags |= 1u;  // ESI_DIAG_UNSORTED
            t_carry = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(tu >> 32), kWave - 1) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)tu, kWave - 1));
            const int64_t dt = t - t_ref;
            if (ok && (dt >= kMaxSpan || dt <= -kMaxSpan))
                flags |= 4u;  // ESI_DIAG_TIME_RANGE
            const uint32_t key = ok ? (q >> tile_log) : 0u;
            const uint32_t rank = wave_stable_rank_or<NW>(ok, key, mycw, myrep, mygroup);
            packed[st] = ok ? (rank | (key << 16)) : 0xFFFFFFFFu;
            recs[st] = pack_record(dt, q & tmask, ps[st] > 0);
        }
        __syncthreads();
        // exclusive scan over (tile, wave), tile-major: start of each wave's
        // run of each tile inside the sub-batch sorted by tile; each tile's
        // bucket position advances by its count here, and wd keeps the
        // offset from staged to bucket position for this sub-batch
        {
            const int kpt = (K + NT - 1) / NT;  // tiles per thread, consecutive
            const int k0 = tid * kpt;
            uint32_t sum = 0;
            for (int kk = 0; kk < kpt; ++kk) {
                const int k = k0 + kk;
                if (k < K) {
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const uint64_t v = cw[(size_t)k * CW + c];
                        sum += (uint32_t)(v & 0xFFFF) + (uint32_t)((v >> 16) & 0xFFFF) +
                               (uint32_t)((v >> 32) & 0xFFFF) + (uint32_t)(v >> 48);
                    }
                }
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
            if (tid == NT - 1)
                sub_total = run + sum;
            for (int kk = 0; kk < kpt; ++kk) {
                const int k = k0 + kk;
                if (k < K) {
                    const uint32_t s0 = run;
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const uint64_t v = cw[(size_t)k * CW + c];
                        uint64_t starts = 0;
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            starts |= (uint64_t)(run & 0xFFFFu) << (16 * w);
                            run += (uint32_t)(v >> (16 * w)) & 0xFFFFu;
                        }
                        cw[(size_t)k * CW + c] = starts;
                    }
                    const uint32_t g0 = gbase[k];
                    wd[k] = g0 - s0;
                    gbase[k] = g0 + (run - s0);
                }
            }
        }
        __syncthreads();

        // stage the records in tile order (over the rank's scratch)
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            if (packed[s] != 0xFFFFFFFFu) {
                const uint32_t key = packed[s] >> 16;
                const uint32_t pos = (uint32_t)mycw[key * NW] + (packed[s] & 0xFFFFu);
                if (pos < (uint32_t)SUB) {
                    staged[pos] = recs[s];
                    skey[pos] = (uint16_t)key;
                } else {
                    bad = true;
                }
            }
        }
        __syncthreads();

        // the first half of the next sub-batch's events, in flight during
        // the write-back
        load_half(sb + SUB, 0);

        // each tile's run of this sub-batch is appended to its bucket:
        // consecutive staged records of one tile land on consecutive
        // addresses; the counters are cleared for the next sub-batch
        const uint32_t total = min(sub_total, (uint32_t)SUB);
#pragma unroll
        for (int i = 0; i < SUB / NT; ++i) {
            const uint32_t p = (uint32_t)(tid + i * NT);
            const uint32_t k = skey[p];
            const int64_t g = (p < total && k < (uint32_t)K) ? (int64_t)(uint32_t)(wd[k] + p) : -1;
            const bool store = g >= 0 && g < cap;
            bad |= p < total && !store;
            records[store ? g : cap] = staged[p];
        }
        for (int k = tid; k < K * CW; k += NT)
            cw[k] = 0;
        __syncthreads();  // staged, skey and cw are reused by the next sub-batch
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

// Single-stream kernels: one call's ranges, tile columns and segments.
// The histogram runs 1024 threads per range: one workgroup per range, and
// the ranges are as few as the bucketing workgroups resident at once.
constexpr int kHistBlock = 1024;

__global__ __launch_bounds__(kHistBlock) void k_hist(EventsDev ev, int W, int H, int tile_log,
                                                     int K, int64_t E, uint32_t* table,
                                                     uint32_t* tile_tot, DiagDev* diag)
{
    hist_body<kHistBlock>(ev, W, H, tile_log, K, E, table, tile_tot, diag, xcd_block(blockIdx.x, gridDim.x),
              blockIdx.x == 0);
}

__global__ __launch_bounds__(kBlock) void k_seg_sum(const uint32_t* table, int K, int64_t B,
                                                    uint32_t* segsum, uint32_t* tile_tot)
{
    seg_sum_body(table, K, B, segsum, tile_tot, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBlock) void k_seg_down(uint32_t* table, int K, int64_t B,
                                                     const uint32_t* segsum,
                                                     const uint32_t* tile_tot, uint32_t* total,
                                                     DiagDev* diag)
{
    seg_down_body(table, K, B, segsum, tile_tot, total, diag, blockIdx.x, blockIdx.y);
}

template <int SUB, int NW>
__global__ __launch_bounds__(NW * kWave, 2) void k_bucket(EventsDev ev, int W, int H, int tile_log,
                                                       int K, int64_t E, const uint32_t* table,
                                                       uint64_t* records, int64_t cap, DiagDev* diag)
{
    bucket_body<SUB, NW>(ev, W, H, tile_log, K, E, table, records, cap, diag,
                         xcd_block(blockIdx.x, gridDim.x));
}

// ---- integration order: tiles by event count, largest first -----------------
// The integration launch has more tiles than the GPU holds workgroups, and
// the tiles' event counts differ by an order of magnitude (a scene's moving
// edges cross some tiles far more often than others).  Workgroups start in
// index order, so listing the tiles largest first lets the short ones fill
// the end of the launch (longest-processing-time-first list scheduling).
// The tiles are sorted by a size class of their count (leading bit and four
// bits after it); order within a class is whatever the LDS atomics give, a
// schedule only: every tile's result is the same wherever it runs.
constexpr int kOrderBlock = 1024;
constexpr int kOrderClasses = 513;  // 0 for an empty tile, 1 + 16 e + m otherwise

__device__ __forceinline__ uint32_t size_class(uint32_t c)
{
    if (c == 0)
        return 0;
    const int e = 31 - __clz(c);
    const uint32_t m = (e >= 4 ? c >> (e - 4) : c << (4 - e)) & 15u;
    return 1u + 16u * (uint32_t)e + m;
}

__global__ __launch_bounds__(kOrderBlock) void k_order(const uint32_t* tile_tot, int K,
                                                       uint32_t* order)
{
    static_assert(kOrderClasses <= kOrderBlock, "one class per thread");
    __shared__ uint32_t pos[kOrderBlock];
    __shared__ uint32_t wsum[kOrderBlock / kWave];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    pos[tid] = 0;
    __syncthreads();
    // slot kOrderClasses - 1 - class: the largest class first
    for (int k = tid; k < K; k += kOrderBlock)
        atomicAdd(&pos[kOrderClasses - 1 - size_class(tile_tot[k])], 1u);
    __syncthreads();
    const uint32_t v = pos[tid];
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = (uint32_t)__shfl_up((int)inc, o);
        if (lane >= o)
            inc += n;
    }
    if (lane == kWave - 1)
        wsum[wave] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w)
        base += wsum[w];
    pos[tid] = base + inc - v;  // exclusive start of this slot
    __syncthreads();
    for (int k = tid; k < K; k += kOrderBlock) {
        const uint32_t at = atomicAdd(&pos[kOrderClasses - 1 - size_class(tile_tot[k])], 1u);
        if (at < (uint32_t)K)
            order[at] = (uint32_t)k;
    }
}

// ---- batched calls: many streams per launch ---------------------------------

// The stream whose work range [base[i], base[i + 1]) holds w (base[0] = 0,
// non-decreasing; uniform loads).
__device__ __forceinline__ int batch_item(const uint32_t* base, int n, uint32_t w)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (load_const(base, mid) <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One workgroup per (stream, range); each stream's ranges start at a multiple
// of the XCD count, so the XCD mapping of one call carries over.
__global__ __launch_bounds__(kHistBlock) void kb_hist(BatchDev b)
{
    const int i = batch_item(b.unit_base, b.n, blockIdx.x);
    const BatchItem& it = b.items[i];
    const int64_t unit = xcd_block(blockIdx.x - load_const(b.unit_base, i), it.B_pad);
    if (unit >= it.B)
        return;
    hist_body<kHistBlock>(it.ev, it.st.W, it.st.H, it.tile_log, it.K, it.E, it.cs.table, it.cs.tile_tot,
              it.diag, unit, unit == 0);
}

__global__ __launch_bounds__(kBlock) void kb_seg_sum(BatchDev b)
{
    const int i = batch_item(b.seg_base, b.n, blockIdx.x);
    const BatchItem& it = b.items[i];
    const int l = (int)(blockIdx.x - load_const(b.seg_base, i));
    seg_sum_body(it.cs.table, it.K, it.B, it.cs.blocksum, it.cs.tile_tot, l % it.cols,
                 l / it.cols);
}

__global__ __launch_bounds__(kBlock) void kb_seg_down(BatchDev b)
{
    const int i = batch_item(b.seg_base, b.n, blockIdx.x);
    const BatchItem& it = b.items[i];
    const int l = (int)(blockIdx.x - load_const(b.seg_base, i));
    seg_down_body(it.cs.table, it.K, it.B, it.cs.blocksum, it.cs.tile_tot, it.cs.total, it.diag,
                  l % it.cols, l / it.cols);
}

template <int SUB>
__global__ __launch_bounds__(kBlock, 2) void kb_bucket(BatchDev b)
{
    const int i = batch_item(b.unit_base, b.n, blockIdx.x);
    const BatchItem& it = b.items[i];
    const int64_t unit = xcd_block(blockIdx.x - load_const(b.unit_base, i), it.B_pad);
    if (unit >= it.B)
        return;
    bucket_body<SUB, kWavesPerBlock>(it.ev, it.st.W, it.st.H, it.tile_log, it.K, it.E,
                                     it.cs.table, it.cs.records, it.ev.n, it.diag, unit);
}

// LDS of bucket_body: staged records, per-wave counters, two tile arrays,
// staged tiles
template <int SUB, int NW>
size_t bucket_lds(int K)
{
    return sizeof(uint64_t) * (SUB + (size_t)K * (NW / 4)) + 2 * sizeof(uint32_t) * K +
           sizeof(uint16_t) * SUB;
}

}  // namespace

bool bucket_wide(int K) { return K >= kWideTiles; }

int bucket_slots(int K)
{
    int dev = 0, cus = 0, per_cu = 0;
    const hipError_t occ =
        bucket_wide(K)
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bucket<kSubWide, kWavesWide>,
                                                           kWavesWide * kWave,
                                                           bucket_lds<kSubWide, kWavesWide>(K))
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bucket<kSub, kWavesPerBlock>,
                                                           kBlock,
                                                           bucket_lds<kSub, kWavesPerBlock>(K));
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        occ != hipSuccess) {
        (void)hipGetLastError();
        return 1024;
    }
    return std::max(1, cus) * std::max(1, per_cu);
}

int bucket_slots_batch(int K)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kb_bucket<kSub>, kBlock,
                                                     bucket_lds<kSub, kWavesPerBlock>(K)) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 1024;
    }
    return std::max(1, cus) * std::max(1, per_cu);
}

size_t scan_segments(int64_t B) { return (size_t)((B + kSegRows - 1) / kSegRows); }

hipError_t launch_bucket_batch(const BatchDev& b, uint32_t units, uint32_t seg_blocks, int kmax,
                               hipStream_t stream)
{
    if (units == 0)
        return hipSuccess;
    hipLaunchKernelGGL(kb_hist, dim3(units), dim3(kHistBlock), sizeof(uint32_t) * kmax, stream, b);
    if (seg_blocks) {
        hipLaunchKernelGGL(kb_seg_sum, dim3(seg_blocks), dim3(kBlock), 0, stream, b);
        hipLaunchKernelGGL(kb_seg_down, dim3(seg_blocks), dim3(kBlock), 0, stream, b);
    }
    hipLaunchKernelGGL(kb_bucket<kSub>, dim3(units), dim3(kBlock),
                       (bucket_lds<kSub, kWavesPerBlock>(kmax)), stream, b);
    return hipGetLastError();
}

hipError_t launch_bucket(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                         const CallScratch& cs, DiagDev* diag, hipStream_t stream)
{
    const int K = sc.ntiles;
    const int64_t B = sc.nunits;
    const int nseg = (int)scan_segments(B);
    hipLaunchKernelGGL(k_hist, dim3((unsigned)B), dim3(kHistBlock), sizeof(uint32_t) * K, stream, ev,
                       st.W, st.H, sc.tile_log, K, sc.unit_events, cs.table, cs.tile_tot, diag);
    const dim3 grid((unsigned)((K + kBlock - 1) / kBlock), (unsigned)nseg);
    hipLaunchKernelGGL(k_seg_sum, grid, dim3(kBlock), 0, stream, cs.table, K, B, cs.blocksum,
                       cs.tile_tot);
    hipLaunchKernelGGL(k_seg_down, grid, dim3(kBlock), 0, stream, cs.table, K, B, cs.blocksum,
                       cs.tile_tot, cs.total, diag);
    if (sc.ordered)
        hipLaunchKernelGGL(k_order, dim3(1), dim3(kOrderBlock), 0, stream, cs.tile_tot, K,
                           cs.order);
    if (bucket_wide(K))
        hipLaunchKernelGGL((k_bucket<kSubWide, kWavesWide>), dim3((unsigned)B),
                           dim3(kWavesWide * kWave), (bucket_lds<kSubWide, kWavesWide>(K)), stream,
                           ev, st.W, st.H, sc.tile_log, K, sc.unit_events, cs.table, cs.records,
                           ev.n, diag);
    else
        hipLaunchKernelGGL((k_bucket<kSub, kWavesPerBlock>), dim3((unsigned)B), dim3(kBlock),
                           (bucket_lds<kSub, kWavesPerBlock>(K)), stream, ev, st.W, st.H,
                           sc.tile_log, K, sc.unit_events, cs.table, cs.records, ev.n, diag);
    return hipGetLastError();
}

}  // namespace esi
