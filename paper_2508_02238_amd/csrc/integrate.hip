// integrate.hip -- per-tile integration of the bucketed events and frames.
//
// One workgroup (256 threads) owns a tile of 256 * PPT consecutive pixels;
// thread `tid` owns pixels tid + 256 i (i < PPT), so that each wave writes a
// frame row piece of 256 contiguous bytes per pixel slot.  The pixel state
// (S, T, N, P) stays in registers for the whole call, S in FP64.
//
// The tile's records (array order inside the tile, from the bucketing pass)
// are consumed in chunks of at most CHUNK records, each paired with a
// segment of at most kFrameGroup frames: the frames that every record of the
// chunk precedes or belongs to and that no later record can reach.
//   1. each wave holds its quarter of the chunk's records in registers
//      (prefetched while the previous chunk was processed);
//   2. each record finds the first frame of the segment that includes it
//      (ballots over the segment's frame times bound each wave step's
//      records, then a binary search inside those bounds), then a
//      stable counting sort by pixel inside the tile (per-wave stable ranks,
//      an exclusive scan over (pixel, wave) counters, a scatter into LDS) makes
//      each pixel's events of the chunk contiguous and in array order;
//   3. phase A: each thread runs the events of its pixels through Alg. 2 in
//      array order and records a change list: for every frame of the segment
//      at which the pixel's visible state changes, the frame index and the
//      state after the last event that frame includes.  A pixel's run of more
//      than scan_run events (hot pixels, same-time bursts) is left to its
//      whole wave instead, which composes the run's per-event clamp-affine
//      maps with a DPP scan, 64 events at a time (3b), so that one long run
//      does not hold the other 63 lanes;
//   4. phase B: the segment's frames, every thread writing its pixels' values
//      (Eq. (14)); a frame compares its index with the pixel's next change
//      and only lanes with a change touch LDS.
// Frames after the last event form segments with no records.
//
// Decay at a frame: with t_b the segment's first frame time, a visible state
// (S, T) keeps A = 1 + k (T - t_b) and a frame at t_f has kt = k (t_f - t_b),
// so the base of Eq. (4) is u = A - kt = 1 - k (t_f - T).  A segment's frames
// span at most kMaxSegmentDecay decay lengths, which bounds the rounding of u
// by a few ulp of that span (a longer gap gives a one-frame segment, kt = 0).
// Under the exponential decay the factors separate instead:
// exp(-k (t_f - T)) = exp(k (T - t_b)) exp(-k (t_f - t_b)), so a visible
// state keeps G = exp(k (T - t_b)), a frame E = exp(-k (t_f - t_b)), and the
// frame's decay is min(G E, 1) (the 1 for a T after t_f); a segment then spans
// at most kMaxSegmentExp decay lengths, so that G and E stay normal numbers.
//
// Chunk boundaries come from a few scalar loads (first and last record of
// the window, first frame time after it) prefetched one chunk ahead; only a
// chunk that ends because its frame segment is full searches the records.
// The next chunk's records and frame times are loaded before this chunk's
// frame stores and waited for in one place: on CDNA one counter tracks vector
// loads and stores, and a load waited for after a burst of stores would wait
// for the stores too.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "esi_internal.hpp"

namespace esi {
namespace {

// s_waitcnt immediate (gfx9 encoding): vmcnt = 0, expcnt and lgkmcnt not waited.
constexpr int kWaitVmcnt0 = 0x0F70;
constexpr int kFrameGroup = 112;                    // frames per segment, at most
constexpr int kSearchTop = 64;                      // largest power of two <= kFrameGroup
constexpr double kMaxSegmentDecay = 1073741824.0;   // 2^30
constexpr double kMaxSegmentExp = 600.0;            // e^600 and e^-600 are normal doubles
constexpr int kNever = 0x7FFFFFFF;                  // "no further change"
constexpr uint64_t kLpxMask = (uint64_t)0x7FFF << 48;

// A tile of NB * PPT pixels: NB threads, PPT pixels each (thread t holds
// pixels t, t + NB, ...).  BIG (two pixels per thread only): chunks of 2048
// records at three workgroups per CU instead of 1536 at four.
template <int PPT, int NB, bool BIG = false>
struct TileCfg {
    static constexpr int TILE = NB * PPT;
    static constexpr int WAVES = NB / kWave;
    static constexpr int TILE_BITS = TILE == 256 ? 8 : TILE == 512 ? 9 : TILE == 1024 ? 10 : 11;
    // records per chunk: LDS holds them three times over (records, states,
    // frame indices) next to the (pixel, wave) counters of the tile; five
    // workgroups share a CU at one pixel per thread, four at two
    static constexpr int CHUNK = PPT == 1 ? 1280 : PPT == 2 ? (BIG ? 2048 : 1536) : 1024;
    static constexpr int PER_WAVE = CHUNK / WAVES;  // records per wave per chunk
    static constexpr int STEPS = PER_WAVE / kWave;  // records per lane per chunk
};

// Number of leading entries of tfl[0, n) that are < t (n <= kFrameGroup), in
// a fixed number of steps (binary lifting: the steps add up to at least
// kFrameGroup); for non-decreasing tfl this is the lower bound of t.
__device__ __forceinline__ int frames_before(const int64_t* tfl, int n, int64_t t)
{
    static_assert(2 * kSearchTop > kFrameGroup && kSearchTop <= kFrameGroup, "search steps");
    int pos = 0;
#pragma unroll
    for (int step = kSearchTop; step >= 1; step >>= 1) {
        const int probe = pos + step;
        const int64_t v = tfl[min(probe, kFrameGroup) - 1];
        pos = (probe <= n && v < t) ? probe : pos;
    }
    return pos;
}

template <int PPT>
struct Pixels {
    // state after every event applied so far (Alg. 2)
    double S[PPT];
    int64_t T[PPT];
    uint32_t N[PPT];  // this call's events (plus the stored count if loaded early)
    int32_t P[PPT];   // their polarity sum, likewise
    uint32_t touched; // bit i: pixel slot i has events in this call
    // the state the frames see: Sv = S / (s_max - s_min) and Av = 1 + k (T - t_b)
    // (exponential decay: Av = exp(k (T - t_b)))
    double Sv[PPT], Av[PPT];
    // change list of the segment: byte offsets of the next change's entry in
    // chg_S / chg_A (8-byte entries) and of the frame index after it in chg_j
    // (2-byte entries)
    uint32_t eo[PPT], jo[PPT];
    int jn[PPT];  // segment frame of the next change (>= kFrameGroup: none)
};

// Take the next change of pixel slot i: its state becomes the visible one and
// the frame of the change after it is read.  Pixel l's frame indices sit at
// chg_j[entry + l] and are followed by a 0xFFFF sentinel, so no test of the
// list's end is needed.
template <int PPT>
__device__ __forceinline__ void take_change(Pixels<PPT>& px, int i, const double* chg_S,
                                            const double* chg_A, const uint16_t* chg_j)
{
    px.Sv[i] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(chg_S) + px.eo[i]);
    px.Av[i] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(chg_A) + px.eo[i]);
    px.jn[i] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(chg_j) + px.jo[i]);
    px.eo[i] += 8u;
    px.jo[i] += 2u;
}

// Buffer resource for one frame row piece of `bytes` bytes: stores at or past
// `bytes` (pixel slots off the sensor in the last tile) are dropped by the
// buffer range check.  Word 3 is the gfx9 raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(void* row, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(row, (short)0, (int)bytes, 0x00020000);
}

constexpr int kNontemporal = 2;  // cache policy of the frame stores: streaming

// One frame (index jj of the segment) of Eq. (14): take the pixel's next
// change if it belongs to this frame, then
//   F = clamp(Sv u^b) + f_off,  u = clamp(Av - kt, 0, 1)    (decayed snapshot)
//   F = Sv + f_off                                        (lazy snapshot)
// with Sv = S / (s_max - s_min) and f_off = -s_min / (s_max - s_min), i.e.
// F = (v - s_min) / (s_max - s_min).  CLAMP: the clamp of Eq. (13) on the
// decayed value, a no-op when s_min <= 0 <= s_max and the state is in range
// (then Sv u^b lies between 0 and Sv).  OUT: 1 FP32 frames, 2 8-bit codes,
// 3 both; fr / ur: this frame's row piece of the tile.
template <int PPT, int NB, int BK, bool LAZY, bool CLAMP, int OUT>
__device__ __forceinline__ void frame_step(const MethodParams& mp, Pixels<PPT>& px, int jj, double kt,
                                           const double* chg_S, const double* chg_A,
                                           const uint16_t* chg_j, __amdgpu_buffer_rsrc_t fr,
                                           __amdgpu_buffer_rsrc_t ur)
{
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int l = (int)threadIdx.x + i * NB;
        if (px.jn[i] == jj)
            take_change<PPT>(px, i, chg_S, chg_A, chg_j);
        double F;
        if (LAZY) {
            F = px.Sv[i] + mp.f_off;
        } else if (BK == kDecayExp) {
            // kt holds the frame's factor E here and Av the state's G
            double w = px.Sv[i] * fmin(px.Av[i] * kt, 1.0);
            if (CLAMP)
                w = fmin(fmax(w, mp.sv_min), mp.sv_max);
            F = w + mp.f_off;
        } else {
            const double u = fmin(fmax(px.Av[i] - kt, 0.0), 1.0);
            if (BK == kDecayB2 && !CLAMP) {
                F = __fma_rn(px.Sv[i] * u, u, mp.f_off);
            } else if (BK == kDecayB1 && !CLAMP) {
                F = __fma_rn(px.Sv[i], u, mp.f_off);
            } else {
                double w = px.Sv[i] * power_b<BK>(u, mp.b);
                if (CLAMP)
                    w = fmin(fmax(w, mp.sv_min), mp.sv_max);
                F = w + mp.f_off;
            }
        }
        const float Ff = (float)F;
        if (OUT & 1)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(Ff), fr, l * 4, 0, kNontemporal);
        if (OUT & 2)
            __builtin_amdgcn_raw_buffer_store_b8(frame_code(Ff), ur, l, 0, kNontemporal);
    }
}

// Phase B over frames [jj0, jj1) of one segment (at most 64: kt of frame jj
// is lane jj - jj0 of ktv); frow / urow point at the tile's piece of frame
// jj0 (`fbytes` / `ubytes` of it on the sensor) and advance.
template <int PPT, int NB, int BK, bool LAZY, bool CLAMP, int OUT>
__device__ __forceinline__ void walk_frames(const MethodParams& mp, Pixels<PPT>& px, int jj0, int jj1,
                                            double ktv, const double* chg_S, const double* chg_A,
                                            const uint16_t* chg_j, float*& frow, uint8_t*& urow,
                                            int64_t npix, uint32_t fbytes, uint32_t ubytes)
{
    for (int jj = jj0; jj < jj1; ++jj) {
        const double kt = LAZY ? 0.0 : readlane_f64(ktv, jj - jj0);
        const __amdgpu_buffer_rsrc_t fr = row_rsrc((OUT & 1) ? (void*)frow : nullptr, fbytes);
        const __amdgpu_buffer_rsrc_t ur = row_rsrc((OUT & 2) ? (void*)urow : nullptr, ubytes);
        frame_step<PPT, NB, BK, LAZY, CLAMP, OUT>(mp, px, jj, kt, chg_S, chg_A, chg_j, fr, ur);
        if (OUT & 1)
            frow += npix;
        if (OUT & 2)
            urow += npix;
    }
}

// Phase B over the nfw frames of one segment; ktv0 / ktv1 hold k (t_f - t_b)
// of frames lane and 64 + lane (exponential decay: exp(-k (t_f - t_b))).
template <int PPT, int NB, int BK, bool LAZY, bool CLAMP, int OUT>
__device__ __forceinline__ void walk_segment(const MethodParams& mp, Pixels<PPT>& px, int nfw,
                                             double ktv0, double ktv1, const double* chg_S,
                                             const double* chg_A, const uint16_t* chg_j,
                                             float* frow, uint8_t* urow, int64_t npix,
                                             uint32_t fbytes, uint32_t ubytes)
{
    walk_frames<PPT, NB, BK, LAZY, CLAMP, OUT>(mp, px, 0, min(nfw, kWave), ktv0, chg_S, chg_A,
                                               chg_j, frow, urow, npix, fbytes, ubytes);
    if (nfw > kWave)
        walk_frames<PPT, NB, BK, LAZY, CLAMP, OUT>(mp, px, kWave, nfw, ktv1, chg_S, chg_A, chg_j,
                                                   frow, urow, npix, fbytes, ubytes);
}

// Output mode of a call: 0-2 decayed snapshots (FP32, 8-bit, both), 3-5 the
// same with the clamp, 6-8 lazy.
__device__ __forceinline__ int walk_mode(const MethodParams& mp, const FrameOut& fo)
{
    const int out = (fo.frames && fo.frames_u8) ? 2 : (fo.frames ? 0 : 1);
    return (mp.lazy ? 6 : (mp.need_clamp ? 3 : 0)) + out;
}

template <int PPT, int NB, int BK>
__device__ __forceinline__ void walk_dispatch(int mode, const MethodParams& mp, Pixels<PPT>& px,
                                              int nfw, double ktv0, double ktv1,
                                              const double* chg_S, const double* chg_A,
                                              const uint16_t* chg_j, float* frow, uint8_t* urow,
                                              int64_t npix, uint32_t fbytes, uint32_t ubytes)
{
#define ESI_WALK(L, C, O)                                                                     \
    walk_segment<PPT, NB, BK, L, C, O>(mp, px, nfw, ktv0, ktv1, chg_S, chg_A, chg_j, frow, urow, \
                                   npix, fbytes, ubytes)
    switch (mode) {
    case 0: ESI_WALK(false, false, 1); break;
    case 1: ESI_WALK(false, false, 2); break;
    case 2: ESI_WALK(false, false, 3); break;
    case 3: ESI_WALK(false, true, 1); break;
    case 4: ESI_WALK(false, true, 2); break;
    case 5: ESI_WALK(false, true, 3); break;
    case 6: ESI_WALK(true, false, 1); break;
    case 7: ESI_WALK(true, false, 2); break;
    default: ESI_WALK(true, false, 3); break;
    }
#undef ESI_WALK
}

// Scalars that place one chunk: its record window [cs, cs + avail), the
// times of the window's last record and of the record after it, and the
// frame times that bound its segment.
struct ChunkCtl {
    uint32_t avail;
    int64_t t_first;          // time of the window's first record (0 if none)
    int64_t t_last, t_after;  // t_after = INT64_MAX when the window ends the tile
    int64_t tb, tf_hi;        // frame j and frame min(j + kFrameGroup, nf) - 1
};

template <int CHUNK>
__device__ __forceinline__ ChunkCtl chunk_ctl(const uint64_t* records, uint32_t cs, uint32_t re,
                                              int64_t t_ref, const FrameOut& fo, int j)
{
    ChunkCtl c;
    c.avail = min((uint32_t)CHUNK, re - cs);
    c.t_first = c.avail ? t_ref + record_dt(load_const(records, cs)) : 0;
    c.t_last = c.avail ? t_ref + record_dt(load_const(records, cs + c.avail - 1)) : 0;
    c.t_after = (cs + c.avail < re) ? t_ref + record_dt(load_const(records, cs + c.avail)) : INT64_MAX;
    c.tb = (j < fo.nf) ? load_const(fo.t_frames, j) : 0;
    c.tf_hi = (j < fo.nf) ? load_const(fo.t_frames, min(j + kFrameGroup, fo.nf) - 1) : 0;
    return c;
}

// One pixel per thread: five workgroups per CU (at most 96 VGPRs, 32 KB of
// LDS each), so that a 640x480 sensor's 1200 tiles are all resident at once.
// Two pixels per thread: four (at most 128 VGPRs, 40 KB).  Four pixels: two
// (at most 256 VGPRs; the batched kernel holds the next tile's state besides
// its own).  (Tiles of 512 pixels as 512 threads x 1 pixel ran 7% slower than
// 256 x 2 on the 1280x720 spoke workload: two workgroups per CU, eight-wave
// barriers.)
template <int PPT, int NB, bool BIG = false>
constexpr int min_blocks_per_cu()
{
    return PPT == 1 ? 5 : PPT == 2 ? (BIG ? 3 : 4) : PPT == 4 ? 2 : 1;
}

// A tile's record window [rs, re) in its bucket and the call's time origin
// (scalar loads; a batched workgroup loads the next tile's while it works on
// the current one).
struct TileBounds {
    uint32_t rs, re;
    int64_t t_ref;
};

__device__ __forceinline__ TileBounds tile_bounds(const uint32_t* table, const uint32_t* total,
                                                  const int64_t* ev_t, int K, int tile)
{
    TileBounds tb{0, 0, 0};
    if (table) {
        tb.rs = load_const(table, tile);
        tb.re = (tile + 1 < K) ? load_const(table, tile + 1) : load_const(total, 0);
        tb.t_ref = load_const(ev_t, 0);
    }
    return tb;
}

// PPT consecutive 16-bit counters as one LDS word (2, 4, 8 or 16 bytes).
template <int PPT>
struct CounterWord;
template <>
struct CounterWord<1> {
    using T = uint16_t;
    __device__ static uint32_t get(T v, int) { return v; }
    __device__ static void set(T& v, int, uint32_t x) { v = (uint16_t)x; }
};
template <>
struct CounterWord<2> {
    using T = uint32_t;
    __device__ static uint32_t get(T v, int i) { return (v >> (16 * i)) & 0xFFFFu; }
    __device__ static void set(T& v, int i, uint32_t x) { v |= (x & 0xFFFFu) << (16 * i); }
};
template <>
struct CounterWord<4> {
    using T = uint64_t;
    __device__ static uint32_t get(T v, int i) { return (uint32_t)(v >> (16 * i)) & 0xFFFFu; }
    __device__ static void set(T& v, int i, uint32_t x) { v |= (uint64_t)(x & 0xFFFFu) << (16 * i); }
};
template <>
struct CounterWord<8> {
    using T = uint4;
    __device__ static uint32_t get(const T& v, int i)
    {
        const uint32_t w = i < 2 ? v.x : i < 4 ? v.y : i < 6 ? v.z : v.w;
        return (w >> (16 * (i & 1))) & 0xFFFFu;
    }
    __device__ static void set(T& v, int i, uint32_t x)
    {
        const uint32_t b = (x & 0xFFFFu) << (16 * (i & 1));
        if (i < 2)
            v.x |= b;
        else if (i < 4)
            v.y |= b;
        else if (i < 6)
            v.z |= b;
        else
            v.w |= b;
    }
};

// One tile's stored state (S as its FP32 pair, T, N, P) per pixel slot,
// loaded by the batched kernel while the previous tile finishes.
template <int PPT>
struct TileState {
    float s_hi[PPT], s_lo[PPT];
    int64_t T[PPT];
    uint32_t N[PPT];
    int32_t P[PPT];
};

template <int PPT, int NB>
__device__ __forceinline__ void load_tile_state(const StateDev& st, int tile, TileState<PPT>& ts)
{
    const int64_t q0 = (int64_t)tile * (NB * PPT) + threadIdx.x;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * NB;
        const bool in = q < st.npix;
        ts.s_hi[i] = in ? st.S_hi[q] : 0.0f;
        ts.s_lo[i] = in ? st.S_lo[q] : 0.0f;
        ts.T[i] = in ? st.T[q] : 0;
        ts.N[i] = in ? st.N[q] : 0u;
        ts.P[i] = in ? st.P[q] : 0;
    }
}

// No state loaded ahead: the body loads its own.
struct NoPrefetch {
    __device__ void operator()() const {}
};

// SCAN: phase A's wave scan of long runs compiled in (section 3b).
// EARLY_NP: N and P are loaded with S and T at the start of the tile, so that
// its end waits for no load (batched calls, whose workgroups go on to the
// next tile, and the larger tiles); otherwise they are read and updated at the
// write-back (one pixel per thread, one tile per workgroup: loading them
// first only lengthens the first wait).
template <int PPT, int NB, int BK, bool SCAN, bool EARLY_NP, bool PRE = false,
          typename Next = NoPrefetch, bool BIG = false>
__device__ __forceinline__ void integrate_body(const uint64_t* __restrict__ records,
                                               const uint32_t* __restrict__ table,
                                               const uint32_t* __restrict__ total,
                                               const int64_t* __restrict__ ev_t, int K,
                                               StateDev st, MethodParams mp, FrameOut fo,
                                               DiagDev* diag, int tile, const TileBounds& tb,
                                               const TileState<PPT>* pre = nullptr,
                                               Next next = Next{})
{
    using Cfg = TileCfg<PPT, NB, BIG>;
    constexpr int TILE = Cfg::TILE;
    constexpr int WAVES = Cfg::WAVES;
    constexpr int CHUNK = Cfg::CHUNK;
    constexpr int PER_WAVE = Cfg::PER_WAVE;
    constexpr int STEPS = Cfg::STEPS;
    static_assert(kFrameGroup <= NB, "one frame time per thread");
    static_assert(kFrameGroup < 128, "segment frame index in 7 bits");
    static_assert(PER_WAVE % kWave == 0, "chunk size");
    static_assert(CHUNK < 65536, "16-bit counters");
    static_assert((1 << Cfg::TILE_BITS) == TILE, "tile key bits");
    // (one spare entry each: the change lists' reads one past a last entry)
    __shared__ uint64_t sorted[CHUNK + 1];  // records sorted by pixel (frame index over the pixel field)
    __shared__ double ktvs[CHUNK + 1];      // k (t - t_first) of the sorted records; then
    double* chg_S = ktvs;                 // change lists: S / (s_max - s_min) after the change
    __shared__ uint16_t chg_j[CHUNK + TILE];  // change lists: frame index in the segment
    __shared__ __align__(16) uint16_t cnt[WAVES][TILE];
    // representative lane per (wave, pixel) and lane masks per wave for the
    // LDS stable rank (one and two pixels per thread; larger tiles, whose
    // threads hold more registers, use the ballot rank)
    constexpr bool kOrRank = PPT <= 2;
    __shared__ uint8_t rrep[WAVES][kOrRank ? TILE : 1];
    __shared__ uint64_t rgroup[WAVES][kOrRank ? kWave : 1];
    __shared__ int64_t tfl[kFrameGroup];  // frame times of the segment
    __shared__ uint32_t scan_w[WAVES];
    __shared__ uint32_t cut_w[WAVES];
    double* chg_A = reinterpret_cast<double*>(sorted);  // change lists: A after the change

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int64_t q0 = (int64_t)tile * TILE + tid;
    const int64_t npix = st.npix;
    const int nf = fo.nf;
    const int mode = walk_mode(mp, fo);
    // pixels of the tile on the sensor: the frame stores' range
    const uint32_t tile_px = (uint32_t)min((int64_t)TILE, npix - (int64_t)tile * TILE);

    Pixels<PPT> px;
    bool in[PPT];
    px.touched = 0u;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * NB;
        in[i] = q < npix;
        if constexpr (PRE) {
            px.S[i] = (double)pre->s_hi[i] + (double)pre->s_lo[i];
            px.T[i] = pre->T[i];
            px.N[i] = pre->N[i];
            px.P[i] = pre->P[i];
        } else {
            px.S[i] = in[i] ? (double)st.S_hi[q] + (double)st.S_lo[q] : 0.0;
            px.T[i] = in[i] ? st.T[q] : 0;
            px.N[i] = (EARLY_NP && in[i]) ? st.N[q] : 0u;
            px.P[i] = (EARLY_NP && in[i]) ? st.P[q] : 0;
        }
    }

    // the tile's records [rs, re)
    const uint32_t rs = tb.rs, re = tb.re;
    const int64_t t_ref = tb.t_ref;

    int j = 0;  // first frame of the segment (uniform)
    uint32_t cs = rs;
    bool bad = false;
    ChunkCtl c = chunk_ctl<CHUNK>(records, cs, re, t_ref, fo, j);

    // records of the first chunk and the first frame times; clamped indices,
    // no select on loaded values, so all loads stay in flight
    uint64_t rr[STEPS], rr_next[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
        rr[s] = 0;
    if (c.avail > 0) {
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            rr[s] = records[cs + min((uint32_t)(wave * PER_WAVE + s * kWave + lane), c.avail - 1u)];
    }
    int64_t tfv = 0, tfv_next = 0;
    if (nf > 0)
        tfv = fo.t_frames[min(tid, nf - 1)];
    // nothing may be pending on these at the loop head, or the compiler waits
    // there for everything outstanding, frame stores included
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);

    while (cs < re || j < nf) {
        // ---- chunk and segment bounds (uniform) ----
        const int jmax0 = min(j + kFrameGroup, nf);
        int jmax = jmax0;
        if (jmax > j + 1 &&
            mp.k * (double)(c.tf_hi - c.tb) > (BK == kDecayExp ? kMaxSegmentExp : kMaxSegmentDecay))
            jmax = j + 1;
        const int64_t tf_lim = (jmax < nf) ? (jmax == jmax0 ? c.tf_hi : c.tb) : INT64_MAX;
        uint32_t cn;
        if (c.avail == 0) {
            cn = 0;
        } else if (jmax == nf || c.t_last <= tf_lim) {
            cn = c.avail;
        } else {
            // the segment is full before the window ends: the chunk stops at
            // the first record later than the segment's last frame (each wave
            // finds it among the records it holds)
            uint32_t first = (uint32_t)CHUNK;
#pragma unroll
            for (int s = STEPS - 1; s >= 0; --s) {
                const uint32_t base = (uint32_t)(wave * PER_WAVE + s * kWave);
                const bool over = base + lane < c.avail && t_ref + record_dt(rr[s]) > tf_lim;
                const uint64_t m = __ballot(over);
                if (m)
                    first = base + (uint32_t)__ffsll((long long)m) - 1u;
            }
            if (lane == 0)
                cut_w[wave] = first;
            __syncthreads();
            cn = c.avail;
#pragma unroll
            for (int w = 0; w < WAVES; ++w)
                cn = min(cn, cut_w[w]);
        }
        const uint32_t ce = cs + cn;
        // frames the chunk completes: all of the segment unless the record
        // after the chunk (t_after) comes before its end
        const bool search = (cn == c.avail) && (ce < re);
        const int64_t tb = c.tb;

        // prefetch the next chunk's records (before this chunk's frame stores)
        const uint32_t avail1 = min((uint32_t)CHUNK, re - ce);
        if (avail1 > 0) {
#pragma unroll
            for (int s = 0; s < STEPS; ++s)
                rr_next[s] = records[ce + min((uint32_t)(wave * PER_WAVE + s * kWave + lane), avail1 - 1u)];
        }

        // the segment's frame times; the visible state before this chunk's
        // events
        if (tid < kFrameGroup)
            tfl[tid] = tfv;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            px.Sv[i] = px.S[i] * mp.inv_range;
            px.Av[i] = (BK == kDecayExp) ? exp(mp.k * (double)(px.T[i] - tb))
                                         : __fma_rn(mp.k, (double)(px.T[i] - tb), 1.0);
        }
        uint32_t rank[STEPS];
        if (cn > 0) {
            // 2a. stable ranks inside the wave (the ballot rank of the larger
            // tiles skips a wave step with no record of the chunk: sparse
            // chunks fill only their first steps)
            for (int k = lane; k < TILE / 4; k += kWave)  // four counters per store
                reinterpret_cast<uint64_t*>(cnt[wave])[k] = 0;
            wave_sync();
#pragma unroll
            for (int s = 0; s < STEPS; ++s) {
                rank[s] = 0;
                if (!kOrRank && (uint32_t)(wave * PER_WAVE + s * kWave) >= cn)  // uniform
                    continue;
                const uint32_t c_ = (uint32_t)(wave * PER_WAVE + s * kWave + lane);
                const uint32_t key = record_lpx(rr[s]) & (TILE - 1);
                if (kOrRank)
                    rank[s] = wave_stable_rank_or(c_ < cn, key, cnt[wave], rrep[wave], rgroup[wave]);
                else
                    rank[s] = wave_stable_rank<Cfg::TILE_BITS>(c_ < cn, key, cnt[wave]);
            }
        }
        __syncthreads();
        // decay bases k (t_f - t_b) of the segment's frames, one per lane:
        // frames lane and 64 + lane
        double ktv0 = mp.k * (double)(tfl[lane] - tb);
        double ktv1 = mp.k * (double)(tfl[min(kWave + lane, kFrameGroup - 1)] - tb);
        if (BK == kDecayExp) {  // the frames' factors exp(-k (t_f - t_b))
            ktv0 = exp(-ktv0);
            ktv1 = exp(-ktv1);
        }
        int j_end = jmax;
        if (search)
            j_end = j + frames_before(tfl, jmax - j, c.t_after);
        if (cn == 0 && j_end == j)
            j_end = min(j + 1, nf);  // progress even with unsorted frame times
        const int nfw = j_end - j;

        // prefetch the next segment's frame times and the next chunk's bounds
        if (j_end < nf)
            tfv_next = fo.t_frames[min(j_end + tid, nf - 1)];
        const ChunkCtl c1 = chunk_ctl<CHUNK>(records, ce, re, t_ref, fo, j_end);

        if (cn > 0) {
            // 2b. the segment frame of each record (the number of segment
            // frames earlier than it), kept with its rank.  A wave step's 64
            // records are consecutive in the tile's array order, so (events
            // and frames sorted) their frames lie between those of the
            // step's first and last record.  Those two counts come from
            // ballots over the segment's frame times, one per lane (frames
            // lane and 64 + lane); each record then searches its step's
            // range by binary lifting, the steps side by side with as many
            // halvings as the widest range needs (none when no frame time
            // falls inside any step).  Unsorted input still gives a count in
            // [0, nfw].
            {
                const int64_t f0 = tfl[lane];
                const int64_t f1 = tfl[min(kWave + lane, kFrameGroup - 1)];
                const bool v0 = lane < nfw, v1 = kWave + lane < nfw;
                auto frames_below = [&](int64_t t) -> int {  // t uniform
                    int c = __popcll(__ballot(v0 && f0 < t));
                    if (nfw > kWave)
                        c += __popcll(__ballot(v1 && f1 < t));
                    return c;
                };
                int jc[STEPS], hi[STEPS];  // hi uniform
                int64_t tr[STEPS];
                int span = 0;
#pragma unroll
                for (int s = 0; s < STEPS; ++s) {
                    tr[s] = t_ref + record_dt(rr[s]);
                    const int ca = frames_below(readlane_i64(tr[s], 0));
                    const int cz = frames_below(readlane_i64(tr[s], kWave - 1));
                    jc[s] = min(ca, cz);
                    hi[s] = max(ca, cz);
                    span = max(span, hi[s] - jc[s]);
                }
                if (span > 0) {
                    for (int step = 1 << (31 - __clz(span)); step >= 1; step >>= 1) {
#pragma unroll
                        for (int s = 0; s < STEPS; ++s) {
                            const int probe = jc[s] + step;
                            const int64_t v = tfl[max(min(probe, hi[s]) - 1, 0)];
                            jc[s] = (probe <= hi[s] && v < tr[s]) ? probe : jc[s];
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < STEPS; ++s)
                    rank[s] |= (uint32_t)jc[s] << 16;
            }
            // 2c. exclusive scan over (pixel, wave), pixel-major
            // (each thread's PPT consecutive counters of a wave are read and
            // written as one LDS access of 2 PPT bytes)
            {
                using Word = CounterWord<PPT>;
                typename Word::T cw[WAVES];
                uint32_t sum = 0;
#pragma unroll
                for (int w = 0; w < WAVES; ++w) {
                    cw[w] = reinterpret_cast<const typename Word::T*>(cnt[w])[tid];
#pragma unroll
                    for (int i = 0; i < PPT; ++i)
                        sum += Word::get(cw[w], i);
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
                typename Word::T out[WAVES];
#pragma unroll
                for (int w = 0; w < WAVES; ++w)
                    out[w] = typename Word::T{};
#pragma unroll
                for (int i = 0; i < PPT; ++i)
#pragma unroll
                    for (int w = 0; w < WAVES; ++w) {
                        Word::set(out[w], i, run);
                        run += Word::get(cw[w], i);
                    }
#pragma unroll
                for (int w = 0; w < WAVES; ++w)
                    reinterpret_cast<typename Word::T*>(cnt[w])[tid] = out[w];
            }
            __syncthreads();
            // 2d. scatter into pixel order, the frame index over the pixel
            // field, and each record's k (t - t_first) (every index is
            // checked, so that a broken invariant can only flag an error,
            // never leave the chunk)
            const int64_t dt_first = c.t_first - t_ref;
#pragma unroll
            for (int s = 0; s < STEPS; ++s) {
                const uint32_t c_ = (uint32_t)(wave * PER_WAVE + s * kWave + lane);
                if (c_ < cn) {
                    const uint32_t at = (uint32_t)cnt[wave][record_lpx(rr[s]) & (TILE - 1)] + (rank[s] & 0xFFFFu);
                    if (at < cn) {
                        sorted[at] = (rr[s] & ~kLpxMask) | ((uint64_t)(rank[s] >> 16) << 48);
                        // k (t - t_first) with the frame index and a
                        // negative-polarity bit in its 8 lowest mantissa bits
                        // (a relative change below 2^-44)
                        const double kt = mp.k * (double)(record_dt(rr[s]) - dt_first);
                        const uint64_t kb = ((uint64_t)__double_as_longlong(kt) & ~(uint64_t)0xFF) |
                                            (uint64_t)(rank[s] >> 16) |
                                            ((uint64_t)(record_pos(rr[s]) ^ 1u) << 7);
                        ktvs[at] = __longlong_as_double((long long)kb);
                    } else {
                        bad = true;
                    }
                }
            }
            __syncthreads();

            // 3. phase A: each pixel's events of the chunk in array order
            // (Alg. 2).  With A = 1 + k (T - t_first) per pixel and
            // kt = k (t - t_first) per event, the base of Eq. (4) is
            // u = clamp(A - kt, 0, 1) = max(1 - k max(t - T, 0), 0), and after
            // the event A = 1 + kt.  N, P and T are settled once per run.
            // The change list keeps, per segment frame jc that first includes
            // some event, the state after the last such event, written once
            // the next event belongs to a later frame (or the run ends); its
            // decay base is A + k (t_first - t_b) (exponential decay: the
            // factor exp of that minus 1).  Entries go over the
            // pixel's own slots of `sorted`/`ktvs`, behind the read position
            // (an entry written at event e lands at or before e - 1, while the
            // loop has already read e + 1).  Events after the segment
            // (jc == nfw) make no entry.
            const double dA = mp.k * (double)(c.t_first - tb);
            const uint64_t c_bits = (uint64_t)__double_as_longlong(mp.C);
            const uint32_t c_hi = (uint32_t)(c_bits >> 32), c_lo = (uint32_t)c_bits;
            // clamp bounds in canonical form once, not on every event
            const double s_min = __builtin_canonicalize(mp.s_min);
            const double s_max = __builtin_canonicalize(mp.s_max);
            // runs longer than mp.scan_run are left to the wave's scan (3b):
            // only their lane masks (scalar registers) live across the loop
            uint64_t lmask[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int l = tid + i * NB;
                const uint32_t end = min((l + 1 < TILE) ? (uint32_t)cnt[0][l + 1] : cn, cn);
                const uint32_t beg = min((uint32_t)cnt[0][l], end);
                const bool lng = SCAN && end - beg > (uint32_t)mp.scan_run;
                lmask[i] = __ballot(lng);
                if (lng)
                    continue;
                double S = px.S[i];
                double A = __fma_rn(mp.k, (double)(px.T[i] - c.t_first), 1.0);
                uint32_t w = beg, nneg = 0;
                int jc_prev = nfw;  // frame of the events applied so far (nfw: none)
                auto run = [&](auto decay_then_add) {
                    // the next event's kt is read one iteration ahead
                    // (indices up to end <= CHUNK: the spare entry)
                    double kt_next = ktvs[beg];
                    for (uint32_t e = beg; e < end; ++e) {
                        const double kt = kt_next;
                        kt_next = ktvs[e + 1];
                        const uint32_t low = (uint32_t)__double_as_longlong(kt);
                        const int jc = (int)(low & 0x7Fu);
                        const uint32_t neg = (low >> 7) & 1u;
                        if (jc != jc_prev && jc_prev < nfw) {
                            // the group of event e - 1 is complete
                            chg_S[w] = S * mp.inv_range;
                            chg_A[w] = (BK == kDecayExp) ? exp(A + dA - 1.0) : A + dA;
                            chg_j[w + l] = (uint16_t)jc_prev;
                            ++w;
                        }
                        jc_prev = jc;
                        const double d = decay_from_base<BK>(A - kt, mp.b);
                        // +C or -C: the polarity flips the sign bit of C
                        const double s = __hiloint2double((int)(c_hi + (neg << 31)), (int)c_lo);
                        if constexpr (decltype(decay_then_add)::value)
                            S = fmin(fmax(__fma_rn(S, d, s), s_min), s_max);
                        else
                            S = fmin(fmax((S + s) * d, s_min), s_max);
                        A = 1.0 + kt;
                        nneg += neg;
                    }
                };
                if (mp.decay_then_add)
                    run(std::true_type{});
                else
                    run(std::false_type{});
                if (end > beg) {
                    const uint64_t rl = sorted[end - 1];  // the run's last event
                    if (jc_prev < nfw) {
                        chg_S[w] = S * mp.inv_range;
                        chg_A[w] = (BK == kDecayExp) ? exp(A + dA - 1.0) : A + dA;
                        chg_j[w + l] = (uint16_t)jc_prev;
                        ++w;
                    }
                    px.T[i] = t_ref + record_dt(rl);
                }
                px.S[i] = S;
                px.N[i] += end - beg;
                px.P[i] += (int32_t)(end - beg) - 2 * (int32_t)nneg;
                px.touched |= (end > beg ? 1u : 0u) << i;
                chg_j[w + l] = 0xFFFF;  // end of the list
                // the first change's frame; eo at its entry, jo at the frame
                // index after it
                px.jn[i] = chg_j[beg + (uint32_t)l];
                px.eo[i] = 8u * beg;
                px.jo[i] = 2u * (beg + (uint32_t)l + 1u);
            }

            // 3b. each run longer than mp.scan_run, one after the other, by
            // the whole wave of its pixel, 64 events at a time: lane e takes
            // event b0 + e and builds its map (the decay from the previous
            // event's time, lane e - 1's kt, or the pixel's A for the run's
            // first event), the wave scans the maps (wave_scan), and lane e
            // applies the composed map to the state before the block, which
            // gives the state after its event.  The change-list entries are
            // the events whose next event belongs to a later frame (or that
            // end the run), at positions counted with a ballot; they land at
            // or before their own event, behind every read of the block, and
            // the next block only reads later events.
#pragma unroll
            for (int i = 0; i < (SCAN ? PPT : 0); ++i) {
                uint64_t todo = lmask[i];
                while (todo) {
                    const int owner = (int)__builtin_ctzll(todo);
                    todo &= todo - 1ull;
                    const uint32_t l = (uint32_t)(tid - lane + owner + i * NB);
                    const uint32_t end = min((l + 1 < TILE) ? (uint32_t)cnt[0][l + 1] : cn, cn);
                    const uint32_t beg = min((uint32_t)cnt[0][l], end);
                    double S = readlane_f64(px.S[i], owner);
                    const int64_t T0 =
                        (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                                       (int)((uint64_t)px.T[i] >> 32), owner) << 32) |
                                  (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)px.T[i], owner));
                    double A = __fma_rn(mp.k, (double)(T0 - c.t_first), 1.0);
                    // the run's last event, read before any entry can overwrite it
                    const int64_t t_last = t_ref + record_dt(sorted[end - 1]);
                    uint32_t w = beg, nneg = 0;
                    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
                        const uint32_t e = b0 + (uint32_t)lane;
                        const bool valid = e < end;
                        const bool has_next = e + 1u < end;
                        const double kt = ktvs[valid ? e : b0];
                        const double kt_n = ktvs[has_next ? e + 1u : b0];
                        const uint32_t low = (uint32_t)__double_as_longlong(kt);
                        const int jc = (int)(low & 0x7Fu);
                        const uint32_t neg = (low >> 7) & 1u;
                        const int jc_n =
                            has_next ? (int)((uint32_t)__double_as_longlong(kt_n) & 0x7Fu) : -1;
                        // the previous event's kt (wave_shr:1); lane 0 takes A
                        const double kt_p = dpp_f64<0x138>(0.0, kt);
                        const double A_p = (lane == 0) ? A : 1.0 + kt_p;
                        const double d = decay_from_base<BK>(A_p - kt, mp.b);
                        const double sc = __hiloint2double((int)(c_hi + (neg << 31)), (int)c_lo);
                        ClampAffine f = clamp_affine_identity();
                        if (valid) {
                            f.a = d;
                            f.b = mp.decay_then_add ? sc : d * sc;
                            f.lo = s_min;
                            f.hi = s_max;
                        }
                        f = wave_scan(f);
                        const double S_e = apply(f, S);
                        const bool ge = valid && jc < nfw && jc_n != jc;
                        const uint64_t gm = __ballot(ge);
                        if (ge) {
                            const uint32_t at = w + (uint32_t)__popcll(gm & ((1ull << lane) - 1ull));
                            const double A_e = 1.0 + kt;
                            chg_S[at] = S_e * mp.inv_range;
                            chg_A[at] = (BK == kDecayExp) ? exp(A_e + dA - 1.0) : A_e + dA;
                            chg_j[at + l] = (uint16_t)jc;
                        }
                        const int last = (int)min(end - b0, (uint32_t)kWave) - 1;
                        S = readlane_f64(S_e, last);
                        A = 1.0 + readlane_f64(kt, last);
                        w += (uint32_t)__popcll(gm);
                        nneg += (uint32_t)__popcll(__ballot(valid && neg != 0u));
                    }
                    if (lane == owner) {
                        px.S[i] = S;
                        px.T[i] = t_last;
                        px.N[i] += end - beg;
                        px.P[i] += (int32_t)(end - beg) - 2 * (int32_t)nneg;
                        px.touched |= 1u << i;
                        chg_j[w + l] = 0xFFFF;
                        px.jn[i] = chg_j[beg + l];
                        px.eo[i] = 8u * beg;
                        px.jo[i] = 2u * (beg + l + 1u);
                    }
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < PPT; ++i)
                px.jn[i] = kNever;
        }

        // Wait for the prefetched records and frame times now: this also
        // drains the frame stores of the previous segment (one counter covers
        // loads and stores), which have had the whole sort to complete.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        // the next tile's state, loaded during this tile's last frames
        if constexpr (PRE) {
            if (!(ce < re || j_end < nf))
                next();
        }
        // 4. phase B: the frames this chunk completes
        if (nfw > 0) {
            const size_t base = (size_t)j * (size_t)fo.stride + (size_t)tile * TILE;
            walk_dispatch<PPT, NB, BK>(mode, mp, px, nfw, ktv0, ktv1, chg_S, chg_A, chg_j,
                                   fo.frames ? fo.frames + base : nullptr,
                                   fo.frames_u8 ? fo.frames_u8 + base : nullptr, fo.stride,
                                   4u * tile_px, tile_px);
        }
        j = j_end;
        cs = ce;
        c = c1;
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            rr[s] = rr_next[s];
        tfv = tfv_next;
        __syncthreads();  // LDS is reused by the next chunk
    }

#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * NB;
        // a pixel without events in this call keeps its stored state as it
        // is (S, T unchanged, no re-rounding), so only touched pixels write
        if (in[i] && ((px.touched >> i) & 1u)) {
            const float hi = (float)px.S[i];
            st.S_hi[q] = hi;
            st.S_lo[q] = (float)(px.S[i] - (double)hi);
            st.T[q] = px.T[i];
            st.N[q] = EARLY_NP ? px.N[i] : st.N[q] + px.N[i];
            st.P[q] = EARLY_NP ? px.P[i] : st.P[q] + px.P[i];
        }
    }
    if (bad)
        atomicOr(&diag->flags, 8u);  // ESI_DIAG_INTERNAL: never expected
    // frame times must be non-decreasing; the first workgroup checks
    if (tile == 0) {
        bool unsorted = false;
        for (int jj = 1 + tid; jj < nf; jj += NB)
            unsorted |= fo.t_frames[jj] < fo.t_frames[jj - 1];
        if (unsorted)
            atomicOr(&diag->flags, 2u);  // ESI_DIAG_FRAMES_UNSORTED
    }
}

// One workgroup per tile of one call.  Workgroups start in index order, so
// with `order` (the tiles by event count, largest first) the longest tiles
// start first and the short ones fill the end of the launch.
template <int PPT, int NB, int BK, bool SCAN, bool BIG = false>
__global__ __launch_bounds__(NB, (min_blocks_per_cu<PPT, NB, BIG>())) void k_integrate(
    const uint64_t* __restrict__ records, const uint32_t* __restrict__ table,
    const uint32_t* __restrict__ total, const int64_t* __restrict__ ev_t,
    const uint32_t* __restrict__ order, int K, StateDev st, MethodParams mp, FrameOut fo,
    DiagDev* diag)
{
    const int tile = order ? (int)load_const(order, blockIdx.x) : (int)blockIdx.x;
    integrate_body<PPT, NB, BK, SCAN, (PPT >= 2), false, NoPrefetch, BIG>(
        records, table, total, ev_t, K, st, mp, fo, diag, tile,
        tile_bounds(table, total, ev_t, K, tile));
}

// Batched: the tiles of items [i0, i1) (one tile size and decay kind), work
// indices [tile0, tile0 + tiles) laid out item by item; each workgroup takes
// a contiguous share of them, so it looks its item up once and then only
// steps to the next item.
template <int PPT, int NB, int BK, bool SCAN, bool BIG = false>
__global__ __launch_bounds__(NB, (min_blocks_per_cu<PPT, NB, BIG>())) void kb_integrate(
    BatchDev b, int i0, int i1, uint32_t tile0, uint32_t tiles)
{
    const uint32_t per = (tiles + gridDim.x - 1) / gridDim.x;
    uint32_t w = tile0 + blockIdx.x * per;
    const uint32_t w_end = min(tile0 + tiles, w + per);
    if (w >= w_end)
        return;
    // the item holding w: the last with tile_base <= w
    int lo = i0, hi = i1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (load_const(b.tile_base, mid) <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    int i = lo;
    uint32_t first = load_const(b.tile_base, i), next = load_const(b.tile_base, i + 1);
    // the larger tiles load each next tile's state while the current one
    // finishes (its last frames and write-back)
    constexpr bool kPre = PPT >= 4;
    TileState<PPT> cur, nxt;
    bool have = false;
    for (; w < w_end; ++w) {
        while (w >= next) {
            ++i;
            first = next;
            next = load_const(b.tile_base, i + 1);
        }
        const BatchItem& it = b.items[i];
        const int tile = (int)(w - first);
        if constexpr (kPre) {
            if (!have)
                load_tile_state<PPT, NB>(it.st, tile, cur);
            // the tile after this one: its item and index
            const bool more = w + 1 < w_end;
            int i2 = i;
            uint32_t f2 = first;
            if (more && w + 1 >= next) {
                i2 = i + 1;
                f2 = next;
                while (w + 1 >= load_const(b.tile_base, i2 + 1)) {
                    ++i2;
                    f2 = load_const(b.tile_base, i2);
                }
            }
            bool loaded = false;
            auto prefetch = [&]() {
                if (more) {
                    load_tile_state<PPT, NB>(b.items[i2].st, (int)(w + 1 - f2), nxt);
                    loaded = true;
                }
            };
            integrate_body<PPT, NB, BK, SCAN, true, true>(
                it.cs.records, it.cs.table, it.cs.total, it.ev.t, it.K, it.st, it.mp, it.fo,
                it.diag, tile, tile_bounds(it.cs.table, it.cs.total, it.ev.t, it.K, tile), &cur,
                prefetch);
            if (loaded)
                cur = nxt;
            have = loaded;
        } else {
            integrate_body<PPT, NB, BK, SCAN, true, false, NoPrefetch, BIG>(
                it.cs.records, it.cs.table, it.cs.total, it.ev.t, it.K, it.st, it.mp, it.fo,
                it.diag, tile, tile_bounds(it.cs.table, it.cs.total, it.ev.t, it.K, tile));
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

template <int BK>
__global__ __launch_bounds__(kBlock) void k_snapshot(StateDev st, MethodParams mp, int64_t t_f,
                                                     float* frame, uint8_t* u8)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= st.npix)
        return;
    const double S = (double)st.S_hi[q] + (double)st.S_lo[q];
    const float F = frame_value<BK>(mp, S, st.T[q], t_f);
    if (frame)
        frame[q] = F;
    if (u8)
        u8[q] = frame_code(F);
}

__global__ __launch_bounds__(kBlock) void k_reset(StateDev st, int64_t t0, DiagDev* diag)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < st.npix) {
        st.S_hi[q] = 0.0f;
        st.S_lo[q] = 0.0f;
        st.T[q] = t0;
        st.N[q] = 0;
        st.P[q] = 0;
    }
    if (q == 0 && diag) {
        diag->dropped = 0;
        diag->accepted = 0;
        diag->flags = 0;
    }
}


template <int PPT, int NB, int BK>
hipError_t launch_integrate_t(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                              const CallScratch& cs, const MethodParams& mp, const FrameOut& fo,
                              DiagDev* diag, hipStream_t stream)
{
    const bool has = ev.n > 0;
    // tiles of one pixel per thread leave the scan out when it is off: its
    // code alone slows that kernel (section 3b)
    auto go = [&](auto scan, auto big) {
        hipLaunchKernelGGL((k_integrate<PPT, NB, BK, decltype(scan)::value, decltype(big)::value>),
                           dim3(sc.ntiles), dim3(NB), 0, stream, has ? cs.records : nullptr,
                           has ? cs.table : nullptr, has ? cs.total : nullptr,
                           has ? ev.t : nullptr, (has && sc.ordered) ? cs.order : nullptr,
                           sc.ntiles, st, mp, fo, diag);
    };
    if constexpr (PPT == 2) {
        if (sc.big_chunk) {
            go(std::true_type{}, std::true_type{});
            return hipGetLastError();
        }
    }
    if (PPT == 1 && mp.scan_run == kScanOff)
        go(std::false_type{}, std::false_type{});
    else
        go(std::true_type{}, std::false_type{});
    return hipGetLastError();
}

template <int PPT, int NB>
hipError_t launch_integrate_p(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                              const CallScratch& cs, const MethodParams& mp, const FrameOut& fo,
                              DiagDev* diag, hipStream_t stream)
{
    switch (decay_kind(mp)) {
    case kDecayB1:
        return launch_integrate_t<PPT, NB, kDecayB1>(ev, st, sc, cs, mp, fo, diag, stream);
    case kDecayB2:
        return launch_integrate_t<PPT, NB, kDecayB2>(ev, st, sc, cs, mp, fo, diag, stream);
    case kDecayExp:
        return launch_integrate_t<PPT, NB, kDecayExp>(ev, st, sc, cs, mp, fo, diag, stream);
    default:
        return launch_integrate_t<PPT, NB, kDecayPow>(ev, st, sc, cs, mp, fo, diag, stream);
    }
}

}  // namespace

int integrate_slots(int ppt, bool big)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
        switch (ppt) {
        case 1:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate<1, 256, kDecayB2, true>, 256, 0);
            break;
        case 2:
            e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                          &per_cu, k_integrate<2, 256, kDecayB2, true, true>, 256, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                          &per_cu, k_integrate<2, 256, kDecayB2, true>, 256, 0);
            break;
        case 4:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate<4, 256, kDecayB2, true>, 256, 0);
            break;
        default:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate<8, 256, kDecayB2, true>, 256, 0);
        }
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1 << 30;  // unknown: never ordered
    }
    return std::max(1, cus) * std::max(1, per_cu);
}

int decay_kind(const MethodParams& mp)
{
    if (mp.exp_decay)
        return kDecayExp;
    return mp.b == 1.0 ? kDecayB1 : (mp.b == 2.0 ? kDecayB2 : kDecayPow);
}

hipError_t launch_integrate(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                            const CallScratch& cs, const MethodParams& mp, const FrameOut& fo,
                            DiagDev* diag, hipStream_t stream)
{
    switch (sc.ppt) {
    // 256 threads per tile, 1, 2, 4 or 8 pixels each
    case 1:
        return launch_integrate_p<1, 256>(ev, st, sc, cs, mp, fo, diag, stream);
    case 2:
        return launch_integrate_p<2, 256>(ev, st, sc, cs, mp, fo, diag, stream);
    case 4:
        return launch_integrate_p<4, 256>(ev, st, sc, cs, mp, fo, diag, stream);
    case 8:
        return launch_integrate_p<8, 256>(ev, st, sc, cs, mp, fo, diag, stream);
    default:
        return hipErrorInvalidValue;
    }
}

namespace {

template <int PPT, int BK, bool SCAN, bool BIG = false>
hipError_t launch_integrate_batch_s(const BatchDev& b, int i0, int i1, uint32_t tile0,
                                    uint32_t tiles, hipStream_t stream)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                     kb_integrate<PPT, 256, BK, SCAN, BIG>, 256,
                                                     0) != hipSuccess)
        return hipGetLastError();
    // eight workgroups per slot: contiguous shares, balanced by the
    // dispatcher (64 streams of 10 ms windows: 1, 2, 4, 8, 16 and 32 per slot
    // gave 587, 550, 531, 522, 548 and 582 us per window)
    const uint32_t grid = std::min<uint32_t>(tiles, 8u * (uint32_t)std::max(1, cus * per_cu));
    hipLaunchKernelGGL((kb_integrate<PPT, 256, BK, SCAN, BIG>), dim3(grid), dim3(256), 0, stream,
                       b, i0, i1, tile0, tiles);
    return hipGetLastError();
}

// scan: the items of the launch have the scan on (their class; tiles of
// one pixel per thread only leave it out)
template <int PPT, int BK>
hipError_t launch_integrate_batch_t(const BatchDev& b, int i0, int i1, uint32_t tile0,
                                    uint32_t tiles, bool scan, bool big, hipStream_t stream)
{
    if constexpr (PPT == 2) {
        if (big)
            return launch_integrate_batch_s<PPT, BK, true, true>(b, i0, i1, tile0, tiles, stream);
    }
    if (PPT == 1 && !scan)
        return launch_integrate_batch_s<PPT, BK, false>(b, i0, i1, tile0, tiles, stream);
    return launch_integrate_batch_s<PPT, BK, true>(b, i0, i1, tile0, tiles, stream);
}

template <int PPT>
hipError_t launch_integrate_batch_p(const BatchDev& b, int i0, int i1, uint32_t tile0,
                                    uint32_t tiles, int bk, bool scan, bool big,
                                    hipStream_t stream)
{
    switch (bk) {
    case kDecayB1:
        return launch_integrate_batch_t<PPT, kDecayB1>(b, i0, i1, tile0, tiles, scan, big, stream);
    case kDecayB2:
        return launch_integrate_batch_t<PPT, kDecayB2>(b, i0, i1, tile0, tiles, scan, big, stream);
    case kDecayExp:
        return launch_integrate_batch_t<PPT, kDecayExp>(b, i0, i1, tile0, tiles, scan, big, stream);
    default:
        return launch_integrate_batch_t<PPT, kDecayPow>(b, i0, i1, tile0, tiles, scan, big, stream);
    }
}

}  // namespace

hipError_t launch_integrate_batch(const BatchDev& b, int i0, int i1, uint32_t tile0,
                                  uint32_t tiles, int ppt, int bk, bool scan, bool big,
                                  hipStream_t stream)
{
    if (tiles == 0)
        return hipSuccess;
    switch (ppt) {
    case 1:
        return launch_integrate_batch_p<1>(b, i0, i1, tile0, tiles, bk, scan, big, stream);
    case 2:
        return launch_integrate_batch_p<2>(b, i0, i1, tile0, tiles, bk, scan, big, stream);
    case 4:
        return launch_integrate_batch_p<4>(b, i0, i1, tile0, tiles, bk, scan, big, stream);
    case 8:
        return launch_integrate_batch_p<8>(b, i0, i1, tile0, tiles, bk, scan, big, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_snapshot(const StateDev& st, const MethodParams& mp, int64_t t_f, float* frame,
                           uint8_t* u8, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((st.npix + kBlock - 1) / kBlock);
    switch (decay_kind(mp)) {
    case kDecayB1:
        hipLaunchKernelGGL(k_snapshot<kDecayB1>, dim3(blocks), dim3(kBlock), 0, stream, st, mp,
                           t_f, frame, u8);
        break;
    case kDecayB2:
        hipLaunchKernelGGL(k_snapshot<kDecayB2>, dim3(blocks), dim3(kBlock), 0, stream, st, mp,
                           t_f, frame, u8);
        break;
    case kDecayExp:
        hipLaunchKernelGGL(k_snapshot<kDecayExp>, dim3(blocks), dim3(kBlock), 0, stream, st, mp,
                           t_f, frame, u8);
        break;
    default:
        hipLaunchKernelGGL(k_snapshot<kDecayPow>, dim3(blocks), dim3(kBlock), 0, stream, st, mp,
                           t_f, frame, u8);
    }
    return hipGetLastError();
}

hipError_t launch_reset(const StateDev& st, int64_t t0, DiagDev* diag, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((st.npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(kBlock), 0, stream, st, t0, diag);
    return hipGetLastError();
}

}  // namespace esi
