// integrate.hip -- per-tile integration of the bucketed events and frames.
//
// One workgroup (256 threads) owns a tile of 256 * PPT consecutive pixels;
// thread `tid` owns pixels tid + 256 i (i < PPT), so that each wave writes a
// frame row piece of 256 contiguous bytes per pixel slot.  The pixel state
// (S, T, N, P) stays in registers for the whole call, S in FP64.
//
// The tile's records (array order inside the tile, from the bucketing pass)
// are consumed in chunks of at most CHUNK records that complete at most
// kFrameGroup frames:
//   1. each wave holds its quarter of the chunk's records in registers
//      (prefetched while the previous chunk was processed);
//   2. stable counting sort by pixel inside the tile: per-wave stable ranks,
//      an exclusive scan over (pixel, wave) counters, a scatter into LDS, so
//      each pixel's events of the chunk are contiguous and in array order;
//   3. phase A: each thread runs the events of its pixels through Alg. 2 in
//      array order and records a change list: for every frame of the chunk
//      at which the pixel's visible state changes, the frame index and the
//      state after the last event that frame includes;
//   4. phase B: the chunk's frames, every thread writing its pixels' values
//      (Eq. (14)); a frame only compares its index with the pixel's next
//      change and selects, with no branch and no loop per event.
// Frames after the last event are written from the final state.
//
// Frame times are read through the scalar path (wave-uniform index): on
// CDNA one counter tracks vector loads and stores, and waiting for a vector
// load issued after a burst of frame stores would wait for the stores too.
// For the same reason the next chunk's records and frame times are loaded
// before this chunk's frame stores and waited for in one place.
#include <hip/hip_runtime.h>

#include "esi_internal.hpp"

namespace esi {
namespace {

// s_waitcnt immediate (gfx9 encoding): vmcnt = 0, expcnt and lgkmcnt not waited.
constexpr int kWaitVmcnt0 = 0x0F70;
constexpr int kFrameGroup = 128;  // frames completed by one chunk, at most
constexpr bool kMaskedReload = true;

// Records per chunk: LDS holds the chunk three times over (records, states,
// frame indices) next to the (pixel, wave) counters of the tile.
constexpr int chunk_records(int ppt) { return ppt >= 4 ? 1024 : 1792; }

struct FrameOut {
    const int64_t* t_frames;
    int nf;
    float* frames;
    uint8_t* frames_u8;
};

// First index in [lo, hi) whose frame time is >= t (hi if none); frame times
// are non-decreasing (otherwise the result is some index in [lo, hi]).
__device__ __forceinline__ int first_frame_at_or_after(const int64_t* tf, int lo, int hi, int64_t t)
{
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (load_const(tf, mid) < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// First record index in [lo, hi) whose time is > t (hi if none).
__device__ __forceinline__ uint32_t first_record_after(const uint64_t* rec, uint32_t lo, uint32_t hi,
                                                       int64_t t_ref, int64_t t)
{
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (t_ref + record_dt(load_const(rec, mid)) <= t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// First index in [0, n) of the LDS frame-time window with tfl[idx] >= t.
__device__ __forceinline__ int lds_lower_bound(const int64_t* tfl, int n, int64_t t)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tfl[mid] < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <int PPT>
struct Pixels {
    // state after every event applied so far (Alg. 2)
    double S[PPT];
    int64_t T[PPT];
    uint32_t N[PPT];
    int32_t P[PPT];
    // the state the frames see (after the events up to the last frame
    // written): Sf and Af = 1 + k (Tf - t_base), so that the decay base of a
    // frame at t_f is u = Af - k (t_f - t_base)
    double Sf[PPT], Af[PPT];
    // this chunk's change list: entries cbase + idx, ... of chg_*
    uint32_t cbase[PPT], nch[PPT], idx[PPT];
    int jn[PPT];        // frame index (in the chunk) of the next change
    double Sn[PPT], An[PPT];  // its state
};

// Phase B: frames [j0, j1) of the call.  jj = j - j0 indexes the chunk's
// change lists and kt[jj] = k (t_f - t_base) (kt == nullptr: computed here).
// Per pixel and frame: take the next change if it belongs to this frame
// (only those lanes touch LDS), then v = clamp(Sf u^b), u = clamp(Af - kt, 0, 1),
// F = (v - s_min)/(s_max - s_min).
template <int PPT, int BK, int CHUNK_ENTRIES>
__device__ __forceinline__ void walk_frames(const MethodParams& mp, Pixels<PPT>& px,
                                            const FrameOut& fo, int j0, int j1, int64_t t_base,
                                            const double* kt, const double* chg_S,
                                            const double* chg_A, const uint16_t* chg_j,
                                            int64_t q0, int64_t npix)
{
    int64_t t_next_f = (j0 < j1 && !kt) ? load_const(fo.t_frames, j0) : 0;
    for (int j = j0; j < j1; ++j) {
        const int jj = j - j0;
        double ktf;
        if (kt) {
            ktf = kt[jj];
        } else {
            ktf = mp.k * (double)(t_next_f - t_base);
            if (j + 1 < j1)
                t_next_f = load_const(fo.t_frames, j + 1);  // one frame ahead
        }
        float F[PPT];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            if (kMaskedReload) {
                if (px.jn[i] == jj) {
                    px.Sf[i] = px.Sn[i];
                    px.Af[i] = px.An[i];
                    ++px.idx[i];
                    const uint32_t e = min(px.cbase[i] + px.idx[i], (uint32_t)(CHUNK_ENTRIES - 1));
                    px.Sn[i] = chg_S[e];
                    px.An[i] = chg_A[e];
                    px.jn[i] = (px.idx[i] < px.nch[i]) ? (int)chg_j[e] : 0x7FFFFFFF;
                }
            } else {
                const bool c = px.jn[i] == jj;
                px.Sf[i] = c ? px.Sn[i] : px.Sf[i];
                px.Af[i] = c ? px.An[i] : px.Af[i];
                px.idx[i] += c ? 1u : 0u;
                const uint32_t e = min(px.cbase[i] + px.idx[i], (uint32_t)(CHUNK_ENTRIES - 1));
                px.Sn[i] = chg_S[e];
                px.An[i] = chg_A[e];
                px.jn[i] = (px.idx[i] < px.nch[i]) ? (int)chg_j[e] : 0x7FFFFFFF;
            }
            double v = px.Sf[i];
            if (!mp.lazy) {
                const double u = fmin(fmax(px.Af[i] - ktf, 0.0), 1.0);
                v = clamp_s(mp, px.Sf[i] * power_b<BK>(u, mp.b));
            }
            F[i] = (float)((v - mp.s_min) * mp.inv_range);
        }
        float* frow = fo.frames ? fo.frames + (size_t)j * (size_t)npix : nullptr;
        uint8_t* urow = fo.frames_u8 ? fo.frames_u8 + (size_t)j * (size_t)npix : nullptr;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int64_t q = q0 + (int64_t)i * kBlock;
            if (q < npix) {
                if (frow)
                    __builtin_nontemporal_store(F[i], frow + q);
                if (urow)
                    urow[q] = frame_code(F[i]);
            }
        }
    }
}

template <int PPT, int BK>
__global__ __launch_bounds__(kBlock) void k_integrate(
    const uint64_t* __restrict__ records, const uint32_t* __restrict__ table,
    const uint32_t* __restrict__ total, const int64_t* __restrict__ ev_t, int K, StateDev st,
    MethodParams mp, FrameOut fo, DiagDev* diag)
{
    constexpr int TILE = kBlock * PPT;
    constexpr int CHUNK = chunk_records(PPT);             // records per chunk, at most
    constexpr int PER_WAVE = CHUNK / kWavesPerBlock;      // records per wave per chunk
    constexpr int STEPS = PER_WAVE / kWave;               // records per lane per chunk
    static_assert(kFrameGroup <= kBlock, "one frame time per thread");
    static_assert(PER_WAVE % kWave == 0, "chunk size");
    __shared__ uint64_t sorted[CHUNK];    // records sorted by pixel; then event times (double)
    __shared__ double chg_S[CHUNK];       // change lists: S after the change
    __shared__ uint16_t chg_j[CHUNK];     // change lists: frame index in the chunk
    __shared__ uint32_t cnt[kWavesPerBlock][TILE];
    __shared__ int64_t tfl[kFrameGroup];  // frame times of the chunk
    __shared__ double ktl[kFrameGroup];   // k (t_f - t_base) of the chunk's frames
    __shared__ uint32_t scan_w[kWavesPerBlock];
    double* chg_A = (double*)sorted;      // change lists: A after the change

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int tile = blockIdx.x;
    const int64_t q0 = (int64_t)tile * TILE + tid;
    const int64_t npix = st.npix;
    const int kbits = key_bits_for((uint32_t)TILE);

    Pixels<PPT> px;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * kBlock;
        const bool in = q < npix;
        px.S[i] = in ? (double)st.S_hi[q] + (double)st.S_lo[q] : 0.0;
        px.T[i] = in ? st.T[q] : 0;
        px.N[i] = in ? st.N[q] : 0u;
        px.P[i] = in ? st.P[q] : 0;
        px.Sf[i] = px.S[i];
        px.cbase[i] = 0;
        px.nch[i] = 0;
        px.idx[i] = 0;
        px.jn[i] = 0x7FFFFFFF;
        px.Sn[i] = 0.0;
        px.An[i] = 0.0;
    }

    // the tile's records [rs, re); read-only here, so scalar loads
    uint32_t rs = 0, re = 0;
    int64_t t_ref = 0;
    if (table) {
        rs = load_const(table, tile);
        re = (tile + 1 < K) ? load_const(table, tile + 1) : load_const(total, 0);
        t_ref = load_const(ev_t, 0);
    }

    // frame decay bases are measured from t_base (first frame time) so that
    // A = 1 + k (T - t_base) keeps its precision
    const int64_t t_base = (fo.nf > 0) ? load_const(fo.t_frames, 0) : 0;
#pragma unroll
    for (int i = 0; i < PPT; ++i)
        px.Af[i] = __fma_rn(mp.k, (double)(px.T[i] - t_base), 1.0);

    int j = 0;  // next frame to write (uniform)
    bool bad = false;

    // records of the first chunk and the first frame times; clamped indices,
    // no select on loaded values, so all loads stay in flight
    uint64_t rr[STEPS], rr_next[STEPS];
    int64_t tf_cur = 0, tf_nxt = 0;
    if (rs < re) {
        const int cn0 = (int)(min(rs + (uint32_t)CHUNK, re) - rs);
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            rr[s] = records[rs + min(wave * PER_WAVE + s * kWave + lane, cn0 - 1)];
        if (fo.nf > 0)
            tf_cur = fo.t_frames[min(tid, fo.nf - 1)];
    }
    // nothing may be pending on `rr` at the loop head, or the compiler waits
    // there for everything outstanding, frame stores included
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);

    for (uint32_t cs = rs; cs < re;) {
        // this chunk: at most CHUNK records, completing at most kFrameGroup
        // frames (records after the group's last frame wait for the next one)
        uint32_t ce = min(cs + (uint32_t)CHUNK, re);
        const int jmax = min(j + kFrameGroup, fo.nf);
        if (j < fo.nf && jmax < fo.nf)
            ce = first_record_after(records, cs, ce, t_ref, load_const(fo.t_frames, jmax - 1));
        const int cn = (int)(ce - cs);
        const int64_t t_next = (ce < re) ? t_ref + record_dt(load_const(records, ce)) : INT64_MAX;
        int j_end = (t_next == INT64_MAX) ? jmax
                                          : min(first_frame_at_or_after(fo.t_frames, j, fo.nf, t_next), jmax);
        if (cn == 0 && j_end == j)
            j_end = min(j + 1, fo.nf);  // progress even with unsorted frame times
        const int nfw = j_end - j;     // frames of this chunk

        // prefetch the next chunk's records and frame times (before this
        // chunk's frame stores are issued)
        if (ce < re) {
            const int cn1 = (int)(min(ce + (uint32_t)CHUNK, re) - ce);
#pragma unroll
            for (int s = 0; s < STEPS; ++s)
                rr_next[s] = records[ce + min(wave * PER_WAVE + s * kWave + lane, cn1 - 1)];
        }
        if (j_end < fo.nf)
            tf_nxt = fo.t_frames[min(j_end + tid, fo.nf - 1)];

        if (tid < kFrameGroup) {
            tfl[tid] = tf_cur;
            ktl[tid] = mp.k * (double)(tf_cur - t_base);
        }
        // 2a. stable ranks inside the wave
        for (int k = lane; k < TILE; k += kWave)
            cnt[wave][k] = 0;
        wave_sync();
        uint32_t rank[STEPS];
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int c = wave * PER_WAVE + s * kWave + lane;
            rank[s] = wave_stable_rank(c < cn, record_lpx(rr[s]) & (TILE - 1), kbits, cnt[wave]);
        }
        __syncthreads();
        // 2b. exclusive scan over (pixel, wave), pixel-major
        {
            uint32_t v[PPT][kWavesPerBlock];
            uint32_t sum = 0;
#pragma unroll
            for (int i = 0; i < PPT; ++i)
#pragma unroll
                for (int w = 0; w < kWavesPerBlock; ++w) {
                    v[i][w] = cnt[w][tid * PPT + i];
                    sum += v[i][w];
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
#pragma unroll
            for (int i = 0; i < PPT; ++i)
#pragma unroll
                for (int w = 0; w < kWavesPerBlock; ++w) {
                    cnt[w][tid * PPT + i] = run;
                    run += v[i][w];
                }
        }
        __syncthreads();
        // 2c. scatter into pixel order (every index is checked, so that a
        // broken invariant can only flag an error, never leave the chunk)
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int c = wave * PER_WAVE + s * kWave + lane;
            if (c < cn) {
                const uint32_t at = cnt[wave][record_lpx(rr[s]) & (TILE - 1)] + rank[s];
                if (at < (uint32_t)cn)
                    sorted[at] = rr[s];
                else
                    bad = true;
            }
        }
        __syncthreads();

        // 3. phase A: each pixel's events of the chunk in array order; the
        // change list keeps, per frame index jc of the chunk that first
        // includes some event, the state after the last such event.  Entries
        // go over the pixel's own slots of `sorted`/chg_*, behind the read
        // position.  Events after the chunk's last frame (jc == nfw) make no
        // entry: the frames of later chunks see the final state.
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int l = tid + i * kBlock;
            const uint32_t end = min((l + 1 < TILE) ? cnt[0][l + 1] : (uint32_t)cn, (uint32_t)cn);
            const uint32_t beg = min(cnt[0][l], end);
            uint32_t w = beg;          // change list write position
            int jc_prev = -1;
            for (uint32_t e = beg; e < end; ++e) {
                const uint64_t r = sorted[e];
                const int64_t t = t_ref + record_dt(r);
                apply_event<BK>(mp, px.S[i], px.T[i], px.N[i], px.P[i], t, record_pos(r));
                const int jc = lds_lower_bound(tfl, nfw, t);
                if (jc < nfw) {
                    if (jc != jc_prev && jc_prev >= 0)
                        ++w;           // a new entry; the previous one is final
                    chg_S[w] = px.S[i];
                    chg_A[w] = __fma_rn(mp.k, (double)(t - t_base), 1.0);
                    chg_j[w] = (uint16_t)jc;
                    jc_prev = jc;
                }
            }
            px.cbase[i] = beg;
            px.nch[i] = (jc_prev >= 0) ? (w - beg + 1u) : 0u;
            px.idx[i] = 0;
            const uint32_t e0 = min(beg, (uint32_t)max(cn - 1, 0));
            px.jn[i] = px.nch[i] ? (int)chg_j[e0] : 0x7FFFFFFF;
            px.Sn[i] = chg_S[e0];
            px.An[i] = chg_A[e0];
        }
        // Wait for the prefetched records and frame times now: this also
        // drains the frame stores of the previous chunk (one counter covers
        // loads and stores), which have had the whole sort to complete.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        // 4. phase B: the frames this chunk completes
        walk_frames<PPT, BK, CHUNK>(mp, px, fo, j, j_end, t_base, ktl, chg_S, chg_A, chg_j, q0,
                                    npix);
        j = j_end;
        // the frames of later chunks see every event of this one
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            px.Sf[i] = px.S[i];
            px.Af[i] = __fma_rn(mp.k, (double)(px.T[i] - t_base), 1.0);
            px.nch[i] = 0;
            px.jn[i] = 0x7FFFFFFF;
        }
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            rr[s] = rr_next[s];
        tf_cur = tf_nxt;
        cs = ce;
        __syncthreads();  // LDS is reused by the next chunk
    }
    // frames after the last event (no change lists: nch = 0, jn never hit)
    walk_frames<PPT, BK, CHUNK>(mp, px, fo, j, fo.nf, t_base, nullptr, chg_S, chg_A, chg_j, q0,
                                npix);

#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * kBlock;
        if (q < npix) {
            const float hi = (float)px.S[i];
            st.S_hi[q] = hi;
            st.S_lo[q] = (float)(px.S[i] - (double)hi);
            st.T[q] = px.T[i];
            st.N[q] = px.N[i];
            st.P[q] = px.P[i];
        }
    }
    if (bad)
        atomicOr(&diag->flags, 8u);  // ESI_DIAG_INTERNAL: never expected
    // frame times must be non-decreasing; the first workgroup checks
    if (tile == 0) {
        bool unsorted = false;
        for (int jj = 1 + tid; jj < fo.nf; jj += kBlock)
            unsorted |= fo.t_frames[jj] < fo.t_frames[jj - 1];
        if (unsorted)
            atomicOr(&diag->flags, 2u);  // ESI_DIAG_FRAMES_UNSORTED
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

int decay_kind(double b) { return b == 1.0 ? kDecayB1 : (b == 2.0 ? kDecayB2 : kDecayPow); }

template <int PPT, int BK>
hipError_t launch_integrate_t(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                              const CallScratch& cs, const MethodParams& mp,
                              const int64_t* t_frames, int nf, float* frames, uint8_t* frames_u8,
                              DiagDev* diag, hipStream_t stream)
{
    FrameOut fo{t_frames, nf, frames, frames_u8};
    const bool has = ev.n > 0;
    hipLaunchKernelGGL((k_integrate<PPT, BK>), dim3(sc.ntiles), dim3(kBlock), 0, stream,
                       has ? cs.records : nullptr, has ? cs.table : nullptr,
                       has ? cs.total : nullptr, has ? ev.t : nullptr, sc.ntiles, st, mp, fo, diag);
    return hipGetLastError();
}

template <int PPT>
hipError_t launch_integrate_p(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                              const CallScratch& cs, const MethodParams& mp,
                              const int64_t* t_frames, int nf, float* frames, uint8_t* frames_u8,
                              DiagDev* diag, hipStream_t stream)
{
    switch (decay_kind(mp.b)) {
    case kDecayB1:
        return launch_integrate_t<PPT, kDecayB1>(ev, st, sc, cs, mp, t_frames, nf, frames,
                                                 frames_u8, diag, stream);
    case kDecayB2:
        return launch_integrate_t<PPT, kDecayB2>(ev, st, sc, cs, mp, t_frames, nf, frames,
                                                 frames_u8, diag, stream);
    default:
        return launch_integrate_t<PPT, kDecayPow>(ev, st, sc, cs, mp, t_frames, nf, frames,
                                                  frames_u8, diag, stream);
    }
}

}  // namespace

hipError_t launch_integrate(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                            const CallScratch& cs, const MethodParams& mp,
                            const int64_t* t_frames, int nf, float* frames, uint8_t* frames_u8,
                            DiagDev* diag, hipStream_t stream)
{
    switch (sc.ppt) {
    case 1:
        return launch_integrate_p<1>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    case 2:
        return launch_integrate_p<2>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    case 4:
        return launch_integrate_p<4>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    case 8:
        return launch_integrate_p<8>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_snapshot(const StateDev& st, const MethodParams& mp, int64_t t_f, float* frame,
                           uint8_t* u8, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((st.npix + kBlock - 1) / kBlock);
    switch (decay_kind(mp.b)) {
    case kDecayB1:
        hipLaunchKernelGGL(k_snapshot<kDecayB1>, dim3(blocks), dim3(kBlock), 0, stream, st, mp,
                           t_f, frame, u8);
        break;
    case kDecayB2:
        hipLaunchKernelGGL(k_snapshot<kDecayB2>, dim3(blocks), dim3(kBlock), 0, stream, st, mp,
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
