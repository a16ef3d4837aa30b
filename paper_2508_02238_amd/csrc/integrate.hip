// integrate.hip -- per-tile integration of the bucketed events and frames.
//
// One workgroup (256 threads) owns a tile of 256 * PPT consecutive pixels;
// thread `tid` owns pixels tid + 256 i (i < PPT), so that each wave writes a
// frame row piece of 256 contiguous bytes per pixel slot.  The pixel state
// (S, T, N, P) stays in registers for the whole call, S in FP64.
//
// The tile's records (array order inside the tile, from the bucketing pass)
// are consumed in chunks of kChunk:
//   1. each wave loads its quarter of the chunk into registers;
//   2. stable counting sort by pixel inside the tile: per-wave stable ranks,
//      an exclusive scan over (pixel, wave) counters, a scatter into LDS, so
//      each pixel's events of the chunk are contiguous and in array order;
//   3. every frame j with t_frames[j] earlier than the next chunk's first
//      event is complete after this chunk: for each such frame each thread
//      applies its pixels' events with t <= t_frames[j] (Alg. 2 event loop)
//      and writes the frame value (Eq. (14)); then it applies the rest of
//      the chunk.
// Frames after the last event are written from the final state.
//
// The frame loop index and the frame times are wave-uniform (scalar loads):
// on CDNA a wait for a vector load also waits for every earlier store, so a
// per-frame vector load would stall on the previous frame's stores.
// Between events the decayed snapshot is advanced incrementally:
// u = 1 - k (t_f - T) drops by k (t_f - t_f') from one frame to the next.
#include <hip/hip_runtime.h>

#include "esi_internal.hpp"

namespace esi {
namespace {

// s_waitcnt immediate (gfx9 encoding): vmcnt = 0, expcnt and lgkmcnt not waited.
constexpr int kWaitVmcnt0 = 0x0F70;

struct FrameOut {
    const int64_t* t_frames;
    int nf;
    float* frames;
    uint8_t* frames_u8;
};

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// First index in [lo, nf) whose frame time is >= t (nf if none); frame times
// are non-decreasing (otherwise the result is some index in [lo, nf]).
__device__ __forceinline__ int first_frame_at_or_after(const int64_t* tf, int lo, int nf, int64_t t)
{
    int hi = nf;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (load_const(tf, mid) < t)
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
    // the state as the frames see it: after the events up to the last
    // frame written
    double Sf[PPT];
    int64_t Tf[PPT];
    double u[PPT];      // 1 - k (t_f - Tf) at the last frame time written
    bool fresh[PPT];    // u is valid (Tf unchanged since the last frame)
};

// Phase B: frames [j0, j1).  Each pixel's events of the chunk were applied in
// phase A, which left the state after each event in post_S; here a pixel only
// moves its pointer past the events with t <= t_f and takes the state of the
// last one (ptr/end/tn: the pixel's next event in `sorted` and its time).
template <int PPT, int BK>
__device__ __forceinline__ void walk_frames(const MethodParams& mp, Pixels<PPT>& px,
                                            const FrameOut& fo, int j0, int j1, int64_t& tf_prev,
                                            const uint64_t* sorted, const double* post_S,
                                            uint32_t* ptr, const uint32_t* end, int64_t* tn,
                                            int64_t t_ref, int64_t q0, int64_t npix)
{
    int64_t t_next_f = (j0 < j1) ? load_const(fo.t_frames, j0) : 0;
    for (int j = j0; j < j1; ++j) {
        const int64_t t_f = t_next_f;
        if (j + 1 < j1)
            t_next_f = load_const(fo.t_frames, j + 1);  // one frame ahead
        const double dk = mp.k * (double)(t_f - tf_prev);
        tf_prev = t_f;
        float F[PPT];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            if (ptr[i] < end[i] && tn[i] <= t_f) {
                do {
                    px.Sf[i] = post_S[ptr[i]];
                    px.Tf[i] = tn[i];
                    ++ptr[i];
                    tn[i] = (ptr[i] < end[i]) ? t_ref + record_dt(sorted[ptr[i]]) : INT64_MAX;
                } while (ptr[i] < end[i] && tn[i] <= t_f);
                px.fresh[i] = false;
            }
            if (px.fresh[i]) {
                px.u[i] -= dk;
            } else {
                px.u[i] = __fma_rn(-mp.k, (double)(t_f - px.Tf[i]), 1.0);
                px.fresh[i] = true;
            }
            F[i] = frame_value_u<BK>(mp, px.Sf[i], px.u[i]);
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int64_t q = q0 + (int64_t)i * kBlock;
            if (q < npix) {
                const size_t o = (size_t)j * (size_t)npix + (size_t)q;
                if (fo.frames)
                    __builtin_nontemporal_store(F[i], fo.frames + o);
                if (fo.frames_u8)
                    fo.frames_u8[o] = frame_code(F[i]);
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
    constexpr int PER_WAVE = kChunk / kWavesPerBlock;     // records per wave per chunk
    constexpr int STEPS = PER_WAVE / kWave;               // records per lane per chunk
    __shared__ uint64_t sorted[kChunk];
    __shared__ double post_S[kChunk];
    __shared__ uint32_t cnt[kWavesPerBlock][TILE];
    __shared__ uint32_t scan_w[kWavesPerBlock];

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
        px.Tf[i] = px.T[i];
        px.u[i] = 1.0;
        px.fresh[i] = false;
    }

    // the tile's records [rs, re); read-only here, so scalar loads
    uint32_t rs = 0, re = 0;
    int64_t t_ref = 0;
    if (table) {
        rs = load_const(table, tile);
        re = (tile + 1 < K) ? load_const(table, tile + 1) : load_const(total, 0);
        t_ref = load_const(ev_t, 0);
    }

    int j = 0;               // next frame to write (uniform)
    int64_t tf_prev = 0;     // time of the last frame written (uniform)
    bool bad = false;
    uint32_t ptr[PPT], end[PPT];
    int64_t tn[PPT];

    // Records of a chunk, this wave's quarter, step-major (array order).
    // Clamped indices: no select on loaded values, all loads stay in flight.
    uint64_t rr[STEPS], rr_next[STEPS];
    if (rs < re) {
        const int cn0 = (int)(min(rs + (uint32_t)kChunk, re) - rs);
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            rr[s] = records[rs + min(wave * PER_WAVE + s * kWave + lane, cn0 - 1)];
    }
    // nothing may be pending on `rr` at the loop head, or the compiler waits
    // there for everything outstanding, frame stores included
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    for (uint32_t cs = rs; cs < re; cs += kChunk) {
        const uint32_t ce = min(cs + (uint32_t)kChunk, re);
        const int cn = (int)(ce - cs);
        const int64_t t_next = (ce < re) ? t_ref + record_dt(load_const(records, ce)) : INT64_MAX;
        // prefetch the next chunk before this chunk's frame stores are issued
        if (ce < re) {
            const int cn1 = (int)(min(ce + (uint32_t)kChunk, re) - ce);
#pragma unroll
            for (int s = 0; s < STEPS; ++s)
                rr_next[s] = records[ce + min(wave * PER_WAVE + s * kWave + lane, cn1 - 1)];
        }

        // 2a. stable ranks inside the wave
        for (int k = lane; k < TILE; k += kWave)
            cnt[wave][k] = 0;
        wave_sync();
        uint32_t rank[STEPS];
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int c = wave * PER_WAVE + s * kWave + lane;
            rank[s] = wave_stable_rank(c < cn, (record_lpx(rr[s]) & (TILE - 1)), kbits, cnt[wave]);
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
                const uint32_t at = cnt[wave][(record_lpx(rr[s]) & (TILE - 1))] + rank[s];
                if (at < (uint32_t)cn)
                    sorted[at] = rr[s];
                else
                    bad = true;
            }
        }
        __syncthreads();

        // 3. phase A: each pixel's events of the chunk, in array order
        // (Alg. 2 event loop); the state after each event goes to post_S
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int l = tid + i * kBlock;
            end[i] = min((l + 1 < TILE) ? cnt[0][l + 1] : (uint32_t)cn, (uint32_t)cn);
            ptr[i] = min(cnt[0][l], end[i]);
            for (uint32_t e = ptr[i]; e < end[i]; ++e) {
                const uint64_t r = sorted[e];
                apply_event<BK>(mp, px.S[i], px.T[i], px.N[i], px.P[i], t_ref + record_dt(r),
                                record_pos(r));
                post_S[e] = px.S[i];
            }
            tn[i] = (ptr[i] < end[i]) ? t_ref + record_dt(sorted[ptr[i]]) : INT64_MAX;
        }
        // 4. phase B: the frames this chunk completes
        const int j_end = (t_next == INT64_MAX)
                              ? fo.nf
                              : first_frame_at_or_after(fo.t_frames, j, fo.nf, t_next);
        // Wait for the prefetched records now: this also drains the frame
        // stores of the previous chunk (one counter covers loads and stores),
        // which have had the whole sort to complete.  Waiting after this
        // chunk's stores instead would stall on all of them.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        walk_frames<PPT, BK>(mp, px, fo, j, j_end, tf_prev, sorted, post_S, ptr, end, tn, t_ref,
                             q0, npix);
        j = j_end;
        // the frames of later chunks see every event of this one
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            if (px.Tf[i] != px.T[i] || ptr[i] < end[i]) {
                px.Sf[i] = px.S[i];
                px.Tf[i] = px.T[i];
                px.fresh[i] = false;
            }
        }
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            rr[s] = rr_next[s];
        __syncthreads();  // LDS is reused by the next chunk
    }
    // frames after the last event
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        ptr[i] = 0;
        end[i] = 0;
        tn[i] = INT64_MAX;
    }
    walk_frames<PPT, BK>(mp, px, fo, j, fo.nf, tf_prev, sorted, post_S, ptr, end, tn, t_ref, q0,
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
