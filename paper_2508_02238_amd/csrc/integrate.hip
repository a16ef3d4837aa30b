// integrate.hip -- per-tile integration of the bucketed events and frames.
//
// One workgroup (256 threads) owns a tile of 256 * PPT consecutive pixels;
// thread `tid` owns pixels tid + 256 i (i < PPT), so that a frame row of the
// tile is written by the workgroup as contiguous 1 KB pieces.  The pixel
// state (S, T, N, P) stays in registers for the whole call, in FP64 for S.
//
// The tile's records (array order inside the tile, from the bucketing pass)
// are consumed in chunks of kChunk:
//   1. each wave loads its quarter of the chunk into registers;
//   2. stable counting sort by pixel inside the tile: per-wave stable ranks,
//      an exclusive scan over (pixel, wave) counters, a scatter into LDS, so
//      each pixel's events of the chunk are contiguous and in array order;
//   3. every frame j with t_frames[j] earlier than the next chunk's first
//      event is now complete up to t_frames[j]: each thread applies its
//      pixels' events with t <= t_frames[j] (Alg. 2 event loop) and writes
//      the frame value (Eq. (14)); then applies the rest of the chunk.
// Frames after the last event are written from the final state.
#include <hip/hip_runtime.h>

#include "esi_internal.hpp"

namespace esi {
namespace {

struct FrameOut {
    const int64_t* t_frames;
    int nf;
    float* frames;
    uint8_t* frames_u8;
};

template <int PPT>
struct Pixels {
    double S[PPT];
    int64_t T[PPT];
    uint32_t N[PPT];
    int32_t P[PPT];
};

template <int PPT>
__device__ __forceinline__ void write_frame(const MethodParams& mp, const Pixels<PPT>& px,
                                            const FrameOut& fo, int j, int64_t q0, int64_t npix,
                                            int64_t t_f)
{
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * kBlock;
        if (q < npix) {
            const float F = frame_value(mp, px.S[i], px.T[i], t_f);
            const size_t o = (size_t)j * (size_t)npix + (size_t)q;
            if (fo.frames)
                __builtin_nontemporal_store(F, fo.frames + o);
            if (fo.frames_u8)
                fo.frames_u8[o] = frame_code(F);
        }
    }
}

template <int PPT>
__global__ __launch_bounds__(kBlock) void k_integrate(
    const uint64_t* __restrict__ records, const uint32_t* __restrict__ table,
    const uint32_t* __restrict__ total, const int64_t* __restrict__ ev_t, int K, int tile_log,
    StateDev st, MethodParams mp, FrameOut fo, DiagDev* diag)
{
    constexpr int TILE = kBlock * PPT;
    constexpr int PER_WAVE = kChunk / kWavesPerBlock;     // records per wave per chunk
    constexpr int STEPS = PER_WAVE / kWave;               // records per lane per chunk
    __shared__ uint64_t sorted[kChunk];
    __shared__ uint32_t cnt[kWavesPerBlock][TILE];
    __shared__ uint32_t tag[kWavesPerBlock][128];
    __shared__ uint32_t scan_w[kWavesPerBlock];

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int tile = blockIdx.x;
    const int64_t q0 = (int64_t)tile * TILE + tid;
    const int64_t npix = st.npix;

    Pixels<PPT> px;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int64_t q = q0 + (int64_t)i * kBlock;
        if (q < npix) {
            px.S[i] = (double)st.S_hi[q] + (double)st.S_lo[q];
            px.T[i] = st.T[q];
            px.N[i] = st.N[q];
            px.P[i] = st.P[q];
        } else {
            px.S[i] = 0.0;
            px.T[i] = 0;
            px.N[i] = 0;
            px.P[i] = 0;
        }
    }

    uint32_t rs = 0, re = 0;
    int64_t t_ref = 0;
    if (table) {
        rs = table[tile];
        re = (tile + 1 < K) ? table[tile + 1] : *total;
        t_ref = ev_t[0];
    }
    for (int k = lane; k < 128; k += kWave)
        tag[wave][k] = 0xFFFFFFFFu;

    int j = 0;  // next frame to write
    bool bad = false;
    for (uint32_t cs = rs; cs < re; cs += kChunk) {
        const uint32_t ce = min(cs + (uint32_t)kChunk, re);
        const int cn = (int)(ce - cs);
        const int64_t t_next = (ce < re) ? t_ref + record_dt(records[ce]) : INT64_MAX;

        // 1. this wave's quarter of the chunk, in array order (step-major)
        uint64_t rr[STEPS];
        uint32_t rank[STEPS];
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int c = wave * PER_WAVE + s * kWave + lane;
            rr[s] = (c < cn) ? records[cs + c] : 0ull;
        }
        for (int k = lane; k < TILE; k += kWave)
            cnt[wave][k] = 0;
        wave_sync();
        // 2a. stable ranks inside the wave
        bool ranked = true;
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int c = wave * PER_WAVE + s * kWave + lane;
            ranked &= wave_stable_rank(c < cn, record_lpx(rr[s]), cnt[wave], tag[wave], rank[s]);
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
                const uint32_t at = cnt[wave][record_lpx(rr[s])] + rank[s];
                if (ranked && at < (uint32_t)cn)
                    sorted[at] = rr[s];
                else
                    bad = true;
            }
        }
        __syncthreads();

        // 3. walk frames and events
        uint32_t ptr[PPT], end[PPT];
        int64_t tn[PPT];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int l = tid + i * kBlock;
            end[i] = min((l + 1 < TILE) ? cnt[0][l + 1] : (uint32_t)cn, (uint32_t)cn);
            ptr[i] = min(cnt[0][l], end[i]);
            tn[i] = (ptr[i] < end[i]) ? t_ref + record_dt(sorted[ptr[i]]) : INT64_MAX;
        }
        for (; j < fo.nf; ++j) {
            const int64_t t_f = fo.t_frames[j];
            if (t_f >= t_next)
                break;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                while (ptr[i] < end[i] && tn[i] <= t_f) {
                    const uint64_t r = sorted[ptr[i]];
                    apply_event(mp, px.S[i], px.T[i], px.N[i], px.P[i], tn[i], record_pos(r));
                    ++ptr[i];
                    tn[i] = (ptr[i] < end[i]) ? t_ref + record_dt(sorted[ptr[i]]) : INT64_MAX;
                }
            }
            write_frame<PPT>(mp, px, fo, j, q0, npix, t_f);
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            while (ptr[i] < end[i]) {
                const uint64_t r = sorted[ptr[i]];
                apply_event(mp, px.S[i], px.T[i], px.N[i], px.P[i], t_ref + record_dt(r),
                            record_pos(r));
                ++ptr[i];
            }
        }
        __syncthreads();  // LDS is reused by the next chunk
    }
    for (; j < fo.nf; ++j)
        write_frame<PPT>(mp, px, fo, j, q0, npix, fo.t_frames[j]);

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
        bool bad = false;
        for (int jj = 1 + tid; jj < fo.nf; jj += kBlock)
            bad |= fo.t_frames[jj] < fo.t_frames[jj - 1];
        if (bad)
            atomicOr(&diag->flags, 2u);  // ESI_DIAG_FRAMES_UNSORTED
    }
}

__global__ __launch_bounds__(kBlock) void k_snapshot(StateDev st, MethodParams mp, int64_t t_f,
                                                     float* frame, uint8_t* u8)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= st.npix)
        return;
    const double S = (double)st.S_hi[q] + (double)st.S_lo[q];
    const float F = frame_value(mp, S, st.T[q], t_f);
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

template <int PPT>
hipError_t launch_integrate_t(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                              const CallScratch& cs, const MethodParams& mp,
                              const int64_t* t_frames, int nf, float* frames, uint8_t* frames_u8,
                              DiagDev* diag, hipStream_t stream)
{
    FrameOut fo{t_frames, nf, frames, frames_u8};
    const bool has = ev.n > 0;
    hipLaunchKernelGGL(k_integrate<PPT>, dim3(sc.ntiles), dim3(kBlock), 0, stream,
                       has ? cs.records : nullptr, has ? cs.table : nullptr,
                       has ? cs.total : nullptr, has ? ev.t : nullptr, sc.ntiles, sc.tile_log, st,
                       mp, fo, diag);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_integrate(const EventsDev& ev, const StateDev& st, const Schedule& sc,
                            const CallScratch& cs, const MethodParams& mp,
                            const int64_t* t_frames, int nf, float* frames, uint8_t* frames_u8,
                            DiagDev* diag, hipStream_t stream)
{
    switch (sc.ppt) {
    case 1:
        return launch_integrate_t<1>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    case 2:
        return launch_integrate_t<2>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    case 4:
        return launch_integrate_t<4>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    case 8:
        return launch_integrate_t<8>(ev, st, sc, cs, mp, t_frames, nf, frames, frames_u8, diag, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_snapshot(const StateDev& st, const MethodParams& mp, int64_t t_f, float* frame,
                           uint8_t* u8, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((st.npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_snapshot, dim3(blocks), dim3(kBlock), 0, stream, st, mp, t_f, frame, u8);
    return hipGetLastError();
}

hipError_t launch_reset(const StateDev& st, int64_t t0, DiagDev* diag, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((st.npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(kBlock), 0, stream, st, t0, diag);
    return hipGetLastError();
}

}  // namespace esi
