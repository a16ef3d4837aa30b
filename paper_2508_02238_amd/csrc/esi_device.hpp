// esi_device.hpp -- device-side arithmetic of ESI shared by the kernels.
//
// Per event (Alg. 2, event loop): S <- (S + p C) d(dt), T <- t, S <- clamp(S)
// with d(dt) = max(1 - k dt, 0)^b (Eq. (4)) and the clamp of Eq. (13).
// All of it runs in FP64 in registers: on CDNA4 an FP64 FMA issues at the
// same rate as an unpacked FP32 one, and FP64 keeps long runs of decay
// factors close to 1 well inside a 1e-5 relative error without compensated
// FP32 arithmetic.  Frames (Eq. (14)) are rounded to FP32 once, at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace esi {

constexpr int kWave = 64;
constexpr int kBlock = 256;           // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;

// Per-call constants of the method.
struct MethodParams {
    double C, k, b, s_min, s_max, inv_range;  // inv_range = 1 / (s_max - s_min)
    int b_kind;                               // 1, 2, 3, 4: integer power; 0: pow()
    int decay_then_add;
    int lazy;
};

// Eq. (4) as a truncated power: d(dt) = max(1 - k dt, 0)^b, dt >= 0 integer us.
__device__ __forceinline__ double decay(const MethodParams& mp, int64_t dt)
{
    const double u = __fma_rn(-mp.k, (double)dt, 1.0);
    if (!(u > 0.0))
        return 0.0;
    switch (mp.b_kind) {
    case 1:
        return u;
    case 2:
        return u * u;
    case 3:
        return u * u * u;
    case 4: {
        const double u2 = u * u;
        return u2 * u2;
    }
    default:
        return pow(u, mp.b);
    }
}

__device__ __forceinline__ double clamp_s(const MethodParams& mp, double s)
{
    return fmin(fmax(s, mp.s_min), mp.s_max);
}

// One event of Alg. 2 at a pixel whose state is (S, T, N, P).
__device__ __forceinline__ void apply_event(const MethodParams& mp, double& S, int64_t& T,
                                            uint32_t& N, int32_t& P, int64_t t, int pos)
{
    int64_t dt = t - T;
    dt = dt < 0 ? 0 : dt;
    const double d = decay(mp, dt);
    const double s = pos ? mp.C : -mp.C;
    const double v = mp.decay_then_add ? __fma_rn(S, d, s) : (S + s) * d;
    S = clamp_s(mp, v);
    T = t;
    N += 1u;
    P += pos ? 1 : -1;
}

// Eq. (14) of the state seen at t_f (decayed to t_f unless lazy), in [0, 1].
__device__ __forceinline__ float frame_value(const MethodParams& mp, double S, int64_t T,
                                             int64_t t_f)
{
    double v = S;
    if (!mp.lazy) {
        int64_t dt = t_f - T;
        dt = dt < 0 ? 0 : dt;
        v = clamp_s(mp, S * decay(mp, dt));
    }
    return (float)((v - mp.s_min) * mp.inv_range);
}

// 8-bit code: floor(255 F + 1/2) in FP32 with separately rounded operations.
__device__ __forceinline__ uint8_t frame_code(float F)
{
    float a = __fadd_rn(__fmul_rn(255.0f, F), 0.5f);
    a = floorf(a);
    a = fminf(fmaxf(a, 0.0f), 255.0f);
    return (uint8_t)a;
}

// Tile-bucketed event record, 64 bits:
//   [0, 48)  t - t_ref, two's complement (t_ref = the call's first event time)
//   [48, 63) pixel index inside its tile
//   63       polarity (1: +1)
__device__ __forceinline__ uint64_t pack_record(int64_t dt, uint32_t lpx, int pos)
{
    return ((uint64_t)dt & 0xFFFFFFFFFFFFull) | ((uint64_t)lpx << 48) | ((uint64_t)pos << 63);
}
__device__ __forceinline__ int64_t record_dt(uint64_t r) { return ((int64_t)(r << 16)) >> 16; }
__device__ __forceinline__ uint32_t record_lpx(uint64_t r) { return (uint32_t)(r >> 48) & 0x7FFFu; }
__device__ __forceinline__ int record_pos(uint64_t r) { return (int)(r >> 63); }

constexpr int64_t kMaxSpan = (int64_t)1 << 47;

// Ordering point for LDS traffic between the lanes of one wave: the lanes
// of a wave issue in lockstep and LDS serves a wave's requests in order, so a
// fence at wavefront scope plus a compiler barrier suffice.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Stable multisplit rank inside one wave step.  Lane l holds an element with
// key `key` (valid when `ok`); lanes are in array order.  On return, for valid
// lanes, `pos` = counter[key] (before this step) + number of lower valid lanes
// with the same key, and counter[key] has been advanced by the number of
// valid lanes with that key.  `tag` is a 128-entry per-wave LDS array holding
// 0xFFFFFFFF on entry (and on return).  Leader election: the lowest lane of
// each hash slot wins an atomic min; lanes whose key differs from their
// leader's retry in a later round; peers of a leader are found by matching
// the 6 bits of the leader's lane id with ballots.  Every round completes at
// least the leader of each slot, so 64 rounds always suffice; the bound also
// guarantees termination.  Returns false on a lane left unranked (never
// expected).
__device__ __forceinline__ bool wave_stable_rank(bool ok, uint32_t key, uint32_t* counter,
                                                 uint32_t* tag, uint32_t& pos)
{
    const uint32_t lane = __lane_id();
    const uint32_t slot = key & 127u;
    uint64_t pending = __ballot(ok);
    pos = 0;
    for (int round = 0; pending && round < kWave; ++round) {
        const bool mine_pending = (pending >> lane) & 1ull;
        if (mine_pending)
            atomicMin(&tag[slot], lane);
        wave_sync();
        const uint32_t leader = mine_pending ? (tag[slot] & 63u) : lane;
        const uint32_t lkey = (uint32_t)__shfl((int)key, (int)leader);
        const bool mine = mine_pending && (lkey == key);
        uint64_t peers = __ballot(mine);
#pragma unroll
        for (int bit = 0; bit < 6; ++bit) {
            const bool lb = (leader >> bit) & 1u;
            const uint64_t bm = __ballot(mine && lb);
            peers &= lb ? bm : ~bm;
        }
        const uint64_t below = peers & ((1ull << lane) - 1ull);
        const uint32_t r = (uint32_t)__popcll(below);
        const uint32_t c = (uint32_t)__popcll(peers);
        uint32_t old = 0;
        if (mine && lane == leader) {
            old = counter[key];
            counter[key] = old + c;
            tag[slot] = 0xFFFFFFFFu;
        }
        wave_sync();
        old = (uint32_t)__shfl((int)old, (int)leader);
        if (mine)
            pos = old + r;
        pending &= ~__ballot(mine);
    }
    return !((pending >> lane) & 1ull);
}

}  // namespace esi
