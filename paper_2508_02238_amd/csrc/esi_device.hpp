// esi_device.hpp -- device-side arithmetic and wave primitives shared by the
// kernels.
//
// Per event (Alg. 2, event loop): S <- (S + p C) d(dt), T <- t, S <- clamp(S)
// with d(dt) = max(1 - k dt, 0)^b (Eq. (4)) and the clamp of Eq. (13).  The
// kernels run it in FP64 registers: on CDNA4 an FP64 FMA issues at the same
// rate as an unpacked FP32 one, and FP64 keeps long runs of decay factors
// close to 1 well inside a 1e-5 relative error without compensated FP32
// arithmetic.  Frames (Eq. (14)) are rounded to FP32 once, at the end.
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
    double f_off;                             // -s_min * inv_range
    double sv_min, sv_max;                    // s_min * inv_range, s_max * inv_range
    int decay_then_add;
    int lazy;
    int exp_decay;   // d = exp(-k dt) instead of Eq. (4)
    int need_clamp;  // a decayed state can leave [s_min, s_max]
    // a pixel's run of more than scan_run events in one chunk goes through
    // the wave's scan of its per-event maps instead of one lane's loop
    // (kScanOff: never)
    int scan_run;
};

constexpr int kScanOff = 0x7FFFFFFF;

// How the decay is evaluated: Eq. (4), d = max(1 - k dt, 0)^b, with b = 1 and
// b = 2 exactly by multiplication and any other b by pow(); or the
// exponential decay exp(-k dt) of the accumulator plugin the paper compares
// against (Sec. II; Sec. IV ties its lower runtime to that cheaper function).
enum DecayKind { kDecayB1 = 1, kDecayB2 = 2, kDecayPow = 0, kDecayExp = 3 };

__device__ __noinline__ double decay_pow(double u, double b) { return pow(u, b); }

// u^b for u in [0, 1].
template <int BK>
__device__ __forceinline__ double power_b(double u, double b)
{
    if (BK == kDecayB1)
        return u;
    if (BK == kDecayB2)
        return u * u;
    return decay_pow(u, b);
}

// The decay from its base x = 1 - k dt (dt >= 0, so x <= 1 up to rounding):
// Eq. (4) clamps x to [0, 1] and raises it to b; the exponential decay is
// exp(x - 1).
template <int BK>
__device__ __forceinline__ double decay_from_base(double x, double b)
{
    if (BK == kDecayExp)
        return exp(fmin(x, 1.0) - 1.0);
    return power_b<BK>(fmin(fmax(x, 0.0), 1.0), b);
}

// Eq. (4) as a truncated power: d(dt) = max(1 - k dt, 0)^b, dt >= 0 integer
// us; or exp(-k dt).
template <int BK>
__device__ __forceinline__ double decay(const MethodParams& mp, int64_t dt)
{
    if (BK == kDecayExp)
        return exp(-mp.k * (double)dt);
    const double u = __fma_rn(-mp.k, (double)dt, 1.0);
    return (u > 0.0) ? power_b<BK>(u, mp.b) : 0.0;
}

__device__ __forceinline__ double clamp_s(const MethodParams& mp, double s)
{
    return fmin(fmax(s, mp.s_min), mp.s_max);
}

// Eq. (14) of the state seen at t_f (decayed to t_f unless lazy), in [0, 1].
template <int BK>
__device__ __forceinline__ float frame_value(const MethodParams& mp, double S, int64_t T,
                                             int64_t t_f)
{
    double v = S;
    if (!mp.lazy) {
        int64_t dt = t_f - T;
        dt = dt < 0 ? 0 : dt;
        v = clamp_s(mp, S * decay<BK>(mp, dt));
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

// Read-only data that stays unchanged for the whole kernel, read at a
// wave-uniform index: through the constant address space the compiler emits
// scalar loads (a vector load would be waited for with the same counter as
// the kernel's earlier stores).
template <typename T>
__device__ __forceinline__ T load_const(const T* p, int64_t i)
{
    return ((const __attribute__((address_space(4))) T*)p)[i];
}

// Ordering point for LDS traffic between the lanes of one wave: the lanes
// of a wave issue in lockstep and LDS serves a wave's requests in order, so a
// fence at wavefront scope plus a compiler barrier suffice.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---- the per-event map of Alg. 2 and its composition ------------------------
//
// One event of a pixel maps the state S to clamp(a S + b, lo, hi) (Eq. (13)'s
// clamp after the add and the decay of Alg. 1/2): add then decay gives
// a = d, b = d p C; decay then add gives a = d, b = p C; lo, hi = S_min, S_max.
// With a >= 0 these maps are closed under composition (Eq. (5) unrolls the
// same recurrence into products of decay factors):
//   (g after f)(x) = clamp(g.a f.a x + g.a f.b + g.b, L, H),
//   L = clamp(g.a f.lo + g.b, g.lo, g.hi),  H = clamp(g.a f.hi + g.b, g.lo, g.hi),
// because x -> g.a x + g.b is non-decreasing and a clamp of a clamp is the
// clamp to the clamped bounds.  Composition is associative, so the states
// after every event of a run are an inclusive scan of its maps.
struct ClampAffine {
    double a, b, lo, hi;
};

__device__ __forceinline__ ClampAffine clamp_affine_identity()
{
    return ClampAffine{1.0, 0.0, -1.7976931348623157e308, 1.7976931348623157e308};
}

// g after f.
__device__ __forceinline__ ClampAffine compose(const ClampAffine& f, const ClampAffine& g)
{
    ClampAffine r;
    r.a = g.a * f.a;
    r.b = __fma_rn(g.a, f.b, g.b);
    r.lo = fmin(fmax(__fma_rn(g.a, f.lo, g.b), g.lo), g.hi);
    r.hi = fmin(fmax(__fma_rn(g.a, f.hi, g.b), g.lo), g.hi);
    return r;
}

__device__ __forceinline__ double apply(const ClampAffine& f, double x)
{
    return fmin(fmax(__fma_rn(f.a, x, f.b), f.lo), f.hi);
}

// A double moved across lanes by a DPP control (two 32-bit moves); lanes the
// control gives no source (or that ROW_MASK leaves out) take `old`.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_f64(double old, double src)
{
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), CTRL, ROW_MASK,
                                               0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void scan_step(ClampAffine& m)
{
    const ClampAffine id = clamp_affine_identity();
    ClampAffine p;
    p.a = dpp_f64<CTRL, ROW_MASK>(id.a, m.a);
    p.b = dpp_f64<CTRL, ROW_MASK>(id.b, m.b);
    p.lo = dpp_f64<CTRL, ROW_MASK>(id.lo, m.lo);
    p.hi = dpp_f64<CTRL, ROW_MASK>(id.hi, m.hi);
    m = compose(p, m);  // the earlier lanes' map first
}

// Inclusive scan of the lanes' maps in lane order: lane l returns map_l after
// ... after map_0.  Rows of 16 lanes first (shifts by 1, 2, 4, 8), then row
// 0's total into row 1 and row 2's into row 3 (row_bcast:15), then rows 0-1's
// total into rows 2 and 3 (row_bcast:31).  Lanes without a source compose
// the identity.
__device__ __forceinline__ ClampAffine wave_scan(ClampAffine m)
{
    scan_step<0x111, 0xF>(m);  // row_shr:1
    scan_step<0x112, 0xF>(m);  // row_shr:2
    scan_step<0x114, 0xF>(m);  // row_shr:4
    scan_step<0x118, 0xF>(m);  // row_shr:8
    scan_step<0x142, 0xA>(m);  // row_bcast:15 into rows 1 and 3
    scan_step<0x143, 0xC>(m);  // row_bcast:31 into rows 2 and 3
    return m;
}

// Lane l's double, read by the whole wave (l uniform).
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFF), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Lane l's 64-bit integer, read by the whole wave (l uniform).
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l)
{
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xFFFFFFFF), l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Stable multisplit rank inside one wave step.  Lane l holds an element with
// key `key` < 2^KEY_BITS (valid when `ok`); lanes are in array order.
// Returns, for valid lanes, counter[key] (before this step) plus the number of
// lower valid lanes with the same key, and advances counter[key] by the
// number of valid lanes with that key.  The lanes sharing a key are found by
// matching the key one bit at a time with ballots (a wave-wide match), so the
// ranks are stable without atomics.
template <int KEY_BITS, typename CounterT>
__device__ __forceinline__ uint32_t wave_stable_rank(bool ok, uint32_t key, CounterT* counter)
{
    const uint32_t lane = __lane_id();
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < KEY_BITS; ++bit) {
        const bool lb = (key >> bit) & 1u;
        const uint64_t bm = __ballot(lb);
        peers &= lb ? bm : ~bm;
    }
    const uint32_t r = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    const uint32_t c = (uint32_t)__popcll(peers);
    const uint32_t base = ok ? (uint32_t)counter[key] : 0u;
    wave_sync();  // every lane has read its counter before the update
    if (ok && r + 1u == c)
        counter[key] = (CounterT)(base + c);  // the last lane of each key group
    wave_sync();
    return base + r;
}

// The same rank with the key's lanes found through LDS: the lanes of a key
// agree on a representative lane (each writes its lane number to slot[key],
// one write per key survives), clear the representative's word of `group`,
// and OR their own lane bits into it; the word then holds the key's lane
// mask.  OR is order-independent, so the result does not depend on how LDS
// serialises lanes that hit one word.  slot: one byte per key, group: 64
// words; neither needs initialisation.  The counter of key k is
// counter[k * STRIDE].
template <int STRIDE = 1, typename CounterT>
__device__ __forceinline__ uint32_t wave_stable_rank_or(bool ok, uint32_t key, CounterT* counter,
                                                        uint8_t* slot, uint64_t* group)
{
    const uint32_t lane = __lane_id();
    if (ok)
        slot[key] = (uint8_t)lane;
    wave_sync();
    uint32_t rep = 0, base = 0;
    if (ok) {
        rep = slot[key];
        base = (uint32_t)counter[key * STRIDE];
        group[rep] = 0;
        __hip_atomic_fetch_or(&group[rep], 1ull << lane, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    wave_sync();
    const uint64_t peers = ok ? group[rep] : 0ull;
    const uint32_t r = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    const uint32_t c = (uint32_t)__popcll(peers);
    if (ok && r + 1u == c)
        counter[key * STRIDE] = (CounterT)(base + c);  // the last lane of each key group
    wave_sync();
    return base + r;
}

}  // namespace esi
