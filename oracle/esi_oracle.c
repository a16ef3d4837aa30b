/*
 * esi_oracle.c -- plain, serial, FP64 CPU oracle for Event-based Single
 * Integration (ESI), Dong et al., "An Event-based Fast Intensity
 * Reconstruction Scheme for UAV Real-time Perception" (arXiv 2508.02238).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the package smoke check and the
 * CPU-baseline leg of the benchmark may call this file; the GPU library never
 * includes, links or calls it, and it shares no header, helper or constant
 * with the GPU library.
 *
 * What it computes, in the paper's order (Sec. III, Alg. 1 and Alg. 2):
 *   per event e_i = (x_i, y_i, p_i, t_i), in array order:
 *     S(x,y) <- S(x,y) + p_i * C                       (Alg. 2: accumulate the event)
 *     dt     <- t_i - T(x,y)                           (Alg. 2: time since the last event)
 *     S(x,y) <- S(x,y) * d(dt),  d from Eq. (4)        (Alg. 2: decay step)
 *     T(x,y) <- t_i                                    (Alg. 2: new last-event time)
 *     S(x,y) <- min(max(S, S_min), S_max)              (Eq. (13), applied per event as in Alg. 2)
 *   frame:  B = (S - S_min) / (S_max - S_min)           (Eq. (14), normalised to [0,1];
 *                                                        the 8-bit code is 255 times this)
 *
 * Readings taken where the paper is silent, ambiguous or garbled (each is
 * listed with its reason in the design notes of the repository):
 *   - Eq. (4) max{(1-kt)^b, 0} is read as a truncated power max(1-kt, 0)^b,
 *     so d = 0 once kt >= 1 (the power of a negative base is undefined for
 *     non-integer b).
 *   - dt is clamped at 0 for a time that goes backwards; equal times give d = 1.
 *   - T starts at t0 (default 0, as in Alg. 1/2), not at the first event.
 *   - Polarity: p > 0 is +1, anything else is -1.
 *   - Events with x >= W or y >= H are dropped and counted.
 *   - A frame at time t_f holds every event with t <= t_f (the condition
 *     t_n <= t < t_{n+1} under Eq. (5)).  It is a read-only snapshot: by
 *     default the state is decayed to t_f and clamped (the decay-to-query-time
 *     of Eq. (3)); flag LAZY maps S as stored, as Alg. 2's final loop does.
 *   - flag DECAY_THEN_ADD swaps the first two steps (decay, then add).
 *   - flag DECAY_EXP replaces Eq. (4) by the plain exponential decay
 *     d(dt) = exp(-k dt) of the accumulator plugin the paper compares against
 *     (Sec. II, and the runtime discussion of Sec. IV); b is then unused.
 *
 * Parity pins for every function here live in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define ORACLE_DECAY_THEN_ADD 1u
#define ORACLE_SNAPSHOT_LAZY 2u
#define ORACLE_DECAY_EXP 4u

/* Eq. (4): d(t) = max{(1 - k t)^b, 0}, read as max(1 - k t, 0)^b. */
double esi_oracle_decay(double dt, double k, double b)
{
    double u = 1.0 - k * dt;
    if (u <= 0.0)
        return 0.0;
    return pow(u, b);
}

/* The exponential decay of the accumulator plugin: d(t) = exp(-k t). */
double esi_oracle_decay_exp(double dt, double k)
{
    return exp(-k * dt);
}

/* The decay a call uses: Eq. (4), or the exponential one under DECAY_EXP. */
static double decay_of(double dt, double k, double b, uint32_t flags)
{
    if (flags & ORACLE_DECAY_EXP)
        return esi_oracle_decay_exp(dt, k);
    return esi_oracle_decay(dt, k, b);
}

/* Eq. (13). */
static double clamp_s(double s, double s_min, double s_max)
{
    if (s < s_min)
        s = s_min;
    if (s > s_max)
        s = s_max;
    return s;
}

/* Alg. 1/2 initialisation: S = 0, T = t0 (reading: the stream origin), plus
 * the per-pixel event count N and signed polarity sum P kept for exact
 * count parity. */
void esi_oracle_init_state(int64_t npix, int64_t t0, double *S, int64_t *T,
                           uint32_t *N, int32_t *P)
{
    for (int64_t q = 0; q < npix; ++q) {
        S[q] = 0.0;
        T[q] = t0;
        N[q] = 0;
        P[q] = 0;
    }
}

/* The value a pixel shows in a frame taken at t_f: Eq. (14) of the clamped
 * (Eq. (13)) estimate, decayed to t_f unless LAZY. */
static double frame_value(double S, int64_t T, int64_t t_f, double k, double b,
                          double s_min, double s_max, uint32_t flags)
{
    double v = S;
    if (!(flags & ORACLE_SNAPSHOT_LAZY)) {
        int64_t dt = t_f - T;
        if (dt < 0)
            dt = 0;
        v = clamp_s(S * decay_of((double)dt, k, b, flags), s_min, s_max);
    }
    return (v - s_min) / (s_max - s_min);
}

/* A standalone frame of the whole state at t_f (Alg. 2's final loop, Eq. (14)). */
void esi_oracle_snapshot(int64_t npix, const double *S, const int64_t *T,
                         int64_t t_f, double k, double b, double s_min,
                         double s_max, uint32_t flags, double *frame)
{
    for (int64_t q = 0; q < npix; ++q)
        frame[q] = frame_value(S[q], T[q], t_f, k, b, s_min, s_max, flags);
}

/* The 8-bit code of Eq. (14) for a normalised value F in [0, 1]: 255 F rounded
 * half up, clamped to [0, 255].  The paper gives no rounding rule; this
 * decision is taken in FP32 (the precision the GPU frames are kept in) with
 * separately rounded multiply and add. */
uint8_t esi_oracle_u8(double F)
{
    volatile float f = (float)F;
    volatile float m = 255.0f * f;
    volatile float a = m + 0.5f;
    float r = floorf(a);
    if (r < 0.0f)
        r = 0.0f;
    if (r > 255.0f)
        r = 255.0f;
    return (uint8_t)r;
}

/* A frame's rows [r0, r1) of the state at t_f (Eq. (14)); the part of
 * esi_oracle_snapshot that one row band owns. */
static void snapshot_rows(int32_t W, int32_t r0, int32_t r1, const double *S,
                          const int64_t *T, int64_t t_f, double k, double b,
                          double s_min, double s_max, uint32_t flags, double *frame)
{
    for (int64_t q = (int64_t)r0 * W; q < (int64_t)r1 * W; ++q)
        frame[q] = frame_value(S[q], T[q], t_f, k, b, s_min, s_max, flags);
}

/*
 * Alg. 2's event loop restricted to the pixels of rows [r0, r1): the events
 * of other rows are passed over (each pixel's update reads and writes only
 * that pixel, so the bands of a sensor are independent), and the frames are
 * written for these rows only.  Out-of-range events are counted by the band
 * that starts at row 0, decreasing times by every band.  The arguments are
 * those of esi_oracle_integrate below, which is this loop over all rows.
 */
void esi_oracle_integrate_rows(int32_t W, int32_t H, int32_t r0, int32_t r1,
                               double C, double k, double b, double s_min,
                               double s_max, uint32_t flags, double *S,
                               int64_t *T, uint32_t *N, int32_t *P, int64_t n,
                               const uint16_t *x, const uint16_t *y,
                               const int64_t *t, const int8_t *p, int32_t nf,
                               const int64_t *t_frames, const uint8_t *frame_sel,
                               double *frames, uint64_t *dropped, int32_t *unsorted)
{
    const int64_t npix = (int64_t)W * (int64_t)H;
    int32_t j = 0;
    int64_t nsel = 0;

    for (int64_t i = 0; i < n; ++i) {
        /* Frames strictly before this event's time see none of it. */
        while (j < nf && t_frames[j] < t[i]) {
            if (!frame_sel || frame_sel[j]) {
                if (frames)
                    snapshot_rows(W, r0, r1, S, T, t_frames[j], k, b, s_min,
                                  s_max, flags, frames + nsel * npix);
                ++nsel;
            }
            ++j;
        }
        if (i > 0 && t[i] < t[i - 1])
            *unsorted = 1;
        if (x[i] >= W || y[i] >= H) {
            if (r0 == 0)
                ++*dropped;
            continue;
        }
        if (y[i] < r0 || y[i] >= r1)
            continue;
        const int64_t q = (int64_t)y[i] * W + x[i];
        const int pol = (p[i] > 0) ? 1 : -1;
        int64_t dt = t[i] - T[q];
        if (dt < 0)
            dt = 0;
        const double d = decay_of((double)dt, k, b, flags);
        if (flags & ORACLE_DECAY_THEN_ADD)
            S[q] = S[q] * d + pol * C;
        else
            S[q] = (S[q] + pol * C) * d;
        T[q] = t[i];
        S[q] = clamp_s(S[q], s_min, s_max);
        N[q] += 1;
        P[q] += pol;
    }
    while (j < nf) {
        if (!frame_sel || frame_sel[j]) {
            if (frames)
                snapshot_rows(W, r0, r1, S, T, t_frames[j], k, b, s_min, s_max,
                              flags, frames + nsel * npix);
            ++nsel;
        }
        ++j;
    }
}

/*
 * Integrate n events into the state (Alg. 2's event loop) and emit frames.
 *
 * State arrays S, T, N, P have W*H entries, row-major q = y*W + x; they are
 * read and updated in place, so consecutive calls continue one stream.
 * t_frames[0..nf) are the frame times (non-decreasing).  Frame j is emitted
 * just before the first event with t > t_frames[j], or after the last event.
 * frame_sel (may be NULL = all) marks which frames are written out; the
 * selected frames are stored one after another in `frames` (W*H doubles each,
 * may be NULL).  Skipping a frame changes nothing else: frames are read-only.
 * *dropped counts out-of-range events, *unsorted is set to 1 if some event's
 * time is below its predecessor's in array order.
 */
void esi_oracle_integrate(int32_t W, int32_t H, double C, double k, double b,
                          double s_min, double s_max, uint32_t flags,
                          double *S, int64_t *T, uint32_t *N, int32_t *P,
                          int64_t n, const uint16_t *x, const uint16_t *y,
                          const int64_t *t, const int8_t *p, int32_t nf,
                          const int64_t *t_frames, const uint8_t *frame_sel,
                          double *frames, uint64_t *dropped, int32_t *unsorted)
{
    esi_oracle_integrate_rows(W, H, 0, H, C, k, b, s_min, s_max, flags, S, T, N,
                              P, n, x, y, t, p, nf, t_frames, frame_sel, frames,
                              dropped, unsorted);
}
