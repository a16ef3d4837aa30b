/*
 * esi.h -- C ABI of the MI355X (gfx950) implementation of Event-based Single
 * Integration (ESI): Dong et al., "An Event-based Fast Intensity
 * Reconstruction Scheme for UAV Real-time Perception", arXiv 2508.02238.
 *
 * What the library computes (Sec. III of the paper):
 *   For every event e_i = (x_i, y_i, p_i, t_i), in the order given, at the
 *   event's pixel q = y*W + x (Alg. 2, event loop):
 *       S[q] <- (S[q] + p_i C) * d(t_i - T[q])        add, then decay (Alg. 1/2)
 *       T[q] <- t_i
 *       S[q] <- min(max(S[q], S_min), S_max)           clamp, Eq. (13)
 *   with the decay of Eq. (4), d(t) = max(1 - k t, 0)^b.
 *   A frame at time t_f holds, for each pixel, the state after all events
 *   with t <= t_f (Eq. (5): t_n <= t < t_{n+1}), mapped by Eq. (14) to
 *       F = (v - S_min) / (S_max - S_min) in [0, 1]   (8-bit code: 255 F)
 *   where v = clamp(S[q] d(t_f - T[q])) is the state decayed to t_f (the
 *   decay-to-query-time of Eq. (3)); ESI_SNAPSHOT_LAZY gives v = S[q], as
 *   the final loop of Alg. 2 maps S directly.  Frames never change state.
 *
 * Readings where the paper is silent (the same in the CPU reference used to
 * test this library):
 *   - d = 0 once k t >= 1 (the truncated power), equal times give d = 1, and
 *     a time below T[q] is treated as dt = 0 (T[q] still becomes t_i).
 *   - T starts at params.t0_us (Alg. 1/2 start it at 0, the default).
 *   - polarity p > 0 is +1, anything else -1 (accepts {+1,-1} and {1,0}).
 *   - events with x >= W or y >= H are dropped and counted, not an error.
 *   - events of one pixel are applied in array order, also when times tie
 *     (the clamp makes the order matter).
 *   - the 8-bit code is floor(255 F + 1/2) in FP32, at most 255.
 *
 * Layout and ownership:
 *   - Every pointer argument marked "device" is device memory of the GPU the
 *     state was created on (hipMalloc, torch tensors); the caller owns it and
 *     keeps it alive until the stream has consumed it.
 *   - The library owns the state (per pixel S: f32 plus an f32 correction
 *     term, T: i64, N: u32 event count, P: i32 signed polarity sum; 24 B per
 *     pixel in HBM) and its scratch, allocated on the stream.
 *   - All compute calls are asynchronous and ordered on `stream`; one state
 *     is used by one stream at a time, and a state is not thread-safe.
 *   - Frames are [n_frames][H][W] row-major, FP32 normalised to [0, 1], and
 *     optionally as 8-bit codes in a second [n_frames][H][W] buffer.
 *
 * Errors: every call returns an esi_status.  Invalid arguments are detected
 * on the host before anything is enqueued and leave the state unchanged.
 * A HIP runtime failure returns ESI_ERR_HIP and poisons the state: every
 * later compute call returns ESI_ERR_POISONED until esi_reset or
 * esi_import_state succeeds.  Conditions found in the data on the device
 * (dropped events, decreasing times, unsorted frame times, a call spanning
 * 2^47 us or more) are not errors: they are counted or flagged and read back
 * with esi_get_diagnostics.
 */
#ifndef ESI_H
#define ESI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ESI_OK = 0,
    ESI_ERR_INVALID_ARG = 1,
    ESI_ERR_OUT_OF_MEMORY = 2,
    ESI_ERR_HIP = 3,
    ESI_ERR_POISONED = 4,
    ESI_ERR_SCRATCH_LIMIT = 5, /* esi_integrate_window_noalloc: call too large */
} esi_status;

/* params.flags */
enum {
    ESI_ADD_THEN_DECAY = 0,        /* Alg. 1/2 order: add p C, then decay (default) */
    ESI_DECAY_THEN_ADD = 1u << 0,  /* decay, then add */
    ESI_SNAPSHOT_DECAYED = 0,      /* frame shows clamp(S d(t_f - T)) (default) */
    ESI_SNAPSHOT_LAZY = 1u << 1,   /* frame shows S as stored (Alg. 2's map loop) */
    ESI_DECAY_EXP = 1u << 2,       /* d(dt) = exp(-k dt) in place of Eq. (4), for every event
                                      and snapshot (b unused): the exponential decay of the
                                      event-accumulator plugin the paper compares ESI with
                                      (Sec. II; Sec. IV attributes the plugin's lower runtime
                                      to this cheaper function) */
};

/* diag.flags */
enum {
    ESI_DIAG_UNSORTED = 1u << 0,     /* some event time below its predecessor's */
    ESI_DIAG_FRAMES_UNSORTED = 1u << 1, /* t_frames decreasing: frames unspecified */
    ESI_DIAG_TIME_RANGE = 1u << 2,   /* a call's events span >= 2^47 us: results unspecified */
    ESI_DIAG_INTERNAL = 1u << 3,     /* an internal consistency check failed (a bug) */
};

/* Inputs of Alg. 1/2 (k, b, C) and the clamp bounds of Eq. (13). */
typedef struct {
    double C;        /* contrast threshold c, log-intensity step per event; > 0 */
    double k_per_us; /* decay rate k of Eq. (4), 1/us; >= 0 (0: no decay, Eq. (2)) */
    double b;        /* decay exponent b of Eq. (4); > 0 */
    double s_min;    /* S_min of Eq. (13)-(14) */
    double s_max;    /* S_max of Eq. (13)-(14); > s_min */
    int64_t t0_us;   /* initial T (stream origin), us */
    uint32_t flags;  /* ESI_* flags above */
} esi_params;

/* Events, structure of arrays in device memory, n entries each. */
typedef struct {
    const uint16_t *x; /* column, [0, W) */
    const uint16_t *y; /* row, [0, H) */
    const int64_t *t;  /* time stamp, us */
    const int8_t *p;   /* polarity */
    size_t n;
} esi_events;

typedef struct {
    uint64_t dropped;      /* events with x >= W or y >= H, all calls so far */
    uint64_t accepted;     /* events integrated, all calls so far */
    uint32_t flags;        /* ESI_DIAG_* seen in any call so far */
    uint32_t poisoned;     /* nonzero after a HIP failure */
    uint64_t calls;        /* esi_integrate_window calls */
} esi_diag;

typedef struct esi_state esi_state;

/* Create a state for a W x H sensor: S = 0, T = t0_us, N = P = 0 (Alg. 1/2
 * initialisation).  1 <= W, H <= 65536 (every 16-bit coordinate).  The state
 * lives on the current HIP device (24 B per pixel: 103 GB for 65536 x 65536;
 * ESI_ERR_OUT_OF_MEMORY if it does not fit).  A sensor of more than 4096000
 * pixels is integrated in bands of rows of at most that many pixels, one pass
 * over the events per band.  On success *out receives the state; the
 * initialisation is enqueued on `stream`. */
esi_status esi_create_state(int32_t width, int32_t height, const esi_params *params,
                            hipStream_t stream, esi_state **out);

/* Free the state and its scratch (synchronises the state's device). */
esi_status esi_destroy_state(esi_state *st);

/* Back to the initial state (S = 0, T = t0_us, N = P = 0); clears the
 * diagnostics and the poisoned flag. */
esi_status esi_reset(esi_state *st, hipStream_t stream);

/* Integrate ev->n events (Alg. 2's event loop, in array order per pixel)
 * and write n_frames frames (Eq. (14)) taken at t_frames[j].
 *   ev        device SoA events; ev->n may be 0.  Expected time-sorted; if
 *             not, the state is still that of array order, the frames of
 *             this call are unspecified and ESI_DIAG_UNSORTED is set.
 *   t_frames  n_frames non-decreasing times (us), in device or host memory
 *             (host memory is detected with hipPointerGetAttributes and
 *             copied to the library's scratch on `stream`; keep it unchanged
 *             until the stream has consumed it); NULL iff n_frames is 0.
 *             Frame j includes the events with t <= t_frames[j] and the
 *             events of earlier calls.
 *   frames    device f32 [n_frames][H][W], or NULL.
 *   frames_u8 device u8 [n_frames][H][W], or NULL.
 * n_frames >= 0; n_frames > 0 needs frames or frames_u8.  The call spans
 * less than 2^47 us (about 4.5 years) from its first event's time, and
 * ev->n < 2^31. */
esi_status esi_integrate_window(esi_state *st, const esi_events *ev, const int64_t *t_frames,
                                int32_t n_frames, float *frames, uint8_t *frames_u8,
                                hipStream_t stream);

/* esi_integrate_window for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the call's scratch (tile
 * histogram, its scan and the 8-byte tile-bucketed event records) in a fixed
 * 64 MiB array that the library holds in each GPU's memory until the process
 * ends, so the call allocates and frees nothing.  The state must exist
 * already (esi_create_state allocates it and looks the array up on its
 * device); inputs and outputs are the caller's, as for esi_integrate_window,
 * except that t_frames must be device memory (ESI_ERR_INVALID_ARG
 * otherwise: nothing is staged).  A call whose scratch exceeds the array
 * (about 8 bytes per event plus 4 bytes per (tile, bucketing range): some
 * 7.9M events on a 1280 x 720 sensor, more on smaller ones) returns
 * ESI_ERR_SCRATCH_LIMIT before anything is enqueued; split it into several
 * calls.  Every call on one GPU uses that GPU's one array: calls that overlap
 * on one GPU (different streams, different threads) race and must be
 * serialised by the caller; each call initialises all of the scratch it
 * reads, so nothing carries over from the previous call. */
esi_status esi_integrate_window_noalloc(esi_state *st, const esi_events *ev,
                                        const int64_t *t_frames, int32_t n_frames,
                                        float *frames, uint8_t *frames_u8, hipStream_t stream);

/* One frame of the current state at t_frame_us (Alg. 2's final loop with
 * Eq. (14); decayed to t_frame_us unless ESI_SNAPSHOT_LAZY).  frame: device
 * f32 [H][W] or NULL; u8: device [H][W] or NULL; not both NULL.  Read-only
 * on the state. */
esi_status esi_snapshot_frame(esi_state *st, int64_t t_frame_us, float *frame, uint8_t *u8,
                              hipStream_t stream);

/* Copy the state to device buffers of W*H entries (any may be NULL):
 * S as f32 (the rounded value), T, N, P. */
esi_status esi_read_state(esi_state *st, float *S, int64_t *T, uint32_t *N, int32_t *P,
                          hipStream_t stream);

/* Bytes of a serialised state (header + 24 B per pixel). */
size_t esi_state_bytes(const esi_state *st);

/* Serialise the state into host memory (bytes >= esi_state_bytes); waits
 * for the state's stream work to finish. */
esi_status esi_export_state(esi_state *st, void *host_buf, size_t bytes);

/* Restore a state written by esi_export_state for the same W, H; clears the
 * poisoned flag.  Waits for the copy to finish. */
esi_status esi_import_state(esi_state *st, const void *host_buf, size_t bytes);

/* Read the diagnostics (waits for the state's stream work to finish). */
esi_status esi_get_diagnostics(esi_state *st, esi_diag *out);

/* Tile size of the integration kernels for later calls on this state: 256,
 * 512, 1024 or 2048 pixels (the smallest allowed: a sensor (or band) whose
 * tiles would be more than 2000 gets the next larger size), or 0 for the
 * default (the smallest size with at most 2000 tiles).  N, P and T do not depend on it, S
 * and frames only to rounding (decay bases are taken per chunk of a tile's
 * events); for calls with few events per tile larger tiles shorten the
 * per-tile chains of dependent memory accesses, for event-dense calls
 * smaller tiles give more workgroups (an autotuner picks it per workload). */
esi_status esi_set_tile_pixels(esi_state *st, int32_t tile_pixels);

/* Phase A's split between its two forms of the same recurrence (Alg. 2's
 * event loop; the per-event maps composed as in Eq. (5)), for later calls on
 * this state: within one chunk of a tile's events, a pixel's run of at most
 * scan_run events is integrated by its own lane, one event after the other,
 * and a longer run by its whole wave, 64 events at a time, as a scan of the
 * per-event clamp-affine maps (hot pixels and same-time bursts).  scan_run
 * >= 0; INT32_MAX turns the scan off; 0 for the default: 64 for tiles of
 * 512 pixels and more, off for 256-pixel tiles (their one-pixel-per-thread
 * kernel is slowed by the scan's code alone, so it is compiled without it
 * unless a threshold is set).  N, P and T do not depend on it, S and frames
 * only to rounding. */
esi_status esi_set_scan_run(esi_state *st, int32_t scan_run);

/* Records per chunk of the integration for tiles of 512 pixels (two pixels
 * per thread), for later calls on this state: 0 or 1536 (the default: four
 * workgroups per CU) or 2048 (three workgroups per CU).  Larger chunks take a
 * tile's events in fewer passes of the in-tile sort and of Alg. 2's event
 * loop; that pays on hot pixels and frame-heavy calls (1280x720 with hot
 * pixels: 8% less integration time), and costs where the tiles outnumber
 * the resident workgroups and differ in length (1280x720 spokes at 100 FPS:
 * 15% more).  Other tile sizes ignore it; esi_integrate_batch takes each
 * state's setting.  Results are the same up to rounding; N, P and T exactly.
 * ESI_ERR_INVALID_ARG for other values. */
esi_status esi_set_chunk(esi_state *st, int32_t records);

/* An upper bound of the device scratch that one state of a W x H sensor
 * allocates for integrate calls (esi_integrate_window or esi_integrate_batch)
 * of at most n_events events each, growth margin included: what a caller that
 * budgets device memory per state (a server admitting sessions) must reserve
 * beside the state itself (esi_state_bytes).  Uses the current device. */
esi_status esi_scratch_bound(int32_t width, int32_t height, size_t n_events, size_t *bytes);

/* Sensor size of a state. */
esi_status esi_get_size(const esi_state *st, int32_t *width, int32_t *height);

/* Per-phase GPU timing of integrate calls, for measurement.  While enabled,
 * every esi_integrate_window call records HIP events on its stream around
 * its two phases: bucketing (histogram, scan and stable scatter of the
 * events by pixel tile) and integration (the per-tile event loop of Alg. 2
 * with the frames of Eq. (14)).  Enabling clears earlier records; up to 1024
 * calls are recorded.  esi_profile_read waits for the recorded calls and
 * returns their number and the summed milliseconds of each phase. */
esi_status esi_profile_enable(esi_state *st, int enable);
esi_status esi_profile_read(esi_state *st, uint32_t *calls, double *bucket_ms,
                            double *integrate_ms);

/* ---- many streams per launch -------------------------------------------
 * The same integration (Alg. 2 per pixel, frames by Eq. (14)) for many
 * independent states at once: each launch of the bucketing and integration
 * kernels covers the work of every stream (per stream: its bucketing ranges,
 * table scan and tiles, laid out one after the other), instead of one set
 * of launches per stream.  Results are those of one esi_integrate_window call
 * per item, bit for bit.
 *
 * A batch object owns the staging of the per-stream descriptors (pinned host
 * memory and a device copy, sized for max_items, 1..4096) on the current
 * device. */
typedef struct esi_batch esi_batch;
esi_status esi_batch_create(int32_t max_items, esi_batch **out);
/* Synchronises the batch's device (earlier calls may still read it). */
esi_status esi_batch_destroy(esi_batch *batch);

/* Item i integrates events[i] into states[i] and writes n_frames[i] frames
 * at t_frames[i] into frames[i] / frames_u8[i], with the rules of
 * esi_integrate_window for each item (buffers in device memory of the
 * batch's device, frame times in device or host memory).  states: n_items distinct states (host array of
 * pointers); events: host array of n_items descriptors.  t_frames, n_frames,
 * frames, frames_u8: host arrays of n_items entries, or NULL for "no frames"
 * / "no such output" for every item.  1 <= n_items <= max_items.  Argument
 * errors return ESI_ERR_INVALID_ARG before anything is enqueued (also for a
 * state of more than 4096000 pixels, which only esi_integrate_window
 * integrates, band by band); t_frames[i] may be host memory (packed into the
 * batch's staging and copied with the descriptors); a poisoned
 * state returns ESI_ERR_POISONED; a HIP failure poisons every state of the
 * call.  The call may wait for the previous call's descriptor copy (host
 * side) and for the stream when a state's scratch must grow; its descriptor
 * copy waits (on the device) for the previous call's kernels, so successive
 * calls on one batch object may use different streams. */
esi_status esi_integrate_batch(esi_batch *batch, int32_t n_items, esi_state *const *states,
                               const esi_events *events, const int64_t *const *t_frames,
                               const int32_t *n_frames, float *const *frames,
                               uint8_t *const *frames_u8, hipStream_t stream);

/* Static text for a status code. */
const char *esi_status_string(esi_status s);

#ifdef __cplusplus
}
#endif

#endif /* ESI_H */
