/*
 * sanitize_driver.c -- runs the CPU oracle and the event generator on small
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitize.py builds and runs it).  The sanitizers abort on their
 * first finding; exit status 0 means every run completed and each checked
 * property held.
 *
 * Runs: every scene of the generator (with and without tuning, noise and hot
 * pixels, several thread counts); on each stream the oracle's whole-stream
 * integration under every flag combination, the same stream in two calls
 * and in row bands (which must give the same state), standalone snapshots
 * and 8-bit codes, and malformed input (events off the sensor, decreasing
 * times, an empty call).
 */
#include "../evgen/evgen.c"

#include <stdio.h>

void esi_oracle_init_state(int64_t npix, int64_t t0, double *S, int64_t *T, uint32_t *N,
                           int32_t *P);
void esi_oracle_snapshot(int64_t npix, const double *S, const int64_t *T, int64_t t_f, double k,
                         double b, double s_min, double s_max, uint32_t flags, double *frame);
uint8_t esi_oracle_u8(double F);
void esi_oracle_integrate_rows(int32_t W, int32_t H, int32_t r0, int32_t r1, double C, double k,
                               double b, double s_min, double s_max, uint32_t flags, double *S,
                               int64_t *T, uint32_t *N, int32_t *P, int64_t n, const uint16_t *x,
                               const uint16_t *y, const int64_t *t, const int8_t *p, int32_t nf,
                               const int64_t *t_frames, const uint8_t *frame_sel, double *frames,
                               uint64_t *dropped, int32_t *unsorted);
void esi_oracle_integrate(int32_t W, int32_t H, double C, double k, double b, double s_min,
                          double s_max, uint32_t flags, double *S, int64_t *T, uint32_t *N,
                          int32_t *P, int64_t n, const uint16_t *x, const uint16_t *y,
                          const int64_t *t, const int8_t *p, int32_t nf, const int64_t *t_frames,
                          const uint8_t *frame_sel, double *frames, uint64_t *dropped,
                          int32_t *unsorted);

static int failures = 0;

#define CHECK(cond, ...)                                                                      \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            fprintf(stderr, "check failed (%s:%d): ", __FILE__, __LINE__);                  \
            fprintf(stderr, __VA_ARGS__);                                                     \
            fputc('\n', stderr);                                                              \
            ++failures;                                                                       \
        }                                                                                     \
    } while (0)

typedef struct {
    int32_t W, H;
    int64_t n;
    uint16_t *x, *y;
    int64_t *t;
    int8_t *p;
} stream_t;

typedef struct {
    double *S;
    int64_t *T;
    uint32_t *N;
    int32_t *P;
} state_t;

static void *xmalloc(size_t bytes)
{
    void *v = malloc(bytes ? bytes : 1);
    if (!v) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return v;
}

static state_t state_new(int64_t npix)
{
    state_t s = {(double *)xmalloc(sizeof(double) * npix), (int64_t *)xmalloc(sizeof(int64_t) * npix),
                 (uint32_t *)xmalloc(sizeof(uint32_t) * npix),
                 (int32_t *)xmalloc(sizeof(int32_t) * npix)};
    esi_oracle_init_state(npix, 0, s.S, s.T, s.N, s.P);
    return s;
}

static void state_free(state_t *s)
{
    free(s->S);
    free(s->T);
    free(s->N);
    free(s->P);
}

static int state_equal(const state_t *a, const state_t *b, int64_t npix)
{
    return !memcmp(a->S, b->S, sizeof(double) * npix) && !memcmp(a->T, b->T, sizeof(int64_t) * npix) &&
           !memcmp(a->N, b->N, sizeof(uint32_t) * npix) && !memcmp(a->P, b->P, sizeof(int32_t) * npix);
}

static int generate(const evgen_cfg *cfg, stream_t *s)
{
    int64_t n = 0;
    double tuned = 0.0;
    void *h = evgen_generate(cfg, &n, &tuned);
    if (!h)
        return 0;
    s->W = cfg->W;
    s->H = cfg->H;
    s->n = n;
    s->x = (uint16_t *)xmalloc(sizeof(uint16_t) * n);
    s->y = (uint16_t *)xmalloc(sizeof(uint16_t) * n);
    s->t = (int64_t *)xmalloc(sizeof(int64_t) * n);
    s->p = (int8_t *)xmalloc((size_t)n);
    evgen_fetch(h, s->x, s->y, s->t, s->p);
    return 1;
}

static void stream_free(stream_t *s)
{
    free(s->x);
    free(s->y);
    free(s->t);
    free(s->p);
}

/* The oracle over one stream: every flag combination, whole, split in two
 * calls, and in row bands; standalone snapshots and 8-bit codes. */
static void exercise(const stream_t *s, int64_t duration_us)
{
    const int64_t npix = (int64_t)s->W * s->H;
    const double C = 0.2, k = 2e-5, b = 2.0, s_min = -1.0, s_max = 1.0;
    const int32_t nf = 8;
    int64_t tf[8];
    for (int j = 0; j < nf; ++j)
        tf[j] = (j + 1) * duration_us / nf - 1;
    const uint32_t flag_sets[] = {0u, 1u, 2u, 4u, 5u, 6u, 7u};
    double *frames = (double *)xmalloc(sizeof(double) * npix * nf);
    double *frames2 = (double *)xmalloc(sizeof(double) * npix * nf);
    double *snap = (double *)xmalloc(sizeof(double) * npix);
    for (size_t fi = 0; fi < sizeof(flag_sets) / sizeof(flag_sets[0]); ++fi) {
        const uint32_t flags = flag_sets[fi];
        const double bb = (flags & 4u) ? 0.0 : b;
        state_t a = state_new(npix), c = state_new(npix), d = state_new(npix);
        uint64_t dropped = 0;
        int32_t unsorted = 0;
        esi_oracle_integrate(s->W, s->H, C, k, bb, s_min, s_max, flags, a.S, a.T, a.N, a.P, s->n,
                             s->x, s->y, s->t, s->p, nf, tf, NULL, frames, &dropped, &unsorted);
        CHECK(dropped == 0 && unsorted == 0, "generated stream: dropped %llu unsorted %d",
              (unsigned long long)dropped, (int)unsorted);
        for (int64_t q = 0; q < npix * nf; ++q)
            CHECK(frames[q] >= 0.0 && frames[q] <= 1.0, "frame value %g out of [0, 1]", frames[q]);
        for (int64_t q = 0; q < npix; ++q)
            CHECK(a.S[q] >= s_min && a.S[q] <= s_max, "S %g outside the clamp", a.S[q]);

        /* two calls split at the middle event: the same state */
        const int64_t h = s->n / 2;
        esi_oracle_integrate(s->W, s->H, C, k, bb, s_min, s_max, flags, c.S, c.T, c.N, c.P, h,
                             s->x, s->y, s->t, s->p, 0, NULL, NULL, NULL, &dropped, &unsorted);
        esi_oracle_integrate(s->W, s->H, C, k, bb, s_min, s_max, flags, c.S, c.T, c.N, c.P,
                             s->n - h, s->x + h, s->y + h, s->t + h, s->p + h, 0, NULL, NULL, NULL,
                             &dropped, &unsorted);
        CHECK(state_equal(&a, &c, npix), "split call changed the state (flags %u)", flags);

        /* row bands: the same state and frames */
        const int32_t bands[] = {0, s->H / 3, s->H / 2 + 1, s->H};
        for (int bi = 0; bi < 3; ++bi)
            esi_oracle_integrate_rows(s->W, s->H, bands[bi], bands[bi + 1], C, k, bb, s_min, s_max,
                                      flags, d.S, d.T, d.N, d.P, s->n, s->x, s->y, s->t, s->p, nf,
                                      tf, NULL, frames2, &dropped, &unsorted);
        CHECK(state_equal(&a, &d, npix), "row bands changed the state (flags %u)", flags);
        CHECK(!memcmp(frames, frames2, sizeof(double) * npix * nf),
              "row bands changed the frames (flags %u)", flags);

        /* a standalone snapshot at the last frame time equals that frame */
        esi_oracle_snapshot(npix, a.S, a.T, tf[nf - 1], k, bb, s_min, s_max, flags, snap);
        if (s->n == 0 || s->t[s->n - 1] <= tf[nf - 1])
            CHECK(!memcmp(snap, frames + (int64_t)(nf - 1) * npix, sizeof(double) * npix),
                  "snapshot differs from the last frame (flags %u)", flags);
        unsigned sum = 0;
        for (int64_t q = 0; q < npix; ++q)
            sum += esi_oracle_u8(snap[q]);
        (void)sum;
        state_free(&a);
        state_free(&c);
        state_free(&d);
    }
    free(frames);
    free(frames2);
    free(snap);
}

/* Malformed input: events off the sensor are dropped and counted, a
 * decreasing time is flagged, an empty call with frames writes them. */
static void malformed(const stream_t *s)
{
    if (s->n < 4)
        return;
    const int64_t npix = (int64_t)s->W * s->H;
    stream_t m = *s;
    m.x = (uint16_t *)xmalloc(sizeof(uint16_t) * s->n);
    m.y = (uint16_t *)xmalloc(sizeof(uint16_t) * s->n);
    m.t = (int64_t *)xmalloc(sizeof(int64_t) * s->n);
    memcpy(m.x, s->x, sizeof(uint16_t) * s->n);
    memcpy(m.y, s->y, sizeof(uint16_t) * s->n);
    memcpy(m.t, s->t, sizeof(int64_t) * s->n);
    m.x[1] = (uint16_t)(s->W + 3);
    m.y[2] = (uint16_t)65535;
    m.t[3] = m.t[0] - 1000; /* earlier than every event before it */
    state_t a = state_new(npix);
    uint64_t dropped = 0;
    int32_t unsorted = 0;
    int64_t tf[2] = {m.t[s->n - 1], m.t[s->n - 1] + 5000000};
    double *frames = (double *)xmalloc(sizeof(double) * npix * 2);
    esi_oracle_integrate(m.W, m.H, 0.2, 2e-5, 1.5, -1.0, 1.0, 0u, a.S, a.T, a.N, a.P, m.n, m.x,
                         m.y, m.t, m.p, 2, tf, NULL, frames, &dropped, &unsorted);
    CHECK(dropped == 2, "dropped %llu, expected 2", (unsigned long long)dropped);
    CHECK(unsorted == 1, "decreasing time not flagged");
    /* an empty call with frames */
    esi_oracle_integrate(m.W, m.H, 0.2, 2e-5, 1.5, -1.0, 1.0, 0u, a.S, a.T, a.N, a.P, 0, NULL, NULL,
                         NULL, NULL, 2, tf, NULL, frames, &dropped, &unsorted);
    for (int64_t q = 0; q < npix * 2; ++q)
        CHECK(frames[q] >= 0.0 && frames[q] <= 1.0, "empty-call frame value %g", frames[q]);
    free(frames);
    state_free(&a);
    free(m.x);
    free(m.y);
    free(m.t);
}

int main(void)
{
    const int64_t D = 200000;
    for (int scene = 0; scene <= 3; ++scene) {
        for (int variant = 0; variant < 3; ++variant) {
            evgen_cfg cfg;
            memset(&cfg, 0, sizeof(cfg));
            cfg.scene = scene;
            cfg.W = variant == 2 ? 37 : 48;
            cfg.H = variant == 2 ? 23 : 32;
            cfg.threads = 1 + variant;
            cfg.duration_us = D;
            cfg.seed = 100 + 10 * (uint64_t)scene + (uint64_t)variant;
            cfg.C_mean = 0.2;
            cfg.C_sigma = variant == 1 ? 0.02 : 0.0;
            cfg.C_lo = 0.15;
            cfg.C_hi = 0.25;
            cfg.target_scene_events = 20000.0;
            cfg.amplitude = scene == 1 ? 1.5 : (scene == 2 ? 0.16 : 0.2);
            cfg.noise_fraction = variant == 0 ? 0.0 : 0.1;
            cfg.step_us = 100.0;
            cfg.grating_period_px = 12.0;
            cfg.grating_speed_px_s = 200.0;
            cfg.tex_speed_px_s = 60.0;
            cfg.tex_vel_tau_s = 0.5;
            cfg.tex_lambda_lo = 6.0;
            cfg.tex_lambda_hi = 30.0;
            cfg.spoke_rev_s = 20.0;
            cfg.spoke_radius_frac = 0.45;
            cfg.spoke_edge_px = 1.0;
            cfg.spoke_count = 4;
            cfg.hot_fraction = variant == 2 ? 0.01 : 0.0;
            cfg.hot_rate_hz = variant == 2 ? 10e3 : 0.0;
            cfg.hot_rate_hi_hz = variant == 2 ? 50e3 : 0.0;
            cfg.tune = variant == 1 && scene != 3;
            stream_t s;
            if (!generate(&cfg, &s)) {
                fprintf(stderr, "evgen_generate failed (scene %d, variant %d)\n", scene, variant);
                return 1;
            }
            for (int64_t i = 1; i < s.n; ++i)
                CHECK(s.t[i - 1] <= s.t[i], "generated stream not time-sorted at %lld", (long long)i);
            for (int64_t i = 0; i < s.n; ++i)
                CHECK(s.x[i] < s.W && s.y[i] < s.H && (s.p[i] == 1 || s.p[i] == -1) && s.t[i] >= 0 &&
                          s.t[i] < D,
                      "generated event %lld out of range", (long long)i);
            exercise(&s, D);
            malformed(&s);
            printf("scene %d variant %d: %lld events\n", scene, variant, (long long)s.n);
            stream_free(&s);
        }
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
