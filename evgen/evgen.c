/*
 * evgen.c -- seeded synthetic DVS event streams.
 *
 * Inputs for both the GPU path and the CPU oracle; this file holds no part of
 * the integration method.  It is an ideal event-camera forward model
 * (Sec. III-A, Eq. (1), read as L(t2) = L(t1) + c * (signed events)): each
 * pixel keeps a reference log intensity L_ref, and every time the scene's
 * log intensity L(q, t) moves C_q above (below) it, the pixel emits a +1 (-1)
 * event and L_ref moves by +C_q (-C_q).  Crossing times are found on linear
 * pieces of L (sinusoid scenes: linear interpolation between samples; the
 * spoke scene: exact, its ramps are linear) and floored to integer
 * microseconds, so several crossings can share one time stamp.
 *
 * Scenes:
 *   0 grating  one sinusoid in x, period lambda px, drifting at v px/s.
 *   1 texture  sum of 8 random 2-D sinusoids, translated by a 2-D random walk
 *              (Ornstein-Uhlenbeck velocity).
 *   2 spokes   N radial spokes in a disc rotating at f rev/s, trapezoid
 *              profile with edges e px wide.
 *   3 none     no scene (noise and hot pixels only).
 * Plus per-pixel Poisson noise (uniform in time, random polarity) and
 * optional hot pixels (Poisson at a high rate, 3/4 positive; the rate is one
 * value, or per pixel log-uniform between two).
 *
 * On request one scene parameter is tuned so that the number of scene events
 * hits a target (bisection on the count over a pixel subsample): the
 * amplitude of the grating, the speed of the texture, the disc radius of the
 * spokes.  The count is monotone in each of them.  The noise rate is set from
 * the target and the noise fraction.
 *
 * Output order: time-sorted; ties in a fixed order (pixel bands in q order,
 * then generation order inside a band), so the stream does not depend on the
 * number of threads.  Random numbers: SplitMix64 (Steele, Lea, Flood 2014),
 * keyed by (seed, pixel, purpose).
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t scene, W, H, threads;
    int64_t duration_us;
    uint64_t seed;
    double C_mean, C_sigma, C_lo, C_hi; /* sensor threshold per pixel */
    double target_scene_events;         /* tune to this many scene events (<= 0: no tuning) */
    double amplitude;                   /* log-intensity amplitude */
    double noise_fraction;              /* noise / (scene + noise) events */
    double step_us;                     /* sampling step of sinusoid scenes */
    double grating_period_px, grating_speed_px_s;
    double tex_speed_px_s, tex_vel_tau_s, tex_lambda_lo, tex_lambda_hi;
    double spoke_rev_s, spoke_radius_frac, spoke_edge_px;
    int32_t spoke_count;
    double hot_fraction, hot_rate_hz;
    double hot_rate_hi_hz; /* > hot_rate_hz: each hot pixel's rate log-uniform in between */
    int32_t tune; /* nonzero: tune the scene parameter to target_scene_events */
} evgen_cfg;

typedef struct {
    int64_t t;
    uint32_t q;
    int8_t p;
} rec_t;

/* ---------------------------------------------------------------- RNG --- */
static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t rng_key(uint64_t seed, uint64_t a, uint64_t b)
{
    return mix64(seed + 0x9E3779B97F4A7C15ULL * (mix64(a + 0x632BE59BD9B4E019ULL) ^ (b + 1)));
}
static inline uint64_t rng_next(uint64_t *s)
{
    *s += 0x9E3779B97F4A7C15ULL;
    return mix64(*s);
}
static inline double rng_unif(uint64_t *s) /* [0, 1) */
{
    return (double)(rng_next(s) >> 11) * (1.0 / 9007199254740992.0);
}
static inline double rng_normal(uint64_t *s)
{
    double u1 = rng_unif(s), u2 = rng_unif(s);
    if (u1 < 1e-300)
        u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

enum { PURPOSE_C = 1, PURPOSE_NOISE = 2, PURPOSE_SCENE = 3, PURPOSE_HOT = 4 };

/* ------------------------------------------------------ event buffers --- */
typedef struct {
    rec_t *v;
    size_t n, cap;
} vec_t;

static int vec_push(vec_t *a, int64_t t, uint32_t q, int8_t p)
{
    if (a->n == a->cap) {
        size_t nc = a->cap ? a->cap * 2 : 4096;
        rec_t *nv = (rec_t *)realloc(a->v, nc * sizeof(rec_t));
        if (!nv)
            return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n].t = t;
    a->v[a->n].q = q;
    a->v[a->n].p = p;
    a->n++;
    return 0;
}

/* -------------------------------------------------------------- scenes --- */
#define MAXC 8
#define GROUP 8

typedef struct {
    const evgen_cfg *cfg;
    double A;          /* amplitude */
    double radius;     /* spokes: disc radius in px */
    double noise_rate; /* per pixel, events per us */
    /* sinusoid scenes */
    int ncomp;
    double kx[MAXC], ky[MAXC], ph[MAXC], w[MAXC];
    double *cs, *sn;   /* [nsteps+1][MAXC]: cos / sin of k_i . o(t_step) */
    double *ox, *oy;   /* unit-speed offset path, [nsteps+1] */
    int64_t nsteps;
    double dt;         /* sample step, us */
} scene_t;

static double pixel_C(const evgen_cfg *c, uint32_t q)
{
    if (c->C_sigma <= 0.0)
        return c->C_mean;
    uint64_t s = rng_key(c->seed, q, PURPOSE_C);
    for (int it = 0; it < 64; ++it) {
        double v = c->C_mean + c->C_sigma * rng_normal(&s);
        if (v >= c->C_lo && v <= c->C_hi)
            return v;
    }
    return c->C_mean;
}

static int64_t floor_time(double te, int64_t D)
{
    int64_t ti = (int64_t)floor(te);
    if (ti >= D)
        ti = D - 1;
    if (ti < 0)
        ti = 0;
    return ti;
}

/* Linear piece of L from (ta, La) to (tb, Lb): emit every crossing of the
 * reference level and move it.  `out` NULL: count only. */
static int emit_piece(vec_t *out, uint32_t q, double C, double *Lref, double ta,
                      double La, double tb, double Lb, int64_t D, int64_t *count)
{
    while (Lb - *Lref >= C) {
        double lev = *Lref + C;
        double f = (Lb > La) ? (lev - La) / (Lb - La) : 1.0;
        if (f < 0.0)
            f = 0.0;
        if (out && vec_push(out, floor_time(ta + f * (tb - ta), D), q, 1))
            return -1;
        ++*count;
        *Lref = lev;
    }
    while (*Lref - Lb >= C) {
        double lev = *Lref - C;
        double f = (La > Lb) ? (La - lev) / (La - Lb) : 1.0;
        if (f < 0.0)
            f = 0.0;
        if (out && vec_push(out, floor_time(ta + f * (tb - ta), D), q, -1))
            return -1;
        ++*count;
        *Lref = lev;
    }
    return 0;
}

/* Per-step tables of a sinusoid scene for a speed scale s: the offset is
 * s * o_unit(t) (texture) or (v t, 0) (grating). */
static void sinusoid_tables(scene_t *s, double speed_scale)
{
    for (int64_t k = 0; k <= s->nsteps; ++k) {
        double ox = speed_scale * s->ox[k], oy = speed_scale * s->oy[k];
        for (int i = 0; i < MAXC; ++i) {
            double a = (i < s->ncomp) ? s->kx[i] * ox + s->ky[i] * oy : 0.0;
            s->cs[k * MAXC + i] = cos(a);
            s->sn[k * MAXC + i] = sin(a);
        }
    }
}

static int setup_sinusoids(scene_t *s)
{
    const evgen_cfg *c = s->cfg;
    s->dt = c->step_us > 0 ? c->step_us : 100.0;
    s->nsteps = (int64_t)ceil((double)c->duration_us / s->dt);
    size_t m = (size_t)(s->nsteps + 1);
    s->cs = (double *)malloc(sizeof(double) * MAXC * m);
    s->sn = (double *)malloc(sizeof(double) * MAXC * m);
    s->ox = (double *)malloc(sizeof(double) * m);
    s->oy = (double *)malloc(sizeof(double) * m);
    if (!s->cs || !s->sn || !s->ox || !s->oy)
        return -1;
    if (c->scene == 0) {
        s->ncomp = 1;
        s->kx[0] = 6.283185307179586 / c->grating_period_px;
        s->ky[0] = 0.0;
        s->ph[0] = 0.0;
        s->w[0] = 1.0;
        for (int64_t k = 0; k <= s->nsteps; ++k) {
            s->ox[k] = c->grating_speed_px_s * (k * s->dt) * 1e-6;
            s->oy[k] = 0.0;
        }
        return 0;
    }
    uint64_t r = rng_key(c->seed, 0xFFFFFFFFu, PURPOSE_SCENE);
    s->ncomp = MAXC;
    for (int i = 0; i < MAXC; ++i) {
        double lam = c->tex_lambda_lo + (c->tex_lambda_hi - c->tex_lambda_lo) * rng_unif(&r);
        double dir = 3.141592653589793 * rng_unif(&r);
        s->kx[i] = 6.283185307179586 / lam * cos(dir);
        s->ky[i] = 6.283185307179586 / lam * sin(dir);
        s->ph[i] = 6.283185307179586 * rng_unif(&r);
        s->w[i] = (0.5 + 0.5 * rng_unif(&r)) / sqrt((double)MAXC);
    }
    /* unit-rms velocity per axis, Ornstein-Uhlenbeck with time constant tau */
    double tau = c->tex_vel_tau_s, dt_s = s->dt * 1e-6;
    double a = exp(-dt_s / tau), bn = sqrt(1.0 - a * a);
    double vx = rng_normal(&r), vy = rng_normal(&r), ox = 0.0, oy = 0.0;
    for (int64_t k = 0; k <= s->nsteps; ++k) {
        s->ox[k] = ox;
        s->oy[k] = oy;
        ox += vx * dt_s;
        oy += vy * dt_s;
        vx = a * vx + bn * rng_normal(&r);
        vy = a * vy + bn * rng_normal(&r);
    }
    return 0;
}

/* A group of up to GROUP consecutive pixels of a sinusoid scene. */
static int group_sinusoid(const scene_t *s, uint32_t q0, int ng, vec_t *out, int64_t *count)
{
    const evgen_cfg *c = s->cfg;
    const int64_t D = c->duration_us;
    double sp[MAXC][GROUP], cp[MAXC][GROUP], Lprev[GROUP], Lref[GROUP], Cq[GROUP];
    memset(sp, 0, sizeof(sp));
    memset(cp, 0, sizeof(cp));
    for (int g = 0; g < GROUP; ++g) {
        uint32_t q = q0 + (uint32_t)(g < ng ? g : 0);
        double x = (double)(q % (uint32_t)c->W), y = (double)(q / (uint32_t)c->W);
        for (int i = 0; i < s->ncomp; ++i) {
            double a = s->kx[i] * x + s->ky[i] * y + s->ph[i];
            sp[i][g] = s->A * s->w[i] * sin(a);
            cp[i][g] = s->A * s->w[i] * cos(a);
        }
        Cq[g] = pixel_C(c, q);
    }
    for (int g = 0; g < GROUP; ++g) {
        double acc = 0.0;
        for (int i = 0; i < MAXC; ++i)
            acc += sp[i][g] * s->cs[i] - cp[i][g] * s->sn[i];
        Lprev[g] = acc;
        Lref[g] = acc;
    }
    for (int64_t k = 1; k <= s->nsteps; ++k) {
        const double *co = s->cs + k * MAXC, *so = s->sn + k * MAXC;
        double L[GROUP];
        for (int g = 0; g < GROUP; ++g)
            L[g] = 0.0;
        for (int i = 0; i < MAXC; ++i) {
            const double ci = co[i], si = so[i];
            for (int g = 0; g < GROUP; ++g)
                L[g] += sp[i][g] * ci - cp[i][g] * si;
        }
        double ta = (k - 1) * s->dt, tb = k * s->dt;
        if (tb > (double)D)
            tb = (double)D;
        for (int g = 0; g < ng; ++g) {
            if (fabs(L[g] - Lref[g]) >= Cq[g]) {
                if (emit_piece(out, q0 + (uint32_t)g, Cq[g], &Lref[g], ta, Lprev[g], tb,
                               L[g], D, count))
                    return -1;
            }
            Lprev[g] = L[g];
        }
    }
    return 0;
}

/* Spokes.  A pixel at radius r and angle theta sees the pattern coordinate
 * u(t) = u0 - f t (in spoke periods).  Over one period the profile is +1 on
 * [h, 1/2 - h] and -1 on [1/2 + h, 1 - h], with linear ramps of half-width
 * h (h = edge width / (2 r) in radians, times N / 2pi) centred on the
 * multiples of 1/2: (u - cc)/h around an integer cc, (cc - u)/h around a
 * half-integer cc. */
static double spoke_profile(double u, double h)
{
    double v = u - floor(u);
    if (v < h)
        return v / h;
    if (v > 1.0 - h)
        return (v - 1.0) / h;
    if (v < 0.5 - h)
        return 1.0;
    if (v > 0.5 + h)
        return -1.0;
    return (0.5 - v) / h;
}

static int pixel_spokes(const scene_t *s, uint32_t q, vec_t *out, int64_t *count)
{
    const evgen_cfg *c = s->cfg;
    const int64_t D = c->duration_us;
    const int32_t x = (int32_t)(q % (uint32_t)c->W), y = (int32_t)(q / (uint32_t)c->W);
    const double cx = 0.5 * (c->W - 1), cy = 0.5 * (c->H - 1);
    const double dx = x - cx, dy = y - cy, r = sqrt(dx * dx + dy * dy);
    const double N = (double)c->spoke_count;
    if (r > s->radius || r < 2.0)
        return 0;
    const double h = 0.5 * (c->spoke_edge_px / r) * N / 6.283185307179586;
    if (h >= 0.24)
        return 0;
    const double u0 = atan2(dy, dx) * N / 6.283185307179586;
    const double f = N * c->spoke_rev_s * 1e-6;
    const double A = s->A, C = pixel_C(c, q);
    double Lref = A * spoke_profile(u0, h);
    const double u_end = u0 - f * (double)D;
    for (int64_t k2 = (int64_t)floor(2.0 * (u0 + h));; --k2) {
        const double cc = 0.5 * (double)k2;
        if (cc + h <= u_end)
            break;
        double ua = cc + h, ub = cc - h;
        if (ua > u0)
            ua = u0;
        if (ub < u_end)
            ub = u_end;
        if (ua <= ub)
            continue;
        const double sgn = (k2 % 2 == 0) ? 1.0 : -1.0;
        const double La = A * sgn * (ua - cc) / h, Lb = A * sgn * (ub - cc) / h;
        if (emit_piece(out, q, C, &Lref, (u0 - ua) / f, La, (u0 - ub) / f, Lb, D, count))
            return -1;
    }
    return 0;
}

static int pixel_noise(const scene_t *s, uint32_t q, vec_t *out, int64_t *count)
{
    const evgen_cfg *c = s->cfg;
    const int64_t D = c->duration_us;
    if (s->noise_rate > 0.0) {
        uint64_t r = rng_key(c->seed, q, PURPOSE_NOISE);
        double t = 0.0;
        for (;;) {
            t += -log(1.0 - rng_unif(&r)) / s->noise_rate;
            if (t >= (double)D)
                break;
            int8_t p = (rng_next(&r) >> 63) ? 1 : -1;
            if (out && vec_push(out, (int64_t)t, q, p))
                return -1;
            ++*count;
        }
    }
    if (c->hot_fraction > 0.0 && c->hot_rate_hz > 0.0) {
        uint64_t r = rng_key(c->seed, q, PURPOSE_HOT);
        if (rng_unif(&r) < c->hot_fraction) {
            double hz = c->hot_rate_hz;
            if (c->hot_rate_hi_hz > hz)
                hz *= exp(rng_unif(&r) * log(c->hot_rate_hi_hz / hz));
            double rate = hz * 1e-6, t = 0.0;
            for (;;) {
                t += -log(1.0 - rng_unif(&r)) / rate;
                if (t >= (double)D)
                    break;
                int8_t p = (rng_next(&r) >> 62) ? 1 : -1;
                if (out && vec_push(out, (int64_t)t, q, p))
                    return -1;
                ++*count;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------ worker threads --- */
#define NBANDS 256

typedef struct {
    const scene_t *s;
    vec_t band[NBANDS];
    int64_t band_lo[NBANDS + 1];
    int64_t band_count[NBANDS];
    int next_band;
    pthread_mutex_t mu;
    int err;
    int counting;  /* count scene events only, on every stride-th group */
    int stride;
} job_t;

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    const scene_t *s = j->s;
    const evgen_cfg *c = s->cfg;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int b = j->next_band++;
        pthread_mutex_unlock(&j->mu);
        if (b >= NBANDS)
            break;
        vec_t *out = j->counting ? NULL : &j->band[b];
        int64_t cnt = 0;
        int64_t lo = j->band_lo[b], hi = j->band_lo[b + 1];
        for (int64_t q0 = lo; q0 < hi; q0 += GROUP) {
            int ng = (int)((hi - q0) < GROUP ? (hi - q0) : GROUP);
            if (j->counting && ((q0 / GROUP) % j->stride))
                continue;
            int rc = 0;
            if (c->scene == 0 || c->scene == 1)
                rc = group_sinusoid(s, (uint32_t)q0, ng, out, &cnt);
            else if (c->scene == 2)
                for (int g = 0; g < ng && !rc; ++g)
                    rc = pixel_spokes(s, (uint32_t)(q0 + g), out, &cnt);
            if (!j->counting)
                for (int g = 0; g < ng && !rc; ++g)
                    rc = pixel_noise(s, (uint32_t)(q0 + g), out, &cnt);
            if (rc) {
                j->err = 1;
                break;
            }
        }
        j->band_count[b] = cnt;
    }
    return NULL;
}

static void run_workers(job_t *j, int threads)
{
    pthread_t th[64];
    if (threads < 1)
        threads = 1;
    if (threads > 64)
        threads = 64;
    j->next_band = 0;
    for (int i = 0; i < threads; ++i)
        pthread_create(&th[i], NULL, worker, j);
    for (int i = 0; i < threads; ++i)
        pthread_join(th[i], NULL);
}

static double count_scene(job_t *j, int threads)
{
    j->counting = 1;
    run_workers(j, threads);
    j->counting = 0;
    double n = 0.0;
    for (int b = 0; b < NBANDS; ++b)
        n += (double)j->band_count[b];
    return n * j->stride;
}

/* ------------------------------------------------ stable radix by time --- */
typedef struct {
    rec_t *src, *dst;
    int64_t lo, hi;
    int shift;
    int64_t *hist; /* [threads][256] */
    int tid;
} radix_arg_t;

static void *radix_count(void *arg)
{
    radix_arg_t *a = (radix_arg_t *)arg;
    int64_t *h = a->hist + (int64_t)a->tid * 256;
    memset(h, 0, 256 * sizeof(int64_t));
    for (int64_t i = a->lo; i < a->hi; ++i)
        h[(a->src[i].t >> a->shift) & 255]++;
    return NULL;
}

static void *radix_scatter(void *arg)
{
    radix_arg_t *a = (radix_arg_t *)arg;
    int64_t *h = a->hist + (int64_t)a->tid * 256;
    for (int64_t i = a->lo; i < a->hi; ++i) {
        int d = (int)((a->src[i].t >> a->shift) & 255);
        a->dst[h[d]++] = a->src[i];
    }
    return NULL;
}

/* Stable LSD radix sort by t (t in [0, D)).  Returns the buffer holding the
 * result (a or b). */
static rec_t *sort_by_time(rec_t *a, rec_t *b, int64_t n, int64_t D, int threads)
{
    int bits = 0;
    while (bits < 63 && ((int64_t)1 << bits) < D)
        ++bits;
    if (threads < 1)
        threads = 1;
    if (threads > 64)
        threads = 64;
    int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * 256 * threads);
    radix_arg_t args[64];
    pthread_t th[64];
    for (int shift = 0; shift < bits; shift += 8) {
        for (int i = 0; i < threads; ++i) {
            args[i] = (radix_arg_t){a, b, n * i / threads, n * (i + 1) / threads, shift, hist, i};
            pthread_create(&th[i], NULL, radix_count, &args[i]);
        }
        for (int i = 0; i < threads; ++i)
            pthread_join(th[i], NULL);
        int64_t run = 0;
        for (int d = 0; d < 256; ++d)
            for (int i = 0; i < threads; ++i) {
                int64_t cnt = hist[i * 256 + d];
                hist[i * 256 + d] = run;
                run += cnt;
            }
        for (int i = 0; i < threads; ++i)
            pthread_create(&th[i], NULL, radix_scatter, &args[i]);
        for (int i = 0; i < threads; ++i)
            pthread_join(th[i], NULL);
        rec_t *tmp = a;
        a = b;
        b = tmp;
    }
    free(hist);
    return a;
}

/* ------------------------------------------------------------- public --- */
typedef struct {
    rec_t *recs;
    int64_t n;
    int32_t W;
} evgen_result;

/* Set the tuned parameter to v. */
static void set_param(scene_t *s, int which, double v)
{
    if (which == 0)
        s->A = v;
    else if (which == 1)
        sinusoid_tables(s, v);
    else
        s->radius = v;
}

/* Generate a stream.  Returns a handle (NULL on failure); *n_out = events,
 * tuned[0] = the tuned parameter (amplitude, speed or radius). */
void *evgen_generate(const evgen_cfg *cfg, int64_t *n_out, double *tuned)
{
    scene_t s;
    memset(&s, 0, sizeof(s));
    s.cfg = cfg;
    const int64_t npix = (int64_t)cfg->W * cfg->H;
    const int64_t D = cfg->duration_us;
    if (npix <= 0 || D <= 0 || npix > 0xFFFFFFFFll || cfg->W > 65535 || cfg->H > 65535)
        return NULL;
    s.A = cfg->amplitude;
    s.radius = cfg->spoke_radius_frac * (cfg->W < cfg->H ? cfg->W : cfg->H);
    if ((cfg->scene == 0 || cfg->scene == 1) && setup_sinusoids(&s))
        return NULL;
    if (cfg->scene == 1)
        sinusoid_tables(&s, cfg->tex_speed_px_s);
    else if (cfg->scene == 0)
        sinusoid_tables(&s, 1.0);

    job_t *j = (job_t *)calloc(1, sizeof(job_t));
    pthread_mutex_init(&j->mu, NULL);
    j->s = &s;
    for (int b = 0; b <= NBANDS; ++b)
        j->band_lo[b] = npix * b / NBANDS;
    j->stride = npix > 40000 ? 16 : 1;

    double param = 0.0;
    const int which = cfg->scene == 0 ? 0 : (cfg->scene == 1 ? 1 : 2);
    if (cfg->scene != 3) {
        param = which == 0 ? s.A : (which == 1 ? cfg->tex_speed_px_s : s.radius);
        if (cfg->tune && cfg->target_scene_events > 0.0) {
            const double target = cfg->target_scene_events;
            double lo = param, hi = param;
            set_param(&s, which, lo);
            double clo = count_scene(j, cfg->threads), chi = clo;
            for (int it = 0; it < 40 && clo > target; ++it) {
                hi = lo;
                chi = clo;
                lo *= 0.5;
                set_param(&s, which, lo);
                clo = count_scene(j, cfg->threads);
            }
            for (int it = 0; it < 40 && chi < target; ++it) {
                lo = hi;
                clo = chi;
                hi *= 2.0;
                set_param(&s, which, hi);
                chi = count_scene(j, cfg->threads);
            }
            for (int it = 0; it < 30 && hi / lo > 1.0 + 1e-4; ++it) {
                double mid = sqrt(lo * hi);
                set_param(&s, which, mid);
                double cm = count_scene(j, cfg->threads);
                if (fabs(cm / target - 1.0) < 0.005) {
                    lo = hi = mid;
                    break;
                }
                if (cm < target)
                    lo = mid;
                else
                    hi = mid;
            }
            param = sqrt(lo * hi);
        }
        set_param(&s, which, param);
    }
    if (cfg->noise_fraction > 0.0 && cfg->noise_fraction < 1.0) {
        double base = cfg->target_scene_events > 0.0 ? cfg->target_scene_events : 0.0;
        if (cfg->scene == 3)
            base = 1e6 * (double)D * 1e-6; /* none: 1 Mev/s of noise per unit fraction */
        double noise_total = base * cfg->noise_fraction / (1.0 - cfg->noise_fraction);
        s.noise_rate = noise_total / ((double)npix * (double)D);
    }

    run_workers(j, cfg->threads);
    int err = j->err;
    int64_t n = 0;
    for (int b = 0; b < NBANDS; ++b)
        n += (int64_t)j->band[b].n;
    rec_t *a = err ? NULL : (rec_t *)malloc(sizeof(rec_t) * (n ? n : 1));
    rec_t *bb = err ? NULL : (rec_t *)malloc(sizeof(rec_t) * (n ? n : 1));
    int64_t off = 0;
    for (int b = 0; b < NBANDS; ++b) {
        if (a && j->band[b].n)
            memcpy(a + off, j->band[b].v, sizeof(rec_t) * j->band[b].n);
        off += (int64_t)j->band[b].n;
        free(j->band[b].v);
    }
    free(j);
    free(s.cs);
    free(s.sn);
    free(s.ox);
    free(s.oy);
    if (!a || !bb) {
        free(a);
        free(bb);
        return NULL;
    }
    rec_t *sorted = sort_by_time(a, bb, n, D, cfg->threads);
    free(sorted == a ? bb : a);
    evgen_result *res = (evgen_result *)malloc(sizeof(evgen_result));
    res->recs = sorted;
    res->n = n;
    res->W = cfg->W;
    *n_out = n;
    if (tuned)
        *tuned = param;
    return res;
}

/* Copy the stream into caller SoA arrays of length n and free the handle. */
void evgen_fetch(void *h, uint16_t *x, uint16_t *y, int64_t *t, int8_t *p)
{
    evgen_result *r = (evgen_result *)h;
    for (int64_t i = 0; i < r->n; ++i) {
        uint32_t q = r->recs[i].q;
        x[i] = (uint16_t)(q % (uint32_t)r->W);
        y[i] = (uint16_t)(q / (uint32_t)r->W);
        t[i] = r->recs[i].t;
        p[i] = r->recs[i].p;
    }
    free(r->recs);
    free(r);
}
