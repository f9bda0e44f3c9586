/*
 * Seeded synthetic inputs for the SparkCL map -> reduce workloads.
 *
 * Shared by the tests, the benchmark and the smoke check as the one source of
 * input bytes: both the oracle and the GPU path read what this writes.  It
 * holds none of the method's arithmetic: no map, no reduction and no Philox.
 *
 * Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used counter-style.  A stream is named by
 * (seed, partition id, tag); its key is the SplitMix64 output for the stream
 * number, and word i of the stream is mix64(key + gamma * (i + 1)).  Any word
 * can be computed on its own, so the fill is split across threads freely and
 * the bytes do not depend on the thread count.
 *
 * Build: gcc -std=c11 -O2 -fPIC -shared -pthread datagen.c -lm.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t datagen_stream_key(uint64_t seed, uint32_t pid, uint32_t tag)
{
    uint64_t stream = ((uint64_t)pid << 8) | (tag & 0xffu);
    return mix64(seed + SM_GAMMA * (stream + 1));
}

static inline uint64_t word(uint64_t key, uint64_t i)
{
    return mix64(key + SM_GAMMA * (i + 1));
}

enum {
    DIST_WORDS = 0,      /* raw 64-bit words                               */
    DIST_U_PM1 = 1,      /* binary32 on the 2^-23 grid in [-1, 1), exact   */
    DIST_U_02 = 2,       /* binary32 on the 2^-23 grid in [0, 2), exact    */
    DIST_NORMAL = 3,     /* N(0,1): Box-Muller in FP64, rounded to float   */
    DIST_NORMAL64 = 4,   /* N(0,1) as double                               */
    DIST_U01_64 = 5      /* uniform in (0, 1) as double                    */
};

static double normal_from(uint64_t w)
{
    /* Box-Muller, cosine branch: two 32-bit halves as uniforms in (0,1). */
    double u1 = ((double)(w >> 32) + 0.5) * 0x1p-32;
    double u2 = ((double)(w & 0xffffffffu) + 0.5) * 0x1p-32;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

typedef struct {
    void *out;
    uint64_t begin, end, key, first;
    int dist;
} job;

static void fill_range(const job *j)
{
    for (uint64_t i = j->begin; i < j->end; ++i) {
        uint64_t w = word(j->key, j->first + i);
        switch (j->dist) {
        case DIST_WORDS:
            ((uint64_t *)j->out)[i] = w;
            break;
        case DIST_U_PM1:
            ((float *)j->out)[i] =
                (float)((double)((int64_t)(w >> 40) - (1ll << 23)) * 0x1p-23);
            break;
        case DIST_U_02:
            ((float *)j->out)[i] = (float)((double)(w >> 40) * 0x1p-23);
            break;
        case DIST_NORMAL:
            ((float *)j->out)[i] = (float)normal_from(w);
            break;
        case DIST_NORMAL64:
            ((double *)j->out)[i] = normal_from(w);
            break;
        case DIST_U01_64:
            ((double *)j->out)[i] = ((double)(w >> 11) + 0.5) * 0x1p-53;
            break;
        default:
            break;
        }
    }
}

static void *fill_thread(void *arg)
{
    fill_range((const job *)arg);
    return NULL;
}

/* Fill out[0..n) with draws first .. first + n - 1 of stream (seed, pid,
 * tag) in distribution `dist`, using up to `nthreads` threads.  Returns 0, or
 * -1 for an unknown distribution. */
int datagen_fill_at(void *out, uint64_t first, uint64_t n, uint64_t seed,
                    uint32_t pid, uint32_t tag, int dist, int nthreads)
{
    if (dist < DIST_WORDS || dist > DIST_U01_64)
        return -1;
    uint64_t key = datagen_stream_key(seed, pid, tag);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 64)
        nthreads = 64;
    if (n < (1u << 16))
        nthreads = 1;
    job jobs[64];
    pthread_t th[64];
    int running[64] = {0};
    uint64_t chunk = (n + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t b = (uint64_t)t * chunk, e = b + chunk;
        if (b > n)
            b = n;
        if (e > n)
            e = n;
        jobs[t] = (job){out, b, e, key, first, dist};
        if (t > 0)
            running[t] = pthread_create(&th[t], NULL, fill_thread, &jobs[t]) == 0;
    }
    fill_range(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) {
        if (running[t])
            pthread_join(th[t], NULL);
        else
            fill_range(&jobs[t]); /* thread could not start: fill here */
    }
    return 0;
}

/* Fill out[0..n) with the first n draws of stream (seed, pid, tag). */
int datagen_fill(void *out, uint64_t n, uint64_t seed, uint32_t pid,
                 uint32_t tag, int dist, int nthreads)
{
    return datagen_fill_at(out, 0, n, seed, pid, tag, dist, nthreads);
}
