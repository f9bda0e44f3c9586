/*
 * SparkCL map -> reduce oracle (see oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU product path.
 *
 * Written for clarity, not speed: one element at a time, in index order, with
 * no blocking, fusion or reordering beyond what the definitions state.
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>

/* ------------------------------------------------------------------------ */
/* O1  POLY: the MapCL elementwise kernel (sec. 3.1.3; the Fig 3 kernel body
 * applies one expression per global id).  Horner's rule, highest coefficient
 * first; each step is fl(fl(t * x) + coef[k]).                               */
static float poly_one(float x, uint32_t degree, const float *coef)
{
    float t = coef[degree];
    for (uint32_t k = degree; k-- > 0;) {
        float prod = t * x;   /* one binary32 multiply */
        t = prod + coef[k];   /* one binary32 add      */
    }
    return t;
}

void oracle_poly_map(const float *x, uint64_t n, uint32_t degree,
                     const float *coef, float *y)
{
    for (uint64_t i = 0; i < n; ++i)
        y[i] = poly_one(x[i], degree, coef);
}

/* O2  FMUL: the two-input kernel of Fig 3 (SparkKernel2, elementwise over
 * data1 and data2), generalised from a + b to x*y + c*x.                     */
static float fmul_one(float x, float y, float c)
{
    float xy = x * y;
    float cx = c * x;
    return xy + cx;
}

void oracle_fmul_map(const float *x, const float *y, uint64_t n, float c,
                     float *z)
{
    for (uint64_t i = 0; i < n; ++i)
        z[i] = fmul_one(x[i], y[i], c);
}

/* O3  ReduceCL sum (sec. 3.1.3): Neumaier's compensated summation in FP64,
 * index order.  s holds the running sum, comp the accumulated rounding error
 * of every s + v step; the result is s + comp.                               */
typedef struct {
    double s, comp;
} neumaier;

static void neumaier_add(neumaier *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->comp += (a->s - t) + v;
    else
        a->comp += (v - t) + a->s;
    a->s = t;
}

static double neumaier_value(const neumaier *a) { return a->s + a->comp; }

double oracle_sum(const float *v, uint64_t n)
{
    neumaier a = {0.0, 0.0};
    for (uint64_t i = 0; i < n; ++i)
        neumaier_add(&a, (double)v[i]);
    return neumaier_value(&a);
}

double oracle_sum_f64(const double *v, uint64_t n)
{
    neumaier a = {0.0, 0.0};
    for (uint64_t i = 0; i < n; ++i)
        neumaier_add(&a, v[i]);
    return neumaier_value(&a);
}

/* O4  ReduceCL max: m starts at -inf; m = v if v > m, index order.           */
float oracle_max(const float *v, uint64_t n)
{
    float m = -INFINITY;
    for (uint64_t i = 0; i < n; ++i)
        if (v[i] > m)
            m = v[i];
    return m;
}

/* ------------------------------------------------------------------------ */
/* O5  Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11).  Not part of the SparkCL paper: the
 * Pi demo (sec. 3.2.1) needs a counter-based generator and this is the one
 * chosen.  A round multiplies counter words 0 and 2 by two odd constants
 * (32x32 -> 64 bit), then forms the new counter from the high halves xor the
 * other counter words xor the round key, and the low halves.  The two key
 * words are bumped by two Weyl constants between rounds.                    */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* O6  MapCLPartition Monte-Carlo count (SparkCLPi, sec. 3.2.1).
 * Sample s of partition pid uses the Philox block for pair j = s / 2 with
 * key = (seed low, seed high) and counter = (j low, j high, pid, 0).  An even
 * sample takes words (0, 1), an odd sample words (2, 3).  The point is
 * (a, b) * 2^-24 with a, b the top 24 bits of the two words; it is a hit iff
 * a^2 + b^2 <= 2^48, i.e. iff the point lies in the closed unit quarter-disc,
 * decided exactly in 64-bit integers.                                        */
uint64_t oracle_mc_count(uint64_t seed, uint32_t pid, uint64_t lo, uint64_t hi)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t hits = 0;
    for (uint64_t s = lo; s < hi; ++s) {
        uint64_t j = s / 2;
        uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), pid, 0u};
        uint32_t r[4];
        oracle_philox4x32_10(ctr, key, r);
        uint32_t wa = (s % 2 == 0) ? r[0] : r[2];
        uint32_t wb = (s % 2 == 0) ? r[1] : r[3];
        uint64_t a = wa >> 8, b = wb >> 8;
        if (a * a + b * b <= (1ull << 48))
            ++hits;
    }
    return hits;
}

/* ------------------------------------------------------------------------ */
/* A whole partition task: the map (O1/O2) evaluated element by element and
 * folded straight into the requested reductions (O3/O4), or the partition
 * kernel (O6).  Spark pipelines a map into the reduce that consumes it, so
 * the oracle does not store the mapped values.                               */
int oracle_task_run(const oracle_task *t, oracle_result *r)
{
    r->sum = 0.0;
    r->max = -INFINITY;
    r->pad = 0;
    r->count = 0;
    r->n = t->n;

    if (t->kernel_id == ORACLE_MC_PI) {
        if (t->reduce_ops != ORACLE_COUNT)
            return -1;
        r->count = oracle_mc_count(t->seed, t->partition_id, 0, t->n);
        return 0;
    }
    if (t->kernel_id != ORACLE_POLY && t->kernel_id != ORACLE_FMUL)
        return -1;
    if (t->reduce_ops == 0 || (t->reduce_ops & ~(uint32_t)(ORACLE_SUM | ORACLE_MAX)))
        return -1;
    if (t->kernel_id == ORACLE_POLY && t->degree > 7)
        return -1;

    neumaier acc = {0.0, 0.0};
    float m = -INFINITY;
    for (uint64_t i = 0; i < t->n; ++i) {
        float v = (t->kernel_id == ORACLE_POLY)
                      ? poly_one(t->in0[i], t->degree, t->coef)
                      : fmul_one(t->in0[i], t->in1[i], t->c);
        neumaier_add(&acc, (double)v);
        if (v > m)
            m = v;
    }
    if (t->reduce_ops & ORACLE_SUM)
        r->sum = neumaier_value(&acc);
    if (t->reduce_ops & ORACLE_MAX)
        r->max = m;
    return 0;
}

/* O7  RDD-level ReduceCL combine (sec. 3.1.3 tree-reduce, sec. 3.2.2): the
 * partition sums folded in FP64 Neumaier in partition order, the max of the
 * maxima, the integer sum of the counts and of the element counts.          */
void oracle_rdd_total(const oracle_result *r, uint64_t ntasks,
                      uint32_t reduce_ops, oracle_result *total)
{
    neumaier acc = {0.0, 0.0};
    float m = -INFINITY;
    uint64_t count = 0, n = 0;
    for (uint64_t i = 0; i < ntasks; ++i) {
        neumaier_add(&acc, r[i].sum);
        if (r[i].max > m)
            m = r[i].max;
        count += r[i].count;
        n += r[i].n;
    }
    total->sum = (reduce_ops & ORACLE_SUM) ? neumaier_value(&acc) : 0.0;
    total->max = (reduce_ops & ORACLE_MAX) ? m : -INFINITY;
    total->pad = 0;
    total->count = (reduce_ops & ORACLE_COUNT) ? count : 0;
    total->n = n;
}

/* ------------------------------------------------------------------------ */
/* O9  Array-valued ReduceCL: the Fig 3 combiner (elementwise over two RDD
 * elements that are arrays) applied along a fixed binary tree (sec. 3.1.3
 * item 3, sec. 3.2.2).  The tree over elements [k0, k1) splits at k0 plus the
 * largest power of two strictly below the count, left part first.            */
static float combine_one(uint32_t combiner, float a, float b)
{
    if (combiner == ORACLE_VADD)
        return a + b;             /* one binary32 add */
    return (b > a) ? b : a;       /* VMAX */
}

static uint32_t largest_pow2_below(uint32_t m) /* m >= 2 */
{
    uint32_t p = 1;
    while (2 * p < m)
        p *= 2;
    return p;
}

static float tree_at(uint32_t combiner, const float *const *arrays,
                     uint32_t k0, uint32_t k1, uint64_t i)
{
    if (k1 - k0 == 1)
        return arrays[k0][i];
    const uint32_t mid = k0 + largest_pow2_below(k1 - k0);
    const float left = tree_at(combiner, arrays, k0, mid, i);
    const float right = tree_at(combiner, arrays, mid, k1, i);
    return combine_one(combiner, left, right);
}

int oracle_tree_reduce_arrays(uint32_t combiner, const float *const *arrays,
                              uint32_t k, uint64_t len, float *out)
{
    if ((combiner != ORACLE_VADD && combiner != ORACLE_VMAX) || k == 0)
        return -1;
    for (uint64_t i = 0; i < len; ++i)
        out[i] = tree_at(combiner, arrays, 0, k, i);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O10 WordCount (sec. 3.2.3).  Tokenise in byte order, hash each word with
 * 64-bit FNV-1a (offset basis 14695981039346656037, prime 1099511628211:
 * for each byte, xor it in, then multiply modulo 2^64), collect the keys,
 * sort them and count the runs.                                              */
static int is_space(uint8_t b)
{
    return b == 0x20 || (b >= 0x09 && b <= 0x0d);
}

uint64_t oracle_fnv1a64(const uint8_t *bytes, uint64_t len)
{
    uint64_t h = 14695981039346656037ull;
    for (uint64_t i = 0; i < len; ++i) {
        h ^= bytes[i];
        h *= 1099511628211ull;
    }
    return h;
}

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y ? 1 : 0;
}

int oracle_wordcount(const uint8_t *text, uint64_t nbytes, uint64_t *keys,
                     uint64_t *counts, uint64_t cap, uint64_t *ndistinct,
                     uint64_t *nwords)
{
    uint64_t nw = 0, room = 1024;
    uint64_t *all = malloc(room * sizeof(uint64_t));
    if (!all)
        return -1;
    uint64_t i = 0;
    while (i < nbytes) {
        if (is_space(text[i])) {
            ++i;
            continue;
        }
        uint64_t j = i;
        while (j < nbytes && !is_space(text[j]))
            ++j;
        if (nw == room) {
            room *= 2;
            uint64_t *grown = realloc(all, room * sizeof(uint64_t));
            if (!grown) {
                free(all);
                return -1;
            }
            all = grown;
        }
        all[nw++] = oracle_fnv1a64(text + i, j - i);
        i = j;
    }
    qsort(all, nw, sizeof(uint64_t), cmp_u64);
    uint64_t nd = 0;
    for (uint64_t k = 0; k < nw;) {
        uint64_t e = k;
        while (e < nw && all[e] == all[k])
            ++e;
        if (nd < cap) {
            keys[nd] = all[k];
            counts[nd] = e - k;
        }
        ++nd;
        k = e;
    }
    free(all);
    *ndistinct = nd;
    *nwords = nw;
    return nd <= cap ? 0 : -1;
}

/* O10 WordCount's words: the first occurrence of each key.  Tokenise in byte
 * order as above, pair every word's key with the offset of its first byte,
 * sort the pairs by key and then offset, and answer each query key with the
 * offset of its first pair (UINT64_MAX when no word has the key).            */
struct key_off {
    uint64_t key, off;
};

static int cmp_key_off(const void *a, const void *b)
{
    const struct key_off *x = a, *y = b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->off < y->off ? -1 : x->off > y->off ? 1 : 0;
}

int oracle_wordcount_first(const uint8_t *text, uint64_t nbytes, const uint64_t *keys,
                           uint64_t nkeys, uint64_t *offsets)
{
    uint64_t nw = 0, room = 1024;
    struct key_off *all = malloc(room * sizeof(*all));
    if (!all)
        return -1;
    uint64_t i = 0;
    while (i < nbytes) {
        if (is_space(text[i])) {
            ++i;
            continue;
        }
        uint64_t j = i;
        while (j < nbytes && !is_space(text[j]))
            ++j;
        if (nw == room) {
            room *= 2;
            struct key_off *grown = realloc(all, room * sizeof(*all));
            if (!grown) {
                free(all);
                return -1;
            }
            all = grown;
        }
        all[nw].key = oracle_fnv1a64(text + i, j - i);
        all[nw].off = i;
        ++nw;
        i = j;
    }
    qsort(all, nw, sizeof(*all), cmp_key_off);
    for (uint64_t q = 0; q < nkeys; ++q) {
        /* the first pair whose key is not below the query */
        uint64_t lo = 0, hi = nw;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (all[mid].key < keys[q])
                lo = mid + 1;
            else
                hi = mid;
        }
        offsets[q] = (lo < nw && all[lo].key == keys[q]) ? all[lo].off : UINT64_MAX;
    }
    free(all);
    return 0;
}
