/*
 * SparkCL map -> reduce oracle: plain, slow, single-threaded CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path never links, loads or calls it, and it shares no source with that path.
 *
 * What it computes, and where the paper defines it:
 *   - MapCL (sec. 3.1.3): an elementwise kernel over a partition's elements; the
 *     Fig 3 kernel body applies one expression per global id.
 *   - MapCLPartition (sec. 3.1.3): a kernel that sees a whole partition and
 *     emits partition-level values (the SparkCLPi demo, sec. 3.2.1).
 *   - ReduceCL (sec. 3.1.3, sec. 3.2.2): a reduction of a partition, then a
 *     tree combine of the partition results into one RDD-level value.
 *
 * Floating point: compile with -O2 -ffp-contract=off on x86-64 (SSE2 scalar
 * arithmetic, no x87).  Every map step is one IEEE binary32 operation in the
 * order written; sums are FP64 Neumaier in index order.
 */
#ifndef SPARKCL_ORACLE_H
#define SPARKCL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Kernel ids of the built-in registry. */
enum { ORACLE_POLY = 1, ORACLE_FMUL = 2, ORACLE_MC_PI = 3 };
/* Reduce-op bits. */
enum { ORACLE_SUM = 1, ORACLE_MAX = 2, ORACLE_COUNT = 4 };

typedef struct {
    uint32_t kernel_id;
    uint32_t reduce_ops;
    uint64_t n;            /* elements (POLY, FMUL) or samples (MC_PI) */
    const float *in0;      /* x */
    const float *in1;      /* y (FMUL only) */
    uint64_t seed;         /* MC_PI key */
    uint32_t partition_id; /* MC_PI counter word 2 */
    uint32_t degree;       /* POLY degree, 0..7 */
    float coef[8];         /* POLY coefficients, coef[k] multiplies x^k */
    float c;               /* FMUL constant */
} oracle_task;

typedef struct {
    double sum;            /* +0.0 when SUM not requested or n == 0 */
    float max;             /* -inf when MAX not requested or n == 0 */
    uint32_t pad;
    uint64_t count;        /* MC_PI hits; 0 otherwise */
    uint64_t n;            /* elements covered */
} oracle_result;

/* O1  POLY map: y_i = Horner(coef, x_i), one binary32 multiply and one
 *     binary32 add per step, highest coefficient first. */
void oracle_poly_map(const float *x, uint64_t n, uint32_t degree,
                     const float *coef, float *y);

/* O2  FMUL map: z_i = fl(fl(x_i * y_i) + fl(c * x_i)). */
void oracle_fmul_map(const float *x, const float *y, uint64_t n, float c,
                     float *z);

/* O3  FP64 Neumaier sum of (double)v_i, i = 0..n-1 in order. */
double oracle_sum(const float *v, uint64_t n);

/* O3' the same summation over doubles (used for the RDD-level combine). */
double oracle_sum_f64(const double *v, uint64_t n);

/* O4  max over v_i in index order, starting from -inf. */
float oracle_max(const float *v, uint64_t n);

/* O5  Philox4x32-10 block function: out = philox(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);

/* O6  Monte-Carlo hit count over samples [lo, hi) of partition `pid`. */
uint64_t oracle_mc_count(uint64_t seed, uint32_t pid, uint64_t lo,
                         uint64_t hi);

/* Full task: map fused with the requested reductions (O1/O2 + O3/O4, or O6).
 * Returns 0, or -1 for an invalid kernel id / op mask / degree. */
int oracle_task_run(const oracle_task *t, oracle_result *r);

/* O7  RDD-level combine of partition results in partition order. */
void oracle_rdd_total(const oracle_result *r, uint64_t ntasks,
                      uint32_t reduce_ops, oracle_result *total);

/* O9  Array-valued ReduceCL (sec. 3.1.3 item 3; Fig 3; sec. 3.2.2): the RDD's
 *     elements are float arrays of one length `len`; a two-input combiner
 *     kernel (Fig 3: c[gid] = a[gid] + b[gid]) is applied pairwise along a tree
 *     until one array is left.  Tree (a reading: the paper names a Spark
 *     tree-reduce and fixes no shape): over elements [k0, k1) the split point
 *     is k0 + the largest power of two strictly below k1 - k0, and the left
 *     part is the left operand.  Each combine is one binary32 operation per
 *     position:  VADD: fl(a + b);  VMAX: (b > a) ? b : a.
 *     Returns 0, or -1 for an unknown combiner or k == 0. */
enum { ORACLE_VADD = 1, ORACLE_VMAX = 2 };
int oracle_tree_reduce_arrays(uint32_t combiner, const float *const *arrays,
                              uint32_t k, uint64_t len, float *out);

/* O10 WordCount (sec. 3.2.3: the Spark word-count demo as a SparkCL kernel).
 *     A word is a maximal run of bytes that are not ASCII whitespace (space,
 *     tab, LF, VT, FF, CR); its key is the 64-bit FNV-1a hash of its bytes
 *     (Fowler, Noll, Vo).  Writes the distinct keys in ascending order with
 *     their counts (up to `cap` of them), *ndistinct and *nwords.  Returns 0,
 *     or -1 if there are more than `cap` distinct keys or memory runs out. */
uint64_t oracle_fnv1a64(const uint8_t *bytes, uint64_t len);
int oracle_wordcount(const uint8_t *text, uint64_t nbytes, uint64_t *keys,
                     uint64_t *counts, uint64_t cap, uint64_t *ndistinct,
                     uint64_t *nwords);
/*     For each of the nkeys query keys, the byte offset of the first word
 *     whose key it is, or UINT64_MAX when no word has it.  Returns 0, or -1
 *     if memory runs out. */
int oracle_wordcount_first(const uint8_t *text, uint64_t nbytes, const uint64_t *keys,
                           uint64_t nkeys, uint64_t *offsets);

#ifdef __cplusplus
}
#endif

#endif
