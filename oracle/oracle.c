/*
 * oracle.c -- FP64 reference for the general strided tensor contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the HIP
 * library.
 *
 * What it computes (Approach, "Supporting tensor computations": the
 * block-scatter tensor-to-matrix mapping lets matrix algorithms run directly
 * on tensors; Introduction, "Challenges": tensor work without explicit
 * conversion between tensors and matrices; Approach, "Variations on
 * functionality": transposition expressed purely through strides).  The paper
 * gives no formula, so the oracle writes out the plain definition of a
 * labelled contraction over strided storage:
 *
 *     C[c] <- alpha * sum_{s} A[addr_A(c,s)] * B[addr_B(c,s)] + beta * C[c]
 *
 * for every multi-index c over C's labels, where s runs over every label that
 * appears in A or B but not in C, and the address of an element is
 * base + sum_d index(label_d) * stride_d.  These are einsum semantics: a label
 * in all three tensors acts as a batch index, a label only in A (or only in
 * B) is summed inside the product, and a label repeated within A or B selects
 * a diagonal.
 *
 * Conventions (the paper is silent; readings listed with the design notes):
 *   - beta == 0: C is not read (BLAS convention), so NaN in C0 does not leak.
 *   - alpha == 0: A and B are not read.
 *   - An empty sum (a summed label of extent 0) contributes 0.
 *   - Summation is sequential in odometer order (first summed label
 *     fastest), in FP64, optionally Neumaier-compensated.
 *   - Optionally emits D[c] = |alpha| * sum_s |A*B| + |beta| * |C0[c]|, the
 *     componentwise condition tensor used by the error bounds.
 *   - split == 1 forms each product from the bf16 hi/lo split of the two
 *     operands (mixed precision, Introduction, "Challenges", and "Supporting
 *     new and mixed precisions"): hi = RNE_bf16(x), lo = RNE_bf16(x - hi),
 *     product = hi_a*hi_b + hi_a*lo_b + lo_a*hi_b, each term exact in FP64.
 *     This is the split-exact reference for the bf16x3 path.
 *   - split == 2 splits each operand three ways, h = RNE_bf16(x),
 *     m = RNE_bf16(x - h), l = RNE_bf16(x - h - m) (the differences are exact
 *     in FP32), and keeps the six products whose orders sum to at most two
 *     units of 2^-8: hh, hm, mh, hl, lh, mm.  Reference for the bf16x6 path.
 *   - split == 16 + s (1 <= s <= 12) is FP64 emulated on 8-bit integer
 *     products with s slices (new and mixed precisions, Introduction,
 *     "Challenges", and "Supporting new and mixed precisions"; the slicing is
 *     the error-free splitting of Ozaki, Ogita, Oishi and Rump, in the integer
 *     form of Ootomo, Ozaki and Yokota).  For one C entry the "row" of A is
 *     every A element its sum reads, and the "column" of B likewise:
 *       1. each is scaled by a power of two, 2^-ea and 2^-eb, where e is the
 *          smallest integer with max|v| <= (127/128) 2^e (0 for an all-zero
 *          row), so every scaled value lies in [-127/128, 127/128];
 *       2. each scaled value v is cut into s signed digits by exact rounding
 *          to nearest (ties to even), the extraction of the error-free
 *          splitting: r_0 = v, d_t = rint(2^7 r_{t-1}), r_t = 2^7 r_{t-1} - d_t,
 *          so v = sum_t d_t 2^-7t + 2^-7s r_s with |d_1| <= 127,
 *          |d_t| <= 64 for t >= 2 and |r_s| <= 1/2;
 *       3. for every digit pair (t, u) with t + u <= s + 1 the digit products
 *          are summed over the sum's index space as exact integers S_tu;
 *       4. the entry's product term is 2^(ea+eb) sum_tu S_tu 2^-7(t+u),
 *          summed in FP64 (compensated, t then u ascending).
 *     A row or column holding a non-finite value gives NaN.
 *
 * Built with -O2 -fopenmp -ffp-contract=off and no fast-math, so results are
 * reproducible on any x86-64 host.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_RANK 8
#define ORACLE_MAX_LABELS (3 * ORACLE_MAX_RANK)

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_SHAPE (-2)
#define ORACLE_ERR_LABEL (-3)

typedef struct {
  int32_t rank;
  const int64_t *extents;
  const int64_t *strides;
  const int32_t *labels;
} oracle_tensor;

/* Round a float to the nearest bfloat16 value, ties to even, by keeping the
 * top 16 bits of its IEEE-754 binary32 encoding after adding half an ulp of
 * the kept part (plus one when the kept part is odd).  NaN stays NaN. */
static float bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, sizeof u);
  if ((u & 0x7f800000u) == 0x7f800000u) {
    if (u & 0x007fffffu) u |= 0x00400000u; /* keep NaN a NaN after truncation */
    u &= 0xffff0000u;
  } else {
    uint32_t keep_odd = (u >> 16) & 1u;
    u += 0x7fffu + keep_odd;
    u &= 0xffff0000u;
  }
  float r;
  memcpy(&r, &u, sizeof r);
  return r;
}

void oracle_bf16_rne(const float *in, float *out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = bf16_rne(in[i]);
}

/* One contraction problem after label analysis. */
typedef struct {
  int nlab;                              /* distinct labels */
  int32_t lab[ORACLE_MAX_LABELS];        /* label values */
  int64_t ext[ORACLE_MAX_LABELS];        /* extent of each label */
  int64_t sA[ORACLE_MAX_LABELS];         /* A stride of each label (sum over repeats) */
  int64_t sB[ORACLE_MAX_LABELS];
  int nout;                              /* C's modes, in C's order */
  int out_lab[ORACLE_MAX_RANK];          /* label slot of C mode d */
  int64_t out_stride[ORACLE_MAX_RANK];   /* C stride of mode d */
  int nsum;                              /* summed labels */
  int sum_lab[ORACLE_MAX_LABELS];        /* label slot of summed label */
  int64_t nentries;                      /* number of C entries */
} problem;

static int find_or_add(problem *p, int32_t label, int64_t extent) {
  for (int i = 0; i < p->nlab; ++i) {
    if (p->lab[i] == label) return p->ext[i] == extent ? i : -2;
  }
  p->lab[p->nlab] = label;
  p->ext[p->nlab] = extent;
  p->sA[p->nlab] = 0;
  p->sB[p->nlab] = 0;
  return p->nlab++;
}

static int check_tensor(const oracle_tensor *t) {
  if (!t) return ORACLE_ERR_ARG;
  if (t->rank < 0 || t->rank > ORACLE_MAX_RANK) return ORACLE_ERR_ARG;
  if (t->rank > 0 && (!t->extents || !t->strides || !t->labels)) return ORACLE_ERR_ARG;
  for (int d = 0; d < t->rank; ++d)
    if (t->extents[d] < 0) return ORACLE_ERR_ARG;
  return ORACLE_OK;
}

static int analyse(const oracle_tensor *A, const oracle_tensor *B, const oracle_tensor *C,
                   problem *p) {
  int rc;
  if ((rc = check_tensor(A)) || (rc = check_tensor(B)) || (rc = check_tensor(C))) return rc;
  memset(p, 0, sizeof *p);
  /* C's labels first, each exactly once. */
  for (int d = 0; d < C->rank; ++d) {
    for (int e = 0; e < d; ++e)
      if (C->labels[e] == C->labels[d]) return ORACLE_ERR_LABEL;
    int slot = find_or_add(p, C->labels[d], C->extents[d]);
    p->out_lab[d] = slot;
    p->out_stride[d] = C->strides[d];
  }
  p->nout = C->rank;
  for (int d = 0; d < A->rank; ++d) {
    int slot = find_or_add(p, A->labels[d], A->extents[d]);
    if (slot == -2) return ORACLE_ERR_SHAPE;
    p->sA[slot] += A->strides[d];
  }
  for (int d = 0; d < B->rank; ++d) {
    int slot = find_or_add(p, B->labels[d], B->extents[d]);
    if (slot == -2) return ORACLE_ERR_SHAPE;
    p->sB[slot] += B->strides[d];
  }
  /* Every output label must come from an input. */
  for (int d = 0; d < C->rank; ++d) {
    int32_t l = C->labels[d];
    int found = 0;
    for (int e = 0; e < A->rank; ++e) found |= (A->labels[e] == l);
    for (int e = 0; e < B->rank; ++e) found |= (B->labels[e] == l);
    if (!found) return ORACLE_ERR_LABEL;
  }
  /* Summed labels: everything that is not an output label, in order of
   * first appearance (A, then B). */
  p->nsum = 0;
  for (int i = C->rank; i < p->nlab; ++i) p->sum_lab[p->nsum++] = i;
  p->nentries = 1;
  for (int d = 0; d < C->rank; ++d) p->nentries *= C->extents[d];
  return ORACLE_OK;
}

typedef struct {
  double sum, comp, abssum;
} accum;

static void acc_add(accum *a, double t, int compensated) {
  if (compensated) {
    double s = a->sum + t;
    if (fabs(a->sum) >= fabs(t))
      a->comp += (a->sum - s) + t;
    else
      a->comp += (t - s) + a->sum;
    a->sum = s;
  } else {
    a->sum += t;
  }
}

/* Element offsets of A and B for the label values in idx[]. */
static void addresses(const problem *p, const int64_t *idx, int64_t *offA, int64_t *offB) {
  int64_t oa = 0, ob = 0;
  for (int l = 0; l < p->nlab; ++l) {
    oa += idx[l] * p->sA[l];
    ob += idx[l] * p->sB[l];
  }
  *offA = oa;
  *offB = ob;
}

/* Odometer step over the summed labels, first summed label fastest. */
static void next_summed(const problem *p, int64_t *idx) {
  for (int s = 0; s < p->nsum; ++s) {
    int l = p->sum_lab[s];
    if (++idx[l] < p->ext[l]) break;
    idx[l] = 0;
  }
}

#define ORACLE_INT8_BASE 16
#define ORACLE_INT8_MAX_SLICES 12

/* Step 1 of the slicing: the smallest integer e with amax <= (127/128) 2^e
 * (amax >= 0, finite); 0 when amax == 0. */
static int scale_exponent(double amax) {
  if (amax == 0.0) return 0;
  int e;
  double f = frexp(amax, &e); /* amax = f 2^e, 0.5 <= f < 1 */
  return f <= 127.0 / 128.0 ? e : e + 1;
}

/* Step 2: the s digits of v = x 2^-e (|v| <= 127/128), by exact rounding to
 * nearest (the default rounding mode: ties to even). */
static void int8_digits(double x, int e, int s, int *d) {
  double r = ldexp(x, -e);
  for (int t = 0; t < s; ++t) {
    double y = ldexp(r, 7);
    double q = rint(y);
    d[t] = (int)q;
    r = y - q;
  }
}

void oracle_int8_digits(const double *x, int64_t n, int e, int s, int8_t *out) {
  int d[ORACLE_INT8_MAX_SLICES];
  for (int64_t i = 0; i < n; ++i) {
    int8_digits(x[i], e, s, d);
    for (int t = 0; t < s; ++t) out[i * s + t] = (int8_t)d[t];
  }
}

/* Steps 1-4 for one output entry; returns the product term (before alpha)
 * and fills *abssum with sum |a b|. */
static double int8_entry(const problem *p, int64_t *idx, const double *a, const double *b, int s,
                         int64_t terms, double *abssum) {
  double amax = 0.0, bmax = 0.0, asum = 0.0;
  int finite = 1;
  for (int q = 0; q < p->nsum; ++q) idx[p->sum_lab[q]] = 0;
  for (int64_t t = 0; t < terms; ++t) {
    int64_t offA, offB;
    addresses(p, idx, &offA, &offB);
    double x = a[offA], y = b[offB];
    if (!isfinite(x) || !isfinite(y)) finite = 0;
    if (fabs(x) > amax) amax = fabs(x);
    if (fabs(y) > bmax) bmax = fabs(y);
    asum += fabs(x * y);
    next_summed(p, idx);
  }
  *abssum = asum;
  if (!finite) return NAN;
  const int ea = scale_exponent(amax), eb = scale_exponent(bmax);
  int64_t S[ORACLE_INT8_MAX_SLICES + 1][ORACLE_INT8_MAX_SLICES + 1];
  memset(S, 0, sizeof S);
  int da[ORACLE_INT8_MAX_SLICES], db[ORACLE_INT8_MAX_SLICES];
  for (int q = 0; q < p->nsum; ++q) idx[p->sum_lab[q]] = 0;
  for (int64_t t = 0; t < terms; ++t) {
    int64_t offA, offB;
    addresses(p, idx, &offA, &offB);
    int8_digits(a[offA], ea, s, da);
    int8_digits(b[offB], eb, s, db);
    for (int i = 1; i <= s; ++i)
      for (int j = 1; i + j <= s + 1; ++j) S[i][j] += (int64_t)da[i - 1] * (int64_t)db[j - 1];
    next_summed(p, idx);
  }
  accum acc = {0.0, 0.0, 0.0};
  for (int i = 1; i <= s; ++i)
    for (int j = 1; i + j <= s + 1; ++j) acc_add(&acc, ldexp((double)S[i][j], -7 * (i + j)), 1);
  return ldexp(acc.sum + acc.comp, ea + eb);
}

/* Sum over the summed labels for one output entry whose label values are in
 * idx[] (output slots filled, summed slots overwritten here). */
static void one_entry(const problem *p, int64_t *idx, const double *a, const double *b,
                      int split, int compensated, accum *out) {
  accum acc = {0.0, 0.0, 0.0};
  int64_t terms = 1;
  for (int s = 0; s < p->nsum; ++s) terms *= p->ext[p->sum_lab[s]];
  if (split > ORACLE_INT8_BASE) {
    acc.sum = int8_entry(p, idx, a, b, split - ORACLE_INT8_BASE, terms, &acc.abssum);
    *out = acc;
    return;
  }
  for (int s = 0; s < p->nsum; ++s) idx[p->sum_lab[s]] = 0;
  for (int64_t t = 0; t < terms; ++t) {
    int64_t offA, offB;
    addresses(p, idx, &offA, &offB);
    double x = a[offA], y = b[offB];
    acc.abssum += fabs(x * y);
    if (split == 1) {
      float xf = (float)x, yf = (float)y;
      float xh = bf16_rne(xf), yh = bf16_rne(yf);
      float xl = bf16_rne(xf - xh), yl = bf16_rne(yf - yh);
      acc_add(&acc, (double)xh * (double)yh, compensated);
      acc_add(&acc, (double)xh * (double)yl, compensated);
      acc_add(&acc, (double)xl * (double)yh, compensated);
    } else if (split == 2) {
      float xf = (float)x, yf = (float)y;
      float xh = bf16_rne(xf), yh = bf16_rne(yf);
      float xr = xf - xh, yr = yf - yh;
      float xm = bf16_rne(xr), ym = bf16_rne(yr);
      float xl = bf16_rne(xr - xm), yl = bf16_rne(yr - ym);
      acc_add(&acc, (double)xh * (double)yh, compensated);
      acc_add(&acc, (double)xh * (double)ym, compensated);
      acc_add(&acc, (double)xm * (double)yh, compensated);
      acc_add(&acc, (double)xh * (double)yl, compensated);
      acc_add(&acc, (double)xm * (double)ym, compensated);
      acc_add(&acc, (double)xl * (double)yh, compensated);
    } else {
      acc_add(&acc, x * y, compensated);
    }
    next_summed(p, idx);
  }
  *out = acc;
}

static double finish(const accum *acc, double alpha, double beta, double c0, int compensated) {
  double ab = compensated ? acc->sum + acc->comp : acc->sum;
  double r = 0.0;
  if (alpha != 0.0) r = alpha * ab;
  if (beta != 0.0) r = r + beta * c0;
  return r;
}

/* Full contraction, result written into c (which holds C0 on entry) at C's
 * strides.  d, if not NULL, receives the condition tensor at C's strides. */
int oracle_contract(double alpha, const oracle_tensor *A, const double *a,
                    const oracle_tensor *B, const double *b, double beta,
                    const oracle_tensor *C, double *c, double *d, int split,
                    int compensated, int nthreads) {
  problem p;
  int rc = analyse(A, B, C, &p);
  if (rc) return rc;
  if (!c || (alpha != 0.0 && (!a || !b))) return ORACLE_ERR_ARG;
  if (split < 0 || (split > 2 && split <= ORACLE_INT8_BASE) ||
      split > ORACLE_INT8_BASE + ORACLE_INT8_MAX_SLICES)
    return ORACLE_ERR_ARG;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t e = 0; e < p.nentries; ++e) {
    int64_t idx[ORACLE_MAX_LABELS];
    memset(idx, 0, sizeof idx);
    /* column-major odometer digits of entry e over C's modes */
    int64_t rem = e, offC = 0;
    for (int m = 0; m < p.nout; ++m) {
      int64_t ext = p.ext[p.out_lab[m]];
      idx[p.out_lab[m]] = rem % ext;
      rem /= ext;
      offC += idx[p.out_lab[m]] * p.out_stride[m];
    }
    accum acc = {0.0, 0.0, 0.0};
    if (alpha != 0.0) one_entry(&p, idx, a, b, split, compensated, &acc);
    double c0 = (beta != 0.0) ? c[offC] : 0.0;
    double r = finish(&acc, alpha, beta, c0, compensated);
    if (d) d[offC] = fabs(alpha) * acc.abssum + fabs(beta) * fabs(c0);
    c[offC] = r;
  }
  return ORACLE_OK;
}

/* Selected entries only: cidx holds n multi-indices over C's modes (row-major
 * n x rank).  C0 is read from c0 at C's strides (only when beta != 0); the
 * results go to out[i] (and the condition numbers to dout[i] if not NULL). */
int oracle_contract_entries(double alpha, const oracle_tensor *A, const double *a,
                            const oracle_tensor *B, const double *b, double beta,
                            const oracle_tensor *C, const double *c0,
                            const int64_t *cidx, int64_t n, double *out, double *dout,
                            int split, int compensated, int nthreads) {
  problem p;
  int rc = analyse(A, B, C, &p);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!cidx || !out))) return ORACLE_ERR_ARG;
  if (beta != 0.0 && n > 0 && !c0) return ORACLE_ERR_ARG;
  if (alpha != 0.0 && (!a || !b)) return ORACLE_ERR_ARG;
  if (split < 0 || (split > 2 && split <= ORACLE_INT8_BASE) ||
      split > ORACLE_INT8_BASE + ORACLE_INT8_MAX_SLICES)
    return ORACLE_ERR_ARG;
  for (int64_t i = 0; i < n; ++i)
    for (int m = 0; m < p.nout; ++m) {
      int64_t v = cidx[i * p.nout + m];
      if (v < 0 || v >= p.ext[p.out_lab[m]]) return ORACLE_ERR_ARG;
    }
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int64_t i = 0; i < n; ++i) {
    int64_t idx[ORACLE_MAX_LABELS];
    memset(idx, 0, sizeof idx);
    int64_t offC = 0;
    for (int m = 0; m < p.nout; ++m) {
      idx[p.out_lab[m]] = cidx[i * p.nout + m];
      offC += idx[p.out_lab[m]] * p.out_stride[m];
    }
    accum acc = {0.0, 0.0, 0.0};
    if (alpha != 0.0) one_entry(&p, idx, a, b, split, compensated, &acc);
    double cv = (beta != 0.0) ? c0[offC] : 0.0;
    out[i] = finish(&acc, alpha, beta, cv, compensated);
    if (dout) dout[i] = fabs(alpha) * acc.abssum + fabs(beta) * fabs(cv);
  }
  return ORACLE_OK;
}
