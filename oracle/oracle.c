/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the binary
 * tensor contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header or table with the
 * GPU path and has its own spec parser.
 *
 * What it computes (Section 2, the contraction equations; the ta.tc operation
 * of Section 5 with its scaling factor alpha; the "=", "+=" and "-=" forms of
 * the operation grammar in Fig. 2):
 *
 *     C[free] = alpha * sum_{contracted} A[...] * B[...]  +  beta * C[free]
 *
 * The free (external) indices each appear in exactly one input and in the
 * output; the contraction (summation) indices appear in both inputs and not
 * in the output (Section 2).  A label in all three tensors (a batch label)
 * indexes the output and both inputs and is not summed.  beta == 0 means C is not read; alpha == 0 means
 * A and B are not read (BLAS convention; the paper only has "=" (beta 0) and
 * "+=" / "-=" (beta 1, alpha negated for "-=")).
 *
 * Arithmetic: IEEE double, compiled with -ffp-contract=off so every multiply
 * and every add rounds on its own.  The summation order is fixed: contracted
 * labels in order of first appearance in A's label string, the last label
 * varying fastest.  Each output element is computed by exactly one thread, so
 * results do not depend on the thread count.
 *
 * Parity pins for this file live in the CPU test suite: brute force over
 * every index tuple, a pure-Python loop on tiny cases, numpy.einsum, all-ones
 * and Kronecker-delta closed forms, chain reassociation, integer exactness,
 * storage-permutation invariance and the pure-GEMM special case.
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXRANK 16
#define OR_MAXLABELS 52

enum {
  OR_OK = 0,
  OR_ERR_SPEC = 1,    /* malformed spec, label not in exactly two tensors */
  OR_ERR_SHAPE = 2,   /* negative extent, extents of one label disagree */
  OR_ERR_NULL = 4,
  OR_ERR_RANGE = 5    /* point index outside the output */
};

typedef struct {
  int rank[3];                 /* 0 = C, 1 = A, 2 = B */
  char lab[3][OR_MAXRANK];
} or_spec_t;

/* Spec grammar: labels '=' labels '*' labels, one ASCII letter per label,
 * blanks ignored.  Returns 0 or OR_ERR_SPEC. */
static int or_parse(const char *s, or_spec_t *sp) {
  int part = 0;
  memset(sp, 0, sizeof(*sp));
  if (!s) return OR_ERR_SPEC;
  for (; *s; ++s) {
    char ch = *s;
    if (ch == ' ' || ch == '\t') continue;
    if (ch == '=') { if (part != 0) return OR_ERR_SPEC; part = 1; continue; }
    if (ch == '*') { if (part != 1) return OR_ERR_SPEC; part = 2; continue; }
    if (!((ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z'))) return OR_ERR_SPEC;
    if (sp->rank[part] >= OR_MAXRANK) return OR_ERR_SPEC;
    for (int i = 0; i < sp->rank[part]; ++i)
      if (sp->lab[part][i] == ch) return OR_ERR_SPEC;   /* repeated in one tensor */
    sp->lab[part][sp->rank[part]++] = ch;
  }
  if (part != 2) return OR_ERR_SPEC;
  return OR_OK;
}

static int or_find(const or_spec_t *sp, int t, char ch) {
  for (int i = 0; i < sp->rank[t]; ++i)
    if (sp->lab[t][i] == ch) return i;
  return -1;
}

/* One row per distinct label: its extent and its element stride in each of
 * the three tensors (0 where the tensor does not hold the label). */
typedef struct {
  int n;
  char ch[OR_MAXLABELS];
  int64_t ext[OR_MAXLABELS];
  int64_t str[3][OR_MAXLABELS];
  int in[3][OR_MAXLABELS];
} or_table_t;

static int or_table(const or_spec_t *sp, const int64_t *dims[3],
                    const int64_t *strides[3], or_table_t *tb) {
  memset(tb, 0, sizeof(*tb));
  for (int t = 0; t < 3; ++t) {
    for (int p = 0; p < sp->rank[t]; ++p) {
      char ch = sp->lab[t][p];
      int row = -1;
      for (int r = 0; r < tb->n; ++r) if (tb->ch[r] == ch) row = r;
      if (row < 0) {
        row = tb->n++;
        tb->ch[row] = ch;
        tb->ext[row] = dims[t][p];
      }
      if (dims[t][p] < 0) return OR_ERR_SHAPE;
      if (tb->ext[row] != dims[t][p]) return OR_ERR_SHAPE;
      tb->in[t][row] = 1;
      tb->str[t][row] = strides[t][p];
    }
  }
  for (int r = 0; r < tb->n; ++r) {
    int cnt = tb->in[0][r] + tb->in[1][r] + tb->in[2][r];
    /* A label in all three tensors is a batch label: it indexes C, A and B
     * alike and is not summed (the label grammar of Section 4 does not forbid
     * it).  The sum below already treats it that way -- it is one of C's
     * labels, so it fixes A's and B's addresses for each output element and
     * is not among A's contracted labels. */
    if (cnt < 2) return OR_ERR_SPEC;       /* in one tensor only */
    if (cnt == 3 && !tb->in[0][r]) return OR_ERR_SPEC;
  }
  return OR_OK;
}

/* Dense row-major element strides for a tensor of the given dims. */
static void or_rowmajor(int rank, const int64_t *dims, int64_t *out) {
  int64_t s = 1;
  for (int p = rank - 1; p >= 0; --p) { out[p] = s; s *= dims[p]; }
}

typedef struct {
  or_spec_t sp;
  or_table_t tb;
  int nfree, nsum;
  int freerow[OR_MAXRANK];     /* table rows of C's labels, in C's order */
  int sumrow[OR_MAXRANK];      /* contracted labels, first appearance in A */
  int64_t nout, nk;
} or_problem_t;

static int or_setup(or_problem_t *pb, const char *spec,
                    const int64_t *dimsA, const int64_t *strA,
                    const int64_t *dimsB, const int64_t *strB,
                    const int64_t *dimsC, const int64_t *strC,
                    int64_t sA[OR_MAXRANK], int64_t sB[OR_MAXRANK], int64_t sC[OR_MAXRANK]) {
  int rc = or_parse(spec, &pb->sp);
  if (rc) return rc;
  const int64_t *dims[3] = {dimsC, dimsA, dimsB};
  const int64_t *given[3] = {strC, strA, strB};
  int64_t *own[3] = {sC, sA, sB};
  for (int t = 0; t < 3; ++t) {
    if (pb->sp.rank[t] > 0 && !dims[t]) return OR_ERR_NULL;
    if (given[t]) memcpy(own[t], given[t], sizeof(int64_t) * pb->sp.rank[t]);
    else or_rowmajor(pb->sp.rank[t], dims[t], own[t]);
  }
  const int64_t *strides[3] = {sC, sA, sB};
  rc = or_table(&pb->sp, dims, strides, &pb->tb);
  if (rc) return rc;
  pb->nfree = 0; pb->nsum = 0; pb->nout = 1; pb->nk = 1;
  for (int p = 0; p < pb->sp.rank[0]; ++p) {
    char ch = pb->sp.lab[0][p];
    for (int r = 0; r < pb->tb.n; ++r) if (pb->tb.ch[r] == ch) pb->freerow[pb->nfree++] = r;
  }
  for (int p = 0; p < pb->sp.rank[1]; ++p) {
    char ch = pb->sp.lab[1][p];
    if (or_find(&pb->sp, 0, ch) >= 0) continue;          /* free label of A */
    for (int r = 0; r < pb->tb.n; ++r) if (pb->tb.ch[r] == ch) pb->sumrow[pb->nsum++] = r;
  }
  for (int i = 0; i < pb->nfree; ++i) pb->nout *= pb->tb.ext[pb->freerow[i]];
  for (int i = 0; i < pb->nsum; ++i) pb->nk *= pb->tb.ext[pb->sumrow[i]];
  return OR_OK;
}

/* The sum for one output element, given that element's label values. */
static double or_sum(const or_problem_t *pb, const int64_t *freeval,
                     const double *A, const double *B) {
  const or_table_t *tb = &pb->tb;
  int64_t baseA = 0, baseB = 0;
  for (int i = 0; i < pb->nfree; ++i) {
    int r = pb->freerow[i];
    baseA += freeval[i] * tb->str[1][r];   /* stride is 0 where A lacks the label */
    baseB += freeval[i] * tb->str[2][r];
  }
  double s = 0.0;
  if (pb->nk == 0) return s;
  int64_t kv[OR_MAXRANK];
  for (int i = 0; i < pb->nsum; ++i) kv[i] = 0;
  for (;;) {
    int64_t offA = baseA, offB = baseB;
    for (int i = 0; i < pb->nsum; ++i) {
      int r = pb->sumrow[i];
      offA += kv[i] * tb->str[1][r];
      offB += kv[i] * tb->str[2][r];
    }
    double prod = A[offA] * B[offB];
    s = s + prod;
    /* odometer: last contracted label fastest */
    int i = pb->nsum - 1;
    while (i >= 0) {
      if (++kv[i] < tb->ext[pb->sumrow[i]]) break;
      kv[i] = 0;
      --i;
    }
    if (i < 0) break;
  }
  return s;
}

static void or_decode(const or_problem_t *pb, int64_t o, int64_t *val) {
  for (int i = pb->nfree - 1; i >= 0; --i) {
    int64_t e = pb->tb.ext[pb->freerow[i]];
    val[i] = o % e;
    o /= e;
  }
}

static int64_t or_addrC(const or_problem_t *pb, const int64_t *val) {
  int64_t a = 0;
  for (int i = 0; i < pb->nfree; ++i) a += val[i] * pb->tb.str[0][pb->freerow[i]];
  return a;
}

/*
 * oracle_contract: C = alpha * contract(A, B) + beta * C over the whole output.
 * The dims and strides arrays are per tensor, in the order of that tensor's labels in the
 * spec; strides are in elements, NULL means dense row-major.  All data is
 * double.  nthreads <= 0 uses the OpenMP default.
 */
int oracle_contract(const char *spec, double alpha,
                    const double *A, const int64_t *dimsA, const int64_t *strA,
                    const double *B, const int64_t *dimsB, const int64_t *strB,
                    double beta,
                    double *C, const int64_t *dimsC, const int64_t *strC,
                    int nthreads) {
  or_problem_t pb;
  int64_t sA[OR_MAXRANK], sB[OR_MAXRANK], sC[OR_MAXRANK];
  int rc = or_setup(&pb, spec, dimsA, strA, dimsB, strB, dimsC, strC, sA, sB, sC);
  if (rc) return rc;
  if (pb.nout == 0) return OR_OK;
  if (!C) return OR_ERR_NULL;
  if (alpha != 0.0 && pb.nk > 0 && (!A || !B)) return OR_ERR_NULL;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int64_t nout = pb.nout;
#pragma omp parallel for schedule(static)
  for (int64_t o = 0; o < nout; ++o) {
    int64_t val[OR_MAXRANK];
    or_decode(&pb, o, val);
    double s = (alpha == 0.0) ? 0.0 : or_sum(&pb, val, A, B);
    int64_t ac = or_addrC(&pb, val);
    double r = alpha * s;
    if (beta != 0.0) r = r + beta * C[ac];
    C[ac] = r;
  }
  return OR_OK;
}

/*
 * oracle_contract_points: the same result, for n selected output elements
 * only.  points holds n rows of C-rank label values (in C's label order);
 * out[i] receives alpha*sum + beta*C0[point i] (C0 read only when beta != 0,
 * C0 may be NULL then).  Lets full-size GPU results be sampled.
 */
int oracle_contract_points(const char *spec, double alpha,
                           const double *A, const int64_t *dimsA, const int64_t *strA,
                           const double *B, const int64_t *dimsB, const int64_t *strB,
                           double beta,
                           const double *C0, const int64_t *dimsC, const int64_t *strC,
                           int64_t n, const int64_t *points, double *out,
                           int nthreads) {
  or_problem_t pb;
  int64_t sA[OR_MAXRANK], sB[OR_MAXRANK], sC[OR_MAXRANK];
  int rc = or_setup(&pb, spec, dimsA, strA, dimsB, strB, dimsC, strC, sA, sB, sC);
  if (rc) return rc;
  if (n > 0 && (!points || !out)) return OR_ERR_NULL;
  if (beta != 0.0 && n > 0 && !C0) return OR_ERR_NULL;
  int rank = pb.nfree;
  for (int64_t i = 0; i < n; ++i)
    for (int p = 0; p < rank; ++p) {
      int64_t v = points[i * rank + p];
      if (v < 0 || v >= pb.tb.ext[pb.freerow[p]]) return OR_ERR_RANGE;
    }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t *val = points + i * rank;
    double s = (alpha == 0.0) ? 0.0 : or_sum(&pb, val, A, B);
    double r = alpha * s;
    if (beta != 0.0) r = r + beta * C0[or_addrC(&pb, val)];
    out[i] = r;
  }
  return OR_OK;
}

/*
 * oracle_bruteforce: a second, structurally different evaluator for tiny
 * inputs.  One odometer runs over every label (free and contracted) in
 * reverse order of first appearance scanning B, A, C -- so the first label of
 * B varies fastest -- and accumulates each product A*B into a zeroed dense
 * buffer indexed by the output position; alpha and beta are applied at the
 * end.  No strides shortcuts: each step recomputes all three addresses from
 * the full label tuple.  C must be dense enough to hold the result at the
 * given strides; acc is a caller-supplied scratch buffer of nout doubles.
 */
int oracle_bruteforce(const char *spec, double alpha,
                      const double *A, const int64_t *dimsA, const int64_t *strA,
                      const double *B, const int64_t *dimsB, const int64_t *strB,
                      double beta,
                      double *C, const int64_t *dimsC, const int64_t *strC,
                      double *acc) {
  or_problem_t pb;
  int64_t sA[OR_MAXRANK], sB[OR_MAXRANK], sC[OR_MAXRANK];
  int rc = or_setup(&pb, spec, dimsA, strA, dimsB, strB, dimsC, strC, sA, sB, sC);
  if (rc) return rc;
  const or_table_t *tb = &pb.tb;
  if (pb.nout == 0) return OR_OK;
  if (!C || !acc) return OR_ERR_NULL;
  /* label order: scan B, then A, then C, keep first appearances */
  int order[OR_MAXLABELS], nl = 0;
  const int scan[3] = {2, 1, 0};
  for (int si = 0; si < 3; ++si) {
    int t = scan[si];
    for (int p = 0; p < pb.sp.rank[t]; ++p) {
      char ch = pb.sp.lab[t][p];
      int row = -1, seen = 0;
      for (int r = 0; r < tb->n; ++r) if (tb->ch[r] == ch) row = r;
      for (int q = 0; q < nl; ++q) if (order[q] == row) seen = 1;
      if (!seen) order[nl++] = row;
    }
  }
  for (int64_t o = 0; o < pb.nout; ++o) acc[o] = 0.0;
  int any_empty = 0;
  for (int q = 0; q < nl; ++q) if (tb->ext[order[q]] == 0) any_empty = 1;
  if (alpha != 0.0 && !any_empty) {
    int64_t v[OR_MAXLABELS];
    for (int q = 0; q < nl; ++q) v[q] = 0;
    for (;;) {
      int64_t offA = 0, offB = 0, dense = 0;
      for (int q = 0; q < nl; ++q) {
        int r = order[q];
        offA += v[q] * tb->str[1][r];
        offB += v[q] * tb->str[2][r];
      }
      /* dense output position in C's label order, last label fastest */
      for (int i = 0; i < pb.nfree; ++i) {
        int r = pb.freerow[i];
        int64_t val = 0;
        for (int q = 0; q < nl; ++q) if (order[q] == r) val = v[q];
        dense = dense * tb->ext[r] + val;
      }
      acc[dense] = acc[dense] + A[offA] * B[offB];
      /* odometer: first entry of `order` fastest */
      int q = 0;
      while (q < nl) {
        if (++v[q] < tb->ext[order[q]]) break;
        v[q] = 0;
        ++q;
      }
      if (q == nl) break;
    }
  }
  for (int64_t o = 0; o < pb.nout; ++o) {
    int64_t val[OR_MAXRANK];
    or_decode(&pb, o, val);
    int64_t ac = or_addrC(&pb, val);
    double r = alpha * acc[o];
    if (beta != 0.0) r = r + beta * C[ac];
    C[ac] = r;
  }
  return OR_OK;
}

/* Number of threads the OpenMP runtime will use for the next parallel loop. */
int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
