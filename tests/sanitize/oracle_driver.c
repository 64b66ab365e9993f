/* oracle_driver.c -- runs the oracle (oracle.c) under the address and
 * undefined-behaviour sanitizers on small random contractions read from
 * stdin, one per line:
 *   <spec> <alpha> <beta> <rank A> <dims A> <rank B> <dims B> <rank C> <dims C>
 * For each it evaluates the contraction, the brute force and every output
 * point, with deterministic pseudo-random inputs, and prints the largest
 * difference between the three. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_contract(const char *spec, double alpha, const double *A, const int64_t *dA, const int64_t *sA,
                    const double *B, const int64_t *dB, const int64_t *sB, double beta, double *C,
                    const int64_t *dC, const int64_t *sC, int nthreads);
int oracle_contract_points(const char *spec, double alpha, const double *A, const int64_t *dA, const int64_t *sA,
                           const double *B, const int64_t *dB, const int64_t *sB, double beta, const double *C,
                           const int64_t *dC, const int64_t *sC, int64_t npts, const int64_t *pts, double *out,
                           int nthreads);
int oracle_bruteforce(const char *spec, double alpha, const double *A, const int64_t *dA, const int64_t *sA,
                      const double *B, const int64_t *dB, const int64_t *sB, double beta, double *C,
                      const int64_t *dC, const int64_t *sC, double *acc);

static int64_t read_dims(int64_t *d, int64_t *s) {
  int r = 0;
  if (scanf("%d", &r) != 1) return -1;
  int64_t n = 1;
  for (int i = 0; i < r; ++i) {
    long long x;
    if (scanf("%lld", &x) != 1) return -1;
    d[i] = x;
  }
  for (int i = r - 1; i >= 0; --i) {
    s[i] = n;
    n *= d[i];
  }
  return n;
}

static double val(uint64_t *st) {
  *st = *st * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)((*st >> 33) % 7) - 3.0;
}

int main(void) {
  char spec[128];
  double alpha, beta, worst = 0.0;
  uint64_t st = 12345;
  long cases = 0;
  while (scanf("%127s %lf %lf", spec, &alpha, &beta) == 3) {
    int64_t dA[16], sA[16], dB[16], sB[16], dC[16], sC[16];
    int64_t nA = read_dims(dA, sA), nB = read_dims(dB, sB), nC = read_dims(dC, sC);
    if (nA < 0 || nB < 0 || nC < 0) return 2;
    double *A = malloc(sizeof(double) * (size_t)(nA ? nA : 1));
    double *B = malloc(sizeof(double) * (size_t)(nB ? nB : 1));
    double *C0 = malloc(sizeof(double) * (size_t)(nC ? nC : 1));
    double *C1 = malloc(sizeof(double) * (size_t)(nC ? nC : 1));
    double *C2 = malloc(sizeof(double) * (size_t)(nC ? nC : 1));
    double *acc = malloc(sizeof(double) * (size_t)(nC ? nC : 1));
    double *pv = malloc(sizeof(double) * (size_t)(nC ? nC : 1));
    for (int64_t i = 0; i < nA; ++i) A[i] = val(&st);
    for (int64_t i = 0; i < nB; ++i) B[i] = val(&st);
    for (int64_t i = 0; i < nC; ++i) C0[i] = val(&st);
    memcpy(C1, C0, sizeof(double) * (size_t)nC);
    memcpy(C2, C0, sizeof(double) * (size_t)nC);
    memset(acc, 0, sizeof(double) * (size_t)(nC ? nC : 1));
    int rc1 = oracle_contract(spec, alpha, A, dA, sA, B, dB, sB, beta, C1, dC, sC, 2);
    int rc2 = oracle_bruteforce(spec, alpha, A, dA, sA, B, dB, sB, beta, C2, dC, sC, acc);
    /* every output point, decoded from its flat index */
    int64_t *pts = malloc(sizeof(int64_t) * 16 * (size_t)(nC ? nC : 1));
    int rank = (int)strcspn(spec, "=");
    for (int64_t o = 0; o < nC; ++o) {
      int64_t x = o;
      for (int q = rank - 1; q >= 0; --q) {
        pts[o * rank + q] = x % dC[q];
        x /= dC[q];
      }
    }
    int rc3 = oracle_contract_points(spec, alpha, A, dA, sA, B, dB, sB, beta, C0, dC, sC, nC, pts, pv, 2);
    if (rc1 || rc2 || rc3) {
      printf("error %d %d %d for %s\n", rc1, rc2, rc3, spec);
      return 1;
    }
    for (int64_t i = 0; i < nC; ++i) {
      double e = fabs(C1[i] - C2[i]) + fabs(C1[i] - pv[i]);
      if (e > worst) worst = e;
    }
    free(A), free(B), free(C0), free(C1), free(C2), free(acc), free(pv), free(pts);
    ++cases;
  }
  printf("cases %ld worst %.3e\n", cases, worst);
  return 0;
}
