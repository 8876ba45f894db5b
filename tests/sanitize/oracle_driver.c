/* Host-side sanitizer run of the oracle (test infrastructure): every oracle
 * routine on small seeded inputs, mixed dims 1..3, grids that do and do not
 * divide, invalid arguments, and a sliced network, built with
 * -fsanitize=address,undefined.  Exits nonzero on a wrong status or a failed
 * round-trip; the sanitizers abort on any out-of-bounds access or undefined
 * behaviour. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_permute(const double*, int32_t, const int64_t*, const int32_t*, double*);
int orc_tensordot(const double*, int32_t, const int64_t*, const double*, int32_t,
                  const int64_t*, int32_t, const int32_t*, const int32_t*, double*);
int orc_tensordot_entries(const double*, int32_t, const int64_t*, const double*, int32_t,
                          const int64_t*, int32_t, const int32_t*, const int32_t*, int64_t,
                          const int64_t*, double*);
int orc_to_blocked(const double*, int32_t, const int64_t*, const int32_t*, double*);
int orc_from_blocked(const double*, int32_t, const int64_t*, const int32_t*, double*);
int orc_block_tensordot(const double*, int32_t, const int64_t*, const int32_t*, const double*,
                        int32_t, const int64_t*, const int32_t*, int32_t, const int32_t*,
                        const int32_t*, double*, int32_t*);
int orc_statevector(int32_t, int32_t, const int32_t*, const int32_t*, const double*, double*);
double orc_norm2(const double*, int64_t);
int orc_contract_network(int32_t, const int32_t*, const int32_t*, const double*, int32_t,
                         const int32_t*, int32_t, const int32_t*, double*, int64_t, int32_t*,
                         int32_t*);

static uint64_t st = 12345;
static uint64_t nxt(void) {
  st += 0x9E3779B97F4A7C15ULL;
  uint64_t z = st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static int below(int n) { return (int)(nxt() % (uint64_t)n); }
static double *fill(int64_t n) {
  double *x = malloc(sizeof(double) * 2 * (n ? n : 1));
  for (int64_t i = 0; i < 2 * n; ++i) x[i] = (double)below(17) - 8.0;
  return x;
}
static int64_t numel(int r, const int64_t *d) {
  int64_t n = 1;
  for (int i = 0; i < r; ++i) n *= d[i];
  return n;
}
#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                \
    }                                                          \
  } while (0)

static int one_case(void) {
  int rA = 1 + below(6), rB = 1 + below(6);
  int k = below((rA < rB ? rA : rB) + 1);
  int64_t dA[8], dB[8];
  int32_t axA[8], axB[8], gA[8], gB[8];
  int32_t pa[8], pb[8];
  for (int i = 0; i < rA; ++i) pa[i] = i;
  for (int i = 0; i < rB; ++i) pb[i] = i;
  for (int i = rA - 1; i > 0; --i) { int j = below(i + 1), t = pa[i]; pa[i] = pa[j]; pa[j] = t; }
  for (int i = rB - 1; i > 0; --i) { int j = below(i + 1), t = pb[i]; pb[i] = pb[j]; pb[j] = t; }
  for (int i = 0; i < rA; ++i) dA[i] = 1 + below(3);
  for (int i = 0; i < rB; ++i) dB[i] = 1 + below(3);
  for (int i = 0; i < k; ++i) {
    axA[i] = pa[i];
    axB[i] = pb[i];
    dB[axB[i]] = dA[axA[i]];
  }
  for (int i = 0; i < rA; ++i) gA[i] = (dA[i] % 2 == 0 && below(2)) ? 2 : 1;
  for (int i = 0; i < rB; ++i) gB[i] = (dB[i] % 2 == 0 && below(2)) ? 2 : 1;
  int64_t nA = numel(rA, dA), nB = numel(rB, dB), nC = nA * nB;
  for (int i = 0; i < k; ++i) nC /= dA[axA[i]] * dA[axA[i]];
  double *A = fill(nA), *B = fill(nB);
  double *C = calloc(2 * (nC ? nC : 1), sizeof(double));
  double *C2 = calloc(2 * (nC ? nC : 1), sizeof(double));
  CHECK(orc_tensordot(A, rA, dA, B, rB, dB, k, axA, axB, C) == 0);
  /* every entry again, one by one */
  int64_t *idx = malloc(sizeof(int64_t) * (nC ? nC : 1));
  for (int64_t i = 0; i < nC; ++i) idx[i] = i;
  CHECK(orc_tensordot_entries(A, rA, dA, B, rB, dB, k, axA, axB, nC, idx, C2) == 0);
  CHECK(memcmp(C, C2, sizeof(double) * 2 * nC) == 0);
  /* blocked: round trip, then the block contraction on the blocked operands */
  double *Ab = fill(nA), *Bb = fill(nB), *back = fill(nA);
  CHECK(orc_to_blocked(A, rA, dA, gA, Ab) == 0);
  CHECK(orc_from_blocked(Ab, rA, dA, gA, back) == 0);
  CHECK(memcmp(A, back, sizeof(double) * 2 * nA) == 0);
  CHECK(orc_to_blocked(B, rB, dB, gB, Bb) == 0);
  int32_t gC[16];
  double *Cb = calloc(2 * (nC ? nC : 1), sizeof(double));
  CHECK(orc_block_tensordot(Ab, rA, dA, gA, Bb, rB, dB, gB, k, axA, axB, Cb, gC) == 0);
  /* permutation of A */
  double *P = fill(nA);
  CHECK(orc_permute(A, rA, dA, pa, P) == 0);
  /* invalid: repeated axis in a permutation, grid 2 on an odd dim */
  if (rA >= 2) {
    int32_t bad[8];
    memcpy(bad, pa, sizeof(bad));
    bad[1] = bad[0];
    CHECK(orc_permute(A, rA, dA, bad, P) != 0);
  }
  for (int i = 0; i < rA; ++i)
    if (dA[i] % 2 == 1) {
      int32_t g2[8];
      memcpy(g2, gA, sizeof(g2));
      g2[i] = 2;
      CHECK(orc_to_blocked(A, rA, dA, g2, Ab) != 0);
      break;
    }
  (void)orc_norm2(A, nA);
  free(A); free(B); free(C); free(C2); free(idx); free(Ab); free(Bb); free(back); free(Cb);
  free(P);
  return 0;
}

static int network_case(void) {
  /* A ring of 6 rank-3 tensors (dims 2): tensor i has bonds (i, i+1) around
   * the ring and one bond to a hub of rank 6; path contracts in order; two
   * sliced bonds.  Unsliced and sliced results must agree to rounding. */
  int32_t ranks[7] = {3, 3, 3, 3, 3, 3, 6};
  int32_t labels[24];
  int pos = 0;
  for (int i = 0; i < 6; ++i) {
    labels[pos++] = i;
    labels[pos++] = (i + 1) % 6;
    labels[pos++] = 10 + i;
  }
  for (int i = 0; i < 6; ++i) labels[pos++] = 10 + i;
  int64_t tot = 6 * 8 + 64;
  double *data = malloc(sizeof(double) * 2 * tot);
  for (int64_t i = 0; i < 2 * tot; ++i) data[i] = ((double)below(1001) - 500.0) / 500.0;
  int32_t path[12] = {0, 1, 7, 2, 8, 3, 9, 4, 10, 5, 11, 6};
  int32_t sliced[2] = {2, 13};
  double out[2], out2[2];
  int32_t orank, olab[64];
  CHECK(orc_contract_network(7, ranks, labels, data, 6, path, 0, sliced, out, 2, &orank, olab) == 0);
  CHECK(orank == 0);
  CHECK(orc_contract_network(7, ranks, labels, data, 6, path, 2, sliced, out2, 2, &orank, olab) == 0);
  CHECK(fabs(out[0] - out2[0]) + fabs(out[1] - out2[1]) <= 1e-12 * (1 + fabs(out[0]) + fabs(out[1])));
  /* a path that uses an id twice is refused */
  int32_t bad[12] = {0, 1, 0, 2, 8, 3, 9, 4, 10, 5, 11, 6};
  CHECK(orc_contract_network(7, ranks, labels, data, 6, bad, 0, sliced, out, 2, &orank, olab) != 0);
  free(data);
  return 0;
}

static int statevector_case(void) {
  /* H on qubit 0, then CNOT chain: GHZ on 5 qubits. */
  const double h = 0.70710678118654752440;
  double mats[2 * 4 + 4 * 2 * 16];
  int32_t nq[5] = {1, 2, 2, 2, 2}, qs[9] = {0, 0, 1, 1, 2, 2, 3, 3, 4};
  double H[8] = {h, 0, h, 0, h, 0, -h, 0};
  memcpy(mats, H, sizeof(H));
  double X[32] = {0};
  int perm[4] = {0, 1, 3, 2};
  for (int r = 0; r < 4; ++r) X[2 * (4 * r + perm[r])] = 1.0;
  for (int g = 0; g < 4; ++g) memcpy(mats + 8 + 32 * g, X, sizeof(X));
  double psi[64];
  CHECK(orc_statevector(5, 5, nq, qs, mats, psi) == 0);
  CHECK(fabs(psi[0] - h) < 1e-15 && fabs(psi[62] - h) < 1e-15);
  CHECK(fabs(orc_norm2(psi, 32) - 1.0) < 1e-15);
  CHECK(orc_statevector(0, 0, nq, qs, mats, psi) != 0);
  return 0;
}

int main(void) {
  for (int t = 0; t < 300; ++t)
    if (one_case()) return 1;
  if (network_case()) return 1;
  if (statevector_case()) return 1;
  printf("oracle sanitizer run: ok\n");
  return 0;
}
