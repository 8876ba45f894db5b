/*
 * Oracle: plain, slow, single-threaded CPU reference for block tensor
 * contraction and sliced tensor-network contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may call,
 * link or load this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the GPU implementation.
 *
 * Arithmetic: complex128 written out as real double arithmetic
 * (re += ar*br - ai*bi; im += ar*bi + ai*br), summed in a fixed sequential
 * order.  Compiled with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math) so every product and sum is an individually rounded IEEE op.
 *
 * Memory conventions (readings of what the paper leaves open):
 *   - tensors are row-major (C order), complex values interleaved (re, im);
 *   - a tensordot output lists A's free axes in A's order, then B's free axes
 *     in B's order (the pairwise contraction formula of Section II.A);
 *   - axesA[i] is paired with axesB[i]; paired dims must be equal;
 *   - a blocked tensor over a uniform grid (Section II.C) is stored
 *     block-major: block coordinates row-major, each block contiguous and
 *     row-major inside.
 *
 * Every function returns 0 on success and a nonzero code on invalid input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_RANK 64

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ESHAPE = 2, ORC_EGRID = 3, ORC_ENOMEM = 5 };

static int64_t orc_numel(int32_t rank, const int64_t* dims) {
  int64_t n = 1;
  for (int32_t j = 0; j < rank; ++j) n *= dims[j];
  return n;
}

/* Row-major strides, in complex elements. */
static void orc_strides(int32_t rank, const int64_t* dims, int64_t* st) {
  int64_t s = 1;
  for (int32_t j = rank - 1; j >= 0; --j) {
    st[j] = s;
    s *= dims[j];
  }
}

static void orc_unravel(int64_t lin, int32_t rank, const int64_t* dims, int64_t* idx) {
  for (int32_t j = rank - 1; j >= 0; --j) {
    idx[j] = lin % dims[j];
    lin /= dims[j];
  }
}

/* ------------------------------------------------------------------------ */
/* Index permutation: out.shape[j] = in.shape[perm[j]] (transpose).           */
/* ------------------------------------------------------------------------ */
int orc_permute(const double* in, int32_t rank, const int64_t* dims, const int32_t* perm,
                double* out) {
  if (rank < 0 || rank > ORC_MAX_RANK) return ORC_EINVAL;
  int seen[ORC_MAX_RANK] = {0};
  for (int32_t j = 0; j < rank; ++j) {
    if (perm[j] < 0 || perm[j] >= rank || seen[perm[j]]) return ORC_EINVAL;
    seen[perm[j]] = 1;
  }
  int64_t in_st[ORC_MAX_RANK], odims[ORC_MAX_RANK], idx[ORC_MAX_RANK];
  orc_strides(rank, dims, in_st);
  for (int32_t j = 0; j < rank; ++j) odims[j] = dims[perm[j]];
  int64_t n = orc_numel(rank, dims);
  for (int64_t o = 0; o < n; ++o) {
    orc_unravel(o, rank, odims, idx);
    int64_t src = 0;
    for (int32_t j = 0; j < rank; ++j) src += idx[j] * in_st[perm[j]];
    out[2 * o] = in[2 * src];
    out[2 * o + 1] = in[2 * src + 1];
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Pairwise contraction (Section II.A; numpy tensordot semantics).           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t nfa, nfb, k;
  int32_t fa[ORC_MAX_RANK], fb[ORC_MAX_RANK];
  int64_t cdims[2 * ORC_MAX_RANK];
  int32_t crank;
  int64_t K;
  int64_t* offa; /* contracted offsets into A, K entries, row-major over pairs */
  int64_t* offb;
  int64_t sta[ORC_MAX_RANK], stb[ORC_MAX_RANK];
} orc_td;

static int orc_td_setup(orc_td* t, int32_t rA, const int64_t* dA, int32_t rB,
                        const int64_t* dB, int32_t k, const int32_t* axA,
                        const int32_t* axB) {
  if (rA < 0 || rB < 0 || rA > ORC_MAX_RANK || rB > ORC_MAX_RANK) return ORC_EINVAL;
  if (k < 0 || k > rA || k > rB) return ORC_EINVAL;
  int ca[ORC_MAX_RANK] = {0}, cb[ORC_MAX_RANK] = {0};
  for (int32_t i = 0; i < k; ++i) {
    if (axA[i] < 0 || axA[i] >= rA || axB[i] < 0 || axB[i] >= rB) return ORC_EINVAL;
    if (ca[axA[i]] || cb[axB[i]]) return ORC_EINVAL;
    ca[axA[i]] = cb[axB[i]] = 1;
    if (dA[axA[i]] != dB[axB[i]]) return ORC_ESHAPE;
  }
  t->k = k;
  t->nfa = t->nfb = 0;
  for (int32_t j = 0; j < rA; ++j)
    if (!ca[j]) t->fa[t->nfa++] = j;
  for (int32_t j = 0; j < rB; ++j)
    if (!cb[j]) t->fb[t->nfb++] = j;
  t->crank = t->nfa + t->nfb;
  for (int32_t j = 0; j < t->nfa; ++j) t->cdims[j] = dA[t->fa[j]];
  for (int32_t j = 0; j < t->nfb; ++j) t->cdims[t->nfa + j] = dB[t->fb[j]];
  orc_strides(rA, dA, t->sta);
  orc_strides(rB, dB, t->stb);
  int64_t kd[ORC_MAX_RANK], kidx[ORC_MAX_RANK];
  t->K = 1;
  for (int32_t i = 0; i < k; ++i) {
    kd[i] = dA[axA[i]];
    t->K *= kd[i];
  }
  t->offa = (int64_t*)malloc(sizeof(int64_t) * (size_t)(t->K > 0 ? t->K : 1));
  t->offb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(t->K > 0 ? t->K : 1));
  if (!t->offa || !t->offb) {
    free(t->offa);
    free(t->offb);
    return ORC_ENOMEM;
  }
  for (int64_t c = 0; c < t->K; ++c) {
    orc_unravel(c, k, kd, kidx);
    int64_t oa = 0, ob = 0;
    for (int32_t i = 0; i < k; ++i) {
      oa += kidx[i] * t->sta[axA[i]];
      ob += kidx[i] * t->stb[axB[i]];
    }
    t->offa[c] = oa;
    t->offb[c] = ob;
  }
  return ORC_OK;
}

static void orc_td_free(orc_td* t) {
  free(t->offa);
  free(t->offb);
}

/* One output entry C[lin], summing over the contracted index in ascending
 * row-major order of the pairing. */
static void orc_td_entry(const orc_td* t, const double* A, const double* B, int64_t lin,
                         double* re_out, double* im_out) {
  int64_t idx[2 * ORC_MAX_RANK];
  orc_unravel(lin, t->crank, t->cdims, idx);
  int64_t ba = 0, bb = 0;
  for (int32_t j = 0; j < t->nfa; ++j) ba += idx[j] * t->sta[t->fa[j]];
  for (int32_t j = 0; j < t->nfb; ++j) bb += idx[t->nfa + j] * t->stb[t->fb[j]];
  double re = 0.0, im = 0.0;
  for (int64_t c = 0; c < t->K; ++c) {
    const double* a = A + 2 * (ba + t->offa[c]);
    const double* b = B + 2 * (bb + t->offb[c]);
    double pr = a[0] * b[0] - a[1] * b[1];
    double pi = a[0] * b[1] + a[1] * b[0];
    re += pr;
    im += pi;
  }
  *re_out = re;
  *im_out = im;
}

int orc_tensordot(const double* A, int32_t rA, const int64_t* dA, const double* B, int32_t rB,
                  const int64_t* dB, int32_t k, const int32_t* axA, const int32_t* axB,
                  double* C) {
  orc_td t;
  int rc = orc_td_setup(&t, rA, dA, rB, dB, k, axA, axB);
  if (rc) return rc;
  int64_t n = orc_numel(t.crank, t.cdims);
  for (int64_t o = 0; o < n; ++o) orc_td_entry(&t, A, B, o, &C[2 * o], &C[2 * o + 1]);
  orc_td_free(&t);
  return ORC_OK;
}

/* Selected output entries only (row-major linear indices into C): lets the
 * tests check outputs of contractions too large to evaluate whole. */
int orc_tensordot_entries(const double* A, int32_t rA, const int64_t* dA, const double* B,
                          int32_t rB, const int64_t* dB, int32_t k, const int32_t* axA,
                          const int32_t* axB, int64_t nent, const int64_t* cidx, double* out) {
  orc_td t;
  int rc = orc_td_setup(&t, rA, dA, rB, dB, k, axA, axB);
  if (rc) return rc;
  int64_t n = orc_numel(t.crank, t.cdims);
  for (int64_t e = 0; e < nent; ++e) {
    if (cidx[e] < 0 || cidx[e] >= n) {
      orc_td_free(&t);
      return ORC_EINVAL;
    }
    orc_td_entry(&t, A, B, cidx[e], &out[2 * e], &out[2 * e + 1]);
  }
  orc_td_free(&t);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Uniform-grid block layout (Section II.C).                                 */
/* ------------------------------------------------------------------------ */
static int orc_check_grid(int32_t rank, const int64_t* dims, const int32_t* grid) {
  for (int32_t j = 0; j < rank; ++j) {
    if (dims[j] < 1) return ORC_ESHAPE;
    if (grid[j] < 1 || dims[j] % grid[j] != 0) return ORC_EGRID;
  }
  return ORC_OK;
}

/* Offset, in the block-major buffer, of the element at dense coordinates x. */
static int64_t orc_blocked_offset(int32_t rank, const int64_t* dims, const int32_t* grid,
                                  const int64_t* x) {
  int64_t blin = 0, ilin = 0, bsize = 1;
  for (int32_t j = 0; j < rank; ++j) {
    int64_t ext = dims[j] / grid[j];
    blin = blin * grid[j] + x[j] / ext;
    ilin = ilin * ext + x[j] % ext;
    bsize *= ext;
  }
  return blin * bsize + ilin;
}

int orc_to_blocked(const double* dense, int32_t rank, const int64_t* dims,
                   const int32_t* grid, double* blocked) {
  if (rank < 0 || rank > ORC_MAX_RANK) return ORC_EINVAL;
  int rc = orc_check_grid(rank, dims, grid);
  if (rc) return rc;
  int64_t n = orc_numel(rank, dims), x[ORC_MAX_RANK];
  for (int64_t o = 0; o < n; ++o) {
    orc_unravel(o, rank, dims, x);
    int64_t d = orc_blocked_offset(rank, dims, grid, x);
    blocked[2 * d] = dense[2 * o];
    blocked[2 * d + 1] = dense[2 * o + 1];
  }
  return ORC_OK;
}

int orc_from_blocked(const double* blocked, int32_t rank, const int64_t* dims,
                     const int32_t* grid, double* dense) {
  if (rank < 0 || rank > ORC_MAX_RANK) return ORC_EINVAL;
  int rc = orc_check_grid(rank, dims, grid);
  if (rc) return rc;
  int64_t n = orc_numel(rank, dims), x[ORC_MAX_RANK];
  for (int64_t o = 0; o < n; ++o) {
    orc_unravel(o, rank, dims, x);
    int64_t s = orc_blocked_offset(rank, dims, grid, x);
    dense[2 * o] = blocked[2 * s];
    dense[2 * o + 1] = blocked[2 * s + 1];
  }
  return ORC_OK;
}

static int64_t orc_gcd(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

/* Copy the sub-tensor with origin org and extents ext out of a block-major
 * buffer (dims, grid) into a dense row-major array. */
static void orc_extract(const double* blocked, int32_t rank, const int64_t* dims,
                        const int32_t* grid, const int64_t* org, const int64_t* ext,
                        double* dst) {
  int64_t n = orc_numel(rank, ext), loc[ORC_MAX_RANK], x[ORC_MAX_RANK];
  for (int64_t o = 0; o < n; ++o) {
    orc_unravel(o, rank, ext, loc);
    for (int32_t j = 0; j < rank; ++j) x[j] = org[j] + loc[j];
    int64_t s = orc_blocked_offset(rank, dims, grid, x);
    dst[2 * o] = blocked[2 * s];
    dst[2 * o + 1] = blocked[2 * s + 1];
  }
}

/* Block tensor contraction, the four steps of Section II.C:
 *   (1) for each block of C, the blocks of A and B it needs are the ones whose
 *       non-contracted coordinates match the C block's;
 *   (2) those are paired by matching coordinates on the contracted axes;
 *   (3) each pair is contracted locally into a partial block;
 *   (4) the partials are added into the C block.
 * Where the two operands split a contracted pair of axes differently, both
 * are viewed on the common refinement (least common multiple of the two grid
 * counts), which leaves the result unchanged.  C's grid is A's free-axis grid
 * followed by B's.  Pairs are visited in ascending row-major order of their
 * contracted block coordinates.  gC receives C's grid (rank rA + rB - 2k). */
typedef struct {
  const orc_td* t;
  const double *Ab, *Bb;
  double* Cb;
  int32_t rA, rB, k, crank;
  const int64_t *dA, *dB;
  const int32_t *gA, *gB, *axA, *axB;
  const int64_t *cgrid, *pg, *extA, *extB;
  int64_t csz, npair, asz, bsz;
} orc_blk_job;

/* The four steps of Section II.C for output block `blk` (row-major block
 * index): pairs in ascending order, each contracted and added into the
 * block's accumulator.  Returns nonzero when out of memory. */
static int orc_block_of_c(const orc_blk_job* J, int64_t blk) {
  const orc_td* t = J->t;
  double* ablk = (double*)malloc(sizeof(double) * 2 * (size_t)J->asz);
  double* bblk = (double*)malloc(sizeof(double) * 2 * (size_t)J->bsz);
  double* part = (double*)malloc(sizeof(double) * 2 * (size_t)J->csz);
  double* acc = (double*)calloc(2 * (size_t)J->csz, sizeof(double));
  int rc = (!ablk || !bblk || !part || !acc) ? ORC_ENOMEM : ORC_OK;
  int64_t cb[2 * ORC_MAX_RANK], pc[ORC_MAX_RANK], orgA[ORC_MAX_RANK], orgB[ORC_MAX_RANK];
  if (!rc) {
    orc_unravel(blk, J->crank, J->cgrid, cb);
    /* Step 1: the free-axis coordinates of this C block fix the A and B
     * block origins on the free axes. */
    for (int32_t j = 0; j < t->nfa; ++j) orgA[t->fa[j]] = cb[j] * J->extA[t->fa[j]];
    for (int32_t j = 0; j < t->nfb; ++j) orgB[t->fb[j]] = cb[t->nfa + j] * J->extB[t->fb[j]];
  }
  for (int64_t p = 0; p < J->npair && !rc; ++p) {
    /* Step 2: pair p matches contracted block coordinates on both sides. */
    orc_unravel(p, J->k, J->pg, pc);
    for (int32_t i = 0; i < J->k; ++i) {
      orgA[J->axA[i]] = pc[i] * J->extA[J->axA[i]];
      orgB[J->axB[i]] = pc[i] * J->extB[J->axB[i]];
    }
    orc_extract(J->Ab, J->rA, J->dA, J->gA, orgA, J->extA, ablk);
    orc_extract(J->Bb, J->rB, J->dB, J->gB, orgB, J->extB, bblk);
    /* Step 3: local contraction of the pair. */
    rc = orc_tensordot(ablk, J->rA, J->extA, bblk, J->rB, J->extB, J->k, J->axA, J->axB, part);
    /* Step 4: add the partial block into the C block. */
    for (int64_t e = 0; e < 2 * J->csz && !rc; ++e) acc[e] += part[e];
  }
  if (!rc) memcpy(J->Cb + 2 * blk * J->csz, acc, sizeof(double) * 2 * (size_t)J->csz);
  free(ablk);
  free(bblk);
  free(part);
  free(acc);
  return rc;
}

int orc_block_tensordot(const double* Ab, int32_t rA, const int64_t* dA, const int32_t* gA,
                        const double* Bb, int32_t rB, const int64_t* dB, const int32_t* gB,
                        int32_t k, const int32_t* axA, const int32_t* axB, double* Cb,
                        int32_t* gC) {
  orc_td t;
  int rc = orc_td_setup(&t, rA, dA, rB, dB, k, axA, axB);
  if (rc) return rc;
  orc_td_free(&t);
  if ((rc = orc_check_grid(rA, dA, gA)) || (rc = orc_check_grid(rB, dB, gB))) return rc;

  /* Refined grids: free axes keep their own counts, contracted pairs use the
   * least common multiple. */
  int64_t rgA[ORC_MAX_RANK], rgB[ORC_MAX_RANK], pg[ORC_MAX_RANK];
  for (int32_t j = 0; j < rA; ++j) rgA[j] = gA[j];
  for (int32_t j = 0; j < rB; ++j) rgB[j] = gB[j];
  for (int32_t i = 0; i < k; ++i) {
    int64_t a = gA[axA[i]], b = gB[axB[i]];
    int64_t l = a / orc_gcd(a, b) * b;
    if (dA[axA[i]] % l != 0) return ORC_EGRID;
    rgA[axA[i]] = rgB[axB[i]] = pg[i] = l;
  }
  int32_t crank = t.crank;
  int64_t cdims[2 * ORC_MAX_RANK], cgrid[2 * ORC_MAX_RANK], cext[2 * ORC_MAX_RANK];
  int32_t cg32[2 * ORC_MAX_RANK];
  for (int32_t j = 0; j < t.nfa; ++j) {
    cdims[j] = dA[t.fa[j]];
    cgrid[j] = gA[t.fa[j]];
  }
  for (int32_t j = 0; j < t.nfb; ++j) {
    cdims[t.nfa + j] = dB[t.fb[j]];
    cgrid[t.nfa + j] = gB[t.fb[j]];
  }
  for (int32_t j = 0; j < crank; ++j) {
    cext[j] = cdims[j] / cgrid[j];
    cg32[j] = (int32_t)cgrid[j];
    if (gC) gC[j] = cg32[j];
  }
  int64_t extA[ORC_MAX_RANK], extB[ORC_MAX_RANK];
  for (int32_t j = 0; j < rA; ++j) extA[j] = dA[j] / rgA[j];
  for (int32_t j = 0; j < rB; ++j) extB[j] = dB[j] / rgB[j];

  orc_blk_job J;
  J.t = &t;
  J.Ab = Ab;
  J.Bb = Bb;
  J.Cb = Cb;
  J.rA = rA;
  J.rB = rB;
  J.k = k;
  J.dA = dA;
  J.dB = dB;
  J.gA = gA;
  J.gB = gB;
  J.axA = axA;
  J.axB = axB;
  J.crank = crank;
  J.cgrid = cgrid;
  J.pg = pg;
  J.extA = extA;
  J.extB = extB;
  J.csz = orc_numel(crank, cext);
  J.npair = orc_numel(k, pg);
  J.asz = orc_numel(rA, extA);
  J.bsz = orc_numel(rB, extB);
  int64_t nCblk = orc_numel(crank, cgrid);
  /* C blocks are independent: each is summed on its own, in the same order,
   * whether the blocks run one after another or (built with ORC_OPENMP, the
   * CPU-baseline build) on several threads. */
#ifdef ORC_OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(max : rc)
#endif
  for (int64_t blk = 0; blk < nCblk; ++blk) {
    int r = orc_block_of_c(&J, blk);
    if (r > rc) rc = r;
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* State-vector simulation (Section II.A: the state as a 2^n tensor).         */
/* Qubit 0 is the most significant bit of the basis index.  A two-qubit gate  */
/* on (a, b) has matrix index 2*bit_a + bit_b.  Gate matrices are row-major,  */
/* complex interleaved, packed one after another.                             */
/* ------------------------------------------------------------------------ */
int orc_statevector(int32_t n, int32_t ngates, const int32_t* nq, const int32_t* qubits,
                    const double* mats, double* psi) {
  if (n < 1 || n > 30) return ORC_EINVAL;
  int64_t dim = (int64_t)1 << n;
  memset(psi, 0, sizeof(double) * 2 * (size_t)dim);
  psi[0] = 1.0;
  const int32_t* q = qubits;
  const double* m = mats;
  for (int32_t g = 0; g < ngates; ++g) {
    if (nq[g] == 1) {
      if (q[0] < 0 || q[0] >= n) return ORC_EINVAL;
      int64_t bit = (int64_t)1 << (n - 1 - q[0]);
      for (int64_t i = 0; i < dim; ++i) {
        if (i & bit) continue;
        double v[4] = {psi[2 * i], psi[2 * i + 1], psi[2 * (i | bit)], psi[2 * (i | bit) + 1]};
        for (int r = 0; r < 2; ++r) {
          double re = 0.0, im = 0.0;
          for (int c = 0; c < 2; ++c) {
            double mr = m[2 * (2 * r + c)], mi = m[2 * (2 * r + c) + 1];
            re += mr * v[2 * c] - mi * v[2 * c + 1];
            im += mr * v[2 * c + 1] + mi * v[2 * c];
          }
          int64_t dst = r ? (i | bit) : i;
          psi[2 * dst] = re;
          psi[2 * dst + 1] = im;
        }
      }
      q += 1;
      m += 8;
    } else if (nq[g] == 2) {
      if (q[0] < 0 || q[0] >= n || q[1] < 0 || q[1] >= n || q[0] == q[1]) return ORC_EINVAL;
      int64_t ba = (int64_t)1 << (n - 1 - q[0]), bb = (int64_t)1 << (n - 1 - q[1]);
      for (int64_t i = 0; i < dim; ++i) {
        if ((i & ba) || (i & bb)) continue;
        int64_t ix[4] = {i, i | bb, i | ba, i | ba | bb}; /* index 2*a + b */
        double v[8];
        for (int c = 0; c < 4; ++c) {
          v[2 * c] = psi[2 * ix[c]];
          v[2 * c + 1] = psi[2 * ix[c] + 1];
        }
        for (int r = 0; r < 4; ++r) {
          double re = 0.0, im = 0.0;
          for (int c = 0; c < 4; ++c) {
            double mr = m[2 * (4 * r + c)], mi = m[2 * (4 * r + c) + 1];
            re += mr * v[2 * c] - mi * v[2 * c + 1];
            im += mr * v[2 * c + 1] + mi * v[2 * c];
          }
          psi[2 * ix[r]] = re;
          psi[2 * ix[r] + 1] = im;
        }
      }
      q += 2;
      m += 32;
    } else {
      return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

/* Sum of squared magnitudes in FP64, ascending order. */
double orc_norm2(const double* x, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[2 * i] * x[2 * i] + x[2 * i + 1] * x[2 * i + 1];
  return s;
}

/* ------------------------------------------------------------------------ */
/* Sliced tensor-network contraction (Sections II.A and II.B).                */
/*                                                                            */
/* Tensors carry integer bond labels; every dim is 2.  path holds nsteps     */
/* pairs in single-static-assignment form (ids >= nt are step results).  A    */
/* label carried by both operands of a step is summed over, in the order the  */
/* labels appear on the first operand.  The result lists the first operand's  */
/* surviving labels, then the second's.                                       */
/*                                                                            */
/* Slicing: each sliced label is projected onto each basis value; slice s     */
/* fixes sliced[i] to bit (nsliced-1-i) of s (the first sliced label is the   */
/* most significant).  The copies are contracted independently and their      */
/* results summed in FP64 in ascending s, which recovers the unsliced result. */
/* out receives the summed final tensor (out_cap doubles available), with its */
/* rank and labels.  orc_contract_network_range sums only the slices          */
/* s_begin <= s < s_end (one projection of Section II.B when s_end =          */
/* s_begin + 1); orc_contract_network sums all of them.                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  double* data;
  int32_t rank;
  int32_t labels[ORC_MAX_RANK];
} orc_nt;

static int orc_project(const double* src, int32_t rank, const int32_t* labels,
                       int32_t nsliced, const int32_t* sliced, int64_t s, orc_nt* dst) {
  int32_t fixed[ORC_MAX_RANK];
  int32_t nk = 0;
  for (int32_t j = 0; j < rank; ++j) {
    fixed[j] = -1;
    for (int32_t i = 0; i < nsliced; ++i)
      if (labels[j] == sliced[i]) fixed[j] = (int32_t)((s >> (nsliced - 1 - i)) & 1);
    if (fixed[j] < 0) dst->labels[nk++] = labels[j];
  }
  dst->rank = nk;
  int64_t n = (int64_t)1 << nk;
  dst->data = (double*)malloc(sizeof(double) * 2 * (size_t)n);
  if (!dst->data) return ORC_ENOMEM;
  for (int64_t o = 0; o < n; ++o) {
    int64_t srcoff = 0;
    int32_t kk = 0;
    for (int32_t j = 0; j < rank; ++j) {
      int64_t bit;
      if (fixed[j] >= 0)
        bit = fixed[j];
      else
        bit = (o >> (nk - 1 - kk++)) & 1;
      srcoff = srcoff * 2 + bit;
    }
    dst->data[2 * o] = src[2 * srcoff];
    dst->data[2 * o + 1] = src[2 * srcoff + 1];
  }
  return ORC_OK;
}

static int orc_step(const orc_nt* a, const orc_nt* b, orc_nt* c) {
  int32_t axA[ORC_MAX_RANK], axB[ORC_MAX_RANK], k = 0;
  for (int32_t i = 0; i < a->rank; ++i)
    for (int32_t j = 0; j < b->rank; ++j)
      if (a->labels[i] == b->labels[j]) {
        axA[k] = i;
        axB[k] = j;
        ++k;
      }
  int32_t crank = a->rank + b->rank - 2 * k;
  if (crank > ORC_MAX_RANK || crank > 40) return ORC_EINVAL;
  int64_t dA[ORC_MAX_RANK], dB[ORC_MAX_RANK];
  for (int32_t j = 0; j < a->rank; ++j) dA[j] = 2;
  for (int32_t j = 0; j < b->rank; ++j) dB[j] = 2;
  c->rank = crank;
  int32_t n = 0;
  for (int32_t i = 0; i < a->rank; ++i) {
    int shared = 0;
    for (int32_t j = 0; j < k; ++j) shared |= (axA[j] == i);
    if (!shared) c->labels[n++] = a->labels[i];
  }
  for (int32_t i = 0; i < b->rank; ++i) {
    int shared = 0;
    for (int32_t j = 0; j < k; ++j) shared |= (axB[j] == i);
    if (!shared) c->labels[n++] = b->labels[i];
  }
  c->data = (double*)malloc(sizeof(double) * 2 * ((size_t)1 << crank));
  if (!c->data) return ORC_ENOMEM;
  return orc_tensordot(a->data, a->rank, dA, b->data, b->rank, dB, k, axA, axB, c->data);
}

int orc_contract_network_range(int32_t nt, const int32_t* ranks, const int32_t* labels,
                               const double* data, int32_t nsteps, const int32_t* path,
                               int32_t nsliced, const int32_t* sliced, int64_t s_begin,
                               int64_t s_end, double* out, int64_t out_cap,
                               int32_t* out_rank, int32_t* out_labels) {
  if (nt < 1 || nsteps != nt - 1 || nsliced < 0 || nsliced > 30) return ORC_EINVAL;
  if (s_begin < 0 || s_end <= s_begin || s_end > ((int64_t)1 << nsliced)) return ORC_EINVAL;
  int32_t ntot = nt + nsteps;
  int64_t* doff = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt);
  int64_t* loff = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt);
  orc_nt* T = (orc_nt*)calloc((size_t)ntot, sizeof(orc_nt));
  if (!doff || !loff || !T) {
    free(doff);
    free(loff);
    free(T);
    return ORC_ENOMEM;
  }
  int64_t d = 0, l = 0;
  for (int32_t i = 0; i < nt; ++i) {
    if (ranks[i] < 0 || ranks[i] > 40) {
      free(doff);
      free(loff);
      free(T);
      return ORC_EINVAL;
    }
    doff[i] = d;
    loff[i] = l;
    d += (int64_t)1 << ranks[i];
    l += ranks[i];
  }
  int rc = ORC_OK;
  int first = 1;
  for (int64_t s = s_begin; s < s_end && !rc; ++s) {
    for (int32_t i = 0; i < nt && !rc; ++i)
      rc = orc_project(data + 2 * doff[i], ranks[i], labels + loff[i], nsliced, sliced, s,
                       &T[i]);
    for (int32_t st = 0; st < nsteps && !rc; ++st) {
      int32_t a = path[2 * st], b = path[2 * st + 1];
      if (a < 0 || b < 0 || a >= nt + st || b >= nt + st || a == b || !T[a].data ||
          !T[b].data) {
        rc = ORC_EINVAL;
        break;
      }
      rc = orc_step(&T[a], &T[b], &T[nt + st]);
      free(T[a].data);
      free(T[b].data);
      T[a].data = T[b].data = NULL;
    }
    if (!rc) {
      orc_nt* f = &T[ntot - 1];
      int64_t n = (int64_t)1 << f->rank;
      if (2 * n > out_cap) {
        rc = ORC_EINVAL;
      } else if (first) {
        *out_rank = f->rank;
        for (int32_t j = 0; j < f->rank; ++j) out_labels[j] = f->labels[j];
        memset(out, 0, sizeof(double) * 2 * (size_t)n);
        first = 0;
      } else if (f->rank != *out_rank) {
        rc = ORC_EINVAL;
      }
      if (!rc)
        for (int64_t e = 0; e < 2 * n; ++e) out[e] += f->data[e];
    }
    for (int32_t i = 0; i < ntot; ++i) {
      free(T[i].data);
      T[i].data = NULL;
    }
  }
  free(doff);
  free(loff);
  free(T);
  return rc;
}

int orc_contract_network(int32_t nt, const int32_t* ranks, const int32_t* labels,
                         const double* data, int32_t nsteps, const int32_t* path,
                         int32_t nsliced, const int32_t* sliced, double* out, int64_t out_cap,
                         int32_t* out_rank, int32_t* out_labels) {
  if (nsliced < 0 || nsliced > 30) return ORC_EINVAL;
  return orc_contract_network_range(nt, ranks, labels, data, nsteps, path, nsliced, sliced, 0,
                                    (int64_t)1 << nsliced, out, out_cap, out_rank, out_labels);
}
