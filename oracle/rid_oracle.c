/*
 * rid_oracle.c -- plain, slow CPU reference for the randomized LUPP
 * interpolative decomposition (Pearce, Chen, Dong, Martinsson, "Adaptive
 * parallelizable algorithms for interpolative decompositions via partially
 * pivoted LU", arXiv 2310.09417).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this file;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header or constant table with the GPU path.
 *
 * Arithmetic: IEEE double, every sum taken in ascending index order, built
 * with -ffp-contract=off so that no multiply-add is fused.  OpenMP is used only
 * across independent outputs (columns of a sketch, candidates of the final
 * solve), so every result is independent of the thread count.
 *
 * Column form throughout: A is m x n (row-major, leading dimension lda), the
 * sketch is Y = Omega * A (l x n), LU with partial pivoting runs on Y^T
 * (n x l) and selects columns of A.  The paper writes the row form
 * (Y = A * Omega, LUPP on Y); the column form is the same algorithm applied to
 * A^T (paper, Sec. 4, last sentence before Sec. 4.1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the OpenMP loops below use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the OpenMP loops from here on (n < 1: the runtime's default);
 * results do not depend on it (only independent outputs are split). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

/* Status codes (same numbering as the library's public header: an interface
 * both sides must agree on, restated here rather than shared). */
enum {
  ORC_OK = 0,
  ORC_NOT_CONVERGED = 1,
  ORC_RANK_DEFICIENT = 2,
  ORC_ERR_ARG = -1,
  ORC_ERR_NONFINITE = -2
};

/* ------------------------------------------------------------------------ */
/* Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 4.2).          */
/* One round maps (c0,c1,c2,c3) with key (k0,k1) to                          */
/*   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));       */
/* the key is advanced by the Weyl constants (W0,W1) between rounds.         */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Gaussian embedding entries (paper Sec. 3.2 and Alg. 1: independent        */
/* Gaussian blocks Omega^(t)).  Entry omega(c, i) of sketch vector c at row  */
/* i is a pure function of (seed, c, i):                                     */
/*   counter = (floor(i/4), c, 0, 0), key = (seed low 32, seed high 32),     */
/*   u_a = (x_a + 1/2) * 2^-32 in (0,1) for the four output words x_a,       */
/*   Box-Muller on (u0,u1) gives rows 4q, 4q+1 and on (u2,u3) rows 4q+2,     */
/*   4q+3:  sqrt(-2 ln u) * (cos 2 pi v, sin 2 pi v).                        */
/* Sketch vectors are numbered globally: block t of width b holds vectors    */
/* t*b .. t*b+b-1, so every block is independent of every other.            */
/* ------------------------------------------------------------------------ */
static void omega_quad(uint64_t seed, uint32_t q, uint32_t c, double w[4]) {
  uint32_t ctr[4] = {q, c, 0u, 0u};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  const double two_pi = 6.283185307179586476925286766559;
  double u[4];
  for (int a = 0; a < 4; ++a) u[a] = ((double)x[a] + 0.5) * 0x1p-32;
  double r0 = sqrt(-2.0 * log(u[0]));
  double r1 = sqrt(-2.0 * log(u[2]));
  w[0] = r0 * cos(two_pi * u[1]);
  w[1] = r0 * sin(two_pi * u[1]);
  w[2] = r1 * cos(two_pi * u[3]);
  w[3] = r1 * sin(two_pi * u[3]);
}

/* Omega block: out[c * m + i] = omega(c0 + c, i), c < w, i < m. */
void orc_omega(uint64_t seed, int64_t c0, int64_t w, int64_t m, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < w; ++c) {
    for (int64_t i = 0; i < m; i += 4) {
      double v[4];
      omega_quad(seed, (uint32_t)(i / 4), (uint32_t)(c0 + c), v);
      for (int a = 0; a < 4 && i + a < m; ++a) out[c * m + i + a] = v[a];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Rounding into a narrower binary floating-point format: p significand bits */
/* (the implicit one included), smallest normal exponent emin, largest      */
/* finite magnitude xmax.  Round to nearest, ties to the even significand;  */
/* magnitudes beyond xmax saturate.  Subnormals keep the spacing of the     */
/* smallest binade.                                                         */
/*   fmt 1: bfloat16       p = 8, emin = -126, xmax = (2 - 2^-7) 2^127       */
/*   fmt 2: OCP FP8 e4m3   p = 4, emin = -6,   xmax = 448                    */
/* fmt 0 returns x unchanged.                                               */
/* ------------------------------------------------------------------------ */
double orc_round_format(double x, int fmt) {
  int p, emin;
  double xmax;
  if (fmt == 1) {
    p = 8;
    emin = -126;
    xmax = ldexp(2.0 - ldexp(1.0, -7), 127);
  } else if (fmt == 2) {
    p = 4;
    emin = -6;
    xmax = 448.0;
  } else {
    return x;
  }
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  (void)frexp(x, &e); /* |x| = f 2^e, f in [0.5, 1): leading bit at 2^(e-1) */
  int lead = e - 1;
  if (lead < emin) lead = emin;
  const double q = ldexp(1.0, lead - (p - 1)); /* spacing of the binade */
  double r = nearbyint(x / q) * q;             /* x / q is exact; ties to even */
  if (fabs(r) > xmax) r = copysign(xmax, x);
  return r;
}

/* The same rounding applied to each of n values (out may alias x). */
void orc_round_format_array(const double* x, int64_t n, int fmt, double* out) {
  for (int64_t t = 0; t < n; ++t) out[t] = orc_round_format(x[t], fmt);
}

/* Omega block rounded into format fmt: out[c * m + i] = round(omega(c0+c, i)). */
void orc_omega_format(uint64_t seed, int64_t c0, int64_t w, int64_t m, int fmt, double* out) {
  orc_omega(seed, c0, w, m, out);
  for (int64_t t = 0; t < w * m; ++t) out[t] = orc_round_format(out[t], fmt);
}

/* Sketch (paper Sec. 2.4): Y(c, j) = sum_{i=0}^{m-1} omega(c0+c, i) * A(i, j),
 * summed in ascending i, with the entries of Omega first rounded into format
 * fmt (0: kept in double).  Y is w x n row-major with leading dimension ldy.
 * Each output column strip is owned by one thread. */
void orc_sketch_format(const double* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                       int64_t c0, int64_t w, int fmt, double* Y, int64_t ldy) {
  double* om = (double*)malloc(sizeof(double) * (size_t)(w > 0 ? w : 1) * (size_t)(m > 0 ? m : 1));
  orc_omega_format(seed, c0, w, m, fmt, om);
  const int64_t strip = 256;
  int64_t nstrips = (n + strip - 1) / strip;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t sidx = 0; sidx < nstrips; ++sidx) {
    int64_t j0 = sidx * strip, j1 = j0 + strip < n ? j0 + strip : n;
    for (int64_t c = 0; c < w; ++c)
      for (int64_t j = j0; j < j1; ++j) Y[c * ldy + j] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      const double* a = A + i * lda;
      for (int64_t c = 0; c < w; ++c) {
        double o = om[c * m + i];
        double* y = Y + c * ldy;
        for (int64_t j = j0; j < j1; ++j) y[j] = y[j] + o * a[j];
      }
    }
  }
  free(om);
}

/* Sketch with the Gaussian entries kept in double. */
void orc_sketch(const double* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                int64_t c0, int64_t w, double* Y, int64_t ldy) {
  orc_sketch_format(A, m, n, lda, seed, c0, w, 0, Y, ldy);
}

/* ------------------------------------------------------------------------ */
/* Sparse sign embedding (paper Sec. 5, random matrix distributions: each    */
/* row of the embedding carries zeta independent Rademacher entries at       */
/* uniformly random coordinates; zeta = 8), column form: in the block of w   */
/* sketch vectors starting at global index c0, column i (row i of A) has     */
/* zw = min(8, w) nonzeros.  Their rows are a uniformly random zw-subset of  */
/* the w, drawn by Floyd's algorithm: for q = 0..zw-1, j = w - zw + q,       */
/* t = floor(u_q (j+1) / 2^32); take t unless already taken, else j.  The    */
/* words u_0..u_7 are Philox4x32-10 with key (seed lo, seed hi) at counters  */
/* (i, c0, SS_TAG, 0) and (i, c0, SS_TAG, 1); the sign of the q-th chosen    */
/* row is bit q of the first word at (i, c0, SS_TAG, 2) (1 = negative).      */
/* Values +-sqrt(w / zw), so that E[Omega^T Omega] = w I as for the unit     */
/* Gaussian (the estimate E = ||S||_F / sqrt(w) stays unbiased).             */
/* ------------------------------------------------------------------------ */
#define ORC_SS_TAG 0x53534e31u /* distinct from the Gaussian stream's zero word */
#define ORC_SS_ZETA 8

static void ss_column(uint64_t seed, uint32_t i, uint32_t c0, int64_t w, int64_t* rows,
                      int* neg, int64_t* zw_out) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t u[8], sg[4];
  const uint32_t c_a[4] = {i, c0, ORC_SS_TAG, 0}, c_b[4] = {i, c0, ORC_SS_TAG, 1},
                 c_s[4] = {i, c0, ORC_SS_TAG, 2};
  orc_philox4x32_10(c_a, key, u);
  orc_philox4x32_10(c_b, key, u + 4);
  orc_philox4x32_10(c_s, key, sg);
  const int64_t zw = w < ORC_SS_ZETA ? w : ORC_SS_ZETA;
  for (int64_t q = 0; q < zw; ++q) {
    const int64_t j = w - zw + q;
    const int64_t t = (int64_t)(((uint64_t)u[q] * (uint64_t)(j + 1)) >> 32);
    int taken = 0;
    for (int64_t r = 0; r < q; ++r)
      if (rows[r] == t) taken = 1;
    rows[q] = taken ? j : t;
    neg[q] = (int)((sg[0] >> q) & 1u);
  }
  *zw_out = zw;
}

/* Sparse sign block: out[c * m + i] = Omega(c0 + c, i) for c < w, i < m. */
void orc_omega_sparse(uint64_t seed, int64_t c0, int64_t w, int64_t m, double* out) {
  for (int64_t t = 0; t < w * m; ++t) out[t] = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    int64_t rows[ORC_SS_ZETA], zw;
    int neg[ORC_SS_ZETA];
    ss_column(seed, (uint32_t)i, (uint32_t)c0, w, rows, neg, &zw);
    const double v = sqrt((double)w / (double)zw);
    for (int64_t q = 0; q < zw; ++q) out[rows[q] * m + i] = neg[q] ? -v : v;
  }
}

/* Sketch with the sparse sign block: Y(c, j) = sum_i Omega(c0+c, i) A(i, j). */
void orc_sketch_sparse(const double* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                       int64_t c0, int64_t w, double* Y, int64_t ldy) {
  double* om = (double*)malloc(sizeof(double) * (size_t)w * (size_t)m);
  orc_omega_sparse(seed, c0, w, m, om);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t c = 0; c < w; ++c) {
      double acc = 0.0;
      for (int64_t i = 0; i < m; ++i) acc = acc + om[c * m + i] * A[i * lda + j];
      Y[c * ldy + j] = acc;
    }
  free(om);
}

/* Sketch of a block in the chosen embedding (0 Gaussian, 1 sparse sign). */
static void sketch_emb(int embedding, const double* A, int64_t m, int64_t n, int64_t lda,
                       uint64_t seed, int64_t c0, int64_t w, double* Y, int64_t ldy) {
  if (embedding == 1)
    orc_sketch_sparse(A, m, n, lda, seed, c0, w, Y, ldy);
  else
    orc_sketch(A, m, n, lda, seed, c0, w, Y, ldy);
}

/* Sum of squares of A in ascending (row, column) order. */
static double frob2(const double* A, int64_t m, int64_t n, int64_t lda, int* nonfinite) {
  double s = 0.0;
  *nonfinite = 0;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double v = A[i * lda + j];
      if (!isfinite(v)) *nonfinite = 1;
      s = s + v * v;
    }
  return s;
}

/* Result record returned to the caller. */
typedef struct {
  int64_t k;          /* rank of the returned ID (= number of skeletons)         */
  double err_est;     /* Schur-complement estimate E for that rank (-1 if none)  */
  int32_t status;     /* ORC_* code                                              */
  int32_t nsteps;     /* number of estimates taken (length of the E history)    */
  double min_gap;     /* min over pivot steps of (|1st| - |2nd|) / |1st|        */
  int64_t min_gap_step;
  double fro_a;       /* ||A||_F                                                 */
  int64_t robust_k;   /* leading pivots decided by more than the rounding floor: */
                      /* (|1st| - |2nd|) > 64 eps sqrt(s+1) max|Y| at every step */
                      /* s < robust_k, eps = 2^-52 (128 units of roundoff)       */
                      /* s < robust_k; later ones may legitimately differ in     */
                      /* any other correct evaluation order                      */
} orc_result;

/*
 * Blocked LUPP interpolative decomposition on the sketch (paper Alg. 1 and
 * Sec. 4.2), column form.
 *
 *   mode 0 (fixed rank, randLUPP): one block of k sketch vectors is factored
 *     (k pivots), then one block of p vectors is drawn only to estimate the
 *     error of that rank-k ID (Sec. 3.2, E_Schur on an independent sample).
 *   mode 1 (adaptive, randLUPPadap): the first block of b vectors is always
 *     factored; each later block of b vectors is first reduced by the current
 *     factorization (U2 = L1^{-1} (P Y)(top), S = (P Y)(bottom) - L2 U2), its
 *     Frobenius norm gives the estimate, and only if that misses the
 *     tolerance is S factored and appended.
 *
 * Z (n x zc) holds P * [Y^(0) ... Y^(t)]^T with its LU factors in place:
 * row r is candidate column perm[r]; for r < k the row holds U (columns
 * >= r) and L1 (columns < r); for r >= k columns < k hold L2.
 *
 * Estimate scaling: Omega has unit variance, so E = ||S||_F / sqrt(w) is the
 * unbiased estimate of the residual norm (E||X w||^2 = ||X||_F^2 per unit
 * vector w).
 *
 * Outputs: J[0..k) pivot order (original column indices); T (k x (n-k),
 * row-major, ldt) with column q belonging to the q-th non-skeleton column in
 * ascending index; E history (up to hist_cap entries).
 */
static int rid_lupp_impl(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                         int64_t k_or_b, int64_t p, double tol, int tol_relative, int64_t kmax,
                         int64_t first_width, uint64_t seed, int estimator, int64_t resid_p,
                         int embedding, int64_t* J, double* T, int64_t ldt, double* E_hist,
                         double* est_hist, int64_t hist_cap, double* gap_hist,
                         const int64_t* force_J, int64_t force_len, double* force_short,
                         orc_result* res);

int orc_rid_lupp(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                 int64_t k_or_b, int64_t p, double tol, int tol_relative, int64_t kmax,
                 uint64_t seed, int64_t* J, double* T, int64_t ldt, double* E_hist,
                 int64_t hist_cap, orc_result* res) {
  return rid_lupp_impl(A, m, n, lda, mode, k_or_b, p, tol, tol_relative, kmax, 0, seed, 0, 0, 0,
                       J, T, ldt, E_hist, NULL, hist_cap, NULL, NULL, 0, NULL, res);
}

/* Same as orc_rid_lupp with the blocks drawn from the sparse sign embedding
 * (embedding 1) instead of the Gaussian one (0). */
int orc_rid_lupp_emb(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                     int64_t k_or_b, int64_t p, double tol, int tol_relative, int64_t kmax,
                     uint64_t seed, int embedding, int64_t* J, double* T, int64_t ldt,
                     double* E_hist, int64_t hist_cap, orc_result* res) {
  return rid_lupp_impl(A, m, n, lda, mode, k_or_b, p, tol, tol_relative, kmax, 0, seed, 0, 0,
                       embedding, J, T, ldt, E_hist, NULL, hist_cap, NULL, NULL, 0, NULL, res);
}

/* Same as orc_rid_lupp with the stopping estimate taken from the residual
 * triangle of Remark 1 (estimator 1: Schur estimate on the set-aside sample,
 * 2: eq. normUest, 3: eq. maxUest; see resid_triangle below).  Adaptive mode:
 * resid_p vectors are set aside once (stream indices ORC_RESID_C0 + j) and the
 * estimate of the current rank is taken after every factored block, so no
 * block is drawn only to be measured.  Fixed-rank mode: the p oversampling
 * vectors are the sample.  est_hist receives the three estimates of every
 * step (3 entries per step).  embedding: 0 Gaussian, 1 sparse sign (the
 * sample is drawn from the same embedding). */
int orc_rid_lupp_est(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                     int64_t k_or_b, int64_t p, int estimator, int64_t resid_p, double tol,
                     int tol_relative, int64_t kmax, uint64_t seed, int embedding, int64_t* J,
                     double* T, int64_t ldt, double* E_hist, double* est_hist, int64_t hist_cap,
                     orc_result* res) {
  return rid_lupp_impl(A, m, n, lda, mode, k_or_b, p, tol, tol_relative, kmax, 0, seed, estimator,
                       resid_p, embedding, J, T, ldt, E_hist, est_hist, hist_cap, NULL, NULL, 0,
                       NULL, res);
}

/* Adaptive variant whose first factored block has first_width vectors
 * (instead of b), e.g. a rank predicted beforehand; the blocks after it have b
 * vectors and the stopping rule is unchanged. */
int orc_rid_adaptive_first(const double* A, int64_t m, int64_t n, int64_t lda, int64_t b,
                           int64_t first_width, double tol, int tol_relative, int64_t kmax,
                           uint64_t seed, int64_t* J, double* T, int64_t ldt, double* E_hist,
                           int64_t hist_cap, orc_result* res) {
  return rid_lupp_impl(A, m, n, lda, 1, b, 0, tol, tol_relative, kmax, first_width, seed, 0, 0, 0,
                       J, T, ldt, E_hist, NULL, hist_cap, NULL, NULL, 0, NULL, res);
}

/* Same as orc_rid_lupp, also reporting every pivot step's decision margin:
 * gap_hist[s] = (|best| - |runner-up|) / (sqrt(s + 1) max|Y|) for s < k (+inf
 * when step s had a single candidate).  A step is decided above the rounding
 * floor of a precision with machine epsilon eps when gap_hist[s] > 64 eps
 * (robust_k is that count for eps = 2^-52); test diagnostics only. */
int orc_rid_lupp_gaps(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                      int64_t k_or_b, int64_t p, double tol, int tol_relative, int64_t kmax,
                      uint64_t seed, int64_t* J, double* T, int64_t ldt, double* E_hist,
                      int64_t hist_cap, double* gap_hist, orc_result* res) {
  return rid_lupp_impl(A, m, n, lda, mode, k_or_b, p, tol, tol_relative, kmax, 0, seed, 0, 0, 0,
                       J, T, ldt, E_hist, NULL, hist_cap, gap_hist, NULL, 0, NULL, res);
}

/* Same as orc_rid_lupp_gaps with the first force_len pivots given: step s
 * takes candidate column force_J[s] (which must not be pivoted yet) instead of
 * the largest one, and force_short[s] = (|largest| - |forced|) / (sqrt(s + 1)
 * max|Y|) is its shortfall on the scale of gap_hist (0 when the forced pivot
 * is a largest one).  The rest of the method is unchanged.  Test diagnostics:
 * it replays another implementation's pivot order, so that each of its
 * decisions can be measured against the rounding floor and its T and E
 * compared with the oracle's for the same skeletons. */
int orc_rid_lupp_forced(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                        int64_t k_or_b, int64_t p, double tol, int tol_relative, int64_t kmax,
                        uint64_t seed, const int64_t* force_J, int64_t force_len, int64_t* J,
                        double* T, int64_t ldt, double* E_hist, int64_t hist_cap,
                        double* gap_hist, double* force_short, orc_result* res) {
  return rid_lupp_impl(A, m, n, lda, mode, k_or_b, p, tol, tol_relative, kmax, 0, seed, 0, 0, 0,
                       J, T, ldt, E_hist, NULL, hist_cap, gap_hist, force_J, force_len,
                       force_short, res);
}

/* ------------------------------------------------------------------------ */
/* Residual triangle (paper Sec. 3.2, Remark 1), column form.                */
/* Z (n x zc) holds the LU factors of the permuted sketch in its first k    */
/* columns (rows in the order perm); Yr (p x n, row c = sample vector c) is  */
/* an independent Gaussian sample.  With P the current row permutation,     */
/*   U2_r = L1^{-1} (P Yr^T)(0:k)      (forward substitution, ascending)     */
/*   S_r  = (P Yr^T)(k:n) - L2 U2_r    (ascending s)                         */
/* and S_r is factored by LU with partial pivoting (ties to the lowest       */
/* original column index; an exactly zero pivot column ends it, the rows of  */
/* U_r not reached stay zero), so that P[Y Yr]^T = [L1 0; L2 L_r] [U1 U2;   */
/* 0 U_r].  Estimates (nr = n - k candidates left):                          */
/*   est[0] = ||S_r||_F / sqrt(p)            (Schur estimate on the sample)  */
/*   est[1] = gamma(k) sqrt(nr) ||U_r||_F     (eq. normUest)                 */
/*   est[2] = gamma(k) sqrt(nr) max |U_r|     (eq. maxUest)                  */
/* gamma(k) = 1 / max(1, k / (4 ln k)), gamma(1) = 1: the reciprocal of the  */
/* asymptotic growth-factor bound k / (4 log k) of LU on Haar matrices,     */
/* never above one because a growth factor is at least one.                 */
/* Ur (p x p, row-major, may be NULL) receives U_r.                          */
/* ------------------------------------------------------------------------ */
#define ORC_RESID_C0 2147483648LL /* stream index of the first set-aside vector */

double orc_growth_scale(int64_t k) {
  if (k < 2) return 1.0;
  const double g = (double)k / (4.0 * log((double)k));
  return g > 1.0 ? 1.0 / g : 1.0;
}

static void resid_triangle(const double* Z, int64_t zc, const int64_t* perm, int64_t n, int64_t k,
                           const double* Yr, int64_t p, double est[3], double* Ur) {
  const int64_t nr = n - k;
  double* W = (double*)malloc(sizeof(double) * (size_t)n * (size_t)p);
  int64_t* oi = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
  for (int64_t r = 0; r < n; ++r)
    for (int64_t q = 0; q < p; ++q) W[r * p + q] = Yr[q * n + perm[r]];
  for (int64_t r = 0; r < k; ++r)
    for (int64_t q = 0; q < p; ++q) {
      double acc = W[r * p + q];
      for (int64_t s = 0; s < r; ++s) acc = acc - Z[r * zc + s] * W[s * p + q];
      W[r * p + q] = acc;
    }
  for (int64_t r = k; r < n; ++r)
    for (int64_t q = 0; q < p; ++q) {
      double acc = W[r * p + q];
      for (int64_t s = 0; s < k; ++s) acc = acc - Z[r * zc + s] * W[s * p + q];
      W[r * p + q] = acc;
    }
  double s2 = 0.0;
  for (int64_t r = k; r < n; ++r)
    for (int64_t q = 0; q < p; ++q) s2 = s2 + W[r * p + q] * W[r * p + q];
  est[0] = sqrt(s2) / sqrt((double)p);
  /* LU with partial pivoting on S_r = W(k:n, :) */
  double* S = W + k * p;
  for (int64_t r = 0; r < nr; ++r) oi[r] = perm[k + r];
  if (Ur)
    for (int64_t t = 0; t < p * p; ++t) Ur[t] = 0.0;
  double fro2 = 0.0, mx = 0.0;
  const int64_t steps = p < nr ? p : nr;
  for (int64_t j = 0; j < steps; ++j) {
    int64_t piv = j;
    double best = fabs(S[j * p + j]);
    for (int64_t r = j + 1; r < nr; ++r) {
      const double v = fabs(S[r * p + j]);
      if (v > best || (v == best && oi[r] < oi[piv])) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0) break;
    if (piv != j) {
      for (int64_t q = 0; q < p; ++q) {
        const double t = S[j * p + q];
        S[j * p + q] = S[piv * p + q];
        S[piv * p + q] = t;
      }
      const int64_t t = oi[j];
      oi[j] = oi[piv];
      oi[piv] = t;
    }
    for (int64_t q = j; q < p; ++q) {
      const double u = S[j * p + q];
      fro2 = fro2 + u * u;
      if (fabs(u) > mx) mx = fabs(u);
      if (Ur) Ur[j * p + q] = u;
    }
    for (int64_t r = j + 1; r < nr; ++r) {
      const double l = S[r * p + j] / S[j * p + j];
      S[r * p + j] = l;
      for (int64_t q = j + 1; q < p; ++q) S[r * p + q] = S[r * p + q] - l * S[j * p + q];
    }
  }
  const double g = orc_growth_scale(k) * sqrt((double)nr);
  est[1] = g * sqrt(fro2);
  est[2] = g * mx;
  free(W);
  free(oi);
}

/* Residual triangle after k LUPP steps on the first l sketch vectors (for
 * tests): Yr = the p vectors c_r .. c_r + p - 1 of the same stream.  Returns
 * ORC_RANK_DEFICIENT when the k steps meet a zero pivot. */
int orc_resid_triangle(const double* A, int64_t m, int64_t n, int64_t lda, int64_t l, int64_t k,
                       uint64_t seed, int64_t c_r, int64_t p, double est[3], double* Ur,
                       int64_t* perm_out) {
  if (k > l || k > n || p < 1) return ORC_ERR_ARG;
  double* Y = (double*)malloc(sizeof(double) * (size_t)l * (size_t)n);
  double* Yr = (double*)malloc(sizeof(double) * (size_t)p * (size_t)n);
  orc_sketch(A, m, n, lda, seed, 0, l, Y, n);
  orc_sketch(A, m, n, lda, seed, c_r, p, Yr, n);
  double* Z = (double*)malloc(sizeof(double) * (size_t)n * (size_t)l);
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int st = ORC_OK;
  for (int64_t r = 0; r < n; ++r) {
    perm[r] = r;
    for (int64_t q = 0; q < l; ++q) Z[r * l + q] = Y[q * n + r];
  }
  for (int64_t s = 0; s < k && st == ORC_OK; ++s) {
    int64_t piv = s;
    double best = fabs(Z[s * l + s]);
    for (int64_t r = s + 1; r < n; ++r) {
      const double v = fabs(Z[r * l + s]);
      if (v > best || (v == best && perm[r] < perm[piv])) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0) {
      st = ORC_RANK_DEFICIENT;
      break;
    }
    if (piv != s) {
      for (int64_t q = 0; q < l; ++q) {
        const double t = Z[s * l + q];
        Z[s * l + q] = Z[piv * l + q];
        Z[piv * l + q] = t;
      }
      const int64_t t = perm[s];
      perm[s] = perm[piv];
      perm[piv] = t;
    }
    for (int64_t r = s + 1; r < n; ++r) {
      const double lv = Z[r * l + s] / Z[s * l + s];
      Z[r * l + s] = lv;
      for (int64_t q = s + 1; q < l; ++q) Z[r * l + q] = Z[r * l + q] - lv * Z[s * l + q];
    }
  }
  if (st == ORC_OK) resid_triangle(Z, l, perm, n, k, Yr, p, est, Ur);
  if (perm_out)
    for (int64_t r = 0; r < n; ++r) perm_out[r] = perm[r];
  free(Y);
  free(Yr);
  free(Z);
  free(perm);
  return st;
}

/* A-posteriori certificate of an ID (the sketched residual of the returned
 * factorization, after Martinsson and Tropp 2020, cited in Remark 1): with
 * Yc = Omega_c A for the p vectors c0 .. c0 + p - 1 of the stream,
 *   cert = ||Yc(:, J^c) - Yc(:, J) T||_F / sqrt(p),
 * J in any order with T (k x (n-k), row-major, ldt) in that order, column q of
 * T for the q-th non-skeleton column in ascending index.  cert^2 is an
 * unbiased estimate of ||A(:, J^c) - A(:, J) T||_F^2.  Sums: s ascending for
 * each entry, then q ascending within c ascending.  Returns ORC_ERR_ARG when J
 * holds an index out of range or twice. */
int orc_certificate(const double* A, int64_t m, int64_t n, int64_t lda, const int64_t* J,
                    int64_t k, const double* T, int64_t ldt, uint64_t seed, int64_t c0, int64_t p,
                    double* cert) {
  if (k < 0 || k > n || p < 1) return ORC_ERR_ARG;
  char* is_skel = (char*)calloc((size_t)n, 1);
  for (int64_t s = 0; s < k; ++s) {
    if (J[s] < 0 || J[s] >= n || is_skel[J[s]]) {
      free(is_skel);
      return ORC_ERR_ARG;
    }
    is_skel[J[s]] = 1;
  }
  int64_t* rest = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n - k > 0 ? n - k : 1));
  int64_t nr = 0;
  for (int64_t j = 0; j < n; ++j)
    if (!is_skel[j]) rest[nr++] = j;
  double* Yc = (double*)malloc(sizeof(double) * (size_t)p * (size_t)n);
  orc_sketch(A, m, n, lda, seed, c0, p, Yc, n);
  double ss = 0.0;
  for (int64_t c = 0; c < p; ++c)
    for (int64_t q = 0; q < nr; ++q) {
      double acc = 0.0;
      for (int64_t s = 0; s < k; ++s) acc = acc + Yc[c * n + J[s]] * T[s * ldt + q];
      const double r = Yc[c * n + rest[q]] - acc;
      ss = ss + r * r;
    }
  *cert = sqrt(ss / (double)p);
  free(is_skel);
  free(rest);
  free(Yc);
  return ORC_OK;
}

static int rid_lupp_impl(const double* A, int64_t m, int64_t n, int64_t lda, int mode,
                         int64_t k_or_b, int64_t p, double tol, int tol_relative, int64_t kmax,
                         int64_t first_width, uint64_t seed, int estimator, int64_t resid_p,
                         int embedding, int64_t* J, double* T, int64_t ldt, double* E_hist,
                         double* est_hist, int64_t hist_cap, double* gap_hist,
                         const int64_t* force_J, int64_t force_len, double* force_short,
                         orc_result* res) {
  memset(res, 0, sizeof(*res));
  res->err_est = -1.0;
  res->min_gap = INFINITY;
  res->min_gap_step = -1;
  if (m < 1 || n < 1 || lda < n || k_or_b < 1 || p < 0 || (mode != 0 && mode != 1) ||
      estimator < 0 || estimator > 3 || (estimator > 0 && mode == 1 && resid_p < 1)) {
    res->status = ORC_ERR_ARG;
    return ORC_ERR_ARG;
  }
  const int64_t mn = m < n ? m : n;
  int64_t kcap, first_w, later_w;
  if (mode == 0) {
    if (k_or_b > mn) {
      res->status = ORC_ERR_ARG;
      return ORC_ERR_ARG;
    }
    kcap = k_or_b;
    first_w = k_or_b;
    later_w = p;
  } else {
    if (kmax < 1) {
      res->status = ORC_ERR_ARG;
      return ORC_ERR_ARG;
    }
    kcap = kmax < mn ? kmax : mn;
    first_w = first_width > 0 ? first_width : k_or_b;
    if (first_w > kcap) first_w = kcap;
    later_w = k_or_b;
  }

  int nonfinite = 0;
  double fa2 = frob2(A, m, n, lda, &nonfinite);
  res->fro_a = sqrt(fa2);
  if (nonfinite) {
    res->status = ORC_ERR_NONFINITE;
    return ORC_ERR_NONFINITE;
  }
  const double thr = tol_relative ? tol * sqrt(fa2) : tol;

  const int64_t zc = kcap + (later_w > first_w ? later_w : first_w) + 1;
  double* Z = (double*)calloc((size_t)n * (size_t)zc, sizeof(double));
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  double* Ynew = (double*)malloc(sizeof(double) * (size_t)n * (size_t)(zc));
  for (int64_t r = 0; r < n; ++r) perm[r] = r;
  /* Remark 1: the sample set aside for the estimate (adaptive mode) */
  double* Yr = NULL;
  if (estimator > 0 && mode == 1) {
    Yr = (double*)malloc(sizeof(double) * (size_t)resid_p * (size_t)n);
    sketch_emb(embedding, A, m, n, lda, seed, ORC_RESID_C0, resid_p, Yr, n);
  }
  double est[3];

  int64_t k = 0;        /* pivots taken so far */
  int64_t cnext = 0;    /* next unused sketch vector */
  double ymax = 0.0;    /* largest |Y| entry drawn so far (scale of the rounding floor) */
  res->robust_k = -1;
  double E = -1.0;
  int status = ORC_OK;
  int first = 1;

  for (;;) {
    int64_t w = first ? first_w : later_w;
    if (w == 0) break; /* fixed rank with p = 0: no estimate */
    /* Draw the next block and apply the current row permutation (P Y^T). */
    sketch_emb(embedding, A, m, n, lda, seed, cnext, w, Ynew, n);
    cnext += w;
    for (int64_t t = 0; t < w * n; ++t)
      if (fabs(Ynew[t]) > ymax) ymax = fabs(Ynew[t]);
    for (int64_t r = 0; r < n; ++r)
      for (int64_t q = 0; q < w; ++q) Z[r * zc + k + q] = Ynew[q * n + perm[r]];

    if (k > 0) {
      /* U2 = L1^{-1} (P Y)(0:k, new): forward substitution, ascending s. */
      for (int64_t r = 0; r < k; ++r)
        for (int64_t q = 0; q < w; ++q) {
          double acc = Z[r * zc + k + q];
          for (int64_t s = 0; s < r; ++s) acc = acc - Z[r * zc + s] * Z[s * zc + k + q];
          Z[r * zc + k + q] = acc;
        }
      /* S = (P Y)(k:n, new) - L2 * U2, ascending s. */
#pragma omp parallel for schedule(static)
      for (int64_t r = k; r < n; ++r)
        for (int64_t q = 0; q < w; ++q) {
          double acc = Z[r * zc + k + q];
          for (int64_t s = 0; s < k; ++s) acc = acc - Z[r * zc + s] * Z[s * zc + k + q];
          Z[r * zc + k + q] = acc;
        }
    }

    if (!first && estimator > 0 && mode == 0) {
      /* fixed rank: the p oversampling vectors are the sample of Remark 1 */
      resid_triangle(Z, zc, perm, n, k, Ynew, w, est, NULL);
      E = est[estimator - 1];
      if (res->nsteps < hist_cap) {
        if (E_hist) E_hist[res->nsteps] = E;
        if (est_hist)
          for (int e = 0; e < 3; ++e) est_hist[3 * res->nsteps + e] = est[e];
      }
      res->nsteps++;
      break;
    }
    if (!first && estimator == 0) {
      /* E = ||S||_F / sqrt(w), rows k..n-1 in order, columns in order. */
      double s2 = 0.0;
      for (int64_t r = k; r < n; ++r)
        for (int64_t q = 0; q < w; ++q) {
          double v = Z[r * zc + k + q];
          s2 = s2 + v * v;
        }
      E = sqrt(s2) / sqrt((double)w);
      if (res->nsteps < hist_cap && E_hist) E_hist[res->nsteps] = E;
      res->nsteps++;
      if (mode == 0) break;                 /* fixed rank: estimate only */
      if (E <= thr) break;                  /* certified at rank k */
      if (k >= kcap) {                      /* cap reached, tolerance missed */
        status = ORC_NOT_CONVERGED;
        break;
      }
    }

    /* LUPP on the block (paper eq. for the Schur update in Sec. 2.3.2). */
    int64_t f = w < kcap - k ? w : kcap - k;
    int deficient = 0;
    for (int64_t s = k; s < k + f; ++s) {
      /* pivot: largest |Z(r, s)| over r >= s; ties -> lowest original index */
      int64_t piv = s;
      double best = fabs(Z[s * zc + s]);
      for (int64_t r = s + 1; r < n; ++r) {
        double v = fabs(Z[r * zc + s]);
        if (v > best || (v == best && perm[r] < perm[piv])) {
          best = v;
          piv = r;
        }
      }
      /* diagnostic: relative gap between the best and the runner-up */
      double second = -1.0;
      for (int64_t r = s; r < n; ++r)
        if (r != piv) {
          double v = fabs(Z[r * zc + s]);
          if (v > second) second = v;
        }
      if (gap_hist) gap_hist[s] = INFINITY;
      if (best > 0.0 && second >= 0.0) {
        if (gap_hist) gap_hist[s] = (best - second) / (sqrt((double)(s + 1)) * ymax);
        double gap = (best - second) / best;
        if (gap < res->min_gap) {
          res->min_gap = gap;
          res->min_gap_step = s;
        }
        const double floor_s = 64.0 * 0x1p-52 * sqrt((double)(s + 1)) * ymax;
        if (res->robust_k < 0 && best - second <= floor_s) res->robust_k = s;
      }
      if (force_J && s < force_len) {
        /* the step takes the given candidate instead; its shortfall from the
         * largest magnitude, on the scale of gap_hist */
        int64_t fr = -1;
        for (int64_t r = s; r < n; ++r)
          if (perm[r] == force_J[s]) {
            fr = r;
            break;
          }
        if (fr < 0) { /* not a remaining candidate */
          free(Z);
          free(perm);
          free(Ynew);
          free(Yr);
          res->status = ORC_ERR_ARG;
          return ORC_ERR_ARG;
        }
        const double v = fabs(Z[fr * zc + s]);
        if (force_short) force_short[s] = ymax > 0.0 ? (best - v) / (sqrt((double)(s + 1)) * ymax) : 0.0;
        piv = fr;
        best = v;
      }
      if (best == 0.0) {
        deficient = 1;
        k = s;
        break;
      }
      if (piv != s) { /* swap whole rows: this also permutes L2 (re-blocking) */
        for (int64_t q = 0; q < zc; ++q) {
          double tmp = Z[s * zc + q];
          Z[s * zc + q] = Z[piv * zc + q];
          Z[piv * zc + q] = tmp;
        }
        int64_t tp = perm[s];
        perm[s] = perm[piv];
        perm[piv] = tp;
      }
      double d = Z[s * zc + s];
#pragma omp parallel for schedule(static)
      for (int64_t r = s + 1; r < n; ++r) {
        double l = Z[r * zc + s] / d;
        Z[r * zc + s] = l;
        for (int64_t q = s + 1; q < k + w; ++q) Z[r * zc + q] = Z[r * zc + q] - l * Z[s * zc + q];
      }
    }
    if (deficient) {
      status = ORC_RANK_DEFICIENT;
      if (E < 0.0) E = 0.0;
      break;
    }
    k += f;
    first = 0;
    if (mode == 1 && k == mn) { /* every column (or row) used: the ID is exact */
      E = 0.0;
      break;
    }
    if (mode == 0 && p == 0) break;
    if (mode == 1 && estimator > 0) {
      /* Remark 1: estimate the error of the rank-k ID from the residual
       * triangle of the set-aside sample; stop as soon as it passes */
      resid_triangle(Z, zc, perm, n, k, Yr, resid_p, est, NULL);
      E = est[estimator - 1];
      if (res->nsteps < hist_cap) {
        if (E_hist) E_hist[res->nsteps] = E;
        if (est_hist)
          for (int e = 0; e < 3; ++e) est_hist[3 * res->nsteps + e] = est[e];
      }
      res->nsteps++;
      if (E <= thr) break;
      if (k >= kcap) {
        status = ORC_NOT_CONVERGED;
        break;
      }
    }
  }

  /* Outputs: skeletons in pivot order and T = L1^{-T} L2^T (paper eq. for the
   * interpolation matrix in Sec. 3.2; last step of Alg. 1). */
  for (int64_t s = 0; s < k; ++s) J[s] = perm[s];
  int64_t nr = n - k;
  /* rank[r - k] = position of candidate r among the non-skeletons in
   * ascending original index */
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
  {
    char* is_skel = (char*)calloc((size_t)n, 1);
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t s = 0; s < k; ++s) is_skel[perm[s]] = 1;
    int64_t q = 0;
    for (int64_t j = 0; j < n; ++j)
      if (!is_skel[j]) slot[j] = q++;
    for (int64_t r = k; r < n; ++r) order[r - k] = slot[perm[r]];
    free(is_skel);
    free(slot);
  }
  if (T && k > 0) {
#pragma omp parallel for schedule(static)
    for (int64_t r = k; r < n; ++r) {
      double* x = (double*)malloc(sizeof(double) * (size_t)k);
      for (int64_t s = k - 1; s >= 0; --s) {
        double acc = Z[r * zc + s];
        for (int64_t s2 = s + 1; s2 < k; ++s2) acc = acc - Z[s2 * zc + s] * x[s2];
        x[s] = acc;
      }
      int64_t q = order[r - k];
      for (int64_t s = 0; s < k; ++s) T[s * ldt + q] = x[s];
      free(x);
    }
  }
  free(order);
  free(Z);
  free(perm);
  free(Ynew);
  free(Yr);
  res->k = k;
  res->err_est = E;
  res->status = status;
  if (res->robust_k < 0 || res->robust_k > k) res->robust_k = k;
  return status;
}

/*
 * Fixed-rank LU factor dump for tests of the bound |L| <= 1 (paper
 * Sec. 2.3.2): factors Y^T (n x l, built from the first l sketch vectors)
 * with k pivot steps and returns L (n x k, rows in pivot order, unit
 * diagonal) and U (k x l).
 */
int orc_lupp_factors(const double* A, int64_t m, int64_t n, int64_t lda, int64_t l,
                     int64_t k, uint64_t seed, double* L, double* U, int64_t* perm_out) {
  if (k > l || k > n) return ORC_ERR_ARG;
  double* Y = (double*)malloc(sizeof(double) * (size_t)l * (size_t)n);
  orc_sketch(A, m, n, lda, seed, 0, l, Y, n);
  double* Z = (double*)malloc(sizeof(double) * (size_t)n * (size_t)l);
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t r = 0; r < n; ++r) {
    perm[r] = r;
    for (int64_t q = 0; q < l; ++q) Z[r * l + q] = Y[q * n + r];
  }
  for (int64_t s = 0; s < k; ++s) {
    int64_t piv = s;
    double best = fabs(Z[s * l + s]);
    for (int64_t r = s + 1; r < n; ++r) {
      double v = fabs(Z[r * l + s]);
      if (v > best || (v == best && perm[r] < perm[piv])) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0) {
      free(Y); free(Z); free(perm);
      return ORC_RANK_DEFICIENT;
    }
    if (piv != s) {
      for (int64_t q = 0; q < l; ++q) {
        double t = Z[s * l + q];
        Z[s * l + q] = Z[piv * l + q];
        Z[piv * l + q] = t;
      }
      int64_t tp = perm[s];
      perm[s] = perm[piv];
      perm[piv] = tp;
    }
    for (int64_t r = s + 1; r < n; ++r) {
      double lv = Z[r * l + s] / Z[s * l + s];
      Z[r * l + s] = lv;
      for (int64_t q = s + 1; q < l; ++q) Z[r * l + q] = Z[r * l + q] - lv * Z[s * l + q];
    }
  }
  for (int64_t r = 0; r < n; ++r) {
    perm_out[r] = perm[r];
    for (int64_t s = 0; s < k; ++s)
      L[r * k + s] = (s < r) ? Z[r * l + s] : (s == r ? 1.0 : 0.0);
  }
  for (int64_t s = 0; s < k; ++s)
    for (int64_t q = 0; q < l; ++q) U[s * l + q] = (q >= s) ? Z[s * l + q] : 0.0;
  free(Y);
  free(Z);
  free(perm);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Row skeletons of C = A(:, J) (paper Sec. 2.4: after the column skeletons */
/* J, a second, direct LUPP on the small m x k matrix C gives the row        */
/* skeletons I; Sec. 2.2, two-sided ID: A ~= W A(I, J) X with W = C A(I,J)^-1 */
/* the row interpolation matrix, W(I, :) = I_k).  LU with partial pivoting   */
/* on C, k steps, physical row swaps, ties to the lowest original row index;  */
/* an exactly zero pivot stops it (ORC_RANK_DEFICIENT, *k_out = steps).       */
/* With P C = [L1; L2] U: W(I^c, :) = L2 L1^{-1}, each row by back            */
/* substitution x L1 = L2(r, :), s descending.  Outputs: I[0..k_out) in pivot */
/* order; Wr ((m - k_out) x ldw, row-major) row q for the q-th non-skeleton   */
/* row in ascending index.  A J entry outside [0, n) gives ORC_ERR_ARG.       */
/* ------------------------------------------------------------------------ */
int orc_lupp_rows(const double* A, int64_t m, int64_t n, int64_t lda, const int64_t* J, int64_t k,
                  int64_t* I, double* Wr, int64_t ldw, int64_t* k_out) {
  *k_out = 0;
  if (k < 1 || k > m || k > n) return ORC_ERR_ARG;
  for (int64_t s = 0; s < k; ++s)
    if (J[s] < 0 || J[s] >= n) return ORC_ERR_ARG;
  double* Z = (double*)malloc(sizeof(double) * (size_t)m * (size_t)k);
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  for (int64_t r = 0; r < m; ++r) {
    perm[r] = r;
    for (int64_t s = 0; s < k; ++s) Z[r * k + s] = A[r * lda + J[s]];
  }
  int st = ORC_OK;
  int64_t kk = k;
  for (int64_t s = 0; s < k; ++s) {
    int64_t piv = s;
    double best = fabs(Z[s * k + s]);
    for (int64_t r = s + 1; r < m; ++r) {
      const double v = fabs(Z[r * k + s]);
      if (v > best || (v == best && perm[r] < perm[piv])) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0) {
      st = ORC_RANK_DEFICIENT;
      kk = s;
      break;
    }
    if (piv != s) {
      for (int64_t q = 0; q < k; ++q) {
        const double t = Z[s * k + q];
        Z[s * k + q] = Z[piv * k + q];
        Z[piv * k + q] = t;
      }
      const int64_t t = perm[s];
      perm[s] = perm[piv];
      perm[piv] = t;
    }
    for (int64_t r = s + 1; r < m; ++r) {
      const double l = Z[r * k + s] / Z[s * k + s];
      Z[r * k + s] = l;
      for (int64_t q = s + 1; q < k; ++q) Z[r * k + q] = Z[r * k + q] - l * Z[s * k + q];
    }
  }
  for (int64_t s = 0; s < kk; ++s) I[s] = perm[s];
  /* slot of each non-skeleton row among the non-skeletons, ascending */
  char* is_skel = (char*)calloc((size_t)m, 1);
  int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  for (int64_t s = 0; s < kk; ++s) is_skel[perm[s]] = 1;
  int64_t q = 0;
  for (int64_t r = 0; r < m; ++r)
    if (!is_skel[r]) slot[r] = q++;
  double* x = (double*)malloc(sizeof(double) * (size_t)(kk > 0 ? kk : 1));
  for (int64_t r = kk; r < m; ++r) {
    for (int64_t s = kk - 1; s >= 0; --s) {
      double acc = Z[r * k + s];
      for (int64_t s2 = s + 1; s2 < kk; ++s2) acc = acc - x[s2] * Z[s2 * k + s];
      x[s] = acc;
    }
    double* w = Wr + slot[perm[r]] * ldw;
    for (int64_t s = 0; s < kk; ++s) w[s] = x[s];
  }
  *k_out = kk;
  free(x);
  free(is_skel);
  free(slot);
  free(Z);
  free(perm);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Probe features of the learned rank (one block).  The first 16 sketch     */
/* vectors (FP64 stream of `seed`), LU with partial pivoting on Y^T for up  */
/* to 16 steps (ties to the lowest column index), and after s steps the     */
/* Schur estimate E_s = ||S_s||_F / sqrt(16 - s) over the remaining probe   */
/* columns (paper Sec. 4.2, eq. errSch; E_0 = ||Y||_F / 4).  Output:        */
/* log2 m, log2 n, log10 of the relative tolerance, log10(E_s / ||A||_F),   */
/* s = 0..15 (values below 1e-30 are floored there).                        */
/* ------------------------------------------------------------------------ */
void orc_rank_features(const double* A, int64_t m, int64_t n, int64_t lda, double tol, int rel,
                       uint64_t seed, double* out) {
  enum { PR = 16 };
  double* Y = (double*)malloc(sizeof(double) * PR * (size_t)n);
  double* M = (double*)malloc(sizeof(double) * PR * (size_t)n);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  orc_sketch(A, m, n, lda, seed, 0, PR, Y, n);
  for (int64_t j = 0; j < n; ++j) {
    idx[j] = j;
    for (int c = 0; c < PR; ++c) M[j * PR + c] = Y[c * n + j];
  }
  int nf = 0;
  const double fa = sqrt(frob2(A, m, n, lda, &nf));
  double E[PR];
  for (int s = 0; s < PR; ++s) E[s] = 0.0;
  {
    double t = 0.0;
    for (int64_t j = 0; j < n; ++j)
      for (int c = 0; c < PR; ++c) t += M[j * PR + c] * M[j * PR + c];
    E[0] = sqrt(t) / 4.0;
  }
  for (int s = 0; s < PR && s < n; ++s) {
    int64_t p = -1;
    double best = -1.0;
    for (int64_t r = s; r < n; ++r) {
      const double v = fabs(M[r * PR + s]);
      if (v > best || (v == best && idx[r] < idx[p])) {
        best = v;
        p = r;
      }
    }
    if (best == 0.0) break;
    if (p != s) {
      for (int c = 0; c < PR; ++c) {
        const double t = M[s * PR + c];
        M[s * PR + c] = M[p * PR + c];
        M[p * PR + c] = t;
      }
      const int64_t ti = idx[s];
      idx[s] = idx[p];
      idx[p] = ti;
    }
    double ss = 0.0;
    for (int64_t r = s + 1; r < n; ++r) {
      const double l = M[r * PR + s] / M[s * PR + s];
      M[r * PR + s] = l;
      for (int c = s + 1; c < PR; ++c) {
        M[r * PR + c] = M[r * PR + c] - l * M[s * PR + c];
        ss += M[r * PR + c] * M[r * PR + c];
      }
    }
    if (s + 1 < PR) E[s + 1] = sqrt(ss / (double)(PR - 1 - s));
  }
  out[0] = log2((double)m);
  out[1] = log2((double)n);
  const double rtol = rel ? tol : (fa > 0.0 ? tol / fa : 1.0);
  out[2] = log10(rtol > 1e-30 ? rtol : 1e-30);
  for (int s = 0; s < PR; ++s) {
    const double r = fa > 0.0 ? E[s] / fa : 0.0;
    out[3 + s] = log10(r > 1e-30 ? r : 1e-30);
  }
  free(Y);
  free(M);
  free(idx);
}
