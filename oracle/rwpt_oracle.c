/*
 * rwpt_oracle.c -- plain, slow, FP64 CPU oracle for the particle mass-transfer
 * step of interacting random-walk particle tracking (Engdahl, Schmidt & Benson,
 * "Accelerating and parallelizing Lagrangian simulations of mixing-limited
 * reactive transport", arXiv:1811.05474).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the GPU path.
 *
 * What it computes (all arithmetic in IEEE binary64 unless stated):
 *   - orc_philox4x32_10: the Philox4x32-10 counter-based generator as
 *     published by Salmon, Moraes, Dror & Shaw (SC'11, "Parallel random
 *     numbers: as easy as 1, 2, 3").
 *   - orc_walk: the random-walk move of Sec. 1.1, Eq. (1)/(2) with zero
 *     velocity (the test problem of Sec. 3 is pure diffusion), i.e.
 *     x <- x + sqrt(2 D_rw dt) dW per dimension, followed by reflection at
 *     zero-flux walls (Sec. 3).
 *   - orc_walk_adv: the same move with a constant velocity v and the
 *     hydrodynamic dispersion of Eq. (1): x <- x + v dt + B dW with
 *     B B^T = 2 dt [(D_rw + aT |v|) I + (aL - aT) v v^T / |v|], then
 *     reflection.  (Eq. (1) prints only the (aL - aT) term in the walk; with
 *     aT = 0, and in 1-D where Eq. (2) follows, the two agree.)
 *   - orc_neighbors: the set of particle pairs whose separation lies within
 *     the cutoff s_max = kappa*sigma (Sec. 2.1 fixed-radius search, Sec. 2.2
 *     ghost pad Delta zeta = kappa sigma with sigma = sqrt(8 D dt)).
 *   - orc_transfer: the explicit ("matrix explicit", Sec. 1.1) mass transfer
 *     of Eqs. (3)-(6): Gaussian co-location weights (Eq. 3), normalisation
 *     (Sec. 1.1, the paragraph after Eq. 3), pairwise exchange (Eq. 4) and
 *     the explicit update (Eq. 6), followed by the irreversible A+B reaction
 *     evaluated per particle after the transfer (Sec. 3 and Sec. 7).
 *
 * Readings of the paper that this file relies on (each one is written out in
 * the design notes of the repository):
 *   - weight: w_ij = exp(-s_ij^2 / (8 D dt)).  The prefactor of Eq. (3) and the
 *     volume ds cancel in the normalisation; in d dimensions |s|^2 is used.
 *   - self term: j = i is included in the row sum (w_ii = 1): mass "stays
 *     put" with the remaining probability.
 *   - sign: Eq. (4) is authoritative (mass flows from high to low); the
 *     matrix form of Eq. (5) carries the opposite sign as printed.
 *   - normalisation: ROW is the literal P_ij = w_ij / sum_j w_ij.  SYM is the
 *     symmetric part (P + P^T)/2, i.e. P_ij = w_ij (1/r_i + 1/r_j)/2, which
 *     makes every pair exchange antisymmetric and conserves mass (the
 *     conservation requirement of Sec. 6).  SYM is the default.  Which
 *     form the paper means is parity unpinned: no printed value decides it.
 *     Each form is pinned by its own mathematics (SYM: symmetric operator
 *     with unit row and column sums, conserved totals; ROW: unit row sums;
 *     both: the two-particle closed form).
 *   - cutoff predicate: a pair is a neighbour iff s^2 <= rc2 where
 *     rc2 = (kappa*kappa) * ((8*D)*dt) evaluated in binary64 and, for the
 *     binary32 predicate, rounded once to binary32; s^2 is evaluated in the
 *     predicate's precision as fma(dz, dz, fma(dy, dy, dx*dx)) with
 *     dx = x_j - x_i, each operation correctly rounded, dimension order.
 *     kappa = +inf selects the full matrix (every pair).
 *   - D = 0: the transfer is skipped (no mass moves).
 *   - reaction: m = max(0, min(A, B)); A -= m; B -= m.  This is the same
 *     update of (A, B) as the paper's conservative-component form
 *     E = min(C1, C2) with C1 = A + E, C2 = B + E.
 *
 * Build:  gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the Philox S-box on a */
/* 128-bit counter with a 64-bit key; the key is bumped by the Weyl          */
/* constants between rounds.                                                 */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];
  uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n1 = lo1;
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  uint32_t n3 = lo0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k[0] += PHILOX_W0; k[1] += PHILOX_W1; }
    philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------------------ */
/* Random walk (Sec. 1.1 Eq. 1-2 at zero velocity, Sec. 3 reflecting walls). */
/* Counter layout: (particle id, step low word, step high word, 0), key =   */
/* the 64-bit seed.  Uniforms u_k = out_k * 2^-32 + 2^-33 in (0, 1];         */
/* Box-Muller: z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = ... sin(2 pi u1),       */
/* z2 = sqrt(-2 ln u2) cos(2 pi u3).                                         */
/* ------------------------------------------------------------------------ */
void orc_normals(uint32_t id, uint64_t seed, uint64_t step, double z[3]) {
  uint32_t ctr[4] = {id, (uint32_t)step, (uint32_t)(step >> 32), 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  const double two32inv = 1.0 / 4294967296.0;
  double u0 = (double)o[0] * two32inv + 0.5 * two32inv;
  double u1 = (double)o[1] * two32inv + 0.5 * two32inv;
  double u2 = (double)o[2] * two32inv + 0.5 * two32inv;
  double u3 = (double)o[3] * two32inv + 0.5 * two32inv;
  const double twopi = 6.283185307179586476925286766559;
  double ra = sqrt(-2.0 * log(u0));
  double rb = sqrt(-2.0 * log(u2));
  z[0] = ra * cos(twopi * u1);
  z[1] = ra * sin(twopi * u1);
  z[2] = rb * cos(twopi * u3);
}

static double reflect(double x, double lo, double hi) {
  /* mirror at the walls until inside the closed box [lo, hi] */
  for (int it = 0; it < 64 && (x < lo || x > hi); ++it) {
    if (x < lo) x = 2.0 * lo - x;
    else x = 2.0 * hi - x;
  }
  if (x < lo) x = lo;
  if (x > hi) x = hi;
  return x;
}

/* x: n*d row-major (particle-major), updated in place. */
int orc_walk(int64_t n, int d, double *x, const uint32_t *id, uint64_t seed, uint64_t step,
             double D_rw, double dt, const double *lo, const double *hi) {
  if (n < 0 || d < 1 || d > 3 || D_rw < 0 || dt <= 0) return ORC_EINVAL;
  if (D_rw == 0.0) return ORC_OK;
  double amp = sqrt(2.0 * D_rw * dt);
  for (int64_t i = 0; i < n; ++i) {
    double z[3];
    orc_normals(id[i], seed, step, z);
    for (int k = 0; k < d; ++k) {
      double v = x[i * d + k] + amp * z[k];
      x[i * d + k] = reflect(v, lo[k], hi[k]);
    }
  }
  return ORC_OK;
}

/* Constant velocity and dispersivities.  The covariance coefficient of the
 * displacement is c_L = D_rw + aL |v| along u = v / |v| and c_T = D_rw + aT |v|
 * across it, so one square root of 2 dt times the tensor applied to dW is
 *   sqrt(2 dt c_T) dW + (sqrt(2 dt c_L) - sqrt(2 dt c_T)) (u . dW) u.
 * With v = 0 the move is that of orc_walk, bit for bit. */
int orc_walk_adv(int64_t n, int d, double *x, const uint32_t *id, uint64_t seed, uint64_t step,
                 double D_rw, double dt, const double *lo, const double *hi, const double *vel,
                 double alpha_l, double alpha_t) {
  if (n < 0 || d < 1 || d > 3 || D_rw < 0 || dt <= 0 || alpha_t < 0 || alpha_l < alpha_t) return ORC_EINVAL;
  double speed2 = 0.0;
  for (int k = 0; k < d; ++k) speed2 += vel[k] * vel[k];
  const double speed = sqrt(speed2);
  double u[3] = {0.0, 0.0, 0.0};
  if (speed > 0.0)
    for (int k = 0; k < d; ++k) u[k] = vel[k] / speed;
  const double amp_t = sqrt(2.0 * dt * (D_rw + alpha_t * speed));
  const double amp_l = sqrt(2.0 * dt * (D_rw + alpha_l * speed));
  const double extra = amp_l - amp_t;
  if (speed == 0.0 && amp_t == 0.0) return ORC_OK;
  for (int64_t i = 0; i < n; ++i) {
    double z[3];
    orc_normals(id[i], seed, step, z);
    double uz = 0.0;
    for (int k = 0; k < d; ++k) uz += u[k] * z[k];
    for (int k = 0; k < d; ++k) {
      const double move = vel[k] * dt + amp_t * z[k] + extra * uz * u[k];
      x[i * d + k] = reflect(x[i * d + k] + move, lo[k], hi[k]);
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cutoff predicate.                                                          */
/* ------------------------------------------------------------------------ */
static double cutoff_rc2(double kappa, double D, double dt) {
  double sigma2 = 8.0 * D * dt;
  return kappa * kappa * sigma2;
}

/* s^2 in binary32: dx*dx rounded, then fma(dy, dy, .) and fma(dz, dz, .),
 * each correctly rounded (C99 fmaf), dimension order.  volatile keeps the
 * compiler from keeping wider intermediates. */
static int within_f32(const double *xi, const double *xj, int d, float rc2f) {
  volatile float acc = 0.0f;
  for (int k = 0; k < d; ++k) {
    volatile float a = (float)xj[k];
    volatile float b = (float)xi[k];
    volatile float dx = a - b;
    if (k == 0) acc = dx * dx;
    else acc = fmaf(dx, dx, acc);
  }
  return acc <= rc2f;
}

static int within_f64(const double *xi, const double *xj, int d, double rc2) {
  volatile double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    volatile double dx = xj[k] - xi[k];
    if (k == 0) acc = dx * dx;
    else acc = fma(dx, dx, acc);
  }
  return acc <= rc2;
}

static int is_neighbor(const double *xi, const double *xj, int d, double rc2, float rc2f,
                       int prec, int full) {
  if (full) return 1;
  if (prec == 32) return within_f32(xi, xj, d, rc2f);
  return within_f64(xi, xj, d, rc2);
}

/* ------------------------------------------------------------------------ */
/* Neighbour candidates: a plain bucket grid with cells no smaller than the   */
/* cutoff (plus a relative margin that covers binary32 rounding of s^2), and */
/* the 3^d surrounding buckets.  Used only to avoid O(N^2) candidate scans;   */
/* every candidate is still decided by the predicate above.                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int d;
  int64_t n;
  int64_t nc[3];
  double lo[3], h[3];
  int64_t ncell;
  int64_t *start; /* ncell + 1 */
  int64_t *items; /* n */
} grid_t;

static void grid_free(grid_t *g) {
  free(g->start);
  free(g->items);
  g->start = NULL;
  g->items = NULL;
}

static int64_t grid_cell_1(const grid_t *g, int k, double v) {
  double u = floor((v - g->lo[k]) / g->h[k]);
  if (u < 0) u = 0;
  if (u > (double)(g->nc[k] - 1)) u = (double)(g->nc[k] - 1);
  return (int64_t)u;
}

static int64_t grid_cell(const grid_t *g, const double *xi) {
  int64_t c = 0;
  for (int k = g->d - 1; k >= 0; --k) c = c * g->nc[k] + grid_cell_1(g, k, xi[k]);
  return c;
}

static int grid_build(grid_t *g, int64_t n, int d, const double *x, double rc) {
  memset(g, 0, sizeof(*g));
  g->d = d;
  g->n = n;
  double hmin = rc * (1.0 + 1e-4) + 1e-300;
  int64_t ncell = 1;
  for (int k = 0; k < d; ++k) {
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
      double v = x[i * d + k];
      if (v < mn) mn = v;
      if (v > mx) mx = v;
    }
    if (n == 0) { mn = 0; mx = 0; }
    double ext = mx - mn;
    int64_t nc = (int64_t)floor(ext / hmin);
    if (nc < 1) nc = 1;
    if (nc > 4096) nc = 4096;
    g->nc[k] = nc;
    g->lo[k] = mn;
  }
  /* keep the bucket table at most a few entries per particle */
  for (;;) {
    ncell = 1;
    int kmax = 0;
    for (int k = 0; k < d; ++k) {
      ncell *= g->nc[k];
      if (g->nc[k] > g->nc[kmax]) kmax = k;
    }
    if (ncell <= 4 * n + 8 || g->nc[kmax] == 1) break;
    g->nc[kmax] = (g->nc[kmax] + 1) / 2;
  }
  for (int k = 0; k < d; ++k) {
    double ext = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double v = x[i * d + k] - g->lo[k];
      if (v > ext) ext = v;
    }
    int64_t nc = g->nc[k];
    g->h[k] = (nc == 1) ? (ext > 0 ? ext * 2.0 : 1.0) : ext / (double)nc;
    if (g->h[k] < hmin) g->h[k] = hmin;
  }
  g->ncell = ncell;
  g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  g->items = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *cellof = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!g->start || !g->items || !cellof) {
    free(cellof);
    grid_free(g);
    return ORC_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    cellof[i] = grid_cell(g, x + i * d);
    g->start[cellof[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
  int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
  if (!fill) {
    free(cellof);
    grid_free(g);
    return ORC_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = cellof[i];
    g->items[g->start[c] + fill[c]++] = i;
  }
  free(fill);
  free(cellof);
  return ORC_OK;
}

/* Visit every candidate j of particle i (3^d buckets around i's bucket). */
typedef void (*visit_fn)(int64_t i, int64_t j, void *ctx);

static void grid_visit(const grid_t *g, const double *x, int64_t i, visit_fn fn, void *ctx) {
  int d = g->d;
  int64_t ci[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) ci[k] = grid_cell_1(g, k, x[i * d + k]);
  int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    lo[k] = ci[k] > 0 ? ci[k] - 1 : 0;
    hi[k] = ci[k] + 1 < g->nc[k] ? ci[k] + 1 : g->nc[k] - 1;
  }
  for (int64_t c2 = lo[2]; c2 <= hi[2]; ++c2)
    for (int64_t c1 = lo[1]; c1 <= hi[1]; ++c1)
      for (int64_t c0 = lo[0]; c0 <= hi[0]; ++c0) {
        int64_t c = c0;
        if (d > 1) c += g->nc[0] * c1;
        if (d > 2) c += g->nc[0] * g->nc[1] * c2;
        for (int64_t t = g->start[c]; t < g->start[c + 1]; ++t) fn(i, g->items[t], ctx);
      }
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists (CSR, columns ascending) -- the "master list" of parents   */
/* and their children within s_max of Sec. 2.1, including j = i.             */
/* Returns the total number of entries; fills rowptr/cols only when cap is   */
/* large enough.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
  const double *x;
  int d;
  double rc2;
  float rc2f;
  int prec;
  int full;
  int64_t count;
  int32_t *buf;
  int64_t bufcap;
} nbr_ctx;

static void nbr_visit(int64_t i, int64_t j, void *vctx) {
  nbr_ctx *c = (nbr_ctx *)vctx;
  if (is_neighbor(c->x + i * c->d, c->x + j * c->d, c->d, c->rc2, c->rc2f, c->prec, c->full)) {
    if (c->count < c->bufcap) c->buf[c->count] = (int32_t)j;
    c->count++;
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* rows/nrows: when rows != NULL only those rows are listed, in the given
 * order (rowptr then has nrows + 1 entries); every entry must lie in [0, n). */
int64_t orc_neighbors_rows(int64_t n, int d, const double *x, double kappa, double D, double dt,
                           int prec, const int64_t *rows, int64_t nrows, int64_t *rowptr,
                           int32_t *cols, int64_t cap) {
  if (n < 0 || d < 1 || d > 3 || D <= 0 || dt <= 0 || !(kappa > 0)) return ORC_EINVAL;
  if (rows) {
    if (nrows < 0) return ORC_EINVAL;
    for (int64_t t = 0; t < nrows; ++t)
      if (rows[t] < 0 || rows[t] >= n) return ORC_EINVAL;
  }
  const int64_t nout = rows ? nrows : n;
  int full = isinf(kappa);
  double rc2 = cutoff_rc2(kappa, D, dt);
  float rc2f = (float)rc2;
  grid_t g;
  int use_grid = !full;
  if (use_grid && grid_build(&g, n, d, x, sqrt(rc2)) != ORC_OK) return ORC_ENOMEM;
  int64_t total = 0;
  int32_t *row = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!row) {
    if (use_grid) grid_free(&g);
    return ORC_ENOMEM;
  }
  if (rowptr && cap >= 0) rowptr[0] = 0;
  for (int64_t t = 0; t < nout; ++t) {
    const int64_t i = rows ? rows[t] : t;
    nbr_ctx c = {x, d, rc2, rc2f, prec, full, 0, row, n};
    if (use_grid) grid_visit(&g, x, i, nbr_visit, &c);
    else
      for (int64_t j = 0; j < n; ++j) nbr_visit(i, j, &c);
    qsort(row, (size_t)c.count, sizeof(int32_t), cmp_i32);
    if (cols && total + c.count <= cap) memcpy(cols + total, row, (size_t)c.count * sizeof(int32_t));
    total += c.count;
    if (rowptr && cap >= 0) rowptr[t + 1] = total;
  }
  free(row);
  if (use_grid) grid_free(&g);
  return total;
}

int64_t orc_neighbors(int64_t n, int d, const double *x, double kappa, double D, double dt,
                      int prec, int64_t *rowptr, int32_t *cols, int64_t cap) {
  return orc_neighbors_rows(n, d, x, kappa, D, dt, prec, NULL, 0, rowptr, cols, cap);
}

/* ------------------------------------------------------------------------ */
/* Mass transfer.                                                             */
/* ------------------------------------------------------------------------ */
#define ORC_NORM_SYM 0
#define ORC_NORM_ROW 1

typedef struct {
  const double *x;
  int d;
  double rc2;
  float rc2f;
  int prec;
  int full;
  double sigma2;
  double acc;
} rowsum_ctx;

static double weight(const double *xi, const double *xj, int d, double sigma2) {
  double s2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double dx = xj[k] - xi[k];
    s2 += dx * dx;
  }
  return exp(-s2 / sigma2); /* Eq. (3) without the prefactor and ds */
}

static void rowsum_visit(int64_t i, int64_t j, void *vctx) {
  rowsum_ctx *c = (rowsum_ctx *)vctx;
  const double *xi = c->x + i * c->d, *xj = c->x + j * c->d;
  if (is_neighbor(xi, xj, c->d, c->rc2, c->rc2f, c->prec, c->full))
    c->acc += weight(xi, xj, c->d, c->sigma2);
}

typedef struct {
  const double *x;
  int d, S;
  double rc2;
  float rc2f;
  int prec;
  int full;
  double sigma2;
  int norm;
  const double *r;
  const double *M;
  int64_t n;
  double acc[64];
} dm_ctx;

static void dm_visit(int64_t i, int64_t j, void *vctx) {
  dm_ctx *c = (dm_ctx *)vctx;
  const double *xi = c->x + i * c->d, *xj = c->x + j * c->d;
  if (!is_neighbor(xi, xj, c->d, c->rc2, c->rc2f, c->prec, c->full)) return;
  double w = weight(xi, xj, c->d, c->sigma2);
  double p;
  if (c->norm == ORC_NORM_ROW) p = w / c->r[i];
  else p = 0.5 * w * (1.0 / c->r[i] + 1.0 / c->r[j]);
  for (int s = 0; s < c->S; ++s) c->acc[s] += p * (c->M[s * c->n + j] - c->M[s * c->n + i]);
}

/*
 * One explicit transfer + reaction step.
 *   x:     n*d row-major positions (the exact values the path stores)
 *   M_in:  S*n species-major masses (M_in[s*n + i])
 *   M_out: S*n (may not alias M_in)
 *   kappa: cutoff in units of sigma = sqrt(8 D dt); +inf = full matrix
 *   norm:  0 = SYM, 1 = ROW
 *   prec:  32 or 64 -- precision of the cutoff predicate only
 *   react_a/react_b: species pair of A + B -> 0, or -1 to disable
 *   rows/nrows: when rows != NULL only those rows are computed, in the given
 *          order (repeats allowed), and M_out is S*nrows laid out as
 *          M_out[s*nrows + t]; every entry must lie in [0, n), else ORC_EINVAL
 *   r_out: optional n row sums
 */
int orc_transfer_rows(int64_t n, int d, int S, const double *x, const double *M_in, double *M_out,
                      double D, double dt, double kappa, int norm, int prec, int react_a,
                      int react_b, const int64_t *rows, int64_t nrows, double *r_out) {
  if (n < 0 || d < 1 || d > 3 || S < 1 || S > 64 || D < 0 || dt <= 0 || !(kappa > 0))
    return ORC_EINVAL;
  if (norm != ORC_NORM_SYM && norm != ORC_NORM_ROW) return ORC_EINVAL;
  if (prec != 32 && prec != 64) return ORC_EINVAL;
  if ((react_a >= 0) != (react_b >= 0) || react_a >= S || react_b >= S ||
      (react_a >= 0 && react_a == react_b))
    return ORC_EINVAL;
  if (rows) {
    if (nrows < 0) return ORC_EINVAL;
    for (int64_t t = 0; t < nrows; ++t)
      if (rows[t] < 0 || rows[t] >= n) return ORC_EINVAL;
  }
  int64_t nout = rows ? nrows : n;
  double *dM = (double *)calloc((size_t)(nout > 0 ? nout : 1) * (size_t)S, sizeof(double));
  double *r = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (!dM || !r) {
    free(dM);
    free(r);
    return ORC_ENOMEM;
  }
  if (D > 0.0) {
    int full = isinf(kappa);
    double sigma2 = 8.0 * D * dt;
    double rc2 = full ? INFINITY : cutoff_rc2(kappa, D, dt);
    float rc2f = (float)rc2;
    grid_t g;
    int use_grid = !full;
    if (use_grid && grid_build(&g, n, d, x, sqrt(rc2)) != ORC_OK) {
      free(dM);
      free(r);
      return ORC_ENOMEM;
    }
    /* row sums r_i = sum_j w_ij, j = i included (normalisation of Sec. 1.1) */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      rowsum_ctx c = {x, d, rc2, rc2f, prec, full, sigma2, 0.0};
      if (use_grid) grid_visit(&g, x, i, rowsum_visit, &c);
      else
        for (int64_t j = 0; j < n; ++j) rowsum_visit(i, j, &c);
      r[i] = c.acc;
    }
    /* exchange, Eq. (4): dM_i = 1/2 sum_j P_ij (M_j - M_i) */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nout; ++t) {
      int64_t i = rows ? rows[t] : t;
      dm_ctx c;
      c.x = x; c.d = d; c.S = S; c.rc2 = rc2; c.rc2f = rc2f; c.prec = prec; c.full = full;
      c.sigma2 = sigma2; c.norm = norm; c.r = r; c.M = M_in; c.n = n;
      for (int s = 0; s < S; ++s) c.acc[s] = 0.0;
      if (use_grid) grid_visit(&g, x, i, dm_visit, &c);
      else
        for (int64_t j = 0; j < n; ++j) dm_visit(i, j, &c);
      for (int s = 0; s < S; ++s) dM[s * nout + t] = 0.5 * c.acc[s];
    }
    if (use_grid) grid_free(&g);
  }
  /* explicit update, Eq. (6), then the per-particle reaction */
  for (int64_t t = 0; t < nout; ++t) {
    int64_t i = rows ? rows[t] : t;
    for (int s = 0; s < S; ++s) M_out[s * nout + t] = M_in[s * n + i] + dM[s * nout + t];
    if (react_a >= 0) {
      double a = M_out[react_a * nout + t], b = M_out[react_b * nout + t];
      double m = a < b ? a : b;
      if (m < 0.0) m = 0.0;
      M_out[react_a * nout + t] = a - m;
      M_out[react_b * nout + t] = b - m;
    }
  }
  if (r_out)
    for (int64_t i = 0; i < n; ++i) r_out[i] = r[i];
  free(dM);
  free(r);
  return ORC_OK;
}

int orc_transfer(int64_t n, int d, int S, const double *x, const double *M_in, double *M_out,
                 double D, double dt, double kappa, int norm, int prec, int react_a, int react_b,
                 double *r_out) {
  return orc_transfer_rows(n, d, S, x, M_in, M_out, D, dt, kappa, norm, prec, react_a, react_b,
                           NULL, 0, r_out);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
