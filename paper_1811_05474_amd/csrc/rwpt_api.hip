// rwpt_api.hip -- host side of the C ABI declared in include/rwpt.h.
//
// Owns the device state of an ensemble, builds the per-realisation cell grid
// and neighbour-row stencil for a given (dt, D), sequences the kernels of one
// explicit step (optionally replayed as a captured HIP graph) and converts
// between the caller's particle order and the cell-sorted device order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rwpt.h"
#include "rwpt_kernels.h"
#include "rwpt_layout.h"

using namespace rwpt;

namespace {

thread_local std::string g_err;  // errors raised before a context exists

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t b) {
    if (b == 0) b = 256;
    if (p && b <= bytes) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

const char* kPhaseNames[PH_N] = {"walk_key", "cell_scan", "scatter", "canon", "rowsum",
                                 "exchange", "audit",     "dense",   "count"};

}  // namespace

struct rwpt_ctx {
  rwpt_config cfg;
  std::string err;
  bool device_ready = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  bool initialized = false;
  int64_t N = 0;
  int32_t n_real = 0;
  int S = 0, dim = 0;
  size_t tsize = 4;
  int64_t cap = 0;
  std::vector<int64_t> real_start;
  std::vector<double> d_scale;

  DevBuf pos0, pos1, mass0, mass1, id, key, slot, tmp_src, tmp_id, tmp_key, skey, r, q;
  DevBuf nb_meta, nb_idx, nb_w, nb_src;  // neighbour cache of the one-lane-per-particle kernels
  DevBuf src_of;                         // previous sorted slot of each sorted particle
  int mcur = 0;                          // mass buffer holding the current masses (0: mass0, 1: mass1)
  DevBuf cell_count, cell_start, scan_part;
  DevBuf d_rp, d_st, d_tiles, d_tile_start, d_real_start, d_blk_real;
  DevBuf audit_part, audit_out, step_ctr, counts, d_chunks, d_chunk_start, chunk_part, audit_done;
  DevBuf bbox, bparts;  // full-matrix path
  DevBuf half_slots, half_own, d_item_start, d_item_real;  // half-stencil tiling
  int64_t half_nitems = 0;
  bool dense = false;   // full-matrix path selected at init
  float dense_escale = 0.0f, dense_skip_s2 = 0.0f;
  int64_t ncell_total = 0;

  std::vector<RealParams> h_rp;
  std::vector<StencilRow> h_st;
  std::vector<Tile> h_tiles;
  std::vector<int32_t> h_tile_start;
  std::vector<AuditChunk> h_chunks;
  std::vector<int32_t> h_chunk_start;
  int32_t ntiles = 0;
  int log2l = 3;
  double refine[3] = {0, 0, 0};

  bool grid_valid = false;
  double g_dt = 0.0, g_D = 0.0;
  bool sorted_valid = false;
  int64_t steps = 0;
  std::vector<double> audit_init;

  // captured steps: [2 * (sort ? 0 : 1) + mcur at the start of the step]
  hipGraphExec_t gx[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t n_captures = 0;  // step graphs captured since the context was created

  bool prof = false;
  struct Ev {
    hipEvent_t a, b;
    int ph;
  };
  std::vector<Ev> ev_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[PH_N] = {0};
  int64_t prof_cnt[PH_N] = {0};
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static rwpt_status fail(rwpt_ctx* c, rwpt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_err = buf;
  return st;
}

#define HIPCHK(c, expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      (void)hipGetLastError();                                                              \
      return fail((c), e_ == hipErrorOutOfMemory ? RWPT_ENOMEM : RWPT_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                        \
    }                                                                                       \
  } while (0)

static int lanes_to_log2(int lanes) {
  switch (lanes) {
    case -1: return kPrivateLists;
    case -2: return kHalfPairs;
    case 1: return 0;
    case 4: return 2;
    case 8: return 3;
    case 16: return 4;
    default: return -2;  // invalid
  }
}

static void default_refine(int dim, double out[3]) {
  // cells per cutoff length: fine along x (the fastest key axis, which trims
  // the candidate ranges), a few per cutoff across the other axes in 1-D and
  // 2-D
  if (dim == 1) {
    out[0] = 16.0; out[1] = 1.0; out[2] = 1.0;
  } else if (dim == 2) {
    out[0] = 16.0; out[1] = 2.0; out[2] = 1.0;
  } else {
    // 3-D neighbourhoods are sparse (one lane per particle): cells of two
    // cutoffs, so each particle's cutoff box overlaps 2 x 2 rows of 2 cells
    out[0] = 0.5; out[1] = 0.5; out[2] = 0.5;
  }
}

// Lanes per particle when the configuration leaves it open: enough tiles to
// fill the chip for small ensembles, fewer lanes per particle (smaller
// candidate unions per lane) otherwise.
static int default_lanes(int dim, int64_t n, bool fp64) {
  // 1-D, binary32: the row-broadcast kernels (4 lanes) beat 16 lanes per
  // particle (32768 particles: exchange 37 vs 54 us)
  if (dim == 1) return fp64 ? 16 : 4;
  if (dim == 3) return -1;  // sparse neighbourhoods: private candidate rows
  // binary32: the row-broadcast kernels at every size (below 4097 tiles each
  // tile takes a whole block); ~225 neighbours per particle, 2e4 - 3e5
  // particles: 0.054 vs 0.058 ms (4 vs 8 lanes) at 2e4, 0.104 vs 0.140 at 1.5e5
  if (!fp64) return 4;
  // binary64 (vector-load tiles; the exp is the cost): 8 lanes per particle
  // beats 4 at every size measured, 0.975 vs 0.993 ms at 1e6, 0.351 vs 0.376
  // at 3e5, 0.068 vs 0.083 at 2e4
  (void)n;
  return 8;
}

static void invalidate_graphs(rwpt_ctx* c) {
  for (int k = 0; k < 4; ++k)
    if (c->gx[k]) {
      (void)hipGraphExecDestroy(c->gx[k]);
      c->gx[k] = nullptr;
    }
}

static rwpt_status ensure_device(rwpt_ctx* c) {
  if (c->device_ready) return RWPT_OK;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(c, RWPT_EDEVICE, "no HIP device available (%s)",
                e != hipSuccess ? hipGetErrorString(e) : "device count 0");
  }
  if (c->cfg.device >= n) return fail(c, RWPT_EDEVICE, "device %d not present (%d devices)", c->cfg.device, n);
  HIPCHK(c, hipSetDevice(c->cfg.device));
  hipDeviceProp_t prop;
  HIPCHK(c, hipGetDeviceProperties(&prop, c->cfg.device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(c, RWPT_EDEVICE, "device %d is %s; this library is built for gfx950", c->cfg.device,
                prop.gcnArchName);
  if (c->cfg.stream) {
    c->stream = (hipStream_t)c->cfg.stream;
    c->own_stream = false;
  } else {
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  HIPCHK(c, c->step_ctr.ensure(sizeof(uint64_t)));

  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->device_ready = true;
  return RWPT_OK;
}

// Record a phase: start event before a launch, stop event after it.
struct PhaseScope {
  rwpt_ctx* c;
  int ph;
  hipEvent_t a = nullptr, b = nullptr;
  PhaseScope(rwpt_ctx* cc, int p) : c(cc), ph(p) {
    if (!c->prof) return;
    a = take();
    b = take();
    if (a) (void)hipEventRecord(a, c->stream);
  }
  hipEvent_t take() {
    if (!c->ev_pool.empty()) {
      hipEvent_t e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~PhaseScope() {
    if (!c->prof || !a || !b) return;
    (void)hipEventRecord(b, c->stream);
    c->ev_pending.push_back({a, b, ph});
  }
};

static void drain_profile(rwpt_ctx* c) {
  if (c->ev_pending.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& ev : c->ev_pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
      c->prof_ms[ev.ph] += ms;
      c->prof_cnt[ev.ph] += 1;
    }
    c->ev_pool.push_back(ev.a);
    c->ev_pool.push_back(ev.b);
  }
  c->ev_pending.clear();
}

// ---------------------------------------------------------------------------
// grid, stencil and tiles for (dt, D)
// ---------------------------------------------------------------------------

// Cell grid, physical parameters and neighbour-row stencil of one realisation
// of nr particles for the step (dt, D_r): the walk amplitudes (Eq. 1/2), the
// cutoff kappa sigma with sigma^2 = 8 D_r dt and its binary32 / binary64
// squares, the weight scale of Eq. 3, cells per axis (refine cells per cutoff
// length, at most about four per particle), and the stencil rows appended to
// st (P.stencil_off, P.n_stencil).  P.cell_off = cell_off; p_begin / p_end
// are left to the caller.
template <typename Rows>
static void real_grid(const rwpt_config& cfg, int dim, double dt, double Dr, int64_t nr, const double refine[3],
                      bool dense, float* dense_escale, float* dense_skip_s2, int64_t cell_off, RealParams& P,
                      Rows& st) {
  memset(&P, 0, sizeof(P));
  double L[3];
  for (int k = 0; k < 3; ++k) {
    P.lo[k] = k < dim ? cfg.box_lo[k] : 0.0;
    P.hi[k] = k < dim ? cfg.box_hi[k] : 1.0;
    L[k] = P.hi[k] - P.lo[k];
  }
  {
    // walk: isotropic share D_rw, plus drift and dispersion with a velocity
    double speed2 = 0.0;
    for (int k = 0; k < dim; ++k) speed2 += cfg.velocity[k] * cfg.velocity[k];
    const double speed = std::sqrt(speed2);
    const double Drw = cfg.rw_ratio * Dr;
    P.amp = std::sqrt(2.0 * dt * (Drw + cfg.alpha_t * speed));
    P.amp_x = std::sqrt(2.0 * dt * (Drw + cfg.alpha_l * speed)) - P.amp;
    for (int k = 0; k < 3; ++k) {
      P.drift[k] = k < dim ? cfg.velocity[k] * dt : 0.0;
      P.udir[k] = (k < dim && speed > 0.0) ? cfg.velocity[k] / speed : 0.0;
    }
    P.moves = (P.amp > 0.0 || speed > 0.0) ? 1 : 0;
  }
  P.active = Dr > 0.0 ? 1 : 0;
  int64_t nc[3] = {1, 1, 1};
  double rcg = 0.0;
  if (P.active) {
    const double sigma2 = 8.0 * Dr * dt;
    const double rc2 = std::isinf(cfg.kappa) ? INFINITY : cfg.kappa * cfg.kappa * sigma2;
    P.rc2_d = rc2;
    P.rc2_f = (float)rc2;
    P.escale_d = -1.0 / sigma2;
    P.escale_f = (float)(-1.4426950408889634073599246810019 / sigma2);
    // geometric cutoff: covers the rounding of s^2 in the predicate
    rcg = std::sqrt(rc2) * (1.0 + 1e-5);
    P.rc_geo = rcg;
    if (dense) {
      // every pair counts; the grid only orders particles so that 32-particle
      // column tiles are compact, and tiles farther apart than the distance
      // where w < 2^-40 are skipped
      *dense_escale = P.escale_f;
      *dense_skip_s2 = (float)(41.0 / std::fabs((double)P.escale_f));
      rcg = std::sqrt(40.0 / std::fabs((double)P.escale_f));
    }
    if (std::isfinite(rcg)) {
      for (int k = 0; k < dim; ++k) {
        double v = std::floor(L[k] * refine[k] / rcg);
        if (!(v >= 1.0)) v = 1.0;
        if (v > (double)(1 << 20)) v = (double)(1 << 20);
        nc[k] = (int64_t)v;
      }
      const int64_t cap_cells = std::max<int64_t>(4 * nr, 64);
      for (;;) {
        int64_t prod = nc[0] * nc[1] * nc[2];
        if (prod <= cap_cells) break;
        int kmax = 0;
        for (int k = 1; k < 3; ++k)
          if (nc[k] > nc[kmax]) kmax = k;
        if (nc[kmax] <= 1) break;
        nc[kmax] = (nc[kmax] + 1) / 2;
      }
    }
  }
  for (int k = 0; k < 3; ++k) {
    P.nc[k] = (int32_t)nc[k];
    P.inv_h[k] = (double)nc[k] / L[k];
  }
  P.cell_off = cell_off;
  P.stencil_off = (int32_t)st.size();
  if (P.active && !dense) {
    const double h[3] = {L[0] / nc[0], L[1] / nc[1], L[2] / nc[2]};
    int Ry = 0, Rz = 0;
    if (dim >= 2) Ry = std::isfinite(rcg) ? (int)std::min<double>(nc[1] - 1, std::ceil(rcg / h[1])) : (int)nc[1] - 1;
    if (dim >= 3) Rz = std::isfinite(rcg) ? (int)std::min<double>(nc[2] - 1, std::ceil(rcg / h[2])) : (int)nc[2] - 1;
    for (int dz = -Rz; dz <= Rz; ++dz)
      for (int dy = -Ry; dy <= Ry; ++dy) {
        int rx;
        if (std::isfinite(rcg)) {
          const double ym = std::max(0, std::abs(dy) - 1) * h[1];
          const double zm = std::max(0, std::abs(dz) - 1) * h[2];
          const double rem = rcg * rcg - ym * ym - zm * zm;
          if (rem < 0.0) continue;
          const double hw = std::sqrt(rem);
          rx = (int)std::min<double>(nc[0] - 1, std::ceil(hw * P.inv_h[0]));
        } else {
          rx = (int)nc[0] - 1;
        }
        st.push_back(StencilRow{dy, dz, rx, 0});
      }
  }
  P.n_stencil = (int32_t)st.size() - P.stencil_off;
}

// Segments of the half-stencil tiling for one realisation: seg_w =
// ceil(2 * the widest reach along x of its stencil rows / (npar - 1)), so that
// at most npar consecutive segments of a row (distinct mod npar) reach any
// cell; the own row's reach; the number of forward stencil rows (dz > 0, or
// dz = 0 and dy > 0).
static void half_segments(RealParams& P, const StencilRow* st, int64_t nr, int64_t target) {
  int rx_max = 0, rx_own = 0, n_fwd = 0;
  for (int f = 0; f < P.n_stencil; ++f) {
    rx_max = std::max(rx_max, st[f].rx);
    if (st[f].dy == 0 && st[f].dz == 0) rx_own = st[f].rx;
    if (st[f].dz > 0 || (st[f].dz == 0 && st[f].dy > 0)) ++n_fwd;
  }
  P.npar = kHalfParities;
  P.seg_w = std::max(1, (2 * rx_max + P.npar - 2) / (P.npar - 1));
  // wider segments where neighbourhoods are sparse, so that a work item has
  // about `target` candidate evaluations on average (any width above the
  // bound keeps the slots single-writer): candidates per particle ~ particles
  // per cell x cells of the stencil
  const int64_t cells = (int64_t)P.nc[0] * P.nc[1] * P.nc[2];
  if (nr > 0 && cells > 0) {
    int64_t stencil_cells = 0;
    for (int f = 0; f < P.n_stencil; ++f) stencil_cells += 2 * st[f].rx + 1;
    const double per_cell = (double)nr / (double)cells;
    const double cand = std::max(1.0, per_cell * (double)stencil_cells);
    const double want = std::ceil((double)target / cand / per_cell);
    if (want > (double)P.seg_w) P.seg_w = (int32_t)std::min<double>(want, (double)P.nc[0]);
  }
  P.nseg = P.active ? (P.nc[0] + P.seg_w - 1) / P.seg_w : 0;
  P.rx_own = rx_own;
  P.n_fwd = n_fwd;
}

static rwpt_status build_grid(rwpt_ctx* c, double dt, double D) {
  if (c->grid_valid && c->g_dt == dt && c->g_D == D) return RWPT_OK;
  const rwpt_config& cfg = c->cfg;
  const int dim = c->dim;
  int lanes = cfg.tile_lanes ? cfg.tile_lanes : default_lanes(dim, c->N, cfg.precision == RWPT_FP64);
  if (c->dense) lanes = 64 / kDenseRowTile;  // tiles of 16 rows (audit partials, D = 0 copy)
  c->log2l = lanes_to_log2(lanes);
  double defr[3];
  default_refine(dim, defr);
  for (int k = 0; k < 3; ++k) c->refine[k] = cfg.cell_refine[k] > 0 ? cfg.cell_refine[k] : defr[k];
  const int G = (c->log2l == kPrivateLists || c->log2l == kHalfPairs) ? 64 : 64 >> c->log2l;
  const bool half = c->log2l == kHalfPairs;

  c->h_rp.assign(c->n_real, RealParams{});
  c->h_st.clear();
  c->h_tiles.clear();
  c->h_tile_start.assign(c->n_real + 1, 0);
  int64_t cell_off = 0;
  for (int r = 0; r < c->n_real; ++r) {
    RealParams& P = c->h_rp[r];
    const int64_t nr = c->real_start[r + 1] - c->real_start[r];
    real_grid(cfg, dim, dt, D * c->d_scale[r], nr, c->refine, c->dense, &c->dense_escale, &c->dense_skip_s2,
              cell_off, P, c->h_st);
    P.p_begin = c->real_start[r];
    P.p_end = c->real_start[r + 1];
    cell_off += (int64_t)P.nc[0] * P.nc[1] * P.nc[2];
    if (half) half_segments(P, c->h_st.data() + P.stencil_off, nr, kHalfTarget);
    c->h_tile_start[r] = (int32_t)c->h_tiles.size();
    for (int64_t b = P.p_begin; b < P.p_end; b += G)
      c->h_tiles.push_back(Tile{(int32_t)b, (int32_t)std::min<int64_t>(b + G, P.p_end), r, 0});
  }
  c->h_tile_start[c->n_real] = (int32_t)c->h_tiles.size();
  c->h_chunks.clear();
  c->h_chunk_start.assign(c->n_real + 1, 0);
  for (int r = 0; r < c->n_real; ++r) {
    c->h_chunk_start[r] = (int32_t)c->h_chunks.size();
    const int32_t t0 = c->h_tile_start[r], t1 = c->h_tile_start[r + 1];
    const int32_t nch = (t1 - t0 + kAuditChunk - 1) / kAuditChunk;
    for (int32_t t = t0; t < t1; t += kAuditChunk)
      c->h_chunks.push_back(AuditChunk{t, std::min<int32_t>(t + kAuditChunk, t1), r, nch});
  }
  c->h_chunk_start[c->n_real] = (int32_t)c->h_chunks.size();
  if (cell_off >= (int64_t)1 << 31) return fail(c, RWPT_EUNSUPPORTED, "cell grid too large (%lld cells)", (long long)cell_off);
  c->ntiles = (int32_t)c->h_tiles.size();
  // half-stencil tiling: work items (row, segment) of every realisation, and
  // slot planes npar (1 + forward rows) deep
  std::vector<int64_t> item_start(c->n_real + 1, 0);
  std::vector<int32_t> item_real(c->n_real, 0);
  int max_fwd = 0;
  c->half_nitems = 0;
  if (half) {
    // dispatch order: realisations by decreasing estimated cost per work item
    // (particles per item x candidates per particle), so that the longest
    // items start first and the short ones fill the end of the launch
    std::vector<double> cost(c->n_real, 0.0);
    for (int r = 0; r < c->n_real; ++r) {
      const RealParams& P = c->h_rp[r];
      const int64_t items = (int64_t)P.nseg * P.nc[1] * P.nc[2];
      const int64_t cells = (int64_t)P.nc[0] * P.nc[1] * P.nc[2];
      if (items <= 0 || cells <= 0) continue;
      int64_t stencil_cells = 0;
      for (int f = 0; f < P.n_stencil; ++f) stencil_cells += 2 * c->h_st[P.stencil_off + f].rx + 1;
      const double nr = (double)(c->real_start[r + 1] - c->real_start[r]);
      cost[r] = (nr / (double)items) * (nr / (double)cells) * (double)stencil_cells;
    }
    std::vector<int32_t> ord(c->n_real);
    for (int r = 0; r < c->n_real; ++r) ord[r] = r;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    for (int k = 0; k < c->n_real; ++k) {
      RealParams& P = c->h_rp[ord[k]];
      P.item_off = c->half_nitems;
      item_start[k] = c->half_nitems;
      item_real[k] = ord[k];
      c->half_nitems += (int64_t)P.nseg * P.nc[1] * P.nc[2];
      max_fwd = std::max(max_fwd, P.n_fwd);
    }
    item_start[c->n_real] = c->half_nitems;
  }

  // device copies
  const int64_t ncell = cell_off;
  const int64_t nscan = (ncell + kScanChunk - 1) / kScanChunk + 1;
  bool regrow = (size_t)(ncell * 4) > c->cell_count.bytes;
  HIPCHK(c, c->cell_count.ensure((size_t)ncell * 4));
  HIPCHK(c, c->cell_start.ensure((size_t)(ncell + 1) * 4));
  HIPCHK(c, c->scan_part.ensure((size_t)nscan * 4));
  HIPCHK(c, c->d_rp.ensure(c->h_rp.size() * sizeof(RealParams)));
  HIPCHK(c, c->d_st.ensure(std::max<size_t>(1, c->h_st.size()) * sizeof(StencilRow)));
  HIPCHK(c, c->d_tiles.ensure(std::max<size_t>(1, c->h_tiles.size()) * sizeof(Tile)));
  HIPCHK(c, c->d_tile_start.ensure(c->h_tile_start.size() * sizeof(int32_t)));
  HIPCHK(c, c->audit_part.ensure((size_t)std::max(1, c->ntiles) * (c->S + 1) * sizeof(double)));
  HIPCHK(c, c->counts.ensure((size_t)std::max(1, c->ntiles) * 2 * sizeof(unsigned long long)));
  if (c->log2l == kPrivateLists) {
    HIPCHK(c, c->nb_meta.ensure((size_t)c->cap * sizeof(uint16_t)));
    HIPCHK(c, c->nb_idx.ensure((size_t)std::max(1, c->ntiles) * kCacheWave * sizeof(uint32_t)));
    HIPCHK(c, c->nb_w.ensure((size_t)std::max(1, c->ntiles) * kCacheWave * c->tsize));
    HIPCHK(c, c->nb_src.ensure((size_t)std::max(1, c->ntiles) * kCacheWave * sizeof(uint32_t)));
  }
  if (half) {
    const int Sa = padded_species(c->S);
    HIPCHK(c, c->half_slots.ensure((size_t)kHalfParities * (1 + max_fwd) * c->cap * Sa * sizeof(float)));
    HIPCHK(c, c->half_own.ensure((size_t)c->cap * Sa * sizeof(double)));
    HIPCHK(c, c->d_item_start.ensure(item_start.size() * sizeof(int64_t)));
    HIPCHK(c, hipMemcpyAsync(c->d_item_start.p, item_start.data(), item_start.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, c->d_item_real.ensure(item_real.size() * sizeof(int32_t)));
    HIPCHK(c, hipMemcpyAsync(c->d_item_real.p, item_real.data(), item_real.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
  }
  if (c->dense) {
    const int ncb = dense_ncb(c->S, c->cfg.norm);
    HIPCHK(c, c->bbox.ensure((size_t)(c->cap / kDenseColTile + 1) * 2 * c->dim * sizeof(float)));
    HIPCHK(c, c->bparts.ensure((size_t)3 * 16 * ncb * c->cap * sizeof(uint16_t)));
  }
  HIPCHK(c, c->d_chunks.ensure(std::max<size_t>(1, c->h_chunks.size()) * sizeof(AuditChunk)));
  HIPCHK(c, c->d_chunk_start.ensure(c->h_chunk_start.size() * sizeof(int32_t)));
  HIPCHK(c, c->chunk_part.ensure(std::max<size_t>(1, c->h_chunks.size()) * (c->S + 1) * sizeof(double)));
  if (!c->h_chunks.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_chunks.p, c->h_chunks.data(), c->h_chunks.size() * sizeof(AuditChunk),
                             hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_chunk_start.p, c->h_chunk_start.data(),
                           c->h_chunk_start.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_rp.p, c->h_rp.data(), c->h_rp.size() * sizeof(RealParams),
                           hipMemcpyHostToDevice, c->stream));
  if (!c->h_st.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_st.p, c->h_st.data(), c->h_st.size() * sizeof(StencilRow),
                             hipMemcpyHostToDevice, c->stream));
  if (!c->h_tiles.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_tiles.p, c->h_tiles.data(), c->h_tiles.size() * sizeof(Tile),
                             hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_tile_start.p, c->h_tile_start.data(),
                           c->h_tile_start.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  (void)regrow;
  HIPCHK(c, hipMemsetAsync(c->cell_count.p, 0, (size_t)ncell * 4, c->stream));
  // the host vectors above must stay alive until the copies finish
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->ncell_total = ncell;
  c->grid_valid = true;
  c->g_dt = dt;
  c->g_D = D;
  c->sorted_valid = false;
  invalidate_graphs(c);
  return RWPT_OK;
}

static DevBuf& mass_buf(rwpt_ctx* c, int k) { return k ? c->mass1 : c->mass0; }

// Steps whose sort leaves the masses in place (the exchange reads them
// through src_of): the one-lane-per-particle kernels of the sparse path.
static bool masses_stay(const rwpt_ctx* c) { return !c->dense && c->log2l == kPrivateLists; }

static PairArgs pair_args(rwpt_ctx* c) {
  PairArgs a;
  memset(&a, 0, sizeof(a));
  a.pos = c->pos0.p;
  a.mass_in = mass_buf(c, c->mcur).p;
  a.mass_out = mass_buf(c, c->mcur ^ 1).p;
  a.q_in = c->q.p;
  a.q_out = c->q.p;
  a.r_out = c->cfg.norm == RWPT_NORM_ROW ? c->r.as<double>() : nullptr;  // read by the exchange
  a.skey = c->skey.as<uint32_t>();
  a.cell_start = c->cell_start.as<uint32_t>();
  a.tiles = c->d_tiles.as<Tile>();
  a.ntiles = c->ntiles;
  a.rp = c->d_rp.as<RealParams>();
  a.st = c->d_st.as<StencilRow>();
  a.S = c->S;
  a.react_a = c->cfg.react_a;
  a.react_b = c->cfg.react_b;
  a.norm = c->cfg.norm;
  a.audit_part = c->audit_part.as<double>();
  a.counts = c->counts.as<unsigned long long>();
  a.nb_meta = c->nb_meta.as<uint16_t>();
  a.nb_idx = c->nb_idx.as<uint32_t>();
  a.nb_w = c->nb_w.p;
  a.nb_src = c->nb_src.as<uint32_t>();
  a.src_of = c->src_of.as<uint32_t>();
  a.indirect = 0;
  a.half_slots = c->half_slots.as<float>();
  a.half_own = c->half_own.as<double>();
  a.half_item_start = c->d_item_start.as<int64_t>();
  a.half_item_real = c->d_item_real.as<int32_t>();
  a.half_nitems = c->half_nitems;
  a.half_cap = c->cap;
  a.n_real = c->n_real;
  return a;
}

// Sort into the cell grid: [walk] -> key -> counting sort -> canonical order.
// Leaves positions in pos0, ids in id, keys in skey; the masses move to the
// other buffer in the new order (mcur flips), or, with move_mass false, stay
// where they are and src_of records each sorted particle's previous slot.
static rwpt_status enqueue_sort(rwpt_ctx* c, bool walk, bool move_mass) {
  const int fp64 = c->cfg.precision == RWPT_FP64;
  const int32_t n = (int32_t)c->N;
  {
    PhaseScope ps(c, PH_WALK_KEY);
    HIPCHK(c, launch_walk_key(fp64, c->dim, c->pos0.p, c->pos1.p, c->id.as<uint32_t>(), n,
                              c->d_rp.as<RealParams>(), c->d_real_start.as<int64_t>(),
                              c->d_blk_real.as<int32_t>(), c->n_real,
                              c->step_ctr.as<uint64_t>(), c->cfg.seed, walk ? 1 : 0,
                              c->cell_count.as<uint32_t>(), c->key.as<uint32_t>(),
                              c->slot.as<uint32_t>(), c->stream));
  }
  {
    PhaseScope ps(c, PH_SCAN);
    HIPCHK(c, launch_cell_scan(c->cell_count.as<uint32_t>(), c->cell_start.as<uint32_t>(), c->ncell_total,
                               c->scan_part.as<uint32_t>(), c->stream));
  }
  {
    PhaseScope ps(c, PH_SCATTER);
    HIPCHK(c, launch_scatter(n, c->key.as<uint32_t>(), c->slot.as<uint32_t>(), c->cell_start.as<uint32_t>(),
                             c->id.as<uint32_t>(), c->tmp_src.as<uint32_t>(), c->tmp_id.as<uint32_t>(),
                             c->tmp_key.as<uint32_t>(), c->stream));
  }
  {
    PhaseScope ps(c, PH_CANON);
    HIPCHK(c, launch_canon(fp64, c->dim, n, c->tmp_src.as<uint32_t>(), c->tmp_id.as<uint32_t>(),
                           c->tmp_key.as<uint32_t>(), c->cell_start.as<uint32_t>(), c->pos1.p, c->pos0.p,
                           mass_buf(c, c->mcur).p, mass_buf(c, c->mcur ^ 1).p, c->S,
                           c->id.as<uint32_t>(), c->skey.as<uint32_t>(),
                           move_mass ? nullptr : c->src_of.as<uint32_t>(), c->stream));
  }
  if (move_mass) c->mcur ^= 1;
  return RWPT_OK;
}

// One explicit step.  Positions in pos0; the masses are read from buffer
// mcur (in the previous sorted order when the sort left them in place) and
// the updated masses are written, in the current sorted order, to the other
// buffer, which becomes mcur.
static rwpt_status enqueue_step(rwpt_ctx* c, bool sort, bool walk) {
  const int fp64 = c->cfg.precision == RWPT_FP64;
  const bool stay = sort && masses_stay(c);
  if (sort) {
    rwpt_status st = enqueue_sort(c, walk, !stay);
    if (st != RWPT_OK) return st;
  }
  PairArgs a = pair_args(c);
  a.indirect = stay ? 1 : 0;
  if (c->dense && c->h_rp[0].active) {
    DenseArgs da;
    memset(&da, 0, sizeof(da));
    da.pos = c->pos0.as<float>();
    da.cap = c->cap;
    da.n = (int32_t)c->N;
    da.mass_in = mass_buf(c, c->mcur).as<float>();
    da.mass_out = mass_buf(c, c->mcur ^ 1).as<float>();
    da.q = c->q.as<float>();
    da.r = c->r.as<double>();
    da.bbox = c->bbox.as<float>();
    da.escale = c->dense_escale;
    da.skip_s2 = c->dense_skip_s2;
    da.bparts = c->bparts.as<__bf16>();
    da.ncb = dense_ncb(c->S, c->cfg.norm);
    da.S = c->S;
    da.react_a = c->cfg.react_a;
    da.react_b = c->cfg.react_b;
    da.norm = c->cfg.norm;
    da.audit_part = c->audit_part.as<double>();
    PhaseScope ps(c, PH_DENSE);
    HIPCHK(c, launch_dense_step(c->dim, da, c->stream));
  } else {
    // the one-lane-per-particle exchange reads the row-sum pass's neighbour
    // cache, so that pass runs for either normalisation
    if (c->cfg.norm == RWPT_NORM_SYM || c->log2l == kPrivateLists || c->log2l == kHalfPairs) {
      PhaseScope ps(c, PH_ROWSUM);
      HIPCHK(c, launch_rowsum(fp64, c->dim, c->log2l, a, c->stream));
    }
    PhaseScope ps(c, PH_EXCHANGE);
    HIPCHK(c, launch_exchange(fp64, c->dim, c->log2l, a, c->stream));
  }
  c->mcur ^= 1;
  {
    PhaseScope ps(c, PH_AUDIT);
    HIPCHK(c, launch_audit_reduce(c->audit_part.as<double>(), c->S + 1, c->d_chunks.as<AuditChunk>(),
                                  (int32_t)c->h_chunks.size(), c->chunk_part.as<double>(),
                                  c->d_chunk_start.as<int32_t>(), c->n_real, c->audit_out.as<double>(),
                                  c->audit_done.as<uint32_t>(), c->step_ctr.as<uint64_t>(), 1, c->stream));
  }
  return RWPT_OK;
}

// Flips of mcur in one step: the exchange always writes the other buffer; a
// sort that moves the masses flips once more.
static int step_flips(const rwpt_ctx* c, bool sort) { return (sort && !masses_stay(c)) ? 0 : 1; }


static rwpt_status ensure_sorted(rwpt_ctx* c) {
  if (c->sorted_valid) return RWPT_OK;
  rwpt_status st = enqueue_sort(c, false, true);  // masses follow into the sorted order
  if (st != RWPT_OK) return st;
  c->sorted_valid = true;
  return RWPT_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Scratch area of the allocation-free entry point
// ---------------------------------------------------------------------------

// Device memory of rwpt_transfer_noalloc: one fixed area per device, part of
// the library's code object (held by every device the library is loaded on
// until the process ends).  Host code never uses the name `scratch` as an
// address: it looks up the area's device address once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};  // device address of `scratch` on each device
}  // namespace

// Device address of the scratch area on the current device, looked up on the
// first call on that device (with it current).
static rwpt_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kScratchDevices) {
    (void)hipGetLastError();
    return fail(nullptr, RWPT_EDEVICE, "no current HIP device (%s)", e != hipSuccess ? hipGetErrorString(e) : "ordinal out of range");
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(nullptr, RWPT_EDEVICE, "scratch area of device %d: %s", dev,
                  e != hipSuccess ? hipGetErrorString(e) : "null address");
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RWPT_OK;
}

// Fixed-capacity list of stencil rows (no host allocation).
struct RowBuf {
  StencilRow* rows;
  int cap;
  int n;
  size_t size() const { return (size_t)n; }
  void push_back(const StencilRow& r) {
    if (n < cap) rows[n] = r;
    ++n;
  }
};

// Bump allocation of 256-byte-aligned pieces of the scratch area.
struct ScratchLayout {
  size_t used = 0;
  size_t take(size_t bytes) {
    const size_t at = used;
    used += (bytes + 255) / 256 * 256;
    return at;
  }
};

// Validation of a configuration (the messages go to the thread's error slot).
static rwpt_status check_config(const rwpt_config& c) {
  if (c.dim < 1 || c.dim > 3) return fail(nullptr, RWPT_EINVAL, "dim must be 1, 2 or 3 (got %d)", c.dim);
  if (c.n_species < 1 || c.n_species > 8)
    return fail(nullptr, RWPT_EINVAL, "n_species must be in 1..8 (got %d)", c.n_species);
  const bool ra = c.react_a >= 0, rb = c.react_b >= 0;
  if (ra != rb || c.react_a < -1 || c.react_b < -1)
    return fail(nullptr, RWPT_EINVAL, "react_a/react_b must both be -1 or both valid species");
  if (ra && (c.react_a >= c.n_species || c.react_b >= c.n_species || c.react_a == c.react_b))
    return fail(nullptr, RWPT_EINVAL, "reaction species (%d, %d) invalid for S = %d", c.react_a,
                c.react_b, c.n_species);
  for (int k = 0; k < c.dim; ++k)
    if (!std::isfinite(c.box_lo[k]) || !std::isfinite(c.box_hi[k]) || !(c.box_lo[k] < c.box_hi[k]))
      return fail(nullptr, RWPT_EINVAL, "box axis %d must satisfy finite lo < hi", k);
  if (!(c.kappa > 0.0)) return fail(nullptr, RWPT_EINVAL, "kappa must be > 0 (or INFINITY)");
  if (!std::isfinite(c.rw_ratio) || c.rw_ratio < 0.0)
    return fail(nullptr, RWPT_EINVAL, "rw_ratio must be finite and >= 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(c.velocity[k])) return fail(nullptr, RWPT_EINVAL, "velocity[%d] is not finite", k);
  if (!std::isfinite(c.alpha_l) || !std::isfinite(c.alpha_t) || c.alpha_t < 0.0 || c.alpha_l < c.alpha_t)
    return fail(nullptr, RWPT_EINVAL, "dispersivities must satisfy alpha_l >= alpha_t >= 0");
  if (c.precision != RWPT_FP32 && c.precision != RWPT_FP64)
    return fail(nullptr, RWPT_EINVAL, "precision must be RWPT_FP32 or RWPT_FP64");
  if (c.norm != RWPT_NORM_SYM && c.norm != RWPT_NORM_ROW)
    return fail(nullptr, RWPT_EINVAL, "norm must be RWPT_NORM_SYM or RWPT_NORM_ROW");
  if (c.path < RWPT_PATH_AUTO || c.path > RWPT_PATH_DENSE)
    return fail(nullptr, RWPT_EINVAL, "path must be AUTO, SPARSE or DENSE");
  if (c.path == RWPT_PATH_DENSE && !std::isinf(c.kappa))
    return fail(nullptr, RWPT_EINVAL, "the dense path evaluates every pair: kappa must be INFINITY");
  if (c.path == RWPT_PATH_DENSE && c.precision != RWPT_FP32)
    return fail(nullptr, RWPT_EUNSUPPORTED, "the dense (matrix-core) path is binary32 only");
  if (c.tile_lanes != 0 && lanes_to_log2(c.tile_lanes) == -2)
    return fail(nullptr, RWPT_EINVAL, "tile_lanes must be -2, -1, 0, 1, 4, 8 or 16 (got %d)", c.tile_lanes);
  if (c.tile_lanes == -2 && c.precision != RWPT_FP32)
    return fail(nullptr, RWPT_EUNSUPPORTED, "the half-stencil tiling (tile_lanes -2) is binary32 only");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(c.cell_refine[k]) || c.cell_refine[k] < 0.0 || c.cell_refine[k] > 64.0)
      return fail(nullptr, RWPT_EINVAL, "cell_refine[%d] must be in [0, 64]", k);
  if (c.device < 0) return fail(nullptr, RWPT_EINVAL, "device must be >= 0");
  if (c.use_graph != 0 && c.use_graph != 1) return fail(nullptr, RWPT_EINVAL, "use_graph must be 0 or 1");
  return RWPT_OK;
}

extern "C" {

const char* rwpt_version(void) { return "rwpt-mi355x 0.1 (gfx950)"; }

void rwpt_config_default(rwpt_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->dim = 2;
  cfg->n_species = 2;
  cfg->react_a = 0;
  cfg->react_b = 1;
  for (int k = 0; k < 3; ++k) {
    cfg->box_lo[k] = 0.0;
    cfg->box_hi[k] = 1.0;
  }
  cfg->kappa = 3.0;
  cfg->rw_ratio = 1.0;
  cfg->precision = RWPT_FP32;
  cfg->norm = RWPT_NORM_SYM;
  cfg->path = RWPT_PATH_AUTO;
  cfg->tile_lanes = 0;
  cfg->device = 0;
  cfg->use_graph = 1;
  cfg->seed = 0;
  cfg->stream = nullptr;
  for (int k = 0; k < 3; ++k) cfg->velocity[k] = 0.0;
  cfg->alpha_l = 0.0;
  cfg->alpha_t = 0.0;
}

rwpt_status rwpt_create(const rwpt_config* cfg, rwpt_ctx** out) {
  if (!out) return fail(nullptr, RWPT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, RWPT_EINVAL, "cfg is NULL");
  const rwpt_config& c = *cfg;
  rwpt_status st = check_config(c);
  if (st != RWPT_OK) return st;
  rwpt_ctx* ctx = new (std::nothrow) rwpt_ctx();
  if (!ctx) return fail(nullptr, RWPT_ENOMEM, "out of host memory");
  ctx->cfg = c;
  ctx->S = c.n_species;
  ctx->dim = c.dim;
  ctx->tsize = c.precision == RWPT_FP64 ? 8 : 4;
  *out = ctx;
  return RWPT_OK;
}

static double neumaier_sum(const std::vector<double>& v) {
  double s = 0.0, comp = 0.0;
  for (double x : v) {
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) comp += (s - t) + x;
    else comp += (x - t) + s;
    s = t;
  }
  return s + comp;
}

rwpt_status rwpt_init_ensemble(rwpt_ctx* c, int32_t n_real, const int64_t* n_per_real, const double* pos,
                               const double* mass, const double* d_scale) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (n_real < 1) return fail(c, RWPT_EINVAL, "n_real must be >= 1");
  if (!n_per_real) return fail(c, RWPT_EINVAL, "n_per_real is NULL");
  int64_t N = 0;
  for (int r = 0; r < n_real; ++r) {
    if (n_per_real[r] < 0) return fail(c, RWPT_EINVAL, "n_per_real[%d] < 0", r);
    N += n_per_real[r];
    if (N > (int64_t)INT32_MAX - 64) return fail(c, RWPT_EINVAL, "too many particles");
  }
  const int dim = c->dim, S = c->S;
  if (N > 0 && (!pos || !mass)) return fail(c, RWPT_EINVAL, "pos/mass is NULL");
  for (int64_t i = 0; i < N; ++i)
    for (int k = 0; k < dim; ++k) {
      const double v = pos[i * dim + k];
      if (!std::isfinite(v) || v < c->cfg.box_lo[k] || v > c->cfg.box_hi[k])
        return fail(c, RWPT_EINVAL, "position of particle %lld axis %d (%g) is outside the box or not finite",
                    (long long)i, k, v);
    }
  for (int64_t i = 0; i < N * S; ++i)
    if (!std::isfinite(mass[i])) return fail(c, RWPT_EINVAL, "mass entry %lld is not finite", (long long)i);
  if (d_scale)
    for (int r = 0; r < n_real; ++r)
      if (!std::isfinite(d_scale[r]) || d_scale[r] < 0.0)
        return fail(c, RWPT_EINVAL, "d_scale[%d] must be finite and >= 0", r);
  rwpt_status st = ensure_device(c);
  if (st != RWPT_OK) return st;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  invalidate_graphs(c);
  c->initialized = false;
  c->grid_valid = false;
  c->sorted_valid = false;
  c->N = N;
  c->n_real = n_real;
  c->real_start.assign(n_real + 1, 0);
  for (int r = 0; r < n_real; ++r) c->real_start[r + 1] = c->real_start[r] + n_per_real[r];
  c->d_scale.assign(n_real, 1.0);
  if (d_scale)
    for (int r = 0; r < n_real; ++r) c->d_scale[r] = d_scale[r];
  // full-matrix path on matrix cores: one realisation, binary32, kappa = inf
  const bool dense_ok = std::isinf(c->cfg.kappa) && c->cfg.precision == RWPT_FP32 && n_real == 1 &&
                        N <= kDenseMaxN;
  if (c->cfg.path == RWPT_PATH_DENSE && !dense_ok)
    return fail(c, RWPT_EUNSUPPORTED, "the dense path needs one realisation of at most %lld particles",
                (long long)kDenseMaxN);
  c->dense = dense_ok && c->cfg.path != RWPT_PATH_SPARSE;
  c->cap = std::max<int64_t>(64, (N + 63) / 64 * 64);
  const size_t ts = c->tsize, cap = (size_t)c->cap;
  const int PS = dim;  // position slots per particle (particle-major, packed)
  HIPCHK(c, c->pos0.ensure(PS * cap * ts));
  HIPCHK(c, c->pos1.ensure(PS * cap * ts));
  const int Sa = padded_species(S);  // species slots per particle
  HIPCHK(c, c->mass0.ensure(Sa * cap * ts));
  HIPCHK(c, c->mass1.ensure(Sa * cap * ts));
  // unused species slots stay zero for the lifetime of the ensemble
  HIPCHK(c, hipMemsetAsync(c->mass0.p, 0, Sa * cap * ts, c->stream));
  HIPCHK(c, hipMemsetAsync(c->mass1.p, 0, Sa * cap * ts, c->stream));
  c->mcur = 0;  // the loaded masses go to mass0
  HIPCHK(c, c->src_of.ensure(cap * 4));
  HIPCHK(c, c->id.ensure(cap * 4));
  HIPCHK(c, c->key.ensure(cap * 4));
  HIPCHK(c, c->slot.ensure(cap * 4));
  HIPCHK(c, c->tmp_src.ensure(cap * 4));
  HIPCHK(c, c->tmp_id.ensure(cap * 4));
  HIPCHK(c, c->tmp_key.ensure(cap * 4));
  HIPCHK(c, c->skey.ensure(cap * 4));
  HIPCHK(c, c->r.ensure(cap * 8));
  HIPCHK(c, c->q.ensure(cap * ts));
  HIPCHK(c, c->d_real_start.ensure((n_real + 1) * sizeof(int64_t)));
  HIPCHK(c, c->audit_out.ensure((size_t)n_real * (S + 1) * sizeof(double)));
  // completion counters of the audit kernel (one per realisation)
  HIPCHK(c, c->audit_done.ensure((size_t)n_real * sizeof(uint32_t)));
  HIPCHK(c, hipMemsetAsync(c->audit_done.p, 0, (size_t)n_real * sizeof(uint32_t), c->stream));

  // host staging: particle-major in the path's precision
  std::vector<unsigned char> hp(PS * cap * ts, 0), hm(Sa * cap * ts, 0);
  std::vector<uint32_t> hid(cap, 0);
  c->audit_init.assign((size_t)n_real * (S + 1), 0.0);
  std::vector<double> rounded_mass((size_t)N * S);
  for (int64_t i = 0; i < N; ++i) {
    hid[i] = (uint32_t)i;
    for (int k = 0; k < dim; ++k) {
      const double v = pos[i * dim + k];
      if (ts == 8) ((double*)hp.data())[PS * i + k] = v;
      else ((float*)hp.data())[PS * i + k] = (float)v;
    }
    for (int s = 0; s < S; ++s) {
      const double v = mass[(size_t)s * N + i];
      double vr;
      if (ts == 8) {
        ((double*)hm.data())[Sa * i + s] = v;
        vr = v;
      } else {
        const float f = (float)v;
        ((float*)hm.data())[Sa * i + s] = f;
        vr = (double)f;
      }
      rounded_mass[(size_t)s * N + i] = vr;
    }
  }
  for (int r = 0; r < n_real; ++r) {
    const int64_t b = c->real_start[r], e = c->real_start[r + 1];
    std::vector<double> acc;
    for (int s = 0; s < S; ++s) {
      acc.assign(rounded_mass.begin() + (size_t)s * N + b, rounded_mass.begin() + (size_t)s * N + e);
      c->audit_init[(size_t)r * (S + 1) + s] = neumaier_sum(acc);
    }
    if (c->cfg.react_a >= 0) {
      acc.clear();
      for (int64_t i = b; i < e; ++i) {
        acc.push_back(rounded_mass[(size_t)c->cfg.react_a * N + i]);
        acc.push_back(-rounded_mass[(size_t)c->cfg.react_b * N + i]);
      }
      c->audit_init[(size_t)r * (S + 1) + S] = neumaier_sum(acc);
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->pos0.p, hp.data(), hp.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->mass0.p, hm.data(), hm.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->id.p, hid.data(), cap * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_real_start.p, c->real_start.data(), (n_real + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, c->stream));
  // realisation of the first particle of every block of the walk launch
  // (realisations keep their sizes and stay contiguous through every sort)
  const int64_t nblk = (N + kBlock - 1) / kBlock;
  std::vector<int32_t> blk_real((size_t)std::max<int64_t>(1, nblk), 0);
  for (int64_t b = 0, rr = 0; b < nblk; ++b) {
    while (rr + 1 < n_real && c->real_start[rr + 1] <= b * kBlock) ++rr;
    blk_real[b] = (int32_t)rr;
  }
  HIPCHK(c, c->d_blk_real.ensure(blk_real.size() * sizeof(int32_t)));
  HIPCHK(c, hipMemcpyAsync(c->d_blk_real.p, blk_real.data(), blk_real.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->step_ctr.p, 0, sizeof(uint64_t), c->stream));
  HIPCHK(c, hipMemcpyAsync(c->audit_out.p, c->audit_init.data(), c->audit_init.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->steps = 0;
  c->initialized = true;
  return RWPT_OK;
}

rwpt_status rwpt_init_ensemble_device(rwpt_ctx* c, int32_t n_real, const int64_t* n_per_real,
                                      const double* pos_dev, const double* mass_dev, const double* d_scale) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (n_real < 1) return fail(c, RWPT_EINVAL, "n_real must be >= 1");
  if (!n_per_real) return fail(c, RWPT_EINVAL, "n_per_real is NULL");
  int64_t N = 0;
  for (int r = 0; r < n_real; ++r) {
    if (n_per_real[r] < 0) return fail(c, RWPT_EINVAL, "n_per_real[%d] < 0", r);
    N += n_per_real[r];
    if (N > (int64_t)INT32_MAX - 64) return fail(c, RWPT_EINVAL, "too many particles");
  }
  if (N > 0 && (!pos_dev || !mass_dev)) return fail(c, RWPT_EINVAL, "pos/mass is NULL");
  rwpt_status st = ensure_device(c);
  if (st != RWPT_OK) return st;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  std::vector<double> hp((size_t)N * c->dim), hm((size_t)N * c->S);
  if (N > 0) {
    HIPCHK(c, hipMemcpyAsync(hp.data(), pos_dev, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(hm.data(), mass_dev, hm.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return rwpt_init_ensemble(c, n_real, n_per_real, hp.data(), hm.data(), d_scale);
}

rwpt_status rwpt_step(rwpt_ctx* c, double dt, double D, int32_t n_steps) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!std::isfinite(dt) || dt <= 0.0) return fail(c, RWPT_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(D) || D < 0.0) return fail(c, RWPT_EINVAL, "D must be finite and >= 0");
  if (n_steps < 0) return fail(c, RWPT_EINVAL, "n_steps must be >= 0");
  if (!c->initialized) return fail(c, RWPT_ESTATE, "rwpt_step before rwpt_init_ensemble");
  if (n_steps == 0) return RWPT_OK;
  if (c->N == 0) {
    c->steps += n_steps;
    return RWPT_OK;
  }
  HIPCHK(c, hipSetDevice(c->cfg.device));
  rwpt_status st = build_grid(c, dt, D);
  if (st != RWPT_OK) return st;
  bool advect = false;
  for (int k = 0; k < c->dim; ++k) advect = advect || c->cfg.velocity[k] != 0.0;
  const bool walk = (c->cfg.rw_ratio > 0.0 && D > 0.0) || advect;
  for (int32_t it = 0; it < n_steps; ++it) {
    const bool sort = walk || !c->sorted_valid;
    if (c->cfg.use_graph && !c->prof) {
      // a captured step bakes in the buffers of the mass parity it starts from
      const int m0 = c->mcur;
      hipGraphExec_t& gx = c->gx[2 * (sort ? 0 : 1) + m0];
      if (!gx) {
        hipGraph_t g = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        rwpt_status s2 = enqueue_step(c, sort, walk);
        hipError_t ec = hipStreamEndCapture(c->stream, &g);
        c->mcur = m0;  // capture records the step; it runs at the launch below
        if (s2 != RWPT_OK) {
          if (g) (void)hipGraphDestroy(g);
          return s2;
        }
        HIPCHK(c, ec);
        hipError_t ei = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(c, ei);
        ++c->n_captures;
      }
      HIPCHK(c, hipGraphLaunch(gx, c->stream));
      c->mcur = m0 ^ step_flips(c, sort);
    } else {
      st = enqueue_step(c, sort, walk);
      if (st != RWPT_OK) return st;
    }
    c->sorted_valid = true;
    c->steps += 1;
  }
  return RWPT_OK;
}

rwpt_status rwpt_sync(rwpt_ctx* c) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  if (!c->device_ready) return RWPT_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RWPT_OK;
}

// Copy `comps` components per particle (particle-major, `stride` slots per
// particle on the device) back to the caller's order.
static rwpt_status fetch_sorted(rwpt_ctx* c, const DevBuf& buf, int comps, int stride, double* out,
                                bool species_major) {
  const int64_t N = c->N;
  if (N == 0) return RWPT_OK;
  const size_t ts = c->tsize, cap = (size_t)c->cap;
  std::vector<unsigned char> h(stride * cap * ts);
  std::vector<uint32_t> hid(N);
  HIPCHK(c, hipMemcpyAsync(h.data(), buf.p, h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(hid.data(), c->id.p, N * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t p = 0; p < N; ++p) {
    const uint32_t o = hid[p];
    if ((int64_t)o >= N) return fail(c, RWPT_EDEVICE, "corrupt id map");
    for (int k = 0; k < comps; ++k) {
      const size_t e = (size_t)stride * p + k;
      const double v = ts == 8 ? ((const double*)h.data())[e] : (double)((const float*)h.data())[e];
      if (species_major) out[(size_t)k * N + o] = v;
      else out[(size_t)o * comps + k] = v;
    }
  }
  return RWPT_OK;
}

rwpt_status rwpt_query_masses(rwpt_ctx* c, double* out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!c->initialized) return fail(c, RWPT_ESTATE, "query before rwpt_init_ensemble");
  if (!out && c->N > 0) return fail(c, RWPT_EINVAL, "out is NULL");
  return fetch_sorted(c, mass_buf(c, c->mcur), c->S, padded_species(c->S), out, true);
}

rwpt_status rwpt_query_positions(rwpt_ctx* c, double* out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!c->initialized) return fail(c, RWPT_ESTATE, "query before rwpt_init_ensemble");
  if (!out && c->N > 0) return fail(c, RWPT_EINVAL, "out is NULL");
  return fetch_sorted(c, c->pos0, c->dim, c->dim, out, false);
}

rwpt_status rwpt_audit(rwpt_ctx* c, double* out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!c->initialized) return fail(c, RWPT_ESTATE, "audit before rwpt_init_ensemble");
  if (!out) return fail(c, RWPT_EINVAL, "out is NULL");
  const size_t n = (size_t)c->n_real * (c->S + 1);
  if (c->steps == 0 || c->N == 0) {
    memcpy(out, c->audit_init.data(), n * sizeof(double));
    return RWPT_OK;
  }
  HIPCHK(c, hipMemcpyAsync(out, c->audit_out.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RWPT_OK;
}

rwpt_status rwpt_steps_taken(rwpt_ctx* c, int64_t* out) {
  if (!c || !out) return fail(c, RWPT_EINVAL, "NULL argument");
  *out = c->steps;
  return RWPT_OK;
}

rwpt_status rwpt_count_pairs(rwpt_ctx* c, double dt, double D, int64_t* pairs_out, int64_t* evals_out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!pairs_out) return fail(c, RWPT_EINVAL, "pairs_out is NULL");
  if (!std::isfinite(dt) || dt <= 0.0 || !std::isfinite(D) || D < 0.0)
    return fail(c, RWPT_EINVAL, "dt must be > 0 and D >= 0");
  if (!c->initialized) return fail(c, RWPT_ESTATE, "count before rwpt_init_ensemble");
  *pairs_out = 0;
  if (evals_out) *evals_out = 0;
  if (c->N == 0) return RWPT_OK;
  if (c->dense) {
    // the full-matrix path evaluates every ordered pair of the realisation
    const int64_t n = c->N;
    *pairs_out = D > 0.0 ? n * (n - 1) : 0;
    if (evals_out) *evals_out = D > 0.0 ? n * n : 0;
    return RWPT_OK;
  }
  rwpt_status st = build_grid(c, dt, D);
  if (st != RWPT_OK) return st;
  st = ensure_sorted(c);
  if (st != RWPT_OK) return st;
  PairArgs a = pair_args(c);
  {
    PhaseScope ps(c, PH_COUNT);
    HIPCHK(c, launch_count(c->cfg.precision == RWPT_FP64, c->dim, c->log2l, a, c->stream));
  }
  std::vector<unsigned long long> h((size_t)c->ntiles * 2);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->counts.p, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  unsigned long long p = 0, e = 0;
  for (int32_t t = 0; t < c->ntiles; ++t) {
    p += h[2 * t];
    e += h[2 * t + 1];
  }
  *pairs_out = (int64_t)p;
  if (evals_out) *evals_out = (int64_t)e;
  return RWPT_OK;
}

rwpt_status rwpt_neighbors(rwpt_ctx* c, double dt, double D, int64_t* rowptr, int32_t* cols, int64_t* nnz_out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!nnz_out) return fail(c, RWPT_EINVAL, "nnz_out is NULL");
  if (!std::isfinite(dt) || dt <= 0.0 || !std::isfinite(D) || D < 0.0)
    return fail(c, RWPT_EINVAL, "dt must be > 0 and D >= 0");
  if (!c->initialized) return fail(c, RWPT_ESTATE, "neighbors before rwpt_init_ensemble");
  const int64_t N = c->N;
  if (N == 0) {
    *nnz_out = 0;
    if (rowptr) rowptr[0] = 0;
    return RWPT_OK;
  }
  if (c->dense) return fail(c, RWPT_EUNSUPPORTED, "the full-matrix path has no neighbour lists (every pair)");
  rwpt_status st = build_grid(c, dt, D);
  if (st != RWPT_OK) return st;
  st = ensure_sorted(c);
  if (st != RWPT_OK) return st;
  const int fp64 = c->cfg.precision == RWPT_FP64;
  DevBuf cursor, rp, pairs;
  HIPCHK(c, cursor.ensure((size_t)c->cap * 4));
  HIPCHK(c, hipMemsetAsync(cursor.p, 0, (size_t)c->cap * 4, c->stream));
  PairArgs a = pair_args(c);
  a.nbr_cursor = cursor.as<uint32_t>();
  rwpt_status result = RWPT_OK;
  do {
    hipError_t e = launch_nbr_count(fp64, c->dim, c->log2l, a, c->stream);
    if (e != hipSuccess) { result = fail(c, RWPT_EDEVICE, "nbr count: %s", hipGetErrorString(e)); break; }
    std::vector<uint32_t> cnt(N);
    e = hipMemcpyAsync(cnt.data(), cursor.p, N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { result = fail(c, RWPT_EDEVICE, "nbr copy: %s", hipGetErrorString(e)); break; }
    std::vector<unsigned long long> off(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) off[i + 1] = off[i] + cnt[i];
    const int64_t nnz = (int64_t)off[N];
    *nnz_out = nnz;
    if (!cols || !rowptr) break;
    if (hipMemsetAsync(cursor.p, 0, (size_t)c->cap * 4, c->stream) != hipSuccess ||
        rp.ensure((N + 1) * 8) != hipSuccess || pairs.ensure((size_t)std::max<int64_t>(1, nnz) * 8) != hipSuccess) {
      result = fail(c, RWPT_ENOMEM, "neighbour export buffers");
      break;
    }
    e = hipMemcpyAsync(rp.p, off.data(), (N + 1) * 8, hipMemcpyHostToDevice, c->stream);
    a.nbr_rowptr = rp.as<unsigned long long>();
    a.nbr_pairs = pairs.as<uint32_t>();
    if (e == hipSuccess) e = launch_nbr_fill(fp64, c->dim, c->log2l, a, c->stream);
    std::vector<uint32_t> hp((size_t)nnz * 2);
    std::vector<uint32_t> hid(N);
    if (e == hipSuccess && nnz) e = hipMemcpyAsync(hp.data(), pairs.p, (size_t)nnz * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hid.data(), c->id.p, N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { result = fail(c, RWPT_EDEVICE, "nbr fill: %s", hipGetErrorString(e)); break; }
    // convert to the caller's order: rows by original id, ascending columns
    std::vector<int64_t> rc(N + 1, 0);
    for (int64_t p = 0; p < N; ++p) rc[hid[p] + 1] = cnt[p];
    for (int64_t i = 0; i < N; ++i) rc[i + 1] += rc[i];
    for (int64_t i = 0; i <= N; ++i) rowptr[i] = rc[i];
    std::vector<int64_t> fillpos(rc.begin(), rc.end() - 1);
    for (int64_t t = 0; t < nnz; ++t) {
      const uint32_t oi = hid[hp[2 * t]], oj = hid[hp[2 * t + 1]];
      cols[fillpos[oi]++] = (int32_t)oj;
    }
    for (int64_t i = 0; i < N; ++i) std::sort(cols + rc[i], cols + rc[i + 1]);
  } while (0);
  cursor.release();
  rp.release();
  pairs.release();
  return result;
}

rwpt_status rwpt_debug_rowsums(rwpt_ctx* c, double dt, double D, int32_t unit_weights, double* r_out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!std::isfinite(dt) || dt <= 0.0 || !std::isfinite(D) || D < 0.0)
    return fail(c, RWPT_EINVAL, "dt must be > 0 and D >= 0");
  if (unit_weights != 0 && unit_weights != 1) return fail(c, RWPT_EINVAL, "unit_weights must be 0 or 1");
  if (!c->initialized) return fail(c, RWPT_ESTATE, "debug_rowsums before rwpt_init_ensemble");
  const int64_t N = c->N;
  if (N > 0 && !r_out) return fail(c, RWPT_EINVAL, "r_out is NULL");
  if (N == 0) return RWPT_OK;
  if (c->dense) return fail(c, RWPT_EUNSUPPORTED, "the full-matrix path has no sparse row-sum pass");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  rwpt_status st = build_grid(c, dt, D);
  if (st != RWPT_OK) return st;
  st = ensure_sorted(c);
  if (st != RWPT_OK) return st;
  PairArgs a = pair_args(c);
  a.r_out = c->r.as<double>();
  DevBuf rp_unit;
  rwpt_status result = RWPT_OK;
  do {
    if (unit_weights) {
      // every weight exp(0) = 1: r_i counts the neighbours within the cutoff
      std::vector<RealParams> h = c->h_rp;
      for (RealParams& P : h) {
        P.escale_d = 0.0;
        P.escale_f = 0.0f;
      }
      hipError_t e = rp_unit.ensure(h.size() * sizeof(RealParams));
      if (e == hipSuccess)
        e = hipMemcpyAsync(rp_unit.p, h.data(), h.size() * sizeof(RealParams), hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        result = fail(c, RWPT_EDEVICE, "debug_rowsums parameters: %s", hipGetErrorString(e));
        break;
      }
      a.rp = rp_unit.as<RealParams>();
    }
    hipError_t e = launch_rowsum(c->cfg.precision == RWPT_FP64, c->dim, c->log2l, a, c->stream);
    std::vector<double> hr(N);
    std::vector<uint32_t> hid(N);
    if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), c->r.p, N * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hid.data(), c->id.p, N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      result = fail(c, RWPT_EDEVICE, "debug_rowsums: %s", hipGetErrorString(e));
      break;
    }
    for (int64_t p = 0; p < N; ++p) {
      if ((int64_t)hid[p] >= N) {
        result = fail(c, RWPT_EDEVICE, "corrupt id map");
        break;
      }
      r_out[hid[p]] = hr[p];
    }
  } while (0);
  rp_unit.release();
  return result;
}

rwpt_status rwpt_profile_enable(rwpt_ctx* c, int32_t on) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  if (!on && c->prof) drain_profile(c);
  c->prof = on != 0;
  return RWPT_OK;
}

rwpt_status rwpt_profile_reset(rwpt_ctx* c) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  drain_profile(c);
  for (int p = 0; p < PH_N; ++p) {
    c->prof_ms[p] = 0.0;
    c->prof_cnt[p] = 0;
  }
  return RWPT_OK;
}

rwpt_status rwpt_profile_read(rwpt_ctx* c, double* ms, int64_t* cnt, int32_t* n_phases) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  drain_profile(c);
  if (n_phases) *n_phases = PH_N;
  for (int p = 0; p < PH_N; ++p) {
    if (ms) ms[p] = c->prof_ms[p];
    if (cnt) cnt[p] = c->prof_cnt[p];
  }
  return RWPT_OK;
}

const char* rwpt_profile_phase_name(int32_t phase) {
  if (phase < 0 || phase >= PH_N) return "";
  return kPhaseNames[phase];
}

rwpt_status rwpt_stats(rwpt_ctx* c, rwpt_stats_t* out) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!out) return fail(c, RWPT_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  out->n_particles = c->initialized ? c->N : 0;
  out->n_real = c->initialized ? c->n_real : 0;
  out->ordered_pairs = -1;
  out->candidate_evals = -1;
  if (c->initialized) {
    rwpt_status st = rwpt_steps_taken(c, &out->steps_taken);
    if (st != RWPT_OK) return st;
  }
  if (c->initialized && c->grid_valid) {
    out->tile_lanes = c->log2l == kPrivateLists ? -1 : (c->log2l == kHalfPairs ? -2 : (1 << c->log2l));
    for (int k = 0; k < 3; ++k) out->cell_refine[k] = c->refine[k];
    out->n_cells = c->ncell_total;
    int64_t pairs = 0, evals = 0;
    rwpt_status st = rwpt_count_pairs(c, c->g_dt, c->g_D, &pairs, &evals);
    if (st != RWPT_OK) return st;
    out->ordered_pairs = pairs;
    out->candidate_evals = evals;
  }
  int32_t np = 0;
  if (c->device_ready) {
    rwpt_status st = rwpt_profile_read(c, out->phase_ms, out->phase_launches, &np);
    if (st != RWPT_OK) return st;
  }
  out->n_phases = np;
  out->graph_captures = c->n_captures;
  return RWPT_OK;
}

// Timed launches of one probe kernel: one untimed launch, then `timed`
// launches between two events on the context's stream.
static hipError_t probe_time(rwpt_ctx* c, int kind, int blocks, int reps, int timed, float* out, float* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  // cutoff 1 on the probe's lattice of spacing 1/8 in [0, 2); weight exp(-s^2)
  const float rc2 = 1.0f, esc = -1.4426950408889634f, h = 1.0f;
  const int slots = species_slots(c->cfg.n_species);
  if (e == hipSuccess) e = launch_probe(kind, c->dim, slots, blocks, reps, rc2, esc, h, out, c->stream);
  if (e == hipSuccess) e = hipEventRecord(a, c->stream);
  for (int t = 0; t < timed && e == hipSuccess; ++t)
    e = launch_probe(kind, c->dim, slots, blocks, reps, rc2, esc, h, out, c->stream);
  if (e == hipSuccess) e = hipEventRecord(b, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return e;
}

rwpt_status rwpt_probe_rate(rwpt_ctx* c, int32_t kind, double* per_s) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!per_s) return fail(c, RWPT_EINVAL, "per_s is NULL");
  if (kind < PROBE_FMA || kind > PROBE_EXCHANGE) return fail(c, RWPT_EINVAL, "probe kind %d not in 0..3", kind);
  rwpt_status st = ensure_device(c);
  if (st != RWPT_OK) return st;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  int cus = 0;
  HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->cfg.device));
  const int blocks = (cus > 0 ? cus : 1) * 8;  // 8 blocks of 4 waves per CU: 8 waves per SIMD
  const int reps = (kind == PROBE_FMA || kind == PROBE_EXP) ? 500 : 1000;
  const int timed = 3;
  DevBuf out;
  hipError_t e = out.ensure((size_t)blocks * probe_block() * sizeof(float));
  float ms = 0.0f;
  if (e == hipSuccess) e = probe_time(c, kind, blocks, reps, timed, out.as<float>(), &ms);
  out.release();
  HIPCHK(c, e);
  if (!(ms > 0.0f)) return fail(c, RWPT_EDEVICE, "probe kind %d: non-positive elapsed time", kind);
  *per_s = (double)blocks * probe_block() * (double)probe_ops_per_lane(kind, reps) * timed / (ms * 1e-3);
  return RWPT_OK;
}

rwpt_status rwpt_get_tiling(rwpt_ctx* c, int32_t* tile_lanes, double* cell_refine3) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  int lanes = c->cfg.tile_lanes ? c->cfg.tile_lanes : default_lanes(c->dim, c->N, c->cfg.precision == RWPT_FP64);
  double defr[3];
  default_refine(c->dim, defr);
  if (tile_lanes) *tile_lanes = lanes;
  if (cell_refine3)
    for (int k = 0; k < 3; ++k) cell_refine3[k] = c->cfg.cell_refine[k] > 0 ? c->cfg.cell_refine[k] : defr[k];
  return RWPT_OK;
}

// Candidate tilings per dimension: lanes per particle x cells per cutoff.
static std::vector<std::pair<int, std::array<double, 3>>> tuning_candidates(int dim, bool fp64) {
  std::vector<std::array<double, 3>> refs;
  if (dim == 1) refs = {{4, 1, 1}, {8, 1, 1}, {16, 1, 1}, {32, 1, 1}};
  else if (dim == 2) refs = {{8, 1, 1}, {16, 1, 1}, {4, 2, 1}, {8, 2, 1}, {8, 3, 1}, {16, 3, 1}, {8, 4, 1}};
  else refs = {{0.5, 0.5, 0.5}, {1, 0.5, 0.5}, {2, 1, 1}, {4, 1, 1}, {8, 1, 1}, {4, 2, 2}, {8, 0.5, 0.5}};
  std::vector<std::pair<int, std::array<double, 3>>> out;
  for (int lanes : {-2, -1, 1, 4, 8, 16})
    if (lanes != -2 || !fp64)
      for (auto& r : refs) out.push_back({lanes, r});
  return out;
}

// Everything that shapes the cell grids and the work of the pair kernels:
// sizes, species, (dt, D), cutoff, precision, normalisation, walk share, the
// box, the velocity and dispersivities, and the realisation sizes and D
// scales (FNV-1a hash of their bits).
static std::string tuning_key(const rwpt_ctx* c, double dt, double D) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t k = 0; k < n; ++k) {
      h ^= b[k];
      h *= 1099511628211ull;
    }
  };
  mix(c->real_start.data(), c->real_start.size() * sizeof(int64_t));
  mix(c->d_scale.data(), c->d_scale.size() * sizeof(double));
  char buf[512];
  snprintf(buf, sizeof(buf),
           "dim=%d N=%lld S=%d nreal=%d D=%.6g dt=%.6g kappa=%.6g prec=%d norm=%d rw=%.6g "
           "box=%.6g,%.6g,%.6g:%.6g,%.6g,%.6g v=%.6g,%.6g,%.6g aL=%.6g aT=%.6g real=%016llx",
           c->dim, (long long)c->N, c->S, c->n_real, D, dt, c->cfg.kappa, c->cfg.precision, c->cfg.norm,
           c->cfg.rw_ratio, c->cfg.box_lo[0], c->cfg.box_lo[1], c->cfg.box_lo[2], c->cfg.box_hi[0],
           c->cfg.box_hi[1], c->cfg.box_hi[2], c->cfg.velocity[0], c->cfg.velocity[1], c->cfg.velocity[2],
           c->cfg.alpha_l, c->cfg.alpha_t, (unsigned long long)h);
  return buf;
}

static bool tuning_cache_lookup(const std::string& key, int* lanes, double ref[3]) {
  const char* path = getenv("RWPT_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char* bar = strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    if (key == line) {
      int l;
      double r0, r1, r2;
      if (sscanf(bar + 1, "%d %lf %lf %lf", &l, &r0, &r1, &r2) == 4 && lanes_to_log2(l) != -2) {
        *lanes = l;
        ref[0] = r0;
        ref[1] = r1;
        ref[2] = r2;
        found = true;
      }
    }
  }
  fclose(f);
  return found;
}

static void tuning_cache_store(const std::string& key, int lanes, const double ref[3]) {
  const char* path = getenv("RWPT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s|%d %.17g %.17g %.17g\n", key.c_str(), lanes, ref[0], ref[1], ref[2]);
  fclose(f);
}

rwpt_status rwpt_autotune(rwpt_ctx* c, double dt, double D, int32_t trial_steps) {
  if (!c) return fail(nullptr, RWPT_EINVAL, "ctx is NULL");
  c->err.clear();
  if (!std::isfinite(dt) || dt <= 0.0 || !std::isfinite(D) || D < 0.0)
    return fail(c, RWPT_EINVAL, "dt must be > 0 and D >= 0");
  if (trial_steps < 1 || trial_steps > 1000) return fail(c, RWPT_EINVAL, "trial_steps must be in 1..1000");
  if (!c->initialized) return fail(c, RWPT_ESTATE, "autotune before rwpt_init_ensemble");
  if (c->N == 0 || c->dense) return RWPT_OK;
  const std::string key = tuning_key(c, dt, D);
  int best_lanes = 0;
  double best_ref[3] = {0, 0, 0};
  if (tuning_cache_lookup(key, &best_lanes, best_ref)) {
    c->cfg.tile_lanes = best_lanes;
    for (int k = 0; k < 3; ++k) c->cfg.cell_refine[k] = best_ref[k];
    c->grid_valid = false;
    c->sorted_valid = false;
    invalidate_graphs(c);
    return RWPT_OK;
  }
  HIPCHK(c, hipSetDevice(c->cfg.device));
  // snapshot of the state the tuning steps will overwrite
  const size_t ts = c->tsize, cap = (size_t)c->cap;
  const int Sa = padded_species(c->S);
  const size_t npos = c->dim * cap * ts, nmass = Sa * cap * ts, naud = (size_t)c->n_real * (c->S + 1) * 8;
  DevBuf sp, sm, si, sa, sc;
  rwpt_status result = RWPT_OK;
  const rwpt_config saved_cfg = c->cfg;
  const int64_t saved_steps = c->steps;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  do {
    if (sp.ensure(npos) != hipSuccess || sm.ensure(nmass) != hipSuccess || si.ensure(cap * 4) != hipSuccess ||
        sa.ensure(naud) != hipSuccess || sc.ensure(8) != hipSuccess) {
      result = fail(c, RWPT_ENOMEM, "autotune snapshot");
      break;
    }
    hipError_t e = hipMemcpyAsync(sp.p, c->pos0.p, npos, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sm.p, mass_buf(c, c->mcur).p, nmass, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(si.p, c->id.p, cap * 4, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sa.p, c->audit_out.p, naud, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.p, c->step_ctr.p, 8, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      result = fail(c, RWPT_EDEVICE, "autotune setup: %s", hipGetErrorString(e));
      break;
    }
    auto restore = [&]() -> hipError_t {
      hipError_t r = hipMemcpyAsync(c->pos0.p, sp.p, npos, hipMemcpyDeviceToDevice, c->stream);
      if (r == hipSuccess) r = hipMemcpyAsync(c->mass0.p, sm.p, nmass, hipMemcpyDeviceToDevice, c->stream);
      c->mcur = 0;
      if (r == hipSuccess) r = hipMemcpyAsync(c->id.p, si.p, cap * 4, hipMemcpyDeviceToDevice, c->stream);
      if (r == hipSuccess) r = hipMemcpyAsync(c->audit_out.p, sa.p, naud, hipMemcpyDeviceToDevice, c->stream);
      if (r == hipSuccess) r = hipMemcpyAsync(c->step_ctr.p, sc.p, 8, hipMemcpyDeviceToDevice, c->stream);
      c->steps = saved_steps;
      c->grid_valid = false;
      c->sorted_valid = false;
      invalidate_graphs(c);
      return r;
    };
    float best_ms = INFINITY;
    const bool was_prof = c->prof;
    c->prof = false;
    for (auto& cand : tuning_candidates(c->dim, c->cfg.precision == RWPT_FP64)) {
      c->cfg.tile_lanes = cand.first;
      for (int k = 0; k < 3; ++k) c->cfg.cell_refine[k] = cand.second[k];
      if (restore() != hipSuccess) {
        result = fail(c, RWPT_EDEVICE, "autotune restore");
        break;
      }
      // untimed warm-up: builds the grid, sorts and captures the step graphs.
      // A step's graph depends on the mass buffer it starts from, which
      // alternates when the step flips it once (a sort that leaves the masses
      // in place, or a step without a sort); three steps capture every graph
      // the timed steps replay, so no capture falls inside the timed window.
      const int warm = c->cfg.use_graph ? 3 : 1;
      rwpt_status st = rwpt_step(c, dt, D, warm);
      if (st == RWPT_EUNSUPPORTED) {
        c->err.clear();  // e.g. a grid too large for this candidate: skip it
        continue;
      }
      if (st != RWPT_OK) {
        result = st;
        break;
      }
      e = hipEventRecord(e0, c->stream);
      st = rwpt_step(c, dt, D, trial_steps);
      if (st != RWPT_OK) {
        result = st;
        break;
      }
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        result = fail(c, RWPT_EDEVICE, "autotune timing: %s", hipGetErrorString(e));
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best_lanes = cand.first;
        for (int k = 0; k < 3; ++k) best_ref[k] = cand.second[k];
      }
    }
    c->prof = was_prof;
    if (result != RWPT_OK) break;
    if (!(best_ms < INFINITY)) {
      result = fail(c, RWPT_EUNSUPPORTED, "autotune: no candidate tiling is supported for this ensemble");
      break;
    }
    c->cfg.tile_lanes = best_lanes;
    for (int k = 0; k < 3; ++k) c->cfg.cell_refine[k] = best_ref[k];
    if (restore() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
      result = fail(c, RWPT_EDEVICE, "autotune final restore");
      break;
    }
    tuning_cache_store(key, best_lanes, best_ref);
  } while (0);
  if (result != RWPT_OK) {
    // leave the context usable with the caller's original tiling and state
    c->cfg = saved_cfg;
    if (sp.p && sm.p && si.p && sa.p && sc.p) {
      (void)hipMemcpyAsync(c->pos0.p, sp.p, npos, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(c->mass0.p, sm.p, nmass, hipMemcpyDeviceToDevice, c->stream);
      c->mcur = 0;
      (void)hipMemcpyAsync(c->id.p, si.p, cap * 4, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(c->audit_out.p, sa.p, naud, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(c->step_ctr.p, sc.p, 8, hipMemcpyDeviceToDevice, c->stream);
    }
    c->steps = saved_steps;
    c->grid_valid = false;
    c->sorted_valid = false;
    invalidate_graphs(c);
  }
  (void)hipStreamSynchronize(c->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  sp.release();
  sm.release();
  si.release();
  sa.release();
  sc.release();
  return result;
}

rwpt_status rwpt_transfer_noalloc(const rwpt_config* cfg, int32_t n, const void* pos, const void* mass_in,
                                  void* mass_out, double dt, double D) {
  if (!cfg) return fail(nullptr, RWPT_EINVAL, "cfg is NULL");
  const rwpt_config& c = *cfg;
  rwpt_status st = check_config(c);
  if (st != RWPT_OK) return st;
  if (c.path == RWPT_PATH_DENSE)
    return fail(nullptr, RWPT_EUNSUPPORTED, "rwpt_transfer_noalloc runs the sparse path only");
  if (n < 0 || n > INT32_MAX - 64) return fail(nullptr, RWPT_EINVAL, "n must be in 0..2^31 - 65 (got %d)", n);
  if (!std::isfinite(dt) || dt <= 0.0) return fail(nullptr, RWPT_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(D) || D < 0.0) return fail(nullptr, RWPT_EINVAL, "D must be finite and >= 0");
  if (n > 0 && (!pos || !mass_in || !mass_out)) return fail(nullptr, RWPT_EINVAL, "pos/mass_in/mass_out is NULL");
  if (n > 0 && (mass_in == mass_out)) return fail(nullptr, RWPT_EINVAL, "mass_out may not alias mass_in");
  if (n == 0) return RWPT_OK;
  const int dim = c.dim, S = c.n_species;
  const int fp64 = c.precision == RWPT_FP64;
  const size_t ts = fp64 ? 8 : 4;
  const int lanes = c.tile_lanes ? c.tile_lanes : default_lanes(dim, n, fp64);
  if (lanes == -2)
    return fail(nullptr, RWPT_EUNSUPPORTED, "rwpt_transfer_noalloc does not take the half-stencil tiling");
  const int log2l = lanes_to_log2(lanes);
  const int G = log2l == kPrivateLists ? 64 : 64 >> log2l;
  double refine[3], defr[3];
  default_refine(dim, defr);
  for (int k = 0; k < 3; ++k) refine[k] = c.cell_refine[k] > 0 ? c.cell_refine[k] : defr[k];
  // grid of the realisation for (dt, D): parameters and stencil rows, kept in
  // kernel arguments
  NoAllocParams na;
  memset(&na, 0, sizeof(na));
  RowBuf rows{na.st, kNoAllocStencil, 0};
  float unused_escale = 0.0f, unused_skip = 0.0f;
  real_grid(c, dim, dt, D, n, refine, false, &unused_escale, &unused_skip, 0, na.P, rows);
  if (rows.n > kNoAllocStencil)
    return fail(nullptr, RWPT_EUNSUPPORTED, "the cutoff spans %d stencil rows; the allocation-free path takes at most %d",
                rows.n, kNoAllocStencil);
  na.n_st = rows.n;
  na.P.p_begin = 0;
  na.P.p_end = n;
  const int64_t ncell = (int64_t)na.P.nc[0] * na.P.nc[1] * na.P.nc[2];
  const int32_t ntiles = (int32_t)((n + G - 1) / G);
  const int64_t cap = (int64_t)(n + 63) / 64 * 64;
  const int PS = dim, Sa = padded_species(S);
  const int64_t nscan = (ncell + kScanChunk - 1) / kScanChunk + 1;
  // the pieces of the scratch area this call uses
  ScratchLayout L;
  const size_t o_pos0 = L.take(PS * cap * ts), o_pos1 = L.take(PS * cap * ts);
  const size_t o_m0 = L.take(Sa * cap * ts), o_m1 = L.take(Sa * cap * ts);
  const size_t o_id = L.take(cap * 4), o_key = L.take(cap * 4), o_slot = L.take(cap * 4);
  const size_t o_tsrc = L.take(cap * 4), o_tid = L.take(cap * 4), o_tkey = L.take(cap * 4);
  const size_t o_skey = L.take(cap * 4), o_r = L.take(cap * 8), o_q = L.take(cap * ts);
  const size_t o_cnt = L.take(ncell * 4), o_start = L.take((ncell + 1) * 4), o_scan = L.take(nscan * 4);
  const size_t o_rp = L.take(sizeof(RealParams)), o_st = L.take(kNoAllocStencil * sizeof(StencilRow));
  const size_t o_tiles = L.take((size_t)ntiles * sizeof(Tile));
  const size_t o_blk = L.take((size_t)((n + kBlock - 1) / kBlock) * 4), o_ctr = L.take(8);
  const size_t o_rs = L.take(2 * sizeof(int64_t));
  const size_t o_aud = L.take((size_t)ntiles * (S + 1) * 8);
  size_t o_meta = 0, o_nidx = 0, o_nw = 0, o_nsrc = 0;
  if (log2l == kPrivateLists) {
    o_meta = L.take(cap * 2);
    o_nidx = L.take((size_t)ntiles * kCacheWave * 4);
    o_nw = L.take((size_t)ntiles * kCacheWave * ts);
    o_nsrc = L.take((size_t)ntiles * kCacheWave * 4);
  }
  if (L.used > kScratchBytes)
    return fail(nullptr, RWPT_EUNSUPPORTED,
                "%d particles (dim %d, %d species, binary%d, %lld cells) need %zu bytes of scratch; "
                "the allocation-free path has %zu",
                n, dim, S, fp64 ? 64 : 32, (long long)ncell, L.used, kScratchBytes);
  void* base = nullptr;
  st = scratch_on_current_device(&base);
  if (st != RWPT_OK) return st;
  unsigned char* b = (unsigned char*)base;
  auto at = [&](size_t off) { return (void*)(b + off); };
  hipStream_t s = (hipStream_t)c.stream;
#define NACHK(expr)                                                                                 \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) {                                                                         \
      (void)hipGetLastError();                                                                      \
      return fail(nullptr, RWPT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));                   \
    }                                                                                               \
  } while (0)
  // set-up: parameters, stencil, tiles, ids, cleared counts, caller layouts
  NACHK(launch_noalloc_setup(fp64, dim, S, na, n, pos, mass_in, at(o_pos0), at(o_m0), (uint32_t*)at(o_id),
                             (Tile*)at(o_tiles), G, ntiles, (RealParams*)at(o_rp), (StencilRow*)at(o_st),
                             (int64_t*)at(o_rs), (int32_t*)at(o_blk), (uint32_t*)at(o_cnt), ncell, s));
  // cell keys (no walk), counting sort, canonical order with the masses moved
  NACHK(launch_walk_key(fp64, dim, at(o_pos0), at(o_pos1), (uint32_t*)at(o_id), n, (RealParams*)at(o_rp),
                        (int64_t*)at(o_rs), (int32_t*)at(o_blk), 1, (uint64_t*)at(o_ctr), c.seed, 0, (uint32_t*)at(o_cnt),
                        (uint32_t*)at(o_key), (uint32_t*)at(o_slot), s));
  NACHK(launch_cell_scan((uint32_t*)at(o_cnt), (uint32_t*)at(o_start), ncell, (uint32_t*)at(o_scan), s));
  NACHK(launch_scatter(n, (uint32_t*)at(o_key), (uint32_t*)at(o_slot), (uint32_t*)at(o_start), (uint32_t*)at(o_id),
                       (uint32_t*)at(o_tsrc), (uint32_t*)at(o_tid), (uint32_t*)at(o_tkey), s));
  NACHK(launch_canon(fp64, dim, n, (uint32_t*)at(o_tsrc), (uint32_t*)at(o_tid), (uint32_t*)at(o_tkey),
                     (uint32_t*)at(o_start), at(o_pos1), at(o_pos0), at(o_m0), at(o_m1), S, (uint32_t*)at(o_id),
                     (uint32_t*)at(o_skey), nullptr, s));
  // row sums, then the exchange + reaction into the other mass buffer
  PairArgs a;
  memset(&a, 0, sizeof(a));
  a.pos = at(o_pos0);
  a.mass_in = at(o_m1);
  a.mass_out = at(o_m0);
  a.q_in = at(o_q);
  a.q_out = at(o_q);
  a.r_out = (double*)at(o_r);
  a.skey = (uint32_t*)at(o_skey);
  a.cell_start = (uint32_t*)at(o_start);
  a.tiles = (Tile*)at(o_tiles);
  a.ntiles = ntiles;
  a.rp = (RealParams*)at(o_rp);
  a.st = (StencilRow*)at(o_st);
  a.S = S;
  a.react_a = c.react_a;
  a.react_b = c.react_b;
  a.norm = c.norm;
  a.audit_part = (double*)at(o_aud);
  if (log2l == kPrivateLists) {
    a.nb_meta = (uint16_t*)at(o_meta);
    a.nb_idx = (uint32_t*)at(o_nidx);
    a.nb_w = at(o_nw);
    a.nb_src = (uint32_t*)at(o_nsrc);
  }
  a.indirect = 0;
  if (c.norm == RWPT_NORM_SYM || log2l == kPrivateLists) NACHK(launch_rowsum(fp64, dim, log2l, a, s));
  NACHK(launch_exchange(fp64, dim, log2l, a, s));
  NACHK(launch_noalloc_store(fp64, S, n, at(o_m0), (uint32_t*)at(o_id), mass_out, s));
#undef NACHK
  return RWPT_OK;
}

const char* rwpt_last_error(const rwpt_ctx* c) {
  if (!c) return g_err.c_str();
  return c->err.c_str();
}

void rwpt_destroy(rwpt_ctx* c) {
  if (!c) return;
  if (c->device_ready) {
    (void)hipSetDevice(c->cfg.device);
    (void)hipStreamSynchronize(c->stream);
    drain_profile(c);
    invalidate_graphs(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    DevBuf* bufs[] = {&c->pos0, &c->pos1, &c->mass0, &c->mass1, &c->id, &c->key, &c->slot,
                      &c->tmp_src, &c->tmp_id, &c->tmp_key, &c->skey, &c->r, &c->q, &c->cell_count,
                      &c->cell_start, &c->scan_part, &c->d_rp, &c->d_st, &c->d_tiles,
                      &c->d_tile_start, &c->d_real_start, &c->d_blk_real, &c->audit_part, &c->audit_out,
                      &c->step_ctr, &c->counts, &c->d_chunks, &c->d_chunk_start, &c->chunk_part,
                      &c->audit_done, &c->bbox, &c->bparts, &c->nb_meta, &c->nb_idx, &c->nb_w,
                      &c->nb_src, &c->src_of, &c->half_slots, &c->half_own, &c->d_item_start,
                      &c->d_item_real};
    for (DevBuf* b : bufs) b->release();
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

}  // extern "C"
