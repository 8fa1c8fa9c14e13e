// rwpt_device.h -- structures shared by the host code and the HIP kernels of
// the mass-transfer library (never by the CPU oracle).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rwpt {

// Cell grid and physical parameters of one realisation, for one (dt, D).
struct RealParams {
  double lo[3];        // reflecting-box lower corner
  double hi[3];        // reflecting-box upper corner
  double inv_h[3];     // 1 / cell size per axis
  int32_t nc[3];       // cells per axis (unused axes: 1)
  int32_t n_stencil;   // number of neighbour-row offsets
  int32_t stencil_off; // first entry in the stencil table
  int32_t active;      // 1 if D_r > 0 (transfer on)
  int64_t cell_off;    // first global cell index of this realisation
  int64_t p_begin;     // first particle (sorted order keeps realisations contiguous)
  int64_t p_end;
  double rc2_d;        // cutoff^2 = (kappa*kappa) * ((8*D_r)*dt), binary64
  double escale_d;     // -1 / sigma^2, sigma^2 = 8 D_r dt
  float rc2_f;         // rc2_d rounded once to binary32
  float escale_f;      // -log2(e) / sigma^2 rounded to binary32 (for exp2)
  double amp;          // isotropic walk amplitude sqrt(2 dt (D_rw + alpha_t |v|))
  double rc_geo;       // geometric cutoff sqrt(rc2_d) (1 + 1e-5): covers the rounding of s^2
  double drift[3];     // v dt
  double udir[3];      // v / |v| (zero without a velocity)
  double amp_x;        // sqrt(2 dt (D_rw + alpha_l |v|)) - amp: extra amplitude along udir
  int32_t moves;       // 1 if the walk moves particles of this realisation
  // half-stencil tiling: the cell rows are cut into segments of seg_w cells,
  // seg_w >= 2 * the widest stencil reach / (npar - 1), one work item per
  // (row, segment); at most npar consecutive segments reach a cell
  int32_t seg_w;       // cells per segment
  int32_t nseg;        // segments per cell row (0: no pair work)
  int32_t npar;        // slot planes per direction (segment index mod npar)
  int32_t rx_own;      // stencil reach along x on the particle's own row
  int32_t n_fwd;       // forward stencil rows (dz > 0, or dz = 0 and dy > 0)
  int64_t item_off;    // first work item of this realisation
};

// Offset (dy, dz) of a neighbour row of cells and how many cells (rx) to
// extend the x-range of the tile on that row.
struct StencilRow {
  int32_t dy, dz, rx, pad;
};

// A run of consecutive particles (in cell-sorted order) handled by one wave.
struct Tile {
  int32_t begin, end, real, pad;
};

// Arguments of the pair kernels.  Floating-point arrays are binary32 or
// binary64 according to the kernel instantiation.
struct PairArgs {
  const void* pos;         // [cap][d] particle-major (packed), cell-sorted
  const void* mass_in;     // [cap][SP] particle-major (SP = 2, 4, 8 species slots)
  void* mass_out;          // [cap][SP]
  const void* q_in;        // 1 / r_i for the symmetric normalisation, [cap]
  void* q_out;             // written by the row-sum pass
  double* r_out;           // r_i = sum_j w_ij, written by the row-sum pass (null: not kept; the
                           // symmetric normalisation needs only q)
  const uint32_t* skey;    // global cell key of each sorted particle
  const uint32_t* cell_start;
  const Tile* tiles;
  int32_t ntiles;
  const RealParams* rp;
  const StencilRow* st;
  int32_t S;
  int32_t react_a, react_b;
  int32_t norm;            // 0 = symmetric, 1 = row
  double* audit_part;      // [ntiles][S + 1]
  unsigned long long* counts;  // count mode: [ntiles][2] (pairs j != i, evaluations)
  uint32_t* nbr_cursor;    // neighbour export: per-particle counts / write cursors
  const unsigned long long* nbr_rowptr;  // neighbour export: exclusive offsets
  uint32_t* nbr_pairs;     // neighbour export: (i, j) sorted-slot pairs
  // neighbour cache of the one-lane-per-particle kernels (written by the
  // row-sum pass, read by the exchange pass)
  uint16_t* nb_meta;       // [cap]: (offset in the wave's region << 4) | count, or the miss code
  uint32_t* nb_idx;        // [ntiles][kCacheWave] sorted index j of each cached neighbour
  void* nb_w;              // [ntiles][kCacheWave] its weight w_ij (binary32 or binary64)
  uint32_t* nb_src;        // [ntiles][kCacheWave] src_of[j] of each cached neighbour (indirect mode)
  // indirect mode (one lane per particle after a sort): the masses are still
  // in the previous sorted order; particle i's are at mass_in[SP * src_of[i]]
  const uint32_t* src_of;  // [cap] previous sorted slot of each sorted particle
  int32_t indirect;
  // half-stencil tiling: the far-end sums of each work item go to slot planes
  // [npar * direction + segment mod npar][cap][V] (V = 1 for the row sums,
  // species slots for the exchange); each particle's own sums to
  // half_own[cap][V]
  float* half_slots;
  double* half_own;
  // work items in dispatch order: the realisations by decreasing cost per
  // item, each realisation's items in (row, segment) order; position k of
  // that order holds realisation half_item_real[k] and starts at item
  // half_item_start[k]
  const int64_t* half_item_start;  // [n_real + 1]
  const int32_t* half_item_real;   // [n_real]
  int64_t half_nitems;
  int64_t half_cap;                // particles per slot plane
  int32_t n_real;
};

}  // namespace rwpt
