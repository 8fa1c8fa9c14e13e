// rwpt_kernels.h -- host-callable launchers of the HIP kernels (internal).
#pragma once
#include "rwpt_device.h"

namespace rwpt {

// Phase identifiers used for per-phase timing.
enum Phase {
  PH_WALK_KEY = 0,
  PH_SCAN,
  PH_SCATTER,
  PH_CANON,
  PH_ROWSUM,
  PH_EXCHANGE,
  PH_AUDIT,
  PH_DENSE,
  PH_COUNT,
  PH_N
};

constexpr int kBlock = 256;        // threads per block of every kernel
constexpr int kScanItems = 16;     // counts per thread in the cell-count scan
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int64_t kScanDirectMax = 256;  // up to this many scan blocks (one partial per thread), no top-level scan launch

// Random walk + reflection (optional) and cell key / in-cell slot of every particle.
// pos_in/pos_out may not alias.  blk_real[b] is the realisation of particle
// b * kBlock (one entry per block of the launch).
hipError_t launch_walk_key(int fp64, int dim, const void* pos_in, void* pos_out,
                           const uint32_t* id, int32_t n, const RealParams* rp,
                           const int64_t* real_start, const int32_t* blk_real, int32_t n_real,
                           const uint64_t* step_ctr,
                           uint64_t seed, int32_t do_walk, uint32_t* cell_count, uint32_t* key,
                           uint32_t* slot, hipStream_t s);

// Exclusive scan of cell_count[0..ncell) into cell_start[0..ncell]; zeroes cell_count.
// partials must hold ceil(ncell / kScanChunk) + 1 entries.
hipError_t launch_cell_scan(uint32_t* cell_count, uint32_t* cell_start, int64_t ncell,
                            uint32_t* partials, hipStream_t s);

// Place every particle at cell_start[key] + slot (arrival order inside a cell).
hipError_t launch_scatter(int32_t n, const uint32_t* key, const uint32_t* slot,
                          const uint32_t* cell_start, const uint32_t* id, uint32_t* tmp_src,
                          uint32_t* tmp_id, uint32_t* tmp_key, hipStream_t s);

// Reorder inside every cell by particle id (canonical order), gathering
// positions, ids and keys into the sorted arrays, and the masses too when
// src_out is NULL; otherwise the masses stay in the previous order and
// src_out[i] receives the previous slot of sorted particle i.
hipError_t launch_canon(int fp64, int dim, int32_t n, const uint32_t* tmp_src,
                        const uint32_t* tmp_id, const uint32_t* tmp_key,
                        const uint32_t* cell_start, const void* pos_in, void* pos_out,
                        const void* mass_in, void* mass_out, int32_t S,
                        uint32_t* id_out, uint32_t* skey, uint32_t* src_out, hipStream_t s);

// Species slots per particle the mass arrays hold for S species: the kernels
// are instantiated for 2, 4 or 8 species and read every slot of their
// instantiation, so slots S..padded_species(S)-1 are allocated and kept zero.
inline int padded_species(int S) { return S <= 2 ? 2 : (S <= 4 ? 4 : 8); }

// Pair kernels (one wave per tile).  log2l: lanes per particle = 1 << log2l,
// or kPrivateLists: one lane per particle with its own candidate rows (tiles
// of 64 particles).
constexpr int kPrivateLists = -1;
// Neighbour cache of the one-lane-per-particle kernels: the row-sum pass keeps
// every in-cutoff neighbour j != i of a lane (sorted index and weight) for the
// exchange pass, in a region of kCacheWave entries owned by the lane's wave.
// A lane with more than kCacheLane neighbours, or whose entries would not fit
// its wave's region, is marked kCacheMiss and searches its stencil again.
constexpr int kCacheLane = 8;
constexpr int kCacheWave = 256;
constexpr uint32_t kCacheMiss = 15;
// Half-stencil tiling (binary32): every unordered pair evaluated once, its
// far-end share accumulated into slot planes and summed by a finalizer.
constexpr int kHalfPairs = -4;
// Slot planes per direction of the half-stencil tiling: segments of
// ceil(2 * reach / (kHalfParities - 1)) cells, so that a cell row of a
// realisation gives enough work items to fill the device.
constexpr int kHalfParities = 2;
// Candidate evaluations per work item of the half-stencil tiling aimed at on
// average (segments are widened up to this where neighbourhoods are sparse).
constexpr int64_t kHalfTarget = 32768;
// Consecutive blocks of the half-stencil launch that one XCD takes in turn.
constexpr int64_t kHalfGroup = 16;
hipError_t launch_rowsum(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s);
hipError_t launch_exchange(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s);
hipError_t launch_count(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s);
hipError_t launch_nbr_count(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s);
hipError_t launch_nbr_fill(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s);

// Per-realisation FP64 reduction of the per-tile audit partials in two fixed-
// order levels (chunks of at most kAuditChunk tiles inside one realisation,
// then the chunks of each realisation) in one launch; `done` holds n_real
// zeroed completion counters that the kernel returns to zero.  Optionally
// advances the step counter.
// Few, large chunks: every chunk block of a realisation with more than one
// chunk ends in a device-scope fence and a completion atomic on a shared
// counter, which serialise across blocks; a realisation of one chunk needs
// neither.
constexpr int kAuditChunk = 2048;
struct AuditChunk {
  int32_t begin, end;  // tiles [begin, end) of one realisation
  int32_t real;        // that realisation
  int32_t n_in_real;   // chunks of that realisation
};
hipError_t launch_audit_reduce(const double* part, int32_t S1, const AuditChunk* chunks, int32_t nchunks,
                               double* chunk_part, const int32_t* chunk_start, int32_t n_real,
                               double* out, uint32_t* done, uint64_t* step_ctr, int32_t bump,
                               hipStream_t s);

// Allocation-free transfer of one realisation in caller arrays.  Its grid
// parameters and stencil rows travel as kernel arguments (at most
// kNoAllocStencil rows) and are written to device memory by the set-up
// launch, which also converts the caller's layouts (positions n x dim
// row-major, masses S x n species-major), fills the tiles of G particles, the
// realisation starts {0, n} and the walk's realisation table, and clears ncell
// cell counts.
constexpr int kNoAllocStencil = 64;
struct NoAllocParams {
  RealParams P;
  StencilRow st[kNoAllocStencil];
  int32_t n_st;
};
hipError_t launch_noalloc_setup(int fp64, int dim, int S, const NoAllocParams& a, int32_t n, const void* pos,
                                const void* mass, void* pos_out, void* mass_out, uint32_t* id, Tile* tiles,
                                int32_t G, int32_t ntiles, RealParams* rp, StencilRow* st, int64_t* real_start,
                                int32_t* blk_real, uint32_t* cell_count, int64_t ncell, hipStream_t s);
// Sorted masses (particle-major) back to the caller's order (S x n species-major).
hipError_t launch_noalloc_store(int fp64, int S, int32_t n, const void* mass_sorted, const uint32_t* id,
                                void* mass, hipStream_t s);

// Full-matrix path of one realisation (binary32 state, bf16-split MFMA).
struct DenseArgs {
  const float* pos;        // [cap][PS] particle-major, sorted
  int64_t cap;
  int32_t n;               // particles (one realisation)
  const float* mass_in;    // [cap][SP] particle-major
  float* mass_out;
  float* q;                // written by the row-sum pass, read by the exchange
  double* r;
  float* bbox;             // [ceil(n / 32)][2 dim]
  float escale;            // -log2(e) / sigma^2
  float skip_s2;           // column tiles at squared distance > skip_s2 hold weights < 2^-40
  __bf16* bparts;          // [3][16 ncb][cap]
  int32_t ncb;             // column blocks of 16 (1 or 2)
  int32_t S, react_a, react_b, norm;
  double* audit_part;      // [ceil(n / 16)][S + 1]
};
constexpr int kDenseRowTile = 16;
constexpr int kDenseColTile = 32;
constexpr int64_t kDenseMaxN = (int64_t)1 << 17;
// column blocks of 16 the contraction needs: [M_s, q M_s, q, 1] (symmetric) or [M_s, 1] (row)
inline int dense_ncb(int S, int norm) { return ((norm == 0 ? 2 * S + 2 : S + 1) + 15) / 16; }
hipError_t launch_dense_step(int dim, const DenseArgs& a, hipStream_t s);

// Instruction-rate probes (register-only kernels of rwpt_probe.hip): binary32
// FMA, binary32 exp2, and the per-candidate code of the row-broadcast row-sum
// and symmetric exchange kernels.  `reps` is iterations (FMA, exp) or chunks
// of 16 candidates (row sum, exchange) per lane; out holds one float per
// thread of the grid (blocks * probe_block()).
enum ProbeKind { PROBE_FMA = 0, PROBE_EXP = 1, PROBE_ROWSUM = 2, PROBE_EXCHANGE = 3 };
int probe_block();
int64_t probe_ops_per_lane(int kind, int reps);
hipError_t launch_probe(int kind, int dim, int slots, int blocks, int reps, float rc2, float esc, float h, float* out,
                        hipStream_t s);

}  // namespace rwpt
