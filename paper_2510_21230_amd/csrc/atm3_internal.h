// Internal declarations shared by the translation units of libatm3.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "atm3.h"

namespace atm3 {

// Grid of linked cells and the FP64 constants every binning step uses.
struct Grid {
  int32_t n[3];     // cells per dimension, floor(L_d / rc)
  int64_t ncells;   // n[0]*n[1]*n[2]
  double box[3];    // L_d
  double inv[3];    // n_d / L_d  (FP64, correctly rounded on host and device)
  double side[3];   // L_d / n_d
};

// Device scratch of one evaluation, owned by the context (grow-only).
enum Buf {
  B_CELL_OF = 0,  // int32 [N]   linear cell per molecule (input order)
  B_RANK,         // int32 [N]   arrival rank within the cell (unstable)
  B_COUNT,        // int32 [C]   molecules per cell
  B_START,        // int32 [C+1] exclusive prefix of counts
  B_PERM,         // int32 [N]   sorted slot -> input index (stable)
  B_SORTED,       // double4[N]  cell-centred FP64 coordinates, .w = input index
  B_FPART,        // double[8][3][N] per-corner partial forces (sorted order)
  B_BLKD,         // double[C][3] per-block e_lj', w_lj', e_atm'
  B_BLKI,         // int32 [C][2] per-block pair and triplet counts
  B_DEFER,        // int32 [2C+3] [0] count, [1] status, [2..C+2) queued base cells, [C+2] count, [C+3..) of the wide tier
  B_RED,          // first-stage reduction partials
  B_TILE,         // int32 per-tile sums of the cell-count scan
  B_FMASK,        // uint32 [N][14] forward-shell pair masks (sorted order)
  B_FMOK,         // int32 [C] the mask words of a cell were written
  // learned surrogate (atm3_surrogate.hip); slot = sorted molecule index
  B_SN_ALL,       // int32 [N]   neighbours per slot
  B_SN_UP,        // int32 [N]   neighbours with a larger slot
  B_SN_START,     // int32 [N+1] first neighbour entry of each slot
  B_SN_UPSTART,   // int32 [N+1] first pair of each slot
  B_SN_LOFILL,    // int32 [N]   fill counters of the lower entries
  B_SN_TILE,      // int32 scan tiles
  B_SN_NB,        // int32 [2P]  neighbour entries: 2*pair + (slot is the pair's second)
  B_SP_IJ,        // int2 [P]    pair slots (i < j)
  B_SP_REC,       // float4 [P]  r_i - r_j and |r_i - r_j|
  B_SP_ST,        // float2 [P]  pair outputs s, t
  B_SD,           // float [N][64] descriptors (normalised, or raw when fitting)
  B_SDB,          // bf16 [N][64]
  B_SQ,           // int32 [N+1] fallback queue (count, slots)
  B_SRED,         // double reduction partials
  B_SRED2,        // double [256][4] second-stage reduction partials
  B_SF3,          // float4 [N] surrogate three-body force per slot
  B_SE,           // float [N]  error estimate per slot
  B_SG,           // float4 [N] dL/dF per slot
  B_SGE,          // float [N]  dL/de per slot
  B_TH1,          // bf16 [P][128] hidden activations (training)
  B_TH2,
  B_TH3,
  B_TG16,         // bf16 [P][16] radial inputs (training)
  B_TDOUT,        // float [P][2] dL/d(s, t)
  B_TDOUTB,       // bf16 [P][2]
  B_TDZ3,         // float [P][128] layer deltas
  B_TDZ2,
  B_TDZ1,
  B_TDZ3B,        // bf16 [P][128]
  B_TDZ2B,
  B_TDZ1B,
  B_TDA,          // float [N][128] dL/dA
  B_TDAB,         // bf16 [N][128]
  B_TPART,        // float split-K partial products
  B_ZHIST,        // uint32 [nbins] z histogram of the slab correction
  B_MDSLOT,       // atm3_result of the step in flight + step counter (graph-launched MD)
  B_PDEFER,       // int32 [C] base cells the shell-pruned product tier handed on
  B_NBUF
};

struct Scratch {
  void* p[B_NBUF] = {};
  size_t cap[B_NBUF] = {};
};

}  // namespace atm3

namespace atm3 {
constexpr int NPHASE = 4;
// HIP event pairs recorded around each timed phase (reused between reads).
struct PhaseTimer {
  std::vector<hipEvent_t> ev;  // start/stop interleaved
  size_t used = 0;             // event pairs recorded since the last read
  double total_ms = 0.0;
  int64_t launches = 0;
};
}  // namespace atm3

struct atm3_ctx {
  int device = 0;
  bool profile = false;
  atm3::PhaseTimer timer[atm3::NPHASE];
  hipStream_t stream = nullptr;
  std::string err;
  atm3::Scratch s;               // owned device scratch (grow-only)
  void** buf = s.p;              // buffer table the launches use: s.p, or a
  size_t* bufcap = s.cap;        // carve of the fixed array (no allocation)
  bool fixed = false;            // inside atm3_compute_forces_noalloc
  atm3_result* dres = nullptr;  // device result of the synchronous path
  atm3_result* hres = nullptr;  // pinned host copy
};

namespace atm3 {

// Record the start / stop event of a timed phase (no-ops unless profiling).
hipError_t phase_begin(atm3_ctx* ctx, int phase);
hipError_t phase_end(atm3_ctx* ctx, int phase);

// Status helpers (set ctx->err and return the code).
int fail(atm3_ctx* ctx, int code, const std::string& msg);
int hip_fail(atm3_ctx* ctx, hipError_t e, const char* what);
int ensure(atm3_ctx* ctx, Buf b, size_t bytes);

// Device scratch sizes of one pairwise-cutoff evaluation of n molecules on
// grid g (every buffer the binning, block, reduction and candidate-count
// launches use); zero for the buffers they do not touch.
void plan_pair_path(int64_t n, const Grid& g, size_t bytes[B_NBUF]);

// Grid from box and cutoff; returns false if any n_d < 1 or sizes overflow.
bool make_grid(const double box[3], double rc, Grid* g);

// Binning (atm3_binning.hip): fills B_CELL_OF, B_COUNT, B_START, B_PERM,
// B_SORTED from the FP64 positions.
hipError_t launch_binning(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g);

// Sets bad_dev[0] to 1 if any of the 3n coordinates is not finite.
hipError_t launch_check_finite(hipStream_t st, const double* pos, int64_t n, int32_t* bad_dev);

// Exclusive prefix sum of count[0..n) into start[0..n], start[n] = total;
// tile_sum needs n/1024 + 2 entries.
hipError_t launch_scan(hipStream_t st, const int32_t* count, int32_t* start, int64_t n, int32_t* tile_sum);

// Forces (atm3_forces.hip): block kernels, per-corner partial forces, final
// gather into `forces` and the reduction into `res_dev`.
size_t reduce_scratch_bytes();
hipError_t launch_forces(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g,
                         const atm3_params& p, float* forces, atm3_result* res_dev);

// Variants (atm3_variants.hip): candidate counts of the cell sets from the
// cell populations (patches n_candidates and, with `triple`, turns the block
// kernels' 3c01 triplet count into the per-molecule one), and the one-sided
// evaluation of the product cutoff for every cell set.
hipError_t launch_variant_counts(atm3_ctx* ctx, const Grid& g, const atm3_params& p, atm3_result* res_dev,
                                 bool triple);
hipError_t launch_onesided(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p,
                           float* forces, atm3_result* res_dev);
// Diagonal of the virial tensor into out_dev[0..5] (LJ xx, yy, zz; ATM xx,
// yy, zz) and the status into out_dev[6]; needs the binning of `pos`.
hipError_t launch_virial_diag(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p,
                              double* out_dev);

}  // namespace atm3
