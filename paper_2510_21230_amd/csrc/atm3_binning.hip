// Linked-cell binning on gfx950: wrap + cell index in FP64 (bit-exact, no
// contraction), counting sort into cell order, stable within each cell, and
// the gather of cell-centred FP64 coordinates the force kernels stage in LDS.
//
// Paper, Sec. 4 (preamble): cells are ordered lexicographically and the cell
// side equals (here: is at least) the cutoff radius.  The cell of a molecule
// is floor(x * n/L) of its wrapped coordinate, clamped to [0, n-1].
//
// This translation unit is compiled with -ffp-contract=off; the pragma below
// states the same requirement in the source.
#pragma clang fp contract(off)

#include "atm3_internal.h"

namespace atm3 {
namespace {

struct BinArgs {
  int32_t n[3];
  double box[3];
  double inv[3];
  double side[3];
};

// x <- x - L*floor(x/L); c = clamp(floor(x * inv), 0, n-1).
__device__ __forceinline__ int cell_coord(double x, double L, double inv, int n, double* xw) {
  double f = floor(x / L);
  double w = x - L * f;
  double t = floor(w * inv);
  int c = (t < 0.0) ? 0 : (t > (double)(n - 1) ? n - 1 : (int)t);
  *xw = w;
  return c;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// One thread per molecule: linear cell and arrival rank within the cell.
// Consecutive molecules often share a cell (lattice order, or an MD state
// that started from one), and atomics of a wave to one address are
// serialised: each run of equal cells in consecutive lanes takes one atomic,
// by its first lane, which reserves the run's length; the run's lanes take
// the ranks that follow the returned count in lane order.
__global__ __launch_bounds__(256) void k_bin_count(const double* __restrict__ pos, int32_t n, BinArgs g,
                                                   int32_t* __restrict__ cell_of, int32_t* __restrict__ rank,
                                                   int32_t* __restrict__ count) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int32_t c = -1;  // lanes past n form runs of their own and add nothing
  if (i < n) {
    double w;
    const int cx = cell_coord(pos[3 * (int64_t)i + 0], g.box[0], g.inv[0], g.n[0], &w);
    const int cy = cell_coord(pos[3 * (int64_t)i + 1], g.box[1], g.inv[1], g.n[1], &w);
    const int cz = cell_coord(pos[3 * (int64_t)i + 2], g.box[2], g.inv[2], g.n[2], &w);
    c = (cz * g.n[1] + cy) * g.n[0] + cx;
    cell_of[i] = c;
  }
  const int32_t prev = __shfl_up(c, 1);
  const unsigned long long heads = __ballot(lane == 0 || c != prev);
  const unsigned long long upto = (2ull << lane) - 1ull;  // lanes 0..lane (all 64 for lane 63)
  const int head = 63 - __clzll(heads & upto);          // first lane of this lane's run
  const unsigned long long later = heads & ~upto;
  const int next = later ? __ffsll((long long)later) - 1 : 64;  // first lane of the next run
  int32_t base = 0;
  if (c >= 0 && lane == head) base = atomicAdd(&count[c], next - lane);
  base = __shfl(base, head);
  if (c >= 0) rank[i] = base + (lane - head);
}

// Exclusive prefix over the cell counts: each workgroup scans a tile of 1024
// cells (4 consecutive cells per thread) and records the tile sum; then
// either each tile's workgroup sums the tile sums before it and adds them
// (k_scan_fix, up to SCAN_SUMS_MAX tiles), or one workgroup scans the tile
// sums and a third launch adds the tile offsets.
constexpr int TILE = 1024;

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t* __restrict__ count, int32_t* __restrict__ start,
                                                    int32_t* __restrict__ tile_sum, int64_t ncells) {
  __shared__ int32_t ws[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * TILE + 4 * tid;
  int v[4];
  for (int k = 0; k < 4; ++k) v[k] = (c0 + k < ncells) ? count[c0 + k] : 0;
  const int s = v[0] + v[1] + v[2] + v[3];
  const int incl = wave_incl_scan(s, lane);
  if (lane == 63) ws[wave] = incl;
  __syncthreads();
  int run = incl - s;
  for (int q = 0; q < wave; ++q) run += ws[q];
  for (int k = 0; k < 4; ++k) {
    if (c0 + k < ncells) start[c0 + k] = run;
    run += v[k];
  }
  if (tid == 255) tile_sum[blockIdx.x] = run;
}

__global__ __launch_bounds__(1024) void k_scan_sums(int32_t* __restrict__ tile_sum, int32_t ntiles) {
  __shared__ int32_t ws[16];
  __shared__ int32_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += 1024) {
    const int t = base + tid;
    const int v = (t < ntiles) ? tile_sum[t] : 0;
    const int incl = wave_incl_scan(v, lane);
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    int pre = carry;
    for (int q = 0; q < wave; ++q) pre += ws[q];
    if (t < ntiles) tile_sum[t] = pre + incl - v;
    __syncthreads();
    if (tid == 1023) carry = pre + incl;
    __syncthreads();
  }
  if (tid == 0) tile_sum[ntiles] = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t* __restrict__ start, const int32_t* __restrict__ tile_sum,
                                                  int64_t ncells, int32_t ntiles) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < ncells) start[c] += tile_sum[c / TILE];
  if (c == 0) start[ncells] = tile_sum[ntiles];
}

// The last two steps in one launch, for at most SCAN_SUMS_MAX tiles:
// workgroup t adds the sum of the tile sums before tile t (each thread sums
// a strided share in a fixed order, then the waves, then the workgroup) to
// the tile's 1,024 prefixes; the last workgroup also writes the total.
constexpr int SCAN_SUMS_MAX = 4096;
__global__ __launch_bounds__(256) void k_scan_fix(int32_t* __restrict__ start, const int32_t* __restrict__ tile_sum,
                                                  int64_t ncells, int32_t ntiles) {
  __shared__ int32_t ws[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = blockIdx.x;
  const bool last = t == ntiles - 1;
  const int upto = last ? ntiles : t;  // the last tile also needs its own sum
  int v = 0;
  for (int q = tid; q < upto; q += 256) v += tile_sum[q];
  const int w = __shfl(wave_incl_scan(v, lane), 63);
  if (lane == 0) ws[wave] = w;
  __syncthreads();
  const int all = ws[0] + ws[1] + ws[2] + ws[3];
  const int off = last ? all - tile_sum[t] : all;
  const int64_t c0 = (int64_t)t * TILE + 4 * tid;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (c0 + k < ncells) start[c0 + k] += off;
  if (last && tid == 0) start[ncells] = all;
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ cell_of, const int32_t* __restrict__ rank,
                                                 const int32_t* __restrict__ start, int32_t n,
                                                 int32_t* __restrict__ perm) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  perm[start[cell_of[i]] + rank[i]] = i;
}

// Restore input order inside each cell (atomic ranks arrive in any order).
// A cell of at most 32 molecules is loaded into registers with independent
// loads, and each entry goes to the slot given by the number of smaller
// entries (the indices are distinct); a larger cell is insertion-sorted in
// place.
__global__ __launch_bounds__(256) void k_cellsort(const int32_t* __restrict__ start, int64_t ncells,
                                                  int32_t* __restrict__ perm) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int32_t lo = start[c], hi = start[c + 1], m = hi - lo;
  if (m <= 1) return;
  if (m <= 32) {
    int32_t v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = (k < m) ? perm[lo + k] : INT32_MAX;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      int r = 0;
#pragma unroll
      for (int q = 0; q < 32; ++q) r += v[q] < v[k];
      if (k < m) perm[lo + r] = v[k];
    }
    return;
  }
  for (int32_t a = lo + 1; a < hi; ++a) {
    int32_t v = perm[a];
    int32_t b = a - 1;
    while (b >= lo && perm[b] > v) {
      perm[b + 1] = perm[b];
      --b;
    }
    perm[b + 1] = v;
  }
}

// One thread per sorted slot: FP64 coordinates relative to the centre of the
// molecule's cell, x_wrapped - (c + 1/2) * side, and the input index in .w.
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ pos, const int32_t* __restrict__ perm,
                                                int32_t n, BinArgs g, double4* __restrict__ sorted) {
  int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t i = perm[s];
  double loc[3];
  for (int d = 0; d < 3; ++d) {
    double w;
    int c = cell_coord(pos[3 * (int64_t)i + d], g.box[d], g.inv[d], g.n[d], &w);
    double centre = ((double)c + 0.5) * g.side[d];
    loc[d] = w - centre;
  }
  sorted[s] = make_double4(loc[0], loc[1], loc[2], (double)i);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_binning(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& gr) {
  BinArgs g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = gr.n[d];
    g.box[d] = gr.box[d];
    g.inv[d] = gr.inv[d];
    g.side[d] = gr.side[d];
  }
  hipStream_t st = ctx->stream;
  int32_t* cell_of = (int32_t*)ctx->buf[B_CELL_OF];
  int32_t* rank = (int32_t*)ctx->buf[B_RANK];
  int32_t* count = (int32_t*)ctx->buf[B_COUNT];
  int32_t* start = (int32_t*)ctx->buf[B_START];
  int32_t* perm = (int32_t*)ctx->buf[B_PERM];
  double4* sorted = (double4*)ctx->buf[B_SORTED];
  const int32_t nn = (int32_t)n;
  unsigned fb = blocks_for(gr.ncells, 256);
  if (fb > 4096) fb = 4096;
  hipError_t e = phase_begin(ctx, ATM3_PHASE_BINNING);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_i32, dim3(fb), dim3(256), 0, st, count, gr.ncells, 0);
  hipLaunchKernelGGL(k_bin_count, dim3(blocks_for(n, 256)), dim3(256), 0, st, pos, nn, g, cell_of, rank, count);
  const int32_t ntiles = (int32_t)((gr.ncells + TILE - 1) / TILE);
  int32_t* tile_sum = (int32_t*)ctx->buf[B_TILE];
  if ((e = launch_scan(st, count, start, gr.ncells, tile_sum)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, cell_of, rank, start, nn, perm);
  hipLaunchKernelGGL(k_cellsort, dim3(blocks_for(gr.ncells, 256)), dim3(256), 0, st, start, gr.ncells, perm);
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, st, pos, perm, nn, g, sorted);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return phase_end(ctx, ATM3_PHASE_BINNING);
}

hipError_t launch_scan(hipStream_t st, const int32_t* count, int32_t* start, int64_t n, int32_t* tile_sum) {
  const int32_t ntiles = (int32_t)((n + TILE - 1) / TILE);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles > 0 ? ntiles : 1), dim3(256), 0, st, count, start, tile_sum, n);
  if (ntiles >= 1 && ntiles <= SCAN_SUMS_MAX) {
    hipLaunchKernelGGL(k_scan_fix, dim3(ntiles), dim3(256), 0, st, start, tile_sum, n, ntiles);
  } else {
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, tile_sum, ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n > 0 ? n : 1, 256)), dim3(256), 0, st, start, tile_sum, n,
                       ntiles);
  }
  return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void k_nonfinite(const double* __restrict__ x, int64_t m, int32_t* __restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad[0] = 1;
}
}  // namespace

hipError_t launch_check_finite(hipStream_t st, const double* pos, int64_t n, int32_t* bad_dev) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, bad_dev, (int64_t)1, 0);
  unsigned nb = blocks_for(3 * n, 256);
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_nonfinite, dim3(nb), dim3(256), 0, st, pos, 3 * n, bad_dev);
  return hipGetLastError();
}

}  // namespace atm3
