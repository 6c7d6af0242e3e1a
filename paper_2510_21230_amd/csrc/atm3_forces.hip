// Fused Lennard-Jones + Axilrod-Teller-Muto kernel over 2x2x2 cell blocks.
//
// Work unit: one workgroup per base cell b, staging the molecules of the
// eight cells b + o, o in {0,1}^3 (the 3c08 neighbourhood of Sec. 4) in LDS.
// A molecule's corner code is the 3-bit o of its cell.  A pair or triplet is
// owned by the block whose base is the componentwise minimum of its cells,
// i.e. iff the AND of the corner codes is 0; every pair/triplet whose cells
// span at most one step per dimension is then counted exactly once over all
// blocks (for a single base cell: the one-cell set, 13 two-cell sets and 44
// three-cell sets; Sec. 3 eqs. celltriplet, twoonetriplets, carttriplets).
//
// Per block:
//  1. stage FP32 block-frame coordinates (cell-centred + corner shift, from
//     FP64) with their FP32 residuals, and corner codes;
//  2. upper-triangle pair bit masks by wave ballots: bit j of row i (j > i)
//     set iff r_ij^2 < rc^2; FP32 test with a guard band, FP64 re-check with
//     the oracle's exact minimum-image formula inside the band;
//  3. row-major lists of the upper pairs and of the pairs the block owns
//     (one thread per mask word, offsets from one scan); LJ over the owned
//     pairs in FP64 (coordinates as FP32 value + residual);
//  4. per pair the owned third molecules
//     K(i,j) = mask_i & mask_j & allowed(code_i & code_j), all above j,
//     as single-word work items of at most NCLS (12) molecules each, placed in
//     order of size by a block scan of per-thread class counts;
//  5. ATM per triplet in FP32 (eq. atm and its gradient in squared sides,
//     eq. forcepairs).  Each thread takes whole items in rounds, largest
//     first, so the lanes of a wave finish their items together; p_i, p_j
//     and the pair's force sums stay in registers for an item and only F_k
//     is scattered per triplet;
//  6. per-corner partial forces to HBM (each (corner, molecule) written by
//     exactly one block, no global atomics); per-block energy and count
//     partials.
// Force and energy accumulation is 64-bit fixed point (units of 2^-32):
// every contribution is converted to an integer number of units (rounded to
// nearest on this path, |value| < 2^18; rounded down on the general path,
// |value| < 2^31) and added with LDS integer atomics, so the sums are exact
// and independent of the order of arrival.  Blocks of more than 128
// molecules, beyond the capacities, or with a value outside the range of
// this path take a general path that materialises the triplets in rounds.
// Wave scans and sums use DPP lane moves, which leave the LDS to the
// atomics.  A gather kernel sums the eight corner partials per molecule; two
// reduction kernels sum the per-block partials in fixed order.  Every result
// is reproducible bit for bit from run to run.
#include "atm3_internal.h"
#include "atm3_terms.h"

namespace atm3 {
namespace {

constexpr int WG = 256;
constexpr int NWAVE = WG / 64;
constexpr int RBLK = 256;  // workgroups of the first reduction stage
constexpr double FIX_SCALE = 4294967296.0;        // 2^32
constexpr double FIX_INV = 2.3283064365386963e-10;  // 2^-32
constexpr double FIX_LIMIT = 2147483648.0;        // |value| < 2^31

typedef unsigned long long u64;

struct ForceArgs {
  const double4* sorted;  // cell-centred FP64 coordinates, .w = input index
  const int32_t* start;   // cell_start
  const double* pos;      // FP64 input positions (exact re-checks only)
  u64* fpart;             // [8][3][N] fixed point
  double* blkd;           // [C][3]: e_lj', w_lj', e_atm'
  int32_t* blki;          // [C][2]: pairs, triplets
  int32_t* defer;         // [0] count, [1] status, [2..] base cells
  const uint32_t* fmask;  // [N][14] forward-shell pair masks (k_fmask)
  const int32_t* fm_ok;   // [C] 1 if a cell's mask words were written
  int32_t ntot;
  int32_t nx, ny, nz;
  int32_t ncells;
  int32_t terms;
  double half[3];  // side_d / 2
  float lo2, hi2;  // FP32 guard band around rc^2
  double rc2;      // rc^2 in FP64 (exact decision)
  double box[3];
  double sig2;   // sigma^2
  double eps24;  // 24 eps
  float k3nu, k15nu, k075nu;  // 3 nu, 1.875 nu, 0.75 nu
};

// Bits strictly above position i within 64-bit word w.
__device__ __forceinline__ u64 above(int i, int w) {
  int d = i - 64 * w;
  if (d < 0) return ~0ull;
  if (d >= 63) return 0ull;
  return ~0ull << (d + 1);
}


// d in units of 2^-32 as a two's-complement 64-bit integer, rounded toward
// minus infinity: floor(d) in the high word, the fraction in the low word
// (both exact in FP64).  Out-of-range or non-finite values set *bad.
__device__ __forceinline__ u64 to_fix(double d, int* bad) {
  if (!(fabs(d) < FIX_LIMIT)) {
    *bad = 1;
    return 0ull;
  }
  const double hi = floor(d);
  const double lo = (d - hi) * FIX_SCALE;  // in [0, 2^32)
  return ((u64)(uint32_t)(int32_t)hi << 32) | (u64)(uint32_t)lo;
}

__device__ __forceinline__ double from_fix(u64 v) { return (double)(long long)v * FIX_INV; }

__device__ __forceinline__ void add_fix(u64* ax, u64* ay, u64* az, int m, double x, double y, double z, int* bad) {
  atomicAdd(&ax[m], to_fix(x, bad));
  atomicAdd(&ay[m], to_fix(y, bad));
  atomicAdd(&az[m], to_fix(z, bad));
}

// Wave-wide inclusive prefix sums with DPP lane moves (row shifts within
// each 16-lane row, then the row broadcasts of lanes 15 and 31); no LDS
// traffic.  Lanes with no source lane read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_mv(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ u64 dpp_mv64(u64 v) {
  return ((u64)dpp_mv<CTRL, ROWS>((uint32_t)(v >> 32)) << 32) | dpp_mv<CTRL, ROWS>((uint32_t)v);
}
__device__ __forceinline__ int wave_incl_scan(int v) {
  uint32_t x = (uint32_t)v;
  x += dpp_mv<0x111, 0xf>(x);  // row_shr:1
  x += dpp_mv<0x112, 0xf>(x);  // row_shr:2
  x += dpp_mv<0x114, 0xf>(x);  // row_shr:4
  x += dpp_mv<0x118, 0xf>(x);  // row_shr:8
  x += dpp_mv<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_mv<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return (int)x;
}
__device__ __forceinline__ u64 wave_incl_scan64(u64 x) {
  x += dpp_mv64<0x111, 0xf>(x);
  x += dpp_mv64<0x112, 0xf>(x);
  x += dpp_mv64<0x114, 0xf>(x);
  x += dpp_mv64<0x118, 0xf>(x);
  x += dpp_mv64<0x142, 0xa>(x);
  x += dpp_mv64<0x143, 0xc>(x);
  return x;
}
__device__ __forceinline__ double wave_incl_scan_d(double v) {
  v += __longlong_as_double((long long)dpp_mv64<0x111, 0xf>((u64)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_mv64<0x112, 0xf>((u64)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_mv64<0x114, 0xf>((u64)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_mv64<0x118, 0xf>((u64)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_mv64<0x142, 0xa>((u64)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_mv64<0x143, 0xc>((u64)__double_as_longlong(v)));
  return v;
}
__device__ __forceinline__ u64 lane63(u64 v) {
  return ((u64)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), 63) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
}
// Wave totals, in every lane (fixed summation order).
__device__ __forceinline__ double wave_sum(double v) {
  return __longlong_as_double((long long)lane63((u64)__double_as_longlong(wave_incl_scan_d(v))));
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
  return (long long)lane63(wave_incl_scan64((u64)v));
}

__device__ __forceinline__ double comb2(double n) { return n * (n - 1.0) * 0.5; }
__device__ __forceinline__ double comb3(double n) { return n * (n - 1.0) * (n - 2.0) / 6.0; }

// Molecule triplets of the cell sets a base cell visits (3c08), from the
// populations N[o] of its eight corner cells: eq. (celltriplet) for the base
// cell, eq. (twoonetriplets) for the 13 cell pairs and eq. (carttriplets) for
// the 44 cell triples whose componentwise minimum is the base (corner codes
// with AND == 0).  In FP64: every term and partial sum is an integer below
// 2^53 for populations up to 2^15 per cell (blocks of more than 512
// molecules are an error of the evaluation anyway), so the count is exact.
__device__ double candidates_3c08(const int32_t* N) {
  double n[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) n[o] = (double)N[o];
  double t = comb3(n[0]);
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int q = p + 1; q < 8; ++q) {
      if ((p & q) == 0) t += n[q] * comb2(n[p]) + n[p] * comb2(n[q]);
#pragma unroll
      for (int r = q + 1; r < 8; ++r)
        if ((p & q & r) == 0) t += n[p] * n[q] * n[r];
    }
  return t;
}

// One ATM triplet in FP32 from block-frame positions: returns the energy
// term without nu (Q^-3/2 + 3/8 P Q^-5/2) and the forces on i and j; the
// force on k is -(F_i + F_j) (eq. newton3rdlaw).

// Shared per-block bookkeeping of both paths.
struct BlockHead {
  int32_t cbase[9];
  int32_t cstart[8];
  int32_t okc[8];  // the corner cells' mask words exist (fm_ok)
  int32_t bad;
  double red[3][NWAVE];
  long long redi[NWAVE];
};

// Cell ranges of the eight corners of base cell b; returns the population.
__device__ int block_cells(const ForceArgs& a, int b, BlockHead& H) {
  const int tid = threadIdx.x;
  const int bx = b % a.nx, by = (b / a.nx) % a.ny, bz = b / (a.nx * a.ny);
  if (tid < 64) {  // wave 0: lane o < 8 takes corner o, a scan gives the offsets
    int cnt = 0;
    if (tid < 8) {
      int cx = bx + (tid & 1), cy = by + ((tid >> 1) & 1), cz = bz + (tid >> 2);
      if (cx >= a.nx) cx -= a.nx;
      if (cy >= a.ny) cy -= a.ny;
      if (cz >= a.nz) cz -= a.nz;
      const int c = (cz * a.ny + cy) * a.nx + cx;
      const int s0 = a.start[c];
      H.cstart[tid] = s0;
      cnt = a.start[c + 1] - s0;
      H.okc[tid] = a.fm_ok ? a.fm_ok[c] : 0;
    }
    const int incl = wave_incl_scan(cnt);
    if (tid < 8) H.cbase[tid + 1] = incl;
    if (tid == 0) {
      H.cbase[0] = 0;
      H.bad = 0;
    }
  }
  __syncthreads();
  return H.cbase[8];
}

// Sorted slot of staged molecule t: the staging order is corner by corner.
__device__ __forceinline__ int slot_of(const BlockHead& H, const uint8_t* scode, int t) {
  const int o = scode[t];
  return H.cstart[o] + (t - H.cbase[o]);
}

// Stage block-frame coordinates, corner codes, input and sorted indices, and
// clear the force accumulators.  With slo, the FP32 residuals p - (float)p
// of the coordinates are kept as well (x in sp[t].w, y and z in slo[t]), so
// that hi + lo carries the FP64 coordinate to about 48 bits.
__device__ void block_stage(const ForceArgs& a, const BlockHead& H, int n, double4* dp, float4* sp, float2* slo,
                            u64* ax, u64* ay, u64* az, uint8_t* scode, int32_t* sorig, int32_t* sslot) {
  // corner boundaries read once (independent broadcast loads, no chain of
  // dependent reads per molecule)
  int cb[8];
#pragma unroll
  for (int k = 1; k < 8; ++k) cb[k] = H.cbase[k];
  for (int t = threadIdx.x; t < n; t += WG) {
    int o = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) o += (cb[k] <= t) ? 1 : 0;
    const int s = H.cstart[o] + (t - H.cbase[o]);
    const double4 v = a.sorted[s];
    const double px = v.x + ((o & 1) ? a.half[0] : -a.half[0]);
    const double py = v.y + ((o & 2) ? a.half[1] : -a.half[1]);
    const double pz = v.z + ((o & 4) ? a.half[2] : -a.half[2]);
    if (dp) dp[t] = make_double4(px, py, pz, 0.0);
    const float hx = (float)px, hy = (float)py, hz = (float)pz;
    if (slo) {
      sp[t] = make_float4(hx, hy, hz, (float)(px - (double)hx));
      slo[t] = make_float2((float)(py - (double)hy), (float)(pz - (double)hz));
    } else {
      sp[t] = make_float4(hx, hy, hz, 0.f);
    }
    ax[t] = 0ull;
    ay[t] = 0ull;
    az[t] = 0ull;
    scode[t] = (uint8_t)o;
    if (sorig) sorig[t] = (int32_t)v.w;
    if (sslot) sslot[t] = s;
  }
}

// Allowed-third masks: bit j of allow[c] iff (code_j & c) == 0.
template <int NW>
__device__ void block_allow(int n, const uint8_t* scode, u64* allow) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int item = wave; item < 8 * NW; item += NWAVE) {
    const int c = item / NW, w = item % NW;
    const int j = 64 * w + lane;
    const bool ok = (j < n) && ((scode[j] & c) == 0);
    const u64 bits = __ballot(ok);
    if (lane == 0) allow[item] = bits;
  }
}

// Upper-triangle mask word (bits j > i of word w) of row i, one wave; i, w
// and n are wave-uniform, so the lane-validity mask is scalar work.
__device__ __forceinline__ u64 mask_word(const ForceArgs& a, int i, int w, int n, const float4 pi, const float4 pj,
                                         const int32_t* sorig) {
  const int lane = threadIdx.x & 63;
  const int lo = i + 1 - 64 * w, hi = n - 64 * w;  // valid lanes: lo <= lane < hi
  u64 valid = (hi >= 64) ? ~0ull : ((hi <= 0) ? 0ull : ((1ull << hi) - 1ull));
  valid &= (lo <= 0) ? ~0ull : ((lo >= 64) ? 0ull : (~0ull << lo));
  const float ex = pi.x - pj.x, ey = pi.y - pj.y, ez = pi.z - pj.z;
  const float r2 = ex * ex + ey * ey + ez * ez;
  u64 bits = __ballot(r2 < a.lo2) & valid;
  const u64 maybe = __ballot(r2 < a.hi2) & valid & ~bits;
  if (maybe) {
    bool exq = false;
    if ((maybe >> lane) & 1ull) exq = exact_r2(a.pos, sorig[i], sorig[64 * w + lane], a.box[0], a.box[1], a.box[2]) < a.rc2;
    bits |= __ballot(exq);
  }
  return bits;
}

__device__ __forceinline__ float dist2f(const float4 p, const float4 q) {
  const float ex = p.x - q.x, ey = p.y - q.y, ez = p.z - q.z;
  return ex * ex + ey * ey + ez * ez;
}

// Exact (FP64 minimum-image) cutoff test of the lanes in `maybe` for row i,
// word w; returns the bits that pass.
__device__ __forceinline__ u64 exact_bits(const ForceArgs& a, int i, int w, u64 maybe, const BlockHead& H,
                                          const uint8_t* scode) {
  const int lane = threadIdx.x & 63;
  bool in = false;
  if ((maybe >> lane) & 1ull) {
    const int oi = (int)a.sorted[slot_of(H, scode, i)].w, oj = (int)a.sorted[slot_of(H, scode, 64 * w + lane)].w;
    in = exact_r2(a.pos, oi, oj, a.box[0], a.box[1], a.box[2]) < a.rc2;
  }
  return __ballot(in);
}

// Per-corner partials (fixed point) and block energy / count partials.
__device__ void block_flush(const ForceArgs& a, int b, int n, const uint8_t* scode, const int32_t* sslot,
                            const u64* ax, const u64* ay, const u64* az, BlockHead& H, double e_lj, double w_lj,
                            double e_atm, long long n_pair, int n_trip, int bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = a.ntot;
  for (int t = tid; t < n; t += WG) {
    const int o = scode[t], s = sslot ? sslot[t] : slot_of(H, scode, t);
    a.fpart[(int64_t)(o * 3 + 0) * N + s] = ax[t];
    a.fpart[(int64_t)(o * 3 + 1) * N + s] = ay[t];
    a.fpart[(int64_t)(o * 3 + 2) * N + s] = az[t];
  }
  const double r0 = wave_sum(e_lj), r1 = wave_sum(w_lj), r2 = wave_sum(e_atm);
  const long long i0 = wave_sum_ll(n_pair);
  const bool anybad = __ballot(bad != 0) != 0ull;
  if (lane == 0) {
    H.red[0][wave] = r0;
    H.red[1][wave] = r1;
    H.red[2][wave] = r2;
    H.redi[wave] = i0;
    if (anybad) H.bad = 1;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0, s1 = 0, s2 = 0;
    long long npr = 0;
    for (int q = 0; q < NWAVE; ++q) {
      s0 += H.red[0][q];
      s1 += H.red[1][q];
      s2 += H.red[2][q];
      npr += H.redi[q];
    }
    a.blkd[3 * (int64_t)b + 0] = s0;
    a.blkd[3 * (int64_t)b + 1] = s1;
    a.blkd[3 * (int64_t)b + 2] = s2;
    a.blki[2 * (int64_t)b + 0] = (int32_t)npr;
    a.blki[2 * (int64_t)b + 1] = n_trip;
    if (H.bad) atomicMin(&a.defer[1], ATM3_ERANGE);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Forward-shell pair masks, computed once per evaluation for every pair of
// neighbouring molecules (the 2x2x2 blocks would otherwise test a pair of one
// cell in 8 blocks, of face-neighbour cells in 4, of edge neighbours in 2).
// For the molecule in sorted slot s of cell A and the k-th forward cell B_k
// of A (FWD order: A itself, then the 13 neighbours at offsets whose
// (dz, dy, dx) is lexicographically positive), word fmask[14 s + k] has bit t
// set iff molecule t of B_k (t after s within A itself) lies inside rc by the
// exact decision.  Cells of more than 32 molecules get no words; fm_ok[c]
// says whether cell c's words were written.  One workgroup per row segment of
// FM_G cells along x stages the forward region of the segment in LDS (the
// segment's row and four neighbouring rows, one cell wider on each side).
// ---------------------------------------------------------------------------
constexpr int FM_G = 8;
constexpr int FM_W = FM_G + 2;          // staged cells per row
constexpr int FM_ROWS = 5;              // (dy, dz) = (0,0), (1,0), (-1,1), (0,1), (1,1)
constexpr int FM_CELLS = FM_ROWS * FM_W;
constexpr int FM_CAP = 1280;            // staged molecules

// Index in FWD of the forward offset (dx, dy, dz) (lexicographically
// positive in (dz, dy, dx), or zero).
__device__ __forceinline__ int fwd_index(int dx, int dy, int dz) {
  return dz == 0 ? (dy == 0 ? dx : 3 + dx) : 9 + 3 * dy + dx;
}

struct FmArgs {
  const double4* sorted;
  const int32_t* start;
  const double* pos;
  uint32_t* fmask;  // [N][14]
  int32_t* fm_ok;   // [C]
  int32_t nx, ny, nz;
  double side[3];
  double box[3];
  float lo2, hi2;
  double rc2;
  int32_t* defer;  // the hand-on queues, emptied here for the block kernels
  int32_t ncells;
};

__global__ __launch_bounds__(256) void k_fmask(FmArgs a) {
  __shared__ float4 sp[FM_CAP];
  __shared__ int32_t cst[FM_CELLS + 1];  // staged start of each staged cell
  __shared__ int32_t cgs[FM_CELLS];      // sorted start of each staged cell
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) {  // queue counts and status (the block kernels run after this launch)
    a.defer[0] = 0;
    a.defer[1] = ATM3_OK;
    a.defer[2 + a.ncells] = 0;
  }
  const int nseg = (a.nx + FM_G - 1) / FM_G;
  const int g = blockIdx.x;
  const int seg = g % nseg, y = (g / nseg) % a.ny, z = g / (nseg * a.ny);
  const int x0 = seg * FM_G;
  const int nown = (a.nx - x0 < FM_G) ? a.nx - x0 : FM_G;  // own cells x0 .. x0 + nown - 1
  // staged cell (r, c): row r (dy, dz), column c -> x = x0 - 1 + c
  if (tid < FM_CELLS) {
    const int r = tid / FM_W, c = tid % FM_W;
    const int dy = (r == 0) ? 0 : (r == 1 ? 1 : r - 3), dz = (r < 2) ? 0 : 1;
    int cx = x0 - 1 + c, cy = y + dy, cz = z + dz;
    cx = (cx % a.nx + a.nx) % a.nx;
    cy = (cy % a.ny + a.ny) % a.ny;
    cz = (cz % a.nz + a.nz) % a.nz;
    const int cell = (cz * a.ny + cy) * a.nx + cx;
    const int s0 = a.start[cell];
    cgs[tid] = s0;
    cst[tid + 1] = a.start[cell + 1] - s0;
  }
  __syncthreads();
  if (tid == 0) {
    cst[0] = 0;
    for (int q = 0; q < FM_CELLS; ++q) cst[q + 1] += cst[q];
  }
  __syncthreads();
  const int M = cst[FM_CELLS];
  const bool fits = M <= FM_CAP;
  // own cells' validity: staged in full and at most 32 molecules each
  if (tid < nown) {
    const int pop = cst[tid + 2] - cst[tid + 1];
    a.fm_ok[(z * a.ny + y) * a.nx + x0 + tid] = (fits && pop <= 32) ? 1 : 0;
  }
  if (!fits) return;  // uniform
  // stage FP32 positions in the frame of own cell x0's centre
  for (int m = tid; m < M; m += 256) {
    int q = 0;  // staged cell of m: the last q with cst[q] <= m
    for (int step = 32; step > 0; step >>= 1)
      if (q + step < FM_CELLS && cst[q + step] <= m) q += step;
    const int r = q / FM_W, c = q % FM_W;
    const double ox = (double)(c - 1) * a.side[0];
    const double oy = (double)((r == 0) ? 0 : (r == 1 ? 1 : r - 3)) * a.side[1];
    const double oz = (double)((r < 2) ? 0 : 1) * a.side[2];
    const double4 v = a.sorted[cgs[q] + (m - cst[q])];
    sp[m] = make_float4((float)(v.x + ox), (float)(v.y + oy), (float)(v.z + oz), 0.f);
  }
  __syncthreads();
  // lanes = (own molecule, forward row) pairs: staged row r holds, for
  // (dy, dz) = (0,0), (1,0), (-1,1), (0,1), (1,1), the cells at dx = 0, 1
  // (row 0) or dx = -1, 0, 1; they are contiguous in the staging, and one
  // lane builds their 2-3 words (forward index k = 0, 1 in row 0, else
  // 2 + 3 (r - 1) + dx + 1)
  const int own0 = cst[1], nmol = cst[1 + nown] - own0;
  // consecutive lanes take consecutive molecules of one row: the lanes of
  // one own cell read the same candidates at the same time (LDS broadcast)
  for (int task = tid; task < FM_ROWS * nmol; task += 256) {
    const int r = task / nmol, ai = task - nmol * r;
    const int am = own0 + ai;  // staged index of the molecule
    int ca = 1;
    while (cst[ca + 1] <= am) ++ca;  // its staged cell (row 0)
    if (cst[ca + 1] - cst[ca] > 32) continue;
    const float4 pa = sp[am];
    const int slot_a = cgs[ca] + (am - cst[ca]);
    const int dx0 = (r == 0) ? 0 : -1;
    for (int dx = dx0; dx <= 1; ++dx) {
      const int k = (r == 0) ? dx : 2 + 3 * (r - 1) + dx + 1;
      const int cb = r * FM_W + ca + dx;
      const int b0 = cst[cb], pop = cst[cb + 1] - b0;
      if (pop > 32) continue;
      const int t0 = (k == 0) ? am - cst[ca] + 1 : 0;
      uint32_t word = 0u, maybe = 0u;  // inside; inside the guard band
      for (int t = t0; t < pop; ++t) {
        const float4 pb = sp[b0 + t];
        const float ex = pa.x - pb.x, ey = pa.y - pb.y, ez = pa.z - pb.z;
        const float r2 = ex * ex + ey * ey + ez * ez;
        word |= (r2 < a.lo2 ? 1u : 0u) << t;
        maybe |= (r2 < a.hi2 ? 1u : 0u) << t;
      }
      maybe &= ~word;
      while (maybe) {  // the exact decision (oracle expression) inside the band
        const int t = __builtin_ctz(maybe);
        maybe &= maybe - 1u;
        const int ia = (int)a.sorted[slot_a].w;
        const int ib = (int)a.sorted[cgs[cb] + t].w;
        if (exact_r2(a.pos, ia, ib, a.box[0], a.box[1], a.box[2]) < a.rc2) word |= 1u << t;
      }
      a.fmask[(size_t)slot_a * 14 + k] = word;
    }
  }
}

// ---------------------------------------------------------------------------
// Fast tiers: at most 64*NW molecules per block (NW = 2: 128, NW = 4: 256).
// Upper-triangle pair masks are built one wave per row.  One pass over the
// mask words lists the upper pairs (PCAP at most) and the upper pairs the
// block owns (PCAP/2 at most).  One pass over the pairs forms each pair's
// owned third molecules K(i,j) = mask_i & mask_j & allowed(code_i & code_j)
// word by word, counts the work items per size class and lists the non-empty
// (pair, word) entries; a second pass over only those entries cuts each K
// word into items of at most NCLS third molecules and places them, largest
// class first, at slots taken from per-class LDS cursors.  Placement order
// within a class does not matter: every force and energy term is summed as a
// fixed-point integer.
// ---------------------------------------------------------------------------
// x in units of 2^-32, rounded to nearest, as a two's-complement 64-bit
// value, for |x| < FAST_LIMIT (the caller checks the bound): adding 1.5 * 2^20
// in FP64 leaves x * 2^32 + 2^51 in the 52 mantissa bits (the sum lies in
// [2^20, 2^21), whose ulp is 2^-32), and one integer subtraction removes the
// exponent field and the offset.
constexpr float FAST_LIMIT = 262144.f;  // 2^18
__device__ __forceinline__ u64 to_fix_m(double x) {
  const double t = x + 1572864.0;
  return (u64)__double_as_longlong(t) - 0x4138000000000000ull;
}
__device__ __forceinline__ u64 to_fix_m(float x) { return to_fix_m((double)x); }

// Adds (x, y, z) with to_fix_m; *far is raised when the bound is not met
// (NaN included).
__device__ __forceinline__ void add_fix_m(u64* ax, u64* ay, u64* az, int m, double x, double y, double z, int* far) {
  *far |= !(fabs(x) + fabs(y) + fabs(z) < (double)FAST_LIMIT);
  atomicAdd(&ax[m], to_fix_m(x));
  atomicAdd(&ay[m], to_fix_m(y));
  atomicAdd(&az[m], to_fix_m(z));
}

// Work items hold at most NCLS third molecules: a K word of more bits is cut
// into runs of NCLS set bits, lowest first, and a shorter last run, so that
// the items of a wave have near-equal sizes.
constexpr int NCLS = 12;
// work items of the four-word tier (2x2x2 blocks at rc 3.0 and density 0.75
// need about 2,000, 2,500 at the 99th percentile)
constexpr int WIDE_KCAP = 3072;

// Pairs (i, j), i before j, whose corner codes can own a third molecule:
// bit c' of PAIR_OK[c] is set iff some corner k >= c' (the third comes after
// j, corner by corner) has k & c & c' == 0.  Rows of corners 4-7 own none.
__device__ __forceinline__ uint32_t pair_ok(int c) {
  return c < 4 ? ((0x383C7EFFu >> (8 * c)) & 0xffu) : 0u;
}

template <int NW, int PCAP, int KCAP>
struct LdsTier {
  static constexpr int MAXB = 64 * NW;
  BlockHead h;
  float4 sp[MAXB];   // FP32 coordinates, .w = residual of x
  float2 slo[MAXB];  // residuals of y and z
  u64 ax[MAXB], ay[MAXB], az[MAXB];
  alignas(16) u64 mask[MAXB * NW];  // bits j > i only
  u64 allow[8 * NW];
  u64 ucol[4 * NW];      // bits j of corners c' with pair_ok(c) bit c', rows c < 4
  uint16_t plist[PCAP];  // i | j << 8: owned upper pairs, then the others that can own a third molecule
  u64 kset[KCAP];         // third molecules of each item (bits of word w)
  uint16_t kmeta[KCAP];   // q | w << 13: pair plist[q], mask word w
  uint16_t nelist[KCAP];  // the same for every non-empty K word
  u64 tot[4][16];            // block totals in 16 slots (by lane): e_lj', w_lj', e_atm' (2^-32 units), LJ pairs
  int32_t ccnt[NCLS + 1];    // items per class
  int32_t cfull[16];         // items of NCLS third molecules, in 16 slots (by lane)
  int32_t cursor[NCLS + 1];
  int32_t nne;  // entries of nelist
  int32_t cnt2[NWAVE];
  uint8_t scode[MAXB];
};

// One ATM triplet of the pair (i, j) with third molecule k, in FP32, for the
// per-pair accumulation of the fast path.  With c_x, c_y, c_z as in
// atm_triplet (eq. forcepairs): F_i(j)k = c_x r_ij is summed over k as a
// scalar (r_ij is fixed for the pair), F_i(k)j = c_y r_ik and F_j(k)i =
// c_z r_jk are added to the pair's accumulators, and F_k = -(c_y r_ik +
// c_z r_jk) (eq. newton3rdlaw) is returned.  x = |r_ij|^2 and ix = 1/x are
// the pair's.  Adds the energy term without nu to *eu and raises *mx to
// max(|c_y|, |c_z|): every side of a triplet the fast path takes is within
// rc, so |F_k| <= (|c_y| + |c_z|) rc <= 2 rc max(|c_y|, |c_z|) per component.
struct PairAcc {
  float cx, fix, fiy, fiz, fjx, fjy, fjz, eu, mx;
};
__device__ __forceinline__ void atm_third(const float4 pi, const float4 pj, const float4 pk, float x, float ix,
                                          float k3nu, float k15nu, float k075nu, PairAcc& q, float& fkx, float& fky,
                                          float& fkz) {
  const float ikx = pi.x - pk.x, iky = pi.y - pk.y, ikz = pi.z - pk.z;
  const float jkx = pj.x - pk.x, jky = pj.y - pk.y, jkz = pj.z - pk.z;
  const float y = ikx * ikx + iky * iky + ikz * ikz;
  const float z = jkx * jkx + jky * jky + jkz * jkz;
  // eq. (atm) in squared sides, as in atm_triplet
  const float s = x + y + z;
  const float A = fmaf(-2.f, x, s), B = fmaf(-2.f, y, s), C = fmaf(-2.f, z, s);
  const float AB = A * B, AC = A * C, BC = B * C;
  const float P = AB * C;
  const float S = AB + AC + BC;
  const float xy = x * y, xz = x * z;
  const float t1 = __builtin_amdgcn_rsqf(xy * z);
  const float t2 = t1 * t1, t3 = t2 * t1, t5 = t3 * t2;
  const float u = P * t5;
  q.eu += fmaf(0.375f, u, t3);
  const float G = fmaf(k15nu, u, k3nu * t3);
  const float H = k075nu * t5;
  // 1/y = xz t2, 1/z = xy t2; -H dP/dx = 2H BC - H S (cyclic)
  const float Gt2 = G * t2, H2 = H + H, nHS = -H * S;
  const float cx = fmaf(G, ix, fmaf(H2, BC, nHS));
  const float cy = fmaf(Gt2, xz, fmaf(H2, AC, nHS));
  const float cz = fmaf(Gt2, xy, fmaf(H2, AB, nHS));
  q.cx += cx;
  q.fix = fmaf(cy, ikx, q.fix);
  q.fiy = fmaf(cy, iky, q.fiy);
  q.fiz = fmaf(cy, ikz, q.fiz);
  q.fjx = fmaf(cz, jkx, q.fjx);
  q.fjy = fmaf(cz, jky, q.fjy);
  q.fjz = fmaf(cz, jkz, q.fjz);
  fkx = -fmaf(cy, ikx, cz * jkx);
  fky = -fmaf(cy, iky, cz * jky);
  fkz = -fmaf(cy, ikz, cz * jkz);
  q.mx = fmaxf(q.mx, fmaxf(fabsf(cy), fabsf(cz)));
}

template <int NW, int PCAP, int KCAP>
__device__ bool do_block_fast(const ForceArgs& a, int b, LdsTier<NW, PCAP, KCAP>& L) {
  constexpr int MAXB = 64 * NW;
  constexpr int WPT = MAXB * NW / WG;  // mask words per thread in the list pass
  static_assert(MAXB * NW % WG == 0 && WPT >= 1, "whole mask words per thread");
  static_assert(KCAP < 65536 && PCAP <= 8192 && PCAP < 65536, "16-bit counts and 13-bit pair indices");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool do_lj = (a.terms & ATM3_TERM_LJ) != 0;
  const bool do_atm = (a.terms & ATM3_TERM_ATM) != 0;

  const int n = block_cells(a, b, L.h);
  if (n > MAXB) return false;
  block_stage(a, L.h, n, nullptr, L.sp, L.slo, L.ax, L.ay, L.az, L.scode, nullptr, nullptr);
  if (tid == 0) L.nne = 0;
  if (tid <= NCLS) L.ccnt[tid] = 0;
  if (tid < 64) L.tot[tid >> 4][tid & 15] = 0ull;
  if (tid < 16) L.cfull[tid] = 0;
  const bool use_fm = (L.h.okc[0] & L.h.okc[1] & L.h.okc[2] & L.h.okc[3] & L.h.okc[4] & L.h.okc[5] &
                       L.h.okc[6] & L.h.okc[7]) != 0;
  __syncthreads();
  block_allow<NW>(n, L.scode, L.allow);
  for (int item = wave; item < 4 * NW; item += NWAVE) {  // ucol[c][w], c < 4
    const int c = item / NW, w = item % NW;
    const int j = 64 * w + lane;
    const bool ok = (j < n) && ((pair_ok(c) >> L.scode[j]) & 1u);
    const u64 bits = __ballot(ok);
    if (lane == 0) L.ucol[item] = bits;
  }

  // 2. upper-triangle mask words.  When every corner cell has forward-shell
  //    words (k_fmask), row i of corner o is assembled from the words of the
  //    corners o' >= o: their offsets o' - o are forward offsets, and corner
  //    o' occupies staged positions cbase[o'] ...
  if (use_fm) {
    // one thread per mask word (row i, word w): the words of the corners
    // o2 >= corner of i whose staged range meets word w, shifted into
    // place and ORed in registers, then one store (rows past n are zero)
    for (int q = tid; q < MAXB * NW; q += WG) {
      const int i = q / NW, w = q - (q / NW) * NW;
      u64 acc = 0ull;
      if (i < n) {
        const int o = L.scode[i];
        const size_t rowbase = (size_t)(L.h.cstart[o] + (i - L.h.cbase[o])) * 14;
#pragma unroll
        for (int o2 = 0; o2 < 8; ++o2) {
          const int sh = L.h.cbase[o2] - 64 * w;  // bit of the corner's first molecule in word w
          if (o2 < o || sh >= 64 || L.h.cbase[o2 + 1] - 64 * w <= 0 || L.h.cbase[o2 + 1] == L.h.cbase[o2]) continue;
          const int dx = (o2 & 1) - (o & 1), dy = ((o2 >> 1) & 1) - ((o >> 1) & 1), dz = (o2 >> 2) - (o >> 2);
          const u64 wd = a.fmask[rowbase + fwd_index(dx, dy, dz)];
          acc |= sh >= 0 ? (wd << sh) : (wd >> (-sh));
        }
      }
      L.mask[q] = acc;
    }
  } else {
    //  ... else one wave per row (rows wave, wave + 4, ...).  Lane l holds
    //  molecules l + 64 w in registers (a far-away position past the last
    //  molecule); a row's position is read from them with readlane (scalar
    //  registers), which keeps this phase off the LDS.
    const float4 far4 = make_float4(1e18f, 1e18f, 1e18f, 0.f);
    float4 pj[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) pj[w] = (64 * w + lane < n) ? L.sp[64 * w + lane] : far4;
    auto rl = [](const float4 v, int l) {  // l wave-uniform
      return make_float4(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l)),
                         __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l)),
                         __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.z), l)), 0.f);
    };
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    for (int i = wv; i < n; i += NWAVE) {
      const int wi = i >> 6, li = i & 63;
      float4 pi = rl(pj[0], li);
#pragma unroll
      for (int w = 1; w < NW; ++w)
        if (w == wi) pi = rl(pj[w], li);
      u64 words[NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        words[w] = 0ull;
        if (w < wi) continue;
        const float r2 = dist2f(pi, pj[w]);
        const u64 tri = (w > wi) ? ~0ull : (li == 63 ? 0ull : (~0ull << (li + 1)));
        u64 bits = __ballot(r2 < a.lo2) & tri;
        const u64 maybe = __ballot(r2 < a.hi2) & tri & ~bits;
        if (maybe) bits |= exact_bits(a, i, w, maybe, L.h, L.scode);
        words[w] = bits;
      }
      if (lane == 0) {
#pragma unroll
        for (int w = 0; w < NW; w += 2)
          *reinterpret_cast<ulonglong2*>(&L.mask[i * NW + w]) = make_ulonglong2(words[w], words[w + 1]);
      }
    }
    for (int i = n + wv; i < MAXB; i += NWAVE)
      if (lane < NW) L.mask[i * NW + lane] = 0ull;
  }
  __syncthreads();

  // 3. pair list: thread t lists the bits of mask words t, t + WG, ...; the
  //    pairs the block owns (corner codes AND to 0, LJ and ATM) come first,
  //    then the other pairs that can own a third molecule (ATM only); both
  //    offsets come from one scan of (owned count | other count << 16)
  int np, no;
  {
    u64 wo[WPT], wn[WPT];
    int packed = 0;
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const int wd = tid + WG * k, ri = wd / NW, rw = wd % NW;
      const u64 m = L.mask[wd];
      const int ci = (ri < n) ? L.scode[ri] : 4;
      wo[k] = (ri < n) ? (m & L.allow[ci * NW + rw]) : 0ull;
      wn[k] = (ci < 4) ? (m & L.ucol[ci * NW + rw] & ~wo[k]) : 0ull;
      packed += __popcll(wo[k]) | (__popcll(wn[k]) << 16);
    }
    const int incl = wave_incl_scan(packed);
    if (lane == 63) L.cnt2[wave] = incl;
    __syncthreads();
    int pre = incl - packed, tot = 0;
    for (int w = 0; w < NWAVE; ++w) {
      const int v = L.cnt2[w];
      if (w < wave) pre += v;
      tot += v;
    }
    no = tot & 0xffff;
    np = no + (tot >> 16);
    if (np > PCAP) return false;  // uniform: block totals
    int o = pre & 0xffff, p = no + (pre >> 16);
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const int wd = tid + WG * k, ri = wd / NW, jb = 64 * (wd % NW);
      // bits walked as 32-bit halves (one find-first-set and two operations
      // per bit instead of their 64-bit sequences)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int base = ri | ((jb + 32 * h) << 8);
        uint32_t x = (uint32_t)(wo[k] >> (32 * h)), y = (uint32_t)(wn[k] >> (32 * h));
        while (x) {
          L.plist[o++] = (uint16_t)(base + (__builtin_ctz(x) << 8));
          x &= x - 1u;
        }
        while (y) {
          L.plist[p++] = (uint16_t)(base + (__builtin_ctz(y) << 8));
          y &= y - 1u;
        }
      }
    }
  }
  __syncthreads();

  double e_lj = 0.0, w_lj = 0.0;
  long long n_pair = 0;
  int far = 0;  // a value beyond FAST_LIMIT: the block goes to the general path

  int ntr = 0, mytr = 0, myfull = 0;
  // 4a. per pair q (lanes = pairs, rounds of WG): the LJ term of the owned
  //     pairs (q < no; FP64 on the coordinates with their residuals), and
  //     each non-zero word of K(i,j) as an entry of nelist, its items
  //     counted per size class
  // lane tid takes pair q0 + (37 tid mod WG): neighbouring lanes then hold
  // pairs of different rows (the list is row by row), whose F_i atomics do
  // not collide on one address
  const int nq = do_atm ? np : no;
  const int qp = (tid * 37) & (WG - 1);
  for (int q0 = 0; q0 < nq; q0 += WG) {  // uniform trip count
    const int q = q0 + qp;
    uint32_t wm = 0u;  // bit w: word w of K(i,j) is non-empty
    if (q < nq) {
      const int e = L.plist[q];
      const int i = e & 255, j = e >> 8;
      if (do_lj && q < no) {
        const float4 hi = L.sp[i], hj = L.sp[j];
        const float2 li = L.slo[i], lj = L.slo[j];
        const double ex = ((double)hi.x - (double)hj.x) + ((double)hi.w - (double)hj.w);
        const double ey = ((double)hi.y - (double)hj.y) + ((double)li.x - (double)lj.x);
        const double ez = ((double)hi.z - (double)hj.z) + ((double)li.y - (double)lj.y);
        const double f = lj_pair(ex, ey, ez, a.sig2, a.eps24, &e_lj, &w_lj);
        add_fix_m(L.ax, L.ay, L.az, i, f * ex, f * ey, f * ez, &far);
        add_fix_m(L.ax, L.ay, L.az, j, -f * ex, -f * ey, -f * ez, &far);
        ++n_pair;
      }
      if (do_atm) {
        const u64* al = &L.allow[(L.scode[i] & L.scode[j]) * NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const u64 K = L.mask[i * NW + w] & L.mask[j * NW + w] & al[w];
          const int c = __popcll(K);
          if (c) {
            mytr += c;
            const int full = (c - 1) / NCLS;  // runs of NCLS bits, then the rest
            myfull += full;
            atomicAdd(&L.ccnt[c - NCLS * full], 1);
            wm |= 1u << w;
          }
        }
      }
    }
    if (do_atm) {  // append the entries to nelist (offsets by a wave scan)
      const int cnt = __popc(wm);
      int at = atomicAdd(&L.nne, cnt);
#pragma unroll
      for (int w = 0; w < NW; ++w)
        if ((wm >> w) & 1u) {
          if (at < KCAP) L.nelist[at] = (uint16_t)(q | (w << 13));
          ++at;
        }
    }
  }
  {  // this thread's LJ totals into the block totals (fixed point, rounded
     // to the nearest unit, so that the many per-thread sums carry no bias;
     // 16 slots, so that the lanes of a wave do not all add to one address)
    int bad = 0;
    if (e_lj != 0.0) atomicAdd(&L.tot[0][lane & 15], to_fix(e_lj + 0.5 * FIX_INV, &bad));
    if (w_lj != 0.0) atomicAdd(&L.tot[1][lane & 15], to_fix(w_lj + 0.5 * FIX_INV, &bad));
    if (n_pair) atomicAdd(&L.tot[3][lane & 15], (u64)n_pair);
    far |= bad;
  }
  __syncthreads();  // the LJ phase's chunks are done
  if (do_atm) {
    // class totals (block-uniform) and the class cursors, largest first
    const int wt = wave_incl_scan(mytr);
    if (lane == 63) L.cnt2[wave] = wt;
    if (myfull) atomicAdd(&L.cfull[lane & 15], myfull);
    __syncthreads();
    for (int v = 0; v < NWAVE; ++v) ntr += L.cnt2[v];
    if (wave == 0) {
      // lane l holds class NCLS - l (largest first); a scan gives the
      // cursors, and the total goes to ccnt[0] (no item has 0 molecules)
      int cnt = 0;
      if (lane < NCLS) cnt = L.ccnt[NCLS - lane];
      if (lane == 0)
        for (int s = 0; s < 16; ++s) cnt += L.cfull[s];
      const int incl = wave_incl_scan(cnt);
      if (lane < NCLS) L.cursor[NCLS - lane] = incl - cnt;
      if (lane == NCLS - 1) L.ccnt[0] = incl;
    }
    __syncthreads();
    const int ne = L.ccnt[0], nne = L.nne;
    if (ne > KCAP || nne > KCAP) return false;  // uniform: block totals

    // 4b. items: the non-empty K words (lanes = entries, entry 37 tid mod WG
    //     + WG r, so that neighbouring lanes hold pairs of different rows,
    //     whose K overlap less: fewer same-address F_k atomics later) cut
    //     into runs and placed at their class cursors
    //    Three entries per thread at a time: their K words, then the slots
    //    of their first items (independent atomics, issued together), then
    //    the stores and any further items
    for (int r0 = 0; WG * r0 < nne; r0 += 3) {
      u64 Kb[3];
      int vb[3], slot[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int p = ((tid * 37) & (WG - 1)) + WG * (r0 + b);
        Kb[b] = 0ull;
        vb[b] = 0;
        if (p < nne) {
          const int v = L.nelist[p];
          const int e = L.plist[v & 8191], w = v >> 13;
          const int i = e & 255, j = e >> 8;
          Kb[b] = L.mask[i * NW + w] & L.mask[j * NW + w] & L.allow[(L.scode[i] & L.scode[j]) * NW + w];
          vb[b] = v;
        }
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int pc = __popcll(Kb[b]), c = pc < NCLS ? pc : NCLS;
        slot[b] = c ? atomicAdd(&L.cursor[c], 1) : 0;
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        u64 K = Kb[b];
        int at = slot[b];
        while (K) {
          u64 run = K;
          if (__popcll(K) > NCLS) {  // the lowest NCLS bits
            u64 x = K;
#pragma unroll
            for (int t = 0; t < NCLS; ++t) x &= x - 1ull;
            run = K ^ x;
          }
          K ^= run;
          L.kset[at] = run;
          L.kmeta[at] = (uint16_t)vb[b];
          if (K) {
            const int pc = __popcll(K);
            at = atomicAdd(&L.cursor[pc < NCLS ? pc : NCLS], 1);
          }
        }
      }
    }
    __syncthreads();

    // 5. ATM: each thread takes whole items, item tid + WG r in round r, so
    //    the 64 items of a wave have similar sizes and finish together; the
    //    pair's sums stay in registers for an item and only F_k is added per
    //    triplet; the item's energy is added in fixed point.  All of it is
    //    converted with to_fix_m; a value beyond its range sends the block to
    //    the general path.
    u64 eacc = 0ull;
    float tmx = 0.f;  // max of the item totals (NaN-propagating)
    float cmx = 0.f;  // max |c_y|, |c_z|: |F_k| stays below 2 rc cmx
    for (int p = tid; p < ne; p += WG) {
      const int v = L.kmeta[p];
      const int e = L.plist[v & 8191];
      const int ci = e & 255, cj = e >> 8;
      // items of pairs with an odd j walk K from the top: pairs of one row
      // have overlapping K, and lanes holding them would otherwise hit the
      // same F_k address in the same instruction.  The direction is a
      // property of the item, not of the lane it lands on, so that every
      // item's FP32 sums are the same from run to run.  Bit t of the walked
      // word is molecule 64 w + t (upward) or 64 w + 63 - t: its byte
      // offset in sp is o16 + s16 t, half of it in ax
      const bool up = (cj & 1) == 0;
      const int o16 = 16 * (64 * (v >> 13) + (up ? 0 : 63)), s16 = up ? 16 : -16;
      u64 K = L.kset[p];
      if (!up) K = __builtin_bitreverse64(K);
      const float4 pi = L.sp[ci], pj = L.sp[cj];
      const float ijx = pi.x - pj.x, ijy = pi.y - pj.y, ijz = pi.z - pj.z;
      const float x = ijx * ijx + ijy * ijy + ijz * ijz;
      const float ix = __builtin_amdgcn_rcpf(x);
      PairAcc q = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, cmx};
      do {  // an item is a non-empty run of K
        const int t = __builtin_ctzll(K);
        K &= K - 1ull;
        const int a16 = o16 + __mul24(t, s16), a8 = a16 >> 1;
        const float4 pk = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(L.sp) + a16);
        float fkx, fky, fkz;
        atm_third(pi, pj, pk, x, ix, a.k3nu, a.k15nu, a.k075nu, q, fkx, fky, fkz);
        atomicAdd(reinterpret_cast<u64*>(reinterpret_cast<char*>(L.ax) + a8), to_fix_m(fkx));
        atomicAdd(reinterpret_cast<u64*>(reinterpret_cast<char*>(L.ay) + a8), to_fix_m(fky));
        atomicAdd(reinterpret_cast<u64*>(reinterpret_cast<char*>(L.az) + a8), to_fix_m(fkz));
      } while (K);
      cmx = q.mx;
      const float fix = fmaf(q.cx, ijx, q.fix), fiy = fmaf(q.cx, ijy, q.fiy), fiz = fmaf(q.cx, ijz, q.fiz);
      const float fjx = fmaf(-q.cx, ijx, q.fjx), fjy = fmaf(-q.cx, ijy, q.fjy), fjz = fmaf(-q.cx, ijz, q.fjz);
      // a NaN or infinite c_y or c_z makes F_i or F_j NaN or infinite as well
      const float tot = fabsf(fix) + fabsf(fiy) + fabsf(fiz) + fabsf(fjx) + fabsf(fjy) + fabsf(fjz) + fabsf(q.eu);
      tmx = fmaxf(tmx, tot == tot ? tot : INFINITY);
      atomicAdd(&L.ax[ci], to_fix_m(fix));
      atomicAdd(&L.ay[ci], to_fix_m(fiy));
      atomicAdd(&L.az[ci], to_fix_m(fiz));
      atomicAdd(&L.ax[cj], to_fix_m(fjx));
      atomicAdd(&L.ay[cj], to_fix_m(fjy));
      atomicAdd(&L.az[cj], to_fix_m(fjz));
      eacc += to_fix_m(q.eu);
    }
    // sides within sqrt(hi2) (the FP32 guard above rc), with 2.5% margin
    far |= !(cmx * (2.05f * sqrtf(a.hi2)) < FAST_LIMIT);
    far |= !(tmx < FAST_LIMIT);
    if (eacc) atomicAdd(&L.tot[2][lane & 15], eacc);
  }
  if (__syncthreads_or(far)) return false;  // uniform
  // per-corner partial forces (each (corner, molecule) written by exactly
  // one block) and the block's totals
  const int N = a.ntot;
  for (int q = tid; q < n; q += WG) {
    const int o = L.scode[q], s = L.h.cstart[o] + (q - L.h.cbase[o]);
    a.fpart[(int64_t)(o * 3 + 0) * N + s] = L.ax[q];
    a.fpart[(int64_t)(o * 3 + 1) * N + s] = L.ay[q];
    a.fpart[(int64_t)(o * 3 + 2) * N + s] = L.az[q];
  }
  if (tid < 4) {
    u64 s = 0ull;
    for (int k = 0; k < 16; ++k) s += L.tot[tid][k];
    if (tid < 3)
      a.blkd[3 * (int64_t)b + tid] = from_fix(s);
    else
      a.blki[2 * (int64_t)b + 0] = (int32_t)s;
  }
  if (tid == 0) a.blki[2 * (int64_t)b + 1] = do_atm ? ntr : 0;
  return true;
}

// ---------------------------------------------------------------------------
// General path for blocks of up to 64*NW molecules with any number of pairs
// and triplets: pairs are compacted by ballot + prefix offsets in rounds of
// PCAP, triplets materialised in rounds of TCAP.
// ---------------------------------------------------------------------------
template <int NW, int PCAP, int TCAP>
struct LdsBig {
  static constexpr int MAXB = 64 * NW;
  BlockHead h;
  double4 dp[MAXB];
  float4 sp[MAXB];
  u64 ax[MAXB], ay[MAXB], az[MAXB];
  u64 mask[MAXB * NW];
  u64 allow[8 * NW];
  int32_t sorig[MAXB];
  int32_t sslot[MAXB];
  int32_t pw[MAXB * NW];  // upper-pair count per row word -> offsets
  uint32_t plist[PCAP];   // i | j << 10
  int32_t pcnt[PCAP];     // triplets per pair -> offsets
  uint32_t tlist[TCAP];   // i | j << 10 | k << 20
  int32_t wsum[NWAVE];    // block_scan scratch
  uint8_t scode[MAXB];
};

// Exclusive prefix sum of data[0..M) in place, all threads of the block;
// returns the total.  Each thread scans a contiguous chunk.
__device__ int block_scan(int32_t* data, int M, int32_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (M + WG - 1) / WG;
  const int lo = tid * per < M ? tid * per : M;
  const int hi = lo + per < M ? lo + per : M;
  int s = 0;
  for (int q = lo; q < hi; ++q) s += data[q];
  const int incl = wave_incl_scan(s);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int wpre = 0, total = 0;
  for (int q = 0; q < NWAVE; ++q) {
    const int v = wsum[q];
    if (q < wave) wpre += v;
    total += v;
  }
  int run = wpre + incl - s;
  for (int q = lo; q < hi; ++q) {
    const int v = data[q];
    data[q] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

template <int NW, int PCAP, int TCAP>
__device__ bool do_block_big(const ForceArgs& a, int b, LdsBig<NW, PCAP, TCAP>& L) {
  constexpr int MAXB = 64 * NW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool do_lj = (a.terms & ATM3_TERM_LJ) != 0;
  const bool do_atm = (a.terms & ATM3_TERM_ATM) != 0;

  const int n = block_cells(a, b, L.h);
  if (n > MAXB) return false;
  block_stage(a, L.h, n, L.dp, L.sp, nullptr, L.ax, L.ay, L.az, L.scode, L.sorig, L.sslot);
  __syncthreads();
  block_allow<NW>(n, L.scode, L.allow);

  // upper-triangle masks
  for (int i = wave; i < n; i += NWAVE) {
    const float4 pi = L.sp[i];
    for (int w = i >> 6; w < NW; ++w) {
      const int j = 64 * w + lane;
      const float4 pj = (j < n) ? L.sp[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      const u64 bits = mask_word(a, i, w, n, pi, pj, L.sorig);
      if (lane == 0) L.mask[i * NW + w] = bits;
    }
    if (lane == 0)
      for (int w = 0; w < (i >> 6); ++w) L.mask[i * NW + w] = 0ull;
  }
  __syncthreads();
  for (int q = tid; q < n * NW; q += WG) L.pw[q] = __popcll(L.mask[q]);
  __syncthreads();
  const int npairs = block_scan(L.pw, n * NW, L.wsum);

  double e_lj = 0.0, w_lj = 0.0, e_atm = 0.0;
  long long n_pair = 0;
  int n_trip = 0, bad = 0;
  for (int pr = 0; pr < npairs; pr += PCAP) {
    const int np = (npairs - pr < PCAP) ? npairs - pr : PCAP;
    for (int item = wave; item < n * NW; item += NWAVE) {
      const int i = item / NW, w = item % NW;
      const u64 bits = L.mask[item];
      const int base = L.pw[item];
      if (base >= pr + np || base + __popcll(bits) <= pr) continue;
      if ((bits >> lane) & 1ull) {
        const int p = base + __popcll(bits & ((1ull << lane) - 1ull));
        if (p >= pr && p < pr + np) L.plist[p - pr] = (uint32_t)i | ((uint32_t)(64 * w + lane) << 10);
      }
    }
    __syncthreads();

    const int mp = ((np + WG - 1) / WG) | 1;
    const int q0 = tid * mp < np ? tid * mp : np;
    const int q1 = q0 + mp < np ? q0 + mp : np;
    {
      int cur = -1;
      double fx = 0.0, fy = 0.0, fz = 0.0;
      for (int q = q0; q < q1; ++q) {
        const uint32_t e = L.plist[q];
        const int i = e & 1023, j = e >> 10;
        const int cij = L.scode[i] & L.scode[j];
        if (do_atm) {
          const u64* al = &L.allow[cij * NW];
          int c = 0;
          for (int w2 = j >> 6; w2 < NW; ++w2)
            c += __popcll(L.mask[i * NW + w2] & L.mask[j * NW + w2] & al[w2] & above(j, w2));
          L.pcnt[q] = c;
        }
        if (do_lj && cij == 0) {
          if (i != cur) {
            if (cur >= 0) add_fix(L.ax, L.ay, L.az, cur, fx, fy, fz, &bad);
            cur = i;
            fx = fy = fz = 0.0;
          }
          const double4 di = L.dp[i], dj = L.dp[j];
          const double ex = di.x - dj.x, ey = di.y - dj.y, ez = di.z - dj.z;
          const double f = lj_pair(ex, ey, ez, a.sig2, a.eps24, &e_lj, &w_lj);
          fx += f * ex;
          fy += f * ey;
          fz += f * ez;
          add_fix(L.ax, L.ay, L.az, j, -f * ex, -f * ey, -f * ez, &bad);
          ++n_pair;
        }
      }
      if (cur >= 0) add_fix(L.ax, L.ay, L.az, cur, fx, fy, fz, &bad);
    }
    __syncthreads();
    if (!do_atm) continue;

    const int ntr = block_scan(L.pcnt, np, L.wsum);
    n_trip += ntr;
    for (int tr = 0; tr < ntr; tr += TCAP) {
      const int nt = (ntr - tr < TCAP) ? ntr - tr : TCAP;
      for (int q = q0; q < q1; ++q) {
        int off = L.pcnt[q];
        const int end = (q + 1 < np) ? L.pcnt[q + 1] : ntr;
        if (end <= tr || off >= tr + nt) continue;
        const uint32_t e = L.plist[q];
        const int i = e & 1023, j = e >> 10;
        const u64* al = &L.allow[(L.scode[i] & L.scode[j]) * NW];
        for (int w2 = j >> 6; w2 < NW; ++w2) {
          u64 K = L.mask[i * NW + w2] & L.mask[j * NW + w2] & al[w2] & above(j, w2);
          while (K) {
            const int k = 64 * w2 + __builtin_ctzll(K);
            K &= K - 1;
            if (off >= tr && off < tr + nt) L.tlist[off - tr] = e | ((uint32_t)k << 20);
            ++off;
          }
        }
      }
      __syncthreads();
      const int m = ((nt + WG - 1) / WG) | 1;
      const int t0 = tid * m < nt ? tid * m : nt;
      const int t1 = t0 + m < nt ? t0 + m : nt;
      int ci = -1, cj = -1;
      float aix = 0.f, aiy = 0.f, aiz = 0.f, ajx = 0.f, ajy = 0.f, ajz = 0.f;
      float eu = 0.f;
      for (int t = t0; t < t1; ++t) {
        const uint32_t e = L.tlist[t];
        const int i = e & 1023, j = (e >> 10) & 1023, k = e >> 20;
        if (i != ci) {
          if (ci >= 0) add_fix(L.ax, L.ay, L.az, ci, aix, aiy, aiz, &bad);
          ci = i;
          aix = aiy = aiz = 0.f;
        }
        if (j != cj) {
          if (cj >= 0) add_fix(L.ax, L.ay, L.az, cj, ajx, ajy, ajz, &bad);
          cj = j;
          ajx = ajy = ajz = 0.f;
        }
        const Trip r = atm_triplet(L.sp[i], L.sp[j], L.sp[k], a.k3nu, a.k15nu, a.k075nu);
        eu += r.eu;
        aix += r.fix;
        aiy += r.fiy;
        aiz += r.fiz;
        ajx += r.fjx;
        ajy += r.fjy;
        ajz += r.fjz;
        add_fix(L.ax, L.ay, L.az, k, -(double)(r.fix + r.fjx), -(double)(r.fiy + r.fjy), -(double)(r.fiz + r.fjz),
                &bad);
      }
      if (ci >= 0) add_fix(L.ax, L.ay, L.az, ci, aix, aiy, aiz, &bad);
      if (cj >= 0) add_fix(L.ax, L.ay, L.az, cj, ajx, ajy, ajz, &bad);
      e_atm += (double)eu;
      __syncthreads();
    }
  }
  __syncthreads();
  block_flush(a, b, n, L.scode, L.sslot, L.ax, L.ay, L.az, L.h, e_lj, w_lj, e_atm, n_pair, n_trip, bad);
  return true;
}

// Regular blocks; blocks with more than 128 molecules, more than PCAP upper
// pairs, more than KCAP work items or a term beyond the rounding conversion
// are queued (defer[2..]) for the wider tier k_block_wide.
// Workgroup ids are spread over the 8 XCDs round-robin; consecutive ids on
// one XCD map to consecutive base cells so neighbouring blocks share its L2.
template <int PCAP, int KCAP>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(8))) void k_block(ForceArgs a) {
  __shared__ LdsTier<2, PCAP, KCAP> L;
  const int per = (a.ncells + 7) / 8;
  const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if ((blockIdx.x >> 3) >= per || b >= a.ncells) return;
  if (!do_block_fast<2, PCAP, KCAP>(a, b, L)) {
    if (threadIdx.x == 0) {
      const int q = atomicAdd(&a.defer[0], 1);
      a.defer[2 + q] = b;
    }
  }
}

// Four mask words per row (up to 256 molecules: dense liquids, or cutoffs
// up to about 3.2 at the benchmark density) and room for more pairs and
// items.  QUEUED: the blocks k_block queued, looped over by a grid that fills
// the GPU; else every base cell, one workgroup each (spread over the XCDs
// like k_block), for grids whose mean block is past the two-word tier.
// What still does not fit is queued (defer[ncells + 2..]) for k_block_big.
template <int PCAP, int KCAP, bool QUEUED>
__global__ __launch_bounds__(WG) void k_block_wide(ForceArgs a) {
  __shared__ LdsTier<4, PCAP, KCAP> L;
  int32_t* q2 = a.defer + 2 + a.ncells;
  int nq = 1, b = 0;
  if (QUEUED) {
    nq = a.defer[0];
  } else {
    const int per = (a.ncells + 7) / 8;
    b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if ((blockIdx.x >> 3) >= per || b >= a.ncells) return;
  }
  for (int q = QUEUED ? (int)blockIdx.x : 0; q < nq; q += QUEUED ? (int)gridDim.x : 1) {
    if (QUEUED) b = a.defer[2 + q];
    if (!do_block_fast<4, PCAP, KCAP>(a, b, L)) {
      if (threadIdx.x == 0) {
        const int t = atomicAdd(&q2[0], 1);
        q2[1 + t] = b;
      }
    }
    __syncthreads();
  }
}

template <int NW, int PCAP, int TCAP>
__global__ __launch_bounds__(WG) void k_block_big(ForceArgs a) {
  __shared__ LdsBig<NW, PCAP, TCAP> L;
  const int32_t* q2 = a.defer + 2 + a.ncells;
  const int nq = q2[0];
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    const int b = q2[1 + q];
    if (!do_block_big<NW, PCAP, TCAP>(a, b, L)) {
      if (threadIdx.x == 0) {
        atomicMin(&a.defer[1], ATM3_EOVERFLOW);
        for (int k = 0; k < 3; ++k) a.blkd[3 * (int64_t)b + k] = 0.0;
        a.blki[2 * (int64_t)b + 0] = 0;
        a.blki[2 * (int64_t)b + 1] = 0;
      }
      __syncthreads();
    }
  }
}

// Sum the eight corner partials of each molecule (exact, fixed point) and
// write the force in input order.
__global__ __launch_bounds__(256) void k_finalize(const u64* __restrict__ fpart, const int32_t* __restrict__ perm,
                                                  int32_t N, float* __restrict__ forces) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  float f[3];
  for (int d = 0; d < 3; ++d) {
    u64 acc = 0ull;
    for (int o = 0; o < 8; ++o) acc += fpart[(int64_t)(o * 3 + d) * N + s];
    f[d] = (float)from_fix(acc);
  }
  const int64_t i = perm[s];
  forces[3 * i + 0] = f[0];
  forces[3 * i + 1] = f[1];
  forces[3 * i + 2] = f[2];
}

// Partial sums of one reduction workgroup: 4 doubles, 2 counts.
struct RedPart {
  double d[4];
  long long c[2];
};

// Stage 1: workgroup g sums the blocks of its contiguous chunk, and the
// traversal's candidate count of each of those base cells.
struct Red1Args {
  const double* blkd;
  const int32_t* blki;
  const int32_t* start;
  int32_t nx, ny, nz, ncells;
  RedPart* part;
};

__device__ double candidates_of(const Red1Args& a, int b) {
  const int bx = b % a.nx, by = (b / a.nx) % a.ny, bz = b / (a.nx * a.ny);
  int32_t N[8];
  for (int o = 0; o < 8; ++o) {
    int cx = bx + (o & 1), cy = by + ((o >> 1) & 1), cz = bz + (o >> 2);
    if (cx >= a.nx) cx -= a.nx;
    if (cy >= a.ny) cy -= a.ny;
    if (cz >= a.nz) cz -= a.nz;
    const int c = (cz * a.ny + cy) * a.nx + cx;
    N[o] = a.start[c + 1] - a.start[c];
  }
  return candidates_3c08(N);
}

// 1,024 threads per workgroup: at 1M molecules (85,184 blocks) each thread
// takes one block, and 16 waves per CU hide the loads' latency
constexpr int R1WG = 1024;
__global__ __launch_bounds__(R1WG) void k_reduce1(Red1Args ra) {
  __shared__ double sd[4][R1WG / 64];
  __shared__ long long sc[2][R1WG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chunk = (ra.ncells + RBLK - 1) / RBLK;
  const int lo = blockIdx.x * chunk;
  const int hi = lo + chunk < ra.ncells ? lo + chunk : ra.ncells;
  double d[4] = {0, 0, 0, 0};
  long long c[2] = {0, 0};
  for (int b = lo + tid; b < hi; b += R1WG) {
    for (int k = 0; k < 3; ++k) d[k] += ra.blkd[3 * (int64_t)b + k];
    d[3] += candidates_of(ra, b);
    c[0] += ra.blki[2 * (int64_t)b + 0];
    c[1] += ra.blki[2 * (int64_t)b + 1];
  }
  for (int k = 0; k < 4; ++k) d[k] = wave_sum(d[k]);
  c[0] = wave_sum_ll(c[0]);
  c[1] = wave_sum_ll(c[1]);
  if (lane == 0) {
    for (int k = 0; k < 4; ++k) sd[k][wave] = d[k];
    sc[0][wave] = c[0];
    sc[1][wave] = c[1];
  }
  __syncthreads();
  if (tid == 0) {
    RedPart r;
    for (int k = 0; k < 4; ++k) {
      double t = 0.0;
      for (int w = 0; w < R1WG / 64; ++w) t += sd[k][w];
      r.d[k] = t;
    }
    for (int k = 0; k < 2; ++k) {
      long long t = 0;
      for (int w = 0; w < R1WG / 64; ++w) t += sc[k][w];
      r.c[k] = t;
    }
    ra.part[blockIdx.x] = r;
  }
}

struct ReduceArgs {
  const RedPart* part;
  const int32_t* defer;
  int32_t nx, ny, nz;
  double eps4, eps24, nu;
  atm3_result* out;
};

// Stage 2: one workgroup sums the RBLK partials in fixed order.
__global__ __launch_bounds__(RBLK) void k_reduce2(ReduceArgs a) {
  __shared__ double sd[4][RBLK / 64];
  __shared__ long long sc[2][RBLK / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const RedPart p = a.part[tid];
  double d[4];
  long long c[2];
  for (int k = 0; k < 4; ++k) d[k] = wave_sum(p.d[k]);
  for (int k = 0; k < 2; ++k) c[k] = wave_sum_ll(p.c[k]);
  if (lane == 0) {
    for (int k = 0; k < 4; ++k) sd[k][wave] = d[k];
    for (int k = 0; k < 2; ++k) sc[k][wave] = c[k];
  }
  __syncthreads();
  if (tid == 0) {
    double e[4] = {0, 0, 0, 0};
    long long q[2] = {0, 0};
    for (int w = 0; w < RBLK / 64; ++w) {
      for (int k = 0; k < 4; ++k) e[k] += sd[k][w];
      for (int k = 0; k < 2; ++k) q[k] += sc[k][w];
    }
    atm3_result r;
    r.e_lj = a.eps4 * e[0];
    r.w_lj = a.eps24 * e[1];
    r.e_atm = a.nu * e[2];
    r.w_atm = 9.0 * a.nu * e[2];  // degree -9 homogeneity of eq. (atm): W_3 = 9 E_3
    r.n_pairs = q[0];
    r.n_triplets = q[1];
    r.n_candidates = (int64_t)e[3];
    r.ncell[0] = a.nx;
    r.ncell[1] = a.ny;
    r.ncell[2] = a.nz;
    r.status = a.defer[1];
    *a.out = r;
  }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t reduce_scratch_bytes() { return sizeof(RedPart) * RBLK; }

hipError_t launch_forces(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p,
                         float* forces, atm3_result* res_dev) {
  hipStream_t st = ctx->stream;
  ForceArgs a;
  a.sorted = (const double4*)ctx->buf[B_SORTED];
  a.start = (const int32_t*)ctx->buf[B_START];
  a.pos = pos;
  a.fpart = (u64*)ctx->buf[B_FPART];
  a.blkd = (double*)ctx->buf[B_BLKD];
  a.blki = (int32_t*)ctx->buf[B_BLKI];
  a.defer = (int32_t*)ctx->buf[B_DEFER];
  a.ntot = (int32_t)n;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.ncells = (int32_t)g.ncells;
  a.terms = p.terms;
  for (int d = 0; d < 3; ++d) {
    a.half[d] = 0.5 * g.side[d];
    a.box[d] = g.box[d];
  }
  const double rc2 = p.rc * p.rc;
  // guard band: FP32 block-frame r^2 is within ~1e-6 relative of the exact
  // value; a band of 4e-5 relative routes every uncertain pair to FP64
  a.lo2 = (float)(rc2 * (1.0 - 4e-5));
  a.hi2 = (float)(rc2 * (1.0 + 4e-5));
  a.rc2 = rc2;
  a.sig2 = p.sigma * p.sigma;
  a.eps24 = 24.0 * p.eps;
  a.k3nu = (float)(3.0 * p.nu);
  a.k15nu = (float)(1.875 * p.nu);
  a.k075nu = (float)(0.75 * p.nu);

  const int per = (a.ncells + 7) / 8;
  FmArgs fa;
  fa.sorted = a.sorted;
  fa.start = a.start;
  fa.pos = pos;
  fa.fmask = (uint32_t*)ctx->buf[B_FMASK];
  fa.fm_ok = (int32_t*)ctx->buf[B_FMOK];
  fa.nx = a.nx;
  fa.ny = a.ny;
  fa.nz = a.nz;
  for (int d = 0; d < 3; ++d) {
    fa.side[d] = g.side[d];
    fa.box[d] = g.box[d];
  }
  fa.lo2 = a.lo2;
  fa.hi2 = a.hi2;
  fa.rc2 = a.rc2;
  fa.defer = a.defer;
  fa.ncells = a.ncells;
  a.fmask = fa.fmask;
  a.fm_ok = fa.fm_ok;
  // the queued wide tier loops over the queue; its LDS (about 67 KB) admits
  // two workgroups per CU, so 512 of them fill the GPU
  const unsigned wide_grid = (unsigned)(a.ncells < 2 * 256 ? a.ncells : 2 * 256);
  hipError_t e = phase_begin(ctx, ATM3_PHASE_BLOCK);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fmask, dim3((unsigned)(((a.nx + FM_G - 1) / FM_G) * a.ny * a.nz)), dim3(256), 0, st, fa);
  // a grid whose mean 2x2x2 block holds more than 112 molecules would queue
  // a large share of its blocks: they all take the four-word tier directly
  const bool wide_all = 8 * n > 112 * (int64_t)a.ncells;
  if (wide_all)
    hipLaunchKernelGGL((k_block_wide<4096, WIDE_KCAP, false>), dim3(8 * per), dim3(WG), 0, st, a);
  else
    hipLaunchKernelGGL((k_block<1536, 640>), dim3(8 * per), dim3(WG), 0, st, a);
  if ((e = phase_end(ctx, ATM3_PHASE_BLOCK)) != hipSuccess) return e;
  if ((e = phase_begin(ctx, ATM3_PHASE_BIG)) != hipSuccess) return e;
  if (!wide_all) hipLaunchKernelGGL((k_block_wide<4096, WIDE_KCAP, true>), dim3(wide_grid), dim3(WG), 0, st, a);
  hipLaunchKernelGGL((k_block_big<8, 4096, 4096>), dim3(256), dim3(WG), 0, st, a);
  if ((e = phase_end(ctx, ATM3_PHASE_BIG)) != hipSuccess) return e;
  if ((e = phase_begin(ctx, ATM3_PHASE_REDUCE)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const u64*)a.fpart,
                     (const int32_t*)ctx->buf[B_PERM], (int32_t)n, forces);
  RedPart* part = (RedPart*)ctx->buf[B_RED];
  Red1Args r1;
  r1.blkd = a.blkd;
  r1.blki = a.blki;
  r1.start = a.start;
  r1.nx = a.nx;
  r1.ny = a.ny;
  r1.nz = a.nz;
  r1.ncells = a.ncells;
  r1.part = part;
  hipLaunchKernelGGL(k_reduce1, dim3(RBLK), dim3(R1WG), 0, st, r1);
  ReduceArgs r;
  r.part = part;
  r.defer = a.defer;
  r.nx = a.nx;
  r.ny = a.ny;
  r.nz = a.nz;
  r.eps4 = 4.0 * p.eps;
  r.eps24 = 24.0 * p.eps;
  r.nu = p.nu;
  r.out = res_dev;
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(RBLK), 0, st, r);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return phase_end(ctx, ATM3_PHASE_REDUCE);
}

}  // namespace atm3
