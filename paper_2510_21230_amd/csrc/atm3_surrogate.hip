// Learned three-body pair surrogate on gfx950: neighbour lists, invariant
// descriptors, the pair MLP on BF16 MFMA (inference and training), force
// assembly with an error estimate, and the exact one-sided ATM fallback.
//
// Slots are the cell-sorted molecule indices of the binning step.  The
// neighbour lists are deterministic: each slot lists its neighbours with a
// larger slot first (in the fixed order of the 27 neighbour cells and of the
// molecules inside a cell), then the rest by pair number; every pair is stored
// once, as (smaller slot, larger slot).
//
// MFMA use.  v_mfma_f32_32x32x16_bf16: for lane l (h = l / 32) the A operand
// holds row l % 32 and k = 8h .. 8h+7, the B operand column l % 32 and
// k = 8h .. 8h+7, and the 16 accumulators hold column l % 32 and rows
// 8(r/4) + 4h + (r%4), r = 0..15.  The fused pair kernel works in the
// transposed form Z^T = W^T H^T, pairs being the columns: one wave owns 32
// pairs end to end, and the accumulators of a layer are, after ReLU and BF16
// conversion, directly the B operand of the next layer once the input
// features are taken in the order those registers hold them.  The weights
// are stored permuted to that order (k_prep), so no data moves between lanes.
#include <math.h>

#include <new>
#include <string>

#include "atm3_internal.h"
#include "atm3_terms.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace atm3 {
namespace {

constexpr int NR = 16, NDESC = 64, NIN = 80, WID = 128;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * WID, OFF_W2 = OFF_B1 + WID, OFF_B2 = OFF_W2 + WID * WID,
              OFF_W3 = OFF_B2 + WID, OFF_B3 = OFF_W3 + WID * WID, OFF_W4 = OFF_B3 + WID, OFF_B4 = OFF_W4 + WID * 2,
              NPARAM = OFF_B4 + 2;
static_assert(NPARAM == ATM3_MLP_NPARAM, "parameter layout");
constexpr float R0 = 0.8f;
constexpr int NPERM1 = 4 * 5 * 64 * 8;    // layer 1 A fragments: 4 descriptor K-steps + 1 radial (bf16)
constexpr int NPERM = 4 * 4 * 2 * 64 * 8;  // layers 2, 3 A fragments (bf16)
constexpr int NPERM4 = 4 * 2 * 64 * 8;     // output layer A fragments (2 of 32 rows used)
constexpr int MAXSPLIT = 256;

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ __forceinline__ f32x16 mfma32(const bf16x8 a, const bf16x8 b, const f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// max(x, 0) as one integer max on the bit pattern (floats with the sign bit
// set, -0 included, are negative as integers); no NaN canonicalisation.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ float softplusf(float t) { return fmaxf(t, 0.f) + __logf(1.f + __expf(-fabsf(t))); }

// --------------------------------------------------------------------------
// neighbour lists
// --------------------------------------------------------------------------
struct NbArgs {
  const double4* sorted;
  const int32_t* start;
  const int32_t* cell_of;
  const double* pos;
  int32_t nx, ny, nz, n;
  double side[3], box[3];
  double rc2, lo2, hi2;
  int32_t* n_all;
  int32_t* n_up;
  int32_t* lo_fill;
  const int32_t* nb_start;
  const int32_t* up_start;
  int32_t* nb;
  int2* pij;
  float4* prec;
};

// Pairs listed first by each slot s: the molecules of its own cell with a
// larger slot and all molecules of the 13 forward neighbour cells (offsets
// after (0,0,0) in z, y, x order), so that every pair is found exactly once;
// every pair also counts for its second slot.  One wave per cell: the lanes
// run over the concatenated candidates of the cell's 14 half-shell cells (in
// that order, slots ascending within a cell), one molecule s of the cell at
// a time, and the ballot of the accepted lanes gives the count and, in the
// fill pass, the pair numbers in candidate order.  The distance comes from
// the cell-centred FP64 records; inside a 1e-9 relative band around rc^2 the
// decision is the exact minimum-image expression on the input positions.
constexpr int NB_WAVES = 4;
constexpr int NB_PASS = 4;  // candidates held in registers: up to 64 NB_PASS per cell

template <bool FILL>
__global__ __launch_bounds__(64 * NB_WAVES) void k_nb_cells(NbArgs a, int64_t ncells) {
  __shared__ int32_t cs[NB_WAVES][14], cpre[NB_WAVES][15];
  __shared__ double co[NB_WAVES][14][3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * NB_WAVES + w;
  if (c >= ncells) return;  // wave-uniform; no block barriers below
  const int cx = (int)(c % a.nx), cy = (int)((c / a.nx) % a.ny), cz = (int)(c / ((int64_t)a.nx * a.ny));
  if (lane < 14) {
    const int q = 13 + lane;
    const int dz = q / 9 - 1, dy = (q / 3) % 3 - 1, dx = q % 3 - 1;
    int uz = cz + dz, uy = cy + dy, ux = cx + dx;
    uz = uz < 0 ? uz + a.nz : (uz >= a.nz ? uz - a.nz : uz);
    uy = uy < 0 ? uy + a.ny : (uy >= a.ny ? uy - a.ny : uy);
    ux = ux < 0 ? ux + a.nx : (ux >= a.nx ? ux - a.nx : ux);
    const int cc = (uz * a.ny + uy) * a.nx + ux;
    cs[w][lane] = a.start[cc];
    cpre[w][lane + 1] = a.start[cc + 1] - a.start[cc];
    co[w][lane][0] = dx * a.side[0];
    co[w][lane][1] = dy * a.side[1];
    co[w][lane][2] = dz * a.side[2];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
    cpre[w][0] = 0;
    for (int q = 0; q < 14; ++q) cpre[w][q + 1] += cpre[w][q];
  }
  __builtin_amdgcn_wave_barrier();
  const int total = cpre[w][14];
  const int s0 = (int)a.start[c], s1 = (int)a.start[c + 1];
  // one candidate per lane and pass: accept it for slot s (cell-centred FP64
  // distance, exact re-check inside the band), then count or fill by ballot
  auto visit = [&](int s, const double4& me, int pass, int k, int t, bool own, double ox, double oy, double oz,
                   double cx, double cy, double cz, int origc, int p0, int e0) {
    bool in = false;
    double ex = 0.0, ey = 0.0, ez = 0.0, r2 = 0.0;
    if (t >= 0 && (!own || t > s)) {
      ex = (me.x - ox) - cx;
      ey = (me.y - oy) - cy;
      ez = (me.z - oz) - cz;
      r2 = ex * ex + ey * ey + ez * ez;
      if (r2 < a.lo2) in = true;
      else if (r2 >= a.hi2) in = false;
      else in = exact_r2(a.pos, (int)me.w, origc, a.box[0], a.box[1], a.box[2]) < a.rc2;
    }
    const unsigned long long bits = __ballot(in);
    if (in) {
      if (FILL) {
        const int pid = p0 + k + __popcll(bits & ((1ull << lane) - 1ull));
        a.pij[pid] = make_int2(s, t);
        a.prec[pid] = make_float4((float)ex, (float)ey, (float)ez, (float)sqrt(r2));
        a.nb[e0 + (pid - p0)] = 2 * pid;
        // the second-slot entry, appended in any order (k_nb_sort orders it)
        a.nb[a.nb_start[t] + a.n_up[t] + atomicAdd(&a.lo_fill[t], 1)] = 2 * pid + 1;
      } else {
        atomicAdd(&a.n_all[t], 1);  // n_all holds the second-slot counts here
      }
    }
    (void)pass;
    return k + __popcll(bits);
  };
  if (total <= 64 * NB_PASS) {
    // the cell's candidates are the same for each of its molecules: resolve
    // them once into registers
    int tt[NB_PASS], oc[NB_PASS];
    bool own[NB_PASS];
    double ox[NB_PASS], oy[NB_PASS], oz[NB_PASS], cx[NB_PASS], cy[NB_PASS], cz[NB_PASS];
#pragma unroll
    for (int pass = 0; pass < NB_PASS; ++pass) {
      const int idx = 64 * pass + lane;
      tt[pass] = -1;
      oc[pass] = 0;
      own[pass] = false;
      ox[pass] = oy[pass] = oz[pass] = cx[pass] = cy[pass] = cz[pass] = 0.0;
      if (idx < total) {
        int q = 0;
        while (idx >= cpre[w][q + 1]) ++q;
        const int t = cs[w][q] + (idx - cpre[w][q]);
        const double4 o = a.sorted[t];
        tt[pass] = t;
        oc[pass] = (int)o.w;
        own[pass] = q == 0;
        ox[pass] = o.x;
        oy[pass] = o.y;
        oz[pass] = o.z;
        cx[pass] = co[w][q][0];
        cy[pass] = co[w][q][1];
        cz[pass] = co[w][q][2];
      }
    }
    const int npass = (total + 63) / 64;
    for (int s = s0; s < s1; ++s) {
      const double4 me = a.sorted[s];
      int k = 0;
      const int p0 = FILL ? a.up_start[s] : 0, e0 = FILL ? a.nb_start[s] : 0;
#pragma unroll
      for (int pass = 0; pass < NB_PASS; ++pass)
        if (pass < npass)
          k = visit(s, me, pass, k, tt[pass], own[pass], ox[pass], oy[pass], oz[pass], cx[pass], cy[pass], cz[pass],
                    oc[pass], p0, e0);
      if (!FILL && lane == 0) a.n_up[s] = k;
    }
    return;
  }
  for (int s = s0; s < s1; ++s) {
    const double4 me = a.sorted[s];
    int k = 0;
    const int p0 = FILL ? a.up_start[s] : 0, e0 = FILL ? a.nb_start[s] : 0;
    for (int base = 0; base < total; base += 64) {
      const int idx = base + lane;
      int t = -1, q = 0;
      double4 o = make_double4(0.0, 0.0, 0.0, 0.0);
      if (idx < total) {
        while (idx >= cpre[w][q + 1]) ++q;
        t = cs[w][q] + (idx - cpre[w][q]);
        o = a.sorted[t];
      }
      k = visit(s, me, base / 64, k, t, q == 0, o.x, o.y, o.z, co[w][q][0], co[w][q][1], co[w][q][2], (int)o.w, p0,
                e0);
    }
    if (!FILL && lane == 0) a.n_up[s] = k;
  }
}

__global__ __launch_bounds__(256) void k_nb_total(const int32_t* __restrict__ n_up, int32_t n,
                                                  int32_t* __restrict__ n_all) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) n_all[s] += n_up[s];
}

// Sort each slot's second-member entries by pair number.  Up to SORT_REG of
// them are loaded into registers with independent loads and each goes to
// the position given by the number of smaller entries (the entries are
// distinct); longer lists are insertion-sorted in place.
constexpr int SORT_REG = 40;

__global__ __launch_bounds__(256) void k_nb_sort(const int32_t* __restrict__ nb_start,
                                                 const int32_t* __restrict__ n_up, int32_t n,
                                                 int32_t* __restrict__ nb) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int lo = nb_start[s] + n_up[s], hi = nb_start[s + 1];
  const int len = hi - lo;
  if (len <= 1) return;
  if (len <= SORT_REG) {
    int32_t v[SORT_REG];
#pragma unroll
    for (int x = 0; x < SORT_REG; ++x) v[x] = x < len ? nb[lo + x] : INT32_MAX;
#pragma unroll
    for (int x = 0; x < SORT_REG; ++x) {
      int r = 0;
#pragma unroll
      for (int y = 0; y < SORT_REG; ++y) r += v[y] < v[x];
      if (x < len) nb[lo + r] = v[x];
    }
    return;
  }
  for (int x = lo + 1; x < hi; ++x) {
    const int v = nb[x];
    int y = x - 1;
    while (y >= lo && nb[y] > v) {
      nb[y + 1] = nb[y];
      --y;
    }
    nb[y + 1] = v;
  }
}

__global__ void k_zero_i32(int32_t* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_zero_f32(float* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// --------------------------------------------------------------------------
// descriptors: four threads per slot, four radial channels each
// --------------------------------------------------------------------------
struct DescArgs {
  const int32_t* nb_start;
  const int32_t* nb;
  const float4* prec;
  int32_t n, raw;
  float rc, w, inv_w, pi_rc;
  const float* mean;
  const float* inv_sd;
  float* D;
  bf16* Db;
};

__global__ __launch_bounds__(256) void k_desc(DescArgs a) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = gid >> 2, cg = gid & 3;
  if (s >= a.n) return;
  float S[4], V[4][3], Q[4][6];
  for (int c = 0; c < 4; ++c) {
    S[c] = 0.f;
    for (int d = 0; d < 3; ++d) V[c][d] = 0.f;
    for (int d = 0; d < 6; ++d) Q[c][d] = 0.f;
  }
  // channel 4 cg + c has q_c = (r - mu_{4cg})/w - c, so
  // g_{c+1} = g_c exp(2 q_c - 1) and exp(2 q_{c+1} - 1) = exp(2 q_c - 1) e^-2
  const float mu0 = R0 + (float)(4 * cg) * a.w;
  const float em2 = 0.1353352832366127f;  // e^-2
  const float third = 1.f / 3.f;
  const int e1 = a.nb_start[s + 1];
  for (int e = a.nb_start[s]; e < e1; ++e) {
    const int v = a.nb[e];
    const float4 d = a.prec[v >> 1];
    // u = (r_other - r_s)/r: -(r_i - r_j)/r when s is the pair's first slot
    const float sir = ((v & 1) ? 1.f : -1.f) * __builtin_amdgcn_rcpf(d.w);
    const float ux = d.x * sir, uy = d.y * sir, uz = d.z * sir;
    const float fc = 0.5f * (1.f + __cosf(d.w * a.pi_rc));
    const float q0 = (d.w - mu0) * a.inv_w;
    float g = __expf(-q0 * q0) * fc;
    float E = __expf(fmaf(2.f, q0, -1.f));
    const float qxx = ux * ux - third, qyy = uy * uy - third, qzz = uz * uz - third;
    const float qxy = ux * uy, qxz = ux * uz, qyz = uy * uz;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      S[c] += g;
      V[c][0] = fmaf(g, ux, V[c][0]);
      V[c][1] = fmaf(g, uy, V[c][1]);
      V[c][2] = fmaf(g, uz, V[c][2]);
      Q[c][0] = fmaf(g, qxx, Q[c][0]);
      Q[c][1] = fmaf(g, qyy, Q[c][1]);
      Q[c][2] = fmaf(g, qzz, Q[c][2]);
      Q[c][3] = fmaf(g, qxy, Q[c][3]);
      Q[c][4] = fmaf(g, qxz, Q[c][4]);
      Q[c][5] = fmaf(g, qyz, Q[c][5]);
      g *= E;
      E *= em2;
    }
  }
  float f[4][4];  // [invariant k][channel c]
  for (int c = 0; c < 4; ++c) {
    const float vx = V[c][0], vy = V[c][1], vz = V[c][2];
    const float xx = Q[c][0], yy = Q[c][1], zz = Q[c][2], xy = Q[c][3], xz = Q[c][4], yz = Q[c][5];
    f[0][c] = S[c];
    f[1][c] = vx * vx + vy * vy + vz * vz;
    f[2][c] = xx * xx + yy * yy + zz * zz + 2.f * (xy * xy + xz * xz + yz * yz);
    f[3][c] = vx * (xx * vx + xy * vy + xz * vz) + vy * (xy * vx + yy * vy + yz * vz) + vz * (xz * vx + yz * vy + zz * vz);
  }
  // columns 16 k + 4 cg .. 16 k + 4 cg + 3: one 16-byte (8-byte) store each
  for (int k = 0; k < 4; ++k) {
    const int col = 16 * k + 4 * cg;
    float x[4];
    for (int c = 0; c < 4; ++c) x[c] = a.raw ? f[k][c] : (f[k][c] - a.mean[col + c]) * a.inv_sd[col + c];
    if (a.D) *reinterpret_cast<float4*>(a.D + (int64_t)s * NDESC + col) = make_float4(x[0], x[1], x[2], x[3]);
    if (a.Db) {
      const bf16 h0 = (bf16)x[0], h1 = (bf16)x[1], h2 = (bf16)x[2], h3 = (bf16)x[3];
      uint2 u;
      u.x = (uint32_t)__builtin_bit_cast(uint16_t, h0) | (uint32_t)__builtin_bit_cast(uint16_t, h1) << 16;
      u.y = (uint32_t)__builtin_bit_cast(uint16_t, h2) | (uint32_t)__builtin_bit_cast(uint16_t, h3) << 16;
      *reinterpret_cast<uint2*>(a.Db + (int64_t)s * NDESC + col) = u;
    }
  }
}

// Column mean and 1/max(sd, 1e-6) of a [rows][64] FP32 array, FP64 sums in
// fixed order: partial sums per block, then one block combines them.
__global__ __launch_bounds__(256) void k_colstats_part(const float* __restrict__ D, int32_t rows, int32_t chunk,
                                                       double* __restrict__ part) {
  const int col = threadIdx.x & 63, sub = threadIdx.x >> 6;
  __shared__ double s1[4][64], s2[4][64];
  const int r0 = blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  double a1 = 0.0, a2 = 0.0;
  for (int r = r0 + sub; r < r1; r += 4) {
    const double x = D[(int64_t)r * 64 + col];
    a1 += x;
    a2 += x * x;
  }
  s1[sub][col] = a1;
  s2[sub][col] = a2;
  __syncthreads();
  if (sub == 0) {
    part[(int64_t)blockIdx.x * 128 + col] = ((s1[0][col] + s1[1][col]) + s1[2][col]) + s1[3][col];
    part[(int64_t)blockIdx.x * 128 + 64 + col] = ((s2[0][col] + s2[1][col]) + s2[2][col]) + s2[3][col];
  }
}

__global__ void k_colstats_final(const double* __restrict__ part, int32_t nparts, int32_t rows,
                                 float* __restrict__ stats) {
  const int col = threadIdx.x;
  if (col >= 64) return;
  double a1 = 0.0, a2 = 0.0;
  for (int b = 0; b < nparts; ++b) {
    a1 += part[(int64_t)b * 128 + col];
    a2 += part[(int64_t)b * 128 + 64 + col];
  }
  const double m = a1 / rows;
  double var = a2 / rows - m * m;
  if (var < 0.0) var = 0.0;
  const double sd = sqrt(var);
  stats[col] = (float)m;
  stats[64 + col] = (float)(1.0 / (sd > 1e-6 ? sd : 1e-6));
}

// --------------------------------------------------------------------------
// generic BF16 MFMA product: C[m][n] = sum_k A(m,k) B(k,n) over the k range of
// blockIdx.z, with strided operands; one wave per 32 x 32 output block, four
// waves per workgroup along m (blockIdx.x: m, blockIdx.y: n).  Epilogue: bias, ReLU, ReLU'-mask, FP32 and/or
// BF16 stores.
// --------------------------------------------------------------------------
struct GemmArgs {
  const bf16* A;
  int64_t sam, sak;
  const bf16* B;
  int64_t sbk, sbn;
  int32_t M, N, K, kchunk;
  float* C;
  int64_t scm, scn, scz;
  bf16* Cb;
  int64_t sbm2, sbn2;
  const float* bias;
  const bf16* mask;
  int64_t smm, smn;
  int32_t relu;
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = (blockIdx.x * 4 + wave) * 32, n0 = blockIdx.y * 32;
  if (m0 >= a.M) return;  // wave-uniform; no barriers below
  const int kb = blockIdx.z * a.kchunk;
  const int ke = min(a.K, kb + a.kchunk);
  const int h = lane >> 5, row = m0 + (lane & 31), col = n0 + (lane & 31);
  f32x16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * h + e;
      av[e] = (row < a.M && k < ke) ? a.A[row * a.sam + k * a.sak] : (bf16)0.f;
      bv[e] = (col < a.N && k < ke) ? a.B[k * a.sbk + col * a.sbn] : (bf16)0.f;
    }
    acc = mfma32(av, bv, acc);
  }
  const int n = n0 + (lane & 31);
  if (n >= a.N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + 8 * (r >> 2) + 4 * h + (r & 3);
    if (m >= a.M) continue;
    float v = acc[r];
    if (a.bias) v += a.bias[n];
    if (a.relu) v = fmaxf(v, 0.f);
    if (a.mask && !((float)a.mask[m * a.smm + n * a.smn] > 0.f)) v = 0.f;
    if (a.C) a.C[blockIdx.z * a.scz + m * a.scm + n * a.scn] = v;
    if (a.Cb) a.Cb[m * a.sbm2 + n * a.sbn2] = (bf16)v;
  }
}

// out[i] = sum over z of part[z * stride + i], fixed order.
__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ part, int32_t nz, int64_t stride,
                                                   int64_t count, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += part[z * stride + i];
  out[i] = s;
}

// Column sums of a [rows][cols] FP32 array (cols <= 256): per-block partial
// rows, then a fixed-order sum.
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ X, int32_t rows, int32_t cols,
                                                     int32_t chunk, float* __restrict__ part) {
  const int c = threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += X[(int64_t)r * cols + c];
  part[(int64_t)blockIdx.x * cols + c] = s;
}

// --------------------------------------------------------------------------
// weights: BF16 copies and the permuted MFMA fragments of the fused kernel
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ P, bf16* __restrict__ w1b,
                                              bf16* __restrict__ w2b, bf16* __restrict__ w3b,
                                              bf16* __restrict__ wp1, bf16* __restrict__ wp2,
                                              bf16* __restrict__ wp3, bf16* __restrict__ wp4) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < NIN * WID) w1b[idx] = (bf16)P[OFF_W1 + idx];
  if (idx < WID * WID) {
    w2b[idx] = (bf16)P[OFF_W2 + idx];
    w3b[idx] = (bf16)P[OFF_W3 + idx];
  }
  if (idx < NPERM1) {
    // [ob][ks][lane][e]: W1[in = 16 ks + 8h + e][out = 32 ob + lane % 32];
    // K-steps 0..3 take the 64 descriptor inputs, step 4 the 16 radial ones
    const int e = idx & 7, lane = (idx >> 3) & 63, ks = (idx >> 9) % 5, ob = (idx >> 9) / 5;
    const int in = 16 * ks + 8 * (lane >> 5) + e, out = 32 * ob + (lane & 31);
    wp1[idx] = (bf16)P[OFF_W1 + in * WID + out];
  }
  if (idx < NPERM) {
    // [ob][b][ks][lane][e]: input feature 32b + 16ks + 8(e/4) + 4h + e%4
    const int e = idx & 7, lane = (idx >> 3) & 63, ks = (idx >> 9) & 1, b = (idx >> 10) & 3, ob = idx >> 12;
    const int f = 32 * b + 16 * ks + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    const int out = 32 * ob + (lane & 31);
    wp2[idx] = (bf16)P[OFF_W2 + f * WID + out];
    wp3[idx] = (bf16)P[OFF_W3 + f * WID + out];
  }
  if (idx < NPERM4) {
    // [b][ks][lane][e]: W4[f][out] with f as for layers 2 and 3, rows
    // out >= 2 zero
    const int e = idx & 7, lane = (idx >> 3) & 63, ks = (idx >> 9) & 1, b = idx >> 10;
    const int f = 32 * b + 16 * ks + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    const int out = lane & 31;
    wp4[idx] = (bf16)(out < 2 ? P[OFF_W4 + 2 * f + out] : 0.f);
  }
}

// --------------------------------------------------------------------------
// fused pair MLP (persistent; weights in LDS; one wave per 32 pairs)
// --------------------------------------------------------------------------
struct PairArgs {
  const int2* pij;
  const float4* prec;
  const bf16* Db;  // [slot][64] BF16 descriptors
  const bf16* wp1;
  const bf16* wp2;
  const bf16* wp3;
  const bf16* wp4;
  const float* P;
  int32_t np;
  float rc, w, inv_w, pi_rc;
  float2* st;
  bf16* h1;  // training dumps [pair][128] (or NULL)
  bf16* h2;
  bf16* h3;
  bf16* g16;  // [pair][16]
};

// BF16 of max(x, 0) for v[base .. base + 7]: round first, then one packed
// 16-bit integer max per two values (a BF16 with the sign bit set, -0
// included, is negative as an integer); the same bits as rounding the ReLU.
__device__ __forceinline__ bf16x8 relu_bf16x8(const f32x16& v, int base) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 w;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x2 f = {v[base + 2 * q], v[base + 2 * q + 1]};
    s16x2 t = __builtin_bit_cast(s16x2, __builtin_convertvector(f, bf16x2));
    t = __builtin_elementwise_max(t, (s16x2)0);
    w[q] = __builtin_bit_cast(uint32_t, t);
  }
  return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ void dump4(bf16* dst, const f32x16& v, int base_reg) {
  // four consecutive features from registers base_reg .. base_reg+3 (after ReLU)
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 t;
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = (bf16)relu(v[base_reg + q]);
  *(bf16x4*)dst = t;
}

// one workgroup per CU: 16 waves for inference, 8 when the activations are
// dumped for training (more registers live)
template <bool DUMP>
constexpr int pm_threads() { return DUMP ? 512 : 1024; }

template <bool DUMP>
__global__ __launch_bounds__(pm_threads<DUMP>()) void k_pair_mlp(PairArgs a) {
  constexpr int PM_THREADS = pm_threads<DUMP>(), PM_WAVES = PM_THREADS / 64;
  __shared__ bf16x8 w1s[4 * 5 * 64];
  __shared__ bf16x8 w2s[32 * 64];
  __shared__ bf16x8 w3s[32 * 64];
  __shared__ float bsh[3 * WID];
  __shared__ bf16x8 w4f[4 * 2 * 64];
  const int tid = threadIdx.x;
  for (int q = tid; q < 4 * 5 * 64; q += PM_THREADS) w1s[q] = ((const bf16x8*)a.wp1)[q];
  for (int q = tid; q < 32 * 64; q += PM_THREADS) {
    w2s[q] = ((const bf16x8*)a.wp2)[q];
    w3s[q] = ((const bf16x8*)a.wp3)[q];
  }
  for (int q = tid; q < WID; q += PM_THREADS) {
    bsh[q] = a.P[OFF_B1 + q];
    bsh[WID + q] = a.P[OFF_B2 + q];
    bsh[2 * WID + q] = a.P[OFF_B3 + q];
  }
  for (int q = tid; q < 4 * 2 * 64; q += PM_THREADS) w4f[q] = ((const bf16x8*)a.wp4)[q];
  const float b40 = a.P[OFF_B4], b41 = a.P[OFF_B4 + 1];
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6, h = lane >> 5, cn = lane & 31;
  // bias K-step: B operand with a single 1 at k = 0 (lanes h = 0), the A
  // operand then carries the bias of row m at k = 0
  bf16x8 ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = (bf16)((e == 0 && h == 0) ? 1.f : 0.f);
  const f32x16 zero16 = {};
  const int ntiles = (a.np + 31) / 32;
  for (int tile = blockIdx.x * PM_WAVES + wave; tile < ntiles; tile += gridDim.x * PM_WAVES) {
    // keeps the weight fragments in LDS: without it the loop-invariant LDS
    // reads are hoisted out of the tile loop into (spilled) registers
    asm volatile("" ::: "memory");
    const int p = tile * 32 + cn;
    const bool valid = p < a.np;
    int i = 0, j = 0;
    float4 d = make_float4(0.f, 0.f, 0.f, 1.f);
    if (valid) {
      const int2 ij = a.pij[p];
      i = ij.x;
      j = ij.y;
      d = a.prec[p];
    }
    // radial inputs, channels 8h .. 8h+7
    // (g_{e+1} = g_e exp(2 q_e - 1), the factor shrinking by e^-2 per channel)
    const float fc = valid ? 0.5f * (1.f + __cosf(d.w * a.pi_rc)) : 0.f;
    bf16x8 gb;
    {
      const float q0 = (d.w - (R0 + (float)(8 * h) * a.w)) * a.inv_w;
      float g = __expf(-q0 * q0) * fc, E = __expf(fmaf(2.f, q0, -1.f));
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        gb[e] = (bf16)g;
        g *= E;
        E *= 0.1353352832366127f;  // e^-2
      }
    }
    if (DUMP && valid) *(bf16x8*)(a.g16 + (int64_t)p * 16 + 8 * h) = gb;
    // descriptor inputs D_i + D_j, features 16 ks + 8h .. +7 (BF16 sum of
    // BF16 values, exact in FP32, rounded once)
    bf16x8 xb[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (valid) {
        const bf16x8 di = *(const bf16x8*)(a.Db + (int64_t)i * NDESC + 16 * ks + 8 * h);
        const bf16x8 dj = *(const bf16x8*)(a.Db + (int64_t)j * NDESC + 16 * ks + 8 * h);
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[ks][e] = (bf16)((float)di[e] + (float)dj[e]);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[ks][e] = (bf16)0.f;
      }
    }

    // layer 1: Z1^T = W1^T X^T + b1
    f32x16 acc[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      bf16x8 bb;
#pragma unroll
      for (int e = 0; e < 8; ++e) bb[e] = (bf16)((e == 0 && h == 0) ? bsh[32 * ob + cn] : 0.f);
      f32x16 c = mfma32(bb, ones, zero16);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) c = mfma32(w1s[(ob * 5 + ks) * 64 + lane], xb[ks], c);
      acc[ob] = mfma32(w1s[(ob * 5 + 4) * 64 + lane], gb, c);
    }

    // layers 2 and 3
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      bf16x8 hb[4][2];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) hb[b][ks] = relu_bf16x8(acc[b], 8 * ks);
      bf16* dump = layer == 0 ? a.h1 : a.h2;
      if (DUMP && valid) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) dump4(dump + (int64_t)p * WID + 32 * b + 8 * q + 4 * h, acc[b], 4 * q);
      }
      const bf16x8* ws = layer == 0 ? w2s : w3s;
      const float* bl = bsh + (layer + 1) * WID;
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) {
        bf16x8 bb;
#pragma unroll
        for (int e = 0; e < 8; ++e) bb[e] = (bf16)((e == 0 && h == 0) ? bl[32 * ob + cn] : 0.f);
        f32x16 c = mfma32(bb, ones, zero16);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) c = mfma32(ws[((ob * 4 + b) * 2 + ks) * 64 + lane], hb[b][ks], c);
        acc[ob] = c;
      }
    }

    // output layer on MFMA: rows 0 and 1 of W4^T relu(z3) are s and t (the
    // other 30 rows of the A operand are zero); b4 is added in FP32
    {
      bf16x8 hb[4][2];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) hb[b][ks] = relu_bf16x8(acc[b], 8 * ks);
      if (DUMP && valid) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) dump4(a.h3 + (int64_t)p * WID + 32 * b + 8 * q + 4 * h, acc[b], 4 * q);
      }
      f32x16 c = zero16;
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) c = mfma32(w4f[(b * 2 + ks) * 64 + lane], hb[b][ks], c);
      // C row m = 8 (r / 4) + 4 h + r % 4: rows 0 and 1 sit in registers 0
      // and 1 of the lanes with h = 0
      if (h == 0 && valid) a.st[p] = make_float2(c[0] + b40, c[1] + b41);
    }
  }
}

// --------------------------------------------------------------------------
// per-molecule force assembly
// --------------------------------------------------------------------------
struct MolArgs {
  const int32_t* nb_start;
  const int32_t* nb;
  const float4* prec;
  const float2* st;
  const double4* sorted;
  int32_t n, with_lj;
  double sig2, eps24;
  float thr;
  float* forces;   // input order (or NULL)
  float* err_out;  // input order (or NULL)
  float4* f3s;     // slot order surrogate force (or NULL)
  float* es;       // slot order error estimate (or NULL)
  int32_t* flag;   // per slot: 1 if the slot takes the exact fallback (or NULL)
  double* red;     // per block: sum (s12 - s6), sum (2 s12 - s6)
};

// Sums over groups of 8 lanes with DPP row shifts: afterwards lanes 7 and 15
// of each 16-lane row hold the sums of lanes 0-7 and 8-15 of that row.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <typename T>
__device__ __forceinline__ T sum8(T v) {
  if constexpr (sizeof(T) == 4) {
    v += dpp_f<0x111>(v);  // row_shr:1
    v += dpp_f<0x112>(v);  // row_shr:2
    v += dpp_f<0x114>(v);  // row_shr:4
  } else {
    v += dpp_d<0x111>(v);
    v += dpp_d<0x112>(v);
    v += dpp_d<0x114>(v);
  }
  return v;
}
// Whole-wave sum in every lane: each 16-lane row, then the four row totals;
// fixed order.
__device__ __forceinline__ double wave_total(double v) {
  v = sum8(v);
  v += dpp_d<0x118>(v);  // row_shr:8: lane 15 of each row holds its row total
  auto rl = [&](int l) {
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | lo);
  };
  return ((rl(15) + rl(31)) + rl(47)) + rl(63);
}

// Eight lanes per slot: each takes every eighth of the slot's neighbour
// entries, and DPP group sums combine them (no LDS traffic).
__global__ __launch_bounds__(256) void k_mol(MolArgs a) {
  __shared__ double r0[4], r1[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane & 7;
  const int s = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 3);
  float fx = 0.f, fy = 0.f, fz = 0.f, e = 0.f;
  double lx = 0.0, ly = 0.0, lz = 0.0, elj = 0.0, wlj = 0.0;
  if (s < a.n) {
    const int e1 = a.nb_start[s + 1];
    for (int q = a.nb_start[s] + g; q < e1; q += 8) {
      const int v = a.nb[q];
      const int pid = v >> 1;
      const float4 d = a.prec[pid];
      const float2 o = a.st[pid];
      const float sg = (v & 1) ? -1.f : 1.f;  // r_s - r_other = sg * (r_i - r_j)
      const float k = sg * o.x / d.w;
      fx = fmaf(k, d.x, fx);
      fy = fmaf(k, d.y, fy);
      fz = fmaf(k, d.z, fz);
      e += softplusf(o.y);
      if (a.with_lj) {
        const double dx = (double)d.x, dy = (double)d.y, dz = (double)d.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        double ir2 = __builtin_amdgcn_rcp(r2);  // refined by two Newton steps
        ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
        ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
        const double s2 = a.sig2 * ir2;
        const double s6 = s2 * s2 * s2, s12 = s6 * s6;
        const double f = a.eps24 * (2.0 * s12 - s6) * ir2 * (double)sg;
        lx += f * dx;
        ly += f * dy;
        lz += f * dz;
        if (!(v & 1)) {
          elj += s12 - s6;
          wlj += 2.0 * s12 - s6;
        }
      }
    }
  }
  fx = sum8(fx);
  fy = sum8(fy);
  fz = sum8(fz);
  e = sum8(e);
  if (a.with_lj) {
    lx = sum8(lx);
    ly = sum8(ly);
    lz = sum8(lz);
  }
  if (g == 7 && s < a.n) {
    const int orig = (int)a.sorted[s].w;
    const bool fall = a.flag && e > a.thr;
    if (a.forces) {
      a.forces[3 * (int64_t)orig + 0] = (float)(lx + (fall ? 0.0 : (double)fx));
      a.forces[3 * (int64_t)orig + 1] = (float)(ly + (fall ? 0.0 : (double)fy));
      a.forces[3 * (int64_t)orig + 2] = (float)(lz + (fall ? 0.0 : (double)fz));
    }
    if (a.err_out) a.err_out[orig] = e;
    if (a.f3s) a.f3s[s] = make_float4(fx, fy, fz, 0.f);
    if (a.es) a.es[s] = e;
    if (a.flag) a.flag[s] = fall ? 1 : 0;
  }
  if (a.red) {
    elj = wave_total(elj);
    wlj = wave_total(wlj);
    if (lane == 0) {
      r0[wave] = elj;
      r1[wave] = wlj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.red[2 * blockIdx.x + 0] = ((r0[0] + r0[1]) + r0[2]) + r0[3];
      a.red[2 * blockIdx.x + 1] = ((r1[0] + r1[1]) + r1[2]) + r1[3];
    }
  }
}

// --------------------------------------------------------------------------
// exact one-sided ATM force of the queued molecules (one wave each)
// --------------------------------------------------------------------------
struct FallArgs {
  const int32_t* queue;
  const int32_t* nb_start;
  const int32_t* nb;
  const int2* pij;
  const float4* prec;
  const double4* sorted;
  const double* pos;
  double box[3];
  double rc2;
  float lo2, hi2;
  float k3nu, k15nu, k075nu;
  float* forces;
  unsigned long long* ntrip;
};

__global__ __launch_bounds__(256) void k_fallback(FallArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nq = a.queue[0];
  unsigned long long cnt_total = 0;
  for (int qi = blockIdx.x * 4 + wave; qi < nq; qi += gridDim.x * 4) {
    const int s = a.queue[1 + qi];
    const int b0 = a.nb_start[s];
    const int m = a.nb_start[s + 1] - b0;
    const long long T = (long long)m * (m - 1) / 2;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    unsigned cnt = 0;
    const float4 ps = make_float4(0.f, 0.f, 0.f, 0.f);
    for (long long q = lane; q < T; q += 64) {
      // (x, y), x < y: row x holds m-1-x pairs
      int x = (int)((2.0 * m - 1.0 - sqrt((2.0 * m - 1.0) * (2.0 * m - 1.0) - 8.0 * (double)q)) * 0.5);
      if (x < 0) x = 0;
      while (x > 0 && (long long)x * (2 * m - x - 1) / 2 > q) --x;
      while ((long long)(x + 1) * (2 * m - x - 2) / 2 <= q) ++x;
      const int y = (int)(q - (long long)x * (2 * m - x - 1) / 2) + x + 1;
      const int va = a.nb[b0 + x], vb = a.nb[b0 + y];
      const float4 da = a.prec[va >> 1], db = a.prec[vb >> 1];
      const float sa = (va & 1) ? 1.f : -1.f, sb = (vb & 1) ? 1.f : -1.f;  // r_other - r_s
      const float4 pj = make_float4(sa * da.x, sa * da.y, sa * da.z, 0.f);
      const float4 pk = make_float4(sb * db.x, sb * db.y, sb * db.z, 0.f);
      const float ex = pj.x - pk.x, ey = pj.y - pk.y, ez = pj.z - pk.z;
      const float z = ex * ex + ey * ey + ez * ez;
      bool in = z < a.lo2;
      if (!in && z < a.hi2) {
        const int2 pa = a.pij[va >> 1], pb = a.pij[vb >> 1];
        const int ta = (va & 1) ? pa.x : pa.y, tb = (vb & 1) ? pb.x : pb.y;
        in = exact_r2(a.pos, (int)a.sorted[ta].w, (int)a.sorted[tb].w, a.box[0], a.box[1], a.box[2]) < a.rc2;
      }
      if (in) {
        const Trip r = atm_triplet(ps, pj, pk, a.k3nu, a.k15nu, a.k075nu);
        fx += (double)r.fix;
        fy += (double)r.fiy;
        fz += (double)r.fiz;
        ++cnt;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      fx += __shfl_xor(fx, off);
      fy += __shfl_xor(fy, off);
      fz += __shfl_xor(fz, off);
      cnt += __shfl_xor(cnt, off);
    }
    if (lane == 0) {
      const int64_t orig = (int64_t)a.sorted[s].w;
      a.forces[3 * orig + 0] += (float)fx;
      a.forces[3 * orig + 1] += (float)fy;
      a.forces[3 * orig + 2] += (float)fz;
      cnt_total += cnt;
    }
  }
  if (lane == 0 && cnt_total) atomicAdd(a.ntrip, cnt_total);
}

// --------------------------------------------------------------------------
// training
// --------------------------------------------------------------------------
struct LossArgs {
  const float4* f3s;
  const float* es;
  const float* target;  // input order [n][3]
  const double4* sorted;
  int32_t n;
  float lam, inv_n;
  float4* gF;
  float* ge;
  double* red;  // per block loss partial
};

__global__ __launch_bounds__(256) void k_loss(LossArgs a) {
  __shared__ double r0[4];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (s < a.n) {
    const int64_t orig = (int64_t)a.sorted[s].w;
    const float4 F = a.f3s[s];
    const float dx = F.x - a.target[3 * orig], dy = F.y - a.target[3 * orig + 1], dz = F.z - a.target[3 * orig + 2];
    const float q2 = dx * dx + dy * dy + dz * dz;
    const float nrm = sqrtf(q2);
    const float de = a.es[s] - nrm;
    a.gF[s] = make_float4(2.f * dx * a.inv_n, 2.f * dy * a.inv_n, 2.f * dz * a.inv_n, 0.f);
    a.ge[s] = 2.f * a.lam * de * a.inv_n;
    l = (double)q2 + (double)a.lam * (double)de * (double)de;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if (lane == 0) r0[wave] = l;
  __syncthreads();
  if (threadIdx.x == 0) a.red[blockIdx.x] = ((r0[0] + r0[1]) + r0[2]) + r0[3];
}

// dL/d(s, t) per pair and the output-layer delta dz3 = (W4 dout) * (h3 > 0);
// 32 threads per pair, four features each.
struct DoutArgs {
  const int2* pij;
  const float4* prec;
  const float2* st;
  const float4* gF;
  const float* ge;
  const bf16* h3;
  const float* P;
  int32_t np;
  float* dout;
  bf16* doutb;
  float* dz3;
  bf16* dz3b;
};

__global__ __launch_bounds__(256) void k_dout(DoutArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = gid >> 5;
  const int fg = gid & 31;
  if (p >= a.np) return;
  const int2 ij = a.pij[p];
  const float4 d = a.prec[p];
  const float ir = 1.f / d.w;
  const float4 gi = a.gF[ij.x], gj = a.gF[ij.y];
  const float ds = ((gi.x - gj.x) * d.x + (gi.y - gj.y) * d.y + (gi.z - gj.z) * d.z) * ir;
  const float t = a.st[p].y;
  const float sig = 1.f / (1.f + __expf(-t));
  const float dt = (a.ge[ij.x] + a.ge[ij.y]) * sig;
  if (fg == 0) {
    a.dout[2 * p] = ds;
    a.dout[2 * p + 1] = dt;
    a.doutb[2 * p] = (bf16)ds;
    a.doutb[2 * p + 1] = (bf16)dt;
  }
  for (int q = 0; q < 4; ++q) {
    const int f = 4 * fg + q;
    float v = a.P[OFF_W4 + 2 * f] * ds + a.P[OFF_W4 + 2 * f + 1] * dt;
    if (!((float)a.h3[p * WID + f] > 0.f)) v = 0.f;
    a.dz3[p * WID + f] = v;
    a.dz3b[p * WID + f] = (bf16)v;
  }
}

// dA_s = sum of dz1 over the slot's pairs (entry order), 32 threads per slot.
__global__ __launch_bounds__(256) void k_dA(const int32_t* __restrict__ nb_start, const int32_t* __restrict__ nb,
                                            const float* __restrict__ dz1, int32_t n, float* __restrict__ dA,
                                            bf16* __restrict__ dAb) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = gid >> 5;
  const int fg = gid & 31;
  if (s >= n) return;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const int e1 = nb_start[s + 1];
  for (int e = nb_start[s]; e < e1; ++e) {
    const float4 v = ((const float4*)dz1)[(int64_t)(nb[e] >> 1) * 32 + fg];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  ((float4*)dA)[s * 32 + fg] = acc;
  bf16* o = dAb + s * WID + 4 * fg;
  o[0] = (bf16)acc.x;
  o[1] = (bf16)acc.y;
  o[2] = (bf16)acc.z;
  o[3] = (bf16)acc.w;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int32_t count, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Fixed-order sum of per-block FP64 partials (rows of `cols` values,
// cols <= 4): workgroup g sums rows [g chunk, (g + 1) chunk) into row g of
// out, each thread a strided set of them, then a tree in LDS; the order
// depends only on the row count.
__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ part, int32_t rows, int32_t cols,
                                                  double* __restrict__ out, int32_t chunk) {
  __shared__ double t[4][256];
  const int tid = threadIdx.x;
  const int lo = blockIdx.x * chunk, hi = lo + chunk < rows ? lo + chunk : rows;
  for (int c = 0; c < cols; ++c) {
    double s = 0.0;
    for (int r = lo + tid; r < hi; r += 256) s += part[(int64_t)r * cols + c];
    t[c][tid] = s;
  }
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half)
      for (int c = 0; c < cols; ++c) t[c][tid] += t[c][tid + half];
    __syncthreads();
  }
  if (tid < cols) out[(int64_t)blockIdx.x * cols + tid] = t[tid][0];
}

// Fallback queue from the per-slot flags: queue[0] = count, then the flagged
// slots in slot order (positions from an exclusive scan of the flags).
__global__ __launch_bounds__(256) void k_queue(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                               int32_t n, int32_t* __restrict__ queue) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && flag[s]) queue[1 + pos[s]] = s;
  if (s == 0) queue[0] = pos[n];
}

}  // namespace
}  // namespace atm3

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace atm3;

struct atm3_mlp {
  int device = 0;
  float* params = nullptr;  // [NPARAM] FP32 masters
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* grad = nullptr;    // own gradient buffer
  float* stats = nullptr;   // mean[64], inv_sd[64]
  bf16* w1b = nullptr;
  bf16* w2b = nullptr;
  bf16* w3b = nullptr;
  bf16* wp1 = nullptr;
  bf16* wp2 = nullptr;
  bf16* wp3 = nullptr;
  bf16* wp4 = nullptr;
  double* dsum = nullptr;   // small device reduction outputs
  int64_t step = 0;
};

namespace {

// splitmix64 (Steele, Lea, Flood) and Box-Muller for the seeded initial weights
uint64_t splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double unit_open(uint64_t* s) { return ((double)(splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

double normal(uint64_t* s) {
  const double u1 = unit_open(s), u2 = unit_open(s);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
}

hipError_t prep_weights(atm3_ctx* ctx, atm3_mlp* m) {
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(NPERM > NIN * WID ? NPERM : NIN * WID, 256)), dim3(256), 0,
                     ctx->stream, m->params, m->w1b, m->w2b, m->w3b, m->wp1, m->wp2, m->wp3, m->wp4);
  return hipGetLastError();
}

int begin(atm3_ctx* ctx, atm3_mlp* m) {
  if (!ctx || !m) return ATM3_EINVAL;
  ctx->err.clear();
  if (m->device != ctx->device) return fail(ctx, ATM3_EINVAL, "model and context are on different devices");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return ATM3_OK;
}

// Geometry of one surrogate evaluation, after sur_prepare.
struct SurGeom {
  Grid g;
  int64_t n = 0;
  int64_t np = 0;
  double rc = 0.0;
};

template <class T>
T* buf(atm3_ctx* ctx, Buf b) {
  return (T*)ctx->buf[b];
}

// Binning, neighbour lists and descriptors (FP32 and BF16).
int sur_prepare(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double* box, double rc, bool raw,
                bool fp32_desc, SurGeom* G) {
  if (!pos) return fail(ctx, ATM3_EINVAL, "pos is NULL");
  if (n < 1 || n > (int64_t)1 << 26) return fail(ctx, ATM3_EINVAL, "n must be in [1, 2^26]");
  if (!box) return fail(ctx, ATM3_EINVAL, "box is NULL");
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0) || !isfinite(box[d])) return fail(ctx, ATM3_EINVAL, "box lengths must be finite and > 0");
  if (!(rc > R0 + 0.1) || !isfinite(rc)) return fail(ctx, ATM3_EINVAL, "rc must be finite and > 0.9");
  if (!make_grid(box, rc, &G->g)) return fail(ctx, ATM3_EINVAL, "cell grid out of range");
  for (int d = 0; d < 3; ++d)
    if (G->g.n[d] < 3)
      return fail(ctx, ATM3_EINVAL, "box too small: floor(L/rc) = " + std::to_string(G->g.n[d]) + " < 3 cells");
  G->n = n;
  G->rc = rc;
  const size_t N = (size_t)n, C = (size_t)G->g.ncells;
  int r;
  if ((r = ensure(ctx, B_CELL_OF, 4 * N))) return r;
  if ((r = ensure(ctx, B_RANK, 4 * N))) return r;
  if ((r = ensure(ctx, B_COUNT, 4 * C))) return r;
  if ((r = ensure(ctx, B_START, 4 * (C + 1)))) return r;
  if ((r = ensure(ctx, B_PERM, 4 * N))) return r;
  if ((r = ensure(ctx, B_SORTED, 32 * N))) return r;
  if ((r = ensure(ctx, B_TILE, 4 * (C / 1024 + 2)))) return r;
  if ((r = ensure(ctx, B_SN_ALL, 4 * N))) return r;
  if ((r = ensure(ctx, B_SN_UP, 4 * N))) return r;
  if ((r = ensure(ctx, B_SN_START, 4 * (N + 1)))) return r;
  if ((r = ensure(ctx, B_SN_UPSTART, 4 * (N + 1)))) return r;
  if ((r = ensure(ctx, B_SN_LOFILL, 4 * N))) return r;
  if ((r = ensure(ctx, B_SN_TILE, 4 * (N / 1024 + 2)))) return r;
  if ((r = ensure(ctx, B_SD, 4 * 64 * N))) return r;
  if ((r = ensure(ctx, B_SDB, 2 * 64 * N))) return r;
  hipStream_t st = ctx->stream;
  hipError_t e = launch_binning(ctx, pos, n, G->g);
  if (e != hipSuccess) return hip_fail(ctx, e, "binning launch");

  NbArgs a;
  a.sorted = buf<double4>(ctx, B_SORTED);
  a.start = buf<int32_t>(ctx, B_START);
  a.cell_of = buf<int32_t>(ctx, B_CELL_OF);
  a.pos = pos;
  a.nx = G->g.n[0];
  a.ny = G->g.n[1];
  a.nz = G->g.n[2];
  a.n = (int32_t)n;
  for (int d = 0; d < 3; ++d) {
    a.side[d] = G->g.side[d];
    a.box[d] = box[d];
  }
  a.rc2 = rc * rc;
  a.lo2 = a.rc2 * (1.0 - 1e-9);
  a.hi2 = a.rc2 * (1.0 + 1e-9);
  a.n_all = buf<int32_t>(ctx, B_SN_ALL);
  a.n_up = buf<int32_t>(ctx, B_SN_UP);
  a.nb_start = buf<int32_t>(ctx, B_SN_START);
  a.up_start = buf<int32_t>(ctx, B_SN_UPSTART);
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n, 256) < 4096 ? blocks_for(n, 256) : 4096), dim3(256), 0, st,
                     a.n_all, n);
  const unsigned cell_blocks = blocks_for(G->g.ncells, NB_WAVES);
  hipLaunchKernelGGL(k_nb_cells<false>, dim3(cell_blocks), dim3(64 * NB_WAVES), 0, st, a, G->g.ncells);
  hipLaunchKernelGGL(k_nb_total, dim3(blocks_for(n, 256)), dim3(256), 0, st, a.n_up, (int32_t)n, a.n_all);
  if ((e = launch_scan(st, a.n_all, buf<int32_t>(ctx, B_SN_START), n, buf<int32_t>(ctx, B_SN_TILE))) != hipSuccess)
    return hip_fail(ctx, e, "scan");
  if ((e = launch_scan(st, a.n_up, buf<int32_t>(ctx, B_SN_UPSTART), n, buf<int32_t>(ctx, B_SN_TILE))) != hipSuccess)
    return hip_fail(ctx, e, "scan");
  int32_t tot[2];
  e = hipMemcpyAsync(&tot[0], buf<int32_t>(ctx, B_SN_UPSTART) + n, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&tot[1], buf<int32_t>(ctx, B_SN_START) + n, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "pair count");
  const int64_t P = tot[0];
  if (P < 0 || P >= ((int64_t)1 << 30) || tot[1] != 2 * tot[0])
    return fail(ctx, ATM3_EINVAL, "too many neighbour pairs for 32-bit lists");
  G->np = P;
  if ((r = ensure(ctx, B_SN_NB, 4 * (size_t)(2 * P)))) return r;
  if ((r = ensure(ctx, B_SP_IJ, 8 * (size_t)P))) return r;
  if ((r = ensure(ctx, B_SP_REC, 16 * (size_t)P))) return r;
  if ((r = ensure(ctx, B_SP_ST, 8 * (size_t)P))) return r;
  a.nb = buf<int32_t>(ctx, B_SN_NB);
  a.pij = buf<int2>(ctx, B_SP_IJ);
  a.prec = buf<float4>(ctx, B_SP_REC);
  a.lo_fill = buf<int32_t>(ctx, B_SN_LOFILL);
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n, 256) < 4096 ? blocks_for(n, 256) : 4096), dim3(256), 0, st,
                     a.lo_fill, n);
  hipLaunchKernelGGL(k_nb_cells<true>, dim3(cell_blocks), dim3(64 * NB_WAVES), 0, st, a, G->g.ncells);
  hipLaunchKernelGGL(k_nb_sort, dim3(blocks_for(n, 256)), dim3(256), 0, st, a.nb_start, a.n_up, (int32_t)n, a.nb);

  DescArgs da;
  da.nb_start = a.nb_start;
  da.nb = a.nb;
  da.prec = a.prec;
  da.n = (int32_t)n;
  da.raw = raw ? 1 : 0;
  da.rc = (float)rc;
  da.w = (float)((rc - R0) / (NR - 1));
  da.inv_w = (float)((NR - 1) / (rc - R0));
  da.pi_rc = (float)(3.14159265358979323846 / rc);
  da.mean = m->stats;
  da.inv_sd = m->stats + 64;
  da.D = fp32_desc ? buf<float>(ctx, B_SD) : nullptr;
  da.Db = buf<bf16>(ctx, B_SDB);
  hipLaunchKernelGGL(k_desc, dim3(blocks_for(4 * n, 256)), dim3(256), 0, st, da);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "surrogate preparation launch");
  return ATM3_OK;
}

int sur_pairs_forward(atm3_ctx* ctx, atm3_mlp* m, const SurGeom& G, bool dump) {
  if (G.np == 0) return ATM3_OK;
  PairArgs pa;
  pa.pij = buf<int2>(ctx, B_SP_IJ);
  pa.prec = buf<float4>(ctx, B_SP_REC);
  pa.Db = buf<bf16>(ctx, B_SDB);
  pa.wp1 = m->wp1;
  pa.wp2 = m->wp2;
  pa.wp3 = m->wp3;
  pa.wp4 = m->wp4;
  pa.P = m->params;
  pa.np = (int32_t)G.np;
  pa.rc = (float)G.rc;
  pa.w = (float)((G.rc - R0) / (NR - 1));
  pa.inv_w = (float)((NR - 1) / (G.rc - R0));
  pa.pi_rc = (float)(3.14159265358979323846 / G.rc);
  pa.st = buf<float2>(ctx, B_SP_ST);
  pa.h1 = dump ? buf<bf16>(ctx, B_TH1) : nullptr;
  pa.h2 = dump ? buf<bf16>(ctx, B_TH2) : nullptr;
  pa.h3 = dump ? buf<bf16>(ctx, B_TH3) : nullptr;
  pa.g16 = dump ? buf<bf16>(ctx, B_TG16) : nullptr;
  int dev_cu = 256;
  (void)hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
  const int64_t tiles = (G.np + 31) / 32;
  int64_t grid = dev_cu;  // one 8-wave workgroup per CU: one LDS copy of the weights
  if (grid * 8 > tiles) grid = (tiles + 7) / 8;
  if (dump)
    hipLaunchKernelGGL(k_pair_mlp<true>, dim3((unsigned)grid), dim3(pm_threads<true>()), 0, ctx->stream, pa);
  else
    hipLaunchKernelGGL(k_pair_mlp<false>, dim3((unsigned)grid), dim3(pm_threads<false>()), 0, ctx->stream, pa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "pair MLP launch");
  return ATM3_OK;
}

// Fixed-order sum of `rows` rows of `cols` doubles into out: one workgroup
// for short inputs, else 256 contiguous chunks, then their sums.  B_SRED2
// must hold 256 x 4 doubles.
void sum_rows(atm3_ctx* ctx, hipStream_t st, const double* part, int32_t rows, int32_t cols, double* out) {
  if (rows <= 8192) {
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, st, part, rows, cols, out, rows);
    return;
  }
  const int32_t chunk = (rows + 255) / 256, g1 = (rows + chunk - 1) / chunk;
  double* tmp = buf<double>(ctx, B_SRED2);
  hipLaunchKernelGGL(k_sum_rows, dim3(g1), dim3(256), 0, st, part, rows, cols, tmp, chunk);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, st, (const double*)tmp, g1, cols, out, g1);
}

int sur_mol(atm3_ctx* ctx, const SurGeom& G, const atm3_params* p, float thr, bool with_lj, bool queue, float* forces,
            float* err_out, bool keep_slot) {
  int r;
  const size_t N = (size_t)G.n;
  const unsigned nb = blocks_for(G.n, 32);  // k_mol: eight lanes per slot
  if ((r = ensure(ctx, B_SRED, 16 * (size_t)nb + 64))) return r;
  if ((r = ensure(ctx, B_SRED2, 8 * 256 * 4))) return r;
  if ((r = ensure(ctx, B_SQ, 4 * (N + 1)))) return r;
  if ((r = ensure(ctx, B_SF3, 16 * N))) return r;
  if ((r = ensure(ctx, B_SE, 4 * N))) return r;
  MolArgs ma;
  ma.nb_start = buf<int32_t>(ctx, B_SN_START);
  ma.nb = buf<int32_t>(ctx, B_SN_NB);
  ma.prec = buf<float4>(ctx, B_SP_REC);
  ma.st = buf<float2>(ctx, B_SP_ST);
  ma.sorted = buf<double4>(ctx, B_SORTED);
  ma.n = (int32_t)G.n;
  ma.with_lj = with_lj ? 1 : 0;
  ma.sig2 = p ? p->sigma * p->sigma : 1.0;
  ma.eps24 = p ? 24.0 * p->eps : 0.0;
  ma.thr = thr;
  ma.forces = forces;
  ma.err_out = err_out;
  ma.f3s = keep_slot ? buf<float4>(ctx, B_SF3) : nullptr;
  ma.es = keep_slot ? buf<float>(ctx, B_SE) : nullptr;
  ma.flag = queue ? buf<int32_t>(ctx, B_SN_LOFILL) : nullptr;  // free after the list build
  ma.red = buf<double>(ctx, B_SRED);
  hipLaunchKernelGGL(k_mol, dim3(nb), dim3(256), 0, ctx->stream, ma);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && queue) {
    int32_t* qpos = buf<int32_t>(ctx, B_SN_UPSTART) + 0;  // reused: N+1 entries
    // the pair offsets of B_SN_UPSTART are no longer needed once the lists exist
    e = launch_scan(ctx->stream, ma.flag, qpos, G.n, buf<int32_t>(ctx, B_SN_TILE));
    if (e == hipSuccess)
      hipLaunchKernelGGL(k_queue, dim3(blocks_for(G.n, 256)), dim3(256), 0, ctx->stream, ma.flag, qpos,
                         (int32_t)G.n, buf<int32_t>(ctx, B_SQ));
    if (e == hipSuccess) e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "force assembly launch");
  return ATM3_OK;
}

// C[M][N] (+)= op products through k_gemm, split over K with a fixed-order sum.
int gemm_splitk(atm3_ctx* ctx, GemmArgs ga, float* out) {
  int r;
  const int64_t MN = (int64_t)ga.M * ga.N;
  int splits = (int)((ga.K + 4095) / 4096);
  if (splits < 1) splits = 1;
  if (splits > MAXSPLIT) splits = MAXSPLIT;
  int64_t chunk = (ga.K + splits - 1) / splits;
  chunk = (chunk + 15) / 16 * 16;
  splits = (int)((ga.K + chunk - 1) / chunk);
  if (splits < 1) splits = 1;
  if ((r = ensure(ctx, B_TPART, 4 * (size_t)MN * splits))) return r;
  ga.kchunk = (int32_t)chunk;
  ga.C = buf<float>(ctx, B_TPART);
  ga.scm = ga.N;
  ga.scn = 1;
  ga.scz = MN;
  hipLaunchKernelGGL(k_gemm, dim3(blocks_for(ga.M, 128), blocks_for(ga.N, 32), splits), dim3(256), 0, ctx->stream,
                     ga);
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(MN, 256)), dim3(256), 0, ctx->stream, buf<float>(ctx, B_TPART),
                     splits, MN, MN, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "gemm launch");
  return ATM3_OK;
}

int colsum(atm3_ctx* ctx, const float* X, int64_t rows, int cols, float* out) {
  int r;
  const int chunk = 4096;
  const int parts = (int)((rows + chunk - 1) / chunk);
  const int np = parts > 0 ? parts : 1;
  if ((r = ensure(ctx, B_TPART, 4 * (size_t)cols * np))) return r;
  if (rows > 0)
    hipLaunchKernelGGL(k_colsum_part, dim3(parts), dim3(256), 0, ctx->stream, X, (int32_t)rows, cols, chunk,
                       buf<float>(ctx, B_TPART));
  else
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, ctx->stream, buf<float>(ctx, B_TPART), (int64_t)cols);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, ctx->stream, buf<float>(ctx, B_TPART), np, (int64_t)cols,
                     (int64_t)cols, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "column sum launch");
  return ATM3_OK;
}

int do_grad(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double* box, double rc,
            const float* target, float lam, float* grad, double* loss_out) {
  if (!target) return fail(ctx, ATM3_EINVAL, "f3_target is NULL");
  SurGeom G;
  int r = sur_prepare(ctx, m, pos, n, box, rc, false, false, &G);
  if (r) return r;
  const size_t P = (size_t)G.np, N = (size_t)n;
  if ((r = ensure(ctx, B_TH1, 2 * 128 * P))) return r;
  if ((r = ensure(ctx, B_TH2, 2 * 128 * P))) return r;
  if ((r = ensure(ctx, B_TH3, 2 * 128 * P))) return r;
  if ((r = ensure(ctx, B_TG16, 2 * 16 * P))) return r;
  if ((r = sur_pairs_forward(ctx, m, G, true))) return r;
  if ((r = sur_mol(ctx, G, nullptr, 0.f, false, false, nullptr, nullptr, true))) return r;
  hipStream_t st = ctx->stream;
  const unsigned nbk = blocks_for(n, 256);
  if ((r = ensure(ctx, B_SG, 16 * N))) return r;
  if ((r = ensure(ctx, B_SGE, 4 * N))) return r;
  if ((r = ensure(ctx, B_SRED, 8 * (size_t)nbk + 64))) return r;
  LossArgs la;
  la.f3s = buf<float4>(ctx, B_SF3);
  la.es = buf<float>(ctx, B_SE);
  la.target = target;
  la.sorted = buf<double4>(ctx, B_SORTED);
  la.n = (int32_t)n;
  la.lam = lam;
  la.inv_n = (float)(1.0 / (double)n);
  la.gF = buf<float4>(ctx, B_SG);
  la.ge = buf<float>(ctx, B_SGE);
  la.red = buf<double>(ctx, B_SRED);
  hipLaunchKernelGGL(k_loss, dim3(nbk), dim3(256), 0, st, la);
  sum_rows(ctx, st, la.red, (int32_t)nbk, 1, m->dsum);
  if (grad) {
    if ((r = ensure(ctx, B_TDOUT, 8 * P + 8))) return r;
    if ((r = ensure(ctx, B_TDOUTB, 4 * P + 4))) return r;
    if ((r = ensure(ctx, B_TDZ3, 4 * 128 * P))) return r;
    if ((r = ensure(ctx, B_TDZ2, 4 * 128 * P))) return r;
    if ((r = ensure(ctx, B_TDZ1, 4 * 128 * P))) return r;
    if ((r = ensure(ctx, B_TDZ3B, 2 * 128 * P))) return r;
    if ((r = ensure(ctx, B_TDZ2B, 2 * 128 * P))) return r;
    if ((r = ensure(ctx, B_TDZ1B, 2 * 128 * P))) return r;
    if ((r = ensure(ctx, B_TDA, 4 * 128 * N))) return r;
    if ((r = ensure(ctx, B_TDAB, 2 * 128 * N))) return r;
    const int64_t np = (int64_t)P;
    if (np > 0) {
      DoutArgs oa;
      oa.pij = buf<int2>(ctx, B_SP_IJ);
      oa.prec = buf<float4>(ctx, B_SP_REC);
      oa.st = buf<float2>(ctx, B_SP_ST);
      oa.gF = la.gF;
      oa.ge = la.ge;
      oa.h3 = buf<bf16>(ctx, B_TH3);
      oa.P = m->params;
      oa.np = (int32_t)np;
      oa.dout = buf<float>(ctx, B_TDOUT);
      oa.doutb = buf<bf16>(ctx, B_TDOUTB);
      oa.dz3 = buf<float>(ctx, B_TDZ3);
      oa.dz3b = buf<bf16>(ctx, B_TDZ3B);
      hipLaunchKernelGGL(k_dout, dim3(blocks_for(32 * np, 256)), dim3(256), 0, st, oa);
      // dz2 = (dz3 W3^T) * (h2 > 0); dz1 = (dz2 W2^T) * (h1 > 0)
      for (int layer = 0; layer < 2; ++layer) {
        GemmArgs ga = {};
        ga.A = layer == 0 ? buf<bf16>(ctx, B_TDZ3B) : buf<bf16>(ctx, B_TDZ2B);
        ga.sam = 128;
        ga.sak = 1;
        ga.B = layer == 0 ? m->w3b : m->w2b;  // B(k, n) = W[n][k]
        ga.sbk = 1;
        ga.sbn = 128;
        ga.M = (int32_t)np;
        ga.N = 128;
        ga.K = 128;
        ga.kchunk = 128;
        ga.C = layer == 0 ? buf<float>(ctx, B_TDZ2) : buf<float>(ctx, B_TDZ1);
        ga.scm = 128;
        ga.scn = 1;
        ga.Cb = layer == 0 ? buf<bf16>(ctx, B_TDZ2B) : buf<bf16>(ctx, B_TDZ1B);
        ga.sbm2 = 128;
        ga.sbn2 = 1;
        ga.mask = layer == 0 ? buf<bf16>(ctx, B_TH2) : buf<bf16>(ctx, B_TH1);
        ga.smm = 128;
        ga.smn = 1;
        hipLaunchKernelGGL(k_gemm, dim3(blocks_for(np, 128), 4, 1), dim3(256), 0, st, ga);
      }
    }
    // weight gradients (split-K over pairs), bias gradients (column sums)
    struct WG {
      Buf x;
      int xcols;
      Buf y;
      int ycols;
      int off;
    };
    const WG wg[4] = {{B_TH3, 128, B_TDOUTB, 2, OFF_W4},
                      {B_TH2, 128, B_TDZ3B, 128, OFF_W3},
                      {B_TH1, 128, B_TDZ2B, 128, OFF_W2},
                      {B_TG16, 16, B_TDZ1B, 128, OFF_W1 + NDESC * WID}};
    for (const WG& w : wg) {
      GemmArgs ga = {};
      ga.A = buf<bf16>(ctx, w.x);  // A(m, k) = X[k][m]
      ga.sam = 1;
      ga.sak = w.xcols;
      ga.B = buf<bf16>(ctx, w.y);  // B(k, n) = Y[k][n]
      ga.sbk = w.ycols;
      ga.sbn = 1;
      ga.M = w.xcols;
      ga.N = w.ycols;
      ga.K = (int32_t)np;
      if ((r = gemm_splitk(ctx, ga, grad + w.off))) return r;
    }
    if ((r = colsum(ctx, buf<float>(ctx, B_TDOUT), np, 2, grad + OFF_B4))) return r;
    if ((r = colsum(ctx, buf<float>(ctx, B_TDZ3), np, 128, grad + OFF_B3))) return r;
    if ((r = colsum(ctx, buf<float>(ctx, B_TDZ2), np, 128, grad + OFF_B2))) return r;
    if ((r = colsum(ctx, buf<float>(ctx, B_TDZ1), np, 128, grad + OFF_B1))) return r;
    // dA per slot, then dW1a = D^T dA (split-K over molecules)
    hipLaunchKernelGGL(k_dA, dim3(blocks_for(32 * (int64_t)n, 256)), dim3(256), 0, st, buf<int32_t>(ctx, B_SN_START),
                       buf<int32_t>(ctx, B_SN_NB), buf<float>(ctx, B_TDZ1), (int32_t)n, buf<float>(ctx, B_TDA),
                       buf<bf16>(ctx, B_TDAB));
    GemmArgs ga = {};
    ga.A = buf<bf16>(ctx, B_SDB);
    ga.sam = 1;
    ga.sak = 64;
    ga.B = buf<bf16>(ctx, B_TDAB);
    ga.sbk = 128;
    ga.sbn = 1;
    ga.M = 64;
    ga.N = 128;
    ga.K = (int32_t)n;
    if ((r = gemm_splitk(ctx, ga, grad + OFF_W1))) return r;
  }
  double loss = 0.0;
  hipError_t e = hipMemcpyAsync(&loss, m->dsum, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "loss copy");
  if (loss_out) *loss_out = loss / (double)n;
  return ATM3_OK;
}

int do_adam(atm3_ctx* ctx, atm3_mlp* m, const float* grad, float lr, float b1, float b2, float eps) {
  if (!grad) return fail(ctx, ATM3_EINVAL, "grad is NULL");
  if (!(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(ctx, ATM3_EINVAL, "invalid Adam hyper-parameters");
  m->step += 1;
  const float c1 = (float)(1.0 - pow((double)b1, (double)m->step));
  const float c2 = (float)(1.0 - pow((double)b2, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(NPARAM, 256)), dim3(256), 0, ctx->stream, m->params, m->m, m->v, grad,
                     NPARAM, lr, b1, b2, eps, c1, c2);
  hipError_t e = prep_weights(ctx, m);
  if (e != hipSuccess) return hip_fail(ctx, e, "Adam launch");
  return ATM3_OK;
}

}  // namespace

extern "C" {

int atm3_mlp_create(atm3_ctx* ctx, uint64_t seed, atm3_mlp** out) {
  if (!ctx || !out) return ATM3_EINVAL;
  ctx->err.clear();
  *out = nullptr;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  atm3_mlp* m = new (std::nothrow) atm3_mlp();
  if (!m) return fail(ctx, ATM3_ENOMEM, "host allocation");
  m->device = ctx->device;
  bool ok = hipMalloc(&m->params, 4 * NPARAM) == hipSuccess && hipMalloc(&m->m, 4 * NPARAM) == hipSuccess &&
            hipMalloc(&m->v, 4 * NPARAM) == hipSuccess && hipMalloc(&m->grad, 4 * NPARAM) == hipSuccess &&
            hipMalloc(&m->stats, 4 * 128) == hipSuccess && hipMalloc(&m->w1b, 2 * NIN * WID) == hipSuccess &&
            hipMalloc(&m->w2b, 2 * WID * WID) == hipSuccess && hipMalloc(&m->w3b, 2 * WID * WID) == hipSuccess &&
            hipMalloc(&m->wp1, 2 * NPERM1) == hipSuccess && hipMalloc(&m->wp2, 2 * NPERM) == hipSuccess &&
            hipMalloc(&m->wp3, 2 * NPERM) == hipSuccess && hipMalloc(&m->wp4, 2 * NPERM4) == hipSuccess &&
            hipMalloc(&m->dsum, 64) == hipSuccess;
  if (!ok) {
    atm3_mlp_destroy(m);
    return fail(ctx, ATM3_ENOMEM, "device allocation for the model");
  }
  std::vector<float> h(NPARAM, 0.f);
  uint64_t s = seed;
  for (int i = 0; i < NIN * WID; ++i) h[OFF_W1 + i] = (float)(normal(&s) * sqrt(2.0 / NIN));
  for (int i = 0; i < WID * WID; ++i) h[OFF_W2 + i] = (float)(normal(&s) * sqrt(2.0 / WID));
  for (int i = 0; i < WID * WID; ++i) h[OFF_W3 + i] = (float)(normal(&s) * sqrt(2.0 / WID));
  for (int i = 0; i < 2 * WID; ++i) h[OFF_W4 + i] = (float)(0.1 * normal(&s) * sqrt(1.0 / WID));
  h[OFF_B4 + 1] = -3.f;
  std::vector<float> st(128, 0.f);
  for (int i = 64; i < 128; ++i) st[i] = 1.f;
  e = hipMemcpy(m->params, h.data(), 4 * NPARAM, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stats, st.data(), 4 * 128, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->m, 0, 4 * NPARAM);
  if (e == hipSuccess) e = hipMemset(m->v, 0, 4 * NPARAM);
  if (e == hipSuccess) e = prep_weights(ctx, m);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    atm3_mlp_destroy(m);
    return hip_fail(ctx, e, "model initialisation");
  }
  *out = m;
  return ATM3_OK;
}

void atm3_mlp_destroy(atm3_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  void* ps[] = {m->params, m->m,   m->v,   m->grad, m->stats, m->w1b, m->w2b,
                m->w3b,    m->wp1, m->wp2, m->wp3,  m->wp4,   m->dsum};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  delete m;
}

int atm3_mlp_set_params(atm3_ctx* ctx, atm3_mlp* m, const float* host, int64_t n) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!host || n != NPARAM) return fail(ctx, ATM3_EINVAL, "parameter count must be ATM3_MLP_NPARAM");
  hipError_t e = hipMemcpy(m->params, host, 4 * NPARAM, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->m, 0, 4 * NPARAM);
  if (e == hipSuccess) e = hipMemset(m->v, 0, 4 * NPARAM);
  if (e == hipSuccess) e = prep_weights(ctx, m);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "set params");
  m->step = 0;
  return ATM3_OK;
}

int atm3_mlp_get_params(atm3_ctx* ctx, atm3_mlp* m, float* host, int64_t n) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!host || n != NPARAM) return fail(ctx, ATM3_EINVAL, "parameter count must be ATM3_MLP_NPARAM");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(host, m->params, 4 * NPARAM, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "get params");
  return ATM3_OK;
}

int atm3_mlp_set_stats(atm3_ctx* ctx, atm3_mlp* m, const float* mean, const float* inv_sd) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!mean || !inv_sd) return fail(ctx, ATM3_EINVAL, "NULL statistics");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(m->stats, mean, 4 * 64, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stats + 64, inv_sd, 4 * 64, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "set stats");
  return ATM3_OK;
}

int atm3_mlp_get_stats(atm3_ctx* ctx, atm3_mlp* m, float* mean, float* inv_sd) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!mean || !inv_sd) return fail(ctx, ATM3_EINVAL, "NULL statistics");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(mean, m->stats, 4 * 64, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(inv_sd, m->stats + 64, 4 * 64, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "get stats");
  return ATM3_OK;
}

int atm3_mlp_fit_stats(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double box[3], double rc) {
  int r = begin(ctx, m);
  if (r) return r;
  SurGeom G;
  if ((r = sur_prepare(ctx, m, pos, n, box, rc, true, true, &G))) return r;
  const int chunk = 2048;
  const int parts = (int)((n + chunk - 1) / chunk);
  if ((r = ensure(ctx, B_SRED, 8 * 128 * (size_t)parts))) return r;
  hipLaunchKernelGGL(k_colstats_part, dim3(parts), dim3(256), 0, ctx->stream, buf<float>(ctx, B_SD), (int32_t)n,
                     chunk, buf<double>(ctx, B_SRED));
  hipLaunchKernelGGL(k_colstats_final, dim3(1), dim3(64), 0, ctx->stream, buf<double>(ctx, B_SRED), parts,
                     (int32_t)n, m->stats);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "fit stats");
  return ATM3_OK;
}

int atm3_surrogate_forces(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double box[3],
                          const atm3_params* p, float thr, float* forces, float* err_est, atm3_result* out,
                          int64_t* n_fallback) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!p || !forces || !out) return fail(ctx, ATM3_EINVAL, "params, forces or result is NULL");
  if (!(p->sigma > 0.0) || !isfinite(p->eps) || !isfinite(p->nu))
    return fail(ctx, ATM3_EINVAL, "sigma must be > 0, eps and nu finite");
  if (p->truncation != ATM3_TRUNC_PAIR) return fail(ctx, ATM3_EINVAL, "the surrogate uses the pairwise cutoff");
  SurGeom G;
  if ((r = sur_prepare(ctx, m, pos, n, box, p->rc, false, false, &G))) return r;
  if ((r = sur_pairs_forward(ctx, m, G, false))) return r;
  if ((r = sur_mol(ctx, G, p, thr, true, true, forces, err_est, false))) return r;
  hipStream_t st = ctx->stream;
  const unsigned nbk = blocks_for(n, 32);  // k_mol's partials: one row per block of 32 slots
  unsigned long long* ntrip = (unsigned long long*)(m->dsum + 4);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, (int32_t*)ntrip, (int64_t)2);
  FallArgs fa;
  fa.queue = buf<int32_t>(ctx, B_SQ);
  fa.nb_start = buf<int32_t>(ctx, B_SN_START);
  fa.nb = buf<int32_t>(ctx, B_SN_NB);
  fa.pij = buf<int2>(ctx, B_SP_IJ);
  fa.prec = buf<float4>(ctx, B_SP_REC);
  fa.sorted = buf<double4>(ctx, B_SORTED);
  fa.pos = pos;
  for (int d = 0; d < 3; ++d) fa.box[d] = box[d];
  fa.rc2 = p->rc * p->rc;
  fa.lo2 = (float)(fa.rc2 * (1.0 - 4e-5));
  fa.hi2 = (float)(fa.rc2 * (1.0 + 4e-5));
  fa.k3nu = (float)(3.0 * p->nu);
  fa.k15nu = (float)(1.875 * p->nu);
  fa.k075nu = (float)(0.75 * p->nu);
  fa.forces = forces;
  fa.ntrip = ntrip;
  int dev_cu = 256;
  (void)hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
  hipLaunchKernelGGL(k_fallback, dim3(8 * dev_cu), dim3(256), 0, st, fa);
  sum_rows(ctx, st, buf<double>(ctx, B_SRED), (int32_t)nbk, 2, m->dsum);
  hipError_t e = hipGetLastError();
  double sums[2];
  unsigned long long nt = 0;
  int32_t nq = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(sums, m->dsum, 16, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nt, ntrip, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nq, buf<int32_t>(ctx, B_SQ), 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "surrogate evaluation");
  atm3_result res = {};
  res.e_lj = 4.0 * p->eps * sums[0];
  res.w_lj = 24.0 * p->eps * sums[1];
  res.e_atm = NAN;
  res.w_atm = NAN;
  res.n_pairs = G.np;
  res.n_triplets = (int64_t)nt;
  res.n_candidates = 0;
  for (int d = 0; d < 3; ++d) res.ncell[d] = G.g.n[d];
  res.status = ATM3_OK;
  *out = res;
  if (n_fallback) *n_fallback = nq;
  return ATM3_OK;
}

int atm3_mlp_grad(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double box[3], double rc,
                  const float* f3_target, float lam, float* grad_dev, double* loss_out) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!(lam >= 0.f)) return fail(ctx, ATM3_EINVAL, "lam must be >= 0");
  return do_grad(ctx, m, pos, n, box, rc, f3_target, lam, grad_dev, loss_out);
}

int atm3_mlp_adam(atm3_ctx* ctx, atm3_mlp* m, const float* grad_dev, float lr, float beta1, float beta2, float eps) {
  int r = begin(ctx, m);
  if (r) return r;
  return do_adam(ctx, m, grad_dev, lr, beta1, beta2, eps);
}

int atm3_mlp_train_step(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double box[3], double rc,
                        const float* f3_target, float lam, float lr, double* loss_out) {
  int r = begin(ctx, m);
  if (r) return r;
  if (!(lam >= 0.f)) return fail(ctx, ATM3_EINVAL, "lam must be >= 0");
  if ((r = do_grad(ctx, m, pos, n, box, rc, f3_target, lam, m->grad, loss_out))) return r;
  return do_adam(ctx, m, m->grad, lr, 0.9f, 0.999f, 1e-8f);
}

int atm3_surrogate_pairs(atm3_ctx* ctx, atm3_mlp* m, const double* pos, int64_t n, const double box[3], double rc,
                         int64_t cap, int32_t* pair_ij, float* st_out, float* desc, float* f3, float* err,
                         int64_t* n_pairs) {
  int r = begin(ctx, m);
  if (r) return r;
  if (cap < 0) return fail(ctx, ATM3_EINVAL, "cap must be >= 0");
  SurGeom G;
  if ((r = sur_prepare(ctx, m, pos, n, box, rc, false, desc != nullptr, &G))) return r;
  if ((r = sur_pairs_forward(ctx, m, G, false))) return r;
  if ((r = sur_mol(ctx, G, nullptr, 0.f, false, false, nullptr, err, true))) return r;
  hipStream_t st = ctx->stream;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "surrogate evaluation");
  // gather to input order on the host side of the boundary: small copies
  const int64_t np = G.np < cap ? G.np : cap;
  std::vector<int32_t> perm(n);
  e = hipMemcpy(perm.data(), buf<int32_t>(ctx, B_PERM), 4 * (size_t)n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "copy");
  if (pair_ij && np > 0) {
    std::vector<int2> ij(np);
    e = hipMemcpy(ij.data(), buf<int2>(ctx, B_SP_IJ), 8 * (size_t)np, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy");
    std::vector<int32_t> o(2 * np);
    for (int64_t q = 0; q < np; ++q) {
      o[2 * q] = perm[ij[q].x];
      o[2 * q + 1] = perm[ij[q].y];
    }
    e = hipMemcpy(pair_ij, o.data(), 8 * (size_t)np, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy");
  }
  if (st_out && np > 0) {
    e = hipMemcpy(st_out, buf<float2>(ctx, B_SP_ST), 8 * (size_t)np, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy");
  }
  if (desc || f3) {
    std::vector<float> d(64 * (size_t)n), o(64 * (size_t)n);
    std::vector<float4> f(n);
    if (desc) {
      e = hipMemcpy(d.data(), buf<float>(ctx, B_SD), 4 * 64 * (size_t)n, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(ctx, e, "copy");
      for (int64_t s = 0; s < n; ++s)
        for (int c = 0; c < 64; ++c) o[64 * (size_t)perm[s] + c] = d[64 * (size_t)s + c];
      e = hipMemcpy(desc, o.data(), 4 * 64 * (size_t)n, hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(ctx, e, "copy");
    }
    if (f3) {
      e = hipMemcpy(f.data(), buf<float4>(ctx, B_SF3), 16 * (size_t)n, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(ctx, e, "copy");
      std::vector<float> g3(3 * (size_t)n);
      for (int64_t s = 0; s < n; ++s) {
        g3[3 * (size_t)perm[s] + 0] = f[s].x;
        g3[3 * (size_t)perm[s] + 1] = f[s].y;
        g3[3 * (size_t)perm[s] + 2] = f[s].z;
      }
      e = hipMemcpy(f3, g3.data(), 12 * (size_t)n, hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(ctx, e, "copy");
    }
  }
  if (n_pairs) *n_pairs = G.np;
  return ATM3_OK;
}

}  // extern "C"
