// The product truncation rule and the 3c18 / 3c01 cell sets (Sec. 2, Sec. 4).
//
// Pairwise cutoff: the three cell sets visit the same triplets (all three
// pairs are within rc, so their cells are neighbours and fit the 3c08 block,
// the 3c18 forward set and every 27-neighbourhood), so the block kernel's
// forces, energies and triplets serve all of them; only the number of
// candidate molecule triplets differs.  k_cand_* count those from the cell
// populations (eqs. celltriplet, twoonetriplets, carttriplets summed over
// the visited cell sets), and for 3c01, where every molecule of a triplet
// takes its own share, the triplet count becomes receiving incidences.
//
// Product cutoff: a triplet may have sides beyond rc, so there is no pair
// filter.  For 3c08 and 3c18, k_prod_block stages each base cell's cell set
// and evaluates each of its triplets once (forces on all three, exact fixed
// point).  For 3c01, where each molecule takes its own share, k_onesided
// evaluates for every molecule m every pair (j, k) of candidates from the
// 27 cells around m: the visited-set test on the cell offsets, the
// truncation test on the exact FP64 minimum-image squared sides (sorted,
// multiplied left to right, strict), and the ATM force on m (FP32 per
// triplet, FP64 sums); it also gives the LJ forces of the other two.
// Energies and virials are credited once per triplet (a third per receiving
// molecule for 3c01); counts once per triplet (3c01: once per receiving
// molecule).
#include <math.h>

#include <algorithm>

#include "atm3_internal.h"
#include "atm3_terms.h"

namespace atm3 {
namespace {

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

__device__ __forceinline__ int wrap_off(int off, int n) {
  off %= n;
  if (off < 0) off += n;
  if (off > n / 2) off -= n;
  return off;
}

// ---------------------------------------------------------------------------
// candidate counts of the 3c18 and 3c01 cell sets (pairwise cutoff path)
// ---------------------------------------------------------------------------
struct CandArgs {
  const int32_t* start;
  int32_t nx, ny, nz;
  int64_t ncells;
  int32_t variant;
  unsigned long long* part;  // per block
};

__global__ __launch_bounds__(256) void k_cand(CandArgs a) {
  __shared__ unsigned long long ws[4];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = 0;
  if (c < a.ncells) {
    const int cx = (int)(c % a.nx), cy = (int)((c / a.nx) % a.ny), cz = (int)(c / ((int64_t)a.nx * a.ny));
    const long long nb = a.start[c + 1] - a.start[c];
    if (a.variant == ATM3_VARIANT_3C08) {
      // base cell c: molecule triplets of its 2x2x2 block whose cells have
      // c as componentwise minimum (corner codes AND to 0): eq.
      // (celltriplet) for the cell itself, eq. (twoonetriplets) for the 13
      // cell pairs, eq. (carttriplets) for the 44 cell triples
      long long N[8];
      for (int o = 0; o < 8; ++o) {
        const int ux = wrapc(cx + (o & 1), a.nx), uy = wrapc(cy + ((o >> 1) & 1), a.ny), uz = wrapc(cz + (o >> 2), a.nz);
        const int64_t cc = ((int64_t)uz * a.ny + uy) * a.nx + ux;
        N[o] = a.start[cc + 1] - a.start[cc];
      }
      long long t = N[0] * (N[0] - 1) * (N[0] - 2) / 6;
      for (int p = 0; p < 8; ++p)
        for (int q = p + 1; q < 8; ++q) {
          if ((p & q) == 0) t += N[q] * (N[p] * (N[p] - 1) / 2) + N[p] * (N[q] * (N[q] - 1) / 2);
          for (int r = q + 1; r < 8; ++r)
            if ((p & q & r) == 0) t += N[p] * N[q] * N[r];
        }
      v = (unsigned long long)t;
    } else if (a.variant == ATM3_VARIANT_3C01) {
      // every molecule of cell c: pairs of the other molecules of its 27 cells
      long long s = 0;
      for (int q = 0; q < 27; ++q) {
        const int ux = wrapc(cx + q % 3 - 1, a.nx), uy = wrapc(cy + (q / 3) % 3 - 1, a.ny),
                  uz = wrapc(cz + q / 9 - 1, a.nz);
        const int64_t cc = ((int64_t)uz * a.ny + uy) * a.nx + ux;
        s += a.start[cc + 1] - a.start[cc];
      }
      v = (unsigned long long)(nb * ((s - 1) * (s - 2) / 2));
    } else {
      // base cell c with two cells of {c} + its 13 forward neighbours
      long long sf = 0, sf2 = 0, two = 0;
      for (int q = 14; q < 27; ++q) {
        const int ux = wrapc(cx + q % 3 - 1, a.nx), uy = wrapc(cy + (q / 3) % 3 - 1, a.ny),
                  uz = wrapc(cz + q / 9 - 1, a.nz);
        const int64_t cc = ((int64_t)uz * a.ny + uy) * a.nx + ux;
        const long long nf = a.start[cc + 1] - a.start[cc];
        sf += nf;
        sf2 += nf * nf;
        two += nf * (nf - 1) / 2;
      }
      const long long t = nb * (nb - 1) * (nb - 2) / 6 + (nb * (nb - 1) / 2) * sf + nb * two +
                          nb * ((sf * sf - sf2) / 2);
      v = (unsigned long long)t;
    }
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) a.part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// n_candidates of the result; with `triple`, a 3c01 triplet count made by
// the block kernel (each triplet once) becomes the 3c01 count (once per
// receiving molecule).
__global__ void k_cand_final(const unsigned long long* __restrict__ part, int32_t np, int32_t variant,
                             int32_t triple, atm3_result* __restrict__ res) {
  if (threadIdx.x != 0) return;
  unsigned long long s = 0;
  for (int b = 0; b < np; ++b) s += part[b];
  res->n_candidates = (int64_t)s;
  if (triple && variant == ATM3_VARIANT_3C01) res->n_triplets *= 3;
}

// ---------------------------------------------------------------------------
// one-sided evaluation under the product cutoff
// ---------------------------------------------------------------------------
constexpr int CAND_CAP = 2048;  // candidates per cell neighbourhood (LDS)
constexpr int OS_WAVES = 8;     // waves per block
constexpr int OS_SPLIT = 2;     // waves per molecule (rows xa split by parity)
constexpr int OS_MOLS = OS_WAVES / OS_SPLIT;  // molecules per group
constexpr int OS_QCAP = 128;    // per-wave queue of pairs that passed the FP32 test
constexpr int OS_NB = 27;       // neighbour cells, the cell included

struct OneArgs {
  const double4* sorted;
  const int32_t* start;
  const double* pos;
  int32_t nx, ny, nz, variant, terms, groups;
  double side[3], box[3];
  double rc2, rc6, sig2, eps4, eps24;
  float boxf[3], invf[3];
  float rc2hi, lo6f, hi6f, small2;  // FP32 thresholds of the exact decisions
  float k3nu, k15nu, k075nu;
  float* forces;
  double* fout;               // if set, FP64 forces go here instead of `forces`
  double* tpart;              // if set, per block LJ W_xx, W_yy, W_zz (half per molecule)
  double* dpart;              // per block: e_lj, w_lj, e_atm, unused
  unsigned long long* ipart;  // per block: n_pairs, n_triplets, unused, overflow
};

// Truncation test of the oracle: squared sides sorted ascending, multiplied
// left to right, strict comparison with (rc^2 rc^2) rc^2.
__device__ __noinline__ bool product_ok(double x, double y, double z, double rc6) {
#pragma clang fp contract(off)
  double s0 = x, s1 = y, s2 = z, t;
  if (s1 < s0) { t = s0; s0 = s1; s1 = t; }
  if (s2 < s1) { t = s1; s1 = s2; s2 = t; }
  if (s1 < s0) { t = s0; s0 = s1; s1 = t; }
  return ((s0 * s1) * s2) < rc6;
}

struct Off {
  int x, y, z;
};

__device__ __forceinline__ Off unpack_off(uint32_t u) {
  return Off{(int)(u & 255u) - 8, (int)((u >> 8) & 255u) - 8, (int)((u >> 16) & 255u) - 8};
}

__device__ __forceinline__ bool lex_less(const Off& p, const Off& q) {
  if (p.z != q.z) return p.z < q.z;
  if (p.y != q.y) return p.y < q.y;
  return p.x < q.x;
}

__device__ __forceinline__ Off rel(const Off& a, const Off& b, int nx, int ny, int nz) {
  return Off{wrap_off(a.x - b.x, nx), wrap_off(a.y - b.y, ny), wrap_off(a.z - b.z, nz)};
}

__device__ __forceinline__ bool near1(const Off& a, const Off& b) {
  const int dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
}

__device__ __forceinline__ bool adjacent(const Off& a, const Off& b, int nx, int ny, int nz) {
  return near1(rel(b, a, nx, ny, nz), Off{0, 0, 0});
}

// Visited test of the triplet labelled t0 < t1 < t2 (by input index) with
// cell offsets o0, o1, o2 (relative to any common cell); for 3c01 returns the
// receiving mask (bit q: molecule t_q takes its share), else 7 or 0.
__device__ __forceinline__ int visited_mask(int variant, const Off& o0, const Off& o1, const Off& o2, int nx, int ny,
                                            int nz) {
  if (variant == ATM3_VARIANT_3C01) {
    const bool a01 = adjacent(o0, o1, nx, ny, nz), a02 = adjacent(o0, o2, nx, ny, nz),
               a12 = adjacent(o1, o2, nx, ny, nz);
    return (a01 && a02 ? 1 : 0) | (a01 && a12 ? 2 : 0) | (a02 && a12 ? 4 : 0);
  }
  const Off z0{0, 0, 0};
  const Off r1 = rel(o1, o0, nx, ny, nz), r2 = rel(o2, o0, nx, ny, nz);
  if (variant == ATM3_VARIANT_3C08) {
    const int lx = min(0, min(r1.x, r2.x)), hx = max(0, max(r1.x, r2.x));
    const int ly = min(0, min(r1.y, r2.y)), hy = max(0, max(r1.y, r2.y));
    const int lz = min(0, min(r1.z, r2.z)), hz = max(0, max(r1.z, r2.z));
    return (hx - lx <= 1 && hy - ly <= 1 && hz - lz <= 1) ? 7 : 0;
  }
  // 3c18: lexicographically smallest cell as base; the others within one
  // step of it in every dimension
  Off b = z0;
  if (lex_less(r1, b)) b = r1;
  if (lex_less(r2, b)) b = r2;
  return (near1(z0, b) && near1(r1, b) && near1(r2, b)) ? 7 : 0;
}

// Minimum image of an FP32 displacement (for the FP32 pre-test and the force
// arithmetic; every decision is taken again in FP64 near its boundary).
__device__ __forceinline__ float3 wrapf(float3 d, const float* L, const float* inv) {
  d.x = fmaf(-L[0], rintf(d.x * inv[0]), d.x);
  d.y = fmaf(-L[1], rintf(d.y * inv[1]), d.y);
  d.z = fmaf(-L[2], rintf(d.z * inv[2]), d.z);
  return d;
}

__device__ __forceinline__ float sq3(float3 d) { return fmaf(d.z, d.z, fmaf(d.y, d.y, d.x * d.x)); }

// Energy term of eq. (atm) and the force on molecule i of the triplet (i, j,
// k) from r_ij = -va, r_ik = -vb and the squared sides x = |r_ij|^2,
// y = |r_ik|^2, z = |r_jk|^2 (eq. forcepairs: F_i = c_x r_ij + c_y r_ik).
__device__ __forceinline__ float atm_on_i(float3 va, float3 vb, float x, float y, float z, float k3nu, float k15nu,
                                          float k075nu, float3* f) {
  const float s = x + y + z;
  const float A = fmaf(-2.f, x, s), B = fmaf(-2.f, y, s), C = fmaf(-2.f, z, s);
  const float AB = A * B, AC = A * C, BC = B * C;
  const float P = AB * C;
  const float S = AB + AC + BC;
  const float Q = (x * y) * z;
  const float t1 = __builtin_amdgcn_rsqf(Q);
  const float t2 = t1 * t1, t3 = t2 * t1, t5 = t3 * t2;
  const float G = fmaf(k15nu * P, t5, k3nu * t3);
  const float H = k075nu * t5;
  const float cx = fmaf(G, (y * z) * t2, -H * fmaf(-2.f, BC, S));
  const float cy = fmaf(G, (x * z) * t2, -H * fmaf(-2.f, AC, S));
  f->x = -fmaf(cx, va.x, cy * vb.x);
  f->y = -fmaf(cx, va.y, cy * vb.y);
  f->z = -fmaf(cx, va.z, cy * vb.z);
  return fmaf(0.375f * P, t5, t3);
}

struct OneLds {
  float4 p[CAND_CAP];         // candidate position relative to the centre cell's centre; .w = input index
  uint32_t off[CAND_CAP];     // packed cell offset (dx+8) | (dy+8) << 8 | (dz+8) << 16
  uint32_t q[OS_WAVES][OS_QCAP];  // queued pairs xa | xb << 16
  int32_t cnt[OS_NB + 1], base[OS_NB + 1];
  int32_t cell[OS_NB + 1];
  double facc[OS_WAVES][3];
  double red[OS_WAVES][3];
  unsigned long long redi[OS_WAVES][2];
  double tred[OS_WAVES][3];
  int32_t nc;
};

// One block per (cell, group slice): the candidates of the cell's
// neighbourhood are staged once in LDS and shared by every molecule of the
// cell; each molecule is handled by OS_SPLIT waves (candidate rows split by
// parity), each lane taking the partners xb > xa of row xa.  Pairs that pass
// the FP32 product test with a relative guard band are queued and evaluated
// 64 at a time; pairs inside the band take the oracle's FP64 decision.  WV:
// molecule-candidate vectors need a minimum-image wrap (fewer than 4 cells
// per dimension); WJ: candidate-candidate vectors do (fewer than 8).
template <bool WV, bool WJ, bool TENSOR = false>
__global__ __launch_bounds__(64 * OS_WAVES) void k_onesided(OneArgs a) {
  __shared__ OneLds L;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c = blockIdx.x / a.groups;
  const int g = blockIdx.x % a.groups;
  const int cx = (int)(c % a.nx), cy = (int)((c / a.nx) % a.ny), cz = (int)(c / ((int64_t)a.nx * a.ny));
  constexpr int R = 1, span = 3, nnb = OS_NB, q0 = 13;
  double e_lj = 0.0, w_lj = 0.0, e3 = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
  unsigned long long npair = 0, ntrip = 0, over = 0;
  // neighbour cells (dx fastest) and their populations
  if (threadIdx.x < nnb) {
    const int q = threadIdx.x;
    const int dx = q % span - R, dy = (q / span) % span - R, dz = q / (span * span) - R;
    const int ux = wrapc(cx + dx, a.nx), uy = wrapc(cy + dy, a.ny), uz = wrapc(cz + dz, a.nz);
    const int cc = (uz * a.ny + uy) * a.nx + ux;
    L.cell[q] = cc;
    L.cnt[q] = a.start[cc + 1] - a.start[cc];
  }
  __syncthreads();
  if (w == 0) {
    int run = 0;
    for (int b0 = 0; b0 < nnb; b0 += 64) {
      const int q = b0 + lane;
      const int v = q < nnb ? L.cnt[q] : 0;
      int incl = v;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
      }
      if (q < nnb) L.base[q] = run + incl - v;
      run += __shfl(incl, 63);
    }
    if (lane == 0) L.nc = run;
  }
  __syncthreads();
  const int nc = L.nc;
  if (nc > CAND_CAP) {
    over = 1;
  } else {
    for (int q = w; q < nnb; q += OS_WAVES) {
      const int dx = q % span - R, dy = (q / span) % span - R, dz = q / (span * span) - R;
      const int t0 = a.start[L.cell[q]], m = L.cnt[q], b = L.base[q];
      const uint32_t ou = (uint32_t)(dx + 8) | ((uint32_t)(dy + 8) << 8) | ((uint32_t)(dz + 8) << 16);
      for (int t = lane; t < m; t += 64) {
        const double4 o = a.sorted[t0 + t];
        L.p[b + t] = make_float4((float)(o.x + dx * a.side[0]), (float)(o.y + dy * a.side[1]),
                                 (float)(o.z + dz * a.side[2]), __int_as_float((int)o.w));
        L.off[b + t] = ou;
      }
    }
  }
  __syncthreads();
  const int pop = L.cnt[q0];
  if (!over) {
    for (int gg = g; gg * OS_MOLS < pop; gg += a.groups) {
      const int ml = gg * OS_MOLS + w / OS_SPLIT, h = w % OS_SPLIT;
      double fx = 0.0, fy = 0.0, fz = 0.0;
      if (ml < pop) {
        const int self = L.base[q0] + ml;
        const float4 pm4 = L.p[self];
        const float3 pm = make_float3(pm4.x, pm4.y, pm4.z);
        const int om = __float_as_int(pm4.w);
        auto vec = [&](const float4 p) {
          float3 d = make_float3(p.x - pm.x, p.y - pm.y, p.z - pm.z);
          if (WV) d = wrapf(d, a.boxf, a.invf);
          return d;
        };
        // Lennard-Jones pairs containing m (FP64 on the exact squared distance)
        if (a.terms & ATM3_TERM_LJ) {
          for (int q = lane + 64 * h; q < nc; q += 64 * OS_SPLIT) {
            const float4 pj = L.p[q];
            const float3 v = vec(pj);
            if (q == self || !(sq3(v) < a.rc2hi)) continue;
            const int oj = __float_as_int(pj.w);
            const double x = exact_r2(a.pos, om, oj, a.box[0], a.box[1], a.box[2]);
            if (!(x < a.rc2)) continue;
            const double s2 = a.sig2 / x, s6 = s2 * s2 * s2, s12 = s6 * s6;
            const double f = a.eps24 * (2.0 * s12 - s6) / x;  // F_m = f (r_m - r_j)
            fx -= f * (double)v.x;
            fy -= f * (double)v.y;
            fz -= f * (double)v.z;
            e_lj += 0.5 * a.eps4 * (s12 - s6);
            w_lj += 0.5 * f * x;
            if (TENSOR) {
              tx += 0.5 * f * (double)(v.x * v.x);
              ty += 0.5 * f * (double)(v.y * v.y);
              tz += 0.5 * f * (double)(v.z * v.z);
            }
            npair += (om < oj) ? 1 : 0;
          }
        }
        if (a.terms & ATM3_TERM_ATM) {
          uint32_t* qb = L.q[w];
          int qn = 0;
          // evaluate the queued pairs [qn - cnt, qn), one per lane
          auto drain = [&](int cnt) {
            if (lane < cnt) {
              const uint32_t e = qb[qn - cnt + lane];
              const int xa = (int)(e & 0xffffu), xb = (int)(e >> 16);
              const float4 pa = L.p[xa], pb = L.p[xb];
              const float3 va = vec(pa), vb = vec(pb);
              float3 jk = make_float3(vb.x - va.x, vb.y - va.y, vb.z - va.z);
              if (WJ) jk = wrapf(jk, a.boxf, a.invf);
              const float x = sq3(va), y = sq3(vb), z = sq3(jk);
              const float pf = (x * y) * z;
              const int oa = __float_as_int(pa.w), ob = __float_as_int(pb.w);
              bool in = true;
              if (!(pf < a.lo6f) || fminf(x, fminf(y, z)) < a.small2)
                in = product_ok(exact_r2(a.pos, om, oa, a.box[0], a.box[1], a.box[2]),
                                exact_r2(a.pos, om, ob, a.box[0], a.box[1], a.box[2]),
                                exact_r2(a.pos, oa, ob, a.box[0], a.box[1], a.box[2]), a.rc6);
              if (in) {
                // label by input index: t0 < t1 < t2
                const Off z0{0, 0, 0}, fa = unpack_off(L.off[xa]), fb = unpack_off(L.off[xb]);
                int i0 = om, i1 = oa, i2 = ob;
                Off o0 = z0, o1 = fa, o2 = fb, to;
                int ti;
                if (i1 < i0) { ti = i0; i0 = i1; i1 = ti; to = o0; o0 = o1; o1 = to; }
                if (i2 < i1) { ti = i1; i1 = i2; i2 = ti; to = o1; o1 = o2; o2 = to; }
                if (i1 < i0) { ti = i0; i0 = i1; i1 = ti; to = o0; o0 = o1; o1 = to; }
                const int me = (om > oa ? 1 : 0) + (om > ob ? 1 : 0);
                const int vm = visited_mask(a.variant, o0, o1, o2, a.nx, a.ny, a.nz);
                if ((vm >> me) & 1) {
                  float3 f;
                  const float eu = atm_on_i(va, vb, x, y, z, a.k3nu, a.k15nu, a.k075nu, &f);
                  fx += (double)f.x;
                  fy += (double)f.y;
                  fz += (double)f.z;
                  e3 += (double)eu;
                  if (a.variant == ATM3_VARIANT_3C01 || me == 0) ++ntrip;
                }
              }
            }
            qn -= cnt;
          };
          for (int xa = h; xa + 1 < nc; xa += OS_SPLIT) {
            if (xa == self) continue;
            const float3 va = vec(L.p[xa]);
            const float xa2 = sq3(va);
            for (int xb0 = xa + 1; xb0 < nc; xb0 += 64) {
              const int xb = xb0 + lane;
              bool acc = false;
              if (xb < nc && xb != self) {
                const float3 vb = vec(L.p[xb]);
                float3 jk = make_float3(vb.x - va.x, vb.y - va.y, vb.z - va.z);
                if (WJ) jk = wrapf(jk, a.boxf, a.invf);
                const float y = sq3(vb), z = sq3(jk);
                acc = (xa2 * y) * z < a.hi6f || fminf(xa2, fminf(y, z)) < a.small2;
              }
              const unsigned long long bits = __ballot(acc);
              if (acc) qb[qn + __popcll(bits & ((1ull << lane) - 1ull))] = (uint32_t)xa | ((uint32_t)xb << 16);
              qn += __popcll(bits);
              __builtin_amdgcn_wave_barrier();
              if (qn >= 64) {
                drain(64);
                __builtin_amdgcn_wave_barrier();
              }
            }
          }
          if (qn > 0) drain(qn);
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o);
        fy += __shfl_xor(fy, o);
        fz += __shfl_xor(fz, o);
      }
      if (lane == 0) {
        L.facc[w][0] = fx;
        L.facc[w][1] = fy;
        L.facc[w][2] = fz;
      }
      __syncthreads();
      if (threadIdx.x < OS_MOLS) {
        const int m2 = gg * OS_MOLS + threadIdx.x;
        if (m2 < pop) {
          const int om = __float_as_int(L.p[L.base[q0] + m2].w);
          double s[3] = {0.0, 0.0, 0.0};
          for (int hh = 0; hh < OS_SPLIT; ++hh)
            for (int d = 0; d < 3; ++d) s[d] += L.facc[threadIdx.x * OS_SPLIT + hh][d];
          for (int d = 0; d < 3; ++d) {
            if (a.fout) a.fout[3 * (int64_t)om + d] = s[d];
            else a.forces[3 * (int64_t)om + d] = (float)s[d];
          }
        }
      }
      __syncthreads();
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    e_lj += __shfl_xor(e_lj, o);
    w_lj += __shfl_xor(w_lj, o);
    e3 += __shfl_xor(e3, o);
    npair += __shfl_xor(npair, o);
    ntrip += __shfl_xor(ntrip, o);
  }
  if (TENSOR)
    for (int o = 32; o > 0; o >>= 1) {
      tx += __shfl_xor(tx, o);
      ty += __shfl_xor(ty, o);
      tz += __shfl_xor(tz, o);
    }
  if (lane == 0) {
    L.red[w][0] = e_lj;
    L.red[w][1] = w_lj;
    L.red[w][2] = e3;
    L.redi[w][0] = npair;
    L.redi[w][1] = ntrip;
    L.tred[w][0] = tx;
    L.tred[w][1] = ty;
    L.tred[w][2] = tz;
  }
  __syncthreads();
  if (TENSOR && threadIdx.x < 3) {
    double t = 0.0;
    for (int q = 0; q < OS_WAVES; ++q) t += L.tred[q][threadIdx.x];
    a.tpart[3 * (int64_t)blockIdx.x + threadIdx.x] = t;
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      double sum = 0.0;
      for (int q = 0; q < OS_WAVES; ++q) sum += L.red[q][k];
      a.dpart[4 * (int64_t)blockIdx.x + k] = sum;
    }
    a.dpart[4 * (int64_t)blockIdx.x + 3] = 0.0;
    unsigned long long s0 = 0, s1 = 0;
    for (int q = 0; q < OS_WAVES; ++q) {
      s0 += L.redi[q][0];
      s1 += L.redi[q][1];
    }
    a.ipart[4 * (int64_t)blockIdx.x + 0] = s0;
    a.ipart[4 * (int64_t)blockIdx.x + 1] = s1;
    a.ipart[4 * (int64_t)blockIdx.x + 2] = 0;
    a.ipart[4 * (int64_t)blockIdx.x + 3] = over;
  }
}

// ---------------------------------------------------------------------------
// product cutoff, 3c08 and 3c18: one block per base cell, each triplet once
// ---------------------------------------------------------------------------
// The cell set of base cell b is staged in LDS (3c08: the 2x2x2 block with b
// as its minimum corner; 3c18: b and its 13 lexicographically greater
// neighbours, b first).  A staged triplet i < j < k belongs to b iff its
// corner codes AND to zero (3c08) or i lies in b (3c18; every other staged
// cell is lexicographically greater than b).  Waves take the rows (i, j)
// (j = wave mod 4), lanes the third molecules k > j; FP32 pre-test, queue and
// exact decision as in the one-sided kernel; the ATM force on all three
// molecules from the three minimum-image vectors (eq. forcepairs), rounded to
// 2^-32 fixed point and summed with integer atomics (LDS per block, then
// global per molecule), so the sums are exact and reproducible.
constexpr int PB_CAP = 512;   // molecules of one cell set
constexpr int PB_WAVES = 4;
constexpr int PB_QCAP = 128;
constexpr double FIX_SCALE = 4294967296.0;  // 2^32
constexpr float PB_FIX_LIMIT = 262144.f;    // 2^18: a contribution beyond is reported

struct ProdArgs {
  const double4* sorted;
  const int32_t* start;
  const double* pos;
  int32_t nx, ny, nz, splits;  // `splits` blocks share a base cell's rows
  double side[3], box[3];
  double rc6;
  float boxf[3], invf[3];
  float lo6f, hi6f, small2;
  float k3nu, k15nu, k075nu;
  unsigned long long* acc;    // [3 n] fixed-point ATM forces, input order
  double* dpart;              // per block: 0, 0, 3 sum u, 0
  unsigned long long* ipart;  // per block: 0, n_triplets, range flag, overflow
  // virial-tensor mode only: the pairwise cutoff instead of the product
  // (rc^2 with the same relative band), and per-block W_xx, W_yy, W_zz
  int32_t pair;
  double rc2;
  float lo2f, hi2f;
  double* tpart;
  // shell-pruned tier: 1 / t1 and log2(rc^6 (1 + 1e-3) / t1^2); per base
  // cell, 1 if k_prod_fast handed the cell on (k_prod_block skips the others)
  float pf_inv_t1, pf_lh;
  int32_t* pdefer;
  // with pdefer: the LJ pairs the cell set owns (Newton 3, fixed point), as
  // the one-sided kernel is not run then
  int32_t lj;
  double sig2, eps4, eps24;
};

struct ProdLds {
  float4 p[PB_CAP];  // position relative to the base cell's centre; .w = input index
  uint8_t code[PB_CAP];
  unsigned long long f[3][PB_CAP];
  uint32_t q[PB_WAVES][PB_QCAP];  // queued triplets i | j << 9 | k << 18
  int32_t cnt[16], base[16], cell[16];
  double red[PB_WAVES];
  unsigned long long redi[PB_WAVES][2];
  double tred[PB_WAVES][3];
  double redl[PB_WAVES][2];
  unsigned long long redp[PB_WAVES];
};

// The exact minimum-image difference r_a - r_b of input molecules (as in
// exact_r2, whose squared length it returns).
__device__ __forceinline__ double exact_vec(const double* __restrict__ pos, int a, int b, const double* box,
                                            double& ex, double& ey, double& ez) {
#pragma clang fp contract(off)
  double d0 = pos[3 * (int64_t)a + 0] - pos[3 * (int64_t)b + 0];
  d0 = d0 - box[0] * rint(d0 / box[0]);
  double d1 = pos[3 * (int64_t)a + 1] - pos[3 * (int64_t)b + 1];
  d1 = d1 - box[1] * rint(d1 / box[1]);
  double d2 = pos[3 * (int64_t)a + 2] - pos[3 * (int64_t)b + 2];
  d2 = d2 - box[2] * rint(d2 / box[2]);
  ex = d0;
  ey = d1;
  ez = d2;
  double s = d0 * d0;
  s = s + d1 * d1;
  s = s + d2 * d2;
  return s;
}

// eq. (atm) and eq. (forcepairs) from the three pair vectors r_ij = r_i - r_j,
// r_ik, r_jk and their squared lengths x, y, z: F_i = c_x r_ij + c_y r_ik,
// F_j = -c_x r_ij + c_z r_jk (F_k = -F_i - F_j); returns u / nu.
__device__ __forceinline__ float atm_vec(float3 ij, float3 ik, float3 jk, float x, float y, float z, float k3nu,
                                         float k15nu, float k075nu, float3* fi, float3* fj, float3* c = nullptr) {
  const float s = x + y + z;
  const float A = fmaf(-2.f, x, s), B = fmaf(-2.f, y, s), C = fmaf(-2.f, z, s);
  const float AB = A * B, AC = A * C, BC = B * C;
  const float P = AB * C;
  const float S = AB + AC + BC;
  const float xy = x * y, yz = y * z, xz = x * z;
  const float Q = xy * z;
  const float t1 = __builtin_amdgcn_rsqf(Q);
  const float t2 = t1 * t1, t3 = t2 * t1, t5 = t3 * t2;
  const float G = fmaf(k15nu * P, t5, k3nu * t3);
  const float H = k075nu * t5;
  const float cx = fmaf(G, yz * t2, -H * fmaf(-2.f, BC, S));
  const float cy = fmaf(G, xz * t2, -H * fmaf(-2.f, AC, S));
  const float cz = fmaf(G, xy * t2, -H * fmaf(-2.f, AB, S));
  fi->x = fmaf(cx, ij.x, cy * ik.x);
  fi->y = fmaf(cx, ij.y, cy * ik.y);
  fi->z = fmaf(cx, ij.z, cy * ik.z);
  fj->x = fmaf(cz, jk.x, -cx * ij.x);
  fj->y = fmaf(cz, jk.y, -cx * ij.y);
  fj->z = fmaf(cz, jk.z, -cx * ij.z);
  if (c) *c = make_float3(cx, cy, cz);
  return fmaf(0.375f * P, t5, t3);
}

__device__ __forceinline__ unsigned long long fix32(float v) {
  return (unsigned long long)(long long)rint((double)v * FIX_SCALE);
}

template <int VAR, bool WR, bool TENSOR = false>
__global__ __launch_bounds__(64 * PB_WAVES) void k_prod_block(ProdArgs a) {
  __shared__ ProdLds L;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t b = blockIdx.x / a.splits;
  const int split = blockIdx.x % a.splits;
  if (a.pdefer != nullptr && a.pdefer[b] == 0) {  // done by k_prod_fast
    if (threadIdx.x < 4) {
      a.dpart[4 * (int64_t)blockIdx.x + threadIdx.x] = 0.0;
      a.ipart[4 * (int64_t)blockIdx.x + threadIdx.x] = 0ull;
    }
    return;
  }
  const int bx = (int)(b % a.nx), by = (int)((b / a.nx) % a.ny), bz = (int)(b / ((int64_t)a.nx * a.ny));
  constexpr int NCS = (VAR == ATM3_VARIANT_3C08) ? 8 : 14;
  // offsets of the cell set; 3c18: base, then the forward half in z-major order
  auto offs = [](int q, int& dx, int& dy, int& dz) {
    if (VAR == ATM3_VARIANT_3C08) {
      dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
    } else {
      const int t = q == 0 ? 13 : 13 + q;  // index in the 27-cube, z-major
      dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    }
  };
  if (threadIdx.x < NCS) {
    int dx, dy, dz;
    offs(threadIdx.x, dx, dy, dz);
    const int ux = wrapc(bx + dx, a.nx), uy = wrapc(by + dy, a.ny), uz = wrapc(bz + dz, a.nz);
    const int cc = (uz * a.ny + uy) * a.nx + ux;
    L.cell[threadIdx.x] = cc;
    L.cnt[threadIdx.x] = a.start[cc + 1] - a.start[cc];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < NCS; ++q) {
      L.base[q] = s;
      s += L.cnt[q];
    }
    L.base[NCS] = s;
  }
  __syncthreads();
  const int n = L.base[NCS];
  double e3 = 0.0, tx = 0.0, ty = 0.0, tz = 0.0, elj = 0.0, wlj = 0.0;
  unsigned long long ntrip = 0, rng = 0, npair = 0;
  const unsigned long long over = n > PB_CAP ? 1 : 0;
  const bool pair = TENSOR && a.pair;
  if (!over) {
    for (int q = w; q < NCS; q += PB_WAVES) {
      int dx, dy, dz;
      offs(q, dx, dy, dz);
      const int t0 = a.start[L.cell[q]], m = L.cnt[q], bb = L.base[q];
      const uint8_t code = (VAR == ATM3_VARIANT_3C08) ? (uint8_t)q : (uint8_t)(q == 0 ? 0 : 1);
      for (int t = lane; t < m; t += 64) {
        const double4 o = a.sorted[t0 + t];
        L.p[bb + t] = make_float4((float)(o.x + dx * a.side[0]), (float)(o.y + dy * a.side[1]),
                                  (float)(o.z + dz * a.side[2]), __int_as_float((int)o.w));
        L.code[bb + t] = code;
      }
    }
    for (int t = threadIdx.x; t < n; t += 64 * PB_WAVES) L.f[0][t] = L.f[1][t] = L.f[2][t] = 0ull;
  }
  __syncthreads();
  if (!over) {
    auto dvec = [&](const float4 u, const float4 v) {  // minimum image of u - v
      float3 d = make_float3(u.x - v.x, u.y - v.y, u.z - v.z);
      if (WR) d = wrapf(d, a.boxf, a.invf);
      return d;
    };
    if (!TENSOR && a.lj) {
      // the LJ pairs the cell set owns (3c08: corner codes AND to zero;
      // 3c18: the first molecule in the base cell), a wave per row i, rows
      // shared by the `splits` blocks of the cell; the oracle's FP64
      // distance decides, FP64 forces in fixed point
      const int imax_lj = (VAR == ATM3_VARIANT_3C08) ? n : min(n, L.cnt[0]);
      for (int i = split * PB_WAVES + w; i < imax_lj; i += a.splits * PB_WAVES) {
        const float4 pi = L.p[i];
        const int ci = L.code[i];
        for (int j = i + 1 + lane; j < n; j += 64) {
          if (VAR == ATM3_VARIANT_3C08 && (ci & L.code[j]) != 0) continue;
          const float4 pj = L.p[j];
          if (!(sq3(dvec(pi, pj)) < a.hi2f)) continue;
          double ex, ey, ez;
          if (!(exact_vec(a.pos, __float_as_int(pi.w), __float_as_int(pj.w), a.box, ex, ey, ez) < a.rc2)) continue;
          const double f = lj_pair(ex, ey, ez, a.sig2, a.eps24, &elj, &wlj);
          const double gx = f * ex, gy = f * ey, gz = f * ez;
          if (!(fabs(gx) + fabs(gy) + fabs(gz) < (double)PB_FIX_LIMIT)) {
            rng = 1;
          } else {
            const unsigned long long vx = (unsigned long long)(long long)rint(gx * FIX_SCALE);
            const unsigned long long vy = (unsigned long long)(long long)rint(gy * FIX_SCALE);
            const unsigned long long vz = (unsigned long long)(long long)rint(gz * FIX_SCALE);
            atomicAdd(&L.f[0][i], vx);
            atomicAdd(&L.f[1][i], vy);
            atomicAdd(&L.f[2][i], vz);
            atomicAdd(&L.f[0][j], 0ull - vx);
            atomicAdd(&L.f[1][j], 0ull - vy);
            atomicAdd(&L.f[2][j], 0ull - vz);
          }
          ++npair;
        }
      }
    }
    uint32_t* qb = L.q[w];
    int qn = 0;
    auto drain = [&](int cnt) {
      if (lane < cnt) {
        const uint32_t e = qb[qn - cnt + lane];
        const int i = (int)(e & 511u), j = (int)((e >> 9) & 511u), k = (int)(e >> 18);
        const float4 pi = L.p[i], pj = L.p[j], pk = L.p[k];
        const float3 ij = dvec(pi, pj), ik = dvec(pi, pk), jk = dvec(pj, pk);
        const float x = sq3(ij), y = sq3(ik), z = sq3(jk);
        bool in = true;
        const bool near = pair ? !(fmaxf(x, fmaxf(y, z)) < a.lo2f) : !((x * y) * z < a.lo6f);
        if (near || fminf(x, fminf(y, z)) < a.small2) {
          const int oi = __float_as_int(pi.w), oj = __float_as_int(pj.w), ok = __float_as_int(pk.w);
          const double ex = exact_r2(a.pos, oi, oj, a.box[0], a.box[1], a.box[2]);
          const double ey = exact_r2(a.pos, oi, ok, a.box[0], a.box[1], a.box[2]);
          const double ez = exact_r2(a.pos, oj, ok, a.box[0], a.box[1], a.box[2]);
          in = pair ? (ex < a.rc2 && ey < a.rc2 && ez < a.rc2) : product_ok(ex, ey, ez, a.rc6);
        }
        if (in) {
          float3 fi, fj, c;
          const float u = atm_vec(ij, ik, jk, x, y, z, a.k3nu, a.k15nu, a.k075nu, &fi, &fj, &c);
          if (TENSOR) {
            // virial of the three force pairs: c_x r_ij r_ij + c_y r_ik r_ik + c_z r_jk r_jk
            tx += (double)fmaf(c.x, ij.x * ij.x, fmaf(c.y, ik.x * ik.x, c.z * (jk.x * jk.x)));
            ty += (double)fmaf(c.x, ij.y * ij.y, fmaf(c.y, ik.y * ik.y, c.z * (jk.y * jk.y)));
            tz += (double)fmaf(c.x, ij.z * ij.z, fmaf(c.y, ik.z * ik.z, c.z * (jk.z * jk.z)));
          }
          const float3 fk = make_float3(-(fi.x + fj.x), -(fi.y + fj.y), -(fi.z + fj.z));
          const float mx = fmaxf(fmaxf(fmaxf(fabsf(fi.x), fabsf(fi.y)), fmaxf(fabsf(fi.z), fabsf(fj.x))),
                                 fmaxf(fmaxf(fabsf(fj.y), fabsf(fj.z)),
                                       fmaxf(fabsf(fk.x), fmaxf(fabsf(fk.y), fabsf(fk.z)))));
          if (!(mx < PB_FIX_LIMIT)) {
            rng = 1;
          } else {
            atomicAdd(&L.f[0][i], fix32(fi.x));
            atomicAdd(&L.f[1][i], fix32(fi.y));
            atomicAdd(&L.f[2][i], fix32(fi.z));
            atomicAdd(&L.f[0][j], fix32(fj.x));
            atomicAdd(&L.f[1][j], fix32(fj.y));
            atomicAdd(&L.f[2][j], fix32(fj.z));
            atomicAdd(&L.f[0][k], fix32(fk.x));
            atomicAdd(&L.f[1][k], fix32(fk.y));
            atomicAdd(&L.f[2][k], fix32(fk.z));
          }
          e3 += 3.0 * (double)u;
          ++ntrip;
        }
      }
      qn -= cnt;
    };
    const int imax = (VAR == ATM3_VARIANT_3C08) ? n : min(n, L.cnt[0]);
    // rows (i, j) with j = split * PB_WAVES + wave modulo splits * PB_WAVES
    const int stride = a.splits * PB_WAVES, mine = split * PB_WAVES + w;
    for (int i = 0; i < imax; ++i) {
      const float4 pi = L.p[i];
      const int ci = L.code[i];
      int j = i + 1 + (((mine - (i + 1)) % stride) + stride) % stride;
      for (; j + 1 < n; j += stride) {
        const float4 pj = L.p[j];
        const int cij = ci & L.code[j];
        const float3 ij = dvec(pi, pj);
        const float x = sq3(ij);
        for (int k0 = j + 1; k0 < n; k0 += 64) {
          const int k = k0 + lane;
          bool acc = false;
          if (k < n && (VAR != ATM3_VARIANT_3C08 || (L.code[k] & cij) == 0)) {
            const float4 pk = L.p[k];
            const float y = sq3(dvec(pi, pk)), z = sq3(dvec(pj, pk));
            acc = (pair ? fmaxf(x, fmaxf(y, z)) < a.hi2f : (x * y) * z < a.hi6f) || fminf(x, fminf(y, z)) < a.small2;
          }
          const unsigned long long bits = __ballot(acc);
          if (acc)
            qb[qn + __popcll(bits & ((1ull << lane) - 1ull))] =
                (uint32_t)i | ((uint32_t)j << 9) | ((uint32_t)k << 18);
          qn += __popcll(bits);
          __builtin_amdgcn_wave_barrier();
          if (qn >= 64) {
            drain(64);
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
    }
    if (qn > 0) drain(qn);
  }
  __syncthreads();
  if (!over) {
    for (int t = threadIdx.x; t < n; t += 64 * PB_WAVES) {
      const int o = __float_as_int(L.p[t].w);
      for (int d = 0; d < 3; ++d) {
        const unsigned long long v = L.f[d][t];
        if (v) atomicAdd(&a.acc[3 * (int64_t)o + d], v);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    e3 += __shfl_xor(e3, o);
    ntrip += __shfl_xor(ntrip, o);
    rng |= __shfl_xor(rng, o);
    elj += __shfl_xor(elj, o);
    wlj += __shfl_xor(wlj, o);
    npair += __shfl_xor(npair, o);
    if (TENSOR) {
      tx += __shfl_xor(tx, o);
      ty += __shfl_xor(ty, o);
      tz += __shfl_xor(tz, o);
    }
  }
  if (lane == 0) {
    L.red[w] = e3;
    L.redi[w][0] = ntrip;
    L.redi[w][1] = rng;
    L.redl[w][0] = elj;
    L.redl[w][1] = wlj;
    L.redp[w] = npair;
    if (TENSOR) {
      L.tred[w][0] = tx;
      L.tred[w][1] = ty;
      L.tred[w][2] = tz;
    }
  }
  __syncthreads();
  if (TENSOR && threadIdx.x < 3) {
    double t = 0.0;
    for (int q = 0; q < PB_WAVES; ++q) t += L.tred[q][threadIdx.x];
    a.tpart[3 * (int64_t)blockIdx.x + threadIdx.x] = t;
  }
  if (threadIdx.x == 0) {
    double s = 0.0, sl = 0.0, sw = 0.0;
    unsigned long long t = 0, r = 0, sp = 0;
    for (int q = 0; q < PB_WAVES; ++q) {
      s += L.red[q];
      t += L.redi[q][0];
      r |= L.redi[q][1];
      sl += L.redl[q][0];
      sw += L.redl[q][1];
      sp += L.redp[q];
    }
    const int64_t blk = blockIdx.x;
    a.dpart[4 * blk + 0] = a.eps4 * sl;
    a.dpart[4 * blk + 1] = a.eps24 * sw;
    a.dpart[4 * blk + 2] = s;
    a.dpart[4 * blk + 3] = 0.0;
    a.ipart[4 * blk + 0] = sp;
    a.ipart[4 * blk + 1] = t;
    a.ipart[4 * blk + 2] = r;
    a.ipart[4 * blk + 3] = over;
  }
}

// ---------------------------------------------------------------------------
// product cutoff, 3c08 and 3c18: shell-pruned tier
// ---------------------------------------------------------------------------
// Same cell sets and ownership as k_prod_block, with the third molecules
// pruned before any triplet is evaluated.  Each triplet of a cell set is
// enumerated once, by its designated pair: the pair with the smallest FP32
// squared side (ties: the smaller pair key i << 8 | j, i < j, in staging
// order).  A triplet inside the product cutoff has its shortest side inside
// rc (x^3 <= x y z < rc^6), so the rows are the pairs within rc (a relative
// band wider), and the third molecules k of row (i, j), squared side x, are
// those with y = |r_ik|^2 >= x, z = |r_jk|^2 >= x and x y z < rc^6.
// Shells: every staged squared distance D falls in one of 16 shells, shell
// 0 below t1 = rc^2 (1 + 1e-4) / 8 and shell a >= 1 from t1 2^((a - 1) / 2)
// up (one more than the FP32 exponent of (D / t1)^2), held as four bit
// planes per row and mask word.  A lane per row keeps the k whose shells
// with i and with j are both at least x's and whose shell lower bounds allow
// x y z < rc^6 (1 + 1e-3): with y >= t1 2^((a - 1) / 2) and z likewise that
// is a + b <= 1 + ceil(2 log2(rc^6 (1 + 1e-3) / (t1^2 x))), a bit-sliced add
// and compare over 64 molecules at once.  The kept set holds every triplet
// inside the cutoff and about half as many again on the benchmark fluid.
// It is cut into work items of at most PF_NCLS molecules, counting-sorted by
// size, and a lane per item takes the designation test, the product test
// (FP32 with a relative band, the oracle's FP64 test inside it and for sides
// under a quarter cell) and the ATM force on all three molecules (eq.
// forcepairs: the pair's two forces summed over its items in registers),
// in 2^-32 fixed point, as is the energy.  Blocks beyond the tier (more
// molecules, rows or items than it holds) set their flag in `pdefer` and
// k_prod_block evaluates them.
constexpr int PF_WG = 256;
constexpr int PF_NCLS = 12;                    // third molecules per work item at most
constexpr int PF_NSH = 16;                     // shells: four bit planes
constexpr float PF_FIX_LIMIT = 262144.f;       // 2^18: the fixed-point conversion's range

template <int NW, int PCAP, int KCAP>
struct ProdFastLds {
  static constexpr int MAXB = 64 * NW;
  float4 p[MAXB];                        // block-frame position, .w = input index
  float lo[3][MAXB];                     // residuals: coordinate - (double)p
  alignas(16) unsigned long long pl[MAXB][NW][4];  // bit k of plane b: bit b of the shell of (i, k)
  unsigned long long own[8][NW];         // 3c08: k with code & m == 0; 3c18: [0] base cell, [1] all
  unsigned long long f[3][MAXB];         // ATM forces, 2^-32 units
  uint16_t plist[PCAP];                  // rows i | j << 8, i < j
  unsigned long long kset[KCAP];         // third molecules of an item (bits of word w)
  uint16_t kmeta[KCAP];                  // row | w << 12
  uint8_t code[MAXB];
  int32_t cnt[16], base[16], cell[16], gst[16];  // populations, staged offsets, cells, first sorted slots
  int32_t ccnt[2][PF_NCLS + 1], cursor[PF_NCLS + 1];  // class counts per half of the workgroup
  int32_t wsum[PF_WG / 64];
  int32_t nrows, nitems, abort, nsub;
  unsigned long long red[PF_WG / 64][4];
  double redd[PF_WG / 64][2];
};

// 2^-32 fixed point by a magic add in FP64 (|v| < 2^19; the caller checks).
__device__ __forceinline__ unsigned long long pf_fix(float v) {
  const double t = (double)v + 1572864.0;
  return (unsigned long long)__double_as_longlong(t) - 0x4138000000000000ull;
}

__device__ __forceinline__ unsigned long long pf_fixd(double v) {
  const double t = v + 1572864.0;
  return (unsigned long long)__double_as_longlong(t) - 0x4138000000000000ull;
}

// Shell of a squared distance d (inv_t1 = 1 / t1): shell a >= 1 holds
// t1 2^((a - 1) / 2) <= d, that is 2^(a - 1) <= (d / t1)^2, so a is one more
// than the binary exponent of (d / t1)^2 (in FP32, a monotone function of
// d); 0 below t1, at most PF_NSH - 1.
__device__ __forceinline__ int pf_shell(float d, float inv_t1) {
  const float u = d * inv_t1;
  const int e = (int)(__float_as_uint(u * u) >> 23) - 126;
  return min(max(e, 0), PF_NSH - 1);
}

// Bit-sliced comparisons with a per-lane constant c whose bits are given as
// all-ones / zero masks m[b]: values (planes v[]) >= c, and <= c.
template <int NB>
__device__ __forceinline__ unsigned long long pf_ge(const unsigned long long* v, const unsigned long long* m) {
  unsigned long long lt = 0ull, eq = ~0ull;
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    lt |= eq & ~v[b] & m[b];
    eq &= ~(v[b] ^ m[b]);
  }
  return ~lt;
}
template <int NB>
__device__ __forceinline__ unsigned long long pf_le(const unsigned long long* v, const unsigned long long* m) {
  unsigned long long gt = 0ull, eq = ~0ull;
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    gt |= eq & v[b] & ~m[b];
    eq &= ~(v[b] ^ m[b]);
  }
  return ~gt;
}

// Exclusive prefix over the block of one value per thread; *total gets the sum.
__device__ __forceinline__ int pf_scan(int v, int32_t* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int s = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(s, o);
    if (lane >= o) s += t;
  }
  if (lane == 63) wsum[wave] = s;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < PF_WG / 64; ++q) {
    before += q < wave ? wsum[q] : 0;
    all += wsum[q];
  }
  __syncthreads();
  *total = all;
  return before + s - v;
}

// RPT rows per thread and round.  A round whose items exceed KCAP runs as
// two halves; a half that alone exceeds it hands the block on.  On the
// benchmark fluid 3c08 takes rounds of 512 rows (at most about 1,600 of
// 2,048 items).  3c18 takes rounds of 1,024: its first rows, those of the
// base cell's molecules, take third molecules from the whole set and split
// into halves, but most of its rows have no base-cell member, must take
// the third molecule from the base cell, and make items of one or two
// candidates; small rounds of those were dominated by their barriers
// (rounds of 256 rows: 16.3 ms per evaluation, 512: 15.2, 1,024: 14.8;
// 1,536 and more hand sets on)
template <int VAR, int NW, int PCAP, int KCAP, int RPT>
__global__ __launch_bounds__(PF_WG) void k_prod_fast(ProdArgs a) {
  using Lds = ProdFastLds<NW, PCAP, KCAP>;
  constexpr int MAXB = Lds::MAXB;
  constexpr int NCS = (VAR == ATM3_VARIANT_3C08) ? 8 : 14;
  static_assert(PCAP <= 4096 && NW <= 4 && MAXB <= 256, "12-bit rows, 2-bit words, 8-bit molecule indices");
  static_assert(PF_WG == 256, "two halves of 128 threads (tid >> 7)");
  __shared__ Lds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ncells = (int64_t)a.nx * a.ny * a.nz;
  const int64_t per = (ncells + 7) / 8;
  const int64_t b = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if ((int64_t)(blockIdx.x >> 3) >= per || b >= ncells) return;
  const int bx = (int)(b % a.nx), by = (int)((b / a.nx) % a.ny), bz = (int)(b / ((int64_t)a.nx * a.ny));
  auto offs = [](int q, int& dx, int& dy, int& dz) {
    if (VAR == ATM3_VARIANT_3C08) {
      dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
    } else {
      const int t = q == 0 ? 13 : 13 + q;  // base, then the forward half of the 27-cube in z-major order
      dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    }
  };
  if (tid < NCS) {
    int dx, dy, dz;
    offs(tid, dx, dy, dz);
    const int ux = wrapc(bx + dx, a.nx), uy = wrapc(by + dy, a.ny), uz = wrapc(bz + dz, a.nz);
    const int cc = (uz * a.ny + uy) * a.nx + ux;
    L.cell[tid] = cc;
    L.gst[tid] = a.start[cc];
    L.cnt[tid] = a.start[cc + 1] - L.gst[tid];
  }
  if (tid < 2 * (PF_NCLS + 1)) L.ccnt[tid / (PF_NCLS + 1)][tid % (PF_NCLS + 1)] = 0;
  if (tid == 0) L.abort = 0;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int q = 0; q < NCS; ++q) {
      L.base[q] = s;
      s += L.cnt[q];
    }
    L.base[NCS] = s;
  }
  __syncthreads();
  const int n = L.base[NCS];
  unsigned long long eacc = 0ull;
  int ntr = 0, far = 0, npair = 0;
  double elj = 0.0, wlj = 0.0;
  bool fits = n <= MAXB;
  if (fits) {
    // 1. stage the cell set (block frame: relative to the base cell's centre),
    //    a thread per molecule: its cell q is the number of later cells
    //    whose staged range starts at or before it, so that every record is
    //    fetched in one round of independent loads
    for (int t = tid; t < n; t += PF_WG) {
      int q = 0;
#pragma unroll
      for (int c = 1; c < NCS; ++c) q += (L.base[c] <= t) ? 1 : 0;
      int dx, dy, dz;
      offs(q, dx, dy, dz);
      const uint8_t code = (VAR == ATM3_VARIANT_3C08) ? (uint8_t)q : (uint8_t)(q == 0 ? 0 : 1);
      const double4 o = a.sorted[L.gst[q] + (t - L.base[q])];
      const double vx = o.x + dx * a.side[0], vy = o.y + dy * a.side[1], vz = o.z + dz * a.side[2];
      const float hx = (float)vx, hy = (float)vy, hz = (float)vz;
      L.p[t] = make_float4(hx, hy, hz, __int_as_float((int)o.w));
      L.lo[0][t] = (float)(vx - (double)hx);
      L.lo[1][t] = (float)(vy - (double)hy);
      L.lo[2][t] = (float)(vz - (double)hz);
      L.code[t] = code;
    }
    for (int t = tid; t < n; t += PF_WG) L.f[0][t] = L.f[1][t] = L.f[2][t] = 0ull;
    __syncthreads();
    // 2. shell planes, a wave per row, and the ownership masks.  shell(i, k)
    //    equals shell(k, i) bit for bit (the FP32 differences are exact
    //    negatives of each other and sq3 sums in a fixed order), so row i
    //    computes its words w >= i / 64 only; the words below the diagonal of
    //    64 x 64 blocks are bit transposes of the blocks above, next
    for (int i = wave; i < n; i += PF_WG / 64) {
      const float4 pi = L.p[i];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        if (w < (i >> 6)) continue;  // uniform: one row per wave
        const int k = 64 * w + lane;
        int s = 0;
        if (k < n) {
          const float4 pk = L.p[k];
          s = pf_shell(sq3(make_float3(pi.x - pk.x, pi.y - pk.y, pi.z - pk.z)), a.pf_inv_t1);
        }
        const unsigned long long b0 = __ballot(s & 1), b1 = __ballot(s & 2), b2 = __ballot(s & 4),
                                 b3 = __ballot(s & 8);
        if (lane == 0) {
          *(ulonglong2*)&L.pl[i][w][0] = make_ulonglong2(b0, b1);
          *(ulonglong2*)&L.pl[i][w][2] = make_ulonglong2(b2, b3);
        }
      }
    }
    constexpr int NOWN = (VAR == ATM3_VARIANT_3C08) ? 8 : 2;
    for (int task = wave; task < NOWN * NW; task += PF_WG / 64) {
      const int m = task / NW, w = task - (task / NW) * NW;
      const int k = 64 * w + lane;
      bool okk = false;
      if (k < n) okk = (VAR == ATM3_VARIANT_3C08) ? (L.code[k] & m) == 0 : (m == 1 || L.code[k] == 0);
      const unsigned long long bits = __ballot(okk);
      if (lane == 0) L.own[m][w] = bits;
    }
    __syncthreads();
    // block (I, K), K > I, plane b: lane l holds row 64 I + l's word K (zero
    // past n); six butterfly stages (lanes l and l ^ h exchange their words,
    // h = 32 ... 1, and each keeps its own bit groups of size h on its side
    // of the diagonal and takes the partner's from the other) leave in lane
    // l the column 64 K + l over those rows, which is row 64 K + l's word I
    {
      constexpr int NBLK = NW * (NW - 1) / 2;
      for (int task = wave; task < 4 * NBLK; task += PF_WG / 64) {
        const int blk = task >> 2, b = task & 3;
        int I = 0, t = blk;  // the blk-th pair I < K in order
        while (t >= NW - 1 - I) t -= NW - 1 - I++;
        const int K = I + 1 + t;
        if (64 * K >= n) continue;  // uniform: no rows in word K
        const int r = 64 * I + lane;
        unsigned long long x = r < n ? L.pl[r][K][b] : 0ull;
#pragma unroll
        for (int st = 5; st >= 0; --st) {
          const int h = 1 << st;
          const unsigned long long m = h == 32 ? 0x00000000FFFFFFFFull
                                     : h == 16 ? 0x0000FFFF0000FFFFull
                                     : h == 8  ? 0x00FF00FF00FF00FFull
                                     : h == 4  ? 0x0F0F0F0F0F0F0F0Full
                                     : h == 2  ? 0x3333333333333333ull
                                               : 0x5555555555555555ull;
          const unsigned long long y = __shfl_xor(x, h);
          x = (lane & h) ? ((x & ~m) | ((y & ~m) >> h)) : ((x & m) | ((y & m) << h));
        }
        L.pl[64 * K + lane][I][b] = x;
      }
    }
    __syncthreads();
    // 3. rows: pairs i < j with shell <= 6 (D < t1 * 8 = rc^2 (1 + 1e-4)), a thread per molecule i
    unsigned long long rw[NW];
    int cnt = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      rw[w] = 0ull;
      if (tid < n) {
        const unsigned long long* v = L.pl[tid][w];
        const int lo = tid - 64 * w + 1;  // bits k > tid
        const unsigned long long gt = lo <= 0 ? ~0ull : (lo >= 64 ? 0ull : (~0ull << lo));
        rw[w] = ~v[3] & ~(v[2] & v[1] & v[0]) & gt & L.own[VAR == ATM3_VARIANT_3C08 ? 0 : 1][w];
        cnt += __popcll(rw[w]);
      }
    }
    int nrows = 0;
    int off = pf_scan(cnt, L.wsum, &nrows);
    if (nrows > PCAP) {
      fits = false;
    } else {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        unsigned long long bits = rw[w];
        while (bits) {
          const int j = 64 * w + __builtin_ctzll(bits);
          bits &= bits - 1;
          L.plist[off++] = (uint16_t)(tid | (j << 8));
        }
      }
    }
    __syncthreads();
    // 4. rounds of PF_WG * RPT rows: kept third molecules, items, ATM.
    //    row_words: the K words of row q (zero past the rows), with the
    //    row's LJ term when `lj` (once per row)
    auto row_words = [&](int q, unsigned long long* Kq, bool lj) {
#pragma unroll
      for (int w = 0; w < NW; ++w) Kq[w] = 0ull;
      if (q >= nrows) return;
      const int pr = L.plist[q], i = pr & 255, j = pr >> 8;
      const float4 pi = L.p[i], pj = L.p[j];
      const float x = sq3(make_float3(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z));
      const int ax = pf_shell(x, a.pf_inv_t1);
      int cmax = 31;
      // 2 log2(rc^6 (1 + 1e-3) / (t1^2 x)) from a constant and log2 x; the
      // 1e-3 added before rounding up covers the rounding of both forms
      if (ax > 0) cmax = min(31, (int)ceilf(2.f * (a.pf_lh - __log2f(x)) + 1e-3f) + 1);
      unsigned long long mx[4], mc[5];
#pragma unroll
      for (int t = 0; t < 4; ++t) mx[t] = ((ax >> t) & 1) ? ~0ull : 0ull;
#pragma unroll
      for (int t = 0; t < 5; ++t) mc[t] = ((cmax >> t) & 1) ? ~0ull : 0ull;
      const int ci = L.code[i], cj = L.code[j];
      const int om = (VAR == ATM3_VARIANT_3C08) ? (ci & cj) : ((ci == 0 || cj == 0) ? 1 : 0);
      // the LJ term of an owned pair within rc (FP32 test, the oracle's
      // FP64 test in a relative band; FP64 on the coordinates with their
      // residuals), Newton 3 in fixed point
      if (lj && a.lj && ((VAR == ATM3_VARIANT_3C08) ? om == 0 : om == 1) && x < a.hi2f) {
        bool in = x < a.lo2f;
        if (!in)
          in = exact_r2(a.pos, __float_as_int(pi.w), __float_as_int(pj.w), a.box[0], a.box[1], a.box[2]) < a.rc2;
        if (in) {
          const double ex = ((double)pi.x - (double)pj.x) + ((double)L.lo[0][i] - (double)L.lo[0][j]);
          const double ey = ((double)pi.y - (double)pj.y) + ((double)L.lo[1][i] - (double)L.lo[1][j]);
          const double ez = ((double)pi.z - (double)pj.z) + ((double)L.lo[2][i] - (double)L.lo[2][j]);
          const double f = lj_pair(ex, ey, ez, a.sig2, a.eps24, &elj, &wlj);
          const double gx = f * ex, gy = f * ey, gz = f * ez;
          far |= !(fabs(gx) + fabs(gy) + fabs(gz) < (double)PF_FIX_LIMIT);
          atomicAdd(&L.f[0][i], pf_fixd(gx));
          atomicAdd(&L.f[1][i], pf_fixd(gy));
          atomicAdd(&L.f[2][i], pf_fixd(gz));
          atomicAdd(&L.f[0][j], pf_fixd(-gx));
          atomicAdd(&L.f[1][j], pf_fixd(-gy));
          atomicAdd(&L.f[2][j], pf_fixd(-gz));
          ++npair;
        }
      }
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        // words holding no molecule the row may take (rows whose third
        // molecule must lie in the base cell, or corner 0 of 3c08) are skipped
        const unsigned long long ow = L.own[om][w];
        if (ow == 0ull) continue;
        unsigned long long vi[4], vj[4], s[5];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          vi[t] = L.pl[i][w][t];
          vj[t] = L.pl[j][w][t];
        }
        // s = shell(i, k) + shell(j, k), five planes
        unsigned long long c = 0ull;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const unsigned long long h = vi[t] ^ vj[t];
          s[t] = h ^ c;
          c = (vi[t] & vj[t]) | (c & h);
        }
        s[4] = c;
        // shells >= ax: the row's own shell is at most 6, so the top plane
        // alone decides shells of 8 and more, three planes the others
        unsigned long long kw = (vi[3] | pf_ge<3>(vi, mx)) & (vj[3] | pf_ge<3>(vj, mx)) & pf_le<5>(s, mc) & ow;
        if ((i >> 6) == w) kw &= ~(1ull << (i & 63));
        if ((j >> 6) == w) kw &= ~(1ull << (j & 63));
        Kq[w] = kw;
      }
    };
    // items of one row per size class, in the counters of this thread's half
    auto count_items = [&](const unsigned long long* Kq) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int p = __popcll(Kq[w]);
        if (p >= PF_NCLS) atomicAdd(&L.ccnt[tid >> 7][PF_NCLS], p / PF_NCLS);
        if (p % PF_NCLS) atomicAdd(&L.ccnt[tid >> 7][p % PF_NCLS], 1);
      }
    };
    // class cursors, largest items first, by wave 0 (lane l takes class
    // PF_NCLS - l, a scan gives the cursors): both halves (sub < 0) or one.
    // With `decide`, the round's class totals first choose one pass (both
    // halves, if their items fit KCAP together) or two (sub 0 now), and
    // flag the block when one half alone overflows
    auto wave_incl = [&](int v) {
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (lane >= o) v += t;
      }
      return v;
    };
    auto set_cursors = [&](int sub, bool decide) {
      if (wave == 0) {
        const int c = PF_NCLS - lane;
        const int c0 = lane < PF_NCLS ? L.ccnt[0][c] : 0, c1 = lane < PF_NCLS ? L.ccnt[1][c] : 0;
        if (decide) {
          const int t0 = __shfl(wave_incl(c0), 63), t1 = __shfl(wave_incl(c1), 63);
          const int nsub = (t0 + t1 <= KCAP) ? 1 : 2;
          if (lane == 0) {
            L.nsub = nsub;
            if (t0 > KCAP || t1 > KCAP) L.abort = 1;
          }
          sub = nsub == 1 ? -1 : 0;
        }
        const int v = sub < 0 ? c0 + c1 : (sub == 0 ? c0 : c1);
        const int incl = wave_incl(v);
        if (lane < PF_NCLS) L.cursor[c] = incl - v;
        if (lane == PF_NCLS - 1) L.nitems = incl;
      }
    };
    // this thread's items: runs of PF_NCLS set bits, lowest first, then the
    // rest.  The slot of the first item of every word (the whole word when
    // it has at most PF_NCLS bits) comes from an atomic per word, all of
    // them issued before any is waited for; then the stores, and the further
    // items of words with more bits
    auto place_items = [&](int r0, unsigned long long (&K)[RPT][NW]) {
      int slot[RPT][NW];
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr)
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const int pc = __popcll(K[rr][w]), c = pc < PF_NCLS ? pc : PF_NCLS;
          slot[rr][w] = c ? atomicAdd(&L.cursor[c], 1) : 0;
        }
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr) {
        const int q = r0 + rr * PF_WG + tid;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          unsigned long long bits = K[rr][w];
          int at = slot[rr][w];
          while (bits) {
            unsigned long long run = bits;
            if (__popcll(bits) > PF_NCLS) {  // the lowest PF_NCLS bits
              unsigned long long t = bits;
              for (int u = 0; u < PF_NCLS; ++u) t &= t - 1ull;
              run = bits ^ t;
            }
            bits ^= run;
            L.kset[at] = run;
            L.kmeta[at] = (uint16_t)(q | (w << 12));
            if (bits) {
              const int pc = __popcll(bits);
              at = atomicAdd(&L.cursor[pc < PF_NCLS ? pc : PF_NCLS], 1);
            }
          }
        }
      }
    };
    // a thread per item: designation, product test, ATM on all three molecules
    auto atm_pass = [&]() {
      const int nitems = L.nitems;
      for (int e = tid; e < nitems; e += PF_WG) {
        const int meta = L.kmeta[e], q = meta & 0xfff, w = meta >> 12;
        unsigned long long bits = L.kset[e];
        const int pr = L.plist[q], i = pr & 255, j = pr >> 8;
        const float4 pi = L.p[i], pj = L.p[j];
        const float ijx = pi.x - pj.x, ijy = pi.y - pj.y, ijz = pi.z - pj.z;
        const float x = sq3(make_float3(ijx, ijy, ijz));
        const float ix = __builtin_amdgcn_rcpf(x);  // 1 ulp, as in the pairwise-cutoff block kernel
        const int kij = (i << 8) | j;
        // a designated candidate has x as its shortest side, so the
        // quarter-cell test of the oracle's FP64 path reads x alone
        const bool xsmall = x < a.small2;
        float cxs = 0.f, fix = 0.f, fiy = 0.f, fiz = 0.f, fjx = 0.f, fjy = 0.f, fjz = 0.f, eu = 0.f;
        int nt = 0;
        while (bits) {
          const int k = 64 * w + __builtin_ctzll(bits);
          bits &= bits - 1ull;
          const float4 pk = L.p[k];
          const float ikx = pi.x - pk.x, iky = pi.y - pk.y, ikz = pi.z - pk.z;
          const float jkx = pj.x - pk.x, jky = pj.y - pk.y, jkz = pj.z - pk.z;
          const float y = sq3(make_float3(ikx, iky, ikz)), z = sq3(make_float3(jkx, jky, jkz));
          // designation and product tests as one mask (bitwise, so that they
          // compile to lane masks, not to a branch per condition); the pair
          // keys break ties of squared sides only, which a wave almost never
          // has; the oracle's FP64 test runs only for designated candidates
          // in the band or with a side under a quarter cell
          bool des = (y > x) & (z > x);
          if ((y == x) | (z == x)) {
            const int kik = k < i ? ((k << 8) | i) : ((i << 8) | k);
            const int kjk = k < j ? ((k << 8) | j) : ((j << 8) | k);
            des = ((y > x) | ((y == x) & (kik > kij))) & ((z > x) | ((z == x) & (kjk > kij)));
          }
          const float prod = (x * y) * z;
          bool in = des & (prod < a.lo6f);
          if (des & ((!in & (prod < a.hi6f)) | xsmall)) {
            const int oi = __float_as_int(pi.w), oj = __float_as_int(pj.w), ok = __float_as_int(pk.w);
            const double ex = exact_r2(a.pos, oi, oj, a.box[0], a.box[1], a.box[2]);
            const double ey = exact_r2(a.pos, oi, ok, a.box[0], a.box[1], a.box[2]);
            const double ez = exact_r2(a.pos, oj, ok, a.box[0], a.box[1], a.box[2]);
            in = product_ok(ex, ey, ez, a.rc6);
          }
          if (!in) continue;
          // eq. (atm) in squared sides and eq. (forcepairs), as atm_vec
          const float s = x + y + z;
          const float A = fmaf(-2.f, x, s), B = fmaf(-2.f, y, s), C = fmaf(-2.f, z, s);
          const float AB = A * B, AC = A * C, BC = B * C;
          const float P = AB * C, S = AB + AC + BC;
          const float xy = x * y, xz = x * z;
          const float t1 = __builtin_amdgcn_rsqf(xy * z);
          const float t2 = t1 * t1, t3 = t2 * t1, t5 = t3 * t2;
          const float u = P * t5;
          eu += fmaf(0.375f, u, t3);
          const float G = fmaf(a.k15nu, u, a.k3nu * t3);
          const float H = a.k075nu * t5;
          const float Gt2 = G * t2, H2 = H + H, nHS = -H * S;
          const float cx = fmaf(G, ix, fmaf(H2, BC, nHS));
          const float cy = fmaf(Gt2, xz, fmaf(H2, AC, nHS));
          const float cz = fmaf(Gt2, xy, fmaf(H2, AB, nHS));
          cxs += cx;
          fix = fmaf(cy, ikx, fix);
          fiy = fmaf(cy, iky, fiy);
          fiz = fmaf(cy, ikz, fiz);
          fjx = fmaf(cz, jkx, fjx);
          fjy = fmaf(cz, jky, fjy);
          fjz = fmaf(cz, jkz, fjz);
          const float fkx = -fmaf(cy, ikx, cz * jkx), fky = -fmaf(cy, iky, cz * jky), fkz = -fmaf(cy, ikz, cz * jkz);
          far |= !(fmaxf(fabsf(fkx), fmaxf(fabsf(fky), fabsf(fkz))) < PF_FIX_LIMIT);
          atomicAdd(&L.f[0][k], pf_fix(fkx));
          atomicAdd(&L.f[1][k], pf_fix(fky));
          atomicAdd(&L.f[2][k], pf_fix(fkz));
          ++nt;
        }
        if (nt) {
          const float Fix = fmaf(cxs, ijx, fix), Fiy = fmaf(cxs, ijy, fiy), Fiz = fmaf(cxs, ijz, fiz);
          const float Fjx = fmaf(-cxs, ijx, fjx), Fjy = fmaf(-cxs, ijy, fjy), Fjz = fmaf(-cxs, ijz, fjz);
          far |= !(fmaxf(fmaxf(fabsf(Fix), fmaxf(fabsf(Fiy), fabsf(Fiz))),
                         fmaxf(fabsf(Fjx), fmaxf(fabsf(Fjy), fabsf(Fjz)))) < PF_FIX_LIMIT);
          far |= !(fabsf(eu) < PF_FIX_LIMIT);
          atomicAdd(&L.f[0][i], pf_fix(Fix));
          atomicAdd(&L.f[1][i], pf_fix(Fiy));
          atomicAdd(&L.f[2][i], pf_fix(Fiz));
          atomicAdd(&L.f[0][j], pf_fix(Fjx));
          atomicAdd(&L.f[1][j], pf_fix(Fjy));
          atomicAdd(&L.f[2][j], pf_fix(Fjz));
          eacc += pf_fix(eu);
          ntr += nt;
        }
      }
    };
    for (int r0 = 0; fits && r0 < nrows; r0 += PF_WG * RPT) {
      unsigned long long K[RPT][NW];
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr) {
        row_words(r0 + rr * PF_WG + tid, K[rr], true);
        count_items(K[rr]);
      }
      __syncthreads();
      // the round's items: in one pass if they fit KCAP, else the two halves
      // of the workgroup's rows one after the other, the second half forming
      // its K words again (the block is handed on only if one half alone
      // overflows)
      set_cursors(0, true);
      __syncthreads();
      if (L.abort) {
        fits = false;
        break;
      }
      const int nsub = L.nsub;
      if (nsub == 1 || (tid >> 7) == 0) place_items(r0, K);
      __syncthreads();
      atm_pass();
      __syncthreads();
      if (nsub == 2) {
        set_cursors(1, false);
        __syncthreads();
        if ((tid >> 7) == 1) {
#pragma unroll
          for (int rr = 0; rr < RPT; ++rr) row_words(r0 + rr * PF_WG + tid, K[rr], false);
          place_items(r0, K);
        }
        __syncthreads();
        atm_pass();
        __syncthreads();
      }
      if (tid < 2 * (PF_NCLS + 1)) L.ccnt[tid / (PF_NCLS + 1)][tid % (PF_NCLS + 1)] = 0;
      __syncthreads();
    }
  }
  // 5. forces to the per-molecule accumulators, block partials, or the flag
  //    that hands the base cell to k_prod_block
  const unsigned long long far_all = (unsigned long long)far;
  if (fits) {
    for (int t = tid; t < n; t += PF_WG) {
      const int o = __float_as_int(L.p[t].w);
      for (int d = 0; d < 3; ++d) {
        const unsigned long long v = L.f[d][t];
        if (v) atomicAdd(&a.acc[3 * (int64_t)o + d], v);
      }
    }
  }
  unsigned long long e = eacc, nt = (unsigned long long)ntr, fr = far_all, np2 = (unsigned long long)npair;
  for (int o = 32; o > 0; o >>= 1) {
    e += __shfl_xor(e, o);
    nt += __shfl_xor(nt, o);
    fr |= __shfl_xor(fr, o);
    np2 += __shfl_xor(np2, o);
    elj += __shfl_xor(elj, o);
    wlj += __shfl_xor(wlj, o);
  }
  if (lane == 0) {
    L.red[wave][0] = e;
    L.red[wave][1] = nt;
    L.red[wave][2] = fr;
    L.red[wave][3] = np2;
    L.redd[wave][0] = elj;
    L.redd[wave][1] = wlj;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long se = 0, st = 0, sf = 0, sp = 0;
    double sel = 0.0, swl = 0.0;
    for (int q = 0; q < PF_WG / 64; ++q) {
      se += L.red[q][0];
      st += L.red[q][1];
      sf |= L.red[q][2];
      sp += L.red[q][3];
      sel += L.redd[q][0];
      swl += L.redd[q][1];
    }
    a.pdefer[b] = fits ? 0 : 1;
    a.dpart[4 * b + 0] = fits ? a.eps4 * sel : 0.0;
    a.dpart[4 * b + 1] = fits ? a.eps24 * swl : 0.0;
    a.dpart[4 * b + 2] = fits ? 3.0 * (double)(long long)se * (1.0 / FIX_SCALE) : 0.0;
    a.dpart[4 * b + 3] = 0.0;
    a.ipart[4 * b + 0] = fits ? sp : 0;
    a.ipart[4 * b + 1] = fits ? st : 0;
    a.ipart[4 * b + 2] = fits ? sf : 0;
    a.ipart[4 * b + 3] = 0;
  }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = 0ull;
}

// forces = FP64 LJ force (when computed) + fixed-point ATM force, rounded once.
__global__ __launch_bounds__(256) void k_prod_forces(const double* __restrict__ lj,
                                                     const unsigned long long* __restrict__ acc, int64_t m,
                                                     float* __restrict__ forces) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double f3 = (double)(long long)acc[i] * (1.0 / FIX_SCALE);
  forces[i] = (float)(lj ? lj[i] + f3 : f3);
}

// First stage of the fixed-order sums: block g adds the partials
// [g * chunk, (g + 1) * chunk) of dpart / ipart into entry g of dout / iout.
__global__ __launch_bounds__(256) void k_partials_sum(const double* __restrict__ dpart,
                                                      const unsigned long long* __restrict__ ipart, int32_t nb,
                                                      int32_t chunk, double* __restrict__ dout,
                                                      unsigned long long* __restrict__ iout) {
  __shared__ double sd[3][256];
  __shared__ unsigned long long si[4][256];
  const int tid = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min((int64_t)nb, lo + chunk);
  double d[3] = {0.0, 0.0, 0.0};
  unsigned long long c[4] = {0, 0, 0, 0};
  for (int64_t b = lo + tid; b < hi; b += 256) {
    for (int k = 0; k < 3; ++k) d[k] += dpart[4 * b + k];
    for (int k = 0; k < 4; ++k) c[k] += ipart[4 * b + k];
  }
  for (int k = 0; k < 3; ++k) sd[k][tid] = d[k];
  for (int k = 0; k < 4; ++k) si[k][tid] = c[k];
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half) {
      for (int k = 0; k < 3; ++k) sd[k][tid] += sd[k][tid + half];
      for (int k = 0; k < 4; ++k) si[k][tid] += si[k][tid + half];
    }
    __syncthreads();
  }
  if (tid < 4) {
    dout[4 * (int64_t)blockIdx.x + tid] = tid < 3 ? sd[tid][0] : 0.0;
    iout[4 * (int64_t)blockIdx.x + tid] = si[tid][0];
  }
}

// Fixed-order sums of the per-block partials into the result.  The ATM
// energy partials hold 3 u / nu per triplet (once per receiving molecule in
// the one-sided kernel, three times u once per triplet in the block kernel),
// so E3 = nu * sum / 3; W3 = 9 E3 (the ATM potential is homogeneous of
// degree -9 in the positions).  Integer slot 2 flags a force contribution
// beyond the fixed-point range.
__global__ __launch_bounds__(256) void k_onesided_final(const double* __restrict__ dpart,
                                                        const unsigned long long* __restrict__ ipart, int32_t nb,
                                                        double nu, int32_t nx, int32_t ny, int32_t nz,
                                                        atm3_result* __restrict__ res) {
  // fixed-order parallel sums: strided per thread, then a tree in LDS
  __shared__ double sd[3][256];
  __shared__ unsigned long long si[4][256];
  const int tid = threadIdx.x;
  double d[3] = {0.0, 0.0, 0.0};
  unsigned long long c[4] = {0, 0, 0, 0};
  for (int b = tid; b < nb; b += 256) {
    for (int k = 0; k < 3; ++k) d[k] += dpart[4 * (int64_t)b + k];
    for (int k = 0; k < 4; ++k) c[k] += ipart[4 * (int64_t)b + k];
  }
  for (int k = 0; k < 3; ++k) sd[k][tid] = d[k];
  for (int k = 0; k < 4; ++k) si[k][tid] = c[k];
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half) {
      for (int k = 0; k < 3; ++k) sd[k][tid] += sd[k][tid + half];
      for (int k = 0; k < 4; ++k) si[k][tid] += si[k][tid + half];
    }
    __syncthreads();
  }
  if (tid != 0) return;
  atm3_result r;
  r.e_lj = sd[0][0];
  r.w_lj = sd[1][0];
  r.e_atm = nu * sd[2][0] / 3.0;
  r.w_atm = 9.0 * r.e_atm;
  r.n_pairs = (int64_t)si[0][0];
  r.n_triplets = (int64_t)si[1][0];
  r.n_candidates = 0;  // from the cell populations afterwards
  r.ncell[0] = nx;
  r.ncell[1] = ny;
  r.ncell[2] = nz;
  r.status = si[3][0] ? ATM3_EOVERFLOW : (si[2][0] ? ATM3_ERANGE : ATM3_OK);
  *res = r;
}

}  // namespace

hipError_t launch_variant_counts(atm3_ctx* ctx, const Grid& g, const atm3_params& p, atm3_result* res_dev,
                                 bool triple) {
  const unsigned nb = blocks_for(g.ncells, 256);
  if (ensure(ctx, B_SRED, 8 * (size_t)nb + 64)) return hipErrorOutOfMemory;
  CandArgs a;
  a.start = (const int32_t*)ctx->buf[B_START];
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.ncells = g.ncells;
  a.variant = p.variant;
  a.part = (unsigned long long*)ctx->buf[B_SRED];
  hipLaunchKernelGGL(k_cand, dim3(nb), dim3(256), 0, ctx->stream, a);
  hipLaunchKernelGGL(k_cand_final, dim3(1), dim3(64), 0, ctx->stream, a.part, (int32_t)nb, p.variant,
                     triple ? 1 : 0, res_dev);
  return hipGetLastError();
}

namespace {

// One-sided kernel arguments for `terms`.
OneArgs one_args(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p, int terms,
                 float* forces, int* groups_out, bool* wv, bool* wj) {
  OneArgs a;
  // blocks per cell: about one group of OS_MOLS molecules each; for LJ alone
  // (little work per molecule) the staged neighbourhood is shared by the
  // whole cell, one block per cell once the grid fills the GPU
  const int64_t per_cell = (n + g.ncells - 1) / g.ncells;
  int64_t groups64 = std::min<int64_t>(64, std::max<int64_t>(1, (per_cell + OS_MOLS - 1) / OS_MOLS));
  if (!(terms & ATM3_TERM_ATM)) groups64 = std::min<int64_t>(groups64, (2048 + g.ncells - 1) / g.ncells);
  const int groups = (int)groups64;
  a.sorted = (const double4*)ctx->buf[B_SORTED];
  a.start = (const int32_t*)ctx->buf[B_START];
  a.pos = pos;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.variant = p.variant;
  a.terms = terms;
  a.groups = groups;
  double smin = g.side[0];
  *wv = *wj = false;
  for (int d = 0; d < 3; ++d) {
    a.side[d] = g.side[d];
    a.box[d] = g.box[d];
    a.boxf[d] = (float)g.box[d];
    a.invf[d] = (float)(1.0 / g.box[d]);
    smin = std::min(smin, g.side[d]);
    // molecule-partner vectors span under 2 cells, partner-partner under 4
    *wv = *wv || g.n[d] < 4;
    *wj = *wj || g.n[d] < 8;
  }
  a.rc2 = p.rc * p.rc;
  a.rc6 = (a.rc2 * a.rc2) * a.rc2;
  // FP32 pre-tests: a relative band of 1e-4 around each boundary, and every
  // side shorter than a quarter cell, go to the exact FP64 decision (the
  // FP32 squared sides err by less than 3e-5 relative outside that range)
  a.rc2hi = (float)(a.rc2 * (1.0 + 1e-4));
  a.lo6f = (float)(a.rc6 * (1.0 - 1e-4));
  a.hi6f = (float)(a.rc6 * (1.0 + 1e-4));
  a.small2 = (float)(0.0625 * smin * smin);
  a.sig2 = p.sigma * p.sigma;
  a.eps4 = 4.0 * p.eps;
  a.eps24 = 24.0 * p.eps;
  a.k3nu = (float)(3.0 * p.nu);
  a.k15nu = (float)(1.875 * p.nu);
  a.k075nu = (float)(0.75 * p.nu);
  a.forces = forces;
  a.fout = nullptr;
  a.tpart = nullptr;
  *groups_out = groups;
  return a;
}

template <bool TENSOR = false>
void launch_one(const OneArgs& a, unsigned nb, bool wv, bool wj, hipStream_t st) {
  if (wv)
    hipLaunchKernelGGL((k_onesided<true, true, TENSOR>), dim3(nb), dim3(64 * OS_WAVES), 0, st, a);
  else if (wj)
    hipLaunchKernelGGL((k_onesided<false, true, TENSOR>), dim3(nb), dim3(64 * OS_WAVES), 0, st, a);
  else
    hipLaunchKernelGGL((k_onesided<false, false, TENSOR>), dim3(nb), dim3(64 * OS_WAVES), 0, st, a);
}

// Block-kernel arguments for base-cell grids of `splits` blocks per cell;
// *wr: the grid needs minimum-image wraps inside a cell set (vectors span
// under 2 cells for 3c08, 3 for 3c18).
ProdArgs prod_args(const OneArgs& a, const Grid& g, int variant, int splits, unsigned long long* acc, bool* wr) {
  ProdArgs b;
  b.sorted = a.sorted;
  b.start = a.start;
  b.pos = a.pos;
  b.nx = g.n[0];
  b.ny = g.n[1];
  b.nz = g.n[2];
  b.splits = splits;
  *wr = false;
  for (int d = 0; d < 3; ++d) {
    b.side[d] = a.side[d];
    b.box[d] = a.box[d];
    b.boxf[d] = a.boxf[d];
    b.invf[d] = a.invf[d];
    *wr = *wr || g.n[d] < (variant == ATM3_VARIANT_3C08 ? 4 : 6);
  }
  b.rc6 = a.rc6;
  b.lo6f = a.lo6f;
  b.hi6f = a.hi6f;
  b.small2 = a.small2;
  b.k3nu = a.k3nu;
  b.k15nu = a.k15nu;
  b.k075nu = a.k075nu;
  b.acc = acc;
  b.pair = 0;
  b.rc2 = a.rc2;
  b.lo2f = (float)(a.rc2 * (1.0 - 1e-4));
  b.hi2f = (float)(a.rc2 * (1.0 + 1e-4));
  b.tpart = nullptr;
  const double t1 = a.rc2 * (1.0 + 1e-4) / 8.0;
  b.pf_inv_t1 = (float)(1.0 / t1);
  b.pf_lh = (float)std::log2(a.rc6 * (1.0 + 1e-3) / (t1 * t1));
  b.pdefer = nullptr;
  b.lj = 0;
  b.sig2 = a.sig2;
  b.eps4 = a.eps4;
  b.eps24 = a.eps24;
  return b;
}

template <bool TENSOR>
void launch_prod(const ProdArgs& b, int variant, bool wr, unsigned nb, hipStream_t st) {
  if (variant == ATM3_VARIANT_3C08) {
    if (wr) hipLaunchKernelGGL((k_prod_block<ATM3_VARIANT_3C08, true, TENSOR>), dim3(nb), dim3(64 * PB_WAVES), 0, st, b);
    else hipLaunchKernelGGL((k_prod_block<ATM3_VARIANT_3C08, false, TENSOR>), dim3(nb), dim3(64 * PB_WAVES), 0, st, b);
  } else {
    if (wr) hipLaunchKernelGGL((k_prod_block<ATM3_VARIANT_3C18, true, TENSOR>), dim3(nb), dim3(64 * PB_WAVES), 0, st, b);
    else hipLaunchKernelGGL((k_prod_block<ATM3_VARIANT_3C18, false, TENSOR>), dim3(nb), dim3(64 * PB_WAVES), 0, st, b);
  }
}

inline int prod_splits(const Grid& g) {
  // small grids: several blocks per base cell so that about 2048 run
  return (int)std::min<int64_t>(8, std::max<int64_t>(1, (2048 + g.ncells - 1) / g.ncells));
}

// Fixed-order sums of the virial-tensor partials: out[0..2] LJ, out[3..5]
// ATM (blocks nb1..nb), out[6] the status as a number.
__global__ __launch_bounds__(256) void k_tensor_final(const double* __restrict__ tpart,
                                                      const unsigned long long* __restrict__ ipart, int32_t nb1,
                                                      int32_t nb, double* __restrict__ out) {
  __shared__ double sd[6][256];
  __shared__ unsigned long long sf[2][256];
  const int tid = threadIdx.x;
  double d[6] = {0, 0, 0, 0, 0, 0};
  unsigned long long over = 0, rng = 0;
  for (int b = tid; b < nb; b += 256) {
    for (int k = 0; k < 3; ++k) d[(b < nb1 ? 0 : 3) + k] += tpart[3 * (int64_t)b + k];
    rng |= ipart[4 * (int64_t)b + 2];
    over |= ipart[4 * (int64_t)b + 3];
  }
  for (int k = 0; k < 6; ++k) sd[k][tid] = d[k];
  sf[0][tid] = over;
  sf[1][tid] = rng;
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half) {
      for (int k = 0; k < 6; ++k) sd[k][tid] += sd[k][tid + half];
      sf[0][tid] |= sf[0][tid + half];
      sf[1][tid] |= sf[1][tid + half];
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int k = 0; k < 6; ++k) out[k] = sd[k][0];
    out[6] = sf[0][0] ? (double)ATM3_EOVERFLOW : (sf[1][0] ? (double)ATM3_ERANGE : 0.0);
  }
}

}  // namespace

hipError_t launch_virial_diag(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p,
                              double* out_dev) {
  const bool lj = (p.terms & ATM3_TERM_LJ) != 0, atm = (p.terms & ATM3_TERM_ATM) != 0;
  const bool pair = p.truncation == ATM3_TRUNC_PAIR;
  // the pairwise cutoff includes the same triplets for every cell set
  const int variant = pair ? ATM3_VARIANT_3C08 : p.variant;
  int groups = 1;
  bool wv = false, wj = false;
  OneArgs a = one_args(ctx, pos, n, g, p, ATM3_TERM_LJ, nullptr, &groups, &wv, &wj);
  const int splits = prod_splits(g);
  const int64_t nb1_64 = lj ? g.ncells * groups : 0, nb2_64 = atm ? g.ncells * splits : 0;
  if (nb1_64 + nb2_64 > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  const unsigned nb1 = (unsigned)nb1_64, nb2 = (unsigned)nb2_64, nb = nb1 + nb2;
  if (ensure(ctx, B_SRED, 88 * (size_t)nb + 64)) return hipErrorOutOfMemory;
  double* dpart = (double*)ctx->buf[B_SRED];
  unsigned long long* ipart = (unsigned long long*)(dpart + 4 * (size_t)nb);
  double* tpart = (double*)(ipart + 4 * (size_t)nb);
  unsigned long long* acc = (unsigned long long*)ctx->buf[B_FPART];
  double* ljf = (double*)(acc + 3 * n);
  hipStream_t st = ctx->stream;
  if (nb1) {
    a.dpart = dpart;
    a.ipart = ipart;
    a.fout = ljf;
    a.tpart = tpart;
    launch_one<true>(a, nb1, wv, wj, st);
  }
  if (nb2) {
    hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(3 * n, 256)), dim3(256), 0, st, acc, 3 * n);
    bool wr = false;
    ProdArgs b = prod_args(a, g, variant, splits, acc, &wr);
    b.pair = pair ? 1 : 0;
    b.dpart = dpart + 4 * (size_t)nb1;
    b.ipart = ipart + 4 * (size_t)nb1;
    b.tpart = tpart + 3 * (size_t)nb1;
    launch_prod<true>(b, variant, wr, nb2, st);
  }
  hipLaunchKernelGGL(k_tensor_final, dim3(1), dim3(256), 0, st, (const double*)tpart,
                     (const unsigned long long*)ipart, (int32_t)nb1, (int32_t)nb, out_dev);
  return hipGetLastError();
}

hipError_t launch_onesided(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p,
                           float* forces, atm3_result* res_dev) {
  const bool lj = (p.terms & ATM3_TERM_LJ) != 0, atm = (p.terms & ATM3_TERM_ATM) != 0;
  // 3c01 (every molecule takes its own share) runs the one-sided kernel for
  // both terms; 3c08 and 3c18 run it for LJ only and the block
  // kernel for ATM
  const bool blockwise = p.variant != ATM3_VARIANT_3C01;
  // the shell-pruned tier takes every base cell first where the cell sets
  // need no minimum-image wrap, with the LJ pairs the sets own; k_prod_block
  // the cells it hands on
  bool wr_set = false;
  for (int d = 0; d < 3; ++d) wr_set = wr_set || g.n[d] < (p.variant == ATM3_VARIANT_3C08 ? 4 : 6);
  const bool fast = blockwise && atm && !wr_set;
  const int one_terms = fast ? 0 : (blockwise ? (p.terms & ATM3_TERM_LJ) : p.terms);
  int groups = 1;
  bool wv = false, wj = false;
  OneArgs a = one_args(ctx, pos, n, g, p, one_terms ? one_terms : ATM3_TERM_LJ, forces, &groups, &wv, &wj);
  const int64_t nb1_64 = one_terms ? g.ncells * groups : 0;
  const int splits = prod_splits(g);
  const int64_t nb2_64 = (blockwise && atm) ? g.ncells * splits : 0;
  const int64_t nbf_64 = fast ? g.ncells : 0;
  if (nb1_64 + nb2_64 + nbf_64 > (int64_t)INT32_MAX || 8 * ((g.ncells + 7) / 8) > (int64_t)INT32_MAX)
    return hipErrorInvalidValue;
  const unsigned nb1 = (unsigned)nb1_64, nbf = (unsigned)nbf_64, nb2 = (unsigned)nb2_64, nb = nb1 + nbf + nb2;
  if (nbf && ensure(ctx, B_PDEFER, 4 * (size_t)g.ncells)) return hipErrorOutOfMemory;
  // room for the per-block partials and, afterwards, the candidate partials
  // of launch_variant_counts (so that its ensure does not reallocate)
  const size_t need = 64 * (size_t)nb + 64 * 256 + 64, need_c = 8 * (size_t)blocks_for(g.ncells, 256) + 64;
  if (ensure(ctx, B_SRED, need > need_c ? need : need_c)) return hipErrorOutOfMemory;
  double* dpart = (double*)ctx->buf[B_SRED];
  unsigned long long* ipart = (unsigned long long*)(dpart + 4 * (size_t)nb);
  // B_FPART (24 doubles per molecule) holds the fixed-point ATM forces and
  // the FP64 LJ forces of the block path
  unsigned long long* acc = (unsigned long long*)ctx->buf[B_FPART];
  double* ljf = (double*)(acc + 3 * n);
  hipStream_t st = ctx->stream;
  hipError_t e = phase_begin(ctx, ATM3_PHASE_BLOCK);
  if (e != hipSuccess) return e;
  if (blockwise)
    hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(3 * n, 256)), dim3(256), 0, st, acc, 3 * n);
  if (nb1) {
    a.dpart = dpart;
    a.ipart = ipart;
    if (blockwise) a.fout = ljf;
    launch_one(a, nb1, wv, wj, st);
  }
  if (nb2) {
    bool wr = false;
    ProdArgs b = prod_args(a, g, p.variant, splits, acc, &wr);
    if (nbf) {
      b.pdefer = (int32_t*)ctx->buf[B_PDEFER];
      b.lj = lj ? 1 : 0;
      b.dpart = dpart + 4 * (size_t)nb1;
      b.ipart = ipart + 4 * (size_t)nb1;
      const unsigned grid = (unsigned)(8 * ((g.ncells + 7) / 8));
      // a grid whose mean 3c08 block holds more than 112 molecules (cutoffs
      // from about 2.8 at density 0.75) would hand on most of its blocks:
      // three mask words (192 molecules) and rounds of 256 rows instead
      if (p.variant == ATM3_VARIANT_3C08 && 8 * n > 112 * g.ncells)
        hipLaunchKernelGGL((k_prod_fast<ATM3_VARIANT_3C08, 3, 4096, 1536, 1>), dim3(grid), dim3(PF_WG), 0, st, b);
      else if (p.variant == ATM3_VARIANT_3C08)
        hipLaunchKernelGGL((k_prod_fast<ATM3_VARIANT_3C08, 2, 2048, 2048, 2>), dim3(grid), dim3(PF_WG), 0, st, b);
      else
        hipLaunchKernelGGL((k_prod_fast<ATM3_VARIANT_3C18, 3, 4096, 1536, 4>), dim3(grid), dim3(PF_WG), 0, st, b);
    }
    b.dpart = dpart + 4 * (size_t)(nb1 + nbf);
    b.ipart = ipart + 4 * (size_t)(nb1 + nbf);
    launch_prod<false>(b, p.variant, wr, nb2, st);
  }
  if (blockwise)
    hipLaunchKernelGGL(k_prod_forces, dim3(blocks_for(3 * n, 256)), dim3(256), 0, st,
                       (lj && nb1) ? (const double*)ljf : nullptr,
                       (const unsigned long long*)acc, 3 * n, forces);
  e = phase_end(ctx, ATM3_PHASE_BLOCK);
  if (e != hipSuccess) return e;
  // two stages: 256 blocks over the partials, then one over their sums
  const int32_t chunk = (int32_t)std::max<int64_t>(1, ((int64_t)nb + 255) / 256);
  const int32_t ng = (int32_t)(((int64_t)nb + chunk - 1) / chunk);
  double* dsum = (double*)(ipart + 4 * (size_t)nb);
  unsigned long long* isum = (unsigned long long*)(dsum + 4 * 256);
  if (ng > 0)
    hipLaunchKernelGGL(k_partials_sum, dim3(ng), dim3(256), 0, st, (const double*)dpart,
                       (const unsigned long long*)ipart, (int32_t)nb, chunk, dsum, isum);
  hipLaunchKernelGGL(k_onesided_final, dim3(1), dim3(256), 0, st, dsum, isum, ng, p.nu, g.n[0], g.n[1],
                     g.n[2], res_dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the candidates of the variant's cell sets, from the cell populations
  // (B_SRED is free again once k_onesided_final has run)
  return launch_variant_counts(ctx, g, p, res_dev, false);
}

}  // namespace atm3
