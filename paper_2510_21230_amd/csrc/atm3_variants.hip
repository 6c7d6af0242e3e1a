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
// filter.  k_onesided evaluates, one wave per molecule m, every pair (j, k)
// of candidates from the cells around m (1 cell for 3c08 and 3c01, 2 for
// 3c18): the visited-set test on the cell offsets, the truncation test on
// the exact FP64 minimum-image squared sides (sorted, multiplied left to
// right, strict), and the ATM force on m (FP32 per triplet, FP64 sums).
// Energies and virials are credited a third per receiving molecule; counts
// once per triplet (3c01: once per receiving molecule).
#include <math.h>

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
    if (a.variant == ATM3_VARIANT_3C01) {
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

__global__ void k_cand_final(const unsigned long long* __restrict__ part, int32_t np, int32_t variant,
                             atm3_result* __restrict__ res) {
  if (threadIdx.x != 0) return;
  unsigned long long s = 0;
  for (int b = 0; b < np; ++b) s += part[b];
  res->n_candidates = (int64_t)s;
  if (variant == ATM3_VARIANT_3C01) res->n_triplets *= 3;
}

// ---------------------------------------------------------------------------
// one-sided evaluation under the product cutoff
// ---------------------------------------------------------------------------
constexpr int CAND_CAP = 2048;  // candidates per molecule (LDS, per wave)
constexpr int OS_WAVES = 2;

struct OneArgs {
  const double4* sorted;
  const int32_t* start;
  const int32_t* cell_of;
  const double* pos;
  int32_t n, nx, ny, nz, reach, variant, terms;
  double side[3], box[3];
  double rc2, rc6, sig2, eps4, eps24, nu;
  float k3nu, k15nu, k075nu;
  float* forces;
  double* dpart;              // per block: e_lj, w_lj, e_atm, w_atm
  unsigned long long* ipart;  // per block: n_pairs, n_triplets, n_candidates, overflow
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

__device__ __forceinline__ bool lex_less(const Off& p, const Off& q) {
  if (p.z != q.z) return p.z < q.z;
  if (p.y != q.y) return p.y < q.y;
  return p.x < q.x;
}

__device__ __forceinline__ Off rel(const Off& a, const Off& b, int nx, int ny, int nz) {
  return Off{wrap_off(a.x - b.x, nx), wrap_off(a.y - b.y, ny), wrap_off(a.z - b.z, nz)};
}

__device__ __forceinline__ bool adjacent(const Off& a, const Off& b, int nx, int ny, int nz) {
  const Off r = rel(b, a, nx, ny, nz);
  return r.x >= -1 && r.x <= 1 && r.y >= -1 && r.y <= 1 && r.z >= -1 && r.z <= 1;
}

// Visited test of the triplet labelled t0 < t1 < t2 (by input index) with
// cell offsets o0, o1, o2 (relative to any common cell); for 3c01 returns the
// receiving mask (bit q: molecule t_q takes its share), else 7 or 0.
__device__ int visited_mask(int variant, const Off& o0, const Off& o1, const Off& o2, int nx, int ny, int nz) {
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
  const Off* o[3] = {&z0, &r1, &r2};
  int m = 0;
  if (lex_less(r1, *o[m])) m = 1;
  if (lex_less(r2, *o[m])) m = 2;
  for (int t = 0; t < 3; ++t) {
    if (t == m) continue;
    const int dx = o[t]->x - o[m]->x, dy = o[t]->y - o[m]->y, dz = o[t]->z - o[m]->z;
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return 0;
  }
  return 7;
}

struct OneLds {
  int32_t orig[OS_WAVES][CAND_CAP];
  int8_t off[OS_WAVES][CAND_CAP][4];
  float4 v[OS_WAVES][CAND_CAP];      // r_j - r_m (FP32), .w unused
  double x[OS_WAVES][CAND_CAP];      // exact squared distance to m
  double red[OS_WAVES][4];
  unsigned long long redi[OS_WAVES][4];
};

__global__ __launch_bounds__(64 * OS_WAVES) void k_onesided(OneArgs a) {
  __shared__ OneLds L;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double e_lj = 0.0, w_lj = 0.0, e3 = 0.0;
  unsigned long long npair = 0, ntrip = 0, ncand = 0, over = 0;
  const int s = blockIdx.x * OS_WAVES + w;
  if (s < a.n) {
    const double4 me = a.sorted[s];
    const int om = (int)me.w;
    const int c = a.cell_of[om];
    const int cx = c % a.nx, cy = (c / a.nx) % a.ny, cz = c / (a.nx * a.ny);
    // candidates: molecules of the cells within `reach` of m's cell
    int nc = 0;
    const int R = a.reach, span = 2 * R + 1;
    for (int q = 0; q < span * span * span; ++q) {
      const int dx = q % span - R, dy = (q / span) % span - R, dz = q / (span * span) - R;
      const int ux = wrapc(cx + dx, a.nx), uy = wrapc(cy + dy, a.ny), uz = wrapc(cz + dz, a.nz);
      const int cc = (uz * a.ny + uy) * a.nx + ux;
      const int t0 = a.start[cc], t1 = a.start[cc + 1];
      for (int b = t0; b < t1; b += 64) {
        const int t = b + lane;
        const bool ok = t < t1 && t != s;
        const unsigned long long bits = __ballot(ok);
        const int slot = nc + __popcll(bits & ((1ull << lane) - 1ull));
        if (ok && slot < CAND_CAP) {
          const double4 o = a.sorted[t];
          const int oj = (int)o.w;
          L.orig[w][slot] = oj;
          L.off[w][slot][0] = (int8_t)dx;
          L.off[w][slot][1] = (int8_t)dy;
          L.off[w][slot][2] = (int8_t)dz;
          // r_j - r_m = loc_j - loc_m + offset of j's cell
          const double ex = (o.x - me.x) + dx * a.side[0], ey = (o.y - me.y) + dy * a.side[1],
                       ez = (o.z - me.z) + dz * a.side[2];
          L.v[w][slot] = make_float4((float)ex, (float)ey, (float)ez, 0.f);
          L.x[w][slot] = exact_r2(a.pos, om, oj, a.box[0], a.box[1], a.box[2]);
        }
        nc += __popcll(bits);
      }
    }
    if (nc > CAND_CAP) {
      over = 1;
      nc = CAND_CAP;
    }
    __builtin_amdgcn_wave_barrier();
    double fx = 0.0, fy = 0.0, fz = 0.0;
    // Lennard-Jones pairs containing m (FP64)
    if (a.terms & ATM3_TERM_LJ) {
      for (int q = lane; q < nc; q += 64) {
        const double x = L.x[w][q];
        if (!(x < a.rc2)) continue;
        const float4 vj = L.v[w][q];
        const double s2 = a.sig2 / x, s6 = s2 * s2 * s2, s12 = s6 * s6;
        const double f = a.eps24 * (2.0 * s12 - s6) / x;  // F_m = f (r_m - r_j)
        fx -= f * (double)vj.x;
        fy -= f * (double)vj.y;
        fz -= f * (double)vj.z;
        e_lj += 0.5 * a.eps4 * (s12 - s6);
        w_lj += 0.5 * f * x;
        npair += (om < L.orig[w][q]) ? 1 : 0;
      }
    }
    // ATM triplets containing m
    if (a.terms & ATM3_TERM_ATM) {
      const Off om_off{0, 0, 0};
      const float4 pm = make_float4(0.f, 0.f, 0.f, 0.f);
      const long long T = (long long)nc * (nc - 1) / 2;
      for (long long q = lane; q < T; q += 64) {
        int xa = (int)((2.0 * nc - 1.0 - sqrt((2.0 * nc - 1.0) * (2.0 * nc - 1.0) - 8.0 * (double)q)) * 0.5);
        if (xa < 0) xa = 0;
        while (xa > 0 && (long long)xa * (2 * nc - xa - 1) / 2 > q) --xa;
        while ((long long)(xa + 1) * (2 * nc - xa - 2) / 2 <= q) ++xa;
        const int xb = (int)(q - (long long)xa * (2 * nc - xa - 1) / 2) + xa + 1;
        const int oj = L.orig[w][xa], ok = L.orig[w][xb];
        const Off fj{L.off[w][xa][0], L.off[w][xa][1], L.off[w][xa][2]};
        const Off fk{L.off[w][xb][0], L.off[w][xb][1], L.off[w][xb][2]};
        // label by input index: t0 < t1 < t2
        int id[3] = {om, oj, ok};
        Off of[3] = {om_off, fj, fk};
        int me_pos = 0;
        if (id[1] < id[0]) { int ti = id[0]; id[0] = id[1]; id[1] = ti; Off to = of[0]; of[0] = of[1]; of[1] = to; }
        if (id[2] < id[1]) { int ti = id[1]; id[1] = id[2]; id[2] = ti; Off to = of[1]; of[1] = of[2]; of[2] = to; }
        if (id[1] < id[0]) { int ti = id[0]; id[0] = id[1]; id[1] = ti; Off to = of[0]; of[0] = of[1]; of[1] = to; }
        me_pos = (id[0] == om) ? 0 : (id[1] == om ? 1 : 2);
        const int vm = visited_mask(a.variant, of[0], of[1], of[2], a.nx, a.ny, a.nz);
        const bool mine = (vm >> me_pos) & 1;
        if (a.variant == ATM3_VARIANT_3C01) ncand += mine ? 1 : 0;
        else ncand += (vm && me_pos == 0) ? 1 : 0;
        if (!mine) continue;
        const double z = exact_r2(a.pos, oj, ok, a.box[0], a.box[1], a.box[2]);
        if (!product_ok(L.x[w][xa], L.x[w][xb], z, a.rc6)) continue;
        const Trip r = atm_triplet(pm, L.v[w][xa], L.v[w][xb], a.k3nu, a.k15nu, a.k075nu);
        fx += (double)r.fix;
        fy += (double)r.fiy;
        fz += (double)r.fiz;
        e3 += (double)r.eu;
        if (a.variant == ATM3_VARIANT_3C01 || me_pos == 0) ++ntrip;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      fx += __shfl_xor(fx, off);
      fy += __shfl_xor(fy, off);
      fz += __shfl_xor(fz, off);
    }
    if (lane == 0) {
      a.forces[3 * (int64_t)om + 0] = (float)fx;
      a.forces[3 * (int64_t)om + 1] = (float)fy;
      a.forces[3 * (int64_t)om + 2] = (float)fz;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    e_lj += __shfl_xor(e_lj, off);
    w_lj += __shfl_xor(w_lj, off);
    e3 += __shfl_xor(e3, off);
    npair += __shfl_xor(npair, off);
    ntrip += __shfl_xor(ntrip, off);
    ncand += __shfl_xor(ncand, off);
  }
  if (lane == 0) {
    L.red[w][0] = e_lj;
    L.red[w][1] = w_lj;
    L.red[w][2] = e3;
    L.redi[w][0] = npair;
    L.redi[w][1] = ntrip;
    L.redi[w][2] = ncand;
    L.redi[w][3] = over;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      double sum = 0.0;
      for (int q = 0; q < OS_WAVES; ++q) sum += L.red[q][k];
      a.dpart[4 * (int64_t)blockIdx.x + k] = sum;
    }
    for (int k = 0; k < 4; ++k) {
      unsigned long long sum = 0;
      for (int q = 0; q < OS_WAVES; ++q) sum += L.redi[q][k];
      a.ipart[4 * (int64_t)blockIdx.x + k] = sum;
    }
  }
}

// Fixed-order sums of the per-block partials into the result.  The ATM
// energy collected per molecule is the sum over triplets of u / nu counted
// once per receiving molecule, so E3 = nu * sum / 3; W3 = 9 E3 (the ATM
// potential is homogeneous of degree -9 in the positions).
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
  r.n_candidates = (int64_t)si[2][0];
  r.ncell[0] = nx;
  r.ncell[1] = ny;
  r.ncell[2] = nz;
  r.status = si[3][0] ? ATM3_EOVERFLOW : ATM3_OK;
  *res = r;
}

}  // namespace

hipError_t launch_variant_counts(atm3_ctx* ctx, const Grid& g, const atm3_params& p, atm3_result* res_dev) {
  const unsigned nb = blocks_for(g.ncells, 256);
  if (ensure(ctx, B_SRED, 8 * (size_t)nb + 64)) return hipErrorOutOfMemory;
  CandArgs a;
  a.start = (const int32_t*)ctx->s.p[B_START];
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.ncells = g.ncells;
  a.variant = p.variant;
  a.part = (unsigned long long*)ctx->s.p[B_SRED];
  hipLaunchKernelGGL(k_cand, dim3(nb), dim3(256), 0, ctx->stream, a);
  hipLaunchKernelGGL(k_cand_final, dim3(1), dim3(64), 0, ctx->stream, a.part, (int32_t)nb, p.variant, res_dev);
  return hipGetLastError();
}

hipError_t launch_onesided(atm3_ctx* ctx, const double* pos, int64_t n, const Grid& g, const atm3_params& p,
                           float* forces, atm3_result* res_dev) {
  const unsigned nb = blocks_for(n, OS_WAVES);
  if (ensure(ctx, B_SRED, 64 * (size_t)nb + 64)) return hipErrorOutOfMemory;
  OneArgs a;
  a.sorted = (const double4*)ctx->s.p[B_SORTED];
  a.start = (const int32_t*)ctx->s.p[B_START];
  a.cell_of = (const int32_t*)ctx->s.p[B_CELL_OF];
  a.pos = pos;
  a.n = (int32_t)n;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.reach = (p.variant == ATM3_VARIANT_3C18) ? 2 : 1;
  a.variant = p.variant;
  a.terms = p.terms;
  for (int d = 0; d < 3; ++d) {
    a.side[d] = g.side[d];
    a.box[d] = g.box[d];
  }
  a.rc2 = p.rc * p.rc;
  a.rc6 = (a.rc2 * a.rc2) * a.rc2;
  a.sig2 = p.sigma * p.sigma;
  a.eps4 = 4.0 * p.eps;
  a.eps24 = 24.0 * p.eps;
  a.nu = p.nu;
  a.k3nu = (float)(3.0 * p.nu);
  a.k15nu = (float)(1.875 * p.nu);
  a.k075nu = (float)(0.75 * p.nu);
  a.forces = forces;
  a.dpart = (double*)ctx->s.p[B_SRED];
  a.ipart = (unsigned long long*)((double*)ctx->s.p[B_SRED] + 4 * (size_t)nb);
  hipError_t e = phase_begin(ctx, ATM3_PHASE_BLOCK);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_onesided, dim3(nb), dim3(64 * OS_WAVES), 0, ctx->stream, a);
  e = phase_end(ctx, ATM3_PHASE_BLOCK);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_onesided_final, dim3(1), dim3(256), 0, ctx->stream, a.dpart, a.ipart, (int32_t)nb, p.nu, g.n[0],
                     g.n[1], g.n[2], res_dev);
  return hipGetLastError();
}

}  // namespace atm3
