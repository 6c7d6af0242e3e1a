// Device math shared by the exact block kernel and the surrogate's exact
// fallback: the ATM triplet term, the Lennard-Jones pair term and the exact
// minimum-image distance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace atm3 {

// Exact squared minimum-image distance between input molecules a and b: the
// oracle's expression, FP64, no contraction, evaluated left to right.
static __device__ __noinline__ double exact_r2(const double* __restrict__ pos, int a, int b, double Lx, double Ly,
                                        double Lz) {
#pragma clang fp contract(off)
  double d0 = pos[3 * (int64_t)a + 0] - pos[3 * (int64_t)b + 0];
  d0 = d0 - Lx * rint(d0 / Lx);
  double d1 = pos[3 * (int64_t)a + 1] - pos[3 * (int64_t)b + 1];
  d1 = d1 - Ly * rint(d1 / Ly);
  double d2 = pos[3 * (int64_t)a + 2] - pos[3 * (int64_t)b + 2];
  d2 = d2 - Lz * rint(d2 / Lz);
  double s = d0 * d0;
  s = s + d1 * d1;
  s = s + d2 * d2;
  return s;
}

struct Trip {
  float eu, fix, fiy, fiz, fjx, fjy, fjz;
};

static __device__ __forceinline__ Trip atm_triplet(const float4 pi, const float4 pj, const float4 pk, float k3nu,
                                            float k15nu, float k075nu) {
  const float ijx = pi.x - pj.x, ijy = pi.y - pj.y, ijz = pi.z - pj.z;
  const float ikx = pi.x - pk.x, iky = pi.y - pk.y, ikz = pi.z - pk.z;
  const float jkx = pj.x - pk.x, jky = pj.y - pk.y, jkz = pj.z - pk.z;
  const float x = ijx * ijx + ijy * ijy + ijz * ijz;
  const float y = ikx * ikx + iky * iky + ikz * ikz;
  const float z = jkx * jkx + jky * jky + jkz * jkz;
  // eq. (atm) in squared sides: u = nu [Q^-3/2 + 3/8 P Q^-5/2],
  // Q = xyz, P = (y+z-x)(x+z-y)(x+y-z) = A B C.
  const float s = x + y + z;
  const float A = fmaf(-2.f, x, s), B = fmaf(-2.f, y, s), C = fmaf(-2.f, z, s);
  const float AB = A * B, AC = A * C, BC = B * C;
  const float P = AB * C;
  const float S = AB + AC + BC;
  const float xy = x * y, yz = y * z, xz = x * z;
  const float Q = xy * z;
  const float t1 = __builtin_amdgcn_rsqf(Q);
  const float t2 = t1 * t1, t3 = t2 * t1, t5 = t3 * t2;
  Trip r;
  r.eu = fmaf(0.375f * P, t5, t3);
  // c_x = -2 du/dx = nu [3 t3 / x + 15/8 P t5 / x - 3/4 t5 dP/dx],
  // dP/dx = S - 2BC (cyclic for y, z); 1/x = yz / Q.
  const float G = fmaf(k15nu * P, t5, k3nu * t3);
  const float H = k075nu * t5;
  const float cx = fmaf(G, yz * t2, -H * fmaf(-2.f, BC, S));
  const float cy = fmaf(G, xz * t2, -H * fmaf(-2.f, AC, S));
  const float cz = fmaf(G, xy * t2, -H * fmaf(-2.f, AB, S));
  // eq. (forcepairs): F_i = F_i(j)k + F_i(k)j, F_j = -F_i(j)k + F_j(k)i,
  // with F_i(j)k = c_x r_ij, F_i(k)j = c_y r_ik, F_j(k)i = c_z r_jk.
  r.fix = fmaf(cx, ijx, cy * ikx);
  r.fiy = fmaf(cx, ijy, cy * iky);
  r.fiz = fmaf(cx, ijz, cy * ikz);
  r.fjx = fmaf(cz, jkx, -cx * ijx);
  r.fjy = fmaf(cz, jky, -cx * ijy);
  r.fjz = fmaf(cz, jkz, -cx * ijz);
  return r;
}

// LJ pair term in FP64 on block-frame displacement e = r_i - r_j; returns
// the force factor f (F_i = f e) and adds s12 - s6 and 2 s12 - s6 to the
// energy and virial accumulators (scaled by 4 eps and 24 eps at the end).
static __device__ __forceinline__ double lj_pair(double ex, double ey, double ez, double sig2, double eps24, double* e_lj,
                                          double* w_lj) {
  // 4 eps [(s/r)^12 - (s/r)^6]; F_i = 24 eps [2 (s/r)^12 - (s/r)^6] r_ij / r^2
  const double r2 = ex * ex + ey * ey + ez * ez;
  double ir2 = __builtin_amdgcn_rcp(r2);  // refined by two Newton steps
  ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
  ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
  const double s2 = sig2 * ir2;
  const double s6 = s2 * s2 * s2;
  const double s12 = s6 * s6;
  *e_lj += s12 - s6;
  const double g = 2.0 * s12 - s6;
  *w_lj += g;
  return eps24 * g * ir2;
}

}  // namespace atm3
