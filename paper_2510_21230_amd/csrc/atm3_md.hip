// Velocity Verlet (NVE) on FP64 positions and velocities with FP32 forces,
// unit mass, reduced Lennard-Jones units (the MD runs of the paper's
// validation, Sec. 5): half kick + drift, then after the force evaluation the
// second half kick; kinetic energy by a fixed-order FP64 reduction; an
// isokinetic velocity rescaling for constant-temperature runs (Sec. 5.1 runs
// NVT without naming its thermostat).
#include <math.h>
#include <string.h>

#include "atm3_internal.h"

namespace atm3 {
namespace {

__global__ __launch_bounds__(256) void k_kick_drift(double* __restrict__ x, double* __restrict__ v,
                                                    const float* __restrict__ f, int64_t m, double hdt, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double vi = v[i] + hdt * (double)f[i];
  v[i] = vi;
  x[i] = x[i] + dt * vi;
}

__global__ __launch_bounds__(256) void k_kick(double* __restrict__ v, const float* __restrict__ f, int64_t m,
                                              double hdt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  v[i] = v[i] + hdt * (double)f[i];
}

constexpr int KE_CHUNK = 4096;

__global__ __launch_bounds__(256) void k_ke_part(const double* __restrict__ v, int64_t m, double* __restrict__ part) {
  __shared__ double ws[4];
  const int64_t b0 = (int64_t)blockIdx.x * KE_CHUNK;
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b0 + KE_CHUNK && i < m; i += 256) s += v[i] * v[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

__global__ void k_ke_final(const double* __restrict__ part, int32_t np, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < np; ++b) s += part[b];
  out[0] = 0.5 * s;
}

// v *= sqrt(ke_target / ke), ke from k_ke_final (left unchanged when ke is 0).
__global__ __launch_bounds__(256) void k_rescale(double* __restrict__ v, int64_t m, const double* __restrict__ ke,
                                                 double ke_target) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double k = ke[0];
  if (k > 0.0) v[i] = v[i] * sqrt(ke_target / k);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int md_check(atm3_ctx* ctx, const void* a, const void* b, int64_t n, double dt) {
  if (!ctx) return ATM3_EINVAL;
  ctx->err.clear();
  if (!a || !b) return fail(ctx, ATM3_EINVAL, "NULL device pointer");
  if (n < 1 || n > ((int64_t)1 << 40)) return fail(ctx, ATM3_EINVAL, "n out of range");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(ctx, ATM3_EINVAL, "dt must be finite and > 0");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return ATM3_OK;
}

}  // namespace
}  // namespace atm3

using namespace atm3;

extern "C" {

int atm3_md_kick_drift(atm3_ctx* ctx, double* pos, double* vel, const float* forces, int64_t n, double dt) {
  int r = md_check(ctx, pos, vel, n, dt);
  if (r) return r;
  if (!forces) return fail(ctx, ATM3_EINVAL, "forces is NULL");
  const int64_t m = 3 * n;
  hipLaunchKernelGGL(k_kick_drift, dim3(blocks_for(m, 256)), dim3(256), 0, ctx->stream, pos, vel, forces, m,
                     0.5 * dt, dt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "kick-drift launch");
  return ATM3_OK;
}

int atm3_md_kick(atm3_ctx* ctx, double* vel, const float* forces, int64_t n, double dt) {
  int r = md_check(ctx, vel, forces, n, dt);
  if (r) return r;
  const int64_t m = 3 * n;
  hipLaunchKernelGGL(k_kick, dim3(blocks_for(m, 256)), dim3(256), 0, ctx->stream, vel, forces, m, 0.5 * dt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "kick launch");
  return ATM3_OK;
}

int atm3_md_kinetic(atm3_ctx* ctx, const double* vel, int64_t n, double* ke_out) {
  int r = md_check(ctx, vel, ke_out, n, 1.0);
  if (r) return r;
  const int64_t m = 3 * n;
  const int np = (int)((m + KE_CHUNK - 1) / KE_CHUNK);
  if ((r = ensure(ctx, B_SRED, 8 * (size_t)np + 64))) return r;
  double* part = (double*)ctx->s.p[B_SRED];
  hipLaunchKernelGGL(k_ke_part, dim3(np), dim3(256), 0, ctx->stream, vel, m, part + 1);
  hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(64), 0, ctx->stream, part + 1, np, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->hres, part, 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kinetic energy");
  memcpy(ke_out, ctx->hres, 8);
  return ATM3_OK;
}

int atm3_md_rescale(atm3_ctx* ctx, double* vel, int64_t n, double temperature, int64_t dof) {
  int r = md_check(ctx, vel, vel, n, 1.0);
  if (r) return r;
  if (!(temperature > 0.0) || !isfinite(temperature)) return fail(ctx, ATM3_EINVAL, "temperature must be > 0");
  if (dof < 1 || dof > 3 * n) return fail(ctx, ATM3_EINVAL, "dof must be in [1, 3n]");
  const int64_t m = 3 * n;
  const int np = (int)((m + KE_CHUNK - 1) / KE_CHUNK);
  if ((r = ensure(ctx, B_SRED, 8 * (size_t)np + 64))) return r;
  double* part = (double*)ctx->s.p[B_SRED];
  hipLaunchKernelGGL(k_ke_part, dim3(np), dim3(256), 0, ctx->stream, vel, m, part + 1);
  hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(64), 0, ctx->stream, part + 1, np, part);
  hipLaunchKernelGGL(k_rescale, dim3(blocks_for(m, 256)), dim3(256), 0, ctx->stream, vel, m, (const double*)part,
                     0.5 * (double)dof * temperature);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "rescale launch");
  return ATM3_OK;
}

}  // extern "C"
