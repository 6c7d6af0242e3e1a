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

// Planar long-range correction of the LJ force (the slab runs of Sec. 5.2
// add one and cite it without stating it).  A sheet of areal density s_a at
// height offset xi pulls a molecule, through its molecules beyond rc, with
// F_z = 2 pi s_a xi phi(max(rc, |xi|)), phi the LJ potential; the sheets
// are the bins of the instantaneous z histogram, and every molecule of a bin
// takes the force at the bin's centre (bin pairs act with opposite forces:
// no net momentum).
constexpr int LRC_MAXBINS = 4096;

__global__ void k_zero_u32(uint32_t* p, int32_t m) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// z <- z - L_z floor(z / L_z), k = floor(z * (nbins / L_z)) clamped (FP64,
// no contraction: the bin is bit-exact).
__device__ __forceinline__ int zbin(double z, double lz, double inv, int nbins) {
#pragma clang fp contract(off)
  z = z - lz * floor(z / lz);
  const int k = (int)floor(z * inv);
  return k < 0 ? 0 : (k >= nbins ? nbins - 1 : k);
}

__global__ __launch_bounds__(256) void k_zhist(const double* __restrict__ pos, int64_t n, double lz, double inv,
                                               int32_t nbins, uint32_t* __restrict__ hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&hist[zbin(pos[3 * i + 2], lz, inv, nbins)], 1u);
}

struct LrcArgs {
  const double* pos;
  int64_t n;
  const uint32_t* hist;
  double* fbin;  // [nbins] force at each bin centre
  int32_t nbins;
  double lz, inv, dz, coef, rc, sigma, eps4;  // coef = 2 pi / (L_x L_y)
  float* forces;
  long long* hist_sum;
};

// Force at each bin centre (one thread per bin, fixed order over the bins);
// the histogram sums for profile sampling.
__global__ __launch_bounds__(256) void k_lrc_bins(LrcArgs a) {
  __shared__ double sh[LRC_MAXBINS];
  for (int k = threadIdx.x; k < a.nbins; k += blockDim.x) sh[k] = (double)a.hist[k];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.nbins) return;
  if (a.hist_sum) a.hist_sum[b] += (long long)a.hist[b];
  const double zb = (b + 0.5) * a.dz;
  double f = 0.0;
  for (int k = 0; k < a.nbins; ++k) {
    if (sh[k] == 0.0) continue;
    double xi = zb - (k + 0.5) * a.dz;
    xi -= a.lz * rint(xi / a.lz);
    const double r = fmax(a.rc, fabs(xi));
    const double s2 = (a.sigma / r) * (a.sigma / r), s6 = s2 * s2 * s2;
    f += sh[k] * xi * (a.eps4 * (s6 * s6 - s6));
  }
  a.fbin[b] = a.coef * f;
}

__global__ __launch_bounds__(256) void k_lrc_apply(LrcArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int b = zbin(a.pos[3 * i + 2], a.lz, a.inv, a.nbins);
  a.forces[3 * i + 2] = (float)((double)a.forces[3 * i + 2] + a.fbin[b]);
}

// Step counter of a graph-launched run: the result of every sample_every-th
// step goes to its row (the graph's kernels take fixed arguments, so the row
// is chosen on the device), and every step's status is folded into the
// status of row nsamp (the minimum: the most negative failure code wins).
__global__ void k_md_store(const uint64_t* __restrict__ slot, uint8_t* __restrict__ rows, int64_t stride,
                           int64_t* __restrict__ ctr, int64_t sample_every, int64_t nsamp) {
  __shared__ int64_t c;
  if (threadIdx.x == 0) {
    c = ++ctr[0];
    const int32_t st = ((const atm3_result*)slot)->status;
    atomicMin(&((atm3_result*)(rows + nsamp * stride))->status, st);
  }
  __syncthreads();
  if (c % sample_every != 0 || c / sample_every > nsamp) return;
  uint64_t* dst = (uint64_t*)(rows + (c / sample_every - 1) * stride);
  for (int k = threadIdx.x; k < (int)(sizeof(atm3_result) / 8); k += blockDim.x) dst[k] = slot[k];
}

// Folds one evaluation's status into the run-wide status word.
__global__ void k_md_fold(const atm3_result* __restrict__ slot, int32_t* __restrict__ status) {
  if (threadIdx.x == 0) atomicMin(status, slot->status);
}

__global__ void k_zero_i64(int64_t* p) {
  if (threadIdx.x == 0) p[0] = 0;
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
  double* part = (double*)ctx->buf[B_SRED];
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
  double* part = (double*)ctx->buf[B_SRED];
  hipLaunchKernelGGL(k_ke_part, dim3(np), dim3(256), 0, ctx->stream, vel, m, part + 1);
  hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(64), 0, ctx->stream, part + 1, np, part);
  hipLaunchKernelGGL(k_rescale, dim3(blocks_for(m, 256)), dim3(256), 0, ctx->stream, vel, m, (const double*)part,
                     0.5 * (double)dof * temperature);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "rescale launch");
  return ATM3_OK;
}

int atm3_md_slab_lrc(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3], int32_t nbins, double rc,
                     double eps, double sigma, float* forces, int64_t* hist_sum) {
  int r = md_check(ctx, pos, forces, n, 1.0);
  if (r) return r;
  if (!box) return fail(ctx, ATM3_EINVAL, "box is NULL");
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0) || !isfinite(box[d])) return fail(ctx, ATM3_EINVAL, "box lengths must be finite and > 0");
  if (nbins < 1 || nbins > LRC_MAXBINS) return fail(ctx, ATM3_EINVAL, "nbins must be in [1, 4096]");
  if (!(rc > 0.0) || !(2.0 * rc <= box[2])) return fail(ctx, ATM3_EINVAL, "rc must be > 0 and at most L_z / 2");
  if (!(eps > 0.0) || !(sigma > 0.0)) return fail(ctx, ATM3_EINVAL, "eps and sigma must be > 0");
  // histogram (uint32) and bin forces (FP64) in one scratch buffer
  if ((r = ensure(ctx, B_ZHIST, 12 * (size_t)nbins + 16))) return r;
  uint32_t* hist = (uint32_t*)ctx->buf[B_ZHIST];
  double* fbin = (double*)((char*)ctx->buf[B_ZHIST] + ((4 * (size_t)nbins + 15) & ~(size_t)15));
  const double inv = (double)nbins / box[2];
  hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nbins, 256)), dim3(256), 0, ctx->stream, hist, nbins);
  hipLaunchKernelGGL(k_zhist, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, pos, n, box[2], inv, nbins,
                     hist);
  LrcArgs a;
  a.pos = pos;
  a.n = n;
  a.hist = hist;
  a.fbin = fbin;
  a.nbins = nbins;
  a.lz = box[2];
  a.inv = inv;
  a.dz = box[2] / nbins;
  a.coef = 2.0 * M_PI / (box[0] * box[1]);
  a.rc = rc;
  a.sigma = sigma;
  a.eps4 = 4.0 * eps;
  a.forces = forces;
  a.hist_sum = (long long*)hist_sum;
  hipLaunchKernelGGL(k_lrc_bins, dim3(blocks_for(nbins, 256)), dim3(256), 0, ctx->stream, a);
  hipLaunchKernelGGL(k_lrc_apply, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "slab correction launch");
  return ATM3_OK;
}

int atm3_md_nvt_graph(atm3_ctx* ctx, double* pos, double* vel, int64_t n, const double box[3],
                      const atm3_params* params, int64_t steps, double dt, double temperature, int64_t dof,
                      int64_t sample_every, float* forces, void* rows, int64_t row_stride, int32_t lrc_bins,
                      int64_t* profile) {
  static_assert(sizeof(atm3_result) % 8 == 0, "result rows are copied in 8-byte words");
  int r = md_check(ctx, pos, vel, n, dt);
  if (r) return r;
  if (!params || !box || !forces || !rows) return fail(ctx, ATM3_EINVAL, "NULL argument");
  if (steps < 1 || sample_every < 1) return fail(ctx, ATM3_EINVAL, "steps and sample_every must be >= 1");
  if (row_stride < (int64_t)sizeof(atm3_result) || row_stride % 8)
    return fail(ctx, ATM3_EINVAL, "row_stride must be a multiple of 8 of at least sizeof(atm3_result)");
  if (params->flags & ATM3_FLAG_CHECK_FINITE) return fail(ctx, ATM3_EINVAL, "the finite check cannot be captured");
  if (ctx->profile) return fail(ctx, ATM3_EINVAL, "phase profiling cannot be captured");
  if (!(temperature > 0.0) || !isfinite(temperature)) return fail(ctx, ATM3_EINVAL, "temperature must be > 0");
  if (dof < 1 || dof > 3 * n) return fail(ctx, ATM3_EINVAL, "dof must be in [1, 3n]");
  if ((r = ensure(ctx, B_MDSLOT, sizeof(atm3_result) + 64))) return r;
  atm3_result* slot = (atm3_result*)ctx->buf[B_MDSLOT];
  int64_t* ctr = (int64_t*)((char*)ctx->buf[B_MDSLOT] + ((sizeof(atm3_result) + 15) & ~(size_t)15));
  // every scratch buffer a step uses is sized before the capture (no
  // allocation or synchronisation may happen inside it): the initial forces,
  // and the kinetic-energy partials of the thermostat
  if ((r = atm3_compute_forces_async(ctx, pos, n, box, params, forces, slot))) return r;
  if (lrc_bins && (r = atm3_md_slab_lrc(ctx, pos, n, box, lrc_bins, params->rc, params->eps, params->sigma,
                                         forces, nullptr)))
    return r;
  const int np = (int)((3 * n + KE_CHUNK - 1) / KE_CHUNK);
  if ((r = ensure(ctx, B_SRED, 8 * (size_t)np + 64))) return r;
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, ctx->stream, ctr);
  hipLaunchKernelGGL(k_md_fold, dim3(1), dim3(64), 0, ctx->stream, slot,
                     &((atm3_result*)((uint8_t*)rows + (steps / sample_every) * row_stride))->status);

  hipStream_t user = ctx->stream, s = nullptr;
  hipEvent_t e0 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&e0, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(e0, user);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, e0, 0);
  if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    ctx->stream = s;
    const int64_t nsamp = steps / sample_every;
    r = atm3_md_kick_drift(ctx, pos, vel, forces, n, dt);
    if (!r) r = atm3_compute_forces_async(ctx, pos, n, box, params, forces, slot);
    if (!r && lrc_bins)
      r = atm3_md_slab_lrc(ctx, pos, n, box, lrc_bins, params->rc, params->eps, params->sigma, forces, profile);
    if (!r) r = atm3_md_kick(ctx, vel, forces, n, dt);
    if (!r) r = atm3_md_rescale(ctx, vel, n, temperature, dof);
    if (!r) {
      hipLaunchKernelGGL(k_md_store, dim3(1), dim3(64), 0, s, (const uint64_t*)slot, (uint8_t*)rows, row_stride, ctr,
                         sample_every, nsamp);
      e = hipGetLastError();
    }
    ctx->stream = user;
    hipError_t ec = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = ec;
  }
  if (!r && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  for (int64_t k = 0; !r && e == hipSuccess && k < steps; ++k) e = hipGraphLaunch(exec, s);
  if (s) {
    hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (e0) (void)hipEventDestroy(e0);
  if (s) (void)hipStreamDestroy(s);
  ctx->stream = user;
  if (r) return r;
  if (e != hipSuccess) return hip_fail(ctx, e, "graph-launched MD");
  return ATM3_OK;
}

}  // extern "C"
