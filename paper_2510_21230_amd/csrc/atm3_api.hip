// C ABI of libatm3.so: context, scratch ownership, argument checks, launches.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "atm3_internal.h"

namespace atm3 {

int fail(atm3_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(atm3_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? ATM3_ENOMEM : ATM3_EDEVICE, m);
}

int ensure(atm3_ctx* ctx, Buf b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->fixed) {  // carve of the fixed array: never allocate
    if (ctx->bufcap[b] >= bytes) return ATM3_OK;
    return fail(ctx, ATM3_EINVAL, "evaluation exceeds the fixed scratch array of the no-allocation entry point");
  }
  if (ctx->s.cap[b] >= bytes) return ATM3_OK;
  if (ctx->s.p[b]) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    (void)hipFree(ctx->s.p[b]);
    ctx->s.p[b] = nullptr;
    ctx->s.cap[b] = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom for slightly larger inputs
  hipError_t e = hipMalloc(&ctx->s.p[b], want);
  if (e != hipSuccess) {
    ctx->s.p[b] = nullptr;
    return hip_fail(ctx, e, "hipMalloc (scratch)");
  }
  ctx->s.cap[b] = want;
  return ATM3_OK;
}

void plan_pair_path(int64_t n, const Grid& g, size_t bytes[B_NBUF]) {
  for (int b = 0; b < B_NBUF; ++b) bytes[b] = 0;
  const size_t N = (size_t)n, C = (size_t)g.ncells;
  bytes[B_CELL_OF] = 4 * N;
  bytes[B_RANK] = 4 * N;
  bytes[B_COUNT] = 4 * C;
  bytes[B_START] = 4 * (C + 1);
  bytes[B_PERM] = 4 * N;
  bytes[B_SORTED] = 32 * N;
  bytes[B_FPART] = 8 * 24 * N;
  bytes[B_BLKD] = 8 * 3 * C;
  bytes[B_BLKI] = 4 * 2 * C;
  bytes[B_DEFER] = 4 * (2 * C + 3);
  bytes[B_RED] = reduce_scratch_bytes();
  bytes[B_TILE] = 4 * (C / 1024 + 2);
  bytes[B_FMASK] = 4 * 14 * N;
  bytes[B_FMOK] = 4 * C;
  bytes[B_SRED] = 8 * ((C + 255) / 256) + 64;  // candidate counts of 3c18 / 3c01
}

static hipError_t phase_event(atm3_ctx* ctx, int phase, int which) {
  if (!ctx->profile) return hipSuccess;
  PhaseTimer& t = ctx->timer[phase];
  const size_t k = 2 * t.used + (size_t)which;
  while (t.ev.size() <= k) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    t.ev.push_back(e);
  }
  hipError_t err = hipEventRecord(t.ev[k], ctx->stream);
  if (which == 1) ++t.used;
  return err;
}

hipError_t phase_begin(atm3_ctx* ctx, int phase) { return phase_event(ctx, phase, 0); }
hipError_t phase_end(atm3_ctx* ctx, int phase) { return phase_event(ctx, phase, 1); }

bool make_grid(const double box[3], double rc, Grid* g) {
  int64_t total = 1;
  for (int d = 0; d < 3; ++d) {
    double q = floor(box[d] / rc);
    if (!(q >= 1.0) || q > 1.0e6) return false;
    g->n[d] = (int32_t)q;
    g->box[d] = box[d];
    g->inv[d] = (double)g->n[d] / box[d];
    g->side[d] = box[d] / (double)g->n[d];
    total *= g->n[d];
  }
  if (total > (int64_t)1 << 30) return false;
  g->ncells = total;
  return true;
}

}  // namespace atm3

using namespace atm3;

namespace {

int set_device(atm3_ctx* ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return ATM3_OK;
}

int check_box(atm3_ctx* ctx, const double* box, double rc) {
  if (!box) return fail(ctx, ATM3_EINVAL, "box is NULL");
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0) || !isfinite(box[d])) return fail(ctx, ATM3_EINVAL, "box lengths must be finite and > 0");
  if (!(rc > 0.0) || !isfinite(rc)) return fail(ctx, ATM3_EINVAL, "rc must be finite and > 0");
  return ATM3_OK;
}

// Argument checks and the cell grid, without touching device memory.
int validate(atm3_ctx* ctx, const double* pos, int64_t n, const double* box, const atm3_params* p, Grid* g) {
  if (!ctx) return ATM3_EINVAL;
  ctx->err.clear();
  if (!p) return fail(ctx, ATM3_EINVAL, "params is NULL");
  if (!pos) return fail(ctx, ATM3_EINVAL, "pos is NULL");
  if (n < 1 || n > (int64_t)0x7fffffff / 3) return fail(ctx, ATM3_EINVAL, "n must be in [1, 2^31/3)");
  int rc = check_box(ctx, box, p->rc);
  if (rc) return rc;
  if (!(p->sigma > 0.0) || !isfinite(p->sigma)) return fail(ctx, ATM3_EINVAL, "sigma must be finite and > 0");
  if (!isfinite(p->eps) || !isfinite(p->nu)) return fail(ctx, ATM3_EINVAL, "eps and nu must be finite");
  if (p->truncation != ATM3_TRUNC_PAIR && p->truncation != ATM3_TRUNC_PRODUCT)
    return fail(ctx, ATM3_EINVAL, "truncation must be ATM3_TRUNC_PAIR or ATM3_TRUNC_PRODUCT");
  if (p->variant < ATM3_VARIANT_3C08 || p->variant > ATM3_VARIANT_3C01)
    return fail(ctx, ATM3_EINVAL, "variant must be 3c08, 3c18 or 3c01");
  if (p->terms < 1 || p->terms > 3) return fail(ctx, ATM3_EINVAL, "terms must be a non-empty OR of ATM3_TERM_*");
  if (p->flags & ~ATM3_FLAG_CHECK_FINITE) return fail(ctx, ATM3_EINVAL, "unknown bits in flags");
  if (!make_grid(box, p->rc, g)) return fail(ctx, ATM3_EINVAL, "cell grid out of range (floor(L/rc) < 1 or too many cells)");
  // 3 cells per dimension keep the 27 neighbours of a cell distinct; 3c18
  // needs 5: its base cell is the lexicographically smallest of wrapped
  // offsets spanning two steps, which for 3 or 4 cells depends on the
  // labelling
  const int need = (p->variant == ATM3_VARIANT_3C18) ? 5 : 3;
  for (int d = 0; d < 3; ++d)
    if (g->n[d] < need)
      return fail(ctx, ATM3_EINVAL,
                  "box too small: floor(L/rc) = " + std::to_string(g->n[d]) + " < " + std::to_string(need) +
                      " cells in some dimension");
  return set_device(ctx);
}

// The finite check of ATM3_FLAG_CHECK_FINITE (blocks until it has run).
int check_finite(atm3_ctx* ctx, const double* pos, int64_t n) {
  int32_t* bad = (int32_t*)ctx->buf[B_DEFER];
  hipError_t e = launch_check_finite(ctx->stream, pos, n, bad);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->hres, bad, 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "finite check");
  int32_t flag = 0;
  memcpy(&flag, ctx->hres, 4);
  if (flag) return fail(ctx, ATM3_ERANGE, "a position is not finite");
  return ATM3_OK;
}

int prepare(atm3_ctx* ctx, const double* pos, int64_t n, const double* box, const atm3_params* p, Grid* g) {
  int r = validate(ctx, pos, n, box, p, g);
  if (r) return r;
  size_t bytes[B_NBUF];
  plan_pair_path(n, *g, bytes);
  for (int b = 0; b < B_NBUF; ++b)
    if (bytes[b] && b != B_SRED && (r = ensure(ctx, (Buf)b, bytes[b]))) return r;
  if (p->flags & ATM3_FLAG_CHECK_FINITE) return check_finite(ctx, pos, n);
  return ATM3_OK;
}

// The fixed device array of the no-allocation entry point, one copy per
// device, and its device address on each device (hipGetSymbolAddress once
// per device, with that device current, at context creation).  Host code
// uses only these addresses, never the array's name.
constexpr int NOALLOC_MAXDEV = 64;
std::mutex noalloc_mu;
void* noalloc_addr[NOALLOC_MAXDEV] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[ATM3_NOALLOC_BYTES];

namespace {

int noalloc_init(atm3_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= NOALLOC_MAXDEV) return ATM3_EDEVICE;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (noalloc_addr[ctx->device]) return ATM3_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return ATM3_EDEVICE;
  noalloc_addr[ctx->device] = ptr;
  return ATM3_OK;
}

}  // namespace

extern "C" {

const char* atm3_version(void) { return "atm3 0.1 (gfx950)"; }

int atm3_create(atm3_ctx** out, int device_ordinal) {
  if (!out) return ATM3_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device_ordinal < 0 || device_ordinal >= count)
    return ATM3_EDEVICE;
  atm3_ctx* ctx = new (std::nothrow) atm3_ctx();
  if (!ctx) return ATM3_ENOMEM;
  ctx->device = device_ordinal;
  if (hipSetDevice(device_ordinal) != hipSuccess) {
    delete ctx;
    return ATM3_EDEVICE;
  }
  if (hipMalloc(&ctx->dres, sizeof(atm3_result)) != hipSuccess) {
    delete ctx;
    return ATM3_ENOMEM;
  }
  if (hipHostMalloc(&ctx->hres, sizeof(atm3_result), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(ctx->dres);
    delete ctx;
    return ATM3_ENOMEM;
  }
  if (noalloc_init(ctx) != ATM3_OK) {
    (void)hipHostFree(ctx->hres);
    (void)hipFree(ctx->dres);
    delete ctx;
    return ATM3_EDEVICE;
  }
  *out = ctx;
  return ATM3_OK;
}

void atm3_destroy(atm3_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (int b = 0; b < B_NBUF; ++b)
    if (ctx->s.p[b]) (void)hipFree(ctx->s.p[b]);
  for (int q = 0; q < NPHASE; ++q)
    for (hipEvent_t e : ctx->timer[q].ev) (void)hipEventDestroy(e);
  if (ctx->dres) (void)hipFree(ctx->dres);
  if (ctx->hres) (void)hipHostFree(ctx->hres);
  delete ctx;
}

int atm3_set_stream(atm3_ctx* ctx, void* hip_stream) {
  if (!ctx) return ATM3_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return ATM3_OK;
}

int atm3_profile_enable(atm3_ctx* ctx, int enable) {
  if (!ctx) return ATM3_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  ctx->profile = enable != 0;
  for (int q = 0; q < NPHASE; ++q) {
    ctx->timer[q].used = 0;
    ctx->timer[q].total_ms = 0.0;
    ctx->timer[q].launches = 0;
  }
  return ATM3_OK;
}

int atm3_profile_read(atm3_ctx* ctx, int phase, double* total_ms, int64_t* launches) {
  if (!ctx || phase < 0 || phase >= NPHASE || !total_ms || !launches) return ATM3_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  PhaseTimer& t = ctx->timer[phase];
  for (size_t k = 0; k < t.used; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
    t.total_ms += ms;
    ++t.launches;
  }
  t.used = 0;
  *total_ms = t.total_ms;
  *launches = t.launches;
  return ATM3_OK;
}

const char* atm3_last_error(const atm3_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

int atm3_bin_cells(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3], double rc, int32_t* cell_of,
                   int32_t* cell_start, int32_t* perm, int32_t ncell_out[3]) {
  if (!ctx) return ATM3_EINVAL;
  ctx->err.clear();
  int r = check_box(ctx, box, rc);
  if (r) return r;
  Grid g;
  if (!make_grid(box, rc, &g)) return fail(ctx, ATM3_EINVAL, "cell grid out of range");
  if (ncell_out)
    for (int d = 0; d < 3; ++d) ncell_out[d] = g.n[d];
  if (!cell_start) return ATM3_OK;
  if (!pos || !cell_of || !perm) return fail(ctx, ATM3_EINVAL, "NULL device pointer");
  if (n < 1 || n > (int64_t)0x7fffffff / 3) return fail(ctx, ATM3_EINVAL, "n must be in [1, 2^31/3)");
  if ((r = set_device(ctx))) return r;
  const size_t N = (size_t)n, C = (size_t)g.ncells;
  if ((r = ensure(ctx, B_CELL_OF, 4 * N))) return r;
  if ((r = ensure(ctx, B_RANK, 4 * N))) return r;
  if ((r = ensure(ctx, B_COUNT, 4 * C))) return r;
  if ((r = ensure(ctx, B_START, 4 * (C + 1)))) return r;
  if ((r = ensure(ctx, B_PERM, 4 * N))) return r;
  if ((r = ensure(ctx, B_SORTED, 32 * N))) return r;
  if ((r = ensure(ctx, B_TILE, 4 * (C / 1024 + 2)))) return r;
  hipError_t e = launch_binning(ctx, pos, n, g);
  if (e != hipSuccess) return hip_fail(ctx, e, "binning launch");
  e = hipMemcpyAsync(cell_of, ctx->buf[B_CELL_OF], 4 * N, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cell_start, ctx->buf[B_START], 4 * (C + 1), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(perm, ctx->buf[B_PERM], 4 * N, hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync");
  return ATM3_OK;
}

int atm3_compute_forces_async(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                              const atm3_params* params, float* forces, atm3_result* out_dev) {
  Grid g;
  int r = prepare(ctx, pos, n, box, params, &g);
  if (r) return r;
  if (!forces || !out_dev) return fail(ctx, ATM3_EINVAL, "forces / result pointer is NULL");
  hipError_t e = launch_binning(ctx, pos, n, g);
  if (e != hipSuccess) return hip_fail(ctx, e, "binning launch");
  if (params->truncation == ATM3_TRUNC_PRODUCT) {
    e = launch_onesided(ctx, pos, n, g, *params, forces, out_dev);
  } else {
    e = launch_forces(ctx, pos, n, g, *params, forces, out_dev);
    if (e == hipSuccess && params->variant != ATM3_VARIANT_3C08)
      e = launch_variant_counts(ctx, g, *params, out_dev, true);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "force launch");
  return ATM3_OK;
}

int atm3_compute_forces_noalloc(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                                const atm3_params* params, float* forces, atm3_result* out_dev) {
  Grid g;
  int r = validate(ctx, pos, n, box, params, &g);
  if (r) return r;
  if (!forces || !out_dev) return fail(ctx, ATM3_EINVAL, "forces / result pointer is NULL");
  if (params->truncation != ATM3_TRUNC_PAIR)
    return fail(ctx, ATM3_EINVAL, "the no-allocation entry point evaluates the pairwise cutoff only");
  if (ctx->profile) return fail(ctx, ATM3_EINVAL, "phase timing is not available without allocation");
  if (n > ATM3_NOALLOC_MAX_N || g.ncells > ATM3_NOALLOC_MAX_CELLS)
    return fail(ctx, ATM3_EINVAL,
                "no-allocation limits exceeded: n = " + std::to_string(n) + " (max " +
                    std::to_string(ATM3_NOALLOC_MAX_N) + "), cells = " + std::to_string(g.ncells) + " (max " +
                    std::to_string(ATM3_NOALLOC_MAX_CELLS) + ")");
  unsigned char* base = (unsigned char*)noalloc_addr[ctx->device];
  if (!base) return fail(ctx, ATM3_EDEVICE, "the fixed scratch array has no address on this device");
  size_t bytes[B_NBUF];
  plan_pair_path(n, g, bytes);
  void* table[B_NBUF] = {};
  size_t cap[B_NBUF] = {};
  size_t off = 0;
  for (int b = 0; b < B_NBUF; ++b) {
    if (!bytes[b]) continue;
    off = (off + 255) & ~(size_t)255;
    table[b] = base + off;
    cap[b] = bytes[b];
    off += bytes[b];
  }
  if (off > (size_t)ATM3_NOALLOC_BYTES)
    return fail(ctx, ATM3_EINVAL, "evaluation exceeds the fixed scratch array of the no-allocation entry point");
  ctx->buf = table;
  ctx->bufcap = cap;
  ctx->fixed = true;
  hipError_t e = hipSuccess;
  if (params->flags & ATM3_FLAG_CHECK_FINITE) r = check_finite(ctx, pos, n);
  if (!r) e = launch_binning(ctx, pos, n, g);
  if (!r && e == hipSuccess) e = launch_forces(ctx, pos, n, g, *params, forces, out_dev);
  if (!r && e == hipSuccess && params->variant != ATM3_VARIANT_3C08)
    e = launch_variant_counts(ctx, g, *params, out_dev, true);
  ctx->buf = ctx->s.p;
  ctx->bufcap = ctx->s.cap;
  ctx->fixed = false;
  if (r) return r;
  if (e != hipSuccess) return hip_fail(ctx, e, "force launch");
  return ATM3_OK;
}

int atm3_virial_diag(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3], const atm3_params* params,
                     double w_out[6]) {
  static_assert(sizeof(atm3_result) >= 7 * sizeof(double), "the result buffers hold the tensor and its status");
  Grid g;
  int r = prepare(ctx, pos, n, box, params, &g);
  if (r) return r;
  if (!w_out) return fail(ctx, ATM3_EINVAL, "w_out is NULL");
  if (params->truncation == ATM3_TRUNC_PRODUCT && params->variant == ATM3_VARIANT_3C01)
    return fail(ctx, ATM3_EINVAL, "the virial tensor is not available for 3c01 under the product rule");
  hipError_t e = launch_binning(ctx, pos, n, g);
  if (e == hipSuccess) e = launch_virial_diag(ctx, pos, n, g, *params, (double*)ctx->dres);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->hres, ctx->dres, 7 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "virial tensor");
  double h[7];
  memcpy(h, ctx->hres, sizeof(h));
  const int status = (int)h[6];
  if (status == ATM3_EOVERFLOW)
    return fail(ctx, status, "the cells within reach of a cell hold more than 2048 molecules, or a cell set more than 512");
  if (status == ATM3_ERANGE) return fail(ctx, status, "an ATM force term reached 2^18 (fixed-point accumulator range)");
  for (int k = 0; k < 6; ++k) w_out[k] = h[k];
  return ATM3_OK;
}

int atm3_compute_forces(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3], const atm3_params* params,
                        float* forces, atm3_result* out) {
  if (!out) return fail(ctx, ATM3_EINVAL, "result pointer is NULL");
  int r = atm3_compute_forces_async(ctx, pos, n, box, params, forces, ctx ? ctx->dres : nullptr);
  if (r) return r;
  hipError_t e = hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(atm3_result), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "result copy");
  *out = *ctx->hres;
  if (out->status == ATM3_EOVERFLOW)
    return fail(ctx, out->status,
                params->truncation == ATM3_TRUNC_PRODUCT
                    ? "the cells within reach of a cell hold more than 2048 molecules, or a 3c08 / 3c18 cell set more than 512"
                    : "a 2x2x2 block of cells holds more than 512 molecules");
  if (out->status == ATM3_ERANGE)
    return fail(ctx, out->status,
                params->truncation == ATM3_TRUNC_PRODUCT
                    ? "an ATM force term reached 2^18 (fixed-point accumulator range)"
                    : "a force contribution or sum reached 2^31 (fixed-point accumulator range)");
  if (out->status != ATM3_OK) return fail(ctx, out->status, "evaluation failed");
  return ATM3_OK;
}

}  // extern "C"
