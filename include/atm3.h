/*
 * atm3 -- linked-cell Lennard-Jones + Axilrod-Teller-Muto forces on MI355X.
 *
 * C ABI of libatm3.so.  Plain pointers and sizes only; device pointers are
 * HIP device memory of the context's device (for example the data pointer of
 * a contiguous torch tensor on that device).  No function throws across this
 * boundary; each returns ATM3_OK (0) or a negative status, and
 * atm3_last_error() gives the message of the last failure on that context.
 *
 * The computation follows "Linked Cell Traversal Algorithms for Three-Body
 * Interactions in Molecular Dynamics" (Pinzon Escobar, Muehlhaeusser,
 * Bungartz, Neumann):
 *   Sec. 2  truncation conditions (pairwise, product); eq. (forcepairs) and
 *           eq. (newton3rdlaw): three force pairs per triplet; eq. (atm) the
 *           ATM energy, eq. (ATMGradient) its radial derivative;
 *   Sec. 3  triplets of molecules stored in one, two or three cells,
 *           eqs. (celltriplet), (twoonetriplets), (carttriplets);
 *   Sec. 4  linked cells of side >= rc in lexicographic order, and the cell
 *           sets visited by the 3c01, 3c18 and 3c08 traversals;
 *   Sec. 5  the Lennard-Jones pair term in reduced units and the three-body
 *           virial W_3 of eq. (P_3).
 *
 * Units: reduced Lennard-Jones units.  Positions are FP64, forces FP32,
 * energies and virials FP64.  The virial returned is W = sum over pairs /
 * triplets of r.F (eq. P_3 for the three-body part), not a pressure.
 *
 * Threading: one context per host thread; all work of a context is enqueued
 * on its stream, in order.
 */
#ifndef ATM3_H
#define ATM3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define ATM3_OK 0
#define ATM3_EINVAL (-1)    /* invalid argument (message says which)          */
#define ATM3_EDEVICE (-2)   /* HIP runtime error or bad device ordinal        */
#define ATM3_ENOMEM (-3)    /* device allocation failed                       */
#define ATM3_ERANGE (-4)    /* non-finite input, or a force term beyond the
                               fixed-point range (see atm3_compute_forces)   */
#define ATM3_EOVERFLOW (-5) /* too many molecules in a cell neighbourhood   */

/* Truncation conditions of Sec. 2. */
#define ATM3_TRUNC_PAIR 0    /* a triplet counts iff all three sides < rc        */
#define ATM3_TRUNC_PRODUCT 1 /* iff r_ij * r_ik * r_jk < rc^3 (squared: < rc^6) */

/* Cell sets visited (Sec. 4). */
#define ATM3_VARIANT_3C08 0 /* cells of one 2x2x2 block, each triplet once       */
#define ATM3_VARIANT_3C18 1 /* base cell + two cells of base or its 13 forward
                               neighbours                                      */
#define ATM3_VARIANT_3C01 2 /* per molecule, 27-cell neighbourhood, no Newton 3  */

/* Terms. */
#define ATM3_TERM_LJ 1
#define ATM3_TERM_ATM 2

/* Flags. */
#define ATM3_FLAG_CHECK_FINITE 2 /* reject non-finite positions with ATM3_ERANGE
                                    (the check blocks until it has run)      */

typedef struct atm3_ctx atm3_ctx;

typedef struct {
  double eps;         /* LJ well depth epsilon (> = 0)                          */
  double sigma;       /* LJ diameter sigma (> 0)                                */
  double nu;          /* ATM strength nu                                        */
  double rc;          /* cutoff radius (> 0); cell side = L_d / floor(L_d/rc)   */
  int32_t truncation; /* ATM3_TRUNC_*                                           */
  int32_t variant;    /* ATM3_VARIANT_*                                         */
  int32_t terms;      /* OR of ATM3_TERM_* (non-zero)                           */
  int32_t flags;      /* OR of ATM3_FLAG_*                                      */
} atm3_params;

typedef struct {
  double e_lj;          /* LJ energy (unshifted, truncated at rc)              */
  double e_atm;         /* ATM energy, eq. (atm) summed over included triplets */
  double w_lj;          /* LJ virial sum r.F                                   */
  double w_atm;         /* three-body virial W_3, eq. (P_3)                    */
  int64_t n_pairs;      /* included LJ pairs                                   */
  int64_t n_triplets;   /* included triplets (3c01: receiving incidences)      */
  int64_t n_candidates; /* molecule triplets of the visited cell sets          */
  int32_t ncell[3];     /* cells per dimension                                 */
  int32_t status;       /* ATM3_OK or the failure status of the evaluation     */
} atm3_result;

/* Create a context on HIP device `device_ordinal`.  The context owns all
 * device scratch (grown on demand, freed by atm3_destroy) and starts on the
 * device's null stream.  Returns ATM3_EDEVICE for a bad ordinal. */
int atm3_create(atm3_ctx** out, int device_ordinal);

/* Free the context and its scratch.  NULL is ignored. */
void atm3_destroy(atm3_ctx* ctx);

/* Set the HIP stream (hipStream_t passed as void*; NULL = null stream) on
 * which all later work of this context is enqueued. */
int atm3_set_stream(atm3_ctx* ctx, void* hip_stream);

/* Message of the last failed call on this context ("" if none).  The string
 * is owned by the context and valid until its next call. */
const char* atm3_last_error(const atm3_ctx* ctx);

/* Version string of the library (static storage). */
const char* atm3_version(void);

/* Linked-cell binning (Sec. 4): cells of side L_d / n_d with
 * n_d = floor(L_d / rc) >= 1, lexicographic linear index
 * c = (c_z * n_y + c_y) * n_x + c_x.  Each position is wrapped
 * x <- x - L*floor(x/L) and binned c_d = floor(x * (n_d / L_d)) clamped to
 * [0, n_d - 1], in FP64 without contraction (bit-exact).
 *   pos        device, n*3 FP64, molecule-major (x, y, z), caller-owned
 *   n          number of molecules, 1 <= n < 2^31
 *   box        host, 3 FP64 box lengths > 0 (orthorhombic, periodic)
 *   cell_of    device, n int32: linear cell of each molecule (input order)
 *   cell_start device, ncells+1 int32: exclusive prefix of cell populations
 *   perm       device, n int32: sorted slot -> input index; molecules of a
 *              cell are contiguous and keep their input order (stable)
 *   ncell_out  host, 3 int32: cells per dimension
 * The caller sizes cell_start from the cell counts floor(L_d/rc); pass
 * cell_start = NULL to only query ncell_out.  Synchronous only with respect
 * to ncell_out; the device outputs are enqueued on the context stream. */
int atm3_bin_cells(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3], double rc,
                   int32_t* cell_of, int32_t* cell_start, int32_t* perm, int32_t ncell_out[3]);

/* One evaluation of LJ + ATM forces, energies, virials and counts.
 *   pos     device, n*3 FP64 positions (any periodic image)
 *   forces  device, n*3 FP32 output, input order, overwritten
 *   out     host result; the call blocks until the evaluation is done
 * Preconditions (ATM3_EINVAL otherwise): n >= 1; rc > 0; sigma > 0; every
 * n_d >= 3 (the 27 neighbours of a cell are distinct), n_d >= 5 for 3c18.
 * Every distance is the minimum image.  Returns ATM3_EOVERFLOW if some
 * 2x2x2 block of cells holds more than 512 molecules (pair rule), or, under
 * the product rule, the 27 cells around one cell hold more than 2048 or
 * one 3c08 / 3c18 cell set more than 512.
 * Returns ATM3_ERANGE if a force term or sum reaches 2^31 in magnitude
 * (pair rule) or an ATM or LJ force term reaches 2^18 (product rule with
 * 3c08 / 3c18).  Forces are accumulated exactly in 64-bit fixed point with 2^-32
 * resolution and are undefined after either error.  Results are
 * reproducible bit for bit between calls. */
int atm3_compute_forces(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                        const atm3_params* params, float* forces, atm3_result* out);

/* Diagonal of the virial tensor, W_aa = sum over force pairs of r_a F_a: the
 * LJ pairs, and the three force pairs F_i(j)k, F_i(k)j, F_j(k)i of eq.
 * (forcepairs) of every included triplet (the pressure tensor behind the
 * surface tensions that motivate three-body forces at interfaces, Sec. 1).
 * The trace is the scalar virial of atm3_compute_forces.
 *   w_out  host, 6 FP64: LJ xx, yy, zz, then ATM xx, yy, zz (FP64 sums of
 *          FP32 terms)
 * Same arguments and preconditions as atm3_compute_forces; the pairwise
 * cutoff uses the 3c08 sets (every cell set includes the same triplets),
 * the product cutoff 3c08 or 3c18 (ATM3_EINVAL for 3c01).  Blocks until
 * done.  ATM3_EOVERFLOW / ATM3_ERANGE as for the product rule. */
int atm3_virial_diag(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                     const atm3_params* params, double w_out[6]);

/* As atm3_compute_forces, but enqueue only: the result struct is written to
 * `out_dev` (device memory, sizeof(atm3_result) bytes) by the last kernel,
 * including its `status`.  Nothing blocks.  Argument checks happen on the
 * host before anything is enqueued. */
int atm3_compute_forces_async(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                              const atm3_params* params, float* forces, atm3_result* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * atm3_compute_forces_async with the pairwise cutoff (any cell set), but
 * every scratch buffer of the evaluation is carved from one fixed device
 * array of ATM3_NOALLOC_BYTES that the library holds on each device it runs
 * on until the process ends.  The call allocates nothing; the caller still
 * provides pos, forces and out_dev.  Outputs are bit-identical to
 * atm3_compute_forces_async with the same arguments.
 * Limits: n <= ATM3_NOALLOC_MAX_N and at most ATM3_NOALLOC_MAX_CELLS cells
 * (ATM3_EINVAL beyond them, before anything is enqueued); the product
 * cutoff and enabled phase timing return ATM3_EINVAL.
 * Every call on a device shares that device's array and leaves its last
 * contents there: calls that overlap on one device (two contexts, two
 * streams, or two threads) race and give undefined results; calls ordered
 * on one stream are safe.  Other errors as atm3_compute_forces_async. */
#define ATM3_NOALLOC_MAX_N 65536
#define ATM3_NOALLOC_MAX_CELLS 65536
#define ATM3_NOALLOC_BYTES (24 << 20)
int atm3_compute_forces_noalloc(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                                const atm3_params* params, float* forces, atm3_result* out_dev);

/* Kernel timing with HIP events recorded on the context stream around each
 * phase of atm3_compute_forces[_async]:
 *   ATM3_PHASE_BINNING  wrap/cell index, counting sort, coordinate gather
 *   ATM3_PHASE_BLOCK    the fused LJ + ATM kernel over 2x2x2 cell blocks
 *   ATM3_PHASE_BIG      the same for blocks of more than 128 molecules
 *   ATM3_PHASE_REDUCE   per-molecule force gather and the global reduction
 * atm3_profile_enable(ctx, 1) starts recording (and clears the totals);
 * atm3_profile_read() waits for the stream, then returns the summed elapsed
 * milliseconds and number of timed launches of one phase. */
#define ATM3_PHASE_BINNING 0
#define ATM3_PHASE_BLOCK 1
#define ATM3_PHASE_BIG 2
#define ATM3_PHASE_REDUCE 3
int atm3_profile_enable(atm3_ctx* ctx, int enable);
int atm3_profile_read(atm3_ctx* ctx, int phase, double* total_ms, int64_t* launches);


/* ------------------------------------------------------------------------
 * Learned three-body pair surrogate.
 *
 * The paper computes the ATM forces exactly; this model is an addition whose
 * error is always measured against the exact evaluation above.  Per
 * molecule i, 64 rotation-, translation- and permutation-invariant
 * descriptors D_i are built from its neighbours j (minimum-image
 * r_ij^2 < rc^2, the exact path's pair rule, Sec. 2): for 16 radial channels
 * g_a(r) = exp(-((r - mu_a)/w)^2) fc(r), mu_a = 0.8 + a w,
 * w = (rc - 0.8)/15, fc(r) = (1 + cos(pi r/rc))/2, with u_ij = (r_j - r_i)/r_ij:
 *   S_a = sum g_a, V_a = sum g_a u, Q_a = sum g_a (u u^T - I/3),
 *   D_raw = [S_a, |V_a|^2, Q_a:Q_a, V_a^T Q_a V_a], D = (D_raw - mean) * inv_sd.
 * A pair MLP on x_ij = [D_i + D_j, g(r_ij)] (80 inputs, symmetric in i, j),
 * 80 -> 128 -> 128 -> 128 -> 2 with ReLU, gives s_ij and t_ij; the
 * three-body force is F_i = sum_j s_ij (r_i - r_j)/r_ij (Newton 3 holds
 * exactly) and the error estimate e_i = sum_j softplus(t_ij).  Matrix
 * products run on BF16 MFMA with FP32 accumulation.
 *
 * Parameters: ATM3_MLP_NPARAM FP32 values in the order
 *   W1 [80][128] (rows: 64 descriptor inputs, then 16 radial inputs), b1[128],
 *   W2 [128][128], b2[128], W3 [128][128], b3[128], W4 [128][2], b4[2],
 * each matrix [input][output] row-major.  Descriptor statistics: mean[64],
 * inv_sd[64].
 * ---------------------------------------------------------------------- */
#define ATM3_MLP_NPARAM 43650
#define ATM3_MLP_NDESC 64

typedef struct atm3_mlp atm3_mlp;

/* Create a model on the context's device with seeded He-initialised
 * weights (zero biases, b4 = (0, -3)) and identity statistics (mean 0,
 * inv_sd 1).  The model holds its parameters, Adam moments and BF16 copies;
 * use it only with the context it was created with. */
int atm3_mlp_create(atm3_ctx* ctx, uint64_t seed, atm3_mlp** out);
void atm3_mlp_destroy(atm3_mlp* mlp);

/* Copy parameters from / to host memory (n must be ATM3_MLP_NPARAM).
 * Setting parameters clears the Adam moments. */
int atm3_mlp_set_params(atm3_ctx* ctx, atm3_mlp* mlp, const float* host, int64_t n);
int atm3_mlp_get_params(atm3_ctx* ctx, atm3_mlp* mlp, float* host, int64_t n);

/* Descriptor statistics from / to host memory (64 + 64 values). */
int atm3_mlp_set_stats(atm3_ctx* ctx, atm3_mlp* mlp, const float* mean, const float* inv_sd);
int atm3_mlp_get_stats(atm3_ctx* ctx, atm3_mlp* mlp, float* mean, float* inv_sd);

/* Fit the statistics to one configuration: per-feature mean and
 * 1/max(sd, 1e-6) of the raw descriptors (population sd, FP64 sums). */
int atm3_mlp_fit_stats(atm3_ctx* ctx, atm3_mlp* mlp, const double* pos, int64_t n, const double box[3],
                       double rc);

/* Forces with the surrogate three-body term.
 *   forces    device, n*3 FP32, input order: exact LJ (pair list, FP64
 *             arithmetic on FP32 displacements) plus, per molecule, the
 *             surrogate three-body force, or, where e_i > err_threshold,
 *             the exact one-sided ATM force of that molecule (all included
 *             triplets containing it, eqs. atm, ATMGradient, forcepairs)
 *   err_est   device, n FP32 error estimates e_i (may be NULL)
 *   out       host result: e_lj, w_lj, n_pairs as the exact path; e_atm and
 *             w_atm are NaN (the surrogate has no energy); n_triplets counts
 *             the triplets the fallback evaluated
 *   n_fallback host, number of molecules that took the exact fallback
 * params: eps, sigma, nu, rc as for atm3_compute_forces (the pair rule).
 * Blocks until done.  ATM3_EINVAL for fewer than 3 cells per dimension or
 * more than 2^30 pairs. */
int atm3_surrogate_forces(atm3_ctx* ctx, atm3_mlp* mlp, const double* pos, int64_t n, const double box[3],
                          const atm3_params* params, float err_threshold, float* forces, float* err_est,
                          atm3_result* out, int64_t* n_fallback);

/* Gradient of the training loss
 *   L = mean_i |F_i - T_i|^2 + lam * mean_i (e_i - |F_i - T_i|)^2
 * (the second target held constant) at one configuration, with F the
 * surrogate three-body force and T = f3_target (device, n*3 FP32, input
 * order; for example the ATM-only forces of atm3_compute_forces).
 *   grad_dev device, ATM3_MLP_NPARAM FP32 (may be NULL: only the loss)
 *   loss_out host, L
 * Blocks until done. */
int atm3_mlp_grad(atm3_ctx* ctx, atm3_mlp* mlp, const double* pos, int64_t n, const double box[3], double rc,
                  const float* f3_target, float lam, float* grad_dev, double* loss_out);

/* One Adam step (bias-corrected) with the gradient grad_dev (device,
 * ATM3_MLP_NPARAM FP32); refreshes the BF16 weight copies. */
int atm3_mlp_adam(atm3_ctx* ctx, atm3_mlp* mlp, const float* grad_dev, float lr, float beta1, float beta2,
                  float eps);

/* atm3_mlp_grad followed by atm3_mlp_adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) on the model's own gradient buffer. */
int atm3_mlp_train_step(atm3_ctx* ctx, atm3_mlp* mlp, const double* pos, int64_t n, const double box[3], double rc,
                        const float* f3_target, float lam, float lr, double* loss_out);

/* Inspection of one surrogate evaluation (no fallback):
 *   pair_ij  device, 2*cap int32: input indices of each pair
 *   st       device, 2*cap FP32: s, t of each pair
 *   desc     device, n*64 FP32 normalised descriptors, input order
 *   f3       device, n*3 FP32 surrogate three-body force, input order
 *   err      device, n FP32 error estimate, input order
 *   n_pairs  host, number of pairs (entries beyond cap are not written)
 * Any of the device outputs may be NULL. */
int atm3_surrogate_pairs(atm3_ctx* ctx, atm3_mlp* mlp, const double* pos, int64_t n, const double box[3],
                         double rc, int64_t cap, int32_t* pair_ij, float* st, float* desc, float* f3, float* err,
                         int64_t* n_pairs);

/* ------------------------------------------------------------------------
 * Molecular dynamics driver: velocity Verlet (NVE), unit mass, reduced LJ
 * units, FP64 positions and velocities (device, n*3, molecule-major), FP32
 * forces (device, n*3, e.g. from atm3_compute_forces).  One step is
 *   atm3_md_kick_drift(dt)   v += dt/2 F(x);  x += dt v
 *   (new forces F(x))
 *   atm3_md_kick(dt)         v += dt/2 F(x)
 * Positions are not wrapped (the force routines accept any image).  Both
 * only enqueue.  atm3_md_kinetic returns sum v^2 / 2 (FP64, fixed-order
 * reduction) and blocks. */
int atm3_md_kick_drift(atm3_ctx* ctx, double* pos, double* vel, const float* forces, int64_t n, double dt);
int atm3_md_kick(atm3_ctx* ctx, double* vel, const float* forces, int64_t n, double dt);
int atm3_md_kinetic(atm3_ctx* ctx, const double* vel, int64_t n, double* ke_out);

/* Isokinetic thermostat for the NVT runs of Sec. 5.1 (the paper does not name
 * its thermostat): scales the device velocities `vel` (n*3 FP64, in place)
 * so that sum v^2 / 2 = dof * temperature / 2, with dof degrees of freedom
 * (3n - 3 for zero total momentum).  Velocities that are all zero are left
 * as they are.  Only enqueues (kinetic energy reduced on the device).
 * Errors: ATM3_EINVAL for a NULL pointer, n < 1, temperature <= 0 or not
 * finite, dof outside [1, 3n]. */
int atm3_md_rescale(atm3_ctx* ctx, double* vel, int64_t n, double temperature, int64_t dof);

/* Long-range correction of the LJ forces in planar geometry, for the slab
 * runs of Sec. 5.2 (the paper adds one and cites it without stating it).
 * The instantaneous density profile along z is binned into nbins bins over
 * L_z: a molecule's bin is k = floor(z' * (nbins / L_z)), clamped to
 * [0, nbins - 1], with z' = z - L_z floor(z / L_z) (FP64, bit-exact).  Each
 * bin is taken as a uniform sheet of areal density n_k / (L_x L_y) at its
 * centre.  Its molecules beyond rc pull a molecule at height offset xi
 * along z with 2 pi s_a xi phi(max(rc, |xi|)), where phi is the LJ
 * potential 4 eps [(sigma/r)^12 - (sigma/r)^6] and xi the minimum image.
 * Every molecule of bin b takes the force at b's centre (FP64 sum over the
 * bins), added in FP64 to forces[3i + 2]; bin pairs act with opposite
 * forces, so no net momentum is added.
 *   pos       device, n*3 FP64 positions
 *   forces    device, n*3 FP32, updated in place (z components)
 *   hist_sum  device, nbins int64, or NULL: this call's bin counts are added
 *             (density profile sampling)
 * Only enqueues.  Errors: ATM3_EINVAL for a NULL pointer, n < 1, a box length
 * not finite and > 0, nbins outside [1, 4096], rc <= 0 or rc > L_z / 2,
 * eps or sigma <= 0. */
int atm3_md_slab_lrc(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3], int32_t nbins, double rc,
                     double eps, double sigma, float* forces, int64_t* hist_sum);

/* `steps` NVT steps (the isokinetic runs of Sec. 5.1 and 5.2) with every
 * step captured once as a HIP graph and launched `steps` times, instead of
 * some twenty kernel launches per step from the host.  One step is:
 * atm3_md_kick_drift; atm3_compute_forces_async; atm3_md_slab_lrc if
 * lrc_bins > 0 (histogram added to `profile` if not NULL); atm3_md_kick;
 * atm3_md_rescale to `temperature` with `dof` degrees of freedom.  The
 * result struct of step k (k = 1..steps) is written to
 * rows + (k / sample_every - 1) * row_stride when sample_every divides k,
 * and the status of every evaluation (the initial one and every step,
 * sampled or not) is folded into the status
 * field of the row after the last sample, rows + nsamp * row_stride with
 * nsamp = steps / sample_every, as the minimum of the statuses (so any
 * failure, being negative, stays there); the caller sets that field to
 * ATM3_OK before the call.
 * Before the first step the forces at the initial positions are computed
 * (with the correction).  The trajectory and the rows are bit-identical to
 * the same calls made one by one.
 *   pos, vel  device, n*3 FP64, updated in place
 *   forces    device, n*3 FP32 scratch, holds the last step's forces
 *   rows      device, (steps / sample_every + 1) * row_stride bytes,
 *             caller-owned
 *   profile   device, lrc_bins int64, or NULL
 * Ordered after the work already enqueued on the context stream; returns
 * when the run has finished.  Errors: ATM3_EINVAL for the conditions of the
 * calls it makes, steps or sample_every < 1, row_stride not a multiple of 8
 * or below sizeof(atm3_result), ATM3_FLAG_CHECK_FINITE set, or profiling
 * enabled (neither can be captured); a failed evaluation is reported in the
 * folded status of row nsamp, and in its own row if it was sampled. */
int atm3_md_nvt_graph(atm3_ctx* ctx, double* pos, double* vel, int64_t n, const double box[3],
                      const atm3_params* params, int64_t steps, double dt, double temperature, int64_t dof,
                      int64_t sample_every, float* forces, void* rows, int64_t row_stride, int32_t lrc_bins,
                      int64_t* profile);

#ifdef __cplusplus
}
#endif

#endif /* ATM3_H */
