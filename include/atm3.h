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
#define ATM3_ERANGE (-4)    /* non-finite input, or a force beyond +-2^31     */
#define ATM3_EOVERFLOW (-5) /* a 2x2x2 cell block holds more than 512 molecules */

/* Truncation conditions of Sec. 2. */
#define ATM3_TRUNC_PAIR 0    /* a triplet counts iff all three sides < rc        */
#define ATM3_TRUNC_PRODUCT 1 /* iff r_ij * r_ik * r_jk < rc^3 (squared: < rc^6) */

/* Cell sets visited (Sec. 4). */
#define ATM3_VARIANT_3C08 0 /* cells of one 2x2x2 block, each triplet once       */
#define ATM3_VARIANT_3C18 1 /* base cell + two of its 13 forward neighbours      */
#define ATM3_VARIANT_3C01 2 /* per molecule, 27-cell neighbourhood, no Newton 3  */

/* Terms. */
#define ATM3_TERM_LJ 1
#define ATM3_TERM_ATM 2

/* Flags. */
#define ATM3_FLAG_CHECK_FINITE 2 /* reject non-finite positions with ATM3_ERANGE */

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
 * n_d >= 3, and n_d >= 5 for the product rule with 3c08, n_d >= 7 for the
 * product rule with 3c18 or 3c01 (so cell shifts equal minimum images).
 * Returns ATM3_EOVERFLOW if some 2x2x2 block of cells holds more than 512
 * molecules, ATM3_ERANGE if a force term or sum reaches 2^31 in magnitude
 * (forces are accumulated exactly in 64-bit fixed point with 2^-32
 * resolution); forces are undefined in both cases.  Results are
 * reproducible bit for bit between calls. */
int atm3_compute_forces(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
                        const atm3_params* params, float* forces, atm3_result* out);

/* As atm3_compute_forces, but enqueue only: the result struct is written to
 * `out_dev` (device memory, sizeof(atm3_result) bytes) by the last kernel,
 * including its `status`.  Nothing blocks.  Argument checks happen on the
 * host before anything is enqueued. */
int atm3_compute_forces_async(atm3_ctx* ctx, const double* pos, int64_t n, const double box[3],
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

#ifdef __cplusplus
}
#endif

#endif /* ATM3_H */
