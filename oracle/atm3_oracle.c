/*
 * FP64 CPU oracle for linked-cell Lennard-Jones + Axilrod-Teller-Muto forces.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * Paper: "Linked Cell Traversal Algorithms for Three-Body Interactions in
 * Molecular Dynamics" (Pinzon Escobar, Muehlhaeusser, Bungartz, Neumann).
 * Every function cites the passage it follows.  The method is exact, so the
 * oracle computes the plain definition directly: brute force over all pairs
 * and triplets, with the inclusion rule "truncation condition AND the cell
 * sets the chosen traversal visits" evaluated per pair / triplet.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA contraction,
 * so every FP64 decision below is the IEEE result of the expression as
 * written, left to right).
 *
 * Readings of the paper fixed here (each also listed in the design notes):
 *  - force is MINUS the gradient of the potential;
 *  - cutoff comparisons are strict: a pair is inside iff r^2 < rc^2;
 *  - product rule: the three squared sides, sorted ascending, multiplied left
 *    to right, compared strictly against (rc^2*rc^2)*rc^2;
 *  - Lennard-Jones is the unshifted 12-6 form truncated at rc, over pairs of
 *    molecules whose cells are neighbours (all variants);
 *  - 3c08 visits a triplet iff its three cells fit in one 2x2x2 block of
 *    cells; 3c18 iff, in the local frame, the two cells other than the
 *    lexicographically smallest one are that cell itself or its forward
 *    neighbours; 3c01 (no Newton 3) gives molecule m its share of a triplet
 *    iff both other cells are in the 27-cell neighbourhood of m's cell, and
 *    credits energy and virial one third per receiving molecule.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double eps, sigma, nu, rc;
  int32_t truncation; /* 0 = pairwise cutoff, 1 = product cutoff (Sec. 2) */
  int32_t variant;    /* 0 = 3c08, 1 = 3c18, 2 = 3c01 (Sec. 4)           */
  int32_t terms;      /* bit0 Lennard-Jones, bit1 ATM                    */
  int32_t pad;
} orc_params;

typedef struct {
  double e_lj, e_atm, w_lj, w_atm;
  int64_t n_pairs, n_triplets, n_candidates;
  int64_t n_distinct; /* distinct included triplets (3c01: at least one receiver) */
} orc_result;

/* ------------------------------------------------------------------------ */
/* Linked cells (Sec. 4 preamble): cell side >= rc, lexicographic order.    */
/* ------------------------------------------------------------------------ */

/* Number of cells per dimension: floor(L_d / rc), so the side L_d/n_d >= rc. */
int orc_grid(const double box[3], double rc, int32_t ncell[3]) {
  for (int d = 0; d < 3; ++d) {
    double q = floor(box[d] / rc);
    if (!(q >= 1.0) || q > 2147483647.0) return -1;
    ncell[d] = (int32_t)q;
  }
  return 0;
}

/* Wrap into the box and assign the cell: x <- x - L*floor(x/L),
 * c = floor(x * (n/L)) clamped to [0, n-1]; linear index (cz*ny + cy)*nx + cx
 * with x fastest (lexicographic cell order).  Outputs per molecule the three
 * cell coordinates and the linear index. */
void orc_bin(const double* pos, int64_t n, const double box[3],
             const int32_t ncell[3], int32_t* cxyz, int32_t* clin) {
  double inv[3];
  for (int d = 0; d < 3; ++d) inv[d] = (double)ncell[d] / box[d];
  for (int64_t i = 0; i < n; ++i) {
    int32_t c[3];
    for (int d = 0; d < 3; ++d) {
      double x = pos[3 * i + d];
      double f = floor(x / box[d]);
      double xw = x - box[d] * f;
      double t = floor(xw * inv[d]);
      int32_t ci = (t < 0.0) ? 0 : (t > (double)(ncell[d] - 1) ? ncell[d] - 1 : (int32_t)t);
      c[d] = ci;
      if (cxyz) cxyz[3 * i + d] = ci;
    }
    if (clin) clin[i] = (c[2] * ncell[1] + c[1]) * ncell[0] + c[0];
  }
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* Minimum-image displacement a - b: d -= L * rint(d / L) per component. */
static inline void min_image(const double* a, const double* b, const double box[3], double d[3]) {
  for (int k = 0; k < 3; ++k) {
    double t = a[k] - b[k];
    d[k] = t - box[k] * rint(t / box[k]);
  }
}

/* Squared length, evaluated left to right, no fused multiply-add. */
static inline double sqlen(const double d[3]) {
  double s = d[0] * d[0];
  s = s + d[1] * d[1];
  s = s + d[2] * d[2];
  return s;
}

/* Periodic cell offset b - a mapped to the symmetric window around 0. */
static inline int wrap_off(int off, int n) {
  off %= n;
  if (off < 0) off += n;
  if (off > n / 2) off -= n;
  return off;
}

/* ------------------------------------------------------------------------ */
/* Potentials                                                                */
/* ------------------------------------------------------------------------ */

/* Lennard-Jones 12-6 in reduced units (Sec. 5): u = 4 eps [(s/r)^12-(s/r)^6];
 * returns u and f with F_i = f * r_ij (f = -(du/dr)/r). */
static inline void lj_pair(double r2, double eps, double sigma, double* u, double* f) {
  double s2 = (sigma * sigma) / r2;
  double s6 = s2 * s2 * s2;
  double s12 = s6 * s6;
  *u = 4.0 * eps * (s12 - s6);
  *f = 24.0 * eps * (2.0 * s12 - s6) / r2;
}

/* Axilrod-Teller-Muto energy, eq. (atm): the law-of-cosines form in the three
 * side lengths a = r_ij, b = r_ik, c = r_jk. */
double orc_atm_energy(double a, double b, double c, double nu) {
  double x = a * a, y = b * b, z = c * c;
  double a3 = a * a * a, b3 = b * b * b, c3 = c * c * c;
  double a5 = a3 * a * a, b5 = b3 * b * b, c5 = c3 * c * c;
  double first = 1.0 / (a3 * b3 * c3);
  double second = 3.0 * (-x + y + z) * (x - y + z) * (x + y - z) / (8.0 * a5 * b5 * c5);
  return nu * (first + second);
}

/* Radial derivative of the ATM energy with respect to the side a, with b and
 * c the two other sides: eq. (ATMGradient), its eleven terms written out as
 * printed (with a = r_ij, b = r_ik, c = r_jk).  The derivatives with respect
 * to the other two sides follow by cycling the roles (Sec. 2). */
double orc_atm_dudr(double a, double b, double c, double nu) {
  double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
  double b3 = b * b * b, b5 = b3 * b * b;
  double c3 = c * c * c, c5 = c3 * c * c;
  double s = 0.0;
  s += -1.0 / (a4 * b3 * c3);
  s += -1.0 / (8.0 * b5 * c5);
  s += 5.0 * b / (8.0 * a6 * c5);
  s += 5.0 * c / (8.0 * a6 * b5);
  s += -1.0 / (8.0 * a2 * b3 * c5);
  s += -1.0 / (8.0 * a2 * b5 * c3);
  s += -3.0 / (8.0 * a4 * b * c5);
  s += -3.0 / (8.0 * a4 * b5 * c);
  s += -5.0 / (8.0 * a6 * b * c3);
  s += -5.0 / (8.0 * a6 * b3 * c);
  s += 6.0 / (8.0 * a4 * b3 * c3);
  return 3.0 * nu * s;
}

/* The three force pairs of eq. (forcepairs) for one triplet:
 *   F_i(j)k = -(du/dr_ij) r_ij/|r_ij|,  F_i(k)j = -(du/dr_ik) r_ik/|r_ik|,
 *   F_j(k)i = -(du/dr_jk) r_jk/|r_jk|,
 * with r_ab = r_a - r_b.  Also returns the energy (eq. atm) and the triplet's
 * virial term of eq. (P_3). */
static void atm_force_pairs(const double rij[3], const double rik[3], const double rjk[3],
                            double x, double y, double z, double nu,
                            double fij[3], double fik[3], double fjk[3],
                            double* u, double* w) {
  double a = sqrt(x), b = sqrt(y), c = sqrt(z);
  double gij = orc_atm_dudr(a, b, c, nu);
  double gik = orc_atm_dudr(b, a, c, nu);
  double gjk = orc_atm_dudr(c, a, b, nu);
  double sij = -gij / a, sik = -gik / b, sjk = -gjk / c;
  for (int d = 0; d < 3; ++d) {
    fij[d] = sij * rij[d];
    fik[d] = sik * rik[d];
    fjk[d] = sjk * rjk[d];
  }
  *u = orc_atm_energy(a, b, c, nu);
  double wij = rij[0] * fij[0] + rij[1] * fij[1] + rij[2] * fij[2];
  double wik = rik[0] * fik[0] + rik[1] * fik[1] + rik[2] * fik[2];
  double wjk = rjk[0] * fjk[0] + rjk[1] * fjk[1] + rjk[2] * fjk[2];
  *w = wij + wik + wjk;
}

/* ------------------------------------------------------------------------ */
/* Inclusion rules                                                           */
/* ------------------------------------------------------------------------ */

/* Truncation (Sec. 2): pairwise -> every side inside rc; product -> the
 * product of the sides below rc^3, tested on squared sides in ascending order
 * so the decision does not depend on how the triplet is labelled. */
static inline int truncation_ok(double x, double y, double z, double rc, int rule) {
  double rc2 = rc * rc;
  if (rule == 0) return (x < rc2) && (y < rc2) && (z < rc2);
  double s0 = x, s1 = y, s2 = z, t;
  if (s1 < s0) { t = s0; s0 = s1; s1 = t; }
  if (s2 < s1) { t = s1; s1 = s2; s2 = t; }
  if (s1 < s0) { t = s0; s0 = s1; s1 = t; }
  double rc6 = (rc2 * rc2) * rc2;
  return ((s0 * s1) * s2) < rc6;
}

/* Pair visited by the cell traversal: the two cells are equal or neighbours. */
static inline int cells_adjacent(const int32_t* ca, const int32_t* cb, const int32_t n[3]) {
  for (int d = 0; d < 3; ++d) {
    int o = wrap_off(cb[d] - ca[d], n[d]);
    if (o < -1 || o > 1) return 0;
  }
  return 1;
}

/* Lexicographic order of cell offsets: z most significant, x least. */
static inline int lex_less(const int* p, const int* q) {
  if (p[2] != q[2]) return p[2] < q[2];
  if (p[1] != q[1]) return p[1] < q[1];
  return p[0] < q[0];
}

/* 3c08 (Sec. 4, Fig. c08): the triplet's cells lie in one 2x2x2 block, i.e.
 * in every dimension the three cell coordinates span at most one step. */
static int visited_3c08(const int32_t* ci, const int32_t* cj, const int32_t* ck, const int32_t n[3]) {
  for (int d = 0; d < 3; ++d) {
    int oj = wrap_off(cj[d] - ci[d], n[d]);
    int ok = wrap_off(ck[d] - ci[d], n[d]);
    int lo = 0, hi = 0;
    if (oj < lo) lo = oj;
    if (oj > hi) hi = oj;
    if (ok < lo) lo = ok;
    if (ok > hi) hi = ok;
    if (hi - lo > 1) return 0;
  }
  return 1;
}

/* 3c18 (Sec. 4, Fig. c18): take the lexicographically smallest of the three
 * cells as base cell C_b; the other two must each be C_b itself or one of its
 * forward neighbours (offset components in {-1,0,1}, lexicographically
 * positive).  Following the worked example (base pair (4,5) pairs with
 * {6,7,8}), both C_n1 and C_n2 are forward neighbours of the base cell. */
static int visited_3c18(const int32_t* ci, const int32_t* cj, const int32_t* ck, const int32_t n[3]) {
  int o[3][3];
  for (int d = 0; d < 3; ++d) {
    o[0][d] = 0;
    o[1][d] = wrap_off(cj[d] - ci[d], n[d]);
    o[2][d] = wrap_off(ck[d] - ci[d], n[d]);
  }
  int m = 0;
  if (lex_less(o[1], o[m])) m = 1;
  if (lex_less(o[2], o[m])) m = 2;
  for (int t = 0; t < 3; ++t) {
    if (t == m) continue;
    int r[3], zero = 1;
    for (int d = 0; d < 3; ++d) {
      r[d] = o[t][d] - o[m][d];
      if (r[d] < -1 || r[d] > 1) return 0;
      if (r[d] != 0) zero = 0;
    }
    (void)zero; /* same cell as the base, or lexicographically after it */
  }
  return 1;
}

/* 3c01 (Sec. 4, Fig. c01): molecule m (cell cm) takes its share of the
 * triplet iff both other molecules lie in cells of m's 27-neighbourhood. */
static inline int visited_3c01(const int32_t* cm, const int32_t* ca, const int32_t* cb, const int32_t n[3]) {
  return cells_adjacent(cm, ca, n) && cells_adjacent(cm, cb, n);
}

/* ------------------------------------------------------------------------ */
/* Brute force: all pairs and all triplets, O(N^3).                          */
/* ------------------------------------------------------------------------ */

/* Full evaluation: forces (N*3, input order), energies, virials (W = sum of
 * r.F, eq. (P_3) for the three-body part) and counts.  n_candidates is the
 * number of molecule triplets the traversal visits regardless of distance
 * (3c01: receiving-molecule incidences), i.e. what eqs. (celltriplet),
 * (twoonetriplets) and (carttriplets) count over the visited cell sets;
 * n_distinct counts every included triplet once (for 3c01, n_triplets counts
 * receiving molecules, up to three per triplet).
 * If wdiag is not NULL it receives the diagonal of the virial tensor,
 * W_aa = sum over the force pairs of r_a F_a (the LJ pairs, and the three
 * force pairs of eq. (forcepairs) of each included triplet, credited like
 * the energy): wdiag[0..2] LJ xx, yy, zz, wdiag[3..5] ATM xx, yy, zz.
 * Returns 0, or -1 on invalid arguments. */
int orc_brute_tensor(const double* pos, int64_t n, const double box[3], const orc_params* p,
                     double* forces, orc_result* res, double* wdiag) {
  int32_t nc[3];
  if (n < 1 || orc_grid(box, p->rc, nc) != 0) return -1;
  int32_t* cx = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)n);
  double* r2 = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  if (!cx || !r2) { free(cx); free(r2); return -1; }
  orc_bin(pos, n, box, nc, cx, NULL);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double d[3];
      min_image(pos + 3 * i, pos + 3 * j, box, d);
      r2[i * n + j] = sqlen(d);
    }
  memset(forces, 0, sizeof(double) * 3 * (size_t)n);
  double rc2 = p->rc * p->rc;
  double e2 = 0, w2 = 0, e3 = 0, w3 = 0;
  double t2x = 0, t2y = 0, t2z = 0, t3x = 0, t3y = 0, t3z = 0;
  int64_t np = 0, nt = 0, ndist = 0, ncand = 0;

  if (p->terms & 1) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i + 1; j < n; ++j) {
        double x = r2[i * n + j];
        if (!(x < rc2) || !cells_adjacent(cx + 3 * i, cx + 3 * j, nc)) continue;
        double d[3], u, f;
        min_image(pos + 3 * i, pos + 3 * j, box, d);
        lj_pair(x, p->eps, p->sigma, &u, &f);
        for (int k = 0; k < 3; ++k) {
          forces[3 * i + k] += f * d[k];
          forces[3 * j + k] -= f * d[k];
        }
        e2 += u;
        w2 += f * x;
        t2x += f * d[0] * d[0];
        t2y += f * d[1] * d[1];
        t2z += f * d[2] * d[2];
        ++np;
      }
  }

  if (p->terms & 2) {
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double* fb = (double*)calloc((size_t)nth * 3 * (size_t)n, sizeof(double));
    if (!fb) { free(cx); free(r2); return -1; }
#pragma omp parallel reduction(+ : e3, w3, nt, ndist, ncand, t3x, t3y, t3z)
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      double* F = fb + (size_t)tid * 3 * (size_t)n;
#pragma omp for schedule(dynamic, 4)
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
          for (int64_t k = j + 1; k < n; ++k) {
            const int32_t *ci = cx + 3 * i, *cj = cx + 3 * j, *ck = cx + 3 * k;
            double x = r2[i * n + j], y = r2[i * n + k], z = r2[j * n + k];
            int recv[3] = {1, 1, 1};
            if (p->variant == 0) {
              if (!visited_3c08(ci, cj, ck, nc)) continue;
              ++ncand;
            } else if (p->variant == 1) {
              if (!visited_3c18(ci, cj, ck, nc)) continue;
              ++ncand;
            } else {
              recv[0] = visited_3c01(ci, cj, ck, nc);
              recv[1] = visited_3c01(cj, ci, ck, nc);
              recv[2] = visited_3c01(ck, ci, cj, nc);
              int nr = recv[0] + recv[1] + recv[2];
              if (nr == 0) continue;
              ncand += nr;
            }
            if (!truncation_ok(x, y, z, p->rc, p->truncation)) continue;
            double rij[3], rik[3], rjk[3], fij[3], fik[3], fjk[3], u, w;
            min_image(pos + 3 * i, pos + 3 * j, box, rij);
            min_image(pos + 3 * i, pos + 3 * k, box, rik);
            min_image(pos + 3 * j, pos + 3 * k, box, rjk);
            atm_force_pairs(rij, rik, rjk, x, y, z, p->nu, fij, fik, fjk, &u, &w);
            int nr = recv[0] + recv[1] + recv[2];
            for (int d = 0; d < 3; ++d) {
              if (recv[0]) F[3 * i + d] += fij[d] + fik[d];
              if (recv[1]) F[3 * j + d] += -fij[d] + fjk[d];
              if (recv[2]) F[3 * k + d] += -fik[d] - fjk[d];
            }
            const double share = (nr == 3) ? 1.0 : (double)nr / 3.0;
            if (nr == 3) {
              e3 += u;
              w3 += w;
            } else {
              e3 += u * (double)nr / 3.0;
              w3 += w * (double)nr / 3.0;
            }
            t3x += share * (rij[0] * fij[0] + rik[0] * fik[0] + rjk[0] * fjk[0]);
            t3y += share * (rij[1] * fij[1] + rik[1] * fik[1] + rjk[1] * fjk[1]);
            t3z += share * (rij[2] * fij[2] + rik[2] * fik[2] + rjk[2] * fjk[2]);
            nt += (p->variant == 2) ? nr : 1;
            ++ndist;
          }
    }
    for (int t = 0; t < nth; ++t)
      for (int64_t q = 0; q < 3 * n; ++q) forces[q] += fb[(size_t)t * 3 * (size_t)n + q];
    free(fb);
  }
  res->e_lj = e2;
  res->w_lj = w2;
  res->e_atm = e3;
  res->w_atm = w3;
  res->n_pairs = np;
  res->n_triplets = nt;
  res->n_candidates = ncand;
  res->n_distinct = ndist;
  if (wdiag) {
    wdiag[0] = t2x;
    wdiag[1] = t2y;
    wdiag[2] = t2z;
    wdiag[3] = t3x;
    wdiag[4] = t3y;
    wdiag[5] = t3z;
  }
  free(cx);
  free(r2);
  return 0;
}

int orc_brute(const double* pos, int64_t n, const double box[3], const orc_params* p,
              double* forces, orc_result* res) {
  return orc_brute_tensor(pos, n, box, p, forces, res, NULL);
}

/* ------------------------------------------------------------------------ */
/* Per-molecule evaluation: the force on each listed molecule, summed over    */
/* every included pair and triplet that contains it.  Same inclusion rules as */
/* orc_brute; the candidate partners of molecule m are the molecules of the   */
/* cells within `reach` cells of m's cell (a necessary condition of every     */
/* visited set: 1 for pairs and pairwise-cutoff triplets, 2 otherwise).      */
/* If `list` is NULL all molecules are evaluated and the totals (energy,     */
/* virial, counts; each pair/triplet credited once) are returned in `res`;   */
/* with a list the totals hold the listed molecules' shares only.            */
/* ------------------------------------------------------------------------ */
int orc_molecules(const double* pos, int64_t n, const double box[3], const orc_params* p,
                  const int64_t* list, int64_t nlist, double* forces, orc_result* res) {
  int32_t nc[3];
  if (n < 1 || orc_grid(box, p->rc, nc) != 0) return -1;
  int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
  int32_t* cx = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)n);
  int32_t* cl = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* start = (int64_t*)calloc((size_t)ncells + 1, sizeof(int64_t));
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!cx || !cl || !start || !order) { free(cx); free(cl); free(start); free(order); return -1; }
  orc_bin(pos, n, box, nc, cx, cl);
  /* bucket the molecules by cell (plain counting sort, input order kept) */
  for (int64_t i = 0; i < n; ++i) start[cl[i] + 1]++;
  for (int64_t c = 0; c < ncells; ++c) start[c + 1] += start[c];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncells);
    memcpy(fill, start, sizeof(int64_t) * (size_t)ncells);
    for (int64_t i = 0; i < n; ++i) order[fill[cl[i]]++] = i;
    free(fill);
  }
  int reach = (p->truncation == 0) ? 1 : 2;
  int64_t count = list ? nlist : n;
  double rc2 = p->rc * p->rc;
  double e2 = 0, w2 = 0, e3 = 0, w3 = 0;
  int64_t np = 0, nt = 0;
  int fail = 0;

#pragma omp parallel reduction(+ : e2, w2, e3, w3, np, nt) reduction(| : fail)
  {
    int64_t cap = 4096;
    int64_t* cand = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < count; ++q) {
      int64_t m = list ? list[q] : q;
      const int32_t* cm = cx + 3 * m;
      double F[3] = {0, 0, 0};
      /* gather candidate partners */
      int64_t nca = 0;
      for (int dz = -reach; dz <= reach; ++dz)
        for (int dy = -reach; dy <= reach; ++dy)
          for (int dx = -reach; dx <= reach; ++dx) {
            int c3[3] = {cm[0] + dx, cm[1] + dy, cm[2] + dz};
            int skip = 0;
            for (int d = 0; d < 3; ++d) {
              int span = 2 * reach + 1;
              if (span > nc[d] && (d == 0 ? dx : (d == 1 ? dy : dz)) != 0) {
                /* small grids: visit each distinct periodic cell once */
                int off = d == 0 ? dx : (d == 1 ? dy : dz);
                int w = wrap_off(off, nc[d]);
                if (w != off) skip = 1;
              }
              c3[d] = ((c3[d] % nc[d]) + nc[d]) % nc[d];
            }
            if (skip) continue;
            int64_t c = ((int64_t)c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
            for (int64_t s = start[c]; s < start[c + 1]; ++s) {
              int64_t j = order[s];
              if (j == m) continue;
              if (nca == cap) {
                cap *= 2;
                cand = (int64_t*)realloc(cand, sizeof(int64_t) * (size_t)cap);
              }
              cand[nca++] = j;
            }
          }
      /* Lennard-Jones pairs containing m */
      if (p->terms & 1) {
        for (int64_t a = 0; a < nca; ++a) {
          int64_t j = cand[a];
          double d[3], u, f;
          min_image(pos + 3 * m, pos + 3 * j, box, d);
          double x = sqlen(d);
          if (!(x < rc2) || !cells_adjacent(cm, cx + 3 * j, nc)) continue;
          lj_pair(x, p->eps, p->sigma, &u, &f);
          for (int k = 0; k < 3; ++k) F[k] += f * d[k];
          if (m < j) {
            e2 += u;
            w2 += f * x;
            ++np;
          }
        }
      }
      /* ATM triplets containing m */
      if (p->terms & 2) {
        /* pairwise cutoff: both partners must be inside rc of m */
        int64_t nuse = nca;
        if (p->truncation == 0) {
          nuse = 0;
          for (int64_t a = 0; a < nca; ++a) {
            double d[3];
            min_image(pos + 3 * m, pos + 3 * cand[a], box, d);
            if (sqlen(d) < rc2) cand[nuse++] = cand[a];
          }
        }
        for (int64_t a = 0; a < nuse; ++a)
          for (int64_t b = a + 1; b < nuse; ++b) {
            int64_t j = cand[a], k = cand[b];
            /* label the triplet i<j<k by input index */
            int64_t t0 = m, t1 = j, t2 = k, tt;
            if (t1 < t0) { tt = t0; t0 = t1; t1 = tt; }
            if (t2 < t1) { tt = t1; t1 = t2; t2 = tt; }
            if (t1 < t0) { tt = t0; t0 = t1; t1 = tt; }
            const int32_t *ci = cx + 3 * t0, *cj = cx + 3 * t1, *ck = cx + 3 * t2;
            int recv[3] = {1, 1, 1};
            if (p->variant == 0) {
              if (!visited_3c08(ci, cj, ck, nc)) continue;
            } else if (p->variant == 1) {
              if (!visited_3c18(ci, cj, ck, nc)) continue;
            } else {
              recv[0] = visited_3c01(ci, cj, ck, nc);
              recv[1] = visited_3c01(cj, ci, ck, nc);
              recv[2] = visited_3c01(ck, ci, cj, nc);
            }
            int me = (m == t0) ? 0 : (m == t1 ? 1 : 2);
            int nr = recv[0] + recv[1] + recv[2];
            if (nr == 0) continue;
            double rij[3], rik[3], rjk[3];
            min_image(pos + 3 * t0, pos + 3 * t1, box, rij);
            min_image(pos + 3 * t0, pos + 3 * t2, box, rik);
            min_image(pos + 3 * t1, pos + 3 * t2, box, rjk);
            double x = sqlen(rij), y = sqlen(rik), z = sqlen(rjk);
            if (!truncation_ok(x, y, z, p->rc, p->truncation)) continue;
            double fij[3], fik[3], fjk[3], u, w;
            atm_force_pairs(rij, rik, rjk, x, y, z, p->nu, fij, fik, fjk, &u, &w);
            if (recv[me]) {
              for (int d = 0; d < 3; ++d) {
                if (me == 0) F[d] += fij[d] + fik[d];
                else if (me == 1) F[d] += -fij[d] + fjk[d];
                else F[d] += -fik[d] - fjk[d];
              }
            }
            if (p->variant == 2) {
              if (recv[me]) {
                e3 += u / 3.0;
                w3 += w / 3.0;
                ++nt;
              }
            } else if (m == t0) {
              e3 += u;
              w3 += w;
              ++nt;
            }
          }
      }
      for (int k = 0; k < 3; ++k) forces[3 * q + k] = F[k];
    }
    free(cand);
  }
  (void)fail;
  res->e_lj = e2;
  res->w_lj = w2;
  res->e_atm = e3;
  res->w_atm = w3;
  res->n_pairs = np;
  res->n_triplets = nt;
  res->n_candidates = -1;
  res->n_distinct = -1;
  free(cx);
  free(cl);
  free(start);
  free(order);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Linked-cell evaluation with Newton's third law over the 3c08 cell sets   */
/* (Sec. 4): the CPU reference of the method's own structure, used to time  */
/* the oracle against the GPU.  Every base cell b takes the 2x2x2 block of  */
/* cells b + o, o in {0,1}^3 (corner code o = ox + 2 oy + 4 oz); a pair or  */
/* triplet of molecules of the block belongs to b iff b is the             */
/* componentwise minimum of its cells, i.e. the AND of the corner codes is */
/* 0, so every pair and triplet of the 3c08 sets is evaluated exactly once */
/* (eqs. celltriplet, twoonetriplets, carttriplets count them).  Pairwise   */
/* cutoff only: under it these sets hold every included triplet.  The       */
/* arithmetic per pair and per triplet is that of orc_brute (minimum image, */
/* eq. ATMGradient term by term, eq. forcepairs, eq. P_3); only the order   */
/* of the force sums differs.  Base cells [b0, b1) only when b1 > b0 (a     */
/* bounded sample for timing: the forces then hold that sample's share).   */
/* Returns 0, or -1 on invalid arguments, the product cutoff, or fewer than */
/* 3 cells per dimension.                                                   */
/* ------------------------------------------------------------------------ */
static int64_t comb2_(int64_t m) { return m * (m - 1) / 2; }
static int64_t comb3_(int64_t m) { return m * (m - 1) * (m - 2) / 6; }

int orc_cells(const double* pos, int64_t n, const double box[3], const orc_params* p,
              int64_t b0, int64_t b1, double* forces, orc_result* res) {
  int32_t nc[3];
  if (n < 1 || p->truncation != 0 || orc_grid(box, p->rc, nc) != 0) return -1;
  for (int d = 0; d < 3; ++d)
    if (nc[d] < 3) return -1;
  const int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
  if (b1 <= b0) { b0 = 0; b1 = ncells; }
  if (b0 < 0 || b1 > ncells) return -1;
  int32_t* cl = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* start = (int64_t*)calloc((size_t)ncells + 1, sizeof(int64_t));
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!cl || !start || !order) { free(cl); free(start); free(order); return -1; }
  orc_bin(pos, n, box, nc, NULL, cl);
  for (int64_t i = 0; i < n; ++i) start[cl[i] + 1]++;
  for (int64_t c = 0; c < ncells; ++c) start[c + 1] += start[c];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncells);
    memcpy(fill, start, sizeof(int64_t) * (size_t)ncells);
    for (int64_t i = 0; i < n; ++i) order[fill[cl[i]]++] = i;
    free(fill);
  }
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  double* fb = (double*)calloc((size_t)nth * 3 * (size_t)n, sizeof(double));
  if (!fb) { free(cl); free(start); free(order); return -1; }
  const double rc2 = p->rc * p->rc;
  double e2 = 0, w2 = 0, e3 = 0, w3 = 0;
  int64_t np = 0, nt = 0, ncand = 0;
  int fail = 0;

#pragma omp parallel reduction(+ : e2, w2, e3, w3, np, nt, ncand) reduction(| : fail)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* F = fb + (size_t)tid * 3 * (size_t)n;
    int64_t cap = 0;
    int64_t* loc = NULL;  /* molecules of the block */
    int* code = NULL;     /* their corner codes     */
    double* dv = NULL;    /* minimum-image r_a - r_b of every ordered pair */
    double* r2 = NULL;    /* its squared length                            */
#pragma omp for schedule(dynamic, 8)
    for (int64_t b = b0; b < b1; ++b) {
      const int bx = (int)(b % nc[0]), by = (int)((b / nc[0]) % nc[1]), bz = (int)(b / ((int64_t)nc[0] * nc[1]));
      int64_t pop[8], m = 0;
      for (int o = 0; o < 8; ++o) {
        int cx = (bx + (o & 1)) % nc[0], cy = (by + ((o >> 1) & 1)) % nc[1], cz = (bz + (o >> 2)) % nc[2];
        int64_t c = ((int64_t)cz * nc[1] + cy) * nc[0] + cx;
        pop[o] = start[c + 1] - start[c];
        m += pop[o];
      }
      /* molecule triplets of the visited cell sets, eqs. (celltriplet),
       * (twoonetriplets), (carttriplets) */
      ncand += comb3_(pop[0]);
      for (int o = 0; o < 8; ++o)
        for (int q = o + 1; q < 8; ++q) {
          if ((o & q) == 0) ncand += pop[q] * comb2_(pop[o]) + pop[o] * comb2_(pop[q]);
          for (int r = q + 1; r < 8; ++r)
            if ((o & q & r) == 0) ncand += pop[o] * pop[q] * pop[r];
        }
      if (m > cap) {
        cap = 2 * m;
        free(loc); free(code); free(dv); free(r2);
        loc = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
        code = (int*)malloc(sizeof(int) * (size_t)cap);
        dv = (double*)malloc(sizeof(double) * 3 * (size_t)cap * (size_t)cap);
        r2 = (double*)malloc(sizeof(double) * (size_t)cap * (size_t)cap);
        if (!loc || !code || !dv || !r2) { fail = 1; cap = 0; continue; }
      }
      m = 0;
      for (int o = 0; o < 8; ++o) {
        int cx = (bx + (o & 1)) % nc[0], cy = (by + ((o >> 1) & 1)) % nc[1], cz = (bz + (o >> 2)) % nc[2];
        int64_t c = ((int64_t)cz * nc[1] + cy) * nc[0] + cx;
        for (int64_t s = start[c]; s < start[c + 1]; ++s) {
          loc[m] = order[s];
          code[m] = o;
          ++m;
        }
      }
      for (int64_t a = 0; a < m; ++a)
        for (int64_t q = a + 1; q < m; ++q) {
          double* d = dv + 3 * (a * m + q);
          min_image(pos + 3 * loc[a], pos + 3 * loc[q], box, d);
          r2[a * m + q] = sqlen(d);
        }
      if (p->terms & 1) {
        for (int64_t a = 0; a < m; ++a)
          for (int64_t q = a + 1; q < m; ++q) {
            const double x = r2[a * m + q];
            if ((code[a] & code[q]) != 0 || !(x < rc2)) continue;
            const double* d = dv + 3 * (a * m + q);
            double u, f;
            lj_pair(x, p->eps, p->sigma, &u, &f);
            for (int k = 0; k < 3; ++k) {
              F[3 * loc[a] + k] += f * d[k];
              F[3 * loc[q] + k] -= f * d[k];
            }
            e2 += u;
            w2 += f * x;
            ++np;
          }
      }
      if (p->terms & 2) {
        for (int64_t a = 0; a < m; ++a)
          for (int64_t q = a + 1; q < m; ++q) {
            const double x = r2[a * m + q];
            if (!(x < rc2)) continue;
            for (int64_t k = q + 1; k < m; ++k) {
              if ((code[a] & code[q] & code[k]) != 0) continue;
              const double y = r2[a * m + k], z = r2[q * m + k];
              if (!truncation_ok(x, y, z, p->rc, 0)) continue;
              double fij[3], fik[3], fjk[3], u, w;
              atm_force_pairs(dv + 3 * (a * m + q), dv + 3 * (a * m + k), dv + 3 * (q * m + k), x, y, z, p->nu,
                              fij, fik, fjk, &u, &w);
              for (int d = 0; d < 3; ++d) {
                F[3 * loc[a] + d] += fij[d] + fik[d];
                F[3 * loc[q] + d] += -fij[d] + fjk[d];
                F[3 * loc[k] + d] += -fik[d] - fjk[d];
              }
              e3 += u;
              w3 += w;
              ++nt;
            }
          }
      }
    }
    free(loc); free(code); free(dv); free(r2);
  }
  memset(forces, 0, sizeof(double) * 3 * (size_t)n);
  for (int t = 0; t < nth; ++t)
    for (int64_t q = 0; q < 3 * n; ++q) forces[q] += fb[(size_t)t * 3 * (size_t)n + q];
  free(fb);
  free(cl);
  free(start);
  free(order);
  res->e_lj = e2;
  res->w_lj = w2;
  res->e_atm = e3;
  res->w_atm = w3;
  res->n_pairs = np;
  res->n_triplets = nt;
  res->n_candidates = ncand;
  res->n_distinct = nt;
  return fail ? -1 : 0;
}

/* Sets the number of OpenMP threads of the oracle's parallel loops. */
void orc_set_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Single-triplet helpers for pinning tests: energy, the three force pairs and
 * the virial of one triplet given the three displacement vectors. */
void orc_triplet(const double rij[3], const double rik[3], const double rjk[3], double nu,
                 double fi[3], double fj[3], double fk[3], double* u, double* w) {
  double fij[3], fik[3], fjk[3];
  double x = sqlen(rij), y = sqlen(rik), z = sqlen(rjk);
  atm_force_pairs(rij, rik, rjk, x, y, z, nu, fij, fik, fjk, u, w);
  for (int d = 0; d < 3; ++d) {
    fi[d] = fij[d] + fik[d];
    fj[d] = -fij[d] + fjk[d];
    fk[d] = -fik[d] - fjk[d];
  }
}

/* Visited-set predicate exposed for tests: variant 0/1 return 0/1 for the
 * triplet; variant 2 returns a 3-bit mask of receiving molecules. */
int orc_visited(const int32_t* ci, const int32_t* cj, const int32_t* ck, const int32_t n[3], int variant) {
  if (variant == 0) return visited_3c08(ci, cj, ck, n);
  if (variant == 1) return visited_3c18(ci, cj, ck, n);
  return visited_3c01(ci, cj, ck, n) | (visited_3c01(cj, ci, ck, n) << 1) |
         (visited_3c01(ck, ci, cj, n) << 2);
}
