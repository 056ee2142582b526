/* Plain C float64 twin of the oracle's operator-state product (oracle/apply.py).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; it is compiled into its own shared object for the tests, the
 * smoke check and the CPU-baseline leg of the benchmark.  It includes no
 * header of the HIP library and shares no table or helper with it.
 *
 * What it computes is the plain definition of H|psi> for H = sum_k c_k P_k
 * with letter-form strings (Section 2.2): a string with X-or-Y positions
 * `flip`, Y-or-Z positions `sign` and n_y letters Y acts on a basis state as
 *
 *     P |s> = i^n_y (-1)^popcount(s & sign) |s xor flip>,
 *
 * letter by letter (X|b> = |1-b>, Y|b> = i(-1)^b|1-b>, Z|b> = (-1)^b|b>).
 * Two evaluation orders are provided, both ungrouped and term by term:
 *   - scatter (the source-driven form of Section 2.4): every source s of a
 *     list adds c_k P_k psi_s to out[s xor flip_k] for every term k;
 *   - targets (Eq. reverse_sum without the grouping): a selected target t
 *     gathers sum_k c_k i^n_y (-1)^popcount(s_k & sign_k) psi[s_k] with
 *     s_k = t xor flip_k.
 * In a spin sector (Section 2.4, spin-resolved product basis) sources and
 * targets outside the sector are dropped (the projection P H P psi).  A
 * configuration's index is found by lookup in position tables that the
 * caller builds from the explicitly enumerated ascending spin strings, never
 * by a combinatorial rank formula.  All arithmetic is float64; threads
 * (OpenMP) split sources or targets, and the scatter sums the per-thread
 * partial vectors in thread order.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Configuration space: the full space of n_qubits (index = bit pattern), or
 * the (N_alpha, N_beta) sector of n_orb orbitals, alpha = qubits 0..n_orb-1,
 * beta = n_orb..2 n_orb-1, index = pos_a[alpha] * dim_b + pos_b[beta]. */
typedef struct {
  int32_t sector;          /* 0: full space, 1: spin sector */
  int32_t n_bits;          /* full: n_qubits; sector: n_orb */
  uint64_t dim;            /* number of configurations */
  uint64_t dim_b;          /* sector: number of beta strings */
  const int32_t* pos_a;    /* sector: 2^n_orb entries, position of an alpha string or -1 */
  const int32_t* pos_b;    /* sector: same for beta strings */
  const uint64_t* str_a;   /* sector: alpha strings, ascending */
  const uint64_t* str_b;   /* sector: beta strings, ascending */
} orc_space;

static inline int64_t index_of(const orc_space* sp, uint64_t bits) {
  if (!sp->sector) return bits < sp->dim ? (int64_t)bits : -1;
  const uint64_t mask = (1ull << sp->n_bits) - 1ull;
  const uint64_t hi = bits >> sp->n_bits;
  if (hi > mask) return -1;
  const int32_t ia = sp->pos_a[bits & mask], ib = sp->pos_b[hi];
  if (ia < 0 || ib < 0) return -1;
  return (int64_t)ia * (int64_t)sp->dim_b + ib;
}

static inline uint64_t bits_of(const orc_space* sp, uint64_t index) {
  if (!sp->sector) return index;
  return sp->str_a[index / sp->dim_b] | (sp->str_b[index % sp->dim_b] << sp->n_bits);
}

/* c_k i^n_y as (re, im) pairs */
static double* term_factors(uint64_t n_terms, const uint8_t* n_y, const double* coeff) {
  double* f = (double*)malloc(2 * (n_terms ? n_terms : 1) * sizeof(double));
  if (!f) return NULL;
  for (uint64_t k = 0; k < n_terms; ++k) {
    double re = coeff[2 * k], im = coeff[2 * k + 1];
    for (int r = 0; r < (n_y[k] & 3); ++r) { /* multiply by i */
      const double t = re;
      re = -im;
      im = t;
    }
    f[2 * k] = re;
    f[2 * k + 1] = im;
  }
  return f;
}

static int threads_for(int n_threads) { return n_threads > 0 ? n_threads : omp_get_max_threads(); }

/* out[t] = sum over the listed sources s (all of the space when src is NULL)
 * and every term k with t = s xor flip_k in the space of c_k P_k psi_s.
 * out holds dim interleaved (re, im) float64 pairs and is overwritten.
 * Returns 0, or -1 when memory runs out; *used = threads used. */
int orc_apply_scatter(const orc_space* sp, uint64_t n_terms, const uint64_t* flip, const uint64_t* sign,
                      const uint8_t* n_y, const double* coeff, const double* psi, uint64_t n_src,
                      const int64_t* src, double* out, int n_threads, int* used) {
  const int nt = threads_for(n_threads);
  const uint64_t n = src ? n_src : sp->dim;
  double* fac = term_factors(n_terms, n_y, coeff);
  double** part = (double**)calloc((size_t)nt, sizeof(double*));
  if (!fac || !part) {
    free(fac);
    free(part);
    return -1;
  }
  int fail = 0;
  for (int i = 0; i < nt; ++i) {
    part[i] = i == 0 ? out : (double*)malloc(2 * sp->dim * sizeof(double));
    if (!part[i]) fail = 1;
  }
  if (!fail) {
#pragma omp parallel num_threads(nt)
    {
      const int me = omp_get_thread_num();
      double* acc = part[me];
      memset(acc, 0, 2 * sp->dim * sizeof(double));
      const uint64_t lo = n * (uint64_t)me / (uint64_t)nt, hi = n * (uint64_t)(me + 1) / (uint64_t)nt;
      for (uint64_t j = lo; j < hi; ++j) {
        const uint64_t si = src ? (uint64_t)src[j] : j;
        const uint64_t s = bits_of(sp, si);
        const double pr = psi[2 * si], pi = psi[2 * si + 1];
        if (pr == 0.0 && pi == 0.0) continue;
        for (uint64_t k = 0; k < n_terms; ++k) {
          const int64_t ti = index_of(sp, s ^ flip[k]);
          if (ti < 0) continue;
          const double sg = (__builtin_popcountll(s & sign[k]) & 1) ? -1.0 : 1.0;
          const double fr = sg * fac[2 * k], fi = sg * fac[2 * k + 1];
          acc[2 * ti] += fr * pr - fi * pi;
          acc[2 * ti + 1] += fr * pi + fi * pr;
        }
      }
    }
    for (int i = 1; i < nt; ++i)
      for (uint64_t t = 0; t < 2 * sp->dim; ++t) out[t] += part[i][t];
  }
  for (int i = 1; i < nt; ++i) free(part[i]);
  free(part);
  free(fac);
  if (used) *used = nt;
  return fail ? -1 : 0;
}

/* out[j] = (P H P psi)[tgt[j]] for n_tgt selected targets, each summed over
 * the terms in their order.  out holds n_tgt interleaved pairs. */
int orc_apply_targets(const orc_space* sp, uint64_t n_terms, const uint64_t* flip, const uint64_t* sign,
                      const uint8_t* n_y, const double* coeff, const double* psi, uint64_t n_tgt,
                      const int64_t* tgt, double* out, int n_threads, int* used) {
  const int nt = threads_for(n_threads);
  double* fac = term_factors(n_terms, n_y, coeff);
  if (!fac) return -1;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64)
  for (uint64_t j = 0; j < n_tgt; ++j) {
    const uint64_t t = bits_of(sp, (uint64_t)tgt[j]);
    double ar = 0.0, ai = 0.0;
    for (uint64_t k = 0; k < n_terms; ++k) {
      const uint64_t s = t ^ flip[k];
      const int64_t si = index_of(sp, s);
      if (si < 0) continue;
      const double sg = (__builtin_popcountll(s & sign[k]) & 1) ? -1.0 : 1.0;
      const double fr = sg * fac[2 * k], fi = sg * fac[2 * k + 1];
      const double pr = psi[2 * si], pi = psi[2 * si + 1];
      ar += fr * pr - fi * pi;
      ai += fr * pi + fi * pr;
    }
    out[2 * j] = ar;
    out[2 * j + 1] = ai;
  }
  free(fac);
  if (used) *used = nt;
  return 0;
}
