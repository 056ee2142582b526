// Device-side layout of the grouped operator and the configuration spaces.
#pragma once

#include <memory>

#include "host_plan.h"
#include "pbs_internal.h"

// Operator grouped by X-mask (Eq. topological_group) plus the tables of the
// spin-sector kernel.
//
// CSR form (full-space kernel): group g has mask xg[g] and terms
// off[g]..off[g+1]-1 with Z-masks zk[] and XZ-form coefficients ck[] (re, im).
//
// Sector form (n_qubits even, split at h = n_qubits/2 into alpha = low half,
// beta = high half).  Terms are ordered by (X_alpha, popcount(X_beta),
// X_beta, z_beta', z_alpha):
//   class c      : distinct X_alpha, groups cls_g0[c]..cls_g0[c+1]-1; the
//                  group with X_beta = 0 (if any) is cls_zg[c], the groups
//                  with popcount(X_beta) = 2 are cls_p0[c]..cls_p1[c]-1 and
//                  cls_pm[c] is their row in the pair map (or -1)
//   group g      : X_beta = pg_xb[g], uniques pg_u0[g]..pg_u0[g+1]-1
//   unique u     : beta Z-mask u_zb[u], terms u_t0[u]..u_t0[u+1]-1
//   term t       : alpha Z-mask pt_za[t], coefficient pt_c[t] (re, im)
//   pair map     : pmap[cls_pm[c] * n_pairs + pair(p, q)] = group with
//                  X_beta = {p, q} in class c, or -1; pair(p, q) = q(q-1)/2 + p
//                  for p < q
//   quad map     : qmap[cls_qm[c] * n_quads + quad(X_beta)] = group with that
//                  four-orbital X_beta in class c, or -1; quad(X) is the
//                  colexicographic rank sum_j C(b_j, j + 1) of X's bits
//                  b_0 < b_1 < b_2 < b_3 (built when C(h, 4) <= kMaxQuads)
// Exact rewrites valid inside any fixed-(N_alpha, N_beta) sector:
//  * a term whose X_alpha or X_beta has odd popcount never maps a sector
//    configuration into the sector and is removed;
//  * a sector-preserving move with mask X flips exactly |X|/2 set bits of
//    both the source s and the target t = s ^ X, so
//    (-1)^popcount(z & s) = (-1)^(|X|/2) (-1)^popcount((z ^ X) & s): z_beta
//    is replaced by whichever of z_beta, z_beta ^ X_beta lacks X_beta's
//    lowest bit, with the sign moved into the coefficient;
//  * (-1)^popcount(z & s) = (-1)^popcount(z & X) (-1)^popcount(z & t), so
//    the constant factor (-1)^popcount(z & X) of both halves is moved into the
//    coefficient and the kernel evaluates parities against the target
//    strings, which each thread already holds.
// Terms with equal z_beta' share one unique entry, whose alpha parities are
// folded per target row at run time.
namespace pbs {
// Per-class record read by the sector kernel in one load.
struct ClassMeta {
  uint32_t xa;      // X_alpha of the class
  uint32_t g0, g1;  // its groups
  int32_t zg;       // the X_beta = 0 group, or -1
  uint32_t p1;      // end of the popcount-2 groups (they start after zg)
  int32_t pm;       // pair-map row, or -1
  uint32_t ua;      // first unique of the class
  uint32_t u_z;     // end of the X_beta = 0 group's uniques
  uint32_t u_p;     // end of the pair groups' uniques
  uint32_t u_end;   // end of the class's uniques
  uint32_t flags;   // kClassSimple | kClassPairsSingle
  uint32_t q1;      // end of the popcount-4 groups (they start at p1)
  int32_t qm;       // quad-map row, or -1
  uint32_t u_q;     // end of the quad groups' uniques
  uint32_t pad[2];
};
constexpr uint32_t kClassSimple = 1u;       // only an X_beta = 0 group, few uniques
constexpr uint32_t kClassPairsSingle = 2u;  // every pair group has exactly one unique
constexpr uint32_t kSimpleCap = 64;         // uniques of a "simple" class
constexpr uint32_t kMaxQuads = 2048;        // largest C(h, 4) given a quad map (h <= 16)

// Spin-factorized phase evaluation of one beta sector (Section 2.4,
// Eqs. svd_weights, precomp_alpha, precomp_beta, svd_sreverse_sum and
// dot_product; Algorithm grouped_hvec).  A group's coefficients in sector
// form make a matrix M[mu][nu] over its distinct alpha Z-masks (rows) and
// its uniques (columns, beta Z-masks); with a rank-R factorization M = P Q
// its phase sum at target (t_a, t_b) is sum_r A_r(t_a) F_r(t_b), where
//   A_r = sum_mu P[mu][r] (-1)^popcount(Za_mu & t_a)   ("factor uniques",
//         folded per workgroup like the unfactored uniques), and
//   F_r = sum_nu Q[r][nu] (-1)^popcount(Zb_nu & t_b)   (precomputed here for
//         every beta string of the sector).
// Factored groups: the X_beta = 0 group of every non-simple class (tables
// fz, one per class and rank, indexed by beta column), and the pair and quad
// groups of the class with X_alpha = 0 (tables indexed by the target's move:
// em/fp for its single moves, eq/fq for its double moves).  Real
// coefficients only.
struct FactorPlan {
  uint32_t n_orb = 0, n_beta = 0;  // the beta sector the tables are for
  uint64_t dim_beta = 0;
  uint32_t n_fu = 0, n_ft = 0;     // factor uniques and their terms
  DevBuf<uint32_t> fu_t0;          // [n_fu + 1]
  DevBuf<uint32_t> ft_za;          // [n_ft] alpha Z-mask (sector form)
  DevBuf<double> ft_c;             // [n_ft] P[mu][r]
  // per class: first factor unique of its X_beta = 0 group, rank (0 = not
  // factored), offset of its fz rows (in doubles), 0
  DevBuf<uint4> cls_f;
  DevBuf<double> fz;
  uint32_t max_r1 = 0;
  // the X_alpha = 0 class (c0 < n_class when its pair and quad groups are factored)
  uint32_t c0 = 0xffffffffu;
  uint32_t c0_fu0 = 0, c0_fq = 0, c0_fu1 = 0;  // its pair-group, then quad-group factor uniques
  uint32_t t_zero = 0, t_pair = 0, t_quad = 0;  // most terms of one factor unique, per kind
  uint32_t r2 = 0, r3 = 0;          // rank of every factored pair / quad group (padded with zeros)
  uint32_t n_moves = 0, n_qmoves = 0;
  DevBuf<uint32_t> em;   // [n_moves][dim_beta]: source column | (4 + factor offset, or 0) << 16
  DevBuf<double> fp;     // [n_moves][r2][dim_beta]
  DevBuf<uint32_t> eq;   // [n_qmoves][dim_beta]: source column | (4 + factor offset, or 0) << 16
  DevBuf<double> fq;     // [n_qmoves][r3][dim_beta]
  // ranks found (for reporting): groups factored per kind and the largest rank
  uint32_t n_f1 = 0, n_f2 = 0, n_f3 = 0;
  // Alpha side of the alpha sector N_alpha (Eq. precomp_alpha) for the
  // simple classes (one X_beta = 0 group whose uniques all have beta Z-mask
  // 0, so a target's phase sum for the class depends on t_alpha alone):
  // for alpha row i, entries alist_off[i] .. alist_off[i + 1] - 1 hold, in
  // class order, the source row rank of every simple class whose source
  // lies in the sector and the class's folded coefficient at t_alpha.
  uint32_t n_alpha = 0;
  bool alist = false;
  DevBuf<uint32_t> alist_off;  // [dim_alpha + 1]
  DevBuf<uint32_t> alist_src;
  DevBuf<double> alist_c;
  // Alpha side of the "image" classes (X_beta = 0 group factored with rank
  // <= 2 or absent, every other group a single-unique pair group): for alpha
  // row i, entries plist_off[i] .. plist_off[i + 1] - 1 list, in class order,
  // the image classes whose source lies in the sector (source row rank,
  // class), and entry e's image pimg[e * n_img ..] holds the folded
  // coefficient of the class's pair group for each orbital pair (0 when
  // absent), a 0 for padding moves, then the X_beta = 0 group's folded
  // factors A_0, A_1.
  bool plist = false;
  uint32_t n_img = 0;
  DevBuf<uint32_t> plist_off, plist_src, plist_cls;
  DevBuf<double> pimg;
  DevBuf<uint32_t> pimg_flag;  // [n_class]: 1 for image classes
  // the operator's non-simple classes without the X_alpha = 0 class (when
  // its tables exist), without the image classes, and without both
  std::vector<uint32_t> ns_sizes;  // [3]
  DevBuf<uint32_t> ns_rest[3];
  // sizes for the rows kernel: longest alpha list, and the uniques and
  // groups of all non-simple classes
  uint32_t alist_max = 0, ns_uniques = 0, ns_groups = 0;
};
}  // namespace pbs

struct pbs_grouped {
  uint32_t n_qubits = 0;
  uint64_t n_groups = 0;
  uint64_t n_terms = 0;
  pbs::DevBuf<uint64_t> xg;
  pbs::DevBuf<uint32_t> off;
  pbs::DevBuf<uint64_t> zk;
  pbs::DevBuf<double> ck;

  bool has_sector = false;
  uint32_t half = 0;
  uint32_t n_class = 0, n_pgroup = 0, n_unique = 0, n_pterm = 0;
  uint32_t n_pairs = 0, n_pmap = 0;
  uint32_t n_quads = 0, n_qmap = 0;
  uint32_t max_quad_uniques = 0;  // largest u_q - u_p over classes with a quad-map row
  pbs::DevBuf<uint32_t> cls_xa, cls_g0;
  pbs::DevBuf<int32_t> cls_zg, cls_p0, cls_p1, cls_pm, pmap;
  pbs::DevBuf<int32_t> cls_q1, cls_qm, qmap;
  pbs::DevBuf<uint32_t> pg_pc;  // popcount(X_beta) of each group
  pbs::DevBuf<pbs::ClassMeta> cls_meta;
  // class schedule of the sector kernel: maximal runs of consecutive simple
  // classes as (first, end) pairs, then the other classes in order
  uint32_t n_runs = 0, n_ns = 0;
  pbs::DevBuf<uint32_t> runs, ns_list;
  uint32_t quad_cnt = 0;  // uniques of every mapped quad group when all are equal, else 0
  // When every pair group of every kClassPairsSingle class has the beta
  // Z-mask zpair[pair(p, q)] (a function of its two orbitals only, as for
  // Jordan-Wigner strings), the kernel evaluates each move's beta parity
  // once per target instead of once per class.
  bool pair_sign = false;
  pbs::DevBuf<uint32_t> zpair;
  pbs::DevBuf<uint32_t> pg_xb, pg_u0;
  pbs::DevBuf<uint32_t> u_zb, u_t0;
  pbs::DevBuf<uint32_t> pt_za;
  pbs::DevBuf<double> pt_c;
  bool real_coef = false;  // every sector-form coefficient has a zero imaginary part
  // spin-factorized evaluation of one beta sector (pbs_grouped_factor) and
  // whether applies use it
  std::unique_ptr<pbs::FactorPlan> fplan;
  uint32_t fact_on = 7u;  // which factored parts applies use (pbs_grouped_set_factored)
};

// Full space (D = 2^n) or spin sector.
struct pbs_space {
  bool sector = false;
  uint32_t n_qubits = 0;
  uint64_t dim = 0;
  uint32_t n_orb = 0, n_alpha = 0, n_beta = 0;
  uint64_t dim_alpha = 0, dim_beta = 0;
  uint32_t n_chunks = 0;              // 8-bit chunks of an n_orb-bit spin string
  pbs::DevBuf<uint32_t> str_alpha;    // [dim_alpha] ascending
  pbs::DevBuf<uint32_t> str_beta;     // [dim_beta] ascending
  // rank_tab[(c * (n_orb + 1) + k) * 256 + b]: contribution of byte b of chunk c
  // to the combinatorial rank when k ones lie below the chunk.
  pbs::DevBuf<uint32_t> rank_tab;
  // the same tables as uint16 when n_orb <= 16 (every entry is below 2^16)
  pbs::DevBuf<uint16_t> rank_tab16;
};

namespace pbs {
uint64_t host_binom(uint32_t n, uint32_t r);  // exact binomial coefficient (space.hip)

inline size_t rank_tab_entries(uint32_t n_orb) {
  return static_cast<size_t>((n_orb + 7) / 8) * (n_orb + 1) * 256;
}
}  // namespace pbs
