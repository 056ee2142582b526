// Host-side planning that needs no device: the sector kernel's LDS layout,
// the rank-revealing factorization of a group's sector-form coefficients
// (Section 2.4, Eq. svd_weights) and the work list of a batched launch.
// Plain C++17 with no HIP header, so that the same code also builds with the
// host compiler under AddressSanitizer and UndefinedBehaviorSanitizer.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace pbs {

// ------------------------------------------------------ sector LDS layout
constexpr int kMaxMoves = 56;         // pair moves cached per lane (N_beta (n_orb - N_beta) <= 56)
constexpr uint32_t kRowCapBytes = 64u * 1024u;
constexpr uint32_t kListMinBytes = 4096u;  // simple-class row list when no row is staged
// LDS copy of the uint16 rank tables (n_orb <= 16): chunk 0 with no ones
// below it, then chunk 1 for 0..8 ones below it (zeros when n_orb <= 8)
constexpr uint32_t kRank16Lds = 10u * 256u;
// Fixed LDS placement (the kernel declares no static LDS, so these are
// absolute addresses): workgroup scratch at byte 0, the pair map at kPuOff
// (an 8-byte slot per orbital pair, at most C(32, 2) + 1 entries) and the
// staged row at kRowOff, so per-move addresses need no base register.
constexpr uint32_t kMiscBytes = 256;  // ballot counts and the energy reduction
constexpr uint32_t kPuOff = kMiscBytes;
constexpr uint32_t kPuBytes = 4096;
constexpr uint32_t kRowOff = kPuOff + kPuBytes;
constexpr uint32_t kZeroSlots = 4;     // zero entries after the folded uniques (absent groups, padding)
constexpr uint32_t kFCapMin = 1024;    // folded uniques: smallest LDS capacity planned for
constexpr uint32_t kFCapMax = 4096;    // and the largest (offsets are packed in 16 bits)
constexpr uint32_t kMaxR1 = 32;        // largest factored rank of an X_beta = 0 group
constexpr uint32_t kFactZeroSlots = 4;  // zero factors at the start of the class-0 fold

inline uint32_t align16(uint32_t v) { return (v + 15u) & ~15u; }

// What the layout depends on: the device's LDS per workgroup (less the
// static arrays), the sector, the amplitude size and the operator's table
// sizes.
struct SectorLayoutIn {
  uint32_t lds_limit = 0;
  uint32_t n_orb = 0, n_beta = 0;
  uint64_t dim_beta = 0;
  uint32_t elem_bytes = 8;
  bool realc = true;      // real coefficients (8-byte folded uniques)
  bool allow_row = true;  // a source row may be staged whole
  bool allow_enum = true, allow_qenum = true;
  uint64_t n_pmap = 0, n_qmap = 0;  // pair and quad map entries (0: no map)
  uint32_t n_pairs = 0, n_quads = 0, max_quad_uniques = 0;
  bool a_region = false;  // folded factors of an X_beta = 0 group need a place
};

// Byte offsets of every region and the choices that decide them.  Regions:
// [0, kMiscBytes) scratch, [kPuOff, kPuOff + kPuBytes) pair map (the X_beta
// = 0 factors at off_a inside it when they fit), [kRowOff, kRowOff +
// row_region) staged row or row list, then rank tables, folded uniques,
// their Z-masks, the quad map and, when not in the pair map, the X_beta = 0
// factors; lds is the end of the last region.
struct SectorLayout {
  bool r16 = false, enum_ok = false, qenum_ok = false, row_lds = false;
  uint32_t n_moves = 0, n_qmoves = 0, list_cap = 0, f_cap = 0;
  uint32_t row_region = 0, rank_bytes = 0, off_rank = 0, off_f = 0, f_bytes = 0, off_fz = 0, fz_bytes = 0;
  uint32_t off_qu = 0, qu_bytes = 0, off_a = 0, a_bytes = 0, lds = 0;
  bool a_in_pair_map = false;
};

// Returns false when the operator's orbital pairs do not fit the pair map.
// The folded uniques get what is left of half the LDS, so that two
// workgroups share a compute unit, unless the fixed parts alone need more.
inline bool sector_layout(const SectorLayoutIn& in, SectorLayout* out) {
  SectorLayout L;
  if (in.n_pairs + 1u > kPuBytes / 8u) return false;
  const uint32_t limit = in.lds_limit;
  const uint32_t half = limit / 2u - 512u;
  L.r16 = in.n_orb <= 16;
  L.rank_bytes = L.r16 ? align16(kRank16Lds * 2u) : 0u;
  const uint32_t per_unique = (in.realc ? 8u : 16u) + 4u;
  const uint32_t f_min = (kFCapMin + kZeroSlots) * per_unique + 64u;
  L.n_moves = in.n_beta * (in.n_orb - in.n_beta);
  L.enum_ok = in.allow_enum && in.n_pmap > 0 && L.n_moves <= static_cast<uint32_t>(kMaxMoves) &&
              in.dim_beta < 65536 && in.n_pairs < 65536;
  const uint32_t pu_bytes = kMiscBytes + kPuBytes;
  auto pairs = [](uint64_t m) { return m < 2 ? uint64_t{0} : m * (m - 1) / 2; };
  const uint64_t n_ep = pairs(in.n_orb - in.n_beta), n_op = pairs(in.n_beta);
  L.qenum_ok = in.allow_qenum && L.r16 && L.enum_ok && in.n_qmap > 0 && in.n_quads > 0 && n_op * n_ep > 0;
  L.n_qmoves = static_cast<uint32_t>(n_op * n_ep);
  const uint64_t row_bytes = in.dim_beta * in.elem_bytes;
  const uint64_t row_space = row_bytes > kListMinBytes ? row_bytes : kListMinBytes;
  L.row_lds = in.allow_row && row_bytes <= kRowCapBytes && L.rank_bytes + f_min + pu_bytes + row_space <= limit;
  L.row_region = align16(static_cast<uint32_t>(L.row_lds ? row_space : kListMinBytes));
  L.list_cap = L.row_region / 8u;
  // The double-move phase needs its quad map and every quad unique of a
  // class in LDS at once; it is kept only if that still lets two workgroups
  // share a compute unit (or if two never fit anyway).
  const uint32_t base_fixed = L.rank_bytes + L.row_region + pu_bytes;
  const uint32_t qu_need = align16(in.n_quads * 4u);
  const uint32_t q_need = (in.max_quad_uniques + kZeroSlots) * per_unique + 64u;
  if (L.qenum_ok) {
    const bool two_without = base_fixed + f_min <= half;
    const uint32_t cap = two_without ? half : limit;
    if (base_fixed + qu_need + std::max(q_need, f_min) > cap || in.max_quad_uniques >= kFCapMax) L.qenum_ok = false;
  }
  L.qu_bytes = L.qenum_ok ? qu_need : 0u;
  // the folded factors of an X_beta = 0 group sit after the pair map when
  // its fixed region has room (n_orb <= 16), else in a region of their own
  const uint32_t a_in_pu = align16((in.n_pairs + 1u) * 8u);
  L.a_in_pair_map = a_in_pu + kMaxR1 * 8u <= kPuBytes;
  L.a_bytes = (in.a_region && !L.a_in_pair_map) ? align16(kMaxR1 * 8u) : 0u;
  const uint32_t fixed = base_fixed + L.qu_bytes + L.a_bytes;
  const uint32_t budget = fixed + f_min <= half ? half : limit;
  L.f_cap = std::min(kFCapMax, (budget - fixed - 64u) / per_unique - kZeroSlots);
  uint32_t off = kRowOff + L.row_region;
  L.off_rank = off;
  off += L.rank_bytes;
  L.off_f = off;
  L.f_bytes = align16((L.f_cap + kZeroSlots) * (per_unique - 4u));
  off += L.f_bytes;
  L.off_fz = off;
  L.fz_bytes = align16((L.f_cap + kZeroSlots) * 4u);
  off += L.fz_bytes;
  L.off_qu = off;
  off += L.qu_bytes;
  L.off_a = L.a_in_pair_map ? kPuOff + a_in_pu : off;
  off += L.a_bytes;
  L.lds = off;
  *out = L;
  return true;
}

// ------------------------------------------- spin-factorized coefficients
// M = P Q by pivoted Gram-Schmidt on the rows of M (rows x cols, row-major):
// the next basis vector is the remaining row of largest norm, orthogonalised
// twice against the basis; stops when every remaining row is below
// rtol * (largest row norm of M).  Q (rank x cols, orthonormal rows) is
// returned through the argument, the rank as the result.
inline uint32_t factor_rows(const std::vector<double>& M, uint32_t rows, uint32_t cols, double rtol,
                            std::vector<double>& Q) {
  std::vector<double> res = M;
  Q.clear();
  double scale = 0.0;
  for (uint32_t i = 0; i < rows; ++i) {
    double s = 0.0;
    for (uint32_t j = 0; j < cols; ++j) s += M[static_cast<size_t>(i) * cols + j] * M[static_cast<size_t>(i) * cols + j];
    scale = std::max(scale, std::sqrt(s));
  }
  if (scale == 0.0) return 0;
  uint32_t r = 0;
  std::vector<double> q(cols);
  while (r < rows && r < cols) {
    uint32_t best = 0;
    double bn = -1.0;
    for (uint32_t i = 0; i < rows; ++i) {
      double s = 0.0;
      for (uint32_t j = 0; j < cols; ++j)
        s += res[static_cast<size_t>(i) * cols + j] * res[static_cast<size_t>(i) * cols + j];
      if (s > bn) {
        bn = s;
        best = i;
      }
    }
    if (std::sqrt(bn) <= rtol * scale) break;
    for (uint32_t j = 0; j < cols; ++j) q[j] = res[static_cast<size_t>(best) * cols + j];
    for (int pass = 0; pass < 2; ++pass) {
      for (uint32_t k = 0; k < r; ++k) {
        double d = 0.0;
        for (uint32_t j = 0; j < cols; ++j) d += q[j] * Q[static_cast<size_t>(k) * cols + j];
        for (uint32_t j = 0; j < cols; ++j) q[j] -= d * Q[static_cast<size_t>(k) * cols + j];
      }
      double nn = 0.0;
      for (uint32_t j = 0; j < cols; ++j) nn += q[j] * q[j];
      nn = std::sqrt(nn);
      for (uint32_t j = 0; j < cols; ++j) q[j] /= nn;
    }
    Q.insert(Q.end(), q.begin(), q.end());
    ++r;
    for (uint32_t i = 0; i < rows; ++i) {
      double d = 0.0;
      for (uint32_t j = 0; j < cols; ++j) d += res[static_cast<size_t>(i) * cols + j] * q[j];
      for (uint32_t j = 0; j < cols; ++j) res[static_cast<size_t>(i) * cols + j] -= d * q[j];
    }
  }
  return r;
}

// The sector-form tables of the groups on the host: group g's uniques are
// [pg_u0[g], pg_u0[g + 1]); unique u has beta Z-mask u_zb[u] and terms
// [u_t0[u], u_t0[u + 1]) with alpha Z-masks pt_za and real coefficients pt_c.
struct HostTables {
  std::vector<uint32_t> pg_u0, u_zb, u_t0, pt_za, pg_xb;
  std::vector<double> pt_c;
};

// One group's factors: for each r, the alpha terms (Za, P[mu][r]) and the
// beta list (Zb, Q[r][nu]); exact zeros are left out.
struct GroupFactors {
  uint32_t rank = 0;
  uint32_t n_uniques = 0;
  std::vector<std::vector<std::pair<uint32_t, double>>> a, b;
};

inline GroupFactors factor_group(const HostTables& T, uint32_t g, double rtol = 1e-14) {
  GroupFactors F;
  const uint32_t u0 = T.pg_u0[g], u1 = T.pg_u0[g + 1];
  F.n_uniques = u1 - u0;
  // rows: the distinct alpha Z-masks, ascending
  std::vector<uint32_t> za(T.pt_za.begin() + T.u_t0[u0], T.pt_za.begin() + T.u_t0[u1]);
  std::sort(za.begin(), za.end());
  za.erase(std::unique(za.begin(), za.end()), za.end());
  auto row_of = [&](uint32_t z) {
    return static_cast<uint32_t>(std::lower_bound(za.begin(), za.end(), z) - za.begin());
  };
  const uint32_t nr = static_cast<uint32_t>(za.size()), nc = u1 - u0;
  std::vector<double> M(static_cast<size_t>(nr) * nc, 0.0);
  for (uint32_t u = u0; u < u1; ++u)
    // terms whose beta Z-masks differ by X_beta share one unique in sector
    // form and may share an alpha Z-mask too: their coefficients add
    for (uint32_t t = T.u_t0[u]; t < T.u_t0[u + 1]; ++t)
      M[static_cast<size_t>(row_of(T.pt_za[t])) * nc + (u - u0)] += T.pt_c[t];
  std::vector<double> Q;
  F.rank = factor_rows(M, nr, nc, rtol, Q);
  F.a.resize(F.rank);
  F.b.resize(F.rank);
  for (uint32_t r = 0; r < F.rank; ++r) {
    for (uint32_t mu = 0; mu < nr; ++mu) {
      double p = 0.0;
      for (uint32_t nu = 0; nu < nc; ++nu) p += M[static_cast<size_t>(mu) * nc + nu] * Q[static_cast<size_t>(r) * nc + nu];
      if (p != 0.0) F.a[r].emplace_back(za[mu], p);
    }
    for (uint32_t nu = 0; nu < nc; ++nu)
      if (Q[static_cast<size_t>(r) * nc + nu] != 0.0) F.b[r].emplace_back(T.u_zb[u0 + nu], Q[static_cast<size_t>(r) * nc + nu]);
  }
  return F;
}

// ------------------------------------------------- batched launch work list
// Jobs in launch order (largest cost first, ties in the caller's order,
// unless the caller fixed the order) and each job's first work item in that
// order; total = all items.
struct BatchPlan {
  std::vector<uint32_t> order;
  std::vector<uint64_t> base;  // indexed by launch position
  uint64_t total = 0;
};

inline BatchPlan batch_plan(const std::vector<double>& cost, const std::vector<uint64_t>& items, bool keep_order) {
  BatchPlan B;
  const size_t n = cost.size();
  B.order.resize(n);
  for (size_t i = 0; i < n; ++i) B.order[i] = static_cast<uint32_t>(i);
  if (!keep_order)
    std::stable_sort(B.order.begin(), B.order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
  B.base.resize(n);
  uint64_t base = 0;
  for (size_t k = 0; k < n; ++k) {
    B.base[k] = base;
    base += items[B.order[k]];
  }
  B.total = base;
  return B;
}

}  // namespace pbs
