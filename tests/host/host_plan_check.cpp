// Host checks of the device-free planning code (csrc/host_plan.h), built by
// tests/test_host_sanitize.py with the host compiler under AddressSanitizer
// and UndefinedBehaviorSanitizer.  Prints one line per check group and
// returns non-zero on the first failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2606_28952_amd/csrc/host_plan.h"

using namespace pbs;

static int g_fail = 0;
#define CHECK(cond, ...)                                 \
  do {                                                   \
    if (!(cond)) {                                       \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                 \
      std::fprintf(stderr, "\n");                        \
      ++g_fail;                                          \
      return;                                            \
    }                                                    \
  } while (0)

static double fro(const std::vector<double>& a) {
  double s = 0.0;
  for (double v : a) s += v * v;
  return std::sqrt(s);
}

// factor_rows: a random rows x cols matrix of rank k is factored with rank
// k, Q has orthonormal rows and M Q^T Q reproduces M.
static void check_factor_rows() {
  std::mt19937_64 rng(11);
  std::normal_distribution<double> nd;
  int cases = 0;
  for (uint32_t rows : {1u, 2u, 5u, 17u, 40u})
    for (uint32_t cols : {1u, 3u, 8u, 33u})
      for (uint32_t k = 0; k <= std::min(rows, cols); k += (k < 3 ? 1 : 5)) {
        std::vector<double> A(static_cast<size_t>(rows) * k), B(static_cast<size_t>(k) * cols), M(rows * cols, 0.0);
        for (double& v : A) v = nd(rng);
        for (double& v : B) v = nd(rng);
        for (uint32_t i = 0; i < rows; ++i)
          for (uint32_t j = 0; j < cols; ++j)
            for (uint32_t r = 0; r < k; ++r) M[i * cols + j] += A[i * k + r] * B[r * cols + j];
        std::vector<double> Q;
        const uint32_t rank = factor_rows(M, rows, cols, 1e-12, Q);
        CHECK(rank == k, "rank %u, expected %u (%u x %u)", rank, k, rows, cols);
        CHECK(Q.size() == static_cast<size_t>(rank) * cols, "Q size");
        for (uint32_t a = 0; a < rank; ++a)
          for (uint32_t b = 0; b < rank; ++b) {
            double d = 0.0;
            for (uint32_t j = 0; j < cols; ++j) d += Q[a * cols + j] * Q[b * cols + j];
            CHECK(std::fabs(d - (a == b ? 1.0 : 0.0)) < 1e-12, "Q not orthonormal (%u, %u): %g", a, b, d);
          }
        std::vector<double> R = M;
        for (uint32_t i = 0; i < rows; ++i)
          for (uint32_t r = 0; r < rank; ++r) {
            double p = 0.0;
            for (uint32_t j = 0; j < cols; ++j) p += M[i * cols + j] * Q[r * cols + j];
            for (uint32_t j = 0; j < cols; ++j) R[i * cols + j] -= p * Q[r * cols + j];
          }
        CHECK(fro(R) <= 1e-12 * std::max(1.0, fro(M)), "residual %g", fro(R));
        ++cases;
      }
  // duplicated and negated rows add no rank; a zero matrix has rank 0
  std::vector<double> M = {1, 2, 3, 2, 4, 6, -1, -2, -3}, Q;
  CHECK(factor_rows(M, 3, 3, 1e-14, Q) == 1, "duplicated rows");
  CHECK(factor_rows(std::vector<double>(12, 0.0), 3, 4, 1e-14, Q) == 0 && Q.empty(), "zero matrix");
  std::printf("factor_rows: %d random cases\n", cases);
}

// factor_group: for random groups, sum_r A_r(ta) F_r(tb) equals the direct
// phase sum sum_k c_k (-1)^(|za_k & ta| + |zb_u & tb|) at every pair of
// spin strings of n bits.
static void check_factor_group() {
  std::mt19937_64 rng(12);
  const uint32_t n = 6;
  int cases = 0;
  for (int rep = 0; rep < 40; ++rep) {
    HostTables T;
    T.pg_u0 = {0};
    T.u_t0 = {0};
    const uint32_t n_groups = 1 + rng() % 4;
    for (uint32_t g = 0; g < n_groups; ++g) {
      const uint32_t nu = 1 + rng() % 6;
      for (uint32_t u = 0; u < nu; ++u) {
        T.u_zb.push_back(static_cast<uint32_t>(rng() % (1u << n)));
        const uint32_t nt = 1 + rng() % 5;
        for (uint32_t t = 0; t < nt; ++t) {
          // few distinct alpha masks, so that the rank is often below both sizes
          T.pt_za.push_back(static_cast<uint32_t>(rng() % 4) * 5u);
          T.pt_c.push_back(std::ldexp(static_cast<double>(static_cast<int>(rng() % 2001) - 1000), -7));
        }
        T.u_t0.push_back(static_cast<uint32_t>(T.pt_za.size()));
      }
      T.pg_u0.push_back(static_cast<uint32_t>(T.u_zb.size()));
      T.pg_xb.push_back(0);
    }
    for (uint32_t g = 0; g < n_groups; ++g) {
      const GroupFactors F = factor_group(T, g);
      CHECK(F.n_uniques == T.pg_u0[g + 1] - T.pg_u0[g], "uniques");
      CHECK(F.a.size() == F.rank && F.b.size() == F.rank, "factor lists");
      std::set<uint32_t> za(T.pt_za.begin() + T.u_t0[T.pg_u0[g]], T.pt_za.begin() + T.u_t0[T.pg_u0[g + 1]]);
      CHECK(F.rank <= std::min<size_t>(za.size(), F.n_uniques), "rank above the matrix size");
      for (uint32_t ta = 0; ta < (1u << n); ++ta)
        for (uint32_t tb = 0; tb < (1u << n); ++tb) {
          double want = 0.0, got = 0.0;
          for (uint32_t u = T.pg_u0[g]; u < T.pg_u0[g + 1]; ++u)
            for (uint32_t t = T.u_t0[u]; t < T.u_t0[u + 1]; ++t)
              want += ((__builtin_popcount(T.pt_za[t] & ta) + __builtin_popcount(T.u_zb[u] & tb)) & 1) ? -T.pt_c[t]
                                                                                                       : T.pt_c[t];
          for (uint32_t r = 0; r < F.rank; ++r) {
            double A = 0.0, B = 0.0;
            for (const auto& e : F.a[r]) A += (__builtin_popcount(e.first & ta) & 1) ? -e.second : e.second;
            for (const auto& e : F.b[r]) B += (__builtin_popcount(e.first & tb) & 1) ? -e.second : e.second;
            got += A * B;
          }
          CHECK(std::fabs(got - want) <= 1e-12 * (1.0 + std::fabs(want)), "group %u at (%u, %u): %.17g vs %.17g", g,
                ta, tb, got, want);
        }
      ++cases;
    }
  }
  std::printf("factor_group: %d groups, every (alpha, beta) string pair of %u bits\n", cases, n);
}

// batch_plan: launch order is a permutation, costs do not increase along
// it, ties keep the caller's order, and every job's items follow the
// previous job's without gap or overlap.
static void check_batch_plan() {
  std::mt19937_64 rng(13);
  int cases = 0;
  for (uint32_t n : {0u, 1u, 2u, 7u, 64u, 300u}) {
    for (bool keep : {false, true}) {
      std::vector<double> cost(n);
      std::vector<uint64_t> items(n);
      for (uint32_t i = 0; i < n; ++i) {
        cost[i] = static_cast<double>(rng() % 5);  // many ties
        items[i] = rng() % 1000;
      }
      const BatchPlan P = batch_plan(cost, items, keep);
      CHECK(P.order.size() == n && P.base.size() == n, "sizes");
      std::vector<int> seen(n, 0);
      for (uint32_t k = 0; k < n; ++k) {
        CHECK(P.order[k] < n && !seen[P.order[k]]++, "not a permutation");
        if (keep) CHECK(P.order[k] == k, "given order changed");
        if (!keep && k > 0) {
          CHECK(cost[P.order[k - 1]] >= cost[P.order[k]], "cost increases");
          if (cost[P.order[k - 1]] == cost[P.order[k]]) CHECK(P.order[k - 1] < P.order[k], "tie reordered");
        }
        const uint64_t next = k + 1 < n ? P.base[k + 1] : P.total;
        CHECK(next - P.base[k] == items[P.order[k]], "items of job %u", k);
      }
      CHECK(n > 0 || P.total == 0, "empty batch");
      CHECK(n == 0 || P.base[0] == 0, "first base");
      ++cases;
    }
  }
  std::printf("batch_plan: %d cases\n", cases);
}

// sector_layout: over sectors, amplitude sizes, coefficient kinds, device
// LDS sizes and table sizes, the regions are disjoint, lie below the
// layout's end, which stays within the device's LDS, and the pair map, the
// folded uniques' capacity and the row region hold what the kernels put
// there.
static void check_sector_layout() {
  int cases = 0, rows_staged = 0, two_per_cu = 0;
  for (uint32_t limit : {65536u - 1024u, 163840u - 1024u})
    for (uint32_t n_orb = 2; n_orb <= 24; ++n_orb)
      for (uint32_t n_beta = 0; n_beta <= n_orb; n_beta += 1 + n_orb / 6)
        for (uint32_t elem : {8u, 16u})
          for (bool realc : {true, false})
            for (uint32_t quads : {0u, 35u, 1820u})
              for (bool a_region : {false, true}) {
                SectorLayoutIn in;
                in.lds_limit = limit;
                in.n_orb = n_orb;
                in.n_beta = n_beta;
                uint64_t d = 1;  // C(n_orb, n_beta)
                for (uint32_t i = 0; i < n_beta; ++i) d = d * (n_orb - i) / (i + 1);
                in.dim_beta = d;
                in.elem_bytes = elem;
                in.realc = realc;
                in.n_pmap = 1;
                in.n_qmap = quads ? 1 : 0;
                in.n_pairs = n_orb * (n_orb - 1) / 2;
                in.n_quads = quads;
                in.max_quad_uniques = quads / 4;
                in.a_region = a_region;
                SectorLayout L;
                const bool ok = sector_layout(in, &L);
                CHECK(ok == (in.n_pairs + 1 <= kPuBytes / 8), "pair map refusal at n_orb %u", n_orb);
                if (!ok) continue;
                ++cases;
                CHECK(L.lds <= limit, "LDS %u above the limit %u (n_orb %u, n_beta %u)", L.lds, limit, n_orb, n_beta);
                CHECK(L.f_cap >= 1 && L.f_cap <= kFCapMax, "f_cap %u", L.f_cap);
                CHECK(L.f_bytes >= (L.f_cap + kZeroSlots) * (realc ? 8u : 16u), "folded uniques region");
                CHECK(L.fz_bytes >= (L.f_cap + kZeroSlots) * 4u, "Z-mask region");
                CHECK(L.list_cap * 8u <= L.row_region, "row list capacity");
                if (L.row_lds) {
                  CHECK(d * elem <= L.row_region, "staged row does not fit");
                  ++rows_staged;
                }
                CHECK(L.r16 == (n_orb <= 16) && (L.rank_bytes >= (L.r16 ? kRank16Lds * 2u : 0u)), "rank tables");
                CHECK((in.n_pairs + 1u) * 8u <= kPuBytes, "pair map");
                if (a_region && L.a_in_pair_map)
                  CHECK(L.off_a >= kPuOff + (in.n_pairs + 1u) * 8u && L.off_a + kMaxR1 * 8u <= kPuOff + kPuBytes,
                        "X_beta = 0 factors outside the pair map's free tail");
                // every region [off, off + size): disjoint, 16-byte aligned, below lds
                struct Reg {
                  uint32_t off, size;
                };
                std::vector<Reg> regs = {{0, kMiscBytes},
                                         {kPuOff, kPuBytes},
                                         {kRowOff, L.row_region},
                                         {L.off_rank, L.rank_bytes},
                                         {L.off_f, L.f_bytes},
                                         {L.off_fz, L.fz_bytes},
                                         {L.off_qu, L.qu_bytes}};
                if (!L.a_in_pair_map) regs.push_back({L.off_a, L.a_bytes});
                for (size_t i = 0; i < regs.size(); ++i) {
                  CHECK(regs[i].off % 16 == 0, "region %zu misaligned", i);
                  CHECK(regs[i].off + regs[i].size <= L.lds, "region %zu ends past lds", i);
                  for (size_t j = 0; j < i; ++j)
                    CHECK(regs[i].size == 0 || regs[j].size == 0 || regs[i].off >= regs[j].off + regs[j].size ||
                              regs[j].off >= regs[i].off + regs[i].size,
                          "regions %zu and %zu overlap", j, i);
                }
                if (2u * (L.lds + 1024u) <= limit + 1024u) ++two_per_cu;
              }
  // the 28-qubit (7, 7) sector of complex64 amplitudes on a 160 KB device
  // stages its rows and keeps two workgroups per compute unit
  SectorLayoutIn in;
  in.lds_limit = 163840u - 1024u;
  in.n_orb = 14;
  in.n_beta = 7;
  in.dim_beta = 3432;
  in.elem_bytes = 8;
  in.n_pmap = 1;
  in.n_pairs = 91;
  in.a_region = true;
  SectorLayout L;
  CHECK(sector_layout(in, &L) && L.row_lds && L.enum_ok && L.a_in_pair_map && 2u * (L.lds + 1024u) <= 163840u,
        "28-qubit sector layout (lds %u)", L.lds);
  std::printf("sector_layout: %d cases, %d with a staged row, %d with two workgroups per CU\n", cases, rows_staged,
              two_per_cu);
}

int main() {
  check_factor_rows();
  check_factor_group();
  check_batch_plan();
  check_sector_layout();
  if (g_fail) {
    std::printf("%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("all host plan checks passed\n");
  return 0;
}
