// Spin-factorized phase evaluation (Section 2.4: Eqs. svd_weights,
// precomp_alpha, precomp_beta, svd_sreverse_sum and dot_product; Algorithm
// grouped_hvec; the rank distribution of Table svd_rank_dist).
//
// In a spin sector every group's phase sum separates into alpha and beta
// parities: with its sector-form coefficients arranged as a matrix
// M[mu][nu] (rows: the group's distinct alpha Z-masks, columns: its uniques,
// i.e. distinct beta Z-masks),
//   sum_k C_k (-1)^popcount(Z_k & t) = sum_{mu,nu} M[mu][nu] a_mu(t_a) b_nu(t_b),
// a_mu = (-1)^popcount(Za_mu & t_a), b_nu = (-1)^popcount(Zb_nu & t_b).  A
// rank-R factorization M = P Q turns this into sum_r A_r(t_a) F_r(t_b).  The
// sector kernel folds the A_r once per workgroup (all its lanes share t_a);
// this file factors the groups on the host and precomputes F_r for every
// beta string of a sector on the device, laid out per target move so that
// the kernel's loads are coalesced.  The paper computes the factors by an
// SVD; here a rank-revealing Gram-Schmidt factorization (Q with orthonormal
// rows, P = M Q^T, columns chosen by largest remaining norm) gives the same
// exact ranks on these matrices with the same rounding-level residual.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "handles.h"

namespace pbs {
namespace {

// colexicographic rank of a spin string among the n-bit words of its
// popcount (ascending integer order): sum_i C(pos_i, i + 1)
__device__ inline uint32_t colex_rank(uint32_t s) {
  uint32_t r = 0, i = 1;
  while (s) {
    const uint32_t b = __ffs(s) - 1;
    s &= s - 1;
    uint32_t c = 1;  // C(b, i)
    for (uint32_t k = 1; k <= i; ++k) c = c * (b - i + k) / k;
    r += b >= i ? c : 0u;
    ++i;
  }
  return r;
}

// k-th set bit (k from 0) of w
__device__ inline uint32_t kth_bit(uint32_t w, uint32_t k) {
  for (uint32_t i = 0; i < k; ++i) w &= w - 1;
  return __ffs(w) - 1;
}

// i-th pair (a < b) of n items in the order (0,1), (0,2), ..., (1,2), ...
__device__ inline void pair_at(uint32_t i, uint32_t n, uint32_t& a, uint32_t& b) {
  a = 0;
  while (i >= n - 1 - a) {
    i -= n - 1 - a;
    ++a;
  }
  b = a + 1 + i;
}

__device__ inline double eval_rows(const uint32_t* q_zb, const double* q_c, uint32_t lo, uint32_t hi, uint32_t tb) {
  double f = 0.0;
  for (uint32_t k = lo; k < hi; ++k) f += (__popc(q_zb[k] & tb) & 1u) ? -q_c[k] : q_c[k];
  return f;
}

// F rows of the X_beta = 0 groups: f[i * db + j] = sum over row i's list.
__global__ void k_fact_rows(uint32_t n_rows, uint64_t db, const uint32_t* str_b, const uint32_t* q_lo,
                            const uint32_t* q_zb, const double* q_c, double* f) {
  const uint64_t n = static_cast<uint64_t>(n_rows) * db;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t row = static_cast<uint32_t>(i / db);
    f[i] = eval_rows(q_zb, q_c, q_lo[row], q_lo[row + 1], str_b[i % db]);
  }
}

// Single moves (occupied p -> empty q, p outer, both ascending):
// em[m * db + j] = source column | (factor slot << 16), fp[(m * r2 + r) * db + j].
__global__ void k_fact_moves(uint64_t db, uint32_t n_orb, uint32_t n_beta, uint32_t r2, const uint32_t* str_b,
                             const int32_t* pk, const uint32_t* q_lo, const uint32_t* q_zb, const double* q_c,
                             uint32_t* em, double* fp) {
  const uint32_t ne = n_orb - n_beta, n_moves = n_beta * ne;
  const uint32_t full = (n_orb == 32) ? 0xffffffffu : ((1u << n_orb) - 1u);
  const uint64_t n = static_cast<uint64_t>(n_moves) * db;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t m = static_cast<uint32_t>(i / db);
    const uint64_t j = i % db;
    const uint32_t tb = str_b[j];
    const uint32_t p = kth_bit(tb, m / ne), q = kth_bit(~tb & full, m % ne);
    const uint32_t lo = p < q ? p : q, hi = p < q ? q : p;
    const int32_t k = pk[hi * (hi - 1) / 2 + lo];
    em[static_cast<uint64_t>(m) * db + j] =
        colex_rank(tb ^ (1u << p) ^ (1u << q)) | ((k >= 0 ? kFactZeroSlots + static_cast<uint32_t>(k) * r2 : 0u) << 16);
    for (uint32_t r = 0; r < r2; ++r) {
      const uint32_t row = static_cast<uint32_t>(k) * r2 + r;
      fp[(static_cast<uint64_t>(m) * r2 + r) * db + j] = k >= 0 ? eval_rows(q_zb, q_c, q_lo[row], q_lo[row + 1], tb)
                                                                : 0.0;
    }
  }
}

// Double moves: occupied pair (a < b) outer, empty pair (c < d) inner, each
// in the order of pair_at over the target's occupied / empty orbitals.
// eq[qm * db + j] = source column | (factor slot << 16); fq[(qm * r3 + r) * db + j].
__global__ void k_fact_quads(uint64_t db, uint32_t n_orb, uint32_t n_beta, uint32_t r3, uint32_t slot0,
                             const uint32_t* str_b, const int32_t* qk, const uint32_t* q_lo, const uint32_t* q_zb,
                             const double* q_c, uint32_t* eq, double* fq) {
  const uint32_t ne = n_orb - n_beta;
  const uint32_t n_op = n_beta * (n_beta - 1) / 2, n_ep = ne * (ne - 1) / 2, n_q = n_op * n_ep;
  const uint32_t full = (n_orb == 32) ? 0xffffffffu : ((1u << n_orb) - 1u);
  const uint64_t n = static_cast<uint64_t>(n_q) * db;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t qm = static_cast<uint32_t>(i / db);
    const uint64_t j = i % db;
    const uint32_t tb = str_b[j], emp = ~tb & full;
    uint32_t a, b, c, d;
    pair_at(qm / n_ep, n_beta, a, b);
    pair_at(qm % n_ep, ne, c, d);
    const uint32_t X = (1u << kth_bit(tb, a)) | (1u << kth_bit(tb, b)) | (1u << kth_bit(emp, c)) |
                       (1u << kth_bit(emp, d));
    const int32_t k = qk[colex_rank(X)];
    eq[static_cast<uint64_t>(qm) * db + j] =
        colex_rank(tb ^ X) | ((k >= 0 ? slot0 + static_cast<uint32_t>(k) * r3 : 0u) << 16);
    for (uint32_t r = 0; r < r3; ++r) {
      const uint32_t row = static_cast<uint32_t>(k) * r3 + r;
      fq[(static_cast<uint64_t>(qm) * r3 + r) * db + j] = k >= 0 ? eval_rows(q_zb, q_c, q_lo[row], q_lo[row + 1], tb)
                                                                 : 0.0;
    }
  }
}

// Position of this thread's flag among the workgroup's set flags (in thread
// order) and their total; 256 threads.
__device__ inline void block_compact(bool flag, uint32_t* s_cnt, uint32_t& pos, uint32_t& total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint64_t bal = __ballot(flag);
  if (lane == 0) s_cnt[wave] = static_cast<uint32_t>(__popcll(bal));
  __syncthreads();
  pos = static_cast<uint32_t>(__popcll(bal & ((1ull << lane) - 1ull)));
  total = 0;
  for (uint32_t w = 0; w < 4; ++w) {
    pos += w < wave ? s_cnt[w] : 0u;
    total += s_cnt[w];
  }
  __syncthreads();
}

// Alpha lists (Eq. precomp_alpha for the simple classes): one workgroup per
// alpha row, its threads over the simple classes in class order; pass 0
// counts the classes whose source row lies in the sector, pass 1 writes
// their source rank and folded coefficient sum_t c_t (-1)^popcount(za_t & t_alpha)
// in class order.
__global__ __launch_bounds__(256) void k_alpha_list(uint32_t pass, uint64_t da, uint32_t n_alpha,
                                                    const uint32_t* str_a, const uint32_t* simple, uint32_t n_simple,
                                                    const ClassMeta* meta, const uint32_t* u_t0,
                                                    const uint32_t* pt_za, const double* pt_c, const uint32_t* off,
                                                    uint32_t* count, uint32_t* src, double* coef) {
  __shared__ uint32_t s_cnt[4];
  for (uint64_t i = blockIdx.x; i < da; i += gridDim.x) {
    const uint32_t ta = str_a[i];
    uint32_t n = pass ? off[i] : 0u;
    for (uint32_t k0 = 0; k0 < n_simple; k0 += 256) {
      const uint32_t k = k0 + threadIdx.x;
      const ClassMeta* m = k < n_simple ? meta + simple[k] : nullptr;
      const uint32_t sa = m ? ta ^ m->xa : 0u;
      const bool v = m && static_cast<uint32_t>(__popc(sa)) == n_alpha;
      uint32_t pos, total;
      block_compact(v, s_cnt, pos, total);
      if (pass && v) {
        double f = 0.0;
        for (uint32_t t = u_t0[m->ua]; t < u_t0[m->u_end]; ++t)
          f += (__popc(pt_za[t] & ta) & 1u) ? -pt_c[2 * t] : pt_c[2 * t];
        src[n + pos] = colex_rank(sa);
        coef[n + pos] = f;
      }
      n += total;
    }
    if (!pass && threadIdx.x == 0) count[i] = n;
  }
}

// Image-class lists: one workgroup per alpha row; pass 0 counts the image
// classes whose source row lies in the sector, pass 1 writes (source rank,
// class, row) in class order.
__global__ __launch_bounds__(256) void k_pair_list(uint32_t pass, uint64_t da, uint32_t n_alpha,
                                                   const uint32_t* str_a, const uint32_t* cls, uint32_t n_cls,
                                                   const ClassMeta* meta, const uint32_t* off, uint32_t* count,
                                                   uint32_t* src, uint32_t* ent_cls, uint32_t* ent_row) {
  __shared__ uint32_t s_cnt[4];
  for (uint64_t i = blockIdx.x; i < da; i += gridDim.x) {
    const uint32_t ta = str_a[i];
    uint32_t n = pass ? off[i] : 0u;
    for (uint32_t k0 = 0; k0 < n_cls; k0 += 256) {
      const uint32_t k = k0 + threadIdx.x;
      const uint32_t sa = k < n_cls ? ta ^ meta[cls[k]].xa : 0u;
      const bool v = k < n_cls && static_cast<uint32_t>(__popc(sa)) == n_alpha;
      uint32_t pos, total;
      block_compact(v, s_cnt, pos, total);
      if (pass && v) {
        src[n + pos] = colex_rank(sa);
        ent_cls[n + pos] = cls[k];
        ent_row[n + pos] = static_cast<uint32_t>(i);
      }
      n += total;
    }
    if (!pass && threadIdx.x == 0) count[i] = n;
  }
}

// Images: one workgroup per entry (an alpha row and one of its image
// classes), one thread per slot j < n_img: the folded coefficient of the
// class's pair group on orbital pair j, 0 for slot n_pairs, then the
// X_beta = 0 group's folded factors.  The entry's class, row and class
// record are uniform across the workgroup; the pair-map row is read
// coalesced.
constexpr uint32_t kImgBlock = 128;
__global__ __launch_bounds__(kImgBlock) void k_pair_images(uint32_t n_img, uint32_t n_pairs, const uint32_t* str_a,
                                                           const uint32_t* ent_cls, const uint32_t* ent_row,
                                                           const ClassMeta* meta, const int32_t* pmap,
                                                           const uint32_t* pg_u0, const uint32_t* u_t0,
                                                           const uint32_t* pt_za, const double* pt_c,
                                                           const uint4* cls_f, const uint32_t* fu_t0,
                                                           const uint32_t* ft_za, const double* ft_c, double* img) {
  const uint64_t e = blockIdx.x;
  const uint32_t c = ent_cls[e], ta = str_a[ent_row[e]];
  const int32_t* prow = pmap + static_cast<uint64_t>(meta[c].pm) * n_pairs;
  const uint4 cf = cls_f[c];
  for (uint32_t j = threadIdx.x; j < n_img; j += kImgBlock) {
    double f = 0.0;
    if (j < n_pairs) {
      const int32_t g = prow[j];
      if (g >= 0) {
        const uint32_t u = pg_u0[g];
        for (uint32_t t = u_t0[u]; t < u_t0[u + 1]; ++t) f += (__popc(pt_za[t] & ta) & 1u) ? -pt_c[2 * t] : pt_c[2 * t];
      }
    } else if (j > n_pairs) {
      const uint32_t r = j - n_pairs - 1;
      if (r < cf.y) {
        const uint32_t u = cf.x + r;
        for (uint32_t t = fu_t0[u]; t < fu_t0[u + 1]; ++t) f += (__popc(ft_za[t] & ta) & 1u) ? -ft_c[t] : ft_c[t];
      }
    }
    img[e * n_img + j] = f;
  }
}

// ---------------------------------------------------------------- host side

// Pinned host staging for the build's small host<->device copies, one buffer
// per device for the process's lifetime, used by one build at a time.  Copies
// through it are stream-ordered and asynchronous: an upload returns at once,
// and several downloads complete with one wait.  A copy that does not fit
// goes through pageable memory (synchronously, as before) and the buffer
// grows for the next build.
class Staging {
 public:
  explicit Staging(hipStream_t s) : s_(s) {
    int dev = 0;
    PBS_HIP(hipGetDevice(&dev));
    PBS_REQUIRE(dev >= 0 && dev < kMaxDevices, PBS_ERR_RANGE, "device index beyond the staging table");
    pool_ = &pools()[dev];
    pool_->mu.lock();
    if (!pool_->base && hipHostMalloc(&pool_->base, kInitial, hipHostMallocDefault) == hipSuccess)
      pool_->cap = kInitial;
    (void)hipGetLastError();
  }
  ~Staging() {
    // queued copies read or fill the buffer until the stream reaches them
    (void)hipStreamSynchronize(s_);
    if (wanted_ > pool_->cap) {
      if (pool_->base) (void)hipHostFree(pool_->base);
      pool_->base = nullptr;
      pool_->cap = 0;
      const size_t grown = wanted_ + wanted_ / 4;
      if (hipHostMalloc(&pool_->base, grown, hipHostMallocDefault) == hipSuccess) pool_->cap = grown;
    }
    (void)hipGetLastError();
    pool_->mu.unlock();
  }
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;

  // handle-owned buffer (hipMalloc), filled from h
  template <class T>
  void upload(DevBuf<T>& d, const std::vector<T>& h) {
    d.alloc(h.size());
    put(d.get(), h);
  }
  // temporary of the build, from the call's scratch arena
  template <class T>
  void upload_temp(DevBuf<T>& d, const std::vector<T>& h) {
    d = DevBuf<T>(h.size(), s_);
    put(d.get(), h);
  }
  // n values of d into out, complete after wait()
  template <class T>
  void fetch(std::vector<T>& out, const DevBuf<T>& d, size_t n) {
    out.resize(n);
    if (!n) return;
    const size_t bytes = n * sizeof(T);
    if (void* p = take(bytes)) {
      PBS_HIP(hipMemcpyAsync(p, d.get(), bytes, hipMemcpyDeviceToHost, s_));
      pending_.push_back({out.data(), p, bytes});
    } else {
      PBS_HIP(hipMemcpyAsync(out.data(), d.get(), bytes, hipMemcpyDeviceToHost, s_));
    }
  }
  // waits for the stream and moves the fetched values into place
  void wait() {
    PBS_HIP(hipStreamSynchronize(s_));
    for (const Pending& q : pending_) std::memcpy(q.dst, q.src, q.bytes);
    pending_.clear();
  }

 private:
  static constexpr int kMaxDevices = 64;
  static constexpr size_t kInitial = size_t(8) << 20;
  struct Pool {
    void* base = nullptr;
    size_t cap = 0;
    std::mutex mu;
  };
  struct Pending {
    void* dst;
    const void* src;
    size_t bytes;
  };
  static Pool* pools() {
    static Pool table[kMaxDevices];  // lives until the process ends
    return table;
  }
  void* take(size_t bytes) {
    const size_t need = (bytes + 255) & ~static_cast<size_t>(255);
    const size_t at = top_;
    top_ += need;
    wanted_ = std::max(wanted_, top_);
    if (!pool_->base || top_ > pool_->cap) return nullptr;
    return static_cast<char*>(pool_->base) + at;
  }
  template <class T>
  void put(T* dst, const std::vector<T>& h) {
    if (h.empty()) return;
    const size_t bytes = h.size() * sizeof(T);
    if (void* p = take(bytes)) {
      std::memcpy(p, h.data(), bytes);
      PBS_HIP(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, s_));
    } else {
      PBS_HIP(hipMemcpyAsync(dst, h.data(), bytes, hipMemcpyHostToDevice, s_));
      PBS_HIP(hipStreamSynchronize(s_));  // h may change once we return
    }
  }

  hipStream_t s_;
  Pool* pool_ = nullptr;
  size_t top_ = 0, wanted_ = 0;
  std::vector<Pending> pending_;
};

void build_plan(pbs_grouped& h, const pbs_space& sp, hipStream_t s) {
  auto plan = std::make_unique<FactorPlan>();
  FactorPlan& F = *plan;
  F.n_orb = sp.n_orb;
  F.n_beta = sp.n_beta;
  F.dim_beta = sp.dim_beta;
  const uint64_t db = sp.dim_beta;
  Staging st(s);
  HostTables T;
  std::vector<double> pt_c2;
  std::vector<ClassMeta> meta;
  std::vector<uint32_t> ns;
  st.fetch(T.pg_u0, h.pg_u0, h.n_pgroup + 1);
  st.fetch(T.u_zb, h.u_zb, h.n_unique);
  st.fetch(T.u_t0, h.u_t0, h.n_unique + 1);
  st.fetch(T.pt_za, h.pt_za, h.n_pterm);
  st.fetch(T.pg_xb, h.pg_xb, h.n_pgroup);
  st.fetch(pt_c2, h.pt_c, 2ull * h.n_pterm);
  st.fetch(meta, h.cls_meta, h.n_class);
  st.fetch(ns, h.ns_list, h.n_ns);
  st.wait();
  T.pt_c.resize(h.n_pterm);
  for (uint32_t t = 0; t < h.n_pterm; ++t) T.pt_c[t] = pt_c2[2ull * t];

  // factor uniques (alpha side) and the beta lists of the table rows
  std::vector<uint32_t> fu_t0{0}, ft_za;
  std::vector<double> ft_c;
  std::vector<uint32_t> q_lo{0}, q_zb;
  std::vector<double> q_c;
  auto add_factor = [&](const std::vector<std::pair<uint32_t, double>>* a) {
    if (a)
      for (auto& t : *a) {
        ft_za.push_back(t.first);
        ft_c.push_back(t.second);
      }
    fu_t0.push_back(static_cast<uint32_t>(ft_za.size()));
  };
  auto add_row = [&](const std::vector<std::pair<uint32_t, double>>* b) {
    if (b)
      for (auto& t : *b) {
        q_zb.push_back(t.first);
        q_c.push_back(t.second);
      }
    q_lo.push_back(static_cast<uint32_t>(q_zb.size()));
  };

  // the class with X_alpha = 0: its pair groups (single moves) and quad groups
  // (double moves), when the sector kernel enumerates both
  const uint32_t ne = sp.n_orb - sp.n_beta;
  const uint32_t n_moves = sp.n_beta * ne;
  const uint64_t n_qmoves = host_binom(sp.n_beta, 2) * host_binom(ne, 2);
  uint32_t c0 = 0xffffffffu;
  for (uint32_t c : ns)
    if (meta[c].xa == 0) c0 = c;
  std::vector<GroupFactors> pf, qf;
  if (c0 != 0xffffffffu && sp.n_orb <= 16 && n_moves > 0 && n_qmoves > 0 && db < 65536) {
    const ClassMeta& m = meta[c0];
    const uint32_t gz_end = m.zg >= 0 ? m.g0 + 1 : m.g0;
    uint32_t r2 = 0, r3 = 0;
    for (uint32_t g = gz_end; g < m.p1; ++g) {
      pf.push_back(factor_group(T, g));
      r2 = std::max(r2, pf.back().rank);
    }
    for (uint32_t g = m.p1; g < m.q1; ++g) {
      qf.push_back(factor_group(T, g));
      r3 = std::max(r3, qf.back().rank);
    }
    const uint64_t n_fold = static_cast<uint64_t>(pf.size()) * r2 + static_cast<uint64_t>(qf.size()) * r3;
    // the tables hold every move of a target, present group or not: used
    // only when most orbital pairs / quadruples have a group (two-body
    // operators with dense integrals), where they replace long phase sums
    const bool dense = 2 * pf.size() >= h.n_pairs && 2 * qf.size() >= h.n_quads;
    if (dense && r2 >= 1 && r2 <= 2 && r3 >= 1 && r3 <= 2 && kFactZeroSlots + n_fold <= 4096) {
      F.c0 = c0;
      F.r2 = r2;
      F.r3 = r3;
    } else {
      pf.clear();
      qf.clear();
    }
  }
  std::vector<int32_t> pk(h.n_pairs + 1, -1), qk(h.n_quads ? h.n_quads : 1, -1);
  if (F.c0 != 0xffffffffu) {
    const ClassMeta& m = meta[c0];
    const uint32_t gz_end = m.zg >= 0 ? m.g0 + 1 : m.g0;
    F.c0_fu0 = 0;
    for (uint32_t k = 0; k < pf.size(); ++k) {
      const uint32_t x = T.pg_xb[gz_end + k];
      const uint32_t lo = static_cast<uint32_t>(__builtin_ctz(x)), hi = 31u - static_cast<uint32_t>(__builtin_clz(x));
      pk[hi * (hi - 1) / 2 + lo] = static_cast<int32_t>(k);
      for (uint32_t r = 0; r < F.r2; ++r) add_factor(r < pf[k].rank ? &pf[k].a[r] : nullptr);
    }
    F.c0_fq = static_cast<uint32_t>(fu_t0.size() - 1);
    for (uint32_t k = 0; k < qf.size(); ++k) {
      uint32_t x = T.pg_xb[m.p1 + k], id = 0;
      for (uint32_t j = 1; j <= 4; ++j) {
        const uint32_t b = static_cast<uint32_t>(__builtin_ctz(x));
        x &= x - 1;
        id += static_cast<uint32_t>(host_binom(b, j));
      }
      qk[id] = static_cast<int32_t>(k);
      for (uint32_t r = 0; r < F.r3; ++r) add_factor(r < qf[k].rank ? &qf[k].a[r] : nullptr);
    }
    F.c0_fu1 = static_cast<uint32_t>(fu_t0.size() - 1);
    F.n_f2 = static_cast<uint32_t>(pf.size());
    F.n_f3 = static_cast<uint32_t>(qf.size());
    F.n_moves = n_moves;
    F.n_qmoves = static_cast<uint32_t>(n_qmoves);
  }
  const uint32_t rows_p = static_cast<uint32_t>(q_lo.size() - 1);
  for (uint32_t k = 0; k < pf.size(); ++k)
    for (uint32_t r = 0; r < F.r2; ++r) add_row(r < pf[k].rank ? &pf[k].b[r] : nullptr);
  const uint32_t rows_q = static_cast<uint32_t>(q_lo.size() - 1);
  for (uint32_t k = 0; k < qf.size(); ++k)
    for (uint32_t r = 0; r < F.r3; ++r) add_row(r < qf[k].rank ? &qf[k].b[r] : nullptr);
  const uint32_t rows_z = static_cast<uint32_t>(q_lo.size() - 1);

  // X_beta = 0 groups of the non-simple classes, factored when that lowers
  // the number of beta terms a target evaluates
  std::vector<uint4> cls_f(h.n_class, make_uint4(0u, 0u, 0u, 0u));
  uint32_t n_zrows = 0;
  for (uint32_t c : ns) {
    const ClassMeta& m = meta[c];
    if (m.zg < 0) continue;
    GroupFactors G = factor_group(T, static_cast<uint32_t>(m.zg));
    if (G.rank == 0 || G.rank > kMaxR1 || G.rank >= G.n_uniques) continue;
    const uint32_t fu0 = static_cast<uint32_t>(fu_t0.size() - 1);
    for (uint32_t r = 0; r < G.rank; ++r) {
      add_factor(&G.a[r]);
      add_row(&G.b[r]);
    }
    cls_f[c] = make_uint4(fu0, G.rank, 0u, 0u);
    *reinterpret_cast<uint64_t*>(&cls_f[c].z) = static_cast<uint64_t>(n_zrows) * db;
    n_zrows += G.rank;
    F.max_r1 = std::max(F.max_r1, G.rank);
    ++F.n_f1;
  }
  F.n_fu = static_cast<uint32_t>(fu_t0.size() - 1);
  auto most_terms = [&](uint32_t a, uint32_t b) {
    uint32_t t = 0;
    for (uint32_t u = a; u < b; ++u) t = std::max(t, fu_t0[u + 1] - fu_t0[u]);
    return t;
  };
  F.t_pair = most_terms(F.c0_fu0, F.c0_fq);
  F.t_quad = most_terms(F.c0_fq, F.c0_fu1);
  F.t_zero = most_terms(F.c0_fu1, F.n_fu);
  F.n_ft = static_cast<uint32_t>(ft_za.size());
  st.upload(F.fu_t0, fu_t0);
  st.upload(F.ft_za, ft_za);
  st.upload(F.ft_c, ft_c);
  st.upload(F.cls_f, cls_f);
  DevBuf<uint32_t> d_qlo, d_qzb;
  DevBuf<double> d_qc;
  st.upload_temp(d_qlo, q_lo);
  st.upload_temp(d_qzb, q_zb);
  st.upload_temp(d_qc, q_c);

  if (n_zrows) {
    F.fz.alloc(static_cast<uint64_t>(n_zrows) * db);
    const uint64_t n = static_cast<uint64_t>(n_zrows) * db;
    hipLaunchKernelGGL(k_fact_rows, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n_zrows, db, sp.str_beta.get(),
                       d_qlo.get() + rows_z, d_qzb.get(), d_qc.get(), F.fz.get());
    PBS_HIP(hipGetLastError());
  }
  if (F.c0 != 0xffffffffu) {
    DevBuf<int32_t> d_pk, d_qk;
    st.upload_temp(d_pk, pk);
    st.upload_temp(d_qk, qk);
    F.em.alloc(static_cast<uint64_t>(n_moves) * db);
    F.fp.alloc(static_cast<uint64_t>(n_moves) * F.r2 * db);
    F.eq.alloc(n_qmoves * db);
    F.fq.alloc(n_qmoves * F.r3 * db);
    const uint64_t nm = static_cast<uint64_t>(n_moves) * db, nq = n_qmoves * db;
    hipLaunchKernelGGL(k_fact_moves, dim3(grid_for(nm, 256, 65536)), dim3(256), 0, s, db, sp.n_orb, sp.n_beta, F.r2,
                       sp.str_beta.get(), d_pk.get(), d_qlo.get() + rows_p, d_qzb.get(), d_qc.get(), F.em.get(),
                       F.fp.get());
    const uint32_t slot0 = kFactZeroSlots + F.n_f2 * F.r2;
    hipLaunchKernelGGL(k_fact_quads, dim3(grid_for(nq, 256, 65536)), dim3(256), 0, s, db, sp.n_orb, sp.n_beta,
                       F.r3, slot0, sp.str_beta.get(), d_qk.get(), d_qlo.get() + rows_q, d_qzb.get(), d_qc.get(),
                       F.eq.get(), F.fq.get());
    PBS_HIP(hipGetLastError());
  }
  // alpha lists of the simple classes, when every unique of every simple
  // class has beta Z-mask 0
  {
    std::vector<uint32_t> simple;
    bool plain = true;
    for (uint32_t c = 0; c < h.n_class && plain; ++c) {
      if (!(meta[c].flags & kClassSimple)) continue;
      simple.push_back(c);
      for (uint32_t u = meta[c].ua; u < meta[c].u_end; ++u) plain = plain && T.u_zb[u] == 0u;
    }
    const uint64_t da = sp.dim_alpha;
    if (plain && !simple.empty() && sp.n_orb <= 32) {
      DevBuf<uint32_t> d_simple, cnt(da, s);
      st.upload_temp(d_simple, simple);
      const unsigned grid = static_cast<unsigned>(std::min<uint64_t>(da, 65536));
      hipLaunchKernelGGL(k_alpha_list, dim3(grid), dim3(256), 0, s, 0u, da, sp.n_alpha, sp.str_alpha.get(),
                         d_simple.get(), static_cast<uint32_t>(simple.size()), h.cls_meta.get(), h.u_t0.get(),
                         h.pt_za.get(), h.pt_c.get(), nullptr, cnt.get(), nullptr, nullptr);
      PBS_HIP(hipGetLastError());
      std::vector<uint32_t> c, off(da + 1, 0u);
      st.fetch(c, cnt, da);
      st.wait();
      for (uint64_t i = 0; i < da; ++i) {
        off[i + 1] = off[i] + c[i];
        F.alist_max = std::max(F.alist_max, c[i]);
      }
      st.upload(F.alist_off, off);
      F.alist_src.alloc(off[da]);
      F.alist_c.alloc(off[da]);
      if (off[da]) {
        hipLaunchKernelGGL(k_alpha_list, dim3(grid), dim3(256), 0, s, 1u, da, sp.n_alpha, sp.str_alpha.get(),
                           d_simple.get(), static_cast<uint32_t>(simple.size()), h.cls_meta.get(), h.u_t0.get(),
                           h.pt_za.get(), h.pt_c.get(), F.alist_off.get(), nullptr, F.alist_src.get(),
                           F.alist_c.get());
        PBS_HIP(hipGetLastError());
      }
      F.alist = true;
      F.n_alpha = sp.n_alpha;
    }
  }
  // image classes and their per-row images
  std::vector<uint32_t> flag(h.n_class, 0u);
  if (F.alist && h.pair_sign && F.n_alpha == sp.n_alpha) {
    std::vector<uint32_t> icls;
    const std::vector<uint4>& cf = cls_f;  // as uploaded to F.cls_f
    for (uint32_t c : ns) {
      const ClassMeta& m = meta[c];
      if (c == F.c0 || m.pm < 0 || !(m.flags & kClassPairsSingle) || m.p1 != m.g1) continue;
      if (m.zg >= 0 && (cf[c].y == 0 || cf[c].y > 2)) continue;
      icls.push_back(c);
      flag[c] = 1u;
    }
    const uint64_t da = sp.dim_alpha;
    if (!icls.empty()) {
      DevBuf<uint32_t> d_cls, cnt(da, s);
      st.upload_temp(d_cls, icls);
      const unsigned grid = static_cast<unsigned>(std::min<uint64_t>(da, 65536));
      hipLaunchKernelGGL(k_pair_list, dim3(grid), dim3(256), 0, s, 0u, da, sp.n_alpha, sp.str_alpha.get(), d_cls.get(),
                         static_cast<uint32_t>(icls.size()), h.cls_meta.get(), nullptr, cnt.get(), nullptr, nullptr,
                         nullptr);
      PBS_HIP(hipGetLastError());
      std::vector<uint32_t> c, off(da + 1, 0u);
      st.fetch(c, cnt, da);
      st.wait();
      for (uint64_t i = 0; i < da; ++i) off[i + 1] = off[i] + c[i];
      const uint64_t n_ent = off[da];
      st.upload(F.plist_off, off);
      F.plist_src.alloc(n_ent);
      F.plist_cls.alloc(n_ent);
      DevBuf<uint32_t> ent_row(n_ent, s);
      F.n_img = h.n_pairs + 3;
      F.pimg.alloc(n_ent * F.n_img);
      if (n_ent) {
        hipLaunchKernelGGL(k_pair_list, dim3(grid), dim3(256), 0, s, 1u, da, sp.n_alpha, sp.str_alpha.get(),
                           d_cls.get(), static_cast<uint32_t>(icls.size()), h.cls_meta.get(), F.plist_off.get(),
                           nullptr, F.plist_src.get(), F.plist_cls.get(), ent_row.get());
        PBS_REQUIRE(n_ent < (1ull << 31), PBS_ERR_RANGE, "more than 2^31 alpha-image entries");
        hipLaunchKernelGGL(k_pair_images, dim3(static_cast<unsigned>(n_ent)), dim3(kImgBlock), 0, s, F.n_img,
                           h.n_pairs, sp.str_alpha.get(), F.plist_cls.get(), ent_row.get(), h.cls_meta.get(),
                           h.pmap.get(), h.pg_u0.get(), h.u_t0.get(), h.pt_za.get(), h.pt_c.get(), F.cls_f.get(),
                           F.fu_t0.get(), F.ft_za.get(), F.ft_c.get(), F.pimg.get());
        PBS_HIP(hipGetLastError());
      }
      st.upload(F.pimg_flag, flag);
      F.plist = true;
    }
  }
  {
    // the image flags as uploaded to F.pimg_flag, none without images
    if (!F.plist) flag.assign(h.n_class, 0u);
    for (uint32_t c : ns) {
      F.ns_uniques += meta[c].u_end - meta[c].ua;
      F.ns_groups += meta[c].g1 - meta[c].g0;
    }
    F.ns_sizes.assign(3, 0u);
    for (int k = 0; k < 3; ++k) {
      std::vector<uint32_t> l;
      for (uint32_t c : ns)
        if (!((k != 1 && c == F.c0) || (k != 0 && flag[c]))) l.push_back(c);
      F.ns_sizes[k] = static_cast<uint32_t>(l.size());
      st.upload(F.ns_rest[k], l);
    }
  }
  PBS_HIP(hipStreamSynchronize(s));
  h.fplan = std::move(plan);
}

}  // namespace
}  // namespace pbs

using namespace pbs;

extern "C" {

pbs_status pbs_grouped_factor(pbs_grouped* h, const pbs_space* sp, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(h != nullptr && sp != nullptr, PBS_ERR_ARG, "null handle");
    PBS_REQUIRE(sp->sector, PBS_ERR_ARG, "factored evaluation needs a spin-sector space");
    PBS_REQUIRE(h->has_sector && h->half == sp->n_orb, PBS_ERR_ARG, "operator lacks sector tables for this split");
    PBS_REQUIRE(h->real_coef, PBS_ERR_UNSUPPORTED, "factored evaluation needs real sector-form coefficients");
    h->fplan.reset();
    Scratch scratch(as_stream(stream));  // temporaries of this call
    build_plan(*h, *sp, as_stream(stream));
  });
}

pbs_status pbs_grouped_set_factored(pbs_grouped* h, int32_t mode) {
  return guarded([&] {
    PBS_REQUIRE(h != nullptr, PBS_ERR_ARG, "null handle");
    PBS_REQUIRE(mode >= 0 && mode <= 7, PBS_ERR_ARG, "factored-evaluation mode must be 0..7");
    h->fact_on = static_cast<uint32_t>(mode);
  });
}

pbs_status pbs_grouped_factor_info(const pbs_grouped* h, uint32_t* info) {
  return guarded([&] {
    PBS_REQUIRE(h != nullptr && info != nullptr, PBS_ERR_ARG, "null argument");
    const FactorPlan* F = h->fplan.get();
    info[0] = F ? 1u : 0u;
    info[1] = F ? F->n_f1 : 0u;
    info[2] = F ? F->max_r1 : 0u;
    info[3] = F ? F->n_f2 : 0u;
    info[4] = F ? F->r2 : 0u;
    info[5] = F ? F->n_f3 : 0u;
    info[6] = F ? F->r3 : 0u;
    info[7] = F ? F->n_beta : 0u;
    info[8] = F && F->alist ? 1u : 0u;
    info[9] = F ? F->n_alpha : 0u;
    info[10] = F && F->plist ? 1u : 0u;
  });
}

}  // extern "C"
