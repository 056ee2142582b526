// Operator-state product by target-driven summation over X-mask groups
// (Section 2.4, Eq. reverse_sum) and, in spin sectors, over the
// spin-resolved product basis (Eq. sreverse_sum); the fused energy of
// Eq. vqe_energy.
//
// Every output amplitude is produced by exactly one thread, which gathers
// the source amplitudes psi[t ^ X_g] of all groups and multiplies each by
// its group's phase sum sum_k C_k (-1)^popcount(Z_k & s); there are no
// atomics and results are bitwise reproducible.  Amplitudes are read in
// their storage type (complex128 or complex64) and everything else --
// coefficients, phase sums, accumulators, reductions -- is float64.
//
// Sector kernel layout: a workgroup owns one target alpha string t_a (one
// row of the alpha-major state) and a range of beta columns; each lane holds
// NT targets of that row.  Groups are visited class by class (classes share
// X_alpha), so the source row s_a = t_a ^ X_alpha, its validity and its rank
// are uniform across the workgroup, and so are the alpha parities of all
// terms: each unique beta Z-mask's coefficient is folded over its terms'
// alpha parities once per group visit and applied to NT targets.
#include "handles.h"

namespace pbs {
namespace {

constexpr int kBlock = 256;

template <class T>
struct Amp;
template <>
struct Amp<double2> {
  __device__ static inline void load(const double2* p, uint64_t i, double& r, double& m) {
    const double2 v = p[i];
    r = v.x;
    m = v.y;
  }
  __device__ static inline void store(double2* p, uint64_t i, double r, double m) { p[i] = make_double2(r, m); }
};
template <>
struct Amp<float2> {
  __device__ static inline void load(const float2* p, uint64_t i, double& r, double& m) {
    const float2 v = p[i];
    r = static_cast<double>(v.x);
    m = static_cast<double>(v.y);
  }
  __device__ static inline void store(float2* p, uint64_t i, double r, double m) {
    p[i] = make_float2(static_cast<float>(r), static_cast<float>(m));
  }
};

// v * (-1)^(p & 1) by flipping the sign bit.
__device__ inline double signed_by(double v, uint32_t p) {
  return __hiloint2double(__double2hiint(v) ^ static_cast<int>((p & 1u) << 31), __double2loint(v));
}

__device__ inline void block_reduce3_store(double a, double b, double c, double* dst) {
  __shared__ double red[3][kBlock / 64];
  for (int d = 32; d > 0; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
    c += __shfl_xor(c, d, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
    red[2][wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      s0 += red[0][w];
      s1 += red[1][w];
      s2 += red[2][w];
    }
    dst[0] = s0;
    dst[1] = s1;
    dst[2] = s2;
  }
}

// ---------------------------------------------------------------- full space
template <class T, bool EXPVAL>
__global__ __launch_bounds__(kBlock) void k_apply_full(uint64_t dim, uint32_t n_groups, const uint64_t* __restrict__ xg,
                                                       const uint32_t* __restrict__ off,
                                                       const uint64_t* __restrict__ zk,
                                                       const double2* __restrict__ ck, const T* __restrict__ psi,
                                                       T* __restrict__ out, double* __restrict__ partial) {
  double e_re = 0.0, e_im = 0.0, nrm = 0.0;
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(kBlock) + threadIdx.x; t < dim;
       t += static_cast<uint64_t>(gridDim.x) * kBlock) {
    double acc_r = 0.0, acc_i = 0.0;
    for (uint32_t g = 0; g < n_groups; ++g) {
      const uint64_t s = t ^ xg[g];
      double fr = 0.0, fi = 0.0;
      const uint32_t k1 = off[g + 1];
      for (uint32_t k = off[g]; k < k1; ++k) {
        const uint32_t par = static_cast<uint32_t>(__popcll(zk[k] & s));
        const double2 c = ck[k];
        fr += signed_by(c.x, par);
        fi += signed_by(c.y, par);
      }
      double ar, ai;
      Amp<T>::load(psi, s, ar, ai);
      acc_r = fma(ar, fr, fma(-ai, fi, acc_r));
      acc_i = fma(ar, fi, fma(ai, fr, acc_i));
    }
    if (EXPVAL) {
      double pr, pi;
      Amp<T>::load(psi, t, pr, pi);
      e_re = fma(pr, acc_r, fma(pi, acc_i, e_re));
      e_im = fma(pr, acc_i, fma(-pi, acc_r, e_im));
      nrm = fma(pr, pr, fma(pi, pi, nrm));
    } else {
      Amp<T>::store(out, t, acc_r, acc_i);
    }
  }
  if (EXPVAL) block_reduce3_store(e_re, e_im, nrm, partial + 3ull * blockIdx.x);
}

// ---------------------------------------------------------------- spin sector
struct SectorArgs {
  uint32_t n_orb, n_alpha, n_beta, n_chunks;
  uint64_t dim_beta;
  uint32_t cols;  // beta columns per workgroup
  uint32_t n_class;
  const uint32_t* str_a;
  const uint32_t* str_b;
  const uint32_t* rank_tab;
  const uint32_t* cls_xa;
  const uint32_t* cls_g0;
  const uint32_t* pg_xb;
  const uint32_t* pg_u0;
  const uint32_t* u_zb;
  const uint32_t* u_t0;
  const uint32_t* pt_za;
  const double2* pt_c;
};

__device__ inline uint32_t rank_of(uint32_t s, uint32_t n_orb, uint32_t n_chunks, const uint32_t* tab) {
  uint32_t r = 0, below = 0;
  for (uint32_t c = 0; c < n_chunks; ++c) {
    const uint32_t byte = (s >> (8 * c)) & 255u;
    r += tab[(c * (n_orb + 1) + below) * 256 + byte];
    below += __popc(byte);
  }
  return r;
}

constexpr uint32_t kRankLdsEntries = 2 * 17 * 256;  // n_orb <= 16

template <class T, int NT, bool EXPVAL, bool RANK_LDS>
__global__ __launch_bounds__(kBlock) void k_apply_sector(SectorArgs P, const T* __restrict__ psi, T* __restrict__ out,
                                                         double* __restrict__ partial) {
  __shared__ uint32_t s_rank[RANK_LDS ? kRankLdsEntries : 1];
  const uint32_t* rtab = P.rank_tab;
  if (RANK_LDS) {
    const uint32_t n = P.n_chunks * (P.n_orb + 1) * 256;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) s_rank[i] = P.rank_tab[i];
    __syncthreads();
    rtab = s_rank;
  }
  const uint64_t db = P.dim_beta;
  const uint64_t ia = blockIdx.x;
  const uint32_t col0 = blockIdx.y * P.cols;
  const uint32_t col1 = (col0 + P.cols < db) ? col0 + P.cols : static_cast<uint32_t>(db);
  const uint32_t ta = P.str_a[ia];

  uint32_t tb[NT];
  bool live[NT];
  double acc_r[NT], acc_i[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const uint32_t c = col0 + threadIdx.x + j * kBlock;
    live[j] = c < col1;
    tb[j] = live[j] ? P.str_b[c] : 0u;
    acc_r[j] = 0.0;
    acc_i[j] = 0.0;
  }

  for (uint32_t cl = 0; cl < P.n_class; ++cl) {
    const uint32_t sa = ta ^ P.cls_xa[cl];
    if (static_cast<uint32_t>(__popc(sa)) != P.n_alpha) continue;  // uniform
    const uint64_t row = static_cast<uint64_t>(rank_of(sa, P.n_orb, P.n_chunks, rtab)) * db;
    const uint32_t g1 = P.cls_g0[cl + 1];
    for (uint32_t g = P.cls_g0[cl]; g < g1; ++g) {
      const uint32_t xb = P.pg_xb[g];
      uint32_t sb[NT];
      double fr[NT], fi[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        sb[j] = tb[j] ^ xb;
        fr[j] = 0.0;
        fi[j] = 0.0;
      }
      const uint32_t u1 = P.pg_u0[g + 1];
      for (uint32_t u = P.pg_u0[g]; u < u1; ++u) {
        double Fr = 0.0, Fi = 0.0;
        const uint32_t t1 = P.u_t0[u + 1];
        for (uint32_t t = P.u_t0[u]; t < t1; ++t) {
          const uint32_t par = __popc(P.pt_za[t] & sa);
          const double2 c = P.pt_c[t];
          Fr += signed_by(c.x, par);
          Fi += signed_by(c.y, par);
        }
        const uint32_t zb = P.u_zb[u];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const uint32_t par = __popc(zb & sb[j]);
          fr[j] += signed_by(Fr, par);
          fi[j] += signed_by(Fi, par);
        }
      }
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        if (live[j] && static_cast<uint32_t>(__popc(sb[j])) == P.n_beta) {
          const uint64_t src = row + rank_of(sb[j], P.n_orb, P.n_chunks, rtab);
          double ar, ai;
          Amp<T>::load(psi, src, ar, ai);
          acc_r[j] = fma(ar, fr[j], fma(-ai, fi[j], acc_r[j]));
          acc_i[j] = fma(ar, fi[j], fma(ai, fr[j], acc_i[j]));
        }
      }
    }
  }

  double e_re = 0.0, e_im = 0.0, nrm = 0.0;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    if (!live[j]) continue;
    const uint64_t t = ia * db + col0 + threadIdx.x + j * kBlock;
    if (EXPVAL) {
      double pr, pi;
      Amp<T>::load(psi, t, pr, pi);
      e_re = fma(pr, acc_r[j], fma(pi, acc_i[j], e_re));
      e_im = fma(pr, acc_i[j], fma(-pi, acc_r[j], e_im));
      nrm = fma(pr, pr, fma(pi, pi, nrm));
    } else {
      Amp<T>::store(out, t, acc_r[j], acc_i[j]);
    }
  }
  if (EXPVAL) block_reduce3_store(e_re, e_im, nrm, partial + 3ull * (blockIdx.y * gridDim.x + blockIdx.x));
}

// Sums per-workgroup partials in a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_expval_finish(const double* partial, uint64_t nparts, double* result) {
  double a = 0, b = 0, c = 0;
  for (uint64_t i = threadIdx.x; i < nparts; i += kBlock) {
    a += partial[3 * i];
    b += partial[3 * i + 1];
    c += partial[3 * i + 2];
  }
  block_reduce3_store(a, b, c, result);
}

// ---------------------------------------------------------------- launch planning
struct Launch {
  dim3 grid;
  int nt = 0;
  uint32_t cols = 0;
  uint64_t parts = 0;
};

constexpr unsigned kFullGridCap = 1u << 16;

Launch plan_launch(const pbs_space& sp) {
  Launch L;
  if (!sp.sector) {
    L.grid = dim3(grid_for(sp.dim, kBlock, kFullGridCap));
    L.parts = L.grid.x;
    return L;
  }
  const uint64_t db = sp.dim_beta;
  int nt = 8;
  if (db <= 2 * kBlock) nt = 2;
  else if (db <= 4 * kBlock) nt = 4;
  const uint64_t per = static_cast<uint64_t>(nt) * kBlock;
  const uint64_t chunks = (db + per - 1) / per;
  L.nt = nt;
  L.cols = static_cast<uint32_t>((db + chunks - 1) / chunks);
  L.grid = dim3(static_cast<unsigned>(sp.dim_alpha), static_cast<unsigned>(chunks));
  L.parts = sp.dim_alpha * chunks;
  return L;
}

void validate(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt) {
  PBS_REQUIRE(h != nullptr && sp != nullptr, PBS_ERR_ARG, "null handle");
  PBS_REQUIRE(dt == PBS_C128 || dt == PBS_C64, PBS_ERR_ARG, "unknown dtype");
  PBS_REQUIRE(h->n_qubits == sp->n_qubits, PBS_ERR_ARG,
              "operator has " + std::to_string(h->n_qubits) + " qubits, space has " + std::to_string(sp->n_qubits));
  if (sp->sector) {
    PBS_REQUIRE(h->has_sector && h->half == sp->n_orb, PBS_ERR_ARG, "operator lacks sector tables for this split");
  }
}

template <class T, bool EXPVAL>
void launch(const pbs_grouped& h, const pbs_space& sp, const void* psi, void* out, double* partial, hipStream_t s) {
  const Launch L = plan_launch(sp);
  const T* p = static_cast<const T*>(psi);
  T* o = static_cast<T*>(out);
  if (!sp.sector) {
    hipLaunchKernelGGL((k_apply_full<T, EXPVAL>), L.grid, dim3(kBlock), 0, s, sp.dim,
                       static_cast<uint32_t>(h.n_groups), h.xg.get(), h.off.get(), h.zk.get(),
                       reinterpret_cast<const double2*>(h.ck.get()), p, o, partial);
  } else {
    SectorArgs a;
    a.n_orb = sp.n_orb;
    a.n_alpha = sp.n_alpha;
    a.n_beta = sp.n_beta;
    a.n_chunks = sp.n_chunks;
    a.dim_beta = sp.dim_beta;
    a.cols = L.cols;
    a.n_class = h.n_class;
    a.str_a = sp.str_alpha.get();
    a.str_b = sp.str_beta.get();
    a.rank_tab = sp.rank_tab.get();
    a.cls_xa = h.cls_xa.get();
    a.cls_g0 = h.cls_g0.get();
    a.pg_xb = h.pg_xb.get();
    a.pg_u0 = h.pg_u0.get();
    a.u_zb = h.u_zb.get();
    a.u_t0 = h.u_t0.get();
    a.pt_za = h.pt_za.get();
    a.pt_c = reinterpret_cast<const double2*>(h.pt_c.get());
    const bool lds = sp.n_orb <= 16;
#define PBS_SECTOR(NTV)                                                                                     \
  if (lds)                                                                                                  \
    hipLaunchKernelGGL((k_apply_sector<T, NTV, EXPVAL, true>), L.grid, dim3(kBlock), 0, s, a, p, o, partial);  \
  else                                                                                                      \
    hipLaunchKernelGGL((k_apply_sector<T, NTV, EXPVAL, false>), L.grid, dim3(kBlock), 0, s, a, p, o, partial);
    if (L.nt == 2) {
      PBS_SECTOR(2)
    } else if (L.nt == 4) {
      PBS_SECTOR(4)
    } else {
      PBS_SECTOR(8)
    }
#undef PBS_SECTOR
  }
  PBS_HIP(hipGetLastError());
}

}  // namespace
}  // namespace pbs

using namespace pbs;

extern "C" {

pbs_status pbs_apply_pauli_sum(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                               void* stream) {
  return guarded([&] {
    validate(h, sp, dt);
    PBS_REQUIRE(psi != nullptr && out != nullptr, PBS_ERR_ARG, "null state pointer");
    const uint64_t bytes = sp->dim * (dt == PBS_C128 ? 16ull : 8ull);
    const auto a = reinterpret_cast<uintptr_t>(psi), b = reinterpret_cast<uintptr_t>(out);
    PBS_REQUIRE(a + bytes <= b || b + bytes <= a, PBS_ERR_ARG, "out overlaps psi");
    hipStream_t s = as_stream(stream);
    if (dt == PBS_C128)
      launch<double2, false>(*h, *sp, psi, out, nullptr, s);
    else
      launch<float2, false>(*h, *sp, psi, out, nullptr, s);
  });
}

pbs_status pbs_expval_workspace_bytes(const pbs_space* sp, uint64_t* bytes) {
  return guarded([&] {
    PBS_REQUIRE(sp != nullptr && bytes != nullptr, PBS_ERR_ARG, "null argument");
    *bytes = plan_launch(*sp).parts * 3 * sizeof(double);
  });
}

pbs_status pbs_expval(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, double* result,
                      void* work, uint64_t work_bytes, void* stream) {
  return guarded([&] {
    validate(h, sp, dt);
    PBS_REQUIRE(psi != nullptr && result != nullptr && work != nullptr, PBS_ERR_ARG, "null pointer");
    const uint64_t need = plan_launch(*sp).parts * 3 * sizeof(double);
    PBS_REQUIRE(work_bytes >= need, PBS_ERR_ARG,
                "workspace of " + std::to_string(work_bytes) + " bytes, need " + std::to_string(need));
    hipStream_t s = as_stream(stream);
    double* partial = static_cast<double*>(work);
    if (dt == PBS_C128)
      launch<double2, true>(*h, *sp, psi, nullptr, partial, s);
    else
      launch<float2, true>(*h, *sp, psi, nullptr, partial, s);
    hipLaunchKernelGGL(k_expval_finish, dim3(1), dim3(kBlock), 0, s, partial, plan_launch(*sp).parts, result);
    PBS_HIP(hipGetLastError());
  });
}

}  // extern "C"
