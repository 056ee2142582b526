// Real-time propagation psi <- exp(-i H dt) psi by short-iterative Lanczos
// (Section 2.1, Eq. real_time_evolution; the paper lists Krylov propagation
// among the consumers of the operator engine without fixing an algorithm, so
// this is the textbook method of Park and Light, 1986).
//
// Device work per Lanczos vector: one operator-state product (the sector or
// full-space apply), the three-term recurrence (alpha_j from one dot with the
// newest vector) followed by one full pass of classical Gram-Schmidt against
// all basis vectors (two multi-axpy sweeps: the first subtracts the
// recurrence terms and returns the projections, the second subtracts those
// and returns the norm), and a scale.  Inner products accumulate in float64 with a fixed-order two-stage
// reduction (deterministic).  The k x k tridiagonal matrix (k <= 16) is
// diagonalised on the host by cyclic Jacobi rotations and exp(-i T dt) e_1
// combines the basis vectors on the device.
#include <cmath>

#include "handles.h"

namespace pbs {
// the apply launcher lives in apply.hip
void apply_launch(const pbs_grouped& h, const pbs_space& sp, pbs_dtype dt, const void* psi, void* out, hipStream_t s);

namespace {

constexpr int kKB = 256;
constexpr int kMaxK = 16;
constexpr unsigned kKGrid = 4096;  // up to 16 waves per SIMD for the streaming kernels

template <class T>
struct KAmp;
template <>
struct KAmp<double2> {
  __device__ static inline double2 ld(const double2* p, uint64_t i) { return p[i]; }
  __device__ static inline void st(double2* p, uint64_t i, double r, double m) { p[i] = make_double2(r, m); }
  // the value st() stores, read back as float64
  __device__ static inline double2 stored(double r, double m) { return make_double2(r, m); }
};
template <>
struct KAmp<float2> {
  __device__ static inline double2 ld(const float2* p, uint64_t i) {
    const float2 v = p[i];
    return make_double2(v.x, v.y);
  }
  __device__ static inline void st(float2* p, uint64_t i, double r, double m) {
    p[i] = make_float2(static_cast<float>(r), static_cast<float>(m));
  }
  __device__ static inline double2 stored(double r, double m) {
    return make_double2(static_cast<float>(r), static_cast<float>(m));
  }
};

struct Coeffs {
  double re[kMaxK];
  double im[kMaxK];
};

// Block partials of ND complex sums held by every thread (ar, ai):
// partial[b * 2 * ND + 2i + {0,1}], wave shuffles then a fixed-order sum over
// the block's waves.
template <int ND>
__device__ inline void block_partials(const double (&ar)[ND], const double (&ai)[ND], double* __restrict__ partial) {
  __shared__ double red[2 * ND][kKB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    double a = ar[i], b = ai[i];
    for (int d = 32; d > 0; d >>= 1) {
      a += __shfl_xor(a, d, 64);
      b += __shfl_xor(b, d, 64);
    }
    if (lane == 0) {
      red[2 * i][wave] = a;
      red[2 * i + 1][wave] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * ND) {
    double s = 0.0;
    for (int w = 0; w < kKB / 64; ++w) s += red[threadIdx.x][w];
    partial[static_cast<uint64_t>(blockIdx.x) * 2 * ND + threadIdx.x] = s;
  }
}

// partial[b * 2 * NV + 2i + {0,1}] = sum over block b's elements of conj(x_i) * y.
// The vector count is a template argument so that the kernel holds exactly
// NV accumulator pairs (registers, hence resident waves, follow NV).
template <class T, int NV>
__global__ __launch_bounds__(kKB) void k_multidot(uint64_t n, const T* __restrict__ xbase, uint64_t stride,
                                                  const T* __restrict__ y, double* __restrict__ partial) {
  double ar[NV], ai[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) ar[i] = ai[i] = 0.0;
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(kKB) + threadIdx.x; t < n;
       t += static_cast<uint64_t>(gridDim.x) * kKB) {
    const double2 w = KAmp<T>::ld(y, t);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 v = KAmp<T>::ld(xbase + i * stride, t);
      ar[i] = fma(v.x, w.x, fma(v.y, w.y, ar[i]));
      ai[i] = fma(v.x, w.y, fma(-v.y, w.x, ai[i]));
    }
  }
  block_partials<NV>(ar, ai, partial);
}

// out[j] = sum over blocks of partial[b * nvals + j], fixed order.
__global__ __launch_bounds__(kKB) void k_sum_partials(const double* partial, int nblocks, int nvals, double* out) {
  __shared__ double red[kKB];
  for (int j = 0; j < nvals; ++j) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kKB) s += partial[static_cast<uint64_t>(b) * nvals + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kKB / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
    __syncthreads();
  }
}

// y <- beta_scale * y + sum_i c_i x_i   (float64 arithmetic, one rounding to T)
template <class T>
__global__ __launch_bounds__(kKB) void k_multiaxpy(uint64_t n, int nv, const T* __restrict__ xbase, uint64_t stride,
                                                   Coeffs c, double y_scale, T* __restrict__ y) {
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(kKB) + threadIdx.x; t < n;
       t += static_cast<uint64_t>(gridDim.x) * kKB) {
    double r = 0.0, m = 0.0;
    if (y_scale != 0.0) {
      const double2 w = KAmp<T>::ld(y, t);
      r = y_scale * w.x;
      m = y_scale * w.y;
    }
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) {
      if (i < nv) {
        const double2 v = KAmp<T>::ld(xbase + i * stride, t);
        r = fma(c.re[i], v.x, fma(-c.im[i], v.y, r));
        m = fma(c.re[i], v.y, fma(c.im[i], v.x, m));
      }
    }
    KAmp<T>::st(y, t, r, m);
  }
}

// Fused Gram-Schmidt pass: y <- y + sum_i c_i x_i, and from the same sweep
// over the elements the block partials that k_multidot would write for the
// updated y as stored: with NORM = false the inner products conj(x_i) y of
// the same x_i (the next pass's projections), with NORM = true |y|^2 (as
// k_multidot(y, y)).  Each thread visits the same elements in the same order
// as in k_multidot, so the reduced values are those of the unfused sequence
// bit for bit; y is read and written once instead of read three times and
// written once.
template <class T, bool NORM, int NV>
__global__ __launch_bounds__(kKB) void k_multiaxpy_dot(uint64_t n, const T* __restrict__ xbase, uint64_t stride,
                                                       Coeffs c, T* __restrict__ y, double* __restrict__ partial) {
  constexpr int kD = NORM ? 1 : NV;
  double ar[kD], ai[kD];
#pragma unroll
  for (int i = 0; i < kD; ++i) ar[i] = ai[i] = 0.0;
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(kKB) + threadIdx.x; t < n;
       t += static_cast<uint64_t>(gridDim.x) * kKB) {
    const double2 w0 = KAmp<T>::ld(y, t);
    double r = w0.x, m = w0.y;
    double2 v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      v[i] = KAmp<T>::ld(xbase + i * stride, t);
      r = fma(c.re[i], v[i].x, fma(-c.im[i], v[i].y, r));
      m = fma(c.re[i], v[i].y, fma(c.im[i], v[i].x, m));
    }
    KAmp<T>::st(y, t, r, m);
    const double2 w = KAmp<T>::stored(r, m);
    if (NORM) {
      ar[0] = fma(w.x, w.x, fma(w.y, w.y, ar[0]));
      ai[0] = fma(w.x, w.y, fma(-w.y, w.x, ai[0]));
    } else {
#pragma unroll
      for (int i = 0; i < kD; ++i) {
        ar[i] = fma(v[i].x, w.x, fma(v[i].y, w.y, ar[i]));
        ai[i] = fma(v[i].x, w.y, fma(-v[i].y, w.x, ai[i]));
      }
    }
  }
  block_partials<kD>(ar, ai, partial);
}

// Launches K<NV> for the runtime count nv in 1..kMaxK.
template <template <int> class K, int NV = 1, class... A>
void launch_nv(int nv, dim3 grid, hipStream_t s, A... args) {
  if constexpr (NV <= kMaxK) {
    if (nv == NV) {
      hipLaunchKernelGGL(K<NV>::fn(), grid, dim3(kKB), 0, s, args...);
      return;
    }
    launch_nv<K, NV + 1>(nv, grid, s, args...);
  } else {
    PBS_REQUIRE(false, PBS_ERR_RANGE, "vector count outside 1..16");
  }
}
template <class T>
struct DotK {
  template <int NV>
  struct K {
    static auto fn() { return k_multidot<T, NV>; }
  };
};
template <class T, bool NORM>
struct AxpyDotK {
  template <int NV>
  struct K {
    static auto fn() { return k_multiaxpy_dot<T, NORM, NV>; }
  };
};

template <class T>
__global__ __launch_bounds__(kKB) void k_scale_copy(uint64_t n, const T* __restrict__ x, double s, T* __restrict__ y) {
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(kKB) + threadIdx.x; t < n;
       t += static_cast<uint64_t>(gridDim.x) * kKB) {
    const double2 v = KAmp<T>::ld(x, t);
    KAmp<T>::st(y, t, s * v.x, s * v.y);
  }
}

// Cyclic Jacobi eigen-decomposition of a symmetric k x k matrix (row-major);
// on return a holds the eigenvalues on its diagonal and u the eigenvectors
// (columns).
void jacobi_eigen(int k, std::vector<double>& a, std::vector<double>& u) {
  u.assign(static_cast<size_t>(k) * k, 0.0);
  for (int i = 0; i < k; ++i) u[i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < k; ++i) {
      diag += a[i * k + i] * a[i * k + i];
      for (int j = i + 1; j < k; ++j) off += a[i * k + j] * a[i * k + j];
    }
    if (off <= 1e-34 * (diag + 1e-300)) break;
    for (int p = 0; p < k; ++p) {
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[p * k + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {  // A <- A J (columns p, q)
          const double arp = a[r * k + p], arq = a[r * k + q];
          a[r * k + p] = c * arp - s * arq;
          a[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {  // A <- J^T A (rows p, q)
          const double apr = a[p * k + r], aqr = a[q * k + r];
          a[p * k + r] = c * apr - s * aqr;
          a[q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {  // U <- U J
          const double urp = u[r * k + p], urq = u[r * k + q];
          u[r * k + p] = c * urp - s * urq;
          u[r * k + q] = s * urp + c * urq;
        }
      }
    }
  }
}

size_t elem_size(pbs_dtype dt) { return dt == PBS_C128 ? 16 : 8; }

size_t partial_doubles() { return static_cast<size_t>(kKGrid) * 2 * kMaxK; }

uint64_t workspace_bytes(const pbs_space& sp, pbs_dtype dt, uint32_t m) {
  const uint64_t vec = sp.dim * elem_size(dt);
  return (m + 1) * ((vec + 255) & ~255ull) + (partial_doubles() + 2 * kMaxK) * sizeof(double);
}

template <class T>
class Lanczos {
 public:
  Lanczos(const pbs_grouped& h, const pbs_space& sp, pbs_dtype dt, uint32_t m, unsigned char* work, hipStream_t s)
      : h_(h), sp_(sp), dt_(dt), m_(m), s_(s), n_(sp.dim) {
    stride_ = (n_ * sizeof(T) + 255) & ~255ull;
    V_ = reinterpret_cast<T*>(work);
    W_ = reinterpret_cast<T*>(work + m * stride_);
    partial_ = reinterpret_cast<double*>(work + (m + 1) * stride_);
    dots_ = partial_ + partial_doubles();
    grid_ = grid_for(n_, kKB, kKGrid);
  }
  T* vec(uint32_t i) const { return reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(V_) + i * stride_); }
  uint64_t stride_elems() const { return stride_ / sizeof(T); }

  // returns sum_i conj(x_i) y for x_0..x_{nv-1} starting at xbase
  void dots(const T* xbase, int nv, const T* y, double* host) {
    launch_nv<DotK<T>::template K>(nv, dim3(grid_), s_, n_, xbase, stride_elems(), y, partial_);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kKB), 0, s_, partial_, static_cast<int>(grid_), 2 * nv, dots_);
    PBS_HIP(hipGetLastError());
    PBS_HIP(hipMemcpyAsync(host, dots_, 2 * nv * sizeof(double), hipMemcpyDeviceToHost, s_));
    PBS_HIP(hipStreamSynchronize(s_));
  }
  // y <- y + sum_i c_i x_i, then (host) sum_i conj(x_i) y, or |y|^2 with norm
  void axpy_dots(const T* xbase, int nv, const double* cre, const double* cim, T* y, bool norm, double* host) {
    Coeffs c{};
    for (int i = 0; i < nv; ++i) {
      c.re[i] = cre[i];
      c.im[i] = cim[i];
    }
    if (norm)
      launch_nv<AxpyDotK<T, true>::template K>(nv, dim3(grid_), s_, n_, xbase, stride_elems(), c, y, partial_);
    else
      launch_nv<AxpyDotK<T, false>::template K>(nv, dim3(grid_), s_, n_, xbase, stride_elems(), c, y, partial_);
    const int nd = norm ? 1 : nv;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kKB), 0, s_, partial_, static_cast<int>(grid_), 2 * nd, dots_);
    PBS_HIP(hipGetLastError());
    PBS_HIP(hipMemcpyAsync(host, dots_, 2 * nd * sizeof(double), hipMemcpyDeviceToHost, s_));
    PBS_HIP(hipStreamSynchronize(s_));
  }
  void axpy(const T* xbase, int nv, const double* cre, const double* cim, double y_scale, T* y) {
    Coeffs c{};
    for (int i = 0; i < nv; ++i) {
      c.re[i] = cre[i];
      c.im[i] = cim[i];
    }
    hipLaunchKernelGGL((k_multiaxpy<T>), dim3(grid_), dim3(kKB), 0, s_, n_, nv, xbase, stride_elems(), c, y_scale, y);
    PBS_HIP(hipGetLastError());
  }

  void step(T* psi, double dt, double* info) {
    double d[2 * kMaxK];
    dots(psi, 1, psi, d);
    const double nrm = std::sqrt(d[0]);
    info[0] = nrm;
    if (!(nrm > 0.0)) {
      info[1] = 0.0;
      info[2] = 0.0;
      info[3] = 0.0;
      return;
    }
    hipLaunchKernelGGL((k_scale_copy<T>), dim3(grid_), dim3(kKB), 0, s_, n_, psi, 1.0 / nrm, vec(0));
    PBS_HIP(hipGetLastError());
    std::vector<double> alpha, beta;
    double scale = 0.0, last_b = 0.0;
    uint32_t k = 0;
    for (uint32_t j = 0; j < m_; ++j) {
      apply_launch(h_, sp_, dt_, vec(j), W_, s_);
      // the three-term recurrence: alpha_j = <v_j, w> on the fresh product
      // (H is Hermitian, so w has no other component in exact arithmetic)
      dots(vec(j), 1, W_, d);
      alpha.push_back(d[0]);
      double nre[kMaxK] = {}, nim[kMaxK] = {};
      nre[j] = -d[0];
      nim[j] = -d[1];
      if (j > 0) nre[j - 1] = -beta[j - 1];
      // subtract alpha_j v_j + beta_{j-1} v_{j-1}, and in the same sweep the
      // projections on every basis vector (full re-orthogonalisation)
      axpy_dots(vec(0), static_cast<int>(j + 1), nre, nim, W_, false, d);
      for (uint32_t i = 0; i <= j; ++i) {
        nre[i] = -d[2 * i];
        nim[i] = -d[2 * i + 1];
      }
      // subtract those, and in the same sweep |w|^2
      axpy_dots(vec(0), static_cast<int>(j + 1), nre, nim, W_, true, d);
      const double b = std::sqrt(std::max(d[0], 0.0));
      last_b = b;
      scale = std::max(scale, std::max(std::fabs(alpha.back()), b));
      k = j + 1;
      if (j + 1 == m_ || b <= 1e-14 * scale) break;
      beta.push_back(b);
      hipLaunchKernelGGL((k_scale_copy<T>), dim3(grid_), dim3(kKB), 0, s_, n_, W_, 1.0 / b, vec(j + 1));
      PBS_HIP(hipGetLastError());
    }
    // exp(-i T dt) e_1 from the eigen-decomposition of the tridiagonal T
    std::vector<double> a(static_cast<size_t>(k) * k, 0.0), u;
    for (uint32_t i = 0; i < k; ++i) a[i * k + i] = alpha[i];
    for (uint32_t i = 0; i + 1 < k; ++i) a[i * k + i + 1] = a[(i + 1) * k + i] = beta[i];
    jacobi_eigen(static_cast<int>(k), a, u);
    double cre[kMaxK], cim[kMaxK];
    for (uint32_t r = 0; r < k; ++r) {
      double sr = 0.0, si = 0.0;
      for (uint32_t q = 0; q < k; ++q) {
        const double lam = a[q * k + q];
        const double w = u[r * k + q] * u[0 * k + q];
        sr += w * std::cos(lam * dt);
        si -= w * std::sin(lam * dt);
      }
      cre[r] = nrm * sr;
      cim[r] = nrm * si;
    }
    axpy(vec(0), static_cast<int>(k), cre, cim, 0.0, psi);
    PBS_HIP(hipStreamSynchronize(s_));
    info[1] = alpha[0];
    info[2] = static_cast<double>(k);
    info[3] = last_b;
  }

 private:
  const pbs_grouped& h_;
  const pbs_space& sp_;
  pbs_dtype dt_;
  uint32_t m_;
  hipStream_t s_;
  uint64_t n_;
  uint64_t stride_ = 0;
  T* V_ = nullptr;
  T* W_ = nullptr;
  double* partial_ = nullptr;
  double* dots_ = nullptr;
  unsigned grid_ = 1;
};

}  // namespace
}  // namespace pbs

using namespace pbs;

extern "C" {

pbs_status pbs_krylov_workspace_bytes(const pbs_space* sp, pbs_dtype dt, uint32_t m, uint64_t* bytes) {
  return guarded([&] {
    PBS_REQUIRE(sp != nullptr && bytes != nullptr, PBS_ERR_ARG, "null argument");
    PBS_REQUIRE(dt == PBS_C128 || dt == PBS_C64, PBS_ERR_ARG, "unknown dtype");
    PBS_REQUIRE(m >= 1 && m <= static_cast<uint32_t>(kMaxK), PBS_ERR_RANGE, "m must be 1..16");
    *bytes = workspace_bytes(*sp, dt, m);
  });
}

pbs_status pbs_krylov_step(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, void* psi, double dt_step,
                           uint32_t m, void* work, uint64_t work_bytes, double* info, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(h != nullptr && sp != nullptr && psi != nullptr && work != nullptr && info != nullptr,
                PBS_ERR_ARG, "null argument");
    PBS_REQUIRE(dt == PBS_C128 || dt == PBS_C64, PBS_ERR_ARG, "unknown dtype");
    PBS_REQUIRE(m >= 1 && m <= static_cast<uint32_t>(kMaxK), PBS_ERR_RANGE, "m must be 1..16");
    PBS_REQUIRE(std::isfinite(dt_step), PBS_ERR_ARG, "dt is not finite");
    PBS_REQUIRE(work_bytes >= workspace_bytes(*sp, dt, m), PBS_ERR_ARG, "workspace too small");
    const auto a = reinterpret_cast<uintptr_t>(psi), w = reinterpret_cast<uintptr_t>(work);
    const uint64_t pb = sp->dim * elem_size(dt);
    PBS_REQUIRE(a + pb <= w || w + work_bytes <= a, PBS_ERR_ARG, "psi overlaps the workspace");
    hipStream_t s = as_stream(stream);
    unsigned char* wk = static_cast<unsigned char*>(work);
    if (dt == PBS_C128) {
      Lanczos<double2> L(*h, *sp, dt, m, wk, s);
      L.step(static_cast<double2*>(psi), dt_step, info);
    } else {
      Lanczos<float2> L(*h, *sp, dt, m, wk, s);
      L.step(static_cast<float2*>(psi), dt_step, info);
    }
  });
}

}  // extern "C"
