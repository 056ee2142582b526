// Variational layer on top of the operator-state product: an ansatz of
// Pauli rotations exp(i theta_k P_k) acting on a reference basis state in the
// full 2^n space, its energy <psi(theta)|H|psi(theta)> (Section 2.1, Eq.
// vqe_energy) and the gradient of that energy by the adjoint method.
//
// A number- and S_z-conserving H acts on each (N_alpha, N_beta) sector of the
// full space separately, so the full-space product H|psi> is computed by
// permuting psi into sector blocks (each block alpha-major, the layout of a
// sector space), running the batched sector kernel over all blocks in one
// launch, and permuting back.  Rotations and overlaps are bandwidth-bound
// passes over the full-space vectors.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "sector.h"

namespace pbs {
namespace {

// XZ form of a Hermitian letter-form string: P|s> = omega (-1)^popcount(z & s) |s ^ x>
// with omega = i^popcount(x & z) (Section 2.3).
struct Rot {
  uint64_t x, z;
  uint32_t omega;  // power of i, 0..3
};

// i^k * (r, m)
__device__ inline void times_i_pow(uint32_t k, double& r, double& m) {
  const double a = r, b = m;
  switch (k & 3u) {
    case 0: break;
    case 1: r = -b; m = a; break;
    case 2: r = -a; m = -b; break;
    default: r = b; m = -a; break;
  }
}

// psi <- (cos theta + i sin theta P) psi over pairs (t, t ^ x), t with the
// highest bit of x clear; x = 0 is a diagonal phase.
template <class T>
__global__ __launch_bounds__(kBlock) void k_rotate(T* __restrict__ psi, uint64_t dim, uint64_t x, uint64_t z,
                                                    uint32_t omega, double c, double s) {
  if (x == 0) {
    for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < dim;
         t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
      double pr, pi;
      Amp<T>::load(psi, t, pr, pi);
      double fr = 0.0, fi = signed_by(s, __popcll(z & t));  // i s (-1)^(z.t) omega
      times_i_pow(omega, fr, fi);
      const double gr = c + fr, gi = fi;
      Amp<T>::store(psi, t, pr * gr - pi * gi, pr * gi + pi * gr);
    }
    return;
  }
  const uint32_t h = 63u - static_cast<uint32_t>(__clzll(static_cast<long long>(x)));
  const uint64_t low = (1ull << h) - 1ull;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < dim / 2;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t t = ((i & ~low) << 1) | (i & low);  // bit h clear
    const uint64_t u = t ^ x;
    double ar, ai, br, bi;
    Amp<T>::load(psi, t, ar, ai);
    Amp<T>::load(psi, u, br, bi);
    // (P psi)[t] = omega (-1)^(z.u) psi[u], (P psi)[u] = omega (-1)^(z.t) psi[t]
    double pr = signed_by(br, __popcll(z & u)), pi = signed_by(bi, __popcll(z & u));
    double qr = signed_by(ar, __popcll(z & t)), qi = signed_by(ai, __popcll(z & t));
    times_i_pow(omega + 1u, pr, pi);  // i * omega
    times_i_pow(omega + 1u, qr, qi);
    Amp<T>::store(psi, t, c * ar + s * pr, c * ai + s * pi);
    Amp<T>::store(psi, u, c * br + s * qr, c * bi + s * qi);
  }
}

// One step of the adjoint sweep in a single pass: workgroup partials of
// <lam|P|psi> = sum_t conj(lam[t]) (P psi)[t], then psi <- R^dagger psi and
// lam <- R^dagger lam
// with R^dagger = cos theta - i sin theta P, all from the same loads.  c, s
// are cos(-theta), sin(-theta).
template <class T>
__global__ __launch_bounds__(kBlock) void k_adjoint_step(T* __restrict__ psi, T* __restrict__ lam, uint64_t dim,
                                                          uint64_t x, uint64_t z, uint32_t omega, double c, double s,
                                                          double* __restrict__ partial) {
  double sr = 0.0, si = 0.0;
  if (x == 0) {
    for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < dim;
         t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
      double pr, pi, lr, li;
      Amp<T>::load(psi, t, pr, pi);
      Amp<T>::load(lam, t, lr, li);
      double wr = signed_by(1.0, __popcll(z & t)), wi = 0.0;  // P|t> = w |t>
      times_i_pow(omega, wr, wi);
      const double qr = wr * pr - wi * pi, qi = wr * pi + wi * pr;  // (P psi)[t]
      sr = fma(lr, qr, fma(li, qi, sr));
      si = fma(lr, qi, fma(-li, qr, si));
      const double gr = c - s * wi, gi = s * wr;  // c + i s w
      Amp<T>::store(psi, t, pr * gr - pi * gi, pr * gi + pi * gr);
      Amp<T>::store(lam, t, lr * gr - li * gi, lr * gi + li * gr);
    }
  } else {
    const uint32_t h = 63u - static_cast<uint32_t>(__clzll(static_cast<long long>(x)));
    const uint64_t low = (1ull << h) - 1ull;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < dim / 2;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
      const uint64_t t = ((i & ~low) << 1) | (i & low);
      const uint64_t u = t ^ x;
      double atr, ati, aur, aui, btr, bti, bur, bui;  // psi[t], psi[u], lam[t], lam[u]
      Amp<T>::load(psi, t, atr, ati);
      Amp<T>::load(psi, u, aur, aui);
      Amp<T>::load(lam, t, btr, bti);
      Amp<T>::load(lam, u, bur, bui);
      const uint32_t pu = __popcll(z & u), pt = __popcll(z & t);
      // (P v)[t] = omega (-1)^(z.u) v[u], (P v)[u] = omega (-1)^(z.t) v[t]
      double ptr = signed_by(aur, pu), pti = signed_by(aui, pu);
      double pur = signed_by(atr, pt), pui = signed_by(ati, pt);
      double qtr = signed_by(bur, pu), qti = signed_by(bui, pu);
      double qur = signed_by(btr, pt), qui = signed_by(bti, pt);
      times_i_pow(omega, ptr, pti);
      times_i_pow(omega, pur, pui);
      times_i_pow(omega, qtr, qti);
      times_i_pow(omega, qur, qui);
      sr = fma(btr, ptr, fma(bti, pti, sr));
      si = fma(btr, pti, fma(-bti, ptr, si));
      sr = fma(bur, pur, fma(bui, pui, sr));
      si = fma(bur, pui, fma(-bui, pur, si));
      // v <- c v + i s (P v)
      Amp<T>::store(psi, t, c * atr - s * pti, c * ati + s * ptr);
      Amp<T>::store(psi, u, c * aur - s * pui, c * aui + s * pur);
      Amp<T>::store(lam, t, c * btr - s * qti, c * bti + s * qtr);
      Amp<T>::store(lam, u, c * bur - s * qui, c * bui + s * qur);
    }
  }
  block_reduce3_store<kBlock>(sr, si, 0.0, partial + 3ull * blockIdx.x);
}

// ---------------------------------------------------------------- K rotations per pass
// K consecutive rotations whose X masks are linearly independent over GF(2)
// act together on the orbits t ^ span{x_0 .. x_{K-1}} of 2^K indices.
// Gaussian elimination gives a basis b_j of the span with leading bit p_j and
// bit p_i of b_j clear for i < j; projecting the span onto the pivot bits is
// then one to one, so every orbit holds exactly one index with all pivot bits
// clear, enumerated by inserting zero bits at the sorted pivots into i.
// Element e of an orbit is t0 ^ (sum over the set bits j of e of x_j), so
// rotation j pairs the elements that differ in bit j of e.
struct PairRot {
  uint64_t x, z;
  uint32_t omega;
  double c, s;
};

struct Cx {
  double r, i;
};

// (P v)[t] for the pair (t, u = t ^ x): omega (-1)^(z.u) v[u]
__device__ inline Cx pauli_image(const Cx& vu, uint64_t z, uint64_t u, uint32_t omega) {
  const uint32_t p = __popcll(z & u);
  double r = signed_by(vu.r, p), m = signed_by(vu.i, p);
  times_i_pow(omega, r, m);
  return Cx{r, m};
}

// (vt, vu) <- (c vt + i s (P v)[t], c vu + i s (P v)[u])
__device__ inline void rotate_pair(Cx& vt, Cx& vu, uint64_t t, uint64_t u, const PairRot& R) {
  const Cx pt = pauli_image(vu, R.z, u, R.omega), pu = pauli_image(vt, R.z, t, R.omega);
  vt = Cx{R.c * vt.r - R.s * pt.i, R.c * vt.i + R.s * pt.r};
  vu = Cx{R.c * vu.r - R.s * pu.i, R.c * vu.i + R.s * pu.r};
}

// acc += conj(l[t]) (P a)[t] + conj(l[u]) (P a)[u]
__device__ inline void overlap_pair(const Cx& at, const Cx& au, const Cx& lt, const Cx& lu, uint64_t t, uint64_t u,
                                    const PairRot& R, double& sr, double& si) {
  const Cx pt = pauli_image(au, R.z, u, R.omega), pu = pauli_image(at, R.z, t, R.omega);
  sr = fma(lt.r, pt.r, fma(lt.i, pt.i, sr));
  si = fma(lt.r, pt.i, fma(-lt.i, pt.r, si));
  sr = fma(lu.r, pu.r, fma(lu.i, pu.i, sr));
  si = fma(lu.r, pu.i, fma(-lu.i, pu.r, si));
}

// One adjoint step on the pair (t, u = t ^ x) of both vectors:
// acc += conj(l) (P p) over the pair, then p <- R p and l <- R l with the
// pair's two Z parities evaluated once.
__device__ inline void adjoint_pair(Cx& pt, Cx& pu, Cx& lt, Cx& lu, uint64_t t, uint64_t u, const PairRot& R,
                                    double& sr, double& si) {
  const uint32_t qt = __popcll(R.z & t), qu = __popcll(R.z & u);
  auto image = [&](const Cx& v, uint32_t q) {
    double r = signed_by(v.r, q), m = signed_by(v.i, q);
    times_i_pow(R.omega, r, m);
    return Cx{r, m};
  };
  const Cx a_t = image(pu, qu), a_u = image(pt, qt);  // (P p)[t], (P p)[u]
  sr = fma(lt.r, a_t.r, fma(lt.i, a_t.i, sr));
  si = fma(lt.r, a_t.i, fma(-lt.i, a_t.r, si));
  sr = fma(lu.r, a_u.r, fma(lu.i, a_u.i, sr));
  si = fma(lu.r, a_u.i, fma(-lu.i, a_u.r, si));
  const Cx b_t = image(lu, qu), b_u = image(lt, qt);  // (P l)[t], (P l)[u]
  pt = Cx{R.c * pt.r - R.s * a_t.i, R.c * pt.i + R.s * a_t.r};
  pu = Cx{R.c * pu.r - R.s * a_u.i, R.c * pu.i + R.s * a_u.r};
  lt = Cx{R.c * lt.r - R.s * b_t.i, R.c * lt.i + R.s * b_t.r};
  lu = Cx{R.c * lu.r - R.s * b_u.i, R.c * lu.i + R.s * b_u.r};
}

__device__ inline uint64_t insert_zero(uint64_t v, uint32_t b) {
  const uint64_t low = (1ull << b) - 1ull;
  return ((v & ~low) << 1) | (v & low);
}

template <class T>
__device__ inline Cx load_cx(const T* p, uint64_t i) {
  Cx v;
  Amp<T>::load(p, i, v.r, v.i);
  return v;
}

template <class T>
__device__ inline void store_cx(T* p, uint64_t i, const Cx& v) {
  Amp<T>::store(p, i, v.r, v.i);
}

template <int K>
struct RotGroup {
  PairRot r[K];      // in application order
  uint32_t piv[K];   // pivot bits, ascending
};

template <int K>
__device__ inline uint64_t orbit_base(uint64_t i, const RotGroup<K>& G) {
  uint64_t t = i;
#pragma unroll
  for (int j = 0; j < K; ++j) t = insert_zero(t, G.piv[j]);
  return t;
}

// psi <- R_{K-1} ... R_0 psi
template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_rotate_group(T* __restrict__ psi, uint64_t dim, RotGroup<K> G) {
  constexpr int N = 1 << K;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < (dim >> K);
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    uint64_t t[N];
    t[0] = orbit_base(i, G);
#pragma unroll
    for (int e = 1; e < N; ++e) t[e] = t[e & (e - 1)] ^ G.r[__builtin_ctz(e)].x;
    Cx v[N];
#pragma unroll
    for (int e = 0; e < N; ++e) v[e] = load_cx(psi, t[e]);
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int e = 0; e < N; ++e)
        if (!(e & (1 << j))) rotate_pair(v[e], v[e | (1 << j)], t[e], t[e | (1 << j)], G.r[j]);
#pragma unroll
    for (int e = 0; e < N; ++e) store_cx(psi, t[e], v[e]);
  }
}

// K adjoint steps in one pass: with psi and lam taken after rotation K-1 on
// entry, for j = K-1 down to 0: partials of <lam|P_j|psi>, then R_j^dagger
// on both vectors (G carries cos, sin of -theta).  partial_j = partial +
// 3 * stride * j.
template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_adjoint_group(T* __restrict__ psi, T* __restrict__ lam, uint64_t dim,
                                                           RotGroup<K> G, double* __restrict__ partial,
                                                           uint64_t stride) {
  constexpr int N = 1 << K;
  double ov[2 * K];
#pragma unroll
  for (int j = 0; j < 2 * K; ++j) ov[j] = 0.0;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < (dim >> K);
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    uint64_t t[N];
    t[0] = orbit_base(i, G);
#pragma unroll
    for (int e = 1; e < N; ++e) t[e] = t[e & (e - 1)] ^ G.r[__builtin_ctz(e)].x;
    Cx p[N], l[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
      p[e] = load_cx(psi, t[e]);
      l[e] = load_cx(lam, t[e]);
    }
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
#pragma unroll
      for (int e = 0; e < N; ++e)
        if (!(e & (1 << j)))
          adjoint_pair(p[e], p[e | (1 << j)], l[e], l[e | (1 << j)], t[e], t[e | (1 << j)], G.r[j], ov[2 * j],
                       ov[2 * j + 1]);
    }
#pragma unroll
    for (int e = 0; e < N; ++e) {
      store_cx(psi, t[e], p[e]);
      store_cx(lam, t[e], l[e]);
    }
  }
  __shared__ double red[2 * K][kBlock / 64];
#pragma unroll
  for (int j = 0; j < 2 * K; ++j)
    for (int d = 32; d > 0; d >>= 1) ov[j] += __shfl_xor(ov[j], d, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) red[j][wave] = ov[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double sr = 0.0, si = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) {
        sr += red[2 * j][w];
        si += red[2 * j + 1][w];
      }
      double* out = partial + 3ull * stride * j + 3ull * blockIdx.x;
      out[0] = sr;
      out[1] = si;
      out[2] = 0.0;
    }
  }
}

// out[k] = (sum of the partials of overlap k, real and imaginary parts), fixed order.
__global__ __launch_bounds__(kBlock) void k_sum_overlaps(const double* partial, uint32_t nparts, double* out) {
  const double* p = partial + 3ull * nparts * blockIdx.x;
  double a = 0.0, b = 0.0;
  for (uint32_t i = threadIdx.x; i < nparts; i += kBlock) {
    a += p[3ull * i];
    b += p[3ull * i + 1];
  }
  double r[3];
  block_reduce3_store<kBlock>(a, b, 0.0, r);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = r[0];
    out[2 * blockIdx.x + 1] = r[1];
  }
}

__global__ void k_basis_state(double2* psi64, float2* psi32, uint64_t dim, uint64_t ref) {
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < dim;
       t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const double v = t == ref ? 1.0 : 0.0;
    if (psi64) psi64[t] = make_double2(v, 0.0);
    if (psi32) psi32[t] = make_float2(static_cast<float>(v), 0.0f);
  }
}

constexpr uint64_t kTransposed = 1ull << 63;  // block offset flag: stored as sector (N_beta, N_alpha)

// Colexicographic rank of a spin string from T[c][k][byte] tables.
__device__ inline uint32_t colex_rank(uint32_t s, uint32_t n_orb, uint32_t n_chunks, const uint32_t* tab) {
  uint32_t r = 0, below = 0;
  for (uint32_t c = 0; c < n_chunks; ++c) {
    const uint32_t byte = (s >> (8 * c)) & 255u;
    r += tab[(c * (n_orb + 1) + below) * 256 + byte];
    below += __popc(byte);
  }
  return r;
}

// Full-space index s = alpha | beta << n_orb  <->  sector-block index
// off[N_alpha][N_beta] + rank(alpha) C(n_orb, N_beta) + rank(beta), or, for a
// block flagged transposed (top bit of its offset), + rank(beta) C(n_orb,
// N_alpha) + rank(alpha): the layout of sector (N_beta, N_alpha).
template <class T, bool TO_BLOCKS>
__global__ __launch_bounds__(kBlock) void k_fock_permute(const T* __restrict__ in, T* __restrict__ out, uint64_t dim,
                                                          uint32_t n_orb, uint32_t n_chunks,
                                                          const uint32_t* __restrict__ tab,
                                                          const uint64_t* __restrict__ off,
                                                          const uint32_t* __restrict__ binom_n) {
  const uint32_t mask = (1u << n_orb) - 1u;
  for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < dim;
       s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t a = static_cast<uint32_t>(s) & mask, b = static_cast<uint32_t>(s >> n_orb);
    const uint32_t pa = __popc(a), pb = __popc(b);
    const uint64_t o = off[pa * (n_orb + 1) + pb];
    const uint64_t ra = colex_rank(a, n_orb, n_chunks, tab), rb = colex_rank(b, n_orb, n_chunks, tab);
    const uint64_t j = (o & ~kTransposed) + ((o & kTransposed) ? rb * binom_n[pa] + ra : ra * binom_n[pb] + rb);
    if (TO_BLOCKS)
      out[j] = in[s];
    else
      out[s] = in[j];
  }
}

Rot rot_of(uint64_t x, uint64_t z) { return Rot{x, z, static_cast<uint32_t>(__builtin_popcountll(x & z) & 3)}; }

// Whether H conserves N_alpha and N_beta (H commutes with both), decided on
// the grouped XZ form.  Group g couples s to t = s ^ X_g with matrix element
// f_g(s) = sum_k C_k (-1)^popcount(Z_k & s).  The numbers are conserved iff
// f_g(s) = 0 for every s on which X_g flips unequal numbers of set and unset
// bits in either half; that set depends only on the bits of s inside X_g, so
// splitting Z_k into its parts inside and outside X_g (the characters of the
// outside bits are independent) leaves, per distinct outside part, a function
// of the |X_g| inside bits to evaluate at every bad pattern.  Sums that cancel
// are accepted up to 1e-12 of the absolute coefficient sum (rounding).
bool conserves_spin_numbers(const pbs_grouped& h, hipStream_t s, std::string* why) {
  const uint32_t n = h.half;
  std::vector<uint64_t> xg(h.n_groups), zk(h.n_terms);
  std::vector<uint32_t> off(h.n_groups + 1);
  std::vector<double> ck(2 * h.n_terms);
  PBS_HIP(hipMemcpyAsync(xg.data(), h.xg.get(), xg.size() * 8, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(off.data(), h.off.get(), off.size() * 4, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(zk.data(), h.zk.get(), zk.size() * 8, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(ck.data(), h.ck.get(), ck.size() * 8, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipStreamSynchronize(s));
  const uint64_t mask = (1ull << n) - 1ull;
  for (uint64_t g = 0; g < h.n_groups; ++g) {
    const uint64_t x = xg[g];
    if (x == 0) continue;  // diagonal
    const int fa = __builtin_popcountll(x & mask), fb = __builtin_popcountll(x >> n);
    const int m = fa + fb;
    if (m > 20) {
      *why = "a group flips more than 20 qubits; conservation of N_alpha and N_beta cannot be checked";
      return false;
    }
    uint32_t bit[64];
    for (int i = 0, q = 0; q < 64; ++q)
      if ((x >> q) & 1ull) bit[i++] = static_cast<uint32_t>(q);
    // inside patterns u (bit i of u = qubit bit[i] of s) that change N_alpha or N_beta
    std::vector<uint32_t> bad;
    for (uint32_t u = 0; u < (1u << m); ++u) {
      const int ua = __builtin_popcount(u & ((1u << fa) - 1u)), ub = __builtin_popcount(u >> fa);
      if (2 * ua != fa || 2 * ub != fb) bad.push_back(u);
    }
    // terms of the group ordered by their Z part outside X
    std::vector<uint32_t> ks;
    for (uint32_t k = off[g]; k < off[g + 1]; ++k) ks.push_back(k);
    std::stable_sort(ks.begin(), ks.end(), [&](uint32_t a, uint32_t b) { return (zk[a] & ~x) < (zk[b] & ~x); });
    for (size_t i0 = 0; i0 < ks.size();) {
      size_t i1 = i0;
      double scale = 0.0;
      while (i1 < ks.size() && (zk[ks[i1]] & ~x) == (zk[ks[i0]] & ~x)) {
        scale += std::fabs(ck[2 * ks[i1]]) + std::fabs(ck[2 * ks[i1] + 1]);
        ++i1;
      }
      for (uint32_t u : bad) {
        double fr = 0.0, fi = 0.0;
        for (size_t i = i0; i < i1; ++i) {
          const uint64_t zin = zk[ks[i]] & x;
          int par = 0;
          for (int b = 0; b < m; ++b) par ^= static_cast<int>(((u >> b) & 1u) & ((zin >> bit[b]) & 1ull));
          fr += par ? -ck[2 * ks[i]] : ck[2 * ks[i]];
          fi += par ? -ck[2 * ks[i] + 1] : ck[2 * ks[i] + 1];
        }
        if (std::fabs(fr) + std::fabs(fi) > 1e-12 * scale) {
          char buf[96];
          std::snprintf(buf, sizeof(buf), "the group with X mask 0x%llx changes N_alpha or N_beta",
                        static_cast<unsigned long long>(x));
          *why = buf;
          return false;
        }
      }
      i0 = i1;
    }
  }
  return true;
}


// True when exchanging the two qubit halves maps the operator onto itself
// term by term (bit-identical coefficients), as for the Jordan-Wigner
// Hamiltonian of spin-free integrals.  Then H = S H S for the half-exchange
// S, so block (N_alpha, N_beta) of H psi equals, element for element, block
// (N_beta, N_alpha) of H (S psi).
bool halves_symmetric(const pbs_grouped& h, hipStream_t s) {
  const uint32_t n = h.half;
  std::vector<uint64_t> xg(h.n_groups), zk(h.n_terms);
  std::vector<uint32_t> off(h.n_groups + 1);
  std::vector<double> ck(2 * h.n_terms);
  PBS_HIP(hipMemcpyAsync(xg.data(), h.xg.get(), xg.size() * 8, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(off.data(), h.off.get(), off.size() * 4, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(zk.data(), h.zk.get(), zk.size() * 8, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(ck.data(), h.ck.get(), ck.size() * 8, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipStreamSynchronize(s));
  struct Term {
    uint64_t x, z, cr, ci;
    bool operator<(const Term& o) const {
      return x != o.x ? x < o.x : z != o.z ? z < o.z : cr != o.cr ? cr < o.cr : ci < o.ci;
    }
    bool operator==(const Term& o) const { return x == o.x && z == o.z && cr == o.cr && ci == o.ci; }
  };
  const uint64_t mask = (1ull << n) - 1ull;
  auto swap = [&](uint64_t v) { return (v >> n) | ((v & mask) << n); };
  std::vector<Term> a, b;
  a.reserve(h.n_terms);
  b.reserve(h.n_terms);
  for (uint64_t g = 0; g < h.n_groups; ++g) {
    for (uint32_t k = off[g]; k < off[g + 1]; ++k) {
      uint64_t cr, ci;
      std::memcpy(&cr, &ck[2 * k], 8);
      std::memcpy(&ci, &ck[2 * k + 1], 8);
      a.push_back(Term{xg[g], zk[k], cr, ci});
      b.push_back(Term{swap(xg[g]), swap(zk[k]), cr, ci});
    }
  }
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  return a == b;
}

}  // namespace
}  // namespace pbs

using namespace pbs;

struct pbs_vqe {
  uint32_t n_orb = 0, n_qubits = 0, n_rot = 0;
  pbs_dtype dt = PBS_C128;
  uint64_t dim = 0, ref = 0;
  std::vector<Rot> rots;
  std::vector<pbs_space*> spaces;  // one per nonempty (N_alpha, N_beta) block, alpha-major order
  pbs_batch* batch = nullptr;
  uint32_t n_jobs = 0;
  DevBuf<uint32_t> rank_tab, binom_n;
  DevBuf<uint64_t> off;
  DevBuf<char> psi, lam, blk_in, blk_out;
  DevBuf<double> energies, partial, overlaps;
  uint32_t nparts = 0;
  bool evaluated = false;  // blk_in holds psi(theta) of the last evaluation
  uint32_t n_transposed = 0;  // blocks stored as sector (N_beta, N_alpha)
  uint32_t group_fwd = 3, group_adj = 3;  // most rotations fused per forward / adjoint pass (1..3)
  ~pbs_vqe() {
    if (batch) pbs_batch_destroy(batch);
    for (pbs_space* sp : spaces) pbs_space_destroy(sp);
  }
};

namespace pbs {
namespace {
constexpr unsigned kVqeGrid = 4096;
constexpr uint32_t kMaxRotations = 4096;  // overlap partials: 3 doubles x <= 4096 workgroups per rotation

PairRot pair_rot(const Rot& r, double angle) { return PairRot{r.x, r.z, r.omega, cos(angle), sin(angle)}; }

// Rotations first .. first+K-1 as one group, or false when their X masks are
// not linearly independent (a zero or repeated mask included).
template <int K>
bool make_group(const pbs_vqe& v, uint32_t first, const double* theta, double sign, RotGroup<K>& G) {
  uint64_t basis[K];
  for (int j = 0; j < K; ++j) {
    uint64_t y = v.rots[first + j].x;
    for (int i = 0; i < j; ++i)
      if ((y >> G.piv[i]) & 1ull) y ^= basis[i];
    if (y == 0) return false;
    basis[j] = y;
    G.piv[j] = 63u - static_cast<uint32_t>(__builtin_clzll(y));
    G.r[j] = pair_rot(v.rots[first + j], sign * theta[first + j]);
  }
  std::sort(G.piv, G.piv + K);
  return true;
}

template <class T>
void rotate_all(pbs_vqe& v, T* psi, const double* theta, bool inverse, uint32_t k, hipStream_t s) {
  const Rot& r = v.rots[k];
  const double th = inverse ? -theta[k] : theta[k];
  hipLaunchKernelGGL((k_rotate<T>), dim3(grid_for(v.dim, kBlock, kVqeGrid)), dim3(kBlock), 0, s, psi, v.dim, r.x,
                     r.z, r.omega, cos(th), sin(th));
}

template <class T>
void energy_grad(pbs_vqe& v, const double* theta, double* energy, double* grad, hipStream_t s) {
  T* psi = reinterpret_cast<T*>(v.psi.get());
  T* lam = reinterpret_cast<T*>(v.lam.get());
  T* bin = reinterpret_cast<T*>(v.blk_in.get());
  T* bout = reinterpret_cast<T*>(v.blk_out.get());
  const dim3 grid(grid_for(v.dim, kBlock, kVqeGrid));
  hipLaunchKernelGGL(k_basis_state, grid, dim3(kBlock), 0, s, sizeof(T) == 16 ? reinterpret_cast<double2*>(psi) : nullptr,
                     sizeof(T) == 8 ? reinterpret_cast<float2*>(psi) : nullptr, v.dim, v.ref);
  for (uint32_t k = 0; k < v.n_rot;) {
    RotGroup<3> G3;
    RotGroup<2> G2;
    if (v.group_fwd >= 3 && k + 2 < v.n_rot && v.dim >= 8 && make_group<3>(v, k, theta, 1.0, G3)) {
      hipLaunchKernelGGL((k_rotate_group<T, 3>), dim3(grid_for(v.dim / 8, kBlock, kVqeGrid)), dim3(kBlock), 0, s,
                         psi, v.dim, G3);
      k += 3;
    } else if (v.group_fwd >= 2 && k + 1 < v.n_rot && make_group<2>(v, k, theta, 1.0, G2)) {
      hipLaunchKernelGGL((k_rotate_group<T, 2>), dim3(grid_for(v.dim / 4, kBlock, kVqeGrid)), dim3(kBlock), 0, s,
                         psi, v.dim, G2);
      k += 2;
    } else {
      rotate_all<T>(v, psi, theta, false, k, s);
      k += 1;
    }
  }
  // H psi through the sector blocks, with each block's energy
  const pbs_space& sp0 = *v.spaces[0];
  hipLaunchKernelGGL((k_fock_permute<T, true>), grid, dim3(kBlock), 0, s, psi, bin, v.dim, v.n_orb, sp0.n_chunks,
                     v.rank_tab.get(), v.off.get(), v.binom_n.get());
  PBS_HIP(hipGetLastError());
  const pbs_status st = pbs_batch_run(v.batch, v.energies.get(), s);
  PBS_REQUIRE(st == PBS_OK, st, std::string("batched sector apply failed: ") + pbs_last_error());
  std::vector<double> e(3ull * v.n_jobs);
  PBS_HIP(hipMemcpyAsync(e.data(), v.energies.get(), e.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  if (grad && v.n_rot > 0) {
    hipLaunchKernelGGL((k_fock_permute<T, false>), grid, dim3(kBlock), 0, s, bout, lam, v.dim, v.n_orb,
                       sp0.n_chunks, v.rank_tab.get(), v.off.get(), v.binom_n.get());
    // adjoint sweep: g_k = -2 Im <lam_k|P_k|psi_k>, then undo rotation k on both vectors
    for (uint32_t k = v.n_rot; k > 0;) {
      RotGroup<3> G3;
      RotGroup<2> G2;
      if (v.group_adj >= 3 && k >= 3 && v.dim >= 8 && make_group<3>(v, k - 3, theta, -1.0, G3)) {
        hipLaunchKernelGGL((k_adjoint_group<T, 3>), dim3(v.nparts), dim3(kBlock), 0, s, psi, lam, v.dim, G3,
                           v.partial.get() + 3ull * v.nparts * (k - 3), static_cast<uint64_t>(v.nparts));
        k -= 3;
      } else if (v.group_adj >= 2 && k >= 2 && make_group<2>(v, k - 2, theta, -1.0, G2)) {
        hipLaunchKernelGGL((k_adjoint_group<T, 2>), dim3(v.nparts), dim3(kBlock), 0, s, psi, lam, v.dim, G2,
                           v.partial.get() + 3ull * v.nparts * (k - 2), static_cast<uint64_t>(v.nparts));
        k -= 2;
      } else {
        --k;
        const Rot& r = v.rots[k];
        hipLaunchKernelGGL((k_adjoint_step<T>), dim3(v.nparts), dim3(kBlock), 0, s, psi, lam, v.dim, r.x, r.z,
                           r.omega, cos(-theta[k]), sin(-theta[k]), v.partial.get() + 3ull * v.nparts * k);
      }
    }
    hipLaunchKernelGGL(k_sum_overlaps, dim3(v.n_rot), dim3(kBlock), 0, s, v.partial.get(), v.nparts,
                       v.overlaps.get());
    PBS_HIP(hipGetLastError());
    std::vector<double> ov(2ull * v.n_rot);
    PBS_HIP(hipMemcpyAsync(ov.data(), v.overlaps.get(), ov.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    PBS_HIP(hipStreamSynchronize(s));
    for (uint32_t k = 0; k < v.n_rot; ++k) grad[k] = -2.0 * ov[2 * k + 1];
  }
  PBS_HIP(hipGetLastError());
  PBS_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (uint32_t j = 0; j < v.n_jobs; ++j) acc += e[3 * j];
  *energy = acc;
  v.evaluated = true;
}

template <class T>
void state_out(const pbs_vqe& v, T* psi_out, hipStream_t s) {
  const pbs_space& sp0 = *v.spaces[0];
  hipLaunchKernelGGL((k_fock_permute<T, false>), dim3(grid_for(v.dim, kBlock, kVqeGrid)), dim3(kBlock), 0, s,
                     reinterpret_cast<const T*>(v.blk_in.get()), psi_out, v.dim, v.n_orb, sp0.n_chunks,
                     v.rank_tab.get(), v.off.get(), v.binom_n.get());
  PBS_HIP(hipGetLastError());
}
}  // namespace
}  // namespace pbs

extern "C" {

pbs_status pbs_vqe_create(const pbs_grouped* h, uint32_t n_orb, uint32_t n_rot, const uint64_t* x, const uint64_t* z,
                          uint64_t ref, pbs_dtype dt, void* stream, pbs_vqe** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(h != nullptr, PBS_ERR_ARG, "null pbs_grouped");
    PBS_REQUIRE(dt == PBS_C128 || dt == PBS_C64, PBS_ERR_ARG, "unknown dtype");
    PBS_REQUIRE(n_orb >= 1 && n_orb <= 14, PBS_ERR_RANGE, "the full space needs 1 <= n_orb <= 14");
    PBS_REQUIRE(h->n_qubits == 2 * n_orb && h->has_sector && h->half == n_orb, PBS_ERR_ARG,
                "operator must act on 2 n_orb qubits with sector tables");
    PBS_REQUIRE(n_rot <= kMaxRotations, PBS_ERR_RANGE,
                "at most " + std::to_string(kMaxRotations) + " rotations (the gradient keeps per-rotation partials)");
    PBS_REQUIRE(n_rot == 0 || (x != nullptr && z != nullptr), PBS_ERR_ARG, "null rotation strings");
    const uint64_t dim = 1ull << (2 * n_orb);
    PBS_REQUIRE(ref < dim, PBS_ERR_ARG, "reference state outside the space");
    for (uint32_t k = 0; k < n_rot; ++k)
      PBS_REQUIRE(((x[k] | z[k]) >> (2 * n_orb)) == 0, PBS_ERR_ARG,
                  "rotation " + std::to_string(k) + " acts beyond the qubits");
    hipStream_t s = as_stream(stream);
    auto* v = new pbs_vqe();
    try {
      v->n_orb = n_orb;
      v->n_qubits = 2 * n_orb;
      v->n_rot = n_rot;
      v->dt = dt;
      v->dim = dim;
      // measured at 24 qubits: three-rotation adjoint passes need 328 registers
      // per lane (one wave per SIMD), which pays off for complex128 only
      v->group_adj = dt == PBS_C128 ? 3u : 2u;
      v->ref = ref;
      for (uint32_t k = 0; k < n_rot; ++k) v->rots.push_back(rot_of(x[k], z[k]));
      const size_t esz = dt == PBS_C128 ? 16 : 8;
      v->psi.alloc(dim * esz);
      v->lam.alloc(dim * esz);
      v->blk_in.alloc(dim * esz);
      v->blk_out.alloc(dim * esz);
      // sector blocks, alpha-major over (N_alpha, N_beta).  A block with fewer
      // beta strings than a workgroup has lanes (and than alpha strings) is
      // stored and applied as sector (N_beta, N_alpha) when the operator is
      // symmetric under exchanging the halves, so its rows are long.
      std::vector<uint64_t> off((n_orb + 1) * (n_orb + 1), 0);
      std::vector<uint32_t> bn(n_orb + 1);
      for (uint32_t k = 0; k <= n_orb; ++k) bn[k] = static_cast<uint32_t>(host_binom(n_orb, k));
      std::string why;
      PBS_REQUIRE(conserves_spin_numbers(*h, s, &why), PBS_ERR_UNSUPPORTED,
                  "the energy is evaluated block by block over (N_alpha, N_beta) sectors, which needs an operator "
                  "that conserves N_alpha and N_beta: " + why);
      const bool sym = halves_symmetric(*h, s);
      std::vector<const pbs_grouped*> hs;
      std::vector<const pbs_space*> sps;
      std::vector<const void*> ins;
      std::vector<void*> outs;
      uint64_t acc = 0;
      for (uint32_t na = 0; na <= n_orb; ++na) {
        for (uint32_t nb = 0; nb <= n_orb; ++nb) {
          const bool tr = sym && bn[nb] < static_cast<uint32_t>(kSB) && bn[nb] < bn[na];
          off[na * (n_orb + 1) + nb] = acc | (tr ? kTransposed : 0ull);
          v->n_transposed += tr ? 1u : 0u;
          pbs_space* sp = nullptr;
          const pbs_status st = pbs_space_sector(n_orb, tr ? nb : na, tr ? na : nb, stream, &sp);
          PBS_REQUIRE(st == PBS_OK, st, std::string("sector space: ") + pbs_last_error());
          v->spaces.push_back(sp);
          hs.push_back(h);
          sps.push_back(sp);
          ins.push_back(v->blk_in.get() + acc * esz);
          outs.push_back(v->blk_out.get() + acc * esz);
          acc += sp->dim;
        }
      }
      PBS_REQUIRE(acc == dim, PBS_ERR_DEVICE, "sector blocks do not tile the full space");
      v->n_jobs = static_cast<uint32_t>(sps.size());
      const pbs_status st = pbs_batch_create(v->n_jobs, hs.data(), sps.data(), dt, ins.data(), outs.data(), &v->batch);
      PBS_REQUIRE(st == PBS_OK, st, std::string("batch: ") + pbs_last_error());
      const pbs_space& sp0 = *v->spaces[0];
      v->rank_tab.alloc(sp0.rank_tab.n);
      PBS_HIP(hipMemcpyAsync(v->rank_tab.get(), sp0.rank_tab.get(), sp0.rank_tab.n * 4, hipMemcpyDeviceToDevice, s));
      v->off.alloc(off.size());
      v->binom_n.alloc(bn.size());
      PBS_HIP(hipMemcpyAsync(v->off.get(), off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
      PBS_HIP(hipMemcpyAsync(v->binom_n.get(), bn.data(), bn.size() * 4, hipMemcpyHostToDevice, s));
      v->energies.alloc(3ull * v->n_jobs);
      v->nparts = grid_for(dim / 2, kBlock, 4096);  // one pair per thread and pass, up to 4096 workgroups
      v->partial.alloc(3ull * v->nparts * (n_rot ? n_rot : 1));
      v->overlaps.alloc(2ull * (n_rot ? n_rot : 1));
      PBS_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete v;
      throw;
    }
    *out = v;
  });
}

pbs_status pbs_vqe_energy_grad(pbs_vqe* v, const double* theta, double* energy, double* grad, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr && energy != nullptr, PBS_ERR_ARG, "null argument");
    PBS_REQUIRE(v->n_rot == 0 || theta != nullptr, PBS_ERR_ARG, "null parameters");
    hipStream_t s = as_stream(stream);
    if (v->dt == PBS_C128)
      energy_grad<double2>(*v, theta, energy, grad, s);
    else
      energy_grad<float2>(*v, theta, energy, grad, s);
  });
}

pbs_status pbs_vqe_state(const pbs_vqe* v, void* psi_out, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr && psi_out != nullptr, PBS_ERR_ARG, "null argument");
    PBS_REQUIRE(v->evaluated, PBS_ERR_ARG, "no state before the first evaluation");
    if (v->dt == PBS_C128)
      state_out(*v, static_cast<double2*>(psi_out), as_stream(stream));
    else
      state_out(*v, static_cast<float2*>(psi_out), as_stream(stream));
  });
}

pbs_status pbs_vqe_minimize(pbs_vqe* v, double* theta, uint32_t max_iter, double g_tol, double f_tol, void* stream,
                            double* energy, uint32_t* iters, uint32_t* evals, int32_t* reason) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr && theta != nullptr, PBS_ERR_ARG, "null argument");
    PBS_REQUIRE(v->n_rot >= 1, PBS_ERR_ARG, "nothing to optimise: the ansatz has no rotations");
    hipStream_t s = as_stream(stream);
    const Objective fg = [&](const double* th, double* f, double* g) {
      if (v->dt == PBS_C128)
        energy_grad<double2>(*v, th, f, g, s);
      else
        energy_grad<float2>(*v, th, f, g, s);
    };
    // energies of a complex64 state carry float32 rounding noise
    const double noise = v->dt == PBS_C128 ? 1e-13 : 1e-6;
    const LbfgsResult r = lbfgs_minimize(v->n_rot, theta, fg, max_iter, 10, g_tol, f_tol, noise);
    if (energy) *energy = r.f;
    if (iters) *iters = r.iters;
    if (evals) *evals = r.evals;
    if (reason) *reason = r.reason;
  });
}

pbs_status pbs_vqe_tune(pbs_vqe* v, uint32_t reps, void* stream, uint32_t* config, double* ms) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr, PBS_ERR_ARG, "null pbs_vqe");
    PBS_REQUIRE(v->evaluated, PBS_ERR_ARG, "tune after the first evaluation (the blocks hold a state then)");
    const pbs_status st = pbs_batch_tune(v->batch, reps, stream, config, ms);
    PBS_REQUIRE(st == PBS_OK, st, std::string("batch tuning: ") + pbs_last_error());
  });
}

pbs_status pbs_vqe_set_config(pbs_vqe* v, uint32_t config) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr, PBS_ERR_ARG, "null pbs_vqe");
    const pbs_status st = pbs_batch_set_config(v->batch, config);
    PBS_REQUIRE(st == PBS_OK, st, std::string("batch schedule: ") + pbs_last_error());
  });
}

pbs_status pbs_vqe_set_groups(pbs_vqe* v, uint32_t forward, uint32_t adjoint) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr, PBS_ERR_ARG, "null pbs_vqe");
    PBS_REQUIRE(forward >= 1 && forward <= 3 && adjoint >= 1 && adjoint <= 3, PBS_ERR_RANGE,
                "rotations fused per pass must be 1, 2 or 3");
    v->group_fwd = forward;
    v->group_adj = adjoint;
  });
}

pbs_status pbs_vqe_info(const pbs_vqe* v, uint32_t* n_blocks, uint32_t* n_transposed) {
  return guarded([&] {
    PBS_REQUIRE(v != nullptr, PBS_ERR_ARG, "null pbs_vqe");
    if (n_blocks) *n_blocks = v->n_jobs;
    if (n_transposed) *n_transposed = v->n_transposed;
  });
}

void pbs_vqe_destroy(pbs_vqe* v) { delete v; }

}  // extern "C"
