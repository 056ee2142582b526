// Pauli-string products, Pauli sums, canonical reduction and the direct
// Jordan-Wigner construction (Sections 2.2-2.3, Algorithm 1).
#include <cmath>
#include <mutex>

#include "exact_sum.h"
#include "pbs_internal.h"

namespace pbs {

namespace {
thread_local std::string g_last_error;

// ---------------------------------------------------------------- products
// Letter form -> XZ form adds one factor i per Y (Section 2.2: chi = gamma +
// popcount(X & Z)); the product rule of Eq. pauli_prod_phase adds
// 2 popcount(Z_left & X_right); back to letter form subtracts popcount(X & Z).
__global__ void k_pauli_mul(uint64_t n, int W, const uint64_t* xa, const uint64_t* za, const uint8_t* pa,
                            const uint64_t* xb, const uint64_t* zb, const uint8_t* pb, uint64_t* xo, uint64_t* zo,
                            uint8_t* po) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    uint32_t e = static_cast<uint32_t>(pa[i]) + static_cast<uint32_t>(pb[i]);
    for (int w = 0; w < W; ++w) {
      const uint64_t a_x = xa[i * W + w], a_z = za[i * W + w];
      const uint64_t b_x = xb[i * W + w], b_z = zb[i * W + w];
      const uint64_t m_x = a_x ^ b_x, m_z = a_z ^ b_z;
      e += __popcll(a_x & a_z) + __popcll(b_x & b_z) + 2u * __popcll(a_z & b_x);
      e += 3u * __popcll(m_x & m_z);  // subtract popcount mod 4
      xo[i * W + w] = m_x;
      zo[i * W + w] = m_z;
    }
    po[i] = static_cast<uint8_t>(e & 3u);
  }
}

// i^g * (re, im)
__device__ inline void rotate(uint32_t g, double& re, double& im) {
  const double r = re, m = im;
  switch (g & 3u) {
    case 0: break;
    case 1: re = -m; im = r; break;
    case 2: re = -r; im = -m; break;
    default: re = m; im = -r; break;
  }
}

// AoS strings + interleaved coefficients -> SoA keys (z words, then x words) and re/im.
__global__ void k_to_soa(uint64_t m, int W, const uint64_t* x, const uint64_t* z, const double* c, uint64_t* keys,
                         double* re, double* im) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    for (int w = 0; w < W; ++w) {
      keys[static_cast<uint64_t>(w) * m + i] = z[i * W + w];
      keys[static_cast<uint64_t>(W + w) * m + i] = x[i * W + w];
    }
    re[i] = c[2 * i];
    im[i] = c[2 * i + 1];
  }
}

__global__ void k_segment_starts(const uint32_t* heads, const uint32_t* segid, uint64_t m, uint32_t* start) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (heads[i]) start[segid[i]] = static_cast<uint32_t>(i);
}

// Fast path of the correctly rounded segment sums.  Cascaded TWO-SUM (the
// Sum2 scheme of Ogita, Rump and Oishi, 2005) gives s = fl(sum x) and the
// exact rounding errors q_j, so the exact sum is T = s + sum q_j.  The lanes
// of a wave sum strided parts of a run and are merged by TWO-SUM as well, so
// at most N = n + 64 error terms arise; any summation tree of them gives
// |fl(sum q_j) - sum q_j| <= gamma_N sum |q_j| and sum |q_j| <= e / (1 - gamma_N)
// for e = fl(sum |q_j|), gamma_N = N u / (1 - N u), u = 2^-53, so for N u <= 1/4
// the compensation c is within 2 N u e.  With r = fl(s + c) and its exact
// error er, |T - r| <= |er| + 2 N u e; when this (rounded upward) is below
// half the smaller gap next to r, r is the round-to-nearest value of T.  T is
// also a multiple of g, the smallest unit in the last place among the
// inputs, so r = 0 with a bound below g proves T = 0.  When every q_j is
// zero, s is exact.
struct Sum2 {
  double s = 0.0, c = 0.0, e = 0.0;
  int emin = 2047;  // smallest max(biased exponent, 1) over nonzero inputs
};

__device__ inline void sum2_add(Sum2& a, double v) {
  double t, q;
  two_sum(a.s, v, t, q);
  a.s = t;
  a.c += q;
  a.e += fabs(q);
  const int be = static_cast<int>((static_cast<uint64_t>(__double_as_longlong(v)) >> 52) & 0x7ffu);
  if (v != 0.0) a.emin = min(a.emin, max(be, 1));
}

__device__ inline void sum2_merge(Sum2& a, double s, double c, double e, int emin) {
  double t, q;
  two_sum(a.s, s, t, q);
  a.s = t;
  a.c = (a.c + c) + q;
  a.e = (a.e + e) + fabs(q);
  a.emin = min(a.emin, emin);
}

__device__ inline void sum2_wave_merge(Sum2& a) {
  for (int d = 32; d > 0; d >>= 1)
    sum2_merge(a, __shfl_xor(a.s, d, 64), __shfl_xor(a.c, d, 64), __shfl_xor(a.e, d, 64),
               __shfl_xor(a.emin, d, 64));
}

// True when r is proven to be the correctly rounded sum (N error terms at most).
__device__ inline bool sum2_round(const Sum2& a, uint32_t N, double& r) {
  if (a.e == 0.0) {
    r = a.s + 0.0;
    return true;
  }
  if (N >= (1u << 30)) return false;
  double rr, er;
  two_sum(a.s, a.c, rr, er);
  if (!isfinite(rr)) return false;
  const double two_nu = static_cast<double>(N) * 0x1p-52;  // exact: N < 2^30
  const double bound = (fabs(er) + two_nu * a.e * (1.0 + 0x1p-50)) * (1.0 + 0x1p-50);
  if (rr == 0.0) {  // s + c = 0 exactly; T is a multiple of g with |T| <= bound
    if (a.emin < 2047 && bound < ldexp(1.0, a.emin - 1075)) {
      r = 0.0;
      return true;
    }
    return false;
  }
  const double ar = fabs(rr);
  const double below = __longlong_as_double(__double_as_longlong(ar) - 1);  // next double toward zero
  if (bound < 0.5 * (ar - below)) {
    r = rr + 0.0;
    return true;
  }
  return false;
}

// One wave per run of equal keys: certified fast sums, then the drop test;
// runs the fast path cannot certify are queued for k_segment_sum_exact.
__global__ __launch_bounds__(256) void k_segment_sum(uint32_t nseg, uint64_t m, const uint32_t* start,
                                                     const uint32_t* order, const double* re, const double* im,
                                                     double eps_drop, double* out_re, double* out_im, uint32_t* keep,
                                                     uint32_t* n_slow, uint32_t* slow) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t u = wave; u < nseg; u += n_waves) {
    const uint32_t b = start[u];
    const uint32_t e = (u + 1 < nseg) ? start[u + 1] : static_cast<uint32_t>(m);
    Sum2 ar, ai;
    for (uint32_t j = b + lane; j < e; j += 64) {
      const uint32_t v = order[j];
      sum2_add(ar, re[v]);
      sum2_add(ai, im[v]);
    }
    sum2_wave_merge(ar);
    sum2_wave_merge(ai);
    if (lane == 0) {
      double r, i;
      if (sum2_round(ar, e - b + 64, r) && sum2_round(ai, e - b + 64, i)) {
        out_re[u] = r;
        out_im[u] = i;
        keep[u] = (fmax(fabs(r), fabs(i)) > eps_drop) ? 1u : 0u;
      } else {
        slow[atomicAdd(n_slow, 1u)] = u;
      }
    }
  }
}

// Exact expansions for the queued runs (their order in the queue does not
// matter: each run's result depends on its contributions only).
__global__ void k_segment_sum_exact(uint32_t nseg, uint64_t m, const uint32_t* start, const uint32_t* order,
                                    const double* re, const double* im, double eps_drop, const uint32_t* n_slow,
                                    const uint32_t* slow, double* out_re, double* out_im, uint32_t* keep,
                                    uint32_t* overflow) {
  const uint32_t n = *n_slow;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const uint32_t u = slow[k];
    const uint32_t b = start[u];
    const uint32_t e = (u + 1 < nseg) ? start[u + 1] : static_cast<uint32_t>(m);
    ExactAcc ar, ai;
    acc_init(ar);
    acc_init(ai);
    for (uint32_t j = b; j < e; ++j) {
      const uint32_t v = order[j];
      acc_add(ar, re[v]);
      acc_add(ai, im[v]);
    }
    if (ar.overflow | ai.overflow) atomicOr(overflow, 1u);
    const double r = acc_round(ar), i = acc_round(ai);
    out_re[u] = r;
    out_im[u] = i;
    keep[u] = (fmax(fabs(r), fabs(i)) > eps_drop) ? 1u : 0u;
  }
}

__global__ void k_compact_terms(uint32_t nseg, uint64_t m, int W, const uint32_t* start, const uint32_t* keep,
                                const uint32_t* pos, const uint64_t* keys, const double* sre, const double* sim,
                                uint64_t* x, uint64_t* z, double* c) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nseg; u += gridDim.x * blockDim.x) {
    if (!keep[u]) continue;
    const uint64_t o = pos[u];
    const uint64_t i = start[u];
    for (int w = 0; w < W; ++w) {
      z[o * W + w] = keys[static_cast<uint64_t>(w) * m + i];
      x[o * W + w] = keys[static_cast<uint64_t>(W + w) * m + i];
    }
    c[2 * o] = sre[u];
    c[2 * o + 1] = sim[u];
  }
}

// ---------------------------------------------------------------- sum x sum
// One thread per pair (k, l).  The coefficient a_k b_l is carried exactly as
// four rows of TWO-PRODUCT pieces (p = fl(a*b), e = fma(a, b, -p)) so the
// canonical reduction rounds the exact pair sums once.
__global__ void k_sum_mul(uint64_t na, uint64_t nb, int W, const uint64_t* xa, const uint64_t* za, const double* ca,
                          const uint64_t* xb, const uint64_t* zb, const double* cb, uint64_t* keys, double* re,
                          double* im) {
  const uint64_t npairs = na * nb;
  const uint64_t m = 4 * npairs;
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < npairs;
       t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t k = t / nb, l = t % nb;
    uint32_t g = 0;
    for (int w = 0; w < W; ++w) {
      const uint64_t a_x = xa[k * W + w], a_z = za[k * W + w];
      const uint64_t b_x = xb[l * W + w], b_z = zb[l * W + w];
      const uint64_t m_x = a_x ^ b_x, m_z = a_z ^ b_z;
      g += __popcll(a_x & a_z) + __popcll(b_x & b_z) + 2u * __popcll(a_z & b_x) + 3u * __popcll(m_x & m_z);
      for (int r = 0; r < 4; ++r) {
        keys[static_cast<uint64_t>(w) * m + 4 * t + r] = m_z;
        keys[static_cast<uint64_t>(W + w) * m + 4 * t + r] = m_x;
      }
    }
    const double ar = ca[2 * k], ai = ca[2 * k + 1], br = cb[2 * l], bi = cb[2 * l + 1];
    const double p1 = ar * br, e1 = fma(ar, br, -p1);
    const double p2 = ai * bi, e2 = fma(ai, bi, -p2);
    const double p3 = ar * bi, e3 = fma(ar, bi, -p3);
    const double p4 = ai * br, e4 = fma(ai, br, -p4);
    double r0 = p1, i0 = p3, r1 = e1, i1 = e3, r2 = -p2, i2 = p4, r3 = -e2, i3 = e4;
    rotate(g, r0, i0);
    rotate(g, r1, i1);
    rotate(g, r2, i2);
    rotate(g, r3, i3);
    re[4 * t] = r0; im[4 * t] = i0;
    re[4 * t + 1] = r1; im[4 * t + 1] = i1;
    re[4 * t + 2] = r2; im[4 * t + 2] = i2;
    re[4 * t + 3] = r3; im[4 * t + 3] = i3;
  }
}

// ---------------------------------------------------------------- Jordan-Wigner
// Ladder operator a+_p or a_p is 1/2 (X_p -+ i Y_p) Z_{<p}; term 0 is X_p Z_{<p}
// (letter phase 0), term 1 is Y_p Z_{<p} (letter phase 3 for a+, 1 for a).
// In XZ form term 1 carries one more factor i for its Y.
struct Str {
  uint64_t x[kMaxWords];
  uint64_t z[kMaxWords];
  uint32_t e;  // XZ-form exponent of i
};

__device__ inline void ladder_mul(Str& s, int W, uint32_t p, bool dagger, int term) {
  // right-multiply s by the chosen ladder term: e += e2 + 2 popcount(z_s & x_2)
  const int pw = static_cast<int>(p >> 6);
  const uint64_t pbit = 1ull << (p & 63u);
  uint32_t e2 = 0;
  if (term) e2 = (dagger ? 3u : 1u) + 1u;
  uint32_t cross = __popcll(s.z[pw] & pbit);
  s.e += e2 + 2u * cross;
  for (int w = 0; w < W; ++w) {
    uint64_t zmask;
    if (w < pw) zmask = ~0ull;
    else if (w > pw) zmask = 0ull;
    else zmask = pbit - 1ull;
    if (term && w == pw) zmask |= pbit;
    s.z[w] ^= zmask;
  }
  s.x[pw] ^= pbit;
}

__device__ inline void emit_contribution(const Str& s, int W, double mag, uint64_t m, uint64_t row, uint64_t* keys,
                                         double* re, double* im) {
  uint32_t g = s.e;
  for (int w = 0; w < W; ++w) {
    g += 3u * __popcll(s.x[w] & s.z[w]);
    keys[static_cast<uint64_t>(w) * m + row] = s.z[w];
    keys[static_cast<uint64_t>(W + w) * m + row] = s.x[w];
  }
  double r = mag, i = 0.0;
  rotate(g, r, i);
  re[row] = r;
  im[row] = i;
}

__global__ void k_flag_abs_gt(const double* h, uint64_t n, double eps, uint32_t* flag) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    flag[i] = fabs(h[i]) > eps ? 1u : 0u;
}

__global__ void k_jw_identity(int W, uint64_t m, double e0, uint64_t* keys, double* re, double* im) {
  for (int w = 0; w < 2 * W; ++w) keys[static_cast<uint64_t>(w) * m] = 0ull;
  re[0] = e0;
  im[0] = 0.0;
}

__global__ void k_jw_one_body(uint32_t n, int W, const double* h1, const uint32_t* flag, const uint32_t* off,
                              uint64_t base, uint64_t m, uint64_t* keys, double* re, double* im) {
  const uint64_t total = static_cast<uint64_t>(n) * n;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (!flag[i]) continue;
    const uint32_t P = static_cast<uint32_t>(i / n), Q = static_cast<uint32_t>(i % n);
    const double mag = h1[i] * 0.25;  // h * (1/2)^2, exact
    const uint64_t row0 = base + 4ull * off[i];
    for (int combo = 0; combo < 4; ++combo) {
      Str s;
      for (int w = 0; w < W; ++w) s.x[w] = s.z[w] = 0ull;
      s.e = 0;
      ladder_mul(s, W, P, true, combo & 1);
      ladder_mul(s, W, Q, false, (combo >> 1) & 1);
      emit_contribution(s, W, mag, m, row0 + combo, keys, re, im);
    }
  }
}

__global__ void k_jw_two_body(uint32_t n, int W, const double* h2, const uint32_t* flag, const uint32_t* off,
                              uint64_t base, uint64_t m, uint64_t* keys, double* re, double* im) {
  const uint64_t n2 = static_cast<uint64_t>(n) * n;
  const uint64_t total = n2 * n2;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (!flag[i]) continue;
    const uint32_t S = static_cast<uint32_t>(i % n);
    const uint32_t R = static_cast<uint32_t>((i / n) % n);
    const uint32_t Q = static_cast<uint32_t>((i / n2) % n);
    const uint32_t P = static_cast<uint32_t>(i / (n2 * n));
    const double mag = h2[i] * (0.5 * 0.0625);  // 1/2 * h * (1/2)^4, exact
    const uint64_t row0 = base + 16ull * off[i];
    for (int combo = 0; combo < 16; ++combo) {
      Str s;
      for (int w = 0; w < W; ++w) s.x[w] = s.z[w] = 0ull;
      s.e = 0;
      ladder_mul(s, W, P, true, combo & 1);
      ladder_mul(s, W, Q, true, (combo >> 1) & 1);
      ladder_mul(s, W, R, false, (combo >> 2) & 1);
      ladder_mul(s, W, S, false, (combo >> 3) & 1);
      emit_contribution(s, W, mag, m, row0 + combo, keys, re, im);
    }
  }
}

// OR of all mask bits at or above n_qubits (must be zero for a valid sum).
__global__ void k_stray_bits(const uint64_t* x, const uint64_t* z, uint64_t m, int W, uint32_t n_qubits,
                             unsigned long long* out) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    uint64_t bad = 0;
    for (int w = 0; w < W; ++w) {
      const int top = static_cast<int>(n_qubits) - 64 * w;
      const uint64_t keep = top >= 64 ? ~0ull : ((1ull << top) - 1ull);
      bad |= (x[i * W + w] | z[i * W + w]) & ~keep;
    }
    if (bad) atomicOr(out, 1ull);
  }
}

void check_sum(const pbs_sum* s) { PBS_REQUIRE(s != nullptr, PBS_ERR_ARG, "null pbs_sum"); }

}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------- scratch arena
struct Scratch::Arena {
  std::mutex mu;
  void* base = nullptr;
  size_t cap = 0;
};

namespace {
thread_local Scratch* tl_scratch = nullptr;

Scratch::Arena* device_arena() {
  static std::mutex mu;
  static Scratch::Arena* arenas[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!arenas[dev]) arenas[dev] = new Scratch::Arena();  // lives until the process ends
  return arenas[dev];
}
}  // namespace

Scratch::Scratch(hipStream_t s) : arena_(device_arena()), stream_(s), outer_(tl_scratch) {
  if (outer_) {  // nested scope: share the outer scope's arena and cursor
    arena_ = nullptr;
  } else if (arena_) {
    arena_->mu.lock();
  }
  tl_scratch = this;
}

Scratch::~Scratch() {
  tl_scratch = outer_;
  if (!arena_) return;
  // temporaries may still be in use by queued work on the stream
  (void)hipStreamSynchronize(stream_);
  if (wanted_ > arena_->cap) {
    if (arena_->base) (void)hipFree(arena_->base);
    arena_->base = nullptr;
    arena_->cap = 0;
    const size_t grown = wanted_ + wanted_ / 4;
    if (hipMalloc(&arena_->base, grown) == hipSuccess)
      arena_->cap = grown;
    else
      arena_->base = nullptr;
  }
  (void)hipGetLastError();
  arena_->mu.unlock();
}

void* Scratch::take(size_t bytes) {
  if (outer_) return outer_->take(bytes);
  const size_t need = (bytes + 255) & ~static_cast<size_t>(255);
  const size_t at = top_;
  top_ += need;
  wanted_ = top_ > wanted_ ? top_ : wanted_;
  if (!arena_ || !arena_->base || top_ > arena_->cap) return nullptr;
  return static_cast<char*>(arena_->base) + at;
}

Scratch* Scratch::current() { return tl_scratch; }
void clear_last_error() { g_last_error.clear(); }

void canonicalize_soa(uint32_t n_qubits, int W, uint64_t m, DevBuf<uint64_t>& keys, DevBuf<double>& re,
                      DevBuf<double>& im, double eps_drop, pbs_sum& out, hipStream_t s) {
  PBS_REQUIRE(m < (1ull << 32), PBS_ERR_RANGE, "more than 2^32 - 1 contributions");
  out.n_qubits = n_qubits;
  out.words = W;
  out.canonical = true;
  if (m == 0) {
    out.n_terms = 0;
    out.x.release();
    out.z.release();
    out.coeff.release();
    return;
  }
  const int nw = 2 * W;
  DevBuf<uint32_t> order(m, s);
  iota_u32(order.get(), m, s);
  radix_sort_keys(keys.get(), order.get(), m, nw, s);
  DevBuf<uint32_t> heads(m, s), segid(m, s), cnt(2, s);
  mark_heads(keys.get(), m, nw, heads.get(), s);
  exclusive_scan_u32(heads.get(), segid.get(), m, cnt.get(), s);
  const uint32_t nseg = read_scalar(cnt.get(), s);
  DevBuf<uint32_t> start(nseg, s), keep(nseg, s), pos(nseg, s), flags(2, s), slow(nseg, s);
  DevBuf<double> sre(nseg, s), sim(nseg, s);
  uint32_t* overflow = flags.get();
  uint32_t* n_slow = flags.get() + 1;
  PBS_HIP(hipMemsetAsync(flags.get(), 0, 2 * sizeof(uint32_t), s));
  hipLaunchKernelGGL(k_segment_starts, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, heads.get(), segid.get(), m,
                     start.get());
  hipLaunchKernelGGL(k_segment_sum, dim3(grid_for(64ull * nseg, 256, 65536)), dim3(256), 0, s, nseg, m, start.get(),
                     order.get(), re.get(), im.get(), eps_drop, sre.get(), sim.get(), keep.get(), n_slow, slow.get());
  hipLaunchKernelGGL(k_segment_sum_exact, dim3(grid_for(nseg, 64, 65536)), dim3(64), 0, s, nseg, m, start.get(),
                     order.get(), re.get(), im.get(), eps_drop, n_slow, slow.get(), sre.get(), sim.get(), keep.get(),
                     overflow);
  PBS_HIP(hipGetLastError());
  exclusive_scan_u32(keep.get(), pos.get(), nseg, cnt.get() + 1, s);
  const uint32_t nkeep = read_scalar(cnt.get() + 1, s);
  PBS_REQUIRE(read_scalar(overflow, s) == 0, PBS_ERR_RANGE,
              "exact summation needed more than the supported number of expansion components");
  out.n_terms = nkeep;
  out.x.alloc(static_cast<uint64_t>(nkeep) * W);
  out.z.alloc(static_cast<uint64_t>(nkeep) * W);
  out.coeff.alloc(2ull * nkeep);
  if (nkeep) {
    hipLaunchKernelGGL(k_compact_terms, dim3(grid_for(nseg, 256, 65536)), dim3(256), 0, s, nseg, m, W, start.get(),
                       keep.get(), pos.get(), keys.get(), sre.get(), sim.get(), out.x.get(), out.z.get(),
                       out.coeff.get());
    PBS_HIP(hipGetLastError());
  }
  PBS_HIP(hipStreamSynchronize(s));
}

}  // namespace pbs

using namespace pbs;

extern "C" {

const char* pbs_last_error(void) { return g_last_error.c_str(); }

int32_t pbs_abi_version(void) { return 1; }

pbs_status pbs_pauli_mul(uint32_t n_qubits, uint64_t n, const uint64_t* xa, const uint64_t* za, const uint8_t* pa,
                         const uint64_t* xb, const uint64_t* zb, const uint8_t* pb, uint64_t* xo, uint64_t* zo,
                         uint8_t* po, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(n_qubits >= 1 && n_qubits <= kMaxQubitsSum, PBS_ERR_RANGE, "n_qubits must be 1..256");
    if (n == 0) return;
    PBS_REQUIRE(xa && za && pa && xb && zb && pb && xo && zo && po, PBS_ERR_ARG, "null array");
    const int W = words_for(n_qubits);
    hipLaunchKernelGGL(k_pauli_mul, dim3(grid_for(n, 256, 65536)), dim3(256), 0, as_stream(stream), n, W, xa, za, pa,
                       xb, zb, pb, xo, zo, po);
    PBS_HIP(hipGetLastError());
  });
}

pbs_status pbs_sum_create(uint32_t n_qubits, uint64_t n_terms, const uint64_t* x, const uint64_t* z,
                          const double* coeff, void* stream, pbs_sum** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(n_qubits >= 1 && n_qubits <= kMaxQubitsSum, PBS_ERR_RANGE, "n_qubits must be 1..256");
    PBS_REQUIRE(n_terms < (1ull << 32), PBS_ERR_RANGE, "n_terms must be below 2^32");
    PBS_REQUIRE(n_terms == 0 || (x && z && coeff), PBS_ERR_ARG, "null array");
    hipStream_t s = as_stream(stream);
    Scratch scratch(s);  // temporaries of this call
    auto* sum = new pbs_sum();
    try {
      sum->n_qubits = n_qubits;
      sum->words = words_for(n_qubits);
      sum->n_terms = n_terms;
      sum->canonical = false;
      const uint64_t nw = n_terms * sum->words;
      sum->x.alloc(nw);
      sum->z.alloc(nw);
      sum->coeff.alloc(2 * n_terms);
      if (n_terms) {
        PBS_HIP(hipMemcpyAsync(sum->x.get(), x, nw * 8, hipMemcpyDefault, s));
        PBS_HIP(hipMemcpyAsync(sum->z.get(), z, nw * 8, hipMemcpyDefault, s));
        PBS_HIP(hipMemcpyAsync(sum->coeff.get(), coeff, 2 * n_terms * 8, hipMemcpyDefault, s));
        DevBuf<unsigned long long> stray(1, s);
        PBS_HIP(hipMemsetAsync(stray.get(), 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_stray_bits, dim3(grid_for(n_terms, 256, 4096)), dim3(256), 0, s, sum->x.get(),
                           sum->z.get(), n_terms, sum->words, n_qubits, stray.get());
        PBS_HIP(hipGetLastError());
        PBS_REQUIRE(read_scalar(stray.get(), s) == 0, PBS_ERR_ARG, "mask bits set at or above n_qubits");
      }
      PBS_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete sum;
      throw;
    }
    *out = sum;
  });
}

pbs_status pbs_sum_info(const pbs_sum* s, uint32_t* n_qubits, uint64_t* n_terms, int32_t* canonical) {
  return guarded([&] {
    check_sum(s);
    if (n_qubits) *n_qubits = s->n_qubits;
    if (n_terms) *n_terms = s->n_terms;
    if (canonical) *canonical = s->canonical ? 1 : 0;
  });
}

pbs_status pbs_sum_read(const pbs_sum* s, uint64_t* x, uint64_t* z, double* coeff, void* stream) {
  return guarded([&] {
    check_sum(s);
    hipStream_t st = as_stream(stream);
    const uint64_t nw = s->n_terms * s->words;
    if (s->n_terms) {
      if (x) PBS_HIP(hipMemcpyAsync(x, s->x.get(), nw * 8, hipMemcpyDefault, st));
      if (z) PBS_HIP(hipMemcpyAsync(z, s->z.get(), nw * 8, hipMemcpyDefault, st));
      if (coeff) PBS_HIP(hipMemcpyAsync(coeff, s->coeff.get(), 2 * s->n_terms * 8, hipMemcpyDefault, st));
    }
    PBS_HIP(hipStreamSynchronize(st));
  });
}

pbs_status pbs_sum_view(const pbs_sum* s, uint32_t* n_qubits, uint64_t* n_terms, const uint64_t** x,
                        const uint64_t** z, const double** coeff) {
  return guarded([&] {
    check_sum(s);
    if (n_qubits) *n_qubits = s->n_qubits;
    if (n_terms) *n_terms = s->n_terms;
    const bool any = s->n_terms > 0;
    if (x) *x = any ? s->x.get() : nullptr;
    if (z) *z = any ? s->z.get() : nullptr;
    if (coeff) *coeff = any ? s->coeff.get() : nullptr;
  });
}

void pbs_sum_destroy(pbs_sum* s) { delete s; }

pbs_status pbs_pauli_canonicalize(pbs_sum* sum, double eps_drop, void* stream) {
  return guarded([&] {
    check_sum(sum);
    PBS_REQUIRE(!std::isnan(eps_drop), PBS_ERR_ARG, "eps_drop is NaN");
    hipStream_t s = as_stream(stream);
    Scratch scratch(s);  // temporaries of this call
    const uint64_t m = sum->n_terms;
    const int W = sum->words;
    DevBuf<uint64_t> keys(m * 2 * W, s);
    DevBuf<double> re(m, s), im(m, s);
    if (m) {
      hipLaunchKernelGGL(k_to_soa, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, m, W, sum->x.get(), sum->z.get(),
                         sum->coeff.get(), keys.get(), re.get(), im.get());
      PBS_HIP(hipGetLastError());
    }
    pbs_sum tmp;
    canonicalize_soa(sum->n_qubits, W, m, keys, re, im, eps_drop, tmp, s);
    sum->x = std::move(tmp.x);
    sum->z = std::move(tmp.z);
    sum->coeff = std::move(tmp.coeff);
    sum->n_terms = tmp.n_terms;
    sum->canonical = true;
  });
}

pbs_status pbs_pauli_sum_mul(const pbs_sum* a, const pbs_sum* b, double eps_drop, void* stream, pbs_sum** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    check_sum(a);
    check_sum(b);
    PBS_REQUIRE(a->n_qubits == b->n_qubits, PBS_ERR_ARG, "qubit counts differ");
    PBS_REQUIRE(!std::isnan(eps_drop), PBS_ERR_ARG, "eps_drop is NaN");
    const uint64_t np = a->n_terms * b->n_terms;
    PBS_REQUIRE(a->n_terms < (1ull << 30) && b->n_terms < (1ull << 30) && np < (1ull << 30), PBS_ERR_RANGE,
                "product has 2^30 or more term pairs");
    hipStream_t s = as_stream(stream);
    Scratch scratch(s);  // temporaries of this call
    const int W = a->words;
    const uint64_t m = 4 * np;
    DevBuf<uint64_t> keys(m * 2 * W, s);
    DevBuf<double> re(m, s), im(m, s);
    if (np) {
      hipLaunchKernelGGL(k_sum_mul, dim3(grid_for(np, 256, 65536)), dim3(256), 0, s, a->n_terms, b->n_terms, W,
                         a->x.get(), a->z.get(), a->coeff.get(), b->x.get(), b->z.get(), b->coeff.get(), keys.get(),
                         re.get(), im.get());
      PBS_HIP(hipGetLastError());
    }
    auto* res = new pbs_sum();
    try {
      canonicalize_soa(a->n_qubits, W, m, keys, re, im, eps_drop, *res, s);
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
  });
}

pbs_status pbs_jw_transform(uint32_t n_spin_orb, const double* h1, const double* h2, double e0, double eps,
                            double eps_drop, void* stream, pbs_sum** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(n_spin_orb >= 1 && n_spin_orb <= 255, PBS_ERR_RANGE, "n_spin_orb must be 1..255");
    PBS_REQUIRE(h1 != nullptr, PBS_ERR_ARG, "null h1");
    PBS_REQUIRE(!std::isnan(eps) && !std::isnan(eps_drop), PBS_ERR_ARG, "threshold is NaN");
    hipStream_t s = as_stream(stream);
    Scratch scratch(s);  // temporaries of this call
    const uint32_t n = n_spin_orb;
    const int W = words_for(n);
    const uint64_t n2 = static_cast<uint64_t>(n) * n;
    const uint64_t n4 = h2 ? n2 * n2 : 0;
    DevBuf<uint32_t> flag1(n2, s), off1(n2, s), cnt(2, s);
    hipLaunchKernelGGL(k_flag_abs_gt, dim3(grid_for(n2, 256, 65536)), dim3(256), 0, s, h1, n2, eps, flag1.get());
    exclusive_scan_u32(flag1.get(), off1.get(), n2, cnt.get(), s);
    DevBuf<uint32_t> flag2(n4, s), off2(n4, s);
    uint64_t k2 = 0;
    if (n4) {
      hipLaunchKernelGGL(k_flag_abs_gt, dim3(grid_for(n4, 256, 65536)), dim3(256), 0, s, h2, n4, eps, flag2.get());
      exclusive_scan_u32(flag2.get(), off2.get(), n4, cnt.get() + 1, s);
      k2 = read_scalar(cnt.get() + 1, s);
    }
    const uint64_t k1 = read_scalar(cnt.get(), s);
    const uint64_t m = 1 + 4 * k1 + 16 * k2;
    PBS_REQUIRE(m < (1ull << 32), PBS_ERR_RANGE, "more than 2^32 - 1 Pauli contributions");
    DevBuf<uint64_t> keys(m * 2 * W, s);
    DevBuf<double> re(m, s), im(m, s);
    hipLaunchKernelGGL(k_jw_identity, dim3(1), dim3(1), 0, s, W, m, e0, keys.get(), re.get(), im.get());
    if (k1)
      hipLaunchKernelGGL(k_jw_one_body, dim3(grid_for(n2, 256, 65536)), dim3(256), 0, s, n, W, h1, flag1.get(),
                         off1.get(), 1ull, m, keys.get(), re.get(), im.get());
    if (k2)
      hipLaunchKernelGGL(k_jw_two_body, dim3(grid_for(n4, 256, 65536)), dim3(256), 0, s, n, W, h2, flag2.get(),
                         off2.get(), 1ull + 4 * k1, m, keys.get(), re.get(), im.get());
    PBS_HIP(hipGetLastError());
    auto* res = new pbs_sum();
    try {
      canonicalize_soa(n, W, m, keys, re, im, eps_drop, *res, s);
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
  });
}

}  // extern "C"
