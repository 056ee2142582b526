// Warm-start network for the variational layer: a 1 -> H -> H -> O multilayer
// perceptron with tanh hidden layers that maps a geometry coordinate to the
// ansatz parameters, trained by full-batch Adam on the mean squared error.
//
// Every product takes bfloat16 operands and accumulates in float32 on the
// matrix cores (v_mfma_f32_16x16x32_bf16, one wavefront per 16x16 output
// tile).  Master weights, biases, Adam moments, activations kept for the
// backward pass and all bias gradients are float32; bf16 copies of W2 and W3
// are refreshed by the optimizer step.  Rounding points: R and W1 in the
// first layer, h1/W2 and h2/W3 in the forward products, dL/dy, dL/dz2 and the
// weights and activations they meet in the backward products.
//
// Batch rows are padded to a multiple of 32 (the K step of a weight-gradient
// product) and the output width to a multiple of 32 (the K step of dL/dh2);
// padded rows carry zero output error, padded output columns zero weights, so
// neither contributes to any gradient.
#include <cmath>
#include <vector>

#include "pbs_internal.h"

namespace pbs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr unsigned kMlpBlock = 256;  // 4 wavefronts, one output tile each
constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kAdamEps = 1e-8f;

// float -> bfloat16, round to nearest, ties to even (quiet NaN kept).
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
__device__ inline float round_bf16(float f) { return from_bf16(to_bf16(f)); }

enum Epi : int {
  kEpiTanh = 0,   // out = tanh(acc + bias); also bf16 copy
  kEpiOutput = 1, // y = acc + bias; optional output error dL/dy and loss partials
  kEpiStore = 2,  // out = acc (weight gradients)
  kEpiDTanh = 3,  // out = acc * (1 - h^2); optional bf16 copy
};

struct Gemm {
  // C[m][n] = sum_k A(m,k) B(k,n) over bf16 operands.
  const uint16_t* a;  // A(m,k) = a[m*lda + k] if A is k-contiguous, else a[k*lda + m]
  const uint16_t* b;  // B(k,n) = b[n*ldb + k] if B is k-contiguous, else b[k*ldb + n]
  uint32_t lda, ldb;
  uint32_t M, N, K;   // M, N multiples of 16; K a multiple of 32
  uint32_t m_valid, n_valid;
  const float* bias;  // kEpiTanh, kEpiOutput (n_valid entries)
  float* out;         // float32 result, ld ldo (may be null for kEpiOutput)
  uint32_t ldo;
  uint16_t* outb;     // bf16 copy / bf16 output error, ld ldb16
  uint32_t ldb16;
  float* out2;        // kEpiOutput: float32 output error, ld ldb16
  const float* aux;   // kEpiDTanh: activations (ld ldaux); kEpiOutput: targets (ld ldaux) or null
  uint32_t ldaux;
  float scale;        // kEpiOutput: 2 / (n * O)
  float* partial;     // kEpiOutput: per-tile sum of squared errors
};

template <bool KCONTIG>
__device__ inline bf16x8 load_frag(const uint16_t* p, uint32_t ld, uint32_t row, uint32_t k) {
  if (KCONTIG) {
    const uint4 w = *reinterpret_cast<const uint4*>(p + static_cast<size_t>(row) * ld + k);
    return __builtin_bit_cast(bf16x8, w);
  } else {
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t lo = p[static_cast<size_t>(k + 2 * e) * ld + row];
      const uint32_t hi = p[static_cast<size_t>(k + 2 * e + 1) * ld + row];
      w[e] = lo | (hi << 16);
    }
    return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
  }
}

// One wavefront per 16x16 tile of C.  Lane l holds row l%16 of the A slice
// and column l%16 of the B slice for k = 8*(l/16) .. 8*(l/16)+7 of each
// 32-wide K step, and receives C rows 4*(l/16) .. 4*(l/16)+3 of column l%16.
template <int EPI, bool AK, bool BK>
__global__ __launch_bounds__(kMlpBlock) void k_mlp_gemm(Gemm g) {
  const uint32_t tiles_n = g.N / 16;
  const uint32_t tile = blockIdx.x * (kMlpBlock / 64) + (threadIdx.x >> 6);
  if (tile >= (g.M / 16) * tiles_n) return;
  const uint32_t tm = tile / tiles_n, tn = tile % tiles_n;
  const uint32_t lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (uint32_t k0 = 0; k0 < g.K; k0 += 32) {
    const bf16x8 fa = load_frag<AK>(g.a, g.lda, tm * 16 + r, k0 + 8 * q);
    const bf16x8 fb = load_frag<BK>(g.b, g.ldb, tn * 16 + r, k0 + 8 * q);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc, 0, 0, 0);
  }
  const uint32_t n = tn * 16 + r;
  float sq = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t m = tm * 16 + 4 * q + i;
    const float v = acc[i];
    if (EPI == kEpiTanh) {
      if (m < g.m_valid && n < g.n_valid) {
        const float h = tanhf(v + g.bias[n]);
        g.out[static_cast<size_t>(m) * g.ldo + n] = h;
        g.outb[static_cast<size_t>(m) * g.ldb16 + n] = to_bf16(h);
      }
    } else if (EPI == kEpiOutput) {
      const bool valid = m < g.m_valid && n < g.n_valid;
      const float y = v + (n < g.n_valid ? g.bias[n] : 0.f);
      if (valid && g.out) g.out[static_cast<size_t>(m) * g.ldo + n] = y;
      if (g.aux) {
        const float d = valid ? y - g.aux[static_cast<size_t>(m) * g.ldaux + n] : 0.f;
        const float dy = g.scale * d;
        g.out2[static_cast<size_t>(m) * g.ldb16 + n] = dy;
        g.outb[static_cast<size_t>(m) * g.ldb16 + n] = to_bf16(dy);
        sq = fmaf(d, d, sq);
      }
    } else if (EPI == kEpiStore) {
      if (m < g.m_valid && n < g.n_valid) g.out[static_cast<size_t>(m) * g.ldo + n] = v;
    } else {
      if (m < g.m_valid && n < g.n_valid) {
        const float h = g.aux[static_cast<size_t>(m) * g.ldaux + n];
        const float d = v * (1.f - h * h);
        g.out[static_cast<size_t>(m) * g.ldo + n] = d;
        if (g.outb) g.outb[static_cast<size_t>(m) * g.ldb16 + n] = to_bf16(d);
      }
    }
  }
  if (EPI == kEpiOutput && g.aux) {
    for (int d = 32; d > 0; d >>= 1) sq += __shfl_xor(sq, d, 64);
    if (lane == 0) g.partial[tile] = sq;
  }
}

// h1 = tanh(bf16(x) bf16(W1) + b1) over the padded batch (x = 0 beyond n).
__global__ __launch_bounds__(kMlpBlock) void k_mlp_input(const float* __restrict__ x, uint32_t n, uint32_t rows,
                                                          uint32_t H, const float* __restrict__ w1,
                                                          const float* __restrict__ b1, float* __restrict__ h1,
                                                          uint16_t* __restrict__ h1b) {
  const uint32_t idx = blockIdx.x * kMlpBlock + threadIdx.x;
  if (idx >= rows * H) return;
  const uint32_t b = idx / H, j = idx % H;
  const float xv = b < n ? round_bf16(x[b]) : 0.f;
  const float h = tanhf(fmaf(xv, round_bf16(w1[j]), b1[j]));
  h1[idx] = h;
  h1b[idx] = to_bf16(h);
}

// Column sums over the padded batch: first-layer weight and bias gradients,
// the other bias gradients, and the loss from the output tiles' partials.
__global__ __launch_bounds__(kMlpBlock) void k_mlp_colsum(const float* __restrict__ x, uint32_t n, uint32_t rows,
                                                           uint32_t H, uint32_t O, uint32_t Op,
                                                           const float* __restrict__ dz1,
                                                           const float* __restrict__ dz2,
                                                           const float* __restrict__ dy,
                                                           const float* __restrict__ partial, uint32_t n_partial,
                                                           float* __restrict__ grad, float* __restrict__ loss,
                                                           const uint32_t* __restrict__ steps, uint32_t n_slots) {
  const uint32_t c = blockIdx.x * kMlpBlock + threadIdx.x;
  const size_t off_b1 = H, off_b2 = 3ull * H + static_cast<size_t>(H) * H - H;
  const size_t off_b3 = 3ull * H + static_cast<size_t>(H) * H + static_cast<size_t>(O) * H;
  if (c < H) {
    float sw = 0.f, sb = 0.f;
    for (uint32_t b = 0; b < rows; ++b) {
      const float d = dz1[static_cast<size_t>(b) * H + c];
      sb += d;
      if (b < n) sw = fmaf(d, round_bf16(x[b]), sw);
    }
    grad[c] = sw;
    grad[off_b1 + c] = sb;
  } else if (c < 2 * H) {
    const uint32_t j = c - H;
    float s = 0.f;
    for (uint32_t b = 0; b < rows; ++b) s += dz2[static_cast<size_t>(b) * H + j];
    grad[off_b2 + j] = s;
  } else if (c < 2 * H + O) {
    const uint32_t j = c - 2 * H;
    float s = 0.f;
    for (uint32_t b = 0; b < rows; ++b) s += dy[static_cast<size_t>(b) * Op + j];
    grad[off_b3 + j] = s;
  } else if (c == 2 * H + O && loss) {
    float s = 0.f;
    for (uint32_t t = 0; t < n_partial; ++t) s += partial[t];
    // during training, loss[steps[0] - steps[1]]: the step count and the
    // count at the start of the current call, both kept on the device
    const uint32_t slot = steps ? steps[0] - steps[1] : 0u;
    if (slot < n_slots) loss[slot] = s / (static_cast<float>(n) * static_cast<float>(O));
  }
}

// Adam with bias correction for step *steps + 1 (the count is kept on the
// device so that one captured step can be replayed); refreshes the bf16
// copies of W2 and W3.
__global__ __launch_bounds__(kMlpBlock) void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                                                         float* __restrict__ m1, float* __restrict__ m2,
                                                         uint64_t count, float lr, const uint32_t* __restrict__ steps,
                                                         uint64_t off_w2, uint64_t n_w2, uint16_t* __restrict__ w2b,
                                                         uint64_t off_w3, uint64_t n_w3,
                                                         uint16_t* __restrict__ w3b) {
  const double t = static_cast<double>(*steps) + 1.0;
  const float bc1 = static_cast<float>(1.0 / (1.0 - pow(static_cast<double>(kBeta1), t)));
  const float bc2 = static_cast<float>(1.0 / (1.0 - pow(static_cast<double>(kBeta2), t)));
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(kMlpBlock) + threadIdx.x; i < count;
       i += static_cast<uint64_t>(gridDim.x) * kMlpBlock) {
    const float gi = g[i];
    const float a = kBeta1 * m1[i] + (1.f - kBeta1) * gi;
    const float v = kBeta2 * m2[i] + (1.f - kBeta2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float w = p[i] - lr * (a * bc1) / (sqrtf(v * bc2) + kAdamEps);
    p[i] = w;
    if (i - off_w2 < n_w2) w2b[i - off_w2] = to_bf16(w);
    if (i - off_w3 < n_w3) w3b[i - off_w3] = to_bf16(w);
  }
}

__global__ void k_mlp_tick(uint32_t* steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) steps[0] += 1u;
}

// Start of a training call: the loss slots of the call count from here.
__global__ void k_mlp_mark(uint32_t* steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) steps[1] = steps[0];
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_refresh(const float* __restrict__ p, uint64_t off_w2,
                                                            uint64_t n_w2, uint16_t* __restrict__ w2b,
                                                            uint64_t off_w3, uint64_t n_w3,
                                                            uint16_t* __restrict__ w3b) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(kMlpBlock) + threadIdx.x; i < n_w2 + n_w3;
       i += static_cast<uint64_t>(gridDim.x) * kMlpBlock) {
    if (i < n_w2)
      w2b[i] = to_bf16(p[off_w2 + i]);
    else
      w3b[i - n_w2] = to_bf16(p[off_w3 + i - n_w2]);
  }
}

inline uint32_t round_up32(uint32_t v) { return (v + 31u) & ~31u; }

}  // namespace
}  // namespace pbs

using namespace pbs;

struct pbs_mlp {
  uint32_t H = 0, O = 0, Op = 0, max_rows = 0;
  uint64_t count = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
  uint64_t step = 0;  // Adam steps requested through direct calls (a bound, not the count)
  DevBuf<float> params, grads, mom1, mom2;
  DevBuf<uint16_t> w2b, w3b;
  DevBuf<float> h1, h2, dy, dz2, dz1, partial, loss;
  DevBuf<uint32_t> steps;  // [Adam steps taken, steps taken when the current call began], on the device
  DevBuf<uint16_t> h1b, h2b, dyb, dz2b;
};

namespace pbs {
namespace {

template <int EPI, bool AK, bool BK>
void launch_gemm(const Gemm& g, hipStream_t s) {
  const uint32_t tiles = (g.M / 16) * (g.N / 16);
  hipLaunchKernelGGL((k_mlp_gemm<EPI, AK, BK>), dim3((tiles + 3) / 4), dim3(kMlpBlock), 0, s, g);
}

// Forward pass over rows = round_up32(n) padded rows.  With targets the
// output error and loss partials are written for a following backward pass.
void forward(pbs_mlp& m, uint32_t n, const float* x, float* y, const float* t, hipStream_t s) {
  const uint32_t rows = round_up32(n), H = m.H;
  const float* p = m.params.get();
  hipLaunchKernelGGL(k_mlp_input, dim3((rows * H + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0, s, x, n, rows, H,
                     p, p + H, m.h1.get(), m.h1b.get());
  Gemm g{};
  g.a = m.h1b.get();
  g.lda = H;
  g.b = m.w2b.get();
  g.ldb = H;
  g.M = rows;
  g.N = H;
  g.K = H;
  g.m_valid = rows;
  g.n_valid = H;
  g.bias = p + m.off_b2;
  g.out = m.h2.get();
  g.ldo = H;
  g.outb = m.h2b.get();
  g.ldb16 = H;
  launch_gemm<kEpiTanh, true, true>(g, s);
  Gemm o{};
  o.a = m.h2b.get();
  o.lda = H;
  o.b = m.w3b.get();
  o.ldb = H;
  o.M = rows;
  o.N = m.Op;
  o.K = H;
  o.m_valid = n;
  o.n_valid = m.O;
  o.bias = p + m.off_b3;
  o.out = y;
  o.ldo = m.O;
  o.outb = m.dyb.get();
  o.ldb16 = m.Op;
  o.out2 = m.dy.get();
  o.aux = t;
  o.ldaux = m.O;
  o.scale = 2.0f / (static_cast<float>(n) * static_cast<float>(m.O));
  o.partial = m.partial.get();
  launch_gemm<kEpiOutput, true, true>(o, s);
}

// Backward pass after forward(..., t): gradients into grad (packed layout).
void backward(pbs_mlp& m, uint32_t n, const float* x, float* grad, float* loss, const uint32_t* steps, uint32_t n_slots,
              hipStream_t s) {
  const uint32_t rows = round_up32(n), H = m.H, Op = m.Op;
  // dW3[j][k] = sum_b dy[b][j] h2[b][k]
  Gemm w3{};
  w3.a = m.dyb.get();
  w3.lda = Op;
  w3.b = m.h2b.get();
  w3.ldb = H;
  w3.M = Op;
  w3.N = H;
  w3.K = rows;
  w3.m_valid = m.O;
  w3.n_valid = H;
  w3.out = grad + m.off_w3;
  w3.ldo = H;
  launch_gemm<kEpiStore, false, false>(w3, s);
  // dz2[b][k] = (sum_j dy[b][j] W3[j][k]) (1 - h2^2)
  Gemm z2{};
  z2.a = m.dyb.get();
  z2.lda = Op;
  z2.b = m.w3b.get();
  z2.ldb = H;
  z2.M = rows;
  z2.N = H;
  z2.K = Op;
  z2.m_valid = rows;
  z2.n_valid = H;
  z2.out = m.dz2.get();
  z2.ldo = H;
  z2.outb = m.dz2b.get();
  z2.ldb16 = H;
  z2.aux = m.h2.get();
  z2.ldaux = H;
  launch_gemm<kEpiDTanh, true, false>(z2, s);
  // dW2[j][k] = sum_b dz2[b][j] h1[b][k]
  Gemm w2{};
  w2.a = m.dz2b.get();
  w2.lda = H;
  w2.b = m.h1b.get();
  w2.ldb = H;
  w2.M = H;
  w2.N = H;
  w2.K = rows;
  w2.m_valid = H;
  w2.n_valid = H;
  w2.out = grad + m.off_w2;
  w2.ldo = H;
  launch_gemm<kEpiStore, false, false>(w2, s);
  // dz1[b][k] = (sum_j dz2[b][j] W2[j][k]) (1 - h1^2)
  Gemm z1{};
  z1.a = m.dz2b.get();
  z1.lda = H;
  z1.b = m.w2b.get();
  z1.ldb = H;
  z1.M = rows;
  z1.N = H;
  z1.K = H;
  z1.m_valid = rows;
  z1.n_valid = H;
  z1.out = m.dz1.get();
  z1.ldo = H;
  z1.aux = m.h1.get();
  z1.ldaux = H;
  launch_gemm<kEpiDTanh, true, false>(z1, s);
  const uint32_t cols = 2 * H + m.O + 1;
  hipLaunchKernelGGL(k_mlp_colsum, dim3((cols + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0, s, x, n, rows, H,
                     m.O, Op, m.dz1.get(), m.dz2.get(), m.dy.get(), m.partial.get(), (rows / 16) * (Op / 16), grad,
                     loss, steps, n_slots);
}

void adam(pbs_mlp& m, float lr, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(m.count, kMlpBlock, 1024)), dim3(kMlpBlock), 0, s, m.params.get(),
                     m.grads.get(), m.mom1.get(), m.mom2.get(), m.count, lr, m.steps.get(), m.off_w2,
                     static_cast<uint64_t>(m.H) * m.H, m.w2b.get(), m.off_w3, static_cast<uint64_t>(m.O) * m.H,
                     m.w3b.get());
  hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(64), 0, s, m.steps.get());
}

// One training step: forward, backward (loss into the call's next slot of
// losses, of which there are n_slots), Adam.
void train_step(pbs_mlp& m, uint32_t n, const float* x, const float* t, float lr, float* losses, uint32_t n_slots,
                hipStream_t s) {
  forward(m, n, x, nullptr, t, s);
  backward(m, n, x, m.grads.get(), losses, losses ? m.steps.get() : nullptr, n_slots, s);
  adam(m, lr, s);
}

void load_params(pbs_mlp& m, const float* params, hipStream_t s) {
  PBS_HIP(hipMemcpyAsync(m.params.get(), params, m.count * sizeof(float), hipMemcpyDefault, s));
  PBS_HIP(hipMemsetAsync(m.mom1.get(), 0, m.count * sizeof(float), s));
  PBS_HIP(hipMemsetAsync(m.mom2.get(), 0, m.count * sizeof(float), s));
  PBS_HIP(hipMemsetAsync(m.steps.get(), 0, 2 * sizeof(uint32_t), s));
  m.step = 0;
  const uint64_t n2 = static_cast<uint64_t>(m.H) * m.H, n3 = static_cast<uint64_t>(m.O) * m.H;
  hipLaunchKernelGGL(k_mlp_refresh, dim3(grid_for(n2 + n3, kMlpBlock, 1024)), dim3(kMlpBlock), 0, s,
                     m.params.get(), m.off_w2, n2, m.w2b.get(), m.off_w3, n3, m.w3b.get());
  PBS_HIP(hipGetLastError());
}

void check_batch(const pbs_mlp* m, uint32_t n) {
  PBS_REQUIRE(m != nullptr, PBS_ERR_ARG, "null pbs_mlp");
  PBS_REQUIRE(n >= 1 && n <= m->max_rows, PBS_ERR_RANGE,
              "batch of " + std::to_string(n) + " rows outside 1.." + std::to_string(m->max_rows));
}

}  // namespace
}  // namespace pbs

extern "C" {

pbs_status pbs_mlp_param_count(uint32_t hidden, uint32_t n_out, uint64_t* count) {
  return guarded([&] {
    PBS_REQUIRE(count != nullptr, PBS_ERR_ARG, "null output");
    *count = 3ull * hidden + static_cast<uint64_t>(hidden) * hidden + static_cast<uint64_t>(n_out) * hidden + n_out;
  });
}

pbs_status pbs_mlp_create(uint32_t hidden, uint32_t n_out, uint32_t max_batch, const float* params, void* stream,
                          pbs_mlp** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(hidden >= 32 && hidden <= 1024 && hidden % 32 == 0, PBS_ERR_RANGE,
                "hidden width must be a multiple of 32 in 32..1024");
    PBS_REQUIRE(n_out >= 1 && n_out <= 1024, PBS_ERR_RANGE, "output width must be in 1..1024");
    PBS_REQUIRE(max_batch >= 1 && max_batch <= 4096, PBS_ERR_RANGE, "max_batch must be in 1..4096");
    PBS_REQUIRE(params != nullptr, PBS_ERR_ARG, "null initial parameters");
    hipStream_t s = as_stream(stream);
    auto* m = new pbs_mlp();
    try {
      const uint32_t H = hidden, O = n_out, Op = round_up32(n_out), R = round_up32(max_batch);
      m->H = H;
      m->O = O;
      m->Op = Op;
      m->max_rows = max_batch;
      m->count = 3ull * H + static_cast<uint64_t>(H) * H + static_cast<uint64_t>(O) * H + O;
      m->off_w2 = 2ull * H;
      m->off_b2 = m->off_w2 + static_cast<uint64_t>(H) * H;
      m->off_w3 = m->off_b2 + H;
      m->off_b3 = m->off_w3 + static_cast<uint64_t>(O) * H;
      m->params.alloc(m->count);
      m->grads.alloc(m->count);
      m->mom1.alloc(m->count);
      m->mom2.alloc(m->count);
      m->w2b.alloc(static_cast<size_t>(H) * H);
      m->w3b.alloc(static_cast<size_t>(Op) * H);
      PBS_HIP(hipMemsetAsync(m->w3b.get(), 0, static_cast<size_t>(Op) * H * 2, s));  // padded rows stay zero
      const size_t act = static_cast<size_t>(R) * H, outs = static_cast<size_t>(R) * Op;
      m->h1.alloc(act);
      m->h2.alloc(act);
      m->dz2.alloc(act);
      m->dz1.alloc(act);
      m->h1b.alloc(act);
      m->h2b.alloc(act);
      m->dz2b.alloc(act);
      m->dy.alloc(outs);
      m->dyb.alloc(outs);
      m->partial.alloc((R / 16) * (Op / 16));
      m->loss.alloc(1);
      m->steps.alloc(2);
      load_params(*m, params, s);
      PBS_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

pbs_status pbs_mlp_set_params(pbs_mlp* m, const float* params, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(m != nullptr && params != nullptr, PBS_ERR_ARG, "null argument");
    load_params(*m, params, as_stream(stream));
    PBS_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pbs_status pbs_mlp_get_params(const pbs_mlp* m, float* params, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(m != nullptr && params != nullptr, PBS_ERR_ARG, "null argument");
    PBS_HIP(hipMemcpyAsync(params, m->params.get(), m->count * sizeof(float), hipMemcpyDefault, as_stream(stream)));
    PBS_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pbs_status pbs_mlp_forward(pbs_mlp* m, uint32_t n, const float* x, float* y, void* stream) {
  return guarded([&] {
    check_batch(m, n);
    PBS_REQUIRE(x != nullptr && y != nullptr, PBS_ERR_ARG, "null argument");
    forward(*m, n, x, y, nullptr, as_stream(stream));
    PBS_HIP(hipGetLastError());
  });
}

pbs_status pbs_mlp_loss_grad(pbs_mlp* m, uint32_t n, const float* x, const float* t, float* loss, float* grad,
                             void* stream) {
  return guarded([&] {
    check_batch(m, n);
    PBS_REQUIRE(x != nullptr && t != nullptr && grad != nullptr, PBS_ERR_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    forward(*m, n, x, nullptr, t, s);
    backward(*m, n, x, grad, loss, nullptr, 1u, s);
    PBS_HIP(hipGetLastError());
  });
}

pbs_status pbs_mlp_train(pbs_mlp* m, uint32_t n, const float* x, const float* t, uint32_t n_steps, float lr,
                         float* losses, void* stream) {
  return guarded([&] {
    check_batch(m, n);
    PBS_REQUIRE(x != nullptr && t != nullptr, PBS_ERR_ARG, "null argument");
    PBS_REQUIRE(lr > 0.f && std::isfinite(lr), PBS_ERR_ARG, "learning rate must be positive");
    PBS_REQUIRE(m->step + n_steps < (1ull << 32), PBS_ERR_RANGE, "step count beyond 2^32");
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_mlp_mark, dim3(1), dim3(64), 0, s, m->steps.get());
    for (uint32_t i = 0; i < n_steps; ++i) train_step(*m, n, x, t, lr, losses, n_steps, s);
    m->step += n_steps;
    PBS_HIP(hipGetLastError());
  });
}

void pbs_mlp_destroy(pbs_mlp* m) { delete m; }

}  // extern "C"
