// Device primitives: exclusive scan, stable LSD radix sort on multiword keys,
// segment-head marking.  They carry the canonical reduction of Section 2.3
// (radix sort of the binary symplectic keys, then a linear merge) and the
// grouping of Eq. topological_group.
#include "pbs_internal.h"

namespace pbs {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr uint64_t kScanTile = kScanBlock * kScanItems;

// Exclusive scan of one value per thread across a 256-thread block (4 wave64s).
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_wave, uint32_t& block_total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) lds_wave[wave] = incl;
  __syncthreads();
  uint32_t wave_off = 0;
  uint32_t total = 0;
  for (int w = 0; w < kScanBlock / 64; ++w) {
    uint32_t t = lds_wave[w];
    if (w < wave) wave_off += t;
    total += t;
  }
  __syncthreads();
  block_total = total;
  return wave_off + incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(const uint32_t* in, uint64_t n, uint32_t* partial) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    uint64_t i = base + j;
    if (i < n) s += in[i];
  }
  uint32_t total;
  (void)block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single block: exclusive scan of the per-tile partial sums.
__global__ __launch_bounds__(kScanBlock) void k_scan_partials_scan(uint32_t* partial, uint64_t nb, uint32_t* total_out) {
  __shared__ uint32_t lds[kScanBlock / 64];
  uint32_t carry = 0;
  for (uint64_t c = 0; c < nb; c += kScanBlock) {
    uint64_t i = c + threadIdx.x;
    uint32_t v = i < nb ? partial[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, lds, tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t* in, uint32_t* out, uint64_t n, const uint32_t* partial) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    uint64_t i = base + j;
    v[j] = i < n ? in[i] : 0u;
    s += v[j];
  }
  uint32_t tot;
  uint32_t run = partial[blockIdx.x] + block_exclusive_scan(s, lds, tot);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    uint64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
}

// Single block: the whole scan for short inputs (at most kScanSingleTiles
// tiles), tile after tile with a running carry; in == out is allowed (each
// thread reads its items before the block scan and writes them after it).
constexpr uint64_t kScanSingleTiles = 16;
__global__ __launch_bounds__(kScanBlock) void k_scan_single(const uint32_t* in, uint32_t* out, uint64_t n,
                                                            uint32_t* total_out) {
  __shared__ uint32_t lds[kScanBlock / 64];
  uint32_t carry = 0;
  for (uint64_t c = 0; c < n; c += kScanTile) {
    const uint64_t base = c + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const uint64_t i = base + j;
      v[j] = i < n ? in[i] : 0u;
      s += v[j];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(s, lds, tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const uint64_t i = base + j;
      if (i < n) out[i] = run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// ---------------------------------------------------------------- radix sort
constexpr int kSortBlock = 256;
constexpr uint32_t kSortTile = 4096;

// OR over all items of (key ^ key[0]) per word: the bits that vary.
__global__ __launch_bounds__(256) void k_varying_bits(const uint64_t* keys, uint64_t m, int nw, unsigned long long* out) {
  for (int w = 0; w < nw; ++w) {
    const uint64_t* k = keys + static_cast<uint64_t>(w) * m;
    const uint64_t ref = k[0];
    uint64_t acc = 0;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < m; i += gridDim.x * 256ull) acc |= (k[i] ^ ref);
    // wave reduction
    for (int d = 32; d > 0; d >>= 1) acc |= __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicOr(out + w, static_cast<unsigned long long>(acc));
  }
}

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint64_t* key, uint64_t m, uint32_t shift, uint32_t* counts,
                                                           uint32_t nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t start = static_cast<uint64_t>(blockIdx.x) * kSortTile;
  const uint64_t end = start + kSortTile < m ? start + kSortTile : m;
  for (uint64_t i = start + threadIdx.x; i < end; i += kSortBlock) {
    atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[static_cast<uint64_t>(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items of a tile are ranked in index order, 256 at a time.
// Within a wave, items with equal digits are matched by eight ballots; waves
// are ordered through per-wave digit counts in LDS.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const uint64_t* kin, uint64_t* kout, int nw, const uint32_t* vin,
                                                              uint32_t* vout, uint64_t m, int word, uint32_t shift,
                                                              const uint32_t* offsets, uint32_t nblk) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kSortBlock / 64][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  base[tid] = offsets[static_cast<uint64_t>(tid) * nblk + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kSortBlock / 64; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t start = static_cast<uint64_t>(blockIdx.x) * kSortTile;
  const uint64_t end = start + kSortTile < m ? start + kSortTile : m;
  const uint64_t* kd = kin + static_cast<uint64_t>(word) * m;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint64_t c = start; c < end; c += kSortBlock) {
    const uint64_t i = c + tid;
    const bool valid = i < end;
    const uint32_t dg = valid ? static_cast<uint32_t>((kd[i] >> shift) & 255u) : 0u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const unsigned long long mb = __ballot(bit);
      peers &= bit ? mb : ~mb;
    }
    const uint32_t rank = static_cast<uint32_t>(__popcll(peers & below));
    if (valid && rank == 0) wcnt[wave][dg] = static_cast<uint32_t>(__popcll(peers));
    __syncthreads();
    if (valid) {
      uint32_t pos = base[dg] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dg];
      if (pos >= m) pos = static_cast<uint32_t>(i);  // unreachable with consistent counts; keeps writes in bounds
      for (int w = 0; w < nw; ++w) kout[static_cast<uint64_t>(w) * m + pos] = kin[static_cast<uint64_t>(w) * m + i];
      vout[pos] = vin[i];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kSortBlock / 64; ++w) {
      add += wcnt[w][tid];
      wcnt[w][tid] = 0;
    }
    base[tid] += add;
    __syncthreads();
  }
}

__global__ void k_mark_heads(const uint64_t* keys, uint64_t m, int nw, uint32_t* heads) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    uint32_t h = 1;
    if (i > 0) {
      h = 0;
      for (int w = 0; w < nw; ++w) {
        if (keys[static_cast<uint64_t>(w) * m + i] != keys[static_cast<uint64_t>(w) * m + i - 1]) {
          h = 1;
          break;
        }
      }
    }
    heads[i] = h;
  }
}

__global__ void k_iota(uint32_t* v, uint64_t m) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    v[i] = static_cast<uint32_t>(i);
}

}  // namespace

void iota_u32(uint32_t* v, uint64_t m, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, v, m);
  PBS_HIP(hipGetLastError());
}

size_t scan_scratch_bytes(uint64_t n) { return ((n + kScanTile - 1) / kScanTile + 1) * sizeof(uint32_t); }

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total, hipStream_t s) {
  PBS_REQUIRE(n < (1ull << 32), PBS_ERR_RANGE, "scan length exceeds 2^32");
  if (n == 0) {
    if (total) PBS_HIP(hipMemsetAsync(total, 0, sizeof(uint32_t), s));
    return;
  }
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= kScanSingleTiles) {  // one launch, no temporary
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanBlock), 0, s, in, out, n, total);
    PBS_HIP(hipGetLastError());
    return;
  }
  DevBuf<uint32_t> partial(nb, s);
  hipLaunchKernelGGL(k_scan_partials, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, s, in, n, partial.get());
  hipLaunchKernelGGL(k_scan_partials_scan, dim3(1), dim3(kScanBlock), 0, s, partial.get(), nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, s, in, out, n, partial.get());
  PBS_HIP(hipGetLastError());
  // `partial` is released on return: a temporary of the call's scratch scope
  // stays reserved until the scope ends (which waits for the stream); one
  // from hipMalloc must not be freed under queued work
  if (!partial.borrowed) PBS_HIP(hipStreamSynchronize(s));
}

void mark_heads(const uint64_t* keys, uint64_t m, int nw, uint32_t* heads, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_mark_heads, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, keys, m, nw, heads);
  PBS_HIP(hipGetLastError());
}

void radix_sort_keys(uint64_t* keys, uint32_t* vals, uint64_t m, int nw, hipStream_t s) {
  PBS_REQUIRE(m < (1ull << 32), PBS_ERR_RANGE, "sort length exceeds 2^32");
  if (m <= 1) return;
  DevBuf<unsigned long long> vary(nw, s);
  PBS_HIP(hipMemsetAsync(vary.get(), 0, nw * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_varying_bits, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s, keys, m, nw, vary.get());
  PBS_HIP(hipGetLastError());
  std::vector<unsigned long long> hv(nw);
  PBS_HIP(hipMemcpyAsync(hv.data(), vary.get(), nw * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  PBS_HIP(hipStreamSynchronize(s));

  const uint32_t nblk = static_cast<uint32_t>((m + kSortTile - 1) / kSortTile);
  DevBuf<uint64_t> ktmp(m * nw, s);
  DevBuf<uint32_t> vtmp(m, s);
  DevBuf<uint32_t> counts(static_cast<uint64_t>(nblk) * 256, s);
  uint64_t* kcur = keys;
  uint32_t* vcur = vals;
  uint64_t* kalt = ktmp.get();
  uint32_t* valt = vtmp.get();
  for (int w = 0; w < nw; ++w) {
    for (uint32_t shift = 0; shift < 64; shift += 8) {
      if (((hv[w] >> shift) & 255ull) == 0) continue;  // digit equal for every item
      hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortBlock), 0, s, kcur + static_cast<uint64_t>(w) * m, m, shift,
                         counts.get(), nblk);
      exclusive_scan_u32(counts.get(), counts.get(), static_cast<uint64_t>(nblk) * 256, nullptr, s);
      hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortBlock), 0, s, kcur, kalt, nw, vcur, valt, m, w, shift,
                         counts.get(), nblk);
      PBS_HIP(hipGetLastError());
      std::swap(kcur, kalt);
      std::swap(vcur, valt);
    }
  }
  if (kcur != keys) {
    PBS_HIP(hipMemcpyAsync(keys, kcur, m * nw * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    PBS_HIP(hipMemcpyAsync(vals, vcur, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
  // temporaries of the call's scratch scope stay reserved until it ends;
  // hipMalloc'd ones are freed on return, after the queued work
  if (!(vary.borrowed && ktmp.borrowed && vtmp.borrowed && counts.borrowed)) PBS_HIP(hipStreamSynchronize(s));
}

}  // namespace pbs
