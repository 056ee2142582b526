// Configuration spaces: full 2^n space and fixed-(N_alpha, N_beta) spin
// sectors of the spin-resolved product basis (Section 2.4; Eq. fcidim).
//
// Spin strings of n_orb bits with N ones are listed in ascending integer
// order.  The position of a string in that list is its combinatorial
// (colexicographic) rank, sum_i C(p_i, i + 1) over its set bits p_0 < p_1 <
// ...; it is evaluated one 8-bit chunk at a time from tables
// T[c][k][byte] = sum over the set bits q_j of `byte` of C(8c + q_j, k + j + 1),
// where k is the number of ones below the chunk.  Unranking reads the list.
#include "handles.h"

namespace pbs {
namespace {

__host__ __device__ inline uint64_t binom(uint32_t n, uint32_t r) {
  if (r > n) return 0;
  if (r > n - r) r = n - r;
  uint64_t v = 1;
  for (uint32_t i = 1; i <= r; ++i) v = v * (n - r + i) / i;  // exact at every step
  return v;
}

__global__ void k_rank_tables(uint32_t n_orb, uint32_t n_chunks, uint32_t* tab) {
  const uint32_t total = n_chunks * (n_orb + 1) * 256;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const uint32_t b = e & 255u;
    const uint32_t k = (e >> 8) % (n_orb + 1);
    const uint32_t c = (e >> 8) / (n_orb + 1);
    uint64_t v = 0;
    uint32_t j = 0;
    for (uint32_t q = 0; q < 8; ++q) {
      if ((b >> q) & 1u) {
        v += binom(8 * c + q, k + j + 1);
        ++j;
      }
    }
    tab[e] = static_cast<uint32_t>(v);
  }
}

// Greedy combinatorial unranking: the largest q with C(q, r) <= rest is the
// position of the r-th one (counting from the top).
__global__ void k_unrank_all(uint32_t n_orb, uint32_t n_ones, uint64_t count, uint32_t* out) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    uint64_t rest = i;
    uint32_t word = 0;
    uint32_t q = n_orb;
    for (uint32_t r = n_ones; r >= 1; --r) {
      do {
        --q;
      } while (binom(q, r) > rest);
      word |= 1u << q;
      rest -= binom(q, r);
    }
    out[i] = word;
  }
}

__global__ void k_narrow_u16(const uint32_t* in, uint64_t n, uint16_t* out) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<uint16_t>(in[i]);
}

__device__ inline uint32_t rank_string(uint32_t s, uint32_t n_orb, uint32_t n_chunks, const uint32_t* tab) {
  uint32_t r = 0;
  uint32_t below = 0;
  for (uint32_t c = 0; c < n_chunks; ++c) {
    const uint32_t byte = (s >> (8 * c)) & 255u;
    r += tab[(c * (n_orb + 1) + below) * 256 + byte];
    below += __popc(byte);
  }
  return r;
}

__global__ void k_space_rank(bool sector, uint32_t n_qubits, uint32_t n_orb, uint32_t na, uint32_t nb, uint64_t db,
                             uint32_t n_chunks, const uint32_t* tab, uint64_t n, const uint64_t* bits, int64_t* idx) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t b = bits[i];
    if (!sector) {
      idx[i] = (n_qubits >= 64 || (b >> n_qubits) == 0) ? static_cast<int64_t>(b) : -1;
      continue;
    }
    const uint64_t mask = (n_orb == 32) ? 0xffffffffull : ((1ull << n_orb) - 1ull);
    const uint32_t a = static_cast<uint32_t>(b & mask);
    const uint32_t be = static_cast<uint32_t>((b >> n_orb) & mask);
    const bool high = (2 * n_orb < 64) && ((b >> (2 * n_orb)) != 0);
    if (high || static_cast<uint32_t>(__popc(a)) != na || static_cast<uint32_t>(__popc(be)) != nb) {
      idx[i] = -1;
      continue;
    }
    const uint64_t ra = rank_string(a, n_orb, n_chunks, tab);
    const uint64_t rb = rank_string(be, n_orb, n_chunks, tab);
    idx[i] = static_cast<int64_t>(ra * db + rb);
  }
}

__global__ void k_space_unrank(bool sector, uint32_t n_orb, uint64_t dim, uint64_t db, const uint32_t* sa,
                               const uint32_t* sb, uint64_t n, const int64_t* idx, uint64_t* bits) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const int64_t v = idx[i];
    if (v < 0 || static_cast<uint64_t>(v) >= dim) {
      bits[i] = ~0ull;
      continue;
    }
    if (!sector) {
      bits[i] = static_cast<uint64_t>(v);
      continue;
    }
    const uint64_t ia = static_cast<uint64_t>(v) / db, ib = static_cast<uint64_t>(v) % db;
    bits[i] = static_cast<uint64_t>(sa[ia]) | (static_cast<uint64_t>(sb[ib]) << n_orb);
  }
}

void check_space(const pbs_space* sp) { PBS_REQUIRE(sp != nullptr, PBS_ERR_ARG, "null pbs_space"); }

}  // namespace

uint64_t host_binom(uint32_t n, uint32_t r) { return binom(n, r); }

}  // namespace pbs

using namespace pbs;

extern "C" {

pbs_status pbs_space_full(uint32_t n_qubits, pbs_space** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(n_qubits >= 1 && n_qubits <= 40, PBS_ERR_RANGE, "full space supports 1..40 qubits");
    auto* sp = new pbs_space();
    sp->sector = false;
    sp->n_qubits = n_qubits;
    sp->dim = 1ull << n_qubits;
    *out = sp;
  });
}

pbs_status pbs_space_sector(uint32_t n_orb, uint32_t n_alpha, uint32_t n_beta, void* stream, pbs_space** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(n_orb >= 1 && n_orb <= 32, PBS_ERR_RANGE, "n_orb must be 1..32");
    PBS_REQUIRE(n_alpha <= n_orb && n_beta <= n_orb, PBS_ERR_ARG, "more electrons of one spin than orbitals");
    const uint64_t da = binom(n_orb, n_alpha), db = binom(n_orb, n_beta);
    PBS_REQUIRE(da < (1ull << 32) && db < (1ull << 32), PBS_ERR_RANGE, "spin-string count exceeds 2^32");
    PBS_REQUIRE(da * db < (1ull << 40), PBS_ERR_RANGE, "sector dimension exceeds 2^40");
    hipStream_t s = as_stream(stream);
    auto* sp = new pbs_space();
    try {
      sp->sector = true;
      sp->n_qubits = 2 * n_orb;
      sp->n_orb = n_orb;
      sp->n_alpha = n_alpha;
      sp->n_beta = n_beta;
      sp->dim_alpha = da;
      sp->dim_beta = db;
      sp->dim = da * db;
      sp->n_chunks = (n_orb + 7) / 8;
      const size_t nt = rank_tab_entries(n_orb);
      sp->rank_tab.alloc(nt);
      sp->str_alpha.alloc(da);
      sp->str_beta.alloc(db);
      hipLaunchKernelGGL(k_rank_tables, dim3(grid_for(nt, 256, 4096)), dim3(256), 0, s, n_orb, sp->n_chunks,
                         sp->rank_tab.get());
      if (n_orb <= 16) {
        sp->rank_tab16.alloc(nt);
        hipLaunchKernelGGL(k_narrow_u16, dim3(grid_for(nt, 256, 4096)), dim3(256), 0, s, sp->rank_tab.get(), nt,
                           sp->rank_tab16.get());
      }
      hipLaunchKernelGGL(k_unrank_all, dim3(grid_for(da, 256, 65536)), dim3(256), 0, s, n_orb, n_alpha, da,
                         sp->str_alpha.get());
      hipLaunchKernelGGL(k_unrank_all, dim3(grid_for(db, 256, 65536)), dim3(256), 0, s, n_orb, n_beta, db,
                         sp->str_beta.get());
      PBS_HIP(hipGetLastError());
      PBS_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete sp;
      throw;
    }
    *out = sp;
  });
}

pbs_status pbs_space_dim(const pbs_space* sp, uint64_t* dim) {
  return guarded([&] {
    check_space(sp);
    PBS_REQUIRE(dim != nullptr, PBS_ERR_ARG, "null output");
    *dim = sp->dim;
  });
}

pbs_status pbs_space_shape(const pbs_space* sp, uint32_t* n_orb, uint32_t* n_alpha, uint32_t* n_beta,
                           uint64_t* dim_alpha, uint64_t* dim_beta) {
  return guarded([&] {
    check_space(sp);
    if (n_orb) *n_orb = sp->n_orb;
    if (n_alpha) *n_alpha = sp->n_alpha;
    if (n_beta) *n_beta = sp->n_beta;
    if (dim_alpha) *dim_alpha = sp->dim_alpha;
    if (dim_beta) *dim_beta = sp->dim_beta;
    PBS_REQUIRE(sp->sector, PBS_ERR_ARG, "not a sector space");
  });
}

pbs_status pbs_space_rank(const pbs_space* sp, uint64_t n, const uint64_t* bits, int64_t* idx, void* stream) {
  return guarded([&] {
    check_space(sp);
    if (n == 0) return;
    PBS_REQUIRE(bits && idx, PBS_ERR_ARG, "null array");
    hipLaunchKernelGGL(k_space_rank, dim3(grid_for(n, 256, 65536)), dim3(256), 0, as_stream(stream), sp->sector,
                       sp->n_qubits, sp->n_orb, sp->n_alpha, sp->n_beta, sp->dim_beta, sp->n_chunks,
                       sp->rank_tab.get(), n, bits, idx);
    PBS_HIP(hipGetLastError());
  });
}

pbs_status pbs_space_unrank(const pbs_space* sp, uint64_t n, const int64_t* idx, uint64_t* bits, void* stream) {
  return guarded([&] {
    check_space(sp);
    if (n == 0) return;
    PBS_REQUIRE(bits && idx, PBS_ERR_ARG, "null array");
    hipLaunchKernelGGL(k_space_unrank, dim3(grid_for(n, 256, 65536)), dim3(256), 0, as_stream(stream), sp->sector,
                       sp->n_orb, sp->dim, sp->dim_beta, sp->str_alpha.get(), sp->str_beta.get(), n, idx, bits);
    PBS_HIP(hipGetLastError());
  });
}

void pbs_space_destroy(pbs_space* sp) { delete sp; }

}  // extern "C"
