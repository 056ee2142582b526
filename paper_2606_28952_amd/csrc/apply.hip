// Operator-state product H|psi> (Section 2.4, Eq. reverse_sum; in spin
// sectors Eq. sreverse_sum) and the fused energy of Eq. vqe_energy: the
// full-space kernel, launch planning of the sector kernels (whose device code
// lives in sector.h), and the C ABI entry points, single and batched.
#include <mutex>

#include "sector.h"

namespace pbs {
namespace {

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
      if (out) Amp<T>::store(out, t, acc_r, acc_i);
    } else {
      Amp<T>::store(out, t, acc_r, acc_i);
    }
  }
  if (EXPVAL) block_reduce3_store<kBlock>(e_re, e_im, nrm, partial + 3ull * blockIdx.x);
}


// Per-job sums of workgroup partials (one workgroup per job, fixed order).
__global__ __launch_bounds__(kBlock) void k_batch_finish(const BatchJob* jobs, uint32_t n_jobs, uint32_t total_blocks,
                                                         const double* partial, double* result) {
  const uint32_t j = blockIdx.x;
  const uint32_t b0 = jobs[j].block_base;
  const uint32_t b1 = j + 1 < n_jobs ? jobs[j + 1].block_base : total_blocks;
  double a = 0, b = 0, c = 0;
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
    a += partial[3ull * i];
    b += partial[3ull * i + 1];
    c += partial[3ull * i + 2];
  }
  block_reduce3_store<kBlock>(a, b, c, result + 3ull * jobs[j].slot);
}

// Sums per-workgroup partials in a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_expval_finish(const double* partial, uint64_t nparts, double* result) {
  double a = 0, b = 0, c = 0;
  for (uint64_t i = threadIdx.x; i < nparts; i += kBlock) {
    a += partial[3 * i];
    b += partial[3 * i + 1];
    c += partial[3 * i + 2];
  }
  block_reduce3_store<kBlock>(a, b, c, result);
}

// ---------------------------------------------------------------- launch planning
struct Launch {
  uint32_t chunks = 0;  // beta-column chunks per row
  dim3 grid;
  dim3 block;
  uint64_t parts = 0;
  size_t lds = 0;
};

int device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  return v;
}

// Fills the sector kernel's arguments and LDS layout for this operator/space.
// LDS holds the rank tables (n_orb <= 16), the staged source row (or the
// simple-class row list), the folded uniques and the pair map.  The folded
// uniques get what is left of half the device's LDS, so that two workgroups
// share a compute unit, unless the fixed parts alone need more.
Launch plan_sector(const pbs_grouped& h, const pbs_space& sp, size_t elem_bytes, bool allow_row, bool realc,
                   SectorArgs* a_out, bool* r16, bool allow_enum = true, bool allow_qenum = true,
                   bool allow_fact = true) {
  SectorArgs a{};
  a.n_orb = sp.n_orb;
  a.n_alpha = sp.n_alpha;
  a.n_beta = sp.n_beta;
  a.n_chunks = sp.n_chunks;
  a.dim_beta = static_cast<uint32_t>(sp.dim_beta);
  a.n_class = h.n_class;
  a.n_pairs = h.n_pairs;
  a.n_moves = sp.n_beta * (sp.n_orb - sp.n_beta);
  a.str_a = sp.str_alpha.get();
  a.str_b = sp.str_beta.get();
  a.rank16 = sp.rank_tab16.get();
  a.rank32 = sp.rank_tab.get();
  a.meta = h.cls_meta.get();
  a.pmap = h.pmap.get();
  a.qmap = h.qmap.get();
  a.quad_cnt = h.quad_cnt;
  a.pair_sign = h.pair_sign ? 1u : 0u;
  a.zpair = h.zpair.get();
  a.n_runs = h.n_runs;
  a.n_ns = h.n_ns;
  a.runs = h.runs.get();
  a.ns_list = h.ns_list.get();
  a.pg_xb = h.pg_xb.get();
  a.pg_u0 = h.pg_u0.get();
  a.u_zb = h.u_zb.get();
  a.u_t0 = h.u_t0.get();
  a.pt_za = h.pt_za.get();
  a.pt_c = reinterpret_cast<const double2*>(h.pt_c.get());

  // spin-factorized evaluation when the operator carries tables for this
  // beta sector (real coefficients)
  const FactorPlan* F = h.fplan.get();
  const bool fact_ok = allow_fact && realc && F != nullptr && F->n_orb == sp.n_orb;
  const bool fact = fact_ok && (h.fact_on & (kFactZero | kFactMoves)) && F->n_beta == sp.n_beta &&
                    F->dim_beta == sp.dim_beta;
  const bool fact_a = fact_ok && (h.fact_on & kFactAlpha) && F->alist && F->n_alpha == sp.n_alpha;
  SectorLayoutIn in;
  in.lds_limit = static_cast<uint32_t>(device_lds_limit()) - 1024u;  // static shared arrays
  in.n_orb = sp.n_orb;
  in.n_beta = sp.n_beta;
  in.dim_beta = sp.dim_beta;
  in.elem_bytes = static_cast<uint32_t>(elem_bytes);
  in.realc = realc;
  in.allow_row = allow_row;
  in.allow_enum = allow_enum;
  in.allow_qenum = allow_qenum;
  in.n_pmap = h.n_pmap;
  in.n_qmap = h.n_qmap;
  in.n_pairs = h.n_pairs;
  in.n_quads = h.n_quads;
  in.max_quad_uniques = h.max_quad_uniques;
  in.a_region = fact || fact_a;
  SectorLayout Y;
  PBS_REQUIRE(sector_layout(in, &Y), PBS_ERR_RANGE, "too many orbital pairs for the pair map");
  *r16 = Y.r16;
  a.enum_ok = Y.enum_ok ? 1u : 0u;
  a.qenum_ok = Y.qenum_ok ? 1u : 0u;
  a.n_quads = h.n_quads;
  a.n_qmoves = Y.n_qmoves;
  a.row_lds = Y.row_lds ? 1u : 0u;
  a.list_cap = Y.list_cap;
  a.f_cap = Y.f_cap;
  a.off_rank = Y.off_rank;
  a.off_f = Y.off_f;
  a.off_fz = Y.off_fz;
  a.off_qu = Y.off_qu;
  a.off_a = Y.off_a;
  a.fact = fact ? (h.fact_on & kFactZero) : 0u;
  a.f_c0 = 0xffffffffu;
  if (fact_a) {
    a.alist_off = F->alist_off.get();
    a.alist_src = F->alist_src.get();
    a.alist_c = F->alist_c.get();
    // image classes need the cached single moves (with their beta parities)
    // and the X_beta = 0 rows of this beta sector
    if (F->plist && a.enum_ok && a.row_lds && h.pair_sign && F->n_beta == sp.n_beta && F->dim_beta == sp.dim_beta) {
      a.plist_off = F->plist_off.get();
      a.plist_src = F->plist_src.get();
      a.plist_cls = F->plist_cls.get();
      a.pimg = F->pimg.get();
      a.pimg_flag = F->pimg_flag.get();
      a.n_img = F->n_img;
      a.cls_f = F->cls_f.get();
      a.fz = F->fz.get();
    }
  }
  if (fact) {
    a.fu_t0 = F->fu_t0.get();
    a.ft_za = F->ft_za.get();
    a.ft_c = F->ft_c.get();
    a.cls_f = F->cls_f.get();
    a.fz = F->fz.get();
    a.f_tz = F->t_zero;
    // the X_alpha = 0 class through the move tables: needs room for its
    // folded factors
    if ((h.fact_on & kFactMoves) && a.row_lds && F->c0 != 0xffffffffu && F->n_moves == a.n_moves &&
        kFactZeroSlots + (F->c0_fu1 - F->c0_fu0) <= a.f_cap) {
      a.fact |= kFactMoves;
      a.f_c0 = F->c0;
      a.f_r2 = F->r2;
      a.f_r3 = F->r3;
      a.f_c0_fu0 = F->c0_fu0;
      a.f_c0_fq = F->c0_fq;
      a.f_c0_fu1 = F->c0_fu1;
      a.f_tp = F->t_pair;
      a.f_tq = F->t_quad;
      a.f_n_qmoves = F->n_qmoves;
      a.em = F->em.get();
      a.fp = F->fp.get();
      a.eq = F->eq.get();
      a.fq = F->fq.get();
    }
  }
  // classes that pass Q and the image pass evaluate leave the class list
  if (a.fact && a.f_c0 != 0xffffffffu) {
    const int k = a.plist_off ? 2 : 0;
    a.ns_list = F->ns_rest[k].get();
    a.n_ns = F->ns_sizes[k];
  } else if (a.plist_off) {
    a.ns_list = F->ns_rest[1].get();
    a.n_ns = F->ns_sizes[1];
  }
  *a_out = a;

  Launch L;
  const uint64_t chunks = (sp.dim_beta + kSB - 1) / kSB;
  L.grid = dim3(static_cast<unsigned>(sp.dim_alpha * chunks));
  L.chunks = static_cast<uint32_t>(chunks);
  L.block = dim3(kSB);
  L.parts = sp.dim_alpha * chunks;
  L.lds = Y.lds;
  return L;
}

constexpr unsigned kFullGridCap = 1u << 16;

// Fixed workspace of pbs_expval_noalloc (per-workgroup energy partials): one
// copy per device, alive until the process ends.  Host code never uses the
// array's name as an address; it uses the device address looked up once per
// device by noalloc_scratch().
static_assert(PBS_EXPVAL_NOALLOC_MAX_BYTES % 256 == 0, "workspace size");
static __device__ __align__(256) double scratch[PBS_EXPVAL_NOALLOC_MAX_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
double* noalloc_scratch() {
  int dev = 0;
  PBS_HIP(hipGetDevice(&dev));
  PBS_REQUIRE(dev >= 0 && dev < kMaxDevices, PBS_ERR_RANGE, "device ordinal beyond the fixed workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    PBS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PBS_REQUIRE(p != nullptr, PBS_ERR_DEVICE, "no device address for the fixed workspace");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

uint64_t partial_count(const pbs_space& sp) {
  if (!sp.sector) return grid_for(sp.dim, kBlock, kFullGridCap);
  return sp.dim_alpha * ((sp.dim_beta + kSB - 1) / kSB);
}

void validate(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt) {
  PBS_REQUIRE(h != nullptr && sp != nullptr, PBS_ERR_ARG, "null handle");
  PBS_REQUIRE(dt == PBS_C128 || dt == PBS_C64, PBS_ERR_ARG, "unknown dtype");
  PBS_REQUIRE(h->n_qubits == sp->n_qubits, PBS_ERR_ARG,
              "operator has " + std::to_string(h->n_qubits) + " qubits, space has " + std::to_string(sp->n_qubits));
  if (sp->sector) {
    PBS_REQUIRE(h->has_sector && h->half == sp->n_orb, PBS_ERR_ARG, "operator lacks sector tables for this split");
    PBS_REQUIRE(sp->dim_alpha * ((sp->dim_beta + kSB - 1) / kSB) < (1ull << 31), PBS_ERR_RANGE,
                "sector needs more than 2^31 workgroups");
  }
}

// Layout of the rows kernel when it applies (see k_apply_rows): factored
// alpha lists, rows not staged, every non-simple class in LDS.
bool plan_rows(const pbs_grouped& h, const SectorArgs& a, bool r16, bool expval, RowsLayout* Lr, size_t* lds) {
  const FactorPlan* F = h.fplan.get();
  if (!r16 || a.row_lds || a.alist_off == nullptr || F == nullptr || a.ns_list != h.ns_list.get()) return false;
  if (F->ns_uniques >= 65536u || F->ns_uniques + F->ns_groups == 0) return false;
  RowsLayout L{};
  uint32_t off = kMiscBytes;
  L.off_rank = off;
  off += align16(kRank16Lds * 2u);
  L.off_lsrc = off;
  off += align16(F->alist_max * 4u);
  L.off_lc = off;
  off += align16(F->alist_max * 8u);
  L.off_cls = off;
  off += align16(a.n_ns * 16u);
  L.off_grp = off;
  off += align16(F->ns_groups * 8u);
  L.off_f = off;
  off += align16(F->ns_uniques * 8u);
  L.off_fz = off;
  off += align16(F->ns_uniques * 4u);
  L.off_e = off;  // per-thread energy sums (the fused energy pass only)
  if (expval) off += 3u * kSB * 8u;
  if (off > 60u * 1024u) return false;
  *Lr = L;
  *lds = off;
  return true;
}

// Launches the apply (EXPVAL: with the energy partials) for target alpha
// rows [row_begin, row_end) of a sector space (the whole space by default);
// out holds those rows only, from row_begin's first column.  Returns the
// number of energy partials written.
template <class T, bool EXPVAL>
uint64_t launch(const pbs_grouped& h, const pbs_space& sp, const void* psi, void* out, double* partial,
                hipStream_t s, uint64_t row_begin = 0, uint64_t row_end = ~0ull) {
  const T* p = static_cast<const T*>(psi);
  T* o = static_cast<T*>(out);
  if (!sp.sector) {
    const dim3 grid(grid_for(sp.dim, kBlock, kFullGridCap));
    hipLaunchKernelGGL((k_apply_full<T, EXPVAL>), grid, dim3(kBlock), 0, s, sp.dim,
                       static_cast<uint32_t>(h.n_groups), h.xg.get(), h.off.get(), h.zk.get(),
                       reinterpret_cast<const double2*>(h.ck.get()), p, o, partial);
  } else {
    SectorArgs a;
    bool r16 = false;
    const Launch L = plan_sector(h, sp, sizeof(T), true, h.real_coef, &a, &r16);
    const pbs_dtype dt = sizeof(T) == 16 ? PBS_C128 : PBS_C64;
    row_end = std::min<uint64_t>(row_end, sp.dim_alpha);
    const uint64_t rows = row_end - row_begin;
    if (rows == 0) return 0;
    a.row_begin = static_cast<uint32_t>(row_begin);
    // the kernels store target t = row * dim_beta + column at out[t]: shift
    // the base so that row_begin's first column lands at out[0]
    if (o) o = reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(o) - row_begin * sp.dim_beta * sizeof(T));
    RowsLayout Lr;
    size_t lds_rows = 0;
    if (h.real_coef && plan_rows(h, a, r16, EXPVAL, &Lr, &lds_rows)) {
      // one workgroup per alpha row, sweeping all of its columns
      hipLaunchKernelGGL((k_apply_rows<T, EXPVAL>), dim3(static_cast<unsigned>(rows)), dim3(kSB), lds_rows, s, a, Lr,
                         p, o, partial);
      PBS_HIP(hipGetLastError());
      return rows;
    }
    void* kern = sector_kernel(dt, EXPVAL, false, r16, a.row_lds != 0, h.real_coef);
    if (L.lds > 64 * 1024)
      PBS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(L.lds)));
    void* args[] = {&a, &p, &o, &partial};
    const uint64_t parts = rows * L.chunks;
    PBS_HIP(hipLaunchKernel(kern, dim3(static_cast<unsigned>(parts)), L.block, args, L.lds, s));
    PBS_HIP(hipGetLastError());
    return parts;
  }
  PBS_HIP(hipGetLastError());
  return partial_count(sp);
}

}  // namespace

void apply_launch(const pbs_grouped& h, const pbs_space& sp, pbs_dtype dt, const void* psi, void* out,
                  hipStream_t s) {
  validate(&h, &sp, dt);
  if (dt == PBS_C128)
    launch<double2, false>(h, sp, psi, out, nullptr, s);
  else
    launch<float2, false>(h, sp, psi, out, nullptr, s);
}

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
    *bytes = partial_count(*sp) * 3 * sizeof(double);
  });
}

pbs_status pbs_expval(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                      double* result, void* work, uint64_t work_bytes, void* stream) {
  return guarded([&] {
    validate(h, sp, dt);
    PBS_REQUIRE(psi != nullptr && result != nullptr && work != nullptr, PBS_ERR_ARG, "null pointer");
    if (out) {
      const uint64_t bytes = sp->dim * (dt == PBS_C128 ? 16ull : 8ull);
      const auto a = reinterpret_cast<uintptr_t>(psi), b = reinterpret_cast<uintptr_t>(out);
      PBS_REQUIRE(a + bytes <= b || b + bytes <= a, PBS_ERR_ARG, "out overlaps psi");
    }
    const uint64_t need = partial_count(*sp) * 3 * sizeof(double);
    PBS_REQUIRE(work_bytes >= need, PBS_ERR_ARG,
                "workspace of " + std::to_string(work_bytes) + " bytes, need " + std::to_string(need));
    hipStream_t s = as_stream(stream);
    double* partial = static_cast<double*>(work);
    const uint64_t parts = dt == PBS_C128 ? launch<double2, true>(*h, *sp, psi, out, partial, s)
                                          : launch<float2, true>(*h, *sp, psi, out, partial, s);
    hipLaunchKernelGGL(k_expval_finish, dim3(1), dim3(kBlock), 0, s, partial, parts, result);
    PBS_HIP(hipGetLastError());
  });
}

}  // extern "C"

namespace {
// Checks of a target-row range call: a sector space, rows within it, and an
// output shard of (row_end - row_begin) rows that does not overlap psi.
void check_rows(const pbs_space* sp, pbs_dtype dt, const void* psi, const void* out, uint64_t row_begin,
                uint64_t row_end) {
  PBS_REQUIRE(sp->sector, PBS_ERR_ARG, "a row range needs a spin-sector space");
  PBS_REQUIRE(row_begin <= row_end && row_end <= sp->dim_alpha, PBS_ERR_RANGE,
              "rows [" + std::to_string(row_begin) + ", " + std::to_string(row_end) + ") outside the sector's " +
                  std::to_string(sp->dim_alpha) + " alpha rows");
  PBS_REQUIRE(psi != nullptr, PBS_ERR_ARG, "null state pointer");
  if (out) {
    const uint64_t elem = dt == PBS_C128 ? 16ull : 8ull;
    const auto a = reinterpret_cast<uintptr_t>(psi), b = reinterpret_cast<uintptr_t>(out);
    const uint64_t in_bytes = sp->dim * elem, out_bytes = (row_end - row_begin) * sp->dim_beta * elem;
    PBS_REQUIRE(a + in_bytes <= b || b + out_bytes <= a, PBS_ERR_ARG, "out overlaps psi");
  }
}
}  // namespace

extern "C" {

pbs_status pbs_apply_pauli_sum_rows(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi,
                                    void* out, uint64_t row_begin, uint64_t row_end, void* stream) {
  return guarded([&] {
    validate(h, sp, dt);
    check_rows(sp, dt, psi, out, row_begin, row_end);
    PBS_REQUIRE(out != nullptr || row_begin == row_end, PBS_ERR_ARG, "null output pointer");
    hipStream_t s = as_stream(stream);
    if (dt == PBS_C128)
      launch<double2, false>(*h, *sp, psi, out, nullptr, s, row_begin, row_end);
    else
      launch<float2, false>(*h, *sp, psi, out, nullptr, s, row_begin, row_end);
  });
}

pbs_status pbs_expval_rows(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                           uint64_t row_begin, uint64_t row_end, double* result, void* work, uint64_t work_bytes,
                           void* stream) {
  return guarded([&] {
    validate(h, sp, dt);
    PBS_REQUIRE(result != nullptr && work != nullptr, PBS_ERR_ARG, "null pointer");
    check_rows(sp, dt, psi, out, row_begin, row_end);
    // at most one partial per (row, column chunk) of the share
    const uint64_t need = (row_end - row_begin) * ((sp->dim_beta + kSB - 1) / kSB) * 3 * sizeof(double);
    PBS_REQUIRE(work_bytes >= need, PBS_ERR_ARG,
                "workspace of " + std::to_string(work_bytes) + " bytes, need " + std::to_string(need));
    hipStream_t s = as_stream(stream);
    double* partial = static_cast<double*>(work);
    const uint64_t parts = dt == PBS_C128 ? launch<double2, true>(*h, *sp, psi, out, partial, s, row_begin, row_end)
                                          : launch<float2, true>(*h, *sp, psi, out, partial, s, row_begin, row_end);
    hipLaunchKernelGGL(k_expval_finish, dim3(1), dim3(kBlock), 0, s, partial, parts, result);
    PBS_HIP(hipGetLastError());
  });
}

pbs_status pbs_expval_noalloc(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                              double* result, void* stream) {
  return guarded([&] {
    validate(h, sp, dt);
    PBS_REQUIRE(psi != nullptr && result != nullptr, PBS_ERR_ARG, "null pointer");
    if (out) {
      const uint64_t bytes = sp->dim * (dt == PBS_C128 ? 16ull : 8ull);
      const auto a = reinterpret_cast<uintptr_t>(psi), b = reinterpret_cast<uintptr_t>(out);
      PBS_REQUIRE(a + bytes <= b || b + bytes <= a, PBS_ERR_ARG, "out overlaps psi");
    }
    const uint64_t need = partial_count(*sp) * 3 * sizeof(double);
    PBS_REQUIRE(need <= PBS_EXPVAL_NOALLOC_MAX_BYTES, PBS_ERR_RANGE,
                "space needs " + std::to_string(need) + " bytes of energy partials, the fixed workspace holds " +
                    std::to_string(static_cast<uint64_t>(PBS_EXPVAL_NOALLOC_MAX_BYTES)));
    double* partial = noalloc_scratch();
    hipStream_t s = as_stream(stream);
    const uint64_t parts = dt == PBS_C128 ? launch<double2, true>(*h, *sp, psi, out, partial, s)
                                          : launch<float2, true>(*h, *sp, psi, out, partial, s);
    hipLaunchKernelGGL(k_expval_finish, dim3(1), dim3(kBlock), 0, s, partial, parts, result);
    PBS_HIP(hipGetLastError());
  });
}

}  // extern "C"

struct pbs_batch {
  uint32_t n_jobs = 0;
  uint32_t total_blocks = 0;  // work items (alpha row, column chunk) over all jobs
  uint32_t grid = 0;          // workgroups launched (fewer than the items when persistent)
  pbs_dtype dt = PBS_C64;
  bool r16 = false, row_lds = false, realc = false;
  size_t lds = 0;
  uint32_t config = 0;     // schedule in use (PBS_BATCH_* bits)
  double tuned_ms = -1.0;  // time of that schedule when chosen by pbs_batch_tune
  std::vector<const pbs_grouped*> h;
  std::vector<const pbs_space*> sp;
  std::vector<const void*> psi;
  std::vector<void*> out;
  pbs::DevBuf<pbs::BatchJob> jobs;
  pbs::DevBuf<double> partial;
};

namespace pbs {
namespace {

constexpr uint32_t kBatchConfigs = 256;  // six PBS_BATCH_* flags and the 2-bit workgroup order

// Builds and uploads the job table of batch B for schedule `config`:
// PBS_BATCH_GIVEN_ORDER keeps the caller's job order (else largest first),
// PBS_BATCH_NO_ROW_STAGING gathers source rows from HBM/L2 instead of staging
// them in LDS, PBS_BATCH_NO_DOUBLE_MOVES scans double-flip groups instead of
// enumerating each target's double moves, PBS_BATCH_NO_SINGLE_MOVES scans
// pair groups instead of enumerating single moves, and the order field
// (PBS_BATCH_ORDER_*) maps a job's workgroups to (row, chunk): by default as
// a single launch does (rows fastest when rows are staged, else a row's
// chunks kept on one XCD), or forced plain row-major, rows fastest or
// XCD-grouped.  Synchronizes (plain copy).
void fill_batch(pbs_batch& B, uint32_t config) {
  const uint32_t n = B.n_jobs;
  const size_t esz = B.dt == PBS_C128 ? 16 : 8;
  const bool given = config & PBS_BATCH_GIVEN_ORDER, allow_row = !(config & PBS_BATCH_NO_ROW_STAGING);
  const bool qenum = !(config & PBS_BATCH_NO_DOUBLE_MOVES), penum = !(config & PBS_BATCH_NO_SINGLE_MOVES);
  const bool factd = !(config & PBS_BATCH_NO_FACTORED);
  std::vector<BatchJob> jobs(n);
  std::vector<double> cost(n);
  std::vector<uint64_t> items(n);
  // one launch shares one kernel variant: rows staged only if every job's
  // row fits, LDS rank tables only if every job has n_orb <= 16
  bool r16 = true, rowlds = allow_row, realc = true;
  for (uint32_t i = 0; i < n; ++i) realc = realc && B.h[i]->real_coef;
  for (uint32_t i = 0; i < n; ++i) {
    bool job_r16 = false;
    plan_sector(*B.h[i], *B.sp[i], esz, allow_row, realc, &jobs[i].args, &job_r16, penum, qenum, factd);
    r16 = r16 && job_r16;
    rowlds = rowlds && jobs[i].args.row_lds;
  }
  size_t lds = 0;
  for (uint32_t i = 0; i < n; ++i) {
    bool job_r16 = false;
    const Launch L =
        plan_sector(*B.h[i], *B.sp[i], esz, rowlds, realc, &jobs[i].args, &job_r16, penum, qenum, factd);
    if (!r16) jobs[i].args.rank16 = nullptr;
    jobs[i].psi = B.psi[i];
    jobs[i].out = B.out[i];
    jobs[i].chunks = L.chunks;
    jobs[i].block_base = 0;
    jobs[i].slot = i;  // original position (energies are written there)
    jobs[i].rows = static_cast<uint32_t>(B.sp[i]->dim_alpha);
    jobs[i].pad = 0;
    lds = std::max(lds, L.lds);
    cost[i] = static_cast<double>(B.sp[i]->dim) * static_cast<double>(B.h[i]->n_pterm + 1);
    items[i] = static_cast<uint64_t>(B.sp[i]->dim_alpha) * L.chunks;
  }
  // largest jobs first, so the launch does not end on a long straggler
  const BatchPlan plan = batch_plan(cost, items, given);
  const uint32_t order_field = config & PBS_BATCH_ORDER_MASK;
  const uint32_t grid_order = order_field == PBS_BATCH_ORDER_PLAIN     ? kOrderPlain
                              : order_field == PBS_BATCH_ORDER_ROW_FAST ? kOrderRowFast
                              : order_field == PBS_BATCH_ORDER_XCD_ROWS ? kOrderXcdRows
                              : (rowlds ? kOrderRowFast : kOrderXcdRows);
  for (uint32_t i = 0; i < n; ++i) jobs[i].order = grid_order;
  PBS_REQUIRE(plan.total < (1ull << 31), PBS_ERR_RANGE, "batch needs more than 2^31 workgroups");
  std::vector<BatchJob> sorted(n);
  for (uint32_t k = 0; k < n; ++k) {
    sorted[k] = jobs[plan.order[k]];
    sorted[k].block_base = static_cast<uint32_t>(plan.base[k]);
  }
  const uint64_t base = plan.total;
  if (lds > 64 * 1024) {
    for (bool ev : {false, true})
      PBS_HIP(hipFuncSetAttribute(sector_kernel(B.dt, ev, true, r16, rowlds, realc),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  }
  if (B.partial.n < 3ull * base) B.partial.alloc(3ull * base);
  if (B.jobs.n < n) B.jobs.alloc(n);
  PBS_HIP(hipMemcpy(B.jobs.get(), sorted.data(), n * sizeof(BatchJob), hipMemcpyHostToDevice));
  B.total_blocks = static_cast<uint32_t>(base);
  B.r16 = r16;
  B.row_lds = rowlds;
  B.realc = realc;
  B.lds = lds;
  B.grid = B.total_blocks;
  if (config & PBS_BATCH_PERSISTENT) {
    // as many workgroups as are resident at once (both kernel forms share
    // their resources); each walks the item list with a fixed stride
    int dev = 0, cus = 0, per_cu = 0;
    PBS_HIP(hipGetDevice(&dev));
    PBS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PBS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sector_kernel(B.dt, false, true, r16, rowlds, realc),
                                                         kSB, lds));
    const uint64_t resident = static_cast<uint64_t>(std::max(cus, 1)) * static_cast<uint64_t>(std::max(per_cu, 1));
    B.grid = static_cast<uint32_t>(std::min<uint64_t>(B.total_blocks, resident));
  }
  B.config = config;
}

void launch_batch(const pbs_batch& b, double* energies, hipStream_t s) {
  const bool ev = energies != nullptr;
  void* kern = sector_kernel(b.dt, ev, true, b.r16, b.row_lds, b.realc);
  const BatchJob* jobs = b.jobs.get();
  uint32_t n = b.n_jobs, items = b.total_blocks;
  double* partial = b.partial.get();
  void* args[] = {&jobs, &n, &items, &partial};
  PBS_HIP(hipLaunchKernel(kern, dim3(b.grid), dim3(kSB), args, b.lds, s));
  if (ev) {
    hipLaunchKernelGGL(k_batch_finish, dim3(n), dim3(kBlock), 0, s, jobs, n, b.total_blocks, partial, energies);
    PBS_HIP(hipGetLastError());
  }
}

}  // namespace
}  // namespace pbs

extern "C" {

pbs_status pbs_batch_create(uint32_t n, const pbs_grouped* const* h, const pbs_space* const* sp, pbs_dtype dt,
                            const void* const* psi, void* const* out, pbs_batch** batch) {
  return guarded([&] {
    PBS_REQUIRE(batch != nullptr, PBS_ERR_ARG, "null output handle");
    *batch = nullptr;
    PBS_REQUIRE(n >= 1 && h && sp && psi && out, PBS_ERR_ARG, "empty batch or null array");
    const size_t esz = dt == PBS_C128 ? 16 : 8;
    for (uint32_t i = 0; i < n; ++i) {
      validate(h[i], sp[i], dt);
      PBS_REQUIRE(sp[i]->sector, PBS_ERR_UNSUPPORTED, "batched apply runs on spin-sector spaces");
      PBS_REQUIRE(psi[i] && out[i], PBS_ERR_ARG, "null state pointer in job " + std::to_string(i));
      const uint64_t bytes = sp[i]->dim * esz;
      const auto a = reinterpret_cast<uintptr_t>(psi[i]), b = reinterpret_cast<uintptr_t>(out[i]);
      PBS_REQUIRE(a + bytes <= b || b + bytes <= a, PBS_ERR_ARG, "out overlaps psi in job " + std::to_string(i));
    }
    for (uint32_t i = 0; i < n; ++i) {  // outputs of different jobs must not overlap
      const uint64_t bi = sp[i]->dim * esz;
      for (uint32_t j = i + 1; j < n; ++j) {
        const uint64_t bj = sp[j]->dim * esz;
        const auto x = reinterpret_cast<uintptr_t>(out[i]), y = reinterpret_cast<uintptr_t>(out[j]);
        PBS_REQUIRE(x + bi <= y || y + bj <= x, PBS_ERR_ARG, "outputs of jobs overlap");
      }
    }
    auto* B = new pbs_batch();
    try {
      B->n_jobs = n;
      B->dt = dt;
      B->h.assign(h, h + n);
      B->sp.assign(sp, sp + n);
      B->psi.assign(psi, psi + n);
      B->out.assign(out, out + n);
      fill_batch(*B, 0u);
    } catch (...) {
      delete B;
      throw;
    }
    *batch = B;
  });
}

pbs_status pbs_batch_set_config(pbs_batch* b, uint32_t config) {
  return guarded([&] {
    PBS_REQUIRE(b != nullptr, PBS_ERR_ARG, "null pbs_batch");
    PBS_REQUIRE(config < kBatchConfigs, PBS_ERR_ARG, "unknown schedule bits");
    fill_batch(*b, config);
    b->tuned_ms = -1.0;
  });
}

pbs_status pbs_batch_tune(pbs_batch* b, uint32_t reps, void* stream, uint32_t* config, double* ms) {
  return guarded([&] {
    PBS_REQUIRE(b != nullptr, PBS_ERR_ARG, "null pbs_batch");
    PBS_REQUIRE(reps >= 1 && reps <= 100, PBS_ERR_RANGE, "reps must be in 1..100");
    hipStream_t s = as_stream(stream);
    hipEvent_t e0, e1;
    PBS_HIP(hipEventCreate(&e0));
    PBS_HIP(hipEventCreate(&e1));
    std::vector<std::pair<std::string, double>> seen;  // job table + variant -> time
    // time of schedule c (schedules with the same table and variant share one measurement)
    auto time_config = [&](uint32_t c) {
      fill_batch(*b, c);
      std::string key(1, static_cast<char>(b->row_lds));
      std::vector<BatchJob> table(b->n_jobs);
      PBS_HIP(hipMemcpy(table.data(), b->jobs.get(), b->n_jobs * sizeof(BatchJob), hipMemcpyDeviceToHost));
      key.append(reinterpret_cast<const char*>(table.data()), table.size() * sizeof(BatchJob));
      for (const auto& e : seen)
        if (e.first == key) return e.second;
      launch_batch(*b, nullptr, s);  // warm-up
      PBS_HIP(hipEventRecord(e0, s));
      for (uint32_t r = 0; r < reps; ++r) launch_batch(*b, nullptr, s);
      PBS_HIP(hipEventRecord(e1, s));
      PBS_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      PBS_HIP(hipEventElapsedTime(&t, e0, e1));
      const double per = static_cast<double>(t) / reps;
      seen.emplace_back(std::move(key), per);
      return per;
    };
    uint32_t best = 0;
    double best_ms = 0.0;
    try {
      // greedy: the workgroup order first (default flags), then the four
      // flags with that order
      best_ms = time_config(0);
      for (uint32_t o = 1; o < 4; ++o) {
        const uint32_t c = o << 4;
        const double t = time_config(c);
        if (t < best_ms) {
          best = c;
          best_ms = t;
        }
      }
      const uint32_t ord = best & PBS_BATCH_ORDER_MASK;
      for (uint32_t f = 1; f < kBatchConfigs; ++f) {
        if (f & PBS_BATCH_ORDER_MASK) continue;
        const double t = time_config(ord | f);
        if (t < best_ms) {
          best = ord | f;
          best_ms = t;
        }
      }
      fill_batch(*b, best);
      b->tuned_ms = best_ms;
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    PBS_HIP(hipEventDestroy(e0));
    PBS_HIP(hipEventDestroy(e1));
    if (config) *config = best;
    if (ms) *ms = best_ms;
  });
}

pbs_status pbs_batch_info(const pbs_batch* b, uint32_t* config, double* tuned_ms, uint32_t* workgroups) {
  return guarded([&] {
    PBS_REQUIRE(b != nullptr, PBS_ERR_ARG, "null pbs_batch");
    if (config) *config = b->config;
    if (tuned_ms) *tuned_ms = b->tuned_ms;
    if (workgroups) *workgroups = b->total_blocks;
  });
}

pbs_status pbs_batch_run(const pbs_batch* b, double* energies, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(b != nullptr, PBS_ERR_ARG, "null pbs_batch");
    launch_batch(*b, energies, as_stream(stream));
  });
}

void pbs_batch_destroy(pbs_batch* b) { delete b; }

}  // extern "C"
