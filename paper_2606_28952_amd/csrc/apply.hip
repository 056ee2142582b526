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
// row of the alpha-major state) and kSB consecutive beta columns, one target
// per lane.  Groups are visited class by class (a class shares X_alpha), so
// the source row s_a = t_a ^ X_alpha, its validity and its rank are uniform
// across the workgroup, and so are the alpha parities of every term: the
// coefficients of each unique beta Z-mask are folded over their terms' alpha
// parities cooperatively into LDS once per class.  Per class:
//  * the group with X_beta = 0 gathers from the lane's own column;
//  * groups whose X_beta flips two orbitals are visited by enumerating the
//    lane's valid pair moves (occupied -> empty, the same count for every
//    target of a sector), cached in registers with their source ranks, and a
//    per-class pair map; invalid moves are never visited;
//  * other groups are scanned with a per-lane validity test;
//  * consecutive classes holding only an X_beta = 0 group share one fold;
//  * the source row is staged in LDS as float64 when it fits.
// Parities are evaluated against the target strings each lane holds; the
// constant (-1)^popcount(z & X) factors were moved into the coefficients
// when the tables were built.
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

// Read-only load through the constant address space: uniform addresses
// become scalar loads (the tables are never written by the kernels).
__device__ inline uint32_t ldc(const uint32_t* p) { return *((const __attribute__((address_space(4))) uint32_t*)(p)); }

__device__ inline ClassMeta ld_meta(const ClassMeta* p) {
  static_assert(sizeof(ClassMeta) == 12 * sizeof(uint32_t), "ClassMeta layout");
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
  uint32_t w[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) w[i] = ldc(q + i);
  ClassMeta m;
  memcpy(&m, w, sizeof(m));
  return m;
}

template <int B>
__device__ inline void block_reduce3_store(double a, double b, double c, double* dst) {
  __shared__ double red[3][B / 64];
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
    for (int w = 0; w < B / 64; ++w) {
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
      if (out) Amp<T>::store(out, t, acc_r, acc_i);
    } else {
      Amp<T>::store(out, t, acc_r, acc_i);
    }
  }
  if (EXPVAL) block_reduce3_store<kBlock>(e_re, e_im, nrm, partial + 3ull * blockIdx.x);
}

// ---------------------------------------------------------------- spin sector
constexpr int kSB = 512;              // lanes per sector workgroup = beta columns per workgroup
constexpr int kMaxMoves = 56;         // pair moves cached per lane (N_beta (n_orb - N_beta) <= 56)
constexpr uint32_t kFCap = 1536;      // folded uniques held in LDS at once (+1 zero slot)
constexpr uint32_t kRowCapBytes = 64u * 1024u;
constexpr uint32_t kListMinBytes = 4096u;  // simple-class row list when no row is staged

struct SectorArgs {
  uint32_t n_orb, n_alpha, n_beta, n_chunks;
  uint32_t dim_beta;
  uint32_t n_class, n_pairs, n_moves;
  uint32_t row_lds, enum_ok;
  uint32_t list_cap;  // entries of the simple-class row list (in the row space)
  uint32_t off_rank, off_row, off_f, off_fz, off_pu;  // LDS byte offsets
  const uint32_t* str_a;
  const uint32_t* str_b;
  const uint16_t* rank16;  // n_orb <= 16
  const uint32_t* rank32;
  const ClassMeta* meta;
  const int32_t* pmap;
  const uint32_t* pg_xb;
  const uint32_t* pg_u0;
  const uint32_t* u_zb;
  const uint32_t* u_t0;
  const uint32_t* pt_za;
  const double2* pt_c;
};

// Combinatorial rank of a spin string: uint16 tables in LDS (n_orb <= 16,
// at most two byte chunks) or uint32 tables in global memory.
template <bool R16>
__device__ inline uint32_t rank_of(uint32_t s, const SectorArgs& P, const uint16_t* t16) {
  if (R16) {
    const uint32_t lo = s & 255u;
    uint32_t r = t16[lo];
    if (P.n_chunks > 1) r += t16[((P.n_orb + 1) + __popc(lo)) * 256 + ((s >> 8) & 255u)];
    return r;
  }
  uint32_t r = 0, below = 0;
  for (uint32_t c = 0; c < P.n_chunks; ++c) {
    const uint32_t byte = (s >> (8 * c)) & 255u;
    r += P.rank32[(c * (P.n_orb + 1) + below) * 256 + byte];
    below += __popc(byte);
  }
  return r;
}

// F[u - ua] = sum over the unique's terms of C_t (-1)^popcount(za_t & ta).
__device__ inline void fold_uniques(const SectorArgs& P, uint32_t ua, uint32_t ub, uint32_t ta, double2* F,
                                    uint32_t* Fz) {
  for (uint32_t u = ua + threadIdx.x; u < ub; u += kSB) {
    double fr = 0.0, fi = 0.0;
    const uint32_t t1 = P.u_t0[u + 1];
    for (uint32_t t = P.u_t0[u]; t < t1; ++t) {
      const uint32_t par = __popc(P.pt_za[t] & ta);
      const double2 c = P.pt_c[t];
      fr += signed_by(c.x, par);
      fi += signed_by(c.y, par);
    }
    F[u - ua] = make_double2(fr, fi);
    Fz[u - ua] = P.u_zb[u];
  }
}

__device__ inline void phase_sum_lds(const double2* F, const uint32_t* Fz, uint32_t b, uint32_t cnt, uint32_t tb,
                                     double& fr, double& fi) {
  for (uint32_t i = 0; i < cnt; ++i) {
    const uint32_t par = __popc(Fz[b + i] & tb);
    const double2 f = F[b + i];
    fr += signed_by(f.x, par);
    fi += signed_by(f.y, par);
  }
}

// Phase sum of group g straight from the term tables (groups too large for LDS).
__device__ inline void phase_sum_direct(const SectorArgs& P, uint32_t g, uint32_t ta, uint32_t tb, double& fr,
                                        double& fi) {
  const uint32_t u1 = P.pg_u0[g + 1];
  for (uint32_t u = P.pg_u0[g]; u < u1; ++u) {
    double gr = 0.0, gi = 0.0;
    const uint32_t t1 = P.u_t0[u + 1];
    for (uint32_t t = P.u_t0[u]; t < t1; ++t) {
      const uint32_t par = __popc(P.pt_za[t] & ta);
      const double2 c = P.pt_c[t];
      gr += signed_by(c.x, par);
      gi += signed_by(c.y, par);
    }
    const uint32_t par = __popc(P.u_zb[u] & tb);
    fr += signed_by(gr, par);
    fi += signed_by(gi, par);
  }
}

__device__ inline void cmul_acc(double fr, double fi, double ar, double ai, double& acc_r, double& acc_i) {
  acc_r = fma(ar, fr, fma(-ai, fi, acc_r));
  acc_i = fma(ar, fi, fma(ai, fr, acc_i));
}

template <class T>
__device__ inline void ld_amp(const T* p, uint64_t i, double& r, double& m) {
  Amp<T>::load(p, i, r, m);
}

// One group of a scanned chunk: validity of X_beta for this lane's target,
// source column rank, phase sum from the folded uniques; invalid targets are
// predicated off (column 0 is read, the coefficient is zeroed).
template <bool R16, class T>
__device__ __forceinline__ void scan_group(const SectorArgs& P, uint32_t g, uint32_t us, uint32_t tb,
                                           const uint16_t* s_rank, const double2* s_F, const uint32_t* s_Fz,
                                           const T* rowp, double& acc_r, double& acc_i) {
  const uint32_t xb = ldc(P.pg_xb + g);
  const uint32_t u0 = ldc(P.pg_u0 + g), u1 = ldc(P.pg_u0 + g + 1);
  const bool valid = 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
  const uint32_t jb = valid ? rank_of<R16>(tb ^ xb, P, s_rank) : 0u;
  double fr = 0.0, fi = 0.0;
  phase_sum_lds(s_F, s_Fz, u0 - us, u1 - u0, tb, fr, fi);
  double a_r, a_i;
  ld_amp<T>(rowp, jb, a_r, a_i);
  if (!valid) fr = fi = 0.0;
  cmul_acc(fr, fi, a_r, a_i, acc_r, acc_i);
}

// Lists, in class order, the simple classes c0 .. c1-1 whose source alpha
// string ta ^ X_alpha lies in the sector: entry = (source row rank, first
// folded unique relative to ua | unique count << 16).  The list is padded to
// a multiple of four with entries that read row 0 against the zero slot.
// Returns the padded length; ends with the list visible to the workgroup.
template <bool R16>
__device__ uint32_t list_valid_rows(const SectorArgs& P, uint32_t c0, uint32_t c1, uint32_t ua, uint32_t ta,
                                    const uint16_t* s_rank, uint2* s_list, uint32_t* s_wcnt) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t base = 0;
  for (uint32_t i0 = c0; i0 < c1; i0 += kSB) {
    const uint32_t cc = i0 + threadIdx.x;
    bool v = false;
    uint2 entry = make_uint2(0u, 0u);
    if (cc < c1) {
      const ClassMeta* m = P.meta + cc;
      const uint32_t sa = ta ^ m->xa;
      v = static_cast<uint32_t>(__popc(sa)) == P.n_alpha;
      if (v) entry = make_uint2(rank_of<R16>(sa, P, s_rank), (m->ua - ua) | ((m->u_end - m->ua) << 16));
    }
    const uint64_t bal = __ballot(v);
    if (lane == 0) s_wcnt[wave] = static_cast<uint32_t>(__popcll(bal));
    __syncthreads();
    uint32_t off = base, total = 0;
    for (uint32_t w = 0; w < kSB / 64; ++w) {
      const uint32_t n = s_wcnt[w];
      off += w < wave ? n : 0u;
      total += n;
    }
    if (v) s_list[off + static_cast<uint32_t>(__popcll(bal & below))] = entry;
    base += total;
    __syncthreads();
  }
  const uint32_t padded = (base + 3u) & ~3u;
  if (threadIdx.x < padded - base) s_list[base + threadIdx.x] = make_uint2(0u, kFCap | (1u << 16));
  __syncthreads();
  return padded;
}

// One workgroup: target alpha string ia (one row of the state), beta columns
// chunk*kSB .. chunk*kSB + kSB - 1, one target per lane.  See the file header
// for the scheme.  `slot` receives the workgroup's energy partials.
template <class T, bool EXPVAL, bool R16, bool ROWLDS>
__device__ __forceinline__ void sector_body(const SectorArgs& P, const T* __restrict__ psi, T* __restrict__ out,
                                            double* __restrict__ slot, uint64_t ia, uint32_t chunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* s_rank = reinterpret_cast<uint16_t*>(smem + P.off_rank);
  T* s_row = reinterpret_cast<T*>(smem + P.off_row);
  double2* s_F = reinterpret_cast<double2*>(smem + P.off_f);
  uint32_t* s_Fz = reinterpret_cast<uint32_t*>(smem + P.off_fz);
  uint32_t* s_pu = reinterpret_cast<uint32_t*>(smem + P.off_pu);
  uint2* s_list = reinterpret_cast<uint2*>(smem + P.off_row);  // shares the staged row's space
  __shared__ uint32_t s_wcnt[kSB / 64];

  if (R16) {
    const uint32_t n = P.n_chunks * (P.n_orb + 1) * 256;
    for (uint32_t i = threadIdx.x; i < n; i += kSB) s_rank[i] = P.rank16[i];
  }
  if (threadIdx.x == 0) {  // zero slot for absent pair groups
    s_F[kFCap] = make_double2(0.0, 0.0);
    s_Fz[kFCap] = 0u;
  }
  __syncthreads();

  const uint32_t db = P.dim_beta;
  const uint32_t col = chunk * kSB + threadIdx.x;
  const bool live = col < db;
  const uint32_t colc = live ? col : 0u;  // in-bounds column for idle lanes
  const uint32_t ta = P.str_a[ia];
  const uint32_t tb = P.str_b[colc];
  const uint32_t n_orb = P.n_orb;

  // Pair moves of this lane's target (occupied p -> empty q), packed as
  // source rank | pair index << 16, occupied-major.
  uint32_t mv[kMaxMoves];
  // padding moves point at pair index n_pairs (the zero slot) and column 0
  const uint32_t pad_move = P.n_pairs << 16;
  if (P.enum_ok) {
    const uint32_t full = (n_orb == 32) ? 0xffffffffu : ((1u << n_orb) - 1u);
    const uint32_t emp = ~tb & full;
    const uint32_t ne = n_orb - P.n_beta;
    uint32_t pm_occ = tb, pm_emp = emp, j = 0;
    uint32_t p = __ffs(pm_occ) - 1;
#pragma unroll
    for (int k = 0; k < kMaxMoves; ++k) {
      mv[k] = pad_move;
      if (static_cast<uint32_t>(k) < P.n_moves) {
        const uint32_t q = __ffs(pm_emp) - 1;
        pm_emp &= pm_emp - 1;
        const uint32_t lo = p < q ? p : q, hi = p < q ? q : p;
        const uint32_t pair = hi * (hi - 1) / 2 + lo;
        mv[k] = rank_of<R16>(tb ^ (1u << p) ^ (1u << q), P, s_rank) | (pair << 16);
        if (++j == ne) {
          j = 0;
          pm_emp = emp;
          pm_occ &= pm_occ - 1;
          p = __ffs(pm_occ) - 1;
        }
      }
    }
  }

  double ar4[4] = {0.0, 0.0, 0.0, 0.0}, ai4[4] = {0.0, 0.0, 0.0, 0.0};
  uint32_t c = 0;
  while (c < P.n_class) {
    const ClassMeta M = ld_meta(P.meta + c);
    if (M.flags & kClassSimple) {
      // consecutive single-group classes share one cooperative fold; their
      // valid source rows are listed (in class order) in LDS and gathered
      // four at a time so the row loads overlap
      const uint32_t ua = M.ua;
      uint32_t ce = c + 1;
      uint32_t ub = M.u_end;
      while (ce < P.n_class && ce - c + 3 < P.list_cap) {
        const ClassMeta N = ld_meta(P.meta + ce);
        if (!(N.flags & kClassSimple) || N.u_end - ua > kFCap) break;
        ub = N.u_end;
        ++ce;
      }
      __syncthreads();
      fold_uniques(P, ua, ub, ta, s_F, s_Fz);
      const uint32_t n_list = list_valid_rows<R16>(P, c, ce, ua, ta, s_rank, s_list, s_wcnt);
      for (uint32_t e0 = 0; e0 < n_list; e0 += 4) {
        uint32_t rk[4], w[4];
        double a_r[4], a_i[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint2 L = s_list[e0 + i];
          rk[i] = __builtin_amdgcn_readfirstlane(L.x);
          w[i] = __builtin_amdgcn_readfirstlane(L.y);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) ld_amp<T>(psi, static_cast<uint64_t>(rk[i]) * db + colc, a_r[i], a_i[i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double fr = 0.0, fi = 0.0;
          phase_sum_lds(s_F, s_Fz, w[i] & 0xffffu, w[i] >> 16, tb, fr, fi);
          cmul_acc(fr, fi, a_r[i], a_i[i], ar4[i], ai4[i]);
        }
      }
      c = ce;
      continue;
    }

    const uint32_t sa = ta ^ M.xa;
    if (static_cast<uint32_t>(__popc(sa)) != P.n_alpha) {
      ++c;
      continue;
    }
    const uint64_t rowoff = static_cast<uint64_t>(rank_of<R16>(sa, P, s_rank)) * db;
    const uint32_t gz_end = M.zg >= 0 ? M.g0 + 1 : M.g0;
    // enumerate pair moves when the class's pair groups are dense enough
    const bool penum = P.enum_ok && M.pm >= 0 && (M.u_p - M.ua) <= kFCap && 2 * (M.p1 - gz_end) >= P.n_moves;
    const bool single = penum && (M.flags & kClassPairsSingle);
    const uint32_t ub_a = penum ? M.u_p : M.u_z;
    const bool fold_a = ub_a > M.ua && ub_a - M.ua <= kFCap;
    const bool stage = P.row_lds && gz_end < M.g1;
    const T* rowg = psi + rowoff;

    // phase A: X_beta = 0 group and, when enumerated, the pair groups
    if (stage || fold_a) {
      __syncthreads();
      if (stage)
        for (uint32_t j = threadIdx.x; j < db; j += kSB) s_row[j] = rowg[j];
      if (fold_a) fold_uniques(P, M.ua, ub_a, ta, s_F, s_Fz);
      if (penum) {
        const int32_t* pm = P.pmap + static_cast<uint64_t>(M.pm) * P.n_pairs;
        for (uint32_t q = threadIdx.x; q <= P.n_pairs; q += kSB) {
          const int32_t g = q < P.n_pairs ? pm[q] : -1;  // entry n_pairs serves the padding moves
          uint32_t v;
          if (single)
            v = g >= 0 ? P.pg_u0[g] - M.ua : kFCap;
          else
            v = g >= 0 ? ((P.pg_u0[g] - M.ua) | ((P.pg_u0[g + 1] - P.pg_u0[g]) << 16)) : 0u;
          s_pu[q] = v;
        }
      }
      __syncthreads();
    }
    if (M.zg >= 0) {
      double fr = 0.0, fi = 0.0;
      if (fold_a)
        phase_sum_lds(s_F, s_Fz, 0, M.u_z - M.ua, tb, fr, fi);
      else
        phase_sum_direct(P, static_cast<uint32_t>(M.zg), ta, tb, fr, fi);
      double a_r, a_i;
      if (ROWLDS && stage)
        ld_amp<T>(s_row, colc, a_r, a_i);
      else
        ld_amp<T>(rowg, colc, a_r, a_i);
      cmul_acc(fr, fi, a_r, a_i, ar4[0], ai4[0]);
    }
    const T* rowp = ROWLDS ? s_row : rowg;  // pair and scanned groups need the staged row
    if (penum) {
      uint32_t n_moves = P.n_moves;
      asm volatile("" : "+s"(n_moves));  // keep the move predicates inside the class loop
      if (single) {
        // straight-line groups of four moves: one unique per pair group; absent
        // groups and padding moves hit the zero slot, so loads issue together
#pragma unroll
        for (int k0 = 0; k0 < kMaxMoves; k0 += 4) {
          if (static_cast<uint32_t>(k0) < n_moves) {
            uint32_t e[4], slot[4], z[4];
            double2 f[4];
            double a_r[4], a_i[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              e[i] = mv[k0 + i];
              asm volatile("" : "+v"(e[i]));  // keep per-move address arithmetic inside the class loop
              slot[i] = s_pu[e[i] >> 16];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              f[i] = s_F[slot[i]];
              z[i] = s_Fz[slot[i]];
              ld_amp<T>(rowp, e[i] & 0xffffu, a_r[i], a_i[i]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t par = __popc(z[i] & tb);
              cmul_acc(signed_by(f[i].x, par), signed_by(f[i].y, par), a_r[i], a_i[i], ar4[i], ai4[i]);
            }
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < kMaxMoves; ++k) {
          if (static_cast<uint32_t>(k) < n_moves) {
            uint32_t e = mv[k];
            asm volatile("" : "+v"(e));
            const uint32_t w = s_pu[e >> 16];
            const uint32_t cnt = w >> 16;
            double fr = 0.0, fi = 0.0;
            phase_sum_lds(s_F, s_Fz, w & 0xffffu, cnt, tb, fr, fi);
            double a_r, a_i;
            ld_amp<T>(rowp, e & 0xffffu, a_r, a_i);
            cmul_acc(fr, fi, a_r, a_i, ar4[k & 3], ai4[k & 3]);
          }
        }
      }
    }

    // phase B: remaining groups, scanned in chunks whose uniques fit in LDS;
    // invalid targets are predicated off (source index clamped, coefficient 0)
    uint32_t gs = penum ? M.p1 : gz_end;
    while (gs < M.g1) {
      const uint32_t us = ldc(P.pg_u0 + gs);
      uint32_t ge = gs;
      while (ge < M.g1 && ldc(P.pg_u0 + ge + 1) - us <= kFCap) ++ge;
      if (ge == gs) {
        const uint32_t xb = P.pg_xb[gs];
        const bool valid = live && 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
        if (valid) {
          double fr = 0.0, fi = 0.0;
          phase_sum_direct(P, gs, ta, tb, fr, fi);
          double a_r, a_i;
          ld_amp<T>(rowp, rank_of<R16>(tb ^ xb, P, s_rank), a_r, a_i);
          cmul_acc(fr, fi, a_r, a_i, ar4[1], ai4[1]);
        }
        ++gs;
        continue;
      }
      __syncthreads();
      fold_uniques(P, us, P.pg_u0[ge], ta, s_F, s_Fz);
      __syncthreads();
      uint32_t g = gs;
      for (; g + 1 < ge; g += 2) {
        scan_group<R16>(P, g, us, tb, s_rank, s_F, s_Fz, rowp, ar4[2], ai4[2]);
        scan_group<R16>(P, g + 1, us, tb, s_rank, s_F, s_Fz, rowp, ar4[3], ai4[3]);
      }
      if (g < ge) scan_group<R16>(P, g, us, tb, s_rank, s_F, s_Fz, rowp, ar4[2], ai4[2]);
      gs = ge;
    }
    ++c;
  }

  const double acc_r = (ar4[0] + ar4[1]) + (ar4[2] + ar4[3]);
  const double acc_i = (ai4[0] + ai4[1]) + (ai4[2] + ai4[3]);
  double e_re = 0.0, e_im = 0.0, nrm = 0.0;
  if (live) {
    const uint64_t t = ia * db + col;
    if (EXPVAL) {
      double pr, pi;
      Amp<T>::load(psi, t, pr, pi);
      e_re = fma(pr, acc_r, pi * acc_i);
      e_im = fma(pr, acc_i, -pi * acc_r);
      nrm = fma(pr, pr, pi * pi);
      if (out) Amp<T>::store(out, t, acc_r, acc_i);
    } else {
      Amp<T>::store(out, t, acc_r, acc_i);
    }
  }
  if (EXPVAL) block_reduce3_store<kSB>(e_re, e_im, nrm, slot);
}

template <class T, bool EXPVAL, bool R16, bool ROWLDS>
__global__ __launch_bounds__(kSB) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_apply_sector(
    SectorArgs P, const T* __restrict__ psi, T* __restrict__ out, double* __restrict__ partial) {
  sector_body<T, EXPVAL, R16, ROWLDS>(P, psi, out, partial + 3ull * (blockIdx.y * gridDim.x + blockIdx.x),
                                      blockIdx.x, blockIdx.y);
}

// A job of a batched launch: one operator on one sector state.
struct BatchJob {
  SectorArgs args;
  const void* psi;
  void* out;
  uint32_t block_base;  // first workgroup of the job
  uint32_t chunks;      // beta-column chunks per row
  uint64_t pad;
};

template <class X>
__device__ inline X ld_words(const X* p) {
  static_assert(sizeof(X) % 4 == 0, "word-sized record");
  constexpr int kW = sizeof(X) / 4;
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
  uint32_t w[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) w[i] = ldc(q + i);
  X v;
  memcpy(&v, w, sizeof(v));
  return v;
}

// All jobs of a batch in one launch: workgroup b belongs to the job with the
// largest block_base <= b (jobs are stored in block order).
template <class T, bool EXPVAL, bool R16, bool ROWLDS>
__global__ __launch_bounds__(kSB) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_apply_sector_batch(
    const BatchJob* __restrict__ jobs, uint32_t n_jobs, double* __restrict__ partial) {
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (ldc(&jobs[mid].block_base) <= blockIdx.x)
      lo = mid;
    else
      hi = mid;
  }
  const BatchJob J = ld_words(jobs + lo);
  const uint32_t b = blockIdx.x - J.block_base;
  sector_body<T, EXPVAL, R16, ROWLDS>(J.args, static_cast<const T*>(J.psi), static_cast<T*>(J.out),
                                      partial + 3ull * blockIdx.x, b / J.chunks, b % J.chunks);
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
  block_reduce3_store<kBlock>(a, b, c, result + 3ull * jobs[j].pad);
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
  dim3 grid;
  dim3 block;
  uint64_t parts = 0;
  size_t lds = 0;
};

inline uint32_t align16(uint32_t v) { return (v + 15u) & ~15u; }

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
Launch plan_sector(const pbs_grouped& h, const pbs_space& sp, size_t elem_bytes, bool allow_row, SectorArgs* a_out,
                   bool* r16) {
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
  a.pg_xb = h.pg_xb.get();
  a.pg_u0 = h.pg_u0.get();
  a.u_zb = h.u_zb.get();
  a.u_t0 = h.u_t0.get();
  a.pt_za = h.pt_za.get();
  a.pt_c = reinterpret_cast<const double2*>(h.pt_c.get());

  const uint32_t limit = static_cast<uint32_t>(device_lds_limit()) - 512u;  // reduction scratch
  *r16 = sp.n_orb <= 16;
  const uint32_t rank_bytes = *r16 ? align16(sp.n_chunks * (sp.n_orb + 1) * 256 * 2) : 0u;
  const uint32_t f_bytes = (kFCap + 1) * 16 + align16((kFCap + 1) * 4);
  a.enum_ok = (h.n_pmap > 0 && a.n_moves <= static_cast<uint32_t>(kMaxMoves) && sp.dim_beta < 65536 &&
               h.n_pairs < 65536)
                  ? 1u
                  : 0u;
  const uint32_t pu_bytes = a.enum_ok ? align16((h.n_pairs + 1) * 4) : 0u;
  const uint64_t row_bytes = sp.dim_beta * elem_bytes;
  const uint64_t row_space = row_bytes > kListMinBytes ? row_bytes : kListMinBytes;
  a.row_lds = (allow_row && row_bytes <= kRowCapBytes && rank_bytes + f_bytes + pu_bytes + row_space <= limit) ? 1u : 0u;
  const uint32_t row_region = align16(static_cast<uint32_t>(a.row_lds ? row_space : kListMinBytes));
  a.list_cap = row_region / 8u;
  uint32_t off = 0;
  a.off_rank = off;
  off += rank_bytes;
  a.off_row = off;
  off += row_region;
  a.off_f = off;
  off += (kFCap + 1) * 16;
  a.off_fz = off;
  off += align16((kFCap + 1) * 4);
  a.off_pu = off;
  off += pu_bytes;
  *a_out = a;

  Launch L;
  const uint64_t chunks = (sp.dim_beta + kSB - 1) / kSB;
  L.grid = dim3(static_cast<unsigned>(sp.dim_alpha), static_cast<unsigned>(chunks));
  L.block = dim3(kSB);
  L.parts = sp.dim_alpha * chunks;
  L.lds = off;
  return L;
}

constexpr unsigned kFullGridCap = 1u << 16;

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
    PBS_REQUIRE(sp->dim_beta < (1ull << 31) && sp->dim_alpha < (1ull << 31), PBS_ERR_RANGE,
                "spin-string count exceeds the launch grid");
  }
}

template <class T, bool EXPVAL>
void launch(const pbs_grouped& h, const pbs_space& sp, const void* psi, void* out, double* partial, hipStream_t s) {
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
    const Launch L = plan_sector(h, sp, sizeof(T), true, &a, &r16);
    auto kern = r16 ? (a.row_lds ? k_apply_sector<T, EXPVAL, true, true> : k_apply_sector<T, EXPVAL, true, false>)
                    : (a.row_lds ? k_apply_sector<T, EXPVAL, false, true> : k_apply_sector<T, EXPVAL, false, false>);
    if (L.lds > 64 * 1024)
      PBS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(L.lds)));
    hipLaunchKernelGGL(kern, L.grid, L.block, L.lds, s, a, p, o, partial);
  }
  PBS_HIP(hipGetLastError());
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
    if (dt == PBS_C128)
      launch<double2, true>(*h, *sp, psi, out, partial, s);
    else
      launch<float2, true>(*h, *sp, psi, out, partial, s);
    hipLaunchKernelGGL(k_expval_finish, dim3(1), dim3(kBlock), 0, s, partial, partial_count(*sp), result);
    PBS_HIP(hipGetLastError());
  });
}

}  // extern "C"

struct pbs_batch {
  uint32_t n_jobs = 0;
  uint32_t total_blocks = 0;
  pbs_dtype dt = PBS_C64;
  bool r16 = false, row_lds = false;
  size_t lds = 0;
  pbs::DevBuf<pbs::BatchJob> jobs;
  pbs::DevBuf<double> partial;
};

namespace pbs {
namespace {
template <class T, bool EXPVAL>
void* batch_kernel(bool r16, bool rowlds) {
  if (r16)
    return rowlds ? reinterpret_cast<void*>(k_apply_sector_batch<T, EXPVAL, true, true>)
                  : reinterpret_cast<void*>(k_apply_sector_batch<T, EXPVAL, true, false>);
  return rowlds ? reinterpret_cast<void*>(k_apply_sector_batch<T, EXPVAL, false, true>)
                : reinterpret_cast<void*>(k_apply_sector_batch<T, EXPVAL, false, false>);
}

void* pick_batch_kernel(pbs_dtype dt, bool expval, bool r16, bool rowlds) {
  if (dt == PBS_C128) return expval ? batch_kernel<double2, true>(r16, rowlds) : batch_kernel<double2, false>(r16, rowlds);
  return expval ? batch_kernel<float2, true>(r16, rowlds) : batch_kernel<float2, false>(r16, rowlds);
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
    std::vector<BatchJob> jobs(n);
    std::vector<double> cost(n);
    std::vector<uint32_t> order(n);
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
    // one launch shares one kernel variant: rows staged only if every job's
    // row fits, LDS rank tables only if every job has n_orb <= 16
    bool r16 = true, rowlds = true;
    for (uint32_t i = 0; i < n; ++i) {
      bool job_r16 = false;
      plan_sector(*h[i], *sp[i], esz, true, &jobs[i].args, &job_r16);
      r16 = r16 && job_r16;
      rowlds = rowlds && jobs[i].args.row_lds;
    }
    size_t lds = 0;
    for (uint32_t i = 0; i < n; ++i) {
      bool job_r16 = false;
      const Launch L = plan_sector(*h[i], *sp[i], esz, rowlds, &jobs[i].args, &job_r16);
      if (!r16) jobs[i].args.rank16 = nullptr;
      jobs[i].psi = psi[i];
      jobs[i].out = out[i];
      jobs[i].chunks = L.grid.y;
      jobs[i].block_base = 0;
      jobs[i].pad = i;  // original position (energies are written there)
      lds = std::max(lds, L.lds);
      cost[i] = static_cast<double>(sp[i]->dim) * static_cast<double>(h[i]->n_pterm + 1);
      order[i] = i;
    }
    // largest jobs first, so the launch does not end on a long straggler
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
    std::vector<BatchJob> sorted(n);
    uint64_t base = 0;
    for (uint32_t k = 0; k < n; ++k) {
      BatchJob J = jobs[order[k]];
      J.block_base = static_cast<uint32_t>(base);
      base += static_cast<uint64_t>(sp[order[k]]->dim_alpha) * J.chunks;
      sorted[k] = J;
    }
    PBS_REQUIRE(base < (1ull << 31), PBS_ERR_RANGE, "batch needs more than 2^31 workgroups");
    auto* B = new pbs_batch();
    try {
      B->n_jobs = n;
      B->total_blocks = static_cast<uint32_t>(base);
      B->dt = dt;
      B->r16 = r16;
      B->row_lds = rowlds;
      B->lds = lds;
      B->jobs.alloc(n);
      B->partial.alloc(3ull * base);
      PBS_HIP(hipMemcpy(B->jobs.get(), sorted.data(), n * sizeof(BatchJob), hipMemcpyHostToDevice));
      if (lds > 64 * 1024) {
        for (bool ev : {false, true})
          PBS_HIP(hipFuncSetAttribute(pick_batch_kernel(dt, ev, r16, rowlds),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
      }
    } catch (...) {
      delete B;
      throw;
    }
    *batch = B;
  });
}

pbs_status pbs_batch_run(const pbs_batch* b, double* energies, void* stream) {
  return guarded([&] {
    PBS_REQUIRE(b != nullptr, PBS_ERR_ARG, "null pbs_batch");
    hipStream_t s = as_stream(stream);
    const bool ev = energies != nullptr;
    void* kern = pick_batch_kernel(b->dt, ev, b->r16, b->row_lds);
    const BatchJob* jobs = b->jobs.get();
    uint32_t n = b->n_jobs;
    double* partial = b->partial.get();
    void* args[] = {&jobs, &n, &partial};
    PBS_HIP(hipLaunchKernel(kern, dim3(b->total_blocks), dim3(kSB), args, b->lds, s));
    if (ev) {
      hipLaunchKernelGGL(k_batch_finish, dim3(n), dim3(kBlock), 0, s, jobs, n, b->total_blocks, partial, energies);
      PBS_HIP(hipGetLastError());
    }
  });
}

void pbs_batch_destroy(pbs_batch* b) { delete b; }

}  // extern "C"
