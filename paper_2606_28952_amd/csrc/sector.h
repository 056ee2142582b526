// Device code of the operator-state product by target-driven summation over
// X-mask groups (Section 2.4, Eq. reverse_sum) and, in spin sectors, over the
// spin-resolved product basis (Eq. sreverse_sum); the fused energy of
// Eq. vqe_energy.  Shared by the library's translation units; each sector
// kernel variant is instantiated in exactly one of the sector_*.hip files.
//
// Every output amplitude is produced by exactly one thread, which gathers
// the source amplitudes psi[t ^ X_g] of all groups and multiplies each by
// its group's phase sum sum_k C_k (-1)^popcount(Z_k & s); there are no
// atomics and results are bitwise reproducible.  Amplitudes are read in
// their storage type (complex128 or complex64) and everything else --
// coefficients, phase sums, accumulators, reductions -- is float64.  When
// every coefficient of the operator is real (real Hamiltonians in XZ form:
// Section 2.3), phase sums are real float64 and each gather costs two FMAs.
//
// Sector kernel layout: a workgroup owns one target alpha string t_a (one
// row of the alpha-major state) and kSB consecutive beta columns, one target
// per lane.  Groups are visited class by class (a class shares X_alpha), so
// the source row s_a = t_a ^ X_alpha, its validity and its rank are uniform
// across the workgroup, and so are the alpha parities of every term: the
// coefficients of each unique beta Z-mask are folded over their terms' alpha
// parities cooperatively into LDS once per class.
//  * Simple classes (a single X_beta = 0 group) come first: runs of them are
//    batched into one fold, their valid source rows are listed in LDS and
//    gathered kGather at a time.
//  * In every other class the source row is staged in LDS when it fits; the
//    group with X_beta = 0 gathers from the lane's own column; groups whose
//    X_beta flips two orbitals are visited by enumerating the lane's valid
//    pair moves (occupied -> empty, the same count for every target of a
//    sector), cached in registers with their source columns and beta
//    parities, through a per-class pair map; groups whose X_beta flips four
//    orbitals by enumerating the valid double moves through a quad map;
//    invalid moves are never visited.  Other groups are scanned with a
//    per-lane validity test.
// Parities are evaluated against the target strings each lane holds; the
// constant (-1)^popcount(z & X) factors were moved into the coefficients
// when the tables were built.
#pragma once

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

// v * (-1)^(bit 31 of e), one bitwise op on the high word (b ^ (a & c)).
__device__ inline double signed_by_bit31(double v, uint32_t e) {
  return __hiloint2double(
      static_cast<int>(__builtin_amdgcn_bitop3_b32(e, static_cast<uint32_t>(__double2hiint(v)), 0x80000000u, 0x6c)),
      __double2loint(v));
}

// Read-only load through the constant address space: uniform addresses
// become scalar loads (the tables are never written by the kernels).
__device__ inline uint32_t ldc(const uint32_t* p) { return *((const __attribute__((address_space(4))) uint32_t*)(p)); }
__device__ inline double ldc(const double* p) { return *((const __attribute__((address_space(4))) double*)(p)); }

// LDS load at an absolute byte address.  The kernels declare no static LDS,
// so the dynamic allocation starts at address 0 and an address computed in a
// register needs no base added.
template <class U>
struct LdsLoad {
  __device__ static __forceinline__ U at(uint32_t byte) {
    typedef __attribute__((address_space(3))) const U* LdsPtr;
    return *(LdsPtr)(static_cast<uintptr_t>(byte));
  }
};
template <class E>
struct LdsLoad<HIP_vector_type<E, 2>> {  // two components (adjacent loads merge)
  __device__ static __forceinline__ HIP_vector_type<E, 2> at(uint32_t byte) {
    HIP_vector_type<E, 2> v;
    v.x = LdsLoad<E>::at(byte);
    v.y = LdsLoad<E>::at(byte + sizeof(E));
    return v;
  }
};
template <class U>
__device__ __forceinline__ U lds_ld(uint32_t byte) {
  return LdsLoad<U>::at(byte);
}

__device__ inline ClassMeta ld_meta(const ClassMeta* p) {
  static_assert(sizeof(ClassMeta) == 16 * sizeof(uint32_t), "ClassMeta layout");
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
  uint32_t w[14];  // the last two words are padding
#pragma unroll
  for (int i = 0; i < 14; ++i) w[i] = ldc(q + i);
  ClassMeta m;
  memcpy(&m, w, sizeof(w));
  m.pad[0] = m.pad[1] = 0;
  return m;
}

// Workgroup sums of (a, b, c) written by thread 0 to dst; red holds 3 B/64
// doubles of LDS.
template <int B>
__device__ inline void block_reduce3_store(double a, double b, double c, double* dst, double (*red)[B / 64]) {
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

template <int B>
__device__ inline void block_reduce3_store(double a, double b, double c, double* dst) {
  __shared__ double red[3][B / 64];
  block_reduce3_store<B>(a, b, c, dst, red);
}

// ---------------------------------------------------------------- coefficients
// Phase-sum arithmetic for complex (double2) or real (double) coefficients.
template <bool REALC>
struct Coef;
template <>
struct Coef<false> {
  using V = double2;
  __device__ static inline V zero() { return make_double2(0.0, 0.0); }
  __device__ static inline V term(const double2* c, uint32_t t) { return c[t]; }
  __device__ static inline void add_signed(V& acc, V c, uint32_t par) {
    acc.x += signed_by(c.x, par);
    acc.y += signed_by(c.y, par);
  }
  __device__ static inline V sign(V c, uint32_t par) { return make_double2(signed_by(c.x, par), signed_by(c.y, par)); }
  __device__ static inline V sign31(V c, uint32_t e) {
    return make_double2(signed_by_bit31(c.x, e), signed_by_bit31(c.y, e));
  }
  __device__ static inline V zeroed_unless(V f, bool keep) { return keep ? f : zero(); }
  // acc += f * a
  __device__ static inline void mac(V f, double ar, double ai, double& acc_r, double& acc_i) {
    acc_r = fma(ar, f.x, fma(-ai, f.y, acc_r));
    acc_i = fma(ar, f.y, fma(ai, f.x, acc_i));
  }
};
template <>
struct Coef<true> {
  using V = double;
  __device__ static inline V zero() { return 0.0; }
  __device__ static inline V term(const double2* c, uint32_t t) { return c[t].x; }
  __device__ static inline void add_signed(V& acc, V c, uint32_t par) { acc += signed_by(c, par); }
  __device__ static inline V sign(V c, uint32_t par) { return signed_by(c, par); }
  __device__ static inline V sign31(V c, uint32_t e) { return signed_by_bit31(c, e); }
  __device__ static inline V zeroed_unless(V f, bool keep) { return keep ? f : 0.0; }
  __device__ static inline void mac(V f, double ar, double ai, double& acc_r, double& acc_i) {
    acc_r = fma(ar, f, acc_r);
    acc_i = fma(ai, f, acc_i);
  }
};

// ---------------------------------------------------------------- spin sector
constexpr int kSB = 512;              // lanes per sector workgroup = beta columns per workgroup
constexpr int kGather = 16;  // simple-class row loads in flight per lane
// the LDS placement constants (kPuOff, kRowOff, ...) are in host_plan.h

constexpr uint32_t kFactZero = 1u;  // X_beta = 0 groups through their F rows
constexpr uint32_t kFactMoves = 2u;  // the X_alpha = 0 class through the move tables
constexpr uint32_t kFactAlpha = 4u;  // simple classes through the alpha lists

struct SectorArgs {
  uint32_t n_orb, n_alpha, n_beta, n_chunks;
  uint32_t dim_beta;
  uint32_t row_begin;  // first target alpha row of the launch (0: the whole sector)
  uint32_t n_class, n_pairs, n_moves;
  uint32_t row_lds, enum_ok;
  uint32_t list_cap;  // entries of the simple-class row list (in the row space)
  uint32_t f_cap;     // folded uniques held in LDS at once; kZeroSlots zeros follow
  uint32_t qenum_ok, n_quads, n_qmoves;  // double-move enumeration (n_orb <= 16)
  uint32_t quad_cnt;                     // uniques of every quad group when all are equal, else 0
  uint32_t pair_sign;                    // beta parities of pair moves cached per target (zpair)
  const uint32_t* zpair;
  uint32_t n_runs, n_ns;                 // class schedule: simple-class runs, other classes
  const uint32_t* runs;                  // (first, end) per run
  const uint32_t* ns_list;
  uint32_t off_rank, off_f, off_fz, off_qu;  // LDS byte offsets (the pair map and row are fixed)
  const uint32_t* str_a;
  const uint32_t* str_b;
  const uint16_t* rank16;  // n_orb <= 16
  const uint32_t* rank32;
  const ClassMeta* meta;
  const int32_t* pmap;
  const int32_t* qmap;
  const uint32_t* pg_xb;
  const uint32_t* pg_u0;
  const uint32_t* u_zb;
  const uint32_t* u_t0;
  const uint32_t* pt_za;
  const double2* pt_c;
  // spin-factorized evaluation (FactorPlan; real coefficients): fact holds
  // kFactZero when X_beta = 0 groups use their F rows (0 when unused); f_c0
  // = the X_alpha = 0 class whose pair and quad groups are evaluated through
  // the move tables, or ~0
  uint32_t fact, f_c0, f_r2, f_r3, f_c0_fu0, f_c0_fu1, f_n_qmoves, off_a;
  // longest factor unique (terms) among: the X_beta = 0 groups', the class-0
  // pair groups' (factor uniques f_c0_fu0 .. f_c0_fq - 1) and quad groups'
  uint32_t f_tz, f_tp, f_tq, f_c0_fq;
  // alpha lists of the simple classes (FactorPlan::alist_*), or null: pass A
  // then reads each row's valid simple classes and coefficients directly
  const uint32_t* alist_off;
  const uint32_t* alist_src;
  const double* alist_c;
  // alpha images of the image classes (FactorPlan::plist, pimg), or null
  const uint32_t* plist_off;
  const uint32_t* plist_src;
  const uint32_t* plist_cls;
  const double* pimg;
  const uint32_t* pimg_flag;
  uint32_t n_img, pad_img;
  const uint32_t* fu_t0;
  const uint32_t* ft_za;
  const double* ft_c;
  const uint4* cls_f;
  const double* fz;
  const uint32_t* em;
  const double* fp;
  const uint32_t* eq;
  const double* fq;
};

// Combinatorial rank of a spin string: uint16 tables in LDS (n_orb <= 16,
// at most two byte chunks) or uint32 tables in global memory.
template <bool R16>
__device__ inline uint32_t rank_of(uint32_t s, const SectorArgs& P, const uint16_t* t16) {
  if (R16) {  // the chunk-1 tables are zero when n_orb <= 8
    const uint32_t lo = s & 255u;
    return t16[lo] + t16[256u + (static_cast<uint32_t>(__popc(lo)) << 8) + ((s >> 8) & 255u)];
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
template <bool REALC>
__device__ inline void fold_uniques(const SectorArgs& P, uint32_t ua, uint32_t ub, uint32_t ta,
                                    typename Coef<REALC>::V* F, uint32_t* Fz, uint32_t lane0 = threadIdx.x,
                                    uint32_t stride = kSB) {
  using C = Coef<REALC>;
  for (uint32_t u = ua + lane0; u < ub; u += stride) {
    typename C::V f = C::zero();
    const uint32_t t1 = P.u_t0[u + 1];
    for (uint32_t t = P.u_t0[u]; t < t1; ++t) C::add_signed(f, C::term(P.pt_c, t), __popc(P.pt_za[t] & ta));
    F[u - ua] = f;
    Fz[u - ua] = P.u_zb[u];
  }
}

// A_r = sum over the factor unique's terms of P[mu][r] (-1)^popcount(za & ta)
// for factor uniques fa .. fb-1, written to A[0 ..).  L consecutive lanes
// share a factor unique (lane j of the set takes terms j, j + L, ...) and
// add their parts in a fixed butterfly, so the loads of a unique's terms are
// issued together and the result does not depend on timing.
template <int L>
__device__ inline void fold_factors_l(const SectorArgs& P, uint32_t fa, uint32_t fb, uint32_t ta, double* A,
                                      uint32_t lane0, uint32_t stride) {
  const uint32_t j = lane0 % L;
  for (uint32_t u0 = fa; u0 < fb; u0 += stride / L) {
    const uint32_t u = u0 + lane0 / L;
    double f = 0.0;
    if (u < fb) {
      const uint32_t t1 = P.fu_t0[u + 1];
      for (uint32_t t = P.fu_t0[u] + j; t < t1; t += L) f += signed_by(P.ft_c[t], __popc(P.ft_za[t] & ta));
    }
#pragma unroll
    for (int d = L / 2; d > 0; d /= 2) f += __shfl_xor(f, d, 64);
    if (u < fb && j == 0) A[u - fa] = f;
  }
}

// lanes per factor unique for a range whose longest factor unique has
// `terms` terms
__device__ inline void fold_factors(const SectorArgs& P, uint32_t fa, uint32_t fb, uint32_t terms, uint32_t ta,
                                    double* A, uint32_t lane0, uint32_t stride) {
  if (terms <= 1)
    fold_factors_l<1>(P, fa, fb, ta, A, lane0, stride);
  else if (terms <= 16)
    fold_factors_l<16>(P, fa, fb, ta, A, lane0, stride);
  else
    fold_factors_l<64>(P, fa, fb, ta, A, lane0, stride);
}

template <bool REALC>
__device__ inline void phase_sum_lds(const typename Coef<REALC>::V* F, const uint32_t* Fz, uint32_t b, uint32_t cnt,
                                     uint32_t tb, typename Coef<REALC>::V& f) {
  for (uint32_t i = 0; i < cnt; ++i) Coef<REALC>::add_signed(f, F[b + i], __popc(Fz[b + i] & tb));
}

// Phase sum of group g straight from the term tables (groups too large for LDS).
template <bool REALC>
__device__ inline void phase_sum_direct(const SectorArgs& P, uint32_t g, uint32_t ta, uint32_t tb,
                                        typename Coef<REALC>::V& f) {
  using C = Coef<REALC>;
  const uint32_t u1 = P.pg_u0[g + 1];
  for (uint32_t u = P.pg_u0[g]; u < u1; ++u) {
    typename C::V h = C::zero();
    const uint32_t t1 = P.u_t0[u + 1];
    for (uint32_t t = P.u_t0[u]; t < t1; ++t) C::add_signed(h, C::term(P.pt_c, t), __popc(P.pt_za[t] & ta));
    C::add_signed(f, h, __popc(P.u_zb[u] & tb));
  }
}

template <class T>
__device__ inline void ld_amp(const T* p, uint64_t i, double& r, double& m) {
  Amp<T>::load(p, i, r, m);
}

// Validity, source column and phase sum of one scanned group (the phase sum
// is zeroed for invalid targets, whose column is 0).
template <bool R16, bool REALC>
__device__ __forceinline__ void scan_prepare(const SectorArgs& P, uint32_t g, uint32_t us, uint32_t tb,
                                             const uint16_t* s_rank, const typename Coef<REALC>::V* s_F,
                                             const uint32_t* s_Fz, uint32_t& jb, typename Coef<REALC>::V& f) {
  using C = Coef<REALC>;
  const uint32_t xb = ldc(P.pg_xb + g);
  const uint32_t u0 = ldc(P.pg_u0 + g), u1 = ldc(P.pg_u0 + g + 1);
  const bool valid = 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
  jb = valid ? rank_of<R16>(tb ^ xb, P, s_rank) : 0u;
  typename C::V h = C::zero();
  phase_sum_lds<REALC>(s_F, s_Fz, u0 - us, u1 - u0, tb, h);
  f = C::zeroed_unless(h, valid);
}

// One group of a scanned chunk: validity of X_beta for this lane's target,
// source column rank, phase sum from the folded uniques; invalid targets are
// predicated off (column 0 is read, the coefficient is zeroed).
template <bool R16, bool REALC, class T>
__device__ __forceinline__ void scan_group(const SectorArgs& P, uint32_t g, uint32_t us, uint32_t tb,
                                           const uint16_t* s_rank, const typename Coef<REALC>::V* s_F,
                                           const uint32_t* s_Fz, const T* rowp, double& acc_r, double& acc_i) {
  using C = Coef<REALC>;
  const uint32_t xb = ldc(P.pg_xb + g);
  const uint32_t u0 = ldc(P.pg_u0 + g), u1 = ldc(P.pg_u0 + g + 1);
  const bool valid = 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
  const uint32_t jb = valid ? rank_of<R16>(tb ^ xb, P, s_rank) : 0u;
  typename C::V f = C::zero();
  phase_sum_lds<REALC>(s_F, s_Fz, u0 - us, u1 - u0, tb, f);
  double a_r, a_i;
  ld_amp<T>(rowp, jb, a_r, a_i);
  C::mac(C::zeroed_unless(f, valid), a_r, a_i, acc_r, acc_i);
}

// One double move of this lane's target: X_beta = X (two occupied and two
// empty orbitals).  The quad map slot gives the folded uniques of X's group
// (absent groups point at the zero slot).
// Source amplitude of a cached pair move: from the staged row at its LDS
// byte offset, or from the global row.
template <class T, bool ROWLDS>
__device__ __forceinline__ void move_amp(const unsigned char* smem, const T* rowg, uint32_t e, double& r, double& m) {
  if (ROWLDS)
    Amp<T>::load(reinterpret_cast<const T*>(smem + kRowOff + (e & 0xffffu)), 0, r, m);
  else
    Amp<T>::load(rowg, e & 0xffffu, r, m);
}

// QC > 0: every quad group has QC uniques (absent groups point at QC zero
// slots), so the phase sum is straight-line; QC = 0: counts from the map.
template <int QC, bool R16, bool REALC, class T>
__device__ __forceinline__ void quad_move(const SectorArgs& P, uint32_t X, uint32_t tb, const uint16_t* s_rank,
                                          const typename Coef<REALC>::V* s_F, const uint32_t* s_Fz,
                                          const uint32_t* s_qu, const T* rowp, double& acc_r, double& acc_i) {
  using C = Coef<REALC>;
  const uint32_t w = s_qu[rank_of<R16>(X, P, s_rank)];
  const uint32_t src = rank_of<R16>(tb ^ X, P, s_rank);
  typename C::V f = C::zero();
  if (QC > 0) {
    const uint32_t b = w & 0xffffu;
#pragma unroll
    for (int i = 0; i < QC; ++i) C::add_signed(f, s_F[b + i], __popc(s_Fz[b + i] & tb));
  } else {
    phase_sum_lds<REALC>(s_F, s_Fz, w & 0xffffu, w >> 16, tb, f);
  }
  double a_r, a_i;
  ld_amp<T>(rowp, src, a_r, a_i);
  C::mac(f, a_r, a_i, acc_r, acc_i);
}

// All C(N_beta, 2) C(n_orb - N_beta, 2) double moves of this lane's target,
// occupied pairs outer, empty pairs inner (two per step).  Every loop bound
// is uniform across the workgroup.
template <int QC, bool R16, bool REALC, class T>
__device__ __forceinline__ void quad_moves(const SectorArgs& P, uint32_t tb, const uint16_t* s_rank,
                                           const typename Coef<REALC>::V* s_F, const uint32_t* s_Fz,
                                           const uint32_t* s_qu, const T* rowp, double (&ar4)[4],
                                           double (&ai4)[4]) {
  const uint32_t nb = P.n_beta, ne = P.n_orb - P.n_beta;
  const uint32_t full = (P.n_orb == 32) ? 0xffffffffu : ((1u << P.n_orb) - 1u);
  const uint32_t emp = ~tb & full;
  uint32_t oa = tb;
  for (uint32_t i = 1; i < nb; ++i) {
    const uint32_t o1 = oa & (0u - oa);
    oa ^= o1;
    uint32_t ob = oa;
    for (uint32_t j = i; j < nb; ++j) {
      const uint32_t o2 = ob & (0u - ob);
      ob ^= o2;
      uint32_t ea = emp;
      for (uint32_t k = 1; k < ne; ++k) {
        const uint32_t e1 = ea & (0u - ea);
        ea ^= e1;
        const uint32_t base = o1 | o2 | e1;
        uint32_t eb = ea;
        uint32_t l = k;
        for (; l + 1 < ne; l += 2) {
          const uint32_t e2 = eb & (0u - eb);
          eb ^= e2;
          const uint32_t e3 = eb & (0u - eb);
          eb ^= e3;
          quad_move<QC, R16, REALC>(P, base | e2, tb, s_rank, s_F, s_Fz, s_qu, rowp, ar4[2], ai4[2]);
          quad_move<QC, R16, REALC>(P, base | e3, tb, s_rank, s_F, s_Fz, s_qu, rowp, ar4[3], ai4[3]);
        }
        if (l < ne) quad_move<QC, R16, REALC>(P, base | (eb & (0u - eb)), tb, s_rank, s_F, s_Fz, s_qu, rowp, ar4[1], ai4[1]);
      }
    }
  }
}

// Factored groups of the X_alpha = 0 class through a move table (single or
// double moves of this lane's beta string, n per string): entry = source
// column | (first folded factor of the move's group, or a zero slot) << 16,
// and F_r of that group at this lane's beta string.  Software-pipelined
// over three register buffers of 8 / R moves: while one buffer is
// evaluated, the table loads of the next two are in flight.
template <int R, class T, bool ROWLDS>
struct MoveTable {
  static constexpr int kU = 8 / R;
  uint32_t e[kU];
  double F[kU][R];
  __device__ __forceinline__ void load(const uint32_t* ent, const double* fv, uint64_t db, uint32_t col, uint32_t q0,
                                       uint32_t n) {
#pragma unroll
    for (int i = 0; i < kU; ++i) {
      const uint32_t m = min(q0 + i, n - 1u);  // past the end: reload the last move (unused)
      e[i] = ent[static_cast<uint64_t>(m) * db + col];
#pragma unroll
      for (int r = 0; r < R; ++r) F[i][r] = fv[(static_cast<uint64_t>(m) * R + r) * db + col];
    }
  }
  __device__ __forceinline__ void eval(const unsigned char* smem, const double* s_A, const T* rowg, uint32_t q0,
                                       uint32_t n, double (&ar4)[4], double (&ai4)[4]) const {
    double a_r[kU], a_i[kU];
#pragma unroll
    for (int i = 0; i < kU; ++i) {
      if (ROWLDS)
        Amp<T>::load(reinterpret_cast<const T*>(smem + kRowOff), e[i] & 0xffffu, a_r[i], a_i[i]);
      else
        Amp<T>::load(rowg, e[i] & 0xffffu, a_r[i], a_i[i]);
    }
#pragma unroll
    for (int i = 0; i < kU; ++i) {
      double f = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) f = fma(s_A[(e[i] >> 16) + r], F[i][r], f);
      f = q0 + i < n ? f : 0.0;  // moves past the end (uniform)
      Coef<true>::mac(f, a_r[i], a_i[i], ar4[i & 3], ai4[i & 3]);
    }
  }
};

template <int R, class T, bool ROWLDS>
__device__ __forceinline__ void fact_table_moves(const unsigned char* smem, const double* s_A, const T* rowg,
                                                 uint32_t n, const uint32_t* ent, const double* fv, uint64_t db,
                                                 uint32_t col, double (&ar4)[4], double (&ai4)[4]) {
  using MT = MoveTable<R, T, ROWLDS>;
  constexpr uint32_t U = MT::kU;
  if (n == 0) return;
  MT b0, b1, b2;
  b0.load(ent, fv, db, col, 0, n);
  b1.load(ent, fv, db, col, U, n);
  for (uint32_t q0 = 0;; q0 += 3 * U) {
    b2.load(ent, fv, db, col, q0 + 2 * U, n);
    b0.eval(smem, s_A, rowg, q0, n, ar4, ai4);
    if (q0 + U >= n) break;
    b0.load(ent, fv, db, col, q0 + 3 * U, n);
    b1.eval(smem, s_A, rowg, q0 + U, n, ar4, ai4);
    if (q0 + 2 * U >= n) break;
    b1.load(ent, fv, db, col, q0 + 4 * U, n);
    b2.eval(smem, s_A, rowg, q0 + 2 * U, n, ar4, ai4);
    if (q0 + 3 * U >= n) break;
  }
}

// Appends to the list, in class order, the simple classes c0 .. c1-1 whose
// source alpha string ta ^ X_alpha lies in the sector: entry = (source row
// rank, first folded unique | unique count << 16), where a class's uniques
// sit at its unique index minus ubase.  Entries start at index `base`; the
// new length is returned (uniform).  Ends with a barrier.
template <bool R16>
__device__ uint32_t append_valid_rows(const SectorArgs& P, uint32_t c0, uint32_t c1, uint32_t ubase, uint32_t ta,
                                      const uint16_t* s_rank, uint2* s_list, uint32_t* s_wcnt, uint32_t base) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  for (uint32_t i0 = c0; i0 < c1; i0 += kSB) {
    const uint32_t cc = i0 + threadIdx.x;
    bool v = false;
    uint2 entry = make_uint2(0u, 0u);
    if (cc < c1) {
      const ClassMeta* m = P.meta + cc;
      const uint32_t sa = ta ^ m->xa;
      v = static_cast<uint32_t>(__popc(sa)) == P.n_alpha;
      if (v) {
        // bit 31: the class's single unique has beta Z-mask 0 (its phase sum
        // is the folded coefficient itself, as for same-spin alpha doubles)
        const uint32_t cnt = m->u_end - m->ua;
        const uint32_t plain = (cnt == 1 && P.u_zb[m->ua] == 0u) ? 0x80000000u : 0u;
        entry = make_uint2(rank_of<R16>(sa, P, s_rank), (m->ua - ubase) | (cnt << 16) | plain);
      }
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
  return base;
}

// Copies the db-element source row into LDS, with 16-byte accesses when the
// row is 16-byte aligned (complex64 pairs; complex128 is 16 bytes anyway).
template <class T>
__device__ __forceinline__ void stage_row(T* s_row, const T* rowg, uint32_t db, uint32_t lane0, uint32_t stride) {
  if (sizeof(T) == 8 && (reinterpret_cast<uintptr_t>(rowg) & 15u) == 0) {
    const uint32_t n2 = db / 2;
    const uint4* src = reinterpret_cast<const uint4*>(rowg);
    uint4* dst = reinterpret_cast<uint4*>(s_row);  // the staged row is 16-byte aligned
    for (uint32_t j = lane0; j < n2; j += stride) dst[j] = src[j];
    if ((db & 1u) && lane0 == 0) s_row[db - 1] = rowg[db - 1];
  } else {
    for (uint32_t j = lane0; j < db; j += stride) s_row[j] = rowg[j];
  }
}

// One workgroup: target alpha string ia (one row of the state), beta columns
// chunk*kSB .. chunk*kSB + kSB - 1, one target per lane.  See the file header
// for the scheme.  `slot` receives the workgroup's energy partials.
template <class T, bool EXPVAL, bool R16, bool ROWLDS, bool REALC>
__device__ __forceinline__ void sector_body(const SectorArgs& P, const T* __restrict__ psi, T* __restrict__ out,
                                            double* __restrict__ slot, uint64_t ia, uint32_t chunk) {
  using C = Coef<REALC>;
  using V = typename C::V;
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* s_rank = reinterpret_cast<uint16_t*>(smem + P.off_rank);
  T* s_row = reinterpret_cast<T*>(smem + kRowOff);
  V* s_F = reinterpret_cast<V*>(smem + P.off_f);
  uint32_t* s_Fz = reinterpret_cast<uint32_t*>(smem + P.off_fz);
  uint32_t* s_pu = reinterpret_cast<uint32_t*>(smem + kPuOff);
  uint32_t* s_qu = reinterpret_cast<uint32_t*>(smem + P.off_qu);
  uint2* s_list = reinterpret_cast<uint2*>(smem + kRowOff);  // shares the staged row's space
  uint32_t* s_wcnt = reinterpret_cast<uint32_t*>(smem);      // kSB / 64 words
  auto* s_red = reinterpret_cast<double(*)[kSB / 64]>(smem + 64);  // 3 x kSB / 64 doubles
  const uint32_t f_cap = P.f_cap;

  if (R16) {
    // 256 entries of chunk 0 (no ones below), then the chunk-1 entries for 0..8
    // ones below (zeros for a single chunk), copied as 32-bit words with every
    // load issued before the first LDS store
    constexpr uint32_t kWords = kRank16Lds / 2u, kIters = (kWords + kSB - 1u) / kSB;
    const uint32_t* r0 = reinterpret_cast<const uint32_t*>(P.rank16);
    const uint32_t* r1 = reinterpret_cast<const uint32_t*>(P.rank16 + (P.n_orb + 1) * 256u);
    uint32_t* s_rank32 = reinterpret_cast<uint32_t*>(s_rank);
    uint32_t v[kIters];
#pragma unroll
    for (uint32_t k = 0; k < kIters; ++k) {
      const uint32_t w = threadIdx.x + k * kSB;
      v[k] = w < 128u ? r0[w] : (w < kWords && P.n_chunks > 1 ? r1[w - 128u] : 0u);
    }
#pragma unroll
    for (uint32_t k = 0; k < kIters; ++k) {
      const uint32_t w = threadIdx.x + k * kSB;
      if (w < kWords) s_rank32[w] = v[k];
    }
  }
  // beta Z-masks of the pair moves, for the move cache below (the pair-map
  // region is free until pass B)
  if (P.enum_ok && P.pair_sign && threadIdx.x <= P.n_pairs)
    reinterpret_cast<uint32_t*>(smem + kPuOff)[threadIdx.x] = P.zpair[threadIdx.x];
  if (threadIdx.x < kZeroSlots) {  // zero slots for absent groups and padding entries
    s_F[f_cap + threadIdx.x] = C::zero();
    s_Fz[f_cap + threadIdx.x] = 0u;
  }
  __syncthreads();

  const uint32_t db = P.dim_beta;
  const uint32_t col = chunk * kSB + threadIdx.x;
  const bool live = col < db;
  const uint32_t colc = live ? col : 0u;  // in-bounds column for idle lanes
  const uint32_t ta = P.str_a[ia];
  const uint32_t tb = P.str_b[colc];
  const uint32_t n_orb = P.n_orb;

  double ar4[4] = {0.0, 0.0, 0.0, 0.0}, ai4[4] = {0.0, 0.0, 0.0, 0.0};

  // pass A through the alpha list: the row's valid simple classes in class
  // order, each a source row rank and a coefficient uniform across the
  // workgroup.  The row's list is copied into LDS (the staged-row region is
  // free here) in pieces; each gather then reads its entry as a broadcast
  // LDS load, and two buffers of kGather / 2 rows keep the next gathers in
  // flight while the current ones are summed.
  if (P.alist_off != nullptr) {
    const uint32_t a0 = ldc(P.alist_off + ia), a1 = ldc(P.alist_off + ia + 1);
    constexpr uint32_t G = kGather / 2;
    const uint32_t cap = (P.list_cap * 8u / 12u) & ~(2u * G - 1u);  // entries per piece (4 + 8 bytes each)
    const uint32_t* s_src = reinterpret_cast<const uint32_t*>(smem + kRowOff);
    const double* s_c = reinterpret_cast<const double*>(smem + kRowOff + 4u * cap);
    const T* psi_col = psi + colc;
    struct Buf {
      double c[G];
      T a[G];
    } b0, b1;
    for (uint32_t p0 = a0; p0 < a1; p0 += cap) {
      const uint32_t n = min(cap, a1 - p0);
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < n; j += kSB) {
        reinterpret_cast<uint32_t*>(smem + kRowOff)[j] = P.alist_src[p0 + j];
        reinterpret_cast<double*>(smem + kRowOff + 4u * cap)[j] = P.alist_c[p0 + j];
      }
      __syncthreads();
      auto load = [&](uint32_t e0, Buf& b) {
#pragma unroll
        for (uint32_t i = 0; i < G; ++i) {
          const uint32_t m = min(e0 + i, n - 1u);
          b.c[i] = e0 + i < n ? s_c[m] : 0.0;
          b.a[i] = psi_col[static_cast<uint64_t>(s_src[m]) * db];
        }
      };
      auto eval = [&](const Buf& b) {
#pragma unroll
        for (uint32_t i = 0; i < G; ++i)
          Coef<true>::mac(b.c[i], static_cast<double>(b.a[i].x), static_cast<double>(b.a[i].y), ar4[i & 3],
                          ai4[i & 3]);
      };
      load(0, b0);
      for (uint32_t e0 = 0; e0 < n; e0 += 2 * G) {
        if (e0 + G < n) load(e0 + G, b1);
        eval(b0);
        if (e0 + G >= n) break;
        if (e0 + 2 * G < n) load(e0 + 2 * G, b0);
        eval(b1);
      }
    }
  }
  // pass A: the simple classes (runs of consecutive ones).  A batch takes
  // whole runs, or pieces of a long run, while their uniques fit in LDS and
  // their classes in the list; each piece is folded at a running offset, the
  // valid source rows of the batch are listed (in class order) and gathered
  // kGather at a time, so the row loads overlap.  This pass runs before the
  // move cache below exists, leaving registers for the loads in flight.
  if (P.alist_off == nullptr) {
    uint32_t r = 0;
    uint32_t c = P.n_runs ? P.runs[0] : 0u;
    while (r < P.n_runs) {
      __syncthreads();  // the previous batch's list and folds are consumed
      uint32_t n_list = 0, fo = 0;
      while (r < P.n_runs) {
        const uint32_t c_end = P.runs[2 * r + 1];
        const uint32_t ua = P.meta[c].ua;
        // the rest of the run if it fits what is left, else its longest piece that does
        uint32_t ce = c_end;
        if (fo + (P.meta[c_end - 1].u_end - ua) > f_cap || n_list + (c_end - c) + kGather - 1 > P.list_cap) {
          ce = c;
          while (ce < c_end && fo + (P.meta[ce].u_end - ua) <= f_cap &&
                 n_list + (ce - c + 1) + kGather - 1 <= P.list_cap)
            ++ce;
        }
        if (ce == c) break;  // nothing fits: close the batch
        const uint32_t ub = P.meta[ce - 1].u_end;
        fold_uniques<REALC>(P, ua, ub, ta, s_F + fo, s_Fz + fo);
        n_list = append_valid_rows<R16>(P, c, ce, ua - fo, ta, s_rank, s_list, s_wcnt, n_list);
        fo += ub - ua;
        c = ce;
        if (c == c_end && ++r < P.n_runs) c = P.runs[2 * r];
      }
      // pad to a multiple of kGather with entries that read row 0 against a zero slot
      const uint32_t padded = (n_list + kGather - 1u) / kGather * kGather;
      if (threadIdx.x < padded - n_list) s_list[n_list + threadIdx.x] = make_uint2(0u, f_cap | (1u << 16) | 0x80000000u);
      __syncthreads();
      for (uint32_t e0 = 0; e0 < padded; e0 += kGather) {
        uint32_t rk[kGather], w[kGather];
        double a_r[kGather], a_i[kGather];
#pragma unroll
        for (int i = 0; i < kGather; ++i) {
          const uint2 L = s_list[e0 + i];
          rk[i] = __builtin_amdgcn_readfirstlane(L.x);
          w[i] = __builtin_amdgcn_readfirstlane(L.y);
        }
#pragma unroll
        for (int i = 0; i < kGather; ++i) ld_amp<T>(psi + static_cast<uint64_t>(rk[i]) * db, colc, a_r[i], a_i[i]);
#pragma unroll
        for (int i = 0; i < kGather; ++i) {
          V f = C::zero();
          if (w[i] >> 31)
            f = s_F[w[i] & 0xffffu];
          else
            phase_sum_lds<REALC>(s_F, s_Fz, w[i] & 0xffffu, (w[i] >> 16) & 0x7fffu, tb, f);
          C::mac(f, a_r[i], a_i[i], ar4[i & 3], ai4[i & 3]);
        }
      }
    }
  }

  // pass Q: with factor tables, the whole X_alpha = 0 class (first of the
  // other classes; its source row is the target row): row staged, factors
  // folded, then its X_beta = 0 group through its F rows and its pair and
  // quad groups through the single- and double-move tables.  It runs before
  // the move cache below takes its registers, and pass B skips the class.
  if constexpr (REALC && ROWLDS) {
    if (P.fact && P.f_c0 != 0xffffffffu) {  // the class is then absent from ns_list
      const ClassMeta M = ld_meta(P.meta + P.f_c0);
      const T* rowg = psi + ia * db;
      const bool stage = P.row_lds != 0;
      const uint32_t* cf = reinterpret_cast<const uint32_t*>(P.cls_f + P.f_c0);
      const uint32_t fz_fu0 = ldc(cf), fz_r = (P.fact & kFactZero) ? ldc(cf + 1) : 0u;
      const uint64_t fz_off = ldc(cf + 2) | (static_cast<uint64_t>(ldc(cf + 3)) << 32);
      double* s_Fd = reinterpret_cast<double*>(smem + P.off_f);
      double* s_A = reinterpret_cast<double*>(smem + P.off_a);
      constexpr uint32_t kZv = 16;  // F rows of the X_beta = 0 group loaded before the folds
      double zv[kZv];
#pragma unroll
      for (uint32_t r = 0; r < kZv; ++r) zv[r] = r < fz_r ? P.fz[fz_off + r * db + colc] : 0.0;
      __syncthreads();  // pass A's list and folds are consumed
      const bool stager = stage && threadIdx.x < kSB / 2;
      const uint32_t lane0 = stage ? threadIdx.x % (kSB / 2) : threadIdx.x;
      const uint32_t stride = stage ? kSB / 2 : kSB;
      if (stager) {
        stage_row<T>(s_row, rowg, db, lane0, stride);
      } else {
        if (lane0 < kFactZeroSlots) s_Fd[lane0] = 0.0;
        fold_factors(P, P.f_c0_fu0, P.f_c0_fq, P.f_tp, ta, s_Fd + kFactZeroSlots, lane0, stride);
        fold_factors(P, P.f_c0_fq, P.f_c0_fu1, P.f_tq, ta, s_Fd + kFactZeroSlots + (P.f_c0_fq - P.f_c0_fu0), lane0,
                     stride);
        if (fz_r) fold_factors(P, fz_fu0, fz_fu0 + fz_r, P.f_tz, ta, s_A, lane0, stride);
      }
      __syncthreads();
      if (M.zg >= 0) {
        double f = 0.0;
        if (fz_r) {
#pragma unroll
          for (uint32_t r = 0; r < kZv; ++r) f = fma(s_A[r < fz_r ? r : 0], zv[r], f);  // zv[r] = 0 past fz_r
          const double* fr = P.fz + fz_off + colc;
          for (uint32_t r = kZv; r < fz_r; ++r) f = fma(s_A[r], fr[r * db], f);
        } else {
          phase_sum_direct<true>(P, static_cast<uint32_t>(M.zg), ta, tb, f);
        }
        double a_r, a_i;
        if (ROWLDS)
          ld_amp<T>(s_row, colc, a_r, a_i);
        else
          ld_amp<T>(rowg, colc, a_r, a_i);
        Coef<true>::mac(f, a_r, a_i, ar4[0], ai4[0]);
      }
      if (P.f_r2 == 1)
        fact_table_moves<1, T, ROWLDS>(smem, s_Fd, rowg, P.n_moves, P.em, P.fp, db, colc, ar4, ai4);
      else
        fact_table_moves<2, T, ROWLDS>(smem, s_Fd, rowg, P.n_moves, P.em, P.fp, db, colc, ar4, ai4);
      if (P.f_r3 == 1)
        fact_table_moves<1, T, ROWLDS>(smem, s_Fd, rowg, P.f_n_qmoves, P.eq, P.fq, db, colc, ar4, ai4);
      else
        fact_table_moves<2, T, ROWLDS>(smem, s_Fd, rowg, P.f_n_qmoves, P.eq, P.fq, db, colc, ar4, ai4);
      // groups beyond the quads (none for two-body operators) are scanned
      uint32_t gs = M.q1;
      while (gs < M.g1) {
        const uint32_t xb = P.pg_xb[gs];
        const bool valid = live && 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
        if (valid) {
          double f = 0.0;
          phase_sum_direct<true>(P, gs, ta, tb, f);
          double a_r, a_i;
          ld_amp<T>(rowg, rank_of<R16>(tb ^ xb, P, s_rank), a_r, a_i);
          Coef<true>::mac(f, a_r, a_i, ar4[1], ai4[1]);
        }
        ++gs;
      }
    }
  }

  // Pair moves of this lane's target (occupied p -> empty q), occupied-major,
  // packed as: bits 0-15 the source column (its LDS byte offset in the staged
  // row when rows are staged), bits 16-27 the pair-map byte offset 8 pair(p, q),
  // bit 31 the move's beta parity popcount(zpair & t_b) when cached.
  uint32_t mv[kMaxMoves];
  // padding moves point at map entry n_pairs (a zero slot) and column 0
  const uint32_t pad_move = (8u * P.n_pairs) << 16;
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
        const uint32_t src = rank_of<R16>(tb ^ (1u << p) ^ (1u << q), P, s_rank);
        const uint32_t par =
            P.pair_sign ? (static_cast<uint32_t>(__popc(lds_ld<uint32_t>(kPuOff + 4u * pair) & tb)) & 1u) : 0u;
        mv[k] = (ROWLDS ? src * static_cast<uint32_t>(sizeof(T)) : src) | ((8u * pair) << 16) | (par << 31);
        if (++j == ne) {
          j = 0;
          pm_emp = emp;
          pm_occ &= pm_occ - 1;
          p = __ffs(pm_occ) - 1;
        }
      }
    }
  }

  // pass B through the alpha images: for each image class of this row (in
  // class order) the source row is staged while the other half of the
  // workgroup copies the class's precomputed image -- the folded pair-group
  // coefficient per orbital pair and the X_beta = 0 group's factors -- into
  // the pair-map region, so each cached move reads its coefficient directly
  // (staged rows only)
  if constexpr (REALC && ROWLDS) {
    if (P.plist_off != nullptr) {
      const uint32_t b0 = ldc(P.plist_off + ia), b1 = ldc(P.plist_off + ia + 1);
      uint32_t n_moves = __builtin_amdgcn_readfirstlane(P.n_moves);
      const uint32_t n_img = P.n_img, n_pairs = P.n_pairs;
      const double* s_Af = reinterpret_cast<const double*>(smem + P.off_a);
      // every lane stages part of the row; lane j < n_img also holds image
      // element j of the next class, loaded while the current class is
      // evaluated
      const uint32_t lane0 = threadIdx.x;
      double imv = (b1 > b0 && lane0 < n_img) ? P.pimg[static_cast<uint64_t>(b0) * n_img + lane0] : 0.0;
      for (uint32_t k = b0; k < b1; ++k) {
        const uint32_t src = ldc(P.plist_src + k), cid = ldc(P.plist_cls + k);
        const uint32_t* cf = reinterpret_cast<const uint32_t*>(P.cls_f + cid);
        const uint32_t fz_r = ldc(cf + 1);
        const uint64_t fz_off = ldc(cf + 2) | (static_cast<uint64_t>(ldc(cf + 3)) << 32);
        const double zv0 = fz_r > 0 ? P.fz[fz_off + colc] : 0.0;
        const double zv1 = fz_r > 1 ? P.fz[fz_off + db + colc] : 0.0;
        const T* rowg = psi + static_cast<uint64_t>(src) * db;
        __syncthreads();
        stage_row<T>(s_row, rowg, db, lane0, kSB);
        {
          const double* im = P.pimg + static_cast<uint64_t>(k) * n_img;
          for (uint32_t j = lane0; j < n_img; j += kSB) {
            const uint32_t at = j <= n_pairs ? kPuOff + 8u * j : P.off_a + 8u * (j - n_pairs - 1u);
            *reinterpret_cast<double*>(smem + at) = j == lane0 ? imv : im[j];
          }
          if (k + 1 < b1 && lane0 < n_img) imv = im[n_img + lane0];
        }
        __syncthreads();
        if (fz_r) {
          const double f = fma(s_Af[0], zv0, s_Af[1] * zv1);
          double a_r, a_i;
          if (ROWLDS)
            ld_amp<T>(s_row, colc, a_r, a_i);
          else
            ld_amp<T>(rowg, colc, a_r, a_i);
          Coef<true>::mac(f, a_r, a_i, ar4[0], ai4[0]);
        }
        uint32_t o16 = 16u, o0 = 0u;
        asm volatile("" : "+s"(o16), "+s"(o0));
#pragma unroll
        for (int k0 = 0; k0 < kMaxMoves; k0 += 4) {
          if (static_cast<uint32_t>(k0) < n_moves) {
            double f[4], a_r[4], a_i[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              f[i] = lds_ld<double>(kPuOff + __builtin_amdgcn_ubfe(mv[k0 + i], o16, 12));
              if (ROWLDS) {
                const T v = lds_ld<T>(kRowOff + __builtin_amdgcn_ubfe(mv[k0 + i], o0, 16));
                a_r[i] = static_cast<double>(v.x);
                a_i[i] = static_cast<double>(v.y);
              } else {
                move_amp<T, false>(smem, rowg, mv[k0 + i], a_r[i], a_i[i]);
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
              Coef<true>::mac(signed_by_bit31(f[i], mv[k0 + i]), a_r[i], a_i[i], ar4[i], ai4[i]);
          }
        }
      }
    }
  }

  // pass B: every other class, in class order
  for (uint32_t ic = 0; ic < P.n_ns; ++ic) {
    const uint32_t cid = P.ns_list[ic];
    const ClassMeta M = ld_meta(P.meta + cid);
    const uint32_t sa = ta ^ M.xa;
    if (static_cast<uint32_t>(__popc(sa)) != P.n_alpha) continue;
    const uint64_t rowoff = static_cast<uint64_t>(rank_of<R16>(sa, P, s_rank)) * db;
    const uint32_t gz_end = M.zg >= 0 ? M.g0 + 1 : M.g0;
    // enumerate pair moves when the class's pair groups are dense enough
    const bool penum = P.enum_ok && M.pm >= 0 && (M.u_p - M.ua) <= f_cap && 2 * (M.p1 - gz_end) >= P.n_moves;
    // single-unique pair groups whose beta parities are cached per move
    const bool single = penum && (M.flags & kClassPairsSingle) && P.pair_sign;
    const uint32_t ub_a = penum ? M.u_p : M.u_z;
    const bool fold_a = ub_a > M.ua && ub_a - M.ua <= f_cap;
    const bool stage = P.row_lds && gz_end < M.g1;
    const T* rowg = psi + rowoff;

    // phase A: X_beta = 0 group and, when enumerated, the pair groups
    if (stage || fold_a) {
      __syncthreads();
      // with a row to stage, half of the workgroup stages it while the other
      // half folds the coefficients and fills the pair map (their global
      // loads overlap); the split is by wave, so no wave diverges
      const bool split = stage && (fold_a || penum);
      const bool stager = !split || threadIdx.x < kSB / 2;
      const uint32_t lane0 = split ? threadIdx.x % (kSB / 2) : threadIdx.x;
      const uint32_t stride = split ? kSB / 2 : kSB;
      const bool folder = !split || !stager;
      if (stage && stager) stage_row<T>(s_row, rowg, db, lane0, stride);
      if (fold_a && folder) fold_uniques<REALC>(P, M.ua, ub_a, ta, s_F, s_Fz, lane0, stride);
      if (penum && folder) {
        const int32_t* pm = P.pmap + static_cast<uint64_t>(M.pm) * P.n_pairs;
        for (uint32_t q = lane0; q <= P.n_pairs; q += stride) {
          const int32_t g = q < P.n_pairs ? pm[q] : -1;  // entry n_pairs serves the padding moves
          uint32_t v;
          if (single)  // LDS byte address of the group's folded unique
            v = P.off_f + (g >= 0 ? P.pg_u0[g] - M.ua : f_cap) * static_cast<uint32_t>(sizeof(V));
          else
            v = g >= 0 ? ((P.pg_u0[g] - M.ua) | ((P.pg_u0[g + 1] - P.pg_u0[g]) << 16)) : 0u;
          s_pu[2 * q] = v;  // 8-byte slots: a move holds 8 pair(p, q) << 16
        }
      }
      __syncthreads();
    }
    if (M.zg >= 0) {
      V f = C::zero();
      if (fold_a)
        phase_sum_lds<REALC>(s_F, s_Fz, 0, M.u_z - M.ua, tb, f);
      else
        phase_sum_direct<REALC>(P, static_cast<uint32_t>(M.zg), ta, tb, f);
      double a_r, a_i;
      if (ROWLDS && stage)
        ld_amp<T>(s_row, colc, a_r, a_i);
      else
        ld_amp<T>(rowg, colc, a_r, a_i);
      C::mac(f, a_r, a_i, ar4[0], ai4[0]);
    }
    const T* rowp = ROWLDS ? s_row : rowg;  // pair and scanned groups need the staged row
    if (penum) {
      uint32_t n_moves = __builtin_amdgcn_readfirstlane(P.n_moves);
      asm volatile("" : "+s"(n_moves));  // keep the move predicates inside the class loop
      if (single) {
        // straight-line groups of four moves: one unique per pair group; absent
        // groups and padding moves hit the zero slot, so loads issue together
        // The field offsets are opaque scalars redefined per class, so the
        // per-move bit-field extracts stay inside the class loop (hoisting
        // them would need 2 registers per cached move) at one VALU each.
        uint32_t o16 = 16u, o0 = 0u;
        asm volatile("" : "+s"(o16), "+s"(o0));
#pragma unroll
        for (int k0 = 0; k0 < kMaxMoves; k0 += 4) {
          if (static_cast<uint32_t>(k0) < n_moves) {
            uint32_t fa[4];
            V f[4];
            double a_r[4], a_i[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fa[i] = lds_ld<uint32_t>(kPuOff + __builtin_amdgcn_ubfe(mv[k0 + i], o16, 12));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              f[i] = lds_ld<V>(fa[i]);
              if (ROWLDS) {
                const T v = lds_ld<T>(kRowOff + __builtin_amdgcn_ubfe(mv[k0 + i], o0, 16));
                a_r[i] = static_cast<double>(v.x);
                a_i[i] = static_cast<double>(v.y);
              } else {
                Amp<T>::load(rowg, __builtin_amdgcn_ubfe(mv[k0 + i], o0, 16), a_r[i], a_i[i]);
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) C::mac(C::sign31(f[i], mv[k0 + i]), a_r[i], a_i[i], ar4[i], ai4[i]);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < kMaxMoves; ++k) {
          if (static_cast<uint32_t>(k) < n_moves) {
            uint32_t e = mv[k];
            asm volatile("" : "+v"(e));
            const uint32_t w = *reinterpret_cast<const uint32_t*>(smem + kPuOff + ((e >> 16) & 0xfffu));
            V f = C::zero();
            phase_sum_lds<REALC>(s_F, s_Fz, w & 0xffffu, w >> 16, tb, f);
            double a_r, a_i;
            move_amp<T, ROWLDS>(smem, rowg, e, a_r, a_i);
            C::mac(f, a_r, a_i, ar4[k & 3], ai4[k & 3]);
          }
        }
      }
    }

    // phase Q: groups whose X_beta flips four orbitals, by enumerating the
    // lane's valid double moves against a per-class quad map
    const bool qenum = penum && P.qenum_ok && M.qm >= 0 && M.u_q - M.u_p <= f_cap &&
                       2 * (M.q1 - M.p1) >= P.n_qmoves;
    if (qenum) {
      __syncthreads();
      fold_uniques<REALC>(P, M.u_p, M.u_q, ta, s_F, s_Fz);
      const int32_t* qm = P.qmap + static_cast<uint64_t>(M.qm) * P.n_quads;
      for (uint32_t q = threadIdx.x; q < P.n_quads; q += kSB) {
        const int32_t g = qm[q];
        s_qu[q] = g >= 0 ? ((P.pg_u0[g] - M.u_p) | ((P.pg_u0[g + 1] - P.pg_u0[g]) << 16)) : (f_cap | (1u << 16));
        // with a uniform count, absent groups read that many zero slots
      }
      __syncthreads();
      if (P.quad_cnt == 3)
        quad_moves<3, R16, REALC>(P, tb, s_rank, s_F, s_Fz, s_qu, rowp, ar4, ai4);
      else
        quad_moves<0, R16, REALC>(P, tb, s_rank, s_F, s_Fz, s_qu, rowp, ar4, ai4);
    }

    // phase B: remaining groups, scanned in chunks whose uniques fit in LDS;
    // invalid targets are predicated off (source index clamped, coefficient 0)
    uint32_t gs = qenum ? M.q1 : (penum ? M.p1 : gz_end);
    while (gs < M.g1) {
      const uint32_t us = ldc(P.pg_u0 + gs);
      uint32_t ge = gs;
      while (ge < M.g1 && ldc(P.pg_u0 + ge + 1) - us <= f_cap) ++ge;
      if (ge == gs) {
        const uint32_t xb = P.pg_xb[gs];
        const bool valid = live && 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
        if (valid) {
          V f = C::zero();
          phase_sum_direct<REALC>(P, gs, ta, tb, f);
          double a_r, a_i;
          ld_amp<T>(rowp, rank_of<R16>(tb ^ xb, P, s_rank), a_r, a_i);
          C::mac(f, a_r, a_i, ar4[1], ai4[1]);
        }
        ++gs;
        continue;
      }
      __syncthreads();
      fold_uniques<REALC>(P, us, P.pg_u0[ge], ta, s_F, s_Fz);
      __syncthreads();
      uint32_t g = gs;
      for (; g + 3 < ge; g += 4) {  // four source loads in flight
        uint32_t jb[4];
        V f[4];
        double a_r[4], a_i[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) scan_prepare<R16, REALC>(P, g + i, us, tb, s_rank, s_F, s_Fz, jb[i], f[i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) ld_amp<T>(rowp, jb[i], a_r[i], a_i[i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) C::mac(f[i], a_r[i], a_i[i], ar4[i], ai4[i]);
      }
      for (; g < ge; ++g) scan_group<R16, REALC>(P, g, us, tb, s_rank, s_F, s_Fz, rowp, ar4[2], ai4[2]);
      gs = ge;
    }
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
  if (EXPVAL) block_reduce3_store<kSB>(e_re, e_im, nrm, slot, s_red);
}

// Order of the workgroups.  With source rows staged in LDS, workgroup b
// takes row b mod dim_alpha and column chunk b / dim_alpha, so the
// workgroups in flight share one column chunk across many rows (measured
// best on the 28-qubit sector).  Without staging, pair-move gathers read
// the source row through L2, so the chunks of one row run back to back on
// one XCD (workgroup b runs on XCD b mod 8): rows are dealt to the XCDs in
// groups of eight, and rows past the last full group take row-major order.
constexpr uint32_t kXcds = 8;
__device__ inline void row_chunk_of(uint32_t b, uint32_t rows, uint32_t chunks, bool row_fast, uint32_t& row,
                                    uint32_t& chunk) {
  if (row_fast) {
    row = b % rows;
    chunk = b / rows;
    return;
  }
  const uint32_t grouped = rows / kXcds * kXcds;
  const uint32_t full = grouped * chunks;
  if (b < full) {
    const uint32_t x = b % kXcds, j = b / kXcds;
    row = j / chunks * kXcds + x;
    chunk = j % chunks;
  } else {
    const uint32_t r = b - full;
    row = grouped + r / chunks;
    chunk = r % chunks;
  }
}

// Rows kernel: one workgroup per alpha row and all of its beta columns, for
// operators whose simple classes come through alpha lists and whose other
// classes' uniques and group records all fit in LDS (few groups, rows too
// long to stage: the 32-qubit Hubbard sector).  Everything the row needs --
// rank tables, the row's alpha list, every valid class's source row, folded
// uniques and group records -- is loaded once; the row's columns are then
// swept chunk by chunk with no barrier, so waves run independently.
// LDS: [0, 256) scratch, then rank tables, the list (source ranks, then
// coefficients), valid classes (source row rank, first and end group
// record), group records (X_beta, first unique | count << 16), folded
// uniques and their beta Z-masks, and for the fused energy pass three
// float64 sums per thread; offsets in RowsLayout.
struct RowsLayout {
  uint32_t off_rank, off_lsrc, off_lc, off_cls, off_grp, off_f, off_fz, off_e;
};

template <class T, bool EXPVAL>
__global__ __launch_bounds__(kSB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 8 : 1, 8))) void k_apply_rows(SectorArgs P, RowsLayout Lr, const T* __restrict__ psi,
                                                    T* __restrict__ out, double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t ia = blockIdx.x + P.row_begin;
  const uint64_t db = P.dim_beta;
  uint16_t* s_rank = reinterpret_cast<uint16_t*>(smem + Lr.off_rank);
  uint32_t* s_lsrc = reinterpret_cast<uint32_t*>(smem + Lr.off_lsrc);
  double* s_lc = reinterpret_cast<double*>(smem + Lr.off_lc);
  uint4* s_cls = reinterpret_cast<uint4*>(smem + Lr.off_cls);
  uint2* s_grp = reinterpret_cast<uint2*>(smem + Lr.off_grp);
  double* s_F = reinterpret_cast<double*>(smem + Lr.off_f);
  uint32_t* s_Fz = reinterpret_cast<uint32_t*>(smem + Lr.off_fz);
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(smem);  // [0]: valid classes, [1]: groups, [2]: uniques
  {  // rank tables (n_orb <= 16), as in the sector kernel
    constexpr uint32_t kWords = kRank16Lds / 2u;
    const uint32_t* r0 = reinterpret_cast<const uint32_t*>(P.rank16);
    const uint32_t* r1 = reinterpret_cast<const uint32_t*>(P.rank16 + (P.n_orb + 1) * 256u);
    uint32_t* s_rank32 = reinterpret_cast<uint32_t*>(s_rank);
    for (uint32_t w = threadIdx.x; w < kWords; w += kSB)
      s_rank32[w] = w < 128u ? r0[w] : (P.n_chunks > 1 ? r1[w - 128u] : 0u);
  }
  const uint32_t ta = P.str_a[ia];
  const uint32_t a0 = ldc(P.alist_off + ia), a1 = ldc(P.alist_off + ia + 1);
  for (uint32_t j = threadIdx.x; j < a1 - a0; j += kSB) {
    s_lsrc[j] = P.alist_src[a0 + j];
    s_lc[j] = P.alist_c[a0 + j];
  }
  // valid classes and their group records (thread 0 walks the classes; few)
  if (threadIdx.x == 0) {
    uint32_t nc = 0, ng = 0, nu = 0;
    for (uint32_t ic = 0; ic < P.n_ns; ++ic) {
      const ClassMeta* m = P.meta + P.ns_list[ic];
      const uint32_t sa = ta ^ m->xa;
      if (static_cast<uint32_t>(__popc(sa)) != P.n_alpha) continue;
      uint32_t r = 0, below = 0;  // rank of the source alpha string
      for (uint32_t c = 0; c < P.n_chunks; ++c) {
        const uint32_t byte = (sa >> (8 * c)) & 255u;
        r += P.rank16[(c * (P.n_orb + 1) + below) * 256 + byte];
        below += __popc(byte);
      }
      s_cls[nc++] = make_uint4(r, ng, ng + (m->g1 - m->g0), nu);
      for (uint32_t g = m->g0; g < m->g1; ++g) {
        const uint32_t u0 = P.pg_u0[g], u1 = P.pg_u0[g + 1];
        s_grp[ng++] = make_uint2(P.pg_xb[g], (nu + (u0 - m->ua)) | ((u1 - u0) << 16));
      }
      nu += m->u_end - m->ua;
    }
    s_cnt[0] = nc;
    s_cnt[1] = ng;
    s_cnt[2] = nu;
  }
  __syncthreads();
  const uint32_t n_cls = s_cnt[0];
  {  // fold every valid class's uniques at the class's offset
    uint32_t nu = 0;
    for (uint32_t ic = 0; ic < P.n_ns; ++ic) {
      const ClassMeta M = ld_meta(P.meta + P.ns_list[ic]);
      if (static_cast<uint32_t>(__popc(ta ^ M.xa)) != P.n_alpha) continue;
      fold_uniques<true>(P, M.ua, M.u_end, ta, s_F + nu, s_Fz + nu);
      nu += M.u_end - M.ua;
    }
  }
  __syncthreads();

  const uint32_t chunks = static_cast<uint32_t>((db + kSB - 1) / kSB);
  const uint32_t n_list = a1 - a0;
  // the energy sums live in LDS (one slot per thread, volatile so they are
  // not promoted back to registers): three doubles held across the sweep
  // would push the kernel past 64 VGPRs and cost a quarter of its waves
  volatile double* s_e = reinterpret_cast<volatile double*>(smem + Lr.off_e);
  if (EXPVAL) {
    s_e[threadIdx.x] = 0.0;
    s_e[kSB + threadIdx.x] = 0.0;
    s_e[2 * kSB + threadIdx.x] = 0.0;
  }
  for (uint32_t ch = 0; ch < chunks; ++ch) {
    const uint32_t col = ch * kSB + threadIdx.x;
    const bool live = col < db;
    const uint32_t colc = live ? col : 0u;
    const uint32_t tb = P.str_b[colc];
    double ar4[4] = {0.0, 0.0, 0.0, 0.0}, ai4[4] = {0.0, 0.0, 0.0, 0.0};
    const T* psi_col = psi + colc;
    // simple classes: the row's list, eight gathers in flight
    for (uint32_t e0 = 0; e0 < n_list; e0 += 8) {
      double c[8];
      T a[8];
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i) {
        const uint32_t m = min(e0 + i, n_list - 1u);
        c[i] = e0 + i < n_list ? s_lc[m] : 0.0;
        a[i] = psi_col[static_cast<uint64_t>(s_lsrc[m]) * db];
      }
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i)
        Coef<true>::mac(c[i], static_cast<double>(a[i].x), static_cast<double>(a[i].y), ar4[i & 3], ai4[i & 3]);
    }
    // other classes: every group, four gathers in flight
    for (uint32_t c = 0; c < n_cls; ++c) {
      const uint4 C = s_cls[c];
      const T* rowp = psi + static_cast<uint64_t>(C.x) * db;
      for (uint32_t g0 = C.y; g0 < C.z; g0 += 4) {
        uint32_t jb[4];
        double f[4], a_r[4], a_i[4];
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
          const uint32_t g = min(g0 + i, C.z - 1u);
          const uint2 R = s_grp[g];
          const uint32_t xb = R.x;
          const bool valid = g0 + i < C.z && 2u * __popc(tb & xb) == static_cast<uint32_t>(__popc(xb));
          jb[i] = valid ? rank_of<true>(tb ^ xb, P, s_rank) : 0u;
          double h = 0.0;
          phase_sum_lds<true>(s_F, s_Fz, R.y & 0xffffu, R.y >> 16, tb, h);
          f[i] = valid ? h : 0.0;
        }
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) ld_amp<T>(rowp, jb[i], a_r[i], a_i[i]);
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) Coef<true>::mac(f[i], a_r[i], a_i[i], ar4[i], ai4[i]);
      }
    }
    const double acc_r = (ar4[0] + ar4[1]) + (ar4[2] + ar4[3]);
    const double acc_i = (ai4[0] + ai4[1]) + (ai4[2] + ai4[3]);
    if (live) {
      const uint64_t t = static_cast<uint64_t>(ia) * db + col;
      if (EXPVAL) {
        double pr, pi;
        Amp<T>::load(psi, t, pr, pi);
        s_e[threadIdx.x] = fma(pr, acc_r, fma(pi, acc_i, s_e[threadIdx.x]));
        s_e[kSB + threadIdx.x] = fma(pr, acc_i, fma(-pi, acc_r, s_e[kSB + threadIdx.x]));
        s_e[2 * kSB + threadIdx.x] = fma(pr, pr, fma(pi, pi, s_e[2 * kSB + threadIdx.x]));
        if (out) Amp<T>::store(out, t, acc_r, acc_i);
      } else {
        Amp<T>::store(out, t, acc_r, acc_i);
      }
    }
  }
  if (EXPVAL)
    block_reduce3_store<kSB>(s_e[threadIdx.x], s_e[kSB + threadIdx.x], s_e[2 * kSB + threadIdx.x],
                             partial + 3ull * blockIdx.x, reinterpret_cast<double(*)[kSB / 64]>(smem + 64));
}

// One-dimensional grid of rows * chunks workgroups for target rows
// [row_begin, row_begin + rows) (all rows unless a row range is asked for).
template <class T, bool EXPVAL, bool R16, bool ROWLDS, bool REALC>
__global__ __launch_bounds__(kSB) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_apply_sector(
    SectorArgs P, const T* __restrict__ psi, T* __restrict__ out, double* __restrict__ partial) {
  const uint32_t chunks = (P.dim_beta + kSB - 1) / kSB;
  uint32_t row, chunk;
  row_chunk_of(blockIdx.x, gridDim.x / chunks, chunks, P.row_lds != 0, row, chunk);
  sector_body<T, EXPVAL, R16, ROWLDS, REALC>(P, psi, out, partial + 3ull * blockIdx.x, row + P.row_begin, chunk);
}

// A job of a batched launch: one operator on one sector state.
struct BatchJob {
  SectorArgs args;
  const void* psi;
  void* out;
  uint32_t block_base;  // first workgroup of the job
  uint32_t chunks;      // beta-column chunks per row
  uint32_t slot;        // the job's position in the caller's list (energies go there)
  uint32_t rows;        // alpha rows
  uint32_t order;       // workgroup -> (row, chunk): kOrderPlain, kOrderRowFast or kOrderXcdRows
  uint32_t pad;
};
constexpr uint32_t kOrderPlain = 0, kOrderRowFast = 1, kOrderXcdRows = 2;

// All jobs of a batch in one launch: work item w (one alpha row and column
// chunk of one job) belongs to the job with the largest block_base <= w
// (jobs are stored in block order, largest first by default).  With a grid
// of one workgroup per item each workgroup takes one item; a persistent
// launch has as many workgroups as fit on the device at once, and
// workgroup i walks items i, i + grid, i + 2 grid, ... of that static list
// (no atomics: the schedule is fixed by the grid size).
template <class T, bool EXPVAL, bool R16, bool ROWLDS, bool REALC>
__global__ __launch_bounds__(kSB) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_apply_sector_batch(
    const BatchJob* __restrict__ jobs, uint32_t n_jobs, uint32_t n_items, double* __restrict__ partial) {
  for (uint32_t w = blockIdx.x; w < n_items; w += gridDim.x) {
    if (w != blockIdx.x) __syncthreads();  // the previous item is done with LDS
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (ldc(&jobs[mid].block_base) <= w)
        lo = mid;
      else
        hi = mid;
    }
    // fields are read from the (read-only) job table where they are used, so
    // the record is not held in registers for the whole kernel
    const BatchJob& J = jobs[lo];
    const uint32_t b = w - J.block_base;
    // a row's chunks share b mod 8 under kOrderXcdRows, hence one XCD whatever
    // the job's first workgroup
    uint32_t row = b / J.chunks, chunk = b % J.chunks;
    if (J.order != kOrderPlain) row_chunk_of(b, J.rows, J.chunks, J.order == kOrderRowFast, row, chunk);
    sector_body<T, EXPVAL, R16, ROWLDS, REALC>(J.args, static_cast<const T*>(J.psi), static_cast<T*>(J.out),
                                               partial + 3ull * w, row, chunk);
  }
}

// Address of one sector kernel variant (single launch or batch).
template <class T, bool EXPVAL, bool R16, bool ROWLDS, bool REALC>
void* sector_variant(bool batch) {
  return batch ? reinterpret_cast<void*>(k_apply_sector_batch<T, EXPVAL, R16, ROWLDS, REALC>)
               : reinterpret_cast<void*>(k_apply_sector<T, EXPVAL, R16, ROWLDS, REALC>);
}

template <class T, bool EXPVAL>
void* sector_variants(bool batch, bool r16, bool rowlds, bool realc) {
  if (r16) {
    if (rowlds) return realc ? sector_variant<T, EXPVAL, true, true, true>(batch)
                             : sector_variant<T, EXPVAL, true, true, false>(batch);
    return realc ? sector_variant<T, EXPVAL, true, false, true>(batch)
                 : sector_variant<T, EXPVAL, true, false, false>(batch);
  }
  if (rowlds) return realc ? sector_variant<T, EXPVAL, false, true, true>(batch)
                           : sector_variant<T, EXPVAL, false, true, false>(batch);
  return realc ? sector_variant<T, EXPVAL, false, false, true>(batch)
               : sector_variant<T, EXPVAL, false, false, false>(batch);
}

}  // namespace

// Each is defined in its own translation unit (sector_<storage>_<mode>.hip)
// so the variants compile in parallel.
void* sector_kernel_c64_apply(bool batch, bool r16, bool rowlds, bool realc);
void* sector_kernel_c64_expval(bool batch, bool r16, bool rowlds, bool realc);
void* sector_kernel_c128_apply(bool batch, bool r16, bool rowlds, bool realc);
void* sector_kernel_c128_expval(bool batch, bool r16, bool rowlds, bool realc);

inline void* sector_kernel(pbs_dtype dt, bool expval, bool batch, bool r16, bool rowlds, bool realc) {
  if (dt == PBS_C128)
    return expval ? sector_kernel_c128_expval(batch, r16, rowlds, realc)
                  : sector_kernel_c128_apply(batch, r16, rowlds, realc);
  return expval ? sector_kernel_c64_expval(batch, r16, rowlds, realc)
                : sector_kernel_c64_apply(batch, r16, rowlds, realc);
}

}  // namespace pbs
