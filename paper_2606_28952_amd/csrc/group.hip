// Grouping of a canonical Pauli sum by X-mask (Section 2.4,
// Eq. topological_group) and the tables of the spin-sector kernel.
#include "handles.h"

namespace pbs {
namespace {

__global__ void k_x_heads(const uint64_t* x, uint64_t m, uint32_t* heads) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    heads[i] = (i == 0 || x[i] != x[i - 1]) ? 1u : 0u;
}

// CSR fill: group masks and offsets from heads; XZ-form coefficients
// C_k = c_k * i^popcount(x_k & z_k) (Section 2.3).
__global__ void k_csr_fill(const uint64_t* x, const uint64_t* z, const double* c, uint64_t m, const uint32_t* heads,
                           const uint32_t* gid, uint64_t* xg, uint32_t* off, uint64_t* zk, double* ck) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (heads[i]) {
      xg[gid[i]] = x[i];
      off[gid[i]] = static_cast<uint32_t>(i);
    }
    zk[i] = z[i];
    const uint32_t y = static_cast<uint32_t>(__popcll(x[i] & z[i])) & 3u;
    const double r = c[2 * i], im = c[2 * i + 1];
    double a = r, b = im;
    if (y == 1) { a = -im; b = r; }
    else if (y == 2) { a = -r; b = -im; }
    else if (y == 3) { a = im; b = -r; }
    ck[2 * i] = a + 0.0;  // exact zeros written as +0.0
    ck[2 * i + 1] = b + 0.0;
  }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

// Sector rewrite of every term: alive flag, sort keys and signed coefficient
// (the exact rewrites listed with pbs_grouped).  Keys, most significant word
// first: (X_alpha << 6 | popcount(X_beta)), (X_beta << 32 | z_beta'), z_alpha.
__global__ void k_sector_terms(const uint64_t* x, const uint64_t* zk, const double* ck, uint64_t m, uint32_t h,
                               uint32_t* alive, uint64_t* k2, uint64_t* k1, uint64_t* k0, double* cre,
                               double* cim) {
  const uint64_t mask = (h == 32) ? 0xffffffffull : ((1ull << h) - 1ull);
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t xa = x[i] & mask, xb = (x[i] >> h) & mask;
    const uint64_t za = zk[i] & mask;
    uint64_t zb = (zk[i] >> h) & mask;
    const uint32_t pa = __popcll(xa), pb = __popcll(xb);
    alive[i] = ((pa & 1u) == 0 && (pb & 1u) == 0) ? 1u : 0u;
    uint32_t flips = 0;
    if (xb != 0 && (zb & (xb & (~xb + 1ull)))) {
      zb ^= xb;
      flips += pb >> 1;
    }
    flips += __popcll(zb & xb) + __popcll(za & xa);
    const double sgn = (flips & 1u) ? -1.0 : 1.0;
    k2[i] = (xa << 6) | pb;
    k1[i] = (xb << 32) | zb;
    k0[i] = za;
    cre[i] = sgn * ck[2 * i];
    cim[i] = sgn * ck[2 * i + 1];
  }
}

__global__ void k_compact_alive(const uint32_t* alive, const uint32_t* pos, uint64_t m, const uint64_t* k2,
                                const uint64_t* k1, const uint64_t* k0, uint64_t* keys_soa, uint64_t ma) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (!alive[i]) continue;
    const uint64_t o = pos[i];
    keys_soa[o] = k0[i];
    keys_soa[ma + o] = k1[i];
    keys_soa[2 * ma + o] = k2[i];
  }
}

__global__ void k_alive_index(const uint32_t* alive, const uint32_t* pos, uint64_t m, uint32_t* src) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (alive[i]) src[pos[i]] = static_cast<uint32_t>(i);
}

// Heads of classes (X_alpha), plan groups (X_alpha, X_beta) and uniques
// (X_alpha, X_beta, z_beta') over the sorted alive terms.
__global__ void k_plan_heads(const uint64_t* keys_soa, uint64_t ma, uint32_t* hc, uint32_t* hg, uint32_t* hu) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < ma;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t w2 = keys_soa[2 * ma + i], w1 = keys_soa[ma + i];
    if (i == 0) {
      hc[i] = hg[i] = hu[i] = 1u;
      continue;
    }
    const uint64_t p2 = keys_soa[2 * ma + i - 1], p1 = keys_soa[ma + i - 1];
    const bool c = (w2 >> 6) != (p2 >> 6);
    const bool g = c || (w1 >> 32) != (p1 >> 32);
    hc[i] = c ? 1u : 0u;
    hg[i] = g ? 1u : 0u;
    hu[i] = (g || w1 != p1) ? 1u : 0u;
  }
}

__global__ void k_plan_fill(const uint64_t* keys_soa, uint64_t ma, const uint32_t* order, const uint32_t* src,
                            const double* cre, const double* cim, const uint32_t* hc, const uint32_t* hg,
                            const uint32_t* hu, const uint32_t* cid, const uint32_t* gid, const uint32_t* uid,
                            uint32_t* cls_xa, uint32_t* cls_g0, uint32_t* pg_xb, uint32_t* pg_pc, uint32_t* pg_u0,
                            uint32_t* u_zb, uint32_t* u_t0, uint32_t* pt_za, double* pt_c) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < ma;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t w2 = keys_soa[2 * ma + i], w1 = keys_soa[ma + i], w0 = keys_soa[i];
    if (hc[i]) {
      cls_xa[cid[i]] = static_cast<uint32_t>(w2 >> 6);
      cls_g0[cid[i]] = gid[i];
    }
    if (hg[i]) {
      pg_xb[gid[i]] = static_cast<uint32_t>(w1 >> 32);
      pg_pc[gid[i]] = static_cast<uint32_t>(w2 & 63u);
      pg_u0[gid[i]] = uid[i];
    }
    if (hu[i]) {
      u_zb[uid[i]] = static_cast<uint32_t>(w1 & 0xffffffffull);
      u_t0[uid[i]] = static_cast<uint32_t>(i);
    }
    pt_za[i] = static_cast<uint32_t>(w0);
    const uint32_t s = src[order[i]];
    pt_c[2 * i] = cre[s];
    pt_c[2 * i + 1] = cim[s];
  }
}

// Flags any coefficient with a nonzero imaginary part.
__global__ void k_any_imag(const double* c, uint64_t m, uint32_t* flag) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (c[2 * i + 1] != 0.0) atomicOr(flag, 1u);
}

// Per class: the X_beta = 0 group, the popcount-2 and popcount-4 ranges,
// and whether the class needs a pair-map and a quad-map row (flags written
// for scans).
__global__ void k_class_meta(uint32_t n_class, const uint32_t* cls_g0, const uint32_t* pg_pc, bool quads,
                             int32_t* zg, int32_t* p0, int32_t* p1, int32_t* q1, uint32_t* has_pairs,
                             uint32_t* has_quads) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_class; c += gridDim.x * blockDim.x) {
    const uint32_t g0 = cls_g0[c], g1 = cls_g0[c + 1];
    // popcounts are ascending within a class: first group with popcount >= v
    auto first_at_least = [&](uint32_t v) {
      uint32_t lo = g0, hi = g1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (pg_pc[mid] < v)
          lo = mid + 1;
        else
          hi = mid;
      }
      return lo;
    };
    const uint32_t a = first_at_least(1), b = first_at_least(3), g = first_at_least(5);
    const int32_t z = a > g0 ? static_cast<int32_t>(g0) : -1;
    zg[c] = z;
    p0[c] = static_cast<int32_t>(a);
    p1[c] = static_cast<int32_t>(b);
    q1[c] = static_cast<int32_t>(g);
    has_pairs[c] = b > a ? 1u : 0u;
    has_quads[c] = quads && g > b ? 1u : 0u;
  }
}

__device__ inline uint32_t small_binom(uint32_t n, uint32_t r) {
  if (r > n) return 0;
  uint32_t v = 1;
  for (uint32_t i = 1; i <= r; ++i) v = v * (n - r + i) / i;  // exact at every step
  return v;
}

// Quad map: the group of each popcount-4 X_beta in its class, at the
// colexicographic rank of X_beta.
// One workgroup per class, its threads over the class's quad groups.
__global__ void k_quad_map(uint32_t n_class, const int32_t* p1, const int32_t* q1, const int32_t* qm,
                           const uint32_t* pg_xb, uint32_t n_quads, int32_t* qmap) {
  for (uint32_t c = blockIdx.x; c < n_class; c += gridDim.x) {
    if (qm[c] < 0) continue;
    for (int32_t g = p1[c] + static_cast<int32_t>(threadIdx.x); g < q1[c]; g += static_cast<int32_t>(blockDim.x)) {
      uint32_t xb = pg_xb[g], id = 0;
      for (uint32_t j = 1; j <= 4; ++j) {
        const uint32_t b = __ffs(xb) - 1;
        xb &= xb - 1;
        id += small_binom(b, j);
      }
      qmap[static_cast<uint64_t>(qm[c]) * n_quads + id] = g;
    }
  }
}

__global__ void k_pair_rows(uint32_t n_class, const uint32_t* has_pairs, const uint32_t* slot, int32_t* pm) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_class; c += gridDim.x * blockDim.x)
    pm[c] = has_pairs[c] ? static_cast<int32_t>(slot[c]) : -1;
}

__global__ void k_class_pack(uint32_t n_class, const uint32_t* cls_xa, const uint32_t* cls_g0, const int32_t* zg,
                             const int32_t* p1, const int32_t* pm, const int32_t* q1, const int32_t* qm,
                             const uint32_t* pg_u0, ClassMeta* meta, uint32_t* max_quad_uniques) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_class; c += gridDim.x * blockDim.x) {
    ClassMeta m;
    m.xa = cls_xa[c];
    m.g0 = cls_g0[c];
    m.g1 = cls_g0[c + 1];
    m.zg = zg[c];
    m.p1 = static_cast<uint32_t>(p1[c]);
    m.pm = pm[c];
    const uint32_t gz_end = m.zg >= 0 ? m.g0 + 1 : m.g0;
    m.ua = pg_u0[m.g0];
    m.u_z = pg_u0[gz_end];
    m.u_p = pg_u0[m.p1];
    m.u_end = pg_u0[m.g1];
    uint32_t f = 0;
    if (m.zg >= 0 && m.g1 == m.g0 + 1 && m.u_end - m.ua <= kSimpleCap) f |= kClassSimple;
    bool single = true;
    for (uint32_t g = gz_end; g < m.p1; ++g) single = single && (pg_u0[g + 1] - pg_u0[g] == 1);
    if (single) f |= kClassPairsSingle;
    m.flags = f;
    m.q1 = static_cast<uint32_t>(q1[c]);
    m.qm = qm[c];
    m.u_q = pg_u0[m.q1];
    m.pad[0] = m.pad[1] = 0;
    meta[c] = m;
    if (m.qm >= 0) atomicMax(max_quad_uniques, m.u_q - m.u_p);
  }
}

__global__ void k_fill_i32(int32_t* p, uint64_t n, int32_t v) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Pair map: the group of each popcount-2 X_beta in its class.
__global__ void k_pair_map(uint32_t n_class, const int32_t* p0, const int32_t* p1, const int32_t* pm,
                           const uint32_t* pg_xb, uint32_t n_pairs, int32_t* pmap) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_class; c += gridDim.x * blockDim.x) {
    if (pm[c] < 0) continue;
    for (int32_t g = p0[c]; g < p1[c]; ++g) {
      const uint32_t xb = pg_xb[g];
      const uint32_t p = __ffs(xb) - 1;
      const uint32_t q = 31 - __clz(xb);
      pmap[static_cast<uint64_t>(pm[c]) * n_pairs + q * (q - 1) / 2 + p] = g;
    }
  }
}

}  // namespace

static void build_sector_tables(pbs_grouped& g, const uint64_t* x, hipStream_t s) {
  const uint64_t m = g.n_terms;
  const uint32_t h = g.n_qubits / 2;
  g.half = h;
  g.n_pairs = h * (h - 1) / 2;
  DevBuf<uint32_t> alive(m, s), apos(m, s), cnt(4, s);
  DevBuf<uint64_t> k2(m, s), k1(m, s), k0(m, s);
  DevBuf<double> cre(m, s), cim(m, s);
  if (m) {
    hipLaunchKernelGGL(k_sector_terms, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, x, g.zk.get(), g.ck.get(), m,
                       h, alive.get(), k2.get(), k1.get(), k0.get(), cre.get(), cim.get());
    PBS_HIP(hipGetLastError());
  }
  exclusive_scan_u32(alive.get(), apos.get(), m, cnt.get(), s);
  const uint64_t ma = read_scalar(cnt.get(), s);
  g.n_pterm = static_cast<uint32_t>(ma);
  g.has_sector = true;
  if (ma == 0) {
    g.real_coef = true;
    g.n_class = g.n_pgroup = g.n_unique = 0;
    g.n_pmap = 0;
    g.cls_g0.alloc(1);
    g.pg_u0.alloc(1);
    g.u_t0.alloc(1);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g.cls_g0.get(), 0u);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g.pg_u0.get(), 0u);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g.u_t0.get(), 0u);
    PBS_HIP(hipStreamSynchronize(s));
    return;
  }
  DevBuf<uint64_t> keys(3 * ma, s);
  DevBuf<uint32_t> src(ma, s), order(ma, s);
  hipLaunchKernelGGL(k_compact_alive, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, alive.get(), apos.get(), m,
                     k2.get(), k1.get(), k0.get(), keys.get(), ma);
  hipLaunchKernelGGL(k_alive_index, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, alive.get(), apos.get(), m,
                     src.get());
  PBS_HIP(hipGetLastError());
  iota_u32(order.get(), ma, s);
  radix_sort_keys(keys.get(), order.get(), ma, 3, s);
  DevBuf<uint32_t> hc(ma, s), hg(ma, s), hu(ma, s), cid(ma, s), gid(ma, s), uid(ma, s);
  hipLaunchKernelGGL(k_plan_heads, dim3(grid_for(ma, 256, 65536)), dim3(256), 0, s, keys.get(), ma, hc.get(),
                     hg.get(), hu.get());
  exclusive_scan_u32(hc.get(), cid.get(), ma, cnt.get() + 1, s);
  exclusive_scan_u32(hg.get(), gid.get(), ma, cnt.get() + 2, s);
  exclusive_scan_u32(hu.get(), uid.get(), ma, cnt.get() + 3, s);
  uint32_t counts[4];
  PBS_HIP(hipMemcpyAsync(counts, cnt.get(), sizeof(counts), hipMemcpyDeviceToHost, s));
  PBS_HIP(hipStreamSynchronize(s));
  g.n_class = counts[1];
  g.n_pgroup = counts[2];
  g.n_unique = counts[3];
  g.cls_xa.alloc(g.n_class);
  g.cls_g0.alloc(g.n_class + 1);
  g.pg_xb.alloc(g.n_pgroup);
  g.pg_pc.alloc(g.n_pgroup);
  g.pg_u0.alloc(g.n_pgroup + 1);
  g.u_zb.alloc(g.n_unique);
  g.u_t0.alloc(g.n_unique + 1);
  g.pt_za.alloc(ma);
  g.pt_c.alloc(2 * ma);
  hipLaunchKernelGGL(k_plan_fill, dim3(grid_for(ma, 256, 65536)), dim3(256), 0, s, keys.get(), ma, order.get(),
                     src.get(), cre.get(), cim.get(), hc.get(), hg.get(), hu.get(), cid.get(), gid.get(), uid.get(),
                     g.cls_xa.get(), g.cls_g0.get(), g.pg_xb.get(), g.pg_pc.get(), g.pg_u0.get(), g.u_zb.get(),
                     g.u_t0.get(), g.pt_za.get(), g.pt_c.get());
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g.cls_g0.get() + g.n_class, g.n_pgroup);
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g.pg_u0.get() + g.n_pgroup, g.n_unique);
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g.u_t0.get() + g.n_unique, static_cast<uint32_t>(ma));
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, cnt.get(), 0u);
  hipLaunchKernelGGL(k_any_imag, dim3(grid_for(ma, 256, 65536)), dim3(256), 0, s, g.pt_c.get(), ma, cnt.get());
  PBS_HIP(hipGetLastError());
  g.real_coef = read_scalar(cnt.get(), s) == 0u;

  // bucket metadata, the pair map and the quad map
  g.cls_zg.alloc(g.n_class);
  g.cls_p0.alloc(g.n_class);
  g.cls_p1.alloc(g.n_class);
  g.cls_pm.alloc(g.n_class);
  g.cls_q1.alloc(g.n_class);
  g.cls_qm.alloc(g.n_class);
  const uint64_t n_quads = host_binom(h, 4);
  g.n_quads = n_quads <= kMaxQuads ? static_cast<uint32_t>(n_quads) : 0u;
  DevBuf<uint32_t> has_pairs(g.n_class, s), has_quads(g.n_class, s), slot(g.n_class, s);
  hipLaunchKernelGGL(k_class_meta, dim3(grid_for(g.n_class, 256, 65536)), dim3(256), 0, s, g.n_class,
                     g.cls_g0.get(), g.pg_pc.get(), g.n_quads > 0, g.cls_zg.get(), g.cls_p0.get(), g.cls_p1.get(),
                     g.cls_q1.get(), has_pairs.get(), has_quads.get());
  exclusive_scan_u32(has_pairs.get(), slot.get(), g.n_class, cnt.get(), s);
  g.n_pmap = read_scalar(cnt.get(), s);
  hipLaunchKernelGGL(k_pair_rows, dim3(grid_for(g.n_class, 256, 65536)), dim3(256), 0, s, g.n_class, has_pairs.get(),
                     slot.get(), g.cls_pm.get());
  const uint64_t pm_entries = static_cast<uint64_t>(g.n_pmap) * g.n_pairs;
  g.pmap.alloc(pm_entries);
  if (pm_entries) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(pm_entries, 256, 65536)), dim3(256), 0, s, g.pmap.get(), pm_entries,
                       -1);
    hipLaunchKernelGGL(k_pair_map, dim3(grid_for(g.n_class, 256, 65536)), dim3(256), 0, s, g.n_class,
                       g.cls_p0.get(), g.cls_p1.get(), g.cls_pm.get(), g.pg_xb.get(), g.n_pairs, g.pmap.get());
  }
  exclusive_scan_u32(has_quads.get(), slot.get(), g.n_class, cnt.get(), s);
  g.n_qmap = read_scalar(cnt.get(), s);
  hipLaunchKernelGGL(k_pair_rows, dim3(grid_for(g.n_class, 256, 65536)), dim3(256), 0, s, g.n_class, has_quads.get(),
                     slot.get(), g.cls_qm.get());
  const uint64_t qm_entries = static_cast<uint64_t>(g.n_qmap) * g.n_quads;
  g.qmap.alloc(qm_entries);
  if (qm_entries) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(qm_entries, 256, 65536)), dim3(256), 0, s, g.qmap.get(), qm_entries,
                       -1);
    hipLaunchKernelGGL(k_quad_map, dim3(std::min<uint32_t>(g.n_class, 65536u)), dim3(256), 0, s, g.n_class,
                       g.cls_p1.get(), g.cls_q1.get(), g.cls_qm.get(), g.pg_xb.get(), g.n_quads, g.qmap.get());
  }
  g.cls_meta.alloc(g.n_class);
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, cnt.get(), 0u);
  hipLaunchKernelGGL(k_class_pack, dim3(grid_for(g.n_class, 256, 65536)), dim3(256), 0, s, g.n_class,
                     g.cls_xa.get(), g.cls_g0.get(), g.cls_zg.get(), g.cls_p1.get(), g.cls_pm.get(), g.cls_q1.get(),
                     g.cls_qm.get(), g.pg_u0.get(), g.cls_meta.get(), cnt.get());
  PBS_HIP(hipGetLastError());
  g.max_quad_uniques = read_scalar(cnt.get(), s);

  // class schedule (host side, once per operator)
  std::vector<ClassMeta> meta(g.n_class);
  std::vector<uint32_t> u0(g.n_pgroup + 1), xb(g.n_pgroup), zb(g.n_unique);
  PBS_HIP(hipMemcpyAsync(meta.data(), g.cls_meta.get(), meta.size() * sizeof(ClassMeta), hipMemcpyDeviceToHost, s));
  PBS_HIP(hipMemcpyAsync(u0.data(), g.pg_u0.get(), u0.size() * 4, hipMemcpyDeviceToHost, s));
  if (!xb.empty()) PBS_HIP(hipMemcpyAsync(xb.data(), g.pg_xb.get(), xb.size() * 4, hipMemcpyDeviceToHost, s));
  if (!zb.empty()) PBS_HIP(hipMemcpyAsync(zb.data(), g.u_zb.get(), zb.size() * 4, hipMemcpyDeviceToHost, s));
  PBS_HIP(hipStreamSynchronize(s));
  std::vector<uint32_t> runs, ns;
  int64_t qcnt = -1;
  for (uint32_t c = 0; c < g.n_class; ++c) {
    const ClassMeta& m = meta[c];
    if (m.flags & kClassSimple) {
      if (!runs.empty() && runs.back() == c) {
        runs.back() = c + 1;
      } else {
        runs.push_back(c);
        runs.push_back(c + 1);
      }
    } else {
      ns.push_back(c);
    }
    if (m.qm >= 0) {
      for (uint32_t q = m.p1; q < m.q1; ++q) {
        const int64_t n = u0[q + 1] - u0[q];
        qcnt = (qcnt == -1 || qcnt == n) ? n : 0;
      }
    }
  }
  // beta Z-masks of the single-unique pair groups, per orbital pair
  std::vector<uint32_t> zp(g.n_pairs + 1, 0u);
  {
    std::vector<char> seen(g.n_pairs + 1, 0);
    bool uniform = true;
    for (uint32_t c = 0; c < g.n_class && uniform; ++c) {
      const ClassMeta& m = meta[c];
      if (!(m.flags & kClassPairsSingle) || m.pm < 0) continue;
      const uint32_t gz_end = m.zg >= 0 ? m.g0 + 1 : m.g0;
      for (uint32_t q = gz_end; q < m.p1; ++q) {
        const uint32_t x = xb[q];
        const uint32_t lo = static_cast<uint32_t>(__builtin_ctz(x)), hi = 31u - static_cast<uint32_t>(__builtin_clz(x));
        const uint32_t pid = hi * (hi - 1) / 2 + lo;
        const uint32_t z = zb[u0[q]];
        if (!seen[pid]) {
          seen[pid] = 1;
          zp[pid] = z;
        } else if (zp[pid] != z) {
          uniform = false;
          break;
        }
      }
    }
    g.pair_sign = uniform && g.n_pairs > 0;
  }
  g.n_runs = static_cast<uint32_t>(runs.size() / 2);
  g.n_ns = static_cast<uint32_t>(ns.size());
  g.quad_cnt = qcnt > 0 ? static_cast<uint32_t>(qcnt) : 0u;
  g.zpair.alloc(zp.size());
  g.runs.alloc(runs.size());
  g.ns_list.alloc(ns.size());
  PBS_HIP(hipMemcpyAsync(g.zpair.get(), zp.data(), zp.size() * 4, hipMemcpyHostToDevice, s));
  if (!runs.empty()) PBS_HIP(hipMemcpyAsync(g.runs.get(), runs.data(), runs.size() * 4, hipMemcpyHostToDevice, s));
  if (!ns.empty()) PBS_HIP(hipMemcpyAsync(g.ns_list.get(), ns.data(), ns.size() * 4, hipMemcpyHostToDevice, s));
  PBS_HIP(hipStreamSynchronize(s));  // the host vectors end here
}

}  // namespace pbs

using namespace pbs;

extern "C" {

pbs_status pbs_group_by_xmask(const pbs_sum* hs, void* stream, pbs_grouped** out) {
  return guarded([&] {
    PBS_REQUIRE(out != nullptr, PBS_ERR_ARG, "null output handle");
    *out = nullptr;
    PBS_REQUIRE(hs != nullptr, PBS_ERR_ARG, "null pbs_sum");
    PBS_REQUIRE(hs->canonical, PBS_ERR_ARG, "group_by_xmask needs a canonical sum");
    PBS_REQUIRE(hs->n_qubits <= 64, PBS_ERR_RANGE, "grouping supports at most 64 qubits");
    hipStream_t s = as_stream(stream);
    Scratch scratch(s);  // temporaries of this call
    auto* g = new pbs_grouped();
    try {
      const uint64_t m = hs->n_terms;
      g->n_qubits = hs->n_qubits;
      g->n_terms = m;
      DevBuf<uint32_t> heads(m, s), gid(m, s), cnt(1, s);
      uint64_t G = 0;
      if (m) {
        hipLaunchKernelGGL(k_x_heads, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, hs->x.get(), m, heads.get());
        exclusive_scan_u32(heads.get(), gid.get(), m, cnt.get(), s);
        G = read_scalar(cnt.get(), s);
      }
      g->n_groups = G;
      g->xg.alloc(G);
      g->off.alloc(G + 1);
      g->zk.alloc(m);
      g->ck.alloc(2 * m);
      hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, g->off.get() + G, static_cast<uint32_t>(m));
      if (m)
        hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(m, 256, 65536)), dim3(256), 0, s, hs->x.get(), hs->z.get(),
                           hs->coeff.get(), m, heads.get(), gid.get(), g->xg.get(), g->off.get(), g->zk.get(),
                           g->ck.get());
      PBS_HIP(hipGetLastError());
      PBS_HIP(hipStreamSynchronize(s));
      if ((g->n_qubits % 2) == 0) build_sector_tables(*g, hs->x.get(), s);
    } catch (...) {
      delete g;
      throw;
    }
    *out = g;
  });
}

pbs_status pbs_grouped_info(const pbs_grouped* g, uint32_t* n_qubits, uint64_t* n_groups, uint64_t* n_terms) {
  return guarded([&] {
    PBS_REQUIRE(g != nullptr, PBS_ERR_ARG, "null pbs_grouped");
    if (n_qubits) *n_qubits = g->n_qubits;
    if (n_groups) *n_groups = g->n_groups;
    if (n_terms) *n_terms = g->n_terms;
  });
}

pbs_status pbs_grouped_read(const pbs_grouped* g, uint64_t* xg, uint64_t* offsets, uint64_t* zk, double* ck,
                            void* stream) {
  return guarded([&] {
    PBS_REQUIRE(g != nullptr, PBS_ERR_ARG, "null pbs_grouped");
    hipStream_t s = as_stream(stream);
    if (xg && g->n_groups) PBS_HIP(hipMemcpyAsync(xg, g->xg.get(), g->n_groups * 8, hipMemcpyDefault, s));
    if (zk && g->n_terms) PBS_HIP(hipMemcpyAsync(zk, g->zk.get(), g->n_terms * 8, hipMemcpyDefault, s));
    if (ck && g->n_terms) PBS_HIP(hipMemcpyAsync(ck, g->ck.get(), g->n_terms * 16, hipMemcpyDefault, s));
    if (offsets) {
      std::vector<uint32_t> o(g->n_groups + 1);
      PBS_HIP(hipMemcpyAsync(o.data(), g->off.get(), o.size() * 4, hipMemcpyDeviceToHost, s));
      PBS_HIP(hipStreamSynchronize(s));
      std::vector<uint64_t> o64(o.begin(), o.end());
      PBS_HIP(hipMemcpyAsync(offsets, o64.data(), o64.size() * 8, hipMemcpyDefault, s));
    }
    PBS_HIP(hipStreamSynchronize(s));
  });
}

void pbs_grouped_destroy(pbs_grouped* g) { delete g; }

}  // extern "C"
