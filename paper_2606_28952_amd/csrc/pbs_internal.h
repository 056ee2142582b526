// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <functional>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pbs.h"

namespace pbs {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  pbs_status code;
  Error(pbs_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);
void clear_last_error();

[[noreturn]] inline void fail(pbs_status code, const std::string& msg) { throw Error(code, msg); }

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fail(PBS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define PBS_HIP(call) ::pbs::hip_check((call), #call)
#define PBS_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) ::pbs::fail((code), (msg)); \
  } while (0)

// Runs `body`, turning exceptions into a status code and a thread-local message.
template <class F>
pbs_status guarded(F&& body) {
  try {
    clear_last_error();
    body();
    return PBS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PBS_ERR_ALLOC;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return PBS_ERR_ARG;
  }
}

// ---------------------------------------------------------------- device memory
// Scratch arena for the temporaries of one handle-building call.  Each
// device keeps one device buffer; a call opens a Scratch scope (which holds
// the device's arena for the call's duration), bump-allocates its
// temporaries from it, and at scope end synchronizes the call's stream and
// releases everything at once.  A request that does not fit falls back to
// hipMalloc and makes the scope grow the arena for the next call.  This
// replaces dozens of hipMalloc/hipFree pairs per call (each hipFree waits for
// the device).
class Scratch {
 public:
  explicit Scratch(hipStream_t s);
  ~Scratch();
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  // 256-byte aligned bytes from the arena, or nullptr when they do not fit
  void* take(size_t bytes);
  static Scratch* current();  // innermost open scope of this thread, or nullptr
  struct Arena;                // one per device (defined with the implementation)

 private:
  Arena* arena_;
  hipStream_t stream_;
  size_t top_ = 0, wanted_ = 0;
  Scratch* outer_;
};

// Owning device buffer.  Allocation happens only in handle-building calls.
// Buffers owned by a handle use hipMalloc; temporaries pass the call's
// stream and come from the thread's open Scratch scope when there is one.
template <class T>
struct DevBuf {
  T* ptr = nullptr;
  size_t n = 0;
  bool borrowed = false;  // from a Scratch arena: not freed here
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(size_t count, hipStream_t) { alloc_temp(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), n(o.n), borrowed(o.borrowed) {
    o.ptr = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      ptr = o.ptr;
      n = o.n;
      borrowed = o.borrowed;
      o.ptr = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptr), count * sizeof(T));
    if (e != hipSuccess) failed(count);
  }
  void alloc_temp(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    if (Scratch* sc = Scratch::current()) {
      if (void* p = sc->take(count * sizeof(T))) {
        ptr = static_cast<T*>(p);
        borrowed = true;
        return;
      }
    }
    alloc(count);
  }
  void release() {
    if (ptr && !borrowed) (void)hipFree(ptr);
    ptr = nullptr;
    n = 0;
    borrowed = false;
  }
  T* get() const { return ptr; }

 private:
  void failed(size_t count) {
    ptr = nullptr;
    n = 0;
    (void)hipGetLastError();
    fail(PBS_ERR_ALLOC, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 1u << 20) {
  uint64_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

// Copies a few values device -> host and waits for the stream.
template <class T>
T read_scalar(const T* dev, hipStream_t s) {
  T v{};
  PBS_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  PBS_HIP(hipStreamSynchronize(s));
  return v;
}

inline int words_for(uint32_t n_qubits) { return n_qubits == 0 ? 1 : static_cast<int>((n_qubits + 63) / 64); }

constexpr int kMaxWords = 4;          // Pauli sums up to 256 qubits
constexpr uint32_t kMaxQubitsSum = 64u * kMaxWords;

// ---------------------------------------------------------------- primitives (prims.hip)
// Exclusive prefix sum of n uint32 values (in may equal out).  When total is
// non-null the sum of all values is written there (device pointer).
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total, hipStream_t s);
// Scratch bytes needed by exclusive_scan_u32 for n values.
size_t scan_scratch_bytes(uint64_t n);

// Stable LSD radix sort of m items keyed by nw 64-bit words (SoA: word w of
// item i at keys[w*m + i], word 0 least significant), carrying a uint32
// payload.  Sorts only the 8-bit digits that differ between items (found by
// a device reduction read back once).  Result ends in keys/vals.
void radix_sort_keys(uint64_t* keys, uint32_t* vals, uint64_t m, int nw, hipStream_t s);

// v[i] = i for i < m.
void iota_u32(uint32_t* v, uint64_t m, hipStream_t s);

// Marks item i as a segment head (1) when its key (nw SoA words) differs from
// item i-1; item 0 is always a head.
void mark_heads(const uint64_t* keys, uint64_t m, int nw, uint32_t* heads, hipStream_t s);

// ---------------------------------------------------------------- sums (algebra.hip)
}  // namespace pbs

struct pbs_sum {
  uint32_t n_qubits = 0;
  int words = 1;
  uint64_t n_terms = 0;
  bool canonical = false;
  pbs::DevBuf<uint64_t> x;      // [n_terms * words], term-major
  pbs::DevBuf<uint64_t> z;      // [n_terms * words]
  pbs::DevBuf<double> coeff;    // [2 * n_terms], letter form (re, im)
};

namespace pbs {
// Canonical reduction of raw contributions held in SoA key arrays
// (keys[w*m + i]: words 0..W-1 are z, W..2W-1 are x) with separate re/im
// arrays; fills `out` (allocates its arrays).
void canonicalize_soa(uint32_t n_qubits, int W, uint64_t m, DevBuf<uint64_t>& keys, DevBuf<double>& re,
                      DevBuf<double>& im, double eps_drop, pbs_sum& out, hipStream_t s);
}  // namespace pbs

namespace pbs {
// ---------------------------------------------------------------- L-BFGS (optim.hip)
using Objective = std::function<void(const double* x, double* f, double* g)>;
enum : int32_t { kStopGradient = 0, kStopDecrease = 1, kStopIterations = 2, kStopLineSearch = 3 };
struct LbfgsResult {
  double f = 0.0, g_inf = 0.0;
  uint32_t iters = 0, evals = 0;
  int32_t reason = kStopIterations;
};
// Minimises fg from x (updated in place); f_noise is the relative rounding
// noise of f allowed in the sufficient-decrease test.  See optim.hip.
LbfgsResult lbfgs_minimize(uint32_t n, double* x, const Objective& fg, uint32_t max_iter, uint32_t history,
                           double g_tol, double f_tol, double f_noise);
}  // namespace pbs
