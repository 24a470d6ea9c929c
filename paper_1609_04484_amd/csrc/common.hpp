// Internal helpers shared by the library's translation units: status and
// error-message plumbing, HIP error checks, small RAII device buffers and
// the geometry-derived constants.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/stokes_ifmm.h"

namespace sbie {

constexpr double kPi = 3.14159265358979323846;

// A failure inside the library: carries a status code to the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

[[noreturn]] inline void fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error(code, buf);
}

#define SBIE_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      ::sbie::fail(SBIE_HIP_ERROR, "%s failed: %s (%s:%d)", #call,            \
                   hipGetErrorString(e_), __FILE__, __LINE__);                \
  } while (0)

#define SBIE_LAUNCH_CHECK() SBIE_HIP(hipGetLastError())

// Run a body and translate exceptions into a status code.
template <class F>
int guarded(F &&f) {
  try {
    set_last_error("");
    return f();
  } catch (const Error &e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return SBIE_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    set_last_error(e.what());
    return SBIE_INVALID_ARGUMENT;
  }
}

// Device buffer owned by the library (plain hipMalloc; used for long-lived
// handles such as factorisations).
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(SBIE_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    n = count;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Scratch from the stream-ordered allocator, released on the same stream.
template <class T>
struct StreamBuf {
  T *p = nullptr;
  hipStream_t s = nullptr;
  StreamBuf(size_t count, hipStream_t st) : s(st) {
    if (count == 0) return;
    if (hipMallocAsync((void **)&p, count * sizeof(T), s) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(SBIE_OUT_OF_MEMORY, "hipMallocAsync of %zu bytes failed", count * sizeof(T));
    }
  }
  StreamBuf(const StreamBuf &) = delete;
  StreamBuf &operator=(const StreamBuf &) = delete;
  ~StreamBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

// Checks on the geometry descriptor that need no device access.
void validate_geom(const sbie_geom *g);
// validate_geom plus the device-side checks of the node and pore data
// (finite values, unit normals, pore nodes on their circles, no repeated
// node, disjoint pores strictly inside the wall); synchronises the stream
// and fails with SBIE_INVALID_GEOMETRY naming the violated conditions.
void validate_geom_device(const sbie_geom *g, hipStream_t s);

inline int64_t n_unknowns(const sbie_geom *g) {
  return 2 * g->n_nodes + 3 * (int64_t)g->n_pores;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Matvec internals (matvec.hip), reused by the solvers.
// ---------------------------------------------------------------------------
struct MatvecWork {
  double *src = nullptr;     // packed source records, 8 doubles per node
  double *psrc = nullptr;    // packed pore records, 8 doubles per pore
  double *part = nullptr;    // partial sums [chunks + pchunks][2 or 4][Nn]
  double *scal = nullptr;    // [0] = flux functional, [1] = wall length
  int chunks = 0;            // source chunks of the pair kernel
  int pchunks = 0;           // pore chunks of the completion kernel
  int tpt = 4;               // targets per thread
  int sym = 0;               // symmetric pair evaluation (plain modes)
  int sym_R = 0;             // superblocks per side of the symmetric evaluation
  double *sym_buf = nullptr; // its partial sums
  size_t doubles() const;
};

// Plan the launch shape and the scratch size (in doubles) for a geometry.
// allow_sym: the plain modes may use the symmetric pair evaluation (one
// partial sum; the compensated mode needs a plan without it).
MatvecWork plan_matvec(const sbie_geom *g, bool allow_sym = true);
size_t matvec_scratch_doubles(const MatvecWork &w, const sbie_geom *g);
void bind_matvec_scratch(MatvecWork &w, const sbie_geom *g, double *base);
// An alternative evaluation of the double-layer pair sum (the fast multipole
// method, fmm.hip): from the packed source records (8 doubles per node:
// x, y, q_xx, q_xy, q_yy, with q_xy the sum of both off-diagonal entries of
// w/pi n sigma^T) it writes part[0..nn) and part[nn..2nn), the x and y
// components of the pair sum at every node (the plain mode's layout).
struct PairSum {
  virtual ~PairSum() = default;
  virtual void run(const double *src, double *part, hipStream_t s) const = 0;
};

// The pair sum of a fast-multipole plan (fmm.hip), and whether the plan was
// built for this geometry (same node arrays and counts).
const PairSum *fmm_pair_sum(const sbie_fmm *f);
bool fmm_same_geometry(const sbie_fmm *f, const sbie_geom *g);

// y = A x.  With `pairs` set, that evaluation replaces the direct pair
// kernel (plain modes only; w.chunks must be 1).
void matvec_run(const sbie_geom *g, const double *x, double *y, int mode,
                MatvecWork &w, hipStream_t s, const PairSum *pairs = nullptr);

// Wall length |Gamma_0| into *out (device scalar).
void wall_length(const sbie_geom *g, double *out, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched matvec over several geometries (matvec.hip): every stage of y = A x
// is one launch for all members, each workgroup finding its member from a
// table of per-member starts.  The per-call member table (pointers, shapes)
// is staged through pinned memory.
// ---------------------------------------------------------------------------
struct BatchMatvec {
  std::vector<const sbie_geom *> geoms;
  std::vector<MatvecWork> work;
  DevBuf<double> scratch;
  DevBuf<char> desc;
  char *hdesc = nullptr;
  hipEvent_t staged = nullptr;   // the last table upload has been consumed
  DevBuf<unsigned long long> queue;   // work counter of the persistent pair stage
  size_t desc_cap = 0;
  int tpt = 4;
  BatchMatvec(const sbie_geom *const *g, int count);
  ~BatchMatvec();
  BatchMatvec(const BatchMatvec &) = delete;
  BatchMatvec &operator=(const BatchMatvec &) = delete;
  // y[a] = A_b u[a] for b = members[a]; all members when `members` is empty
  void run(const std::vector<int> &members, const std::vector<const double *> &u,
           const std::vector<double *> &y, int mode, hipStream_t s);
};

}  // namespace sbie
