// Variable-size batched dense kernels used by the IFMM factorisation and
// solve, templated on the working precision (double or float).
#pragma once
#include <chrono>

#include "common.hpp"

namespace sbie {

// C = alpha op(A) op(B) + beta C, op(A) m x k, op(B) k x n, column-major.
template <class T>
struct GemmDesc {
  int m, n, k;
  int ta, tb;
  const T *A;
  int lda;
  const T *B;
  int ldb;
  T *C;
  int ldc;
  T alpha, beta;
};

// One term of a multi-term GEMV: alpha op(A) x with op(A) rows x cols.  The
// matrix may be stored in a narrower type TA than the vectors and the
// arithmetic (T): entries are widened as they are read.
template <class T, class TA = T>
struct GemvTerm {
  const TA *A;
  const T *x;
  int lda, cols, trans;
  T alpha;
};

// y (rows) = beta y0 + sum of terms [t0, t0 + nt), with y0 = y when null
template <class T>
struct GemvDesc {
  T *y;
  const T *y0;
  int rows;
  int t0, nt;
  T beta;
};

// dst = alpha op(src) (rows x cols of the destination), optionally
// accumulated (acc != 0: dst += alpha op(src)).
template <class T>
struct CopyDesc {
  const T *src;
  int lds;
  T *dst;
  int ldd;
  int rows, cols;
  int trans, acc;
  T alpha;
};

// Staging of host-built descriptor arrays into device memory: a pinned host
// ring and a device ring, both reset at synchronisation points.
struct Stager {
  char *host = nullptr;
  DevBuf<char> dev;
  size_t cap = 0, used = 0;
  explicit Stager(size_t bytes);
  ~Stager();
  Stager(const Stager &) = delete;
  Stager &operator=(const Stager &) = delete;
  // copy bytes to the device ring (stream-ordered); returns the device address
  void *put(const void *src, size_t bytes, hipStream_t s);
  // several host arrays in one transfer: dst[i] receives the device address
  // of part i (each part 256-byte aligned)
  void put_many(const std::vector<std::pair<const void *, size_t>> &parts, std::vector<void *> &dst,
                hipStream_t s);
  void reset() { used = 0; }
};

// A staging ring borrowed from a process-wide pool and returned when the
// lease ends, so that repeated factorisations do not page-lock, map and free
// tens of megabytes each time.  A lease that ends by an exception first
// synchronises its stream (launches in flight may still read the rings); a
// lease that ends normally must end after its stream has been synchronised.
// The pool keeps one ring per concurrent user and device until the process
// ends.
class StagerLease {
 public:
  StagerLease(size_t bytes, hipStream_t s);
  ~StagerLease();
  StagerLease(const StagerLease &) = delete;
  StagerLease &operator=(const StagerLease &) = delete;
  Stager &operator*() { return *st_; }

 private:
  Stager *st_ = nullptr;
  int dev_ = 0;
  hipStream_t s_ = nullptr;
};

// Algorithmic flop counts of the batched products and inverses issued by the
// calling thread (GEMM 2 m n k; Gauss-Jordan inverse 2 n^3), the op log of
// a factorisation.  Reset and read by its caller.
// Host time spent in the batched operations' own code (set up, staging,
// launches), per thread, for the factorisation's verbose report.
struct HostProf {
  enum Slot { kGemm, kStage, kLaunch, kCopy, kInvPrep, kInvLaunch, kOther, kAlloc, kSlots };
  double t[kSlots] = {};
  int64_t n[kSlots] = {};
};
HostProf &host_prof();
struct HostScope {
  int k;
  std::chrono::steady_clock::time_point t0;
  explicit HostScope(int slot) : k(slot), t0(std::chrono::steady_clock::now()) {}
  ~HostScope() {
    HostProf &h = host_prof();
    h.t[k] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ++h.n[k];
  }
};

struct OpFlops {
  double gemm = 0.0, inverse = 0.0;
  double gemm_low = 0.0;   // the part of gemm run with FP16/BF16 inputs
  int64_t gemm_products = 0, inverses = 0;
};
OpFlops &op_flops();

template <class T>
void gemm_batched(const std::vector<GemmDesc<T>> &d, Stager &st, hipStream_t s);
// Products whose result only has to span the right subspace (randomised
// sketches): kF16 / kBF16 round the inputs (after alpha) to FP16 / BF16 and
// accumulate in FP32 on the matrix cores; kWorking is gemm_batched.
enum class GemmInputs : int { kWorking = 0, kF16 = 1, kBF16 = 2 };
template <class T>
void gemm_batched_sketch(const std::vector<GemmDesc<T>> &d, GemmInputs in, Stager &st, hipStream_t s);
template <class T>
void gemv_batched(const std::vector<GemvDesc<T>> &d, const std::vector<GemvTerm<T>> &t,
                  Stager &st, hipStream_t s);
// Device-resident descriptor arrays (prepared once, launched many times).
template <class T, class TA = T>
void gemv_launch(const GemvDesc<T> *d, const GemvTerm<T, TA> *t, int nd, int max_rows,
                 hipStream_t s);
template <class T>
void copy_batched(const std::vector<CopyDesc<T>> &d, Stager &st, hipStream_t s);
template <class T>
void copy_launch(const CopyDesc<T> *d, int nd, int max_rows, hipStream_t s);

// In-place inverses (Gauss-Jordan with partial pivoting); ptrs[b] -> n_b x n_b
// column-major matrix with leading dimension n_b; info[b] != 0 = singular.
template <class T>
void inverse_batched(const std::vector<T *> &ptrs, const std::vector<int> &ns,
                     int32_t *info_dev, Stager &st, hipStream_t s);

// Same, with matrices larger than a threshold inverted by blocked
// Gauss-Jordan with partial pivoting whose rank-nb updates are batched GEMMs
// (spread over all compute units).  Stream-ordered: info_dev is written by
// the last launch, so read it after a synchronisation.
template <class T>
void inverse_batched_blocked(const std::vector<T *> &ptrs, const std::vector<int> &ns,
                             int32_t *info_dev, Stager &st, hipStream_t s);

// Frobenius norms of blocks (rows x cols, ld) into out[b] (double).
template <class T>
struct NormDesc {
  const T *A;
  int lda, rows, cols;
};
template <class T>
void norms_batched(const std::vector<NormDesc<T>> &d, double *out_dev, Stager &st,
                   hipStream_t s);

// Scale each column of blocks to unit norm (zero columns left as zero).
template <class T>
void normalize_columns(T *A, int lda, int rows, int cols, hipStream_t s);
// Same for many blocks (A, lda, rows, cols) in one launch.
template <class T>
void normalize_batched(const std::vector<NormDesc<T>> &d, Stager &st, hipStream_t s);

// Truncated pivoted Gram-Schmidt: R (m x c) holds candidate columns already
// projected against W[:, :r0]; new orthonormal columns (residual column norm
// above tol) are appended to W starting at column r0, at most rmax - r0 of
// them; their number is written to *count.
template <class T>
struct PgsDesc {
  T *R;
  int ldr, m, c;
  T *W;
  int ldw, r0, rmax;
  double tol;
  int *count;
  // the candidates are already orthogonal to W's columns [0, orth_from)
  // (projected out beforehand), so accepted columns are re-orthogonalised
  // only against the later ones; 0 = against all of them
  int orth_from;
};
template <class T>
void pgs_batched(const std::vector<PgsDesc<T>> &d, Stager &st, hipStream_t s);

// Standard normal numbers from a counter-based generator (splitmix64 hash of
// (seed, index) -> two uniforms -> Box-Muller).
template <class T>
void gaussian_fill(T *out, size_t n, uint64_t seed, hipStream_t s);

template <class T>
void fill_value(T *out, size_t n, T v, hipStream_t s);

template <class Tsrc, class Tdst>
void convert(const Tsrc *src, Tdst *dst, size_t n, hipStream_t s);

}  // namespace sbie
