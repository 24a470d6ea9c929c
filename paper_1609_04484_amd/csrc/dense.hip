// Dense kernels for the block-diagonal preconditioner: batched in-place
// Gauss-Jordan inversion with partial pivoting (one workgroup per matrix)
// and block-diagonal matrix-vector products.  (The large wall block is
// inverted by the blocked inverse of batched.hip.)
#include "dense.hpp"

namespace sbie {

namespace {

constexpr int kGJ = 256;

// In-place inverse of column-major n x n matrices (leading dimension n) by
// Gauss-Jordan elimination with partial (row) pivoting; the row swaps are
// undone as column swaps of the inverse at the end.  info[b] = 0 on success,
// k+1 if the k-th pivot was zero or not finite (the matrix is left partly
// eliminated).
__global__ __launch_bounds__(kGJ) void gj_inverse_kernel(
    double *__restrict__ base, const int64_t *__restrict__ off,
    const int32_t *__restrict__ sz, int32_t *__restrict__ info) {
  extern __shared__ double sh[];
  __shared__ double red_v[kGJ];
  __shared__ int red_i[kGJ];
  const int b = blockIdx.x;
  const int n = sz[b];
  double *A = base + off[b];
  double *rowk = sh;
  double *fcol = sh + n;
  int *ipiv = reinterpret_cast<int *>(sh + 2 * n);
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += kGJ) {
      const double v = fabs(A[i + (int64_t)k * n]);
      if (v > best) { best = v; bi = i; }
    }
    red_v[tid] = best;
    red_i[tid] = bi;
    __syncthreads();
    for (int s = kGJ / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double ov = red_v[tid + s];
        const int oi = red_i[tid + s];
        if (ov > red_v[tid] || (ov == red_v[tid] && oi < red_i[tid])) {
          red_v[tid] = ov;
          red_i[tid] = oi;
        }
      }
      __syncthreads();
    }
    const double pv = red_v[0];
    const int p = red_i[0];
    __syncthreads();
    if (!(pv > 0.0) || !isfinite(pv)) {
      if (tid == 0) info[b] = k + 1;
      return;  // uniform across the workgroup
    }
    if (tid == 0) ipiv[k] = p;
    if (p != k) {
      for (int j = tid; j < n; j += kGJ) {
        const double t = A[k + (int64_t)j * n];
        A[k + (int64_t)j * n] = A[p + (int64_t)j * n];
        A[p + (int64_t)j * n] = t;
      }
    }
    __syncthreads();
    const double invd = 1.0 / A[k + (int64_t)k * n];
    for (int j = tid; j < n; j += kGJ)
      rowk[j] = (j == k ? 1.0 : A[k + (int64_t)j * n]) * invd;
    for (int i = tid; i < n; i += kGJ) fcol[i] = i == k ? 0.0 : A[i + (int64_t)k * n];
    __syncthreads();
    for (int i = tid; i < n; i += kGJ) {
      const double f = fcol[i];
      if (i == k) {
        for (int j = 0; j < n; ++j) A[i + (int64_t)j * n] = rowk[j];
      } else {
        for (int j = 0; j < n; ++j) {
          const double a = j == k ? 0.0 : A[i + (int64_t)j * n];
          A[i + (int64_t)j * n] = fma(-f, rowk[j], a);
        }
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = ipiv[k];
    if (p != k) {
      for (int i = tid; i < n; i += kGJ) {
        const double t = A[i + (int64_t)k * n];
        A[i + (int64_t)k * n] = A[i + (int64_t)p * n];
        A[i + (int64_t)p * n] = t;
      }
    }
    __syncthreads();
  }
  if (tid == 0) info[b] = 0;
}

// out[idx[r]] = sum_c M[r + c n] v[idx[c]], one workgroup per block.
__global__ __launch_bounds__(256) void block_gemv_small(
    const double *__restrict__ mats, const int64_t *__restrict__ moff,
    const int64_t *__restrict__ idx, const int64_t *__restrict__ ioff,
    const int32_t *__restrict__ sz, const double *__restrict__ v,
    double *__restrict__ out) {
  extern __shared__ double vs[];
  const int b = blockIdx.x;
  const int n = sz[b];
  const double *M = mats + moff[b];
  const int64_t *ix = idx + ioff[b];
  for (int c = threadIdx.x; c < n; c += blockDim.x) vs[c] = v[ix[c]];
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc = fma(M[r + (int64_t)c * n], vs[c], acc);
    out[ix[r]] = acc;
  }
}

// Split-K partial products of one large block: part[ch][r] =
// sum_{c in chunk ch} M[r + c n] v[idx[c]].
__global__ __launch_bounds__(256) void block_gemv_split(
    const double *__restrict__ M, int64_t n, const int64_t *__restrict__ ix,
    int64_t chunk, const double *__restrict__ v, double *__restrict__ part) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * chunk;
  const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
  if (r >= n) return;
  double acc = 0.0;
  for (int64_t c = c0; c < c1; ++c) acc = fma(M[r + c * n], v[ix[c]], acc);
  part[(int64_t)blockIdx.y * n + r] = acc;
}

__global__ void block_gemv_reduce(const double *__restrict__ part, int64_t n,
                                  int nch, const int64_t *__restrict__ ix,
                                  double *__restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int c = 0; c < nch; ++c) acc += part[(int64_t)c * n + r];
  out[ix[r]] = acc;
}

}  // namespace

void gj_inverse_batched(double *base, const int64_t *off, const int32_t *sz,
                        int nmat, int max_n, int32_t *info, hipStream_t s) {
  if (nmat == 0) return;
  const size_t shmem = (size_t)2 * max_n * sizeof(double) + (size_t)max_n * sizeof(int);
  if (shmem > 60 * 1024)
    fail(SBIE_UNSUPPORTED, "batched inverse limited to n <= 2560 (got %d)", max_n);
  gj_inverse_kernel<<<nmat, kGJ, shmem, s>>>(base, off, sz, info);
  SBIE_LAUNCH_CHECK();
}

void block_gemv(const double *mats, const int64_t *moff_dev, const int64_t *idx,
                const int64_t *ioff_dev, const int32_t *sz_dev, int nsmall,
                int max_small, const double *v, double *out, hipStream_t s) {
  if (nsmall == 0) return;
  block_gemv_small<<<nsmall, 256, (size_t)max_small * sizeof(double), s>>>(
      mats, moff_dev, idx, ioff_dev, sz_dev, v, out);
  SBIE_LAUNCH_CHECK();
}

void big_gemv(const double *M, int64_t n, const int64_t *ix, const double *v,
              double *out, double *part, int nch, hipStream_t s) {
  const int64_t chunk = (n + nch - 1) / nch;
  dim3 grid(ceil_div(n, 256), (unsigned)nch);
  block_gemv_split<<<grid, 256, 0, s>>>(M, n, ix, chunk, v, part);
  SBIE_LAUNCH_CHECK();
  block_gemv_reduce<<<ceil_div(n, 256), 256, 0, s>>>(part, n, nch, ix, out);
  SBIE_LAUNCH_CHECK();
}

}  // namespace sbie
