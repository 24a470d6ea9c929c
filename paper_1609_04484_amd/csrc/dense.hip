// Dense kernels for the preconditioners: batched in-place Gauss-Jordan
// inversion with partial pivoting (one workgroup per matrix), a blocked
// Gauss-Jordan inversion for large well-conditioned blocks whose rank-nb
// updates are plain GEMMs (rocBLAS, FP64 MFMA), and block-diagonal
// matrix-vector products.
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

// dst (rows x cols, ld_dst) = src (rows x cols, ld_src); optionally zero the
// source rows [z0, z1) in the copy.
__global__ void copy_block(const double *__restrict__ src, int64_t ld_src,
                           double *__restrict__ dst, int64_t ld_dst,
                           int64_t rows, int64_t cols, int64_t z0, int64_t z1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= rows || j >= cols) return;
  dst[i + j * ld_dst] = (i >= z0 && i < z1) ? 0.0 : src[i + j * ld_src];
}

__global__ void zero_block(double *__restrict__ dst, int64_t ld, int64_t rows,
                           int64_t cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < rows && j < cols) dst[i + j * ld] = 0.0;
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

void copy_submatrix(const double *src, int64_t ld_src, double *dst,
                    int64_t ld_dst, int64_t rows, int64_t cols, hipStream_t s,
                    int64_t zero_r0, int64_t zero_r1) {
  if (rows == 0 || cols == 0) return;
  dim3 grid(ceil_div(rows, 256), (unsigned)cols);
  copy_block<<<grid, 256, 0, s>>>(src, ld_src, dst, ld_dst, rows, cols, zero_r0, zero_r1);
  SBIE_LAUNCH_CHECK();
}

void blocked_inverse_nopivot(double *M, int64_t n, int nb, hipStream_t s,
                             DenseWork &w) {
  rocblas_handle h = blas_handle(s);
  if ((int64_t)w.C.n < n * nb) w.C.alloc(n * nb);
  if ((int64_t)w.R.n < n * nb) w.R.alloc(n * nb);
  if ((int64_t)w.P.n < (int64_t)nb * nb) w.P.alloc((size_t)nb * nb);
  if (w.meta.n < 4) w.meta.alloc(4);
  int64_t meta_host[2] = {0, 0};
  int32_t hinfo = 0;
  for (int64_t p0 = 0; p0 < n; p0 += nb) {
    const int pb = (int)(n - p0 < nb ? n - p0 : nb);
    // P = M_pp^{-1}
    copy_submatrix(M + p0 + p0 * n, n, w.P.p, pb, pb, pb, s);
    meta_host[0] = 0;
    int32_t szh = pb;
    SBIE_HIP(hipMemcpyAsync(w.meta.p, meta_host, sizeof(int64_t), hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(reinterpret_cast<int32_t *>(w.meta.p + 1), &szh, sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    gj_inverse_batched(w.P.p, w.meta.p, reinterpret_cast<int32_t *>(w.meta.p + 1), 1, pb,
                       reinterpret_cast<int32_t *>(w.meta.p + 2), s);
    SBIE_HIP(hipMemcpyAsync(&hinfo, reinterpret_cast<int32_t *>(w.meta.p + 2), sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) fail(SBIE_BREAKDOWN, "singular diagonal tile at row %lld", (long long)p0);
    // C = M[:, p] with the pivot rows zeroed
    copy_submatrix(M + p0 * n, n, w.C.p, n, n, pb, s, p0, p0 + pb);
    // R = P M[p, :], with its pivot columns zeroed
    const double one = 1.0, zero = 0.0, mone = -1.0;
    SBIE_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, pb, n, pb,
                            &one, w.P.p, pb, M + p0, n, &zero, w.R.p, pb));
    {
      dim3 grid(ceil_div(pb, 256), (unsigned)pb);
      zero_block<<<grid, 256, 0, s>>>(w.R.p + p0 * pb, pb, pb, pb);
      SBIE_LAUNCH_CHECK();
    }
    // M -= C R   (rows and columns outside the pivot block)
    SBIE_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, pb,
                            &mone, w.C.p, n, w.R.p, pb, &one, M, n));
    // M[p, :] = R
    copy_submatrix(w.R.p, pb, M + p0, n, pb, n, s);
    // M[:, p] = -C P, then M_pp = P
    SBIE_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, pb, pb,
                            &mone, w.C.p, n, w.P.p, pb, &zero, M + p0 * n, n));
    copy_submatrix(w.P.p, pb, M + p0 + p0 * n, n, pb, pb, s);
  }
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
