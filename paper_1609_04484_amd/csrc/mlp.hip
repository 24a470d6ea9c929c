// Learned warm start for GMRES: a per-pore multilayer perceptron that maps
// local geometry features of a pore to a truncated Fourier series of the
// density on that pore, plus the kernels that build its inputs, its
// training labels and the initial guess.  All FP32 (network) / FP64 (initial
// guess), hand-written; GEMMs use the batched tile kernel.
//
// Features of pore k (64 floats, zero padded): its radius; the offsets
// (dx, dy) and radii of its 16 nearest pores by centre distance (ties by
// index, zeros when fewer exist); the Poiseuille inflow profile and its slope
// at the centre height and the distances to the two walls.
// Coefficients (64 floats): per velocity component a_0, a_1..a_15, b_1..b_15,
// a_16 of sigma(theta) = a_0 + sum (a_m cos m theta + b_m sin m theta)
// + a_16 cos 16 theta, theta measured at the pore centre.
#include <cmath>
#include <memory>

#include "batched.hpp"
#include "common.hpp"
#include "precond.hpp"

struct sbie_mlp {
  int nl = 0;
  std::vector<int> widths;
  std::vector<size_t> woff, boff;   // parameter offsets (floats)
  size_t nparams = 0;
  sbie::DevBuf<float> p, g, m, v;
  // activations for one batch: Z_l and H_l per layer
  int cap_batch = 0;
  std::vector<sbie::DevBuf<float>> z, h, dz;
  sbie::DevBuf<double> loss;
  // input standardisation h0 = (x - in_mu) * in_scale; the last layer
  // predicts standardised targets, returned as y = z * out_sd + out_mu
  sbie::DevBuf<float> in_mu, in_scale, out_mu, out_sd;
  int64_t step = 0;
  std::unique_ptr<sbie::Stager> st;
};

namespace sbie {
namespace {

constexpr int kFeat = 64;
constexpr int kCoef = 64;
constexpr int kNear = 16;

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

// Z (rows x B) += bias (per row); H = act(Z)
__global__ void bias_act(float *__restrict__ z, float *__restrict__ h, const float *__restrict__ b,
                         int rows, int batch, int act) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * batch) return;
  const int r = (int)(e % rows);
  const float v = z[e] + b[r];
  z[e] = v;
  h[e] = act ? gelu(v) : v;
}

// Loss on standardised targets: with t' = (T - out_mu) / out_sd (per row),
// loss = mean (Y - t')^2 and dY = 2 (Y - t') / (rows * B); loss partial sums
// per block.
__global__ void mse_grad(const float *__restrict__ y, const float *__restrict__ t, float *__restrict__ dy,
                         int rows, int64_t n, float scale, const float *__restrict__ mu,
                         const float *__restrict__ sd, double *__restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % rows);
    const float d = y[e] - (t[e] - mu[r]) / sd[r];
    dy[e] = 2.0f * d * scale;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * (double)scale);
}

__global__ void mul_gelu_grad(float *__restrict__ dz, const float *__restrict__ z, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dz[e] *= gelu_grad(z[e]);
}

// db[r] = sum over the batch of dz[r, :]
__global__ void row_sums(const float *__restrict__ dz, float *__restrict__ db, int rows, int batch) {
  const int r = blockIdx.x;
  float s = 0.0f;
  for (int c = threadIdx.x; c < batch; c += blockDim.x) s += dz[r + (int64_t)c * rows];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) db[r] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// out (rows x B) = (x - mu) * scale  or  x * scale + mu (per row)
__global__ void row_affine(const float *__restrict__ x, float *__restrict__ out, const float *__restrict__ mu,
                           const float *__restrict__ sc, int rows, int64_t n, int inverse) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int r = (int)(e % rows);
  out[e] = inverse ? x[e] * sc[r] + mu[r] : (x[e] - mu[r]) * sc[r];
}

// Mean and standard deviation of every row of X (rows x B, column-major),
// accumulated in FP64 by one wave per row.  Rows with zero spread keep
// scale 1.  invert != 0 stores 1 / std (input scaling), else std.
__global__ void row_stats(const float *__restrict__ x, int rows, int batch, float *__restrict__ mu,
                          float *__restrict__ sc, int invert) {
  const int r = blockIdx.x;
  double s = 0.0, q = 0.0;
  for (int c = threadIdx.x; c < batch; c += 64) {
    const double v = x[r + (int64_t)c * rows];
    s += v;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  const double mean = s / batch;
  for (int c = threadIdx.x; c < batch; c += 64) {
    const double v = x[r + (int64_t)c * rows] - mean;
    q += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
  if (threadIdx.x == 0) {
    const double sd = sqrt(q / batch);
    const bool flat = !(sd > 1e-12 * (fabs(mean) + 1e-30)) || sd < 1e-30;
    mu[r] = (float)mean;
    sc[r] = flat ? 1.0f : (float)(invert ? 1.0 / sd : sd);
  }
}

__global__ void scale_kernel(float *__restrict__ x, int64_t n, float s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] *= s;
}

// Per-pore features (one thread per pore; brute-force 16 nearest).
__global__ void features_kernel(int m, const double *__restrict__ cx, const double *__restrict__ cy,
                                const double *__restrict__ rad, double y_lo, double y_hi,
                                float *__restrict__ f) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double bd[kNear];
  int bi[kNear];
  for (int q = 0; q < kNear; ++q) { bd[q] = 1e300; bi[q] = -1; }
  const double x = cx[k], y = cy[k];
  for (int j = 0; j < m; ++j) {
    if (j == k) continue;
    const double dx = cx[j] - x, dy = cy[j] - y;
    const double d = dx * dx + dy * dy;
    if (d < bd[kNear - 1] || (d == bd[kNear - 1] && j < bi[kNear - 1])) {
      int q = kNear - 1;
      while (q > 0 && (d < bd[q - 1] || (d == bd[q - 1] && j < bi[q - 1]))) {
        bd[q] = bd[q - 1];
        bi[q] = bi[q - 1];
        --q;
      }
      bd[q] = d;
      bi[q] = j;
    }
  }
  float *o = f + (int64_t)k * kFeat;
  o[0] = (float)rad[k];
  for (int q = 0; q < kNear; ++q) {
    const int j = bi[q];
    o[1 + 3 * q] = j >= 0 ? (float)(cx[j] - x) : 0.0f;
    o[2 + 3 * q] = j >= 0 ? (float)(cy[j] - y) : 0.0f;
    o[3 + 3 * q] = j >= 0 ? (float)rad[j] : 0.0f;
  }
  const double hh = 0.5 * (y_hi - y_lo), yc = y - 0.5 * (y_hi + y_lo);
  const double kk = 1.0 / (hh * hh);
  o[49] = (float)(kk * (hh * hh - yc * yc));
  o[50] = (float)(-2.0 * kk * yc);
  o[51] = (float)(y - y_lo);
  o[52] = (float)(y_hi - y);
  for (int q = 53; q < kFeat; ++q) o[q] = 0.0f;
}

// Fourier coefficients of the density on every pore (one wave per pore).
__global__ void labels_kernel(int64_t nn, const int64_t *__restrict__ off, const double *__restrict__ x,
                              const double *__restrict__ y, const double *__restrict__ cx,
                              const double *__restrict__ cy, const double *__restrict__ sigma,
                              float *__restrict__ coef) {
  const int k = blockIdx.x;
  const int64_t a = off[k], b = off[k + 1];
  const double inv_n = 1.0 / (double)(b - a);
  // lane t < 64 computes coefficient t
  const int t = threadIdx.x;
  const int comp = t / 32, q = t % 32;
  int mode;
  bool is_sin;
  if (q == 0) { mode = 0; is_sin = false; }
  else if (q <= 15) { mode = q; is_sin = false; }
  else if (q <= 30) { mode = q - 15; is_sin = true; }
  else { mode = 16; is_sin = false; }
  double s = 0.0;
  for (int64_t j = a; j < b; ++j) {
    const double th = atan2(y[j] - cy[k], x[j] - cx[k]);
    const double sv = sigma[comp * nn + j];
    s += sv * (is_sin ? sin(mode * th) : cos(mode * th));
  }
  s *= (mode == 0 ? 1.0 : 2.0) * inv_n;
  coef[(int64_t)k * kCoef + t] = (float)s;
}

// Initial guess: Fourier series on the pores, the given wall density on the
// wall, and the completion unknowns from the constraint functionals.
__global__ void assemble_x0_kernel(int64_t nn, int m, const int64_t *__restrict__ off,
                                   const double *__restrict__ x, const double *__restrict__ y,
                                   const double *__restrict__ w, const double *__restrict__ cx,
                                   const double *__restrict__ cy, const double *__restrict__ rad,
                                   const float *__restrict__ coef, const double *__restrict__ wall,
                                   double *__restrict__ x0) {
  const int k = blockIdx.x;
  if (k == m) {
    // wall block
    const int64_t a = off[m], b = off[m + 1];
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      x0[j] = wall ? wall[j - a] : 0.0;
      x0[nn + j] = wall ? wall[(b - a) + (j - a)] : 0.0;
    }
    return;
  }
  const int64_t a = off[k], b = off[k + 1];
  const float *c = coef + (int64_t)k * kCoef;
  double sx = 0.0, sy = 0.0, sm = 0.0;
  for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
    const double th = atan2(y[j] - cy[k], x[j] - cx[k]);
    double vx = c[0], vy = c[32];
    for (int md = 1; md <= 15; ++md) {
      const double cs = cos(md * th), sn = sin(md * th);
      vx += c[md] * cs + c[15 + md] * sn;
      vy += c[32 + md] * cs + c[47 + md] * sn;
    }
    vx += c[31] * cos(16.0 * th);
    vy += c[63] * cos(16.0 * th);
    x0[j] = vx;
    x0[nn + j] = vy;
    sx += w[j] * vx;
    sy += w[j] * vy;
    sm += w[j] * ((y[j] - cy[k]) * vx - (x[j] - cx[k]) * vy);
  }
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_down(sx, o, 64);
    sy += __shfl_down(sy, o, 64);
    sm += __shfl_down(sm, o, 64);
  }
  if (threadIdx.x == 0) {
    const double r = rad[k];
    double *lam = x0 + 2 * nn + 3 * (int64_t)k;
    lam[0] = sx / (2.0 * kPi * r);
    lam[1] = sy / (2.0 * kPi * r);
    lam[2] = sm / (2.0 * kPi * r * r);
  }
}

// Wall rows of r = f - y, gathered as [x components | y components].
__global__ void wall_residual(const double *__restrict__ f, const double *__restrict__ y, int64_t nn, int64_t a,
                              int64_t ne, double *__restrict__ rw) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * ne) return;
  const int64_t c = e / ne, i = e % ne;
  const int64_t row = c * nn + a + i;
  rw[e] = f[row] - y[row];
}

__global__ void wall_add(const double *__restrict__ zw, int64_t nn, int64_t a, int64_t ne, double *__restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * ne) return;
  const int64_t c = e / ne, i = e % ne;
  x[c * nn + a + i] += zw[e];
}

// Partial sums of <f, y> and <y, y> per block (256 threads).
__global__ void dot2_partial(const double *__restrict__ f, const double *__restrict__ y, int64_t n,
                             double *__restrict__ part) {
  __shared__ double r1[256], r2[256];
  double a = 0.0, b = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double yy = y[e];
    a += f[e] * yy;
    b += yy * yy;
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      r1[threadIdx.x] += r1[threadIdx.x + st];
      r2[threadIdx.x] += r2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

// alpha = <f, y> / <y, y> from the partial sums (0 when y = 0); one block of
// 256 threads.
__global__ void finish_alpha(const double *__restrict__ part, int np, double *__restrict__ alpha) {
  __shared__ double r1[256], r2[256];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    a += part[2 * q];
    b += part[2 * q + 1];
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      r1[threadIdx.x] += r1[threadIdx.x + st];
      r2[threadIdx.x] += r2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *alpha = r2[0] > 0.0 ? r1[0] / r2[0] : 0.0;
}

__global__ void scale_by(double *__restrict__ x, int64_t n, const double *__restrict__ alpha) {
  const double al = *alpha;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] *= al;
}

void ensure_batch(sbie_mlp *n, int batch) {
  if (batch <= n->cap_batch) return;
  n->z.clear();
  n->h.clear();
  n->dz.clear();
  n->z.resize(n->nl + 1);
  n->h.resize(n->nl + 1);
  n->dz.resize(n->nl + 1);
  for (int l = 0; l <= n->nl; ++l) {
    n->z[l].alloc((size_t)n->widths[l] * batch);
    n->h[l].alloc((size_t)n->widths[l] * batch);
    n->dz[l].alloc((size_t)n->widths[l] * batch);
  }
  n->cap_batch = batch;
}

// forward pass into the cached activations; X is widths[0] x batch
void forward(sbie_mlp *n, const float *X, int batch, hipStream_t s) {
  ensure_batch(n, batch);
  const int64_t n0 = (int64_t)n->widths[0] * batch;
  row_affine<<<ceil_div(n0, 256), 256, 0, s>>>(X, n->h[0].p, n->in_mu.p, n->in_scale.p, n->widths[0], n0, 0);
  SBIE_LAUNCH_CHECK();
  const float *in = n->h[0].p;
  for (int l = 0; l < n->nl; ++l) {
    const int out = n->widths[l + 1], inw = n->widths[l];
    gemm_batched<float>({GemmDesc<float>{out, batch, inw, 0, 0, n->p.p + n->woff[l], out, in, inw,
                                         n->z[l + 1].p, out, 1.0f, 0.0f}},
                        *n->st, s);
    const int64_t ne = (int64_t)out * batch;
    bias_act<<<ceil_div(ne, 256), 256, 0, s>>>(n->z[l + 1].p, n->h[l + 1].p, n->p.p + n->boff[l], out, batch,
                                               l + 1 < n->nl ? 1 : 0);
    SBIE_LAUNCH_CHECK();
    in = n->h[l + 1].p;
  }
}

}  // namespace
}  // namespace sbie

using namespace sbie;

extern "C" int mlp_create(int nlayers, const int32_t *widths, uint64_t seed, sbie_mlp **out,
                          void *stream) {
  return guarded([&]() {
    if (!widths || !out || nlayers < 1 || nlayers > 16) fail(SBIE_INVALID_ARGUMENT, "bad network shape");
    *out = nullptr;
    auto n = std::make_unique<sbie_mlp>();
    n->nl = nlayers;
    for (int l = 0; l <= nlayers; ++l) {
      if (widths[l] <= 0 || widths[l] > 8192) fail(SBIE_INVALID_ARGUMENT, "bad layer width");
      n->widths.push_back(widths[l]);
    }
    size_t o = 0;
    for (int l = 0; l < nlayers; ++l) {
      n->woff.push_back(o);
      o += (size_t)widths[l] * widths[l + 1];
      n->boff.push_back(o);
      o += widths[l + 1];
    }
    n->nparams = o;
    n->p.alloc(o);
    n->g.alloc(o);
    n->m.alloc(o);
    n->v.alloc(o);
    n->loss.alloc(1);
    n->in_mu.alloc(widths[0]);
    n->in_scale.alloc(widths[0]);
    n->out_mu.alloc(widths[nlayers]);
    n->out_sd.alloc(widths[nlayers]);
    n->st = std::make_unique<Stager>((size_t)1 << 20);
    hipStream_t s = (hipStream_t)stream;
    fill_value<float>(n->in_mu.p, widths[0], 0.0f, s);
    fill_value<float>(n->in_scale.p, widths[0], 1.0f, s);
    fill_value<float>(n->out_mu.p, widths[nlayers], 0.0f, s);
    fill_value<float>(n->out_sd.p, widths[nlayers], 1.0f, s);
    fill_value<float>(n->p.p, o, 0.0f, s);
    fill_value<float>(n->m.p, o, 0.0f, s);
    fill_value<float>(n->v.p, o, 0.0f, s);
    // He-normal weights, zero biases
    for (int l = 0; l < nlayers; ++l) {
      const size_t nw = (size_t)widths[l] * widths[l + 1];
      gaussian_fill<float>(n->p.p + n->woff[l], nw, seed * 131 + l, s);
      const int64_t ne = (int64_t)nw;
      scale_kernel<<<ceil_div(ne, 256), 256, 0, s>>>(n->p.p + n->woff[l], ne,
                                                      (float)std::sqrt(2.0 / widths[l]));
      SBIE_LAUNCH_CHECK();
    }
    *out = n.release();
    return SBIE_OK;
  });
}

extern "C" int mlp_destroy(sbie_mlp *n) {
  return guarded([&]() {
    delete n;
    return SBIE_OK;
  });
}

extern "C" int mlp_num_params(const sbie_mlp *n, int64_t *count) {
  return guarded([&]() {
    if (!n || !count) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    *count = (int64_t)n->nparams;
    return SBIE_OK;
  });
}

extern "C" int mlp_get_params(const sbie_mlp *n, float *dst, void *stream) {
  return guarded([&]() {
    if (!n || !dst) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    SBIE_HIP(hipMemcpyAsync(dst, n->p.p, n->nparams * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SBIE_OK;
  });
}

extern "C" int mlp_set_params(sbie_mlp *n, const float *src, void *stream) {
  return guarded([&]() {
    if (!n || !src) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    SBIE_HIP(hipMemcpyAsync(n->p.p, src, n->nparams * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SBIE_OK;
  });
}

extern "C" int mlp_forward(sbie_mlp *n, const float *X, int32_t batch, float *Y, void *stream) {
  return guarded([&]() {
    if (!n || !X || !Y || batch <= 0) fail(SBIE_INVALID_ARGUMENT, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    forward(n, X, batch, s);
    const int outw = n->widths[n->nl];
    const int64_t ne = (int64_t)outw * batch;
    row_affine<<<ceil_div(ne, 256), 256, 0, s>>>(n->h[n->nl].p, Y, n->out_mu.p, n->out_sd.p, outw, ne, 1);
    SBIE_LAUNCH_CHECK();
    return SBIE_OK;
  });
}

extern "C" int mlp_loss_grad(sbie_mlp *n, const float *X, const float *T, int32_t batch, float *grad,
                             double *loss, void *stream) {
  return guarded([&]() {
    if (!n || !X || !T || batch <= 0) fail(SBIE_INVALID_ARGUMENT, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    forward(n, X, batch, s);
    const int L = n->nl;
    const int outw = n->widths[L];
    const int64_t ne = (int64_t)outw * batch;
    fill_value<double>(n->loss.p, 1, 0.0, s);
    mse_grad<<<std::min<int64_t>(ceil_div(ne, 256), 1024), 256, 0, s>>>(
        n->h[L].p, T, n->dz[L].p, outw, ne, 1.0f / (float)ne, n->out_mu.p, n->out_sd.p, n->loss.p);
    SBIE_LAUNCH_CHECK();
    for (int l = L; l >= 1; --l) {
      const int out = n->widths[l], inw = n->widths[l - 1];
      const float *hin = n->h[l - 1].p;
      // dW = dZ H^T, db = row sums of dZ
      gemm_batched<float>({GemmDesc<float>{out, inw, batch, 0, 1, n->dz[l].p, out, hin, inw,
                                           n->g.p + n->woff[l - 1], out, 1.0f, 0.0f}},
                          *n->st, s);
      row_sums<<<out, 256, 0, s>>>(n->dz[l].p, n->g.p + n->boff[l - 1], out, batch);
      SBIE_LAUNCH_CHECK();
      if (l > 1) {
        // dH = W^T dZ, dZ_{l-1} = dH * gelu'(Z_{l-1})
        gemm_batched<float>({GemmDesc<float>{inw, batch, out, 1, 0, n->p.p + n->woff[l - 1], out, n->dz[l].p,
                                             out, n->dz[l - 1].p, inw, 1.0f, 0.0f}},
                            *n->st, s);
        const int64_t nz = (int64_t)inw * batch;
        mul_gelu_grad<<<ceil_div(nz, 256), 256, 0, s>>>(n->dz[l - 1].p, n->z[l - 1].p, nz);
        SBIE_LAUNCH_CHECK();
      }
    }
    if (grad)
      SBIE_HIP(hipMemcpyAsync(grad, n->g.p, n->nparams * 4, hipMemcpyDeviceToDevice, s));
    if (loss) {
      SBIE_HIP(hipMemcpyAsync(loss, n->loss.p, 8, hipMemcpyDeviceToHost, s));
      SBIE_HIP(hipStreamSynchronize(s));
      n->st->reset();  // every descriptor copy has completed
    }
    return SBIE_OK;
  });
}

extern "C" int mlp_set_scaling(sbie_mlp *n, const float *in_mean, const float *in_scale, const float *out_mean,
                               const float *out_std, void *stream) {
  return guarded([&]() {
    if (!n || !in_mean || !in_scale || !out_mean || !out_std) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    const size_t a = (size_t)n->widths[0] * 4, b = (size_t)n->widths[n->nl] * 4;
    SBIE_HIP(hipMemcpyAsync(n->in_mu.p, in_mean, a, hipMemcpyDeviceToDevice, s));
    SBIE_HIP(hipMemcpyAsync(n->in_scale.p, in_scale, a, hipMemcpyDeviceToDevice, s));
    SBIE_HIP(hipMemcpyAsync(n->out_mu.p, out_mean, b, hipMemcpyDeviceToDevice, s));
    SBIE_HIP(hipMemcpyAsync(n->out_sd.p, out_std, b, hipMemcpyDeviceToDevice, s));
    return SBIE_OK;
  });
}

extern "C" int mlp_get_scaling(const sbie_mlp *n, float *in_mean, float *in_scale, float *out_mean,
                               float *out_std, void *stream) {
  return guarded([&]() {
    if (!n || !in_mean || !in_scale || !out_mean || !out_std) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    const size_t a = (size_t)n->widths[0] * 4, b = (size_t)n->widths[n->nl] * 4;
    SBIE_HIP(hipMemcpyAsync(in_mean, n->in_mu.p, a, hipMemcpyDeviceToDevice, s));
    SBIE_HIP(hipMemcpyAsync(in_scale, n->in_scale.p, a, hipMemcpyDeviceToDevice, s));
    SBIE_HIP(hipMemcpyAsync(out_mean, n->out_mu.p, b, hipMemcpyDeviceToDevice, s));
    SBIE_HIP(hipMemcpyAsync(out_std, n->out_sd.p, b, hipMemcpyDeviceToDevice, s));
    return SBIE_OK;
  });
}

extern "C" int mlp_fit_scaling(sbie_mlp *n, const float *X, const float *T, int32_t batch, void *stream) {
  return guarded([&]() {
    if (!n || !X || !T || batch <= 0) fail(SBIE_INVALID_ARGUMENT, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    row_stats<<<n->widths[0], 64, 0, s>>>(X, n->widths[0], batch, n->in_mu.p, n->in_scale.p, 1);
    SBIE_LAUNCH_CHECK();
    row_stats<<<n->widths[n->nl], 64, 0, s>>>(T, n->widths[n->nl], batch, n->out_mu.p, n->out_sd.p, 0);
    SBIE_LAUNCH_CHECK();
    return SBIE_OK;
  });
}

extern "C" int mlp_adam_step(sbie_mlp *n, float lr, float beta1, float beta2, float eps, void *stream) {
  return guarded([&]() {
    if (!n) fail(SBIE_INVALID_ARGUMENT, "null network");
    n->step += 1;
    const float c1 = 1.0f - std::pow(beta1, (float)n->step);
    const float c2 = 1.0f - std::pow(beta2, (float)n->step);
    const int64_t np = (int64_t)n->nparams;
    adam_kernel<<<ceil_div(np, 256), 256, 0, (hipStream_t)stream>>>(n->p.p, n->g.p, n->m.p, n->v.p, np, lr,
                                                                     beta1, beta2, eps, c1, c2);
    SBIE_LAUNCH_CHECK();
    return SBIE_OK;
  });
}

extern "C" int warmstart_features(const sbie_geom *g, double y_lo, double y_hi, float *feats, void *stream) {
  return guarded([&]() {
    validate_geom(g);
    if (!feats) fail(SBIE_INVALID_ARGUMENT, "null output");
    const int m = g->n_pores;
    if (m == 0) return SBIE_OK;
    features_kernel<<<ceil_div(m, 64), 64, 0, (hipStream_t)stream>>>(m, g->cx, g->cy, g->radius, y_lo, y_hi,
                                                                     feats);
    SBIE_LAUNCH_CHECK();
    return SBIE_OK;
  });
}

extern "C" int warmstart_labels(const sbie_geom *g, const double *sigma, float *coeffs, void *stream) {
  return guarded([&]() {
    validate_geom(g);
    if (!sigma || !coeffs) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    const int m = g->n_pores;
    if (m == 0) return SBIE_OK;
    labels_kernel<<<m, 64, 0, (hipStream_t)stream>>>(g->n_nodes, g->curve_off_dev, g->x, g->y, g->cx, g->cy,
                                                     sigma, coeffs);
    SBIE_LAUNCH_CHECK();
    return SBIE_OK;
  });
}

extern "C" int warmstart_assemble(const sbie_geom *g, const float *coeffs, const double *wall_sigma,
                                  double *x0, void *stream) {
  return guarded([&]() {
    validate_geom(g);
    if (!x0 || (g->n_pores > 0 && !coeffs)) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    const int m = g->n_pores;
    assemble_x0_kernel<<<m + 1, 64, 0, (hipStream_t)stream>>>(g->n_nodes, m, g->curve_off_dev, g->x, g->y,
                                                              g->w, g->cx, g->cy, g->radius, coeffs,
                                                              wall_sigma, x0);
    SBIE_LAUNCH_CHECK();
    return SBIE_OK;
  });
}

extern "C" int warmstart_refine(const sbie_geom *g, const sbie_bd *wall_bd, const double *f, double *x0,
                                double *alpha, void *stream) {
  return guarded([&]() {
    validate_geom(g);
    if (!wall_bd || !f || !x0) fail(SBIE_INVALID_ARGUMENT, "null pointer");
    const int m = g->n_pores;
    const int64_t nn = g->n_nodes, a = g->curve_off[m], ne = g->curve_off[m + 1] - a;
    if (bd_size(wall_bd) != 2 * ne)
      fail(SBIE_INVALID_ARGUMENT, "wall preconditioner has %lld unknowns, the wall has %lld",
           (long long)bd_size(wall_bd), (long long)(2 * ne));
    const int64_t n = n_unknowns(g);
    hipStream_t s = (hipStream_t)stream;
    MatvecWork w = plan_matvec(g);
    constexpr int kParts = 256;
    StreamBuf<double> scratch(matvec_scratch_doubles(w, g) + n + 4 * ne + 2 * kParts + 1, s);
    bind_matvec_scratch(w, g, scratch.p);
    double *y = scratch.p + matvec_scratch_doubles(w, g);
    double *rw = y + n, *zw = rw + 2 * ne, *part = zw + 2 * ne, *al = part + 2 * kParts;
    if (ne > 0) {
      matvec_run(g, x0, y, SBIE_MV_FULL, w, s);
      wall_residual<<<ceil_div(2 * ne, 256), 256, 0, s>>>(f, y, nn, a, ne, rw);
      SBIE_LAUNCH_CHECK();
      bd_apply(wall_bd, rw, zw, s);
      wall_add<<<ceil_div(2 * ne, 256), 256, 0, s>>>(zw, nn, a, ne, x0);
      SBIE_LAUNCH_CHECK();
    }
    matvec_run(g, x0, y, SBIE_MV_FULL, w, s);
    dot2_partial<<<kParts, 256, 0, s>>>(f, y, n, part);
    SBIE_LAUNCH_CHECK();
    finish_alpha<<<1, 256, 0, s>>>(part, kParts, al);
    SBIE_LAUNCH_CHECK();
    scale_by<<<std::max(1u, std::min(ceil_div(n, 256), 1024u)), 256, 0, s>>>(x0, n, al);
    SBIE_LAUNCH_CHECK();
    if (alpha) {
      SBIE_HIP(hipMemcpyAsync(alpha, al, 8, hipMemcpyDeviceToHost, s));
      SBIE_HIP(hipStreamSynchronize(s));
    }
    return SBIE_OK;
  });
}
