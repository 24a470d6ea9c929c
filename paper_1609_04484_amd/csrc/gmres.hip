// Flexible GMRES with right preconditioning (Saad's FGMRES).  Section 4 of
// the paper solves the dense system with GMRES and a preconditioner applied
// from the left; here the preconditioner is applied on the right and the
// stored preconditioned directions Z keep the Arnoldi relation A Z = V H
// exact in FP64 whatever the precision of the preconditioner, so the stopping
// test is on the true residual ||f - A x|| <= tol ||f||.
//
// Every vector operation runs on the device: the preconditioner, the matvec,
// classical Gram-Schmidt applied twice (two block dot-products and two block
// updates over the basis V), the norm and the normalisation.  The only
// per-iteration host crossing is the new Hessenberg column (j + 2 doubles),
// which the host needs for its Givens rotations and the convergence test.
// The same driver solves the completed double-layer system and the
// single-layer (first-kind) system of Section 2.1.
#include <chrono>
#include <cmath>
#include <functional>

#include "common.hpp"
#include "precond.hpp"
#include "slp.hpp"

namespace sbie {

namespace {

constexpr int kRows = 8192;  // rows per dot-product chunk

// part[c * nch + ch] = sum over rows of chunk ch of V[:, c] . w
__global__ __launch_bounds__(256) void dot_chunks(const double *__restrict__ V,
                                                  int64_t n, int k,
                                                  const double *__restrict__ w,
                                                  int nch, double *__restrict__ part) {
  const int ch = blockIdx.x;
  const int c = blockIdx.y;
  const int64_t r0 = (int64_t)ch * kRows;
  const int64_t r1 = r0 + kRows < n ? r0 + kRows : n;
  const double *v = V + (int64_t)c * n;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) acc = fma(v[i], w[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)c * nch + ch] = (red[0] + red[1]) + (red[2] + red[3]);
}

// h[c] (+)= sum_ch part[c * nch + ch]
__global__ void reduce_chunks(const double *__restrict__ part, int nch, int k,
                              double *__restrict__ h, int accumulate) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int i = 0; i < nch; ++i) s += part[(int64_t)c * nch + i];
  h[c] = accumulate ? h[c] + s : s;
}

// w -= V[:, 0..k) h
__global__ __launch_bounds__(256) void basis_update(const double *__restrict__ V,
                                                    int64_t n, int k,
                                                    const double *__restrict__ h,
                                                    double *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  for (int c = 0; c < k; ++c) acc = fma(-V[(int64_t)c * n + i], h[c], acc);
  w[i] = acc;
}

// x += Z[:, 0..k) y
__global__ __launch_bounds__(256) void basis_combine(const double *__restrict__ Z,
                                                     int64_t n, int k,
                                                     const double *__restrict__ y,
                                                     double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int c = 0; c < k; ++c) acc = fma(Z[(int64_t)c * n + i], y[c], acc);
  x[i] = acc;
}

// part[ch] = sum over chunk of w^2
__global__ __launch_bounds__(256) void sq_chunks(const double *__restrict__ w, int64_t n,
                                                 double *__restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  const int64_t r1 = r0 + kRows < n ? r0 + kRows : n;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) acc = fma(w[i], w[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void sqrt_sum(const double *__restrict__ part, int nch, double *out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nch; ++i) s += part[i];
  *out = sqrt(s);
}

// v = w / *nrm (if *nrm > 0)
__global__ void scale_by(const double *__restrict__ w, int64_t n,
                         const double *__restrict__ nrm, double *__restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double d = *nrm;
  v[i] = d > 0.0 ? w[i] / d : 0.0;
}

// r = f - r
__global__ void rsub(const double *__restrict__ f, int64_t n, double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) r[i] = f[i] - r[i];
}

__global__ void fill(double *__restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void any_nonfinite(const double *__restrict__ x, int64_t n, int *flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && !isfinite(x[i])) *flag = 1;
}

struct Timer {
  hipEvent_t a, b;
  explicit Timer() {
    SBIE_HIP(hipEventCreate(&a));
    SBIE_HIP(hipEventCreate(&b));
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

}  // namespace

// The operator of a solve: y = A x in plain FP64 sums (Arnoldi) or with
// compensated sums (true residuals).
struct KrylovOp {
  int64_t n;
  std::function<void(const double *, double *, bool, hipStream_t)> apply;
};

int gmres_run_op(const KrylovOp &op, const double *f, double *x,
                 const gmres_params *p, gmres_result *res, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t n = op.n;
  const int max_iter = p->max_iter;
  const int restart = p->restart > 0 && p->restart < max_iter ? p->restart : max_iter;
  const bool use_pc = p->pc != 0;
  const int nch = (int)ceil_div(n, kRows);
  const unsigned nb = ceil_div(n, 256);

  const int64_t basis = (int64_t)restart + 1;
  DevBuf<double> V(basis * n);
  DevBuf<double> Z(use_pc ? (int64_t)restart * n : 0);
  DevBuf<double> wv(n), r(n);
  DevBuf<double> part((size_t)nch * (basis + 1) + 16);
  DevBuf<double> hdev(2 * basis + 4);
  DevBuf<int> flag(1);
  double *hhost = nullptr;
  SBIE_HIP(hipHostMalloc((void **)&hhost, (2 * basis + 4) * sizeof(double), hipHostMallocDefault));
  struct HostFree {
    double *p;
    ~HostFree() { if (p) (void)hipHostFree(p); }
  } hf{hhost};

  Timer tpc, tmv, tar;
  float ms = 0.0f;
  double t_pc = 0.0, t_mv = 0.0, t_ar = 0.0;

  auto norm = [&](const double *v, double *dst) {
    sq_chunks<<<nch, 256, 0, s>>>(v, n, part.p);
    sqrt_sum<<<1, 64, 0, s>>>(part.p, nch, dst);
  };
  auto host_scalar = [&](const double *dev) {
    double h = 0.0;
    SBIE_HIP(hipMemcpyAsync(hhost, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
    h = hhost[0];
    return h;
  };
  auto apply_pc = [&](const double *in, double *out) {
    if (!use_pc) {
      SBIE_HIP(hipMemcpyAsync(out, in, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      return;
    }
    precond_apply(p, in, out, s);
  };

  // non-finite data is an error, not a convergence failure
  SBIE_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  any_nonfinite<<<nb, 256, 0, s>>>(f, n, flag.p);
  int hflag = 0;
  SBIE_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  if (hflag) fail(SBIE_BREAKDOWN, "right-hand side is not finite");

  norm(f, hdev.p);
  const double fnorm = host_scalar(hdev.p);
  if (!p->use_x0) fill<<<nb, 256, 0, s>>>(x, n, 0.0);
  if (p->res_hist) p->res_hist[0] = 1.0;
  if (fnorm == 0.0) {
    fill<<<nb, 256, 0, s>>>(x, n, 0.0);
    SBIE_HIP(hipStreamSynchronize(s));
    res->iters = 0;
    res->status = SBIE_OK;
    res->rel_res_true = 0.0;
    res->rel_res_pc = 0.0;
    return SBIE_OK;
  }

  int total = 0;
  double relres = 0.0;
  int status = SBIE_NOT_CONVERGED;
  std::vector<double> H((size_t)(restart + 1) * restart, 0.0), cs(restart), sn(restart),
      gv(restart + 1), y(restart);
  int hist_pos = 1;
  while (true) {
    // the true residual uses compensated sums: when the density is much
    // larger than the data, plain FP64 sums cannot resolve tol ||f||.  From
    // a zero start the first residual is f itself (A 0 = 0 exactly).
    if (total == 0 && !p->use_x0) {
      SBIE_HIP(hipMemcpyAsync(r.p, f, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      op.apply(x, r.p, true, s);
      rsub<<<nb, 256, 0, s>>>(f, n, r.p);
    }
    norm(r.p, hdev.p);
    const double beta = host_scalar(hdev.p);
    if (!std::isfinite(beta)) fail(SBIE_BREAKDOWN, "residual is not finite");
    relres = beta / fnorm;
    if (relres <= p->tol) { status = SBIE_OK; break; }
    if (total >= max_iter) break;
    const int m = restart < max_iter - total ? restart : max_iter - total;
    scale_by<<<nb, 256, 0, s>>>(r.p, n, hdev.p, V.p);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k_used = 0;
    bool stop = false;
    for (int j = 0; j < m; ++j) {
      double *vj = V.p + (int64_t)j * n;
      double *zj = use_pc ? Z.p + (int64_t)j * n : vj;
      SBIE_HIP(hipEventRecord(tpc.a, s));
      if (use_pc) apply_pc(vj, zj);
      SBIE_HIP(hipEventRecord(tpc.b, s));
      SBIE_HIP(hipEventRecord(tmv.a, s));
      op.apply(zj, wv.p, false, s);
      SBIE_HIP(hipEventRecord(tmv.b, s));
      SBIE_HIP(hipEventRecord(tar.a, s));
      const int k = j + 1;
      // CGS2: h = V^T w; w -= V h; h' = V^T w; w -= V h'; h += h'
      dot_chunks<<<dim3(nch, k), 256, 0, s>>>(V.p, n, k, wv.p, nch, part.p);
      reduce_chunks<<<ceil_div(k, 256), 256, 0, s>>>(part.p, nch, k, hdev.p, 0);
      basis_update<<<nb, 256, 0, s>>>(V.p, n, k, hdev.p, wv.p);
      dot_chunks<<<dim3(nch, k), 256, 0, s>>>(V.p, n, k, wv.p, nch, part.p);
      // second pass: store h' after h, then fold
      reduce_chunks<<<ceil_div(k, 256), 256, 0, s>>>(part.p, nch, k, hdev.p + k + 1, 0);
      basis_update<<<nb, 256, 0, s>>>(V.p, n, k, hdev.p + k + 1, wv.p);
      norm(wv.p, hdev.p + k);
      scale_by<<<nb, 256, 0, s>>>(wv.p, n, hdev.p + k, V.p + (int64_t)k * n);
      SBIE_HIP(hipEventRecord(tar.b, s));
      SBIE_LAUNCH_CHECK();
      // fetch h (k entries), h' (k entries) and ||w||
      SBIE_HIP(hipMemcpyAsync(hhost, hdev.p, (2 * k + 1) * sizeof(double),
                              hipMemcpyDeviceToHost, s));
      SBIE_HIP(hipStreamSynchronize(s));
      SBIE_HIP(hipEventElapsedTime(&ms, tpc.a, tpc.b)); t_pc += ms * 1e-3;
      SBIE_HIP(hipEventElapsedTime(&ms, tmv.a, tmv.b)); t_mv += ms * 1e-3;
      SBIE_HIP(hipEventElapsedTime(&ms, tar.a, tar.b)); t_ar += ms * 1e-3;
      double *col = H.data() + (size_t)j * (restart + 1);
      for (int i = 0; i < k; ++i) col[i] = hhost[i] + hhost[k + 1 + i];
      col[k] = hhost[k];
      if (!std::isfinite(col[k])) fail(SBIE_BREAKDOWN, "Arnoldi produced a non-finite value");
      const bool breakdown = col[k] == 0.0;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      if (den == 0.0) fail(SBIE_BREAKDOWN, "zero Hessenberg column");
      cs[j] = col[j] / den;
      sn[j] = col[j + 1] / den;
      col[j] = den;
      col[j + 1] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++total;
      k_used = j + 1;
      const double est = std::fabs(gv[j + 1]) / fnorm;
      if (p->res_hist && hist_pos <= max_iter + 1) p->res_hist[hist_pos++] = est;
      // the inner cycle aims a little below tol so that the compensated
      // true residual usually confirms convergence without another cycle
      if (est <= 0.5 * p->tol || breakdown || total >= max_iter) { stop = true; break; }
    }
    // y = H^{-1} g (upper triangular)
    for (int i = k_used - 1; i >= 0; --i) {
      double acc = gv[i];
      for (int c = i + 1; c < k_used; ++c) acc -= H[(size_t)c * (restart + 1) + i] * y[c];
      y[i] = acc / H[(size_t)i * (restart + 1) + i];
    }
    SBIE_HIP(hipMemcpyAsync(hdev.p, y.data(), k_used * sizeof(double), hipMemcpyHostToDevice, s));
    basis_combine<<<nb, 256, 0, s>>>(use_pc ? Z.p : V.p, n, k_used, hdev.p, x);
    SBIE_LAUNCH_CHECK();
    SBIE_HIP(hipStreamSynchronize(s));
    (void)stop;
  }
  res->iters = total;
  res->status = status;
  res->rel_res_true = relres;
  // the left-preconditioned residual of the paper's tables; the loop always
  // leaves by one of its two exits right after computing r = f - A x for
  // the final x (compensated), so r is reused
  if (use_pc) {
    apply_pc(r.p, wv.p);
    norm(wv.p, hdev.p);
    apply_pc(f, wv.p);
    norm(wv.p, hdev.p + 1);
    SBIE_HIP(hipMemcpyAsync(hhost, hdev.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
    res->rel_res_pc = hhost[0] / hhost[1];
  } else {
    res->rel_res_pc = relres;
  }
  res->t_precond_s = t_pc;
  res->t_matvec_s = t_mv;
  res->t_arnoldi_s = t_ar;
  res->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return status;
}

int gmres_run(const sbie_geom *g, const double *f, double *x,
              const gmres_params *p, gmres_result *res, hipStream_t s) {
  // plain products (Arnoldi) may use the symmetric pair evaluation; the
  // compensated products (true residuals) use the chunked kernel
  const PairSum *fmm = p->fmm ? fmm_pair_sum(p->fmm) : nullptr;
  MatvecWork mw = plan_matvec(g, !fmm);
  DevBuf<double> mvs(matvec_scratch_doubles(mw, g));
  bind_matvec_scratch(mw, g, mvs.p);
  MatvecWork ma = plan_matvec(g, false);
  DevBuf<double> mas(mw.sym ? matvec_scratch_doubles(ma, g) : 0);
  if (mw.sym) bind_matvec_scratch(ma, g, mas.p);
  MatvecWork &macc = mw.sym ? ma : mw;
  // with a fast-multipole plan: its pair sum in the Arnoldi products (one
  // partial sum), the direct compensated product for true residuals
  MatvecWork mf = plan_matvec(g, false);
  mf.chunks = 1;
  DevBuf<double> mfs(fmm ? matvec_scratch_doubles(mf, g) : 0);
  if (fmm) bind_matvec_scratch(mf, g, mfs.p);
  KrylovOp op{n_unknowns(g), [&](const double *in, double *out, bool accurate, hipStream_t st) {
                if (accurate)
                  matvec_run(g, in, out, SBIE_MV_FULL_ACCURATE, macc, st);
                else if (fmm)
                  matvec_run(g, in, out, SBIE_MV_FULL, mf, st, fmm);
                else
                  matvec_run(g, in, out, SBIE_MV_FULL, mw, st);
              }};
  return gmres_run_op(op, f, x, p, res, s);
}

int gmres_run_slp(const sbie_geom *g, const double *f, double *x,
                  const gmres_params *p, gmres_result *res, hipStream_t s) {
  KrylovOp op{2 * g->n_nodes, [&](const double *in, double *out, bool accurate, hipStream_t st) {
                slp_matvec_run(g, in, out, accurate, st);
              }};
  return gmres_run_op(op, f, x, p, res, s);
}

}  // namespace sbie

extern "C" int gmres_solve(const sbie_geom *g, const double *f, double *sigma,
                           const gmres_params *p, gmres_result *res, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!f || !sigma || !p || !res) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (p->max_iter < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "max_iter < 0");
    if (!(p->tol > 0.0)) sbie::fail(SBIE_INVALID_ARGUMENT, "tol must be positive");
    if (p->pc == 1 && !p->bd) sbie::fail(SBIE_INVALID_ARGUMENT, "pc=1 needs a block-diagonal handle");
    if (p->pc == 2 && !p->ifmm) sbie::fail(SBIE_INVALID_ARGUMENT, "pc=2 needs an IFMM handle");
    if (p->pc < 0 || p->pc > 2) sbie::fail(SBIE_INVALID_ARGUMENT, "unknown preconditioner %d", p->pc);
    const int64_t n = sbie::n_unknowns(g);
    if (f < sigma + n && sigma < f + n) sbie::fail(SBIE_INVALID_ARGUMENT, "f and sigma overlap");
    if (p->pc == 1 && sbie::bd_size(p->bd) != n)
      sbie::fail(SBIE_INVALID_ARGUMENT, "the block-diagonal handle belongs to another operator or geometry");
    if (p->fmm && !sbie::fmm_same_geometry(p->fmm, g))
      sbie::fail(SBIE_INVALID_ARGUMENT, "the fast-multipole plan belongs to another geometry");
    sbie::validate_geom_device(g, (hipStream_t)stream);
    *res = gmres_result{};
    return sbie::gmres_run(g, f, sigma, p, res, (hipStream_t)stream);
  });
}

extern "C" int gmres_solve_slp(const sbie_geom *g, const double *f, double *sigma,
                               const gmres_params *p, gmres_result *res, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!f || !sigma || !p || !res) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (p->max_iter < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "max_iter < 0");
    if (!(p->tol > 0.0)) sbie::fail(SBIE_INVALID_ARGUMENT, "tol must be positive");
    if (p->pc == 2) sbie::fail(SBIE_UNSUPPORTED, "the IFMM preconditioner is built for the double layer only");
    if (p->fmm) sbie::fail(SBIE_UNSUPPORTED, "the fast-multipole plan evaluates the double layer only");
    if (p->pc < 0 || p->pc > 1) sbie::fail(SBIE_INVALID_ARGUMENT, "unknown preconditioner %d", p->pc);
    if (p->pc == 1 && !p->bd) sbie::fail(SBIE_INVALID_ARGUMENT, "pc=1 needs a block-diagonal handle");
    const int64_t n = 2 * g->n_nodes;
    if (f < sigma + n && sigma < f + n) sbie::fail(SBIE_INVALID_ARGUMENT, "f and sigma overlap");
    if (p->pc == 1 && sbie::bd_size(p->bd) != n)
      sbie::fail(SBIE_INVALID_ARGUMENT, "the block-diagonal handle does not belong to the single layer");
    sbie::slp_check_geom(g);
    sbie::validate_geom_device(g, (hipStream_t)stream);
    *res = gmres_result{};
    return sbie::gmres_run_slp(g, f, sigma, p, res, (hipStream_t)stream);
  });
}
