// Lockstep flexible GMRES over a batch of independent geometries.
//
// Every member runs the same FGMRES as gmres_solve (right preconditioning,
// CGS2, host Givens rotations, compensated true residual, inner target
// 0.5 tol), but the members advance together: one batched matvec per step
// (matvec.hip: one launch per stage for the whole batch), one set of batched
// Gram-Schmidt launches over all members' bases, and one device-to-host copy
// of every member's Hessenberg column.  Members may sit at different inner
// steps (after a restart or a failed true-residual check), so each member
// carries its own column count in the per-step table; a member that has
// converged or used its iterations drops out of the active set.  The
// preconditioners are applied member by member (each is its own captured
// graph or block GEMV).
#include <chrono>
#include <cmath>

#include "common.hpp"
#include "precond.hpp"

namespace sbie {

namespace {

constexpr int kRowsB = 8192;  // rows per dot-product chunk

// Per-member table of one Gram-Schmidt step.
struct BArn {
  const double *V;  // basis, n x (restart + 1), column-major
  double *w;        // the new direction
  double *vnext;    // V[:, k]
  double *h;        // [0, k) first pass, [k] norm, [k + 1, 2k + 1) second pass
  double *part;     // partial sums, k x nch
  int64_t n;
  int k, nch;
  int64_t row0, chunk0;  // flattened starts (row blocks, row chunks)
  int64_t member;        // index into the batch-wide arrays
};

__device__ __forceinline__ int find_arn(const BArn *__restrict__ d, int nb, int64_t unit, bool rows) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((rows ? d[mid].row0 : d[mid].chunk0) <= unit) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// part[c * nch + ch] = V[:, c] . w over chunk ch
__global__ __launch_bounds__(256) void dot_b(const BArn *__restrict__ d, int nb) {
  const int b = find_arn(d, nb, blockIdx.x, false);
  const BArn &A = d[b];
  const int c = blockIdx.y;
  if (c >= A.k) return;
  const int ch = (int)(blockIdx.x - A.chunk0);
  const int64_t r0 = (int64_t)ch * kRowsB;
  const int64_t r1 = r0 + kRowsB < A.n ? r0 + kRowsB : A.n;
  const double *v = A.V + (int64_t)c * A.n;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) acc = fma(v[i], A.w[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) A.part[(int64_t)c * A.nch + ch] = (red[0] + red[1]) + (red[2] + red[3]);
}

// one block per member: h_pass[c] = sum of the partials of column c
__global__ void reduce_b(const BArn *__restrict__ d, int pass) {
  const BArn &A = d[blockIdx.x];
  double *h = pass ? A.h + A.k + 1 : A.h;
  for (int c = threadIdx.x; c < A.k; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < A.nch; ++i) s += A.part[(int64_t)c * A.nch + i];
    h[c] = s;
  }
}

// w -= V[:, 0..k) h_pass
__global__ __launch_bounds__(256) void update_b(const BArn *__restrict__ d, int nb, int pass) {
  const int b = find_arn(d, nb, blockIdx.x, true);
  const BArn &A = d[b];
  const int64_t i = ((int64_t)blockIdx.x - A.row0) * 256 + threadIdx.x;
  if (i >= A.n) return;
  const double *h = pass ? A.h + A.k + 1 : A.h;
  double acc = A.w[i];
  for (int c = 0; c < A.k; ++c) acc = fma(-A.V[(int64_t)c * A.n + i], h[c], acc);
  A.w[i] = acc;
}

// part[ch] = sum over chunk of w^2
__global__ __launch_bounds__(256) void sq_b(const BArn *__restrict__ d, int nb) {
  const int b = find_arn(d, nb, blockIdx.x, false);
  const BArn &A = d[b];
  const int ch = (int)(blockIdx.x - A.chunk0);
  const int64_t r0 = (int64_t)ch * kRowsB;
  const int64_t r1 = r0 + kRowsB < A.n ? r0 + kRowsB : A.n;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) acc = fma(A.w[i], A.w[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) A.part[ch] = (red[0] + red[1]) + (red[2] + red[3]);
}

// one thread per member: h[k] = sqrt(sum of partials)
__global__ void norm_b(const BArn *__restrict__ d, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const BArn &A = d[b];
  double s = 0.0;
  for (int i = 0; i < A.nch; ++i) s += A.part[i];
  A.h[A.k] = sqrt(s);
}

// vnext = w / h[k] (zero when the norm is zero)
__global__ __launch_bounds__(256) void scale_b(const BArn *__restrict__ d, int nb) {
  const int b = find_arn(d, nb, blockIdx.x, true);
  const BArn &A = d[b];
  const int64_t i = ((int64_t)blockIdx.x - A.row0) * 256 + threadIdx.x;
  if (i >= A.n) return;
  const double nr = A.h[A.k];
  A.vnext[i] = nr > 0.0 ? A.w[i] / nr : 0.0;
}

// w = f - w (f of the member, from the batch-wide pointer array)
__global__ __launch_bounds__(256) void rsub_b(const BArn *__restrict__ d, int nb, const double *const *__restrict__ f) {
  const int b = find_arn(d, nb, blockIdx.x, true);
  const BArn &A = d[b];
  const int64_t i = ((int64_t)blockIdx.x - A.row0) * 256 + threadIdx.x;
  if (i < A.n) A.w[i] = f[A.member][i] - A.w[i];
}

__global__ __launch_bounds__(256) void combine_one(const double *__restrict__ Z, int64_t n, int k,
                                                   const double *__restrict__ y, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int c = 0; c < k; ++c) acc = fma(Z[(int64_t)c * n + i], y[c], acc);
  x[i] = acc;
}

__global__ void fill_zero(double *__restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

__global__ void nonfinite_flag(const double *__restrict__ x, int64_t n, int *flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && !isfinite(x[i])) *flag = 1;
}

struct Member {
  const sbie_geom *g = nullptr;
  const double *f = nullptr;
  double *x = nullptr;
  gmres_params pc{};
  bool use_pc = false;
  int64_t n = 0;
  int nch = 0;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *h = nullptr, *part = nullptr, *y = nullptr;
  double fnorm = 0.0, relres = 0.0;
  int total = 0, status = SBIE_NOT_CONVERGED;
  int j = 0, m_cycle = 0;
  bool done = false;
  std::vector<double> H, cs, sn, gv, yv;
};

}  // namespace

int gmres_batched_run(const sbie_geom *geoms, int count, const double *const *f, double *const *x,
                      const gmres_member *mem, double tol, int max_iter, int restart_in,
                      gmres_result *res, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const int restart = restart_in > 0 && restart_in < max_iter ? restart_in : (max_iter > 0 ? max_iter : 1);
  const int hstride = 2 * (restart + 1) + 4;
  std::vector<Member> M(count);
  std::vector<const sbie_geom *> gp(count);
  size_t vbytes = 0;
  for (int b = 0; b < count; ++b) {
    Member &a = M[b];
    a.g = &geoms[b];
    gp[b] = a.g;
    a.f = f[b];
    a.x = x[b];
    a.pc.pc = mem[b].pc;
    a.pc.bd = mem[b].bd;
    a.pc.ifmm = mem[b].ifmm;
    a.use_pc = mem[b].pc != 0;
    a.n = n_unknowns(a.g);
    a.nch = (int)ceil_div(a.n, kRowsB);
    vbytes += (size_t)(restart + 1) * a.n + (a.use_pc ? (size_t)restart * a.n : 0) + a.n +
              (size_t)a.nch * (restart + 2) + restart + 8;
    a.H.assign((size_t)(restart + 1) * restart, 0.0);
    a.cs.assign(restart, 0.0);
    a.sn.assign(restart, 0.0);
    a.gv.assign(restart + 1, 0.0);
    a.yv.assign(restart, 0.0);
  }
  DevBuf<double> pool(vbytes);
  DevBuf<double> hall((size_t)hstride * count);
  DevBuf<int> flag(count);
  DevBuf<const double *> fdev(count);
  {
    double *p = pool.p;
    for (int b = 0; b < count; ++b) {
      Member &a = M[b];
      a.V = p; p += (size_t)(restart + 1) * a.n;
      if (a.use_pc) { a.Z = p; p += (size_t)restart * a.n; } else a.Z = a.V;
      a.w = p; p += a.n;
      a.part = p; p += (size_t)a.nch * (restart + 2);
      a.y = p; p += restart + 8;
      a.h = hall.p + (size_t)hstride * b;
    }
  }
  BatchMatvec bmv(gp.data(), count);
  std::vector<const double *> fptr(f, f + count);
  SBIE_HIP(hipMemcpyAsync(fdev.p, fptr.data(), count * sizeof(double *), hipMemcpyHostToDevice, s));
  SBIE_HIP(hipStreamSynchronize(s));  // fptr is pageable host memory

  double *hhost = nullptr, *htab = nullptr;
  SBIE_HIP(hipHostMalloc((void **)&hhost, (size_t)hstride * count * sizeof(double), hipHostMallocDefault));
  const size_t tab_bytes = (size_t)count * sizeof(BArn);
  SBIE_HIP(hipHostMalloc((void **)&htab, tab_bytes, hipHostMallocDefault));
  struct Pinned {
    double *a, *b;
    ~Pinned() {
      if (a) (void)hipHostFree(a);
      if (b) (void)hipHostFree(b);
    }
  } pinned{hhost, htab};
  DevBuf<char> tab(tab_bytes);
  hipEvent_t staged = nullptr;
  SBIE_HIP(hipEventCreateWithFlags(&staged, hipEventDisableTiming));
  struct Ev {
    hipEvent_t e;
    ~Ev() { if (e) { (void)hipEventSynchronize(e); (void)hipEventDestroy(e); } }
  } ev{staged};

  // Upload the per-member table for the listed members; `k` and the
  // destination pointers come from `fill`.
  auto upload = [&](const std::vector<int> &act, auto fill) -> const BArn * {
    SBIE_HIP(hipEventSynchronize(staged));
    BArn *t = reinterpret_cast<BArn *>(htab);
    int64_t r0 = 0, c0 = 0;
    for (size_t q = 0; q < act.size(); ++q) {
      Member &a = M[act[q]];
      BArn &A = t[q];
      A.V = a.V;
      A.w = a.w;
      A.h = a.h;
      A.part = a.part;
      A.n = a.n;
      A.nch = a.nch;
      A.k = 0;
      A.vnext = nullptr;
      A.member = act[q];
      fill(a, A);
      A.row0 = r0;
      A.chunk0 = c0;
      r0 += ceil_div(a.n, 256);
      c0 += a.nch;
    }
    SBIE_HIP(hipMemcpyAsync(tab.p, htab, act.size() * sizeof(BArn), hipMemcpyHostToDevice, s));
    SBIE_HIP(hipEventRecord(staged, s));
    return reinterpret_cast<const BArn *>(tab.p);
  };
  auto rows_of = [&](const std::vector<int> &act) {
    int64_t r = 0;
    for (int b : act) r += ceil_div(M[b].n, 256);
    return (unsigned)r;
  };
  auto chunks_of = [&](const std::vector<int> &act) {
    int64_t c = 0;
    for (int b : act) c += M[b].nch;
    return (unsigned)c;
  };
  auto fetch_h = [&]() {
    SBIE_HIP(hipMemcpyAsync(hhost, hall.p, (size_t)hstride * count * sizeof(double), hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
  };

  std::vector<int> all(count);
  for (int b = 0; b < count; ++b) all[b] = b;

  // non-finite data is an error for that member; ||f|| for everyone
  SBIE_HIP(hipMemsetAsync(flag.p, 0, count * sizeof(int), s));
  for (int b = 0; b < count; ++b) {
    nonfinite_flag<<<ceil_div(M[b].n, 256), 256, 0, s>>>(M[b].f, M[b].n, flag.p + b);
    if (!mem[b].use_x0) fill_zero<<<ceil_div(M[b].n, 256), 256, 0, s>>>(M[b].x, M[b].n);
  }
  SBIE_LAUNCH_CHECK();
  {
    std::vector<int> hflag(count, 0);
    SBIE_HIP(hipMemcpyAsync(hflag.data(), flag.p, count * sizeof(int), hipMemcpyDeviceToHost, s));
    // w = f for the norm
    for (int b = 0; b < count; ++b)
      SBIE_HIP(hipMemcpyAsync(M[b].w, M[b].f, M[b].n * sizeof(double), hipMemcpyDeviceToDevice, s));
    const BArn *dt = upload(all, [](Member &, BArn &A) { A.k = 0; });
    sq_b<<<chunks_of(all), 256, 0, s>>>(dt, count);
    norm_b<<<ceil_div(count, 64), 64, 0, s>>>(dt, count);
    SBIE_LAUNCH_CHECK();
    fetch_h();
    for (int b = 0; b < count; ++b) {
      if (hflag[b]) fail(SBIE_BREAKDOWN, "right-hand side of member %d is not finite", b);
      M[b].fnorm = hhost[(size_t)hstride * b];
      if (M[b].fnorm == 0.0) {
        fill_zero<<<ceil_div(M[b].n, 256), 256, 0, s>>>(M[b].x, M[b].n);
        M[b].done = true;
        M[b].status = SBIE_OK;
        M[b].relres = 0.0;
      }
    }
  }

  double t_step = 0.0;
  std::vector<int> need_res;
  for (int b = 0; b < count; ++b)
    if (!M[b].done) need_res.push_back(b);
  std::vector<int> in_cycle;

  while (!need_res.empty() || !in_cycle.empty()) {
    if (!need_res.empty()) {
      // true residual r = f - A x with compensated sums, for every member
      // that starts a cycle
      std::vector<const double *> u;
      std::vector<double *> out;
      for (int b : need_res) {
        u.push_back(M[b].x);
        out.push_back(M[b].w);
      }
      bmv.run(need_res, u, out, SBIE_MV_FULL_ACCURATE, s);
      const BArn *dt = upload(need_res, [](Member &, BArn &A) { A.k = 0; });
      rsub_b<<<rows_of(need_res), 256, 0, s>>>(dt, (int)need_res.size(), fdev.p);
      sq_b<<<chunks_of(need_res), 256, 0, s>>>(dt, (int)need_res.size());
      norm_b<<<ceil_div(need_res.size(), 64), 64, 0, s>>>(dt, (int)need_res.size());
      SBIE_LAUNCH_CHECK();
      fetch_h();
      std::vector<int> start;
      for (int b : need_res) {
        Member &a = M[b];
        const double beta = hhost[(size_t)hstride * b];
        if (!std::isfinite(beta)) fail(SBIE_BREAKDOWN, "residual of member %d is not finite", b);
        a.relres = beta / a.fnorm;
        if (a.relres <= tol) {
          a.status = SBIE_OK;
          a.done = true;
        } else if (a.total >= max_iter) {
          a.done = true;
        } else {
          a.m_cycle = restart < max_iter - a.total ? restart : max_iter - a.total;
          std::fill(a.H.begin(), a.H.end(), 0.0);
          std::fill(a.gv.begin(), a.gv.end(), 0.0);
          a.gv[0] = beta;
          a.j = 0;
          start.push_back(b);
        }
      }
      if (!start.empty()) {
        // V[:, 0] = r / beta (beta sits in h[0])
        const BArn *ds = upload(start, [](Member &a, BArn &A) {
          A.k = 0;
          A.vnext = a.V;
        });
        scale_b<<<rows_of(start), 256, 0, s>>>(ds, (int)start.size());
        SBIE_LAUNCH_CHECK();
        for (int b : start) in_cycle.push_back(b);
      }
      need_res.clear();
      continue;
    }

    // one lockstep Arnoldi step for every member in a cycle
    auto t0 = std::chrono::steady_clock::now();
    for (int b : in_cycle) {
      Member &a = M[b];
      if (a.use_pc) precond_apply(&a.pc, a.V + (int64_t)a.j * a.n, a.Z + (int64_t)a.j * a.n, s);
    }
    std::vector<const double *> u;
    std::vector<double *> out;
    for (int b : in_cycle) {
      u.push_back(M[b].Z + (int64_t)M[b].j * M[b].n);
      out.push_back(M[b].w);
    }
    bmv.run(in_cycle, u, out, SBIE_MV_FULL, s);
    int kmax = 0;
    for (int b : in_cycle) kmax = std::max(kmax, M[b].j + 1);
    const BArn *dt = upload(in_cycle, [](Member &a, BArn &A) {
      A.k = a.j + 1;
      A.vnext = a.V + (int64_t)(a.j + 1) * a.n;
    });
    const int na = (int)in_cycle.size();
    const unsigned nch = chunks_of(in_cycle), nrow = rows_of(in_cycle);
    for (int pass = 0; pass < 2; ++pass) {
      dot_b<<<dim3(nch, kmax), 256, 0, s>>>(dt, na);
      reduce_b<<<na, 256, 0, s>>>(dt, pass);
      update_b<<<nrow, 256, 0, s>>>(dt, na, pass);
    }
    sq_b<<<nch, 256, 0, s>>>(dt, na);
    norm_b<<<ceil_div(na, 64), 64, 0, s>>>(dt, na);
    scale_b<<<nrow, 256, 0, s>>>(dt, na);
    SBIE_LAUNCH_CHECK();
    fetch_h();
    t_step += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

    std::vector<int> keep;
    for (int b : in_cycle) {
      Member &a = M[b];
      const int j = a.j, k = j + 1;
      const double *hh = hhost + (size_t)hstride * b;
      double *col = a.H.data() + (size_t)j * (restart + 1);
      for (int i = 0; i < k; ++i) col[i] = hh[i] + hh[k + 1 + i];
      col[k] = hh[k];
      if (!std::isfinite(col[k])) fail(SBIE_BREAKDOWN, "Arnoldi of member %d produced a non-finite value", b);
      const bool breakdown = col[k] == 0.0;
      for (int i = 0; i < j; ++i) {
        const double t = a.cs[i] * col[i] + a.sn[i] * col[i + 1];
        col[i + 1] = -a.sn[i] * col[i] + a.cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      if (den == 0.0) fail(SBIE_BREAKDOWN, "zero Hessenberg column in member %d", b);
      a.cs[j] = col[j] / den;
      a.sn[j] = col[j + 1] / den;
      col[j] = den;
      col[j + 1] = 0.0;
      a.gv[j + 1] = -a.sn[j] * a.gv[j];
      a.gv[j] = a.cs[j] * a.gv[j];
      ++a.total;
      const double est = std::fabs(a.gv[j + 1]) / a.fnorm;
      if (est <= 0.5 * tol || breakdown || a.total >= max_iter || k >= a.m_cycle) {
        // end of the cycle: x += Z y with H y = g
        for (int i = k - 1; i >= 0; --i) {
          double acc = a.gv[i];
          for (int c = i + 1; c < k; ++c) acc -= a.H[(size_t)c * (restart + 1) + i] * a.yv[c];
          a.yv[i] = acc / a.H[(size_t)i * (restart + 1) + i];
        }
        SBIE_HIP(hipMemcpyAsync(a.y, a.yv.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
        combine_one<<<ceil_div(a.n, 256), 256, 0, s>>>(a.Z, a.n, k, a.y, a.x);
        SBIE_LAUNCH_CHECK();
        need_res.push_back(b);
      } else {
        a.j = k;
        keep.push_back(b);
      }
    }
    in_cycle.swap(keep);
    if (!need_res.empty()) SBIE_HIP(hipStreamSynchronize(s));  // y uploads come from host vectors
  }

  // the left-preconditioned residual of the paper's tables, member by member
  for (int b = 0; b < count; ++b) {
    Member &a = M[b];
    res[b] = gmres_result{};
    res[b].iters = a.total;
    res[b].status = a.status;
    res[b].rel_res_true = a.relres;
    res[b].rel_res_pc = a.relres;
    if (a.use_pc && a.fnorm > 0.0) {
      matvec_run(a.g, a.x, a.w, SBIE_MV_FULL_ACCURATE, bmv.work[b], s);
      const BArn *dt = upload({b}, [](Member &, BArn &A) { A.k = 0; });
      rsub_b<<<ceil_div(a.n, 256), 256, 0, s>>>(dt, 1, fdev.p);
      precond_apply(&a.pc, a.w, a.V, s);
      precond_apply(&a.pc, a.f, a.V + a.n, s);
      SBIE_HIP(hipMemcpyAsync(a.w, a.V, a.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      sq_b<<<a.nch, 256, 0, s>>>(dt, 1);
      norm_b<<<1, 64, 0, s>>>(dt, 1);
      fetch_h();
      const double num = hhost[(size_t)hstride * b];
      SBIE_HIP(hipMemcpyAsync(a.w, a.V + a.n, a.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      sq_b<<<a.nch, 256, 0, s>>>(dt, 1);
      norm_b<<<1, 64, 0, s>>>(dt, 1);
      SBIE_LAUNCH_CHECK();
      fetch_h();
      const double den = hhost[(size_t)hstride * b];
      res[b].rel_res_pc = den > 0.0 ? num / den : 0.0;
    }
  }
  SBIE_HIP(hipStreamSynchronize(s));
  const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  int worst = SBIE_OK;
  for (int b = 0; b < count; ++b) {
    res[b].t_total_s = el;
    res[b].t_arnoldi_s = t_step;
    if (res[b].status != SBIE_OK) worst = res[b].status;
  }
  return worst;
}

}  // namespace sbie

extern "C" int gmres_solve_batched(const sbie_geom *geoms, int32_t count, const double *const *f,
                                   double *const *sigma, const gmres_member *members, double tol,
                                   int32_t max_iter, int32_t restart, gmres_result *results,
                                   void *stream) {
  return sbie::guarded([&]() {
    if (count < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "count < 0");
    if (count == 0) return (int)SBIE_OK;
    if (!geoms || !f || !sigma || !members || !results) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (max_iter < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "max_iter < 0");
    if (!(tol > 0.0)) sbie::fail(SBIE_INVALID_ARGUMENT, "tol must be positive");
    for (int b = 0; b < count; ++b) {
      sbie::validate_geom(&geoms[b]);
      const gmres_member &m = members[b];
      if (m.pc < 0 || m.pc > 2) sbie::fail(SBIE_INVALID_ARGUMENT, "member %d: unknown preconditioner", b);
      if (m.pc == 1 && !m.bd) sbie::fail(SBIE_INVALID_ARGUMENT, "member %d: pc=1 needs a block-diagonal handle", b);
      if (m.pc == 2 && !m.ifmm) sbie::fail(SBIE_INVALID_ARGUMENT, "member %d: pc=2 needs an IFMM handle", b);
      if (!f[b] || !sigma[b]) sbie::fail(SBIE_INVALID_ARGUMENT, "member %d: null vector", b);
      const int64_t n = sbie::n_unknowns(&geoms[b]);
      if (f[b] < sigma[b] + n && sigma[b] < f[b] + n)
        sbie::fail(SBIE_INVALID_ARGUMENT, "member %d: f and sigma overlap", b);
    }
    for (int b = 0; b < count; ++b) sbie::validate_geom_device(&geoms[b], (hipStream_t)stream);
    return sbie::gmres_batched_run(geoms, count, f, sigma, members, tol, max_iter, restart, results,
                                   (hipStream_t)stream);
  });
}
