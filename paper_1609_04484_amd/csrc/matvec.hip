// Matrix-free application of the completed double-layer operator
// (Section 2.1 double-layer kernel, Section 2.2 Nystrom discretisation).
//
// Launch structure of one y = A x:
//   pack_sources      SoA node data + current density -> 64-byte source records
//                     (x, y, w nx/pi, w ny/pi, sigma_x, sigma_y); pore records
//                     (cx, cy, lambda_x, lambda_y, r mu)
//   wall_flux         flux functional sum_wall w n.sigma and |Gamma_0|
//   dlp_pairs<T>      the O(Nn^2) pair sum, split into (target tile, source
//                     chunk) workgroups; each thread owns T targets; source
//                     records are wave-uniform so they are read through the
//                     scalar data path and broadcast, with no LDS traffic
//   completion_pairs  Stokeslet/rotlet columns, (target tile, pore chunk)
//   epilogue          sums the partials, adds the jump, the smooth diagonal
//                     limit and the wall rank-one term
//   pore_rows         the three constraint rows per pore (one wave per pore)
#include "common.hpp"

namespace sbie {

namespace {

constexpr int kBlock = 256;
constexpr int kPoreChunk = 64;

int g_tpt = 4;        // targets per thread
int g_chunks = 0;     // source chunks (0 = automatic)

// optional event bracketing of the pair kernel
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

__global__ void pack_sources(int64_t nn, int m, const double *__restrict__ x,
                             const double *__restrict__ y,
                             const double *__restrict__ nx,
                             const double *__restrict__ ny,
                             const double *__restrict__ w,
                             const double *__restrict__ rad,
                             const double *__restrict__ cx,
                             const double *__restrict__ cy,
                             const double *__restrict__ u,
                             double *__restrict__ src,
                             double *__restrict__ psrc) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nn) {
    const double s = w[j] * (1.0 / kPi);
    double2 *d = reinterpret_cast<double2 *>(src + 8 * j);
    d[0] = make_double2(x[j], y[j]);
    d[1] = make_double2(s * nx[j], s * ny[j]);
    d[2] = make_double2(u[j], u[nn + j]);
    d[3] = make_double2(0.0, 0.0);
  }
  if (j < m) {
    const double *lam = u + 2 * nn + 3 * j;
    double2 *d = reinterpret_cast<double2 *>(psrc + 8 * j);
    d[0] = make_double2(cx[j], cy[j]);
    d[1] = make_double2(lam[0], lam[1]);
    d[2] = make_double2(rad[j] * lam[2], 0.0);
    d[3] = make_double2(0.0, 0.0);
  }
}

// scal[0] = sum over wall nodes of w (n . sigma); scal[1] = sum of w.
__global__ void wall_flux(int64_t wall_start, int64_t nn,
                          const double *__restrict__ nx,
                          const double *__restrict__ ny,
                          const double *__restrict__ w,
                          const double *__restrict__ u, double *scal,
                          int with_flux) {
  __shared__ double sb[1024], sl[1024];
  double b = 0.0, l = 0.0;
  for (int64_t i = wall_start + threadIdx.x; i < nn; i += blockDim.x) {
    l += w[i];
    if (with_flux) b += w[i] * (nx[i] * u[i] + ny[i] * u[nn + i]);
  }
  sb[threadIdx.x] = b;
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sb[threadIdx.x] += sb[threadIdx.x + s];
      sl[threadIdx.x] += sl[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[0] = sb[0];
    scal[1] = sl[0];
  }
}

// s + c += x with the rounding error of the addition carried in c (Knuth's
// two-sum): used by the compensated mode, whose residuals must resolve
// 1e-10 of the data when the density is much larger than the data.
__device__ __forceinline__ void two_sum_acc(double &s, double &c, double x) {
#pragma clang fp contract(off)
  const double t = s + x;
  const double bp = t - s;
  c += (s - (t - bp)) + (x - bp);
  s = t;
}

// 1/d to full FP64 precision: hardware reciprocal estimate refined by one
// third-order Newton step, r' = r (1 + e + e^2) with e = 1 - d r.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Reciprocals of T positive numbers with one hardware reciprocal: the
// product of all of them is inverted (and refined) once, and each 1/d_t is
// recovered as that inverse times the product of the others (Montgomery's
// batch-inversion trick).  The d_t are squared distances between nodes, so
// their product stays far inside the FP64 range.
template <int T>
__device__ __forceinline__ void batch_recip(const double *d, double *out) {
  if (T == 1) {
    out[0] = recip(d[0]);
  } else if (T == 2) {
    const double r = recip(d[0] * d[1]);
    out[0] = r * d[1];
    out[1] = r * d[0];
  } else if (T == 4) {
    const double p01 = d[0] * d[1], p23 = d[2] * d[3];
    const double r = recip(p01 * p23);
    const double r01 = r * p23, r23 = r * p01;
    out[0] = r01 * d[1];
    out[1] = r01 * d[0];
    out[2] = r23 * d[3];
    out[3] = r23 * d[2];
  } else {
#pragma unroll
    for (int h = 0; h < T; h += 4) batch_recip<4>(d + h, out + h);
  }
}

template <int T, bool ACC>
__global__ __launch_bounds__(kBlock) void dlp_pairs(
    const double *__restrict__ src, const double *__restrict__ xs,
    const double *__restrict__ ys, int64_t nn, int64_t chunk,
    double *__restrict__ part) {
  const int64_t tile0 = (int64_t)blockIdx.x * (kBlock * T) + threadIdx.x;
  double xi[T], yi[T], ax[T], ay[T], cxa[T], cya[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int64_t i = tile0 + (int64_t)t * kBlock;
    // padding targets of the last tile sit far away from every node and at
    // distinct places, so at most one target per thread can coincide with a
    // source (the batched reciprocal multiplies the squared distances)
    xi[t] = i < nn ? xs[i] : xs[nn - 1] + 1.0e3 * (double)(t + 1);
    yi[t] = i < nn ? ys[i] : ys[nn - 1];
    ax[t] = 0.0;
    ay[t] = 0.0;
    cxa[t] = 0.0;
    cya[t] = 0.0;
  }
  // uniform loop bounds kept in scalar registers
  const int64_t j0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * chunk));
  int64_t j1 = j0 + chunk < nn ? j0 + chunk : nn;
  j1 = __builtin_amdgcn_readfirstlane((int)j1);
  for (int64_t j = j0; j < j1; ++j) {
    const double *s = src + 8 * j;  // wave-uniform: scalar loads
    const double sx = s[0], sy = s[1], sax = s[2], say = s[3], ssx = s[4],
                 ssy = s[5];
    double rx[T], ry[T], r2[T], inv[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      rx[t] = xi[t] - sx;
      ry[t] = yi[t] - sy;
      // the self pair has r = 0 exactly: clamping rho^2 keeps 1/rho^4 finite
      // and the pair's factors (r.a)(r.sigma) are exactly zero
      r2[t] = fmax(fma(ry[t], ry[t], rx[t] * rx[t]), 1e-100);
    }
    batch_recip<T>(r2, inv);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const double dn = fma(ry[t], say, rx[t] * sax);
      const double ds = fma(ry[t], ssy, rx[t] * ssx);
      const double c = (dn * ds) * (inv[t] * inv[t]);
      if (ACC) {
        two_sum_acc(ax[t], cxa[t], c * rx[t]);
        two_sum_acc(ay[t], cya[t], c * ry[t]);
      } else {
        ax[t] = fma(c, rx[t], ax[t]);
        ay[t] = fma(c, ry[t], ay[t]);
      }
    }
  }
  double *px = part + (int64_t)blockIdx.y * 4 * nn;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int64_t i = tile0 + (int64_t)t * kBlock;
    if (i < nn) {
      px[i] = ax[t];
      px[nn + i] = ay[t];
      if (ACC) {
        px[2 * nn + i] = cxa[t];
        px[3 * nn + i] = cya[t];
      }
    }
  }
}

// Stokeslet + rotlet columns: sum over pores of S(x_i - c_k) lambda_k
// + r_k R(x_i - c_k) mu_k, without the 1/(4 pi) (applied in the epilogue).
template <bool ACC>
__global__ __launch_bounds__(kBlock) void completion_pairs(
    const double *__restrict__ psrc, const double *__restrict__ xs,
    const double *__restrict__ ys, int64_t nn, int m,
    double *__restrict__ part) {
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < nn ? i0 : nn - 1;
  const double xi = xs[i], yi = ys[i];
  double ax = 0.0, ay = 0.0, cxa = 0.0, cya = 0.0;
  const int k0 = blockIdx.y * kPoreChunk;
  const int k1 = k0 + kPoreChunk < m ? k0 + kPoreChunk : m;
  for (int k = k0; k < k1; ++k) {
    const double *p = psrc + 8 * k;
    const double qx = xi - p[0], qy = yi - p[1];
    const double lx = p[2], ly = p[3], rmu = p[4];
    const double q2 = fma(qy, qy, qx * qx);
    const double inv = 1.0 / q2;
    const double lg = 0.5 * log(q2);
    const double dot = fma(qy, ly, qx * lx) * inv;
    const double tx = -lg * lx + qx * dot + rmu * qy * inv;
    const double ty = -lg * ly + qy * dot - rmu * qx * inv;
    if (ACC) {
      two_sum_acc(ax, cxa, tx);
      two_sum_acc(ay, cya, ty);
    } else {
      ax += tx;
      ay += ty;
    }
  }
  if (i0 < nn) {
    double *px = part + (int64_t)blockIdx.y * 4 * nn;
    px[i0] = ax;
    px[nn + i0] = ay;
    if (ACC) {
      px[2 * nn + i0] = cxa;
      px[3 * nn + i0] = cya;
    }
  }
}

__global__ void epilogue(int64_t nn, int64_t wall_start, int nchunks,
                         int npchunks, int full, int acc,
                         const double *__restrict__ part,
                         const double *__restrict__ nx,
                         const double *__restrict__ ny,
                         const double *__restrict__ w,
                         const double *__restrict__ kappa,
                         const double *__restrict__ u,
                         const double *__restrict__ scal,
                         double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  // (value, error) pairs; the error parts are only used in the compensated
  // mode, where every addition below is a two-sum
  double vx = 0.0, vy = 0.0, ex = 0.0, ey = 0.0;
  auto add = [&](double &v, double &e, double a) {
    if (acc) two_sum_acc(v, e, a); else v += a;
  };
  for (int c = 0; c < nchunks; ++c) {
    const double *p = part + (int64_t)c * 4 * nn;
    add(vx, ex, p[i]);
    add(vy, ey, p[nn + i]);
    if (acc) {
      ex += p[2 * nn + i];
      ey += p[3 * nn + i];
    }
  }
  const double sx = u[i], sy = u[nn + i];
  const double tx = -ny[i], ty = nx[i];
  const double d = w[i] * kappa[i] * (0.5 / kPi) * (tx * sx + ty * sy);
  add(vx, ex, d * tx);
  add(vy, ey, d * ty);
  if (full) {
    double cx = 0.0, cy = 0.0, ecx = 0.0, ecy = 0.0;
    for (int c = 0; c < npchunks; ++c) {
      const double *p = part + (int64_t)(nchunks + c) * 4 * nn;
      add(cx, ecx, p[i]);
      add(cy, ecy, p[nn + i]);
      if (acc) {
        ecx += p[2 * nn + i];
        ecy += p[3 * nn + i];
      }
    }
    add(vx, ex, cx * (0.25 / kPi));
    add(vx, ex, ecx * (0.25 / kPi));
    add(vy, ey, cy * (0.25 / kPi));
    add(vy, ey, ecy * (0.25 / kPi));
    add(vx, ex, -0.5 * sx);
    add(vy, ey, -0.5 * sy);
    if (i >= wall_start) {
      const double f = scal[0] / scal[1];
      add(vx, ex, nx[i] * f);
      add(vy, ey, ny[i] * f);
    }
  }
  out[i] = vx + ex;
  out[nn + i] = vy + ey;
}

// One wave per pore: the constraint rows lambda_k and mu_k.
__global__ void pore_rows(int64_t nn, int m, const int64_t *__restrict__ off,
                          const double *__restrict__ x,
                          const double *__restrict__ y,
                          const double *__restrict__ w,
                          const double *__restrict__ cx,
                          const double *__restrict__ cy,
                          const double *__restrict__ rad,
                          const double *__restrict__ u, int full,
                          double *__restrict__ out) {
  const int k = blockIdx.x;
  if (k >= m) return;
  double sx = 0.0, sy = 0.0, sm = 0.0;
  if (full) {
    const int64_t a = off[k], b = off[k + 1];
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      const double ux = u[j], uy = u[nn + j];
      sx += w[j] * ux;
      sy += w[j] * uy;
      // (x_j - c_k)_perp . sigma = (y_j - cy) ux - (x_j - cx) uy
      sm += w[j] * ((y[j] - cy[k]) * ux - (x[j] - cx[k]) * uy);
    }
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_down(sx, o, 64);
      sy += __shfl_down(sy, o, 64);
      sm += __shfl_down(sm, o, 64);
    }
  }
  if (threadIdx.x == 0) {
    double *o = out + 2 * nn + 3 * (int64_t)k;
    if (full) {
      const double *lam = u + 2 * nn + 3 * (int64_t)k;
      const double r = rad[k];
      o[0] = sx / (2.0 * kPi * r) - lam[0];
      o[1] = sy / (2.0 * kPi * r) - lam[1];
      o[2] = sm / (2.0 * kPi * r * r) - lam[2];
    } else {
      o[0] = o[1] = o[2] = 0.0;
    }
  }
}

__global__ void wall_length_kernel(int64_t wall_start, int64_t nn,
                                   const double *__restrict__ w, double *out) {
  __shared__ double sl[256];
  double l = 0.0;
  for (int64_t i = wall_start + threadIdx.x; i < nn; i += blockDim.x) l += w[i];
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sl[threadIdx.x] += sl[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sl[0];
}

}  // namespace

size_t MatvecWork::doubles() const { return 0; }

MatvecWork plan_matvec(const sbie_geom *g) {
  MatvecWork w;
  w.tpt = g_tpt;
  const int64_t nn = g->n_nodes;
  const int64_t tiles = ceil_div(nn, (int64_t)kBlock * w.tpt);
  if (g_chunks > 0) {
    w.chunks = g_chunks;
  } else {
    int64_t want = (4096 + tiles - 1) / tiles;
    int64_t cap = (nn + 127) / 128;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    w.chunks = (int)want;
  }
  if ((int64_t)w.chunks > nn) w.chunks = (int)nn;
  w.pchunks = g->n_pores > 0 ? (int)ceil_div(g->n_pores, kPoreChunk) : 0;
  return w;
}

size_t matvec_scratch_doubles(const MatvecWork &w, const sbie_geom *g) {
  const int64_t nn = g->n_nodes;
  return (size_t)8 * nn + (size_t)8 * (g->n_pores + 1) +
         (size_t)(w.chunks + w.pchunks) * 4 * nn + 8;
}

void bind_matvec_scratch(MatvecWork &w, const sbie_geom *g, double *base) {
  const int64_t nn = g->n_nodes;
  w.src = base;
  w.psrc = w.src + 8 * nn;
  w.part = w.psrc + 8 * (g->n_pores + 1);
  w.scal = w.part + (size_t)(w.chunks + w.pchunks) * 4 * nn;
}

void matvec_run(const sbie_geom *g, const double *x, double *y, int mode,
                MatvecWork &w, hipStream_t s) {
  const int64_t nn = g->n_nodes;
  const int m = g->n_pores;
  const int full = mode == SBIE_MV_FULL || mode == SBIE_MV_FULL_ACCURATE;
  const bool acc = mode == SBIE_MV_FULL_ACCURATE;
  const int64_t wall_start = g->curve_off[m];
  const int64_t packn = nn > m ? nn : m;
  pack_sources<<<ceil_div(packn, 256), 256, 0, s>>>(
      nn, m, g->x, g->y, g->nx, g->ny, g->w, g->radius, g->cx, g->cy, x,
      w.src, w.psrc);
  SBIE_LAUNCH_CHECK();
  if (full) {
    wall_flux<<<1, 1024, 0, s>>>(wall_start, nn, g->nx, g->ny, g->w, x, w.scal, 1);
    SBIE_LAUNCH_CHECK();
  }
  const int64_t chunk = (nn + w.chunks - 1) / w.chunks;
  dim3 grid(ceil_div(nn, (int64_t)kBlock * w.tpt), w.chunks);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // only the plain pair kernel is timed (the compensated one is a
  // different kernel, launched for true residuals)
  if (g_timing && !acc) {
    SBIE_HIP(hipEventCreate(&ev0));
    SBIE_HIP(hipEventCreate(&ev1));
    SBIE_HIP(hipEventRecord(ev0, s));
  }
  if (acc) {
    dlp_pairs<1, true><<<dim3(ceil_div(nn, kBlock), w.chunks), kBlock, 0, s>>>(
        w.src, g->x, g->y, nn, chunk, w.part);
  } else {
    switch (w.tpt) {
      case 1: dlp_pairs<1, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, chunk, w.part); break;
      case 2: dlp_pairs<2, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, chunk, w.part); break;
      case 4: dlp_pairs<4, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, chunk, w.part); break;
      case 8: dlp_pairs<8, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, chunk, w.part); break;
      default: fail(SBIE_INVALID_ARGUMENT, "targets per thread must be 1, 2, 4 or 8");
    }
  }
  SBIE_LAUNCH_CHECK();
  if (g_timing && !acc) {
    SBIE_HIP(hipEventRecord(ev1, s));
    g_events.emplace_back(ev0, ev1);
  }
  if (full && m > 0) {
    dim3 pg(ceil_div(nn, kBlock), w.pchunks);
    if (acc)
      completion_pairs<true><<<pg, kBlock, 0, s>>>(w.psrc, g->x, g->y, nn, m,
                                                   w.part + (size_t)w.chunks * 4 * nn);
    else
      completion_pairs<false><<<pg, kBlock, 0, s>>>(w.psrc, g->x, g->y, nn, m,
                                                    w.part + (size_t)w.chunks * 4 * nn);
    SBIE_LAUNCH_CHECK();
  }
  epilogue<<<ceil_div(nn, 256), 256, 0, s>>>(nn, wall_start, w.chunks,
                                             full ? w.pchunks : 0, full, acc ? 1 : 0, w.part,
                                             g->nx, g->ny, g->w, g->kappa, x,
                                             w.scal, y);
  SBIE_LAUNCH_CHECK();
  if (m > 0) {
    pore_rows<<<m, 64, 0, s>>>(nn, m, g->curve_off_dev, g->x, g->y, g->w,
                               g->cx, g->cy, g->radius, x, full, y);
    SBIE_LAUNCH_CHECK();
  }
}

void wall_length(const sbie_geom *g, double *out, hipStream_t s) {
  wall_length_kernel<<<1, 256, 0, s>>>(g->curve_off[g->n_pores], g->n_nodes,
                                       g->w, out);
  SBIE_LAUNCH_CHECK();
}

}  // namespace sbie

extern "C" int stokes_dlp_matvec(const sbie_geom *g, const double *x, double *y,
                                 int mode, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!x || !y) sbie::fail(SBIE_INVALID_ARGUMENT, "null vector");
    if (mode != SBIE_MV_FULL && mode != SBIE_MV_DLP_ONLY && mode != SBIE_MV_FULL_ACCURATE)
      sbie::fail(SBIE_INVALID_ARGUMENT, "unknown matvec mode %d", mode);
    const int64_t n = sbie::n_unknowns(g);
    if (x < y + n && y < x + n)
      sbie::fail(SBIE_INVALID_ARGUMENT, "x and y overlap");
    hipStream_t s = (hipStream_t)stream;
    sbie::MatvecWork w = sbie::plan_matvec(g);
    sbie::StreamBuf<double> scratch(sbie::matvec_scratch_doubles(w, g), s);
    sbie::bind_matvec_scratch(w, g, scratch.p);
    sbie::matvec_run(g, x, y, mode, w, s);
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_set_shape(int targets_per_thread,
                                           int source_chunks) {
  return sbie::guarded([&]() {
    if (targets_per_thread != 1 && targets_per_thread != 2 &&
        targets_per_thread != 4 && targets_per_thread != 8)
      sbie::fail(SBIE_INVALID_ARGUMENT, "targets per thread must be 1, 2, 4 or 8");
    if (source_chunks < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "source_chunks < 0");
    sbie::g_tpt = targets_per_thread;
    sbie::g_chunks = source_chunks;
    return SBIE_OK;
  });
}

extern "C" int sbie_kernel_timing(int enable) {
  return sbie::guarded([&]() {
    sbie::g_timing = enable != 0;
    return SBIE_OK;
  });
}

extern "C" int sbie_kernel_time(double *total_ms, int64_t *launches) {
  return sbie::guarded([&]() {
    if (!total_ms || !launches) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    double tot = 0.0;
    for (auto &e : sbie::g_events) {
      SBIE_HIP(hipEventSynchronize(e.second));
      float ms = 0.0f;
      SBIE_HIP(hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    *total_ms = tot;
    *launches = (int64_t)sbie::g_events.size();
    sbie::g_events.clear();
    return SBIE_OK;
  });
}
