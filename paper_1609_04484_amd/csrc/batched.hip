// Variable-size batched dense kernels (double and float instantiations).
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>

#include "batched.hpp"

namespace sbie {

// ----------------------------------------------------------------------------
// Descriptor staging
// ----------------------------------------------------------------------------

Stager::Stager(size_t bytes) : cap(bytes) {
  SBIE_HIP(hipHostMalloc((void **)&host, bytes, hipHostMallocDefault));
  dev.alloc(bytes);
}

Stager::~Stager() {
  if (host) (void)hipHostFree(host);
}

namespace {
std::mutex g_stager_mu;
std::map<int, std::vector<Stager *>> g_stager_pool;   // idle rings per device, kept until exit
}  // namespace

StagerLease::StagerLease(size_t bytes, hipStream_t s) : s_(s) {
  SBIE_HIP(hipGetDevice(&dev_));
  {
    std::lock_guard<std::mutex> lk(g_stager_mu);
    auto &v = g_stager_pool[dev_];
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i]->cap >= bytes) {
        st_ = v[i];
        v.erase(v.begin() + (std::ptrdiff_t)i);
        break;
      }
  }
  if (!st_) st_ = new Stager(bytes);
  st_->reset();
}

StagerLease::~StagerLease() {
  if (std::uncaught_exceptions() > 0) (void)hipStreamSynchronize(s_);
  std::lock_guard<std::mutex> lk(g_stager_mu);
  g_stager_pool[dev_].push_back(st_);
}

HostProf &host_prof() {
  thread_local HostProf h;
  return h;
}

OpFlops &op_flops() {
  thread_local OpFlops f;
  return f;
}

void *Stager::put(const void *src, size_t bytes, hipStream_t s) {
  HostScope hs(HostProf::kStage);
  const size_t need = (bytes + 255) & ~size_t(255);
  if (need > cap) fail(SBIE_OUT_OF_MEMORY, "descriptor batch of %zu bytes exceeds staging", bytes);
  if (used + need > cap) {
    // every earlier copy and every kernel reading earlier descriptors must
    // finish before the rings are reused
    SBIE_HIP(hipStreamSynchronize(s));
    used = 0;
  }
  std::memcpy(host + used, src, bytes);
  SBIE_HIP(hipMemcpyAsync(dev.p + used, host + used, bytes, hipMemcpyHostToDevice, s));
  void *d = dev.p + used;
  used += need;
  return d;
}

void Stager::put_many(const std::vector<std::pair<const void *, size_t>> &parts, std::vector<void *> &dst,
                      hipStream_t s) {
  HostScope hs(HostProf::kStage);
  size_t need = 0;
  for (const auto &p : parts) need += (p.second + 255) & ~size_t(255);
  if (need > cap) fail(SBIE_OUT_OF_MEMORY, "descriptor batch of %zu bytes exceeds staging", need);
  if (used + need > cap) {
    SBIE_HIP(hipStreamSynchronize(s));
    used = 0;
  }
  dst.resize(parts.size());
  size_t o = used;
  for (size_t i = 0; i < parts.size(); ++i) {
    if (parts[i].second) std::memcpy(host + o, parts[i].first, parts[i].second);
    dst[i] = dev.p + o;
    o += (parts[i].second + 255) & ~size_t(255);
  }
  SBIE_HIP(hipMemcpyAsync(dev.p + used, host + used, o - used, hipMemcpyHostToDevice, s));
  used = o;
}

namespace {

constexpr int kBlockedMin = 48;  // larger matrices use the blocked inverse
constexpr int kPanel = 32;

// ----------------------------------------------------------------------------
// GEMM: one 64 x 64 output tile per workgroup, 256 threads (four waves, each a
// 32 x 32 quarter), on the matrix cores
// ----------------------------------------------------------------------------
// FP64 GEMM tile: the output tile is staged through LDS in k-slabs of 16
// (double-buffered), with each of the four waves computing a 32 x 32 quarter as
// 2 x 2 blocks of v_mfma_f64_16x16x4.  Operand layout of that instruction
// (checked on the device): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16], and register v of lane l receives D[l / 16 + 4 v][l % 16].
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// Panel step of the blocked Gauss-Jordan (FP64): rows [k0, k0 + pb) of the
// output take CP (pb x n, leading dimension pb), the other rows of columns
// [k0, k0 + pb) take R (m x pb, leading dimension m), every other entry the
// GEMM update; the values two copies and a product used to write over the
// update afterwards.
struct GjFix {
  const double *R, *CP;
  int k0, pb;
};

template <bool GJ>
__device__ __forceinline__ void gemm_tile_f64(const GemmDesc<double> *__restrict__ descs,
                                              const int2 *__restrict__ tiles, const GjFix *__restrict__ fixes) {
  const int2 tl = tiles[blockIdx.x];
  const GemmDesc<double> d = descs[tl.x];
  const int tiles_m = (d.m + 63) >> 6;
  const int row0 = (tl.y % tiles_m) * 64;
  const int col0 = (tl.y / tiles_m) * 64;
  // two LDS stages: while one is multiplied out, the next k-slab's global
  // values are loaded into registers and then stored into the other stage,
  // so each slab takes one barrier
  __shared__ double As[2][16][65];
  __shared__ double Bs[2][16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  mfma_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  double ra[4], rb[4];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int r, kk;
      if (!d.ta) { r = e & 63; kk = e >> 6; } else { kk = e & 15; r = e >> 4; }
      const int gi = row0 + r, gk = k0 + kk;
      ra[q] = (gi < d.m && gk < d.k) ? (d.ta ? d.A[gk + (size_t)gi * d.lda] : d.A[gi + (size_t)gk * d.lda]) : 0.0;
      int c;
      if (!d.tb) { kk = e & 15; c = e >> 4; } else { c = e & 63; kk = e >> 6; }
      const int gj = col0 + c, gk2 = k0 + kk;
      rb[q] = (gj < d.n && gk2 < d.k) ? (d.tb ? d.B[gj + (size_t)gk2 * d.ldb] : d.B[gk2 + (size_t)gj * d.ldb]) : 0.0;
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if (!d.ta) As[buf][e >> 6][e & 63] = ra[q]; else As[buf][e & 15][e >> 4] = ra[q];
      if (!d.tb) Bs[buf][e & 15][e >> 4] = rb[q]; else Bs[buf][e >> 6][e & 63] = rb[q];
    }
  };
  if (d.k > 0) {
    load_stage(0);
    store_stage(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < d.k; k0 += 16) {
      const bool more = k0 + 16 < d.k;
      if (more) load_stage(k0 + 16);
#pragma unroll
      for (int ks = 0; ks < 16; ks += 4) {
        double a[2], b[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          a[q] = As[cur][ks + lk][wr + 16 * q + li];
          b[q] = Bs[cur][ks + lk][wc + 16 * q + li];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
      }
      // the other stage was last read before the previous barrier
      if (more) store_stage(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wr + 16 * x + lk + 4 * v;
        const int c = col0 + wc + 16 * y + li;
        if (r >= d.m || c >= d.n) continue;
        double *p = d.C + r + (size_t)c * d.ldc;
        if constexpr (GJ) {
          const GjFix &f = fixes[tl.x];
          if (r >= f.k0 && r < f.k0 + f.pb) {
            *p = f.CP[(r - f.k0) + (size_t)c * f.pb];
            continue;
          }
          if (c >= f.k0 && c < f.k0 + f.pb) {
            *p = f.R[r + (size_t)(c - f.k0) * d.m];
            continue;
          }
        }
        double val = d.alpha * acc[x][y][v];
        if (d.beta != 0.0) val = fma(d.beta, *p, val);
        *p = val;
      }
}

__global__ __launch_bounds__(256) void gemm_tiles_mfma(const GemmDesc<double> *__restrict__ descs,
                                                       const int2 *__restrict__ tiles) {
  gemm_tile_f64<false>(descs, tiles, nullptr);
}

__global__ __launch_bounds__(256) void gemm_tiles_mfma_gj(const GemmDesc<double> *__restrict__ descs,
                                                          const int2 *__restrict__ tiles,
                                                          const GjFix *__restrict__ fixes) {
  gemm_tile_f64<true>(descs, tiles, fixes);
}

// FP32 GEMM tile on the matrix cores: the same 64 x 64 tiles, LDS staging
// and 2 x 2 blocks per wave as gemm_tiles_mfma, with v_mfma_f32_16x16x4f32
// (FP32 products accumulated in FP32).  Operand layout as for the FP64
// instruction (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]); the
// result layout differs (checked on the device): register v of lane l
// receives D[4 (l / 16) + v][l % 16].
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gemm_tiles_mfma_f32(const GemmDesc<float> *__restrict__ descs,
                                                           const int2 *__restrict__ tiles) {
  const int2 tl = tiles[blockIdx.x];
  const GemmDesc<float> d = descs[tl.x];
  const int tiles_m = (d.m + 63) >> 6;
  const int row0 = (tl.y % tiles_m) * 64;
  const int col0 = (tl.y / tiles_m) * 64;
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  mfma_f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  float ra[4], rb[4];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int r, kk;
      if (!d.ta) { r = e & 63; kk = e >> 6; } else { kk = e & 15; r = e >> 4; }
      const int gi = row0 + r, gk = k0 + kk;
      ra[q] = (gi < d.m && gk < d.k) ? (d.ta ? d.A[gk + (size_t)gi * d.lda] : d.A[gi + (size_t)gk * d.lda]) : 0.f;
      int c;
      if (!d.tb) { kk = e & 15; c = e >> 4; } else { c = e & 63; kk = e >> 6; }
      const int gj = col0 + c, gk2 = k0 + kk;
      rb[q] = (gj < d.n && gk2 < d.k) ? (d.tb ? d.B[gj + (size_t)gk2 * d.ldb] : d.B[gk2 + (size_t)gj * d.ldb]) : 0.f;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if (!d.ta) As[e >> 6][e & 63] = ra[q]; else As[e & 15][e >> 4] = ra[q];
      if (!d.tb) Bs[e & 15][e >> 4] = rb[q]; else Bs[e >> 6][e & 63] = rb[q];
    }
  };
  if (d.k > 0) load_stage(0);
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    store_stage();
    __syncthreads();
    if (k0 + 16 < d.k) load_stage(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      float a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a[q] = As[ks + lk][wr + 16 * q + li];
        b[q] = Bs[ks + lk][wc + 16 * q + li];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wr + 16 * x + 4 * lk + v;
        const int c = col0 + wc + 16 * y + li;
        if (r >= d.m || c >= d.n) continue;
        float *p = d.C + r + (size_t)c * d.ldc;
        float val = d.alpha * acc[x][y][v];
        if (d.beta != 0.f) val = fmaf(d.beta, *p, val);
        *p = val;
      }
}

// Products with FP16 or BF16 inputs on the matrix cores and FP32
// accumulation (v_mfma_f32_16x16x16f16 / v_mfma_f32_16x16x16bf16_1k), for
// the Gaussian sketches of the recompression, whose results only have to
// span the right column space.  alpha is applied to A in the descriptor's
// precision before the operand is rounded (the callers' alpha is a
// reciprocal block norm, so the rounded entries stay within FP16's range);
// the output is the FP32 accumulator widened to T, plus beta C.  Operand
// layout (checked on the device for both instructions): lane l supplies
// A[l % 16][4 (l / 16) + q] and B[4 (l / 16) + q][l % 16], q = 0..3; results
// as for the FP32 instruction, D[4 (l / 16) + v][l % 16].
typedef _Float16 mfma_h4 __attribute__((ext_vector_type(4)));
typedef short mfma_s4 __attribute__((ext_vector_type(4)));

// FP32 to BF16 bits, rounding to nearest even (finite inputs only).
__device__ __forceinline__ short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <class T, GemmInputs L>
__global__ __launch_bounds__(256) void gemm_tiles_mfma_lowin(const GemmDesc<T> *__restrict__ descs,
                                                             const int2 *__restrict__ tiles) {
  const int2 tl = tiles[blockIdx.x];
  const GemmDesc<T> d = descs[tl.x];
  const int tiles_m = (d.m + 63) >> 6;
  const int row0 = (tl.y % tiles_m) * 64;
  const int col0 = (tl.y / tiles_m) * 64;
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  mfma_f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  float ra[4], rb[4];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int r, kk;
      if (!d.ta) { r = e & 63; kk = e >> 6; } else { kk = e & 15; r = e >> 4; }
      const int gi = row0 + r, gk = k0 + kk;
      ra[q] = (gi < d.m && gk < d.k)
                  ? (float)(d.alpha * (d.ta ? d.A[gk + (size_t)gi * d.lda] : d.A[gi + (size_t)gk * d.lda]))
                  : 0.f;
      int c;
      if (!d.tb) { kk = e & 15; c = e >> 4; } else { c = e & 63; kk = e >> 6; }
      const int gj = col0 + c, gk2 = k0 + kk;
      rb[q] = (gj < d.n && gk2 < d.k) ? (float)(d.tb ? d.B[gj + (size_t)gk2 * d.ldb] : d.B[gk2 + (size_t)gj * d.ldb])
                                      : 0.f;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if (!d.ta) As[e >> 6][e & 63] = ra[q]; else As[e & 15][e >> 4] = ra[q];
      if (!d.tb) Bs[e & 15][e >> 4] = rb[q]; else Bs[e >> 6][e & 63] = rb[q];
    }
  };
  if (d.k > 0) load_stage(0);
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    store_stage();
    __syncthreads();
    if (k0 + 16 < d.k) load_stage(k0 + 16);
    if constexpr (L == GemmInputs::kF16) {
      mfma_h4 a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          a[q][h] = (_Float16)As[4 * lk + h][wr + 16 * q + li];
          b[q][h] = (_Float16)Bs[4 * lk + h][wc + 16 * q + li];
        }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[x], b[y], acc[x][y], 0, 0, 0);
    } else {
      mfma_s4 a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          a[q][h] = bf16_bits(As[4 * lk + h][wr + 16 * q + li]);
          b[q][h] = bf16_bits(Bs[4 * lk + h][wc + 16 * q + li]);
        }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wr + 16 * x + 4 * lk + v;
        const int c = col0 + wc + 16 * y + li;
        if (r >= d.m || c >= d.n) continue;
        T *p = d.C + r + (size_t)c * d.ldc;
        T val = (T)acc[x][y][v];
        if (d.beta != T(0)) val = fma(d.beta, *p, val);
        *p = val;
      }
}

// FP64 and FP32 products go to the matrix cores in their own precision, or
// with inputs rounded to FP16 or BF16 when the caller asks for it.
template <class T>
void launch_gemm_tiles(unsigned nt, const GemmDesc<T> *dd, const int2 *td, hipStream_t s, GemmInputs in) {
  HostScope hs(HostProf::kLaunch);
  if (in == GemmInputs::kF16)
    gemm_tiles_mfma_lowin<T, GemmInputs::kF16><<<nt, 256, 0, s>>>(dd, td);
  else if (in == GemmInputs::kBF16)
    gemm_tiles_mfma_lowin<T, GemmInputs::kBF16><<<nt, 256, 0, s>>>(dd, td);
  else if constexpr (std::is_same<T, double>::value)
    gemm_tiles_mfma<<<nt, 256, 0, s>>>(dd, td);
  else
    gemm_tiles_mfma_f32<<<nt, 256, 0, s>>>(dd, td);
  SBIE_LAUNCH_CHECK();
}

// ----------------------------------------------------------------------------
// GEMV: one workgroup per descriptor (at most 64 rows)
// ----------------------------------------------------------------------------
// The GEMV is bound by how many loads each workgroup keeps in flight: a
// descriptor (at most 64 rows) gets 16 waves.  Untransposed terms: lane =
// row, wave w takes columns w, w + 16, ... with four independent chains;
// transposed terms: wave w takes rows w, w + 16, w + 32, w + 48, lanes
// stride over the columns.  Partial sums meet in LDS.
constexpr int kGemvThreads = 1024;
constexpr int kGemvWaves = kGemvThreads / 64;

// a double moved between lanes by the DPP control CTRL (both halves)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Maximum over the 64 lanes of a wave, returned in every lane (all lanes
// active, no NaN inputs): lane pairs, quads, half rows and rows of 16 by
// DPP, then the four row maxima read from lanes 0, 16, 32 and 48.
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));    // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));    // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));   // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));   // row_mirror
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Minimum of an int over the 64 lanes of a wave, returned in every lane
// (all lanes active), by the same exchanges.
__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// An empty instruction that takes the 32 values as operands: every value
// must be in a register at this point, so their loads are issued together
// instead of one or two at a time between the arithmetic that uses them.
// Lane i < 32 receives lane i + 32 (v_permlane32_swap of v with itself), and
// lane i < 16 receives lane i + 16 (v_permlane16_swap); lane layouts checked
// on the device.
__device__ __forceinline__ double lane_plus32(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_permlane32_swap(hi, hi, false, false)[1],
                          __builtin_amdgcn_permlane32_swap(lo, lo, false, false)[1]);
}
__device__ __forceinline__ double lane_plus16(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_permlane16_swap(hi, hi, false, false)[1],
                          __builtin_amdgcn_permlane16_swap(lo, lo, false, false)[1]);
}

// Sum over the wave as the shfl_down tree forms it (halving distances 32,
// 16, ..., 1), exact in lane 0 only: the two long distances by lane swaps,
// the four within a row of 16 lanes by DPP row shifts (lane i receives lane
// i + d), with the same additions in the same order.
__device__ __forceinline__ double wave_sum_lane0(double v) {
  v += lane_plus32(v);
  v += lane_plus16(v);
  v += dpp_f64<0x108>(v);   // row_shl:8
  v += dpp_f64<0x104>(v);   // row_shl:4
  v += dpp_f64<0x102>(v);   // row_shl:2
  v += dpp_f64<0x101>(v);   // row_shl:1
  return v;
}
__device__ __forceinline__ float wave_sum_lane0(float v) {
  auto mv = [](float x, auto ctrl) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), decltype(ctrl)::value, 0xF, 0xF, false));
  };
  v += __int_as_float(__builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false)[1]);
  v += __int_as_float(__builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false)[1]);
  v += mv(v, std::integral_constant<int, 0x108>{});
  v += mv(v, std::integral_constant<int, 0x104>{});
  v += mv(v, std::integral_constant<int, 0x102>{});
  v += mv(v, std::integral_constant<int, 0x101>{});
  return v;
}

template <class T, class TA>
__global__ __launch_bounds__(kGemvThreads) void gemv_desc(const GemvDesc<T> *__restrict__ descs,
                                                          const GemvTerm<T, TA> *__restrict__ terms) {
  const GemvDesc<T> d = descs[blockIdx.x];
  __shared__ T part[kGemvWaves][64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T acc = T(0);        // untransposed: this thread's partial for row `lane`
  T accw[4];           // transposed: rows wv, wv + 16, wv + 32, wv + 48
#pragma unroll
  for (int q = 0; q < 4; ++q) accw[q] = T(0);
  for (int t = d.t0; t < d.t0 + d.nt; ++t) {
    const GemvTerm<T, TA> tm = terms[t];
    if (!tm.trans) {
      T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
      if (lane < d.rows) {
        const TA *a = tm.A + lane;
        int c = wv;
        for (; c + 3 * kGemvWaves < tm.cols; c += 4 * kGemvWaves) {
          s0 = fma((T)a[(size_t)c * tm.lda], tm.x[c], s0);
          s1 = fma((T)a[(size_t)(c + kGemvWaves) * tm.lda], tm.x[c + kGemvWaves], s1);
          s2 = fma((T)a[(size_t)(c + 2 * kGemvWaves) * tm.lda], tm.x[c + 2 * kGemvWaves], s2);
          s3 = fma((T)a[(size_t)(c + 3 * kGemvWaves) * tm.lda], tm.x[c + 3 * kGemvWaves], s3);
        }
        for (; c < tm.cols; c += kGemvWaves) s0 = fma((T)a[(size_t)c * tm.lda], tm.x[c], s0);
      }
      acc = fma(tm.alpha, (s0 + s1) + (s2 + s3), acc);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wv + kGemvWaves * q;
        if (r >= d.rows) break;
        const TA *col = tm.A + (size_t)r * tm.lda;
        T s = T(0);
        for (int c = lane; c < tm.cols; c += 64) s = fma((T)col[c], tm.x[c], s);
        s = wave_sum_lane0(s);
        if (lane == 0) accw[q] = fma(tm.alpha, s, accw[q]);
      }
    }
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = wv + kGemvWaves * q;
      if (r < d.rows) part[wv][r] += accw[q];
    }
  }
  __syncthreads();
  if (tid < d.rows) {
    T v = T(0);
#pragma unroll
    for (int w = 0; w < kGemvWaves; w += 4)
      v += (part[w][tid] + part[w + 1][tid]) + (part[w + 2][tid] + part[w + 3][tid]);
    T *y = d.y + tid;
    if (d.beta != T(0)) {
      const T base = d.y0 ? d.y0[tid] : *y;
      *y = fma(d.beta, base, v);
    } else {
      *y = v;
    }
  }
}

// ----------------------------------------------------------------------------
// Block copies: blockIdx.x = descriptor, blockIdx.y = 16-column slab
// ----------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void copy_desc(const CopyDesc<T> *__restrict__ descs) {
  const CopyDesc<T> d = descs[blockIdx.x];
  const int c0 = blockIdx.y * 16;
  if (c0 >= d.cols) return;
  // the block's (row, column) pairs are spread over all threads, so short
  // columns (a few rows) still keep the workgroup busy
  const int nc = d.cols - c0 < 16 ? d.cols - c0 : 16;
  const int tot = d.rows * nc;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int c = c0 + e / d.rows, r = e % d.rows;
    T *p = d.dst + r + (size_t)c * d.ldd;
    if (!d.acc && d.alpha == T(0)) {   // zero fill: the source is not read
      *p = T(0);
      continue;
    }
    const T v = d.trans ? d.src[c + (size_t)r * d.lds] : d.src[r + (size_t)c * d.lds];
    *p = d.acc ? fma(d.alpha, v, *p) : d.alpha * v;
  }
}

// Sum of squares of NR entries per column (rows 0, 256, ..., 256 (NR - 1)
// of A) over `cols` columns, accumulated in column order and, within a
// column, in row order; the loads of several columns are issued before
// their products are added, so they are in flight together.
template <class T, int NR>
__device__ __forceinline__ double sumsq_cols(const T *A, int lda, int cols) {
  constexpr int UC = NR == 1 ? 8 : (NR == 2 ? 4 : 3);
  double s = 0.0;
  int c = 0;
  for (; c + UC <= cols; c += UC) {
    double v[UC][NR];
#pragma unroll
    for (int u = 0; u < UC; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k) v[u][k] = (double)A[256 * k + (size_t)(c + u) * lda];
#pragma unroll
    for (int u = 0; u < UC; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k) s = fma(v[u][k], v[u][k], s);
  }
  for (; c < cols; ++c)
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const double v = (double)A[256 * k + (size_t)c * lda];
      s = fma(v, v, s);
    }
  return s;
}

template <class T>
__global__ __launch_bounds__(256) void norm_desc(const NormDesc<T> *__restrict__ descs,
                                                 double *__restrict__ out) {
  const NormDesc<T> d = descs[blockIdx.x];
  const int t = threadIdx.x;
  const int nr = t < d.rows ? (d.rows - 1 - t) / 256 + 1 : 0;   // rows of this thread per column
  double s = 0.0;
  if (nr == 1) s = sumsq_cols<T, 1>(d.A + t, d.lda, d.cols);
  else if (nr == 2) s = sumsq_cols<T, 2>(d.A + t, d.lda, d.cols);
  else if (nr == 3) s = sumsq_cols<T, 3>(d.A + t, d.lda, d.cols);
  else if (nr > 3)
    for (int c = 0; c < d.cols; ++c)
      for (int r = t; r < d.rows; r += 256) {
        const double v = (double)d.A[r + (size_t)c * d.lda];
        s = fma(v, v, s);
      }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt((red[0] + red[1]) + (red[2] + red[3]));
}

template <class T>
__global__ __launch_bounds__(256) void normalize_cols(T *A, int lda, int rows) {
  T *col = A + (size_t)blockIdx.x * lda;
  double s = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) s = fma((double)col[r], (double)col[r], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double nrm = sqrt((red[0] + red[1]) + (red[2] + red[3]));
  const T scale = nrm > 0.0 ? T(1.0 / nrm) : T(0);
  for (int r = threadIdx.x; r < rows; r += 256) col[r] *= scale;
}

// ----------------------------------------------------------------------------
// Gauss-Jordan inversion with partial pivoting, one workgroup per matrix
// ----------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void gj_kernel(T *const *__restrict__ ptrs,
                                                 const int *__restrict__ ns,
                                                 int32_t *__restrict__ info) {
  extern __shared__ unsigned char shraw[];
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  const int b = blockIdx.x;
  const int n = ns[b];
  T *A = ptrs[b];
  T *rowk = reinterpret_cast<T *>(shraw);
  T *fcol = rowk + n;
  int *ipiv = reinterpret_cast<int *>(fcol + n);
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += 256) {
      const double v = fabs((double)A[i + (size_t)k * n]);
      if (v > best) { best = v; bi = i; }
    }
    red_v[tid] = best;
    red_i[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
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
      return;
    }
    if (tid == 0) ipiv[k] = p;
    if (p != k)
      for (int j = tid; j < n; j += 256) {
        const T t = A[k + (size_t)j * n];
        A[k + (size_t)j * n] = A[p + (size_t)j * n];
        A[p + (size_t)j * n] = t;
      }
    __syncthreads();
    const T invd = T(1) / A[k + (size_t)k * n];
    for (int j = tid; j < n; j += 256) rowk[j] = (j == k ? T(1) : A[k + (size_t)j * n]) * invd;
    for (int i = tid; i < n; i += 256) fcol[i] = i == k ? T(0) : A[i + (size_t)k * n];
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
      const T f = fcol[i];
      if (i == k) {
        for (int j = 0; j < n; ++j) A[i + (size_t)j * n] = rowk[j];
      } else {
        for (int j = 0; j < n; ++j) {
          const T a = j == k ? T(0) : A[i + (size_t)j * n];
          A[i + (size_t)j * n] = fma(-f, rowk[j], a);
        }
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = ipiv[k];
    if (p != k)
      for (int i = tid; i < n; i += 256) {
        const T t = A[i + (size_t)k * n];
        A[i + (size_t)k * n] = A[i + (size_t)p * n];
        A[i + (size_t)p * n] = t;
      }
    __syncthreads();
  }
  if (tid == 0) info[b] = 0;
}


// Gauss-Jordan with partial pivoting for n <= 64 with the matrix held in LDS
// (one workgroup per matrix); same contract as gj_kernel.
template <class T>
__global__ __launch_bounds__(256) void gj_small_kernel(T *const *__restrict__ ptrs,
                                                       const int *__restrict__ ns,
                                                       int32_t *__restrict__ info) {
  __shared__ T M[64][65];
  __shared__ T rowk[64], fcol[64];
  __shared__ int ipiv[64];
  __shared__ double red_v[64];
  __shared__ int red_i[64];
  const int b = blockIdx.x;
  const int n = ns[b];
  T *A = ptrs[b];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += 256) M[e % n][e / n] = A[e];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      if (tid >= k && tid < n) { best = fabs((double)M[tid][k]); bi = tid; }
      red_v[tid] = best;
      red_i[tid] = bi;
    }
    __syncthreads();
    for (int st = 32; st > 0; st >>= 1) {
      if (tid < st) {
        const double ov = red_v[tid + st];
        const int oi = red_i[tid + st];
        if (ov > red_v[tid] || (ov == red_v[tid] && oi < red_i[tid])) {
          red_v[tid] = ov;
          red_i[tid] = oi;
        }
      }
      __syncthreads();
    }
    const double pv = red_v[0];
    const int p = red_i[0];
    if (!(pv > 0.0) || !isfinite(pv)) {
      if (tid == 0) info[b] = k + 1;
      return;
    }
    if (tid == 0) ipiv[k] = p;
    if (p != k && tid < n) {
      const T t = M[k][tid];
      M[k][tid] = M[p][tid];
      M[p][tid] = t;
    }
    __syncthreads();
    const T invd = T(1) / M[k][k];
    if (tid < n) {
      rowk[tid] = (tid == k ? T(1) : M[k][tid]) * invd;
      fcol[tid] = tid == k ? T(0) : M[tid][k];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int i = e % n, j = e / n;
      if (i == k) {
        M[i][j] = rowk[j];
      } else {
        const T a = j == k ? T(0) : M[i][j];
        M[i][j] = fma(-fcol[i], rowk[j], a);
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = ipiv[k];
    if (p != k && tid < n) {
      const T t = M[tid][k];
      M[tid][k] = M[tid][p];
      M[tid][p] = t;
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += 256) A[e] = M[e % n][e / n];
  if (tid == 0) info[b] = 0;
}

// ----------------------------------------------------------------------------
// Truncated pivoted Gram-Schmidt (rank-revealing), one workgroup per problem
// ----------------------------------------------------------------------------
// One workgroup of kPgsThreads per candidate block.  In FP64 the candidates
// are only read: their residual norms (squared, in LDS) are downdated by the
// squared projection on every accepted column, and the chosen candidate is
// projected against the accepted columns twice (classical Gram-Schmidt,
// twice) when it is picked, then normalised and appended.  Downdating loses
// about one unit roundoff of the candidate's original norm, far below the
// truncation threshold.  Columns of W below orth_from are left out of the
// projection: the caller has projected them out of the candidates already.
// In FP32 every accepted column is projected out of the candidates in place
// (see pgs_kernel).  Reductions go through wave shuffles, then across the 16
// waves in LDS.
// Sums over the wave of B = 4 or 8 accumulators at once, each formed by the
// same pairings as the halving tree (distances 32, 16, ..., 1; the sum of
// two subtree values is exact under exchange, so the result equals the
// shfl_down tree's in lane 0): at distances 32 and 16 (and 8 for B = 8)
// every lane keeps half of its accumulators and receives the partner's
// half of the same ones, the remaining distances are whole-wave exchanges.
// Returns, in every lane, the total of accumulator wave_sums_slot<B>(lane).
__device__ __forceinline__ void lane_swap32(double P, double Q, double &r0, double &r1) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(P), __double2loint(Q), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(P), __double2hiint(Q), false, false);
  r0 = __hiloint2double(hi[0], lo[0]);   // lanes 32..63: Q of lane - 32
  r1 = __hiloint2double(hi[1], lo[1]);   // lanes 0..31: P of lane + 32
}
__device__ __forceinline__ void lane_swap16(double P, double Q, double &r0, double &r1) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(P), __double2loint(Q), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(P), __double2hiint(Q), false, false);
  r0 = __hiloint2double(hi[0], lo[0]);   // lanes with bit 16 set: Q of lane - 16
  r1 = __hiloint2double(hi[1], lo[1]);   // lanes with bit 16 clear: P of lane + 16
}
template <int B>
__device__ __forceinline__ int wave_sums_slot(int lane) {
  return B == 8 ? ((lane >> 3) & 1) | ((lane >> 3) & 2) | ((lane >> 3) & 4) : ((lane >> 4) & 1) | ((lane >> 4) & 2);
}
template <int B>
__device__ __forceinline__ int wave_sums_lane(int s) {
  return B == 8 ? 8 * (s & 1) + 8 * (s & 2) + 8 * (s & 4) : 16 * (s & 1) + 16 * (s & 2);
}
template <int B>
__device__ __forceinline__ double wave_sums(const double (&a)[B], int lane) {
  static_assert(B == 4 || B == 8, "four or eight accumulators");
  constexpr int H1 = B / 2, H2 = B / 4;
  const bool hi32 = lane & 32, hi16 = lane & 16;
  double b[H1], c[H2];
#pragma unroll
  for (int q = 0; q < H1; ++q) {
    double r0, r1;
    lane_swap32(a[q], a[H1 + q], r0, r1);
    b[q] = hi32 ? a[H1 + q] + r0 : a[q] + r1;
  }
#pragma unroll
  for (int q = 0; q < H2; ++q) {
    double r0, r1;
    lane_swap16(b[q], b[H2 + q], r0, r1);
    c[q] = hi16 ? b[H2 + q] + r0 : b[q] + r1;
  }
  double d;
  if constexpr (H2 == 2) {
    const bool hi8 = lane & 8;
    d = (hi8 ? c[1] : c[0]) + dpp_f64<0x128>(hi8 ? c[0] : c[1]);   // row_ror:8, lane ^ 8
  } else {
    d = c[0] + dpp_f64<0x128>(c[0]);
  }
  d += dpp_f64<0x1B>(dpp_f64<0x141>(d));   // lane ^ 4: half-row mirror, then quad_perm [3,2,1,0]
  d += dpp_f64<0x4E>(d);                   // lane ^ 2
  d += dpp_f64<0xB1>(d);                   // lane ^ 1
  return d;
}

constexpr int kPgsThreads = 1024;
constexpr int kPgsWaves = kPgsThreads / 64;

template <class T>
__global__ __launch_bounds__(kPgsThreads) void pgs_kernel(const PgsDesc<T> *__restrict__ descs) {
  // FP64 columns: residual norms are downdated and the candidates only read.
  // FP32 columns are orthonormal only to about 6e-8, which would spoil a
  // downdated norm at thresholds of tol^2 ~ 1e-9: they are projected in place
  // and re-orthogonalised against the whole basis instead.
  constexpr bool kDowndate = sizeof(T) == sizeof(double);
  extern __shared__ unsigned char shraw[];
  const PgsDesc<T> d = descs[blockIdx.x];
  double *norms = reinterpret_cast<double *>(shraw);   // c
  double *dots = norms + d.c;                           // rmax
  T *q = reinterpret_cast<T *>(dots + d.rmax);          // m
  // red_v / red_i serve the pivot search, red_s the norm of the projected
  // column: each is rewritten only after at least one barrier that follows
  // every read of it, so neither needs a barrier of its own after the reads
  __shared__ double red_v[kPgsWaves], red_s[kPgsWaves];
  __shared__ int red_i[kPgsWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = wv; j < d.c; j += kPgsWaves) {
    const T *col = d.R + (size_t)j * d.ldr;
    double s = 0.0;
    for (int i = lane; i < d.m; i += 64) s = fma((double)col[i], (double)col[i], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) norms[j] = s;
  }
  __syncthreads();
  const double tol2 = d.tol * d.tol;
  int k = 0;
  int guard = 0;
  while (d.r0 + k < d.rmax && guard < d.c + d.rmax) {
    ++guard;
    // pivot: the candidate of largest residual norm (lowest index on ties)
    double best = -1.0;
    int bi = 0;
    for (int j = tid; j < d.c; j += kPgsThreads)
      if (norms[j] > best) { best = norms[j]; bi = j; }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_down(best, o, 64);
      const int oi = __shfl_down(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { red_v[wv] = best; red_i[wv] = bi; }
    __syncthreads();
    double vmax = red_v[0];
    int p = red_i[0];
    for (int w = 1; w < kPgsWaves; ++w)
      if (red_v[w] > vmax || (red_v[w] == vmax && red_i[w] < p)) { vmax = red_v[w]; p = red_i[w]; }
    if (!(vmax > tol2)) break;
    for (int i = tid; i < d.m; i += kPgsThreads) q[i] = d.R[i + (size_t)p * d.ldr];
    __syncthreads();
    const int rc = d.r0 + k;
    const int c0 = kDowndate ? min(d.orth_from, rc) : 0;
    for (int pass = 0; pass < 2 && c0 < rc; ++pass) {
      for (int col = c0 + wv; col < rc; col += kPgsWaves) {
        const T *w = d.W + (size_t)col * d.ldw;
        double s = 0.0;
        for (int i = lane; i < d.m; i += 64) s = fma((double)w[i], (double)q[i], s);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if (lane == 0) dots[col] = s;
      }
      __syncthreads();
      for (int i = tid; i < d.m; i += kPgsThreads) {
        double v = (double)q[i];
        for (int col = c0; col < rc; ++col) v = fma(-(double)d.W[i + (size_t)col * d.ldw], dots[col], v);
        q[i] = (T)v;
      }
      __syncthreads();
    }
    double sq = 0.0;
    for (int i = tid; i < d.m; i += kPgsThreads) sq = fma((double)q[i], (double)q[i], sq);
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_down(sq, o, 64);
    if (lane == 0) red_s[wv] = sq;
    __syncthreads();
    // every thread sums the same values in the same order: a uniform decision
    double nq = 0.0;
    for (int w = 0; w < kPgsWaves; ++w) nq += red_s[w];
    if (nq <= 1e-4 * vmax || !(nq > 0.0)) {
      // numerically inside the current span: retire the column
      if (tid == 0) norms[p] = 0.0;
      __syncthreads();
      continue;
    }
    const double inv = 1.0 / sqrt(nq);
    T *wn = d.W + (size_t)rc * d.ldw;
    for (int i = tid; i < d.m; i += kPgsThreads) {
      const T v = (T)((double)q[i] * inv);
      q[i] = v;
      wn[i] = v;
    }
    if (tid == 0) norms[p] = 0.0;
    __syncthreads();
    ++k;
    for (int j = wv; j < d.c; j += kPgsWaves) {
      // a column already below the tolerance can never be chosen again and
      // its residual norm only decreases: leave it alone
      if (!(norms[j] > tol2)) continue;
      if constexpr (kDowndate) {
        // downdate the residual norm by the projection on the new column;
        // the candidate itself stays as given (read, never written)
        const T *col = d.R + (size_t)j * d.ldr;
        double dt = 0.0;
        for (int i = lane; i < d.m; i += 64) dt = fma((double)q[i], (double)col[i], dt);
        for (int o = 32; o > 0; o >>= 1) dt += __shfl_down(dt, o, 64);
        if (lane == 0) norms[j] = fma(-dt, dt, norms[j]);
      } else {
        // project the new column out of the candidate and recompute its norm
        T *col = d.R + (size_t)j * d.ldr;
        double dt = 0.0;
        for (int i = lane; i < d.m; i += 64) dt = fma((double)q[i], (double)col[i], dt);
        for (int o = 32; o > 0; o >>= 1) dt += __shfl_down(dt, o, 64);
        dt = __shfl(dt, 0, 64);
        double sq2 = 0.0;
        for (int i = lane; i < d.m; i += 64) {
          const T v = (T)((double)col[i] - dt * (double)q[i]);
          col[i] = v;
          sq2 = fma((double)v, (double)v, sq2);
        }
        for (int o = 32; o > 0; o >>= 1) sq2 += __shfl_down(sq2, o, 64);
        if (lane == 0) norms[j] = sq2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) *d.count = k;
}


// Blocked variant for FP64 (candidates read-only, residual norms downdated):
// each step takes the (up to) B candidates of largest residual norm at once,
// projects the block against the columns accepted so far (classical
// Gram-Schmidt twice, 64 columns at a time), orthonormalises it in LDS in
// the order of the norms (a candidate whose residual falls to the tolerance
// inside the block, or into the span, is retired), appends the accepted
// columns and downdates every remaining candidate's norm by them in one pass
// over the candidates.  The candidates and the basis are thus read once per
// block instead of once per column.  The result has the same guarantee as
// the column-by-column pivoting: on exit every candidate's residual norm is
// at most the tolerance; the chosen directions may differ within a block.
constexpr int kPgsChunk = 64;

template <int B>
__global__ __launch_bounds__(kPgsThreads) void pgs_block_kernel(const PgsDesc<double> *__restrict__ descs) {
  extern __shared__ unsigned char shraw[];
  const PgsDesc<double> d = descs[blockIdx.x];
  double *norms = reinterpret_cast<double *>(shraw);   // c
  double *Q = norms + d.c;                              // B x m (block columns)
  __shared__ double dots[kPgsChunk][B];
  __shared__ double vsel[B], nsq[B];
  __shared__ int psel[B];
  __shared__ double cand_v[kPgsWaves][B];
  __shared__ int cand_i[kPgsWaves][B];
  __shared__ int nsel, nacc;
  __shared__ double red_v[kPgsWaves];
  __shared__ int red_i[kPgsWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = wv; j < d.c; j += kPgsWaves) {
    const double *col = d.R + (size_t)j * d.ldr;
    double s = 0.0;
    for (int i = lane; i < d.m; i += 64) s = fma(col[i], col[i], s);
    s = wave_sum_lane0(s);
    if (lane == 0) norms[j] = s;
  }
  __syncthreads();
  const double tol2 = d.tol * d.tol;
  const int c0 = min(d.orth_from, d.r0);
  int k = 0;
  for (int guard = 0; guard < d.c + d.rmax && d.r0 + k < d.rmax; ++guard) {
    // 1. up to B pivots, largest residual norm first (lowest index on ties):
    // each wave lists its own best `room` candidates in that order (DPP
    // maximum of the norms, then minimum of the indices holding it), then
    // wave 0 merges the sorted lists by their heads; a candidate must
    // exceed -1 (taken) and be a number, and the picks stop at the first
    // one not above the tolerance.
    const int room = min(B, d.rmax - d.r0 - k);
    {
      unsigned long long removed = 0;   // bit q: entry tid + q kPgsThreads listed
      for (int i = 0; i < room; ++i) {
        double v = -1.0;
        int bi = 0x7fffffff, bq = -1;
        for (int q = 0, j = tid; j < d.c; j += kPgsThreads, ++q)
          if (!((removed >> q) & 1ull) && norms[j] > v) { v = norms[j]; bi = j; bq = q; }
        const double wmax = wave_max_f64(v);
        const int wi = wave_min_i32(v == wmax ? bi : 0x7fffffff);
        if (lane == 0) { cand_v[wv][i] = wmax; cand_i[wv][i] = wi; }
        if (bq >= 0 && bi == wi) removed |= 1ull << bq;
      }
    }
    __syncthreads();
    if (wv == 0) {
      int head = 0, cnt = 0;            // lane w < kPgsWaves walks wave w's list
      for (; cnt < room; ++cnt) {
        const double hv = (lane < kPgsWaves && head < room) ? cand_v[lane][head] : -1.0;
        const int hi = (lane < kPgsWaves && head < room) ? cand_i[lane][head] : 0x7fffffff;
        const double vmax = wave_max_f64(hv);
        const int p = wave_min_i32(hv == vmax ? hi : 0x7fffffff);
        if (!(vmax > tol2)) break;      // uniform
        if (lane < kPgsWaves && head < room && hi == p) ++head;
        if (lane == 0) {
          vsel[cnt] = vmax;
          psel[cnt] = p;
          norms[p] = -1.0;              // taken (retired below)
        }
      }
      if (lane == 0) nsel = cnt;
    }
    __syncthreads();
    const int ns = nsel;
    if (ns == 0) break;
    // 2. the block's columns into LDS
    for (int e = tid; e < ns * d.m; e += kPgsThreads) {
      const int s = e / d.m, i = e - s * d.m;
      Q[e] = d.R[i + (size_t)psel[s] * d.ldr];
    }
    __syncthreads();
    // 3. project out the basis columns [c0, r0 + k), twice, 64 at a time
    const int rc = d.r0 + k;
    for (int pass = 0; pass < 2; ++pass)
      for (int cb = c0; cb < rc; cb += kPgsChunk) {
        const int ce = min(rc, cb + kPgsChunk);
        for (int col = cb + wv; col < ce; col += kPgsWaves) {
          const double *w = d.W + (size_t)col * d.ldw;
          double acc[B];
#pragma unroll
          for (int s = 0; s < B; ++s) acc[s] = 0.0;
          for (int i = lane; i < d.m; i += 64) {
            const double wi = w[i];
#pragma unroll
            for (int s = 0; s < B; ++s)
              if (s < ns) acc[s] = fma(wi, Q[s * d.m + i], acc[s]);
          }
          const double v = wave_sums<B>(acc, lane);
          if ((lane & (B == 8 ? 7 : 15)) == 0) dots[col - cb][wave_sums_slot<B>(lane)] = v;
        }
        __syncthreads();
        // a thread per row: each basis entry is loaded once for the whole
        // block (same products and order per entry as one thread per entry)
        for (int i = tid; i < d.m; i += kPgsThreads) {
          double v[B];
#pragma unroll
          for (int s = 0; s < B; ++s) v[s] = s < ns ? Q[s * d.m + i] : 0.0;
          for (int col = cb; col < ce; ++col) {
            const double w = d.W[i + (size_t)col * d.ldw];
#pragma unroll
            for (int s = 0; s < B; ++s)
              if (s < ns) v[s] = fma(-w, dots[col - cb][s], v[s]);
          }
#pragma unroll
          for (int s = 0; s < B; ++s)
            if (s < ns) Q[s * d.m + i] = v[s];
        }
        __syncthreads();
      }
    // 4. within the block, in the order of the norms: project against the
    // block columns accepted before it (twice), accept if its residual is
    // above the tolerance and not numerically inside the span
    if (tid == 0) nacc = 0;
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
      double *qs = Q + (size_t)s * d.m;
      const int na = nacc;
      for (int pass = 0; pass < 2 && na > 0; ++pass) {
        for (int t = wv; t < na; t += kPgsWaves) {
          const double *qt = Q + (size_t)t * d.m;
          double v = 0.0;
          for (int i = lane; i < d.m; i += 64) v = fma(qt[i], qs[i], v);
          v = wave_sum_lane0(v);
          if (lane == 0) dots[t][0] = v;
        }
        __syncthreads();
        for (int i = tid; i < d.m; i += kPgsThreads) {
          double v = qs[i];
          for (int t = 0; t < na; ++t) v = fma(-Q[(size_t)t * d.m + i], dots[t][0], v);
          qs[i] = v;
        }
        __syncthreads();
      }
      double sq = 0.0;
      for (int i = tid; i < d.m; i += kPgsThreads) sq = fma(qs[i], qs[i], sq);
      sq = wave_sum_lane0(sq);
      if (lane == 0) red_v[wv] = sq;
      __syncthreads();
      double nq = 0.0;                       // same values, same order: uniform
      for (int w = 0; w < kPgsWaves; ++w) nq += red_v[w];
      __syncthreads();                       // red_v read by everyone
      const bool take = nq > tol2 && nq > 1e-4 * vsel[s];
      if (take) {
        const double inv = 1.0 / sqrt(nq);
        double *dst = Q + (size_t)na * d.m;  // compact: na <= s
        for (int i = tid; i < d.m; i += kPgsThreads) dst[i] = qs[i] * inv;
      }
      __syncthreads();
      if (tid == 0) {
        // a column not taken is inside the span or at the tolerance: retired
        norms[psel[s]] = 0.0;
        if (take) nacc = na + 1;
      }
      __syncthreads();
    }
    const int na = nacc;
    // 5. append the accepted columns, downdate every remaining candidate
    for (int e = tid; e < na * d.m; e += kPgsThreads) {
      const int s = e / d.m, i = e - s * d.m;
      d.W[i + (size_t)(rc + s) * d.ldw] = Q[e];
    }
    for (int j = wv; j < d.c && na > 0; j += kPgsWaves) {
      if (!(norms[j] > tol2)) continue;
      const double *col = d.R + (size_t)j * d.ldr;
      double acc[B];
#pragma unroll
      for (int s = 0; s < B; ++s) acc[s] = 0.0;
      for (int i = lane; i < d.m; i += 64) {
        const double ci = col[i];
#pragma unroll
        for (int s = 0; s < B; ++s)
          if (s < na) acc[s] = fma(Q[s * d.m + i], ci, acc[s]);
      }
      const double tot = wave_sums<B>(acc, lane);
      double dn = 0.0;
#pragma unroll
      for (int s = 0; s < B; ++s) {
        const double v = readlane_f64(tot, wave_sums_lane<B>(s));
        dn = fma(v, v, dn);
      }
      if (lane == 0) norms[j] -= dn;
    }
    k += na;
    __syncthreads();
  }
  if (tid == 0) *d.count = k;
}

// ----------------------------------------------------------------------------
// Blocked Gauss-Jordan with partial pivoting by columns, helper kernels.
// The matrices are column-major, so pivoting by columns makes every
// interchange a copy of contiguous columns; this is Gauss-Jordan with
// partial (row) pivoting applied to the transpose, and the inverse of the
// transpose is the transpose of the inverse.  For the panel of rows
// [k0, k0 + pb) of every matrix: pivot columns are chosen by an elimination
// with partial pivoting of a copy of the wide panel (columns k0..n) -- the
// same columns Gauss-Jordan would choose -- and the interchanges are applied
// to whole columns.  lab[j] follows which original column sits at position
// j; the rows of the finished inverse are put back in that order at the end.
// ----------------------------------------------------------------------------
template <class T>
struct PanelDesc {
  T *A;          // n x n, ld n
  T *work;       // n x pb scratch
  int *ipiv;     // n entries (column chosen at step k; fallback kernel only)
  int *lab;      // n entries: original column now at each position
  int n, k0, pb;
  int32_t *info;
  // when set (register panel kernel only): after the interchanges the same
  // workgroup inverts the pivot block into P (pb x pb, failure into *tinfo)
  // and writes C = A[p, :] with -I in the panel's columns (pb x n, leading
  // dimension pb)
  T *P = nullptr, *C = nullptr;
  int32_t *tinfo = nullptr;
};

template <class T>
__global__ __launch_bounds__(256) void panel_pivot_kernel(const PanelDesc<T> *__restrict__ descs) {
  const PanelDesc<T> d = descs[blockIdx.x];
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  const int tid = threadIdx.x;
  const int h = d.n - d.k0;
  T *W = d.work;
  // W (h x pb): W[r + c h] = A[k0 + c, k0 + r], the panel transposed
  for (int r = tid; r < h; r += 256)
    for (int c = 0; c < d.pb; ++c) W[r + (size_t)c * h] = d.A[(d.k0 + c) + (size_t)(d.k0 + r) * d.n];
  __syncthreads();
  for (int t = 0; t < d.pb; ++t) {
    double best = -1.0;
    int bi = t;
    for (int r = t + tid; r < h; r += 256) {
      const double v = fabs((double)W[r + (size_t)t * h]);
      if (v > best) { best = v; bi = r; }
    }
    red_v[tid] = best;
    red_i[tid] = bi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) {
        const double ov = red_v[tid + st];
        const int oi = red_i[tid + st];
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
      if (tid == 0) *d.info = d.k0 + t + 1;
      return;
    }
    if (tid == 0) d.ipiv[d.k0 + t] = d.k0 + p;
    if (p != t)
      for (int c = tid; c < d.pb; c += 256) {
        const T a = W[t + (size_t)c * h];
        W[t + (size_t)c * h] = W[p + (size_t)c * h];
        W[p + (size_t)c * h] = a;
      }
    __syncthreads();
    const T inv = T(1) / W[t + (size_t)t * h];
    for (int r = t + 1 + tid; r < h; r += 256) W[r + (size_t)t * h] *= inv;
    __syncthreads();
    for (int r = t + 1 + tid; r < h; r += 256) {
      const T l = W[r + (size_t)t * h];
      for (int c = t + 1; c < d.pb; ++c) W[r + (size_t)c * h] = fma(-l, W[t + (size_t)c * h], W[r + (size_t)c * h]);
    }
    __syncthreads();
  }
  // apply the interchanges to whole columns of A, in order
  for (int t = 0; t < d.pb; ++t) {
    const int k = d.k0 + t, p = d.ipiv[k];
    if (p != k) {
      for (int r = tid; r < d.n; r += 256) {
        const T a = d.A[r + (size_t)k * d.n];
        d.A[r + (size_t)k * d.n] = d.A[r + (size_t)p * d.n];
        d.A[r + (size_t)p * d.n] = a;
      }
      if (tid == 0) {
        const int x = d.lab[k];
        d.lab[k] = d.lab[p];
        d.lab[p] = x;
      }
    }
    __syncthreads();
  }
}

// The same elimination for panels of at most kPanelRegRows columns, one
// workgroup barrier per step: each thread keeps one column of the panel in
// registers (column j belongs to thread j; a column's pb entries are
// contiguous in memory), in workgroups of 256, 512 or 768 threads by the
// panel's height.  Below, "row"
// names such a register vector: the elimination is the one of the
// transposed panel.  The pivot is the largest |entry| (a non-finite one
// counts as +inf and stops the panel), the lowest row among equal ones: a
// maximum of doubles and then a minimum of row numbers over each wave, both
// by DPP.  The owner of each wave's best candidate posts its row to LDS
// before the barrier, so after it every thread knows the winner and its row
// at once.  Vectors never move between
// threads; the choice order alone defines the interchanges.  The steps run
// in a loop of four expanded steps, after which the register columns shift
// by four: the code stays small enough for the instruction cache (the fully
// expanded 32 steps were bound by instruction fetch).  Finally the
// interchanges are applied to A as one permutation of the touched columns,
// in three passes separated by barriers (see the end of the kernel).
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// One vector per thread (panels of up to 768 columns).  Three vectors per
// thread in a 256-thread workgroup spilled registers once the steps became
// a loop; a single wave with six vectors per lane measured slower.
constexpr int kPanelRegRows = 768;

// workgroup barrier; for a single wave, LDS completion and a wave barrier
template <int THREADS>
__device__ __forceinline__ void panel_sync() {
  if constexpr (THREADS == 64) {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <class T>
__device__ __forceinline__ void pin_registers(T (&v)[32]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
               "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
               "+v"(v[14]), "+v"(v[15]));
  asm volatile("" : "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]), "+v"(v[20]), "+v"(v[21]),
               "+v"(v[22]), "+v"(v[23]), "+v"(v[24]), "+v"(v[25]), "+v"(v[26]), "+v"(v[27]), "+v"(v[28]),
               "+v"(v[29]), "+v"(v[30]), "+v"(v[31]));
}

// Gauss-Jordan inverse without interchanges, one wave per matrix of order
// n <= NMAX, read from srcs[b] (leading dimension lds[b]) and written to
// ptrs[b] (leading dimension n).  For the pivot blocks of the blocked
// inverse: their columns were chosen by partial pivoting over the whole
// panel, so the diagonal already holds the pivots an interchanging
// elimination of the transposed block would take (the pivots of an
// elimination without interchanges are ratios of leading principal minors,
// the same for a matrix and its transpose).  Lane i keeps row i of
// diag(M, I) (order NMAX) in registers; every lane reads the pivot row from
// the pivot lane (readlane into scalar registers, no LDS round trip) and
// scales it itself.  The steps run in a loop of U expanded steps, after
// which the register columns rotate by U (NMAX steps rotate them back into
// place): the code stays small enough for the instruction cache.
template <class T>
__device__ __forceinline__ T lane_value(T v, int l);
template <>
__device__ __forceinline__ double lane_value<double>(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <>
__device__ __forceinline__ float lane_value<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// One wave (lane i) inverts the matrix of order n <= NMAX at src (leading
// dimension ld) into A (leading dimension n); a failure sets *info.
template <class T, int NMAX>
__device__ __forceinline__ void gj_nopiv_wave(const T *__restrict__ src, int ld, int n, T *__restrict__ A,
                                              int32_t *__restrict__ info, int i) {
  constexpr int U = 8;
  static_assert(NMAX % U == 0 && NMAX <= 64, "the order is a multiple of the expanded steps");
  T r[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) r[c] = (i < n && c < n) ? src[i + (size_t)c * ld] : (i == c ? T(1) : T(0));
  int fail_at = 0;   // 1 + the first step with a zero or non-finite pivot
  for (int k0 = 0; k0 < NMAX; k0 += U) {
    static_for<0, U>([&](auto jc) {
      constexpr int j = decltype(jc)::value;   // register column of step k
      const int k = k0 + j;
      // pivot row k scaled by 1 / pivot, with 1 / pivot in column j
      const T inv = T(1) / lane_value(r[j], k);
      T pr[NMAX];
#pragma unroll
      for (int c = 0; c < NMAX; ++c) pr[c] = c == j ? inv : lane_value(r[c], k) * inv;
      // the elimination runs on after a failure; its values are discarded
      if (fail_at == 0 && !isfinite((double)inv)) fail_at = k + 1;
      if (i == k) {
#pragma unroll
        for (int c = 0; c < NMAX; ++c) r[c] = pr[c];
      } else {
        const T f = r[j];
        r[j] = T(0);
#pragma unroll
        for (int c = 0; c < NMAX; ++c) r[c] = fma(-f, pr[c], r[c]);
      }
    });
    T head[U];
#pragma unroll
    for (int c = 0; c < U; ++c) head[c] = r[c];
#pragma unroll
    for (int c = 0; c + U < NMAX; ++c) r[c] = r[c + U];
#pragma unroll
    for (int c = 0; c < U; ++c) r[NMAX - U + c] = head[c];
  }
  if (fail_at) {
    if (i == 0) *info = fail_at;
    return;
  }
  if (i < n) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c)
      if (c < n) A[i + (size_t)c * n] = r[c];
  }
}

template <class T, int NMAX>
__global__ __launch_bounds__(64) void gj_nopiv_wave_kernel(T *const *__restrict__ ptrs,
                                                           const int *__restrict__ ns,
                                                           int32_t *__restrict__ info,
                                                           const T *const *__restrict__ srcs,
                                                           const int *__restrict__ lds) {
  const int b = blockIdx.x;
  gj_nopiv_wave<T, NMAX>(srcs[b], lds[b], ns[b], ptrs[b], info + b, threadIdx.x);
}

template <class T, int THREADS, int SLOTS>
__global__ __launch_bounds__(THREADS) void panel_pivot_reg_kernel(const PanelDesc<T> *__restrict__ descs) {
  constexpr int PB = 32;
  constexpr int U = 4;   // expanded steps per loop iteration
  constexpr int NW = THREADS / 64;
  static_assert(PB % U == 0, "the panel width is a multiple of the expanded steps");
  const PanelDesc<T> d = descs[blockIdx.x];
  __shared__ double w_val[2][NW];
  __shared__ int w_idx[2][NW];
  __shared__ T w_row[2][NW][PB];
  __shared__ int chosen[PB];
  __shared__ int u_pos[2 * PB], u_src[2 * PB];
  __shared__ int s_nu, s_na;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int h = d.n - d.k0, pb = d.pb;
  T row[SLOTS][PB];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    const int r = tid + THREADS * q;
#pragma unroll
    for (int c = 0; c < PB; ++c)
      row[q][c] = (r < h && c < pb) ? d.A[(d.k0 + c) + (size_t)(d.k0 + r) * d.n] : T(0);
  }
  bool failed = false;
  unsigned used = 0;   // bit q: slot q's vector has been chosen
  for (int t0 = 0; t0 < pb; t0 += U) {
    static_for<0, U>([&](auto jc) {
      constexpr int j = decltype(jc)::value;   // register column of step t
      const int t = t0 + j;
      if (failed || t >= pb) return;
      const int par = t & 1;
      // this thread's best candidate (lowest row on ties)
      double v = -1.0;
      int bi = 0x7fffffff, qb = -1;
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int r = tid + THREADS * q;
        if (r < h && !((used >> q) & 1u)) {
          double a = fabs((double)row[q][j]);
          if (!isfinite(a)) a = HUGE_VAL;
          if (a > v) { v = a; bi = r; qb = q; }
        }
      }
      const double wmax = wave_max_f64(v);
      const int wrow = wave_min_i32(v == wmax ? bi : 0x7fffffff);
      // one owner per wave: the lowest row holding the wave's maximum
      if (qb >= 0 && bi == wrow) {
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
          if (q == qb) {
#pragma unroll
            for (int c = 0; c < PB; ++c) w_row[par][wv][c] = row[q][c];
          }
      }
      if (lane == 0) {
        w_val[par][wv] = wmax;
        w_idx[par][wv] = wrow;
      }
      __syncthreads();
      double wvals[NW];
      int widx[NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        wvals[w] = w_val[par][w];
        widx[w] = w_idx[par][w];
      }
      double pv = wvals[0];
      int p = widx[0], wb = 0;
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const bool better = wvals[w] > pv || (wvals[w] == pv && widx[w] < p);
        pv = better ? wvals[w] : pv;
        p = better ? widx[w] : p;
        wb = better ? w : wb;
      }
      if (!(pv > 0.0) || !isfinite(pv)) {
        if (tid == 0) *d.info = d.k0 + t + 1;
        failed = true;
        return;
      }
      if (tid == 0) chosen[t] = p;
#pragma unroll
      for (int q = 0; q < SLOTS; ++q)
        if (tid + THREADS * q == p) used |= 1u << q;
      // the whole pivot row is read at once (all loads in flight together)
      T prow[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) prow[c] = c < j ? T(0) : w_row[par][wb][c];
      pin_registers(prow);
      const T pinv = T(1) / prow[j];
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int r = tid + THREADS * q;
        if (r < h && !((used >> q) & 1u)) {
          const T l = row[q][j] * pinv;
          row[q][j] = l;
#pragma unroll
          for (int c = j + 1; c < PB; ++c) row[q][c] = fma(-l, prow[c], row[q][c]);
        }
      }
    });
    if (failed) return;   // uniform: every thread read the same keys
    // the next iteration's columns move to register columns 0..U-1
#pragma unroll
    for (int q = 0; q < SLOTS; ++q)
#pragma unroll
      for (int c = 0; c < PB; ++c) row[q][c] = c + U < PB ? row[q][c + U] : T(0);
  }
  // the panel's permutation of columns: position k0 + t receives the t-th
  // chosen column; the columns of [k0, k0 + pb) that were not chosen move,
  // in increasing order, to the positions that chosen columns from beyond
  // the panel left (in the order they were chosen)
  panel_sync<THREADS>();
  if (tid == 0) {
    int nu = 0;
    unsigned top = 0;
    for (int t = 0; t < pb; ++t)
      if (chosen[t] < pb) top |= 1u << chosen[t];
    for (int t = 0; t < pb; ++t)
      if (chosen[t] != t) {
        u_pos[nu] = d.k0 + t;
        u_src[nu] = d.k0 + chosen[t];
        ++nu;
      }
    s_na = nu;
    int x = 0;
    for (int t = 0; t < pb; ++t)
      if (chosen[t] >= pb) {
        while ((top >> x) & 1u) ++x;
        u_pos[nu] = d.k0 + chosen[t];
        u_src[nu] = d.k0 + x;
        ++nu;
        ++x;
      }
    s_nu = nu;
  }
  panel_sync<THREADS>();
  const int nu = s_nu, na = s_na;
  if (nu > 0) {
  {
    // the column labels follow the same permutation (all reads before the
    // barrier, all writes after it)
    const int v = tid < nu ? d.lab[u_src[tid]] : 0;
    panel_sync<THREADS>();
    if (tid < nu) d.lab[u_pos[tid]] = v;
  }
  // Entries [0, na) move chosen columns into the panel, entries [na, nu)
  // move the panel's unchosen columns to the places the chosen ones left
  // beyond the panel.  The sources of the first group are saved to the
  // scratch columns, the second group is copied (its sources lie in the
  // panel, its destinations beyond it), then the first group is written
  // from the scratch copy.  Accesses are whole columns, coalesced.
  for (int i = 0; i < na; ++i)
    for (int r = tid; r < d.n; r += THREADS) d.work[r + (size_t)i * d.n] = d.A[r + (size_t)u_src[i] * d.n];
  __syncthreads();
  for (int i = na; i < nu; ++i)
    for (int r = tid; r < d.n; r += THREADS) d.A[r + (size_t)u_pos[i] * d.n] = d.A[r + (size_t)u_src[i] * d.n];
  __syncthreads();
  for (int i = 0; i < na; ++i)
    for (int r = tid; r < d.n; r += THREADS) d.A[r + (size_t)u_pos[i] * d.n] = d.work[r + (size_t)i * d.n];
  }
  if (d.P == nullptr) return;
  __syncthreads();   // the interchanged columns are visible to every wave
  if (wv == 0) {
    gj_nopiv_wave<T, PB>(d.A + d.k0 + (size_t)d.k0 * d.n, d.n, pb, d.P, d.tinfo, lane);
  } else {
    for (int e = tid - 64; e < pb * d.n; e += THREADS - 64) {
      const int j = e / pb, t = e - j * pb;
      const T v = (j >= d.k0 && j < d.k0 + pb) ? (j - d.k0 == t ? T(-1) : T(0))
                                               : d.A[(d.k0 + t) + (size_t)j * d.n];
      d.C[t + (size_t)j * pb] = v;
    }
  }
}

template <class T>
__global__ void set_diagonal(T *A, int n, T v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) A[i + (size_t)i * n] = v;
}

// Final statuses of a blocked batched inversion (see inverse_batched_blocked).
__global__ void merge_status(const int32_t *__restrict__ stat, int nsmall, int nbm, int npan, int nb,
                             const int *__restrict__ sidx, const int *__restrict__ bidx,
                             const int *__restrict__ tpos, int32_t *__restrict__ info) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nsmall) {
    info[sidx[t]] = stat[t];
    return;
  }
  const int b = t - nsmall;
  if (b >= nbm) return;
  int32_t v = stat[nsmall + b];
  for (int it = 0; it < npan && v == 0; ++it) {
    const int q = tpos[(size_t)it * nbm + b];
    if (q < 0) continue;
    const int32_t w = stat[nsmall + nbm + (size_t)it * nbm + q];
    if (w != 0) v = it * nb + w;
  }
  info[bidx[b]] = v;
}

// Column labels start as the identity.
__global__ void iota_labels(int *const *__restrict__ labs, const int *__restrict__ ns) {
  int *lab = labs[blockIdx.y];
  const int n = ns[blockIdx.y];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n) lab[j] = j;
}

// Undo the column interchanges as a row permutation of the inverse: row k
// of the eliminated matrix is row lab[k] of the inverse.  One workgroup per
// (matrix, block of kUnpermCols columns); each column goes through LDS.
constexpr int kUnpermCols = 16;
template <class T>
__global__ __launch_bounds__(256) void unpermute_rows_kernel(T *const *__restrict__ ptrs,
                                                             const int *__restrict__ ns,
                                                             int *const *__restrict__ labs) {
  extern __shared__ unsigned char shraw[];
  T *buf = reinterpret_cast<T *>(shraw);
  const int n = ns[blockIdx.y];
  const int c0 = blockIdx.x * kUnpermCols;
  if (c0 >= n) return;
  T *A = ptrs[blockIdx.y];
  const int *lab = labs[blockIdx.y];
  const int c1 = min(n, c0 + kUnpermCols);
  for (int c = c0; c < c1; ++c) {
    T *col = A + (size_t)c * n;
    for (int k = threadIdx.x; k < n; k += 256) buf[k] = col[k];
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += 256) col[lab[k]] = buf[k];
    __syncthreads();
  }
}


__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

template <class T>
__global__ void gaussian_kernel(T *out, size_t n, uint64_t seed) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t a = splitmix64(seed * 0x100000001B3ull + 2 * i);
  const uint64_t b = splitmix64(seed * 0x100000001B3ull + 2 * i + 1);
  const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
  out[i] = (T)(sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2));
}

template <class T>
__global__ void fill_kernel(T *out, size_t n, T v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

template <class A, class B>
__global__ void convert_kernel(const A *src, B *dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (B)src[i];
}

}  // namespace

// C = beta C + sum of P partial products (m x n each, leading dimension m)
template <class T>
__global__ void splitk_reduce(const T *__restrict__ part, int P, int m, int n, T *__restrict__ C, int ldc,
                              T beta) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int r = (int)(e % m), c = (int)(e / m);
  T v = T(0);
  for (int p = 0; p < P; ++p) v += part[(int64_t)p * m * n + e];
  T *o = C + r + (size_t)c * ldc;
  *o = beta != T(0) ? fma(beta, *o, v) : v;
}

template <class T>
void gemm_batched_impl(const std::vector<GemmDesc<T>> &d, Stager &st, hipStream_t s, GemmInputs in) {
  HostScope hs(HostProf::kGemm);
  OpFlops &fl = op_flops();
  for (const auto &g : d)
    if (g.m > 0 && g.n > 0 && g.k > 0) {
      fl.gemm += 2.0 * g.m * g.n * g.k;
      ++fl.gemm_products;
    }
  // A batch with few output tiles but a long inner dimension would leave
  // most compute units idle while a handful of workgroups walk the whole k
  // range: such products are split along k into partial products (written
  // to scratch) that one more kernel sums.
  constexpr int64_t kWantTiles = 1024, kMinSlice = 512;
  int64_t total = 0;
  for (const auto &g : d)
    if (g.m > 0 && g.n > 0) total += (int64_t)((g.m + 63) / 64) * ((g.n + 63) / 64);
  if (total == 0) return;
  std::vector<GemmDesc<T>> keep;
  std::vector<int2> tiles;
  struct Split { GemmDesc<T> g; int P; size_t off; };
  std::vector<Split> splits;
  size_t scratch_elems = 0;
  std::vector<GemmDesc<T>> parts;
  for (const auto &g : d) {
    if (g.m <= 0 || g.n <= 0) continue;
    const int64_t nt = (int64_t)((g.m + 63) / 64) * ((g.n + 63) / 64);
    int P = 1;
    if (total < kWantTiles / 2 && g.k >= 4 * kMinSlice)
      P = (int)std::max<int64_t>(1, std::min<int64_t>(g.k / kMinSlice, kWantTiles / total));
    if (P <= 1) {
      parts.push_back(g);
      continue;
    }
    splits.push_back({g, P, scratch_elems});
    scratch_elems += (size_t)P * g.m * g.n;
    (void)nt;
  }
  StreamBuf<T> scratch(scratch_elems, s);
  for (const auto &sp : splits) {
    const GemmDesc<T> &g = sp.g;
    const int slice = (g.k + sp.P - 1) / sp.P;
    for (int p = 0; p < sp.P; ++p) {
      const int k0 = p * slice, kk = std::min(slice, g.k - k0);
      if (kk <= 0) {
        // an empty slice still owns its partial buffer: write zeros
        GemmDesc<T> z = g;
        z.k = 0;
        z.C = scratch.p + sp.off + (size_t)p * g.m * g.n;
        z.ldc = g.m;
        z.beta = T(0);
        parts.push_back(z);
        continue;
      }
      GemmDesc<T> q = g;
      q.k = kk;
      q.A = g.ta ? g.A + k0 : g.A + (size_t)k0 * g.lda;
      q.B = g.tb ? g.B + (size_t)k0 * g.ldb : g.B + k0;
      q.C = scratch.p + sp.off + (size_t)p * g.m * g.n;
      q.ldc = g.m;
      q.beta = T(0);
      parts.push_back(q);
    }
  }
  for (const auto &g : parts) {
    const int id = (int)keep.size();
    keep.push_back(g);
    const int nt = ((g.m + 63) / 64) * ((g.n + 63) / 64);
    for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(id, t));
  }
  for (size_t t0 = 0; t0 < tiles.size(); t0 += 1u << 20) {
    const size_t nt = std::min(tiles.size() - t0, size_t(1) << 20);
    std::vector<void *> dev;
    st.put_many({{keep.data(), keep.size() * sizeof(GemmDesc<T>)}, {tiles.data() + t0, nt * sizeof(int2)}},
                dev, s);
    launch_gemm_tiles<T>((unsigned)nt, (const GemmDesc<T> *)dev[0], (const int2 *)dev[1], s, in);
  }
  for (const auto &sp : splits) {
    const int64_t e = (int64_t)sp.g.m * sp.g.n;
    splitk_reduce<T><<<ceil_div(e, 256), 256, 0, s>>>(scratch.p + sp.off, sp.P, sp.g.m, sp.g.n, sp.g.C,
                                                     sp.g.ldc, sp.g.beta);
    SBIE_LAUNCH_CHECK();
  }
}

template <class T>
void gemm_batched(const std::vector<GemmDesc<T>> &d, Stager &st, hipStream_t s) {
  gemm_batched_impl<T>(d, st, s, GemmInputs::kWorking);
}

template <class T>
void gemm_batched_sketch(const std::vector<GemmDesc<T>> &d, GemmInputs in, Stager &st, hipStream_t s) {
  OpFlops &fl = op_flops();
  if (in != GemmInputs::kWorking)
    for (const auto &g : d)
      if (g.m > 0 && g.n > 0 && g.k > 0) fl.gemm_low += 2.0 * g.m * g.n * g.k;
  gemm_batched_impl<T>(d, st, s, in);
}

template <class T, class TA>
void gemv_launch(const GemvDesc<T> *d, const GemvTerm<T, TA> *t, int nd, int, hipStream_t s) {
  if (nd == 0) return;
  gemv_desc<T, TA><<<nd, kGemvThreads, 0, s>>>(d, t);
  SBIE_LAUNCH_CHECK();
}

template <class T>
void gemv_batched(const std::vector<GemvDesc<T>> &d, const std::vector<GemvTerm<T>> &t,
                  Stager &st, hipStream_t s) {
  if (d.empty()) return;
  std::vector<void *> dev;
  st.put_many({{t.data(), t.size() * sizeof(GemvTerm<T>)}, {d.data(), d.size() * sizeof(GemvDesc<T>)}}, dev, s);
  gemv_launch<T, T>((const GemvDesc<T> *)dev[1], (const GemvTerm<T> *)dev[0], (int)d.size(), 64, s);
}

template <class T>
void copy_launch(const CopyDesc<T> *d, int nd, int max_cols, hipStream_t s) {
  if (nd == 0 || max_cols == 0) return;
  dim3 grid(nd, ceil_div(max_cols, 16));
  copy_desc<T><<<grid, 256, 0, s>>>(d);
  SBIE_LAUNCH_CHECK();
}

template <class T>
void copy_batched(const std::vector<CopyDesc<T>> &d, Stager &st, hipStream_t s) {
  HostScope hs(HostProf::kCopy);
  std::vector<CopyDesc<T>> keep;
  int max_cols = 0;
  for (const auto &c : d)
    if (c.rows > 0 && c.cols > 0) {
      keep.push_back(c);
      max_cols = std::max(max_cols, c.cols);
    }
  if (keep.empty()) return;
  for (size_t b0 = 0; b0 < keep.size(); b0 += 60000) {
    const size_t nb = std::min(keep.size() - b0, size_t(60000));
    auto *dd = (const CopyDesc<T> *)st.put(keep.data() + b0, nb * sizeof(CopyDesc<T>), s);
    copy_launch<T>(dd, (int)nb, max_cols, s);
  }
}

// Gauss-Jordan inverse with partial pivoting of one matrix of order n <=
// NMAX per wave (64 threads), in place: lane i keeps row i of diag(M, I)
// (order NMAX) in registers, so no step needs a barrier.  The pivot is the
// largest |entry| of the column (lowest row on ties), by DPP exchanges; rows
// k and p trade places through LDS; every lane reads the pivot row from the
// pivot lane (readlane) and scales it itself.  The steps run in a loop of
// eight expanded steps, after which the register columns rotate by eight
// (NMAX steps rotate them back), so that the code fits the instruction
// cache.  Same operations as gj_small_kernel; the column interchanges are
// undone through LDS on the way out.
template <class T, int NMAX>
__global__ __launch_bounds__(64) void gj_wave_kernel(T *const *__restrict__ ptrs, const int *__restrict__ ns,
                                                     int32_t *__restrict__ info,
                                                     const T *const *__restrict__ srcs = nullptr,
                                                     const int *__restrict__ lds = nullptr) {
  constexpr int U = 8;
  static_assert(NMAX % U == 0 && NMAX <= 64, "the order is a multiple of the expanded steps");
  __shared__ T xk[NMAX], xp[NMAX];
  __shared__ T out[NMAX][NMAX + 1];
  __shared__ int ipv[NMAX], lab[NMAX];
  const int b = blockIdx.x;
  const int n = ns[b];
  T *A = ptrs[b];
  // the matrix is read from srcs[b] (leading dimension lds[b]) when given,
  // else from A itself; the inverse is written to A (leading dimension n)
  const T *src = srcs ? srcs[b] : A;
  const int ld = srcs ? lds[b] : n;
  const int i = threadIdx.x;
  T r[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) r[c] = (i < n && c < n) ? src[i + (size_t)c * ld] : (i == c ? T(1) : T(0));
  int fail_at = 0;   // 1 + the first step without a positive finite pivot
  for (int k0 = 0; k0 < NMAX; k0 += U) {
    static_for<0, U>([&](auto jc) {
      constexpr int j = decltype(jc)::value;   // register column of step k
      const int k = k0 + j;
      double v = (i >= k && i < NMAX) ? fabs((double)r[j]) : -1.0;
      if (!(v == v)) v = -1.0;                 // a NaN is no candidate
      const double vmax = wave_max_f64(v);
      const int p = wave_min_i32(v == vmax ? i : 0x7fffffff);
      if (fail_at == 0 && (!(vmax > 0.0) || !isfinite(vmax))) fail_at = k + 1;
      if (i == 0) ipv[k] = p < NMAX ? p : k;
      if (p != k && p < NMAX) {
        if (i == k) {
#pragma unroll
          for (int c = 0; c < NMAX; ++c) xk[c] = r[c];
        }
        if (i == p) {
#pragma unroll
          for (int c = 0; c < NMAX; ++c) xp[c] = r[c];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the rows are in LDS
        __builtin_amdgcn_wave_barrier();
        if (i == k) {
#pragma unroll
          for (int c = 0; c < NMAX; ++c) r[c] = xp[c];
        }
        if (i == p) {
#pragma unroll
          for (int c = 0; c < NMAX; ++c) r[c] = xk[c];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
      }
      // pivot row k scaled by 1 / pivot, with 1 / pivot in column j
      const T inv = T(1) / lane_value(r[j], k);
      T pr[NMAX];
#pragma unroll
      for (int c = 0; c < NMAX; ++c) pr[c] = c == j ? inv : lane_value(r[c], k) * inv;
      if (i == k) {
#pragma unroll
        for (int c = 0; c < NMAX; ++c) r[c] = pr[c];
      } else {
        const T f = r[j];
        r[j] = T(0);
#pragma unroll
        for (int c = 0; c < NMAX; ++c) r[c] = fma(-f, pr[c], r[c]);
      }
    });
    T head[U];
#pragma unroll
    for (int c = 0; c < U; ++c) head[c] = r[c];
#pragma unroll
    for (int c = 0; c + U < NMAX; ++c) r[c] = r[c + U];
#pragma unroll
    for (int c = 0; c < U; ++c) r[NMAX - U + c] = head[c];
  }
  if (fail_at) {
    if (i == 0) info[b] = fail_at;
    return;
  }
  // column interchanges in reverse order, as one permutation of labels
  if (i == 0) {
    for (int c = 0; c < n; ++c) lab[c] = c;
    for (int k = n - 1; k >= 0; --k) {
      const int p = ipv[k];
      const int t = lab[k];
      lab[k] = lab[p];
      lab[p] = t;
    }
  }
  if (i < NMAX) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c) out[i][c] = r[c];
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  if (i < n)
    for (int c = 0; c < n; ++c) A[i + (size_t)c * n] = out[i][lab[c]];
}


template <class T>
void inverse_batched(const std::vector<T *> &ptrs, const std::vector<int> &ns,
                     int32_t *info_dev, Stager &st, hipStream_t s) {
  if (ptrs.empty()) return;
  for (int n : ns) op_flops().inverse += 2.0 * n * n * (double)n;
  op_flops().inverses += (int64_t)ns.size();
  int mx = 1;
  for (int n : ns) mx = std::max(mx, n);
  const size_t shmem = 2 * mx * sizeof(T) + mx * sizeof(int);
  if (shmem > 56 * 1024) fail(SBIE_UNSUPPORTED, "dense block of size %d too large to invert", mx);
  std::vector<void *> dev;
  st.put_many({{ptrs.data(), ptrs.size() * sizeof(T *)}, {ns.data(), ns.size() * sizeof(int)}}, dev, s);
  auto *pd = (T *const *)dev[0];
  auto *nd = (const int *)dev[1];
  if (mx <= 32)
    gj_wave_kernel<T, 32><<<(unsigned)ptrs.size(), 64, 0, s>>>(pd, nd, info_dev);
  else if (mx <= 64)
    gj_wave_kernel<T, 64><<<(unsigned)ptrs.size(), 64, 0, s>>>(pd, nd, info_dev);
  else
    gj_kernel<T><<<(unsigned)ptrs.size(), 256, shmem, s>>>(pd, nd, info_dev);
  SBIE_LAUNCH_CHECK();
}


template <class T>
void inverse_batched_blocked(const std::vector<T *> &ptrs, const std::vector<int> &ns,
                             int32_t *info_dev, Stager &st, hipStream_t s) {
  std::unique_ptr<HostScope> prep(new HostScope(HostProf::kInvPrep));
  const int nm = (int)ptrs.size();
  if (nm == 0) return;
  std::vector<T *> sp, bp;
  std::vector<int> sn, bn, sidx, bidx;
  for (int i = 0; i < nm; ++i) {
    if (ns[i] <= kBlockedMin) { sp.push_back(ptrs[i]); sn.push_back(ns[i]); sidx.push_back(i); }
    else { bp.push_back(ptrs[i]); bn.push_back(ns[i]); bidx.push_back(i); }
  }
  // the small ones are counted by inverse_batched
  for (int n : bn) op_flops().inverse += 2.0 * n * n * (double)n;
  op_flops().inverses += (int64_t)bn.size();
  const int nbm = (int)bp.size();
  const int nb = kPanel;
  int maxn = 0;
  for (int n : bn) maxn = std::max(maxn, n);
  const int npan = nbm ? (maxn + nb - 1) / nb : 0;
  if ((size_t)maxn * sizeof(T) > 64 * 1024)
    fail(SBIE_UNSUPPORTED, "matrix of order %d too large for the blocked inverse", maxn);
  // status words: [small matrices | panel pivots per big matrix | tile
  // inverses per (panel, active big matrix)]
  // stream-ordered allocations: no device-wide synchronisation on release
  StreamBuf<int32_t> stat((size_t)sp.size() + nbm + (size_t)npan * std::max(1, nbm) + 1, s);
  const size_t stat_n = (size_t)sp.size() + nbm + (size_t)npan * std::max(1, nbm) + 1;
  fill_value<int>((int *)stat.p, stat_n, 0, s);
  int32_t *info_small = stat.p;
  int32_t *info_panel = stat.p + sp.size();
  int32_t *info_tile = info_panel + nbm;
  if (!sp.empty()) inverse_batched<T>(sp, sn, info_small, st, s);
  std::vector<std::vector<int>> active(npan);
  size_t ws = 0;
  for (int n : bn) ws += (size_t)n * nb;
  // FP64 panel steps take the fused update (R, -P C and the GEMM update in
  // one launch; see gemm_tiles_mfma_gj), which needs -P C in its own buffer
  constexpr bool fused = std::is_same<T, double>::value;
  StreamBuf<T> work(nbm ? ws : 0, s), C(nbm ? ws : 0, s), R(nbm ? ws : 0, s),
      P(nbm ? (size_t)nbm * nb * nb : 0, s), CPb(nbm && fused ? ws : 0, s);
  StreamBuf<int> piv(nbm ? (size_t)nbm * maxn : 0, s), labb(nbm ? (size_t)nbm * maxn : 0, s);
  StreamBuf<T> negid(nbm ? (size_t)nb * nb : 0, s);   // -I of order nb
  if (nbm) {
    fill_value<T>(negid.p, (size_t)nb * nb, T(0), s);
    set_diagonal<T><<<1, 64, 0, s>>>(negid.p, nb, T(-1));
    SBIE_LAUNCH_CHECK();
    std::vector<T *> woff(nbm), coff(nbm), roff(nbm), poff(nbm), cpoff(nbm, nullptr);
    std::vector<int *> ipv(nbm), lbv(nbm);
    size_t o = 0;
    for (int b = 0; b < nbm; ++b) {
      woff[b] = work.p + o;
      coff[b] = C.p + o;
      roff[b] = R.p + o;
      if (fused) cpoff[b] = CPb.p + o;
      o += (size_t)bn[b] * nb;
      poff[b] = P.p + (size_t)b * nb * nb;
      ipv[b] = piv.p + (size_t)b * maxn;
      lbv[b] = labb.p + (size_t)b * maxn;
    }
    std::vector<void *> mdev;
    st.put_many({{bp.data(), bp.size() * sizeof(T *)}, {bn.data(), bn.size() * sizeof(int)},
                 {lbv.data(), lbv.size() * sizeof(int *)}},
                mdev, s);
    auto *mat_dev = (T *const *)mdev[0];
    auto *n_dev = (const int *)mdev[1];
    auto *lab_dev = (int *const *)mdev[2];
    iota_labels<<<dim3(ceil_div(maxn, 256), nbm), 256, 0, s>>>(lab_dev, n_dev);
    SBIE_LAUNCH_CHECK();
    // Every panel step's descriptors are known up front: they are packed
    // into one host blob and uploaded in a single transfer, and the steps
    // then launch back to back with no host work in between.
    std::vector<char> blob;
    auto add = [&](const void *src, size_t bytes) {
      const size_t o = (blob.size() + 255) & ~size_t(255);
      blob.resize(o + std::max<size_t>(bytes, 1));
      if (bytes) std::memcpy(blob.data() + o, src, bytes);
      return o;
    };
    struct GemmPrep { size_t d = 0, t = 0; unsigned nt = 0; };
    struct CopyPrep { size_t d = 0; int n = 0, max_cols = 0; };
    auto prep_gemm = [&](const std::vector<GemmDesc<T>> &g) {
      std::vector<GemmDesc<T>> keep;
      std::vector<int2> tl;
      for (const auto &q : g) {
        if (q.m <= 0 || q.n <= 0) continue;
        const int id = (int)keep.size();
        keep.push_back(q);
        const int nt = ((q.m + 63) / 64) * ((q.n + 63) / 64);
        for (int t = 0; t < nt; ++t) tl.push_back(make_int2(id, t));
      }
      GemmPrep r;
      r.d = add(keep.data(), keep.size() * sizeof(GemmDesc<T>));
      r.t = add(tl.data(), tl.size() * sizeof(int2));
      r.nt = (unsigned)tl.size();
      return r;
    };
    auto prep_copy = [&](const std::vector<CopyDesc<T>> &c) {
      std::vector<CopyDesc<T>> keep;
      CopyPrep r;
      for (const auto &q : c)
        if (q.rows > 0 && q.cols > 0) {
          keep.push_back(q);
          r.max_cols = std::max(r.max_cols, q.cols);
        }
      r.d = add(keep.data(), keep.size() * sizeof(CopyDesc<T>));
      r.n = (int)keep.size();
      return r;
    };
    struct Step {
      size_t pd = 0, pp = 0, pn = 0, psrc = 0, pld = 0, fix = 0;
      int npd = 0, hmax = 0, pmax = 0;
      bool fused_panel = false;
      CopyPrep cC, cRow;
      GemmPrep gR, gUpd, gCol;
    };
    std::vector<Step> steps;
    for (int it = 0; it < npan; ++it) {
      const int k0 = it * nb;
      std::vector<PanelDesc<T>> pd;
      std::vector<T *> pp;
      std::vector<const T *> psrc;
      std::vector<int> pn, pld;
      std::vector<CopyDesc<T>> cC, cRow;
      std::vector<GemmDesc<T>> gR, gUpd, gCol;
      std::vector<GjFix> fix;
      for (int b = 0; b < nbm; ++b) {
        const int n = bn[b];
        if (k0 >= n) continue;
        active[it].push_back(b);
        const int pb = std::min(nb, n - k0);
        T *A = bp[b];
        pd.push_back({A, woff[b], ipv[b], lbv[b], n, k0, pb, info_panel + b});
        pp.push_back(poff[b]);
        pn.push_back(pb);
        psrc.push_back(A + k0 + (size_t)k0 * n);
        pld.push_back(n);
        // p = [k0, k0 + pb).  C = A[p, :] (pb x n) with its pivot columns
        // replaced by -I: then the update A -= R C leaves columns p to be
        // overwritten by R = A[:, p] P, and A[p, :] = -P C puts P itself in
        // the pivot block
        if (k0 > 0) cC.push_back({A + k0, n, coff[b], pb, pb, k0, 0, 0, T(1)});
        cC.push_back({negid.p, nb, coff[b] + (size_t)k0 * pb, pb, pb, pb, 0, 0, T(1)});
        if (k0 + pb < n)
          cC.push_back({A + k0 + (size_t)(k0 + pb) * n, n, coff[b] + (size_t)(k0 + pb) * pb, pb, pb,
                        n - k0 - pb, 0, 0, T(1)});
        gR.push_back({n, pb, pb, 0, 0, A + (size_t)k0 * n, n, poff[b], pb, roff[b], n, T(1), T(0)});
        gUpd.push_back({n, n, pb, 0, 0, roff[b], n, coff[b], pb, A, n, T(-1), T(1)});
        if constexpr (fused) {
          // -P C into its own buffer, in the same launch as R; the update's
          // epilogue then writes R into columns p and -P C into rows p
          gR.push_back({pb, n, pb, 0, 0, poff[b], pb, coff[b], pb, cpoff[b], pb, T(-1), T(0)});
          fix.push_back({(const double *)roff[b], (const double *)cpoff[b], k0, pb});
        } else {
          cRow.push_back({roff[b], n, A + (size_t)k0 * n, n, n, pb, 0, 0, T(1)});
          gCol.push_back({pb, n, pb, 0, 0, poff[b], pb, coff[b], pb, A + k0, n, T(-1), T(0)});
        }
      }
      if (pd.empty()) break;
      Step st_;
      st_.npd = (int)pd.size();
      for (const auto &q : pd) st_.hmax = std::max(st_.hmax, q.n - q.k0);
      // the register panel kernel also inverts the pivot blocks and forms C
      st_.fused_panel = st_.hmax <= kPanelRegRows;
      if (st_.fused_panel)
        for (size_t q = 0; q < pd.size(); ++q) {
          pd[q].P = pp[q];
          pd[q].C = coff[active[it][q]];
          pd[q].tinfo = info_tile + (size_t)it * nbm + q;
        }
      for (int q : pn) st_.pmax = std::max(st_.pmax, q);
      st_.pd = add(pd.data(), pd.size() * sizeof(PanelDesc<T>));
      st_.pp = add(pp.data(), pp.size() * sizeof(T *));
      st_.pn = add(pn.data(), pn.size() * sizeof(int));
      st_.psrc = add(psrc.data(), psrc.size() * sizeof(T *));
      st_.pld = add(pld.data(), pld.size() * sizeof(int));
      st_.cC = prep_copy(cC);
      st_.gR = prep_gemm(gR);
      st_.gUpd = prep_gemm(gUpd);
      st_.cRow = prep_copy(cRow);
      st_.gCol = prep_gemm(gCol);
      // the fused update's fixes follow gUpd's descriptors one to one (all
      // of them have m, n > 0, so prep_gemm keeps every one)
      st_.fix = add(fix.data(), fix.size() * sizeof(GjFix));
      steps.push_back(st_);
    }
    char *db = (char *)st.put(blob.data(), blob.size(), s);
    prep.reset();
    HostScope loop_scope(HostProf::kInvLaunch);
    auto copy_step = [&](const CopyPrep &c) {
      copy_launch<T>((const CopyDesc<T> *)(db + c.d), c.n, c.max_cols, s);
    };
    auto gemm_step = [&](const GemmPrep &g) {
      if (g.nt == 0) return;
      launch_gemm_tiles<T>(g.nt, (const GemmDesc<T> *)(db + g.d), (const int2 *)(db + g.t), s, GemmInputs::kWorking);
    };
    for (size_t it = 0; it < steps.size(); ++it) {
      const Step &q = steps[it];
      const auto *dd = (const PanelDesc<T> *)(db + q.pd);
      static_assert(kPanel <= 32, "the register panels hold 32 entries per vector");
      if (q.hmax <= 256)                                                // choose columns, swap
        panel_pivot_reg_kernel<T, 256, 1><<<(unsigned)q.npd, 256, 0, s>>>(dd);
      else if (q.hmax <= 512)
        panel_pivot_reg_kernel<T, 512, 1><<<(unsigned)q.npd, 512, 0, s>>>(dd);
      else if (q.hmax <= kPanelRegRows)
        panel_pivot_reg_kernel<T, 768, 1><<<(unsigned)q.npd, 768, 0, s>>>(dd);
      else
        panel_pivot_kernel<T><<<(unsigned)q.npd, 256, 0, s>>>(dd);
      SBIE_LAUNCH_CHECK();
      if (!q.fused_panel) {                                             // P = A_pp^-1
        T *const *pp_ = (T *const *)(db + q.pp);
        const int *pn_ = (const int *)(db + q.pn);
        const T *const *ps_ = (const T *const *)(db + q.psrc);
        const int *pl_ = (const int *)(db + q.pld);
        int32_t *inf = info_tile + it * nbm;
        static_assert(kPanel <= 32, "pivot blocks are inverted by 32-row waves");
        gj_nopiv_wave_kernel<T, 32><<<(unsigned)q.npd, 64, 0, s>>>(pp_, pn_, inf, ps_, pl_);
        SBIE_LAUNCH_CHECK();
      }
      if (!q.fused_panel) copy_step(q.cC);                              // C = A[p, :], C[:, p] = -I
      gemm_step(q.gR);                                                  // R = A[:, p] P (and -P C)
      if constexpr (fused) {                                            // A -= R C, A[:, p] = R, A[p, :] = -P C
        if (q.gUpd.nt) {
          gemm_tiles_mfma_gj<<<q.gUpd.nt, 256, 0, s>>>((const GemmDesc<double> *)(db + q.gUpd.d),
                                                       (const int2 *)(db + q.gUpd.t),
                                                       (const GjFix *)(db + q.fix));
          SBIE_LAUNCH_CHECK();
        }
      } else {
        gemm_step(q.gUpd);                                              // A -= R C
        copy_step(q.cRow);                                              // A[:, p] = R
        gemm_step(q.gCol);                                              // A[p, :] = -P C
      }
    }
    unpermute_rows_kernel<T><<<dim3(ceil_div(maxn, kUnpermCols), nbm), 256, (size_t)maxn * sizeof(T), s>>>(
        mat_dev, n_dev, lab_dev);
    SBIE_LAUNCH_CHECK();
  }
  // Merge the statuses on the device (no host round trip): a small matrix
  // reports its own status; a big one its panel-pivot failure, else the
  // first failing pivot-block inverse (as a column index).  tpos[it * nbm +
  // b] is matrix b's slot among the active matrices of panel it, or -1.
  {
    std::vector<int> tpos((size_t)std::max(1, npan) * std::max(1, nbm), -1);
    for (int it = 0; it < npan; ++it)
      for (size_t q = 0; q < active[it].size(); ++q) tpos[(size_t)it * nbm + active[it][q]] = (int)q;
    std::vector<void *> dev;
    st.put_many({{sidx.data(), sidx.size() * sizeof(int)}, {bidx.data(), bidx.size() * sizeof(int)},
                 {tpos.data(), tpos.size() * sizeof(int)}},
                dev, s);
    const int work_items = (int)sidx.size() + nbm;
    merge_status<<<ceil_div(std::max(1, work_items), 256), 256, 0, s>>>(
        stat.p, (int)sidx.size(), nbm, npan, nb, (const int *)dev[0], (const int *)dev[1],
        (const int *)dev[2], info_dev);
    SBIE_LAUNCH_CHECK();
  }
}

template <class T>
void norms_batched(const std::vector<NormDesc<T>> &d, double *out_dev, Stager &st,
                   hipStream_t s) {
  if (d.empty()) return;
  auto *dd = (const NormDesc<T> *)st.put(d.data(), d.size() * sizeof(NormDesc<T>), s);
  norm_desc<T><<<(unsigned)d.size(), 256, 0, s>>>(dd, out_dev);
  SBIE_LAUNCH_CHECK();
}

// Every column of every block to unit norm: blockIdx.x = block, blockIdx.y =
// column (beyond a block's width: nothing to do).
template <class T>
__global__ __launch_bounds__(256) void normalize_cols_desc(const NormDesc<T> *__restrict__ descs) {
  const NormDesc<T> d = descs[blockIdx.x];
  if ((int)blockIdx.y >= d.cols) return;
  T *col = const_cast<T *>(d.A) + (size_t)blockIdx.y * d.lda;
  double s = 0.0;
  for (int r = threadIdx.x; r < d.rows; r += 256) s = fma((double)col[r], (double)col[r], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double nrm = sqrt((red[0] + red[1]) + (red[2] + red[3]));
  const T scale = nrm > 0.0 ? T(1.0 / nrm) : T(0);
  for (int r = threadIdx.x; r < d.rows; r += 256) col[r] *= scale;
}

template <class T>
void normalize_batched(const std::vector<NormDesc<T>> &d, Stager &st, hipStream_t s) {
  int mc = 0;
  for (const auto &q : d) mc = std::max(mc, q.rows > 0 ? q.cols : 0);
  if (d.empty() || mc == 0) return;
  auto *dd = (const NormDesc<T> *)st.put(d.data(), d.size() * sizeof(NormDesc<T>), s);
  normalize_cols_desc<T><<<dim3((unsigned)d.size(), (unsigned)mc), 256, 0, s>>>(dd);
  SBIE_LAUNCH_CHECK();
}

template <class T>
void normalize_columns(T *A, int lda, int rows, int cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return;
  normalize_cols<T><<<cols, 256, 0, s>>>(A, lda, rows);
  SBIE_LAUNCH_CHECK();
}

template <class T>
void pgs_batched(const std::vector<PgsDesc<T>> &d, Stager &st, hipStream_t s) {
  HostScope hs(HostProf::kOther);
  if (d.empty()) return;
  size_t shmem = 0;
  for (const auto &p : d) {
    const size_t b = (size_t)p.c * sizeof(double) + (size_t)p.rmax * sizeof(double) +
                     (size_t)p.m * sizeof(T);
    shmem = std::max(shmem, b);
  }
  if (shmem > 60 * 1024)
    fail(SBIE_UNSUPPORTED, "rank-revealing step too large (%zu bytes of LDS)", shmem);
  auto *dd = (const PgsDesc<T> *)st.put(d.data(), d.size() * sizeof(PgsDesc<T>), s);
  if constexpr (std::is_same<T, double>::value) {
    // blocked pivoting: as many block columns (up to 8) as the LDS holds
    int cmax = 0, mmax = 1;
    for (const auto &p : d) { cmax = std::max(cmax, p.c); mmax = std::max(mmax, p.m); }
    const size_t room = (size_t)48 * 1024 - (size_t)cmax * sizeof(double);
    const int b = (int)std::min<size_t>(8, room / ((size_t)mmax * sizeof(double)));
    if (b >= 4) {
      const size_t sh = (size_t)cmax * sizeof(double) + (size_t)b * mmax * sizeof(double);
      if (b >= 8)
        pgs_block_kernel<8><<<(unsigned)d.size(), kPgsThreads, sh, s>>>(dd);
      else
        pgs_block_kernel<4><<<(unsigned)d.size(), kPgsThreads, (size_t)cmax * sizeof(double) +
                              (size_t)4 * mmax * sizeof(double), s>>>(dd);
      SBIE_LAUNCH_CHECK();
      return;
    }
  }
  pgs_kernel<T><<<(unsigned)d.size(), kPgsThreads, shmem, s>>>(dd);
  SBIE_LAUNCH_CHECK();
}

template <class T>
void gaussian_fill(T *out, size_t n, uint64_t seed, hipStream_t s) {
  if (n == 0) return;
  gaussian_kernel<T><<<ceil_div((int64_t)n, 256), 256, 0, s>>>(out, n, seed);
  SBIE_LAUNCH_CHECK();
}

template <class T>
void fill_value(T *out, size_t n, T v, hipStream_t s) {
  if (n == 0) return;
  fill_kernel<T><<<ceil_div((int64_t)n, 256), 256, 0, s>>>(out, n, v);
  SBIE_LAUNCH_CHECK();
}

template <class A, class B>
void convert(const A *src, B *dst, size_t n, hipStream_t s) {
  if (n == 0) return;
  convert_kernel<A, B><<<ceil_div((int64_t)n, 256), 256, 0, s>>>(src, dst, n);
  SBIE_LAUNCH_CHECK();
}

#define SBIE_INST(T)                                                                     \
  template void gemm_batched<T>(const std::vector<GemmDesc<T>> &, Stager &, hipStream_t); \
  template void gemm_batched_sketch<T>(const std::vector<GemmDesc<T>> &, GemmInputs, Stager &, hipStream_t); \
  template void gemv_batched<T>(const std::vector<GemvDesc<T>> &,                        \
                                const std::vector<GemvTerm<T>> &, Stager &, hipStream_t); \
  template void gemv_launch<T, T>(const GemvDesc<T> *, const GemvTerm<T, T> *, int, int, \
                               hipStream_t);                                             \
  template void copy_batched<T>(const std::vector<CopyDesc<T>> &, Stager &, hipStream_t); \
  template void copy_launch<T>(const CopyDesc<T> *, int, int, hipStream_t);              \
  template void inverse_batched<T>(const std::vector<T *> &, const std::vector<int> &,   \
                                   int32_t *, Stager &, hipStream_t);                    \
  template void inverse_batched_blocked<T>(const std::vector<T *> &,                     \
                                           const std::vector<int> &, int32_t *, Stager &, \
                                           hipStream_t);                                 \
  template void norms_batched<T>(const std::vector<NormDesc<T>> &, double *, Stager &,   \
                                 hipStream_t);                                           \
  template void normalize_columns<T>(T *, int, int, int, hipStream_t);                   \
  template void normalize_batched<T>(const std::vector<NormDesc<T>> &, Stager &, hipStream_t); \
  template void pgs_batched<T>(const std::vector<PgsDesc<T>> &, Stager &, hipStream_t);  \
  template void gaussian_fill<T>(T *, size_t, uint64_t, hipStream_t);                   \
  template void fill_value<T>(T *, size_t, T, hipStream_t);

SBIE_INST(double)
SBIE_INST(float)
template void fill_value<int>(int *, size_t, int, hipStream_t);
template void convert<double, float>(const double *, float *, size_t, hipStream_t);
template void convert<float, double>(const float *, double *, size_t, hipStream_t);
template void convert<double, double>(const double *, double *, size_t, hipStream_t);
template void convert<float, float>(const float *, float *, size_t, hipStream_t);
template void gemv_launch<double, float>(const GemvDesc<double> *, const GemvTerm<double, float> *, int,
                                         int, hipStream_t);

}  // namespace sbie
