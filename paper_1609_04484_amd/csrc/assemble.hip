// Dense blocks A[rows, cols] of the completed double-layer operator: the
// diagonal blocks of the block-diagonal preconditioner (Section 4.1.1), the
// near-field blocks of the IFMM (Section 3.1), and small dense systems.
#include "assemble.hpp"

namespace sbie {

namespace {

__global__ void assemble_kernel(GeomView g, const int64_t *__restrict__ rows,
                                int64_t nr, const int64_t *__restrict__ cols,
                                int64_t nc, double *__restrict__ out,
                                int64_t ld) {
  const int64_t ri = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ci = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  if (ri >= nr || ci >= nc) return;
  out[ri + ci * ld] = op_entry(g, rows[ri], cols[ci]);
}

// Batched square blocks: block b uses indices idx[ioff[b] .. ioff[b]+sz[b])
// for both rows and columns and writes a column-major sz x sz matrix at
// out + ooff[b].
__global__ void assemble_diag_blocks(GeomView g, const int64_t *__restrict__ idx,
                                     const int64_t *__restrict__ ioff,
                                     const int32_t *__restrict__ sz,
                                     const int64_t *__restrict__ ooff,
                                     double *__restrict__ out) {
  const int b = blockIdx.z;
  const int n = sz[b];
  const int ri = blockIdx.x * blockDim.x + threadIdx.x;
  const int ci = blockIdx.y * blockDim.y + threadIdx.y;
  if (ri >= n || ci >= n) return;
  const int64_t *ix = idx + ioff[b];
  out[ooff[b] + ri + (int64_t)ci * n] = op_entry(g, ix[ri], ix[ci]);
}

}  // namespace

void assemble_block(const GeomView &v, const int64_t *rows, int64_t nr,
                    const int64_t *cols, int64_t nc, double *out, int64_t ld,
                    hipStream_t s) {
  if (nr == 0 || nc == 0) return;
  dim3 blk(64, 4);
  dim3 grid(ceil_div(nr, 64), ceil_div(nc, 4));
  if (grid.y > 65535) {
    // tile the column range to respect the grid limit
    const int64_t step = (int64_t)65535 * 4;
    for (int64_t c0 = 0; c0 < nc; c0 += step) {
      const int64_t cn = nc - c0 < step ? nc - c0 : step;
      dim3 g2(ceil_div(nr, 64), ceil_div(cn, 4));
      assemble_kernel<<<g2, blk, 0, s>>>(v, rows, nr, cols + c0, cn, out + c0 * ld, ld);
      SBIE_LAUNCH_CHECK();
    }
    return;
  }
  assemble_kernel<<<grid, blk, 0, s>>>(v, rows, nr, cols, nc, out, ld);
  SBIE_LAUNCH_CHECK();
}

void assemble_diag_batched(const GeomView &v, const int64_t *idx,
                           const int64_t *ioff, const int32_t *sz,
                           const int64_t *ooff, int nblocks, int max_n,
                           double *out, hipStream_t s) {
  if (nblocks == 0) return;
  dim3 blk(64, 4);
  for (int b0 = 0; b0 < nblocks; b0 += 65535) {
    const int nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    dim3 grid(ceil_div(max_n, 64), ceil_div(max_n, 4), nb);
    assemble_diag_blocks<<<grid, blk, 0, s>>>(v, idx, ioff + b0, sz + b0, ooff + b0, out);
    SBIE_LAUNCH_CHECK();
  }
}

}  // namespace sbie

extern "C" int stokes_bie_assemble(const sbie_geom *g, const int64_t *rows,
                                   int64_t nr, const int64_t *cols, int64_t nc,
                                   double *out, int64_t ld, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (nr < 0 || nc < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "negative block size");
    if (nr == 0 || nc == 0) return SBIE_OK;
    if (!rows || !cols || !out) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (ld < nr) sbie::fail(SBIE_INVALID_ARGUMENT, "ld < nr");
    hipStream_t s = (hipStream_t)stream;
    sbie::StreamBuf<double> wl(1, s);
    sbie::wall_length(g, wl.p, s);
    sbie::GeomView v = sbie::make_view(g, wl.p);
    sbie::assemble_block(v, rows, nr, cols, nc, out, ld, s);
    return SBIE_OK;
  });
}
