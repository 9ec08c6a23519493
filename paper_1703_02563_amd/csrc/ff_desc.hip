// Scale-space low-pass and per-pixel descriptors (Sec. 3.2 scale spaces,
// Sec. 3.6 low-pass filtering and replicate border condition).
//
// I^n: integer box filter of half-width h = max(1, n/2), rounded half up,
// computed separably (row sums, then column sums of the row sums; both are
// exact in integers), per 64 x 64 tile in LDS (batches: through a row-sum
// buffer).  Descriptor of scale n: the 16 samples of I^n on a 4x4
// grid with spacing 2n around the pixel, stored as one 16-byte vector per
// pixel so that a patch position costs one 128-bit load; the pixels of each
// row are stored in phase order (x mod n, then x / n), and the map carries a
// replicated border of 3n pixels (desc_col, desc_index).
//
// All (image, scale) jobs of a call run in one launch per stage: blockIdx.z
// selects the job.
#include <algorithm>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

using ffk::clampi;

// Box filter of one (image, scale) job on a 64 x 64 tile of outputs: the
// input tile with its h-wide border (edge pixels replicated) is staged in
// LDS, every staged row gets the row sums of the tile's 64 columns by a
// sliding window over 8 consecutive columns, then every output takes the
// column sum of 2h + 1 row sums, also sliding over 8 rows, rounded half up
// over the box area.  These are the integer sums of the separable
// definition (exact in any order), in one pass over the image.
constexpr int kBT = 64, kBHmax = 32, kBS = kBT + 2 * kBHmax;  // tile, largest half-width (n <= 64), staged side

__global__ __launch_bounds__(256) void k_blur(ffh::DescJobs jobs) {
  __shared__ uint8_t s_in[kBS * kBS];
  __shared__ uint16_t s_row[kBS * kBT];  // (2h + 1) * 255 fits 16 bits
  const ffh::DescJob &jb = jobs.job[blockIdx.z];
  const int W = jobs.W, H = jobs.H;
  const int h = max(1, jb.n >> 1), S = kBT + 2 * h;  // staged rows and columns
  const int x0 = blockIdx.x * kBT, y0 = blockIdx.y * kBT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // staged rows ty + 4u, columns tx and tx + 64: 16 loads in flight per
  // thread before their LDS stores (rows past S read a clamped row, unused)
  const int xa = clampi(x0 - h + tx, W - 1), xb = clampi(x0 - h + tx + 64, W - 1);
  for (int u0 = 0; u0 < S; u0 += 32) {
    uint32_t va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint8_t *row = jb.img + (size_t)clampi(y0 - h + u0 + ty + 4 * u, H - 1) * W;
      va[u] = row[xa];
      vb[u] = row[xb];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = u0 + ty + 4 * u;
      if (r < S) {
        s_in[r * S + tx] = (uint8_t)va[u];
        if (tx + 64 < S) s_in[r * S + tx + 64] = (uint8_t)vb[u];
      }
    }
  }
  __syncthreads();
  // row sums of staged row r for output columns c0 .. c0 + 7 (window of
  // output column c: staged columns c .. c + 2h)
  for (int k = threadIdx.x; k < S * (kBT / 8); k += 256) {
    const int r = k >> 3, c0 = (k & 7) * 8;
    const uint8_t *row = s_in + r * S + c0;
    uint16_t *out = s_row + r * kBT + c0;
    uint32_t sum = 0;
#pragma unroll 8
    for (int dx = 0; dx <= 2 * h; ++dx) sum += row[dx];
    out[0] = (uint16_t)sum;
#pragma unroll
    for (int c = 1; c < 8; ++c) {
      sum += row[c + 2 * h];
      sum -= row[c - 1];
      out[c] = (uint16_t)sum;
    }
  }
  __syncthreads();
  // column sums for output column c, rows r0 .. r0 + 7 (window of output
  // row r: staged rows r .. r + 2h)
  const uint32_t area = (uint32_t)((2 * h + 1) * (2 * h + 1));
  for (int k = threadIdx.x; k < kBT * (kBT / 8); k += 256) {
    const int c = k & (kBT - 1), r0 = (k / kBT) * 8, x = x0 + c;
    const uint16_t *col = s_row + r0 * kBT + c;
    uint32_t sum = 0;
#pragma unroll 8
    for (int dy = 0; dy <= 2 * h; ++dy) sum += col[dy * kBT];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r > 0) {
        sum += col[(r + 2 * h) * kBT];
        sum -= col[(r - 1) * kBT];
      }
      const int y = y0 + r0 + r;
      if (x < W && y < H) jb.blurred[(size_t)y * W + x] = (uint8_t)((sum + area / 2) / area);
    }
  }
}

// The 16 samples of the scale-n descriptor of pixel (x, y) (in the image).
__device__ __forceinline__ uint4 descriptor_at(const uint8_t *blurred, int W, int H, int n, int x, int y) {
  uint32_t w[4];
#pragma unroll
  for (int gy = 0; gy < 4; ++gy) {
    const uint8_t *row = blurred + (size_t)clampi(y + n * (2 * gy - 3), H - 1) * W;
    uint32_t v = 0;
#pragma unroll
    for (int gx = 0; gx < 4; ++gx) v |= (uint32_t)row[clampi(x + n * (2 * gx - 3), W - 1)] << (8 * gx);
    w[gy] = v;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Weight-class row entry (wform_index) of pixel x of blurred row `row`.
__device__ __forceinline__ uint4 wform_entry(const uint8_t *row, int W, int n, int x) {
  auto at = [&](int a) { return (uint32_t)row[clampi(x + n * a, W - 1)]; };
  return make_uint4(at(-6) | at(-5) << 8 | at(5) << 16 | at(6) << 24, at(-4) | at(-3) << 8 | at(3) << 16 | at(4) << 24,
                    at(-2) | at(-1) << 8 | at(1) << 16 | at(2) << 24, at(0));
}

// One workgroup per stored row yp of one map: the four blurred rows its
// descriptors sample (y + n(2gy - 3), clamped) are staged in LDS once, then
// every entry of the padded row (coalesced 16-byte stores) takes its 16
// samples from there.  Entries that are image pixels also go to the
// row-major copy when one is requested.  The weight-class row map has the
// same rows (y + 3n); its row yp is written from a fifth staged row, the
// blurred row y itself.  Dynamic LDS: 5 * row_stride(W).
__host__ __device__ __forceinline__ int desc_row_stride(int W) { return (W + 15) & ~15; }

__global__ __launch_bounds__(256) void k_desc(ffh::DescJobs jobs) {
  extern __shared__ uint8_t s_rows[];
  const ffh::DescJob &jb = jobs.job[blockIdx.y];
  const int W = jobs.W, H = jobs.H, n = jb.n, l2 = ffk::map_log2(n);
  const int P = ffk::desc_pad(n), Wp = W + 2 * P, Hp = H + 2 * P;
  const int yp = blockIdx.x, Ws = desc_row_stride(W);
  if (yp >= Hp) return;  // workgroup-uniform
  const int yr = yp - P, y = clampi(yr, H - 1);
  // staged rows g = 0..3: y + n(2g - 3); g = 4: y itself (weight-class map)
  const int nrows = jb.wform ? 5 : 4;
  auto src_row = [&](int g) { return g < 4 ? clampi(y + n * (2 * g - 3), H - 1) : y; };
  if ((W & 3) == 0) {  // rows start on 4-byte boundaries: dword loads
    const int wq = W >> 2;
    for (int k = threadIdx.x; k < nrows * wq; k += blockDim.x) {
      const int g = k / wq, q = k - g * wq;
      const uint32_t *row = reinterpret_cast<const uint32_t *>(jb.blurred + (size_t)src_row(g) * W);
      reinterpret_cast<uint32_t *>(s_rows + g * Ws)[q] = row[q];
    }
  } else {
    for (int k = threadIdx.x; k < nrows * W; k += blockDim.x) {
      const int g = k / W, x = k - g * W;
      s_rows[g * Ws + x] = jb.blurred[(size_t)src_row(g) * W + x];
    }
  }
  __syncthreads();
  // the weight-class map's rows y in [-3n, H + 3n) are a band of the
  // descriptor map's rows [-4n, H + 4n): stored row y + 3n
  const int ywf = yr + ffk::kWformPad * n;
  if (jb.wform && ywf >= 0 && ywf < H + 2 * ffk::kWformPad * n) {
    uint4 *wout = reinterpret_cast<uint4 *>(jb.wform) + (size_t)ywf * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) wout[x] = wform_entry(s_rows + 4 * Ws, W, n, x);
  }
  uint4 *out = reinterpret_cast<uint4 *>(jb.desc) + (size_t)yp * Wp;
  for (int c = threadIdx.x; c < Wp; c += blockDim.x) {
    const int xr = ffk::desc_pixel(c, l2, Wp) - P, x = clampi(xr, W - 1);
    uint32_t w[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint8_t *row = s_rows + g * Ws;
      uint32_t v = 0;
#pragma unroll
      for (int gx = 0; gx < 4; ++gx) v |= (uint32_t)row[clampi(x + n * (2 * gx - 3), W - 1)] << (8 * gx);
      w[g] = v;
    }
    const uint4 d = make_uint4(w[0], w[1], w[2], w[3]);
    if (jb.desc) out[c] = d;
    if (jb.compact && xr >= 0 && xr < W && yr >= 0 && yr < H)
      reinterpret_cast<uint4 *>(jb.compact)[(size_t)yr * W + xr] = d;
  }
}

// ---- batches: items = (pair, image * L + scale, row) ---------------------
struct RowItem {
  const ffh::BatchPair *bp;
  int im, lv, y;
};

__device__ __forceinline__ RowItem row_item(const ffh::BatchStage &st, int item) {
  const int p = ffk::batch_pair(st.prefix, st.npairs, item);
  const ffh::BatchPair &bp = st.pairs[p];
  const int local = item - st.prefix[p];
  const int z = local / bp.H;
  return {&bp, z / st.L, z % st.L, local % bp.H};
}

__global__ __launch_bounds__(256) void k_hsum_batch(ffh::BatchStage st) {
  ffk::for_items(st.total, [&](int item) {
    const RowItem r = row_item(st, item);
    const int W = r.bp->W, h = max(1, (1 << r.lv) >> 1);
    const uint8_t *row = r.bp->img[r.im] + (size_t)r.y * W;
    uint16_t *out = r.bp->hsum[r.im][r.lv] + (size_t)r.y * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
      uint32_t s = 0;
      for (int dx = -h; dx <= h; ++dx) s += row[clampi(x + dx, W - 1)];
      out[x] = (uint16_t)s;
    }
  });
}

__global__ __launch_bounds__(256) void k_vsum_batch(ffh::BatchStage st) {
  ffk::for_items(st.total, [&](int item) {
    const RowItem r = row_item(st, item);
    const int W = r.bp->W, H = r.bp->H, h = max(1, (1 << r.lv) >> 1);
    const uint32_t area = (uint32_t)((2 * h + 1) * (2 * h + 1));
    const uint16_t *hs = r.bp->hsum[r.im][r.lv];
    uint8_t *out = r.bp->blur[r.im][r.lv] + (size_t)r.y * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
      uint32_t s = 0;
      for (int dy = -h; dy <= h; ++dy) s += hs[(size_t)clampi(r.y + dy, H - 1) * W + x];
      out[x] = (uint8_t)((s + area / 2) / area);
    }
  });
}

// Item (pair, image, scale, image row y): padded row y + P, and for the
// first and last image rows also the border rows they replicate; scale 1
// items also write the row-major copy used by the NN seed.
__global__ __launch_bounds__(256) void k_desc_batch(ffh::BatchStage st) {
  ffk::for_items(st.total, [&](int item) {
    const RowItem r = row_item(st, item);
    const int W = r.bp->W, H = r.bp->H, n = 1 << r.lv;
    const int P = ffk::desc_pad(n), Wp = W + 2 * P;
    const uint8_t *b = r.bp->blur[r.im][r.lv];
    uint4 *map = reinterpret_cast<uint4 *>(r.bp->desc[r.im][r.lv]);
    const int yp0 = r.y == 0 ? 0 : r.y + P, yp1 = r.y == H - 1 ? H + 2 * P : r.y + P + 1;
    for (int c = threadIdx.x; c < Wp; c += blockDim.x) {
      const int xr = ffk::desc_pixel(c, r.lv, Wp) - P;
      const uint4 d = descriptor_at(b, W, H, n, clampi(xr, W - 1), r.y);
      for (int yp = yp0; yp < yp1; ++yp) map[(size_t)yp * Wp + c] = d;
      if (r.lv == 0 && xr >= 0 && xr < W) reinterpret_cast<uint4 *>(r.bp->desc1[r.im])[(size_t)r.y * W + xr] = d;
    }
    // weight-class rows: stored row y + 3n, the first and last image rows
    // replicated into the 3n border rows
    uint4 *wmap = reinterpret_cast<uint4 *>(r.bp->wform[r.im][r.lv]);
    if (wmap) {
      const int Pw = ffk::kWformPad * n;
      const int wy0 = r.y == 0 ? 0 : r.y + Pw, wy1 = r.y == H - 1 ? H + 2 * Pw : r.y + Pw + 1;
      const uint8_t *brow = b + (size_t)r.y * W;
      for (int x = threadIdx.x; x < W; x += blockDim.x) {
        const uint4 e = wform_entry(brow, W, n, x);
        for (int yw = wy0; yw < wy1; ++yw) wmap[(size_t)yw * W + x] = e;
      }
    }
  });
}

}  // namespace

namespace ffh {

hipError_t launch_batch_descriptors(const BatchStage &rows, hipStream_t stream) {
  if (rows.total <= 0) return hipSuccess;
  const dim3 grid(((std::min(rows.total, 4096) + 7) / 8) * 8);
  hipLaunchKernelGGL(k_hsum_batch, grid, dim3(256), 0, stream, rows);
  hipLaunchKernelGGL(k_vsum_batch, grid, dim3(256), 0, stream, rows);
  hipLaunchKernelGGL(k_desc_batch, grid, dim3(256), 0, stream, rows);
  return hipGetLastError();
}

hipError_t launch_descriptors(const DescJobs &jobs, hipStream_t stream) {
  if (jobs.count <= 0) return hipSuccess;
  for (int k = 0; k < jobs.count; ++k)
    if (jobs.job[k].n < 1 || jobs.job[k].n > 2 * kBHmax + 1) return hipErrorInvalidValue;
  const dim3 gb((jobs.W + kBT - 1) / kBT, (jobs.H + kBT - 1) / kBT, jobs.count);
  hipLaunchKernelGGL(k_blur, gb, dim3(256), 0, stream, jobs);
  int pmax = 0;
  for (int k = 0; k < jobs.count; ++k) pmax = std::max(pmax, ffk::desc_pad(jobs.job[k].n));
  const size_t lds = 5 * (size_t)desc_row_stride(jobs.W);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {  // rows wider than 16 K pixels
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_desc),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 gpad(jobs.H + 2 * pmax, jobs.count);
  hipLaunchKernelGGL(k_desc, gpad, dim3(256), lds, stream, jobs);
  return hipGetLastError();
}

}  // namespace ffh
