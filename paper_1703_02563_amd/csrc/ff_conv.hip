// Learned descriptor network kernels: 3x3 convolutions in NHWC with bf16
// operands and float32 accumulation on matrix cores, their backward passes,
// the Adam update, and the quantisation of learned features to bytes.
//
// Convolution as an implicit GEMM: 32 output pixels x 32 output channels per
// wave, K = 9 taps x Cin in chunks of 16 (one v_mfma_f32_32x32x16_bf16 per
// chunk).  A lane holds 8 consecutive input channels of one tap of one pixel
// (16 bytes, zero outside the image: "same" zero padding) and the matching 8
// weights of one output channel.  Layout: activations [B][H][W][C], weights
// [Cout][9][Cin] (tap = 3 * (dy + 1) + (dx + 1)).
//
// The data gradient is the same convolution with the weights rotated by 180
// degrees and transposed ([Cin][9][Cout]).  The weight gradient is a
// contraction over all pixels, also on matrix cores; each workgroup writes
// a partial sum of its rows and a second kernel adds the partials in a fixed
// order, so it is deterministic.
#include <algorithm>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

// The 16 features of one pixel scaled to unit length; returns the scale.
__device__ __forceinline__ float l2norm16(float4 v[4], float delta) {
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += v[k].x * v[k].x + v[k].y * v[k].y + v[k].z * v[k].z + v[k].w * v[k].w;
  const float r = 1.0f / sqrtf(s + delta);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = make_float4(v[k].x * r, v[k].y * r, v[k].z * r, v[k].w * r);
  return r;
}

// Single input channel (the first layer): K = 9 taps padded to 16, lane
// half kh holds taps 8 * kh .. 8 * kh + 7 of one pixel.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_fwd(ffh::ConvArgs a) {
  static_assert(CIN == 1, "Cin 1 (wider inputs: k_conv_fwd_tile)");
  static_assert(COUT <= 32, "Cout <= 32");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 31, kh = lane >> 5;
  const long long P = (long long)a.B * a.H * a.W;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * 32;
  if (p0 >= P) return;  // wave-uniform
  const long long p = p0 + row;
  const bool pv = p < P;
  const int x = pv ? (int)(p % a.W) : 0, y = pv ? (int)((p / a.W) % a.H) : 0;
  const long long img = pv ? p / ((long long)a.W * a.H) : 0;
  const uint16_t *in = a.in;
  const int col = row;  // output channel held by this lane in the B operand
  f32x16 acc = {0};
  uint16_t av[8], bv[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int tap = 8 * kh + e;
    uint16_t va = 0, vb = 0;
    if (tap < 9) {
      const int sx = x + tap % 3 - 1, sy = y + tap / 3 - 1;
      if (pv && sx >= 0 && sx < a.W && sy >= 0 && sy < a.H) va = in[((img * a.H + sy) * a.W + sx)];
      if (col < COUT) vb = a.w[col * 9 + tap];
    }
    av[e] = va;
    bv[e] = vb;
  }
  uint4 ua, ub;
  __builtin_memcpy(&ua, av, 16);
  __builtin_memcpy(&ub, bv, 16);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ua), as_bf16x8(ub), acc, 0, 0, 0);
  if (col >= COUT) return;
  const float bias = a.bias ? a.bias[col] : 0.0f;
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    v[r] = acc[r] + bias;
    if (a.relu) v[r] = fmaxf(v[r], 0.0f);
  }
  const bool full = p0 + 32 <= P;  // wave-uniform: no row outside the batch
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long long q = p0 + 8 * (r >> 2) + 4 * kh + (r & 3);
    if (full || q < P) {
      if (a.out_f32) a.out_f32[q * COUT + col] = v[r];
      if (a.out_bf16) a.out_bf16[q * COUT + col] = f32_to_bf16(v[r]);
    }
  }
}

// Tiled form for Cin >= 16: a workgroup takes kConvRows image rows x 32
// pixels of one image.  The input tile with a one-pixel border (zeros
// outside the image: the "same" padding) is staged in LDS once, instead of
// every tap of every pixel being read from global memory; a pixel occupies
// Cin * 2 + 16 bytes there, so the 16-byte reads of 32 consecutive pixels hit
// distinct banks.  Each wave keeps its weight operands in registers and runs
// every fourth row of the tile.  The products are accumulated in the same
// order as in k_conv_fwd (taps, then channel chunks), so the results are
// identical.
constexpr int kConvRows = 8;

template <int CIN, int COUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_conv_fwd_tile(ffh::ConvArgs a) {
  static_assert(CIN % 16 == 0, "Cin must be a multiple of 16");
  static_assert(COUT <= 32, "Cout <= 32");
  constexpr int KC = CIN / 16, TW = 32, TR = kConvRows, LW = TW + 2;
  constexpr int PX16 = CIN / 8 + 1;  // 16-byte slots per staged pixel (one of padding)
  __shared__ uint4 s_in[(TR + 2) * LW * PX16];
  const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + TR - 1) / TR;
  const int img = blockIdx.x / (tiles_x * tiles_y), t = blockIdx.x % (tiles_x * tiles_y);
  const int x0 = (t % tiles_x) * TW, y0 = (t / tiles_x) * TR;
  const uint4 zero4 = make_uint4(0, 0, 0, 0);
  for (int k = threadIdx.x; k < (TR + 2) * LW * (CIN / 8); k += 256) {
    const int c16 = k % (CIN / 8), px = (k / (CIN / 8)) % LW, ry = k / ((CIN / 8) * LW);
    const int sx = x0 - 1 + px, sy = y0 - 1 + ry;
    uint4 v = zero4;
    if (sx >= 0 && sx < a.W && sy >= 0 && sy < a.H)
      v = reinterpret_cast<const uint4 *>(a.in + (((size_t)img * a.H + sy) * a.W + sx) * CIN)[c16];
    s_in[(ry * LW + px) * PX16 + c16] = v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 31, kh = lane >> 5, col = row;  // A: pixel x0 + row; B: output channel col
  uint4 ub[9 * KC];
  const uint32_t wmask = col < COUT ? 0xFFFFFFFFu : 0u;  // columns beyond Cout multiply by zero
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const uint4 *wsrc = reinterpret_cast<const uint4 *>(a.w + ((size_t)min(col, COUT - 1) * 9 + tap) * CIN);
#pragma unroll
    for (int cc = 0; cc < KC; ++cc) {
      const uint4 w = wsrc[cc * 2 + kh];
      ub[tap * KC + cc] = make_uint4(w.x & wmask, w.y & wmask, w.z & wmask, w.w & wmask);
    }
  }
  __syncthreads();
  const float bias = (a.bias && col < COUT) ? a.bias[col] : 0.0f;
  for (int rr = wave; rr < TR && y0 + rr < a.H; rr += 4) {
    f32x16 acc = {0};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const uint4 *src = s_in + ((rr + tap / 3) * LW + row + tap % 3) * PX16;
#pragma unroll
      for (int cc = 0; cc < KC; ++cc)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(src[cc * 2 + kh]), as_bf16x8(ub[tap * KC + cc]),
                                                      acc, 0, 0, 0);
    }
    if (col < COUT) {
      const size_t q0 = ((size_t)img * a.H + y0 + rr) * a.W;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int x = x0 + 8 * (r >> 2) + 4 * kh + (r & 3);
        float v = acc[r] + bias;
        if (a.relu) v = fmaxf(v, 0.0f);
        if (x < a.W) {
          if (a.out_f32) a.out_f32[(q0 + x) * COUT + col] = v;
          if (a.out_bf16) a.out_bf16[(q0 + x) * COUT + col] = f32_to_bf16(v);
        }
      }
    }
  }
}

// The whole network for inference in one launch (1 -> 32 -> 32 -> 16, ReLU
// after the first two layers, optionally unit length per pixel): a
// workgroup computes a tile of 60 x kNetRows output pixels; the first
// layer's outputs on the tile plus two pixels on every side and the second
// layer's plus one stay in LDS (zero outside the image, the "same" padding
// of the next layer), so the activations never leave the chip.  Every
// layer issues the matrix-core products of k_conv_fwd (first layer) and
// k_conv_fwd_tile (32 pixels of a row per product, taps then channel chunks,
// the same operands, here as the transposed product) and the same bias,
// ReLU and bf16 rounding, and the normalisation is l2norm16: the features
// are bit for bit those of the three convolution launches and the
// normalisation launch.
constexpr int kNetRows = 4, kNetTW = 60, kNetCols = 64, kNetPX = 5;  // 16-byte slots per staged pixel

__global__ __launch_bounds__(256) void k_descnet_fwd(ffh::NetArgs a) {
  constexpr int R1 = kNetRows + 4, R2 = kNetRows + 2, R0 = kNetRows + 6, C0 = kNetCols + 2;
  __shared__ uint16_t s_in[R0][C0];                    // network input, tile + 3 pixels
  __shared__ uint4 s_a1[R1 * kNetCols * kNetPX];         // first layer's outputs, tile + 2 pixels
  __shared__ uint4 s_a2[R2 * kNetCols * kNetPX];         // second layer's outputs, tile + 1 pixel
  float *s_out = reinterpret_cast<float *>(s_a1);        // third layer's outputs (after s_a1 is read)
  const int W = a.W, H = a.H;
  const int tiles_x = (W + kNetTW - 1) / kNetTW, tiles_y = (H + kNetRows - 1) / kNetRows;
  const int img = blockIdx.x / (tiles_x * tiles_y), t = blockIdx.x % (tiles_x * tiles_y);
  const int x0 = (t % tiles_x) * kNetTW, y0 = (t / tiles_x) * kNetRows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = lane & 31, kh = lane >> 5, col = row;
  const size_t plane = (size_t)img * H * W;
  auto inside = [&](int y, int x) { return y >= 0 && y < H && x >= 0 && x < W; };
  // a tile whose first-layer region lies inside the image needs no border
  // zeros (wave-uniform)
  const bool interior = y0 >= 2 && y0 + kNetRows + 2 <= H && x0 >= 2 && x0 + kNetCols - 2 <= W;
  // every weight operand first (the three layers' loads in flight together
  // with the input tile's)
  uint16_t bw1[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int tap = 8 * kh + e;
    bw1[e] = tap < 9 ? a.w1[col * 9 + tap] : (uint16_t)0;
  }
  uint4 ub2[18], ub3[18];
  const uint32_t wmask = col < 16 ? 0xFFFFFFFFu : 0u;  // third layer: columns beyond the 16 outputs multiply by zero
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      ub2[tap * 2 + cc] = reinterpret_cast<const uint4 *>(a.w2 + ((size_t)col * 9 + tap) * 32)[cc * 2 + kh];
      const uint4 w = reinterpret_cast<const uint4 *>(a.w3 + ((size_t)min(col, 15) * 9 + tap) * 32)[cc * 2 + kh];
      ub3[tap * 2 + cc] = make_uint4(w.x & wmask, w.y & wmask, w.z & wmask, w.w & wmask);
    }
  uint4 ub1;
  __builtin_memcpy(&ub1, bw1, 16);
  for (int k = tid; k < R0 * C0; k += 256) {
    const int ry = k / C0, cx = k % C0, y = y0 - 3 + ry, x = x0 - 3 + cx;
    s_in[ry][cx] = inside(y, x) ? a.in[plane + (size_t)y * W + x] : (uint16_t)0;
  }
  __syncthreads();
  // The products are taken transposed, D = W X (weights the first operand,
  // the 32 pixels the columns): a lane then holds 16 output channels of one
  // pixel, channels 8 g + 4 kh .. 8 g + 4 kh + 3 for g = 0..3, and writes
  // them with four 8-byte stores.  Every output element is the same sum of
  // the same products as in the per-layer kernels.
  // bf16 outputs of one pixel (zero outside the image: the next layer's
  // padding) into a staged map
  // the biases of a lane's 16 output channels, per layer
  auto lane_bias = [&](const float *b, int nout, float (&bl)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int co = 8 * (r >> 2) + 4 * kh + (r & 3);
      bl[r] = co < nout ? b[co] : 0.0f;
    }
  };
  auto store_bf16 = [&](uint4 *map, int ry, int c, const f32x16 &acc, const float (&bl)[16], bool in_image) {
    uint8_t *px = reinterpret_cast<uint8_t *>(&map[(ry * kNetCols + c) * kNetPX]);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      uint32_t h[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) h[q] = in_image ? f32_to_bf16(fmaxf(acc[4 * g + q] + bl[4 * g + q], 0.0f)) : 0u;
      *reinterpret_cast<uint2 *>(px + 16 * g + 8 * kh) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
  };
  // first layer: K = 9 taps padded to 16, lane half kh holds taps 8 kh .. 8 kh + 7
  float bl[16];
  lane_bias(a.b1, 32, bl);
  for (int item = wave; item < 2 * R1; item += 4) {
    const int ry = item >> 1, c = 32 * (item & 1) + row;  // this lane's pixel (y0 - 2 + ry, x0 - 2 + c)
    uint16_t av[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int tap = 8 * kh + e;
      av[e] = tap < 9 ? s_in[ry + tap / 3][c + tap % 3] : (uint16_t)0;
    }
    uint4 ua;
    __builtin_memcpy(&ua, av, 16);
    f32x16 acc = {0};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ub1), as_bf16x8(ua), acc, 0, 0, 0);
    store_bf16(s_a1, ry, c, acc, bl, interior || inside(y0 - 2 + ry, x0 - 2 + c));
  }
  __syncthreads();
  // second and third layers: 9 taps x 2 channel chunks of 16 per product, a
  // wave running two row blocks at once (independent accumulator chains)
  auto layer = [&](const uint4 *src_map, const uint4(&ub)[18], int nrows, auto &&store) {
    for (int item = 2 * wave; item < 2 * nrows; item += 8) {
      const int i2 = min(item + 1, 2 * nrows - 1);  // the pair's second block (a repeat when there is none)
      const int ra = item >> 1, ba = 32 * (item & 1), rb = i2 >> 1, bb = 32 * (i2 & 1);
      f32x16 acc0 = {0}, acc1 = {0};
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const uint4 *s0 = src_map + ((ra + tap / 3) * kNetCols + min(ba + row + tap % 3, kNetCols - 1)) * kNetPX;
        const uint4 *s1 = src_map + ((rb + tap / 3) * kNetCols + min(bb + row + tap % 3, kNetCols - 1)) * kNetPX;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ub[tap * 2 + cc]), as_bf16x8(s0[cc * 2 + kh]), acc0,
                                                         0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ub[tap * 2 + cc]), as_bf16x8(s1[cc * 2 + kh]), acc1,
                                                         0, 0, 0);
        }
      }
      store(ra, ba + row, acc0);
      if (i2 != item) store(rb, bb + row, acc1);
    }
  };
  lane_bias(a.b2, 32, bl);
  layer(s_a1, ub2, R2, [&](int ry, int c, const f32x16 &acc) {  // pixel (y0 - 1 + ry, x0 - 1 + c)
    store_bf16(s_a2, ry, c, acc, bl, interior || inside(y0 - 1 + ry, x0 - 1 + c));
  });
  lane_bias(a.b3, 16, bl);
  __syncthreads();  // s_a2 complete; s_a1 no longer read
  layer(s_a2, ub3, kNetRows, [&](int ry, int c, const f32x16 &acc) {  // pixel (y0 + ry, x0 + c): channels < 16
    float *px = s_out + (ry * kNetCols + c) * 16;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int co = 8 * g + 4 * kh;
      *reinterpret_cast<float4 *>(px + co) = make_float4(acc[4 * g] + bl[4 * g], acc[4 * g + 1] + bl[4 * g + 1],
                                                         acc[4 * g + 2] + bl[4 * g + 2], acc[4 * g + 3] + bl[4 * g + 3]);
    }
  });
  __syncthreads();
  for (int k = tid; k < kNetRows * kNetTW; k += 256) {
    const int ry = k / kNetTW, c = k % kNetTW, y = y0 + ry, x = x0 + c;
    if (!inside(y, x)) continue;
    float4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = reinterpret_cast<const float4 *>(s_out + (ry * kNetCols + c) * 16)[q];
    if (a.normalize) l2norm16(v, a.delta);
    float4 *dst = reinterpret_cast<float4 *>(a.out + (plane + (size_t)y * W + x) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = v[q];
  }
}

// W'[ci][tap][co] = W[co][8 - tap][ci]
__global__ __launch_bounds__(256) void k_flip(const uint16_t *w, uint16_t *wf, int cin, int cout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cin * 9 * cout) return;
  const int co = i % cout, tap = (i / cout) % 9, ci = i / (cout * 9);
  wf[i] = w[((size_t)co * 9 + (8 - tap)) * cin + ci];
}

// Partial weight and bias gradients of one row band on matrix cores.
// gw[co][tap][ci] = sum over pixels p of g[p][co] * x[p + d(tap)][ci] is a
// contraction over pixels: per tap, D[co][ci] (32 x 32) += A[co][16 pixels]
// x B[16 pixels][ci] with v_mfma_f32_32x32x16_bf16.  x is bf16 already; the
// float32 gradient is split as g_hi = bf16(g) and g_lo = bf16(g - g_hi) and
// both parts are multiplied (bf16 products are exact in float32, and
// |g - g_hi - g_lo| <= 2^-18 |g|), so every term keeps float32-level
// accuracy.  The bias gradient sum_p g is one more product with B = 1 (for
// Cin = 1 the nine taps and the bias are the columns of one product).  A
// workgroup takes a band of rows; of every 64 pixels of a row each wave
// takes 16.  The tile is staged in LDS channel-major (pixels of a channel
// contiguous; 16-byte loads from global memory, 8 channels or 4 gradients
// each): a lane's 8 pixels of one channel are one aligned 16-byte read, and
// the taps one pixel left or right are assembled from two neighbouring
// reads with byte alignment.  The four waves' sums are added in LDS in a
// fixed order and each workgroup writes one partial; k_wgrad_reduce adds the
// partials in a fixed order, so the result is deterministic.
constexpr int kWgPx = 64;  // pixels of a row per step (16 per wave)
constexpr int kWgX = 80;   // LDS row of image x: pixel x0 - 8 + i at entry i
constexpr int kWgG = 72;   // LDS row of the gradient: pixel x0 + i at entry i

// the 8 bf16 at entries e0 + s .. e0 + s + 7 (s = -1, 0, 1) of an LDS row,
// from the aligned reads lo = [e0 - 8, e0), mid = [e0, e0 + 8), hi = [e0 + 8,
// e0 + 16)
__device__ __forceinline__ uint4 shifted8(uint4 lo, uint4 mid, uint4 hi, int s) {
  if (s == 0) return mid;
  if (s > 0)
    return make_uint4(__builtin_amdgcn_alignbyte(mid.y, mid.x, 2), __builtin_amdgcn_alignbyte(mid.z, mid.y, 2),
                      __builtin_amdgcn_alignbyte(mid.w, mid.z, 2), __builtin_amdgcn_alignbyte(hi.x, mid.w, 2));
  return make_uint4(__builtin_amdgcn_alignbyte(mid.x, lo.w, 2), __builtin_amdgcn_alignbyte(mid.y, mid.x, 2),
                    __builtin_amdgcn_alignbyte(mid.z, mid.y, 2), __builtin_amdgcn_alignbyte(mid.w, mid.z, 2));
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad_partial(ffh::ConvArgs a, int rows_per_block) {
  static_assert((CIN == 1 || CIN == 32) && (COUT == 16 || COUT == 32), "Cin 1 or 32, Cout 16 or 32");
  constexpr int NP = CIN == 1 ? 1 : 10;  // products per pixel block: 9 taps and the bias
  __shared__ __attribute__((aligned(16))) uint16_t s_x[3][CIN][kWgX];  // [dy][ci][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t s_g[2][32][kWgG];   // [hi, lo][co][pixel]
  __shared__ float s_red[4][32 * 32];                                  // the four waves' sums of one product
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, kh = lane >> 5;
  f32x16 acc[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) acc[t] = f32x16{0};
  const uint4 ones = make_uint4(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u);  // bf16 1.0
  for (int e = tid; e < 2 * (32 - COUT) * kWgG; e += 256)  // gradient rows beyond Cout stay zero
    s_g[e / ((32 - COUT) * kWgG)][COUT + (e / kWgG) % (32 - COUT)][e % kWgG] = 0;
  const int nrows = a.B * a.H;
  const int r0 = blockIdx.x * rows_per_block, r1 = min(r0 + rows_per_block, nrows);
  for (int rr = r0; rr < r1; ++rr) {
    const int img = rr / a.H, y = rr % a.H;
    const long long row = (long long)img * a.H + y;
    for (int x0 = 0; x0 < a.W; x0 += kWgPx) {
      __syncthreads();  // the previous step's operands are read
      for (int e = tid; e < kWgPx * (COUT / 4); e += 256) {
        const int v = e % (COUT / 4), px = e / (COUT / 4), x = x0 + px;
        float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (x < a.W) q = *reinterpret_cast<const float4 *>(a.gout + (row * a.W + x) * COUT + 4 * v);
        const float g[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint16_t hi = f32_to_bf16(g[c]);
          s_g[0][4 * v + c][px] = hi;
          s_g[1][4 * v + c][px] = f32_to_bf16(g[c] - bf16_to_f32(hi));
        }
      }
      if constexpr (CIN == 32) {
        for (int e = tid; e < 3 * 66 * 4; e += 256) {
          const int v = e & 3, px = (e >> 2) % 66, dy = (e >> 2) / 66;
          const int sx = x0 + px - 1, sy = y + dy - 1;
          uint4 q = make_uint4(0u, 0u, 0u, 0u);
          if (sx >= 0 && sx < a.W && sy >= 0 && sy < a.H)
            q = *reinterpret_cast<const uint4 *>(a.in + (((long long)img * a.H + sy) * a.W + sx) * 32 + 8 * v);
          const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int c = 0; c < 8; ++c) s_x[dy][8 * v + c][px + 7] = (uint16_t)(w[c >> 1] >> (16 * (c & 1)));
        }
      } else {
        for (int e = tid; e < 3 * 66; e += 256) {
          const int px = e % 66, dy = e / 66;
          const int sx = x0 + px - 1, sy = y + dy - 1;
          uint16_t v = 0;
          if (sx >= 0 && sx < a.W && sy >= 0 && sy < a.H) v = a.in[((long long)img * a.H + sy) * a.W + sx];
          s_x[dy][0][px + 7] = v;
        }
      }
      __syncthreads();
      if (x0 + 16 * wave >= a.W) continue;  // wave-uniform: the wave's pixels are all outside the row
      const int pb = 16 * wave + 8 * kh;    // this lane's 8 pixels (the K index of the products)
      const bf16x8 ahi = as_bf16x8(*reinterpret_cast<const uint4 *>(&s_g[0][col][pb]));
      const bf16x8 alo = as_bf16x8(*reinterpret_cast<const uint4 *>(&s_g[1][col][pb]));
      if constexpr (CIN == 1) {
        // column n of B: tap n (n < 9), the bias (n = 9), nothing beyond
        uint4 bv = make_uint4(0u, 0u, 0u, 0u);
        if (col < 9) {
          const uint16_t *r = s_x[col / 3][0];
          bv = shifted8(*reinterpret_cast<const uint4 *>(r + pb), *reinterpret_cast<const uint4 *>(r + pb + 8),
                        *reinterpret_cast<const uint4 *>(r + pb + 16), col % 3 - 1);
        } else if (col == 9) {
          bv = ones;
        }
        const bf16x8 b = as_bf16x8(bv);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, b, acc[0], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, b, acc[0], 0, 0, 0);
      } else {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const uint16_t *r = s_x[dy][col];
          const uint4 lo = *reinterpret_cast<const uint4 *>(r + pb), mid = *reinterpret_cast<const uint4 *>(r + pb + 8),
                      hi = *reinterpret_cast<const uint4 *>(r + pb + 16);
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const bf16x8 b = as_bf16x8(shifted8(lo, mid, hi, dx - 1));
            const int t = 3 * dy + dx;
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, b, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, b, acc[t], 0, 0, 0);
          }
        }
        const bf16x8 b1 = as_bf16x8(ones);
        acc[9] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, b1, acc[9], 0, 0, 0);
        acc[9] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, b1, acc[9], 0, 0, 0);
      }
    }
  }
  // D[co][n]: a lane holds column n = col, rows co = 8 (r / 4) + 4 kh + r % 4.
  // The four waves' sums of each product are added in a fixed order.
  float *part = a.partial + (size_t)blockIdx.x * (COUT * 9 * CIN + COUT);
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) s_red[wave][(8 * (r >> 2) + 4 * kh + (r & 3)) * 32 + col] = acc[t][r];
    __syncthreads();
    for (int e = tid; e < 32 * 32; e += 256) {
      const int co = e >> 5, n = e & 31;
      if (co >= COUT) continue;
      const float v = ((s_red[0][e] + s_red[1][e]) + s_red[2][e]) + s_red[3][e];
      if constexpr (CIN == 1) {
        if (n < 9) part[co * 9 + n] = v;
        else if (n == 9) part[COUT * 9 + co] = v;
      } else if (t < 9) {
        part[((size_t)co * 9 + t) * CIN + n] = v;
      } else if (n == 0) {
        part[COUT * 9 * CIN + co] = v;
      }
    }
  }
}

// Sum of the per-workgroup partials: 8 lanes per output, each adding a
// contiguous eighth of the partials in order, then the eight sums in a fixed
// tree (deterministic).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *partial, int nblocks, int len, float *gw,
                                                      float *gbias, int nw) {
  const int i = blockIdx.x * 32 + (threadIdx.x >> 3), seg = threadIdx.x & 7;
  float s = 0.0f;
  if (i < len) {
    const int b0 = (int)((long long)nblocks * seg / 8), b1 = (int)((long long)nblocks * (seg + 1) / 8);
    for (int b = b0; b < b1; ++b) s += partial[(size_t)b * len + i];
  }
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  s += __shfl_xor(s, 4);
  if (seg == 0 && i < len) {
    if (i < nw) gw[i] = s;
    else if (gbias) gbias[i - nw] = s;
  }
}

// grad_pre = grad_post where the post-activation is positive, else 0; also
// the bf16 copy for the next matrix-core pass.
__global__ __launch_bounds__(256) void k_relu_bwd(const uint16_t *act, const float *g, float *gout, uint16_t *gout_bf16,
                                                  long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float v = (act == nullptr || bf16_to_f32(act[i]) > 0.0f) ? g[i] : 0.0f;
  if (gout) gout[i] = v;
  if (gout_bf16) gout_bf16[i] = f32_to_bf16(v);
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float *x, uint16_t *y, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = f32_to_bf16(x[i]);
}

// Image bytes -> network input v / 255 - 0.5 (bf16).
__global__ __launch_bounds__(256) void k_image_to_bf16(const uint8_t *img, uint16_t *out, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = f32_to_bf16((float)img[i] * (1.0f / 255.0f) - 0.5f);
}

// Adam (Kingma and Ba 2015) with bias correction; writes the bf16 copy.
__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m, float *v, int count, float lr,
                                              float b1, float b2, float eps, float c1, float c2, uint16_t *p_bf16) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (p_bf16) p_bf16[i] = f32_to_bf16(pi);
}

// Unit length per pixel of 16-channel features: y = f / sqrt(|f|^2 + delta).
__global__ __launch_bounds__(256) void k_l2norm16_fwd(const float4 *f, long long P, float delta, float4 *y,
                                                      float *inv_norm) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = f[p * 4 + k];
  const float r = l2norm16(v, delta);
#pragma unroll
  for (int k = 0; k < 4; ++k) y[p * 4 + k] = v[k];
  if (inv_norm) inv_norm[p] = r;
}

// dL/df = r * (g - y * <g, y>) with r = 1 / sqrt(|f|^2 + delta).
__global__ __launch_bounds__(256) void k_l2norm16_bwd(const float4 *y, const float *inv_norm, const float4 *g,
                                                      long long P, float4 *gin) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float4 yv[4], gv[4];
  float d = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    yv[k] = y[p * 4 + k];
    gv[k] = g[p * 4 + k];
    d += yv[k].x * gv[k].x + yv[k].y * gv[k].y + yv[k].z * gv[k].z + yv[k].w * gv[k].w;
  }
  const float r = inv_norm[p];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    gin[p * 4 + k] = make_float4(r * (gv[k].x - yv[k].x * d), r * (gv[k].y - yv[k].y * d),
                                 r * (gv[k].z - yv[k].z * d), r * (gv[k].w - yv[k].w * d));
}

// Triplet hinge of m (positive, negative) cost pairs: cost[0..m) positives,
// cost[m..2m) negatives.  Loss = weight * sum_k max(0, margin + scale *
// (cost[k] - cost[m + k])); grad[k] = +weight*scale and grad[m + k] =
// -weight*scale where the hinge is active, else 0.  One workgroup: the
// loss is summed in a fixed order (thread-strided partials, then a tree),
// so it is deterministic.
__global__ __launch_bounds__(1024) void k_triplet_hinge(const float *cost, int m, float margin, float scale,
                                                        float weight, float *grad, float *loss) {
  __shared__ float s_part[1024];
  float acc = 0.0f;
  for (int k = threadIdx.x; k < m; k += 1024) {
    const float h = margin + scale * (cost[k] - cost[m + k]);
    const bool on = h > 0.0f;
    acc += on ? h : 0.0f;
    grad[k] = on ? weight * scale : 0.0f;
    grad[m + k] = on ? -weight * scale : 0.0f;
  }
  s_part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_part[threadIdx.x] += s_part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = weight * s_part[0];
}

// Per-map range of float features (block partials, then one block).
__global__ __launch_bounds__(256) void k_minmax_partial(const float *f, long long count, float *part) {
  __shared__ float s_lo[256], s_hi[256];
  float lo = INFINITY, hi = -INFINITY;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long long)gridDim.x * 256) {
    lo = fminf(lo, f[i]);
    hi = fmaxf(hi, f[i]);
  }
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s_lo[threadIdx.x] = fminf(s_lo[threadIdx.x], s_lo[threadIdx.x + s]);
      s_hi[threadIdx.x] = fmaxf(s_hi[threadIdx.x], s_hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_lo[0];
    part[2 * blockIdx.x + 1] = s_hi[0];
  }
}

// The range over the partials (min and max are order-independent), into
// part[2 * nparts], part[2 * nparts + 1].
__global__ __launch_bounds__(256) void k_minmax_final(float *part, int nparts) {
  __shared__ float s_lo[256], s_hi[256];
  float lo = INFINITY, hi = -INFINITY;
  for (int k = threadIdx.x; k < nparts; k += 256) {  // min and max: any order gives the same result
    lo = fminf(lo, part[2 * k]);
    hi = fmaxf(hi, part[2 * k + 1]);
  }
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s_lo[threadIdx.x] = fminf(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
      s_hi[threadIdx.x] = fmaxf(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * nparts] = s_lo[0];
    part[2 * nparts + 1] = s_hi[0];
  }
}

// q = clamp(rint((f - lo) * (255 / (hi - lo))), 0, 255).
__global__ __launch_bounds__(256) void k_quantize(const float *f, long long count, const float *range, uint8_t *q) {
  const float lo = range[0], hi = range[1];
  const float s = hi > lo ? 255.0f / (hi - lo) : 0.0f;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float t = rintf((f[i] - lo) * s);
  q[i] = (uint8_t)fminf(fmaxf(t, 0.0f), 255.0f);
}

}  // namespace

namespace ffh {

static unsigned blocks_of(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_conv_fwd(const ConvArgs &a, hipStream_t stream) {
  const long long P = (long long)a.B * a.H * a.W;
  const unsigned grid = (unsigned)((P + 127) / 128);
  if (P == 0) return hipSuccess;
  const long long tiles = (long long)a.B * ((a.W + 31) / 32) * ((a.H + kConvRows - 1) / kConvRows);
  if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 tgrid((unsigned)tiles);
  if (a.cin == 1 && a.cout == 32) hipLaunchKernelGGL((k_conv_fwd<1, 32>), dim3(grid), dim3(256), 0, stream, a);
  else if (a.cin == 32 && a.cout == 32) hipLaunchKernelGGL((k_conv_fwd_tile<32, 32>), tgrid, dim3(256), 0, stream, a);
  else if (a.cin == 32 && a.cout == 16) hipLaunchKernelGGL((k_conv_fwd_tile<32, 16>), tgrid, dim3(256), 0, stream, a);
  else if (a.cin == 16 && a.cout == 32) hipLaunchKernelGGL((k_conv_fwd_tile<16, 32>), tgrid, dim3(256), 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_descnet_fwd(const NetArgs &a, hipStream_t stream) {
  const long long tiles = (long long)a.B * ((a.W + kNetTW - 1) / kNetTW) * ((a.H + kNetRows - 1) / kNetRows);
  if (tiles <= 0 || tiles > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_descnet_fwd, dim3((unsigned)tiles), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_weight_flip(const uint16_t *w, uint16_t *wf, int cin, int cout, hipStream_t stream) {
  hipLaunchKernelGGL(k_flip, dim3(blocks_of((long long)cin * 9 * cout)), dim3(256), 0, stream, w, wf, cin, cout);
  return hipGetLastError();
}

int wgrad_blocks(int B, int H) { return std::min(B * H, 1024); }

hipError_t launch_wgrad(const ConvArgs &a, float *gw, float *gbias, hipStream_t stream) {
  const int nrows = a.B * a.H, nb = wgrad_blocks(a.B, a.H);
  const int rpb = (nrows + nb - 1) / nb;
  const int used = (nrows + rpb - 1) / rpb;
  if (a.cin == 1 && a.cout == 32) hipLaunchKernelGGL((k_wgrad_partial<1, 32>), dim3(used), dim3(256), 0, stream, a, rpb);
  else if (a.cin == 32 && a.cout == 32) hipLaunchKernelGGL((k_wgrad_partial<32, 32>), dim3(used), dim3(256), 0, stream, a, rpb);
  else if (a.cin == 32 && a.cout == 16) hipLaunchKernelGGL((k_wgrad_partial<32, 16>), dim3(used), dim3(256), 0, stream, a, rpb);
  else return hipErrorInvalidValue;
  const int nw = a.cout * 9 * a.cin, len = nw + a.cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((len + 31) / 32)), dim3(256), 0, stream, a.partial, used, len, gw,
                     gbias, nw);
  return hipGetLastError();
}

hipError_t launch_relu_bwd(const uint16_t *act, const float *g, float *gout, uint16_t *gout_bf16, long long count,
                           hipStream_t stream) {
  if (count > 0)
    hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_of(count)), dim3(256), 0, stream, act, g, gout, gout_bf16, count);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, long long count, hipStream_t stream) {
  if (count > 0) hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks_of(count)), dim3(256), 0, stream, x, y, count);
  return hipGetLastError();
}

hipError_t launch_image_to_bf16(const uint8_t *img, uint16_t *out, long long count, hipStream_t stream) {
  if (count > 0) hipLaunchKernelGGL(k_image_to_bf16, dim3(blocks_of(count)), dim3(256), 0, stream, img, out, count);
  return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int count, float lr, float b1, float b2,
                       float eps, int step, uint16_t *p_bf16, hipStream_t stream) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  if (count > 0)
    hipLaunchKernelGGL(k_adam, dim3(blocks_of(count)), dim3(256), 0, stream, p, g, m, v, count, lr, b1, b2, eps, c1,
                       c2, p_bf16);
  return hipGetLastError();
}

hipError_t launch_l2norm16_fwd(const float *f, long long P, float delta, float *y, float *inv_norm,
                               hipStream_t stream) {
  if (P > 0)
    hipLaunchKernelGGL(k_l2norm16_fwd, dim3(blocks_of(P)), dim3(256), 0, stream, reinterpret_cast<const float4 *>(f),
                       P, delta, reinterpret_cast<float4 *>(y), inv_norm);
  return hipGetLastError();
}

hipError_t launch_l2norm16_bwd(const float *y, const float *inv_norm, const float *g, long long P, float *gin,
                               hipStream_t stream) {
  if (P > 0)
    hipLaunchKernelGGL(k_l2norm16_bwd, dim3(blocks_of(P)), dim3(256), 0, stream, reinterpret_cast<const float4 *>(y),
                       inv_norm, reinterpret_cast<const float4 *>(g), P, reinterpret_cast<float4 *>(gin));
  return hipGetLastError();
}

hipError_t launch_triplet_hinge(const float *cost, int m, float margin, float scale, float weight, float *grad,
                                float *loss, hipStream_t stream) {
  hipLaunchKernelGGL(k_triplet_hinge, dim3(1), dim3(1024), 0, stream, cost, m, margin, scale, weight, grad, loss);
  return hipGetLastError();
}

constexpr int kQuantParts = 1024;

hipError_t launch_quantize(const float *f, long long count, float *part, uint8_t *q, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_minmax_partial, dim3(kQuantParts), dim3(256), 0, stream, f, count, part);
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, stream, part, kQuantParts);
  hipLaunchKernelGGL(k_quantize, dim3(blocks_of(count)), dim3(256), 0, stream, f, count, part + 2 * kQuantParts, q);
  return hipGetLastError();
}

// Two maps with the range of their union: partials of map 1, then of map 2,
// one final reduction over both, both quantised with that range.
hipError_t launch_quantize_pair(const float *f1, const float *f2, long long count, float *part, uint8_t *q1,
                                uint8_t *q2, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_minmax_partial, dim3(kQuantParts), dim3(256), 0, stream, f1, count, part);
  hipLaunchKernelGGL(k_minmax_partial, dim3(kQuantParts), dim3(256), 0, stream, f2, count, part + 2 * kQuantParts);
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, stream, part, 2 * kQuantParts);
  const float *range = part + 4 * kQuantParts;
  hipLaunchKernelGGL(k_quantize, dim3(blocks_of(count)), dim3(256), 0, stream, f1, count, range, q1);
  hipLaunchKernelGGL(k_quantize, dim3(blocks_of(count)), dim3(256), 0, stream, f2, count, range, q2);
  return hipGetLastError();
}

size_t quantize_scratch_bytes() { return (size_t)(2 * kQuantParts + 1) * 2 * sizeof(float); }

}  // namespace ffh
