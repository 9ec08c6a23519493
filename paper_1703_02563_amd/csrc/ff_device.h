// Device-side helpers of the Flow Fields kernels (gfx950).
//
// Patch cost E_n of Eq. 3 on 16-byte descriptors: each patch position adds
// the byte-wise SAD of two descriptors, four bytes per v_sad_u8.  Descriptor
// rows are stored in phase order (desc_col).  Reads
// outside the image take the nearest inside pixel (Sec. 3.6 border
// condition).  The counter-based generator of the random search is
// SplitMix64's output mixer (Steele, Lea, Flood 2014) applied as
// mix(seed ^ mix(counter)), mapped to [0, 2R] by Lemire's multiply-shift.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffk {

constexpr uint32_t kUnset = 0xFFFFFFFFu;

__device__ __forceinline__ int clampi(int v, int hi) { return min(max(v, 0), hi); }

__device__ __forceinline__ uint32_t sad16(const uint4 a, const uint4 b, uint32_t acc) {
  acc = __builtin_amdgcn_sad_u8(a.x, b.x, acc);
  acc = __builtin_amdgcn_sad_u8(a.y, b.y, acc);
  acc = __builtin_amdgcn_sad_u8(a.z, b.z, acc);
  acc = __builtin_amdgcn_sad_u8(a.w, b.w, acc);
  return acc;
}

// Scale-n descriptor maps keep their rows in image order, but the pixels of
// a row are grouped by phase x mod n: pixel x sits at column
// (x mod n) * floor(W / n) + min(x mod n, W mod n) + floor(x / n).  The
// samples x + n*u of a patch row then occupy consecutive columns, as do the
// patch rows of neighbouring grid cells.  For n = 1 this is the identity.
__device__ __forceinline__ int desc_col(int x, int log2n, int W) {
  const int r = x & ((1 << log2n) - 1);
  return r * (W >> log2n) + min(r, W & ((1 << log2n) - 1)) + (x >> log2n);
}

// Scale-n descriptor maps also carry a border of kDescPad * n replicated
// pixels on every side: the map holds D(clamp(x), clamp(y)) for x in
// [-P, W + P), y in [-P, H + P), P = kDescPad * n, rows of width W + 2P in
// phase order.  A patch of radius up to 4 around any in-image target then
// reads the map without clamping.  P is a multiple of n, so phases are unchanged.
constexpr int kDescPad = 4;

__host__ __device__ __forceinline__ int desc_pad(int n) { return kDescPad * n; }

// Layout exponent of the map of scale n: log2 n for a power of two; 0 (the
// pixels of a row in image order) for a sub-scale that is not one.
__host__ __device__ __forceinline__ int map_log2(int n) {
  int l = 0;
  if ((n & (n - 1)) == 0)
    while ((1 << l) < n) ++l;
  return l;
}

// Inverse of desc_col: the pixel stored at column c.
__device__ __forceinline__ int desc_pixel(int c, int log2n, int W) {
  const int q = W >> log2n, m = W & ((1 << log2n) - 1);
  if (c < (q + 1) * m) return c / (q + 1) + ((c % (q + 1)) << log2n);
  const int c2 = c - (q + 1) * m;
  return m + c2 / q + ((c2 % q) << log2n);
}

// Index of pixel (x, y), x in [-P, W + P), y in [-P, H + P), in a padded
// scale-2^log2n descriptor map of a W-wide image.
__device__ __forceinline__ size_t desc_index(int x, int y, int log2n, int W) {
  const int P = kDescPad << log2n, Wp = W + 2 * P;
  return (size_t)(y + P) * Wp + desc_col(x + P, log2n, Wp);
}

// Weight-class row map of a scale-n blurred image I^n: one 16-byte entry per
// pixel (x, y) for y in [-3n, H + 3n) (rows clamped), entry index
// (y + 3n) * W + x.  The entry holds the 13 samples I^n(clamp(x + n a), y),
// a = -6..6, grouped by the multiplicity w(a) = 1,1,2,2,3,3,4,3,3,2,2,1,1 with
// which a sample enters the subsampled patch cost: dword 0 the samples of
// weight 1 (a = -6, -5, 5, 6), dword 1 weight 2 (a = -4, -3, 3, 4), dword 2
// weight 3 (a = -2, -1, 1, 2), dword 3 weight 4 (a = 0, then three zero
// bytes).  For a pixel p and a target q both at least 3n inside the image,
// E_n(p, q - p) = sum over row offsets b = -6..6 of w(b) * (1 s1 + 2 s2 +
// 3 s3 + 4 s4), s_k = the byte SAD of dword k of the entries of rows
// y + n b of the two maps (each descriptor byte is one blurred sample, so the
// 784 byte differences of Eq. 3 are the 169 samples counted w(a) w(b) times).
constexpr int kWformPad = 3;
__host__ __device__ __forceinline__ size_t wform_index(int x, int y, int n, int W) {
  return (size_t)(y + kWformPad * n) * W + x;
}
__host__ __device__ __forceinline__ size_t wform_bytes(int W, int H, int n) {
  return (size_t)W * (H + 2 * kWformPad * n) * 16;
}

__device__ __forceinline__ int flow_x(int32_t f) { return (int)(int16_t)(f & 0xFFFF); }
__device__ __forceinline__ int flow_y(int32_t f) { return f >> 16; }
__device__ __forceinline__ int32_t pack_flow(int fx, int fy) {
  return (int32_t)(((uint32_t)fy << 16) | ((uint32_t)fx & 0xFFFFu));
}

// E_n(p, f) for one candidate flow.
template <int R>
__device__ __forceinline__ uint32_t patch_cost(const uint4 *__restrict__ Da, const uint4 *__restrict__ Db,
                                               int W, int H, int n, int x, int y, int fx, int fy) {
  const int Wm = W - 1, Hm = H - 1, l2 = map_log2(n), P = desc_pad(n), Wp = W + 2 * P;
  uint32_t s = 0;
#pragma unroll 1
  for (int v = -R; v <= R; ++v) {
    const uint4 *ra = Da + (size_t)(clampi(y + n * v, Hm) + P) * Wp;
    const uint4 *rb = Db + (size_t)(clampi(y + fy + n * v, Hm) + P) * Wp;
#pragma unroll
    for (int u = -R; u <= R; ++u) {
      const uint4 a = ra[desc_col(clampi(x + n * u, Wm) + P, l2, Wp)];
      const uint4 b = rb[desc_col(clampi(x + fx + n * u, Wm) + P, l2, Wp)];
      s = sad16(a, b, s);
    }
  }
  return s;
}

// E_n(p, f1) and E_n(p, f2) sharing the reads of image a; a disabled
// candidate is neither read nor summed.
template <int R>
__device__ __forceinline__ void patch_cost2(const uint4 *__restrict__ Da, const uint4 *__restrict__ Db, int W,
                                            int H, int n, int x, int y, int f1x, int f1y, bool en1, int f2x,
                                            int f2y, bool en2, uint32_t &c1, uint32_t &c2) {
  const int Wm = W - 1, Hm = H - 1, l2 = map_log2(n), P = desc_pad(n), Wp = W + 2 * P;
  uint32_t s1 = 0, s2 = 0;
#pragma unroll 1
  for (int v = -R; v <= R; ++v) {
    const uint4 *ra = Da + (size_t)(clampi(y + n * v, Hm) + P) * Wp;
    const uint4 *rb1 = Db + (size_t)(clampi(y + f1y + n * v, Hm) + P) * Wp;
    const uint4 *rb2 = Db + (size_t)(clampi(y + f2y + n * v, Hm) + P) * Wp;
#pragma unroll
    for (int u = -R; u <= R; ++u) {
      const uint4 a = ra[desc_col(clampi(x + n * u, Wm) + P, l2, Wp)];
      if (en1) s1 = sad16(a, rb1[desc_col(clampi(x + f1x + n * u, Wm) + P, l2, Wp)], s1);
      if (en2) s2 = sad16(a, rb2[desc_col(clampi(x + f2x + n * u, Wm) + P, l2, Wp)], s2);
    }
  }
  c1 = s1;
  c2 = s2;
}

// Matching-error policies of the per-step kernels.  Both return a 32-bit
// key: the integer SAD of 16-byte descriptors, or the bit pattern of the
// non-negative float32 sum of squared differences of 16-channel float
// features, which orders exactly like the float values.  The float sum is
// four partial sums, one per group of channels 4k .. 4k+3, each with one
// fused multiply-add per term in the order v, u, c, added as
// (s0 + s1) + (s2 + s3).
struct CostU8 {
  static constexpr int kSub = 0;  // flows in whole pixels
  template <int R>
  __device__ static uint32_t eval(const void *Da, const void *Db, int W, int H, int n, int x, int y, int fx,
                                  int fy) {
    return patch_cost<R>(static_cast<const uint4 *>(Da), static_cast<const uint4 *>(Db), W, H, n, x, y, fx, fy);
  }
  template <int R>
  __device__ static void eval2(const void *Da, const void *Db, int W, int H, int n, int x, int y, int f1x, int f1y,
                               bool en1, int f2x, int f2y, bool en2, uint32_t &c1, uint32_t &c2) {
    patch_cost2<R>(static_cast<const uint4 *>(Da), static_cast<const uint4 *>(Db), W, H, n, x, y, f1x, f1y, en1, f2x,
                   f2y, en2, c1, c2);
  }
  // The terms of patch positions k = g, g + G, ... (k = (v + R)(2R + 1) +
  // u + R) for lane g of G: integers, so the G parts of one evaluation add
  // up to eval's value in any order.
  template <int R, int G>
  __device__ static uint32_t eval_part(const void *Dav, const void *Dbv, int W, int H, int n, int x, int y, int fx,
                                       int fy, int g) {
    const uint4 *Da = static_cast<const uint4 *>(Dav), *Db = static_cast<const uint4 *>(Dbv);
    const int Wm = W - 1, Hm = H - 1, l2 = map_log2(n), P = desc_pad(n), Wp = W + 2 * P;
    constexpr int D = 2 * R + 1;
    uint32_t s = 0;
    // unrolled: all of the lane's loads are in flight together
#pragma unroll
    for (int it = 0; it < (D * D + G - 1) / G; ++it) {
      const int k = g + it * G;
      if (k >= D * D) break;
      const int v = k / D - R, u = k % D - R;
      const uint4 a = Da[(size_t)(clampi(y + n * v, Hm) + P) * Wp + desc_col(clampi(x + n * u, Wm) + P, l2, Wp)];
      const uint4 b =
          Db[(size_t)(clampi(y + fy + n * v, Hm) + P) * Wp + desc_col(clampi(x + fx + n * u, Wm) + P, l2, Wp)];
      s = sad16(a, b, s);
    }
    return s;
  }
};

struct CostF32 {
  static constexpr int kSub = 0;
  template <int R>
  __device__ static uint32_t eval(const void *Da, const void *Db, int W, int H, int n, int x, int y, int fx,
                                  int fy) {
    const float4 *fa = static_cast<const float4 *>(Da), *fb = static_cast<const float4 *>(Db);
    const int Wm = W - 1, Hm = H - 1;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // channels 4k .. 4k+3
#pragma unroll 1
    for (int v = -R; v <= R; ++v) {
      const size_t ra = (size_t)clampi(y + n * v, Hm) * W, rb = (size_t)clampi(y + fy + n * v, Hm) * W;
#pragma unroll
      for (int u = -R; u <= R; ++u) {
        const float4 *a = fa + (ra + clampi(x + n * u, Wm)) * 4;
        const float4 *b = fb + (rb + clampi(x + fx + n * u, Wm)) * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float4 p = a[k], q = b[k];
          float d = p.x - q.x;
          acc[k] = __fmaf_rn(d, d, acc[k]);
          d = p.y - q.y;
          acc[k] = __fmaf_rn(d, d, acc[k]);
          d = p.z - q.z;
          acc[k] = __fmaf_rn(d, d, acc[k]);
          d = p.w - q.w;
          acc[k] = __fmaf_rn(d, d, acc[k]);
        }
      }
    }
    return __float_as_uint((acc[0] + acc[1]) + (acc[2] + acc[3]));
  }
  template <int R>
  __device__ static void eval2(const void *Da, const void *Db, int W, int H, int n, int x, int y, int f1x, int f1y,
                               bool en1, int f2x, int f2y, bool en2, uint32_t &c1, uint32_t &c2) {
    c1 = en1 ? eval<R>(Da, Db, W, H, n, x, y, f1x, f1y) : 0u;
    c2 = en2 ? eval<R>(Da, Db, W, H, n, x, y, f2x, f2y) : 0u;
  }
};

// Four channels of the subpixel cost: |64 a - sum_k w_k b_k| per byte,
// summed into acc.  The bytes go to 16-bit lanes (even and odd bytes); a
// weighted sum of four bytes with weights summing to 64 stays below 2^14 in
// its lane, so the lanes of one 32-bit multiply-add never carry into each
// other, and v_sad_u16 adds both lanes' absolute differences.
__device__ __forceinline__ uint32_t sad_bilinear4(uint32_t a, uint32_t b00, uint32_t b10, uint32_t b01, uint32_t b11,
                                                  uint32_t w00, uint32_t w10, uint32_t w01, uint32_t w11,
                                                  uint32_t acc) {
  constexpr uint32_t m = 0x00FF00FFu;
  const uint32_t ae = (a & m) << 6, ao = ((a >> 8) & m) << 6;
  const uint32_t me = (b00 & m) * w00 + (b10 & m) * w10 + (b01 & m) * w01 + (b11 & m) * w11;
  const uint32_t mo = ((b00 >> 8) & m) * w00 + ((b10 >> 8) & m) * w10 + ((b01 >> 8) & m) * w01 +
                      ((b11 >> 8) & m) * w11;
  acc = __builtin_amdgcn_sad_u16(ae, me, acc);
  return __builtin_amdgcn_sad_u16(ao, mo, acc);
}

// Subpixel matching error (random-search offsets with subpixel accuracy,
// the target patch's colours by bilinear interpolation): flows in 1/8
// pixel; the target t = p + f / 8 lies between pixels (tx0, ty0) and
// (tx0 + 1, ty0 + 1) with fractions ax, ay; image b's descriptors at every
// patch position t + n(u, v) are the bilinear mix of the four pixels'
// descriptors (each read through the border) with weights (8 - ax)(8 - ay),
// ax (8 - ay), (8 - ax) ay, ax ay; E = sum |64 a - mix| over patch positions
// and channels (Eq. 3 times 64, exact).  A corner of weight 0 is read at
// the other corner's column or row (its value does not matter).
struct CostU8Sub {
  static constexpr int kSub = 3;
  template <int R>
  __device__ static uint32_t eval(const void *Dav, const void *Dbv, int W, int H, int n, int x, int y, int fx,
                                  int fy) {
    const uint4 *Da = static_cast<const uint4 *>(Dav), *Db = static_cast<const uint4 *>(Dbv);
    const int tx = x * 8 + fx, ty = y * 8 + fy;  // inside the image: non-negative
    const int tx0 = tx >> 3, ty0 = ty >> 3, ax = tx & 7, ay = ty & 7;
    const int tx1 = tx0 + (ax != 0), ty1 = ty0 + (ay != 0);
    const uint32_t w00 = (8 - ax) * (8 - ay), w10 = ax * (8 - ay), w01 = (8 - ax) * ay, w11 = ax * ay;
    const int Wm = W - 1, Hm = H - 1, l2 = map_log2(n), P = desc_pad(n), Wp = W + 2 * P;
    uint32_t sum = 0;
#pragma unroll 1
    for (int v = -R; v <= R; ++v) {
      const uint4 *ra = Da + (size_t)(clampi(y + n * v, Hm) + P) * Wp;
      const uint4 *r0 = Db + (size_t)(clampi(ty0 + n * v, Hm) + P) * Wp;
      const uint4 *r1 = Db + (size_t)(clampi(ty1 + n * v, Hm) + P) * Wp;
#pragma unroll 1
      for (int u = -R; u <= R; ++u) {
        const uint4 a = ra[desc_col(clampi(x + n * u, Wm) + P, l2, Wp)];
        const int c0 = desc_col(clampi(tx0 + n * u, Wm) + P, l2, Wp), c1 = desc_col(clampi(tx1 + n * u, Wm) + P, l2, Wp);
        const uint4 b00 = r0[c0], b10 = r0[c1], b01 = r1[c0], b11 = r1[c1];
        sum = sad_bilinear4(a.x, b00.x, b10.x, b01.x, b11.x, w00, w10, w01, w11, sum);
        sum = sad_bilinear4(a.y, b00.y, b10.y, b01.y, b11.y, w00, w10, w01, w11, sum);
        sum = sad_bilinear4(a.z, b00.z, b10.z, b01.z, b11.z, w00, w10, w01, w11, sum);
        sum = sad_bilinear4(a.w, b00.w, b10.w, b01.w, b11.w, w00, w10, w01, w11, sum);
      }
    }
    return sum;
  }
  template <int R>
  __device__ static void eval2(const void *Da, const void *Db, int W, int H, int n, int x, int y, int f1x, int f1y,
                               bool en1, int f2x, int f2y, bool en2, uint32_t &c1, uint32_t &c2) {
    c1 = en1 ? eval<R>(Da, Db, W, H, n, x, y, f1x, f1y) : 0u;
    c2 = en2 ? eval<R>(Da, Db, W, H, n, x, y, f2x, f2y) : 0u;
  }
  // The terms of patch positions k = g, g + G, ... (see CostU8::eval_part).
  template <int R, int G>
  __device__ static uint32_t eval_part(const void *Dav, const void *Dbv, int W, int H, int n, int x, int y, int fx,
                                       int fy, int g) {
    const uint4 *Da = static_cast<const uint4 *>(Dav), *Db = static_cast<const uint4 *>(Dbv);
    const int tx = x * 8 + fx, ty = y * 8 + fy;
    const int tx0 = tx >> 3, ty0 = ty >> 3, ax = tx & 7, ay = ty & 7;
    const int tx1 = tx0 + (ax != 0), ty1 = ty0 + (ay != 0);
    const uint32_t w00 = (8 - ax) * (8 - ay), w10 = ax * (8 - ay), w01 = (8 - ax) * ay, w11 = ax * ay;
    const int Wm = W - 1, Hm = H - 1, l2 = map_log2(n), P = desc_pad(n), Wp = W + 2 * P;
    constexpr int D = 2 * R + 1;
    uint32_t sum = 0;
#pragma unroll
    for (int it = 0; it < (D * D + G - 1) / G; ++it) {
      const int k = g + it * G;
      if (k >= D * D) break;
      const int v = k / D - R, u = k % D - R;
      const uint4 a = Da[(size_t)(clampi(y + n * v, Hm) + P) * Wp + desc_col(clampi(x + n * u, Wm) + P, l2, Wp)];
      const uint4 *r0 = Db + (size_t)(clampi(ty0 + n * v, Hm) + P) * Wp;
      const uint4 *r1 = Db + (size_t)(clampi(ty1 + n * v, Hm) + P) * Wp;
      const int c0 = desc_col(clampi(tx0 + n * u, Wm) + P, l2, Wp), c1 = desc_col(clampi(tx1 + n * u, Wm) + P, l2, Wp);
      const uint4 b00 = r0[c0], b10 = r0[c1], b01 = r1[c0], b11 = r1[c1];
      sum = sad_bilinear4(a.x, b00.x, b10.x, b01.x, b11.x, w00, w10, w01, w11, sum);
      sum = sad_bilinear4(a.y, b00.y, b10.y, b01.y, b11.y, w00, w10, w01, w11, sum);
      sum = sad_bilinear4(a.z, b00.z, b10.z, b01.z, b11.z, w00, w10, w01, w11, sum);
      sum = sad_bilinear4(a.w, b00.w, b10.w, b01.w, b11.w, w00, w10, w01, w11, sum);
    }
    return sum;
  }
};

// Target p + f / 2^SB of a flow (in units of 1/2^SB pixel) inside the image.
template <int SB>
__device__ __forceinline__ bool target_in(int W, int H, int x, int y, int fx, int fy) {
  const int tx = x * (1 << SB) + fx, ty = y * (1 << SB) + fy;
  return tx >= 0 && tx <= (W - 1) * (1 << SB) && ty >= 0 && ty <= (H - 1) * (1 << SB);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Random-search offset of cell (i, j): uniform on [-Rn, Rn]^2.
__device__ __forceinline__ void rs_offset(uint64_t seed, int stream_id, int level, int pass, int j, int i,
                                          int Rn, int &ox, int &oy) {
  const uint64_t ctr = ((uint64_t)(stream_id & 0xFF) << 56) | ((uint64_t)(level & 0xFF) << 48) |
                       ((uint64_t)(pass & 0xFFFF) << 32) | ((uint64_t)(j & 0xFFFF) << 16) |
                       (uint64_t)(i & 0xFFFF);
  const uint64_t h = mix64(seed ^ mix64(ctr));
  const uint32_t span = (uint32_t)(2 * Rn + 1);
  ox = (int)__umulhi((uint32_t)h, span) - Rn;
  oy = (int)__umulhi((uint32_t)(h >> 32), span) - Rn;
}

// Workgroups of a launch are dealt to the 8 XCDs round-robin (workgroup b
// runs on XCD b % 8), and every XCD has its own L2.  This bijection of
// [0, nwg) gives each XCD one contiguous range of logical work items, so
// neighbouring tiles (which read neighbouring descriptors) share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
  constexpr int kXcd = 8;
  const int q = nwg / kXcd, r = nwg % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Pair owning `item` in a batch stage: the largest p with prefix[p] <= item.
__device__ __forceinline__ int batch_pair(const int *prefix, int npairs, int item) {
  int lo = 0, hi = npairs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Persistent launch over `total` work items: XCD x (workgroups b with
// b % 8 == x) owns one contiguous range of items and its workgroups stride
// through it.  The grid size must be a positive multiple of 8.
template <typename F>
__device__ __forceinline__ void for_items(int total, F &&f) {
  constexpr int kXcd = 8;
  const int G = gridDim.x, b = blockIdx.x, x = b % kXcd, k = b / kXcd;
  const int gx = G / kXcd;
  const int q = total / kXcd, r = total % kXcd;
  const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  const int cnt = q + (x < r ? 1 : 0);
  for (int it = k; it < cnt; it += gx) f(start + it);
}

// Adds a per-lane count (0, 1 or 2) of the whole wave to a global counter
// with one atomic per wave.
__device__ __forceinline__ void wave_count_add(unsigned long long *counter, int cnt) {
  if (counter == nullptr) return;
  const unsigned long long b1 = __ballot(cnt >= 1);
  const unsigned long long b2 = __ballot(cnt >= 2);
  const int total = __popcll(b1) + __popcll(b2);
  if ((threadIdx.x & 63) == 0 && total) atomicAdd(counter, (unsigned long long)total);
}

// Adds a per-lane count of the whole wave to both entries of a [2] counter
// pair (nullable), one atomic per entry and wave.
__device__ __forceinline__ void wave_count_add2(unsigned long long *counter2, int cnt) {
  if (counter2 == nullptr) return;
  const unsigned long long b1 = __ballot(cnt >= 1);
  const unsigned long long b2 = __ballot(cnt >= 2);
  const int total = __popcll(b1) + __popcll(b2);
  if ((threadIdx.x & 63) == 0 && total) {
    atomicAdd(counter2, (unsigned long long)total);
    atomicAdd(counter2 + 1, (unsigned long long)total);
  }
}

// Adds a per-lane count of any size of the whole wave to a global counter
// (nullable) with one atomic per wave.
__device__ __forceinline__ void wave_sum_add(unsigned long long *counter, int cnt) {
  if (counter == nullptr) return;
  int v = cnt;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(counter, (unsigned long long)v);
}

// The same for both entries of a [2] counter pair (nullable).
__device__ __forceinline__ void wave_sum_add2(unsigned long long *counter2, int cnt) {
  if (counter2 == nullptr) return;
  int v = cnt;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0 && v) {
    atomicAdd(counter2, (unsigned long long)v);
    atomicAdd(counter2 + 1, (unsigned long long)v);
  }
}

}  // namespace ffk
