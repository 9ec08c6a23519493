// Float patch cost of learned 16-channel features and its gradient.
//
// Cost of entry (x, y, fx, fy) at scale n, patch radius r (Eq. 3 with a
// squared-difference data term for learned features, Sec. 3.5; replicate
// border of Sec. 3.6):
//   C = sum_{v=-r..r} sum_{u=-r..r} sum_{c<16} (f1(clamp(p+n(u,v)))[c] - f2(clamp(p+f+n(u,v)))[c])^2
// accumulated in float32 as four partial sums, one per group of channels
// 4k .. 4k+3, each with one fused multiply-add per term in the order v, u, c,
// then added as (s0 + s1) + (s2 + s3) (fixed, so that every caller sees the
// same rounding).
//
// Backward: dL/df1[q] += 2g(f1(q) - f2(t)), dL/df2[t] -= 2g(f1(q) - f2(t))
// per patch position.  Many entries touch the same pixels, and float
// atomics would make the sums depend on arrival order; each contribution is
// therefore rounded once to 64-bit fixed point (2^-32 units) and added with
// integer atomics, which are associative: the result is deterministic.  A
// term of magnitude 2^31 or more, or a sum that leaves the int64 range,
// would wrap: both are detected (the atomic returns the previous value, so
// the adding thread sees a signed overflow) and counted in an overflow word
// after the accumulators; a nonzero count turns every gradient output into
// NaN instead of a wrapped value.
#include "ff_device.h"
#include "ff_internal.h"

namespace {

using ffk::clampi;

constexpr double kFix = 4294967296.0;  // 2^32

template <int R>
__global__ __launch_bounds__(256) void k_cost_fwd(ffh::CostArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.count) return;
  const int4 en = a.entries[e];
  const int n = a.n, Wm = a.W - 1, Hm = a.H - 1;
  const float4 *f1 = reinterpret_cast<const float4 *>(a.f1);
  const float4 *f2 = reinterpret_cast<const float4 *>(a.f2);
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int v = -R; v <= R; ++v) {
    const size_t qrow = (size_t)clampi(en.y + n * v, Hm) * a.W;
    const size_t trow = (size_t)clampi(en.y + en.w + n * v, Hm) * a.W;
#pragma unroll
    for (int u = -R; u <= R; ++u) {
      const float4 *pa = f1 + (qrow + clampi(en.x + n * u, Wm)) * 4;
      const float4 *pb = f2 + (trow + clampi(en.x + en.z + n * u, Wm)) * 4;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 x = pa[k], y = pb[k];
        float d = x.x - y.x;
        acc[k] = __fmaf_rn(d, d, acc[k]);
        d = x.y - y.y;
        acc[k] = __fmaf_rn(d, d, acc[k]);
        d = x.z - y.z;
        acc[k] = __fmaf_rn(d, d, acc[k]);
        d = x.w - y.w;
        acc[k] = __fmaf_rn(d, d, acc[k]);
      }
    }
  }
  a.cost[e] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// One thread per (entry, patch position).
__global__ __launch_bounds__(256) void k_cost_bwd(ffh::CostArgs a) {
  const int side = 2 * a.radius + 1, P = side * side;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)a.count * P) return;
  const int e = (int)(gid / P), k = (int)(gid % P);
  const int v = k / side - a.radius, u = k % side - a.radius;
  const int4 en = a.entries[e];
  const double g2 = 2.0 * (double)a.grad_cost[e];
  if (g2 == 0.0) return;
  unsigned long long *over = reinterpret_cast<unsigned long long *>(a.overflow);
  const int Wm = a.W - 1, Hm = a.H - 1, n = a.n;
  const size_t q = (size_t)clampi(en.y + n * v, Hm) * a.W + clampi(en.x + n * u, Wm);
  const size_t t = (size_t)clampi(en.y + en.w + n * v, Hm) * a.W + clampi(en.x + en.z + n * u, Wm);
  const float *pa = a.f1 + q * 16, *pb = a.f2 + t * 16;
  unsigned long long *acc1 = reinterpret_cast<unsigned long long *>(a.acc1) + q * 16;
  unsigned long long *acc2 = reinterpret_cast<unsigned long long *>(a.acc2) + t * 16;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const double d = g2 * ((double)pa[c] - (double)pb[c]);
    if (!(fabs(d) < 2147483648.0)) {  // |term| >= 2^31 (or NaN): no int64 fixed-point value
      atomicAdd(over, 1ull);
      continue;
    }
    const long long fx = __double2ll_rn(d * kFix);
    if (fx != 0) {
      // signed overflow of old + x: both operands of one sign, the sum of the other
      const long long o1 = (long long)atomicAdd(acc1 + c, (unsigned long long)fx);
      const long long o2 = (long long)atomicAdd(acc2 + c, (unsigned long long)(-fx));
      const long long n1 = (long long)((unsigned long long)o1 + (unsigned long long)fx);
      const long long n2 = (long long)((unsigned long long)o2 - (unsigned long long)fx);
      if ((((o1 ^ n1) & (fx ^ n1)) | ((o2 ^ n2) & (-fx ^ n2))) < 0) atomicAdd(over, 1ull);
    }
  }
}

__global__ __launch_bounds__(256) void k_fixed_to_float(const int64_t *acc, const int64_t *overflow, float *out,
                                                        long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = *overflow ? __builtin_nanf("") : (float)((double)acc[i] * (1.0 / kFix));
}

// Padded, phase-ordered copy of a float feature map (the layout of the
// descriptor maps with 64-byte entries): one thread per 16-byte quarter of a
// stored entry, so consecutive lanes store consecutive bytes.
__global__ __launch_bounds__(256) void k_pad_features(const float4 *f, int W, int H, int log2n, float4 *out) {
  const int P = ffk::desc_pad(1 << log2n), Wp = W + 2 * P, Hp = H + 2 * P;
  const int q = blockIdx.x * blockDim.x + threadIdx.x, yp = blockIdx.y;
  const int c = q >> 2;
  if (c >= Wp || yp >= Hp) return;
  const int x = clampi(ffk::desc_pixel(c, log2n, Wp) - P, W - 1), y = clampi(yp - P, H - 1);
  out[((size_t)yp * Wp + c) * 4 + (q & 3)] = f[((size_t)y * W + x) * 4 + (q & 3)];
}

}  // namespace

namespace ffh {

hipError_t launch_pad_features(const float *f, int W, int H, int n, float *out, hipStream_t stream) {
  const int P = ffk::desc_pad(n);
  const dim3 grid((4 * (W + 2 * P) + 255) / 256, H + 2 * P);
  hipLaunchKernelGGL(k_pad_features, grid, dim3(256), 0, stream, reinterpret_cast<const float4 *>(f), W, H,
                     __builtin_ctz(n), reinterpret_cast<float4 *>(out));
  return hipGetLastError();
}

hipError_t launch_cost_fwd(const CostArgs &a, hipStream_t stream) {
  if (a.count <= 0) return hipSuccess;
  const dim3 grid((a.count + 255) / 256);
  switch (a.radius) {
    case 0: hipLaunchKernelGGL(k_cost_fwd<0>, grid, dim3(256), 0, stream, a); break;
    case 1: hipLaunchKernelGGL(k_cost_fwd<1>, grid, dim3(256), 0, stream, a); break;
    case 2: hipLaunchKernelGGL(k_cost_fwd<2>, grid, dim3(256), 0, stream, a); break;
    case 3: hipLaunchKernelGGL(k_cost_fwd<3>, grid, dim3(256), 0, stream, a); break;
    case 4: hipLaunchKernelGGL(k_cost_fwd<4>, grid, dim3(256), 0, stream, a); break;
    case 5: hipLaunchKernelGGL(k_cost_fwd<5>, grid, dim3(256), 0, stream, a); break;
    case 6: hipLaunchKernelGGL(k_cost_fwd<6>, grid, dim3(256), 0, stream, a); break;
    case 7: hipLaunchKernelGGL(k_cost_fwd<7>, grid, dim3(256), 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cost_bwd(const CostArgs &a, hipStream_t stream) {
  const long long px = (long long)a.W * a.H * 16;
  // acc1, acc2 and the overflow word after them are one array
  hipError_t e = launch_fill_u64(reinterpret_cast<uint64_t *>(a.acc1), 0, 2 * px + 1, stream);
  if (e != hipSuccess) return e;
  const int side = 2 * a.radius + 1;
  const long long work = (long long)a.count * side * side;
  if (work > 0)
    hipLaunchKernelGGL(k_cost_bwd, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, stream, a);
  const dim3 g((unsigned)((px + 255) / 256));
  hipLaunchKernelGGL(k_fixed_to_float, g, dim3(256), 0, stream, a.acc1, a.overflow, a.grad_f1, px);
  hipLaunchKernelGGL(k_fixed_to_float, g, dim3(256), 0, stream, a.acc2, a.overflow, a.grad_f2, px);
  return hipGetLastError();
}

}  // namespace ffh
