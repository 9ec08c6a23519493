// Region filter (Sec. 3.7, after the consistency check): regions of kept
// pixels, two 4-neighbours belonging to one region iff their flows differ by
// less than 3 px; a region of fewer than s pixels is deleted if one of its
// pixels could take in, by the same rule, a removed outlier (a set pixel the
// check did not keep).
//
// Regions are found by union-find in a scratch array of parents with
// parent[x] <= x at all times: a union hooks the larger of two roots under
// the smaller with a compare-and-swap, so every root ends as the smallest
// pixel index of its region, whatever the order of the unions.  A find
// follows strictly decreasing indices and stops; a failed swap returns a
// smaller parent, so the larger of the two roots decreases on every retry
// and a union ends after at most N retries.  Finds halve their paths (a
// parent is lowered with atomicMin to its own parent, an ancestor, so the
// order invariant holds), and once all unions are done every pixel's parent
// is set to its root, so the later passes find roots in one step.  Parents
// are read with device-scope atomic loads (no stale copies in a compute
// unit's cache).
#include <mutex>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

using ffk::kUnset;

__device__ __forceinline__ int rf_load(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int rf_find(const int32_t *parent, int x) {
  for (;;) {
    const int p = rf_load(parent + x);
    if (p == x) return x;
    x = p;
  }
}

// The same with path halving: x's parent is lowered to its grandparent.
__device__ __forceinline__ int rf_find_halve(int32_t *parent, int x) {
  for (;;) {
    const int p = rf_load(parent + x);
    if (p == x) return x;
    const int g = rf_load(parent + p);
    if (g != p) atomicMin(parent + x, g);
    x = p;
  }
}

__device__ __forceinline__ bool rf_linked(int32_t fa, int32_t fb) {
  const int dx = ffk::flow_x(fa) - ffk::flow_x(fb), dy = ffk::flow_y(fa) - ffk::flow_y(fb);
  return dx * dx + dy * dy < 9;
}

// Parents start as the start of each pixel's linked run within its wave
// (64 consecutive pixels of one row, found with a ballot: no atomics), the
// run start itself and unkept pixels as their own parent; parent <= index.
__global__ __launch_bounds__(256) void k_rf_init(const int32_t *flow, const uint8_t *keep, int32_t *parent,
                                                 int32_t *size, uint32_t *flag, int W, int H) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int k = y * W + x;
  const bool in = x < W && y < H;
  const bool hl = in && lane > 0 && keep[k] && keep[k - 1] && rf_linked(flow[k], flow[k - 1]);
  const unsigned long long starts = __ballot(!hl);  // lane 0 always starts a run
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int start = 63 - __clzll(starts & upto);
  if (!in) return;
  parent[k] = k - (lane - start);
  size[k] = 0;
  flag[k] = 0;
}

__device__ __forceinline__ void rf_union(int32_t *parent, int a, int b) {
  int ra = rf_find_halve(parent, a), rb = rf_find_halve(parent, b);
  while (ra != rb) {
    if (ra > rb) {
      const int t = ra;
      ra = rb;
      rb = t;
    }
    const int old = atomicCAS(parent + rb, rb, ra);  // hook rb under ra if rb is still a root
    if (old == rb) return;
    rb = rf_find_halve(parent, old);  // old < rb
    ra = rf_find_halve(parent, ra);
  }
}

// Unions of the links the initial runs do not hold: a horizontal link into
// the previous wave's pixels, and a vertical link unless the left
// neighbour's vertical link already implies it (both rows' runs go on).
__global__ __launch_bounds__(256) void k_rf_union(const int32_t *flow, const uint8_t *keep, int32_t *parent, int W,
                                                  int H) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int k = y * W + x;
  const bool on = x < W && y < H && keep[k] != 0;
  int32_t f = 0;
  if (on) f = flow[k];
  const bool hl = on && x > 0 && keep[k - 1] && rf_linked(f, flow[k - 1]);
  const bool below = on && y + 1 < H && keep[k + W] != 0;
  const bool vl = below && rf_linked(f, flow[k + W]);
  const bool hlb = below && x > 0 && keep[k + W - 1] && rf_linked(flow[k + W], flow[k + W - 1]);
  const bool vl_left = __shfl_up(vl, 1);
  if (hl && lane == 0) rf_union(parent, k, k - 1);
  if (vl && !(lane > 0 && hl && hlb && vl_left)) rf_union(parent, k, k + W);
}

// After the unions: every pixel's parent becomes its root.
__global__ __launch_bounds__(256) void k_rf_flatten(int32_t *parent, int W, int H) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const int k = y * W + x;
  const int r = rf_find(parent, k);
  if (r != k) atomicMin(parent + k, r);
}

// Region sizes, and whether a region borders a removed outlier it could
// take in.  The atomics are aggregated per wave (neighbouring pixels mostly
// share a root): the first pending lane's root is served with one atomic
// for all lanes of that root, until every lane is served (at most 64 rounds,
// the same for all lanes of the wave).
__global__ __launch_bounds__(256) void k_rf_measure(const int32_t *flow, const uint32_t *cost, const uint8_t *keep,
                                                    const int32_t *parent, int32_t *size, uint32_t *flag, int W,
                                                    int H) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  const int k = y * W + x;
  const bool on = x < W && y < H && keep[k] != 0;
  int r = -1;
  bool touches = false;
  if (on) {
    r = rf_find(parent, k);
    const int32_t f = flow[k];
    const int nx[4] = {x + 1, x - 1, x, x}, ny[4] = {y, y, y + 1, y - 1};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      if (nx[d] < 0 || nx[d] >= W || ny[d] < 0 || ny[d] >= H) continue;
      const int kn = ny[d] * W + nx[d];
      touches |= !keep[kn] && cost[kn] != kUnset && rf_linked(f, flow[kn]);
    }
  }
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(on);
  while (pending) {
    const int leader = __ffsll(pending) - 1;
    const int rl = __shfl(r, leader);
    const unsigned long long same = __ballot(on && r == rl) & pending;
    const unsigned long long hit = __ballot(on && r == rl && touches) & pending;
    if (lane == leader) {
      atomicAdd(size + rl, (int)__popcll(same));
      if (hit) atomicOr(flag + rl, 1u);
    }
    pending &= ~same;
  }
}

__global__ __launch_bounds__(256) void k_rf_apply(const uint8_t *keep, const int32_t *parent, const int32_t *size,
                                                  const uint32_t *flag, int W, int H, int s, uint8_t *keep_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const int k = y * W + x;
  uint8_t out = 0;
  if (keep[k]) {
    const int r = rf_find(parent, k);
    out = !(size[r] < s && flag[r] != 0);
  }
  keep_out[k] = out;
}

}  // namespace

namespace ffh {

size_t region_filter_scratch_bytes(int W, int H) { return (size_t)W * H * 3 * sizeof(int32_t); }

hipError_t launch_region_filter(const int16_t *flow, const uint32_t *cost, const uint8_t *keep, int W, int H, int s,
                                void *work, uint8_t *keep_out, hipStream_t stream) {
  const size_t N = (size_t)W * H;
  int32_t *parent = static_cast<int32_t *>(work);
  int32_t *size = parent + N;
  uint32_t *flag = reinterpret_cast<uint32_t *>(size + N);
  const int32_t *f = reinterpret_cast<const int32_t *>(flow);
  const dim3 grid((W + 255) / 256, H), block(256);
  hipLaunchKernelGGL(k_rf_init, grid, block, 0, stream, f, keep, parent, size, flag, W, H);
  hipLaunchKernelGGL(k_rf_union, grid, block, 0, stream, f, keep, parent, W, H);
  hipLaunchKernelGGL(k_rf_flatten, grid, block, 0, stream, parent, W, H);
  hipLaunchKernelGGL(k_rf_measure, grid, block, 0, stream, f, cost, keep, parent, size, flag, W, H);
  hipLaunchKernelGGL(k_rf_apply, grid, block, 0, stream, keep, parent, size, flag, W, H, s, keep_out);
  return hipGetLastError();
}

}  // namespace ffh

// ---- the region filter without caller-provided scratch ----------------------
// Parents, sizes and flags of up to kNoAllocMaxPixels pixels live in a
// static device array.  Its name in host code is only a host-side stand-in:
// the device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is handed
// to the kernels.  Every call on one device shares its copy (k_rf_init
// rewrites all of it that a call reads: parents, sizes and flags), so calls
// that overlap on one device race.

namespace {

constexpr size_t kNoAllocMaxPixels = (size_t)1 << 21;  // 2,097,152 pixels (1920 x 1080 fits): 24 MiB
static __device__ __align__(256) int32_t scratch[3 * kNoAllocMaxPixels];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (nullptr on error).
void *noalloc_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

namespace ffh {

size_t region_filter_noalloc_max_pixels() { return kNoAllocMaxPixels; }

hipError_t launch_region_filter_noalloc(const int16_t *flow, const uint32_t *cost, const uint8_t *keep, int W, int H,
                                        int s, uint8_t *keep_out, hipStream_t stream) {
  void *work = noalloc_scratch();
  if (!work) return hipErrorInvalidDevicePointer;
  return launch_region_filter(flow, cost, keep, W, H, s, work, keep_out, stream);
}

}  // namespace ffh
