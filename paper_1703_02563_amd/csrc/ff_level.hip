// Host side of the temporally blocked level kernel: launch variants and
// run-length tables, and the dispatch to the per-scale translation units
// (ff_level_s0.hip ... ff_level_s6.hip; the kernels are in ff_level_kernels.h).
#include <algorithm>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

constexpr int kH = ffh::kLevelHalo;
// Tile / workgroup variants of the level kernel (tile, threads, load
// schedule, window halo: launch_n in ff_level_kernels.h maps each index to
// its kernel; the tiles and halos here must match it).  Index kNumVariants of the
// per-scale table selects the step-wise schedule instead (one launch per
// half-sweep or random-search step over all cells, no halo): better where
// the grid is too small to give every compute unit a tile.  A variant with
// quad evaluations addresses image b with 32-bit offsets; for a larger map
// its fallback (a halo at least as wide; batches count their work items
// with level_tiles, which follows the fallback) runs instead.
struct Variant {
  int tw, th, halo, fallback;
};
constexpr Variant kVariants[] = {{64, 32, kH, 0}, {32, 16, kH, 1}, {32, 16, kH, 2}, {16, 16, kH, 3},
                                 {32, 32, kH, 4}, {32, 16, kH, 5}, {16, 16, kH, 6}, {32, 32, kH, 7},
                                 {8, 8, kH, 8},   {16, 16, kH, 9}, {16, 16, kH, 10}, {16, 16, 2, 3},
                                 {32, 16, 2, 2},  {16, 16, kH, 3}, {8, 8, kH, 8},   {8, 8, 2, 8},
                                 {32, 16, 4, 2},  {16, 16, 4, 3}};
constexpr int kNumVariants = 18;
static_assert(sizeof(kVariants) / sizeof(kVariants[0]) == kNumVariants, "variant table");

using ScaleLaunch = hipError_t (*)(const ffh::LevelKArgs &, const ffh::BatchStage *, int, hipStream_t);
using ScaleLaunchF32 = hipError_t (*)(const ffh::LevelKArgs &, int, hipStream_t);
constexpr ScaleLaunch kScale[7] = {ffh::launch_level_scale0, ffh::launch_level_scale1, ffh::launch_level_scale2,
                                   ffh::launch_level_scale3, ffh::launch_level_scale4, ffh::launch_level_scale5,
                                   ffh::launch_level_scale6};
constexpr ScaleLaunchF32 kScaleF32[7] = {ffh::launch_level_f32_scale0, ffh::launch_level_f32_scale1,
                                         ffh::launch_level_f32_scale2, ffh::launch_level_f32_scale3,
                                         ffh::launch_level_f32_scale4, ffh::launch_level_f32_scale5,
                                         ffh::launch_level_f32_scale6};

hipError_t dispatch(const ffh::LevelKArgs &a, const ffh::BatchStage *batch, int log2n, int variant,
                    hipStream_t stream) {
  if (log2n < 0 || log2n >= 7 || variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  return kScale[log2n](a, batch, variant, stream);
}

// Window halo of every variant of the float-feature level kernel (image a's
// samples staged in LDS, 64 bytes each; launch_nf32 in ff_level_kernels.h
// maps each index to its tile and kernel): 16x16 / 8x8 / 8x8 / 8x8 / 16x16.
constexpr int kHaloF32[] = {2, 2, 4, 6, 4};
constexpr int kNumVariantsF32 = 5;
static_assert(sizeof(kHaloF32) / sizeof(kHaloF32[0]) == kNumVariantsF32, "float variant table");

// Per-scale float variant (index log2 n); written by ff_set_level_variant_f32.
// 8x8 tiles from n = 4 on, where 16x16 tiles leave most compute units idle.
int g_variant_f32[7] = {0, 0, 1, 1, 1, 1, 1};

hipError_t dispatch_f32(const ffh::LevelKArgs &a, int log2n, hipStream_t stream) {
  if (log2n < 0 || log2n >= 7) return hipErrorInvalidValue;
  return kScaleF32[log2n](a, g_variant_f32[log2n], stream);
}

// Per-scale variant table (index log2 n); written by ff_set_level_variant.
int g_variant[7] = {2, 2, 3, 3, 3, 3, 3};
// Most propagation steps per launch, per cost kind and scale (0: as many as
// the halo allows).  Shorter runs recompute less halo at the price of more
// launches; the float features' evaluations are expensive enough that one
// step per launch is fastest at every scale (measured at 1024x436).
int g_passes[2][7] = {{0, 0, 0, 0, 0, 0, 0}, {1, 1, 1, 1, 1, 1, 1}};

}  // namespace

namespace ffh {

int level_variant_count() { return kNumVariants + 1; }  // + the step-wise schedule

int get_level_variant(int log2n) { return (log2n >= 0 && log2n < 7) ? g_variant[log2n] : -1; }

bool level_stepwise(int log2n) { return get_level_variant(log2n) == kNumVariants; }

int get_level_passes(int log2n, int fcost) {
  return (log2n >= 0 && log2n < 7 && (fcost == 0 || fcost == 1)) ? g_passes[fcost][log2n] : -1;
}

bool set_level_passes(int log2n, int fcost, int passes) {
  if (log2n < 0 || log2n >= 7 || (fcost != 0 && fcost != 1) || passes < 0 || passes > 64) return false;
  g_passes[fcost][log2n] = passes;
  return true;
}

// Blocked kernel variant used where the table asks for the step-wise
// schedule but the caller only has the blocked form (batches, ff_run_level).
static int blocked_variant(int log2n) {
  const int v = get_level_variant(log2n);
  return v == kNumVariants ? 3 : v;
}

int level_variant_count_f32() { return kNumVariantsF32; }

int get_level_variant_f32(int log2n) { return (log2n >= 0 && log2n < 7) ? g_variant_f32[log2n] : -1; }

bool set_level_variant_f32(int log2n, int variant) {
  if (log2n < 0 || log2n >= 7 || variant < 0 || variant >= kNumVariantsF32) return false;
  g_variant_f32[log2n] = variant;
  return true;
}

bool set_level_variant(int log2n, int variant) {
  if (log2n < 0 || log2n >= 7 || variant < 0 || variant >= level_variant_count()) return false;
  g_variant[log2n] = variant;
  return true;
}

static int log2_of(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

int level_window_halo_f32(int log2n) {
  const int v = get_level_variant_f32(log2n);
  return v < 0 ? 2 : kHaloF32[v];
}

int level_window_halo(int log2n) {
  const int v = blocked_variant(log2n);
  return v < 0 ? kLevelHalo : kVariants[v].halo;
}

bool level_map_fits(int W, int H, int log2n) {
  const size_t P = (size_t)ffk::desc_pad(1 << log2n);
  return ((size_t)W + 2 * P) * ((size_t)H + 2 * P) * 16 < ((size_t)1 << 31);
}

// The table's variant, or its fallback where image b's map is too large
// for the 32-bit offsets of the quad evaluations.
static int launch_variant(int log2n, bool map_fits) {
  const int v = blocked_variant(log2n);
  return (v >= 0 && !map_fits) ? kVariants[v].fallback : v;
}

hipError_t launch_level(LevelKArgs a, hipStream_t stream) {
  const int l2 = log2_of(a.n);
  if (a.fcost) return dispatch_f32(a, l2, stream);
  return dispatch(a, nullptr, l2, launch_variant(l2, level_map_fits(a.W, a.H, l2)), stream);
}

hipError_t launch_batch_level(const LevelKArgs &base, const BatchStage &st, bool maps_fit, hipStream_t stream) {
  const int l2 = log2_of(base.n);
  return dispatch(base, &st, l2, launch_variant(l2, maps_fit), stream);
}

int level_tiles(int Wn, int Hn, int log2n, bool maps_fit) {
  const int v = launch_variant(log2n, maps_fit);
  if (v < 0) return 0;
  const Variant t = kVariants[v];
  return ((Wn + t.tw - 1) / t.tw) * ((Hn + t.th - 1) / t.th);
}

void level_halo(int t_begin, int t_end, int halo[4]) {
  halo[0] = halo[1] = halo[2] = halo[3] = 0;
  for (int t = t_begin; t < t_end; ++t) {
    const int d = t & 3;
    halo[(d == 0 || d == 3) ? 0 : 1] += 2;
    halo[(d == 0 || d == 2) ? 2 : 3] += 2;
  }
}

}  // namespace ffh
