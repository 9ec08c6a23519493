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
// with level_tiles, which follows the fallback) runs instead.  Variants 18-25,
// 28, 29 and 31 evaluate interior cells on the weight-class row maps; without
// those maps (a caller that passes none) their descriptor-quad twin (`nowf`,
// same halo, the same tile where one exists) runs.
struct Variant {
  int tw, th, halo, fallback, nowf;
};
constexpr Variant kVariants[] = {
    {64, 32, kH, 0, 0},   {32, 16, kH, 1, 1},   {32, 16, kH, 2, 2},   {16, 16, kH, 3, 3},   {32, 32, kH, 4, 4},
    {32, 16, kH, 5, 5},   {16, 16, kH, 6, 6},   {32, 32, kH, 7, 7},   {8, 8, kH, 8, 8},     {16, 16, kH, 9, 9},
    {16, 16, kH, 10, 10}, {16, 16, 2, 3, 11},   {32, 16, 2, 2, 12},   {16, 16, kH, 3, 13},  {8, 8, kH, 8, 14},
    {8, 8, 2, 8, 15},     {32, 16, 4, 2, 16},   {16, 16, 4, 3, 17},   {32, 16, 4, 2, 16},   {16, 16, 4, 3, 17},
    {32, 16, 2, 2, 12},   {16, 16, 2, 3, 11},   {8, 8, kH, 8, 14},    {8, 8, 2, 8, 15},     {32, 16, 4, 2, 16},
    {64, 32, 4, 0, 16},   {8, 8, kH, 8, 26},    {8, 8, 4, 8, 27},     {8, 8, kH, 8, 26},    {8, 8, 4, 8, 27},
    {16, 16, kH, 10, 30}, {32, 12, 2, 2, 12},   {4, 4, 4, 8, 32}};
constexpr int kNumVariants = 33;
static_assert(sizeof(kVariants) / sizeof(kVariants[0]) == kNumVariants, "variant table");

using ScaleLaunch = hipError_t (*)(const ffh::LevelKArgs &, const ffh::BatchStage *, int, hipStream_t);
using ScaleLaunchF32 = hipError_t (*)(const ffh::LevelKArgs &, int, hipStream_t);
constexpr ScaleLaunchF32 kScaleR2[7] = {ffh::launch_level_r2_scale0, ffh::launch_level_r2_scale1,
                                        ffh::launch_level_r2_scale2, ffh::launch_level_r2_scale3,
                                        ffh::launch_level_r2_scale4, ffh::launch_level_r2_scale5,
                                        ffh::launch_level_r2_scale6};
constexpr ScaleLaunchF32 kScaleR4[7] = {ffh::launch_level_r4_scale0, ffh::launch_level_r4_scale1,
                                        ffh::launch_level_r4_scale2, ffh::launch_level_r4_scale3,
                                        ffh::launch_level_r4_scale4, ffh::launch_level_r4_scale5,
                                        ffh::launch_level_r4_scale6};

// Radius-2 / radius-4 kernel of a table entry: the descriptor-quad variant
// with the same window halo (the run lengths follow the table's halo) -- a
// weight-class variant's quad twin, or for a one-lane variant (all of halo
// kLevelHalo) the quad variant of that halo and a tile of the same class.
int quad_variant(int v) {
  v = kVariants[v].nowf;
  switch (v) {
    case 11: case 12: case 13: case 14: case 15: case 16: case 17: case 26: case 27: case 30: return v;
    default: return kVariants[v].tw >= 16 ? 13 : 14;
  }
}
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

// The built-in launch tables.  Byte descriptors: weight-class evaluations
// on 32x12 tiles (256 threads, six workgroups per compute unit; two steps
// per launch) at n = 1, descriptor quads on 16x16 tiles with 256 threads
// and a halo of 2 at n = 2, with 1024 threads on 16x16 tiles at n = 4, on
// 8x8 tiles at n = 8 and on 4x4 tiles at n = 16 (so that the small grid
// still gives most compute units a workgroup); at most three steps per
// launch (the table tuned at 1024x436, which also halves the time of the
// older one-lane table at 160x120 and 1242x375).
// Float features: 16x16 tiles at n <= 2, 8x8 tiles from n = 4
// on (16x16 tiles leave most compute units idle there), one step per launch
// (the float evaluations are expensive enough that this is fastest at every
// scale, measured at 1024x436).
constexpr ffh::Tuning kDefaultTuning = {{31, 11, 30, 26, 32, 3, 3},
                                        {3, 3, 3, 3, 3, 0, 0},
                                        {0, 0, 1, 1, 1, 1, 1},
                                        {1, 1, 1, 1, 1, 1, 1}};

}  // namespace

namespace ffh {

const Tuning &default_tuning() { return kDefaultTuning; }

int level_variant_count() { return kNumVariants + 1; }  // + the step-wise schedule

int level_variant_count_f32() { return kNumVariantsF32; }

bool level_stepwise(int variant) { return variant == kNumVariants; }

bool tuning_ok(const Tuning &t) {
  for (int k = 0; k < kTuneScales; ++k) {
    if (t.variant[k] < 0 || t.variant[k] >= level_variant_count()) return false;
    if (t.variant_f32[k] < 0 || t.variant_f32[k] >= kNumVariantsF32) return false;
    if (t.passes[k] < 0 || t.passes[k] > 64 || t.passes_f32[k] < 0 || t.passes_f32[k] > 64) return false;
  }
  return true;
}

// Blocked kernel variant used where the table asks for the step-wise
// schedule but the caller only has the blocked form (batches, ff_run_level).
static int blocked_variant(int variant) { return variant == kNumVariants ? 3 : variant; }

static int log2_of(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

int level_window_halo_f32(int variant) {
  return (variant >= 0 && variant < kNumVariantsF32) ? kHaloF32[variant] : 2;
}

int level_window_halo(int variant) {
  const int v = blocked_variant(variant);
  return (v >= 0 && v < kNumVariants) ? kVariants[v].halo : kLevelHalo;
}

bool level_map_fits(int W, int H, int log2n) {
  const size_t P = (size_t)ffk::desc_pad(1 << log2n);
  return ((size_t)W + 2 * P) * ((size_t)H + 2 * P) * 16 < ((size_t)1 << 31);
}

bool level_uses_wform(int variant) {
  return variant >= 0 && variant < kNumVariants && kVariants[variant].nowf != variant;
}

// The table's variant, or its fallback where image b's map is too large
// for the 32-bit offsets of the quad evaluations, or its descriptor-quad
// twin where the weight-class maps are missing.
static int launch_variant(int variant, bool map_fits, bool has_wform) {
  int v = blocked_variant(variant);
  if (v < 0 || v >= kNumVariants) return v;
  if (!map_fits) return kVariants[v].fallback;
  if (!has_wform) v = kVariants[v].nowf;
  return v;
}

static bool dirs_have_wform(const LevelKArgs &a) {
  for (int d = 0; d < a.ndir; ++d)
    if (!a.dir[d].Wa || !a.dir[d].Wb) return false;
  return true;
}

bool level_blocked_ok(int W, int H, int L, int radius) {
  if (radius == 3) return true;
  if (radius != 2 && radius != 4) return false;
  for (int l = 0; l < L; ++l)
    if (!level_map_fits(W, H, l)) return false;
  return true;
}

hipError_t launch_level(LevelKArgs a, hipStream_t stream) {
  const int l2 = log2_of(a.n);
  if (a.fcost) {
    if (l2 < 0 || l2 >= 7) return hipErrorInvalidValue;
    return kScaleF32[l2](a, a.variant, stream);
  }
  if (a.sub_m) {  // a sub-scale stage: the descriptor-quad kernel of the table's window halo
    const int v = blocked_variant(a.variant);
    if (l2 < 0 || l2 >= 7 || v < 0 || v >= kNumVariants || (a.radius != 0 && a.radius != 3)) return hipErrorInvalidValue;
    return dispatch(a, nullptr, l2, quad_variant(v), stream);
  }
  if (a.radius == 2 || a.radius == 4) {
    const int v = blocked_variant(a.variant);
    if (l2 < 0 || l2 >= 7 || v < 0 || v >= kNumVariants || !level_map_fits(a.W, a.H, l2))
      return hipErrorInvalidValue;
    return (a.radius == 2 ? kScaleR2 : kScaleR4)[l2](a, quad_variant(v), stream);
  }
  return dispatch(a, nullptr, l2, launch_variant(a.variant, level_map_fits(a.W, a.H, l2), dirs_have_wform(a)),
                  stream);
}

hipError_t launch_batch_level(const LevelKArgs &base, const BatchStage &st, bool maps_fit, hipStream_t stream) {
  const int l2 = log2_of(base.n);
  return dispatch(base, &st, l2, launch_variant(base.variant, maps_fit, true), stream);
}

int level_tiles(int Wn, int Hn, int variant, bool maps_fit) {
  const int v = launch_variant(variant, maps_fit, true);
  if (v < 0 || v >= kNumVariants) return 0;
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
