// Level kernels of scale 2^6 (see ff_level_kernels.h).
#include "ff_level_kernels.h"

namespace ffh {

hipError_t launch_level_scale6(const LevelKArgs &a, const BatchStage *batch, int variant, hipStream_t stream) {
  return launch_n<6>(a, batch, variant, stream);
}

hipError_t launch_level_f32_scale6(const LevelKArgs &a, int variant, hipStream_t stream) {
  return launch_nf32<6>(a, variant, stream);
}

hipError_t launch_level_r2_scale6(const LevelKArgs &a, int variant, hipStream_t stream) {
  return launch_n_rx<6, 2>(a, variant, stream);
}

hipError_t launch_level_r4_scale6(const LevelKArgs &a, int variant, hipStream_t stream) {
  return launch_n_rx<6, 4>(a, variant, stream);
}

}  // namespace ffh
