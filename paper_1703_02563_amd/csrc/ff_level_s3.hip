// Level kernels of scale 2^3 (see ff_level_kernels.h).
#include "ff_level_kernels.h"

namespace ffh {

hipError_t launch_level_scale3(const LevelKArgs &a, const BatchStage *batch, int variant, hipStream_t stream) {
  return launch_n<3>(a, batch, variant, stream);
}

hipError_t launch_level_f32_scale3(const LevelKArgs &a, int variant, hipStream_t stream) {
  return launch_nf32<3>(a, variant, stream);
}

hipError_t launch_level_r2_scale3(const LevelKArgs &a, int variant, hipStream_t stream) {
  return launch_n_rx<3, 2>(a, variant, stream);
}

hipError_t launch_level_r4_scale3(const LevelKArgs &a, int variant, hipStream_t stream) {
  return launch_n_rx<3, 4>(a, variant, stream);
}

}  // namespace ffh
