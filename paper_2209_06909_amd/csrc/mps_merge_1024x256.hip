// mps_merge_1024x256.hip -- level merges with 1024-output tiles and 256-thread workgroups.
#include "mps_merge.h"

namespace mps {

hipError_t launch_merges_1024x256(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                                  const uint64_t *tile_base, int level, hipStream_t s) {
  return launch_merges_cfg<1024, 256>(kt, a, w, tj, tile_base, level, s);
}

}  // namespace mps
