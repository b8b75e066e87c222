// mps_merge_4096x1024.hip -- level merges with 4096-output tiles and 1024-thread workgroups.
#include "mps_merge.h"

namespace mps {

hipError_t launch_merges_4096x1024(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                                  const uint64_t *tile_base, int level, hipStream_t s) {
  return launch_merges_cfg<4096, 1024>(kt, a, w, tj, tile_base, level, s);
}

}  // namespace mps
