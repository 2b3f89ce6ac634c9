// One instantiation of the batched step kernel (sb_batch_step.hpp): the mode
// and coupling format come from SBT_BATCH_MODE and SBT_BATCH_JP, so that
// the build compiles the pairs in parallel, one object each.
#include "sb_batch_step.hpp"

#if !defined(SBT_BATCH_MODE) || !defined(SBT_BATCH_JP)
#error "build with -DSBT_BATCH_MODE=<0|1|2> -DSBT_BATCH_JP=<0|1>"
#endif

namespace sbt {

template hipError_t launch_batch_steps_tu<SBT_BATCH_MODE, SBT_BATCH_JP>(const BatchArgs &B,
                                                                      hipStream_t st);

}  // namespace sbt
