// One instantiation of the batched step kernel (sb_batch_step.hpp): the mode,
// coupling format and workgroup shape come from SBT_BATCH_MODE, SBT_BATCH_JP
// and SBT_BATCH_TPB, so that the build compiles them in parallel, one object
// each.
#include "sb_batch_step.hpp"

#if !defined(SBT_BATCH_MODE) || !defined(SBT_BATCH_JP) || !defined(SBT_BATCH_TPB)
#error "build with -DSBT_BATCH_MODE=<0|1|2> -DSBT_BATCH_JP=<0|1> -DSBT_BATCH_TPB=<512|1024>"
#endif

namespace sbt {

template hipError_t launch_batch_steps_tu<SBT_BATCH_MODE, SBT_BATCH_JP, SBT_BATCH_TPB>(
    const BatchArgs &B, hipStream_t st);

}  // namespace sbt
