// The batched step kernel for aSB (sb_batch_step.hpp), in its own
// translation unit so the modes compile in parallel.
#include "sb_batch_step.hpp"

namespace sbt {

hipError_t launch_batch_steps_asb(int jprec, const BatchArgs &B, hipStream_t st) {
    return launch_batch_steps_mode<kASB>(jprec, B, st);
}

}  // namespace sbt
