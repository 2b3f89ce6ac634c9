// The batched step kernel for bSB (sb_batch_step.hpp), in its own
// translation unit so the modes compile in parallel.
#include "sb_batch_step.hpp"

namespace sbt {

hipError_t launch_batch_steps_bsb(int jprec, const BatchArgs &B, hipStream_t st) {
    return launch_batch_steps_mode<kBSB>(jprec, B, st);
}

}  // namespace sbt
