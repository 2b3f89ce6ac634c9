// The register-row resident step kernel for aSB
// (sb_resident_reg_step.hpp), in its own translation unit so the modes
// compile in parallel.
#include "sb_resident_reg_step.hpp"

namespace sbt {

hipError_t launch_resident_reg_asb(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    return launch_reg_m<kASB>(A, S, st);
}

}  // namespace sbt
