// Instantiations of the FP64 descending-sweep projection for 1 source
// column, with scaled columns (one translation unit each, so they compile in parallel).
#include "project_fp64_desc_kernel.hpp"

namespace los {

hipError_t project_fp64_desc_launch_n1_sc(const ProjectArgs &a, const ProjectShape &sh,
                                           hipStream_t s) {
  return desc::launch_scaled<1>(a, sh, s);
}

}  // namespace los
