// Instantiations of the FP64 descending-sweep projection for 1 source
// column, plain j_l (one translation unit each, so they compile in parallel).
#include "project_fp64_desc_kernel.hpp"

namespace los {

hipError_t project_fp64_desc_launch_n1(const ProjectArgs &a, const ProjectShape &sh,
                                        hipStream_t s) {
  return desc::launch_plain<1>(a, sh, s);
}

}  // namespace los
