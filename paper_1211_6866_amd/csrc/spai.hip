// SPAI adaptive pattern search (Section 2.1).  Placeholder until the kernel lands.
#include "sai_internal.hpp"

namespace sai {

void spai_patterns(const sai_split_s*, const sai_build_opts&, hipStream_t, const Allocator&,
                   DBuf<int64_t>&, DBuf<int32_t>&, DBuf<int64_t>&, DBuf<int32_t>&, DBuf<int32_t>&,
                   DBuf<int32_t>&) {
  SAI_THROW(SAI_EINVAL, "the SPAI pattern is not available in this build");
}

}  // namespace sai
