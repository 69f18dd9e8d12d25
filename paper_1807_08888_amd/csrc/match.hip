// Top-k labelled subgraph matching on the GPU (placeholder until the
// matching kernels land).
#include "nuri_internal.h"

namespace nuri {

void run_matches(Graph &, const std::vector<const nuri_pattern *> &,
                 const std::vector<uint32_t> &, const QueryOpts &, std::vector<Result> &) {
  throw Error{NURI_EINVAL, "labelled matching is not available in this build"};
}

}  // namespace nuri
