// kNN-PCA surfel ellipsoids (placeholder until the hash-grid kernel lands).
#include "pcs_internal.hpp"

namespace pcs {

size_t knn_scratch_bytes(int64_t n) { return 256 + (size_t)n * 0; }

hipError_t launch_knn_pca(const float*, int64_t, int, float, float, float*, float*, float*, void*,
                          size_t, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace pcs
