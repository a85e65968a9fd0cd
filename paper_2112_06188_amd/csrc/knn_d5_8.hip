// Instantiations of the k-NN traversal for dimensions 5..8.
#include "knn_traverse.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_LAUNCH_D(5) BDL_KNN_LAUNCH_D(6) BDL_KNN_LAUNCH_D(7) BDL_KNN_LAUNCH_D(8)
}  // namespace knn_detail
}  // namespace bdl
