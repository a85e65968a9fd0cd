// Instantiations of the k-NN traversal for dimensions 1..4.
#include "knn_traverse.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_LAUNCH_D(1) BDL_KNN_LAUNCH_D(2) BDL_KNN_LAUNCH_D(3) BDL_KNN_LAUNCH_D(4)
}  // namespace knn_detail
}  // namespace bdl
