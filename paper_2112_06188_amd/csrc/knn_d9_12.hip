// Instantiations of the k-NN traversal for dimensions 9..12.
#include "knn_traverse.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_LAUNCH_D(9) BDL_KNN_LAUNCH_D(10) BDL_KNN_LAUNCH_D(11) BDL_KNN_LAUNCH_D(12)
}  // namespace knn_detail
}  // namespace bdl
