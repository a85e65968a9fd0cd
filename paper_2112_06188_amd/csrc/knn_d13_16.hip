// Instantiations of the k-NN traversal for dimensions 13..16.
#include "knn_traverse.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_LAUNCH_D(13) BDL_KNN_LAUNCH_D(14) BDL_KNN_LAUNCH_D(15) BDL_KNN_LAUNCH_D(16)
}  // namespace knn_detail
}  // namespace bdl
