// Instantiations of the k-NN graph kernel for dimensions 13..16.
#include "knn_graph.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_GRAPH_D(13) BDL_KNN_GRAPH_D(14) BDL_KNN_GRAPH_D(15) BDL_KNN_GRAPH_D(16)
}  // namespace knn_detail
}  // namespace bdl
