// Instantiations of the k-NN graph kernel for dimensions 1..4.
#include "knn_graph.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_GRAPH_D(1) BDL_KNN_GRAPH_D(2) BDL_KNN_GRAPH_D(3) BDL_KNN_GRAPH_D(4)
}  // namespace knn_detail
}  // namespace bdl
