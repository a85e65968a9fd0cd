// Instantiations of the k-NN graph kernel for dimensions 5..8.
#include "knn_graph.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_GRAPH_D(5) BDL_KNN_GRAPH_D(6) BDL_KNN_GRAPH_D(7) BDL_KNN_GRAPH_D(8)
}  // namespace knn_detail
}  // namespace bdl
