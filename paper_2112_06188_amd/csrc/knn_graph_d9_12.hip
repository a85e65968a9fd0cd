// Instantiations of the k-NN graph kernel for dimensions 9..12.
#include "knn_graph.hpp"

namespace bdl {
namespace knn_detail {
BDL_KNN_GRAPH_D(9) BDL_KNN_GRAPH_D(10) BDL_KNN_GRAPH_D(11) BDL_KNN_GRAPH_D(12)
}  // namespace knn_detail
}  // namespace bdl
