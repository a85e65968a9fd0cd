// Internal accessors of a tree for other parts of the library (the request
// loop of the served form); not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "bdl.h"

namespace bdl {

hipStream_t tree_stream(const bdl_tree* t);
int tree_dim(const bdl_tree* t);
// Record msg as this thread's last error (bdl_last_error) and return code.
int tree_fail(int code, const char* msg);

}  // namespace bdl
