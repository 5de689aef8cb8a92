// Kernel instantiations for N = 512.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<512>(const cpra_params&);
}
