// Kernel instantiations for N = 1024.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<1024>(const cpra_params&);
}
