// Kernel instantiations for N = 64.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<64>(const cpra_params&);
}
