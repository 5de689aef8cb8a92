// Kernel instantiations for N = 256.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<256>(const cpra_params&);
}
