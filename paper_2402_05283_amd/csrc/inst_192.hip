// Kernel instantiations for N = 192.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<192>(const cpra_params&);
}
