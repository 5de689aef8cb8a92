// Kernel instantiations for N = 384.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<384>(const cpra_params&);
}
