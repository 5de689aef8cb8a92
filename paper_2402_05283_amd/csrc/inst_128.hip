// Kernel instantiations for N = 128.
#include "impl.hpp"

namespace cpra_impl {
template Ops ops_for_size<128>(const cpra_params&);
}
