// Step, init, codec and diagnostic kernels instantiated for the D3Q39 velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D3Q39() { register_lattice<D3Q39>(); }
}  // namespace lbm
