// Step, init, codec and diagnostic kernels instantiated for the D2Q21 velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q21() { register_lattice<D2Q21>(); }
}  // namespace lbm
