// Step, init, codec and diagnostic kernels instantiated for the D2Q37 velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q37() { register_lattice<D2Q37>(); }
}  // namespace lbm
