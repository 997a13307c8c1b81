// Step, init, codec and diagnostic kernels instantiated for the D2Q17 velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q17() { register_lattice<D2Q17>(); }
}  // namespace lbm
