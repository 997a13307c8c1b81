// Step, init, codec and diagnostic kernels instantiated for the D2Q9 velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q9() { register_lattice<D2Q9>(); }
}  // namespace lbm
