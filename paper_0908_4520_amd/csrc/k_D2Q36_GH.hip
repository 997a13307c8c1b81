// Step, init, codec and diagnostic kernels instantiated for the D2Q36_GH velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q36_GH() { register_lattice<D2Q36_GH>(); }
}  // namespace lbm
