// Step, init, codec and diagnostic kernels instantiated for the D2Q25_CK velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q25_CK() { register_lattice<D2Q25_CK>(); }
}  // namespace lbm
