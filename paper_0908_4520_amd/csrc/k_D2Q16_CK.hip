// Step, init, codec and diagnostic kernels instantiated for the D2Q16_CK velocity set.
#include "kernels_impl.h"

namespace lbm {
void register_D2Q16_CK() { register_lattice<D2Q16_CK>(); }
}  // namespace lbm
