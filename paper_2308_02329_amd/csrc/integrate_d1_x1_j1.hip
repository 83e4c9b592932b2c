// Instantiates the register-resident integrator for d = 1, 1 state
// term(s) and 1 coupling term(s), every supported tile count.
#include "integrate_kernel.h"

namespace chym {
KernelSet lookup_resident_1_1_1(int tiles) { return lookup_tiles<1, 1, 1>(tiles); }
}  // namespace chym
