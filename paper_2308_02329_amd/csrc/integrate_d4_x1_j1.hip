// Instantiates the register-resident integrator for d = 4, 1 state
// term(s) and 1 coupling term(s), every supported tile count.
#include "integrate_kernel.h"

namespace chym {
KernelSet lookup_resident_4_1_1(int tiles) { return lookup_tiles<4, 1, 1>(tiles); }
}  // namespace chym
